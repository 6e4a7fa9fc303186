"""ibm_solve_pressure_noalloc (the full-box pressure solve in the library's fixed work area,
for callers that cannot allocate) against ibm_solve_pressure of a grid with the same
descriptor, through the C ABI: two calls in a row, the second on a smaller grid, FP64 to
1e-12 and FP32 storage to 1e-5 of the solution's maximum; the removed mean too; a grid
beyond the work area is refused."""
import math

import pytest
import torch

import ibm_inputs as I
from tests.gpu_helpers import device

pytestmark = pytest.mark.gpu


def _case(nx, ny, nz):
    return I.Case(nx=nx, ny=ny, nz=nz, lx=2 * math.pi, lz=math.pi, y_lo=-1.2, y_hi=1.0, nu=1e-3, dt=0.01,
                  name=f"poisson_{nx}x{ny}x{nz}")


def _rhs(c, dtype, seed):
    gen = torch.Generator(device=device())
    gen.manual_seed(seed)
    return torch.randn((c.ny - 1, c.nz, c.nx), generator=gen, device=device(), dtype=torch.float64).to(dtype)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_noalloc_solve_matches_handle_solve(precision, tol):
    from paper_2506_14328_amd import IbmGrid, solve_pressure_noalloc
    dtype = torch.float64 if precision == "fp64" else torch.float32
    for n, (shape, seed) in enumerate((((192, 65, 96), 3), ((64, 17, 30), 4))):
        c = _case(*shape)
        print(f"no-alloc solve {precision} call {n + 1}: {shape}", flush=True)
        rhs = _rhs(c, dtype, seed)
        mean = torch.full((1,), float("nan"), dtype=torch.float64, device=device())
        phi = solve_pressure_noalloc(c, rhs, mean_removed=mean)
        g = IbmGrid.from_case(c, precision=precision)
        ref = g.solve_pressure(rhs)
        ref_mean = g.stats()["rhs_mean_removed"]
        g.close()
        torch.cuda.synchronize()
        err = ((phi.double() - ref.double()).abs().max() / ref.double().abs().max()).item()
        print(f"  max |phi - phi_ref| / max |phi_ref| = {err:.2e}; mean {mean.item():.3e} vs {ref_mean:.3e}",
              flush=True)
        assert err <= tol
        assert abs(mean.item() - ref_mean) <= 1e-14 * rhs.double().abs().max().item()


def test_noalloc_rejects_grid_beyond_work_area():
    from paper_2506_14328_amd import solve_pressure_noalloc
    from paper_2506_14328_amd.ibm import IbmError
    c = _case(512, 257, 256)   # 264 MB of FP64 half spectrum
    rhs = torch.zeros((c.ny - 1, c.nz, c.nx), dtype=torch.float64, device=device())
    with pytest.raises(IbmError):
        solve_pressure_noalloc(c, rhs)
