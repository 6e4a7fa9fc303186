"""Wall-shear stress along the south wall (tau(x), tau_1c, tau_1s of Sec. 4.2) through the
C ABI, against the oracle on the same seeded inputs and against closed forms.

* a velocity linear in the distance to the undulated wall gives tau(x_i) = nu a(x_i) and
  the modes of a(x) exactly, a quadratic term b d^2 adds nu b d1 per column (no oracle
  involved);
* the initial state and the state after several steps (open channel, closed wavy channel,
  bare staircase, FP32 storage) against the oracle's profile of its own run;
* error codes.
"""
import ctypes
import math

import numpy as np
import pytest
import torch

import ibm_inputs as I
from oracle.ibm_oracle import OGrid, south_wall_points, wall_shear_modes, wall_shear_profile
from tests.gpu_helpers import case, device, gpu_grid, oracle_run, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    device()


def _say(*a):
    print(*a, flush=True)


def _tau_tol(og, sdf, u_err, ibm=True):
    """Bound on |tau_gpu - tau_oracle| from a velocity difference u_err at the point each
    column reads: nu u_err / d1 at the smallest wall distance."""
    _, d1 = south_wall_points(og, sdf, ibm)
    return og.nu * u_err / float(d1[d1 > 0].min()) + 1e-300


def test_quadratic_field_closed_form():
    c = case("open_small")
    og = OGrid.from_case(c)
    grid = I.coords(c)
    x = grid["xf"]
    eps, alpha = c.geo_params
    yw = eps * (1.0 + np.cos(alpha * x))

    def sdf_of(xx, yy):
        return yy[:, None, None] - eps * (1.0 + np.cos(alpha * xx))[None, None, :] + np.zeros((1, c.nz, 1))

    sdf = (sdf_of(x, grid["yc_g"]), sdf_of(grid["xc"], grid["yf"]), sdf_of(grid["xc"], grid["yc_g"]))
    a0, a1, a2, bq = 1.1, 0.35, -0.6, -0.8
    a = a0 + a1 * np.cos(alpha * x) + a2 * np.sin(alpha * x)
    d = (grid["yc"][:, None, None] - yw[None, None, :]) * np.ones((1, c.nz, 1))
    d1 = d[np.argmax(d > 0, axis=0), np.arange(c.nz)[:, None], np.arange(c.nx)[None, :]]   # (nz, nx)
    z = np.zeros_like(d)
    for quad in (0.0, bq):
        u = np.where(d > 0, a[None, None, :] * d + quad * d * d, 0.0)
        want = og.nu * (a + quad * d1.mean(axis=0))
        for prec, dt, tol in (("fp64", torch.float64, 1e-13), ("fp32", torch.float32, 1e-6)):
            g = gpu_grid(c, sdf, (u, z, z, z), precision=prec)
            tau, (t0, t1c, t1s) = g.wall_shear()
            tau = tau.cpu().numpy()
            scale = og.nu * np.abs(a).max()
            _say(f"[{prec}, b={quad}] max |tau - expected| / scale = {np.abs(tau - want).max() / scale:.2e}")
            assert np.abs(tau - want).max() <= tol * scale
            if quad == 0.0:
                for got, w in ((t0, a0), (t1c, a1), (t1s, a2)):
                    assert abs(got - og.nu * w) <= tol * scale
            g.close()


@pytest.mark.parametrize("name,nsteps,ibm", [("open_small", 0, True), ("open_small", 4, True),
                                             ("wavy_small", 2, True), ("open_small", 2, False)])
def test_wall_shear_parity_fp64(name, nsteps, ibm):
    c = case(name)
    o, sdf, st = oracle_run(c, nsteps, ibm=ibm)
    g = gpu_grid(c, sdf, st, ibm=ibm)
    g.step(nsteps)
    tau, modes = g.wall_shear()
    tau = tau.cpu().numpy()
    ref = wall_shear_profile(o.g, o.u, sdf[0], ibm=ibm)
    ref_modes = wall_shear_modes(o.g, ref)
    scale = max(np.abs(o.u).max(), np.abs(o.v).max(), np.abs(o.w).max())
    u_err = (1e-15 if nsteps == 0 else 1e-12) * scale
    tol = _tau_tol(o.g, sdf[0], u_err, ibm) + 1e-14 * np.abs(ref).max()
    err = np.abs(tau - ref).max()
    _say(f"{name} steps={nsteps} ibm={ibm}: max|dtau| {err:.2e} (bound {tol:.2e}); modes {modes} vs {ref_modes}")
    assert err <= tol
    for got, want in zip(modes, ref_modes):
        assert abs(got - want) <= 2 * tol
    g.close()


def test_wall_shear_fp32_storage_initial_state():
    c = case("open_small")
    sdf = I.make_sdf(c)
    u0, v0, w0 = I.make_initial(c, sdf)
    st32 = [a.astype(np.float32).astype(np.float64) for a in (u0, v0, w0, np.zeros_like(u0))]
    g = gpu_grid(c, sdf, st32, precision="fp32")
    tau, modes = g.wall_shear()
    og = OGrid.from_case(c)
    ref = wall_shear_profile(og, st32[0], sdf[0])
    tol = 1e-13 * np.abs(ref).max()
    assert np.abs(tau.cpu().numpy() - ref).max() <= tol
    for got, want in zip(modes, wall_shear_modes(og, ref)):
        assert abs(got - want) <= 2 * tol
    g.close()


def test_wall_shear_errors():
    from paper_2506_14328_amd import IbmGrid
    c = case("open_small")
    g = IbmGrid.from_case(c)
    out = (ctypes.c_double * 3)()
    assert g.lib.ibm_wall_shear(g._h, 0, None, out) == -4          # before the geometry
    assert g.lib.ibm_wall_shear(g._h, 5, None, out) == -1          # no such instance
    g.close()
