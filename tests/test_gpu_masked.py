"""Masked projection (continuity on the internal pressure cells only; conjugate gradients
preconditioned by the full-box solve) through the C ABI, against the oracle's sparse
direct solve on the same seeded inputs, and by its defining property at full size."""
import math

import numpy as np
import pytest
import torch

import ibm_inputs as I
from tests.gpu_helpers import case, device, gpu_grid, oracle_run, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    device()


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("name,nsteps", [("open_small", 2), ("wavy_small", 2), ("ellip_small", 1),
                                         ("flat_small", 2)])
def test_masked_step_parity(name, nsteps):
    c = case(name, projection=1)
    o, sdf, st = oracle_run(c, nsteps)
    g = gpu_grid(c, sdf, st)
    g.step(nsteps)
    u, v, w, p = [t.cpu().numpy() for t in g.get_state()]
    s = g.stats()
    scale = max(np.abs(o.u).max(), np.abs(o.v).max(), np.abs(o.w).max())
    errs = [np.abs(a - b).max() / scale for a, b in ((u, o.u), (v, o.v), (w, o.w))]
    ep = np.abs(p - o.p).max() / max(np.abs(o.p).max(), scale * scale)
    leak = s["div_max_internal_leak"] * min(o.g.dx, o.g.dy, o.g.dz) / scale
    _say(f"{name}: pcg iterations {s['pcg_iters']}, |r|/|b| {s['poisson_rel_residual']:.1e}; "
         f"u,v,w {['%.1e' % e for e in errs]} p {ep:.1e}; internal divergence * h / U {leak:.1e}")
    assert s["pcg_iters"] > 0 or name == "flat_small"
    assert 0.0 <= s["poisson_rel_residual"] <= 1e-13
    # the velocity to the 1e-12 FP64 target; the pressure, a sum of increments each solved
    # to the residual tolerance 1e-13, against its dynamic scale U^2 as in the other steps
    assert max(errs) <= 1e-12
    assert ep <= 1e-10
    assert leak < 1e-12
    g.close()


@pytest.mark.parametrize("name", ["open_small", "wavy_small"])
def test_masked_graph_equals_eager(name):
    """The masked projection inside a captured graph (fixed iteration budget, convergence
    tested on the device, no host access) gives bit for bit the eager result: the device
    flag stops the iterate at the same iteration in both."""
    c = case(name, projection=1)
    sdf = I.make_sdf(c)
    u0, v0, w0 = I.make_initial(c, sdf)
    st = (u0, v0, w0, np.zeros_like(u0))
    out = []
    for graph in (0, 1):
        g = gpu_grid(c, sdf, st)
        g.tune(graph=graph)
        g.step(4)
        s = g.stats()
        out.append(([t.cpu().numpy() for t in g.get_state()], s["pcg_iters"], s["poisson_rel_residual"]))
        g.close()
    _say(f"{name}: iterations eager {out[0][1]} graph {out[1][1]}, residual {out[1][2]:.1e}")
    assert out[0][1] == out[1][1] and out[1][1] > 0
    assert out[1][2] <= 1e-13
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name,nsteps", [("open_small", 2), ("wavy_small", 2)])
def test_masked_fp32_storage(name, nsteps):
    """The masked projection in FP32 storage: the conjugate gradients in FP64 with the FP32
    full-box solve as preconditioner (flexible beta), phi stored in FP32; against the
    oracle's FP64 direct solve the velocity is within the FP32-storage bar, 1e-5 of the
    largest speed component, the solve reaches its tolerance (1e-9) and continuity holds
    on the internal cells to FP32 rounding.  The captured graph equals the eager steps
    bit for bit."""
    c = case(name, projection=1)
    o, sdf, st = oracle_run(c, nsteps)
    out = []
    for graph in (0, 1):
        g = gpu_grid(c, sdf, st, "fp32")
        g.tune(graph=graph)
        g.step(nsteps)
        s = g.stats()
        out.append(([t.double().cpu().numpy() for t in g.get_state()], s))
        g.close()
    (u, v, w, p), s = out[0]
    scale = max(np.abs(o.u).max(), np.abs(o.v).max(), np.abs(o.w).max())
    errs = [np.abs(a - b).max() / scale for a, b in ((u, o.u), (v, o.v), (w, o.w))]
    leak = s["div_max_internal_leak"] * min(o.g.dx, o.g.dy, o.g.dz) / scale
    _say(f"{name} fp32: pcg iterations {s['pcg_iters']}, |r|/|b| {s['poisson_rel_residual']:.1e}; "
         f"u,v,w {['%.1e' % e for e in errs]}; internal divergence * h / U {leak:.1e}")
    assert s["pcg_iters"] > 0 and 0.0 <= s["poisson_rel_residual"] <= 1e-9
    assert max(errs) < 1e-5
    assert leak < 1e-5
    assert out[1][1]["pcg_iters"] == s["pcg_iters"]
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)


def test_masked_iteration_cap_is_reported():
    """A solve that reaches pcg_max_iter without converging (the device flag unset) makes
    ibm_step return IBM_ERR_UNSTABLE, also with the graph requested (its first step is
    eager)."""
    from paper_2506_14328_amd.ibm import IbmError
    import dataclasses
    c = dataclasses.replace(case("wavy_small", projection=1), pcg_max_iter=8)
    sdf = I.make_sdf(c)
    u0, v0, w0 = I.make_initial(c, sdf)
    g = gpu_grid(c, sdf, (u0, v0, w0, np.zeros_like(u0)))
    g.tune(graph=1)
    with pytest.raises(IbmError):
        g.step(3)          # the first, eager step stops at pcg_max_iter and reports it
    g.close()


def test_masked_equals_full_box_without_solid():
    """A flat channel whose walls are the box walls has no external cell: the masked
    problem is the full-box one and the conjugate gradients stop before the first
    iteration, leaving the full-box solution (gauge shifted to the internal mean, which
    is the full-box mean)."""
    c = case("flat_small", geo_params=(-0.5,))
    c1 = case("flat_small", geo_params=(-0.5,), projection=1)
    sdf = I.make_sdf(c)
    u0, v0, w0 = I.make_initial(c, sdf)
    st = (u0, v0, w0, np.zeros_like(u0))
    out = []
    for cc in (c, c1):
        g = gpu_grid(cc, sdf, st)
        assert g.stats()["n_p_internal"] == cc.nx * (cc.ny - 1) * cc.nz
        g.step(2)
        out.append([t.cpu().numpy() for t in g.get_state()])
        if cc is c1:
            assert g.stats()["pcg_iters"] == 0
        g.close()
    scale = max(np.abs(a).max() for a in out[0][:3])
    for a, b in zip(out[0][:3], out[1][:3]):
        assert np.abs(a - b).max() <= 1e-14 * scale


def test_masked_open_channel_full_size_property():
    """192x65x160 open channel, masked projection: after 3 steps the divergence at every
    internal pressure cell is at rounding level, where the full-box projection leaves a
    leak at the discretisation level; the solve converged (the iteration count and the
    flow rate of both states are printed)."""
    c0 = I.make_case("wavy_open")
    sdf = I.make_sdf(c0)
    u0, v0, w0 = I.make_initial(c0, sdf)
    st = (u0, v0, w0, np.zeros_like(u0))
    leaks = {}
    for proj in (0, 1):
        c = I.Case(**{**c0.__dict__, "projection": proj})
        g = gpu_grid(c, sdf, st)
        g.step(3)
        s = g.stats()
        scale = max(np.abs(u0).max(), 1.0)
        leaks[proj] = s["div_max_internal_leak"] * min(c.dx, c.dy, c.dz) / scale
        _say(f"projection {proj}: internal divergence * h / U {leaks[proj]:.2e}, q {s['q']:.12f}, "
             f"pcg iterations {s['pcg_iters']}, |r|/|b| {s['poisson_rel_residual']:.1e}")
        assert s["nan_flag"] == 0
        if proj == 1:
            assert 0 < s["pcg_iters"] and 0.0 <= s["poisson_rel_residual"] <= 1e-13
        g.close()
    assert leaks[1] < 1e-12
    assert leaks[0] > 1e3 * leaks[1]


def test_masked_and_full_box_instances_in_one_ensemble():
    """An ensemble holding a masked-projection instance and a full-box one steps eagerly
    (the graph knob is ignored while a masked instance is present) and both instances
    match their own oracle runs; the wall shear is read per instance."""
    from paper_2506_14328_amd import IbmGrid
    from oracle.ibm_oracle import wall_shear_profile
    from tests.test_gpu_wall_shear import _tau_tol
    cases = [case("open_small", projection=1), case("wavy_small")]
    runs = [oracle_run(c, 2) for c in cases]
    g = IbmGrid.ensemble(cases, precision="fp64")
    for i, (o, sdf, st) in enumerate(runs):
        g.set_geometry(*[torch.from_numpy(np.ascontiguousarray(a)).to(device()) for a in sdf], inst=i)
        g.set_state(*[torch.from_numpy(np.ascontiguousarray(a)).to(device()) for a in st], inst=i)
    g.tune(graph=1, batch=1)
    g.step(2)
    for i, (o, sdf, st) in enumerate(runs):
        u, v, w, p = [t.cpu().numpy() for t in g.get_state(inst=i)]
        scale = max(np.abs(o.u).max(), np.abs(o.v).max(), np.abs(o.w).max())
        errs = [np.abs(a - b).max() / scale for a, b in ((u, o.u), (v, o.v), (w, o.w))]
        _say(f"instance {i} ({cases[i].name}, projection {cases[i].projection}): {['%.1e' % e for e in errs]}")
        assert max(errs) <= 1e-12
        tau, _ = g.wall_shear(inst=i)
        ref = wall_shear_profile(o.g, o.u, sdf[0])
        tol = _tau_tol(o.g, sdf[0], 1e-11 * scale) + 1e-14 * np.abs(ref).max()
        assert np.abs(tau.cpu().numpy() - ref).max() <= tol
    assert g.stats(inst=0)["pcg_iters"] > 0 and g.stats(inst=1)["pcg_iters"] == 0
    g.close()
