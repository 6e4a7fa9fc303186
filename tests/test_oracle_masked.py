"""Pins of the oracle's masked projection (continuity on the internal pressure cells only,
external faces never corrected; Sec. 3.3 read strictly).

* The sparse operator equals, entry by entry, D (mask) G assembled column by column from
  the oracle's divergence and gradient (pinned on their own) applied to unit vectors,
  on tiny boxes with an undulated wall and with a random mask of solid cells.
* Without any solid the masked problem is the full-box one: same phi as the FFT solver.
* After a masked step the divergence vanishes at every internal pressure cell (the
  property that defines the projection), while the full-box projection leaves a leak
  there; the velocity only changes on internal faces and external faces stay zero.
* The discrete Poiseuille profile between off-grid flat walls stays a fixed point.
* The same on a stretched wall-normal grid (reading R20): the operator against the dense
  assembly, the solve without solid against the stretched FFT solver, no internal leak.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import ibm_inputs as I
from oracle.ibm_oracle import (CFR, OGrid, Oracle, classify, divergence, gradient, masked_laplacian,
                               masked_poisson_solve, poisson_solve)


def _dense_from_operators(g, tags):
    pin = tags["p"]
    cells = np.flatnonzero(pin.ravel())
    M = np.zeros((cells.size, cells.size))
    for col, c in enumerate(cells):
        e = np.zeros(g.shape)
        e.ravel()[c] = 1.0
        gx, gy, gz = gradient(g, e)
        d = divergence(g, np.where(tags["u"], gx, 0.0), np.where(tags["v"], gy, 0.0), np.where(tags["w"], gz, 0.0))
        M[:, col] = d.ravel()[cells]
    return M


def _open(nx=8, ny=7, nz=3, stretched=False, **kw):
    # stretched: faces clustered towards the undulated bottom (spacing ratio 4)
    if stretched:
        kw["y_faces"] = I.bottom_tanh_faces(ny, 0.0, 1.0, 4.0)
    c = I.Case(nx=nx, ny=ny, nz=nz, lx=4 * math.pi, lz=1.0, y_lo=0.0, y_hi=1.0, nu=0.02, dt=0.01, forcing=CFR,
               q_target_or_pi=0.95, seed=3, geometry="wavy_open", geo_params=(0.15, 0.5), top=1, **kw)
    return c, OGrid.from_case(c)


@pytest.mark.parametrize("stretched", [False, True])
def test_operator_matches_dense_assembly_undulated_wall(stretched):
    c, g = _open(stretched=stretched)
    tags = classify(g, *I.make_sdf(c))
    assert not tags["p"].all()
    L, cells = masked_laplacian(g, tags)
    np.testing.assert_allclose(L.toarray(), _dense_from_operators(g, tags), rtol=0, atol=1e-9)


@pytest.mark.parametrize("stretched", [False, True])
def test_operator_matches_dense_assembly_random_mask(stretched):
    c, g = _open(nx=6, ny=6, nz=4, stretched=stretched)
    rng = np.random.default_rng(5)
    su, sv, sw = (rng.uniform(-0.3, 1.0, s.shape) for s in I.make_sdf(c))
    tags = classify(g, su, sv, sw)
    L, cells = masked_laplacian(g, tags)
    np.testing.assert_allclose(L.toarray(), _dense_from_operators(g, tags), rtol=0, atol=1e-9)


@pytest.mark.parametrize("stretched", [False, True])
def test_no_solid_equals_full_box_solve(stretched):
    c, g = _open(nx=8, ny=9, nz=4, stretched=stretched)
    sdf = [np.ones_like(s) for s in I.make_sdf(c)]
    tags = classify(g, *sdf)
    assert tags["p"].all()
    rng = np.random.default_rng(2)
    rhs = rng.standard_normal(g.shape)
    wy = np.broadcast_to(g.dyc[:, None, None], g.shape)
    rhs -= np.sum(wy * rhs) / np.sum(wy)       # consistent: zero volume-weighted mean
    phi_m, res = masked_poisson_solve(g, rhs, tags)
    phi_f, _ = poisson_solve(g, rhs)
    assert res < 1e-12
    # the same solution up to the constant (each solver fixes its own mean)
    dm, df = phi_m - phi_m.mean(), phi_f - phi_f.mean()
    assert np.abs(dm - df).max() < 1e-12 * np.abs(df).max()


@pytest.mark.parametrize("stretched", [False, True])
def test_masked_step_has_no_internal_leak(stretched):
    c, g = _open(nx=16, ny=9, nz=4, stretched=stretched)
    sdf = I.make_sdf(c)
    u0, v0, w0 = I.make_initial(c, sdf)
    out = {}
    for proj in (0, 1):
        o = Oracle(replace(g, projection=proj))
        o.set_geometry(*sdf)
        o.set_state(u0, v0, w0, np.zeros_like(u0))
        o.step(2)
        t = o.tags
        d = divergence(g, o.u, o.v, o.w)
        scale = max(np.abs(o.u).max(), np.abs(o.v).max()) / min(g.dx, g.dy, g.dz)
        out[proj] = np.abs(np.where(t["p"], d, 0.0)).max() / scale
        for comp, f in (("u", o.u), ("v", o.v), ("w", o.w)):
            assert not np.any(np.where(t[comp], 0.0, f))
        if proj == 1:
            assert o.diag["poisson_rel_residual"] < 1e-12
            assert abs(np.sum(np.where(t["p"], o.p, 0.0))) < 1e-10 * np.abs(o.p).max()
    assert out[1] < 1e-13, out
    assert out[0] > 1e-6, out


def test_poiseuille_fixed_point_masked():
    c = I.Case(nx=4, ny=33, nz=4, lx=2 * math.pi, lz=math.pi, y_lo=-1.0, y_hi=1.0, nu=0.01, dt=0.05,
               forcing=CFR, q_target_or_pi=2 * math.pi, geometry="flat", geo_params=(0.37,), projection=1)
    g = OGrid.from_case(c)
    assert g.projection == 1
    o = Oracle(g)
    o.set_geometry(*I.make_sdf(c))
    yc = g.y_lo + (np.arange(g.ny - 1) + 0.5) * g.dy
    hw = 1.0 - 0.37 * g.dy
    delta = yc[0] + hw
    prof = hw * hw - yc * yc + delta * (g.dy - delta)
    a = g.q_target_or_pi / (g.lz * prof.sum() * g.dy)
    u = np.broadcast_to((a * prof)[:, None, None], g.shape).copy()
    o.set_state(u, 0 * u, 0 * u, 0 * u)
    o.step(3)
    assert np.abs(o.u - u).max() < 1e-13 * np.abs(u).max()
    assert np.abs(o.v).max() < 1e-13 and np.abs(o.w).max() < 1e-13
    assert math.isclose(o.pi_last, -2.0 * g.nu * a, rel_tol=1e-11)


def test_disconnected_cells_rejected():
    c, g = _open(nx=4, ny=6, nz=1)
    su, sv, sw = (np.full(s.shape, -1.0) for s in I.make_sdf(c))
    su[2, :, 1] = 1.0                  # one isolated internal u face in row 1 ...
    su[4, :, 1] = 1.0                  # ... and another one two rows above it
    tags = classify(g, su, sv, sw)
    with pytest.raises(ValueError):
        masked_poisson_solve(g, np.zeros(g.shape), tags)
