"""Pins of the oracle's moving immersed walls (rigid translation with velocity U_b; the
box walls at rest).

* Plane Poiseuille flow between immersed walls that slide with velocity U_w along x
  (constant pressure gradient): the discrete Poiseuille profile of walls at rest plus U_w
  is a fixed point of the full step, with the walls 0.37 of a cell inside the box (the
  external neighbour of the first row is the ghost row beyond the box wall, which stores
  zero) and 1.37 cells inside (the neighbour is an external point inside the box, which
  stores U_w).
* A wall velocity normal to the walls is not a steady state, but the source term of a
  sliding wall leaves v and w at zero.
* With U_b = 0 the moving-wall terms vanish (sigma U_b = 0) and every external point
  holds zero, as without the option.
* Galilean pin of sigma on a curved wall: fluid moving with a sphere's velocity stays
  uniform away from the box walls (a planted slip in sigma is caught).
"""
import math

import numpy as np
import pytest

import ibm_inputs as I
from oracle.ibm_oracle import CPG, OGrid, Oracle


def _flat(off, ny=33, nx=4, nz=4, nu=0.01, dt=0.05):
    c = I.Case(nx=nx, ny=ny, nz=nz, lx=2 * math.pi, lz=math.pi, y_lo=-1.0, y_hi=1.0, nu=nu, dt=dt, forcing=CPG,
               q_target_or_pi=-0.02, geometry="flat", geo_params=(off,))
    return c, OGrid.from_case(c)


@pytest.mark.parametrize("off", [0.37, 1.37])
def test_sliding_walls_poiseuille_fixed_point(off):
    c, g = _flat(off)
    o = Oracle(g)
    o.set_geometry(*I.make_sdf(c))
    uw = 0.73
    o.set_wall_velocity(uw, 0.0, 0.0)
    yc = g.y_lo + (np.arange(g.ny - 1) + 0.5) * g.dy
    hw = 1.0 - off * g.dy
    inside = np.abs(yc) < hw
    j0 = int(np.argmax(inside))
    delta = yc[j0] + hw
    a = 0.02 / (2 * g.nu)
    prof = np.where(inside, a * (hw * hw - yc * yc + delta * (g.dy - delta)) + uw, uw)
    u = np.broadcast_to(prof[:, None, None], g.shape).copy()
    o.set_state(u, 0 * u, 0 * u, 0 * u)
    o.step(3)
    assert np.abs(o.u - u).max() < 1e-13 * np.abs(u).max()
    assert np.abs(o.v).max() < 1e-13 and np.abs(o.w).max() < 1e-13
    # the walls' lambda and source split: sigma = lambda where the neighbour stores U_w
    # (inside the box), sigma = nu/(delta dy) where it stores zero (beyond the box wall)
    sig0 = o.sig["u"][j0, 0, 0]
    lam0 = o.lam["u"][j0, 0, 0]
    if off > 1.0:
        assert math.isclose(sig0, lam0, rel_tol=1e-14)
    else:
        assert math.isclose(sig0, g.nu / (delta * g.dy), rel_tol=1e-14)


def test_zero_wall_velocity_is_the_plain_method():
    c, g = _flat(1.37, ny=17)
    sdf = I.make_sdf(c)
    u0, v0, w0 = I.random_fields(c, seed=3, amp=0.1)
    runs = []
    for set_vel in (False, True):
        o = Oracle(g)
        o.set_geometry(*sdf)
        if set_vel:
            o.set_wall_velocity(0.0, 0.0, 0.0)
        o.set_state(u0, v0, w0, np.zeros_like(u0))
        o.step(2)
        runs.append(o)
    assert np.array_equal(runs[0].u, runs[1].u) and np.array_equal(runs[0].v, runs[1].v)
    t = runs[1].tags
    assert not np.any(np.where(t["u"], 0.0, runs[1].u))


def test_wall_shear_of_sliding_wall():
    """The wall shear of the sliding-wall Poiseuille state is that of the walls at rest:
    the discrete momentum balance 2 tau = -Pi n dy holds with u1 - U_w."""
    from oracle.ibm_oracle import wall_shear_profile
    c, g = _flat(0.37)
    sdf = I.make_sdf(c)
    o = Oracle(g)
    o.set_geometry(*sdf)
    uw = 0.4
    o.set_wall_velocity(uw, 0.0, 0.0)
    yc = g.y_lo + (np.arange(g.ny - 1) + 0.5) * g.dy
    hw = 1.0 - 0.37 * g.dy
    delta = yc[0] + hw
    a = 0.02 / (2 * g.nu)
    u = np.broadcast_to((a * (hw * hw - yc * yc + delta * (g.dy - delta)) + uw)[:, None, None], g.shape).copy()
    o.set_state(u, 0 * u, 0 * u, 0 * u)
    o.step(2)
    tau = wall_shear_profile(g, o.u, sdf[0], wall_velocity=uw)
    rows = int(o.tags["u"][:, 0, 0].sum())
    np.testing.assert_allclose(tau, -o.pi_last * rows * g.dy / 2.0, rtol=1e-12)


def _uniform_flow_past_moving_sphere(vel, sig_scale=1.0, steps=1):
    """A sphere (radius 0.35, minimum image in x and z) at least 5 cells from the box walls,
    moving at vel = (U, 0, W) through fluid that moves with it (u = U, v = 0, w = W
    everywhere, zero pressure, no forcing), one RK3 step; sig_scale plants a slip in sigma."""
    c = I.Case(nx=16, ny=17, nz=16, lx=2.0, lz=2.0, y_lo=-1.0, y_hi=1.0, nu=0.02, dt=0.02, forcing=CPG,
               q_target_or_pi=0.0, geometry="flat", geo_params=(0.0,))
    g = OGrid.from_case(c)

    def fn(X, Y, Z):
        dx = X - 1.0
        dx -= c.lx * np.round(dx / c.lx)
        dz = Z - 1.0
        dz -= c.lz * np.round(dz / c.lz)
        return np.sqrt(dx * dx + Y * Y + dz * dz) - 0.35
    o = Oracle(g)
    o.set_geometry(*I._sample(c, fn))
    for comp in "uvw":
        o.sig[comp] = o.sig[comp] * sig_scale
    o.set_wall_velocity(*vel)
    u = np.full(g.shape, vel[0])
    w = np.full(g.shape, vel[2])
    o.set_state(u, 0.0 * u, w, 0.0 * u)
    o.step(steps)
    return g, o


@pytest.mark.parametrize("vel", [(0.8, 0.0, 0.0), (0.3, 0.0, -0.5)])
def test_fluid_moving_with_a_curved_body_stays_uniform(vel):
    """Galilean pin of sigma on a curved wall (reading R19): with the fluid moving at the
    body's velocity, the ghost value of every cut arm is U_b and the near-wall operator
    vanishes, so the implicit update returns U_b exactly when sigma = lambda for arms that
    end at external points inside the box (every arm of a sphere away from the box
    walls).  The box walls at rest disturb only the rows within one stencil width per
    substep of them; everywhere else the step leaves u = U and w = W, v = 0 everywhere.  A
    planted sigma of 0.5 lambda moves the near-wall points by O(U)."""
    g, o = _uniform_flow_past_moving_sphere(vel)
    rows = slice(4, g.ny - 1 - 4)            # more than 3 rows from either box wall
    assert int((o.lam["u"][rows] > 0).sum()) > 0 and int((o.lam["w"][rows] > 0).sum()) > 0
    for comp in "uw":
        ibm = o.lam[comp][rows] > 0            # (the box-wall rows have sigma = 0: at rest)
        assert np.allclose(o.sig[comp][rows][ibm], o.lam[comp][rows][ibm], rtol=1e-14, atol=0.0)
    U, W = vel[0], vel[2]
    scale = max(abs(U), abs(W))
    assert np.abs(o.u[rows] - U).max() <= 1e-14 * scale
    assert np.abs(o.w[rows] - W).max() <= 1e-14 * scale
    assert np.abs(o.v).max() <= 1e-14 * scale
    # the box walls at rest do act on the rows next to them
    assert np.abs(o.u[0] - U).max() > 1e-3 * scale
    # a planted slip in sigma is caught
    g2, o2 = _uniform_flow_past_moving_sphere(vel, sig_scale=0.5)
    assert np.abs(o2.u[rows] - U).max() > 1e-3 * scale
