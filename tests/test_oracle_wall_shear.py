"""Pins of the oracle's wall-shear diagnostic (tau(x), tau_1c, tau_1s of Sec. 4.2).

* A velocity linear in the distance to an undulated wall, with wall gradient
  a(x, z) = a0 + a1 cos(2 pi x/L_x) + a2 sin(2 pi x/L_x) + (a z-dependent part of zero
  spanwise mean), gives tau(x_i) = nu (a0 + a1 cos + a2 sin) exactly and the modes
  (nu a0, nu a1, nu a2): the wall is located from a signed function linear in y, so the
  linear zero crossing is exact; a quadratic term b d^2 adds nu b d1 per column.
* Steady discrete plane Poiseuille flow between off-grid walls (the oracle's own fixed
  point): the shear of the two walls balances the driving pressure gradient over the
  rows exactly, 2 tau = -Pi (rows) dy, the discrete momentum balance.
* Over the flat south box wall (no SDF cut) the wall sits dy/2 below row 0.
* Without the immersed-boundary correction the wall is at the external point below.
* The modes of a trigonometric polynomial in x are its coefficients (discrete
  orthogonality on the periodic grid of u points x_i = i dx).
"""
import math

import numpy as np

from oracle.ibm_oracle import OGrid, south_wall_points, wall_shear_modes, wall_shear_profile


def _grid(nx=32, ny=17, nz=3, nu=0.37):
    return OGrid(nx=nx, ny=ny, nz=nz, lx=4 * math.pi, lz=1.0, y_lo=0.0, y_hi=1.0, nu=nu, dt=0.01, top=1)


def _rows(g):
    """y of u rows -1 .. ny-1 (the SDF layout: row jj = j + 1), x of u points, z of rows."""
    y = g.y_lo + (np.arange(-1, g.ny) + 0.5) * g.dy
    x = np.arange(g.nx) * g.dx
    z = (np.arange(g.nz) + 0.5) * g.dz
    return y, x, z


def test_profile_over_undulated_wall_closed_form():
    g = _grid()
    y, x, z = _rows(g)
    eps, alpha = 0.05, 2 * math.pi / g.lx
    yw = eps * (1.0 + np.cos(alpha * x))                          # (nx,)
    sdf = y[:, None, None] - yw[None, None, :] + 0.0 * z[None, :, None]
    a0, a1, a2 = 1.3, -0.4, 0.25
    ax = a0 + a1 * np.cos(alpha * x) + a2 * np.sin(alpha * x)
    az = 0.3 * (np.arange(g.nz) - (g.nz - 1) / 2.0)              # zero spanwise mean
    a = ax[None, :] + az[:, None]                                 # (nz, nx)
    d = y[1:-1, None, None] - yw[None, None, :]                   # wall distance of u rows
    j1, d1 = south_wall_points(g, sdf)
    assert (j1 >= 0).all() and (j1 <= 2).all() and (j1 > 0).any()
    np.testing.assert_allclose(d1, (y[1:-1][j1] - yw[None, :]), rtol=0, atol=1e-15)
    # linear in the wall distance: exact
    u = np.where(d > 0, a[None] * d, 0.0)
    tau = wall_shear_profile(g, u, sdf)
    np.testing.assert_allclose(tau, g.nu * ax, rtol=0, atol=1e-13)
    t0, t1c, t1s = wall_shear_modes(g, tau)
    assert abs(t0 - g.nu * a0) < 1e-13
    assert abs(t1c - g.nu * a1) < 1e-13
    assert abs(t1s - g.nu * a2) < 1e-13
    # a quadratic term b d^2 adds nu b d1 in each column
    b = -0.9
    tau_q = wall_shear_profile(g, np.where(d > 0, a[None] * d + b * d * d, 0.0), sdf)
    np.testing.assert_allclose(tau_q, g.nu * (ax + b * d1.mean(axis=0)), rtol=0, atol=1e-13)


def test_discrete_momentum_balance_of_steady_poiseuille():
    """Constant-pressure-gradient plane channel, walls 0.37 of a cell inside the box: the
    steady discrete profile u_j = a (h^2 - y_j^2 + delta (dy - delta)) with Pi = -2 nu a is
    a fixed point of the oracle's step (pinned elsewhere); on it the two walls' shear
    balances Pi over the n rows of internal u points: 2 tau = -Pi n dy."""
    import ibm_inputs as I
    from oracle.ibm_oracle import CPG, Oracle
    c = I.Case(nx=4, ny=17, nz=2, lx=2 * math.pi, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.01, dt=0.05, forcing=CPG,
               q_target_or_pi=-0.02, geometry="flat", geo_params=(0.37,))
    g = OGrid.from_case(c)
    sdf = I.make_sdf(c)
    o = Oracle(g)
    o.set_geometry(*sdf)
    yc = g.y_lo + (np.arange(g.ny - 1) + 0.5) * g.dy
    hw = 1.0 - 0.37 * g.dy
    delta = yc[0] + hw
    a = 0.02 / (2 * g.nu)
    u = np.broadcast_to((a * (hw * hw - yc * yc + delta * (g.dy - delta)))[:, None, None], g.shape).copy()
    o.set_state(u, 0 * u, 0 * u, 0 * u)
    o.step(2)
    assert np.abs(o.u - u).max() < 1e-13 * np.abs(u).max()
    rows = int(o.tags["u"][:, 0, 0].sum())
    tau = wall_shear_profile(g, o.u, sdf[0])
    np.testing.assert_allclose(tau, -o.pi_last * rows * g.dy / 2.0, rtol=1e-12)


def test_flat_box_wall_poiseuille():
    g = _grid(nx=8, ny=11, nz=2, nu=0.01)
    y, _, _ = _rows(g)
    sdf = np.ones((g.ny + 1, g.nz, g.nx))                        # no SDF cut anywhere
    yc = y[1:-1]
    u = np.broadcast_to(((yc - g.y_lo) * (g.y_hi - yc))[:, None, None], g.shape).copy()
    j1, d1 = south_wall_points(g, sdf)
    assert (j1 == 0).all() and np.allclose(d1, 0.5 * g.dy)
    tau = wall_shear_profile(g, u, sdf)
    np.testing.assert_allclose(tau, g.nu * (g.y_hi - g.y_lo - 0.5 * g.dy), rtol=1e-13)


def test_staircase_wall_without_correction():
    g = _grid(nx=4, ny=9, nz=2, nu=0.5)
    sdf = np.ones((g.ny + 1, g.nz, g.nx))
    sdf[: 2 + 1] = -0.3                                           # rows -1..1 external
    j1, d1 = south_wall_points(g, sdf, ibm=False)
    assert (j1 == 2).all() and np.allclose(d1, g.dy)
    j1c, d1c = south_wall_points(g, sdf, ibm=True)
    assert (j1c == 2).all() and np.allclose(d1c, g.dy * 1.0 / 1.3)
    # linear in the distance from the staircase wall one row below row 2
    dist = (np.arange(g.ny - 1) - 1) * g.dy
    a = 0.7
    u = np.where(dist > 0, a * dist, 0.0)[:, None, None] * np.ones(g.shape)
    tau = wall_shear_profile(g, u, sdf, ibm=False)
    np.testing.assert_allclose(tau, g.nu * a, rtol=1e-12)
    tau_c = wall_shear_profile(g, u, sdf, ibm=True)
    np.testing.assert_allclose(tau_c, g.nu * a * g.dy / (g.dy / 1.3), rtol=1e-12)


def test_modes_of_trigonometric_polynomial():
    g = _grid(nx=48)
    x = np.arange(g.nx) * g.dx
    al = 2 * math.pi / g.lx
    c0, c1, c2, c3, c4 = 0.11, -0.07, 0.031, 0.5, -0.2
    tau = c0 + c1 * np.cos(al * x) + c2 * np.sin(al * x) + c3 * np.cos(2 * al * x) + c4 * np.sin(5 * al * x)
    t0, t1c, t1s = wall_shear_modes(g, tau)
    assert abs(t0 - c0) < 1e-15 and abs(t1c - c1) < 1e-15 and abs(t1s - c2) < 1e-15
