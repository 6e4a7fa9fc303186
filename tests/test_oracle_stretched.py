"""Pins of the oracle on a stretched wall-normal grid (non-uniform face spacing).

* Faces given explicitly at uniform positions take the stretched code path and reproduce
  the uniform oracle (pinned elsewhere) to rounding.
* The three-point second derivative is exact for quadratics on any spacing (Eq. (3) with
  non-uniform coefficient triples): the Laplacian of a + b y + c y^2 is 2c at every row
  whose stencil stays inside the box, for the centre rows and for the v faces.
* The gradient of a pressure linear in y and the divergence of a v linear in y are their
  slopes; linear interpolation of u to the faces makes d(uv)/dy exact for u linear in y
  and v constant.
* The projection: D G phi equals the right-hand side minus its volume-weighted mean, with
  D and G the divergence and gradient pinned above.
* Plane Poiseuille flow between immersed walls on tanh-stretched grids converges to the
  exact parabola at second order (Sec. 2.3's claim, here with non-uniform spacing).
"""
import math

import numpy as np
import pytest

import ibm_inputs as I
from oracle.ibm_oracle import (CPG, OGrid, Oracle, convection, divergence, gradient_full, laplacian,
                               poisson_solve)


def _grid(ny=13, nx=4, nz=3, gamma=1.3, top=0):
    yf = np.asarray(I.tanh_faces(ny, -1.0, 1.0, gamma))
    return OGrid(nx=nx, ny=ny, nz=nz, lx=2.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.1, dt=0.01, top=top,
                 y_faces=yf)


def _col(a, g):
    return np.broadcast_to(np.asarray(a)[:, None, None], g.shape).copy()


def test_uniform_faces_reduce_to_uniform():
    c = I.Case(nx=16, ny=17, nz=8, lx=2 * math.pi, lz=math.pi, y_lo=-1.2, y_hi=1.0, nu=1.0 / 300.0, dt=0.01,
               forcing=0, q_target_or_pi=2.0 * math.pi, seed=4, geometry="wavy", geo_params=(0.1, math.pi / 2))
    sdf = I.make_sdf(c)
    st = I.laminar_plus_solenoidal(c, sdf, c.seed, amp=0.1)
    ref = Oracle(OGrid.from_case(c))
    gs = OGrid.from_case(c)
    gs.y_faces = np.linspace(c.y_lo, c.y_hi, c.ny)
    assert gs.stretched
    o = Oracle(gs)
    for x in (ref, o):
        x.set_geometry(*sdf)
        x.set_state(*st, np.zeros_like(st[0]))
        x.step(2)
    scale = np.abs(ref.u).max()
    for a, b in ((ref.u, o.u), (ref.v, o.v), (ref.w, o.w)):
        assert np.abs(a - b).max() < 1e-13 * scale
    assert abs(ref.pi_last - o.pi_last) < 1e-12 * abs(ref.pi_last)
    for k in "uvw":
        np.testing.assert_allclose(o.lam[k], ref.lam[k], rtol=1e-12, atol=0)


def test_second_derivative_exact_for_quadratics():
    g = _grid()
    a, b, c = 0.3, -1.7, 2.45
    yc, yf = g.yc, g.yf[:-1]
    fu = _col(a + b * yc + c * yc * yc, g)
    fv = _col(a + b * yf + c * yf * yf, g)
    lu = laplacian(g, fu, comp="u")
    lv = laplacian(g, fv, comp="v")
    # centre rows 1..n-2 (rows 0 and n-1 reach a ghost row); v faces 1..n-2 (face 1 reaches
    # face 0, stored as row 0 here with the quadratic's value; the top face reaches the
    # north wall face, which is not stored)
    np.testing.assert_allclose(lu[1:-1], 2.0 * c, rtol=1e-11)
    np.testing.assert_allclose(lv[1:-1], 2.0 * c, rtol=1e-11)
    # a uniform grid gives the same
    gu = OGrid(nx=4, ny=13, nz=3, lx=2.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.1, dt=0.01)
    yc = gu.yc
    np.testing.assert_allclose(laplacian(gu, _col(a + b * yc + c * yc * yc, gu))[1:-1], 2.0 * c, rtol=1e-11)


def test_gradient_divergence_and_interpolation_exact_for_linear_fields():
    g = _grid()
    s = 0.83
    p = _col(1.0 + s * g.yc, g)
    _, gy, _ = gradient_full(g, p)
    np.testing.assert_allclose(gy[1:], s, rtol=1e-12)
    assert np.all(gy[0] == 0.0)
    v = _col(0.2 + s * g.yf[:-1], g)
    d = divergence(g, np.zeros(g.shape), v, np.zeros(g.shape))
    np.testing.assert_allclose(d[:-1], s, rtol=1e-12)       # the top row reaches the wall face
    # u linear in y, v constant: d(uv)/dy = c b exactly with linear interpolation to faces
    bu, cv = -0.6, 0.35
    u = _col(0.1 + bu * g.yc, g)
    vv = np.full(g.shape, cv)
    nu_, _, _ = convection(g, u, vv, np.zeros(g.shape))
    np.testing.assert_allclose(nu_[1:-1], cv * bu, rtol=1e-12)
    # midpoint averaging would not be exact on this grid
    h = 0.5
    mid = ((h * (u[2:] + u[1:-1])) * cv - (h * (u[1:-1] + u[:-2])) * cv) / g.dyc[1:-1, None, None]
    assert np.abs(mid - cv * bu).max() > 1e-3 * abs(cv * bu)


@pytest.mark.parametrize("top", [0, 1])
def test_projection_consistent_with_divergence_and_gradient(top):
    g = _grid(ny=21, nx=8, nz=6, top=top)
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal(g.shape)
    phi, mean = poisson_solve(g, rhs)
    Gx, Gy, Gz = gradient_full(g, phi)
    dg = divergence(g, Gx, Gy, Gz)
    w = g.dyc[:, None, None] * np.ones(g.shape)
    wmean = float(np.sum(rhs * w) / np.sum(w))
    assert abs(mean - wmean) < 1e-12
    assert np.abs(dg - (rhs - wmean)).max() < 1e-10 * np.abs(rhs).max()


def test_poiseuille_between_immersed_walls_second_order_on_stretched_grids():
    """Walls at y = +-0.8 inside a box [-1, 1] with tanh-stretched faces (gamma = 1);
    constant pressure gradient Pi = -2, nu = 1: exact u = (0.64 - y^2).  Started from the
    exact profile and run to the discrete steady state."""
    errs = []
    for n in (8, 16, 32):
        yf = np.asarray(I.tanh_faces(n + 1, -1.0, 1.0, 1.0))
        hmin = np.diff(yf).min()
        g = OGrid(nx=2, ny=n + 1, nz=1, lx=1.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=1.0, dt=0.4 * hmin ** 2,
                  forcing=CPG, q_target_or_pi=-2.0, y_faces=yf)
        yw = 0.8
        yc = g.yc
        ycg = np.concatenate([[2 * yf[0] - yc[0]], yc, [2 * yf[-1] - yc[-1]]])
        su = np.broadcast_to((yw - np.abs(ycg))[:, None, None], (n + 2, 1, 2)).copy()
        sv = np.broadcast_to((yw - np.abs(yf))[:, None, None], (n + 1, 1, 2)).copy()
        o = Oracle(g)
        o.set_geometry(su, sv, su.copy())
        inside = np.abs(yc) < yw
        ex = np.where(inside, yw * yw - yc * yc, 0.0)
        u0 = np.broadcast_to(ex[:, None, None], g.shape).copy()
        z = np.zeros_like(u0)
        o.set_state(u0, z, z, z)
        o.step(int(1.2 / g.dt) + 1)
        errs.append(np.abs(o.u[:, 0, 0] - ex)[inside].max())
        assert np.abs(o.v).max() == 0.0 and np.abs(o.w).max() == 0.0
    orders = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert errs[-1] < 1e-3
    assert orders[-1] > 1.8, (errs, orders)

