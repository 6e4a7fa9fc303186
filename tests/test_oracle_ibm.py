"""Pins of the oracle's immersed-boundary treatment against what the paper fixes.

* lambda of Eq. (7) for a straight wall at a known distance (closed form);
* a wall lying on the box wall gives delta = dy/2, i.e. the classical
  antisymmetric no-slip ghost, lambda = nu/dy^2;
* corrections of several arms are additive (end of Sec. 2.2);
* the exponential-fit update of Eqs. (13)-(15) is exact for a constant
  right-hand side; its limits lambda = 0 and lambda -> infinity (Sec. 2.4);
* 1 >= B >= 0 for the exponential and Taylor forms (Sec. 2.4);
* the steady discrete plane Poiseuille solution
      u_j = a (h^2 - y_j^2 + delta (dy - delta)),  Pi = -2 nu a
  is a fixed point of the full RK3 step for any dt and any B form
  (constraint (ii) of Sec. 2.4), its error against the exact parabola is
  second order, and the staircase baseline is first order (Sec. 2.3);
* the time integration is second order with the exponential B and first
  order with B = 1 (Sec. 2.5).
"""
import math

import numpy as np
import pytest

import ibm_inputs as I
from oracle.ibm_oracle import (B_EULER, B_EXP, B_TAYLOR2, CFR, CPG, RK_C, OGrid, Oracle,
                               stage_coefficients)


def _flat(ny=33, nx=4, nz=4, off=0.37, nu=0.01, dt=0.05, forcing=CFR, q=2.0 * math.pi, b_mode=B_EXP,
          lx=2 * math.pi, lz=math.pi):
    c = I.Case(nx=nx, ny=ny, nz=nz, lx=lx, lz=lz, y_lo=-1.0, y_hi=1.0, nu=nu, dt=dt, forcing=forcing,
               q_target_or_pi=q, b_mode=b_mode, geometry="flat", geo_params=(off,))
    return c, OGrid.from_case(c)


def test_lambda_flat_wall_closed_form():
    c, g = _flat(off=0.37)
    o = Oracle(g)
    o.set_geometry(*I.make_sdf(c))
    dy = g.dy
    delta = 0.13 * dy        # first u row sits dy/2 above the box wall; wall is 0.37 dy above it
    lam_expected = g.nu * (dy - delta) / (delta * dy * dy)
    assert np.allclose(o.lam["u"][0], lam_expected, rtol=1e-12)
    assert np.allclose(o.lam["u"][-1], lam_expected, rtol=1e-12)
    assert np.allclose(o.lam["w"][0], lam_expected, rtol=1e-12)
    assert np.all(o.lam["u"][1:-1] == 0.0)
    # v: first internal face is 0.63 dy from the wall
    dv = 0.63 * dy
    assert np.allclose(o.lam["v"][1], g.nu * (dy - dv) / (dv * dy * dy), rtol=1e-12)
    assert np.all(o.lam["v"][0] == 0.0)


def test_box_wall_is_antisymmetric_ghost():
    c, g = _flat(off=0.0)
    o = Oracle(g)
    o.set_geometry(*I.make_sdf(c))
    assert np.allclose(o.lam["u"][0], g.nu / g.dy ** 2, rtol=1e-13)
    assert np.allclose(o.lam["w"][-1], g.nu / g.dy ** 2, rtol=1e-13)
    assert np.all(o.lam["v"] == 0.0)


def test_lambda_additive_two_arms():
    """A point whose x-arm and y-arm both cross an inclined plane wall gets the sum of
    the two arm corrections, each with its own exact wall distance."""
    c = I.Case(nx=8, ny=9, nz=4, lx=2.0, lz=1.0, y_lo=-1.0, y_hi=1.0, nu=0.02, dt=0.01)
    g = OGrid.from_case(c)
    dx, dy = c.dx, c.dy
    assert dx == dy
    jP = 4
    ycP = c.y_lo + (jP + 0.5) * dy
    y0 = ycP + 0.1 * dx
    su, sv, sw = I._sample(c, lambda X, Y, Z: (X + (Y - y0)) / math.sqrt(2.0))
    o = Oracle(g)
    o.set_geometry(su, sv, sw)
    assert o.tags["u"][jP, 0, 1] and not o.tags["u"][jP, 0, 0] and not o.tags["u"][jP - 1, 0, 1]
    d = 0.9 * dx        # distance to the plane along +x and along +y from the external neighbours
    lam_arm = g.nu * (dx - d) / (d * dx * dx)
    assert math.isclose(o.lam["u"][jP, 0, 1], 2.0 * lam_arm, rel_tol=1e-12)


@pytest.mark.parametrize("lam", [0.0, 1e-3, 0.7, 13.0, 450.0])
@pytest.mark.parametrize("k", [0, 1, 2])
def test_exponential_update_exact_for_constant_forcing(lam, k):
    """(B u + c_k dt f)/A equals the exact solution of du/dt = -lam u + f over c_k dt."""
    dt, w0, f = 0.03, 0.8, -1.7
    B, A = stage_coefficients(np.array([lam]), k, dt, B_EXP)
    got = (B * w0 + RK_C[k] * dt * f) / A
    tau = RK_C[k] * dt
    x = lam * tau
    # exact solution w0 e^{-x} + f tau (1 - e^{-x})/x, written without cancellation
    exact = w0 + f * tau if lam == 0.0 else w0 * math.exp(-x) + f * tau * (-math.expm1(-x)) / x
    assert abs(got[0] - exact) < 1e-14 * max(1.0, abs(exact))


def test_update_limits_and_bounds():
    x = np.concatenate([[0.0], np.logspace(-8, 4, 200)])
    dt = 1.0
    for mode in (B_EXP, B_TAYLOR2):
        B, A = stage_coefficients(x / RK_C[0], 0, dt, mode)
        assert np.all(B <= 1.0) and np.all(B >= 0.0)
        assert np.all(A >= B)
    B, A = stage_coefficients(np.array([0.1, 1.0, 10.0]) / RK_C[0], 0, dt, B_EXP)
    assert np.allclose(B, [0.1 / math.expm1(0.1), 1 / math.expm1(1.0), 10 / math.expm1(10.0)], rtol=1e-14)
    assert np.allclose(B, [0.9508, 0.5820, 4.54e-4], rtol=2e-3)
    # lambda -> infinity: the update returns zero (exact wall value)
    B, A = stage_coefficients(np.array([1e12]), 0, 0.01, B_EXP)
    assert (B * 3.0 + 0.01 * 5.0) / A < 1e-9
    # Taylor-2 matches exp(-x) to second order
    xs = np.array([1e-2, 5e-3])
    B, A = stage_coefficients(xs / RK_C[0], 0, 1.0, B_TAYLOR2)
    e = np.abs(B / A - np.exp(-xs))
    assert 2.8 < math.log2(e[0] / e[1]) < 3.2


def _discrete_poiseuille(g: OGrid, off: float):
    """Exact steady discrete solution (derived from Eqs. (5)-(7) at the first point)."""
    yc = g.y_lo + (np.arange(g.ny - 1) + 0.5) * g.dy
    hw = 1.0 - off * g.dy
    delta = (yc[0] - (-hw))
    prof = hw * hw - yc * yc + delta * (g.dy - delta)
    # flow-rate constraint: lz * sum(u) dy = Q_t
    a = g.q_target_or_pi / (g.lz * prof.sum() * g.dy)
    return a, a * prof, hw, delta


@pytest.mark.parametrize("b_mode", [B_EXP, B_EULER, B_TAYLOR2])
@pytest.mark.parametrize("dt", [0.05, 0.011])
def test_poiseuille_is_fixed_point(b_mode, dt):
    c, g = _flat(ny=33, dt=dt, b_mode=b_mode)
    o = Oracle(g)
    o.set_geometry(*I.make_sdf(c))
    a, prof, hw, delta = _discrete_poiseuille(g, 0.37)
    u = np.broadcast_to(prof[:, None, None], g.shape).copy()
    o.set_state(u, np.zeros(g.shape), np.zeros(g.shape), np.zeros(g.shape))
    o.step(3)
    assert np.abs(o.u - u).max() < 1e-13 * np.abs(u).max()
    assert np.abs(o.v).max() < 1e-13 and np.abs(o.w).max() < 1e-13
    assert math.isclose(o.pi_last, -2.0 * g.nu * a, rel_tol=1e-11)


def test_poiseuille_cpg_fixed_point():
    c, g = _flat(ny=17, forcing=CPG, q=-0.02)
    o = Oracle(g)
    o.set_geometry(*I.make_sdf(c))
    a = 0.02 / (2 * g.nu)
    yc = g.y_lo + (np.arange(g.ny - 1) + 0.5) * g.dy
    hw = 1.0 - 0.37 * g.dy
    delta = yc[0] + hw
    u = np.broadcast_to((a * (hw * hw - yc * yc + delta * (g.dy - delta)))[:, None, None], g.shape).copy()
    o.set_state(u, 0 * u, 0 * u, 0 * u)
    o.step(2)
    assert np.abs(o.u - u).max() < 1e-13 * np.abs(u).max()


def test_poiseuille_converges_from_noise():
    """Starting from rest plus noise, the solver approaches the discrete fixed point."""
    c, g = _flat(ny=17, nx=4, nz=4, nu=0.05, dt=0.02)
    o = Oracle(g)
    o.set_geometry(*I.make_sdf(c))
    u, v, w = I.random_fields(c, seed=1, amp=1e-3)
    o.set_state(u, v, w, np.zeros(g.shape))
    a, prof, hw, delta = _discrete_poiseuille(g, 0.37)
    e0 = np.abs(o.u - prof[:, None, None]).max()
    o.step(1500)
    e1 = np.abs(o.u - prof[:, None, None]).max()
    assert e1 < 1e-7 * e0, (e0, e1)


def test_poiseuille_spatial_order():
    """Error of the steady IBM solution against the exact parabola is a*delta*(dy-delta):
    exactly second order at fixed delta/dy.  With the bare staircase the wall sits at the
    ghost row and the error is first order (Sec. 2.3)."""
    errs_ibm, errs_st = [], []
    for ny in (17, 33, 65, 129):
        c, g = _flat(ny=ny, dt=0.2 * (2.0 / (ny - 1)) ** 2 / 0.01 * 0.5)
        o = Oracle(g)
        o.set_geometry(*I.make_sdf(c))
        a, prof, hw, delta = _discrete_poiseuille(g, 0.37)
        u = np.broadcast_to(prof[:, None, None], g.shape).copy()
        o.set_state(u, 0 * u, 0 * u, 0 * u)
        o.step(1)
        assert np.abs(o.u - u).max() < 1e-12 * np.abs(u).max()
        yc = g.y_lo + (np.arange(g.ny - 1) + 0.5) * g.dy
        exact = a * (hw * hw - yc * yc)   # same flux normalisation constant a
        errs_ibm.append(np.abs(prof - exact).max())
        # staircase: lambda = 0; the steady profile vanishes on the ghost rows
        os_ = Oracle(g)
        os_.set_geometry(*I.make_sdf(c), ibm=False)
        hs = 1.0 + 0.5 * g.dy
        prof_s = hs * hs - yc * yc
        a_s = g.q_target_or_pi / (g.lz * prof_s.sum() * g.dy)
        us = np.broadcast_to((a_s * prof_s)[:, None, None], g.shape).copy()
        os_.set_state(us, 0 * us, 0 * us, 0 * us)
        os_.step(1)
        assert np.abs(os_.u - us).max() < 1e-12 * np.abs(us).max()
        # compare with the exact parabola through the true wall at the same flux
        prof_e = np.clip(hw * hw - yc * yc, 0, None)
        a_e = g.q_target_or_pi / (g.lz * (4.0 / 3.0) * hw ** 3)
        errs_st.append(np.abs(a_s * prof_s - a_e * prof_e).max())
    p_ibm = [math.log2(errs_ibm[i] / errs_ibm[i + 1]) for i in range(3)]
    p_st = [math.log2(errs_st[i] / errs_st[i + 1]) for i in range(3)]
    assert all(1.95 < p < 2.15 for p in p_ibm) and p_ibm[-1] < 2.05, p_ibm
    assert all(0.8 < p < 1.3 for p in p_st), p_st


def _startup_flow_rate(b_mode, nsteps, T=0.1):
    c, g = _flat(ny=17, nx=2, nz=2, nu=1.0, dt=T / nsteps, forcing=CPG, q=-2.0, b_mode=b_mode, off=0.37)
    o = Oracle(g)
    o.set_geometry(*I.make_sdf(c))
    z = np.zeros(g.shape)
    o.set_state(z, z, z, z)
    o.step(nsteps)
    return o.flow_rate(o.u)


def test_time_order_exponential():
    """Start-up of plane Poiseuille flow under a constant pressure gradient: the flow rate
    at t = T converges with order 2 in dt with the exponential B (Sec. 2.5)."""
    ns = [16, 32, 64]
    qs = [_startup_flow_rate(B_EXP, n) for n in ns]
    qref = _startup_flow_rate(B_EXP, 512)
    e = [abs(q - qref) for q in qs]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert all(1.9 < p < 2.3 for p in orders), (orders, e)


def test_time_order_euler():
    """Same start-up problem with B = 1 (implicit Euler IBM term): first order in dt."""
    ns = [64, 128, 256]
    qs = [_startup_flow_rate(B_EULER, n) for n in ns]
    qref = 2.0 * _startup_flow_rate(B_EULER, 1024) - _startup_flow_rate(B_EULER, 512)
    e = [abs(q - qref) for q in qs]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert all(0.75 < p < 1.25 for p in orders), (orders, e)
