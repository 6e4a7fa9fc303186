"""Pins of the oracle's free-slip north face (the open channel of Sec. 4.2).

* An open channel with a free-slip face at y = H is the lower half of the closed channel
  mirrored about y = H: started from mirrored states, the closed channel's lower half
  equals the open channel after several full RK3 steps (projection, flow-rate control and
  immersed boundary included).  This ties the free-slip treatment to the no-slip one,
  which the other oracle tests pin.
* Over a flat wall at distance delta below the first u row, the steady discrete open
  Poiseuille profile u_j = a ((H - y_w)^2 - (H - y_j)^2 + delta (dy - delta)),
  Pi = -2 nu a, is a fixed point of the full step (the closed-channel solution of
  Sec. 2.4's constraint (ii), centred on the free-slip face).
* The free-slip face contributes no lambda to the top row; a no-slip face does.
"""
import math
from dataclasses import replace

import numpy as np

import ibm_inputs as I
from oracle.ibm_oracle import CFR, OGrid, Oracle


def _open_case(**kw):
    base = dict(nx=16, ny=9, nz=8, lx=4 * math.pi, lz=2 * math.pi, y_lo=0.0, y_hi=1.0, nu=1 / 300.0, dt=0.01,
                forcing=CFR, q_target_or_pi=2 * math.pi * 0.95, seed=7, geometry="wavy_open",
                geo_params=(0.05, 0.5), top=1)
    base.update(kw)
    return I.Case(**base)


def test_open_channel_is_half_of_mirrored_closed_channel():
    co = _open_case()
    n = co.ny - 1
    H = co.y_hi
    cc = replace(co, ny=2 * n + 1, y_hi=2 * H - co.y_lo, top=0, q_target_or_pi=2 * co.q_target_or_pi)
    eps, alpha = co.geo_params

    def s_open(X, Y):
        yw = eps * (1.0 + np.cos(alpha * X))
        dyw = -eps * alpha * np.sin(alpha * X)
        return (Y - yw) / np.sqrt(1.0 + dyw * dyw)

    sdf_o = I.make_sdf(co)
    sdf_c = I._sample(cc, lambda X, Y, Z: np.minimum(s_open(X, Y), s_open(X, 2 * H - Y)))
    u0, v0, w0 = I.make_initial(co, sdf_o)
    uc = np.concatenate([u0, u0[::-1]])
    wc = np.concatenate([w0, w0[::-1]])
    vc = np.concatenate([v0, np.zeros_like(v0[:1]), -v0[1:][::-1]])
    oo = Oracle(OGrid.from_case(co))
    oo.set_geometry(*sdf_o)
    oo.set_state(u0, v0, w0, np.zeros_like(u0))
    oc = Oracle(OGrid.from_case(cc))
    oc.set_geometry(*sdf_c)
    oc.set_state(uc, vc, wc, np.zeros_like(uc))
    assert oo.lam["u"].max() > 0.0            # the undulated wall is an immersed boundary
    oo.step(3)
    oc.step(3)
    for a, b in ((oc.u[:n], oo.u), (oc.v[:n], oo.v), (oc.w[:n], oo.w), (oc.p[:n], oo.p)):
        assert np.abs(a - b).max() <= 1e-12 * max(np.abs(b).max(), 1e-300)
    # the closed channel stays mirror-symmetric
    assert np.abs(oc.u[n:] - oc.u[:n][::-1]).max() <= 1e-12 * np.abs(oc.u).max()
    assert abs(oc.pi_last - oo.pi_last) <= 1e-12 * abs(oo.pi_last)


def _flat_open(ny=17, off=0.37, nu=0.01, dt=0.05):
    c = _open_case(nx=4, ny=ny, nz=4, nu=nu, dt=dt, geometry="flat_open", geo_params=(off,))
    yw = c.y_lo + off * c.dy
    sdf = I._sample(c, lambda X, Y, Z: Y - yw)
    return c, OGrid.from_case(c), sdf, yw


def test_open_poiseuille_is_fixed_point():
    c, g, sdf, yw = _flat_open()
    H = g.y_hi
    yc = g.y_lo + (np.arange(g.ny - 1) + 0.5) * g.dy
    delta = yc[0] - yw
    prof = (H - yw) ** 2 - (H - yc) ** 2 + delta * (g.dy - delta)
    a = g.q_target_or_pi / (g.lz * prof.sum() * g.dy)
    u = np.broadcast_to((a * prof)[:, None, None], g.shape).copy()
    o = Oracle(g)
    o.set_geometry(*sdf)
    o.set_state(u, np.zeros(g.shape), np.zeros(g.shape), np.zeros(g.shape))
    o.step(3)
    assert np.abs(o.u - u).max() < 1e-13 * np.abs(u).max()
    assert np.abs(o.v).max() < 1e-13 and np.abs(o.w).max() < 1e-13
    assert math.isclose(o.pi_last, -2.0 * g.nu * a, rel_tol=1e-11)


def test_free_slip_face_has_no_lambda():
    c, g, sdf, yw = _flat_open()
    o = Oracle(g)
    o.set_geometry(*sdf)
    assert np.all(o.lam["u"][-1] == 0.0) and np.all(o.lam["w"][-1] == 0.0)
    assert np.all(o.lam["u"][0] > 0.0)
    cw = replace(c, top=0)
    ow = Oracle(OGrid.from_case(cw))
    ow.set_geometry(*sdf)
    assert np.allclose(ow.lam["u"][-1], g.nu / g.dy ** 2, rtol=1e-13)   # no-slip box face
