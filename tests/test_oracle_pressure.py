"""Pins of the oracle's pressure path inside the RK3 step (reading R2: -c_k dt G p^{k-1} in
the predictor, the increment phi of the projection, p^k = p^{k-1} + phi, u = u* - c_k dt G phi).

Every other pin of the full step runs with p = 0 or checks a property that a wrong pressure
weighting still satisfies; these involve a non-trivial pressure field:

* steady state (Sec. 2.4, constraint (ii)): a steady solution of the scheme must not depend
  on dt or on the form of B.  At a steady state the substep reduces to the discrete steady
  problem  -N(u) + nu L(u) - lambda u - G p - Pi e_x = 0  at internal points with D u = 0,
  which is checked directly with the (separately pinned) operators, and the state reached
  at dt with the exponential B equals the one reached at dt/2 with B = 1;
* substep identity: at internal points without the immersed-boundary correction (A = B = 1)
  the substep is  u^k - u^{k-1} = dt (a_k H_{k-1} + b_k H_{k-2}) - c_k dt (G p^k + Pi_k e_x),
  the Rai-Moin form of Eq. (16) with the pressure of the new stage: p^k is exactly the
  pressure whose gradient the velocity update used;
* temporal order (Sec. 2.4, Sec. 2.5): on a transient three-dimensional flow over the
  sinusoidal wall, started from a state with a consistent pressure, the velocity converges
  at second order in dt (the pressure at first order, as in incremental pressure-correction
  schemes);
* each pin is shown to catch plausible slips planted in a copy of the oracle (dt instead of
  c_k dt, a_k dt instead of c_k dt, p^k = phi, half the increment, no pressure in the
  predictor, dt in the correction).
"""
import dataclasses
import inspect
import math
import sys
import types

import numpy as np
import pytest

import ibm_inputs as I
import oracle.ibm_oracle as OR
from oracle.ibm_oracle import B_EULER, B_EXP, B_TAYLOR2, CFR, RK_A, RK_B, RK_C


# --------------------------------------------------------------------------------------
# cases
# --------------------------------------------------------------------------------------
def _open(ny=9, nx=32, nz=2, nu=0.05, eps=0.1, alpha=1.0, b_mode=B_EXP, dt=None):
    """Open channel over the undulated bottom eps (1 + cos alpha x), free-slip top at 1,
    Re_b = 1/nu, one wavelength in x; dt at 0.8 of the explicit viscous limit."""
    lx, lz = 2 * math.pi / alpha, 0.5
    dy = 1.0 / (ny - 1)
    if dt is None:
        dt = 0.8 * 2.51 / (4 * nu * ((nx / lx) ** 2 + 1 / dy ** 2 + (nz / lz) ** 2))
    return I.Case(nx=nx, ny=ny, nz=nz, lx=lx, lz=lz, y_lo=0.0, y_hi=1.0, nu=nu, dt=dt, forcing=CFR,
                  q_target_or_pi=lz * (1 - eps), b_mode=b_mode, name="open_steady", seed=1,
                  geometry="wavy_open", geo_params=(eps, alpha), top=1)


def _wavy3d(**kw):
    d = dict(nx=32, ny=13, nz=8, lx=2 * math.pi, lz=math.pi, y_lo=-1.2, y_hi=1.0, nu=1 / 200.0, dt=0.01,
             q_target_or_pi=2 * math.pi, seed=11, geometry="wavy", geo_params=(0.15, math.pi / 2),
             name="wavy_transient")
    d.update(kw)
    return I.Case(**d)


# --------------------------------------------------------------------------------------
# the pins, parameterised by the oracle module (so that planted slips can be run through them)
# --------------------------------------------------------------------------------------
def run_to_steady(M, c, state=None, tol=1e-13, maxsteps=4000):
    """Steps of 10 until the largest change of u, v, w over 10 steps is below tol; returns
    the oracle (None if it blew up or did not settle)."""
    o = M.Oracle(M.OGrid.from_case(c))
    sdf = I.make_sdf(c)
    o.set_geometry(*sdf)
    if state is None:
        # the laminar open-channel profile over the bottom (no perturbation)
        u = I.open_channel_profile(c, *c.geo_params) * (sdf[0][1:-1] > 0.0)
        state = (u, np.zeros_like(u), np.zeros_like(u), np.zeros_like(u))
    o.set_state(*state)
    n = 0
    while n < maxsteps:
        prev = (o.u.copy(), o.v.copy(), o.w.copy())
        with np.errstate(all="ignore"):
            o.step(10)
        n += 10
        du = max(np.abs(a - b).max() for a, b in zip((o.u, o.v, o.w), prev))
        if not np.isfinite(du):
            return None
        if du < tol:
            return o
    return None


def steady_residual(o):
    """Relative residual of the discrete steady problem at the state of o: max over the
    internal points of |H - lambda u - G p - Pi e_x| (against the largest of those terms),
    max |D u| over every cell (times the smallest spacing), and max |G p| at the internal u
    faces (the size of the pressure field)."""
    g, t = o.g, o.tags
    Hu, Hv, Hw = OR.explicit_rhs(g, o.u, o.v, o.w, t)
    Gx, Gy, Gz = OR.gradient(g, o.p)
    res, scale = 0.0, 0.0
    for comp, H, f, G, pi in (("u", Hu, o.u, Gx, o.pi_last), ("v", Hv, o.v, Gy, 0.0), ("w", Hw, o.w, Gz, 0.0)):
        m = t[comp]
        if comp == "v":
            m = m.copy()
            m[0] = False
        lam_u = o.lam[comp] * f
        res = max(res, float(np.abs(np.where(m, H - lam_u - G - pi, 0.0)).max()))
        scale = max(scale, float(np.abs(np.where(m, H, 0.0)).max()), float(np.abs(np.where(m, lam_u, 0.0)).max()),
                    float(np.abs(np.where(m, G, 0.0)).max()))
    div = float(np.abs(OR.divergence(g, o.u, o.v, o.w)).max()) * min(g.dx, g.dy, g.dz)
    gp = float(np.abs(np.where(t["u"], Gx, 0.0)).max())
    return res / scale, div, gp


def substep_identity_error(M, c, nsteps_before=3):
    """Largest violation, relative to max(|u|, |dt H|), of
        u^k - u^{k-1} = dt (a_k H(u^{k-1}) + b_k H(u^{k-2})) - c_k dt (G p^k + Pi_k e_x)
    over the internal points without immersed-boundary correction, the three substeps of one
    step taken after nsteps_before steps of the transient wavy flow (H evaluated with the
    oracle's operators on the saved states)."""
    sdf = I.make_sdf(c)
    u0, v0, w0 = I.make_initial(c, sdf)
    o = M.Oracle(M.OGrid.from_case(c))
    o.set_geometry(*sdf)
    o.set_state(u0, v0, w0, np.zeros_like(u0))
    with np.errstate(all="ignore"):
        o.step(nsteps_before)
    g, t = o.g, o.tags
    states = [(o.u.copy(), o.v.copy(), o.w.copy(), o.p.copy())]
    pis = []
    for k in range(3):
        with np.errstate(all="ignore"):
            o.substep(k)
        states.append((o.u.copy(), o.v.copy(), o.w.copy(), o.p.copy()))
        pis.append(o.pi_last)
    H = [OR.explicit_rhs(g, *s[:3], t) for s in states[:3]]
    worst = 0.0
    for k in range(3):
        new, old = states[k + 1], states[k]
        G = OR.gradient(g, new[3])
        for ci, comp in enumerate("uvw"):
            m = t[comp] & (o.lam[comp] == 0.0)
            if comp == "v":
                m = m.copy()
                m[0] = False
            rhs = g.dt * RK_A[k] * H[k][ci] - RK_C[k] * g.dt * (G[ci] + (pis[k] if comp == "u" else 0.0))
            if k > 0:
                rhs = rhs + g.dt * RK_B[k] * H[k - 1][ci]
            scale = max(float(np.abs(new[ci]).max()), float(np.abs(g.dt * H[k][ci] * m).max()))
            e = float(np.abs(np.where(m, (new[ci] - old[ci]) - rhs, 0.0)).max())
            if not np.isfinite(e):
                return math.inf
            worst = max(worst, e / scale)
    return worst


def _consistent_start(c, T_pre=0.2, n_pre=400):
    """The transient wavy flow after T_pre time units at a small dt: a velocity with the
    pressure it has developed (so that the pressure of the first step is not a start-up
    artefact)."""
    cp = dataclasses.replace(c, dt=T_pre / n_pre)
    sdf = I.make_sdf(cp)
    u0, v0, w0 = I.make_initial(cp, sdf)
    o = OR.Oracle(OR.OGrid.from_case(cp))
    o.set_geometry(*sdf)
    o.set_state(u0, v0, w0, np.zeros_like(u0))
    o.step(n_pre)
    return sdf, (o.u.copy(), o.v.copy(), o.w.copy(), o.p.copy())


def _advance(M, c, sdf, st, T, n):
    o = M.Oracle(M.OGrid.from_case(dataclasses.replace(c, dt=T / n)))
    o.set_geometry(*sdf)
    o.set_state(*st)
    o.step(n)
    inside = o.tags["p"]
    return o.u.copy(), o.v.copy(), o.w.copy(), np.where(inside, o.p - o.p[inside].mean(), 0.0)


def planted(old: str, new: str) -> types.ModuleType:
    """A copy of the oracle module with one slip planted in its source."""
    src = inspect.getsource(OR)
    assert src.count(old) == 1, old
    name = f"oracle_planted_{abs(hash(new))}"
    m = types.ModuleType(name)
    sys.modules[name] = m
    exec(compile(src.replace(old, new), name, "exec"), m.__dict__)
    return m


# --------------------------------------------------------------------------------------
# tests
# --------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def steady_exp():
    o = run_to_steady(OR, _open())
    assert o is not None
    return o


def test_steady_state_solves_the_discrete_steady_problem(steady_exp):
    res, div, gp = steady_residual(steady_exp)
    assert gp > 0.1                    # the pressure field is far from trivial
    assert res < 1e-11, res
    assert div < 1e-13, div
    assert math.isclose(steady_exp.flow_rate(steady_exp.u), steady_exp.g.q_target_or_pi, rel_tol=1e-12)


def test_steady_state_independent_of_dt_and_b_form(steady_exp):
    """The steady state reached at dt with the exponential B equals the one reached from the
    same start at dt/2 with B = 1, and is a fixed point of other dt and B forms."""
    c = _open()
    o2 = run_to_steady(OR, dataclasses.replace(c, dt=c.dt / 2, b_mode=B_EULER))
    assert o2 is not None
    inside = steady_exp.tags["p"]

    def pc(p):
        return np.where(inside, p - p[inside].mean(), 0.0)

    sc_u, sc_p = np.abs(steady_exp.u).max(), np.abs(pc(steady_exp.p)).max()
    assert np.abs(o2.u - steady_exp.u).max() < 1e-11 * sc_u
    assert np.abs(o2.v - steady_exp.v).max() < 1e-11 * sc_u
    assert np.abs(pc(o2.p) - pc(steady_exp.p)).max() < 1e-10 * sc_p
    assert math.isclose(o2.pi_last, steady_exp.pi_last, rel_tol=1e-10)
    st = (steady_exp.u, steady_exp.v, steady_exp.w, steady_exp.p)
    for kw in (dict(dt=c.dt / 2), dict(b_mode=B_EULER), dict(dt=0.37 * c.dt, b_mode=B_TAYLOR2)):
        o = OR.Oracle(OR.OGrid.from_case(dataclasses.replace(c, **kw)))
        o.set_geometry(*I.make_sdf(c))
        o.set_state(*st)
        o.step(20)
        assert np.abs(o.u - steady_exp.u).max() < 1e-12 * sc_u, kw
        assert np.abs(pc(o.p) - pc(steady_exp.p)).max() < 1e-12 * sc_p, kw


def test_substep_identity_with_pressure():
    assert substep_identity_error(OR, _wavy3d()) < 1e-13


def test_time_order_three_dimensional_with_pressure():
    """Velocity order 2 in dt on the transient wavy flow (T = 0.4 from a consistent start,
    dt = T/8 .. T/32 against T/512); the pressure converges at first order."""
    c = _wavy3d()
    sdf, st = _consistent_start(c)
    T = 0.4
    ref = _advance(OR, c, sdf, st, T, 512)
    runs = [_advance(OR, c, sdf, st, T, n) for n in (8, 16, 32)]
    # (w, the smallest component of this flow, converges faster than second order)
    for fi, band in ((0, (1.9, 2.2)), (1, (1.9, 2.2)), (2, (1.9, 3.3)), (3, (0.9, 1.2))):
        e = [np.abs(r[fi] - ref[fi]).max() for r in runs]
        orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
        assert all(band[0] < p < band[1] for p in orders), ("uvwp"[fi], orders, e)
    assert np.abs(ref[3]).max() > 0.01


SLIPS = {
    # the predictor's pressure weighted by dt instead of c_k dt
    "predictor_dt": ("r = dt * RK_A[k] * Hc - ck * dt * Gc", "r = dt * RK_A[k] * Hc - dt * Gc"),
    # the predictor's pressure weighted by a_k dt (the weight of the new explicit term)
    "predictor_akdt": ("r = dt * RK_A[k] * Hc - ck * dt * Gc", "r = dt * RK_A[k] * Hc - RK_A[k] * dt * Gc"),
    # no pressure in the predictor (non-incremental projection with an incremental update)
    "predictor_no_p": ("r = dt * RK_A[k] * Hc - ck * dt * Gc", "r = dt * RK_A[k] * Hc"),
    # non-incremental pressure: p^k = phi
    "p_is_phi": ('self.p = np.where(t["p"], self.p + phi, 0.0)', 'self.p = np.where(t["p"], phi, 0.0)'),
    # half the increment
    "half_increment": ('self.p = np.where(t["p"], self.p + phi, 0.0)',
                       'self.p = np.where(t["p"], self.p + 0.5 * phi, 0.0)'),
    # the full-box correction weighted by dt instead of c_k dt
    "correction_dt": ("            un = us - ck * dt * Gx\n            vn = vs - ck * dt * Gy\n            vn[0] = 0.0  ",
                      "            un = us - dt * Gx\n            vn = vs - dt * Gy\n            vn[0] = 0.0  "),
}


@pytest.mark.parametrize("slip", sorted(SLIPS))
def test_pins_catch_planted_slips(slip):
    """Every planted slip of the pressure path fails the steady-state pin or the substep
    identity (both pass on the oracle itself, above)."""
    M = planted(*SLIPS[slip])
    ident = substep_identity_error(M, _wavy3d())
    o = run_to_steady(M, _open(), maxsteps=1500)
    steady_ok = o is not None and steady_residual(o)[0] < 1e-11
    assert not (ident < 1e-13 and steady_ok), (slip, ident)
