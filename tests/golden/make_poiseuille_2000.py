"""Writes poiseuille_32x33x16_2000steps.txt: the FP64 oracle's state after 2000 RK3 steps
(T = 100) of the 32x33x16 plane-Poiseuille workload from its seeded start, reduced to the
x-z mean profile of u and the norms the GPU test compares.

The steady discrete solution it approaches is the closed form of the IBM's steady
balance at the first fluid point (Sec. 2.3, Eqs. (5)-(7) with constraint (ii) of
Sec. 2.4): u_j = a (h_w^2 - y_j^2 + delta (dy - delta)), with a fixed by the flow rate.

Run from the repository root:  python tests/golden/make_poiseuille_2000.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import ibm_inputs as I                               # noqa: E402
from oracle.ibm_oracle import OGrid, Oracle          # noqa: E402

NSTEPS = 2000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "poiseuille_32x33x16_2000steps.txt")


def main():
    c = I.make_case("poiseuille")
    sdf = I.make_sdf(c)
    u0, v0, w0 = I.make_initial(c, sdf)
    o = Oracle(OGrid.from_case(c))
    o.set_geometry(*sdf)
    o.set_state(u0, v0, w0, np.zeros_like(u0))
    o.step(NSTEPS)
    g = o.g
    yc = g.y_lo + (np.arange(g.ny - 1) + 0.5) * g.dy
    hw = 1.0 - c.geo_params[0] * g.dy
    delta = yc[0] + hw
    prof = hw * hw - yc * yc + delta * (g.dy - delta)
    a = g.q_target_or_pi / (g.lz * prof.sum() * g.dy)
    ud = np.broadcast_to((a * prof)[:, None, None], g.shape)
    exact = np.clip(a * (hw * hw - yc * yc), 0.0, None)
    d = o.u - ud
    with open(OUT, "w") as f:
        f.write("# FP64 oracle, 32x33x16 plane Poiseuille (walls 0.37 cells inside the box), CFR, nu=0.01,\n")
        f.write(f"# dt=0.05, {NSTEPS} RK3 steps from the seeded start; written by make_poiseuille_2000.py\n")
        f.write(f"max_abs_u_minus_discrete = {np.abs(d).max():.17e}\n")
        f.write(f"l2_rel_u_minus_discrete = {np.sqrt((d * d).sum() / (ud * ud).sum()):.17e}\n")
        f.write(f"max_abs_v = {np.abs(o.v).max():.17e}\n")
        f.write(f"max_abs_w = {np.abs(o.w).max():.17e}\n")
        f.write(f"pi_last = {o.pi_last:.17e}\n")
        f.write(f"a = {a:.17e}\n")
        f.write(f"max_abs_discrete_minus_exact = {np.abs(a * prof - exact).max():.17e}\n")
        f.write("# j  y_c  mean_xz(u)\n")
        um = o.u.mean(axis=(1, 2))
        for j in range(g.ny - 1):
            f.write(f"{j} {yc[j]:.17e} {um[j]:.17e}\n")


if __name__ == "__main__":
    main()
