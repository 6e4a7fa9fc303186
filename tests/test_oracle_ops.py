"""Pins of the oracle's discrete operators against properties the mathematics fixes.

* the convective term in divergence form conserves streamwise and spanwise
  momentum (telescoping fluxes, v = 0 on the walls);
* it conserves kinetic energy exactly for a discretely solenoidal field;
* it approximates (u.grad)u to second order away from the walls (manufactured fields);
* the seven-point Laplacian is second-order accurate;
* the staggered divergence and gradient are negative adjoints (summation by parts);
* a uniform field produces no convective or viscous tendency in a periodic box.
"""
import math

import numpy as np
import pytest

import ibm_inputs as I
from oracle.ibm_oracle import OGrid, convection, divergence, gradient, laplacian


def _case(nx=16, ny=13, nz=10, lx=2.0, lz=1.5, ylo=-1.0, yhi=1.0):
    return I.Case(nx=nx, ny=ny, nz=nz, lx=lx, lz=lz, y_lo=ylo, y_hi=yhi, nu=0.01, dt=0.01)


def _og(c):
    return OGrid.from_case(c)


def test_momentum_conservation():
    c = _case()
    g = _og(c)
    u, v, w = I.random_fields(c, seed=7)
    Nu, Nv, Nw = convection(g, u, v, w)
    assert abs(Nu.sum()) < 1e-12 * np.abs(Nu).sum()
    assert abs(Nw.sum()) < 1e-12 * np.abs(Nw).sum()


@pytest.mark.parametrize("seed", [1, 2])
def test_energy_conservation_solenoidal(seed):
    c = _case(nx=12, ny=11, nz=8)
    g = _og(c)
    u, v, w = I.divergence_free_field(c, seed)
    assert np.abs(divergence(g, u, v, w)).max() < 1e-12 * np.abs(u).max() / g.dx
    Nu, Nv, Nw = convection(g, u, v, w)
    e = (u * Nu).sum() + (v[1:] * Nv[1:]).sum() + (w * Nw).sum()
    scale = np.abs(u * Nu).sum() + np.abs(v * Nv).sum() + np.abs(w * Nw).sum()
    assert abs(e) < 1e-13 * scale, (e, scale)


def _manufactured(c):
    """Smooth field periodic in x, z; returns staggered samples and exact (u.grad)u."""
    g = I.coords(c)
    kx = 2 * math.pi / c.lx
    kz = 2 * math.pi / c.lz

    def U(x, y, z): return np.sin(kx * x) * np.cos(y) * np.cos(kz * z) + 0.3
    def V(x, y, z): return np.cos(kx * x) * np.sin(2 * y) * np.cos(kz * z)
    def W(x, y, z): return np.sin(kx * x + kz * z) * np.cos(0.5 * y)

    def grad(f, x, y, z, e=1e-5):
        return ((f(x + e, y, z) - f(x - e, y, z)) / (2 * e), (f(x, y + e, z) - f(x, y - e, z)) / (2 * e),
                (f(x, y, z + e) - f(x, y, z - e)) / (2 * e))

    def adv(F, x, y, z):
        gx, gy, gz = grad(F, x, y, z)
        return U(x, y, z) * gx + V(x, y, z) * gy + W(x, y, z) * gz

    def mesh(yv, zv, xv):
        Y, Z, X = np.meshgrid(yv, zv, xv, indexing="ij")
        return X, Y, Z
    Xu, Yu, Zu = mesh(g["yc"], g["zc"], g["xf"])
    Xv, Yv, Zv = mesh(g["yf"][:-1], g["zc"], g["xc"])
    Xw, Yw, Zw = mesh(g["yc"], g["zf"], g["xc"])
    fields = (U(Xu, Yu, Zu), V(Xv, Yv, Zv), W(Xw, Yw, Zw))
    exact = (adv(U, Xu, Yu, Zu), adv(V, Xv, Yv, Zv), adv(W, Xw, Yw, Zw))
    # divergence-form equals advective form plus u*div(u)
    def divu(x, y, z):
        return grad(U, x, y, z)[0] + grad(V, x, y, z)[1] + grad(W, x, y, z)[2]
    exact = (exact[0] + U(Xu, Yu, Zu) * divu(Xu, Yu, Zu),
             exact[1] + V(Xv, Yv, Zv) * divu(Xv, Yv, Zv),
             exact[2] + W(Xw, Yw, Zw) * divu(Xw, Yw, Zw))
    return fields, exact


def test_convection_second_order_interior():
    errs = []
    for n in (16, 32, 64):
        c = _case(nx=n, ny=n + 1, nz=n, lx=2.0, lz=2.0, ylo=-1.0, yhi=1.0)
        g = _og(c)
        (u, v, w), ex = _manufactured(c)
        N = convection(g, u, v, w)
        sl = slice(3, -3)
        errs.append(max(np.abs(N[q][sl] - ex[q][sl]).max() for q in range(3)))
    p1 = math.log2(errs[0] / errs[1])
    p2 = math.log2(errs[1] / errs[2])
    assert 1.8 < p1 < 2.3 and 1.8 < p2 < 2.3, errs


def test_laplacian_second_order_interior():
    errs = []
    for n in (16, 32, 64):
        c = _case(nx=n, ny=n + 1, nz=n, lx=2.0, lz=2.0)
        g = _og(c)
        cc = I.coords(c)
        Y, Z, X = np.meshgrid(cc["yc"], cc["zc"], cc["xf"], indexing="ij")
        f = np.sin(math.pi * X) * np.cos(1.3 * Y) * np.cos(math.pi * Z)
        ex = -(2 * math.pi ** 2 + 1.69) * f
        L = laplacian(g, f)
        errs.append(np.abs(L[2:-2] - ex[2:-2]).max())
    assert 1.9 < math.log2(errs[0] / errs[1]) < 2.1
    assert 1.9 < math.log2(errs[1] / errs[2]) < 2.1


def test_summation_by_parts():
    """sum_cells phi * D(u) = - sum_faces u * G(phi), with v = 0 on the box walls."""
    c = _case()
    g = _og(c)
    rng = np.random.default_rng(4)
    u, v, w = I.random_fields(c, seed=9)
    phi = rng.standard_normal(g.shape)
    lhs = (phi * divergence(g, u, v, w)).sum()
    Gx, Gy, Gz = gradient(g, phi)
    rhs = -((u * Gx).sum() + (v[1:] * Gy[1:]).sum() + (w * Gz).sum())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_uniform_field_no_tendency():
    c = _case()
    g = _og(c)
    shp = g.shape
    u = np.full(shp, 0.7)
    w = np.full(shp, -0.2)
    v = np.zeros(shp)
    Nu, Nv, Nw = convection(g, u, v, w)
    assert np.abs(Nu).max() < 1e-13 and np.abs(Nw).max() < 1e-13 and np.abs(Nv).max() < 1e-13
    # away from the y ghost rows the Laplacian of a constant vanishes
    assert np.abs(laplacian(g, u)[1:-1]).max() < 1e-12
