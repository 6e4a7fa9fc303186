"""The same synthetic input recipe as ibm_inputs, generated with torch on a device.

Used for the large ragged ensemble, whose inputs are not compared against the oracle
at full size: the sinusoidal-wall signed distances are the same formulas, the
perturbation is the staggered curl of a smoothed, wall-damped random vector potential
drawn from torch's generator (seeded per instance), faded to zero in the solid.  Data
only: none of the solver's arithmetic is here.
"""
from __future__ import annotations

import math

import torch

from . import Case


def _coords(c: Case, dev):
    f64 = torch.float64
    return {
        "xf": torch.arange(c.nx, device=dev, dtype=f64) * c.dx,
        "xc": (torch.arange(c.nx, device=dev, dtype=f64) + 0.5) * c.dx,
        "zf": torch.arange(c.nz, device=dev, dtype=f64) * c.dz,
        "zc": (torch.arange(c.nz, device=dev, dtype=f64) + 0.5) * c.dz,
        "yf": c.y_lo + torch.arange(c.ny, device=dev, dtype=f64) * c.dy,
        "yc_g": c.y_lo + (torch.arange(-1, c.ny, device=dev, dtype=f64) + 0.5) * c.dy,
        "yc": c.y_lo + (torch.arange(c.ny - 1, device=dev, dtype=f64) + 0.5) * c.dy,
    }


def sdf_wavy(c: Case, amp: float, lam: float, dev, top: float = 1.0):
    """Sinusoidal lower wall y_w = -1 + amp sin(2 pi x/lam), flat top at y = top."""
    g = _coords(c, dev)
    k = 2.0 * math.pi / lam

    def fn(y, z, x):
        Y, Z, X = torch.meshgrid(y, z, x, indexing="ij")
        yw = -1.0 + amp * torch.sin(k * X)
        dyw = amp * k * torch.cos(k * X)
        return torch.minimum((Y - yw) / torch.sqrt(1.0 + dyw * dyw), top - Y).contiguous()
    return (fn(g["yc_g"], g["zc"], g["xf"]), fn(g["yf"], g["zc"], g["xc"]), fn(g["yc_g"], g["zf"], g["xc"]))


def _smooth(a: torch.Tensor, passes: int) -> torch.Tensor:
    for _ in range(passes):
        for ax in (1, 2):
            a = 0.25 * torch.roll(a, 1, dims=ax) + 0.5 * a + 0.25 * torch.roll(a, -1, dims=ax)
        b = 0.5 * a
        b[1:] += 0.25 * a[:-1]
        b[:-1] += 0.25 * a[1:]
        a = b
    return a


def laminar_plus_solenoidal(c: Case, sdfs, seed: int, dev, amp: float = 0.1, ub: float = 1.0,
                            dtype=torch.float32):
    g = _coords(c, dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    ym = 0.5 * (c.y_lo + c.y_hi)
    yh = 0.5 * (c.y_hi - c.y_lo)
    damp_f = (1.0 - ((g["yf"] - ym) / yh) ** 2) ** 2
    damp_c = (1.0 - ((g["yc"] - ym) / yh) ** 2) ** 2
    f64 = torch.float64
    psx = _smooth(torch.randn((c.ny, c.nz, c.nx), generator=gen, device=dev, dtype=f64), 2) * damp_f[:, None, None]
    psy = _smooth(torch.randn((c.ny - 1, c.nz, c.nx), generator=gen, device=dev, dtype=f64), 2) * damp_c[:, None, None]
    psz = _smooth(torch.randn((c.ny, c.nz, c.nx), generator=gen, device=dev, dtype=f64), 2) * damp_f[:, None, None]
    psx[0] = 0.0
    psx[-1] = 0.0
    psz[0] = 0.0
    psz[-1] = 0.0
    dx, dy, dz = c.dx, c.dy, c.dz
    up = (psz[1:] - psz[:-1]) / dy - (torch.roll(psy, -1, dims=1) - psy) / dz
    vp = (torch.roll(psx[:-1], -1, dims=1) - psx[:-1]) / dz - (torch.roll(psz[:-1], -1, dims=2) - psz[:-1]) / dx
    wp = (torch.roll(psy, -1, dims=2) - psy) / dx - (psx[1:] - psx[:-1]) / dy
    m = torch.max(torch.stack([up.abs().max(), vp.abs().max(), wp.abs().max()])).clamp_min(1e-300)
    sc = amp * ub / m
    su, sv, sw = sdfs
    width = 2.0 * c.dy

    def env(s):
        t = (s / width).clamp(0.0, 1.0)
        return t * t * (3.0 - 2.0 * t)
    yc = g["yc"][:, None, None]
    lam = 1.5 * ub * (1.0 - yc * yc).clamp_min(0.0)
    u = (lam + sc * up) * env(su[1:-1])
    v = (sc * vp) * env(sv[:-1])
    w = (sc * wp) * env(sw[1:-1])
    v[0] = 0.0
    p = torch.zeros_like(u)
    return tuple(t.to(dtype).contiguous() for t in (u, v, w, p))


def sdf_ellipsoids(c: Case, n: int, seed: int, dev, a_min: float = 0.05, a_max: float = 0.3):
    """Union of the same seeded ellipsoids as ibm_inputs.sdf_ellipsoids, evaluated on dev."""
    from . import _ellipsoid_params
    centres, semi, R = _ellipsoid_params(c, n, seed, a_min, a_max)
    C = torch.tensor(centres, device=dev)
    S = torch.tensor(semi, device=dev)
    Rt = torch.tensor(R, device=dev)
    g = _coords(c, dev)

    def fn(y, z, x):
        Y = y[:, None, None]
        Z = z[None, :, None]
        X = x[None, None, :]
        out = (1.0 - torch.abs(Y)).expand(y.numel(), z.numel(), x.numel()).clone()
        for e in range(n):
            dxp = X - C[e, 0]
            dxp = dxp - c.lx * torch.round(dxp / c.lx)
            dyp = Y - C[e, 1]
            dzp = Z - C[e, 2]
            dzp = dzp - c.lz * torch.round(dzp / c.lz)
            bx = Rt[e, 0, 0] * dxp + Rt[e, 1, 0] * dyp + Rt[e, 2, 0] * dzp
            by = Rt[e, 0, 1] * dxp + Rt[e, 1, 1] * dyp + Rt[e, 2, 1] * dzp
            bz = Rt[e, 0, 2] * dxp + Rt[e, 1, 2] * dyp + Rt[e, 2, 2] * dzp
            rr = torch.sqrt((bx / S[e, 0]) ** 2 + (by / S[e, 1]) ** 2 + (bz / S[e, 2]) ** 2)
            torch.minimum(out, (rr - 1.0) * S[e].min(), out=out)
        return out.contiguous()
    return (fn(g["yc_g"], g["zc"], g["xf"]), fn(g["yf"], g["zc"], g["xc"]), fn(g["yc_g"], g["zf"], g["xc"]))


def make_inputs(c: Case, dev, dtype=torch.float32):
    """(sdf_u, sdf_v, sdf_w), (u, v, w, p) for a wavy or ellipsoid case, on dev."""
    if c.geometry == "wavy":
        sdf = sdf_wavy(c, c.geo_params[0], c.geo_params[1], dev)
    elif c.geometry == "ellipsoids":
        sdf = sdf_ellipsoids(c, int(c.geo_params[0]), c.seed, dev)
    else:
        raise ValueError(c.geometry)
    return sdf, laminar_plus_solenoidal(c, sdf, c.seed, dev, dtype=dtype)
