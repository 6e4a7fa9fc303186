"""Seeded synthetic inputs for the immersed-boundary channel workloads.

This module produces *data only*: signed-distance samples of the solid
boundary on each staggered component grid, and initial velocity fields.
It contains none of the solver's arithmetic (no classification, no wall
distances, no stencils of the method, no time stepping); both the CPU
oracle and the GPU path consume the arrays it returns, and it imports
neither of them.

Array layout (shared contract, x fastest):
  cell-centred and face fields:  shape (ny-1, nz, nx), index [j, k, i]
  v is stored at the south face j of cell j (j = 0..ny-2); the north box
  wall face j = ny-1 is implicit.
SDF layouts (value > 0 in the fluid):
  sdf_u: (ny+1, nz, nx)  rows j = -1..ny-1 at y_c[j], x = i*dx,      z = (k+1/2)*dz
  sdf_v: (ny,   nz, nx)  rows j =  0..ny-1 at y_f[j], x = (i+1/2)*dx, z = (k+1/2)*dz
  sdf_w: (ny+1, nz, nx)  rows j = -1..ny-1 at y_c[j], x = (i+1/2)*dx, z = k*dz
with y_f[j] = y_lo + j*dy, y_c[j] = y_f[j] + dy/2, dy = (y_hi-y_lo)/(ny-1).

Workloads (synthetic stand-ins for the paper's wavy-bottom channel of
Sec. 4.2 and the complex nasal geometry of Sec. 4.3; no dataset is used):
  poiseuille  32x33x16 plane channel, walls off-grid by 0.37 of a cell
  wavy        sinusoidal lower wall y_w = -1 + A sin(2 pi x / lam)
  ellipsoids  union of seeded ellipsoids inside a plane channel
  ensemble    ragged set of wavy channels
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional, Tuple

import numpy as np

__all__ = [
    "Case", "coords", "sdf_flat_channel", "sdf_wavy", "sdf_ellipsoids",
    "laminar_plus_noise", "laminar_plus_solenoidal", "random_fields",
    "divergence_free_field", "make_case", "WORKLOADS", "ensemble_cases", "tanh_faces", "bottom_tanh_faces",
]


@dataclass(frozen=True)
class Case:
    """Box, grid and physical parameters of one channel instance."""
    nx: int
    ny: int            # wall-normal faces including both box walls (cells = ny-1)
    nz: int
    lx: float
    lz: float
    y_lo: float
    y_hi: float
    nu: float
    dt: float
    forcing: int = 0   # 0 = constant flow rate, 1 = constant pressure gradient
    q_target_or_pi: float = 0.0
    b_mode: int = 0    # 0 = exponential, 1 = implicit Euler (B=1), 2 = Taylor-2
    name: str = ""
    seed: int = 0
    geometry: str = "flat"
    geo_params: Tuple = ()
    top: int = 0       # 0 = no-slip north box face, 1 = free-slip north face (open channel)
    projection: int = 0  # 0 = full-box pressure projection, 1 = masked (internal cells only)
    pcg_max_iter: int = 0  # masked: iteration cap per solve (0 = the library's default)
    pcg_tol: float = 0.0   # masked: relative residual tolerance (0 = the library's default)
    y_faces: Optional[Tuple[float, ...]] = None  # stretched wall-normal grid: the ny face y's

    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dz(self) -> float:
        return self.lz / self.nz

    @property
    def dy(self) -> float:
        return (self.y_hi - self.y_lo) / (self.ny - 1)

    @property
    def cells(self) -> int:
        return self.nx * (self.ny - 1) * self.nz


def coords(c: Case) -> Dict[str, np.ndarray]:
    """Sample positions of the staggered grids (1-D per direction)."""
    dx, dy, dz = c.dx, c.dy, c.dz
    out = {
        "xf": np.arange(c.nx) * dx,
        "xc": (np.arange(c.nx) + 0.5) * dx,
        "zf": np.arange(c.nz) * dz,
        "zc": (np.arange(c.nz) + 0.5) * dz,
        "yf": c.y_lo + np.arange(c.ny) * dy,                  # faces 0..ny-1
        "yc_g": c.y_lo + (np.arange(-1, c.ny) + 0.5) * dy,    # centres -1..ny-1 (with ghosts)
        "yc": c.y_lo + (np.arange(c.ny - 1) + 0.5) * dy,      # centres 0..ny-2
        "dyc": np.full(c.ny - 1, dy),                          # cell heights
    }
    if c.y_faces is not None:
        # stretched: centres midway between faces, ghost centres mirrored in the box faces
        yf = np.asarray(c.y_faces, dtype=np.float64)
        yc = 0.5 * (yf[:-1] + yf[1:])
        out["yf"] = yf
        out["yc"] = yc
        out["yc_g"] = np.concatenate([[2.0 * yf[0] - yc[0]], yc, [2.0 * yf[-1] - yc[-1]]])
        out["dyc"] = np.diff(yf)
    return out


def tanh_faces(ny: int, y_lo: float, y_hi: float, gamma: float) -> Tuple[float, ...]:
    """ny wall-normal faces clustered towards both box walls: y = mid + half
    tanh(gamma xi)/tanh(gamma), xi uniform in [-1, 1] (gamma -> 0: uniform)."""
    xi = np.linspace(-1.0, 1.0, ny)
    t = np.tanh(gamma * xi) / math.tanh(gamma)
    y = 0.5 * (y_lo + y_hi) + 0.5 * (y_hi - y_lo) * t
    y[0], y[-1] = y_lo, y_hi
    return tuple(float(a) for a in y)


def bottom_tanh_faces(ny: int, y_lo: float, y_hi: float, ratio: float) -> Tuple[float, ...]:
    """ny wall-normal faces clustered towards the bottom y_lo only: y = y_hi - (y_hi - y_lo)
    tanh(gamma (1 - xi))/tanh(gamma), xi uniform in [0, 1], with gamma chosen (bisection)
    so that the largest spacing (at the top) is `ratio` times the smallest (at the bottom)."""
    xi = np.linspace(0.0, 1.0, ny)

    def faces(gm):
        y = y_hi - (y_hi - y_lo) * np.tanh(gm * (1.0 - xi)) / math.tanh(gm)
        y[0], y[-1] = y_lo, y_hi
        return y

    def spread(gm):
        d = np.diff(faces(gm))
        return d.max() / d.min()

    lo, hi = 1e-6, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if spread(mid) < ratio:
            lo = mid
        else:
            hi = mid
    return tuple(float(a) for a in faces(0.5 * (lo + hi)))


def _mesh(y, z, x):
    Y, Z, X = np.meshgrid(y, z, x, indexing="ij")
    return X, Y, Z


def _sample(c: Case, fn):
    """Evaluate fn(X, Y, Z) on the u, v and w sample grids."""
    g = coords(c)
    su = fn(*_mesh(g["yc_g"], g["zc"], g["xf"]))
    sv = fn(*_mesh(g["yf"], g["zc"], g["xc"]))
    sw = fn(*_mesh(g["yc_g"], g["zf"], g["xc"]))
    return (np.ascontiguousarray(su, dtype=np.float64),
            np.ascontiguousarray(sv, dtype=np.float64),
            np.ascontiguousarray(sw, dtype=np.float64))


def sdf_flat_channel(c: Case, wall_offset_cells: float):
    """Plane channel with walls at y = +-(1 - off*dy): s = (1 - off*dy) - |y|."""
    hw = 1.0 - wall_offset_cells * c.dy
    return _sample(c, lambda X, Y, Z: hw - np.abs(Y))


def sdf_wavy(c: Case, amp: float, lam: float, top: float = 1.0):
    """Sinusoidal lower wall y_w(x) = -1 + amp sin(2 pi x/lam), flat top wall at y = top.

    Lower-wall distance uses the first-order normal-distance estimate
    (y - y_w)/sqrt(1 + y_w'^2); the zero set is exact.
    """
    k = 2.0 * math.pi / lam

    def fn(X, Y, Z):
        yw = -1.0 + amp * np.sin(k * X)
        dyw = amp * k * np.cos(k * X)
        return np.minimum((Y - yw) / np.sqrt(1.0 + dyw * dyw), top - Y)
    return _sample(c, fn)


def wavy_open_wall(x, eps: float, alpha: float):
    """Undulated bottom y_w(x) = eps (1 + cos(alpha x)) of the open channel, and its slope."""
    return eps * (1.0 + np.cos(alpha * x)), -eps * alpha * np.sin(alpha * x)


def sdf_wavy_open(c: Case, eps: float, alpha: float):
    """Open channel over the undulated bottom y_w(x) = eps (1 + cos alpha x): only the bottom
    is a wall (the north box face is free-slip), s = (y - y_w)/sqrt(1 + y_w'^2)."""
    def fn(X, Y, Z):
        yw, dyw = wavy_open_wall(X, eps, alpha)
        return (Y - yw) / np.sqrt(1.0 + dyw * dyw)
    return _sample(c, fn)


def _ellipsoid_params(c: Case, n: int, seed: int, a_min: float, a_max: float):
    rng = np.random.default_rng(seed)
    centres = np.stack([rng.uniform(0.0, c.lx, n),
                        rng.uniform(-1.0, 1.0, n),
                        rng.uniform(0.0, c.lz, n)], axis=1)
    semi = rng.uniform(a_min, a_max, size=(n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    # rotation matrices of unit quaternions (body -> world)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - z * w); R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w); R[:, 2, 1] = 2 * (y * z + x * w); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return centres, semi, R


def sdf_ellipsoids(c: Case, n: int = 64, seed: int = 4, a_min: float = 0.05, a_max: float = 0.3):
    """Union of n seeded ellipsoids in the plane channel y in [-1, 1].

    s = min(min_e s_e, 1 - |y|), s_e = (|R^T (q - c)/r| - 1) * min(r), with
    minimum-image displacements in the periodic x and z directions.
    """
    centres, semi, R = _ellipsoid_params(c, n, seed, a_min, a_max)

    def fn(X, Y, Z):
        out = 1.0 - np.abs(Y)
        for e in range(n):
            dxp = X - centres[e, 0]
            dxp -= c.lx * np.round(dxp / c.lx)
            dyp = Y - centres[e, 1]
            dzp = Z - centres[e, 2]
            dzp -= c.lz * np.round(dzp / c.lz)
            # body-frame coordinates: R^T d
            bx = R[e, 0, 0] * dxp + R[e, 1, 0] * dyp + R[e, 2, 0] * dzp
            by = R[e, 0, 1] * dxp + R[e, 1, 1] * dyp + R[e, 2, 1] * dzp
            bz = R[e, 0, 2] * dxp + R[e, 1, 2] * dyp + R[e, 2, 2] * dzp
            rr = np.sqrt((bx / semi[e, 0]) ** 2 + (by / semi[e, 1]) ** 2 + (bz / semi[e, 2]) ** 2)
            np.minimum(out, (rr - 1.0) * semi[e].min(), out=out)
        return out
    # evaluate plane by plane to bound memory
    g = coords(c)
    outs = []
    for (yy, zz, xx) in ((g["yc_g"], g["zc"], g["xf"]), (g["yf"], g["zc"], g["xc"]),
                         (g["yc_g"], g["zf"], g["xc"])):
        arr = np.empty((yy.size, zz.size, xx.size))
        for j in range(yy.size):
            X, Y, Z = _mesh(yy[j:j + 1], zz, xx)
            arr[j] = fn(X, Y, Z)[0]
        outs.append(arr)
    return tuple(outs)


def random_fields(c: Case, seed: int, amp: float = 1.0):
    """i.i.d. uniform noise in [-amp, amp] on u, v, w (v = 0 on the south box wall)."""
    rng = np.random.default_rng(seed)
    shp = (c.ny - 1, c.nz, c.nx)
    u = rng.uniform(-amp, amp, shp)
    v = rng.uniform(-amp, amp, shp)
    w = rng.uniform(-amp, amp, shp)
    v[0] = 0.0
    return u, v, w


def _smooth(a: np.ndarray, passes: int, axes=(1, 2)) -> np.ndarray:
    for _ in range(passes):
        for ax in axes:
            a = 0.25 * np.roll(a, 1, axis=ax) + 0.5 * a + 0.25 * np.roll(a, -1, axis=ax)
        # y: zero beyond the ends
        b = 0.5 * a
        b[1:] += 0.25 * a[:-1]
        b[:-1] += 0.25 * a[1:]
        a = b
    return a


def divergence_free_field(c: Case, seed: int, smooth_passes: int = 2):
    """Staggered-grid curl of a seeded, smoothed, wall-damped random vector potential.

    The potential lives on cell edges; its curl is discretely solenoidal with
    v = 0 on both box walls (psi_x = psi_z = 0 on the wall faces).
    """
    rng = np.random.default_rng(seed)
    ny1 = c.ny - 1
    g = coords(c)
    damp_f = ((1.0 - ((g["yf"] - 0.5 * (c.y_lo + c.y_hi)) / (0.5 * (c.y_hi - c.y_lo))) ** 2) ** 2)
    damp_c = ((1.0 - ((g["yc"] - 0.5 * (c.y_lo + c.y_hi)) / (0.5 * (c.y_hi - c.y_lo))) ** 2) ** 2)
    psx = _smooth(rng.standard_normal((c.ny, c.nz, c.nx)), smooth_passes) * damp_f[:, None, None]
    psy = _smooth(rng.standard_normal((ny1, c.nz, c.nx)), smooth_passes) * damp_c[:, None, None]
    psz = _smooth(rng.standard_normal((c.ny, c.nz, c.nx)), smooth_passes) * damp_f[:, None, None]
    psx[0] = psx[-1] = 0.0
    psz[0] = psz[-1] = 0.0
    dx, dz = c.dx, c.dz
    dy = g["dyc"][:, None, None]
    u = (psz[1:] - psz[:-1]) / dy - (np.roll(psy, -1, axis=1) - psy) / dz
    v = (np.roll(psx[:-1], -1, axis=1) - psx[:-1]) / dz - (np.roll(psz[:-1], -1, axis=2) - psz[:-1]) / dx
    w = (np.roll(psy, -1, axis=2) - psy) / dx - (psx[1:] - psx[:-1]) / dy
    return u, v, w


def _envelope(s: np.ndarray, width: float) -> np.ndarray:
    """Smooth ramp 0 (s <= 0) -> 1 (s >= width); exactly 0 in the solid."""
    t = np.clip(s / width, 0.0, 1.0)
    return t * t * (3.0 - 2.0 * t)


def laminar_plus_noise(c: Case, seed: int, amp: float = 1e-3):
    """Zero field plus i.i.d. U[-amp, amp] noise (v = 0 on the south box wall)."""
    return random_fields(c, seed, amp)


def open_channel_profile(c: Case, eps: float, alpha: float, ub: float = 1.0) -> np.ndarray:
    """Laminar open-channel profile 1.5 ub (2 eta - eta^2), eta = (y - y_w)/(y_hi - y_w),
    on the u grid (zero below the wall): bulk velocity ub over every column."""
    g = coords(c)
    X, Y, _ = _mesh(g["yc"], g["zc"], g["xf"])
    yw, _ = wavy_open_wall(X, eps, alpha)
    eta = np.clip((Y - yw) / (c.y_hi - yw), 0.0, 1.0)
    return 1.5 * ub * (2.0 * eta - eta * eta)


def laminar_plus_solenoidal(c: Case, sdfs, seed: int, amp: float = 0.1, ub: float = 1.0,
                            env_width: Optional[float] = None, profile: Optional[np.ndarray] = None):
    """Laminar 1.5*ub*(1-y^2) streamwise profile (or the given one on the u grid) plus a
    solenoidal perturbation with max |u'| = amp*ub, both faded to zero in the solid by a
    smooth SDF envelope."""
    g = coords(c)
    su, sv, sw = sdfs
    width = env_width if env_width is not None else 2.0 * c.dy
    eu = _envelope(su[1:-1], width)
    ev = _envelope(sv[:-1], width)
    ew = _envelope(sw[1:-1], width)
    up, vp, wp = divergence_free_field(c, seed)
    m = max(np.abs(up).max(), np.abs(vp).max(), np.abs(wp).max(), 1e-300)
    sc = amp * ub / m
    yc = g["yc"][:, None, None]
    lam = 1.5 * ub * np.clip(1.0 - yc * yc, 0.0, None) if profile is None else profile
    u = (lam + sc * up) * eu
    v = (sc * vp) * ev
    w = (sc * wp) * ew
    v[0] = 0.0
    return (np.ascontiguousarray(u), np.ascontiguousarray(v), np.ascontiguousarray(w))


# --------------------------------------------------------------------------------------
# Workload catalogue
# --------------------------------------------------------------------------------------
WORKLOADS: Dict[str, Case] = {
    # Plane Poiseuille between off-grid walls (0.37 of a cell inside the box walls)
    "poiseuille": Case(nx=32, ny=33, nz=16, lx=2 * math.pi, lz=math.pi, y_lo=-1.0, y_hi=1.0,
                       nu=0.01, dt=0.05, forcing=0, q_target_or_pi=2.0 * math.pi,
                       name="poiseuille_32x33x16", seed=1, geometry="flat", geo_params=(0.37,)),
    # Sinusoidal lower wall, FP64, 192x129x96
    "wavy": Case(nx=192, ny=129, nz=96, lx=2 * math.pi, lz=math.pi, y_lo=-1.2, y_hi=1.0,
                 nu=1.0 / 2800.0, dt=0.008, forcing=0, q_target_or_pi=2.0 * math.pi,
                 name="wavy_192x129x96", seed=2, geometry="wavy", geo_params=(0.1, math.pi / 2)),
    # Same wall at 512x257x256
    "wavy_large": Case(nx=512, ny=257, nz=256, lx=2 * math.pi, lz=math.pi, y_lo=-1.2, y_hi=1.0,
                       nu=1.0 / 2800.0, dt=0.003, forcing=0, q_target_or_pi=2.0 * math.pi,
                       name="wavy_512x257x256", seed=3, geometry="wavy", geo_params=(0.1, math.pi / 2)),
    # Open channel over an undulated bottom y_w = eps (1 + cos alpha x), eps = 0.05,
    # alpha = 1/2 (Lx = 4 pi), spanwise 2 pi, free-slip at y = 1, Re_b = 2800: the
    # coarsest grid of the convergence study (192 x 160 x 64, uniform here)
    "wavy_open": Case(nx=192, ny=65, nz=160, lx=4 * math.pi, lz=2 * math.pi, y_lo=0.0, y_hi=1.0,
                      nu=1.0 / 2800.0, dt=0.008, forcing=0, q_target_or_pi=2 * math.pi * 0.95,
                      name="wavy_open_192x65x160", seed=6, geometry="wavy_open", geo_params=(0.05, 0.5),
                      top=1),
    # Union of 64 seeded ellipsoids, 384x193x192
    "ellipsoids": Case(nx=384, ny=193, nz=192, lx=2 * math.pi, lz=math.pi, y_lo=-1.0, y_hi=1.0,
                       nu=1.0 / 1000.0, dt=0.004, forcing=0, q_target_or_pi=2.0 * math.pi,
                       name="ellipsoids_384x193x192", seed=4, geometry="ellipsoids", geo_params=(64,)),
}


def make_case(name: str, **over) -> Case:
    return replace(WORKLOADS[name], **over)


def make_sdf(c: Case):
    if c.geometry == "flat":
        return sdf_flat_channel(c, c.geo_params[0])
    if c.geometry == "wavy":
        return sdf_wavy(c, c.geo_params[0], c.geo_params[1])
    if c.geometry == "ellipsoids":
        return sdf_ellipsoids(c, int(c.geo_params[0]), seed=c.seed)
    if c.geometry == "wavy_open":
        return sdf_wavy_open(c, c.geo_params[0], c.geo_params[1])
    raise ValueError(c.geometry)


def make_initial(c: Case, sdfs):
    if c.geometry == "flat":
        return laminar_plus_noise(c, c.seed, 1e-3)
    if c.geometry == "wavy_open":
        prof = open_channel_profile(c, c.geo_params[0], c.geo_params[1])
        return laminar_plus_solenoidal(c, sdfs, c.seed, amp=0.1, profile=prof)
    return laminar_plus_solenoidal(c, sdfs, c.seed, amp=0.1)


def ensemble_cases(n: int = 96, seed: int = 5) -> List[Case]:
    """Ragged ensemble of wavy channels drawn from one seed."""
    rng = np.random.default_rng(seed)
    out = []
    for e in range(n):
        nx = int(rng.choice([64, 96, 128, 160]))
        nz = int(rng.choice([64, 96, 128, 160]))
        ny = int(rng.choice([65, 97, 129]))
        amp = float(rng.uniform(0.0, 0.15))
        lam = float(rng.uniform(math.pi / 4, math.pi))
        re = float(rng.uniform(500.0, 3000.0))
        m = max(1, int(round(2 * math.pi / lam)))
        lx = m * lam
        lz = math.pi
        dy = 2.2 / (ny - 1)
        dt = 0.3 * min(lx / nx, dy, lz / nz) / 1.5
        out.append(Case(nx=nx, ny=ny, nz=nz, lx=lx, lz=lz, y_lo=-1.2, y_hi=1.0, nu=1.0 / re, dt=dt,
                        forcing=0, q_target_or_pi=2.0 * lz, name=f"ens{e}", seed=seed * 1000 + e,
                        geometry="wavy", geo_params=(amp, lam)))
    return out
