"""FP64 CPU oracle: one explicit RK3 time step of the implicit, second-order,
discrete-forcing immersed-boundary method on a staggered Cartesian grid,
followed by an FFT / tridiagonal pressure projection.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  It shares no code
with the GPU library and never calls it.

Every function cites the passage of the paper (arXiv 2506.14328) it follows.
Where the paper is silent the reading taken is stated in the docstring
(readings R1..R20; the same list is kept with the design notes).

Conventions
-----------
x streamwise (periodic), y wall-normal (bounded by the box walls y_lo, y_hi),
z spanwise (periodic).  Arrays are indexed [j, k, i] (x fastest):
  p   cell centres          (x_c[i], y_c[j], z_c[k])       shape (ny-1, nz, nx)
  u   west faces            (i*dx,   y_c[j], z_c[k])
  v   south faces           (x_c[i], y_f[j], z_c[k])       (face j = ny-1 is the north
                                                             box wall: implicit zero)
  w   back faces            (x_c[i], y_c[j], k*dz)
Ghost rows of u and w at j = -1 and j = ny-1 lie outside the box; they are
external (value 0) and only carry SDF samples, except that with a free-slip north
face (top = 1, the open channel of Sec. 4.2) the ghost row j = ny-1 mirrors the top
row of u and w (du/dy = dw/dy = 0 on the face) and that face is not a wall for lambda
(reading R16).
Pi is the mean streamwise pressure gradient, entering the u-momentum
equation as -Pi (the paper's notation in Sec. 2.5, Eq. (18)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, Optional, Tuple

import numpy as np
import scipy.fft

# Rai & Moin RK3 coefficients (Sec. 2.4, Eq. (17)): c_k = a_k + b_k.
RK_A = np.array([64.0, 50.0, 90.0]) / 120.0
RK_B = np.array([0.0, -34.0, -50.0]) / 120.0
RK_C = RK_A + RK_B

CFR, CPG = 0, 1
B_EXP, B_EULER, B_TAYLOR2 = 0, 1, 2


@dataclass
class OGrid:
    nx: int
    ny: int
    nz: int
    lx: float
    lz: float
    y_lo: float
    y_hi: float
    nu: float
    dt: float
    forcing: int = CFR
    q_target_or_pi: float = 0.0
    b_mode: int = B_EXP
    top: int = 0          # 0: no-slip north box face; 1: free-slip north face
    projection: int = 0   # 0: full-box projection (reading R6); 1: masked (reading R18)
    # y of the ny v faces (increasing, first y_lo, last y_hi) for a stretched wall-normal
    # grid (Sec. 2.1: non-uniform spacing; reading R20); None: uniform spacing dy
    y_faces: Optional[np.ndarray] = field(default=None, repr=False, compare=False)

    @property
    def stretched(self) -> bool:
        return self.y_faces is not None

    @property
    def yf(self) -> np.ndarray:
        """y of the v faces 0..ny-1 (faces 0 and ny-1 are the box walls)."""
        if self.y_faces is None:
            return self.y_lo + np.arange(self.ny) * self.dy
        return np.asarray(self.y_faces, dtype=np.float64)

    @property
    def yc(self) -> np.ndarray:
        """y of the cell centres (rows of u, w, p), midway between their faces."""
        f = self.yf
        return 0.5 * (f[:-1] + f[1:])

    @property
    def dyc(self) -> np.ndarray:
        """Cell heights y_f[j+1] - y_f[j], rows 0..ny-2 (dy on a uniform grid)."""
        if self.y_faces is None:
            return np.full(self.ny - 1, self.dy)
        return np.diff(self.yf)

    @property
    def hy_lo(self) -> np.ndarray:
        """Distance from centre row j to the row below; the ghost row -1 is the mirror
        image of row 0 in the south box wall (distance dyc[0])."""
        if self.y_faces is None:
            return np.full(self.ny - 1, self.dy)
        out = np.empty(self.ny - 1)
        out[0] = self.dyc[0]
        out[1:] = np.diff(self.yc)
        return out

    @property
    def hy_hi(self) -> np.ndarray:
        """Distance from centre row j to the row above; the ghost row ny-1 is the mirror
        image of the top row in the north face (distance dyc[-1])."""
        if self.y_faces is None:
            return np.full(self.ny - 1, self.dy)
        out = np.empty(self.ny - 1)
        out[-1] = self.dyc[-1]
        out[:-1] = np.diff(self.yc)
        return out

    def face_weights(self) -> Tuple[np.ndarray, np.ndarray]:
        """Linear-interpolation weights of centre rows j-1 and j at face j (rows 0..ny-2;
        at face 0 the ghost row is the mirror image, weights 1/2): (w_lo, w_hi)."""
        d = self.dyc
        dm = np.empty_like(d)
        dm[0] = d[0]
        dm[1:] = d[:-1]
        return d / (dm + d), dm / (dm + d)

    @property
    def dx(self):
        return self.lx / self.nx

    @property
    def dz(self):
        return self.lz / self.nz

    @property
    def dy(self):
        return (self.y_hi - self.y_lo) / (self.ny - 1)

    @property
    def shape(self):
        return (self.ny - 1, self.nz, self.nx)

    @classmethod
    def from_case(cls, c) -> "OGrid":
        yfs = getattr(c, "y_faces", None)
        return cls(c.nx, c.ny, c.nz, c.lx, c.lz, c.y_lo, c.y_hi, c.nu, c.dt,
                   c.forcing, c.q_target_or_pi, c.b_mode, int(getattr(c, "top", 0)),
                   int(getattr(c, "projection", 0)),
                   None if yfs is None else np.asarray(yfs, dtype=np.float64))


def col(a: np.ndarray) -> np.ndarray:
    """A per-row array shaped to broadcast over (row, k, i)."""
    return np.asarray(a)[:, None, None]


def second_derivative_weights(hm, hp):
    """Coefficients d2(-1), d2(+1) of the three-point second derivative with spacings hm
    below and hp above (Eq. (3); d2(0) = -(d2(-1) + d2(+1))); 1/h^2 on a uniform grid."""
    return 2.0 / (hm * (hm + hp)), 2.0 / (hp * (hm + hp))


def y_spacings(g: "OGrid", comp: str) -> Tuple[np.ndarray, np.ndarray]:
    """Spacings (below, above) of the wall-normal stencil of each stored row of a
    component: centre rows for u, w (mirror ghosts at the box faces), face spacings for v
    (face j lies between cells j-1 and j)."""
    if comp in ("u", "w"):
        return g.hy_lo, g.hy_hi
    d = g.dyc
    lo = np.empty_like(d)
    lo[0] = d[0]
    lo[1:] = d[:-1]
    return lo, d


# --------------------------------------------------------------------------------------
# Neighbour access on the staggered arrays (periodic x, z; zero beyond the y rows).
# --------------------------------------------------------------------------------------
def sx(f, d):
    """f at i+d (periodic in x)."""
    return np.roll(f, -d, axis=2)


def sz(f, d):
    """f at k+d (periodic in z)."""
    return np.roll(f, -d, axis=1)


def sy(f, d):
    """f at j+d, zero outside the stored rows (ghost rows / north wall are zero)."""
    out = np.zeros_like(f)
    if d > 0:
        out[:-d] = f[d:]
    elif d < 0:
        out[-d:] = f[:d]
    else:
        out[:] = f
    return out


# --------------------------------------------------------------------------------------
# Geometry: staircase classification and wall distances (Sec. 2.2, Sec. 3.3)
# --------------------------------------------------------------------------------------
def classify(g: OGrid, sdf_u, sdf_v, sdf_w) -> Dict[str, np.ndarray]:
    """Internal/external tags per component grid and for pressure (Sec. 3.3).

    Each velocity grid is compared with the boundary on its own: a point is
    internal iff its signed distance is > 0 (reading R7: s <= 0 is solid).
    v on the two box-wall faces is always external.  A pressure cell is
    internal iff at least one of its six faces is an internal velocity point.
    """
    int_u = sdf_u[1:-1] > 0.0
    int_v = sdf_v[:-1] > 0.0
    int_v[0] = False
    int_w = sdf_w[1:-1] > 0.0
    int_p = (int_u | sx(int_u, 1) | int_v | sy(int_v, 1) | int_w | sz(int_w, 1))
    return {"u": int_u, "v": int_v, "w": int_w, "p": int_p}


def _arm_lambda(nu, h, sP, sQ, extQ, box_dist, d2=None):
    """Contribution nu * d2 (h - delta)/delta of one stencil arm of length h (Eq. (7)).

    delta is the distance from the internal point to the wall along the arm:
    the linear zero crossing of the signed distance between the point and its
    external neighbour (reading R8), or the box wall when that is nearer.
    d2 is the arm's coefficient of the three-point second derivative (Eq. (3)):
    1/h^2 on a uniform spacing (d2 = None), second_derivative_weights otherwise.
    """
    with np.errstate(divide="ignore", invalid="ignore"):
        d_sdf = np.where(sQ <= 0.0, h * sP / (sP - sQ), np.inf)
    delta = np.minimum(d_sdf, box_dist)
    with np.errstate(divide="ignore", invalid="ignore"):
        if d2 is None:
            contrib = np.where(extQ, nu * (h - delta) / (delta * h * h), 0.0)
        else:
            contrib = np.where(extQ, nu * d2 * (h - delta) / delta, 0.0)
    return contrib


def _y_arms(g: OGrid, comp, s_dn, ext_dn, box_dn, s_up, ext_up, box_up):
    """The two wall-normal stencil arms (length, neighbour SDF, external flag, box-wall
    distance, second-derivative coefficient or None for uniform spacing)."""
    if not g.stretched:
        return ((g.dy, s_dn, ext_dn, box_dn, None), (g.dy, s_up, ext_up, box_up, None))
    lo, hi = y_spacings(g, comp)
    d2lo, d2hi = second_derivative_weights(lo, hi)
    return ((col(lo), s_dn, ext_dn, box_dn, col(d2lo)), (col(hi), s_up, ext_up, box_up, col(d2hi)))


def wall_lambda(g: OGrid, sdf_full: np.ndarray, comp: str, internal: np.ndarray) -> np.ndarray:
    """IBM centre-weight correction lambda per point of one component grid.

    Sec. 2.2, Eqs. (5)-(7): the ghost value is the linear extrapolation
    through zero at the wall; substituted into the Laplacian it only changes
    the centre coefficient by lambda = d2(-1) (h - delta)/delta.  The viscous
    factor nu multiplies it (reading R9).  Corrections from different arms
    add up independently (end of Sec. 2.2).
    """
    nu = g.nu
    if comp in ("u", "w"):
        s = sdf_full[1:-1]
        s_dn = sdf_full[:-2]          # row j-1 (ghost row -1 for j = 0)
        s_up = sdf_full[2:]           # row j+1 (ghost row ny-1 for j = ny-2)
        nrow = s.shape[0]
        ext_dn = s_dn <= 0.0
        ext_up = s_up <= 0.0
        ext_dn[0] = True              # ghost rows are outside the box
        box_dn = np.full(s.shape, np.inf)
        box_up = np.full(s.shape, np.inf)
        box_dn[0] = 0.5 * g.dyc[0]    # u, w of row 0 sit half a cell above the south box wall
        if g.top == 0:                # a north box wall half a cell above the top row
            ext_up[-1] = True
            box_up[-1] = 0.5 * g.dyc[-1]
    else:  # v: faces 0..ny-1 are all stored in sdf_full; face 0 and ny-1 are box walls
        s = sdf_full[:-1]
        s_dn = np.zeros_like(s)
        s_dn[1:] = sdf_full[:-2]
        s_up = sdf_full[1:]
        ext_dn = s_dn <= 0.0
        ext_up = s_up <= 0.0
        ext_dn[1] = True              # neighbour face 0 is the south box wall
        ext_up[-1] = True             # neighbour face ny-1 is the north box wall
        box_dn = np.full(s.shape, np.inf)
        box_up = np.full(s.shape, np.inf)
        box_dn[1] = g.dyc[0]
        box_up[-1] = g.dyc[-1]
    lam = np.zeros(s.shape)
    for h, sQ, extQ, bd, d2 in (
        (g.dx, sx(s, -1), sx(s, -1) <= 0.0, np.inf, None),
        (g.dx, sx(s, +1), sx(s, +1) <= 0.0, np.inf, None),
        (g.dz, sz(s, -1), sz(s, -1) <= 0.0, np.inf, None),
        (g.dz, sz(s, +1), sz(s, +1) <= 0.0, np.inf, None),
    ) + _y_arms(g, comp, s_dn, ext_dn, box_dn, s_up, ext_up, box_up):
        lam += _arm_lambda(nu, h, s, sQ, extQ, bd, d2)
    lam = np.where(internal, lam, 0.0)
    return lam


def wall_source(g: OGrid, sdf_full: np.ndarray, comp: str, internal: np.ndarray) -> np.ndarray:
    """Coefficient sigma of the wall velocity U_b in the immersed-boundary term of a
    rigidly moving wall (reading R19): the IBM term of a point becomes
    -lambda u_P + sigma U_b.

    With the ghost value the linear extrapolation through U_b at the wall (Sec. 2.2,
    Eqs. (5)-(7) with a moving wall), u_G = U_b h/delta - u_P (h - delta)/delta, and the
    plain stencil using the stored value of the external neighbour, the difference per
    arm whose wall is the immersed one (the signed-distance crossing nearer than any box
    wall) is lambda_arm (U_b - u_P) when that neighbour stores U_b (an external point
    inside the box), and nu U_b/(delta h) - lambda_arm u_P when it stores zero (the box
    wall face or the ghost row beyond it).  Arms ending on a box wall (at rest) add
    nothing.  Zero at points that are not internal.
    """
    nu = g.nu
    if comp in ("u", "w"):
        s = sdf_full[1:-1]
        s_dn = sdf_full[:-2]
        s_up = sdf_full[2:]
        ext_dn = s_dn <= 0.0
        ext_up = s_up <= 0.0
        ext_dn[0] = True
        box_dn = np.full(s.shape, np.inf)
        box_up = np.full(s.shape, np.inf)
        box_dn[0] = 0.5 * g.dyc[0]
        if g.top == 0:
            ext_up[-1] = True
            box_up[-1] = 0.5 * g.dyc[-1]
    else:
        s = sdf_full[:-1]
        s_dn = np.zeros_like(s)
        s_dn[1:] = sdf_full[:-2]
        s_up = sdf_full[1:]
        ext_dn = s_dn <= 0.0
        ext_up = s_up <= 0.0
        ext_dn[1] = True
        ext_up[-1] = True
        box_dn = np.full(s.shape, np.inf)
        box_up = np.full(s.shape, np.inf)
        box_dn[1] = g.dyc[0]
        box_up[-1] = g.dyc[-1]
    sig = np.zeros(s.shape)
    with np.errstate(divide="ignore", invalid="ignore"):
        for h, sQ, extQ, bd, d2 in (
            (g.dx, sx(s, -1), sx(s, -1) <= 0.0, np.inf, None),
            (g.dx, sx(s, +1), sx(s, +1) <= 0.0, np.inf, None),
            (g.dz, sz(s, -1), sz(s, -1) <= 0.0, np.inf, None),
            (g.dz, sz(s, +1), sz(s, +1) <= 0.0, np.inf, None),
        ) + _y_arms(g, comp, s_dn, ext_dn, box_dn, s_up, ext_up, box_up):
            d_sdf = np.where(sQ <= 0.0, h * s / (s - sQ), np.inf)
            immersed = extQ & (d_sdf < bd)
            stores_zero = np.isfinite(bd)
            if d2 is None:
                arm = np.where(stores_zero, nu / (d_sdf * h), nu * (h - d_sdf) / (d_sdf * h * h))
            else:
                arm = np.where(stores_zero, nu * d2 * h / d_sdf, nu * d2 * (h - d_sdf) / d_sdf)
            sig += np.where(immersed, arm, 0.0)
    return np.where(internal, sig, 0.0)


def stage_coefficients(lam: np.ndarray, k: int, dt: float, b_mode: int = B_EXP):
    """(B, A) of the implicit IBM update for RK stage k (Sec. 2.4, Eqs. (14)-(16)).

    With x = lambda c_k dt (reading R5):
      exponential fit  B = x/(e^x - 1),  A = x + B  (B = 1 at x = 0, B = 0 for huge x)
      implicit Euler   B = 1,            A = 1 + x
      Taylor-2         B = 1/(1 + x/2),  A = x + B   (reciprocal of the Taylor
                                                       expansion of 1/B, Sec. 2.4)
    """
    x = lam * RK_C[k] * dt
    if b_mode == B_EXP:
        with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
            B = np.where(x > 0.0, x / np.expm1(np.minimum(x, 700.0)), 1.0)
        B = np.where(x > 700.0, 0.0, B)
        A = x + B
    elif b_mode == B_EULER:
        B = np.ones_like(x)
        A = 1.0 + x
    elif b_mode == B_TAYLOR2:
        B = 1.0 / (1.0 + 0.5 * x)
        A = x + B
    else:
        raise ValueError(b_mode)
    return B, A


# --------------------------------------------------------------------------------------
# Discrete operators (Sec. 2.1: second-order central differences on the staggered grid)
# --------------------------------------------------------------------------------------
def convection(g: OGrid, u, v, w):
    """Convective terms N(u) in divergence form with two-point averages (reading R1).

    No IBM correction of the convective terms: external and ghost values enter
    as zero (Sec. 3.1 and the opening of Sec. 2).
    """
    dx, dz = g.dx, g.dz
    h = 0.5
    # wall-normal: differences over the cell height (u, w rows) or the centre spacing
    # (v faces); u and w reach a face by linear interpolation between the rows (midpoint
    # averages on a uniform grid; reading R20)
    dy_c = col(g.dyc)
    dy_f = col(g.hy_lo)
    wl, wh = (col(a) for a in g.face_weights())
    wl_p, wh_p = sy(wl, 1), sy(wh, 1)     # weights at face j+1
    if not g.stretched:
        wl = wh = wl_p = wh_p = h
    # u-momentum at (i*dx, y_c[j], z_c[k])
    Nu = ((h * (u + sx(u, 1))) ** 2 - (h * (sx(u, -1) + u)) ** 2) / dx
    Nu += ((wl_p * u + wh_p * sy(u, 1)) * h * (sx(sy(v, 1), -1) + sy(v, 1))
           - (wl * sy(u, -1) + wh * u) * h * (sx(v, -1) + v)) / dy_c
    Nu += (h * (u + sz(u, 1)) * h * (sx(sz(w, 1), -1) + sz(w, 1))
           - h * (sz(u, -1) + u) * h * (sx(w, -1) + w)) / dz
    # v-momentum at (x_c[i], y_f[j], z_c[k])
    Nv = (h * (v + sx(v, 1)) * (wl * sx(sy(u, -1), 1) + wh * sx(u, 1))
          - h * (sx(v, -1) + v) * (wl * sy(u, -1) + wh * u)) / dx
    Nv += ((h * (v + sy(v, 1))) ** 2 - (h * (sy(v, -1) + v)) ** 2) / dy_f
    Nv += (h * (v + sz(v, 1)) * (wl * sz(sy(w, -1), 1) + wh * sz(w, 1))
           - h * (sz(v, -1) + v) * (wl * sy(w, -1) + wh * w)) / dz
    # w-momentum at (x_c[i], y_c[j], k*dz)
    Nw = (h * (w + sx(w, 1)) * h * (sx(sz(u, -1), 1) + sx(u, 1))
          - h * (sx(w, -1) + w) * h * (sz(u, -1) + u)) / dx
    Nw += ((wl_p * w + wh_p * sy(w, 1)) * h * (sz(sy(v, 1), -1) + sy(v, 1))
           - (wl * sy(w, -1) + wh * w) * h * (sz(v, -1) + v)) / dy_c
    Nw += ((h * (w + sz(w, 1))) ** 2 - (h * (sz(w, -1) + w)) ** 2) / dz
    return Nu, Nv, Nw


def laplacian(g: OGrid, f, mirror_top: bool = False, comp: str = "u"):
    """Seven-point Laplacian, Eq. (3), with external/ghost neighbours equal to zero.

    Sec. 2.4: as long as external values are zero and the right-hand side is
    explicit, the unmodified Laplacian is used; the wall enters through lambda.
    mirror_top: the ghost row above the top row equals the top row (free-slip face,
    reading R16).  On a stretched grid the wall-normal part takes the three-point
    coefficients of the row's own spacings (comp selects centre rows or v faces).
    """
    up = sy(f, 1)
    if mirror_top:
        up[-1] = f[-1]
    if g.stretched:
        lo, hi = y_spacings(g, comp)
        dm, dp = (col(a) for a in second_derivative_weights(lo, hi))
        d2y = dm * sy(f, -1) + dp * up - (dm + dp) * f
    else:
        d2y = (up - 2.0 * f + sy(f, -1)) / g.dy ** 2
    return ((sx(f, 1) - 2.0 * f + sx(f, -1)) / g.dx ** 2
            + d2y
            + (sz(f, 1) - 2.0 * f + sz(f, -1)) / g.dz ** 2)


def gradient(g: OGrid, p):
    """G p on the u, v, w faces (row 0 of the v component is the box wall, unused)."""
    return ((p - sx(p, -1)) / g.dx, (p - sy(p, -1)) / col(g.hy_lo), (p - sz(p, -1)) / g.dz)


def divergence(g: OGrid, u, v, w):
    """D u at every cell: forward differences to the cell's faces; v on the north
    box wall face is zero."""
    return (sx(u, 1) - u) / g.dx + (sy(v, 1) - v) / col(g.dyc) + (sz(w, 1) - w) / g.dz


def explicit_rhs(g: OGrid, u, v, w, tags):
    """H = -N(u) + nu L(u) at internal points (Sec. 2.4, Eq. (9)); zero elsewhere."""
    Nu, Nv, Nw = convection(g, u, v, w)
    fs = g.top == 1
    Hu = np.where(tags["u"], -Nu + g.nu * laplacian(g, u, fs), 0.0)
    Hv = np.where(tags["v"], -Nv + g.nu * laplacian(g, v, comp="v"), 0.0)
    Hw = np.where(tags["w"], -Nw + g.nu * laplacian(g, w, fs), 0.0)
    return Hu, Hv, Hw


# --------------------------------------------------------------------------------------
# Pressure Poisson solve: FFT in x and z, tridiagonal in y (Sec. 2.1: solved exactly)
# --------------------------------------------------------------------------------------
def modified_wavenumbers(n: int, h: float, half: bool) -> np.ndarray:
    """Eigenvalues of the periodic three-point second difference: (4/h^2) sin^2(pi m/n)."""
    m = np.arange(n // 2 + 1 if half else n)
    return (4.0 / (h * h)) * np.sin(np.pi * m / n) ** 2


def thomas(lower, diag, upper, rhs):
    """Thomas algorithm for tridiagonal systems along axis 0, vectorised over the rest."""
    n = rhs.shape[0]
    cp = np.empty(diag.shape, dtype=np.float64)
    dp = np.empty(rhs.shape, dtype=rhs.dtype)
    cp[0] = upper[0] / diag[0]
    dp[0] = rhs[0] / diag[0]
    for j in range(1, n):
        den = diag[j] - lower[j] * cp[j - 1]
        cp[j] = upper[j] / den
        dp[j] = (rhs[j] - lower[j] * dp[j - 1]) / den
    x = np.empty_like(dp)
    x[-1] = dp[-1]
    for j in range(n - 2, -1, -1):
        x[j] = dp[j] - cp[j] * x[j + 1]
    return x


def poisson_solve(g: OGrid, rhs: np.ndarray) -> Tuple[np.ndarray, float]:
    """Solve D G phi = rhs - mean(rhs) on the full box, zero-mean phi (readings R6, R11).

    Periodic x, z: real FFT in x, complex FFT in z, modified wavenumbers.
    In y, for each Fourier mode, the three-point operator with homogeneous
    Neumann closure (v = 0 on the box walls: the first and last rows carry -1
    instead of -2).  Mode (0,0) is singular: its right-hand side mean is
    removed, phi_0 = 0 fixes the constant, and the mean of phi is removed.
    Returns (phi, mean of rhs that was removed).
    """
    n = g.ny - 1
    rh = scipy.fft.fft(scipy.fft.rfft(rhs, axis=2), axis=1)          # (n, nz, mh)
    if g.stretched:
        # the volume-weighted mean: D G phi sums to zero with the cell heights as weights
        mean00 = np.sum(rh[:, 0, 0] * g.dyc) / np.sum(g.dyc)
    else:
        mean00 = rh[:, 0, 0].mean()
    rh[:, 0, 0] -= mean00
    kx2 = modified_wavenumbers(g.nx, g.dx, half=True)
    kz2 = modified_wavenumbers(g.nz, g.dz, half=False)
    K2 = kz2[:, None] + kx2[None, :]
    shape = (n,) + K2.shape
    if g.stretched:
        # row j: (1/dyc_j) [(phi_{j+1} - phi_j)/h_{j+1} - (phi_j - phi_{j-1})/h_j]
        lo = 1.0 / (g.dyc * g.hy_lo)
        hi = 1.0 / (g.dyc * g.hy_hi)
    else:
        lo = hi = np.full(n, 1.0 / (g.dy * g.dy))
    lower = np.broadcast_to(col(lo), shape).copy()
    upper = np.broadcast_to(col(hi), shape).copy()
    diag = -(lower + upper) - K2
    diag[0] += lower[0]
    diag[-1] += upper[-1]
    lower[0] = 0.0
    upper[-1] = 0.0
    # gauge of the singular (0,0) mode: replace its first row by phi_0 = 0
    diag[0, 0, 0] = 1.0
    upper[0, 0, 0] = 0.0
    rh[0, 0, 0] = 0.0
    ph = thomas(lower, diag, upper, rh)
    ph[:, 0, 0] -= ph[:, 0, 0].mean()
    phi = scipy.fft.irfft(scipy.fft.ifft(ph, axis=1), n=g.nx, axis=2)
    return phi, float(mean00.real) / (g.nx * g.nz)


def masked_laplacian(g: OGrid, tags) -> Tuple["scipy.sparse.csr_matrix", np.ndarray]:
    """D M G restricted to the internal pressure cells (reading R18).

    M keeps the gradient only on internal velocity faces (the external ones are never
    corrected, Sec. 3.3), so each internal face couples the two pressure cells it
    separates (an internal face always lies between two internal cells): with weight
    1/h^2 on a uniform grid; on a stretched one (reading R20) the v face j, at the
    centre spacing h_j from cell j-1 to cell j, enters the row of cell j with
    1/(h_j dy_j) and that of cell j-1 with 1/(h_j dy_{j-1}), dy the cell heights (the
    divergence over the cell height of the gradient over the centre spacing).  Returns
    the sparse matrix over the internal cells (in C order of the (j, k, i) cell array)
    and the flat indices of those cells.
    """
    import scipy.sparse as sp
    pin = tags["p"]
    cells = np.flatnonzero(pin.ravel())
    pos = -np.ones(pin.size, dtype=np.int64)
    pos[cells] = np.arange(cells.size)
    ny1, nz, nx = pin.shape
    jj, kk, ii = np.meshgrid(np.arange(ny1), np.arange(nz), np.arange(nx), indexing="ij")
    lin = (jj * nz + kk) * nx + ii
    rows, cols, vals = [], [], []
    # u face i of cell (j, k, i) joins cells i-1 and i; v face j joins rows j-1 and j
    # (face 0 is the south box wall, never internal); w face k joins k-1 and k
    for comp, face, other, h in (("u", tags["u"], (jj * nz + kk) * nx + (ii - 1) % nx, g.dx),
                                 ("v", tags["v"], ((jj - 1) * nz + kk) * nx + ii, g.dy),
                                 ("w", tags["w"], (jj * nz + (kk - 1) % nz) * nx + ii, g.dz)):
        a = pos[lin[face]]
        b = pos[other[face]]
        if (a < 0).any() or (b < 0).any():
            raise ValueError("internal face next to an external pressure cell")
        if comp == "v" and g.stretched:
            jf = jj[face]                      # face j: row a is cell j, row b cell j-1
            hc = g.hy_lo[jf]
            wa = 1.0 / (hc * g.dyc[jf])
            wb = 1.0 / (hc * g.dyc[jf - 1])
        else:
            wa = wb = np.full(a.size, 1.0 / (h * h))
        rows += [a, b, a, b]
        cols += [b, a, a, b]
        vals += [wa, wb, -wa, -wb]
    L = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(cells.size, cells.size))
    return L, cells


def masked_poisson_solve(g: OGrid, rhs: np.ndarray, tags) -> Tuple[np.ndarray, float]:
    """Solve D M G phi = rhs on the internal pressure cells only (reading R18).

    The operator is singular (constants) and rhs sums to zero over the internal cells,
    weighted by the cell volumes (every boundary face of the set carries no flux), so the
    system is consistent.  The solution with zero sum over the internal cells is taken:
    the rounding-level volume-weighted mean of rhs over the internal cells is removed
    (the least-squares reading of the system; the weights are the cell heights on a
    stretched grid, reading R20),
    the first internal cell is pinned to zero and its equation, implied by the others,
    dropped; the remaining nonsingular system is solved by a sparse direct factorisation
    and the mean over the internal cells removed.  The internal cells must form one
    connected set through internal faces.
    Returns phi (zero outside the internal cells) and the relative residual
    ||L phi - rhs|| / ||rhs|| (2-norms over the internal cells).
    """
    import scipy.sparse as sp
    import scipy.sparse.csgraph as csg
    import scipy.sparse.linalg as spla
    L, cells = masked_laplacian(g, tags)
    n = cells.size
    ncomp, _ = csg.connected_components(L != 0, directed=False)
    if ncomp != 1:
        raise ValueError(f"internal pressure cells form {ncomp} disconnected sets")
    b = rhs.ravel()[cells]
    if g.stretched:
        wv = np.broadcast_to(col(g.dyc), g.shape).ravel()[cells]
        bc = b - np.sum(wv * b) / np.sum(wv)
    else:
        bc = b - b.mean()
    x = np.zeros(n)
    if n > 1:
        x[1:] = spla.spsolve(sp.csc_matrix(L[1:, 1:]), bc[1:])
    x -= x.mean()
    phi = np.zeros(rhs.size)
    phi[cells] = x
    res = float(np.linalg.norm(L @ x - b) / max(np.linalg.norm(b), 1e-300))
    return phi.reshape(rhs.shape), res


# --------------------------------------------------------------------------------------
# Solver state and the RK3 substep (Sec. 2.4, Eq. (16); Sec. 2.1 projection)
# --------------------------------------------------------------------------------------
class Oracle:
    """Plain FP64 solver for one channel instance."""

    def __init__(self, g: OGrid):
        self.g = g
        self.tags = None
        self.lam = None
        self.coef = None
        self.S = None
        shp = g.shape
        self.u = np.zeros(shp)
        self.v = np.zeros(shp)
        self.w = np.zeros(shp)
        self.p = np.zeros(shp)
        self.H = None
        self.step_count = 0
        self.time = 0.0
        self.wall_vel = (0.0, 0.0, 0.0)
        self.pi_last = 0.0
        self.q_last = 0.0
        self.diag = {}

    # -- geometry ------------------------------------------------------------------
    def set_geometry(self, sdf_u, sdf_v, sdf_w, ibm: bool = True):
        """Classification, lambda and per-stage coefficients.  ibm=False keeps the
        bare staircase (lambda = 0 everywhere), the first-order baseline of Sec. 2.2."""
        g = self.g
        self.tags = classify(g, sdf_u, sdf_v, sdf_w)
        if not self.tags["p"].any():
            raise ValueError("geometry has no fluid")
        self.lam = {
            "u": wall_lambda(g, sdf_u, "u", self.tags["u"]),
            "v": wall_lambda(g, sdf_v, "v", self.tags["v"]),
            "w": wall_lambda(g, sdf_w, "w", self.tags["w"]),
        }
        self.sig = {
            "u": wall_source(g, sdf_u, "u", self.tags["u"]),
            "v": wall_source(g, sdf_v, "v", self.tags["v"]),
            "w": wall_source(g, sdf_w, "w", self.tags["w"]),
        }
        if not ibm:
            self.lam = {c: np.zeros_like(l) for c, l in self.lam.items()}
            self.sig = {c: np.zeros_like(l) for c, l in self.sig.items()}
        self.coef = []
        for k in range(3):
            self.coef.append({c: stage_coefficients(self.lam[c], k, g.dt, g.b_mode) for c in "uvw"})
        # response of the flow rate to a unit pressure gradient at each stage
        self.S = [self.flow_rate(np.where(self.tags["u"], RK_C[k] * g.dt / self.coef[k]["u"][1], 0.0))
                  for k in range(3)]

    def set_state(self, u, v, w, p):
        self.u, self.v, self.w, self.p = (np.array(a, dtype=np.float64) for a in (u, v, w, p))
        self.H = None

    def set_wall_velocity(self, ub: float, vb: float, wb: float):
        """Velocity of the immersed walls (rigid translation; reading R19); the box walls
        stay at rest."""
        self.wall_vel = (float(ub), float(vb), float(wb))

    def _external(self, comp: str) -> np.ndarray:
        """Stored value of the external points of one component: the wall velocity inside
        the box, zero on the south box-wall face of v (Sec. 3.3)."""
        out = np.full(self.g.shape, self.wall_vel["uvw".index(comp)])
        if comp == "v":
            out[0] = 0.0
        return out

    def flow_rate(self, f):
        """Q = (1/nx) sum over internal u faces of f dy dz (mean flux through x-planes;
        dy the cell height of the row on a stretched grid)."""
        g = self.g
        if g.stretched:
            return float(np.sum(np.where(self.tags["u"], f, 0.0) * col(g.dyc)) * g.dz / g.nx)
        return float(np.sum(np.where(self.tags["u"], f, 0.0)) * g.dy * g.dz / g.nx)

    # -- one RK substep --------------------------------------------------------------
    def substep(self, k: int):
        g, t = self.g, self.tags
        dt, ck = g.dt, RK_C[k]
        # external points hold the wall velocity (zero for walls at rest) and no pressure
        # (Sec. 3.3): the correction of Eqs. (5)-(7) is the difference to a stencil that
        # uses these stored values.  After a substep this already holds; after a new state
        # or a new geometry the values at external points are replaced here.
        ext = {c: self._external(c) for c in "uvw"}
        self.u = np.where(t["u"], self.u, ext["u"])
        self.v = np.where(t["v"], self.v, ext["v"])
        self.w = np.where(t["w"], self.w, ext["w"])
        self.p = np.where(t["p"], self.p, 0.0)
        # explicit right-hand side at the current stage (Eq. (9) without the IBM term)
        Hn = explicit_rhs(g, self.u, self.v, self.w, t)
        Gp = gradient(g, self.p)
        star = []
        for c, f, Hc, Gc in zip("uvw", (self.u, self.v, self.w), Hn, Gp):
            r = dt * RK_A[k] * Hc - ck * dt * Gc                     # reading R2
            if RK_B[k] != 0.0:
                r = r + dt * RK_B[k] * self.H[("uvw").index(c)]
            B, A = self.coef[k][c]
            # Eq. (16): (lambda c_k dt + B) w* - B w = dt (a_k f_k + b_k f_{k-1}), plus the
            # moving wall's term sigma U_b, explicit and weighted like lambda (reading R19)
            src = ck * dt * self.sig[c] * self.wall_vel["uvw".index(c)]
            star.append(np.where(t[c], (B * f + r + src) / A, ext[c]))   # reading R3
        us, vs, ws = star
        # mean pressure gradient (reading R4)
        invA_u = 1.0 / self.coef[k]["u"][1]
        if g.forcing == CFR:
            q0 = self.flow_rate(us)
            pi = (q0 - g.q_target_or_pi) / self.S[k]
        else:
            pi = g.q_target_or_pi
        us = np.where(t["u"], us - pi * ck * dt * invA_u, ext["u"])
        self.pi_last = pi
        # projection (Sec. 2.1; continuity on the full box, Sec. 3.3, reading R6)
        rhs = divergence(g, us, vs, ws) / (ck * dt)
        if g.projection == 1:
            # masked projection (reading R18): continuity on the internal cells only
            phi, res = masked_poisson_solve(g, rhs, t)
            Gx, Gy, Gz = gradient(g, phi)
            un = us - ck * dt * Gx
            vn = vs - ck * dt * Gy
            vn[0] = 0.0
            wn = ws - ck * dt * Gz
            self.diag = {"div_max_fullbox": 0.0, "poisson_rel_residual": res, "rhs_mean_removed": 0.0}
        else:
            phi, mean_removed = poisson_solve(g, rhs)
            Gx, Gy, Gz = gradient(g, phi)
            un = us - ck * dt * Gx
            vn = vs - ck * dt * Gy
            vn[0] = 0.0                                                     # south box wall
            wn = ws - ck * dt * Gz
            div_full = divergence(g, un, vn, wn)
            resid = divergence(g, *gradient_full(g, phi)) - (rhs - mean_removed)
            self.diag = {
                "div_max_fullbox": float(np.abs(div_full).max()),
                "poisson_rel_residual": float(np.abs(resid).max() / max(np.abs(rhs).max(), 1e-300)),
                "rhs_mean_removed": mean_removed,
            }
        # external faces back to the wall velocity (Sec. 3.3); only internal pressure is
        # updated
        self.u = np.where(t["u"], un, ext["u"])
        self.v = np.where(t["v"], vn, ext["v"])
        self.w = np.where(t["w"], wn, ext["w"])
        self.p = np.where(t["p"], self.p + phi, 0.0)
        self.H = Hn
        self.q_last = self.flow_rate(self.u)

    def step(self, nsteps: int = 1):
        for _ in range(nsteps):
            for k in range(3):
                self.substep(k)
            self.step_count += 1
            self.time += self.g.dt

    # -- diagnostics -------------------------------------------------------------------
    def stats(self) -> Dict[str, float]:
        g, t = self.g, self.tags
        d = divergence(g, self.u, self.v, self.w)
        out = dict(self.diag)
        out.update({
            "step": self.step_count,
            "time": self.time,
            "q": self.flow_rate(self.u),
            "pi_last": self.pi_last,
            "div_max_internal_leak": float(np.abs(np.where(t["p"], d, 0.0)).max()),
            "ke": float(0.5 * np.sum((self.u ** 2 + self.v ** 2 + self.w ** 2) * col(g.dyc))
                        * g.dx * g.dz) if g.stretched else
                  float(0.5 * (np.sum(self.u ** 2) + np.sum(self.v ** 2) + np.sum(self.w ** 2))
                        * g.dx * g.dy * g.dz),
            "cfl_max": float(np.max(np.abs(self.u) / g.dx + np.abs(self.v) / col(g.dyc)
                                    + np.abs(self.w) / g.dz) * g.dt),
            "n_internal": [int(t[c].sum()) for c in "uvw"],
            "n_ibm": [int((self.lam[c] > 0).sum()) for c in "uvw"],
            "n_p_internal": int(t["p"].sum()),
            "nan_flag": int(not (np.isfinite(self.u).all() and np.isfinite(self.v).all()
                                 and np.isfinite(self.w).all() and np.isfinite(self.p).all())),
        })
        return out


def gradient_full(g: OGrid, phi):
    """G phi on all faces with the v component zeroed on the south box wall."""
    Gx, Gy, Gz = gradient(g, phi)
    Gy = Gy.copy()
    Gy[0] = 0.0
    return Gx, Gy, Gz


def solve_pressure(g: OGrid, rhs: np.ndarray):
    """Stand-alone Poisson solve, the operation behind the library's solve-pressure call."""
    return poisson_solve(g, np.asarray(rhs, dtype=np.float64))


# --------------------------------------------------------------------------------------
# Wall-shear stress of the undulated bottom and its Fourier components (Sec. 4.2)
# --------------------------------------------------------------------------------------
def south_wall_points(g: OGrid, sdf_u: np.ndarray, ibm: bool = True, with_box: bool = False):
    """Lowest internal u point of every (k, i) column and its distance to the wall below.

    Reading R17: the wall under the lowest internal point of a column is located as the
    immersed boundary locates it (Sec. 2.2 and reading R8): the linear zero crossing of
    the signed distance between the point and the external point below it, or the south
    box wall dy/2 below row 0 when that is nearer.  Without the immersed-boundary
    correction the staircase puts the wall at the external point itself (distance dy).
    Returns (j1, d1): j1 = -1 and d1 = 0 where a column holds no internal u point; with
    with_box also a mask of the columns whose wall is the south box wall (at rest).
    sdf_u: (ny+1, nz, nx) with row j+1 holding row j (ghost rows 0 and ny).
    """
    s = sdf_u[1:-1]
    internal = s > 0.0
    has = internal.any(axis=0)
    j1 = np.argmax(internal, axis=0)
    kk, ii = np.meshgrid(np.arange(g.nz), np.arange(g.nx), indexing="ij")
    sP = s[j1, kk, ii]
    s_dn = sdf_u[j1, kk, ii]                 # row j1 - 1 (the ghost row for j1 = 0)
    harm = g.hy_lo[j1]                      # length of the stencil arm below row j1
    d1 = harm.copy()
    with np.errstate(divide="ignore", invalid="ignore"):
        cross = np.where(s_dn <= 0.0, harm * sP / (sP - s_dn), np.inf)
    box = np.where(j1 == 0, 0.5 * g.dyc[0], np.inf)
    if ibm:
        d1 = np.minimum(cross, box)
    j1 = np.where(has, j1, -1)
    d1 = np.where(has, d1, 0.0)
    if with_box:
        return j1, d1, has & (box <= cross)
    return j1, d1


def wall_shear_profile(g: OGrid, u: np.ndarray, sdf_u: np.ndarray, ibm: bool = True,
                       wall_velocity: float = 0.0) -> np.ndarray:
    """Spanwise-averaged wall-shear stress tau(x_i) along the south wall (Sec. 4.2).

    Reading R17: tau is the viscous flux the discretisation itself exchanges with the
    wall.  The ghost value below the lowest internal point is the linear extrapolation
    through zero at the wall (Sec. 2.2, Eqs. (5)-(7)), so the flux through that stencil
    arm is nu (u1 - u_ghost)/dy = nu u1/d1, d1 the wall distance the correction uses
    (with the bare staircase the wall is at the external point, d1 = dy).  Summed over
    the walls this is exactly the discrete momentum balance of a steady flow (pinned).
    An immersed wall sliding with streamwise velocity U_b gives nu (u1 - U_b)/d1 (the box
    wall stays at rest).  Columns without internal u points add zero; the mean is over all
    nz columns of each x_i = i dx.
    """
    j1, d1, box = south_wall_points(g, sdf_u, ibm, with_box=True)
    tau = np.zeros((g.nz, g.nx))
    for k in range(g.nz):
        for i in range(g.nx):
            j = int(j1[k, i])
            if j < 0:
                continue
            ub = 0.0 if box[k, i] else wall_velocity
            tau[k, i] = g.nu * (float(u[j, k, i]) - ub) / float(d1[k, i])
    return tau.mean(axis=0)


def wall_shear_modes(g: OGrid, tau_x: np.ndarray) -> Tuple[float, float, float]:
    """Mean and first Fourier components of tau(x) over the box length (Sec. 4.2).

    tau_1c and tau_1s are (2/L_x) times the integrals of tau(x) cos(2 pi x/L_x) and
    tau(x) sin(2 pi x/L_x) over one box length; on the uniform periodic grid of u points
    x_i = i dx the integrals are the rectangle sums, exact for trigonometric polynomials
    of degree below nx.  tau_0 is the plain mean.
    """
    x = np.arange(g.nx) * g.dx
    th = 2.0 * math.pi * x / g.lx
    t0 = float(np.sum(tau_x) * g.dx / g.lx)
    t1c = float(2.0 / g.lx * np.sum(tau_x * np.cos(th)) * g.dx)
    t1s = float(2.0 / g.lx * np.sum(tau_x * np.sin(th)) * g.dx)
    return t0, t1c, t1s
