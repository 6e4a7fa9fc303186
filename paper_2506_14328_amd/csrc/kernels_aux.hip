// Geometry preprocessing (Sec. 2.2, Sec. 2.4, Sec. 3.3) and diagnostics.
#include "ibm_internal.h"

namespace {

constexpr int BX = 64;
constexpr int BZ = 4;

__device__ __forceinline__ int wrap_p(int i, int n) { return (i + 1 == n) ? 0 : i + 1; }
__device__ __forceinline__ int wrap_m(int i, int n) { return (i == 0) ? n - 1 : i - 1; }

// One arm of a point P towards its neighbour Q (spacing h, second-derivative coefficient
// d2: 1/h^2 on uniform arms), Q external (extQ): the wall lies at delta, the linear zero
// crossing h sP/(sP - sQ) of the signed distance, or at the box wall distance `box` when
// that is nearer (Eq. (7)).  Adds to lam the arm's share nu d2 (h - delta)/delta of the
// Laplacian's centre change, and to src the coefficient of the wall velocity U_b in the
// correction (the ghost extrapolated through U_b): 0 when the nearer wall is a box wall
// (at rest); the arm's lambda share when Q stores U_b (an external point inside the box,
// box = infinity); nu d2 h/delta when Q stores zero (the box-wall face or the ghost beyond
// it, box finite).  delta takes an IEEE division, since delta < h decides whether P
// carries a correction; 1/delta is refined from the hardware estimate.
__device__ __forceinline__ void arm_pair(double nu, double h, double d2, double sP, double sQ, bool extQ,
                                         double box, double& lam, double& src) {
  if (!extQ) return;
  const bool cross = sQ <= 0.0;
  const double delta = cross ? h * sP / (sP - sQ) : INFINITY;
  const double dl = fmin(delta, box);
  const double r = dl > 1e-250 ? recip(dl) : 1.0 / dl;
  const double l = nu * d2 * (h - dl) * r;
  lam += l;
  if (cross && delta < box) src += isinf(box) ? l : nu * d2 * h * r;
}

// Whether that arm changes the Laplacian's centre weight (a positive lambda share):
// min(delta, box) < h.  With the signed distance crossing zero, delta < h holds exactly
// when sQ < 0 up to the rounding of the quotient, so the IEEE quotient is formed only when
// |sQ| is within 2^-40 of sP, where the rounding could decide.
__device__ __forceinline__ bool arm_active(double h, double sP, double sQ, bool extQ, double box) {
  if (!extQ) return false;
  if (box < h) return true;
  if (!(sQ <= 0.0)) return false;
  if (sQ < -sP * 0x1p-40) return true;
  return h * sP / (sP - sQ) < h;
}

// Wall-normal arm data of component q (0 u, 1 v, 2 w) on row j: the arms' spacings, their
// second-derivative coefficients and whether the neighbour below / above is a box wall,
// with that wall's distance (u, w: the south box face is a wall, so is the north one
// unless it is free-slip, half a cell away; v: faces 0 and ny-1 are the walls, one spacing
// away); INFINITY where the neighbour is not a box wall.
struct YArms {
  double hdn, hup, cdn, cup, bdn, bup;
  bool gdn, gup;
};
__device__ __forceinline__ YArms y_arms(const GridParams& g, int q, int j) {
  const bool sy = g.stretched != 0;
  const double* yt = g.ytab;
  const int ys = g.ystr, ny1 = g.ny1;
  const double dy2 = 1.0 / (g.dy * g.dy);
  YArms a;
  a.bdn = a.bup = INFINITY;
  if (q != 1) {
    a.gdn = (j == 0);
    a.gup = (j == ny1 - 1) && !g.top_fs;
    a.hdn = sy ? yt[YT_HC * ys + j] : g.dy;
    a.hup = sy ? yt[YT_HC * ys + j + 1] : g.dy;
    a.cdn = sy ? yt[YT_DCM * ys + j] : dy2;
    a.cup = sy ? yt[YT_DCP * ys + j] : dy2;
    if (a.gdn) a.bdn = sy ? 0.5 * yt[YT_DYC * ys] : 0.5 * g.dy;
    if (a.gup) a.bup = sy ? 0.5 * yt[YT_DYC * ys + ny1 - 1] : 0.5 * g.dy;
  } else {
    a.gdn = (j - 1 == 0);
    a.gup = (j + 1 == ny1);
    a.hdn = sy ? yt[YT_DYC * ys + j - 1] : g.dy;
    a.hup = sy ? yt[YT_DYC * ys + j] : g.dy;
    a.cdn = sy ? yt[YT_DFM * ys + j] : dy2;
    a.cup = sy ? yt[YT_DFP * ys + j] : dy2;
    if (a.gdn) a.bdn = a.hdn;
    if (a.gup) a.bup = a.hup;
  }
  return a;
}

// The seven samples (P, x-, x+, z-, z+, y-, y+) of component q at cell (j, k, i): u and w
// from sample row j + 1 (ghost rows 0 and ny lie outside the box), v on face j (face 0 is
// never internal; its y- sample is clamped to itself).
__device__ __forceinline__ void samples7(const GridParams& g, const double* __restrict__ s, int q, int i, int k,
                                         int j, double* d) {
  const int nx = g.nx, nz = g.nz, plane = nx * nz;
  const int im = wrap_m(i, nx), ip = wrap_p(i, nx);
  const int b = (q == 1 ? j : j + 1) * plane + k * nx;
  d[0] = s[b + i];
  d[1] = s[b + im];
  d[2] = s[b + ip];
  d[3] = s[b + (wrap_m(k, nz) - k) * nx + i];
  d[4] = s[b + (wrap_p(k, nz) - k) * nx + i];
  d[5] = s[(q == 1 && j == 0 ? b : b - plane) + i];
  d[6] = s[b + plane + i];
}

// South-wall point of every (k, i) column of u points: the lowest internal u row j1 and
// its distance d1 to the wall below, located as the immersed boundary locates it (the
// linear zero crossing of the signed distance towards the external point below, or the
// south box wall dy/2 below row 0 when nearer); without the correction the staircase
// wall is at the external point (dy).  j1 = -1, d1 = 0 for a column with no internal u;
// d1 is stored negative where the wall is the south box wall (at rest).
__device__ __forceinline__ void south_wall_point(const GridParams& g, const double* __restrict__ su, int ibm_on,
                                                 int i, int k, int32_t* __restrict__ wj, double* __restrict__ wd) {
  const size_t plane = (size_t)g.nx * g.nz;
  const int col = k * g.nx + i;
  int j1 = -1;
  double sP = 0.0;
  // rows in groups of 8 whose loads are issued together (row j is SDF row j + 1)
  for (int j0 = 0; j0 < g.ny1 && j1 < 0; j0 += 8) {
    double sj[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) sj[q] = (j0 + q < g.ny1) ? su[(size_t)(j0 + q + 1) * plane + col] : 0.0;
#pragma unroll
    for (int q = 7; q >= 0; --q)
      if (sj[q] > 0.0) {
        j1 = j0 + q;
        sP = sj[q];
      }
  }
  double d = 0.0;
  bool box = false;
  if (j1 >= 0) {
    const double sdn = su[(size_t)j1 * plane + col];
    // length of the stencil arm below row j1 and half the first cell
    const double harm = g.stretched ? g.ytab[YT_HC * g.ystr + j1] : g.dy;
    const double half = g.stretched ? 0.5 * g.ytab[YT_DYC * g.ystr] : 0.5 * g.dy;
    const double cross = (sdn <= 0.0) ? harm * sP / (sP - sdn) : INFINITY;
    box = (j1 == 0) && (half <= cross);
    d = ibm_on ? (box ? half : cross) : harm;
  }
  wj[col] = j1;
  wd[col] = box ? -d : d;   // negative: the wall is the south box wall (at rest)
}

// Tags of u, v, w at every cell (j, k, i): internal, and carrying an immersed-boundary
// correction (some stencil arm ends at a wall nearer than its neighbour: lambda > 0,
// Eq. (7); lambda and sigma themselves are computed for the listed points only, by
// k_list_coef); the pressure tag; the counts of the seven tag masks per (row, 64-wide
// chunk), counts[m * nch + row * cpr + chunk] with one zero entry at the end of each array
// (nch = nrows cpr + 1); and the south-wall point of every column (wj, wd).
//  sdf_u, sdf_w: (ny+1, nz, nx), row jj = j+1 holds row j; sdf_v: (ny, nz, nx) faces.
// A block takes a 64 x 4 (x, z) tile through TAG_JC rows, marching up in y: each thread
// keeps the samples of the rows below, at and above its cell in registers and loads one
// new row per step; the x and z neighbours come from the row's tile in LDS (with a halo
// of one point; lanes past the box hold the periodically continued samples).
// With `correct`, first the projection left pending by the last step is applied with the
// cell's old tag and written over its predictor and pressure (f.us, f.vs, f.ws, f.pp):
// this thread alone reads and writes those and the tag, and phi is only read here.
constexpr int TAG_JC = 8;
template <typename T>
__global__ __launch_bounds__(256) void k_geom_tags(GridParams g, const double* __restrict__ su,
                                                  const double* __restrict__ sv, const double* __restrict__ sw,
                                                  int ibm_on, uint8_t* __restrict__ tag, int correct, Fields<T> f,
                                                  const double* __restrict__ wallv, double ck_dt,
                                                  const double* __restrict__ pi, int32_t* __restrict__ wj,
                                                  double* __restrict__ wd, int32_t* __restrict__ counts,
                                                  int32_t* __restrict__ clear) {
  __shared__ double tl[3][BZ + 2][BX + 2];
  const int tx = threadIdx.x, tz = threadIdx.y;
  const int nx = g.nx, nz = g.nz, ny1 = g.ny1, plane = nx * nz;
  const int i = blockIdx.x * BX + tx, k = blockIdx.y * BZ + tz;
  const bool act = i < nx && k < nz;
  const int il = i % nx, kl = k % nz;   // (periodic continuation past the box)
  const int j0 = blockIdx.z * TAG_JC, j1 = min(j0 + TAG_JC, ny1);
  const double* src[3] = {su, sv, sw};
  // sample of component q for cell row j at (x, z) = (ii, kk): u and w on sample row j + 1,
  // v on face j (face -1 clamped to face 0)
  auto smp = [&](int q, int j, int ii, int kk) -> double {
    const int r = q == 1 ? (j < 0 ? 0 : j) : j + 1;
    return src[q][(size_t)r * plane + kk * nx + ii];
  };
  const int ihalo = tx == 0 ? (il == 0 ? nx - 1 : il - 1) : (il + 1 == nx ? 0 : il + 1);
  const bool xh = tx == 0 || tx == BX - 1;
  const int khalo = tz == 0 ? (kl == 0 ? nz - 1 : kl - 1) : (kl + 1 == nz ? 0 : kl + 1);
  const bool zh = tz == 0 || tz == BZ - 1;
  double dn[3], ce[3], up[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    dn[q] = smp(q, j0 - 1, il, kl);
    ce[q] = smp(q, j0, il, kl);
  }
  uint8_t tg = 0;   // this row's tag (0 for lanes past the box)
  for (int j = j0; j < j1; ++j) {
    double hx[3], hz[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      up[q] = smp(q, j + 1, il, kl);
      hx[q] = xh ? smp(q, j, ihalo, kl) : 0.0;
      hz[q] = zh ? smp(q, j, il, khalo) : 0.0;
    }
    __syncthreads();   // the previous row's tile has been read
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      tl[q][tz + 1][tx + 1] = ce[q];
      if (xh) tl[q][tz + 1][tx == 0 ? 0 : BX + 1] = hx[q];
      if (zh) tl[q][tz == 0 ? 0 : BZ + 1][tx + 1] = hz[q];
    }
    __syncthreads();
    if (act) {
      const int c = (j * nz + k) * nx + i;
      if (correct) {
        const int im = wrap_m(i, nx), km = wrap_m(k, nz);
        const Corrected<T> r = corrected_point<T>(g, f, wallv, tag[c], j, c, c - i + im, j > 0 ? c - plane : c,
                                                  c + (km - k) * nx, ck_dt, pi[0]);
        f.us[c] = r.u;
        f.vs[c] = r.v;
        f.ws[c] = r.w;
        f.pp[c] = r.p;
      }
      uint8_t t = 0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double sP = ce[q];
        const bool in = (q == 1) ? (j >= 1 && sP > 0.0) : (sP > 0.0);
        if (!in) continue;
        t |= (q == 0) ? TAG_U : (q == 1 ? TAG_V : TAG_W);
        const double sxm = tl[q][tz + 1][tx], sxp = tl[q][tz + 1][tx + 2];
        const double szm = tl[q][tz][tx + 1], szp = tl[q][tz + 2][tx + 1];
        const YArms ya = y_arms(g, q, j);
        const bool ibm = ibm_on && (arm_active(g.dx, sP, sxm, sxm <= 0.0, INFINITY) ||
                                    arm_active(g.dx, sP, sxp, sxp <= 0.0, INFINITY) ||
                                    arm_active(g.dz, sP, szm, szm <= 0.0, INFINITY) ||
                                    arm_active(g.dz, sP, szp, szp <= 0.0, INFINITY) ||
                                    arm_active(ya.hdn, sP, dn[q], ya.gdn || dn[q] <= 0.0, ya.bdn) ||
                                    arm_active(ya.hup, sP, up[q], ya.gup || up[q] <= 0.0, ya.bup));
        if (ibm) t |= (q == 0) ? TAG_UI : (q == 1 ? TAG_VI : TAG_WI);
      }
      // the pressure cell is internal iff one of its six faces is an internal velocity
      // point: its own west, south and back faces, or the east cell's u, the north cell's v
      // (below the north box face) and the top cell's w
      const bool ue = tl[0][tz + 1][tx + 2] > 0.0, vn = (j + 1 < ny1) && up[1] > 0.0, wt = tl[2][tz + 2][tx + 1] > 0.0;
      if ((t & (TAG_U | TAG_V | TAG_W)) || ue || vn || wt) t |= TAG_P;
      tag[c] = t;
      tg = t;
    }
    // per-(row, 64-wide chunk) counts of the seven masks: a wave is the chunk blockIdx.x of
    // row (j, k)
    if (k < nz) {
      const int nch = g.nrows * ((nx + BX - 1) / BX) + 1;
      const int ch = (j * nz + k) * ((nx + BX - 1) / BX) + blockIdx.x;
      const uint8_t msk[7] = {TAG_U, TAG_V, TAG_W, TAG_P, TAG_UI, TAG_VI, TAG_WI};
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        const uint64_t b = __ballot((tg & msk[m]) != 0);
        if (tx == 0) counts[m * nch + ch] = __popcll(b);
      }
    }
    tg = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      dn[q] = ce[q];
      ce[q] = up[q];
    }
  }
  // one zero entry after each count array; the lists' overflow flag cleared (a kernel, so
  // that a geometry update can be captured)
  if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && tx == 0 && tz == 0) {
    const int nch = g.nrows * ((nx + BX - 1) / BX) + 1;
    for (int m = 0; m < 7; ++m) counts[m * nch + nch - 1] = 0;
    clear[0] = 0;
  }
  // the blocks of the first rows also locate their columns' south-wall points
  if (j0 == 0 && act) south_wall_point(g, su, ibm_on, i, k, wj, wd);
}

// Tiled exclusive scans of several count arrays (ScanSet): block b scans tile
// b - tile_off[m] of array m.  In a tile thread t holds the 4 counts 4t .. 4t+3 (one
// 16-byte load when the array is 16-byte aligned), so that a wave's loads and stores are
// one contiguous kilobyte.
__device__ __forceinline__ int scan_array_of(const ScanSet& s, int b) {
  int m = 0;
  while (m + 1 < s.narr && b >= s.tile_off[m + 1]) ++m;
  return m;
}
__device__ __forceinline__ int4 scan_load4(const int32_t* __restrict__ counts, int n, int e0) {
  int4 v;
  if ((reinterpret_cast<uintptr_t>(counts) & 15) == 0 && e0 + 3 < n) {
    v = *reinterpret_cast<const int4*>(counts + e0);
  } else {
    v.x = e0 < n ? counts[e0] : 0;
    v.y = e0 + 1 < n ? counts[e0 + 1] : 0;
    v.z = e0 + 2 < n ? counts[e0 + 2] : 0;
    v.w = e0 + 3 < n ? counts[e0 + 3] : 0;
  }
  return v;
}
__device__ __forceinline__ int32_t wave_isum(int32_t v) {
  for (int o = IBM_WAVE / 2; o > 0; o >>= 1) v += __shfl_down(v, o, IBM_WAVE);
  return v;
}

// Pass 1: the sum of every tile into s.tsum[b].
__global__ __launch_bounds__(1024) void k_scan_tile_sums(ScanSet s) {
  __shared__ int32_t wsum[16];
  const int b = blockIdx.x, m = scan_array_of(s, b), t = b - s.tile_off[m];
  const int tid = threadIdx.x, lane = tid & (IBM_WAVE - 1), wid = tid / IBM_WAVE;
  const int4 v = scan_load4(s.counts[m], s.n[m], t * SCAN_TILE + 4 * tid);
  const int32_t w = wave_isum(v.x + v.y + v.z + v.w);
  if (lane == 0) wsum[wid] = w;
  __syncthreads();
  if (tid == 0) {
    int32_t tot = 0;
    for (int q = 0; q < 16; ++q) tot += wsum[q];
    s.tsum[b] = tot;
  }
}

// Pass 2: each tile scanned in place from the sum of the tiles before it in its array;
// the array's last tile writes its total.
__global__ __launch_bounds__(1024) void k_scan_tiles(ScanSet s) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t base_sh;
  const int b = blockIdx.x, m = scan_array_of(s, b), t = b - s.tile_off[m];
  const int tid = threadIdx.x, lane = tid & (IBM_WAVE - 1), wid = tid / IBM_WAVE;
  int32_t* counts = s.counts[m];
  const int n = s.n[m], e0 = t * SCAN_TILE + 4 * tid;
  const int4 v = scan_load4(counts, n, e0);
  if (wid == 0) {   // sum of the preceding tiles of this array
    int32_t c = 0;
    for (int q = lane; q < t; q += IBM_WAVE) c += s.tsum[s.tile_off[m] + q];
    c = wave_isum(c);
    if (lane == 0) base_sh = c;
  }
  const int32_t sum = v.x + v.y + v.z + v.w;
  int32_t x = sum;   // inclusive scan over the wave
  for (int o = 1; o < IBM_WAVE; o <<= 1) {
    const int32_t y = __shfl_up(x, o, IBM_WAVE);
    if (lane >= o) x += y;
  }
  if (lane == IBM_WAVE - 1) wsum[wid] = x;
  __syncthreads();
  if (wid == 0) {
    int32_t w = lane < 16 ? wsum[lane] : 0;
    for (int o = 1; o < 16; o <<= 1) {
      const int32_t y = __shfl_up(w, o, IBM_WAVE);
      if (lane >= o) w += y;
    }
    if (lane < 16) wsum[lane] = w;
  }
  __syncthreads();
  int32_t run = base_sh + (wid > 0 ? wsum[wid - 1] : 0) + (x - sum);
  int4 o;
  o.x = run;
  run += v.x;
  o.y = run;
  run += v.y;
  o.z = run;
  run += v.z;
  o.w = run;
  if ((reinterpret_cast<uintptr_t>(counts) & 15) == 0 && e0 + 3 < n) {
    *reinterpret_cast<int4*>(counts + e0) = o;
  } else {
    if (e0 < n) counts[e0] = o.x;
    if (e0 + 1 < n) counts[e0 + 1] = o.y;
    if (e0 + 2 < n) counts[e0 + 2] = o.z;
    if (e0 + 3 < n) counts[e0 + 3] = o.w;
  }
  if (tid == 0 && b + 1 == s.tile_off[m + 1]) s.total[m][0] = base_sh + wsum[15];
}

// Per-stage (B, 1/A) of a point with coefficient lam (Eqs. (14)-(16)): x = lam c_k dt.
__device__ __forceinline__ double2 ibm_stage_coef(double lam, int k, double dt, int b_mode) {
  const double x = lam * rk_c(k) * dt;
  double B, A;
  if (b_mode == 1) {          // implicit Euler: B = 1
    B = 1.0;
    A = 1.0 + x;
  } else if (b_mode == 2) {   // reciprocal of the second-order Taylor expansion of 1/B
    B = 1.0 / (1.0 + 0.5 * x);
    A = x + B;
  } else {                    // exponential fit B = x / (e^x - 1)
    B = (x > 700.0) ? 0.0 : ((x > 0.0) ? x / expm1(x) : 1.0);
    A = x + B;
  }
  return make_double2(B, 1.0 / A);
}

// The ascending cell indices of the u, v and w immersed-boundary points (tag bits
// TAG_UI << c) into the component's list, which starts at list_off[c] and holds cap[c]
// entries: wave w of block b is the 64-wide chunk 4b + w (row r = chunk / cpr), whose
// points go to the chunk's scanned offset offsets[c][chunk] plus their rank among the
// chunk's flagged lanes; a point whose rank reaches the capacity is not written and sets
// overflow[0].  With zphi every cell's phi (zelem bytes each) is zeroed too, with zpi the
// mean pressure gradient: what is left of a projection applied earlier in the update.
__global__ __launch_bounds__(256) void k_compact3(const uint8_t* __restrict__ tag, int nx, int nrows, int cpr,
                                                 const int32_t* __restrict__ off_u, const int32_t* __restrict__ off_v,
                                                 const int32_t* __restrict__ off_w, int32_t* __restrict__ idx,
                                                 int lo_v, int lo_w, int cap_u, int cap_v, int cap_w,
                                                 int32_t* __restrict__ overflow, unsigned char* __restrict__ zphi,
                                                 int zelem, double* __restrict__ zpi) {
  const int lane = threadIdx.x % IBM_WAVE;
  const int ch = blockIdx.x * 4 + threadIdx.x / IBM_WAVE;
  if (ch >= nrows * cpr) return;   // (whole waves)
  const int row = ch / cpr, i = (ch - row * cpr) * IBM_WAVE + lane;
  const bool in = i < nx;
  const int e = row * nx + i;
  const uint8_t t = in ? tag[e] : uint8_t(0);
  if (in && zphi) {
    if (zelem == 8) reinterpret_cast<double*>(zphi)[e] = 0.0;
    else reinterpret_cast<float*>(zphi)[e] = 0.0f;
  }
  if (zpi && ch == 0 && lane == 0) zpi[0] = 0.0;
  const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const uint64_t bal = __ballot((t & (TAG_UI << c)) != 0);
    if (!(t & (TAG_UI << c))) continue;
    const int r = (c == 0 ? off_u : (c == 1 ? off_v : off_w))[ch] + __popcll(bal & below);
    const int cap = c == 0 ? cap_u : (c == 1 ? cap_v : cap_w);
    const int lo = c == 0 ? 0 : (c == 1 ? lo_v : lo_w);
    if (r < cap) idx[lo + r] = e;
    else overflow[0] = 1;
  }
}

// bytes zeros from p (a kernel: no memset nodes in captured graphs): nvec 16-byte vectors
// (p 16-byte aligned, nvec = 0 otherwise), the remaining bytes by thread 0 of block 0
__global__ __launch_bounds__(256) void k_fill_zero(unsigned char* __restrict__ p, int64_t nvec, int64_t bytes) {
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  if (e < nvec) reinterpret_cast<uint4*>(p)[e] = make_uint4(0u, 0u, 0u, 0u);
  if (e == 0)
    for (int64_t b = nvec * 16; b < bytes; ++b) p[b] = 0;
}

// S_k partials: number of internal non-IBM u points (column 0) and sum over IBM u points
// of 1/A_k (columns 1..3).  part layout: [block][4].
__global__ __launch_bounds__(256) void k_s_cells(GridParams g, const uint8_t* __restrict__ tag,
                                                double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  double c = 0.0;
  if (e < g.ncell) c = ((tag[e] & (TAG_U | TAG_UI)) == TAG_U) ? 1.0 : 0.0;
  // a stretched grid weights each row by its cell height
  if (g.stretched && e < g.ncell) c *= g.ytab[YT_DYC * g.ystr + (int)(e / ((int64_t)g.nx * g.nz))];
  const double tot = block_reduce<false>(c, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 4 + 0] = tot;
    part[blockIdx.x * 4 + 1] = 0.0;
    part[blockIdx.x * 4 + 2] = 0.0;
    part[blockIdx.x * 4 + 3] = 0.0;
  }
}
// S3[k] = S_k from the npart partials of part; with sd_out, sd_out[k] = the sum of the nsd
// partials of stage k in part_sd (fixed orders; zero for no partials)
// With cnt7 (uniform grids) the internal non-IBM u points are its internal u count minus
// its immersed-boundary u count (every immersed-boundary u point is internal).  The seven
// sums are accumulated in one pass (all loads issued together), reduced over each wave and
// then over the block's waves (at most 16) in a fixed order.
__device__ __forceinline__ void s_final_block(const double* __restrict__ part, int npart, double scale,
                                              double* __restrict__ S3, const double* __restrict__ part_sd,
                                              int nsd, double* __restrict__ sd_out,
                                              const int32_t* __restrict__ cnt7) {
  __shared__ double wred[16][8];
  const int lane = threadIdx.x % IBM_WAVE, wid = threadIdx.x / IBM_WAVE, nw = blockDim.x / IBM_WAVE;
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int e = threadIdx.x; e < npart; e += blockDim.x) {
    const double2 a = reinterpret_cast<const double2*>(part)[2 * e];
    const double2 b = reinterpret_cast<const double2*>(part)[2 * e + 1];
    acc[0] += a.x;
    acc[1] += a.y;
    acc[2] += b.x;
    acc[3] += b.y;
  }
  if (sd_out)
    for (int e = threadIdx.x; e < nsd; e += blockDim.x) {
      const double2 a = reinterpret_cast<const double2*>(part_sd)[2 * e];
      const double b = part_sd[4 * e + 2];
      acc[4] += a.x;
      acc[5] += a.y;
      acc[6] += b;
    }
#pragma unroll
  for (int q = 0; q < 7; ++q) acc[q] = wave_sum(acc[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < 7; ++q) wred[wid][q] = acc[q];
  __syncthreads();
  if (threadIdx.x < 7) {
    const int q = threadIdx.x;
    double t = wred[0][q];
    for (int w = 1; w < nw; ++w) t += wred[w][q];
    wred[0][q] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double c0 = wred[0][0];
    if (cnt7) c0 += (double)(cnt7[0] - cnt7[4]);
    for (int k = 0; k < 3; ++k) {
      const double ckdt = rk_c(k) * scale;   // scale carries dt dy dz / nx
      S3[k] = (c0 + wred[0][1 + k]) * ckdt;
      if (sd_out) sd_out[k] = wred[0][4 + k];
    }
  }
}
__global__ __launch_bounds__(1024) void k_s_final(const double* __restrict__ part, int npart, double scale,
                                                 double* __restrict__ S3, const double* __restrict__ part_sd,
                                                 int nsd, double* __restrict__ sd_out,
                                                 const int32_t* __restrict__ cnt7) {
  s_final_block(part, npart, scale, S3, part_sd, nsd, sd_out, cnt7);
}

// Per entry of the three immersed-boundary lists (laid end to end: v at n_u, w at
// n_u + n_v; entries beyond each list's count are skipped): its lambda and sigma from the
// signed distances around it (arm_pair over the six arms, Eq. (7)) into lam and L.sig,
// and its per-stage (B, 1/A) into coef[k * n_total + entry].  The first nb2 blocks, which hold the whole
// u list, also write the S_k partials of their u points: per stage the sum of 1/A_k
// (weighted by the row's cell height on a stretched grid) into part[block * 4 + 1 + k], and
// of sigma/A_k (the flow rate a moving wall adds, per unit c_k dt U_b) into
// part_sd[block * 4 + k].
// With fin.done (uniform grids), the last of those blocks to finish also forms S_k from
// every partial (s_final_block): each block writes its partials, makes them visible to
// the device and counts itself in *fin.done; the block that counts last reads them all
// and sets the counter back to zero for the next launch.
struct SFinal {
  unsigned* done;
  double scale;
  double* S3;
  double* sd_out;
  const int32_t* cnt7;
};
__global__ __launch_bounds__(256) void k_list_coef(GridParams g, IbmLists L, const double* __restrict__ su,
                                                  const double* __restrict__ sv, const double* __restrict__ sw,
                                                  double* __restrict__ lam, double* __restrict__ sig,
                                                  double2* __restrict__ coef, double dt, int b_mode, int nb2,
                                                  double* __restrict__ part, double* __restrict__ part_sd,
                                                  SFinal fin) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int cmp = e < L.n_u ? 0 : (e < L.n_u + L.n_v ? 1 : 2);
  const int off = cmp == 0 ? 0 : (cmp == 1 ? L.n_u : L.n_u + L.n_v);
  const int cap = cmp == 0 ? L.n_u : (cmp == 1 ? L.n_v : L.n_w);
  const bool valid = e < L.n_total && e - off < min(L.cnt[cmp], cap);
  double2 cf[3];
  double sg = 0.0;
  if (valid) {
    const unsigned cell = (unsigned)L.idx[e], nx = g.nx, nz = g.nz;
    const unsigned row = cell / nx, i = cell - row * nx, j = row / nz, k = row - j * nz;
    double d[7];
    samples7(g, cmp == 0 ? su : (cmp == 1 ? sv : sw), cmp, (int)i, (int)k, (int)j, d);
    const YArms ya = y_arms(g, cmp, (int)j);
    const double nu = g.nu;
    const double dx2 = 1.0 / (g.dx * g.dx), dz2 = 1.0 / (g.dz * g.dz);
    double l = 0.0;
    arm_pair(nu, g.dx, dx2, d[0], d[1], d[1] <= 0.0, INFINITY, l, sg);
    arm_pair(nu, g.dx, dx2, d[0], d[2], d[2] <= 0.0, INFINITY, l, sg);
    arm_pair(nu, g.dz, dz2, d[0], d[3], d[3] <= 0.0, INFINITY, l, sg);
    arm_pair(nu, g.dz, dz2, d[0], d[4], d[4] <= 0.0, INFINITY, l, sg);
    arm_pair(nu, ya.hdn, ya.cdn, d[0], d[5], ya.gdn || d[5] <= 0.0, ya.bdn, l, sg);
    arm_pair(nu, ya.hup, ya.cup, d[0], d[6], ya.gup || d[6] <= 0.0, ya.bup, l, sg);
    lam[e] = l;
    sig[e] = sg;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cf[k] = ibm_stage_coef(l, k, dt, b_mode);
      coef[(size_t)k * L.n_total + e] = cf[k];
    }
  }
  if ((int)blockIdx.x >= nb2) return;   // (the whole block)
  const bool in = valid && cmp == 0;
  // a stretched grid weights each point by the cell height of its row
  const double wy = (g.stretched && in) ? g.ytab[YT_DYC * g.ystr + L.idx[e] / (g.nx * g.nz)] : 1.0;
  double v[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = in ? cf[k].y * wy : 0.0;
  // the six sums reduced over each wave, then over the block's four waves (fixed order)
  __shared__ double wred[4][6];
  const int lane = threadIdx.x % IBM_WAVE, wid = threadIdx.x / IBM_WAVE;
  double r[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r[k] = wave_sum(v[k]);
    r[3 + k] = wave_sum(sg * v[k]);
  }
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < 6; ++q) wred[wid][q] = r[q];
  __syncthreads();
  __shared__ int last;
  if (threadIdx.x == 0) {
    double t[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) t[q] = ((wred[0][q] + wred[1][q]) + wred[2][q]) + wred[3][q];
    part[blockIdx.x * 4] = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      part[blockIdx.x * 4 + 1 + q] = t[q];
      part_sd[blockIdx.x * 4 + q] = t[3 + q];
    }
    part_sd[blockIdx.x * 4 + 3] = 0.0;
    last = 0;
    if (fin.done) {
      __threadfence();   // the partials visible device-wide before the count
      last = atomicAdd(fin.done, 1u) == (unsigned)(nb2 - 1);
    }
  }
  __syncthreads();
  if (!last) return;
  __threadfence();       // every block's partials visible here
  s_final_block(part, nb2, fin.scale, fin.S3, part_sd, nb2, fin.sd_out, fin.cnt7);
  if (threadIdx.x == 0) fin.done[0] = 0u;
}
// ---------------------------------------------------------------------------------------
// Diagnostics
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double fval(const T* a, int c) { return (double)a[c]; }

// Full-box divergence after the projection and before external faces are reset, the
// Poisson residual D G phi - (rhs - mean) and max |rhs|.  part: [block][3] (max).
template <typename T>
__global__ __launch_bounds__(256) void k_diag(GridParams g, Fields<T> f, IbmLists L, int stage, double ck_dt,
                                             const double* __restrict__ pi, const double* __restrict__ mean,
                                             double* __restrict__ part) {
  __shared__ double red[4];
  const int i = blockIdx.x * BX + threadIdx.x;
  const int k = blockIdx.y * BZ + threadIdx.y;
  const int j = blockIdx.z;
  const int lane = threadIdx.x;
  const int nx = g.nx, nz = g.nz, plane = nx * nz;
  const bool act = (i < nx) && (k < nz);
  const int row = j * nz + k;
  const int c = act ? row * nx + i : 0;
  (void)L;
  (void)stage;
  (void)lane;
  const double pk = pi[0] * ck_dt;
  // u* on the west and east faces (immersed-boundary faces already hold their response)
  auto ust = [&](int cc) {
    const uint8_t t = f.tag[cc];
    return fval(f.us, cc) - (((t & (TAG_U | TAG_UI)) == TAG_U) ? pk : 0.0);
  };
  double uw = 0.0, ue = 0.0;
  if (act) {
    uw = ust(c);
    ue = ust(row * nx + wrap_p(i, nx));
  }
  double dmax = 0.0, rmax = 0.0, hmax = 0.0;
  if (act) {
    const int ip = wrap_p(i, nx), im = wrap_m(i, nx), kp = wrap_p(k, nz), km = wrap_m(k, nz);
    const bool hasN = j + 1 < g.ny1, hasS = j > 0;
    const double ph = fval(f.phi, c);
    const double phe = fval(f.phi, c - i + ip), phw = fval(f.phi, c - i + im);
    const double pht = fval(f.phi, c + (kp - k) * nx), phb = fval(f.phi, c + (km - k) * nx);
    const double phn = hasN ? fval(f.phi, c + plane) : 0.0, phs = hasS ? fval(f.phi, c - plane) : 0.0;
    const double vs = fval(f.vs, c), vn = hasN ? fval(f.vs, c + plane) : 0.0;
    const double wb = fval(f.ws, c), wt = fval(f.ws, c + (kp - k) * nx);
    // gradients of phi on the faces (no flux through the box walls); a stretched grid
    // takes the spacings of face j, face j+1 and cell j
    double iys = g.idy, iyn = g.idy, iyc = g.idy;
    if (g.stretched) {
      iys = g.ytab[YT_IDYF * g.ystr + j];
      iyn = g.ytab[YT_IDYF * g.ystr + j + 1];
      iyc = g.ytab[YT_IDYC * g.ystr + j];
    }
    const double gxw = (ph - phw) * g.idx, gxe = (phe - ph) * g.idx;
    const double gys = hasS ? (ph - phs) * iys : 0.0, gyn = hasN ? (phn - ph) * iyn : 0.0;
    const double gzb = (ph - phb) * g.idz, gzt = (pht - ph) * g.idz;
    const double divs = (ue - uw) * g.idx + (vn - vs) * iyc + (wt - wb) * g.idz;
    const double rhs = divs / ck_dt;
    const double dg = (gxe - gxw) * g.idx + (gyn - gys) * iyc + (gzt - gzb) * g.idz;
    dmax = fabs(divs - ck_dt * dg);
    rmax = fabs(dg - (rhs - mean[0]));
    hmax = fabs(rhs);
  }
  const double a = block_reduce<true>(dmax, red);
  __syncthreads();
  const double b = block_reduce<true>(rmax, red);
  __syncthreads();
  const double cmax = block_reduce<true>(hmax, red);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    part[bid * 3 + 0] = a;
    part[bid * 3 + 1] = b;
    part[bid * 3 + 2] = cmax;
  }
}

// State statistics. part: [block][6] = (sum u over internal u, sum |u|^2, nan count,
//                                      max cfl, max |D u| over internal p, 0)
template <typename T>
__global__ __launch_bounds__(256) void k_stats(GridParams g, Fields<T> f, double* __restrict__ part) {
  __shared__ double red[4];
  const int i = blockIdx.x * BX + threadIdx.x;
  const int k = blockIdx.y * BZ + threadIdx.y;
  const int j = blockIdx.z;
  double qs = 0.0, ke = 0.0, nan = 0.0, cfl = 0.0, leak = 0.0;
  if (i < g.nx && k < g.nz) {
    const int nx = g.nx, nz = g.nz, plane = nx * nz;
    const int ip = wrap_p(i, nx), kp = wrap_p(k, nz);
    const int c = (j * nz + k) * nx + i;
    const uint8_t t = f.tag[c];
    const double u = fval(f.u, c), v = fval(f.v, c), w = fval(f.w, c), p = fval(f.p, c);
    // a stretched grid weights the sums by the cell height and takes it as the spacing
    const double iyc = g.stretched ? g.ytab[YT_IDYC * g.ystr + j] : g.idy;
    const double wy = g.stretched ? g.ytab[YT_DYC * g.ystr + j] : 1.0;
    if (t & TAG_U) qs = g.stretched ? u * wy : u;
    ke = u * u + v * v + w * w;
    if (g.stretched) ke *= wy;
    nan = (isfinite(u) && isfinite(v) && isfinite(w) && isfinite(p)) ? 0.0 : 1.0;
    cfl = (fabs(u) * g.idx + fabs(v) * iyc + fabs(w) * g.idz) * g.dt;
    if (t & TAG_P) {
      const double ue = fval(f.u, c - i + ip);
      const double vn = (j + 1 < g.ny1) ? fval(f.v, c + plane) : 0.0;
      const double wt = fval(f.w, c + (kp - k) * nx);
      leak = fabs((ue - u) * g.idx + (vn - v) * iyc + (wt - w) * g.idz);
    }
  }
  const double a = block_reduce<false>(qs, red);
  __syncthreads();
  const double b = block_reduce<false>(ke, red);
  __syncthreads();
  const double cc = block_reduce<false>(nan, red);
  __syncthreads();
  const double d = block_reduce<true>(isfinite(cfl) ? cfl : 1e300, red);
  __syncthreads();
  const double e = block_reduce<true>(isfinite(leak) ? leak : 1e300, red);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    double* o = part + bid * 6;
    o[0] = a;
    o[1] = b;
    o[2] = cc;
    o[3] = d;
    o[4] = e;
    o[5] = 0.0;
  }
}

// Column-wise reduction of part[npart][nsum + nmax]: sums then maxima.  One block per column.
__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ part, int npart, int nsum,
                                                     int nmax, double* __restrict__ out) {
  __shared__ double red[4];
  const int col = blockIdx.x;
  const int nc = nsum + nmax;
  const bool ismax = col >= nsum;
  double s = 0.0;
  for (int e = threadIdx.x; e < npart; e += blockDim.x) {
    const double v = part[(size_t)e * nc + col];
    s = ismax ? fmax(s, v) : s + v;
  }
  const double r = ismax ? block_reduce<true>(s, red) : block_reduce<false>(s, red);
  if (threadIdx.x == 0) out[col] = r;
}

// Spanwise-averaged wall-shear stress tau(x_i) at the south wall (Sec. 4.2): the viscous
// flux the discretisation exchanges with the wall through the cut stencil arm below the
// lowest internal point, nu u1 / d1 (the ghost value is the linear extrapolation through
// zero at the wall, Eqs. (5)-(7)).  Block (64, 16): x lanes, 16 rows of z columns summed
// in a fixed order.
constexpr int WS_Z = 16;
template <typename T>
__global__ __launch_bounds__(BX * WS_Z) void k_wall_shear(GridParams g, const T* __restrict__ u,
                                                         const int32_t* __restrict__ wj,
                                                         const double* __restrict__ wd,
                                                         const double* __restrict__ wallv,
                                                         double* __restrict__ tau_x) {
  __shared__ double red[WS_Z][BX];
  const int i = blockIdx.x * BX + threadIdx.x;
  const size_t plane = (size_t)g.nx * g.nz;
  double acc = 0.0;
  if (i < g.nx) {
    for (int k = threadIdx.y; k < g.nz; k += WS_Z) {
      const int col = k * g.nx + i;
      const int j1 = wj[col];
      if (j1 >= 0) {
        const double dw = wd[col];
        const double ub = dw < 0.0 ? 0.0 : wallv[0];   // the immersed wall may slide
        acc += ((double)u[(size_t)j1 * plane + col] - ub) / fabs(dw);
      }
    }
  }
  red[threadIdx.y][threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.y == 0 && i < g.nx) {
    double sum = 0.0;
    for (int r = 0; r < WS_Z; ++r) sum += red[r][threadIdx.x];
    tau_x[i] = g.nu * sum / g.nz;
  }
}

// Mean and first Fourier components over the box length of tau(x_i), x_i = i dx:
// out = (sum tau / nx, (2/nx) sum tau cos(2 pi i/nx), (2/nx) sum tau sin(2 pi i/nx)).
__global__ __launch_bounds__(256) void k_tau_modes(const double* __restrict__ tau_x, int nx,
                                                  double* __restrict__ out) {
  __shared__ double red[4];
  double s0 = 0.0, sc = 0.0, ss = 0.0;
  for (int i = threadIdx.x; i < nx; i += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)i / (double)nx, &sn, &cs);
    const double t = tau_x[i];
    s0 += t;
    sc += t * cs;
    ss += t * sn;
  }
  const double r0 = block_reduce<false>(s0, red);
  __syncthreads();
  const double rc = block_reduce<false>(sc, red);
  __syncthreads();
  const double rs = block_reduce<false>(ss, red);
  if (threadIdx.x == 0) {
    out[0] = r0 / nx;
    out[1] = 2.0 * rc / nx;
    out[2] = 2.0 * rs / nx;
  }
}

}  // namespace

static inline dim3 cell_grid(const GridParams& g) {
  return dim3((g.nx + BX - 1) / BX, (g.nz + BZ - 1) / BZ, g.ny1);
}

template <typename T>
hipError_t launch_geom_tags(const GridParams& g, const double* su, const double* sv, const double* sw, int ibm_on,
                            uint8_t* tag, bool correct, const Fields<T>& f, const double* wallv, double ck_dt,
                            const double* pi, int32_t* wj, double* wd, int32_t* counts, int32_t* clear,
                            hipStream_t st) {
  if (correct && (!f.us || !f.vs || !f.ws || !f.pp || !f.phi || !wallv || !pi)) return hipErrorInvalidValue;
  if (!wj || !wd || !counts || !clear) return hipErrorInvalidValue;
  const dim3 grid((g.nx + BX - 1) / BX, (g.nz + BZ - 1) / BZ, (g.ny1 + TAG_JC - 1) / TAG_JC);
  hipLaunchKernelGGL(k_geom_tags<T>, grid, dim3(BX, BZ), 0, st, g, su, sv, sw, ibm_on, tag, correct ? 1 : 0, f,
                     wallv, ck_dt, pi, wj, wd, counts, clear);
  return hipGetLastError();
}
template hipError_t launch_geom_tags<double>(const GridParams&, const double*, const double*, const double*, int,
                                             uint8_t*, bool, const Fields<double>&, const double*, double,
                                             const double*, int32_t*, double*, int32_t*, int32_t*, hipStream_t);
template hipError_t launch_geom_tags<float>(const GridParams&, const double*, const double*, const double*, int,
                                            uint8_t*, bool, const Fields<float>&, const double*, double,
                                            const double*, int32_t*, double*, int32_t*, int32_t*, hipStream_t);



template <typename T>
hipError_t launch_wall_shear(const GridParams& g, const T* u, const int32_t* wj, const double* wd,
                             const double* wallv, double* tau_x, double* modes, hipStream_t st) {
  hipLaunchKernelGGL(k_wall_shear<T>, dim3((g.nx + BX - 1) / BX), dim3(BX, WS_Z), 0, st, g, u, wj, wd, wallv,
                     tau_x);
  if (modes) hipLaunchKernelGGL(k_tau_modes, dim3(1), dim3(256), 0, st, tau_x, g.nx, modes);
  return hipGetLastError();
}
template hipError_t launch_wall_shear<double>(const GridParams&, const double*, const int32_t*, const double*,
                                              const double*, double*, double*, hipStream_t);
template hipError_t launch_wall_shear<float>(const GridParams&, const float*, const int32_t*, const double*,
                                             const double*, double*, double*, hipStream_t);

hipError_t launch_scan_multi(ScanSet set, hipStream_t st) {
  if (set.narr < 1 || set.narr > SCAN_MAX || !set.tsum) return hipErrorInvalidValue;
  set.tile_off[0] = 0;
  for (int m = 0; m < set.narr; ++m) {
    if (set.n[m] < 0) return hipErrorInvalidValue;
    set.tile_off[m + 1] = set.tile_off[m] + scan_tiles(set.n[m]);
  }
  const int ntile = set.tile_off[set.narr];
  if (ntile > set.tsum_cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(ntile), dim3(1024), 0, st, set);
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntile), dim3(1024), 0, st, set);
  return hipGetLastError();
}

hipError_t launch_compact3(const uint8_t* tag, const GridParams& g, int cpr, const int32_t* off_u,
                           const int32_t* off_v, const int32_t* off_w, int32_t* idx, const int cap[3],
                           int32_t* overflow, void* zphi, int zelem, double* zpi, hipStream_t st) {
  const int nchunk = g.nrows * cpr;
  hipLaunchKernelGGL(k_compact3, dim3((nchunk + 3) / 4), dim3(256), 0, st, tag, g.nx, g.nrows, cpr, off_u, off_v,
                     off_w, idx, cap[0], cap[0] + cap[1], cap[0], cap[1], cap[2], overflow, (unsigned char*)zphi,
                     zelem, zpi);
  return hipGetLastError();
}



hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t st) {
  if (bytes <= 0) return hipSuccess;
  const int64_t nvec = ((uintptr_t)p % 16 == 0) ? bytes / 16 : 0;
  const int64_t nb = nvec > 0 ? (nvec + 255) / 256 : 1;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)nb), dim3(256), 0, st, (unsigned char*)p, nvec, bytes);
  return hipGetLastError();
}

hipError_t launch_s_k(const GridParams& g, const uint8_t* tag, const IbmLists& L, const double* su, const double* sv,
                      const double* sw, double* lam, double* sig, double2* coef, double dt, int b_mode, double* part,
                      double scale, double* S3, const int32_t* cnt7, double* sd_out, unsigned* done, hipStream_t st) {
  // (on a uniform grid the internal non-IBM u points are counted by the tag counts, which
  // the final sums read; a stretched grid weights them by row and sums them here)
  const int nb1 = g.stretched ? (int)((g.ncell + 255) / 256) : 0;
  const int nb2 = (L.n_u + 255) / 256;
  const int nbl = (L.n_total + 255) / 256;
  double* part_sd = part + (size_t)(nb1 + nb2) * 4;
  // the final sums in the list kernel's last block on a uniform grid with listed u points;
  // otherwise (the stretched grid's many cell partials, no u list) by a block of their own
  const bool fused = nb1 == 0 && nb2 > 0 && done;
  SFinal fin{};
  if (fused) fin = SFinal{done, scale, S3, sd_out, cnt7};
  if (nb1 > 0) hipLaunchKernelGGL(k_s_cells, dim3(nb1), dim3(256), 0, st, g, tag, part);
  if (nbl > 0)
    hipLaunchKernelGGL(k_list_coef, dim3(nbl), dim3(256), 0, st, g, L, su, sv, sw, lam, sig, coef, dt, b_mode, nb2,
                       part + (size_t)nb1 * 4, part_sd, fin);
  if (!fused)
    hipLaunchKernelGGL(k_s_final, dim3(1), dim3(1024), 0, st, part, nb1 + nb2, scale, S3, part_sd, nb2, sd_out,
                       g.stretched ? nullptr : cnt7);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_diag(const GridParams& g, const Fields<T>& f, const IbmLists& L, int stage, double ck_dt,
                       const double* pi, const double* mean, double* part, int* npart, hipStream_t st) {
  const dim3 grid = cell_grid(g);
  hipLaunchKernelGGL(k_diag<T>, grid, dim3(BX, BZ), 0, st, g, f, L, stage, ck_dt, pi, mean, part);
  *npart = grid.x * grid.y * grid.z;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stats(const GridParams& g, const Fields<T>& f, double* part, int* npart, hipStream_t st) {
  const dim3 grid = cell_grid(g);
  hipLaunchKernelGGL(k_stats<T>, grid, dim3(BX, BZ), 0, st, g, f, part);
  *npart = grid.x * grid.y * grid.z;
  return hipGetLastError();
}

hipError_t launch_reduce_final(const double* part, int npart, int nsum, int nmax, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_final, dim3(nsum + nmax), dim3(256), 0, st, part, npart, nsum, nmax, out);
  return hipGetLastError();
}

template hipError_t launch_diag<double>(const GridParams&, const Fields<double>&, const IbmLists&, int, double,
                                        const double*, const double*, double*, int*, hipStream_t);
template hipError_t launch_diag<float>(const GridParams&, const Fields<float>&, const IbmLists&, int, double,
                                       const double*, const double*, double*, int*, hipStream_t);
template hipError_t launch_stats<double>(const GridParams&, const Fields<double>&, double*, int*, hipStream_t);
template hipError_t launch_stats<float>(const GridParams&, const Fields<float>&, double*, int*, hipStream_t);
