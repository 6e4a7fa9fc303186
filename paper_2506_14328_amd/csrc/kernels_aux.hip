// Geometry preprocessing (Sec. 2.2, Sec. 2.4, Sec. 3.3) and diagnostics.
#include "ibm_internal.h"

namespace {

constexpr int BX = 64;
constexpr int BZ = 4;

__device__ __forceinline__ int wrap_p(int i, int n) { return (i + 1 == n) ? 0 : i + 1; }
__device__ __forceinline__ int wrap_m(int i, int n) { return (i == 0) ? n - 1 : i - 1; }

// Contribution nu (h - delta)/(delta h^2) of one arm whose neighbour is external
// (Eq. (7) with d2(-1) = 1/h^2); delta = linear zero crossing of the signed distance
// between the point and the neighbour, or the box wall distance when that is nearer.
__device__ __forceinline__ double arm(double nu, double h, double sP, double sQ, bool extQ, double box) {
  if (!extQ) return 0.0;
  double delta = (sQ <= 0.0) ? h * sP / (sP - sQ) : INFINITY;
  delta = fmin(delta, box);
  return nu * (h - delta) / (delta * h * h);
}

// The same with the arm's own second-derivative coefficient d2 (stretched wall-normal
// arms): nu d2 (h - delta)/delta.
__device__ __forceinline__ double arm_w(double nu, double h, double d2, double sP, double sQ, bool extQ,
                                        double box) {
  if (!extQ) return 0.0;
  double delta = (sQ <= 0.0) ? h * sP / (sP - sQ) : INFINITY;
  delta = fmin(delta, box);
  return nu * d2 * (h - delta) / delta;
}

// Coefficient of the wall velocity U_b in the correction of one arm whose neighbour is
// external (a rigidly moving immersed wall; the ghost is extrapolated through U_b): 0 when
// the nearer wall is a box wall (at rest); lambda_arm when the neighbour stores U_b (an
// external point inside the box, box = infinity); nu/(delta h) when it stores zero (the
// box-wall face or the ghost beyond it, box finite).
__device__ __forceinline__ double arm_src(double nu, double h, double sP, double sQ, bool extQ, double box) {
  if (!extQ || !(sQ <= 0.0)) return 0.0;
  const double delta = h * sP / (sP - sQ);
  if (!(delta < box)) return 0.0;
  return isinf(box) ? nu * (h - delta) / (delta * h * h) : nu / (delta * h);
}
__device__ __forceinline__ double arm_src_w(double nu, double h, double d2, double sP, double sQ, bool extQ,
                                            double box) {
  if (!extQ || !(sQ <= 0.0)) return 0.0;
  const double delta = h * sP / (sP - sQ);
  if (!(delta < box)) return 0.0;
  return isinf(box) ? nu * d2 * (h - delta) / delta : nu * d2 * h / delta;
}

// Tags of u, v, w and lambda per component at every cell (j, k, i); with sig_* not null
// also the wall-velocity coefficient sigma per component.
//  sdf_u, sdf_w: (ny+1, nz, nx), row jj = j+1 holds row j; sdf_v: (ny, nz, nx) faces.
// With zphi not null the cell's phi (zelem bytes) is zeroed too, and with zpi the mean
// pressure gradient: what is pending of a projection that was applied just before.
__global__ __launch_bounds__(256) void k_geom_lambda(GridParams g, const double* __restrict__ su,
                                                    const double* __restrict__ sv, const double* __restrict__ sw,
                                                    int ibm_on, uint8_t* __restrict__ tag,
                                                    double* __restrict__ lam_u, double* __restrict__ lam_v,
                                                    double* __restrict__ lam_w, double* __restrict__ sig_u,
                                                    double* __restrict__ sig_v, double* __restrict__ sig_w,
                                                    unsigned char* __restrict__ zphi, int zelem,
                                                    double* __restrict__ zpi) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int k = blockIdx.y * BZ + threadIdx.y;
  const int j = blockIdx.z;
  if (i >= g.nx || k >= g.nz) return;
  const int nx = g.nx, nz = g.nz, ny1 = g.ny1;
  const int ip = wrap_p(i, nx), im = wrap_m(i, nx), kp = wrap_p(k, nz), km = wrap_m(k, nz);
  const int plane = nx * nz;
  const int c = (j * nz + k) * nx + i;
  if (zphi) {
    if (zelem == 8) reinterpret_cast<double*>(zphi)[c] = 0.0;
    else reinterpret_cast<float*>(zphi)[c] = 0.0f;
  }
  if (zpi && c == 0) zpi[0] = 0.0;
  const double nu = g.nu, dx = g.dx, dy = g.dy, dz = g.dz;
  const bool sy = g.stretched != 0;
  const double* yt = g.ytab;
  const int ys = g.ystr;
  // wall-normal arms: uniform spacing dy, or the row's own spacing and coefficient
  auto yarm = [&](double h, double d2, double sP, double sQ, bool ext, double box) {
    return sy ? arm_w(nu, h, d2, sP, sQ, ext, box) : arm(nu, h, sP, sQ, ext, box);
  };
  auto ysrc = [&](double h, double d2, double sP, double sQ, bool ext, double box) {
    return sy ? arm_src_w(nu, h, d2, sP, sQ, ext, box) : arm_src(nu, h, sP, sQ, ext, box);
  };
  uint8_t t = 0;
  // u and w: sample row jj = j + 1; ghost rows jj = 0 and jj = ny are outside the box.
  for (int comp = 0; comp < 3; comp += 2) {
    const double* s = comp == 0 ? su : sw;
    const int o = (j + 1) * plane + k * nx;
    const double sP = s[o + i];
    double lam = 0.0, sg = 0.0;
    const bool in = sP > 0.0;
    if (in) {
      const double sxm = s[o + im], sxp = s[o + ip];
      const double szm = s[o + (km - k) * nx + i], szp = s[o + (kp - k) * nx + i];
      const double sdn = s[o - plane + i], sup = s[o + plane + i];
      // the south box face is a wall; so is the north one unless it is free-slip
      const bool gdn = (j == 0), gup = (j == ny1 - 1) && !g.top_fs;
      double hdn = dy, hup = dy, cdn = 0.0, cup = 0.0, bdn = 0.5 * dy, bup = 0.5 * dy;
      if (sy) {
        hdn = yt[YT_HC * ys + j];
        hup = yt[YT_HC * ys + j + 1];
        cdn = yt[YT_DCM * ys + j];
        cup = yt[YT_DCP * ys + j];
        bdn = 0.5 * yt[YT_DYC * ys];
        bup = 0.5 * yt[YT_DYC * ys + ny1 - 1];
      }
      lam += arm(nu, dx, sP, sxm, sxm <= 0.0, INFINITY);
      lam += arm(nu, dx, sP, sxp, sxp <= 0.0, INFINITY);
      lam += arm(nu, dz, sP, szm, szm <= 0.0, INFINITY);
      lam += arm(nu, dz, sP, szp, szp <= 0.0, INFINITY);
      lam += yarm(hdn, cdn, sP, sdn, gdn || sdn <= 0.0, gdn ? bdn : INFINITY);
      lam += yarm(hup, cup, sP, sup, gup || sup <= 0.0, gup ? bup : INFINITY);
      sg += arm_src(nu, dx, sP, sxm, sxm <= 0.0, INFINITY);
      sg += arm_src(nu, dx, sP, sxp, sxp <= 0.0, INFINITY);
      sg += arm_src(nu, dz, sP, szm, szm <= 0.0, INFINITY);
      sg += arm_src(nu, dz, sP, szp, szp <= 0.0, INFINITY);
      sg += ysrc(hdn, cdn, sP, sdn, gdn || sdn <= 0.0, gdn ? bdn : INFINITY);
      sg += ysrc(hup, cup, sP, sup, gup || sup <= 0.0, gup ? bup : INFINITY);
      if (!ibm_on) lam = sg = 0.0;
      t |= (comp == 0) ? TAG_U : TAG_W;
      if (lam > 0.0) t |= (comp == 0) ? TAG_UI : TAG_WI;
    }
    // (stored at immersed-boundary points only: the coefficient kernel reads these arrays
    // at the points of its lists, and skipping the rest saves most of this kernel's writes)
    if (lam > 0.0) {
      (comp == 0 ? lam_u : lam_w)[c] = lam;
      (comp == 0 ? sig_u : sig_w)[c] = sg;
    }
  }
  // v on face j; faces 0 and ny-1 are the box walls.
  {
    const int o = j * plane + k * nx;
    const double sP = sv[o + i];
    double lam = 0.0, sg = 0.0;
    if (j >= 1 && sP > 0.0) {
      const double sxm = sv[o + im], sxp = sv[o + ip];
      const double szm = sv[o + (km - k) * nx + i], szp = sv[o + (kp - k) * nx + i];
      const double sdn = sv[o - plane + i], sup = sv[o + plane + i];
      const bool wdn = (j - 1 == 0), wup = (j + 1 == ny1);
      // face j lies between cells j-1 and j
      double hdn = dy, hup = dy, cdn = 0.0, cup = 0.0;
      if (sy) {
        hdn = yt[YT_DYC * ys + j - 1];
        hup = yt[YT_DYC * ys + j];
        cdn = yt[YT_DFM * ys + j];
        cup = yt[YT_DFP * ys + j];
      }
      lam += arm(nu, dx, sP, sxm, sxm <= 0.0, INFINITY);
      lam += arm(nu, dx, sP, sxp, sxp <= 0.0, INFINITY);
      lam += arm(nu, dz, sP, szm, szm <= 0.0, INFINITY);
      lam += arm(nu, dz, sP, szp, szp <= 0.0, INFINITY);
      lam += yarm(hdn, cdn, sP, sdn, wdn || sdn <= 0.0, wdn ? hdn : INFINITY);
      lam += yarm(hup, cup, sP, sup, wup || sup <= 0.0, wup ? hup : INFINITY);
      sg += arm_src(nu, dx, sP, sxm, sxm <= 0.0, INFINITY);
      sg += arm_src(nu, dx, sP, sxp, sxp <= 0.0, INFINITY);
      sg += arm_src(nu, dz, sP, szm, szm <= 0.0, INFINITY);
      sg += arm_src(nu, dz, sP, szp, szp <= 0.0, INFINITY);
      sg += ysrc(hdn, cdn, sP, sdn, wdn || sdn <= 0.0, wdn ? hdn : INFINITY);
      sg += ysrc(hup, cup, sP, sup, wup || sup <= 0.0, wup ? hup : INFINITY);
      if (!ibm_on) lam = sg = 0.0;
      t |= TAG_V;
      if (lam > 0.0) t |= TAG_VI;
    }
    if (lam > 0.0) {
      lam_v[c] = lam;
      sig_v[c] = sg;
    }
  }
  tag[c] = t;
}

// Pressure cell internal iff one of its six faces is an internal velocity point; then, per
// block of 256 consecutive cells, the number of cells with each of nm tag masks set (mask
// m in bits 8m..8m+7 of masks): counts[m * nblk + block]; block 0 also zeroes *clear (the
// lists' overflow flag, by a kernel so that a geometry update can be captured).  A
// neighbour's tag may gain its pressure bit while it is read here; only its velocity bits,
// which no thread changes, are used.
// With chunks not null (rows of whole 64-wide chunks: nx a multiple of 64) it also
// writes the per-(row, chunk) counts of the three immersed-boundary masks, laid out as
// k_chunk_counts3 writes them (wave w of block b is chunk 4b + w).
__global__ __launch_bounds__(256) void k_geom_ptag_counts(GridParams g, uint8_t* __restrict__ tag, uint64_t masks,
                                                         int nm, int32_t* __restrict__ counts, int nblk,
                                                         int32_t* __restrict__ clear, int32_t* __restrict__ chunks) {
  __shared__ int32_t wc[8][4];
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  uint8_t t = 0;
  if (e < g.ncell) {
    const int nx = g.nx, nz = g.nz;
    const int i = (int)(e % nx), k = (int)((e / nx) % nz), j = (int)(e / ((int64_t)nx * nz));
    t = tag[e];
    const uint8_t te = tag[e - i + wrap_p(i, nx)] & TAG_U;
    const uint8_t tn = (j + 1 < g.ny1) ? (tag[e + (int64_t)nx * nz] & TAG_V) : 0;
    const uint8_t tt = tag[e + (int64_t)(wrap_p(k, nz) - k) * nx] & TAG_W;
    if ((t & (TAG_U | TAG_V | TAG_W)) || te || tn || tt) {
      t |= TAG_P;
      tag[e] = t;
    }
  }
  if (clear && e == 0) clear[0] = 0;
  const int lane = threadIdx.x % IBM_WAVE, wid = threadIdx.x / IBM_WAVE;
  if (chunks) {
    const int64_t nch = g.ncell / IBM_WAVE + 1;   // whole chunks, and one zero entry
    const int64_t ch = e / IBM_WAVE;              // the same for every lane of the wave
    for (int c = 0; c < 3; ++c) {
      const uint64_t b = __ballot((t & (TAG_UI << c)) != 0);
      if (lane == 0 && ch < nch - 1) chunks[c * nch + ch] = __popcll(b);
      if (e == 0) chunks[c * nch + nch - 1] = 0;
    }
  }
  for (int m = 0; m < nm; ++m) {
    const uint8_t mask = uint8_t((masks >> (8 * m)) & 0xffu);
    const uint64_t b = __ballot((t & mask) != 0);
    if (lane == 0) wc[m][wid] = __popcll(b);
  }
  __syncthreads();
  if ((int)threadIdx.x < nm) {
    const int m = threadIdx.x;
    counts[(size_t)m * nblk + blockIdx.x] = wc[m][0] + wc[m][1] + wc[m][2] + wc[m][3];
  }
}

// South-wall point of every (k, i) column of u points: the lowest internal u row j1 and
// its distance d1 to the wall below, located as the immersed boundary locates it (the
// linear zero crossing of the signed distance towards the external point below, or the
// south box wall dy/2 below row 0 when nearer); without the correction the staircase
// wall is at the external point (dy).  j1 = -1, d1 = 0 for a column with no internal u;
// d1 is stored negative where the wall is the south box wall (at rest).
__global__ __launch_bounds__(256) void k_geom_south_wall(GridParams g, const double* __restrict__ su, int ibm_on,
                                                        int32_t* __restrict__ wj, double* __restrict__ wd) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int k = blockIdx.y * BZ + threadIdx.y;
  if (i >= g.nx || k >= g.nz) return;
  const size_t plane = (size_t)g.nx * g.nz;
  const int col = k * g.nx + i;
  int j1 = -1;
  double sP = 0.0;
  for (int j = 0; j < g.ny1; ++j) {
    const double sj = su[(size_t)(j + 1) * plane + col];   // row j is SDF row j + 1
    if (sj > 0.0) {
      j1 = j;
      sP = sj;
      break;
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

// Exclusive prefix sum of nblk counts in place, total[0] = their sum; one block of 1024
// threads, SCAN_PER * 1024 counts per round: each thread adds SCAN_PER consecutive counts,
// the waves scan their threads' sums with shuffles and one wave scans the 16 wave sums.
constexpr int SCAN_PER = 16;
__device__ __forceinline__ void scan_counts_body(int32_t* __restrict__ counts, int nblk,
                                                 int32_t* __restrict__ total) {
  __shared__ int32_t wsum[16];
  const int tid = threadIdx.x, lane = tid & (IBM_WAVE - 1), wid = tid / IBM_WAVE;
  int32_t carry = 0;
  for (int base = 0; base < nblk; base += SCAN_PER * 1024) {
    const int e0 = base + SCAN_PER * tid;
    int32_t v[SCAN_PER];
    int32_t sum = 0;
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) {
      v[q] = (e0 + q < nblk) ? counts[e0 + q] : 0;
      sum += v[q];
    }
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
    int32_t run = carry + (wid > 0 ? wsum[wid - 1] : 0) + (x - sum);
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) {
      if (e0 + q < nblk) counts[e0 + q] = run;
      run += v[q];
    }
    carry += wsum[15];
    __syncthreads();
  }
  if (tid == 0) total[0] = carry;
}

// The same for several arrays at once: block m scans set.counts[m] (set.n[m] counts) and
// writes its sum to set.total[m].
__global__ __launch_bounds__(1024) void k_scan_multi(ScanSet set) {
  const int m = blockIdx.x;
  scan_counts_body(set.counts[m], set.n[m], set.total[m]);
}

// The ascending cell indices of the u, v and w immersed-boundary points (tag bits
// TAG_UI << c) at their scanned block offsets offsets[c * nblk + block], into the
// component's list, which starts at list_off[c] and holds cap[c] entries; a point whose
// rank reaches the capacity is not written and sets overflow[0].
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

// ... and with each listed point its lambda, sigma (from the dense per-component arrays,
// component c at c * n) and per-stage (B, 1/A): coef[k * cap_total + entry].
__global__ __launch_bounds__(256) void k_compact3(const uint8_t* __restrict__ tag, int64_t n,
                                                 const int32_t* __restrict__ offsets, int nblk,
                                                 int32_t* __restrict__ idx, int off_v, int off_w, int cap_u,
                                                 int cap_v, int cap_w, int32_t* __restrict__ overflow,
                                                 const double* __restrict__ lam_dense,
                                                 const double* __restrict__ sig_dense, double dt, int b_mode,
                                                 double* __restrict__ lam_out, double* __restrict__ sig_out,
                                                 double2* __restrict__ coef) {
  __shared__ int32_t wc[3][4];
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  const uint8_t t = (e < n) ? tag[e] : uint8_t(0);
  const int lane = threadIdx.x % IBM_WAVE, wid = threadIdx.x / IBM_WAVE;
  uint64_t bal[3];
  for (int c = 0; c < 3; ++c) {
    bal[c] = __ballot((t & (TAG_UI << c)) != 0);
    if (lane == 0) wc[c][wid] = __popcll(bal[c]);
  }
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  for (int c = 0; c < 3; ++c) {
    if (!(t & (TAG_UI << c))) continue;
    int base = offsets[(size_t)c * nblk + blockIdx.x];
    for (int w = 0; w < wid; ++w) base += wc[c][w];
    const int r = base + __popcll(bal[c] & below);
    const int cap = c == 0 ? cap_u : (c == 1 ? cap_v : cap_w);
    const int off = c == 0 ? 0 : (c == 1 ? off_v : off_w);
    if (r < cap) {
      const int q = off + r;
      idx[q] = (int32_t)e;
      const double lam = lam_dense[(size_t)c * n + e];
      lam_out[q] = lam;
      sig_out[q] = sig_dense[(size_t)c * n + e];
      const int cap_total = cap_u + cap_v + cap_w;
      for (int k = 0; k < 3; ++k) coef[(size_t)k * cap_total + q] = ibm_stage_coef(lam, k, dt, b_mode);
    } else {
      overflow[0] = 1;
    }
  }
}

// Flagged cells per 64-wide chunk of each grid row for the three immersed-boundary masks:
// counts[c * (nrows cpr + 1) + row * cpr + ch]; one extra zero entry per mask.
__global__ __launch_bounds__(256) void k_chunk_counts3(const uint8_t* __restrict__ tag, int nx, int nrows, int cpr,
                                                      int32_t* __restrict__ counts) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int nch = nrows * cpr + 1;
  if (e >= nch) return;
  if (e == nch - 1) {
    for (int c = 0; c < 3; ++c) counts[c * nch + e] = 0;
    return;
  }
  const int row = e / cpr, ch = e - row * cpr;
  const int a = ch * IBM_WAVE, b = min(a + IBM_WAVE, nx);
  const uint8_t* t = tag + (size_t)row * nx;
  int n0 = 0, n1 = 0, n2 = 0;
  for (int i = a; i < b; ++i) {
    const uint8_t v = t[i];
    n0 += (v & TAG_UI) ? 1 : 0;
    n1 += (v & TAG_VI) ? 1 : 0;
    n2 += (v & TAG_WI) ? 1 : 0;
  }
  counts[e] = n0;
  counts[nch + e] = n1;
  counts[2 * nch + e] = n2;
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
// Per block of IBM u points and stage k: sum of 1/A_k into part, and sum of sigma/A_k (the
// flow rate a moving wall adds, per unit c_k dt U_b) into part_sd.
__global__ __launch_bounds__(256) void k_s_list(GridParams g, IbmLists L, double* __restrict__ part,
                                               double* __restrict__ part_sd) {
  __shared__ double red[4];
  const int e = blockIdx.x * 256 + threadIdx.x;
  // the u list holds cnt[0] points (at most its capacity n_u)
  const bool in = e < min(L.cnt[0], L.n_u);
  const double sg = in ? L.sig[e] : 0.0;
  // a stretched grid weights each point by the cell height of its row
  const double wy = (g.stretched && in) ? g.ytab[YT_DYC * g.ystr + L.idx[e] / (g.nx * g.nz)] : 1.0;
  for (int k = 0; k < 3; ++k) {
    double v = in ? L.coef[(size_t)k * L.n_total + e].y : 0.0;
    if (g.stretched) v *= wy;
    const double tot = block_reduce<false>(v, red);
    __syncthreads();
    const double tsd = block_reduce<false>(sg * v, red);
    if (threadIdx.x == 0) {
      part[blockIdx.x * 4 + 1 + k] = tot;
      part_sd[blockIdx.x * 4 + k] = tsd;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x * 4] = 0.0;
    part_sd[blockIdx.x * 4 + 3] = 0.0;
  }
}
// S3[k] = S_k from the npart partials of part; with sd_out, sd_out[k] = the sum of the nsd
// partials of stage k in part_sd (fixed orders; zero for no partials)
// With cnt7 (uniform grids) the internal non-IBM u points are its internal u count minus
// its immersed-boundary u count (every immersed-boundary u point is internal).
__global__ __launch_bounds__(1024) void k_s_final(const double* __restrict__ part, int npart, double scale,
                                                 double* __restrict__ S3, const double* __restrict__ part_sd,
                                                 int nsd, double* __restrict__ sd_out,
                                                 const int32_t* __restrict__ cnt7) {
  __shared__ double red[16];
  double acc[4];
  for (int v = 0; v < 4; ++v) {
    double s = 0.0;
    for (int e = threadIdx.x; e < npart; e += blockDim.x) s += part[e * 4 + v];
    acc[v] = block_reduce<false>(s, red);
    __syncthreads();
  }
  if (cnt7) acc[0] += (double)(cnt7[0] - cnt7[4]);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) {
      const double ckdt = rk_c(k) * scale;   // scale carries dt dy dz / nx
      S3[k] = (acc[0] + acc[1 + k]) * ckdt;
    }
  }
  if (!sd_out) return;
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int e = threadIdx.x; e < nsd; e += blockDim.x) s += part_sd[e * 4 + k];
    const double r = block_reduce<false>(s, red);
    if (threadIdx.x == 0) sd_out[k] = r;
    __syncthreads();
  }
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

hipError_t launch_geom_lambda(const GridParams& g, const double* su, const double* sv, const double* sw,
                              int ibm_on, uint8_t* tag, double* lam_u, double* lam_v, double* lam_w,
                              double* sig_u, double* sig_v, double* sig_w, void* zphi, int zelem, double* zpi,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_geom_lambda, cell_grid(g), dim3(BX, BZ), 0, st, g, su, sv, sw, ibm_on, tag, lam_u, lam_v,
                     lam_w, sig_u, sig_v, sig_w, (unsigned char*)zphi, zelem, zpi);
  return hipGetLastError();
}

hipError_t launch_geom_ptag_counts(const GridParams& g, uint8_t* tag, uint64_t masks, int nm, int32_t* counts,
                                   int nblk, int32_t* clear, int32_t* chunks, hipStream_t st) {
  if ((int64_t)nblk * 256 < g.ncell || nm > 8 || (chunks && g.nx % IBM_WAVE != 0)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_geom_ptag_counts, dim3(nblk), dim3(256), 0, st, g, tag, masks, nm, counts, nblk, clear,
                     chunks);
  return hipGetLastError();
}

hipError_t launch_geom_south_wall(const GridParams& g, const double* su, int ibm_on, int32_t* wj, double* wd,
                                  hipStream_t st) {
  const dim3 grid((g.nx + BX - 1) / BX, (g.nz + BZ - 1) / BZ, 1);
  hipLaunchKernelGGL(k_geom_south_wall, grid, dim3(BX, BZ), 0, st, g, su, ibm_on, wj, wd);
  return hipGetLastError();
}

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

hipError_t launch_scan_multi(const ScanSet& set, hipStream_t st) {
  if (set.narr < 1 || set.narr > SCAN_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scan_multi, dim3(set.narr), dim3(1024), 0, st, set);
  return hipGetLastError();
}

hipError_t launch_compact3(const uint8_t* tag, int64_t n, const int32_t* offsets, int nblk, int32_t* idx,
                           const int cap[3], int32_t* overflow, const double* lam_dense, const double* sig_dense,
                           double dt, int b_mode, double* lam_out, double* sig_out, double2* coef, hipStream_t st) {
  hipLaunchKernelGGL(k_compact3, dim3(nblk), dim3(256), 0, st, tag, n, offsets, nblk, idx, cap[0], cap[0] + cap[1],
                     cap[0], cap[1], cap[2], overflow, lam_dense, sig_dense, dt, b_mode, lam_out, sig_out, coef);
  return hipGetLastError();
}

hipError_t launch_chunk_counts3(const uint8_t* tag, const GridParams& g, int cpr, int32_t* counts, hipStream_t st) {
  const int n = g.nrows * cpr + 1;
  hipLaunchKernelGGL(k_chunk_counts3, dim3((n + 255) / 256), dim3(256), 0, st, tag, g.nx, g.nrows, cpr, counts);
  return hipGetLastError();
}


hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t st) {
  if (bytes <= 0) return hipSuccess;
  const int64_t nvec = ((uintptr_t)p % 16 == 0) ? bytes / 16 : 0;
  const int64_t nb = nvec > 0 ? (nvec + 255) / 256 : 1;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)nb), dim3(256), 0, st, (unsigned char*)p, nvec, bytes);
  return hipGetLastError();
}

hipError_t launch_s_k(const GridParams& g, const uint8_t* tag, const IbmLists& L, double* part, int* npart,
                      hipStream_t st) {
  // (on a uniform grid the internal non-IBM u points are counted by the tag counts, which
  // k_s_final reads; a stretched grid weights them by row and sums them here)
  const int nb1 = g.stretched ? (int)((g.ncell + 255) / 256) : 0;
  const int nb2 = (L.n_u + 255) / 256;
  double* part_sd = part + (size_t)(nb1 + nb2) * 4;
  if (nb1 > 0) hipLaunchKernelGGL(k_s_cells, dim3(nb1), dim3(256), 0, st, g, tag, part);
  if (nb2 > 0) hipLaunchKernelGGL(k_s_list, dim3(nb2), dim3(256), 0, st, g, L, part + (size_t)nb1 * 4, part_sd);
  *npart = nb1 + nb2;
  return hipGetLastError();
}

hipError_t launch_s_k_final(const double* part, int npart, double scale, double* S3, const GridParams& g,
                            const IbmLists& L, const int32_t* cnt7, double* sd_out, hipStream_t st) {
  const int nb1 = g.stretched ? (int)((g.ncell + 255) / 256) : 0;
  const int nb2 = (L.n_u + 255) / 256;
  const double* part_sd = part + (size_t)(nb1 + nb2) * 4;
  hipLaunchKernelGGL(k_s_final, dim3(1), dim3(1024), 0, st, part, npart, scale, S3, part_sd, nb2, sd_out,
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
