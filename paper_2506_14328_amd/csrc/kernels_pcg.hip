// Masked pressure projection: continuity enforced on the internal pressure cells only,
// with the external velocity faces never corrected (Sec. 3.3 read strictly).  The
// singular system D M G phi = D u* / (c_k dt) over the internal cells (M keeps the
// internal faces) is solved by preconditioned conjugate gradients, the preconditioner
// being the full-box FFT/tridiagonal solve of the projection itself; the full-box
// solution is the starting point.  FP64 only.
//
// On a stretched wall-normal grid the operator's rows carry the cell height dy_j in their
// denominators (not symmetric); the solve is then of the symmetric W A x = W b, W the
// diagonal of cell heights: r holds W (b - A x), the preconditioner takes W^-1 r (rs,
// written where r is), and the operator applied to the direction is W A p.
//
// FP32 storage: the conjugate-gradient vectors stay FP64; the preconditioner (the
// full-box solve in the storage precision) takes an FP32 copy of its input (rs) and returns
// an FP32 z, which is inexact by rounding, so the direction update takes the flexible
// (Polak-Ribiere) beta = r . (z - z_prev) / rho_prev, for which the iteration tolerates a
// preconditioner that varies slightly from one application to the next.
//
// Vectors live on the full cell array; r and p are zero outside the internal cells.
// Every reduction writes one partial per block (at most PCG_NPART blocks, grid-stride
// loops); the kernel that needs the total re-adds the partials in the same fixed order
// in every block, so no extra launch and no atomics are needed and the result is
// deterministic.
#include "ibm_internal.h"

namespace {

constexpr int PT = 256;

__device__ __forceinline__ void decode(const GridParams& g, int c, int& j, int& k, int& i) {
  i = c % g.nx;
  const int r = c / g.nx;
  k = r % g.nz;
  j = r / g.nz;
}

// (D M G x) at cell c with MASKED, else the full-box D G x (every face but the box walls).
// Branch-free: every neighbour is loaded (a neighbour beyond a box wall is replaced by the
// cell itself) and a face that does not count is weighted by 0, so that the loads of
// several cells can be in flight together.
template <bool MASKED>
__device__ __forceinline__ double lap(const GridParams& g, const uint8_t* __restrict__ tag,
                                      const double* __restrict__ x, int c, int j, int k, int i) {
  const int nx = g.nx, nz = g.nz, plane = nx * nz;
  const int cw = c - i + (i == 0 ? nx - 1 : i - 1);
  const int ce = c - i + (i + 1 == nx ? 0 : i + 1);
  const int cb = c + ((k == 0 ? nz - 1 : k - 1) - k) * nx;
  const int cf = c + ((k + 1 == nz ? 0 : k + 1) - k) * nx;
  const bool has_s = j > 0, has_n = j + 1 < g.ny1;
  const int cs = has_s ? c - plane : c, cn = has_n ? c + plane : c;
  double fw = 1.0, fe = 1.0, fs = has_s ? 1.0 : 0.0, fn = has_n ? 1.0 : 0.0, fb = 1.0, ff = 1.0;
  if (MASKED) {
    const uint8_t t = tag[c], te = tag[ce], tn = tag[cn], tf = tag[cf];
    fw = (t & TAG_U) ? 1.0 : 0.0;
    fe = (te & TAG_U) ? 1.0 : 0.0;
    fs = (t & TAG_V) ? 1.0 : 0.0;             // v face 0 (the south box wall) is never internal
    fn = (has_n && (tn & TAG_V)) ? 1.0 : 0.0;
    fb = (t & TAG_W) ? 1.0 : 0.0;
    ff = (tf & TAG_W) ? 1.0 : 0.0;
  }
  const double xc = x[c];
  // wall-normal part: idy2 both ways, or the row's own Poisson coefficients
  const double ys = fs * (x[cs] - xc), yn = fn * (x[cn] - xc);
  const double yp = g.stretched ? ys * g.ytab[YT_TLO * g.ystr + j] + yn * g.ytab[YT_THI * g.ystr + j]
                                : (ys + yn) * g.idy2;
  return (fw * (x[cw] - xc) + fe * (x[ce] - xc)) * g.idx2 + yp + (fb * (x[cb] - xc) + ff * (x[cf] - xc)) * g.idz2;
}

// The symmetrising row weight of cell row j: the cell height on a stretched grid, else 1.
__device__ __forceinline__ double row_weight(const GridParams& g, int c) {
  return g.stretched ? g.ytab[YT_DYC * g.ystr + c / (g.nx * g.nz)] : 1.0;
}

// Sum of the nb partials, the same order in every block; every thread gets it.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nb, double* smem) {
  double s = 0.0;
  for (int e = threadIdx.x; e < nb; e += blockDim.x) s += part[e];
  const double r = block_reduce<false>(s, smem);
  __syncthreads();
  if (threadIdx.x == 0) smem[7] = r;
  __syncthreads();
  return smem[7];
}

__device__ __forceinline__ void put_partial(double v, double* smem, double* __restrict__ part) {
  const double r = block_reduce<false>(v, smem);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
  __syncthreads();
}

// r0 = b - D M G x0 with b = D G x0 + mean (the right-hand side the full-box solve x0
// answered, the removed mean added back); partials of |b|^2, sum r0 and sum x0.
__global__ __launch_bounds__(PT) void k_pcg_init(GridParams g, const uint8_t* __restrict__ tag,
                                                const double* __restrict__ x, const double* __restrict__ mean,
                                                double* __restrict__ r, double* __restrict__ pb,
                                                double* __restrict__ prs, double* __restrict__ px) {
  __shared__ double smem[8];
  const double m = mean[0];
  double ab = 0.0, ars = 0.0, ax = 0.0;
  for (int c = blockIdx.x * PT + threadIdx.x; c < g.ncell; c += gridDim.x * PT) {
    double rv = 0.0;
    if (tag[c] & TAG_P) {
      int j, k, i;
      decode(g, c, j, k, i);
      const double wr = row_weight(g, c);
      const double b = lap<false>(g, tag, x, c, j, k, i) + m;
      rv = wr * (b - lap<true>(g, tag, x, c, j, k, i));
      ab += (wr * b) * (wr * b);
      ars += rv;
      ax += x[c];
    }
    r[c] = rv;
  }
  put_partial(ab, smem, pb);
  put_partial(ars, smem, prs);
  put_partial(ax, smem, px);
}

// The operator's range is orthogonal to the constant on the internal cells, and no
// iteration changes the sum of r: its rounding-level mean (from b, which only matches
// the divergence to the full-box solve's accuracy) is removed here.  Partials of |r0|^2.
// With rs (stretched grids, FP32 storage) also rs = W^-1 r in the preconditioner's
// precision P everywhere (zero outside the internal cells).
template <typename P>
__global__ __launch_bounds__(PT) void k_pcg_center(GridParams g, const uint8_t* __restrict__ tag,
                                                  double* __restrict__ r, const double* __restrict__ prs, int nb,
                                                  const int32_t* __restrict__ n_internal, double* __restrict__ pr,
                                                  P* __restrict__ rs) {
  __shared__ double smem[8];
  const double mean = sum_partials(prs, nb, smem) / (double)n_internal[0];
  double ar = 0.0;
  for (int c = blockIdx.x * PT + threadIdx.x; c < g.ncell; c += gridDim.x * PT) {
    double rv = 0.0;
    if (tag[c] & TAG_P) {
      rv = r[c] - mean;
      r[c] = rv;
      ar += rv * rv;
    }
    if (rs) rs[c] = P(rv / row_weight(g, c));
  }
  put_partial(ar, smem, pr);
}

// x = phi (FP32 storage: the full-box solution that starts the iteration, into FP64)
__global__ __launch_bounds__(PT) void k_pcg_load(GridParams g, const float* __restrict__ phi,
                                                double* __restrict__ x) {
  for (int c = blockIdx.x * PT + threadIdx.x; c < g.ncell; c += gridDim.x * PT) x[c] = (double)phi[c];
}

// partials of r . z (r is zero outside the internal cells)
// (with zo, the previous z: partials of r . zo too, for the flexible beta)
template <typename P>
__global__ __launch_bounds__(PT) void k_pcg_rz(GridParams g, const double* __restrict__ r,
                                              const P* __restrict__ z, double* __restrict__ part,
                                              const P* __restrict__ zo, double* __restrict__ part_o) {
  if (g.skip && *g.skip) return;
  __shared__ double smem[8];
  double a = 0.0, ao = 0.0;
  for (int c = blockIdx.x * PT + threadIdx.x; c < g.ncell; c += gridDim.x * PT) {
    a += r[c] * (double)z[c];
    if (zo) ao += r[c] * (double)zo[c];
  }
  put_partial(a, smem, part);
  if (zo) put_partial(ao, smem, part_o);
}

// rho = r . z; p = z + beta p on the internal cells (p = z at it = 0), 0 elsewhere, with
// beta = rho / rho_prev, or (flexible, przo not null) (rho - r . z_prev) / rho_prev; rho
// goes to sc[it & 1], rho_prev is read from the other slot.
template <typename P>
__global__ __launch_bounds__(PT) void k_pcg_dir(GridParams g, const uint8_t* __restrict__ tag,
                                               const P* __restrict__ z, double* __restrict__ p,
                                               const double* __restrict__ prz, const double* __restrict__ przo,
                                               int nb, double* __restrict__ sc, int it) {
  if (g.skip && *g.skip) return;
  __shared__ double smem[8];
  const double rho = sum_partials(prz, nb, smem);
  const double rho_o = (przo && it > 0) ? sum_partials(przo, nb, smem) : 0.0;
  const double rho_prev = it > 0 ? sc[(it + 1) & 1] : 0.0;
  const double beta = rho_prev != 0.0 ? (przo ? (rho - rho_o) / rho_prev : rho / rho_prev) : 0.0;
  for (int c = blockIdx.x * PT + threadIdx.x; c < g.ncell; c += gridDim.x * PT) {
    const bool in = (tag[c] & TAG_P) != 0;
    const double zc = (double)z[c];
    p[c] = in ? (it > 0 ? zc + beta * p[c] : zc) : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[it & 1] = rho;
}

// ap = D M G p on the internal cells (0 elsewhere); partials of p . ap.  Two cells per
// trip, evaluated without branches (p is 0 outside the internal cells).
__global__ __launch_bounds__(PT) void k_pcg_apply(GridParams g, const uint8_t* __restrict__ tag,
                                                 const double* __restrict__ p, double* __restrict__ ap,
                                                 double* __restrict__ part) {
  if (g.skip && *g.skip) return;
  __shared__ double smem[8];
  double a = 0.0;
  const int stride = gridDim.x * PT;
  const int last = (int)g.ncell - 1;
  for (int c0 = blockIdx.x * PT + threadIdx.x; c0 < g.ncell; c0 += 2 * stride) {
    const int c1 = c0 + stride;
    const int c1c = c1 < g.ncell ? c1 : last;
    int j0, k0, i0, j1, k1, i1;
    decode(g, c0, j0, k0, i0);
    decode(g, c1c, j1, k1, i1);
    const double in0 = (tag[c0] & TAG_P) ? 1.0 : 0.0, in1 = (tag[c1c] & TAG_P) ? 1.0 : 0.0;
    const double y0 = in0 * row_weight(g, c0) * lap<true>(g, tag, p, c0, j0, k0, i0);
    const double y1 = in1 * row_weight(g, c1c) * lap<true>(g, tag, p, c1c, j1, k1, i1);
    a += p[c0] * y0;
    ap[c0] = y0;
    if (c1 < g.ncell) {
      a += p[c1] * y1;
      ap[c1] = y1;
    }
  }
  put_partial(a, smem, part);
}

// alpha = rho / (p . ap); x += alpha p, r -= alpha ap on the internal cells; partials of
// |r|^2 and sum x there.
template <typename P>
__global__ __launch_bounds__(PT) void k_pcg_step(GridParams g, const uint8_t* __restrict__ tag,
                                                double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ p, const double* __restrict__ ap,
                                                const double* __restrict__ ppap, int nb,
                                                const double* __restrict__ sc, int it, double* __restrict__ pr,
                                                double* __restrict__ px, P* __restrict__ rs) {
  if (g.skip && *g.skip) return;
  __shared__ double smem[8];
  const double pap = sum_partials(ppap, nb, smem);
  const double alpha = pap != 0.0 ? sc[it & 1] / pap : 0.0;
  double ar = 0.0, ax = 0.0;
  for (int c = blockIdx.x * PT + threadIdx.x; c < g.ncell; c += gridDim.x * PT) {
    if (tag[c] & TAG_P) {
      const double xv = x[c] + alpha * p[c];
      const double rv = r[c] - alpha * ap[c];
      x[c] = xv;
      r[c] = rv;
      if (rs) rs[c] = P(rv / row_weight(g, c));
      ar += rv * rv;
      ax += xv;
    }
  }
  put_partial(ar, smem, pr);
  put_partial(ax, smem, px);
}

// out[0] = sum of the nb partials (one block)
__global__ __launch_bounds__(PT) void k_pcg_total(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double smem[8];
  const double s = sum_partials(part, nb, smem);
  if (threadIdx.x == 0) out[0] = s;
}

// sc[3] <- mean[0]; converged flag cleared (one thread)
__global__ void k_pcg_prep(const double* __restrict__ mean, double* __restrict__ sc, int32_t* __restrict__ stat) {
  if (threadIdx.x == 0) {
    sc[3] = mean[0];
    stat[PCG_DONE] = 0;
    stat[PCG_ITERS] = 0;
  }
}

// Convergence test after `it` iterations (one block): |r|^2 from the partials of the last
// update; unless the solve has already converged, `it` and |r|^2 are recorded and the
// flag set once |r|^2 <= tol2 |b|^2 (|b|^2 in sc[2]).  Every later kernel of the solve
// then returns at once, so the iterate stops exactly at convergence.
__global__ __launch_bounds__(PT) void k_pcg_check(const double* __restrict__ part, int nb,
                                                 const double* __restrict__ sc, double tol2, int it,
                                                 int32_t* __restrict__ stat, double* __restrict__ rr_out) {
  __shared__ double smem[8];
  if (stat[PCG_DONE]) return;
  const double rr = sum_partials(part, nb, smem);
  if (threadIdx.x == 0) {
    stat[PCG_ITERS] = it;
    rr_out[0] = rr;
    if (rr <= tol2 * sc[2]) stat[PCG_DONE] = 1;
  }
}

// mean[0] <- sc[3]
__global__ void k_pcg_post(double* __restrict__ mean, const double* __restrict__ sc) {
  if (threadIdx.x == 0) mean[0] = sc[3];
}

// gauge: phi = x - mean of x over the internal cells there, 0 elsewhere
// (the result into out, in the storage precision: x itself in FP64)
template <typename P>
__global__ __launch_bounds__(PT) void k_pcg_finish(GridParams g, const uint8_t* __restrict__ tag,
                                                  const double* __restrict__ x, const double* __restrict__ px, int nb,
                                                  const int32_t* __restrict__ n_internal, P* __restrict__ out) {
  __shared__ double smem[8];
  const double mean = sum_partials(px, nb, smem) / (double)n_internal[0];
  for (int c = blockIdx.x * PT + threadIdx.x; c < g.ncell; c += gridDim.x * PT)
    out[c] = P((tag[c] & TAG_P) ? x[c] - mean : 0.0);
}

}  // namespace

int pcg_blocks(const GridParams& g) {
  const int64_t nb = (g.ncell + PT - 1) / PT;
  return (int)(nb < PCG_NPART ? nb : PCG_NPART);
}

template <typename P>
hipError_t launch_pcg_init(const GridParams& g, const uint8_t* tag, const double* x, const double* mean, double* r,
                           double* part, const int32_t* n_internal, P* rs, hipStream_t st) {
  const int nb = pcg_blocks(g);
  hipLaunchKernelGGL(k_pcg_init, dim3(nb), dim3(PT), 0, st, g, tag, x, mean, r, part + PCG_B * PCG_NPART,
                     part + PCG_RS * PCG_NPART, part + PCG_X * PCG_NPART);
  hipLaunchKernelGGL(k_pcg_center<P>, dim3(nb), dim3(PT), 0, st, g, tag, r, part + PCG_RS * PCG_NPART, nb,
                     n_internal, part + PCG_R2 * PCG_NPART, rs);
  return hipGetLastError();
}

hipError_t launch_pcg_load(const GridParams& g, const float* phi, double* x, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_load, dim3(pcg_blocks(g)), dim3(PT), 0, st, g, phi, x);
  return hipGetLastError();
}

template <typename P>
hipError_t launch_pcg_rz(const GridParams& g, const double* r, const P* z, const P* zo, double* part,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_rz<P>, dim3(pcg_blocks(g)), dim3(PT), 0, st, g, r, z, part + PCG_RZ * PCG_NPART, zo,
                     part + PCG_RZO * PCG_NPART);
  return hipGetLastError();
}

template <typename P>
hipError_t launch_pcg_dir(const GridParams& g, const uint8_t* tag, const P* z, double* p, double* part,
                          double* sc, int it, bool flexible, hipStream_t st) {
  const int nb = pcg_blocks(g);
  hipLaunchKernelGGL(k_pcg_dir<P>, dim3(nb), dim3(PT), 0, st, g, tag, z, p, part + PCG_RZ * PCG_NPART,
                     flexible ? part + PCG_RZO * PCG_NPART : nullptr, nb, sc, it);
  return hipGetLastError();
}

hipError_t launch_pcg_apply(const GridParams& g, const uint8_t* tag, const double* p, double* ap, double* part,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_apply, dim3(pcg_blocks(g)), dim3(PT), 0, st, g, tag, p, ap, part + PCG_PAP * PCG_NPART);
  return hipGetLastError();
}

template <typename P>
hipError_t launch_pcg_step(const GridParams& g, const uint8_t* tag, double* x, double* r, const double* p,
                           const double* ap, double* part, const double* sc, int it, P* rs, hipStream_t st) {
  const int nb = pcg_blocks(g);
  hipLaunchKernelGGL(k_pcg_step<P>, dim3(nb), dim3(PT), 0, st, g, tag, x, r, p, ap, part + PCG_PAP * PCG_NPART, nb,
                     sc, it, part + PCG_R2 * PCG_NPART, part + PCG_X * PCG_NPART, rs);
  return hipGetLastError();
}

hipError_t launch_pcg_total(const GridParams& g, const double* part, int slot, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_total, dim3(1), dim3(PT), 0, st, part + slot * PCG_NPART, pcg_blocks(g), out);
  return hipGetLastError();
}

hipError_t launch_pcg_prep(const double* mean, double* sc, int32_t* stat, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_prep, dim3(1), dim3(64), 0, st, mean, sc, stat);
  return hipGetLastError();
}

hipError_t launch_pcg_check(const GridParams& g, const double* part, const double* sc, double tol2, int it,
                            int32_t* stat, double* rr_out, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(PT), 0, st, part + PCG_R2 * PCG_NPART, pcg_blocks(g), sc, tol2, it,
                     stat, rr_out);
  return hipGetLastError();
}

hipError_t launch_pcg_post(double* mean, const double* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_post, dim3(1), dim3(64), 0, st, mean, sc);
  return hipGetLastError();
}

template <typename P>
hipError_t launch_pcg_finish(const GridParams& g, const uint8_t* tag, const double* x, const double* part,
                             const int32_t* n_internal, P* out, hipStream_t st) {
  const int nb = pcg_blocks(g);
  hipLaunchKernelGGL(k_pcg_finish<P>, dim3(nb), dim3(PT), 0, st, g, tag, x, part + PCG_X * PCG_NPART, nb,
                     n_internal, out);
  return hipGetLastError();
}

#define IBM_PCG_INST(P)                                                                                          \
  template hipError_t launch_pcg_init<P>(const GridParams&, const uint8_t*, const double*, const double*,      \
                                         double*, double*, const int32_t*, P*, hipStream_t);                    \
  template hipError_t launch_pcg_rz<P>(const GridParams&, const double*, const P*, const P*, double*,           \
                                       hipStream_t);                                                             \
  template hipError_t launch_pcg_dir<P>(const GridParams&, const uint8_t*, const P*, double*, double*, double*, \
                                        int, bool, hipStream_t);                                                 \
  template hipError_t launch_pcg_step<P>(const GridParams&, const uint8_t*, double*, double*, const double*,   \
                                         const double*, double*, const double*, int, P*, hipStream_t);         \
  template hipError_t launch_pcg_finish<P>(const GridParams&, const uint8_t*, const double*, const double*,    \
                                           const int32_t*, P*, hipStream_t);
IBM_PCG_INST(double)
IBM_PCG_INST(float)
#undef IBM_PCG_INST
