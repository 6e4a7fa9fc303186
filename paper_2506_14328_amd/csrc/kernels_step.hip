// Kernels of one RK3 substep (Sec. 2.4, Eq. (16), with the projection of Sec. 2.1):
//   momentum   explicit right-hand side, RK combination, staircase update
//   ibm_fix    implicit centre-weight update at immersed-boundary points
//   cfr        flow-rate reduction -> mean pressure gradient
//   ibm_pi     pressure-gradient response at immersed-boundary u points
//   div_fftx   divergence of u* fused with the real FFT along x
//   fftz       complex FFT along z (forward / inverse)
//   tri        wall-normal tridiagonal solve per Fourier mode (FP64 arithmetic)
//   ifftx      inverse real FFT along x -> phi
//   correct    velocity correction, reset of external faces, pressure update
#include "fft_lds.h"
#include "ibm_internal.h"

namespace {

constexpr int BX = 64;  // x points per block row (one wavefront)
constexpr int BZ = 4;   // z rows per block

__device__ __forceinline__ int wrap_p(int i, int n) { return (i + 1 == n) ? 0 : i + 1; }
__device__ __forceinline__ int wrap_m(int i, int n) { return (i == 0) ? n - 1 : i - 1; }

// ---------------------------------------------------------------------------------------
// momentum: H = -N(u) + nu L(u) at internal points (external/ghost neighbours are zero),
// r = dt (a_k H + b_k H_prev) - c_k dt G p, and the staircase predictor u* = u + r.  At
// immersed-boundary points r is stored and completed by ibm_fix.  Per-block partial sums
// of u* over internal non-IBM u points feed the flow-rate reduction.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_momentum(GridParams g, Fields<T> f, StageConsts s,
                                                 double* __restrict__ qpart) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int k = blockIdx.y * BZ + threadIdx.y;
  const int j = blockIdx.z;
  __shared__ double red[4];
  double qloc = 0.0;
  if (i < g.nx && k < g.nz) {
    const int nx = g.nx, nz = g.nz;
    const int ip = wrap_p(i, nx), im = wrap_m(i, nx);
    const int kp = wrap_p(k, nz), km = wrap_m(k, nz);
    const int plane = nx * nz;
    const int c = (j * nz + k) * nx + i;
    const int cim = c - i + im, cip = c - i + ip;
    const int ckp = c + (kp - k) * nx, ckm = c + (km - k) * nx;
    const bool hasN = (j + 1 < g.ny1), hasS = (j > 0);
    const uint8_t tg = f.tag[c];
    const T h = T(0.5), two = T(2);
    const T idx = T(g.idx), idy = T(g.idy), idz = T(g.idz);
    const T idx2 = T(g.idx2), idy2 = T(g.idy2), idz2 = T(g.idz2), nu = T(g.nu);
    const T akdt = T(s.ak_dt), bkdt = T(s.bk_dt), ckdt = T(s.ck_dt);
    const T* __restrict__ u = f.u;
    const T* __restrict__ v = f.v;
    const T* __restrict__ w = f.w;
    const T* __restrict__ p = f.p;
    const T zero = T(0);

    // ---- u-momentum at (i dx, y_c[j], z_c[k])
    if (tg & TAG_U) {
      const T uc = u[c], ue = u[cip], uw = u[cim];
      const T un = hasN ? u[c + plane] : zero, usb = hasS ? u[c - plane] : zero;
      const T ut = u[ckp], ub = u[ckm];
      const T vnw = hasN ? v[cim + plane] : zero, vne = hasN ? v[c + plane] : zero;
      const T vsw = v[cim], vse = v[c];
      const T wtw = w[ckp - i + im], wte = w[ckp];
      const T wbw = w[cim], wbe = w[c];
      const T a1 = h * (uc + ue), a0 = h * (uw + uc);
      const T N = (a1 * a1 - a0 * a0) * idx +
                  (h * (uc + un) * h * (vnw + vne) - h * (usb + uc) * h * (vsw + vse)) * idy +
                  (h * (uc + ut) * h * (wtw + wte) - h * (ub + uc) * h * (wbw + wbe)) * idz;
      const T L = (ue - two * uc + uw) * idx2 + (un - two * uc + usb) * idy2 + (ut - two * uc + ub) * idz2;
      const T H = -N + nu * L;
      const T G = (p[c] - p[cim]) * idx;
      T r = akdt * H - ckdt * G;
      if (s.use_hold) r += bkdt * f.Hu[c];
      if (s.write_h) f.Hu[c] = H;
      const bool ib = (tg & TAG_UI) != 0;
      const T val = ib ? r : uc + r;
      f.us[c] = val;
      if (!ib) qloc = (double)val;
    } else {
      f.us[c] = zero;
    }

    // ---- v-momentum at (x_c[i], y_f[j], z_c[k]); internal v never sits on face 0
    if (tg & TAG_V) {
      const T vc = v[c], ve = v[cip], vw = v[cim];
      const T vn = hasN ? v[c + plane] : zero, vsb = v[c - plane];
      const T vt = v[ckp], vb = v[ckm];
      const T ue_s = u[cip - plane], ue_n = u[cip], uw_s = u[c - plane], uw_n = u[c];
      const T wt_s = w[ckp - plane], wt_n = w[ckp], wb_s = w[c - plane], wb_n = w[c];
      const T b1 = h * (vc + vn), b0 = h * (vsb + vc);
      const T N = (h * (vc + ve) * h * (ue_s + ue_n) - h * (vw + vc) * h * (uw_s + uw_n)) * idx +
                  (b1 * b1 - b0 * b0) * idy +
                  (h * (vc + vt) * h * (wt_s + wt_n) - h * (vb + vc) * h * (wb_s + wb_n)) * idz;
      const T L = (ve - two * vc + vw) * idx2 + (vn - two * vc + vsb) * idy2 + (vt - two * vc + vb) * idz2;
      const T H = -N + nu * L;
      const T G = (p[c] - p[c - plane]) * idy;
      T r = akdt * H - ckdt * G;
      if (s.use_hold) r += bkdt * f.Hv[c];
      if (s.write_h) f.Hv[c] = H;
      f.vs[c] = (tg & TAG_VI) ? r : vc + r;
    } else {
      f.vs[c] = zero;
    }

    // ---- w-momentum at (x_c[i], y_c[j], k dz)
    if (tg & TAG_W) {
      const T wc = w[c], we = w[cip], ww = w[cim];
      const T wn = hasN ? w[c + plane] : zero, wsb = hasS ? w[c - plane] : zero;
      const T wt = w[ckp], wb = w[ckm];
      const T ue_b = u[ckm - i + ip], ue_t = u[cip], uw_b = u[ckm], uw_t = u[c];
      const T vn_b = hasN ? v[ckm + plane] : zero, vn_t = hasN ? v[c + plane] : zero;
      const T vs_b = v[ckm], vs_t = v[c];
      const T c1 = h * (wc + wt), c0 = h * (wb + wc);
      const T N = (h * (wc + we) * h * (ue_b + ue_t) - h * (ww + wc) * h * (uw_b + uw_t)) * idx +
                  (h * (wc + wn) * h * (vn_b + vn_t) - h * (wsb + wc) * h * (vs_b + vs_t)) * idy +
                  (c1 * c1 - c0 * c0) * idz;
      const T L = (we - two * wc + ww) * idx2 + (wn - two * wc + wsb) * idy2 + (wt - two * wc + wb) * idz2;
      const T H = -N + nu * L;
      const T G = (p[c] - p[ckm]) * idz;
      T r = akdt * H - ckdt * G;
      if (s.use_hold) r += bkdt * f.Hw[c];
      if (s.write_h) f.Hw[c] = H;
      f.ws[c] = (tg & TAG_WI) ? r : wc + r;
    } else {
      f.ws[c] = zero;
    }
  }
  const double tot = block_reduce<false>(qloc, red);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    qpart[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = tot;
}

// ---------------------------------------------------------------------------------------
// ibm_fix: (B u + r) / A at immersed-boundary points (Eq. (16)); u* holds r there.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_ibm_fix(Fields<T> f, IbmLists L, int stage, double* __restrict__ qpart) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  __shared__ double red[4];
  double q = 0.0;
  if (g < L.n_total) {
    const int id = L.idx[g];
    const double2 cf = L.coef[(size_t)stage * L.n_total + g];
    if (g < L.n_u) {
      const T val = T((cf.x * (double)f.u[id] + (double)f.us[id]) * cf.y);
      f.us[id] = val;
      q = (double)val;
    } else if (g < L.n_u + L.n_v) {
      f.vs[id] = T((cf.x * (double)f.v[id] + (double)f.vs[id]) * cf.y);
    } else {
      f.ws[id] = T((cf.x * (double)f.w[id] + (double)f.ws[id]) * cf.y);
    }
  }
  const double tot = block_reduce<false>(q, red);
  if (threadIdx.x == 0) qpart[blockIdx.x] = tot;
}

// ---------------------------------------------------------------------------------------
// cfr: Q(u*_0) = (dy dz / nx) sum u*_0 over internal u; Pi_k = (Q - Q_t) / S_k so that
// Q(u*_0 - Pi_k c_k dt / A) = Q_t exactly.  One block; fixed summation order.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_cfr(const double* __restrict__ qpart, int nq, double scale,
                                              int forcing, double qt, const double* __restrict__ S3,
                                              int stage, double* __restrict__ pi_out,
                                              double* __restrict__ pi_hist) {
  __shared__ double red[16];
  double s = 0.0;
  for (int e = threadIdx.x; e < nq; e += blockDim.x) s += qpart[e];
  const double tot = block_reduce<false>(s, red);
  if (threadIdx.x == 0) {
    const double q0 = tot * scale;
    const double pi = (forcing == 0) ? (q0 - qt) / S3[stage] : qt;
    pi_out[0] = pi;
    pi_hist[0] = pi;
    pi_hist[1] = q0;
  }
}

// u* <- u* - Pi c_k dt / A at immersed-boundary u points (the rest is applied on the fly).
template <typename T>
__global__ __launch_bounds__(256) void k_ibm_pi(Fields<T> f, IbmLists L, int stage, double ck_dt,
                                               const double* __restrict__ pi) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < L.n_u) {
    const int id = L.idx[g];
    const double inva = L.coef[(size_t)stage * L.n_total + g].y;
    f.us[id] = T((double)f.us[id] - pi[0] * ck_dt * inva);
  }
}

// u* on a u face including the pending -Pi c_k dt at internal non-IBM faces.
template <typename T>
__device__ __forceinline__ T ustar_at(const Fields<T>& f, int c, T pick) {
  const uint8_t tg = f.tag[c];
  return f.us[c] - (((tg & (TAG_U | TAG_UI)) == TAG_U) ? pick : T(0));
}

// ---------------------------------------------------------------------------------------
// div_fftx: rhs = D u* / (c_k dt) on every cell, then the real FFT along x of each
// (j, k) row: the nx reals are packed as nx/2 complex numbers z_n = x_{2n} + i x_{2n+1},
// transformed, and unpacked to X_m, m = 0..nx/2.  One wavefront per row, 4 rows/block.
// If rhs_in is given, it replaces the divergence (stand-alone Poisson solve).
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_div_fftx(GridParams g, Fields<T> f, FFTPlan px,
                                                 const double2* __restrict__ rtw, double ck_dt,
                                                 const double* __restrict__ pi, const T* __restrict__ rhs_in) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* sm = reinterpret_cast<cplx<T>*>(smem_raw);
  const int N = g.nhalf;
  const int grp = threadIdx.x / IBM_WAVE, lane = threadIdx.x % IBM_WAVE;
  const int row = blockIdx.x * 4 + grp;
  cplx<T>* A = sm + grp * 2 * N;
  cplx<T>* B = A + N;
  const bool valid = row < g.nrows;
  const int nx = g.nx;
  if (valid) {
    T* Ar = reinterpret_cast<T*>(A);   // interleaved (re, im) == packed reals
    if (rhs_in) {
      for (int i = lane; i < nx; i += IBM_WAVE) Ar[i] = rhs_in[row * nx + i];
    } else {
      const int j = row / g.nz, k = row - (row / g.nz) * g.nz;
      const int kp = wrap_p(k, g.nz);
      const T pick = T(pi[0] * ck_dt);
      const T inv = T(1.0 / ck_dt);
      const T idx = T(g.idx), idy = T(g.idy), idz = T(g.idz);
      const bool hasN = (j + 1 < g.ny1);
      const int plane = nx * g.nz;
      for (int i = lane; i < nx; i += IBM_WAVE) {
        const int c = row * nx + i;
        const int ip = wrap_p(i, nx);
        const T ue = ustar_at(f, c - i + ip, pick), uc = ustar_at(f, c, pick);
        const T vn = hasN ? f.vs[c + plane] : T(0), vc = f.vs[c];
        const T wt = f.ws[c + (kp - k) * nx], wc = f.ws[c];
        Ar[i] = ((ue - uc) * idx + (vn - vc) * idy + (wt - wc) * idz) * inv;
      }
    }
  }
  __syncthreads();
  cplx<T>* R = fft_lds<T>(A, B, 1, px, -1, lane, IBM_WAVE);
  if (valid) {
    cplx<T>* out = f.spec + (size_t)row * g.mh;
    for (int m = lane; m <= N; m += IBM_WAVE) {
      const cplx<T> Zm = R[m == N ? 0 : m];
      const cplx<T> Zc = cconj(R[m == 0 ? 0 : N - m]);
      const cplx<T> s1 = cadd(Zm, Zc), d1 = csub(Zm, Zc);
      const double2 e64 = rtw[m];
      const cplx<T> e = {T(e64.x), T(e64.y)};
      const cplx<T> t = cmul(e, d1);
      out[m] = cplx<T>{T(0.5) * (s1.x + t.y), T(0.5) * (s1.y - t.x)};
    }
  }
}

// ---------------------------------------------------------------------------------------
// fftz: complex FFT along z of the half spectrum, W consecutive x modes per block.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_fftz(GridParams g, cplx<T>* __restrict__ spec, FFTPlan pz, int sign,
                                             int W) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem_raw);
  const int nz = g.nz, mh = g.mh;
  cplx<T>* B = A + nz * W;
  const int j = blockIdx.y;
  const int m0 = blockIdx.x * W;
  cplx<T>* base = spec + (size_t)j * nz * mh;
  for (int e = threadIdx.x; e < nz * W; e += blockDim.x) {
    const int kz = e / W, w = e - kz * W, m = m0 + w;
    A[e] = (m < mh) ? base[kz * mh + m] : cplx<T>{T(0), T(0)};
  }
  __syncthreads();
  const int w = threadIdx.x % W, lane = threadIdx.x / W, nl = blockDim.x / W;
  fft_lds<T>(A + w, B + w, W, pz, sign, lane, nl);
  const cplx<T>* R = (pz.nst & 1) ? B : A;
  for (int e = threadIdx.x; e < nz * W; e += blockDim.x) {
    const int kz = e / W, ww = e - kz * W, m = m0 + ww;
    if (m < mh) base[kz * mh + m] = R[e];
  }
}

// ---------------------------------------------------------------------------------------
// tri: per Fourier mode (kx, kz), solve in y
//   (phi_{j+1} - 2 phi_j + phi_{j-1}) / dy^2 - (kx^2 + kz^2) phi_j = rhat_j / (nx nz)
// with -1 instead of -2 in the first and last rows (no flux through the box walls).
// Mode (0,0): its mean over j is removed, the first row becomes phi_0 = 0, and the
// mean of the solution is removed.  Thomas algorithm in FP64, one thread per mode.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_tri(GridParams g, cplx<T>* __restrict__ spec,
                                            const double* __restrict__ kx2, const double* __restrict__ kz2,
                                            double* __restrict__ cp, double2* __restrict__ dp,
                                            double* __restrict__ mean_out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int Q = g.nmodes;
  if (q >= Q) return;
  const int n = g.ny1;
  const int kz = q / g.mh, m = q - kz * g.mh;
  const double K2 = kx2[m] + kz2[kz];
  const double a = g.idy2;
  const double norm = 1.0 / ((double)g.nx * (double)g.nz);
  const bool zero = (q == 0);
  double mr = 0.0, mi = 0.0;
  if (zero) {
    for (int j = 0; j < n; ++j) {
      const cplx<T> r = spec[(size_t)j * Q];
      mr += (double)r.x;
      mi += (double)r.y;
    }
    mr /= n;
    mi /= n;
    mean_out[0] = mr * norm;
  }
  double cprev = 0.0, dpr = 0.0, dpi = 0.0;
  for (int j = 0; j < n; ++j) {
    const cplx<T> r = spec[(size_t)j * Q + q];
    double rr = ((double)r.x - mr) * norm, ri = ((double)r.y - mi) * norm;
    double b = -2.0 * a - K2;
    if (j == 0 || j == n - 1) b += a;
    double up = (j == n - 1) ? 0.0 : a;
    const double lo = (j == 0) ? 0.0 : a;
    if (zero && j == 0) {
      b = 1.0;
      up = 0.0;
      rr = 0.0;
      ri = 0.0;
    }
    const double den = b - lo * cprev;
    const double cj = up / den;
    dpr = (rr - lo * dpr) / den;
    dpi = (ri - lo * dpi) / den;
    cprev = cj;
    cp[(size_t)j * Q + q] = cj;
    dp[(size_t)j * Q + q] = make_double2(dpr, dpi);
  }
  double xr = dpr, xi = dpi;
  double sr = xr, si = xi;
  if (zero) dp[(size_t)(n - 1) * Q] = make_double2(xr, xi);
  else spec[(size_t)(n - 1) * Q + q] = cplx<T>{T(xr), T(xi)};
  for (int j = n - 2; j >= 0; --j) {
    const double cj = cp[(size_t)j * Q + q];
    const double2 dj = dp[(size_t)j * Q + q];
    xr = dj.x - cj * xr;
    xi = dj.y - cj * xi;
    if (zero) {
      sr += xr;
      si += xi;
      dp[(size_t)j * Q] = make_double2(xr, xi);
    } else {
      spec[(size_t)j * Q + q] = cplx<T>{T(xr), T(xi)};
    }
  }
  if (zero) {
    sr /= n;
    si /= n;
    for (int j = 0; j < n; ++j) {
      const double2 x = dp[(size_t)j * Q];
      spec[(size_t)j * Q] = cplx<T>{T(x.x - sr), T(x.y - si)};
    }
  }
}

// ---------------------------------------------------------------------------------------
// ifftx: inverse real FFT along x of each row: Z_m = (X_m + conj X_{N-m})
//        + i e^{+2 pi i m/nx} (X_m - conj X_{N-m}), m < N = nx/2, z = IDFT_N(Z),
//        x_{2n} = Re z_n, x_{2n+1} = Im z_n.  Unnormalised (tri applied 1/(nx nz)).
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_ifftx(GridParams g, const cplx<T>* __restrict__ spec, T* __restrict__ out,
                                              FFTPlan px, const double2* __restrict__ rtw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* sm = reinterpret_cast<cplx<T>*>(smem_raw);
  const int N = g.nhalf;
  const int grp = threadIdx.x / IBM_WAVE, lane = threadIdx.x % IBM_WAVE;
  const int row = blockIdx.x * 4 + grp;
  cplx<T>* A = sm + grp * 2 * N;
  cplx<T>* B = A + N;
  const bool valid = row < g.nrows;
  if (valid) {
    const cplx<T>* in = spec + (size_t)row * g.mh;
    for (int m = lane; m < N; m += IBM_WAVE) {
      const cplx<T> X = in[m];
      const cplx<T> Xc = cconj(in[N - m]);
      const cplx<T> s1 = cadd(X, Xc), d1 = csub(X, Xc);
      const double2 e64 = rtw[m];
      const cplx<T> e = {T(e64.x), T(-e64.y)};   // e^{+2 pi i m / nx}
      const cplx<T> t = cmul(e, d1);
      A[m] = cplx<T>{s1.x - t.y, s1.y + t.x};
    }
  }
  __syncthreads();
  cplx<T>* R = fft_lds<T>(A, B, 1, px, +1, lane, IBM_WAVE);
  if (valid) {
    const T* Rr = reinterpret_cast<const T*>(R);
    for (int i = lane; i < g.nx; i += IBM_WAVE) out[(size_t)row * g.nx + i] = Rr[i];
  }
}

// ---------------------------------------------------------------------------------------
// correct: u = u* - c_k dt G phi on internal faces (the pending -Pi c_k dt included),
// zero on external faces (Sec. 3.3); p += phi on internal pressure cells only.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_correct(GridParams g, Fields<T> f, double ck_dt,
                                                const double* __restrict__ pi) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int k = blockIdx.y * BZ + threadIdx.y;
  const int j = blockIdx.z;
  if (i >= g.nx || k >= g.nz) return;
  const int nx = g.nx, nz = g.nz;
  const int im = wrap_m(i, nx), km = wrap_m(k, nz);
  const int c = (j * nz + k) * nx + i;
  const int plane = nx * nz;
  const uint8_t tg = f.tag[c];
  const T ckdt = T(ck_dt);
  const T ph = f.phi[c];
  T un = T(0), vn = T(0), wn = T(0);
  if (tg & TAG_U) {
    const T pick = (tg & TAG_UI) ? T(0) : T(pi[0] * ck_dt);
    un = f.us[c] - pick - ckdt * ((ph - f.phi[c - i + im]) * T(g.idx));
  }
  if (tg & TAG_V) vn = f.vs[c] - ckdt * ((ph - f.phi[c - plane]) * T(g.idy));
  if (tg & TAG_W) wn = f.ws[c] - ckdt * ((ph - f.phi[c + (km - k) * nx]) * T(g.idz));
  f.u[c] = un;
  f.v[c] = vn;
  f.w[c] = wn;
  f.p[c] = (tg & TAG_P) ? f.p[c] + ph : T(0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T* __restrict__ src, T* __restrict__ dst, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

}  // namespace

// =======================================================================================
// Launchers
// =======================================================================================
static inline dim3 cell_grid(const GridParams& g) {
  return dim3((g.nx + BX - 1) / BX, (g.nz + BZ - 1) / BZ, g.ny1);
}

template <typename T>
hipError_t launch_momentum(const GridParams& g, const Fields<T>& f, const StageConsts& s, double* qpart,
                           int* nqpart, hipStream_t st) {
  const dim3 grid = cell_grid(g);
  hipLaunchKernelGGL(k_momentum<T>, grid, dim3(BX, BZ), 0, st, g, f, s, qpart);
  *nqpart = grid.x * grid.y * grid.z;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ibm_fix(const GridParams& g, const Fields<T>& f, const IbmLists& L, int stage, double* qpart,
                          int* nqpart, hipStream_t st) {
  (void)g;
  const int nb = (L.n_total + 255) / 256;
  *nqpart = nb;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ibm_fix<T>, dim3(nb), dim3(256), 0, st, f, L, stage, qpart);
  return hipGetLastError();
}

hipError_t launch_cfr(const double* qpart, int nq, double scale, int forcing, double q_target_or_pi,
                      const double* S3, int stage, double* pi_out, double* pi_hist, hipStream_t st) {
  hipLaunchKernelGGL(k_cfr, dim3(1), dim3(1024), 0, st, qpart, nq, scale, forcing, q_target_or_pi, S3, stage,
                     pi_out, pi_hist);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ibm_pi(const Fields<T>& f, const IbmLists& L, int stage, double ck_dt, const double* pi,
                         hipStream_t st) {
  if (L.n_u == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ibm_pi<T>, dim3((L.n_u + 255) / 256), dim3(256), 0, st, f, L, stage, ck_dt, pi);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_div_fftx(const GridParams& g, const Fields<T>& f, const FFTPlan& px, const double2* rtw,
                           double ck_dt, const double* pi, const T* rhs_in, hipStream_t st) {
  const size_t lds = 4 * 2 * (size_t)g.nhalf * sizeof(cplx<T>);
  hipLaunchKernelGGL(k_div_fftx<T>, dim3((g.nrows + 3) / 4), dim3(256), lds, st, g, f, px, rtw, ck_dt, pi,
                     rhs_in);
  return hipGetLastError();
}

template <typename T>
static int fftz_width(int nz) {
  int W = 16;
  while (W > 1 && 2 * (size_t)nz * W * sizeof(cplx<T>) > 65536) W >>= 1;
  return W;
}

template <typename T>
hipError_t launch_fftz(const GridParams& g, cplx<T>* spec, const FFTPlan& pz, int sign, hipStream_t st) {
  const int W = fftz_width<T>(g.nz);
  const size_t lds = 2 * (size_t)g.nz * W * sizeof(cplx<T>);
  hipLaunchKernelGGL(k_fftz<T>, dim3((g.mh + W - 1) / W, g.ny1), dim3(256), lds, st, g, spec, pz, sign, W);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tri(const GridParams& g, cplx<T>* spec, const double* kx2, const double* kz2, double* cp,
                      double2* dp, double* mean_out, hipStream_t st) {
  hipLaunchKernelGGL(k_tri<T>, dim3((g.nmodes + 255) / 256), dim3(256), 0, st, g, spec, kx2, kz2, cp, dp,
                     mean_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ifftx(const GridParams& g, const cplx<T>* spec, T* out, const FFTPlan& px, const double2* rtw,
                        hipStream_t st) {
  const size_t lds = 4 * 2 * (size_t)g.nhalf * sizeof(cplx<T>);
  hipLaunchKernelGGL(k_ifftx<T>, dim3((g.nrows + 3) / 4), dim3(256), lds, st, g, spec, out, px, rtw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_correct(const GridParams& g, const Fields<T>& f, double ck_dt, const double* pi,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_correct<T>, cell_grid(g), dim3(BX, BZ), 0, st, g, f, ck_dt, pi);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(const T* src, T* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_copy<T>, dim3((unsigned)nb), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

#define IBM_INST(T)                                                                                              \
  template hipError_t launch_momentum<T>(const GridParams&, const Fields<T>&, const StageConsts&, double*, int*, \
                                         hipStream_t);                                                           \
  template hipError_t launch_ibm_fix<T>(const GridParams&, const Fields<T>&, const IbmLists&, int, double*,     \
                                        int*, hipStream_t);                                                      \
  template hipError_t launch_ibm_pi<T>(const Fields<T>&, const IbmLists&, int, double, const double*,           \
                                       hipStream_t);                                                             \
  template hipError_t launch_div_fftx<T>(const GridParams&, const Fields<T>&, const FFTPlan&, const double2*,   \
                                         double, const double*, const T*, hipStream_t);                          \
  template hipError_t launch_fftz<T>(const GridParams&, cplx<T>*, const FFTPlan&, int, hipStream_t);            \
  template hipError_t launch_tri<T>(const GridParams&, cplx<T>*, const double*, const double*, double*,         \
                                    double2*, double*, hipStream_t);                                             \
  template hipError_t launch_ifftx<T>(const GridParams&, const cplx<T>*, T*, const FFTPlan&, const double2*,    \
                                      hipStream_t);                                                              \
  template hipError_t launch_correct<T>(const GridParams&, const Fields<T>&, double, const double*,             \
                                        hipStream_t);                                                            \
  template hipError_t launch_copy<T>(const T*, T*, int64_t, hipStream_t);

IBM_INST(double)
IBM_INST(float)
