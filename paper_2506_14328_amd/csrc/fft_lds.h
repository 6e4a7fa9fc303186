// Mixed-radix (8, 4, 2, 3, 5) Stockham FFT on data resident in LDS.
//
// A group of `nlanes` threads transforms one sequence of length p.n whose
// element e sits at buf[e << ls].  Each stage writes its self-sorted result
// (Stockham auto-sort) back into the same LDS buffer, so no bit-reversal pass is
// needed.  Stage with radix R after a span Ns:
//   butterfly b (0 <= b < n/R), k = b mod Ns,
//   inputs  x[b + t n/R] * w^(t k n/(Ns R)),   t = 0..R-1,  w = exp(sign 2 pi i / n)
//   outputs y[(b/Ns) Ns R + k + t Ns] = DFT_R(inputs)[t]
// Every thread of the block must call fft_lds (it contains __syncthreads()).
#pragma once

#include "ibm_internal.h"

// i * z  and  -i * z
template <typename T>
__device__ __forceinline__ cplx<T> mul_i(cplx<T> z) { return {-z.y, z.x}; }
template <typename T>
__device__ __forceinline__ cplx<T> mul_mi(cplx<T> z) { return {z.y, -z.x}; }

template <typename T>
__device__ __forceinline__ void bfly2(cplx<T>* v) {
  cplx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T>
__device__ __forceinline__ void bfly4(cplx<T>* v, int sign) {
  cplx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  cplx<T> t2 = cadd(v[1], v[3]), d = csub(v[1], v[3]);
  cplx<T> t3 = sign < 0 ? mul_mi(d) : mul_i(d);
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <typename T>
__device__ __forceinline__ void bfly3(cplx<T>* v, int sign) {
  const T s3 = T(0.86602540378443864676);  // sqrt(3)/2
  cplx<T> t1 = cadd(v[1], v[2]);
  cplx<T> t2 = {v[0].x - T(0.5) * t1.x, v[0].y - T(0.5) * t1.y};
  cplx<T> d = csub(v[1], v[2]);
  cplx<T> m = mul_i(cplx<T>{T(sign) * s3 * d.x, T(sign) * s3 * d.y});
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, m);
  v[2] = csub(t2, m);
}

template <typename T>
__device__ __forceinline__ void bfly5(cplx<T>* v, int sign) {
  const T c1 = T(0.30901699437494742410);   // cos(2 pi/5)
  const T c2 = T(-0.80901699437494742410);  // cos(4 pi/5)
  const T s1 = T(0.95105651629515357212);   // sin(2 pi/5)
  const T s2 = T(0.58778525229247312917);   // sin(4 pi/5)
  cplx<T> a = v[0];
  cplx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  cplx<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  cplx<T> r1 = {a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y};
  cplx<T> r2 = {a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y};
  const T sg = T(sign);
  cplx<T> q1 = mul_i(cplx<T>{sg * (s1 * t3.x + s2 * t4.x), sg * (s1 * t3.y + s2 * t4.y)});
  cplx<T> q2 = mul_i(cplx<T>{sg * (s2 * t3.x - s1 * t4.x), sg * (s2 * t3.y - s1 * t4.y)});
  v[0] = cadd(a, cadd(t1, t2));
  v[1] = cadd(r1, q1);
  v[4] = csub(r1, q1);
  v[2] = cadd(r2, q2);
  v[3] = csub(r2, q2);
}

// 8-point DFT in place (natural order): two 4-point DFTs of the even and odd inputs,
// combined with the powers of w = exp(sign 2 pi i / 8).
template <typename T>
__device__ __forceinline__ void bfly8(cplx<T>* v, int sign) {
  const T h = T(0.70710678118654752440);   // sqrt(1/2)
  cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
  bfly4(e, sign);
  bfly4(o, sign);
  const T sg = T(sign);
  // w^1 = h (1 + sign i), w^2 = sign i, w^3 = h (-1 + sign i)
  const cplx<T> o1 = {h * (o[1].x - sg * o[1].y), h * (o[1].y + sg * o[1].x)};
  const cplx<T> o2 = {-sg * o[2].y, sg * o[2].x};
  const cplx<T> o3 = {-h * (o[3].x + sg * o[3].y), h * (sg * o[3].x - o[3].y)};
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

// Twiddle w^m = exp(sign 2 pi i m / n) from the table tw[m] = exp(-2 pi i m / n) held in LDS.
template <typename T>
__device__ __forceinline__ cplx<T> tw_at(const cplx<T>* tw, int m, int sign) {
  const cplx<T> t = tw[m];
  return {t.x, sign < 0 ? t.y : -t.y};
}

// Butterflies per thread needed by the largest stage of plan p with nlanes threads.
inline int fft_max_bfly(const FFTPlan& p, int nlanes) {
  int mb = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int nb = p.n / p.radix[s];
    const int b = (nb + nlanes - 1) / nlanes;
    if (b > mb) mb = b;
  }
  return mb <= 1 ? 1 : (mb <= 2 ? 2 : 4);
}

// Copy the plan's twiddle table (n entries) into LDS; caller synchronises.
template <typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* dst, const FFTPlan& p, int tid, int nthr) {
  for (int m = tid; m < p.n; m += nthr) dst[m] = twiddle<T>(p, m, -1);
}

// Quotient b / d for 0 <= b, d < 2^15 with one multiply-high instead of an integer
// division: with m = ceil(2^31 / d) = (2^31 + e) / d, 0 <= e < d, the product 2 b m / 2^32
// equals b / d + b e / (d 2^31), and b e < 2^31 keeps its floor at floor(b / d).
__device__ __forceinline__ uint32_t div_magic(uint32_t d) { return (0x80000000u + d - 1u) / d; }
__device__ __forceinline__ int div_by(int b, uint32_t m) { return (int)__umulhi((uint32_t)b << 1, m); }

// One in-place stage: every thread first computes up to MB butterflies into
// registers, the block synchronises, then the results are written to their
// self-sorted positions.  Requires n/R <= MB * nlanes (the launchers pick MB).
// Element e of the sequence sits at buf[e << ls].
template <typename T, int R, int MB>
__device__ __forceinline__ void fft_stage_r(cplx<T>* buf, int n, int Ns, int ls, const cplx<T>* __restrict__ tw,
                                            int sign, int lane, int nlanes) {
  const int nb = n / R;
  const uint32_t mg = div_magic((uint32_t)Ns);
  const int tstep = div_by(nb, mg);   // n / (Ns R)
  const int nbs = nb << ls, nss = Ns << ls;
  cplx<T> v[MB][R];
  int out[MB];
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int b = lane + q * nlanes;
    out[q] = -1;
    if (b < nb) {
      const int gNs = div_by(b, mg) * Ns;   // (b / Ns) Ns
      const int k = b - gNs;
      out[q] = (b + gNs * (R - 1)) << ls;   // ((b / Ns) Ns R + k) << ls
      const int bi = b << ls;
#pragma unroll
      for (int t = 0; t < R; ++t) v[q][t] = buf[bi + t * nbs];
      if (k != 0) {
        // w1 = w^(k tstep) from the table, higher powers by repeated multiplication
        const cplx<T> w1 = tw_at<T>(tw, k * tstep, sign);
        cplx<T> wt = w1;
#pragma unroll
        for (int t = 1; t < R; ++t) {
          v[q][t] = cmul(v[q][t], wt);
          if (t + 1 < R) wt = cmul(wt, w1);
        }
      }
      if (R == 2) bfly2(v[q]);
      if (R == 3) bfly3(v[q], sign);
      if (R == 4) bfly4(v[q], sign);
      if (R == 5) bfly5(v[q], sign);
      if (R == 8) bfly8(v[q], sign);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    if (out[q] >= 0) {
#pragma unroll
      for (int t = 0; t < R; ++t) buf[out[q] + t * nss] = v[q][t];
    }
  }
  __syncthreads();
}

// Transforms, in place, the sequence held in buf (element e at buf[e << ls], the stride
// a power of two) with twiddles from the LDS table tw (n < 2^15).  Every thread of the
// block must call it.
template <typename T, int MB>
__device__ void fft_lds(cplx<T>* buf, int ls, const FFTPlan& p, const cplx<T>* tw, int sign, int lane,
                        int nlanes) {
  int Ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = (int)((p.rcode >> (4 * s)) & 15u);
    switch (R) {
      case 8: fft_stage_r<T, 8, MB>(buf, p.n, Ns, ls, tw, sign, lane, nlanes); break;
      case 4: fft_stage_r<T, 4, MB>(buf, p.n, Ns, ls, tw, sign, lane, nlanes); break;
      case 2: fft_stage_r<T, 2, MB>(buf, p.n, Ns, ls, tw, sign, lane, nlanes); break;
      case 3: fft_stage_r<T, 3, MB>(buf, p.n, Ns, ls, tw, sign, lane, nlanes); break;
      default: fft_stage_r<T, 5, MB>(buf, p.n, Ns, ls, tw, sign, lane, nlanes); break;
    }
    Ns *= R;
  }
}
