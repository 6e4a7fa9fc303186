// Mixed-radix (4, 2, 3, 5) Stockham FFT on data resident in LDS.
//
// A group of `nlanes` threads transforms one sequence of length p.n whose
// element e sits at buf[e * stride].  Each stage reads from one LDS buffer
// and writes the self-sorted result to the other (Stockham auto-sort), so no
// bit-reversal pass is needed.  Stage with radix R after a span Ns:
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

template <typename T, int R>
__device__ __forceinline__ void fft_stage_r(const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst, int n,
                                            int Ns, int stride, const FFTPlan& p, int sign, int lane,
                                            int nlanes) {
  const int nb = n / R;
  const int tstep = n / (Ns * R);
  for (int b = lane; b < nb; b += nlanes) {
    const int k = b % Ns;
    cplx<T> v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) v[t] = src[(b + t * nb) * stride];
    if (k != 0) {
#pragma unroll
      for (int t = 1; t < R; ++t) v[t] = cmul(v[t], twiddle<T>(p, t * k * tstep, sign));
    }
    if (R == 2) bfly2(v);
    if (R == 3) bfly3(v, sign);
    if (R == 4) bfly4(v, sign);
    if (R == 5) bfly5(v, sign);
    const int o = (b / Ns) * Ns * R + k;
#pragma unroll
    for (int t = 0; t < R; ++t) dst[(o + t * Ns) * stride] = v[t];
  }
}

// Transforms the sequence held in a (stride `stride`); returns the buffer that
// holds the result (a if the number of stages is even, else b).
template <typename T>
__device__ cplx<T>* fft_lds(cplx<T>* a, cplx<T>* b, int stride, const FFTPlan& p, int sign, int lane,
                            int nlanes) {
  int Ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.radix[s];
    switch (R) {
      case 4: fft_stage_r<T, 4>(a, b, p.n, Ns, stride, p, sign, lane, nlanes); break;
      case 2: fft_stage_r<T, 2>(a, b, p.n, Ns, stride, p, sign, lane, nlanes); break;
      case 3: fft_stage_r<T, 3>(a, b, p.n, Ns, stride, p, sign, lane, nlanes); break;
      default: fft_stage_r<T, 5>(a, b, p.n, Ns, stride, p, sign, lane, nlanes); break;
    }
    __syncthreads();
    cplx<T>* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}
