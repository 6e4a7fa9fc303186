// Internal declarations shared by the HIP translation units of libibm.
// Device code targets gfx950 (CDNA4, 64-wide wavefronts) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define IBM_WAVE 64

// Tag bits (one byte per cell, cell layout [j][k][i]).
enum : uint8_t {
  TAG_U = 1u << 0,   // u (west face) internal
  TAG_V = 1u << 1,   // v (south face) internal
  TAG_W = 1u << 2,   // w (back face) internal
  TAG_P = 1u << 3,   // pressure cell internal
  TAG_UI = 1u << 4,  // u carries an immersed-boundary correction (lambda > 0)
  TAG_VI = 1u << 5,
  TAG_WI = 1u << 6,
};

// Kernel ids (profiling).
enum KernelId {
  K_MOMENTUM = 0, K_CFR_PI, K_DIV_FFTX, K_FFTZ_FWD, K_TRI, K_FFTZ_INV, K_IFFTX, K_CORRECT, K_DIAG, K_STATS,
  K_GEOM, K_WALL_SHEAR, K_PCG, K_NUM_KERNELS
};

template <typename T>
struct cplx {
  T x, y;
};

// Geometry and constants of one instance, passed to kernels by value.
struct GridParams {
  int nx, ny1, nz;      // cells per direction (ny1 = ny-1)
  int mh;               // nx/2 + 1 retained x modes
  int nhalf;            // nx/2 (length of the packed complex x transform)
  int nrows;            // ny1*nz rows of nx points
  int nmodes;           // nz*mh Fourier modes per y plane
  int mhs;              // spectrum row stride: mh rounded up to whole 128-byte lines
  int splane;           // spectrum elements per y plane (nz*mhs, plus one line if even)
  int top_fs;           // 1: free-slip north box face (u, w mirrored above the top row)
  int64_t ncell;        // nx*ny1*nz
  double dx, dy, dz;
  double idx, idy, idz;
  double idx2, idy2, idz2;
  double nu, dt;
  // stretched wall-normal grid: stretched = 1 and ytab holds YT_NF per-row tables of
  // ystr = ny1 + 1 doubles each (table f of row j at ytab[f * ystr + j]); a uniform grid
  // has stretched = 0 and a table with the uniform values (used only by batched launches
  // that mix both kinds)
  int stretched;
  int ystr;
  const double* ytab;
  // when set and *skip != 0, the projection kernels (x, z transforms, tridiagonal solve)
  // and the conjugate-gradient kernels return at once: the masked solve has converged
  const int* skip;
};

// Per-row tables of a stretched wall-normal grid (rows j = 0..ny1-1; entry ny1 is padding).
// Cell heights dyc_j = y_f[j+1] - y_f[j]; centre spacings h_j = y_c[j] - y_c[j-1] with the
// ghost centres mirrored in the box faces (h_0 = dyc_0, h_ny1 = dyc_{ny1-1}).
enum YTable {
  YT_IDYC = 0,   // 1 / dyc_j (differences across cell j: divergence, fluxes of u and w rows)
  YT_IDYF,       // 1 / h_j (differences across face j: gradient, flux of v)
  YT_DCM,        // second-derivative weights of centre row j: below 2/(h_j (h_j + h_{j+1}))
  YT_DCP,        //   above 2/(h_{j+1} (h_j + h_{j+1}))
  YT_DFM,        // second-derivative weights of face j: below 2/(dyc_{j-1} (dyc_{j-1} + dyc_j))
  YT_DFP,        //   above 2/(dyc_j (dyc_{j-1} + dyc_j))  (dyc_{-1} = dyc_0)
  YT_WLO,        // interpolation to face j: weight of row j-1, dyc_j / (dyc_{j-1} + dyc_j)
  YT_WHI,        //   weight of row j, dyc_{j-1} / (dyc_{j-1} + dyc_j)
  YT_DYC,        // dyc_j (flow-rate and volume weights); entry ny1: the box height
  YT_TLO,        // pressure Poisson row j: lower coefficient 1/(dyc_j h_j)
  YT_THI,        //   upper coefficient 1/(dyc_j h_{j+1})
  YT_HC,         // h_j (j = 0..ny1: the mirrored ends included)
  YT_NF
};

// Uniform-grid parameters of one descriptor (nx, ny1, nz, spacings, spectrum strides) for
// storage values of ts bytes; ytab, ystr and stretched are left for the caller.
// Spectrum rows start on 128-byte lines (8 FP64 or 16 FP32 complex values per line); a
// plane spans an odd number of lines, so that the rows of one mode in successive planes
// do not all fall on the same memory channels.
inline void grid_params_uniform(int nx, int ny, int nz, double lx, double lz, double y_lo, double y_hi, double nu,
                                double dt, int top_fs, size_t ts, GridParams* out) {
  GridParams& g = *out;
  g.nx = nx;
  g.ny1 = ny - 1;
  g.nz = nz;
  g.nhalf = nx / 2;
  g.mh = nx / 2 + 1;
  g.nrows = g.ny1 * g.nz;
  g.nmodes = g.nz * g.mh;
  g.ncell = (int64_t)g.nx * g.ny1 * g.nz;
  g.dx = lx / nx;
  g.dz = lz / nz;
  g.dy = (y_hi - y_lo) / (ny - 1);
  g.idx = 1.0 / g.dx;
  g.idy = 1.0 / g.dy;
  g.idz = 1.0 / g.dz;
  g.idx2 = 1.0 / (g.dx * g.dx);
  g.idy2 = 1.0 / (g.dy * g.dy);
  g.idz2 = 1.0 / (g.dz * g.dz);
  g.nu = nu;
  g.dt = dt;
  g.top_fs = top_fs;
  const int line = (int)(128 / (2 * ts));
  g.mhs = (g.mh + line - 1) / line * line;
  g.splane = g.nz * g.mhs;
  if ((g.splane / line) % 2 == 0) g.splane += line;
  g.stretched = 0;
  g.ystr = g.ny1 + 1;
  g.ytab = nullptr;
  g.skip = nullptr;
}

// Factors of an FFT length into radix-8/4/2/3/5 stages (host): false if n has another
// prime factor.
bool factor_235(int n, int* radix, int* nst);

// The message ibm_last_error(NULL) returns on this thread (calls without a handle).
void set_last_error(const char* msg);

// Twiddle/stage description of one complex FFT length, resident on the device.
struct FFTPlan {
  int n;                // transform length
  int nst;              // number of radix stages
  int radix[20];        // radix of each stage (8, 4, 2, 3 or 5)
  uint64_t rcode;       // the same, 4 bits per stage (stage s at bits 4s..4s+3), for device code
  const double2* tw64;  // exp(-2 pi i m / n), m = 0..n-1
  const float2* tw32;
};

// ---------------------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.x, -a.y}; }

template <typename T> __device__ __forceinline__ cplx<T> twiddle(const FFTPlan& p, int m, int sign);
template <>
__device__ __forceinline__ cplx<double> twiddle<double>(const FFTPlan& p, int m, int sign) {
  double2 t = p.tw64[m];
  return {t.x, sign < 0 ? t.y : -t.y};
}
template <>
__device__ __forceinline__ cplx<float> twiddle<float>(const FFTPlan& p, int m, int sign) {
  float2 t = p.tw32[m];
  return {t.x, sign < 0 ? t.y : -t.y};
}

// 1/x (x normal, not tiny): the hardware reciprocal estimate refined by two Newton steps,
// each of which squares the relative error, to full FP64 accuracy.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Wave-level and block-level reductions (fixed order: deterministic).
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = IBM_WAVE / 2; o > 0; o >>= 1) v += __shfl_down(v, o, IBM_WAVE);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = IBM_WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, IBM_WAVE));
  return v;
}
// Reduce over the block; result valid in thread 0.  smem holds >= blockDim/64 doubles.
template <bool IS_MAX>
__device__ __forceinline__ double block_reduce(double v, double* smem) {
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthr = blockDim.x * blockDim.y * blockDim.z;
  const int lane = tid & (IBM_WAVE - 1), wid = tid / IBM_WAVE, nw = (nthr + IBM_WAVE - 1) / IBM_WAVE;
  v = IS_MAX ? wave_max(v) : wave_sum(v);
  __syncthreads();
  if (lane == 0) smem[wid] = v;
  __syncthreads();
  double r = IS_MAX ? 0.0 : 0.0;
  if (tid == 0) {
    r = smem[0];
    for (int w = 1; w < nw; ++w) r = IS_MAX ? fmax(r, smem[w]) : r + smem[w];
  }
  return r;
}

// ---------------------------------------------------------------------------------------
// Launchers (one per kernel; defined in the .hip files).  All take the stream.
// ---------------------------------------------------------------------------------------
struct StageConsts {
  double ak_dt, bk_dt, ck_dt;
  int stage;      // 0, 1, 2
  int use_hold;   // b_k != 0
  int write_h;    // H needed by the next stage
};

// Immersed-boundary points: the three component lists, each in linear cell order, laid
// end to end at fixed capacities (so that a new geometry with no more points than the
// capacities needs no reallocation and no host read-back).  choff_c[row * cpr + ch] is the number of points of component c that come
// before the 64-wide chunk ch of grid row `row` (row = j * nz + k); a wavefront that
// covers exactly one such chunk finds a point's list index as that offset plus the
// number of flagged lanes below it (ballot).
struct IbmLists {
  const int32_t* idx;      // [n_u | n_v | n_w] linear cell indices
  const double2* coef;     // [3 stages][n_total] (B, 1/A)
  const double* sig;       // [n_total] coefficient of the wall velocity (moving walls)
  const double* wallv;     // [3] velocity of the immersed walls (device memory)
  const double* sd;        // [3 stages] sum over the IBM u points of sig / A
  int n_cover;             // points the flow-rate kernel visits: n_u, or n_total when the
                           // immersed walls move (it adds their term at every IBM point)
  const int32_t* choff_u;
  const int32_t* choff_v;
  const int32_t* choff_w;
  int n_u, n_v, n_w, n_total;   // capacities of the three lists (laid end to end: v starts
                                // at n_u, w at n_u + n_v) and their sum, the stride of coef
  const int32_t* cnt;      // device: points actually listed per component (<= capacity
                           // unless the geometry overflowed it, which is reported)
  int cpr;                 // 64-wide chunks per row
};

// Index bits of the lanes below `lane` in a 64-bit ballot.
__device__ __forceinline__ int lanes_below(uint64_t mask, int lane) {
  return __popcll(mask & ((1ull << lane) - 1ull));
}



template <typename T>
struct Fields {
  T *u, *v, *w, *p;          // state, materialised on request
  T *us, *vs, *ws;           // predictor (u*) of the current substep
  T *usp, *vsp, *wsp;        // predictor of the previous substep (its projection pending)
  T *pp;                     // pressure before the pending increment phi
  T *pn;                     // pressure after it (written by momentum)
  T *Hu, *Hv, *Hw;           // explicit right-hand side of the previous stage
  T* phi;                    // pressure increment
  cplx<T>* spec;             // spectral work array (ny1, nz, mh)
  const uint8_t* tag;
};

// The state after a projection at point c = (j, k, i) (Sec. 3.3), from its tag tg, its
// west, south and back neighbours cw, cs, cb (cs = c on the first row, whose v is never
// internal): u = u* - c_k dt G phi on internal faces, with the pending -Pi c_k dt on
// internal u faces that carry no immersed-boundary correction; the immersed walls'
// velocity on external faces (v on the south box wall: 0); p = p' + phi on internal
// cells, 0 elsewhere.  Each point reads only its own u*, p' and the phi of its neighbours.
template <typename T>
struct Corrected {
  T u, v, w, p;
};
template <typename T>
__device__ __forceinline__ Corrected<T> corrected_point(const GridParams& g, const Fields<T>& f,
                                                        const double* __restrict__ wallv, uint8_t tg, int j, int c,
                                                        int cw, int cs, int cb, double ck_dt, double pi0) {
  const T ph = f.phi[c], phw = f.phi[cw], phs = f.phi[cs], phb = f.phi[cb];
  const T usv = f.us[c], vsv = f.vs[c], wsv = f.ws[c], pv = f.pp[c];
  const T ckdt = T(ck_dt);
  const T pick = ((tg & (TAG_U | TAG_UI)) == TAG_U) ? T(pi0 * ck_dt) : T(0);
  const T un = usv - pick - ckdt * ((ph - phw) * T(g.idx));
  const T vn = vsv - ckdt * ((ph - phs) * T(g.stretched ? g.ytab[YT_IDYF * g.ystr + j] : g.idy));
  const T wn = wsv - ckdt * ((ph - phb) * T(g.idz));
  Corrected<T> r;
  r.u = (tg & TAG_U) ? un : T(wallv[0]);
  r.v = (tg & TAG_V) ? vn : (j == 0 ? T(0) : T(wallv[1]));
  r.w = (tg & TAG_W) ? wn : T(wallv[2]);
  r.p = (tg & TAG_P) ? pv + ph : T(0);
  return r;
}

// Launch-shape knobs (0 = automatic choice); set directly or by the autotuner.
struct Tuning {
  int mom_jc = 0;     // y planes per momentum block
  int fftz_w = 0;     // x modes per z-FFT block
  int tri_rows = 0;   // rows per thread of the tridiagonal partition solver (4 or 8)
  int tile_order = 0; // momentum tiles: 1 contiguous per XCD (default), 2 interleaved,
                      // 3..8 super-tiles of 2x2, 4x2, 2x4, 4x4, 8x2, 8x4 tiles per XCD
  int mom_cache = 0;  // 1 + bits: bit 0 streaming stores, bit 1 streaming single-use loads
  int mom_tile = 0;   // momentum tile: 0/1 64x4, 2 128x4, 3 64x8, 4 256x4 (FP32), 5 128x8 (FP32),
                      // 6 64x4 with two planes of loads in flight
};

// Flags of the momentum kernel's `order` argument: the tile order (bit 0: contiguous runs
// per XCD) and the cache policy of its single-use accesses.
// Bits MOM_SUPER_SHIFT.. hold log2 of the super-tile's width and depth in tiles (two bits
// each; 0 and 0: no super-tiles).
enum : int { MOM_XCD_CONTIG = 1, MOM_NT_STORE = 2, MOM_NT_LOAD = 4, MOM_SUPER_SHIFT = 4 };

// Arguments of one grid's step kernels, for the batched launches that advance a whole
// ensemble of independent grids with one launch per kernel (block ranges per grid).
template <typename T>
struct MomArgs {
  GridParams g;
  Fields<T> f;
  IbmLists L;
  StageConsts s;
  int jc;
  int ntx;
  int ntz;
  int xcd_order;
  const double* pi_prev;
  double ckdt_prev;
  double* qpart;
  int gx;   // blocks along x of the instance's grid
};

template <typename T>
struct CfrArgs {
  Fields<T> f;
  IbmLists L;
  int stage;
  double ck_dt;
  const double* qpart;
  int nq;
  double scale;
  int forcing;
  double qt;
  const double* S3;
  double* pi_out;
  double* pi_hist;
  int gx;   // blocks along x of the instance's grid
};

template <typename T>
struct DivArgs {
  GridParams g;
  Fields<T> f;
  IbmLists L;
  int stage;
  FFTPlan px;
  const double2* rtw;
  double ck_dt;
  const double* pi;
  const T* rhs_in;
  int ll;   // log2 of the lanes per row
  int gx;   // blocks along x of the instance's grid
};

// Blocks of one z-FFT launch: full blocks (W columns through NJ planes each) plus the
// remainder columns gathered W at a time.
__host__ __device__ inline int fftz_blocks(int mh, int ny1, int W, int NJ) {
  const int gxf = mh / W, rem = mh - gxf * W;
  return gxf * ((ny1 + NJ - 1) / NJ) + (rem * ny1 + W - 1) / W;
}

template <typename T>
struct FftzArgs {
  GridParams g;
  cplx<T>* spec;
  FFTPlan pz;
  int sign;
  int W;
  int gx;   // blocks of the instance's launch
  int nj;   // planes per full block
};

template <typename T>
struct TriArgs {
  GridParams g;
  cplx<T>* spec;
  const double* kx2;
  const double* kz2;
  int P;
  int W;
  double* mean_out;
  int gx;       // blocks of the instance
  int gather;   // modes left over at the end of the z rows gathered into the first blocks
};

template <typename T>
struct IfftxArgs {
  GridParams g;
  const cplx<T>* spec;
  T* out;
  FFTPlan px;
  const double2* rtw;
  int ll;   // log2 of the lanes per row
  int gx;   // blocks along x of the instance's grid
};

template <typename T>
int plan_momentum(const GridParams& g, const Fields<T>& f, const IbmLists& L, const StageConsts& s,
                  const double* pi_prev, double ckdt_prev, const Tuning& tu, double* qpart, MomArgs<T>* a);
template <typename T>
int plan_cfr_pi(const Fields<T>& f, const IbmLists& L, int stage, double ck_dt, const double* qpart, int nq,
                double scale, int forcing, double q_target_or_pi, const double* S3, double* pi_out, double* pi_hist,
                CfrArgs<T>* a);
template <typename T>
int plan_div_fftx(const GridParams& g, const Fields<T>& f, const IbmLists& L, int stage, const FFTPlan& px,
                  const double2* rtw, double ck_dt, const double* pi, DivArgs<T>* a, int* mb, size_t* lds);
template <typename T>
int plan_fftz(const GridParams& g, cplx<T>* spec, const FFTPlan& pz, int sign, const Tuning& tu, FftzArgs<T>* a,
              int* mb, size_t* lds, int* threads);
template <typename T>
int plan_tri(const GridParams& g, cplx<T>* spec, const double* kx2, const double* kz2, double* mean_out,
             const Tuning& tu, TriArgs<T>* a, int* lm, size_t* lds);
template <typename T>
int plan_ifftx(const GridParams& g, const cplx<T>* spec, T* out, const FFTPlan& px, const double2* rtw,
               IfftxArgs<T>* a, int* mb, size_t* lds);
// Batched launches: args and boff (ninst + 1 block offsets) in device memory; ntot blocks.
template <typename T>
hipError_t launch_momentum_b(const MomArgs<T>* args, const int* boff, int ninst, int ntot, bool stretched,
                             hipStream_t st);
template <typename T>
hipError_t launch_cfr_pi_b(const CfrArgs<T>* args, const int* boff, int ninst, int ntot, hipStream_t st);
template <typename T>
hipError_t launch_div_fftx_b(const DivArgs<T>* args, const int* boff, int ninst, int ntot, int mb, size_t lds,
                             hipStream_t st);
template <typename T>
hipError_t launch_fftz_b(const FftzArgs<T>* args, const int* boff, int ninst, int ntot, int mb, int rp, size_t lds,
                         int threads, hipStream_t st);
template <typename T>
hipError_t launch_tri_b(const TriArgs<T>* args, const int* boff, int ninst, int ntot, int lm, size_t lds,
                        bool stretched, hipStream_t st);
template <typename T>
hipError_t launch_ifftx_b(const IfftxArgs<T>* args, const int* boff, int ninst, int ntot, int mb, size_t lds,
                          hipStream_t st);

// step kernels
// pi_prev, ckdt_prev: Pi and c dt of the previous substep, whose projection is pending.
template <typename T>
hipError_t launch_momentum(const GridParams& g, const Fields<T>& f, const IbmLists& L, const StageConsts& s,
                           const double* pi_prev, double ckdt_prev, const Tuning& tu, double* qpart, int* nqpart,
                           hipStream_t st);
template <typename T>
hipError_t launch_cfr_pi(const Fields<T>& f, const IbmLists& L, int stage, double ck_dt, const double* qpart, int nq,
                         double scale, int forcing, double q_target_or_pi, const double* S3, double* pi_out,
                         double* pi_hist, hipStream_t st);
template <typename T>
hipError_t launch_div_fftx(const GridParams& g, const Fields<T>& f, const IbmLists& L, int stage,
                           const FFTPlan& px, const double2* rtw, double ck_dt, const double* pi, const T* rhs_in,
                           hipStream_t st);
template <typename T>
hipError_t launch_fftz(const GridParams& g, cplx<T>* spec, const FFTPlan& pz, int sign, const Tuning& tu,
                       hipStream_t st);
template <typename T>
hipError_t launch_tri(const GridParams& g, cplx<T>* spec, const double* kx2, const double* kz2,
                      double* mean_out, const Tuning& tu, hipStream_t st);
// Valid z-FFT widths for this grid (ascending), written to out; returns the count.
template <typename T>
int fftz_widths(const GridParams& g, const FFTPlan& pz, int* out, int max);
template <typename T>
hipError_t launch_ifftx(const GridParams& g, const cplx<T>* spec, T* out, const FFTPlan& px,
                        const double2* rtw, hipStream_t st);
template <typename T>
// mode bit 0: the state into f.u..f.p; bit 1: into the predictor slot it came from
hipError_t launch_correct(const GridParams& g, const Fields<T>& f, const IbmLists& L, int mode, double ck_dt,
                          const double* pi, hipStream_t st);

// diagnostics
template <typename T>
hipError_t launch_diag(const GridParams& g, const Fields<T>& f, const IbmLists& L, int stage, double ck_dt,
                       const double* pi, const double* mean, double* part, int* npart, hipStream_t st);
template <typename T>
hipError_t launch_stats(const GridParams& g, const Fields<T>& f, double* part, int* npart, hipStream_t st);
hipError_t launch_reduce_final(const double* part, int npart, int nsum, int nmax, double* out,
                               hipStream_t st);

// geometry
// tags (internal, immersed-boundary: some arm shorter than its spacing, and the pressure
// tag), counts[m][row * cpr + chunk] of the seven masks (U, V, W, P, UI, VI, WI) per
// 64-wide row chunk, nrows cpr + 1 entries per mask (the last zero), *clear zeroed, and the
// south-wall point of every (k, i) column of u points: the lowest internal row wj (-1:
// none) and its distance wd to the wall below, negative where that is the south box wall;
// with correct, first the pending projection of the old geometry applied at every point
// with the old tags and written over its predictor and pressure (f.us, f.vs, f.ws, f.pp;
// corrected_point with c_k dt = ck_dt, Pi = pi[0])
template <typename T>
hipError_t launch_geom_tags(const GridParams& g, const double* su, const double* sv, const double* sw, int ibm_on,
                            uint8_t* tag, bool correct, const Fields<T>& f, const double* wallv, double ck_dt,
                            const double* pi, int32_t* wj, double* wd, int32_t* counts, int32_t* clear,
                            hipStream_t st);
// masked projection (conjugate gradients on the internal pressure cells): partial-sum
// slots of PCG_NPART doubles each
constexpr int PCG_NPART = 1024;
enum { PCG_B = 0, PCG_R2, PCG_X, PCG_RZ, PCG_PAP, PCG_RS, PCG_RZO, PCG_NSLOT };
// Device status of the last masked solve (int32 slots): converged flag, iterations, and
// the iteration budget it ran under (0: unbounded eager solve); its final |r|^2 is kept
// as a double in the status's second half.
enum { PCG_DONE = 0, PCG_ITERS, PCG_BUDGET, PCG_NSTAT = 4 };
// sc[3] <- mean[0], the converged flag cleared (a kernel: the solve may be captured)
hipError_t launch_pcg_prep(const double* mean, double* sc, int32_t* stat, hipStream_t st);
// convergence test after `it` iterations: sums the |r|^2 partials; unless already
// converged, records it and |r|^2 and sets the flag when |r|^2 <= tol2 |b|^2
hipError_t launch_pcg_check(const GridParams& g, const double* part, const double* sc, double tol2, int it,
                            int32_t* stat, double* rr_out, hipStream_t st);
// mean[0] <- sc[3] (the removed mean restored for the diagnostics)
hipError_t launch_pcg_post(double* mean, const double* sc, hipStream_t st);
int pcg_blocks(const GridParams& g);
// n_internal: device count of the internal pressure cells
// P: the preconditioner's (storage) precision.  rs: W^-1 r in P, the preconditioner's
// input (stretched grids, FP32 storage; null otherwise: the input is r)
template <typename P>
hipError_t launch_pcg_init(const GridParams& g, const uint8_t* tag, const double* x, const double* mean, double* r,
                           double* part, const int32_t* n_internal, P* rs, hipStream_t st);
// x = phi (FP32 storage: the starting point into FP64)
hipError_t launch_pcg_load(const GridParams& g, const float* phi, double* x, hipStream_t st);
// partials of r . z and (zo not null) r . zo
template <typename P>
hipError_t launch_pcg_rz(const GridParams& g, const double* r, const P* z, const P* zo, double* part,
                         hipStream_t st);
// flexible: the Polak-Ribiere beta from the r . zo partials
template <typename P>
hipError_t launch_pcg_dir(const GridParams& g, const uint8_t* tag, const P* z, double* p, double* part,
                          double* sc, int it, bool flexible, hipStream_t st);
hipError_t launch_pcg_apply(const GridParams& g, const uint8_t* tag, const double* p, double* ap, double* part,
                            hipStream_t st);
template <typename P>
hipError_t launch_pcg_step(const GridParams& g, const uint8_t* tag, double* x, double* r, const double* p,
                           const double* ap, double* part, const double* sc, int it, P* rs, hipStream_t st);
hipError_t launch_pcg_total(const GridParams& g, const double* part, int slot, double* out, hipStream_t st);
// the gauged solution (zero mean over the internal cells) into out (x itself in FP64)
template <typename P>
hipError_t launch_pcg_finish(const GridParams& g, const uint8_t* tag, const double* x, const double* part,
                             const int32_t* n_internal, P* out, hipStream_t st);
// tau_x[nx] and, if modes is not null, modes[3] = (tau_0, tau_1c, tau_1s)
template <typename T>
hipError_t launch_wall_shear(const GridParams& g, const T* u, const int32_t* wj, const double* wd,
                             const double* wallv, double* tau_x, double* modes, hipStream_t st);
// exclusive scans in place of up to SCAN_MAX count arrays, their sums into total[m]: the
// arrays are cut into tiles of SCAN_TILE counts, one block per tile; the tiles' sums go to
// tsum (tsum_cap entries, at least scan_tiles(set)), then each tile is scanned from the
// sum of the tiles before it.  tile_off is filled by the launcher.
constexpr int SCAN_MAX = 12;
constexpr int SCAN_TILE = 4096;
struct ScanSet {
  int32_t* counts[SCAN_MAX];
  int32_t* total[SCAN_MAX];
  int n[SCAN_MAX];
  int tile_off[SCAN_MAX + 1];
  int32_t* tsum;
  int tsum_cap;
  int narr;
};
// tiles of an array of n counts (one tile for an empty array, which writes its zero total)
inline int scan_tiles(int64_t n) { return n > 0 ? (int)((n + SCAN_TILE - 1) / SCAN_TILE) : 1; }
hipError_t launch_scan_multi(ScanSet set, hipStream_t st);
// the u, v, w immersed-boundary lists of capacities cap[] (laid end to end) from the
// scanned per-(row, 64-chunk) offsets of their masks (off_u, off_v, off_w); overflow[0]
// set when a component has more points than its capacity; with zphi every cell's phi
// (zelem bytes) zeroed, with zpi the mean pressure gradient
hipError_t launch_compact3(const uint8_t* tag, const GridParams& g, int cpr, const int32_t* off_u,
                           const int32_t* off_v, const int32_t* off_w, int32_t* idx, const int cap[3],
                           int32_t* overflow, void* zphi, int zelem, double* zpi, hipStream_t st);
hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t st);

// every listed point's lambda and sigma (from the signed distances su, sv, sw) into lam
// and sig, and its per-stage (B, 1/A) into coef (list order), and S3[k] = S_k (Sec. 2.4: c_k dt times the internal non-IBM u points plus the sum of
// 1/A_k over the IBM u points, times scale = dy dz / nx) with sd_out[k] the sum over the
// IBM u points of sig / A_k; part holds the partial sums (4 (ncell/256 + 2 n_u/256 + 2)
// doubles), cnt7 the tag counts (uniform grids), done a device counter that is zero
// between launches
hipError_t launch_s_k(const GridParams& g, const uint8_t* tag, const IbmLists& L, const double* su, const double* sv,
                      const double* sw, double* lam, double* sig, double2* coef, double dt, int b_mode, double* part,
                      double scale, double* S3, const int32_t* cnt7, double* sd_out, unsigned* done, hipStream_t st);

// state copy helpers
template <typename T>
hipError_t launch_copy(const T* src, T* dst, int64_t n, hipStream_t st);
// nvec 16-byte vectors from src to dst (16-byte aligned)
hipError_t launch_stream_copy(const void* src, void* dst, int64_t nvec, hipStream_t st);
constexpr int MIX_MAX = 8;   // most input or output arrays of one stream-mix launch
struct MixPtrs {
  const double2* src[MIX_MAX];
  double2* dst[MIX_MAX];
};
hipError_t launch_stream_mix(const MixPtrs& p, int nsrc, int ndst, int64_t nvec, hipStream_t st);

// RK3 constants (Sec. 2.4, Eq. (17)); c_k = a_k + b_k.
static const double RK_A[3] = {64.0 / 120.0, 50.0 / 120.0, 90.0 / 120.0};
static const double RK_B[3] = {0.0, -34.0 / 120.0, -50.0 / 120.0};
__host__ __device__ __forceinline__ double rk_a(int k) {
  return k == 0 ? 64.0 / 120.0 : (k == 1 ? 50.0 / 120.0 : 90.0 / 120.0);
}
__host__ __device__ __forceinline__ double rk_b(int k) {
  return k == 0 ? 0.0 / 120.0 : (k == 1 ? -34.0 / 120.0 : -50.0 / 120.0);
}
__host__ __device__ __forceinline__ double rk_c(int k) { return rk_a(k) + rk_b(k); }
