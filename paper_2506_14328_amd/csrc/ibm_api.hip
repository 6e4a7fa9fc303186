// Host side of libibm: descriptor validation, device allocation, FFT / tridiagonal
// plans, orchestration of the RK3 substeps on the caller's stream, and the C ABI
// declared in include/ibm.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ibm.h"
#include "ibm_internal.h"

namespace {

thread_local std::string g_last_error;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Instance {
  ibm_grid_desc d{};
  GridParams g{};
  FFTPlan px{}, pz{};
  // device allocations
  std::vector<DevBuf> bufs;
  void *u = nullptr, *v = nullptr, *w = nullptr, *p = nullptr;   // state (materialised on request)
  // Predictor triples and pressures, cycled per substep: between substeps the state is
  // correct(S[cur], phi, P[cur]) with the last substep's Pi and c_k dt.
  void* S[3][3] = {};
  void* P[3] = {};
  int cur = 0;
  bool fresh = true;       // nothing pending: the state is in u, v, w, p (no step since it was set),
                           // or only in the predictor slot cur when state_in_slot
  bool state_in_slot = false;
  void *Hu = nullptr, *Hv = nullptr, *Hw = nullptr, *phi = nullptr, *spec = nullptr;
  uint8_t* tag = nullptr;
  double* qpart = nullptr;
  double* red_part = nullptr;
  double* small = nullptr;         // S3[3] pi[1] pi_hist[2] mean[1] red_out[8] diag_out[4] .. pcg[8]
  int32_t* itotal = nullptr;
  double2* rtw = nullptr;
  double *kx2 = nullptr, *kz2 = nullptr;
  // masked projection: conjugate-gradient vectors r, z, p, A p and partial sums
  double* pcg_v[5] = {};   // r, z, p, A p and (stretched grids) W^-1 r
  // FP32 storage: the FP64 iterate x, two FP32 z (the current and the previous one) and the
  // FP32 preconditioner input
  double* pcg_x = nullptr;
  float* pcg_zf[2] = {};
  float* pcg_rsf = nullptr;
  double* pcg_part = nullptr;
  double wall_vel[3] = {0.0, 0.0, 0.0};   // host copy of the immersed walls' velocity
  int pcg_iters = 0;        // iterations of the last masked solve
  double pcg_res = 0.0;     // its final |r| / |b|
  int pcg_iters_max = 0;    // most iterations of an eager masked solve so far
  bool pcg_seen = false;    // an eager masked solve has run
  int pcg_budget = 0;       // iterations per solve captured in the graph
  int32_t* pcg_stat = nullptr;   // device: PCG_NSTAT int32 slots, then |r|^2 (double)
  // south-wall point per (k, i) column (row, distance) and wall-shear output [nx + 3]
  int32_t* wall_j = nullptr;
  double* wall_d = nullptr;
  double* wall_tau = nullptr;
  // immersed-boundary lists; geometry temporaries (dense lambda, block counts)
  DevBuf ibm_idx, ibm_coef, ibm_lam, ibm_sig, ibm_choff, geo_tmp;
  IbmLists L{};
  Tuning tu{};
  int64_t n_int[3] = {0, 0, 0}, n_ibm[3] = {0, 0, 0}, n_pint = 0;
  int cap[3] = {0, 0, 0};        // immersed-boundary list capacities per component
  bool counts_fresh = true;      // the host counts match the device's
  bool lists_overflowed = false; // a geometry had more points than the capacities
  bool geom_ready = false;
  bool diag_valid = false;
  int64_t step = 0;
  double time = 0.0;

  double* S3() { return small; }
  double* pi() { return small + 3; }
  double* pi_hist() { return small + 4; }
  double* mean() { return small + 6; }
  double* red_out() { return small + 7; }
  double* diag_out() { return small + 15; }
  double* pcg_sc() { return small + 20; }   // rho[2] |b|^2 saved-mean |r|^2
  double* wallv() { return small + 26; }    // velocity of the immersed walls (3)
  double* wall_sd() { return small + 29; }  // per stage: sum over IBM u points of sig / A
  bool moving() const { return wall_vel[0] != 0.0 || wall_vel[1] != 0.0 || wall_vel[2] != 0.0; }
};

}  // namespace

struct ibm_ctx {
  int precision = IBM_FP64;
  hipStream_t stream = nullptr;
  std::vector<Instance> inst;
  std::string err;
  bool diag = false;
  // profiling: bit k of prof_mask selects kernel id k
  uint32_t prof_mask = 0;
  bool prof = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kid;
  size_t ev_used = 0;
  double prof_ms[K_NUM_KERNELS] = {};
  int64_t prof_n[K_NUM_KERNELS] = {};
  // graph execution: one RK3 step of every instance captured once, replayed per step
  bool use_graph = false;
  bool use_batch = false;              // ensembles: one launch per kernel for all instances
  int n_branches = 0;                  // capture streams (instances spread round-robin)
  hipStream_t cap = nullptr;           // capture origin stream
  std::vector<hipStream_t> aux;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // batched launches of an ensemble: per-instance kernel arguments and block offsets,
  // packed in one device buffer (valid for the instances' predictor slots cur0)
  struct Batch {
    bool valid = false;
    std::vector<int> cur0;
    void* dbuf = nullptr;
    const void* mom[3] = {};
    const void* cfr[3] = {};
    const void* div[3] = {};
    const void *fzf = nullptr, *fzi = nullptr, *tri = nullptr, *ifx = nullptr;
    const int *bo_mom = nullptr, *bo_cfr = nullptr, *bo_div = nullptr, *bo_fz = nullptr, *bo_tri = nullptr,
              *bo_ifx = nullptr;
    int n_mom = 0, n_cfr = 0, n_div = 0, n_fz = 0, n_tri = 0, n_ifx = 0;
    int mb_div = 1, mb_fz = 1, rp_fz = 0, mb_ifx = 1, lm_tri = 4, th_fz = 256;
    size_t lds_div = 0, lds_fz = 0, lds_tri = 0, lds_ifx = 0;
    bool stretched = false;   // some instance has a stretched wall-normal grid
  } batch;
};

namespace {

int fail(ibm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  g_last_error = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                        \
  do {                                                                                           \
    hipError_t _e = (expr);                                                                      \
    if (_e != hipSuccess)                                                                        \
      return fail(ctx, IBM_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));       \
  } while (0)

// Synchronises st, after checking that neither st nor the library's own capture stream is
// being captured into a graph (a synchronising call inside a capture is refused with
// IBM_ERR_STATE instead of being left to the runtime).
int sync_stream(ibm_ctx* c, hipStream_t st) {
  // (a query that fails says nothing about a capture: the synchronisation then decides)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(c, IBM_ERR_STATE, "a synchronising call on a stream that is being captured");
  cs = hipStreamCaptureStatusNone;
  if (c && c->cap && hipStreamIsCapturing(c->cap, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(c, IBM_ERR_STATE, "a synchronising call while the library's graph capture is active");
  const hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(c, IBM_ERR_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  return IBM_OK;
}

// IBM_ERR_STATE when the library's stream is being captured into a graph by the caller:
// entry points that synchronise refuse before they enqueue anything, so that the state
// they would leave half-updated stays as it was.
int refuse_capture(ibm_ctx* c) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(c, IBM_ERR_STATE, "this call synchronises the stream, which is being captured into a graph");
  return IBM_OK;
}

#define SYNCHK(ctx, st)                   \
  do {                                    \
    const int _r = sync_stream(ctx, st);  \
    if (_r) return _r;                    \
  } while (0)

template <class F>
hipError_t timed(ibm_ctx* c, int kid, F&& launch) {
  if (c->prof && ((c->prof_mask >> kid) & 1u) && c->ev_used + 1 < c->ev.size()) {
    hipEvent_t a = c->ev[c->ev_used], b = c->ev[c->ev_used + 1];
    c->ev_kid[c->ev_used / 2] = kid;
    c->ev_used += 2;
    hipError_t e = hipEventRecord(a, c->stream);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    return hipEventRecord(b, c->stream);
  }
  return launch();
}

}  // namespace

void set_last_error(const char* msg) { g_last_error = msg; }

// Radices of a length-n transform: the power of two in 8s and 4s (8 8 .. 4 4 rather than
// 8 8 .. 8 2 when the exponent is 1 mod 3, so that no radix-2 stage asks for n/2
// butterflies: the lanes per sequence follow the largest stage's butterfly count), then
// the 3s and the 5s.
bool factor_235(int n, int* radix, int* nst) {
  int k = 0, a = 0;
  while (n % 2 == 0 && a < 40) { ++a; n /= 2; }
  int n8 = a / 3, n4 = 0, n2 = 0;
  if (a % 3 == 2) n4 = 1;
  if (a % 3 == 1) {
    if (n8 > 0) { --n8; n4 = 2; }
    else n2 = 1;
  }
  for (int i = 0; i < n8 && k < 20; ++i) radix[k++] = 8;
  for (int i = 0; i < n4 && k < 20; ++i) radix[k++] = 4;
  for (int i = 0; i < n2 && k < 20; ++i) radix[k++] = 2;
  while (n % 3 == 0 && k < 20) { radix[k++] = 3; n /= 3; }
  while (n % 5 == 0 && k < 20) { radix[k++] = 5; n /= 5; }
  *nst = k;
  return n == 1;
}

namespace {

// Per-row wall-normal tables (the YTable layout) of the faces yf[0..ny1]: the same
// arithmetic as the definitions of the spacings (cell heights, centre spacings with the
// ghost centres mirrored in the box faces).
std::vector<double> y_tables(const double* yf, int ny1) {
  const int ys = ny1 + 1;
  std::vector<double> t((size_t)YT_NF * ys, 0.0);
  std::vector<double> dyc(ny1), yc(ny1), h(ny1 + 1);
  for (int j = 0; j < ny1; ++j) {
    dyc[j] = yf[j + 1] - yf[j];
    yc[j] = 0.5 * (yf[j] + yf[j + 1]);
  }
  h[0] = dyc[0];
  for (int j = 1; j < ny1; ++j) h[j] = yc[j] - yc[j - 1];
  h[ny1] = dyc[ny1 - 1];
  double box = 0.0;
  for (int j = 0; j < ny1; ++j) box += dyc[j];
  auto at = [&](int f, int j) -> double& { return t[(size_t)f * ys + j]; };
  for (int j = 0; j < ny1; ++j) {
    const double dm = j > 0 ? dyc[j - 1] : dyc[0];
    at(YT_IDYC, j) = 1.0 / dyc[j];
    at(YT_DCM, j) = 2.0 / (h[j] * (h[j] + h[j + 1]));
    at(YT_DCP, j) = 2.0 / (h[j + 1] * (h[j] + h[j + 1]));
    at(YT_DFM, j) = 2.0 / (dm * (dm + dyc[j]));
    at(YT_DFP, j) = 2.0 / (dyc[j] * (dm + dyc[j]));
    at(YT_WLO, j) = dyc[j] / (dm + dyc[j]);
    at(YT_WHI, j) = dm / (dm + dyc[j]);
    at(YT_DYC, j) = dyc[j];
    at(YT_TLO, j) = 1.0 / (dyc[j] * h[j]);
    at(YT_THI, j) = 1.0 / (dyc[j] * h[j + 1]);
  }
  for (int j = 0; j <= ny1; ++j) {
    at(YT_IDYF, j) = 1.0 / h[j];
    at(YT_HC, j) = h[j];
  }
  at(YT_WLO, ny1) = 0.5;
  at(YT_WHI, ny1) = 0.5;
  at(YT_DYC, ny1) = box;
  return t;
}

// dy in the flow-rate and volume scale factors: the kernels already weight each row by
// its cell height on a stretched grid
inline double y_scale(const GridParams& g) { return g.stretched ? 1.0 : g.dy; }

int dalloc(ibm_ctx* c, Instance& I, void** out, size_t bytes) {
  if (bytes == 0) bytes = 16;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(c, IBM_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  I.bufs.push_back({p, bytes});
  *out = p;
  return IBM_OK;
}

int make_plan(ibm_ctx* c, Instance& I, int n, FFTPlan* pl) {
  pl->n = n;
  if (!factor_235(n, pl->radix, &pl->nst))
    return fail(c, IBM_ERR_ARG, "FFT length " + std::to_string(n) + " has a prime factor outside {2,3,5}");
  if (pl->nst > 16) return fail(c, IBM_ERR_ARG, "FFT length " + std::to_string(n) + " needs too many stages");
  pl->rcode = 0;
  for (int s = 0; s < pl->nst; ++s) pl->rcode |= (uint64_t)pl->radix[s] << (4 * s);
  std::vector<double2> t64(n);
  std::vector<float2> t32(n);
  for (int m = 0; m < n; ++m) {
    const double a = 2.0 * M_PI * (double)m / (double)n;
    t64[m] = make_double2(std::cos(a), -std::sin(a));
    t32[m] = make_float2((float)t64[m].x, (float)t64[m].y);
  }
  void *d64, *d32;
  int rc;
  if ((rc = dalloc(c, I, &d64, n * sizeof(double2)))) return rc;
  if ((rc = dalloc(c, I, &d32, n * sizeof(float2)))) return rc;
  HIPCHK(c, hipMemcpy(d64, t64.data(), n * sizeof(double2), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(d32, t32.data(), n * sizeof(float2), hipMemcpyHostToDevice));
  pl->tw64 = (const double2*)d64;
  pl->tw32 = (const float2*)d32;
  return IBM_OK;
}

int validate(ibm_ctx* c, const ibm_grid_desc& d) {
  if (d.nx < 2 || (d.nx & 1)) return fail(c, IBM_ERR_ARG, "nx must be even and >= 2");
  if (d.nz < 1) return fail(c, IBM_ERR_ARG, "nz must be >= 1");
  if (d.ny < 3) return fail(c, IBM_ERR_ARG, "ny (wall-normal faces) must be >= 3");
  if (d.nx > 1024 || d.nz > 1024) return fail(c, IBM_ERR_ARG, "nx and nz are limited to 1024");
  if (d.ny > 2049) return fail(c, IBM_ERR_ARG, "ny is limited to 2049 (tridiagonal segments)");
  int r[20], ns;
  if (!factor_235(d.nx / 2, r, &ns) || !factor_235(d.nz, r, &ns))
    return fail(c, IBM_ERR_ARG, "nx/2 and nz must have prime factors in {2,3,5}");
  const double cells = (double)d.nx * (double)(d.ny - 1) * (double)d.nz;
  if (cells * 3.0 > 2.0e9) return fail(c, IBM_ERR_ARG, "grid too large for 32-bit cell indexing");
  if (!(d.dt > 0.0) || !(d.nu > 0.0)) return fail(c, IBM_ERR_ARG, "dt and nu must be > 0");
  if (!(d.lx > 0.0) || !(d.lz > 0.0) || !(d.y_hi > d.y_lo)) return fail(c, IBM_ERR_ARG, "invalid box extents");
  if (d.forcing != IBM_CFR && d.forcing != IBM_CPG) return fail(c, IBM_ERR_ARG, "invalid forcing");
  if (d.b_mode < 0 || d.b_mode > 2) return fail(c, IBM_ERR_ARG, "invalid b_mode");
  if (d.top != IBM_TOP_WALL && d.top != IBM_TOP_FREE_SLIP) return fail(c, IBM_ERR_ARG, "invalid top");
  if (d.projection != IBM_PROJ_FULL_BOX && d.projection != IBM_PROJ_MASKED)
    return fail(c, IBM_ERR_ARG, "invalid projection");
  return IBM_OK;
}

int init_instance(ibm_ctx* c, Instance& I, const ibm_grid_desc& d) {
  I.d = d;
  GridParams& g = I.g;
  const size_t ts = (c->precision == IBM_FP64) ? sizeof(double) : sizeof(float);
  grid_params_uniform(d.nx, d.ny, d.nz, d.lx, d.lz, d.y_lo, d.y_hi, d.nu, d.dt,
                      d.top == IBM_TOP_FREE_SLIP ? 1 : 0, ts, &g);
  int rc;
  if ((rc = make_plan(c, I, g.nhalf, &I.px))) return rc;
  {
    // wall-normal tables (uniform values until ibm_set_y_faces)
    std::vector<double> yf(d.ny);
    for (int j = 0; j < d.ny; ++j) yf[j] = d.y_lo + j * g.dy;
    const std::vector<double> tab = y_tables(yf.data(), g.ny1);
    double* yt = nullptr;
    if ((rc = dalloc(c, I, (void**)&yt, tab.size() * sizeof(double)))) return rc;
    HIPCHK(c, hipMemcpyAsync(yt, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    SYNCHK(c, c->stream);
    g.ytab = yt;
    g.ystr = g.ny1 + 1;
    g.stretched = 0;
  }
  if ((rc = make_plan(c, I, g.nz, &I.pz))) return rc;
  const size_t fb = (size_t)g.ncell * ts;
  void** fields[] = {&I.u, &I.v, &I.w, &I.p, &I.S[0][0], &I.S[0][1], &I.S[0][2], &I.S[1][0], &I.S[1][1],
                     &I.S[1][2], &I.S[2][0], &I.S[2][1], &I.S[2][2], &I.P[0], &I.P[1], &I.P[2],
                     &I.Hu, &I.Hv, &I.Hw, &I.phi};
  for (void** f : fields) {
    if ((rc = dalloc(c, I, f, fb))) return rc;
    HIPCHK(c, hipMemsetAsync(*f, 0, fb, c->stream));
  }
  const size_t nspec = (size_t)g.ny1 * g.splane;
  if ((rc = dalloc(c, I, &I.spec, nspec * 2 * ts))) return rc;
  if ((rc = dalloc(c, I, (void**)&I.tag, (size_t)g.ncell))) return rc;
  HIPCHK(c, hipMemsetAsync(I.tag, 0, (size_t)g.ncell, c->stream));
  const size_t mom_blocks = (size_t)((g.nx + 63) / 64) * ((g.nz + 3) / 4) * g.ny1;
  const size_t lst_blocks = (size_t)((3 * g.ncell + 255) / 256);
  if ((rc = dalloc(c, I, (void**)&I.qpart, (mom_blocks + lst_blocks + 1) * sizeof(double)))) return rc;
  const size_t cell_blocks = (size_t)((g.ncell + 255) / 256);
  const size_t red_n = std::max(mom_blocks * 6, (cell_blocks + lst_blocks) * 4) + 16;
  if ((rc = dalloc(c, I, (void**)&I.red_part, red_n * sizeof(double)))) return rc;
  if ((rc = dalloc(c, I, (void**)&I.small, 32 * sizeof(double)))) return rc;
  HIPCHK(c, hipMemsetAsync(I.small, 0, 32 * sizeof(double), c->stream));
  I.L.wallv = I.wallv();
  I.L.sd = I.wall_sd();
  if ((rc = dalloc(c, I, (void**)&I.itotal, 32 * sizeof(int32_t)))) return rc;
  HIPCHK(c, hipMemsetAsync(I.itotal, 0, 32 * sizeof(int32_t), c->stream));
  if (d.projection == IBM_PROJ_MASKED) {
    for (int q = 0; q < 5; ++q)
      if ((rc = dalloc(c, I, (void**)&I.pcg_v[q], (size_t)g.ncell * sizeof(double)))) return rc;
    if (c->precision == IBM_FP32_STORAGE) {
      if ((rc = dalloc(c, I, (void**)&I.pcg_x, (size_t)g.ncell * sizeof(double)))) return rc;
      for (int q = 0; q < 2; ++q)
        if ((rc = dalloc(c, I, (void**)&I.pcg_zf[q], (size_t)g.ncell * sizeof(float)))) return rc;
      if ((rc = dalloc(c, I, (void**)&I.pcg_rsf, (size_t)g.ncell * sizeof(float)))) return rc;
    }
    if ((rc = dalloc(c, I, (void**)&I.pcg_part, (size_t)PCG_NSLOT * PCG_NPART * sizeof(double)))) return rc;
    if ((rc = dalloc(c, I, (void**)&I.pcg_stat, PCG_NSTAT * sizeof(int32_t) + 2 * sizeof(double)))) return rc;
    HIPCHK(c, hipMemsetAsync(I.pcg_stat, 0, PCG_NSTAT * sizeof(int32_t) + 2 * sizeof(double), c->stream));
  }
  const size_t ncol = (size_t)g.nx * g.nz;
  if ((rc = dalloc(c, I, (void**)&I.wall_j, ncol * sizeof(int32_t)))) return rc;
  if ((rc = dalloc(c, I, (void**)&I.wall_d, ncol * sizeof(double)))) return rc;
  if ((rc = dalloc(c, I, (void**)&I.wall_tau, (g.nx + 3) * sizeof(double)))) return rc;
  // real-FFT unpacking twiddles e^{-2 pi i m/nx}, m = 0..nx/2, and modified wavenumbers
  std::vector<double2> rt(g.mh);
  for (int m = 0; m < g.mh; ++m) {
    const double a = 2.0 * M_PI * (double)m / (double)g.nx;
    rt[m] = make_double2(std::cos(a), -std::sin(a));
  }
  std::vector<double> kx(g.mh), kz(g.nz);
  for (int m = 0; m < g.mh; ++m) {
    const double s = std::sin(M_PI * m / g.nx);
    kx[m] = (4.0 / (g.dx * g.dx)) * (s * s);
  }
  for (int n = 0; n < g.nz; ++n) {
    const double s = std::sin(M_PI * n / g.nz);
    kz[n] = (4.0 / (g.dz * g.dz)) * (s * s);
  }
  if ((rc = dalloc(c, I, (void**)&I.rtw, g.mh * sizeof(double2)))) return rc;
  if ((rc = dalloc(c, I, (void**)&I.kx2, g.mh * sizeof(double)))) return rc;
  if ((rc = dalloc(c, I, (void**)&I.kz2, g.nz * sizeof(double)))) return rc;
  HIPCHK(c, hipMemcpy(I.rtw, rt.data(), g.mh * sizeof(double2), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(I.kx2, kx.data(), g.mh * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(I.kz2, kz.data(), g.nz * sizeof(double), hipMemcpyHostToDevice));
  return IBM_OK;
}

// Pointers of the current substep: the previous predictor / pressure are slot I.cur,
// the ones being written slot nxt (= I.cur when nothing is written).
template <typename T>
Fields<T> fields_of(Instance& I, int nxt = -1) {
  if (nxt < 0) nxt = I.cur;
  Fields<T> f;
  f.u = (T*)I.u; f.v = (T*)I.v; f.w = (T*)I.w; f.p = (T*)I.p;
  f.usp = (T*)I.S[I.cur][0]; f.vsp = (T*)I.S[I.cur][1]; f.wsp = (T*)I.S[I.cur][2];
  f.pp = (T*)I.P[I.cur];
  f.us = (T*)I.S[nxt][0]; f.vs = (T*)I.S[nxt][1]; f.ws = (T*)I.S[nxt][2];
  f.pn = (T*)I.P[nxt];
  f.Hu = (T*)I.Hu; f.Hv = (T*)I.Hv; f.Hw = (T*)I.Hw;
  f.phi = (T*)I.phi;
  f.spec = (cplx<T>*)I.spec;
  f.tag = I.tag;
  return f;
}

// Pointers for explicit predictor slots (previous = cur, written = nxt).
template <typename T>
Fields<T> fields_at(Instance& I, int cur, int nxt) {
  const int save = I.cur;
  I.cur = cur;
  Fields<T> f = fields_of<T>(I, nxt);
  I.cur = save;
  return f;
}

StageConsts stage_consts(const GridParams& g, int k) {
  StageConsts sc;
  sc.ak_dt = rk_a(k) * g.dt;
  sc.bk_dt = rk_b(k) * g.dt;
  sc.ck_dt = rk_c(k) * g.dt;
  sc.stage = k;
  sc.use_hold = (k > 0);
  sc.write_h = (k < 2);
  return sc;
}

#define RUNK(ctx, kid, expr)                                                                     \
  do {                                                                                           \
    hipError_t _e = timed(ctx, kid, [&]() { return (expr); });                                   \
    if (_e != hipSuccess)                                                                        \
      return fail(ctx, IBM_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));       \
  } while (0)

// Pressure solve of the current right-hand side: forward FFTs, tridiagonal, inverse FFTs
// (g: the instance's parameters, with the masked solve's skip flag inside its iterations).
template <typename T>
int poisson(ibm_ctx* c, Instance& I, const GridParams& g, Fields<T>& f, T* phi_out, hipStream_t st) {
  RUNK(c, K_FFTZ_FWD, launch_fftz<T>(g, f.spec, I.pz, -1, I.tu, st));
  RUNK(c, K_TRI, launch_tri<T>(g, f.spec, I.kx2, I.kz2, I.mean(), I.tu, st));
  RUNK(c, K_FFTZ_INV, launch_fftz<T>(g, f.spec, I.pz, +1, I.tu, st));
  RUNK(c, K_IFFTX, launch_ifftx<T>(g, f.spec, phi_out, I.px, I.rtw, st));
  return IBM_OK;
}

// Masked projection of the current substep: f.phi holds the full-box solution, which
// starts the conjugate gradients and is replaced by the masked one (zero mean over the
// internal cells, zero elsewhere).  Convergence is tested on the device after every
// iteration (k_pcg_check); once it holds, every later kernel of the solve returns at once
// (the skip flag in the kernels' grid parameters), so the iterate stops exactly there.
// Eager (capture false): up to pcg_max_iter iterations, the flag read back every
// PCG_CHECK iterations to stop launching (a host synchronisation each time).  Captured
// into a graph (capture true): a fixed budget of I.pcg_budget iterations and no host
// access; a solve that has not converged within the budget is reported by ibm_stats.
// FP32 storage: the iteration in FP64 with an FP32 preconditioner (flexible beta), the
// result stored back into the FP32 phi, default tolerance 1e-9 (phi is stored to about 6e-8).
constexpr int PCG_CHECK = 4;
template <typename T>
int pcg_project(ibm_ctx* c, Instance& I, Fields<T>& f, hipStream_t st, bool capture) {
  constexpr bool f64 = std::is_same<T, double>::value;
  const GridParams& g0 = I.g;
  GridParams g = g0;
  g.skip = I.pcg_stat + PCG_DONE;
  double* x = f64 ? reinterpret_cast<double*>(f.phi) : I.pcg_x;
  double *r = I.pcg_v[0], *p = I.pcg_v[2], *ap = I.pcg_v[3];
  T* zb[2];
  T* rs;
  if constexpr (f64) {
    zb[0] = zb[1] = I.pcg_v[1];
    // on a stretched grid the residual is W (b - A x) and the preconditioner takes W^-1 r
    rs = g0.stretched ? I.pcg_v[4] : nullptr;
  } else {
    zb[0] = I.pcg_zf[0];
    zb[1] = I.pcg_zf[1];
    rs = I.pcg_rsf;   // W^-1 r (W = 1 on a uniform grid), rounded to FP32
  }
  const T* pre_in = rs ? rs : reinterpret_cast<const T*>(r);
  double* part = I.pcg_part;
  double* sc = I.pcg_sc();
  double* rr_dev = reinterpret_cast<double*>(I.pcg_stat + PCG_NSTAT);
  const double tol = I.d.pcg_tol > 0.0 ? I.d.pcg_tol : (f64 ? 1e-13 : 1e-9);
  const int max_iter = I.d.pcg_max_iter > 0 ? I.d.pcg_max_iter : 500;
  const int budget = capture ? I.pcg_budget : max_iter;
  RUNK(c, K_PCG, launch_pcg_prep(I.mean(), sc, I.pcg_stat, st));
  if constexpr (!f64) RUNK(c, K_PCG, launch_pcg_load(g0, f.phi, x, st));
  RUNK(c, K_PCG, launch_pcg_init<T>(g0, I.tag, x, sc + 3, r, part, I.itotal + 3, rs, st));
  RUNK(c, K_PCG, launch_pcg_total(g0, part, PCG_B, sc + 2, st));
  RUNK(c, K_PCG, launch_pcg_check(g0, part, sc, tol * tol, 0, I.pcg_stat, rr_dev, st));
  for (int it = 0; it < budget; ++it) {
    if (!capture && it % PCG_CHECK == 0) {
      int32_t done = 0;
      HIPCHK(c, hipMemcpyAsync(&done, I.pcg_stat + PCG_DONE, sizeof(done), hipMemcpyDeviceToHost, st));
      SYNCHK(c, st);
      if (done) break;
    }
    T* z = zb[it & 1];
    const T* zo = (!f64 && it > 0) ? zb[(it + 1) & 1] : nullptr;
    RUNK(c, K_DIV_FFTX, launch_div_fftx<T>(g, f, I.L, 0, I.px, I.rtw, 1.0, I.pi(), pre_in, st));
    int rc = poisson<T>(c, I, g, f, z, st);
    if (rc) return rc;
    RUNK(c, K_PCG, launch_pcg_rz<T>(g, r, z, zo, part, st));
    RUNK(c, K_PCG, launch_pcg_dir<T>(g, I.tag, z, p, part, sc, it, !f64, st));
    RUNK(c, K_PCG, launch_pcg_apply(g, I.tag, p, ap, part, st));
    RUNK(c, K_PCG, launch_pcg_step<T>(g, I.tag, x, r, p, ap, part, sc, it, rs, st));
    RUNK(c, K_PCG, launch_pcg_check(g0, part, sc, tol * tol, it + 1, I.pcg_stat, rr_dev, st));
  }
  RUNK(c, K_PCG, launch_pcg_finish<T>(g0, I.tag, x, part, I.itotal + 3, f.phi, st));
  RUNK(c, K_PCG, launch_pcg_post(I.mean(), sc, st));
  if (capture) return IBM_OK;
  int32_t stat[PCG_NSTAT];
  double rr = 0.0, bb = 0.0;
  HIPCHK(c, hipMemcpyAsync(stat, I.pcg_stat, sizeof(stat), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipMemcpyAsync(&rr, rr_dev, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipMemcpyAsync(&bb, sc + 2, sizeof(double), hipMemcpyDeviceToHost, st));
  SYNCHK(c, st);
  I.pcg_iters = stat[PCG_ITERS];
  I.pcg_res = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
  I.pcg_iters_max = std::max(I.pcg_iters_max, I.pcg_iters);
  I.pcg_seen = true;
  if (!stat[PCG_DONE]) return fail(c, IBM_ERR_UNSTABLE, "masked projection did not converge");
  return IBM_OK;
}

// Iterations per masked solve captured into a graph: the most a solve has needed so far
// (eager solves, and captured ones as read by ibm_stats) plus a quarter (at least 4), a
// multiple of PCG_CHECK, at least 8 and at most pcg_max_iter.  Iterations past
// convergence cost only their launches (every kernel returns at once).
int pcg_capture_budget(const Instance& I) {
  const int max_iter = I.d.pcg_max_iter > 0 ? I.d.pcg_max_iter : 500;
  int b = std::max(8, I.pcg_iters_max + std::max(4, I.pcg_iters_max / 4));
  b = (b + PCG_CHECK - 1) / PCG_CHECK * PCG_CHECK;
  return std::min(b, max_iter);
}

// nsteps RK3 steps of one instance, launched on st.  count: advance the step/time
// counters (false while the launches are only being captured into a graph).
template <typename T>
int run_steps(ibm_ctx* c, Instance& I, int nsteps, hipStream_t st, bool count = true) {
  const GridParams& g = I.g;
  const double scale = y_scale(g) * g.dz / g.nx;
  for (int s = 0; s < nsteps; ++s) {
    for (int k = 0; k < 3; ++k) {
      StageConsts sc;
      sc.ak_dt = rk_a(k) * g.dt;
      sc.bk_dt = rk_b(k) * g.dt;
      sc.ck_dt = rk_c(k) * g.dt;
      sc.stage = k;
      sc.use_hold = (k > 0);
      sc.write_h = (k < 2);
      int nq = 0;
      const int nxt = (I.cur + 1) % 3;
      Fields<T> fm = fields_of<T>(I, nxt);
      // the previous substep (stage k-1, or stage 2 of the previous step) is projected here
      RUNK(c, K_MOMENTUM, launch_momentum<T>(g, fm, I.L, sc, I.pi(), rk_c((k + 2) % 3) * g.dt, I.tu, I.qpart, &nq,
                                             st));
      I.cur = nxt;
      I.fresh = false;
      Fields<T> f = fields_of<T>(I);
      RUNK(c, K_CFR_PI, launch_cfr_pi<T>(f, I.L, k, sc.ck_dt, I.qpart, nq, scale, I.d.forcing, I.d.q_target_or_pi,
                                         I.S3(), I.pi(), I.pi_hist(), st));
      RUNK(c, K_DIV_FFTX, launch_div_fftx<T>(g, f, I.L, k, I.px, I.rtw, sc.ck_dt, I.pi(), (const T*)nullptr, st));
      int rc = poisson<T>(c, I, I.g, f, f.phi, st);
      if (rc) return rc;
      const bool masked = I.d.projection == IBM_PROJ_MASKED;
      if (masked && (rc = pcg_project<T>(c, I, f, st, !count))) return rc;
      if (c->diag && s == nsteps - 1 && k == 2 && !masked) {
        int np = 0;
        RUNK(c, K_DIAG, launch_diag<T>(g, f, I.L, k, sc.ck_dt, I.pi(), I.mean(), I.red_part, &np, st));
        RUNK(c, K_DIAG, launch_reduce_final(I.red_part, np, 0, 3, I.diag_out(), st));
        I.diag_valid = true;
      }
    }
    if (!count) continue;
    I.step += 1;
    I.time += g.dt;
  }
  return IBM_OK;
}


// Writes the state (u, v, w, p) from the pending projection of the last substep.
// With seed the corrected values replace the predictor and pressure they came from
// instead: once the caller zeroes phi and Pi, the state is the start of the next substep
// (what seed_pending does with copies, in one pass), held in that slot only until a call
// that reads u, v, w, p copies it there.
template <typename T>
int materialize_t(ibm_ctx* c, Instance& I, bool seed) {
  // (recomputed even when it was already written: the host cannot see replays of graphs
  // the caller captured, after which the pending projection is newer than the state)
  if (I.fresh) {
    if (!seed && I.state_in_slot) {
      const size_t fb = (size_t)I.g.ncell * sizeof(T);
      const void* src[4] = {I.S[I.cur][0], I.S[I.cur][1], I.S[I.cur][2], I.P[I.cur]};
      void* dst[4] = {I.u, I.v, I.w, I.p};
      for (int q = 0; q < 4; ++q) HIPCHK(c, hipMemcpyAsync(dst[q], src[q], fb, hipMemcpyDeviceToDevice, c->stream));
      I.state_in_slot = false;
    }
    return IBM_OK;
  }
  Fields<T> f = fields_of<T>(I);
  f.us = f.usp; f.vs = f.vsp; f.ws = f.wsp;   // the predictor awaiting its projection
  RUNK(c, K_CORRECT, launch_correct<T>(I.g, f, I.L, seed ? 2 : 1, rk_c(2) * I.g.dt, I.pi(), c->stream));
  if (seed) {
    I.fresh = true;   // (phi and Pi are zeroed by the caller's next kernel)
    I.state_in_slot = true;
  }
  return IBM_OK;
}

int materialize(ibm_ctx* c, Instance& I, bool seed = false) {
  return c->precision == IBM_FP64 ? materialize_t<double>(c, I, seed) : materialize_t<float>(c, I, seed);
}

// Makes the state in u, v, w, p the starting point of the next step: predictor and
// pressure slot I.cur take copies, phi and Pi are zero (nothing pending).
int seed_pending(ibm_ctx* c, Instance& I) {
  I.state_in_slot = false;   // (every caller has just written u, v, w, p or made them current)
  const size_t fb = (size_t)I.g.ncell * (c->precision == IBM_FP64 ? 8 : 4);
  const void* src[4] = {I.u, I.v, I.w, I.p};
  void* dst[4] = {I.S[I.cur][0], I.S[I.cur][1], I.S[I.cur][2], I.P[I.cur]};
  for (int q = 0; q < 4; ++q) HIPCHK(c, hipMemcpyAsync(dst[q], src[q], fb, hipMemcpyDeviceToDevice, c->stream));
  // zeros by kernels, not memsets: a geometry update may be captured into a graph
  HIPCHK(c, launch_fill_zero(I.phi, (int64_t)fb, c->stream));
  HIPCHK(c, launch_fill_zero(I.pi(), (int64_t)sizeof(double), c->stream));
  I.fresh = true;
  return IBM_OK;
}

void free_buf(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

// What a geometry update does about a projection left pending by the last step.
enum { PENDING_NONE = 0, PENDING_APPLIED, PENDING_FUSE };

// Geometry preprocessing (staircase tags, wall distances, immersed-boundary lists and
// coefficients, S_k), all on the stream.  The first geometry of an instance (or the next
// one after the lists overflowed) reads the point counts back, sizes the lists with room
// to spare and synchronises; later ones run with no host synchronisation and no
// allocation, the counts staying on the device (read by ibm_stats), so that a moving
// body can be advanced between steps at the cost of a few kernels, also inside a graph
// the caller captures.  *sized: whether the lists were (re)allocated.
int set_geometry_impl(ibm_ctx* c, Instance& I, const double* su, const double* sv, const double* sw,
                      bool* sized, int pending) {
  const GridParams& g = I.g;
  hipStream_t st = c->stream;
  const size_t nc = (size_t)g.ncell;
  const int cpr = (g.nx + IBM_WAVE - 1) / IBM_WAVE;
  const size_t nch = (size_t)g.nrows * cpr + 1;
  *sized = false;
  // the scan's tile sums: allocated at the first geometry of the instance and kept
  const int ntile = 7 * scan_tiles((int64_t)nch);
  const size_t tmp_bytes = (size_t)ntile * 4;
  if (!I.geo_tmp.p) {
    if (hipMalloc(&I.geo_tmp.p, tmp_bytes) != hipSuccess) {
      I.geo_tmp.p = nullptr;
      return fail(c, IBM_ERR_OOM, "geometry temporaries");
    }
    I.geo_tmp.bytes = tmp_bytes;
  }
  // per-(row, 64-wide chunk) counts of the seven tag masks, scanned in place into offsets
  // (those of the three immersed-boundary masks index the lists)
  if (!I.ibm_choff.p) {
    if (hipMalloc(&I.ibm_choff.p, 7 * nch * 4) != hipSuccess) {
      I.ibm_choff.p = nullptr;
      return fail(c, IBM_ERR_OOM, "immersed-boundary chunk offsets");
    }
    I.ibm_choff.bytes = 7 * nch * 4;
  }
  int32_t* choff = (int32_t*)I.ibm_choff.p;
  // I.itotal: [0..6] counts of internal u, v, w, p and immersed-boundary u, v, w points,
  // [8] the lists' overflow flag, [24] the S_k blocks' completion counter (zero between
  // launches)
  int32_t* cnt7 = I.itotal;
  int32_t* overflow = I.itotal + 8;
  unsigned* s_done = reinterpret_cast<unsigned*>(I.itotal + 24);
  const bool first = !I.ibm_idx.p || I.lists_overflowed;
  int rc = IBM_OK;
  do {
    // pending: PENDING_APPLIED, a projection applied just before has left phi and Pi to be
    // zeroed; PENDING_FUSE, the tag kernel applies it first (with the old tags, over the
    // predictor slot it came from), phi and Pi zeroed after
    const int esz = c->precision == IBM_FP64 ? 8 : 4;
    const bool fuse = pending == PENDING_FUSE;
    const double ck_dt = rk_c(2) * g.dt;
    hipError_t e = timed(c, K_GEOM, [&]() {
      if (c->precision == IBM_FP64) {
        Fields<double> f = fields_of<double>(I);
        f.us = f.usp; f.vs = f.vsp; f.ws = f.wsp;   // the predictor awaiting its projection
        return launch_geom_tags<double>(g, su, sv, sw, I.d.ibm, I.tag, fuse, f, I.wallv(), ck_dt, I.pi(), I.wall_j,
                                        I.wall_d, choff, overflow, st);
      }
      Fields<float> f = fields_of<float>(I);
      f.us = f.usp; f.vs = f.vsp; f.ws = f.wsp;
      return launch_geom_tags<float>(g, su, sv, sw, I.d.ibm, I.tag, fuse, f, I.wallv(), ck_dt, I.pi(), I.wall_j,
                                     I.wall_d, choff, overflow, st);
    });
    // the seven chunk-count arrays scanned in place (offsets), their totals into cnt7
    ScanSet set{};
    for (int m = 0; m < 7; ++m) {
      set.counts[m] = choff + (size_t)m * nch;
      set.n[m] = (int)nch;
      set.total[m] = cnt7 + m;
    }
    set.narr = 7;
    set.tsum = (int32_t*)I.geo_tmp.p;
    set.tsum_cap = ntile;
    if (e == hipSuccess) e = launch_scan_multi(set, st);
    if (e != hipSuccess) { rc = fail(c, IBM_ERR_DEVICE, std::string("geometry: ") + hipGetErrorString(e)); break; }
    if (first) {
      int32_t cnt[7];
      e = hipMemcpyAsync(cnt, cnt7, sizeof(cnt), hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) { rc = fail(c, IBM_ERR_DEVICE, std::string("geometry counts: ") + hipGetErrorString(e)); break; }
      if ((rc = sync_stream(c, st))) break;
      for (int q = 0; q < 3; ++q) {
        I.n_int[q] = cnt[q];
        I.n_ibm[q] = cnt[4 + q];
      }
      I.n_pint = cnt[3];
      if (I.n_pint == 0) { rc = fail(c, IBM_ERR_ARG, "geometry has no fluid"); break; }
      // list capacities: the counts plus a quarter (at least 1024 more), at most one per cell
      for (int q = 0; q < 3; ++q) {
        const int64_t n = I.n_ibm[q];
        I.cap[q] = (int)std::min<int64_t>((int64_t)nc, n + std::max<int64_t>(n / 4, 1024));
      }
      const int64_t ctot = (int64_t)I.cap[0] + I.cap[1] + I.cap[2];
      free_buf(I.ibm_idx);
      free_buf(I.ibm_coef);
      free_buf(I.ibm_lam);
      free_buf(I.ibm_sig);
      if (hipMalloc(&I.ibm_idx.p, ctot * 4) != hipSuccess || hipMalloc(&I.ibm_coef.p, ctot * 3 * 16) != hipSuccess ||
          hipMalloc(&I.ibm_lam.p, ctot * 8) != hipSuccess || hipMalloc(&I.ibm_sig.p, ctot * 8) != hipSuccess) {
        rc = fail(c, IBM_ERR_OOM, "immersed-boundary lists");
        break;
      }
      I.ibm_idx.bytes = ctot * 4;
      I.ibm_coef.bytes = ctot * 48;
      I.ibm_lam.bytes = ctot * 8;
      I.ibm_sig.bytes = ctot * 8;
      I.lists_overflowed = false;
      I.counts_fresh = true;
      *sized = true;
    } else {
      I.counts_fresh = false;   // the counts are on the device until the next ibm_stats
    }
    int32_t* idx = (int32_t*)I.ibm_idx.p;
    double2* coef = (double2*)I.ibm_coef.p;
    double* lamo = (double*)I.ibm_lam.p;
    double* sigo = (double*)I.ibm_sig.p;
    // (phi and Pi zeroed here: the tag kernel's correction has read phi)
    e = launch_compact3(I.tag, g, cpr, choff + 4 * nch, choff + 5 * nch, choff + 6 * nch, idx, I.cap, overflow,
                        pending ? I.phi : nullptr, esz, pending ? I.pi() : nullptr, st);
    if (e != hipSuccess) { rc = fail(c, IBM_ERR_DEVICE, std::string("ibm lists: ") + hipGetErrorString(e)); break; }
    I.L.choff_u = choff + 4 * nch;
    I.L.choff_v = choff + 5 * nch;
    I.L.choff_w = choff + 6 * nch;
    I.L.cpr = cpr;
    I.L.idx = idx;
    I.L.coef = coef;
    I.L.sig = sigo;
    I.L.wallv = I.wallv();
    I.L.sd = I.wall_sd();
    I.L.cnt = cnt7 + 4;
    I.L.n_u = I.cap[0];
    I.L.n_v = I.cap[1];
    I.L.n_w = I.cap[2];
    I.L.n_total = I.cap[0] + I.cap[1] + I.cap[2];
    I.L.n_cover = I.moving() ? I.L.n_total : I.L.n_u;
    // (with every listed point's lambda, sigma and per-stage coefficients)
    e = launch_s_k(g, I.tag, I.L, su, sv, sw, lamo, sigo, coef, I.d.dt, I.d.b_mode, I.red_part,
                   I.d.dt * y_scale(g) * g.dz / g.nx, I.S3(), cnt7, I.wall_sd(), s_done, st);
    if (e != hipSuccess) { rc = fail(c, IBM_ERR_DEVICE, std::string("S_k: ") + hipGetErrorString(e)); break; }
    if (first && (rc = sync_stream(c, st))) break;
    I.geom_ready = true;
    I.diag_valid = false;
  } while (0);
  return rc;
}

// Host copies of the point counts, refreshed from the device after geometries that ran
// without a read-back (synchronises); IBM_ERR_STATE if such a geometry overflowed the lists
// or left no fluid.
int refresh_counts(ibm_ctx* c, Instance& I) {
  if (I.counts_fresh || !I.geom_ready) return IBM_OK;
  int32_t cnt[9];
  HIPCHK(c, hipMemcpyAsync(cnt, I.itotal, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
  SYNCHK(c, c->stream);
  for (int q = 0; q < 3; ++q) {
    I.n_int[q] = cnt[q];
    I.n_ibm[q] = cnt[4 + q];
  }
  I.n_pint = cnt[3];
  I.counts_fresh = true;
  if (cnt[8]) {
    I.lists_overflowed = true;
    return fail(c, IBM_ERR_STATE,
                "the geometry has more immersed-boundary points than the lists reserved at the first geometry; "
                "give it again with ibm_set_geometry, which then resizes them");
  }
  if (I.n_pint == 0) return fail(c, IBM_ERR_STATE, "the current geometry has no fluid");
  return IBM_OK;
}

int check_inst(ibm_ctx* c, int32_t inst) {
  if (!c) return fail(nullptr, IBM_ERR_ARG, "null handle");
  if (inst < 0 || inst >= (int32_t)c->inst.size()) return fail(c, IBM_ERR_ARG, "instance index out of range");
  return IBM_OK;
}

void drop_batch(ibm_ctx* c) {
  if (c->batch.dbuf) (void)hipFree(c->batch.dbuf);
  c->batch = ibm_ctx::Batch{};
}

void drop_graph(ibm_ctx* c) {
  drop_batch(c);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
}

// Per-instance arguments of every step kernel for the batched launches (each grid's own
// launch shapes; the launch takes the largest template variant and LDS any grid needs).
template <typename T>
int build_batch(ibm_ctx* c) {
  drop_batch(c);
  ibm_ctx::Batch& b = c->batch;
  const int n = (int)c->inst.size();
  std::vector<MomArgs<T>> mom[3];
  std::vector<CfrArgs<T>> cfr[3];
  std::vector<DivArgs<T>> dv[3];
  std::vector<FftzArgs<T>> fzf(n), fzi(n);
  std::vector<TriArgs<T>> tri(n);
  std::vector<IfftxArgs<T>> ifx(n);
  for (int k = 0; k < 3; ++k) {
    mom[k].resize(n);
    cfr[k].resize(n);
    dv[k].resize(n);
  }
  std::vector<int> bo[6];
  std::vector<int> th_own(n, 256);   // each instance's own z-FFT threads
  for (auto& v : bo) v.assign(n + 1, 0);
  b.cur0.resize(n);
  for (int i = 0; i < n; ++i) {
    Instance& I = c->inst[i];
    const GridParams& g = I.g;
    const double scale = y_scale(g) * g.dz / g.nx;
    b.cur0[i] = I.cur;
    b.stretched = b.stretched || I.g.stretched;
    int nq = 0, mb = 1, th = 256, lm = 4;
    size_t lds = 0;
    for (int k = 0; k < 3; ++k) {
      const int ck = (I.cur + k) % 3, nx = (ck + 1) % 3;
      const StageConsts sc = stage_consts(g, k);
      Fields<T> fm = fields_at<T>(I, ck, nx);
      nq = plan_momentum<T>(g, fm, I.L, sc, I.pi(), rk_c((k + 2) % 3) * g.dt, I.tu, I.qpart, &mom[k][i]);
      Fields<T> f = fields_at<T>(I, nx, nx);
      const int nc = plan_cfr_pi<T>(f, I.L, k, sc.ck_dt, I.qpart, nq, scale, I.d.forcing, I.d.q_target_or_pi,
                                    I.S3(), I.pi(), I.pi_hist(), &cfr[k][i]);
      const int nd = plan_div_fftx<T>(g, f, I.L, k, I.px, I.rtw, sc.ck_dt, I.pi(), &dv[k][i], &mb, &lds);
      b.mb_div = std::max(b.mb_div, mb);
      b.lds_div = std::max(b.lds_div, lds);
      if (k == 0) {
        bo[0][i + 1] = nq;
        bo[1][i + 1] = nc;
        bo[2][i + 1] = nd;
      }
    }
    Fields<T> f = fields_of<T>(I);
    bo[3][i + 1] = plan_fftz<T>(g, f.spec, I.pz, -1, I.tu, &fzf[i], &mb, &lds, &th);
    (void)plan_fftz<T>(g, f.spec, I.pz, +1, I.tu, &fzi[i], &mb, &lds, &th);
    th_own[i] = th;
    b.mb_fz = std::max(b.mb_fz, mb);
    b.lds_fz = std::max(b.lds_fz, lds);
    b.th_fz = std::max(b.th_fz, th);
    bo[4][i + 1] = plan_tri<T>(g, f.spec, I.kx2, I.kz2, I.mean(), I.tu, &tri[i], &lm, &lds);
    b.lm_tri = std::max(b.lm_tri, lm);
    b.lds_tri = std::max(b.lds_tri, lds);
    bo[5][i + 1] = plan_ifftx<T>(g, f.spec, f.phi, I.px, I.rtw, &ifx[i], &mb, &lds);
    b.mb_ifx = std::max(b.mb_ifx, mb);
    b.lds_ifx = std::max(b.lds_ifx, lds);
  }
  // z FFTs of instances planned for fewer threads than the launch runs: columns widened
  // by the same factor (at most 64 modes, within the LDS), so that each column keeps the
  // lanes of the instance's own plan
  for (int i = 0; i < n; ++i) {
    const GridParams& g = c->inst[i].g;
    const int f = b.th_fz / th_own[i], W2 = fzf[i].W * f;
    const size_t l2 = ((size_t)W2 + 1) * g.nz * sizeof(cplx<T>);
    if (f > 1 && W2 <= 64 && W2 <= g.mh && l2 <= 163840) {
      fzf[i].W = fzi[i].W = W2;
      b.lds_fz = std::max(b.lds_fz, l2);
      bo[3][i + 1] = fftz_blocks(g.mh, g.ny1, W2, 1);
      fzf[i].gx = fzi[i].gx = bo[3][i + 1];
    }
  }
  // z FFTs: four planes per block with the next plane's columns in registers (RP per
  // thread) when every instance's share of a column, at the launch's thread count, fits 8
  // (the ensemble's many small planes: 307 us per launch with one plane per block, 291
  // with two, 276 with four or eight)
  int per = 0;
  for (int i = 0; i < n; ++i) per = std::max(per, (c->inst[i].g.nz + b.th_fz / fzf[i].W - 1) / (b.th_fz / fzf[i].W));
  b.rp_fz = per <= 4 ? 4 : (per <= 8 ? 8 : 0);
  if (b.rp_fz) {
    for (int i = 0; i < n; ++i) {
      const GridParams& g = c->inst[i].g;
      const int nb = fftz_blocks(g.mh, g.ny1, fzf[i].W, 4);
      fzf[i].nj = fzi[i].nj = 4;
      fzf[i].gx = fzi[i].gx = nb;
      bo[3][i + 1] = nb;
    }
  }
  // block offsets, then the instance of every block (the kernels' lookup table)
  for (auto& v : bo) {
    for (int i = 0; i < n; ++i) v[i + 1] += v[i];
    v.reserve(n + 1 + v[n]);
    for (int i = 0; i < n; ++i) v.insert(v.end(), v[i + 1] - v[i], i);
  }
  // pack everything into one host image (256-byte aligned pieces), then one device copy
  std::vector<unsigned char> img;
  auto put = [&](const void* src, size_t bytes) {
    const size_t off = (img.size() + 255) & ~(size_t)255;
    img.resize(off + bytes);
    memcpy(img.data() + off, src, bytes);
    return off;
  };
  size_t o_mom[3], o_cfr[3], o_div[3];
  for (int k = 0; k < 3; ++k) {
    o_mom[k] = put(mom[k].data(), n * sizeof(MomArgs<T>));
    o_cfr[k] = put(cfr[k].data(), n * sizeof(CfrArgs<T>));
    o_div[k] = put(dv[k].data(), n * sizeof(DivArgs<T>));
  }
  const size_t o_fzf = put(fzf.data(), n * sizeof(FftzArgs<T>)), o_fzi = put(fzi.data(), n * sizeof(FftzArgs<T>));
  const size_t o_tri = put(tri.data(), n * sizeof(TriArgs<T>)), o_ifx = put(ifx.data(), n * sizeof(IfftxArgs<T>));
  size_t o_bo[6];
  for (int q = 0; q < 6; ++q) o_bo[q] = put(bo[q].data(), bo[q].size() * sizeof(int));
  if (hipMalloc(&b.dbuf, img.size()) != hipSuccess) {
    b.dbuf = nullptr;
    return fail(c, IBM_ERR_OOM, "batched launch arguments");
  }
  HIPCHK(c, hipMemcpy(b.dbuf, img.data(), img.size(), hipMemcpyHostToDevice));
  unsigned char* d = (unsigned char*)b.dbuf;
  for (int k = 0; k < 3; ++k) {
    b.mom[k] = d + o_mom[k];
    b.cfr[k] = d + o_cfr[k];
    b.div[k] = d + o_div[k];
  }
  b.fzf = d + o_fzf;
  b.fzi = d + o_fzi;
  b.tri = d + o_tri;
  b.ifx = d + o_ifx;
  b.bo_mom = (const int*)(d + o_bo[0]);
  b.bo_cfr = (const int*)(d + o_bo[1]);
  b.bo_div = (const int*)(d + o_bo[2]);
  b.bo_fz = (const int*)(d + o_bo[3]);
  b.bo_tri = (const int*)(d + o_bo[4]);
  b.bo_ifx = (const int*)(d + o_bo[5]);
  b.n_mom = bo[0][n];
  b.n_cfr = bo[1][n];
  b.n_div = bo[2][n];
  b.n_fz = bo[3][n];
  b.n_tri = bo[4][n];
  b.n_ifx = bo[5][n];
  b.valid = true;
  return IBM_OK;
}

bool batch_current(ibm_ctx* c) {
  if (!c->batch.valid) return false;
  for (size_t i = 0; i < c->inst.size(); ++i)
    if (c->batch.cur0[i] != c->inst[i].cur) return false;
  return true;
}

// nsteps RK3 steps of every instance, one launch per kernel for the whole ensemble.
template <typename T>
int run_steps_batched(ibm_ctx* c, int nsteps, hipStream_t st, bool count = true) {
  const ibm_ctx::Batch& b = c->batch;
  const int n = (int)c->inst.size();
  for (int s = 0; s < nsteps; ++s) {
    for (int k = 0; k < 3; ++k) {
      RUNK(c, K_MOMENTUM, launch_momentum_b<T>((const MomArgs<T>*)b.mom[k], b.bo_mom, n, b.n_mom, b.stretched, st));
      for (Instance& I : c->inst) {
        I.cur = (I.cur + 1) % 3;
        I.fresh = false;
      }
      RUNK(c, K_CFR_PI, launch_cfr_pi_b<T>((const CfrArgs<T>*)b.cfr[k], b.bo_cfr, n, b.n_cfr, st));
      RUNK(c, K_DIV_FFTX, launch_div_fftx_b<T>((const DivArgs<T>*)b.div[k], b.bo_div, n, b.n_div, b.mb_div,
                                               b.lds_div, st));
      RUNK(c, K_FFTZ_FWD, launch_fftz_b<T>((const FftzArgs<T>*)b.fzf, b.bo_fz, n, b.n_fz, b.mb_fz, b.rp_fz, b.lds_fz,
                                           b.th_fz, st));
      RUNK(c, K_TRI, launch_tri_b<T>((const TriArgs<T>*)b.tri, b.bo_tri, n, b.n_tri, b.lm_tri, b.lds_tri, b.stretched, st));
      RUNK(c, K_FFTZ_INV, launch_fftz_b<T>((const FftzArgs<T>*)b.fzi, b.bo_fz, n, b.n_fz, b.mb_fz, b.rp_fz, b.lds_fz,
                                           b.th_fz, st));
      RUNK(c, K_IFFTX, launch_ifftx_b<T>((const IfftxArgs<T>*)b.ifx, b.bo_ifx, n, b.n_ifx, b.mb_ifx, b.lds_ifx,
                                         st));
    }
    if (!count) continue;
    for (Instance& I : c->inst) {
      I.step += 1;
      I.time += I.g.dt;
    }
  }
  return IBM_OK;
}

// Capture one RK3 step of every instance: instance i goes to capture stream i mod B,
// forked from and joined back to the origin stream, so that independent instances are
// independent branches of the graph.
template <typename T>
int build_graph(ibm_ctx* c) {
  drop_graph(c);
  bool masked = false;
  for (Instance& I : c->inst) masked = masked || I.d.projection == IBM_PROJ_MASKED;
  // batched launches have no masked projection: an ensemble with a masked instance is
  // captured as per-instance branches
  if (c->use_batch && c->inst.size() > 1 && !masked) {
    // the batched launches on one stream: seven nodes per substep for the whole ensemble
    int rc = build_batch<T>(c);
    if (rc) return rc;
    if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    rc = run_steps_batched<T>(c, 1, c->cap, false);
    hipGraph_t gr = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->cap, &gr);
    if (!rc && ee != hipSuccess) rc = fail(c, IBM_ERR_DEVICE, std::string("end capture: ") + hipGetErrorString(ee));
    if (rc) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    c->graph = gr;
    const hipError_t e = hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_graph(c);
      return fail(c, IBM_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return IBM_OK;
  }
  const int B = std::max(1, std::min<int>(c->n_branches > 0 ? c->n_branches : 8, (int)c->inst.size()));
  if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  if (!c->ev_fork) HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  while ((int)c->aux.size() < B) {
    hipStream_t s2;
    HIPCHK(c, hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    c->aux.push_back(s2);
    hipEvent_t e;
    HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->ev_join.push_back(e);
  }
  HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  int rc = IBM_OK;
  hipError_t e = hipEventRecord(c->ev_fork, c->cap);
  for (int b = 0; b < B && e == hipSuccess; ++b) e = hipStreamWaitEvent(c->aux[b], c->ev_fork, 0);
  if (e != hipSuccess) rc = fail(c, IBM_ERR_DEVICE, std::string("graph fork: ") + hipGetErrorString(e));
  for (size_t i = 0; i < c->inst.size() && !rc; ++i) rc = run_steps<T>(c, c->inst[i], 1, c->aux[i % B], false);
  for (int b = 0; b < B && !rc; ++b) {
    e = hipEventRecord(c->ev_join[b], c->aux[b]);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->cap, c->ev_join[b], 0);
    if (e != hipSuccess) rc = fail(c, IBM_ERR_DEVICE, std::string("graph join: ") + hipGetErrorString(e));
  }
  hipGraph_t gr = nullptr;
  const hipError_t ee = hipStreamEndCapture(c->cap, &gr);
  if (!rc && ee != hipSuccess) rc = fail(c, IBM_ERR_DEVICE, std::string("end capture: ") + hipGetErrorString(ee));
  if (rc) {
    if (gr) (void)hipGraphDestroy(gr);
    return rc;
  }
  c->graph = gr;
  e = hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(c);
    return fail(c, IBM_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  return IBM_OK;
}

}  // namespace

// =======================================================================================
// C ABI
// =======================================================================================
extern "C" {

int ibm_create_grid(const ibm_grid_desc* desc, int32_t n_inst, int32_t precision, void* hip_stream,
                    ibm_handle* out) {
  if (!desc || !out) return fail(nullptr, IBM_ERR_ARG, "null argument");
  *out = nullptr;
  if (n_inst < 1 || n_inst > 65536) return fail(nullptr, IBM_ERR_ARG, "n_inst must be in 1..65536");
  if (precision != IBM_FP64 && precision != IBM_FP32_STORAGE) return fail(nullptr, IBM_ERR_ARG, "invalid precision");
  ibm_ctx* c = new (std::nothrow) ibm_ctx();
  if (!c) return fail(nullptr, IBM_ERR_OOM, "host allocation");
  c->precision = precision;
  c->stream = (hipStream_t)hip_stream;
  int rc = IBM_OK;
  for (int i = 0; i < n_inst && !rc; ++i) rc = validate(c, desc[i]);
  if (!rc) {
    c->inst.resize(n_inst);
    for (int i = 0; i < n_inst && !rc; ++i) rc = init_instance(c, c->inst[i], desc[i]);
  }
  if (!rc) rc = sync_stream(c, c->stream);
  if (rc) {
    ibm_destroy(c);
    return rc;
  }
  *out = c;
  return IBM_OK;
}

int ibm_set_geometry(ibm_handle h, int32_t inst, const double* sdf_u, const double* sdf_v, const double* sdf_w) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  if (!sdf_u || !sdf_v || !sdf_w) return fail(h, IBM_ERR_ARG, "null SDF pointer");
  Instance& I = h->inst[inst];
  // the first geometry (or one after the lists overflowed) sizes the lists and
  // synchronises; later ones only enqueue kernels and keep the captured graph
  const bool sizing = !I.ibm_idx.p || I.lists_overflowed;
  if (sizing) {
    if ((rc = refuse_capture(h))) return rc;
    drop_graph(h);
  }
  // a pending projection belongs to the old geometry: it is applied (with its tags) and
  // the result made the start of the next substep, which the new tags then act on.  Under
  // a caller's capture it is recorded even if nothing is pending now, since the replays
  // follow steps (with nothing pending it only resets the external points)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(h->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) I.fresh = false;
  const bool pending = !I.fresh;
  int how = PENDING_NONE;
  if (pending && !sizing) {
    // applied by the geometry's first kernel, as materialize(seed) would have
    how = PENDING_FUSE;
    I.fresh = true;
    I.state_in_slot = true;
  } else if (pending) {
    if ((rc = materialize(h, I, true))) return rc;
    how = PENDING_APPLIED;
  }
  bool sized = false;
  if ((rc = set_geometry_impl(h, I, sdf_u, sdf_v, sdf_w, &sized, how))) {
    // (an update that failed before zeroing them must not leave phi and Pi to be applied
    // a second time)
    if (pending) {
      (void)launch_fill_zero(I.phi, (int64_t)I.g.ncell * (h->precision == IBM_FP64 ? 8 : 4), h->stream);
      (void)launch_fill_zero(I.pi(), (int64_t)sizeof(double), h->stream);
    }
    return rc;
  }
  if (sized) drop_graph(h);
  return IBM_OK;
}

int ibm_set_state(ibm_handle h, int32_t inst, const void* u, const void* v, const void* w, const void* p) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  Instance& I = h->inst[inst];
  const size_t fb = (size_t)I.g.ncell * (h->precision == IBM_FP64 ? 8 : 4);
  const void* src[4] = {u, v, w, p};
  void* dst[4] = {I.u, I.v, I.w, I.p};
  for (int q = 0; q < 4; ++q)
    if (!src[q]) return fail(h, IBM_ERR_ARG, "null state pointer");
  for (int q = 0; q < 4; ++q) HIPCHK(h, hipMemcpyAsync(dst[q], src[q], fb, hipMemcpyDeviceToDevice, h->stream));
  I.diag_valid = false;
  return seed_pending(h, I);
}

int ibm_get_state(ibm_handle h, int32_t inst, void* u, void* v, void* w, void* p) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  if ((rc = refuse_capture(h))) return rc;
  Instance& I = h->inst[inst];
  const size_t fb = (size_t)I.g.ncell * (h->precision == IBM_FP64 ? 8 : 4);
  if ((rc = materialize(h, I))) return rc;
  void* dst[4] = {u, v, w, p};
  const void* src[4] = {I.u, I.v, I.w, I.p};
  for (int q = 0; q < 4; ++q) {
    if (!dst[q]) continue;
    HIPCHK(h, hipMemcpyAsync(dst[q], src[q], fb, hipMemcpyDeviceToDevice, h->stream));
  }
  return IBM_OK;
}

int ibm_step(ibm_handle h, int32_t nsteps) {
  if (!h) return fail(nullptr, IBM_ERR_ARG, "null handle");
  if (nsteps < 0) return fail(h, IBM_ERR_ARG, "nsteps < 0");
  for (Instance& I : h->inst)
    if (!I.geom_ready) return fail(h, IBM_ERR_STATE, "ibm_step before ibm_set_geometry");
  bool masked = false;
  for (Instance& I : h->inst) masked = masked || I.d.projection == IBM_PROJ_MASKED;
  // a masked solve synchronises in eager steps and a graph is built by a capture of the
  // library's own: neither inside the caller's capture of the stream
  if (masked || h->use_graph) {
    const int rc = refuse_capture(h);
    if (rc) return rc;
  }
  const bool batched = h->use_batch && h->inst.size() > 1 && !h->diag && !h->prof && !masked;
  if (h->use_graph && !h->diag && !h->prof && masked && nsteps > 0) {
    // a masked instance's iteration budget in the graph comes from its eager solves: a
    // first step runs eagerly when none has been made yet; the graph is rebuilt when a
    // budget changes
    bool need = false;
    for (Instance& I : h->inst) need = need || (I.d.projection == IBM_PROJ_MASKED && !I.pcg_seen);
    if (need) {
      for (Instance& I : h->inst) {
        const int rc = (h->precision == IBM_FP64) ? run_steps<double>(h, I, 1, h->stream)
                                                  : run_steps<float>(h, I, 1, h->stream);
        if (rc) return rc;
      }
      if (--nsteps == 0) return IBM_OK;
    }
    for (Instance& I : h->inst) {
      if (I.d.projection != IBM_PROJ_MASKED) continue;
      const int b = pcg_capture_budget(I);
      if (b != I.pcg_budget) {
        I.pcg_budget = b;
        drop_graph(h);
      }
    }
  }
  if (h->use_graph && !h->diag && !h->prof && nsteps > 0) {
    if (!h->gexec || (batched && !batch_current(h))) {
      const int rc = (h->precision == IBM_FP64) ? build_graph<double>(h) : build_graph<float>(h);
      if (rc) return rc;
    }
    for (int s = 0; s < nsteps; ++s) HIPCHK(h, hipGraphLaunch(h->gexec, h->stream));
    for (Instance& I : h->inst) {
      I.step += nsteps;
      I.time += nsteps * I.g.dt;
      I.fresh = false;
    }
    return IBM_OK;
  }
  if (batched && nsteps > 0) {
    if (!batch_current(h)) {
      const int rc = (h->precision == IBM_FP64) ? build_batch<double>(h) : build_batch<float>(h);
      if (rc) return rc;
    }
    return (h->precision == IBM_FP64) ? run_steps_batched<double>(h, nsteps, h->stream)
                                      : run_steps_batched<float>(h, nsteps, h->stream);
  }
  for (Instance& I : h->inst) {
    const int rc = (h->precision == IBM_FP64) ? run_steps<double>(h, I, nsteps, h->stream)
                                              : run_steps<float>(h, I, nsteps, h->stream);
    if (rc) return rc;
  }
  return IBM_OK;
}

int ibm_solve_pressure(ibm_handle h, int32_t inst, const void* rhs, void* phi) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  if (!rhs || !phi) return fail(h, IBM_ERR_ARG, "null pointer");
  Instance& I = h->inst[inst];
  if (h->precision == IBM_FP64) {
    Fields<double> f = fields_of<double>(I);
    RUNK(h, K_DIV_FFTX, launch_div_fftx<double>(I.g, f, I.L, 0, I.px, I.rtw, 1.0, I.pi(), (const double*)rhs,
                                                 h->stream));
    return poisson<double>(h, I, I.g, f, (double*)phi, h->stream);
  }
  Fields<float> f = fields_of<float>(I);
  RUNK(h, K_DIV_FFTX, launch_div_fftx<float>(I.g, f, I.L, 0, I.px, I.rtw, 1.0, I.pi(), (const float*)rhs,
                                              h->stream));
  return poisson<float>(h, I, I.g, f, (float*)phi, h->stream);
}

int ibm_set_diagnostics(ibm_handle h, int32_t on) {
  if (!h) return fail(nullptr, IBM_ERR_ARG, "null handle");
  h->diag = on != 0;
  drop_graph(h);
  return IBM_OK;
}

int ibm_set_wall_velocity(ibm_handle h, int32_t inst, double ub, double vb, double wb) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  if (!std::isfinite(ub) || !std::isfinite(vb) || !std::isfinite(wb))
    return fail(h, IBM_ERR_ARG, "wall velocity must be finite");
  if ((rc = refuse_capture(h))) return rc;
  Instance& I = h->inst[inst];
  // a pending projection is applied with the walls' previous velocity at external faces
  if ((rc = materialize(h, I))) return rc;
  const double v[3] = {ub, vb, wb};
  HIPCHK(h, hipMemcpyAsync(I.wallv(), v, sizeof(v), hipMemcpyHostToDevice, h->stream));
  SYNCHK(h, h->stream);
  I.wall_vel[0] = ub;
  I.wall_vel[1] = vb;
  I.wall_vel[2] = wb;
  // with moving walls the flow-rate kernel visits every immersed-boundary point (the
  // launch shape changes: captured graphs and batched arguments are rebuilt)
  I.L.n_cover = I.moving() ? I.L.n_total : I.L.n_u;
  drop_graph(h);
  return seed_pending(h, I);
}

int ibm_set_y_faces(ibm_handle h, int32_t inst, const double* y_faces) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  if (!y_faces) return fail(h, IBM_ERR_ARG, "null y_faces");
  if ((rc = refuse_capture(h))) return rc;
  Instance& I = h->inst[inst];
  const int ny = I.g.ny1 + 1;
  const double H = I.d.y_hi - I.d.y_lo;
  for (int j = 0; j < ny; ++j)
    if (!std::isfinite(y_faces[j])) return fail(h, IBM_ERR_ARG, "y_faces must be finite");
  if (std::fabs(y_faces[0] - I.d.y_lo) > 1e-12 * H || std::fabs(y_faces[ny - 1] - I.d.y_hi) > 1e-12 * H)
    return fail(h, IBM_ERR_ARG, "y_faces must start at y_lo and end at y_hi");
  for (int j = 0; j + 1 < ny; ++j)
    if (!(y_faces[j + 1] > y_faces[j])) return fail(h, IBM_ERR_ARG, "y_faces must increase strictly");
  drop_graph(h);
  if ((rc = materialize(h, I))) return rc;
  const std::vector<double> tab = y_tables(y_faces, I.g.ny1);
  HIPCHK(h, hipMemcpyAsync((void*)I.g.ytab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice,
                           h->stream));
  SYNCHK(h, h->stream);
  I.g.stretched = 1;
  // lambda, sigma, the wall distances and S_k depend on the spacing: a geometry is needed
  I.geom_ready = false;
  return IBM_OK;
}

int ibm_wall_shear(ibm_handle h, int32_t inst, double* tau_x, double* modes) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  Instance& I = h->inst[inst];
  if (!I.geom_ready) return fail(h, IBM_ERR_STATE, "ibm_wall_shear before ibm_set_geometry");
  if (modes && (rc = refuse_capture(h))) return rc;
  if ((rc = materialize(h, I))) return rc;
  const GridParams& g = I.g;
  double* tx = tau_x ? tau_x : I.wall_tau;
  double* md = modes ? I.wall_tau + g.nx : nullptr;
  if (h->precision == IBM_FP64) {
    RUNK(h, K_WALL_SHEAR,
         launch_wall_shear<double>(g, (const double*)I.u, I.wall_j, I.wall_d, I.wallv(), tx, md, h->stream));
  } else {
    RUNK(h, K_WALL_SHEAR,
         launch_wall_shear<float>(g, (const float*)I.u, I.wall_j, I.wall_d, I.wallv(), tx, md, h->stream));
  }
  if (modes) {
    HIPCHK(h, hipMemcpyAsync(modes, md, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    SYNCHK(h, h->stream);
  }
  return IBM_OK;
}

int ibm_stats(ibm_handle h, int32_t inst, ibm_stats_t* out) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  if (!out) return fail(h, IBM_ERR_ARG, "null output");
  if ((rc = refuse_capture(h))) return rc;
  Instance& I = h->inst[inst];
  if ((rc = refresh_counts(h, I))) return rc;
  const GridParams& g = I.g;
  if ((rc = materialize(h, I))) return rc;
  int np = 0;
  if (h->precision == IBM_FP64) {
    RUNK(h, K_STATS, launch_stats<double>(g, fields_of<double>(I), I.red_part, &np, h->stream));
  } else {
    RUNK(h, K_STATS, launch_stats<float>(g, fields_of<float>(I), I.red_part, &np, h->stream));
  }
  RUNK(h, K_STATS, launch_reduce_final(I.red_part, np, 3, 3, I.red_out(), h->stream));
  double host[32];
  HIPCHK(h, hipMemcpyAsync(host, I.small, sizeof(host), hipMemcpyDeviceToHost, h->stream));
  // the masked solve's device status: converged flag, iterations, |r|^2
  int32_t pstat[PCG_NSTAT] = {1, 0, 0, 0};
  double prr = 0.0;
  const bool masked = I.d.projection == IBM_PROJ_MASKED;
  if (masked) {
    HIPCHK(h, hipMemcpyAsync(pstat, I.pcg_stat, sizeof(pstat), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(&prr, I.pcg_stat + PCG_NSTAT, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  }
  SYNCHK(h, h->stream);
  const double* ro = host + 7;
  const double* dg = host + 15;
  memset(out, 0, sizeof(*out));
  out->step = I.step;
  out->time = I.time;
  out->q = ro[0] * y_scale(g) * g.dz / g.nx;
  out->pi_last = host[4];
  out->ke = 0.5 * ro[1] * g.dx * y_scale(g) * g.dz;
  out->nan_flag = ro[2] > 0.0 ? 1 : 0;
  out->cfl_max = ro[3];
  out->div_max_internal_leak = ro[4];
  out->rhs_mean_removed = host[6];
  if (masked) {
    // |b|^2 of the last solve is in pcg_sc()[2] = small[22]
    const double bb = host[22];
    out->div_max_fullbox = -1.0;
    out->poisson_rel_residual = I.step > 0 ? (bb > 0.0 ? std::sqrt(prr / bb) : 0.0) : -1.0;
    out->pcg_iters = pstat[PCG_ITERS];
    if (pstat[PCG_DONE]) I.pcg_iters_max = std::max(I.pcg_iters_max, (int)pstat[PCG_ITERS]);
  } else if (I.diag_valid) {
    out->div_max_fullbox = dg[0];
    out->poisson_rel_residual = dg[2] > 0.0 ? dg[1] / dg[2] : 0.0;
  } else {
    out->div_max_fullbox = -1.0;
    out->poisson_rel_residual = -1.0;
  }
  for (int q = 0; q < 3; ++q) {
    out->n_internal[q] = I.n_int[q];
    out->n_ibm[q] = I.n_ibm[q];
  }
  out->n_p_internal = I.n_pint;
  if (out->nan_flag) return fail(h, IBM_ERR_UNSTABLE, "NaN/Inf in the state");
  if (masked && I.step > 0 && !pstat[PCG_DONE])
    return fail(h, IBM_ERR_UNSTABLE,
                I.pcg_budget > 0 ? "masked projection did not converge within the iterations captured (" +
                                       std::to_string(I.pcg_budget) + " per solve)"
                                 : std::string("masked projection did not converge"));
  if (out->cfl_max > std::sqrt(3.0)) return fail(h, IBM_ERR_UNSTABLE, "CFL above sqrt(3)");
  return IBM_OK;
}

int ibm_get_geometry(ibm_handle h, int32_t inst, uint8_t* tags, int64_t* n_ibm3) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  Instance& I = h->inst[inst];
  if (!I.geom_ready) return fail(h, IBM_ERR_STATE, "no geometry");
  if ((rc = refuse_capture(h))) return rc;
  if ((rc = refresh_counts(h, I))) return rc;
  if (tags) HIPCHK(h, hipMemcpyAsync(tags, I.tag, (size_t)I.g.ncell, hipMemcpyDeviceToDevice, h->stream));
  SYNCHK(h, h->stream);
  if (n_ibm3)
    for (int q = 0; q < 3; ++q) n_ibm3[q] = I.n_ibm[q];
  return IBM_OK;
}

int ibm_get_ibm_list(ibm_handle h, int32_t inst, int32_t comp, int32_t* idx, double* lambda, double* coef) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  Instance& I = h->inst[inst];
  if (!I.geom_ready) return fail(h, IBM_ERR_STATE, "no geometry");
  if ((rc = refuse_capture(h))) return rc;
  if (comp < 0 || comp > 2) return fail(h, IBM_ERR_ARG, "comp must be 0, 1 or 2");
  if ((rc = refresh_counts(h, I))) return rc;
  // the component lists lie end to end at their capacities
  const int64_t off = (comp >= 1 ? I.cap[0] : 0) + (comp >= 2 ? I.cap[1] : 0);
  const int64_t n = I.n_ibm[comp];
  const int64_t ntot = I.L.n_total;
  if (n > 0) {
    if (idx)
      HIPCHK(h, hipMemcpyAsync(idx, (int32_t*)I.ibm_idx.p + off, n * 4, hipMemcpyDeviceToDevice, h->stream));
    if (lambda)
      HIPCHK(h, hipMemcpyAsync(lambda, (double*)I.ibm_lam.p + off, n * 8, hipMemcpyDeviceToDevice, h->stream));
    if (coef)
      for (int k = 0; k < 3; ++k)
        HIPCHK(h, hipMemcpyAsync(coef + (size_t)k * n * 2, (double2*)I.ibm_coef.p + k * ntot + off, n * 16,
                                 hipMemcpyDeviceToDevice, h->stream));
  }
  SYNCHK(h, h->stream);
  return IBM_OK;
}

int ibm_tune_set(ibm_handle h, int32_t param, int32_t value) {
  if (!h) return fail(nullptr, IBM_ERR_ARG, "null handle");
  if (value < 0) return fail(h, IBM_ERR_ARG, "tuning value must be >= 0 (0 = automatic)");
  drop_graph(h);
  if (param == IBM_TUNE_GRAPH) {
    h->use_graph = value != 0;
    return IBM_OK;
  }
  if (param == IBM_TUNE_BATCH) {
    h->use_batch = value != 0;
    return IBM_OK;
  }
  if (param == IBM_TUNE_GRAPH_BRANCHES) {
    h->n_branches = value;
    return IBM_OK;
  }
  for (Instance& I : h->inst) {
    switch (param) {
      case IBM_TUNE_MOMENTUM_PLANES: I.tu.mom_jc = value; break;
      case IBM_TUNE_TILE_ORDER:
        if (value > 8) return fail(h, IBM_ERR_ARG, "tile order must be 0..8");
        I.tu.tile_order = value;
        break;
      case IBM_TUNE_MOMENTUM_TILE:
        if (value > 6) return fail(h, IBM_ERR_ARG, "momentum tile must be 0..6");
        I.tu.mom_tile = value;
        break;
      case IBM_TUNE_MOMENTUM_CACHE:
        if (value > 4) return fail(h, IBM_ERR_ARG, "momentum cache policy must be 0..4");
        I.tu.mom_cache = value;
        break;
      case IBM_TUNE_FFTZ_WIDTH: I.tu.fftz_w = value; break;
      case IBM_TUNE_TRI_ROWS:
        if (value != 0 && value != 4 && value != 8) return fail(h, IBM_ERR_ARG, "tri rows must be 0, 4 or 8");
        I.tu.tri_rows = value;
        break;
      default: return fail(h, IBM_ERR_ARG, "unknown tuning parameter");
    }
  }
  return IBM_OK;
}

int ibm_tune_get(ibm_handle h, int32_t param, int32_t* value) {
  if (!h || !value) return fail(h, IBM_ERR_ARG, "null argument");
  const Tuning& t = h->inst[0].tu;
  switch (param) {
    case IBM_TUNE_MOMENTUM_PLANES: *value = t.mom_jc; break;
    case IBM_TUNE_TILE_ORDER: *value = t.tile_order; break;
    case IBM_TUNE_MOMENTUM_CACHE: *value = t.mom_cache; break;
    case IBM_TUNE_MOMENTUM_TILE: *value = t.mom_tile; break;
    case IBM_TUNE_FFTZ_WIDTH: *value = t.fftz_w; break;
    case IBM_TUNE_TRI_ROWS: *value = t.tri_rows; break;
    case IBM_TUNE_GRAPH: *value = h->use_graph ? 1 : 0; break;
    case IBM_TUNE_GRAPH_BRANCHES: *value = h->n_branches; break;
    case IBM_TUNE_BATCH: *value = h->use_batch ? 1 : 0; break;
    default: return fail(h, IBM_ERR_ARG, "unknown tuning parameter");
  }
  return IBM_OK;
}

}  // extern "C"

namespace {
template <typename T>
int autotune_impl(ibm_ctx* c, Instance& I, int steps, int32_t* chosen) {
  const GridParams& g = I.g;
  const size_t fb = (size_t)g.ncell * sizeof(T);
  void* save[4] = {nullptr, nullptr, nullptr, nullptr};
  void* fld[4] = {I.u, I.v, I.w, I.p};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = IBM_OK;
  const int64_t step0 = I.step;
  const double time0 = I.time;
  const bool prof = c->prof, diag = c->diag;
  c->prof = false;
  c->diag = false;
  auto cleanup = [&]() {
    for (void* p : save)
      if (p) (void)hipFree(p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c->prof = prof;
    c->diag = diag;
  };
  for (int q = 0; q < 4; ++q)
    if (hipMalloc(&save[q], fb) != hipSuccess) {
      cleanup();
      return fail(c, IBM_ERR_OOM, "autotune state copy");
    }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(c, IBM_ERR_DEVICE, "autotune events");
  }
  if (!rc) rc = materialize(c, I);
  for (int q = 0; q < 4 && !rc; ++q)
    if (hipMemcpyAsync(save[q], fld[q], fb, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
      rc = fail(c, IBM_ERR_DEVICE, "autotune save");
  // time `steps` steps from the saved state with the current knobs (best of two runs)
  auto trial = [&](float* ms) -> int {
    *ms = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      for (int q = 0; q < 4; ++q)
        if (hipMemcpyAsync(fld[q], save[q], fb, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
          return fail(c, IBM_ERR_DEVICE, "autotune restore");
      int r = seed_pending(c, I);
      if (r) return r;
      r = run_steps<T>(c, I, 1, c->stream);
      if (r) return r;
      if (hipEventRecord(e0, c->stream) != hipSuccess) return fail(c, IBM_ERR_DEVICE, "event");
      r = run_steps<T>(c, I, steps, c->stream);
      if (r) return r;
      float t = 0.f;
      if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&t, e0, e1) != hipSuccess)
        return fail(c, IBM_ERR_DEVICE, "autotune timing");
      if (t < *ms) *ms = t;
    }
    return IBM_OK;
  };
  // candidates per knob, searched one knob at a time
  std::vector<int> to = {1, 2, 3, 4, 5, 6, 7, 8};
  std::vector<int> jc = {0, 2, 4, 6, 8, 10, 12, 14, 16, 20, 24, 32, 48, 64};
  int wv[8];
  const int nw = fftz_widths<T>(g, I.pz, wv, 8);
  std::vector<int> fw(wv, wv + nw);
  std::vector<int> tr = {8, 4};
  std::vector<int>* cand[4] = {&jc, &fw, &tr, &to};
  int* knob[4] = {&I.tu.mom_jc, &I.tu.fftz_w, &I.tu.tri_rows, &I.tu.tile_order};
  // the tile order first (with the default plane chunk), then the others, then the tile
  // order again with the chosen plane chunk
  const int order[5] = {3, 0, 1, 2, 3};
  for (int oq = 0; oq < 5 && !rc; ++oq) {
    const int kq = order[oq];
    float best = 1e30f;
    int bestv = *knob[kq];
    for (int v : *cand[kq]) {
      if (kq == 0 && v > g.ny1) continue;
      *knob[kq] = v;
      float ms = 0.f;
      rc = trial(&ms);
      if (rc) break;
      if (ms < best) {
        best = ms;
        bestv = v;
      }
    }
    *knob[kq] = bestv;
    if (chosen) chosen[kq] = bestv;
  }
  for (int q = 0; q < 4 && !rc; ++q)
    if (hipMemcpyAsync(fld[q], save[q], fb, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
      rc = fail(c, IBM_ERR_DEVICE, "autotune restore");
  if (!rc) rc = seed_pending(c, I);
  if (!rc) rc = sync_stream(c, c->stream);
  I.step = step0;
  I.time = time0;
  I.diag_valid = false;
  cleanup();
  return rc;
}

// Ensembles launched together (one launch per kernel for all instances): the
// knobs that decide how the instances share the GPU (y planes per momentum block, tile
// order) are tuned jointly by timing whole ensemble steps in that launch mode, the same
// value for every instance; the other knobs keep their per-grid values.  The state of
// every instance is saved and restored.
template <typename T>
int autotune_ensemble(ibm_ctx* c, int steps, int32_t* chosen) {
  const size_t ni = c->inst.size();
  std::vector<void*> save(4 * ni, nullptr);
  std::vector<int64_t> step0(ni);
  std::vector<double> time0(ni);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool prof = c->prof, diag = c->diag;
  c->prof = false;
  c->diag = false;
  auto cleanup = [&]() {
    for (void* p : save)
      if (p) (void)hipFree(p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c->prof = prof;
    c->diag = diag;
  };
  int rc = IBM_OK;
  for (size_t i = 0; i < ni && !rc; ++i) {
    Instance& I = c->inst[i];
    step0[i] = I.step;
    time0[i] = I.time;
    const size_t fb = (size_t)I.g.ncell * sizeof(T);
    void* fld[4] = {I.u, I.v, I.w, I.p};
    rc = materialize(c, I);
    for (int q = 0; q < 4 && !rc; ++q) {
      if (hipMalloc(&save[4 * i + q], fb) != hipSuccess)
        rc = fail(c, IBM_ERR_OOM, "autotune state copy");
      else if (hipMemcpyAsync(save[4 * i + q], fld[q], fb, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        rc = fail(c, IBM_ERR_DEVICE, "autotune save");
    }
  }
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = fail(c, IBM_ERR_DEVICE, "autotune events");
  auto restore = [&]() -> int {
    for (size_t i = 0; i < ni; ++i) {
      Instance& I = c->inst[i];
      const size_t fb = (size_t)I.g.ncell * sizeof(T);
      void* fld[4] = {I.u, I.v, I.w, I.p};
      for (int q = 0; q < 4; ++q)
        if (hipMemcpyAsync(fld[q], save[4 * i + q], fb, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
          return fail(c, IBM_ERR_DEVICE, "autotune restore");
      const int r = seed_pending(c, I);
      if (r) return r;
      I.step = step0[i];
      I.time = time0[i];
      I.diag_valid = false;
    }
    return IBM_OK;
  };
  // `steps` ensemble steps in the current launch mode from the saved states, after one
  // step that builds the graph or the batched arguments (best of two runs)
  auto trial = [&](float* ms) -> int {
    *ms = 1e30f;
    drop_graph(c);
    for (int rep = 0; rep < 2; ++rep) {
      int r = restore();
      if (!r) r = ibm_step(c, 1);
      if (r) return r;
      if (hipEventRecord(e0, c->stream) != hipSuccess) return fail(c, IBM_ERR_DEVICE, "event");
      r = ibm_step(c, steps);
      if (r) return r;
      float t = 0.f;
      if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&t, e0, e1) != hipSuccess)
        return fail(c, IBM_ERR_DEVICE, "autotune timing");
      if (t < *ms) *ms = t;
    }
    return IBM_OK;
  };
  const std::vector<int> jc = {0, 8, 16, 24, 32, 48};
  const std::vector<int> to = {1, 2};
  const std::vector<int>* cand[2] = {&jc, &to};
  const int slot[2] = {0, 3};
  for (int kq = 0; kq < 2 && !rc; ++kq) {
    float best = 1e30f;
    int bestv = kq == 0 ? c->inst[0].tu.mom_jc : c->inst[0].tu.tile_order;
    for (int v : *cand[kq]) {
      for (Instance& I : c->inst) (kq == 0 ? I.tu.mom_jc : I.tu.tile_order) = v;
      float ms = 0.f;
      rc = trial(&ms);
      if (rc) break;
      if (ms < best) {
        best = ms;
        bestv = v;
      }
    }
    for (Instance& I : c->inst) (kq == 0 ? I.tu.mom_jc : I.tu.tile_order) = bestv;
    if (chosen) chosen[slot[kq]] = bestv;
  }
  if (chosen && !rc) {
    chosen[1] = c->inst[0].tu.fftz_w;
    chosen[2] = c->inst[0].tu.tri_rows;
  }
  if (!rc) rc = restore();
  if (!rc) rc = sync_stream(c, c->stream);
  drop_graph(c);
  cleanup();
  return rc;
}

}  // namespace

extern "C" {

int ibm_autotune(ibm_handle h, int32_t steps_per_trial, int32_t* chosen) {
  if (!h) return fail(nullptr, IBM_ERR_ARG, "null handle");
  if (steps_per_trial < 1) return fail(h, IBM_ERR_ARG, "steps_per_trial must be >= 1");
  int rc0 = refuse_capture(h);
  if (rc0) return rc0;
  drop_graph(h);
  for (Instance& I : h->inst)
    if (!I.geom_ready) return fail(h, IBM_ERR_STATE, "autotune before ibm_set_geometry");
  // the joint tuner serves ensembles launched as one launch per kernel for all instances;
  // an ensemble of per-instance graph branches is tuned one instance at a time (eager
  // launches), as are single grids
  if (h->inst.size() > 1 && h->use_batch)
    return (h->precision == IBM_FP64) ? autotune_ensemble<double>(h, steps_per_trial, chosen)
                                      : autotune_ensemble<float>(h, steps_per_trial, chosen);
  for (Instance& I : h->inst) {
    if (!I.geom_ready) return fail(h, IBM_ERR_STATE, "autotune before ibm_set_geometry");
    const int rc = (h->precision == IBM_FP64) ? autotune_impl<double>(h, I, steps_per_trial, chosen)
                                              : autotune_impl<float>(h, I, steps_per_trial, chosen);
    if (rc) return rc;
  }
  return IBM_OK;
}

int ibm_profile(ibm_handle h, int32_t on) {
  if (!h) return fail(nullptr, IBM_ERR_ARG, "null handle");
  if (on && h->ev.empty()) {
    const size_t n = 2 * 65536;
    h->ev.resize(n);
    h->ev_kid.resize(n / 2);
    for (size_t e = 0; e < n; ++e) HIPCHK(h, hipEventCreate(&h->ev[e]));
  }
  h->prof = on != 0;
  h->prof_mask = (uint32_t)on;
  return IBM_OK;
}

int ibm_profile_read(ibm_handle h, double* total_ms, int64_t* launches, int32_t max) {
  if (!h) return fail(nullptr, IBM_ERR_ARG, "null handle");
  SYNCHK(h, h->stream);
  for (size_t e = 0; e + 1 < h->ev_used; e += 2) {
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, h->ev[e], h->ev[e + 1]));
    const int kid = h->ev_kid[e / 2];
    h->prof_ms[kid] += ms;
    h->prof_n[kid] += 1;
  }
  h->ev_used = 0;
  for (int k = 0; k < K_NUM_KERNELS && k < max; ++k) {
    if (total_ms) total_ms[k] = h->prof_ms[k];
    if (launches) launches[k] = h->prof_n[k];
    h->prof_ms[k] = 0.0;
    h->prof_n[k] = 0;
  }
  return IBM_OK;
}

const char* ibm_kernel_name(int32_t id) {
  static const char* names[K_NUM_KERNELS] = {"momentum", "cfr_pi", "div_fftx", "fftz_fwd", "tri", "fftz_inv",
                                             "ifftx", "correct", "diag", "stats", "geom",
                                             "wall_shear", "pcg"};
  if (id < 0 || id >= K_NUM_KERNELS) return "unknown";
  return names[id];
}

int32_t ibm_num_kernels(void) { return K_NUM_KERNELS; }

int64_t ibm_device_bytes(ibm_handle h) {
  if (!h) return 0;
  int64_t b = 0;
  for (Instance& I : h->inst) {
    for (auto& x : I.bufs) b += (int64_t)x.bytes;
    b += I.ibm_idx.bytes + I.ibm_coef.bytes + I.ibm_lam.bytes + I.ibm_sig.bytes + I.ibm_choff.bytes +
         I.geo_tmp.bytes;
  }
  return b;
}

int ibm_stream_copy(void* dst, const void* src, int64_t bytes, void* hip_stream) {
  if (!dst || !src) return fail(nullptr, IBM_ERR_ARG, "null pointer");
  if (((uintptr_t)dst | (uintptr_t)src) % 16 != 0) return fail(nullptr, IBM_ERR_ARG, "pointers must be 16-byte aligned");
  if (bytes < 0 || bytes % 16 != 0) return fail(nullptr, IBM_ERR_ARG, "bytes must be a non-negative multiple of 16");
  const uintptr_t d = (uintptr_t)dst, s = (uintptr_t)src;
  if (d < s + (uintptr_t)bytes && s < d + (uintptr_t)bytes && bytes > 0)
    return fail(nullptr, IBM_ERR_ARG, "source and destination overlap");
  const hipError_t e = launch_stream_copy(src, dst, bytes / 16, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(nullptr, IBM_ERR_DEVICE, std::string("stream copy: ") + hipGetErrorString(e));
  return IBM_OK;
}

int ibm_stream_mix(void* const* dst, int32_t ndst, const void* const* src, int32_t nsrc, int64_t bytes,
                   void* hip_stream) {
  if (!dst || !src) return fail(nullptr, IBM_ERR_ARG, "null pointer array");
  if (ndst < 1 || ndst > MIX_MAX || nsrc < 1 || nsrc > MIX_MAX)
    return fail(nullptr, IBM_ERR_ARG, "ndst and nsrc must be 1..8");
  if (bytes < 0 || bytes % 16 != 0) return fail(nullptr, IBM_ERR_ARG, "bytes must be a non-negative multiple of 16");
  MixPtrs p{};
  for (int q = 0; q < nsrc; ++q) {
    if (!src[q] || (uintptr_t)src[q] % 16 != 0) return fail(nullptr, IBM_ERR_ARG, "input arrays must be non-null and 16-byte aligned");
    p.src[q] = (const double2*)src[q];
  }
  for (int q = 0; q < ndst; ++q) {
    if (!dst[q] || (uintptr_t)dst[q] % 16 != 0) return fail(nullptr, IBM_ERR_ARG, "output arrays must be non-null and 16-byte aligned");
    p.dst[q] = (double2*)dst[q];
  }
  // no output may overlap an input or another output
  for (int a = 0; a < ndst; ++a) {
    const uintptr_t d = (uintptr_t)dst[a];
    for (int b = 0; b < nsrc + ndst; ++b) {
      if (b == nsrc + a) continue;
      const uintptr_t o = b < nsrc ? (uintptr_t)src[b] : (uintptr_t)dst[b - nsrc];
      if (bytes > 0 && d < o + (uintptr_t)bytes && o < d + (uintptr_t)bytes)
        return fail(nullptr, IBM_ERR_ARG, "an output array overlaps another array");
    }
  }
  const hipError_t e = launch_stream_mix(p, nsrc, ndst, bytes / 16, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(nullptr, IBM_ERR_DEVICE, std::string("stream mix: ") + hipGetErrorString(e));
  return IBM_OK;
}

int ibm_destroy(ibm_handle h) {
  if (!h) return IBM_OK;
  (void)hipStreamSynchronize(h->stream);
  for (Instance& I : h->inst) {
    for (auto& x : I.bufs) (void)hipFree(x.p);
    I.bufs.clear();
    free_buf(I.ibm_idx);
    free_buf(I.ibm_coef);
    free_buf(I.ibm_lam);
    free_buf(I.ibm_sig);
    free_buf(I.ibm_choff);
    free_buf(I.geo_tmp);
  }
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  drop_graph(h);
  for (hipStream_t s2 : h->aux) (void)hipStreamDestroy(s2);
  for (hipEvent_t e : h->ev_join) (void)hipEventDestroy(e);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  delete h;
  return IBM_OK;
}

const char* ibm_last_error(ibm_handle h) {
  if (h) return h->err.c_str();
  return g_last_error.c_str();
}

}  // extern "C"
