// The stand-alone pressure solve without a handle and without any device allocation
// (ibm_solve_pressure_noalloc): the work area (FFT twiddles, real-FFT unpacking
// twiddles, modified wavenumbers, the removed mean and the half spectrum) lives in one
// file-scope device array of fixed size, resolved to its device address once per GPU.
#include <algorithm>
#include <mutex>

#include "ibm.h"
#include "ibm_internal.h"

namespace {

// The work area of every ibm_solve_pressure_noalloc call on one GPU (each GPU holds its
// own copy for the life of the process).  In host code this name is only a stand-in:
// kernels and copies take the device address returned by hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[IBM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int noalloc_fail(int code, const char* msg) {
  set_last_error(msg);
  return code;
}

// Device address of this GPU's scratch array (looked up once per device, with that
// device current; nullptr on failure).
void* scratch_of_current_device(int* dev_out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  *dev_out = dev;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

// Tables of one solve, computed on the device (sincospi: exact reduction of the
// argument): complex-FFT twiddles e^{-2 pi i m/n} of the x (n = nx/2) and z (n = nz)
// transforms in FP64 and FP32, the real-FFT unpacking twiddles e^{-2 pi i m/nx},
// m = 0..nx/2, and the modified wavenumbers (4/h^2) sin^2(pi m/n) of the periodic
// three-point second difference.
__global__ __launch_bounds__(256) void k_solve_tables(double2* twx64, float2* twx32, int nxh, double2* twz64,
                                                       float2* twz32, int nz, double2* rtw, double* kx2,
                                                       double* kz2, int nx, double dx, double dz) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double s, c;
  if (t < nxh) {
    sincospi(2.0 * t / nxh, &s, &c);
    twx64[t] = make_double2(c, -s);
    twx32[t] = make_float2((float)c, (float)-s);
  }
  if (t < nz) {
    sincospi(2.0 * t / nz, &s, &c);
    twz64[t] = make_double2(c, -s);
    twz32[t] = make_float2((float)c, (float)-s);
    const double sz = sinpi((double)t / nz);
    kz2[t] = (4.0 / (dz * dz)) * (sz * sz);
  }
  if (t <= nx / 2) {
    sincospi(2.0 * t / nx, &s, &c);
    rtw[t] = make_double2(c, -s);
    const double sx = sinpi((double)t / nx);
    kx2[t] = (4.0 / (dx * dx)) * (sx * sx);
  }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

template <typename T>
int solve(const ibm_grid_desc& d, const T* rhs, T* phi, double* mean_removed, hipStream_t st) {
  GridParams g{};
  grid_params_uniform(d.nx, d.ny, d.nz, d.lx, d.lz, d.y_lo, d.y_hi, d.nu, d.dt, 0, sizeof(T), &g);
  FFTPlan px{}, pz{};
  px.n = g.nhalf;
  pz.n = g.nz;
  if (!factor_235(px.n, px.radix, &px.nst) || !factor_235(pz.n, pz.radix, &pz.nst) || px.nst > 16 || pz.nst > 16)
    return noalloc_fail(IBM_ERR_ARG, "nx/2 and nz must have prime factors in {2,3,5}");
  px.rcode = pz.rcode = 0;
  for (int s = 0; s < px.nst; ++s) px.rcode |= (uint64_t)px.radix[s] << (4 * s);
  for (int s = 0; s < pz.nst; ++s) pz.rcode |= (uint64_t)pz.radix[s] << (4 * s);
  // layout of the work area (every part on a 256-byte boundary)
  size_t off[9], at = 0;
  const size_t sz[9] = {(size_t)px.n * sizeof(double2), (size_t)px.n * sizeof(float2),
                        (size_t)pz.n * sizeof(double2), (size_t)pz.n * sizeof(float2),
                        (size_t)g.mh * sizeof(double2), (size_t)g.mh * sizeof(double),
                        (size_t)g.nz * sizeof(double), sizeof(double),
                        (size_t)g.ny1 * g.splane * sizeof(cplx<T>)};
  for (int q = 0; q < 9; ++q) {
    off[q] = at;
    at = align256(at + sz[q]);
  }
  if (at > (size_t)IBM_NOALLOC_SCRATCH_BYTES)
    return noalloc_fail(IBM_ERR_ARG, "grid too large for the fixed work area (IBM_NOALLOC_SCRATCH_BYTES)");
  int dev = -1;
  unsigned char* base = (unsigned char*)scratch_of_current_device(&dev);
  if (!base) return noalloc_fail(IBM_ERR_DEVICE, "device address of the work area not available");
  double2* twx64 = (double2*)(base + off[0]);
  float2* twx32 = (float2*)(base + off[1]);
  double2* twz64 = (double2*)(base + off[2]);
  float2* twz32 = (float2*)(base + off[3]);
  double2* rtw = (double2*)(base + off[4]);
  double* kx2 = (double*)(base + off[5]);
  double* kz2 = (double*)(base + off[6]);
  double* mean = mean_removed ? mean_removed : (double*)(base + off[7]);
  cplx<T>* spec = (cplx<T>*)(base + off[8]);
  px.tw64 = twx64;
  px.tw32 = twx32;
  pz.tw64 = twz64;
  pz.tw32 = twz32;
  const int nt = std::max(std::max(px.n, pz.n), g.mh);
  hipLaunchKernelGGL(k_solve_tables, dim3((nt + 255) / 256), dim3(256), 0, st, twx64, twx32, px.n, twz64, twz32,
                     pz.n, rtw, kx2, kz2, g.nx, g.dx, g.dz);
  hipError_t e = hipGetLastError();
  // the same kernels as ibm_solve_pressure: divergence input replaced by rhs, forward x
  // and z FFTs, tridiagonal solves, inverse transforms
  Fields<T> f{};
  f.spec = spec;
  IbmLists L{};
  const Tuning tu{};
  if (e == hipSuccess) e = launch_div_fftx<T>(g, f, L, 0, px, rtw, 1.0, mean, rhs, st);
  if (e == hipSuccess) e = launch_fftz<T>(g, spec, pz, -1, tu, st);
  if (e == hipSuccess) e = launch_tri<T>(g, spec, kx2, kz2, mean, tu, st);
  if (e == hipSuccess) e = launch_fftz<T>(g, spec, pz, +1, tu, st);
  if (e == hipSuccess) e = launch_ifftx<T>(g, spec, phi, px, rtw, st);
  if (e != hipSuccess) return noalloc_fail(IBM_ERR_DEVICE, hipGetErrorString(e));
  return IBM_OK;
}

}  // namespace

extern "C" {

int ibm_solve_pressure_noalloc(const ibm_grid_desc* desc, int32_t precision, const void* rhs, void* phi,
                               double* mean_removed, void* hip_stream) {
  if (!desc || !rhs || !phi) return noalloc_fail(IBM_ERR_ARG, "null argument");
  const ibm_grid_desc& d = *desc;
  if (d.nx < 2 || (d.nx & 1)) return noalloc_fail(IBM_ERR_ARG, "nx must be even and >= 2");
  if (d.nz < 1 || d.ny < 3) return noalloc_fail(IBM_ERR_ARG, "nz must be >= 1 and ny >= 3");
  if (d.nx > 1024 || d.nz > 1024 || d.ny > 2049) return noalloc_fail(IBM_ERR_ARG, "grid beyond the kernels' limits");
  if (!(d.lx > 0.0) || !(d.lz > 0.0) || !(d.y_hi > d.y_lo)) return noalloc_fail(IBM_ERR_ARG, "invalid box extents");
  if (precision != IBM_FP64 && precision != IBM_FP32_STORAGE) return noalloc_fail(IBM_ERR_ARG, "invalid precision");
  const hipStream_t st = (hipStream_t)hip_stream;
  return precision == IBM_FP64
             ? solve<double>(d, (const double*)rhs, (double*)phi, mean_removed, st)
             : solve<float>(d, (const float*)rhs, (float*)phi, mean_removed, st);
}

}  // extern "C"
