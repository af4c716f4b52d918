// Allocation-free variant of the coarse contraction (hotrg_coarse_noalloc,
// include/hotrg.h): T~ = U T T U (Sec. 2, Fig. 1) as C1 -> C2 -> C3 in
// FP64 with every intermediate in one file-scope device array instead of
// buffers the library allocates, for callers that cannot allocate (code
// under HIP graph capture, serving loops that forbid hipMalloc).
//
// The array lives in this library's code object, so each GPU the library
// runs on holds its own copy (kScratchBytes) until the process ends.  Host
// code never passes the array's name to a kernel -- on the host that name is
// a stand-in, not a device address -- but the address hipGetSymbolAddress
// returns for the current device, looked up once per device when the first
// context on it is created.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "../../include/hotrg.h"
#include "internal.h"

namespace {

constexpr size_t kScratchBytes = HOTRG_NOALLOC_SCRATCH_BYTES;
constexpr size_t kScratchDoubles = kScratchBytes / 8;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

// x[0] = 1.0: the unit scale the operand preparation divides by
__global__ void k_unit(double* x) {
  if (threadIdx.x == 0 && blockIdx.x == 0) x[0] = 1.0;
}

thread_local std::string t_err;

}  // namespace

namespace hotrg {

void noalloc_init_device(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_done[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_err[device] = e;
  g_ptr[device] = e == hipSuccess ? (double*)p : nullptr;
  g_done[device] = true;
}

}  // namespace hotrg

using namespace hotrg;

extern "C" {

hotrg_status hotrg_coarse_noalloc(hotrg_ctx* ctx, const double* T, const double* U, int dx, int dy,
                                  int dn, double* Tt, double* max_abs) {
  if (!ctx || !T || !U || !Tt) {
    set_last_error("NULL argument");
    return HOTRG_ERR_INVALID;
  }
  if (dx < 1 || dy < 1 || dn < 1 || dn > dx * dx) {
    set_last_error("need dx, dy >= 1 and 1 <= dn <= dx*dx");
    return HOTRG_ERR_INVALID;
  }
  // X1, X2 (dn dx^2 dy^2 each), three operand layouts of T (dx^2 dy^2 each),
  // two layouts of U (dx^2 dn each), each starting on a 256-byte boundary
  // (as hipMalloc'd buffers do), after 64 doubles for the unit scale and the
  // max slot
  auto slot = [](double count) { return std::ceil(count / 32.0) * 32.0; };
  const double t4 = (double)dx * dx * dy * dy, u2 = (double)dx * dx * dn;
  const double need = 64.0 + 2.0 * slot(dn * t4) + 3.0 * slot(t4) + 2.0 * slot(u2);
  if (need > (double)kScratchDoubles) {
    t_err = "hotrg_coarse_noalloc: needs " + std::to_string((long long)(need * 8.0)) +
            " bytes of scratch, the maximum is " + std::to_string((long long)kScratchBytes) +
            " (2 dn dx^2 dy^2 + 3 dx^2 dy^2 + 2 dx^2 dn doubles plus alignment)";
    set_last_error(t_err.c_str());
    return HOTRG_ERR_INVALID;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_last_error("hipGetDevice failed");
    return HOTRG_ERR_DEVICE;
  }
  const int cdev = ctx_device(ctx);
  if (cdev != dev && hipSetDevice(cdev) != hipSuccess) {
    set_last_error("hipSetDevice failed");
    return HOTRG_ERR_DEVICE;
  }
  noalloc_init_device(cdev);  // already done when the context was created
  double* base = (cdev >= 0 && cdev < kMaxDevices) ? g_ptr[cdev] : nullptr;
  if (!base) {
    t_err = std::string("scratch array not available on this device: ") +
            hipGetErrorString(cdev >= 0 && cdev < kMaxDevices ? g_err[cdev] : hipErrorInvalidDevice);
    set_last_error(t_err.c_str());
    return HOTRG_ERR_DEVICE;
  }
  auto up32 = [](long long c) { return (c + 31) / 32 * 32; };
  const long long n4 = up32((long long)dx * dx * dy * dy), nu = up32((long long)dx * dx * dn);
  const long long nx = up32((long long)dn * dx * dx * dy * dy);
  // [0] unit scale, [8] max bits (each on its own 64-byte line)
  double* unit = base;
  unsigned long long* mb = max_abs ? (unsigned long long*)max_abs : (unsigned long long*)(base + 8);
  double* Tn = base + 64;
  double* Xt = Tn + n4;
  double* Tp = Xt + n4;
  double* U1 = Tp + n4;
  double* U3 = U1 + nu;
  double* X1 = U3 + nu;
  double* X2 = X1 + nx;
  const hipStream_t s = ctx_stream(ctx);
  hipLaunchKernelGGL(k_unit, dim3(1), dim3(64), 0, s, unit);
  launch_prep(T, false, false, dx, dy, (const unsigned long long*)unit, Tn, Xt, Tp, false, s);
  launch_layout_u(U, dx, dn, U1, U3, false, s);
  coarse_f64_into(ctx, Tn, Tp, U1, U3, dx, dy, dn, X1, X2, Tt, mb, GEMM_NO_TUNE);
  const hipError_t e = hipGetLastError();
  if (cdev != dev) (void)hipSetDevice(dev);
  if (e != hipSuccess) {
    t_err = std::string("kernel launch failed: ") + hipGetErrorString(e);
    set_last_error(t_err.c_str());
    return HOTRG_ERR_DEVICE;
  }
  return HOTRG_OK;
}

}  // extern "C"
