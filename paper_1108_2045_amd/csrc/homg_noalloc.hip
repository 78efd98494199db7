// homg_noalloc.hip -- the residual entry point for callers that cannot
// allocate device memory (see homg_residual_noalloc in include/homg.h).
//
// homg_residual keeps its per-block partial sums of r^2, the solve state and
// the one-entry history in workspace that homg_create allocated.  This
// variant needs no handle: the same workspace is a file-scope device array,
// `scratch`, of a fixed size, which every GPU that runs it holds until the
// process ends.  Its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// passed to kernels and copies; the array's name in host code is a host-side
// stand-in, not a device pointer.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/homg.h"
#include "homg_internal.h"

using namespace homg;

namespace {

// Layout: DevState (32 B) | history[1] (8 B, padded to 64 B) | partials.
constexpr size_t NOALLOC_HEADER = 64;
constexpr size_t NOALLOC_PARTIALS = HOMG_NOALLOC_MAX_PARTIALS;
constexpr size_t NOALLOC_BYTES = NOALLOC_HEADER + sizeof(double) * NOALLOC_PARTIALS;
static_assert(sizeof(DevState) <= 32, "device state must fit the header");

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

// Device address of `scratch` on device dev (looked up once, with dev current).
hipError_t scratch_ptr(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

homg_status nfail(homg_status s, const std::string& msg) {
  set_last_error(msg.c_str());
  return s;
}

int side_k(int64_t n) {
  if (n < 3) return -1;
  int k = 0;
  while ((int64_t(1) << (k + 1)) + 1 <= n) ++k;
  return ((int64_t(1) << k) + 1 == n) ? k : -1;
}

}  // namespace

extern "C" homg_status homg_residual_noalloc(int ndim, int64_t n, const double* f, const double* u,
                                             double* r, double* relres_out, void* stream) {
  if (ndim != 2 && ndim != 3) return nfail(HOMG_ERR_INVALID_ARG, "ndim must be 2 or 3");
  const int k = side_k(n);
  if (k < 1) return nfail(HOMG_ERR_INVALID_ARG, "side must be 2^k + 1 with k >= 1");
  if ((ndim == 2 && k > 15) || (ndim == 3 && k > 10))
    return nfail(HOMG_ERR_UNSUPPORTED, "grid too large");
  if (!f || !u || !r) return nfail(HOMG_ERR_INVALID_ARG, "null f, u or r");
  const int side = int(n);
  if (size_t(partials_bound(ndim, side)) > NOALLOC_PARTIALS)
    return nfail(HOMG_ERR_WORKSPACE, "grid needs more partial sums than the static workspace holds (" +
                                         std::to_string(NOALLOC_PARTIALS) + ")");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
    return nfail(HOMG_ERR_HIP, "cannot query the current device");
  void* base = nullptr;
  if (hipError_t e = scratch_ptr(dev, &base))
    return nfail(HOMG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  char* b = static_cast<char*>(base);
  DevState* st = reinterpret_cast<DevState*>(b);
  double* hist = reinterpret_cast<double*>(b + 32);
  double* partials = reinterpret_cast<double*>(b + NOALLOC_HEADER);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Lay dl = dense_layout(ndim, side);
  const Lay none;
  int count = 0;
  // the same launches as homg_residual with a caller array r; the state
  // reset clears the `done` flag that the residual kernel reads first
  hipError_t e = launch_init_state(st, 0.0, 0, s);
  if (e == hipSuccess) e = launch_norm2(ndim, side, f, dl, partials, &count, s);
  if (e == hipSuccess) e = launch_finalize(partials, count, st, hist, 0, 0, s);
  if (e == hipSuccess)
    e = launch_residual(PREC_F64, ndim, side, u, dl, f, dl, nullptr, none, r, dl, partials, &count, &st->done, s);
  if (e == hipSuccess) e = launch_finalize(partials, count, st, hist, 0, 1, s);
  if (e == hipSuccess && relres_out) e = hipMemcpyAsync(relres_out, hist, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && relres_out) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return nfail(HOMG_ERR_HIP, std::string("residual launch: ") + hipGetErrorString(e));
  return HOMG_OK;
}
