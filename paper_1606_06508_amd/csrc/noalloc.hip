// fh_eval without any allocation: the node table lives in a fixed device
// array of the library instead of a caller workspace.
//
// The array is a file-scope device variable, one copy per GPU the library
// runs on, held until the process ends.  Host code never passes the
// variable's name to a kernel (on the host that name is only a stand-in for
// the device copy): the device address of each GPU's copy is resolved once,
// with hipGetSymbolAddress while that device is current, kept per device,
// and then used like any workspace pointer.  Every call on a GPU uses the
// same array; the status block at its start is cleared by a kernel at the
// start of each call (a kernel, not a memset node, so a captured graph
// replays it correctly), and the packing rewrites the rest.
#include <mutex>

#include "fh_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[FH_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

__global__ void k_noalloc_clear_status(uint32_t* status) {
  // the whole status block: sticky bits, split scales, sign flag, reserved
  if (threadIdx.x < fhk::kStatusBytes / sizeof(uint32_t)) status[threadIdx.x] = 0u;
}

// Device address of the current device's copy of `scratch`, resolved on the
// first call on that device; nullptr on a HIP error.
void* scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
      return nullptr;
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" {

fh_status fh_eval_noalloc(const double* nodes, const double* values, int64_t n, int32_t d,
                          const double* x, int64_t m, double* r_out, double* lambda_out,
                          const double* w, int32_t prec, void* stream) {
  // host-side checks first: no HIP call for a refused problem
  if (n < 1 || n > FH_MAX_NODES || nodes == nullptr || values == nullptr) return FH_E_ARG;
  if (d < 0 || (int64_t)d > n - 1) return FH_E_DEGREE;
  if (m < 0 || (m > 0 && (x == nullptr || r_out == nullptr))) return FH_E_ARG;
  if (prec != FH_FP64 && prec != FH_FP32_SPLIT) return FH_E_ARG;
  // the node tables; offered no room beyond them, fh_eval runs no octet
  // variant (those sort the points into the workspace)
  fhk::NodeTable t;
  const size_t need = fhk::layout_tables(nullptr, n, &t);
  if (n > FH_NOALLOC_MAX_NODES || need > FH_NOALLOC_SCRATCH_BYTES) return FH_E_TOO_LARGE;
  void* ws = scratch_ptr();
  if (ws == nullptr) return FH_E_HIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  k_noalloc_clear_status<<<1, 64, 0, s>>>(static_cast<uint32_t*>(ws));
  if (hipGetLastError() != hipSuccess) return FH_E_HIP;
  return fh_eval(nodes, values, n, d, x, m, r_out, lambda_out, w, prec, ws, need, stream);
}

}  // extern "C"
