// ascc_solve for callers that cannot allocate device memory: the solver state (DIIS history,
// residual, trial amplitudes, statistics) lives in a fixed device array of this translation unit.
//
// The array is a file-scope __device__ variable, so every GPU that runs the library holds one copy
// of it (from the load of the code object until the process ends) at its own device address.  Host
// code never names it: its address is taken once per device with hipGetSymbolAddress, with that
// device current, and only that address is passed on (to the carving solve loop and, through the
// carved arrays, to its kernels).  Every call on one device shares that device's array, so calls
// that overlap on one GPU race; everything the solve reads before writing (the DIIS bookkeeping) is
// reset at the start of each call.
#include <mutex>
#include <string>

#include "../../include/ascc.h"
#include "internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (taken once per device).
int scratch_address(void** out) {
  if (ascc::dry_run()) {
    static void* fake = reinterpret_cast<void*>(ascc::dry_run_address(kScratchBytes));
    *out = fake;
    return ASCC_OK;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    ascc::set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    return ASCC_E_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    ascc::set_error("device index beyond the supported range");
    return ASCC_E_ARG;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      ascc::set_error(std::string("hipGetSymbolAddress of the solver scratch: ") + hipGetErrorString(e));
      return ASCC_E_HIP;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return ASCC_OK;
}

}  // namespace

extern "C" {

int ascc_solve_noalloc(ascc_ints* ints, const ascc_opts* opts, double* d_t1, double* d_t2, ascc_result* res,
                       void* stream) {
  if (!ints || !opts || !d_t1 || !d_t2 || !res) {
    ascc::set_error("NULL argument to ascc_solve_noalloc");
    return ASCC_E_ARG;
  }
  if (opts->diis_size < 1 || opts->diis_size > ascc::kMaxDiis) {
    ascc::set_error("diis_size must be in 1..16");
    return ASCC_E_ARG;
  }
  int no = 0, nv = 0, naux = 0;
  int rc = ascc_ints_shape(ints, &no, &nv, &naux);
  if (rc) return rc;
  const size_t need = ascc::solve_workspace_bytes(no, nv, opts->diis_size);
  if (need > kScratchBytes) {
    ascc::set_error("ascc_solve_noalloc: the solver state of no = " + std::to_string(no) + ", nv = " +
                    std::to_string(nv) + " with " + std::to_string(opts->diis_size) + " DIIS vectors needs " +
                    std::to_string(need) + " bytes, above the fixed " + std::to_string(kScratchBytes) +
                    " (use ascc_solve)");
    return ASCC_E_NOMEM;
  }
  void* base = nullptr;
  if ((rc = scratch_address(&base))) return rc;
  return ascc::solve_impl(ints, opts, d_t1, d_t2, res, stream, static_cast<char*>(base), kScratchBytes);
}

}  // extern "C"
