// qmc_matmul_noalloc: X = Y A with the workspace taken from a static device
// array instead of a caller buffer, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops).  The kernels
// and their order are those of qmc_matmul, all on the caller's stream.
#include <mutex>

#include "internal.hpp"

using namespace qmc;

// The scratch of every allocation-free call on a GPU.  The code object that
// holds it is loaded once per device, so each GPU has its own copy at its own
// address, held until the process ends.  Host code never passes this name to
// a kernel (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[QMC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// the device address of the current device's copy of scratch, looked up on
// the first call on that device (with it current) and kept
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return QMC_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return QMC_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return QMC_ERR_HIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return QMC_OK;
}

}  // namespace

extern "C" int qmc_matmul_noalloc(qmc_plan_t P, const void* A, int64_t t, int64_t lda, void* X,
                                  int64_t ldx, void* stream) {
  if (!P || !A || !X || t < 1 || lda < t || ldx < t) return QMC_ERR_ARG;
  // the timing instrumentation creates HIP events per launch
  if (P->prof_on) return QMC_ERR_ARG;
  if (workspace_bytes(P, t) > QMC_NOALLOC_SCRATCH_BYTES) return QMC_ERR_WORKSPACE;
  const size_t xa = matrix_extent(P->N, t, ldx, P->dtype);
  const size_t aa = matrix_extent(P->s, t, lda, P->dtype);
  if (ranges_overlap(X, xa, A, aa)) return QMC_ERR_ALIAS;
  void* ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc != QMC_OK) return rc;
  // every scratch byte a kernel reads was written earlier in the same call
  // (collapse or outer front, then the fused pass), so nothing is cleared
  return launch_forward(P, A, t, lda, X, ldx, ws, (hipStream_t)stream, QMC_EPI_NONE, nullptr,
                        nullptr, /*single_stream=*/true);
}
