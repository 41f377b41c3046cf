// rBiCGStab without device allocations: the solver's workspace is a static
// device array of fixed size, one per GPU, instead of a caller buffer.  For
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device (hipGetSymbolAddress, with that device
// current) when a context is created there, and only that address is passed
// to kernels.  Every call on a device shares the array and leaves its
// contents behind; the solver initialises every value it reads, so no
// clearing is needed between calls.  Calls that overlap in time on one
// device (two contexts or streams at once) race on it.
#include <mutex>

#include "internal.hpp"

static __device__ __align__(256) unsigned char scratch[KRS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

}  // namespace

using krs::set_err;

namespace krs {

// Looks up (once per device) the device address of the static workspace of
// the context's device; that device must be current.
int noalloc_init(krs_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return set_err(ctx, KRS_ERR_STATE, "device index beyond the static workspace table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[ctx->device]) return KRS_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return set_err(ctx, KRS_ERR_HIP,
                   std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[ctx->device] = p;
  return KRS_OK;
}

}  // namespace krs

extern "C" int krs_rbicgstab_solve_noalloc(krs_ctx* ctx, const krs_matrix* A,
                                           const krs_precond* M, const krs_recycle* rec,
                                           const void* b, void* x, const krs_opts* opts,
                                           krs_stats* stats) {
  if (!ctx || !A || !b || !x || !opts) return KRS_ERR_ARG;
  if (opts->flags & KRS_FLAG_GRAPH)
    return set_err(ctx, KRS_ERR_ARG, "KRS_FLAG_GRAPH instantiates graphs (allocates)");
  if (ctx->timing)
    return set_err(ctx, KRS_ERR_STATE, "kernel timing creates events: disable it first");
  size_t need = 0;
  int rc = krs::workspace_bytes(KRS_SOLVER_RBICGSTAB, A->n, 1, 0, A->dt, &need);
  if (rc) return set_err(ctx, rc, "workspace size");
  if (need > (size_t)KRS_NOALLOC_SCRATCH_BYTES)
    return set_err(ctx, KRS_ERR_WORKSPACE,
                   "system too large for the static workspace (" + std::to_string(need) +
                       " bytes needed, " + std::to_string((size_t)KRS_NOALLOC_SCRATCH_BYTES) +
                       " available)");
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) ws = g_scratch_ptr[ctx->device];
  }
  if (!ws) {
    // the context was created while another device was current: look the
    // address up now, with the context's device current
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return set_err(ctx, KRS_ERR_HIP, "hipGetDevice");
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
      return set_err(ctx, KRS_ERR_HIP, "hipSetDevice");
    rc = krs::noalloc_init(ctx);
    if (cur != ctx->device) (void)hipSetDevice(cur);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ws = g_scratch_ptr[ctx->device];
  }
  return krs_rbicgstab_solve(ctx, A, M, rec, b, x, opts, ws, (size_t)KRS_NOALLOC_SCRATCH_BYTES,
                             stats);
}
