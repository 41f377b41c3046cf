// Per-kernel-class timing with HIP events on the context's stream.
#include "internal.hpp"

namespace krs {

namespace {
hipEvent_t take_event(krs_ctx* ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

hipEvent_t launch_begin(krs_ctx* ctx, int cls) {
  if (!ctx->timing || !((ctx->timing_mask >> cls) & 1u)) return nullptr;
  hipEvent_t a = take_event(ctx);
  if (a && hipEventRecord(a, ctx->stream) != hipSuccess) {
    ctx->pool.push_back(a);
    return nullptr;
  }
  return a;
}

void launch_end(krs_ctx* ctx, int cls, double bytes, hipEvent_t a) {
  ctx->bytes += bytes;
  if (!ctx->timing || !a) return;
  hipEvent_t b = take_event(ctx);
  if (!b || hipEventRecord(b, ctx->stream) != hipSuccess) {
    ctx->pool.push_back(a);
    if (b) ctx->pool.push_back(b);
    return;
  }
  ctx->pending.push_back({cls, a, b, bytes});
}

void timing_flush(krs_ctx* ctx) {
  for (auto& p : ctx->pending) {
    float ms = 0;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->t_launches[p.cls] += 1;
      ctx->t_ms[p.cls] += ms;
      ctx->t_bytes[p.cls] += p.bytes;
    }
    ctx->pool.push_back(p.a);
    ctx->pool.push_back(p.b);
  }
  ctx->pending.clear();
}

void timing_add_bytes(krs_ctx* ctx, int cls, double bytes) {
  ctx->bytes += bytes;
  if (ctx->timing) ctx->t_bytes[cls] += bytes;
}

void timing_release(krs_ctx* ctx) {
  timing_flush(ctx);
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  ctx->pool.clear();
}

}  // namespace krs

extern "C" {

int krs_timing_enable(krs_ctx* ctx, int on) {
  if (!ctx) return KRS_ERR_ARG;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return KRS_ERR_HIP;
  krs::timing_flush(ctx);
  ctx->timing = on != 0;
  return KRS_OK;
}

int krs_timing_classes(krs_ctx* ctx, unsigned int mask) {
  if (!ctx) return KRS_ERR_ARG;
  ctx->timing_mask = mask;
  return KRS_OK;
}

int krs_timing_reset(krs_ctx* ctx) {
  if (!ctx) return KRS_ERR_ARG;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return KRS_ERR_HIP;
  krs::timing_flush(ctx);
  for (int c = 0; c < KRS_K_COUNT; ++c) {
    ctx->t_launches[c] = 0;
    ctx->t_ms[c] = 0;
    ctx->t_bytes[c] = 0;
  }
  return KRS_OK;
}

int krs_timing_read(krs_ctx* ctx, int cls, int64_t* launches, double* ms, double* bytes) {
  if (!ctx || cls < 0 || cls >= KRS_K_COUNT) return KRS_ERR_ARG;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return KRS_ERR_HIP;
  krs::timing_flush(ctx);
  if (launches) *launches = ctx->t_launches[cls];
  if (ms) *ms = ctx->t_ms[cls];
  if (bytes) *bytes = ctx->t_bytes[cls];
  return KRS_OK;
}

}  // extern "C"
