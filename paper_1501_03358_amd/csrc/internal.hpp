// Internal state of the krs library (contexts, handles, workspace carving).
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/krs.h"
#include "kernels.hpp"

struct krs_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  double* pin = nullptr;         // pinned host staging (kPinDoubles)
  double bytes = 0;              // byte-model accumulator of the current call
  // per-kernel-class timing (krs_timing_*)
  struct Pending {
    int cls;
    hipEvent_t a, b;
    double bytes;
  };
  bool timing = false;
  uint32_t timing_mask = 0xffffffffu;   // classes whose launches are timed
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  int64_t t_launches[KRS_K_COUNT] = {};
  double t_ms[KRS_K_COUNT] = {};
  double t_bytes[KRS_K_COUNT] = {};
  // captured rBiCGStab iterations (one pass of the loop per graph), keyed by
  // every pointer and size baked into the launches; least recently used out
  struct Graph {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
    double bytes = 0;              // byte model of one replay
    uint64_t used = 0;
  };
  std::vector<Graph> graphs;
  hipStream_t capture = nullptr;   // private stream, used only to record graphs
  uint64_t clock = 0;
};

struct krs_matrix {
  krs_ctx* ctx = nullptr;
  krs_grid g{};
  krs_dtype dt = KRS_F64;
  const void* bands = nullptr;
  int64_t n = 0;
  int pts = 7;        // 7 or 19 bands
};

struct krs_precond {
  krs_ctx* ctx = nullptr;
  const krs_matrix* A = nullptr;
  krs_precond_desc d{};
  void* tmp = nullptr;           // one vector, needed when global sweeps > 0
  void* pack = nullptr;          // tile-major local-solve coefficients (Schwarz-Jacobi)
};

struct krs_recycle {
  krs_ctx* ctx = nullptr;
  int64_t n = 0;
  int kmax = 0;
  krs_dtype dt = KRS_F64;
  void* U = nullptr;
  void* C = nullptr;
  int64_t ld = 0;
  int dim = 0;
  // hybrid policy state (krs_hybrid_solve)
  bool stale = false;            // A or M changed since C = A~ U
  bool force_rgcrot = false;     // next hybrid system runs rGCROT
  int64_t ref_mv = 0;            // matvecs of the first rBiCGStab system since rGCROT
};

namespace krs {

constexpr int kPinDoubles = 1 << 16;       // 512 KiB pinned staging
constexpr int kMaxM = 64;                  // Arnoldi steps per cycle
constexpr int kMaxK = 62;                  // recycle dimension (block passes take <= 64 columns)
constexpr int kScalarDoubles = 1 << 15;    // device scalar area (256 KiB)
constexpr int64_t kGramPartials = int64_t(1) << 21;   // Gram partial sums (entries)
constexpr int kGramMaxBlocks = 2048;
// Blocks of a Gram product of na x nb entries over n rows: as many as the
// partials hold (one partial per entry and block), at most one per 256 rows.
inline int gram_blocks(int na, int nb, int64_t n) {
  int64_t b = kGramPartials / ((int64_t)(na > 0 ? na : 1) * (nb > 0 ? nb : 1));
  if (b > kGramMaxBlocks) b = kGramMaxBlocks;
  const int64_t by_rows = (n + 255) / 256;
  if (b > by_rows) b = by_rows;
  return b < 1 ? 1 : (int)b;
}
constexpr int64_t kFuseMinN = int64_t(1) << 22;  // fused sweep + matvec from this size
constexpr int kMaxGraphs = 8;                // cached captured iterations per context
constexpr int64_t kGraphMaxN = int64_t(1) << 20;   // larger grids keep the GPU ahead of the host
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
static_assert(sizeof(BatchTable) <= KRS_BATCH_WORKSPACE_BYTES, "batch workspace");
// Leading dimension of multi-vectors: N rounded up to 64 values, plus a pad
// of 1088 values (4 KiB + 256 B in FP32), so that the columns of a block
// product do not all start at the same offset modulo a large power of two
// (on power-of-two grids they would meet the same HBM channels at every row;
// measured at 256^3 FP32: block products 6.23 -> 6.65 TB/s)
constexpr int64_t kLdPad = 1088;
inline int64_t vec_ld(int64_t n) { return (n + 63) / 64 * 64 + kLdPad; }

// Bump allocator over a caller workspace; with base == nullptr it only sizes.
struct Carver {
  char* base;
  size_t cap;
  size_t off = 0;
  bool ok = true;
  Carver(void* b, size_t c) : base((char*)b), cap(c) {}
  void* take(size_t bytes) {
    off = align_up(off);
    void* p = base ? base + off : nullptr;
    off += bytes;
    if (base && off > cap) ok = false;
    return p;
  }
  template <class T>
  T* vec(int64_t count) { return (T*)take(sizeof(T) * (size_t)count); }
};

inline size_t partials_bytes(size_t elem) {
  const size_t red = (size_t)kMaxRedBlocks * (kMaxM + kMaxK + 4);
  const size_t gram = (size_t)kGramPartials;
  return elem * (red > gram ? red : gram);
}

inline Grid3 grid3(const krs_matrix* A) {
  Grid3 g;
  g.nx = (int)A->g.nx;
  g.ny = (int)A->g.ny;
  g.nz = (int)A->g.nz;
  g.px = A->g.periodic[0] ? 1 : 0;
  g.py = A->g.periodic[1] ? 1 : 0;
  g.pz = A->g.periodic[2] ? 1 : 0;
  g.n = A->n;
  g.pts = A->pts;
  return g;
}

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
        .count();
  }
};

inline int set_err(krs_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

}  // namespace krs

#define KRS_CHECK_HIP(ctx, expr)                                                        \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return krs::set_err((ctx), KRS_ERR_HIP,                                          \
                          std::string(#expr) + ": " + hipGetErrorString(_e));          \
  } while (0)

namespace krs {
// kernel-launch bracketing for the timers and the byte model (timing.cpp)
hipEvent_t launch_begin(krs_ctx* ctx, int cls);
void launch_end(krs_ctx* ctx, int cls, double bytes, hipEvent_t a);
// after a stream synchronisation: fold completed event pairs into the totals
void timing_flush(krs_ctx* ctx);
void timing_release(krs_ctx* ctx);
// byte-model bytes of launches whose count is known only after they ran
void timing_add_bytes(krs_ctx* ctx, int cls, double bytes);
}  // namespace krs

// Launch `expr` (returning hipError_t) as kernel class `cls` moving `nbytes`.
#define KRS_LAUNCH(ctx, cls, nbytes, expr)                                              \
  do {                                                                                 \
    hipEvent_t _ev = krs::launch_begin(ctx, (cls));                                    \
    hipError_t _e = (expr);                                                            \
    krs::launch_end(ctx, (cls), (nbytes), _ev);                                        \
    if (_e != hipSuccess)                                                              \
      return krs::set_err((ctx), KRS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// solver entry points implemented in solvers.cpp (dtype dispatched)
namespace krs {
int workspace_bytes(krs_solver solver, int64_t n, int m, int k, krs_dtype dt, size_t* bytes);
int precond_apply(krs_ctx* ctx, const krs_precond* M, const void* r, void* z, void* tmp);
// krs_matrix_create / krs_matrix_create_19pt (pts = 7 or 19 bands)
int matrix_create(krs_ctx* ctx, const krs_grid* g, krs_dtype dt, const void* bands, int pts,
                  krs_matrix** out);
int operator_apply(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, const void* v, void* w,
                   void* tmp);
int precond_pack(krs_ctx* ctx, const krs_precond* M);
size_t precond_pack_bytes(const krs_matrix* A, const krs_precond_desc* d);
int gmres_rgcrot(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, krs_recycle* rec,
                 bool update, const void* b, void* x, const krs_opts* o, void* ws, size_t wsb,
                 krs_stats* st);
int rbicgstab(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, const krs_recycle* rec,
              const void* b, void* x, const krs_opts* o, void* ws, size_t wsb, krs_stats* st);
int recycle_setup(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, krs_recycle* rec,
                  void* ws, size_t wsb);
// per-device lookup of the static workspace of krs_rbicgstab_solve_noalloc
// (noalloc.hip); the context's device must be current
int noalloc_init(krs_ctx* ctx);
// krs_ir_solve_batched (grouped rBiCGStab inner passes; bitwise as alone)
int ir_solve_batched(krs_ctx* ctx, int nsys, const krs_ir_system* sys, const krs_opts* o,
                     void* ws, size_t wsb);
int ir_solve(krs_ctx* ctx, const krs_matrix* A64, const krs_matrix* A32, const krs_precond* M32,
             krs_recycle* rec32, const void* b, void* x, const krs_opts* o, void* ws, size_t wsb,
             krs_stats* st);
}  // namespace krs
