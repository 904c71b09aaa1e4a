// Shared host/device definitions of the SplitSolve HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "splitsolve.h"

typedef double v4d __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ complex helpers (device)

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cneg(double2 a) { return make_double2(-a.x, -a.y); }
// a - b*c
__device__ __forceinline__ double2 cfnms(double2 a, double2 b, double2 c) {
  return make_double2(a.x - b.x * c.x + b.y * c.y, a.y - b.x * c.y - b.y * c.x);
}
// 1/u by scaling with the larger component (avoids overflow of |u|^2 for large entries)
__device__ __forceinline__ double2 crecip(double2 u) {
  if (fabs(u.x) >= fabs(u.y)) {
    double r = u.y / u.x, d = u.x + u.y * r;
    return make_double2(1.0 / d, -r / d);
  } else {
    double r = u.x / u.y, d = u.y + u.x * r;
    return make_double2(r / d, -1.0 / d);
  }
}
// component-wise copies (a plain double2 assignment between address spaces becomes a memcpy that
// keeps register arrays out of registers)
__device__ __forceinline__ void st2(double2 &dst, double2 v) { dst.x = v.x; dst.y = v.y; }
__device__ __forceinline__ double2 ld2(const double2 &s) { return make_double2(s.x, s.y); }
// Lane exchanges inside a row of 16 lanes through DPP (no LDS round trip).  kCtrl: 0xB1 swaps
// neighbours (lane ^ 1), 0x4E swaps pairs (lane ^ 2), 0x141 mirrors each half-row of 8 (lane i <-> 7 - i),
// 0x140 mirrors the row (lane i <-> 15 - i).  Every lane of the row must be active.
template <int kCtrl>
__device__ __forceinline__ int dpp_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, kCtrl, 0xF, 0xF, false);
}
template <int kCtrl>
__device__ __forceinline__ double dpp_double(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_int<kCtrl>((int)(b & 0xffffffffLL));
  const int hi = dpp_int<kCtrl>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Maximum that propagates NaN (fmax drops a NaN operand, which would let a NaN iterate pass a
// convergence test): NaN if either operand is NaN.
__device__ __forceinline__ double nanmax(double a, double b) { return (a != a) ? a : ((b > a || b != b) ? b : a); }

// LAPACK's pivot magnitude |Re| + |Im|
__device__ __forceinline__ double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }

// ------------------------------------------------------------------ host side

namespace ss {

struct Buffer {
  void *ptr = nullptr;
  size_t bytes = 0;
};

enum Slot {
  kSlotM = 0,      // augmented matrices of the batched LU solves
  kSlotPerm,       // row permutations
  kSlotZp,         // first zero pivot per factorization
  kSlotX,          // per-step solutions of the recursion
  kSlotInst,       // per-matrix instance tables
  kSlotDec,        // decimation state
  kSlotObc,        // corner system work
  kSlotMisc,
  kSlotFact,       // kept factorizations of the first-column recursion (for refinement)
  kSlotFactPerm,
  kSlotRef,        // refinement work
  kSlotWarm,       // Newton work of the warm-started self-energies
  kSlotWarmMisc,
  kSlotMlp,        // split-K partial products of the network
  kSlotMlpDz,      // back-propagated gradients
  kSlotLuInv,      // inverses of the LU's diagonal blocks (triangular-solve leaves)
  kSlotSpike,      // partition tables, the second column buffer and the interface systems of the merges
  kSlotCpl,        // FP32 coupling blocks of the next recursion step (BF16-term products)
  kSlotFactInv,    // kept inverses of the diagonal blocks of the kept factorizations (32-column panels)
  kNumSlots
};

}  // namespace ss

struct ss_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  ss::Buffer slot[ss::kNumSlots];
  int *host_word = nullptr;  // pinned word for convergence polls
  bool sync_free = false;    // never wait for the stream inside a call (stream/graph capture)
  int lu_width = 0;          // LU panel width to use where valid for the order (0: the default)
  int lu_tile = 0;           // tile of the LU's general block products: 0 64 x 64, 1 32 x 64
  // what the kept workspaces currently describe (for ss_refine_psi)
  bool fact_valid = false;   // kSlotX + kSlotFact/FactPerm hold a first-column recursion
  bool fact_inv = false;     // and kSlotFactInv the inverses of their 32 x 32 diagonal blocks
  int fact_batch = 0, fact_nb = 0, fact_s = 0;
  double fact_absorb = 0.0;  // absorbing shift of the boundary blocks the kept factors were formed with
  bool corner_valid = false;  // kSlotM/kSlotPerm hold the factored corner systems of ss_apply_obc
  int corner_batch = 0, corner_s = 0, corner_ldm = 0;
  double corner_absorb = 0.0;  // the shift in C' = Sigma + i*absorb*I of the factored corner systems
  // kernel timing probe: launches of `timer_family` are bracketed by event pairs
  std::string timer_family;
  std::vector<hipEvent_t> timer_events;
  size_t timer_used = 0;
  double timer_flops = 0.0;  // algorithmic flops of the timed launches (where the launch site states them)
  double timer_bytes = 0.0;  // algorithmic HBM bytes of the same launches (operands read once, results written once)
  // graph segments: while seg_graphs is set and the stream is being captured, a capture that has grown
  // to seg_limit nodes is closed at the next launch site (into seg_graphs) and a new one begun on the
  // same stream, so no captured graph grows past about seg_limit nodes
  std::vector<hipGraph_t> *seg_graphs = nullptr;
  size_t seg_limit = 0;
  bool seg_failed = false;  // closing or reopening a capture failed (the capture is then broken)
};

namespace ss {

// Grow-only device workspace; a reallocation waits for the stream so no queued kernel still uses it.
ss_status workspace(ss_ctx *ctx, Slot s, size_t bytes, void **out);
ss_status fail(ss_ctx *ctx, ss_status st, const std::string &msg);
ss_status check_launch(ss_ctx *ctx, const char *what);
ss_status host_word(ss_ctx *ctx, int **out);

// A launch site: while the context's stream is captured in segments, starts a new graph segment once
// the current one holds seg_limit nodes (every launch scope passes here before its launches).
void segment_point(ss_ctx *ctx);

// Brackets the launches issued in its scope with a pair of events when `family` is being timed.
struct KernelScope {
  ss_ctx *ctx;
  bool on;
  KernelScope(ss_ctx *c, const char *family, double flops = 0.0, double bytes = 0.0);
  ~KernelScope();
};

__host__ __device__ inline int cdiv(int a, int b) { return (a + b - 1) / b; }

}  // namespace ss

#define SS_TRY(expr)                  \
  do {                                \
    ss_status _st = (expr);           \
    if (_st != SS_OK) return _st;     \
  } while (0)
