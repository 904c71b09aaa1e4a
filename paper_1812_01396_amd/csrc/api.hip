// C ABI entry points: argument validation, context and workspace management.
#include <cmath>
#include <cstdio>
#include <new>

#include "drivers.hpp"
#include "lu.hpp"

namespace ss {

ss_status fail(ss_ctx *ctx, ss_status st, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return st;
}

ss_status check_launch(ss_ctx *ctx, const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, SS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return SS_OK;
}

ss_status workspace(ss_ctx *ctx, Slot s, size_t bytes, void **out) {
  Buffer &b = ctx->slot[s];
  if (bytes == 0) bytes = 256;
  if (b.bytes < bytes) {
    if (ctx->sync_free)
      return fail(ctx, SS_ERR_ARG, "workspace too small in sync-free mode (run the call eagerly once first)");
    if (b.ptr) {
      if (hipStreamSynchronize(ctx->stream) != hipSuccess)
        return fail(ctx, SS_ERR_DEVICE, "workspace: stream synchronize before reallocation failed");
      (void)hipFree(b.ptr);
      b.ptr = nullptr;
      b.bytes = 0;
    }
    const size_t want = bytes + bytes / 8;
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
      (void)hipGetLastError();
      b.ptr = nullptr;
      return fail(ctx, SS_ERR_NOMEM, "workspace: device allocation of " + std::to_string(want) + " bytes failed");
    }
    b.bytes = want;
  }
  *out = b.ptr;
  return SS_OK;
}

ss_status host_word(ss_ctx *ctx, int **out) {
  if (!ctx->host_word) {
    if (hipHostMalloc((void **)&ctx->host_word, sizeof(int)) != hipSuccess) {
      ctx->host_word = nullptr;
      return fail(ctx, SS_ERR_NOMEM, "pinned host word allocation failed");
    }
  }
  *out = ctx->host_word;
  return SS_OK;
}

static hipEvent_t timer_event(ss_ctx *ctx) {
  if (ctx->timer_used == ctx->timer_events.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->timer_events.push_back(e);
  }
  return ctx->timer_events[ctx->timer_used++];
}

void segment_point(ss_ctx *ctx) {
  if (!ctx->seg_graphs || ctx->seg_failed) return;
  hipStreamCaptureStatus status = hipStreamCaptureStatusNone;
  hipGraph_t cur = nullptr;
  size_t nodes = 0;
  if (hipStreamGetCaptureInfo_v2(ctx->stream, &status, nullptr, &cur, nullptr, nullptr) != hipSuccess ||
      status != hipStreamCaptureStatusActive || !cur || hipGraphGetNodes(cur, nullptr, &nodes) != hipSuccess) {
    ctx->seg_failed = true;
    return;
  }
  if (nodes < ctx->seg_limit) return;
  hipGraph_t done = nullptr;
  if (hipStreamEndCapture(ctx->stream, &done) != hipSuccess || !done) {
    ctx->seg_failed = true;
    return;
  }
  ctx->seg_graphs->push_back(done);
  if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) ctx->seg_failed = true;
}

KernelScope::KernelScope(ss_ctx *c, const char *family, double flops, double bytes) : ctx(c), on(false) {
  segment_point(ctx);
  const std::string &tf = ctx->timer_family;
  const bool match = !tf.empty() && (tf == family || (tf[0] == ',' && tf.find(std::string(",") + family + ",") !=
                                                                           std::string::npos));
  if (match) {
    hipEvent_t e = timer_event(ctx);
    if (e && hipEventRecord(e, ctx->stream) == hipSuccess) {
      on = true;
      ctx->timer_flops += flops;
      ctx->timer_bytes += bytes;
    }
  }
}

KernelScope::~KernelScope() {
  if (!on) return;
  hipEvent_t e = timer_event(ctx);
  if (!e || hipEventRecord(e, ctx->stream) != hipSuccess) {
    ctx->timer_used -= e ? 2 : 1;  // drop the unmatched start event
  }
}

static ss_status enter(ss_ctx *ctx) {
  if (!ctx) return SS_ERR_ARG;
  ctx->err.clear();
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SS_ERR_DEVICE, "hipSetDevice failed");
  return SS_OK;
}

}  // namespace ss

using namespace ss;

extern "C" {

const char *ss_status_string(ss_status st) {
  switch (st) {
    case SS_OK: return "ok";
    case SS_ERR_ARG: return "invalid argument";
    case SS_ERR_NOMEM: return "device allocation failed";
    case SS_ERR_DEVICE: return "HIP runtime error";
    case SS_ERR_UNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

const char *ss_last_error(const ss_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

ss_status ss_create(ss_ctx **out, int device, void *hip_stream) {
  if (!out) return SS_ERR_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SS_ERR_ARG;
  // the fixed scratch of ss_transmission_noalloc: its device address, once per device, with that device
  // current (the caller's current device is restored)
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return SS_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return SS_ERR_DEVICE;
  const ss_status sst = transmission_scratch_init(device);
  (void)hipSetDevice(prev);
  if (sst != SS_OK) return sst;
  ss_ctx *ctx = new (std::nothrow) ss_ctx();
  if (!ctx) return SS_ERR_NOMEM;
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  *out = ctx;
  return SS_OK;
}

void ss_destroy(ss_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto &b : ctx->slot)
    if (b.ptr) (void)hipFree(b.ptr);
  if (ctx->host_word) (void)hipHostFree(ctx->host_word);
  for (hipEvent_t e : ctx->timer_events) (void)hipEventDestroy(e);
  delete ctx;
}

ss_status ss_set_stream(ss_ctx *ctx, void *hip_stream) {
  if (!ctx) return SS_ERR_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  return SS_OK;
}

ss_status ss_set_sync_free(ss_ctx *ctx, int on) {
  if (!ctx) return SS_ERR_ARG;
  ctx->sync_free = on != 0;
  return SS_OK;
}

ss_status ss_set_lu_width(ss_ctx *ctx, int width) {
  if (!ctx) return SS_ERR_ARG;
  if (width != 0 && width != 32 && width != 16 && width != 8)
    return ss::fail(ctx, SS_ERR_ARG, "ss_set_lu_width: width must be 0, 32, 16 or 8");
  ctx->lu_width = width;
  return SS_OK;
}

ss_status ss_set_lu_tile(ss_ctx *ctx, int tile) {
  if (!ctx) return SS_ERR_ARG;
  if (tile != 0 && tile != 1) return ss::fail(ctx, SS_ERR_ARG, "ss_set_lu_tile: tile must be 0 or 1");
  ctx->lu_tile = tile;
  return SS_OK;
}

ss_status ss_synchronize(ss_ctx *ctx) {
  SS_TRY(enter(ctx));
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(ctx, SS_ERR_DEVICE, "stream synchronize failed");
  return SS_OK;
}

size_t ss_workspace_bytes(const ss_ctx *ctx) {
  if (!ctx) return 0;
  size_t t = 0;
  for (auto &b : ctx->slot) t += b.bytes;
  return t;
}

namespace {
// One workspace request in call order, as workspace() grants it: grow-only, 9/8 of the request.
void ws_request(size_t *hold, Slot slot, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (hold[slot] < bytes) hold[slot] = bytes + bytes / 8;
}
// Inverses of the diagonal blocks that a batched LU of order n keeps for its triangular leaves.
size_t lu_inverse_bytes(size_t nmat, int n) {
  const size_t w = (size_t)lu_panel_width(n);
  return sizeof(double2) * nmat * (size_t)cdiv(n, (int)w) * 2 * w * w;
}
}  // namespace

ss_status ss_workspace_size(int batch, int nb, int s, int m, int prec, int flags, size_t *bytes) {
  if (!bytes || batch < 0 || nb < 1 || s < 1 || m < 0) return SS_ERR_ARG;
  if (s > SS_MAX_S) return SS_ERR_UNSUPPORTED;
  if (prec != SS_PREC_FP64 && prec != SS_PREC_FP32 && prec != SS_PREC_FP32_LU && prec != SS_PREC_BF16) return SS_ERR_ARG;
  // the requests of the four steps in their order, mirroring the drivers (the decimation, the
  // recursion's sweep, the corner system, the transmission); the precision adds the FP32 coupling
  // blocks of the BF16-term products
  size_t h[kNumSlots] = {};
  const size_t c = sizeof(double2), i4 = sizeof(int), b = (size_t)batch, S = (size_t)s, ss2 = S * S;
  // ss_lead_selfenergy: decimation state and systems, then the final solves
  ws_request(h, kSlotDec, c * 12 * ss2 * b);
  ws_request(h, kSlotPerm, i4 * 2 * b * S);
  ws_request(h, kSlotZp, i4 * 2 * b);
  ws_request(h, kSlotMisc, b * (2 * 8 + 8 + 4 + 4 + 4) + 64 + b * 4 * 8);
  ws_request(h, kSlotLuInv, lu_inverse_bytes(b, s));
  ws_request(h, kSlotObc, c * 2 * b * ss2);
  ws_request(h, kSlotLuInv, lu_inverse_bytes(2 * b, s));
  // ss_precompute_columns: the augmented systems of both recursions and their solution slots
  ws_request(h, kSlotM, c * 2 * b * S * 2 * S);
  ws_request(h, kSlotPerm, i4 * 2 * b * S);
  ws_request(h, kSlotZp, i4 * 3 * b);
  ws_request(h, kSlotX, c * 2 * b * (size_t)nb * ss2);
  if (prec == SS_PREC_BF16) ws_request(h, kSlotCpl, sizeof(float2) * 2 * b * ss2);
  if (flags & SS_KEEP_FACTORS) {
    ws_request(h, kSlotFact, c * b * (size_t)nb * ss2);
    ws_request(h, kSlotFactPerm, i4 * b * (size_t)nb * S);
    if (lu_panel_width(s) == 32) ws_request(h, kSlotFactInv, c * b * (size_t)nb * (size_t)lu_inverse_elems(s, 32));
  }
  ws_request(h, kSlotLuInv, lu_inverse_bytes(2 * b, s));
  // ss_apply_obc: the corner systems [R | C Q b' | I] of order 2s
  const size_t n = 2 * S, nrhs = 2 * S + (size_t)m, ldm = 4 * S + (size_t)m;
  ws_request(h, kSlotM, c * b * n * ldm);
  ws_request(h, kSlotPerm, i4 * b * n);
  ws_request(h, kSlotZp, i4 * b);
  ws_request(h, kSlotObc, c * b * (4 * ss2 + n * nrhs));
  ws_request(h, kSlotLuInv, lu_inverse_bytes(b, 2 * s));
  // ss_transmission: per-tile partial sums
  ws_request(h, kSlotMisc, sizeof(double) * transmission_partials(batch, s));
  size_t t = 0;
  for (int k = 0; k < kNumSlots; ++k) t += h[k];
  *bytes = batch == 0 ? 0 : t;
  return SS_OK;
}

ss_status ss_kernel_timer(ss_ctx *ctx, const char *family) {
  SS_TRY(enter(ctx));
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(ctx, SS_ERR_DEVICE, "stream synchronize failed");
  ctx->timer_family = family ? family : "";
  ctx->timer_used = 0;
  ctx->timer_flops = 0.0;
  ctx->timer_bytes = 0.0;
  return SS_OK;
}

ss_status ss_kernel_timer_read(ss_ctx *ctx, double *total_ms, long long *launches, double *flops,
                               double *bytes) {
  SS_TRY(enter(ctx));
  if (!total_ms || !launches) return fail(ctx, SS_ERR_ARG, "ss_kernel_timer_read: null output");
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(ctx, SS_ERR_DEVICE, "stream synchronize failed");
  double t = 0.0;
  const size_t pairs = ctx->timer_used / 2;
  for (size_t i = 0; i < pairs; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->timer_events[2 * i], ctx->timer_events[2 * i + 1]) != hipSuccess)
      return fail(ctx, SS_ERR_DEVICE, "hipEventElapsedTime failed");
    t += ms;
  }
  *total_ms = t;
  *launches = (long long)pairs;
  if (flops) *flops = ctx->timer_flops;
  if (bytes) *bytes = ctx->timer_bytes;
  ctx->timer_used = 0;
  ctx->timer_flops = 0.0;
  ctx->timer_bytes = 0.0;
  return SS_OK;
}

ss_status ss_lead_selfenergy(ss_ctx *ctx, int batch, int s, int nk, const ss_c128 *H00, const ss_c128 *H01,
                             const ss_c128 *S00, const ss_c128 *S01, const int *kidx, const double *E, double eta,
                             double tol, int max_iter, ss_c128 *sigma, int *iters, double *resid, int *info) {
  SS_TRY(enter(ctx));
  if (batch < 0 || s < 1 || nk < 1) return fail(ctx, SS_ERR_ARG, "ss_lead_selfenergy: batch, s or nk out of range");
  if (s > SS_MAX_S) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_lead_selfenergy: s > SS_MAX_S");
  if (batch == 0) return SS_OK;
  if (!H00 || !H01 || !S00 || !S01 || !E || !sigma)
    return fail(ctx, SS_ERR_ARG, "ss_lead_selfenergy: null input or output pointer");
  if (!(eta >= 0.0)) return fail(ctx, SS_ERR_ARG, "ss_lead_selfenergy: eta must be >= 0");
  ctx->corner_valid = false;  // decimation reuses the corner system's workspace
  return lead_selfenergy(ctx, batch, s, nk, H00, H01, S00, S01, kidx, E, eta, tol, max_iter, sigma, iters, resid,
                         info);
}

ss_status ss_precompute_columns(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E,
                                double absorb, int prec, int flags, ss_c128 *Q, int *info) {
  SS_TRY(enter(ctx));
  if (!hs) return fail(ctx, SS_ERR_ARG, "ss_precompute_columns: null structure");
  if (batch < 0 || hs->nb < 1 || hs->s < 1 || hs->nk < 1)
    return fail(ctx, SS_ERR_ARG, "ss_precompute_columns: batch, nb, s or nk out of range");
  if (hs->s > SS_MAX_S) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_precompute_columns: s > SS_MAX_S");
  if (batch == 0) return SS_OK;
  if (!hs->H_diag || !hs->S_diag || !E || !Q || (hs->nb > 1 && (!hs->H_upper || !hs->S_upper)))
    return fail(ctx, SS_ERR_ARG, "ss_precompute_columns: null input or output pointer");
  if (prec != SS_PREC_FP64 && prec != SS_PREC_FP32 && prec != SS_PREC_FP32_LU && prec != SS_PREC_BF16)
    return fail(ctx, SS_ERR_ARG, "ss_precompute_columns: unknown precision");
  if (flags & ~SS_KEEP_FACTORS) return fail(ctx, SS_ERR_ARG, "ss_precompute_columns: unknown flags");
  if (!(absorb >= 0.0) || !std::isfinite(absorb))
    return fail(ctx, SS_ERR_ARG, "ss_precompute_columns: absorb must be finite and >= 0");
  ctx->corner_valid = false;  // the recursion reuses the corner system's workspace
  return precompute_columns(ctx, hs, batch, kidx, E, absorb, prec, flags, Q, info);
}

ss_status ss_precompute_columns_spike(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E,
                                      double absorb, int prec, int nparts, ss_c128 *Q, int *info) {
  SS_TRY(enter(ctx));
  if (!hs || batch < 0 || hs->nb < 1 || hs->s < 1 || hs->nk < 1)
    return fail(ctx, SS_ERR_ARG, "ss_precompute_columns_spike: size out of range");
  if (hs->s > SS_MAX_S) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_precompute_columns_spike: s > SS_MAX_S");
  if (nparts < 1 || nparts > hs->nb || (nparts & (nparts - 1)) != 0)
    return fail(ctx, SS_ERR_ARG, "ss_precompute_columns_spike: nparts must be a power of two in [1, nb]");
  if (prec != SS_PREC_FP64 && prec != SS_PREC_FP32 && prec != SS_PREC_FP32_LU && prec != SS_PREC_BF16)
    return fail(ctx, SS_ERR_ARG, "ss_precompute_columns_spike: unknown precision");
  if (!(absorb >= 0.0) || !std::isfinite(absorb))
    return fail(ctx, SS_ERR_ARG, "ss_precompute_columns_spike: absorb must be finite and >= 0");
  if (batch == 0) return SS_OK;
  if (!hs->H_diag || !hs->S_diag || (hs->nb > 1 && (!hs->H_upper || !hs->S_upper)) || !E || !Q)
    return fail(ctx, SS_ERR_ARG, "ss_precompute_columns_spike: null pointer");
  ctx->fact_valid = false;
  return precompute_spike(ctx, hs, batch, kidx, E, absorb, prec, nparts, Q, info);
}

ss_status ss_measure_ceilings(ss_ctx *ctx, double *ceil) {
  SS_TRY(enter(ctx));
  if (!ceil) return fail(ctx, SS_ERR_ARG, "ss_measure_ceilings: null output");
  if (ctx->sync_free) return fail(ctx, SS_ERR_ARG, "ss_measure_ceilings: not in sync-free mode");
  return measure_ceilings(ctx, ceil);
}

ss_status ss_lu_factor(ss_ctx *ctx, int nmat, int n, ss_c128 *A, int *perm, int *info) {
  SS_TRY(enter(ctx));
  if (nmat < 0 || n < 1) return fail(ctx, SS_ERR_ARG, "ss_lu_factor: size out of range");
  if (n > kLuMaxN) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_lu_factor: n > 2048");
  if (nmat == 0) return SS_OK;
  if (!A || !perm) return fail(ctx, SS_ERR_ARG, "ss_lu_factor: null pointer");
  return lu_factor_dense(ctx, nmat, n, (double2 *)A, perm, info);
}

ss_status ss_apply_obc(ss_ctx *ctx, int batch, int nb, int s, const ss_c128 *Q, const ss_c128 *sigma, double absorb,
                       int m, const ss_c128 *inj, ss_c128 *psi, ss_c128 *gc, int *info) {
  SS_TRY(enter(ctx));
  if (batch < 0 || nb < 1 || s < 1 || m < 0) return fail(ctx, SS_ERR_ARG, "ss_apply_obc: size out of range");
  if (s > SS_MAX_S) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_apply_obc: s > SS_MAX_S");
  if (batch == 0) return SS_OK;
  if (!Q || !sigma || (m > 0 && (!inj || !psi)))
    return fail(ctx, SS_ERR_ARG, "ss_apply_obc: null input or output pointer");
  if (!(absorb >= 0.0) || !std::isfinite(absorb))
    return fail(ctx, SS_ERR_ARG, "ss_apply_obc: absorb must be finite and >= 0");
  ss_status st = apply_obc(ctx, batch, nb, s, Q, sigma, absorb, m, inj, psi, gc, info);
  ctx->corner_valid = st == SS_OK;
  ctx->corner_absorb = absorb;
  ctx->corner_batch = batch;
  ctx->corner_s = s;
  ctx->corner_ldm = 4 * s + m;
  return st;
}

ss_status ss_transmission(ss_ctx *ctx, int batch, int s, const ss_c128 *gc, const ss_c128 *sigma, double *T) {
  SS_TRY(enter(ctx));
  if (batch < 0 || s < 1) return fail(ctx, SS_ERR_ARG, "ss_transmission: size out of range");
  if (s > SS_MAX_S) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_transmission: s > SS_MAX_S");
  if (batch == 0) return SS_OK;
  if (!gc || !sigma || !T) return fail(ctx, SS_ERR_ARG, "ss_transmission: null pointer");
  return transmission(ctx, batch, s, gc, sigma, T);
}

ss_status ss_transmission_noalloc(ss_ctx *ctx, int batch, int s, const ss_c128 *gc, const ss_c128 *sigma,
                                  double *T) {
  SS_TRY(enter(ctx));
  if (batch < 0 || s < 1) return fail(ctx, SS_ERR_ARG, "ss_transmission_noalloc: size out of range");
  if (s > SS_MAX_S) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_transmission_noalloc: s > SS_MAX_S");
  if (batch == 0) return SS_OK;
  if (!gc || !sigma || !T) return fail(ctx, SS_ERR_ARG, "ss_transmission_noalloc: null pointer");
  return transmission_noalloc(ctx, batch, s, gc, sigma, T);
}

ss_status ss_injection_left(ss_ctx *ctx, int batch, int s, const ss_c128 *sigma, double tol, int mmax,
                            ss_c128 *inj, int *rank) {
  SS_TRY(enter(ctx));
  if (batch < 0 || s < 1 || mmax < 1) return fail(ctx, SS_ERR_ARG, "ss_injection_left: size out of range");
  if (s > SS_MAX_S) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_injection_left: s > SS_MAX_S");
  if (batch == 0) return SS_OK;
  if (!sigma || !inj) return fail(ctx, SS_ERR_ARG, "ss_injection_left: null pointer");
  return injection_left(ctx, batch, s, sigma, tol, mmax, inj, rank);
}

ss_status ss_refine_psi(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E, const ss_c128 *Q,
                        const ss_c128 *sigma, int m, const ss_c128 *inj, ss_c128 *psi, double tol, int max_iter,
                        int *iters, double *resid) {
  SS_TRY(enter(ctx));
  if (!hs || batch < 0 || m < 1 || hs->nb < 1 || hs->s < 1 || hs->nk < 1)
    return fail(ctx, SS_ERR_ARG, "ss_refine_psi: size out of range");
  if (hs->s > SS_MAX_S) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_refine_psi: s > SS_MAX_S");
  if (batch == 0) return SS_OK;
  if (!hs->H_diag || !hs->S_diag || (hs->nb > 1 && (!hs->H_upper || !hs->S_upper)) || !E || !Q || !sigma ||
      !inj || !psi)
    return fail(ctx, SS_ERR_ARG, "ss_refine_psi: null pointer");
  return refine_psi(ctx, hs, batch, kidx, E, Q, sigma, m, inj, psi, tol, max_iter, iters, resid);
}

ss_status ss_transmission_psi(ss_ctx *ctx, int batch, int nb, int s, int m, const ss_c128 *psi, const ss_c128 *sigma,
                              const ss_c128 *psi0, const ss_c128 *gc, double *T) {
  SS_TRY(enter(ctx));
  if (batch < 0 || nb < 1 || s < 1 || m < 1) return fail(ctx, SS_ERR_ARG, "ss_transmission_psi: size out of range");
  if (s > SS_MAX_S) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_transmission_psi: s > SS_MAX_S");
  if (batch == 0) return SS_OK;
  if (!psi || !sigma || !T) return fail(ctx, SS_ERR_ARG, "ss_transmission_psi: null pointer");
  if ((psi0 == nullptr) != (gc == nullptr))
    return fail(ctx, SS_ERR_ARG, "ss_transmission_psi: psi0 and gc are given together or not at all");
  return transmission_psi(ctx, batch, nb, s, m, psi, sigma, psi0, gc, T);
}

ss_status ss_observables(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E, int m,
                         const ss_c128 *psi, double *density, double *current) {
  SS_TRY(enter(ctx));
  if (!hs || batch < 0 || m < 1 || hs->nb < 1 || hs->s < 1 || hs->nk < 1)
    return fail(ctx, SS_ERR_ARG, "ss_observables: size out of range");
  if (hs->s > SS_MAX_S) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_observables: s > SS_MAX_S");
  if (batch == 0 || (!density && !current)) return SS_OK;
  if (!hs->S_diag || (hs->nb > 1 && (!hs->H_upper || !hs->S_upper)) || !E || !psi)
    return fail(ctx, SS_ERR_ARG, "ss_observables: null pointer");
  return observables(ctx, hs, batch, kidx, E, m, psi, density, current);
}

ss_status ss_energy_integral(ss_ctx *ctx, int batch, int n, const double *w, const double *x, double *out) {
  SS_TRY(enter(ctx));
  if (batch < 0 || n < 0) return fail(ctx, SS_ERR_ARG, "ss_energy_integral: size out of range");
  if (n == 0) return SS_OK;
  if (!out || (batch > 0 && (!w || !x))) return fail(ctx, SS_ERR_ARG, "ss_energy_integral: null pointer");
  return energy_integral(ctx, batch, n, w, x, out);
}

// ---------------------------------------------------------------- learned warm start

static bool dims_ok(int nlayer, const int *dims) {
  if (nlayer < 1 || nlayer > 16 || !dims) return false;
  for (int l = 0; l <= nlayer; ++l)
    if (dims[l] < 1) return false;
  return true;
}

size_t ss_mlp_param_count(int nlayer, const int *dims) {
  return dims_ok(nlayer, dims) ? mlp_param_count(nlayer, dims) : 0;
}

ss_status ss_mlp_forward(ss_ctx *ctx, int nlayer, const int *dims, const float *params, int n, const float *X,
                         float *acts) {
  SS_TRY(enter(ctx));
  if (!dims_ok(nlayer, dims) || n < 0) return fail(ctx, SS_ERR_ARG, "ss_mlp_forward: bad layer sizes");
  if (n == 0) return SS_OK;
  if (!params || !X || !acts) return fail(ctx, SS_ERR_ARG, "ss_mlp_forward: null pointer");
  if (n > 65535 * 64) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_mlp_forward: n too large");
  return mlp_forward(ctx, nlayer, dims, params, n, X, acts);
}

ss_status ss_mlp_backward(ss_ctx *ctx, int nlayer, const int *dims, const float *params, int n, const float *X,
                          const float *acts, const float *target, float *grads, double *loss) {
  SS_TRY(enter(ctx));
  if (!dims_ok(nlayer, dims) || n < 1) return fail(ctx, SS_ERR_ARG, "ss_mlp_backward: bad sizes");
  if (!params || !X || !acts || !target || !grads || !loss)
    return fail(ctx, SS_ERR_ARG, "ss_mlp_backward: null pointer");
  if (n > 65535 * 64) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_mlp_backward: n too large");
  return mlp_backward(ctx, nlayer, dims, params, n, X, acts, target, grads, loss);
}

ss_status ss_mlp_adam(ss_ctx *ctx, size_t count, float *params, const float *grads, float *m, float *v, float lr,
                      float beta1, float beta2, float eps, int step) {
  SS_TRY(enter(ctx));
  if (step < 1 || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(ctx, SS_ERR_ARG, "ss_mlp_adam: bad hyper-parameters");
  if (count == 0) return SS_OK;
  if (!params || !grads || !m || !v) return fail(ctx, SS_ERR_ARG, "ss_mlp_adam: null pointer");
  return mlp_adam(ctx, count, params, grads, m, v, lr, beta1, beta2, eps, step);
}

ss_status ss_warm_features(ss_ctx *ctx, int n, const double *E, const double *k, int nfreq, double e_scale, float *X) {
  SS_TRY(enter(ctx));
  if (n < 0 || nfreq < 0 || nfreq > 64 || !(e_scale > 0)) return fail(ctx, SS_ERR_ARG, "ss_warm_features: bad sizes");
  if (n == 0) return SS_OK;
  if (!E || !k || !X) return fail(ctx, SS_ERR_ARG, "ss_warm_features: null pointer");
  return warm_features(ctx, n, E, k, nfreq, e_scale, X);
}

ss_status ss_sigma_moments(ss_ctx *ctx, int n, int s, const ss_c128 *sigma, float std_floor, float *mean, float *std) {
  SS_TRY(enter(ctx));
  if (n < 1 || s < 1 || s > SS_MAX_S) return fail(ctx, SS_ERR_ARG, "ss_sigma_moments: bad sizes");
  if (!sigma || !mean || !std) return fail(ctx, SS_ERR_ARG, "ss_sigma_moments: null pointer");
  return sigma_moments(ctx, n, s, sigma, std_floor, mean, std);
}

ss_status ss_sigma_encode(ss_ctx *ctx, int n, int s, const ss_c128 *sigma, const float *mean, const float *std,
                          float *y) {
  SS_TRY(enter(ctx));
  if (n < 0 || s < 1 || s > SS_MAX_S) return fail(ctx, SS_ERR_ARG, "ss_sigma_encode: bad sizes");
  if (n == 0) return SS_OK;
  if (!sigma || !mean || !std || !y) return fail(ctx, SS_ERR_ARG, "ss_sigma_encode: null pointer");
  return sigma_encode(ctx, n, s, sigma, mean, std, y);
}

ss_status ss_sigma_decode(ss_ctx *ctx, int n, int s, const float *y, const float *mean, const float *std,
                          ss_c128 *sigma) {
  SS_TRY(enter(ctx));
  if (n < 0 || s < 1 || s > SS_MAX_S) return fail(ctx, SS_ERR_ARG, "ss_sigma_decode: bad sizes");
  if (n == 0) return SS_OK;
  if (!sigma || !mean || !std || !y) return fail(ctx, SS_ERR_ARG, "ss_sigma_decode: null pointer");
  return sigma_decode(ctx, n, s, y, mean, std, sigma);
}

ss_status ss_lead_selfenergy_warm(ss_ctx *ctx, int batch, int s, int nk, const ss_c128 *H00, const ss_c128 *H01,
                                  const ss_c128 *S00, const ss_c128 *S01, const int *kidx, const double *E,
                                  double eta, const ss_c128 *sigma_init, double tol, int max_newton, int smith_steps,
                                  ss_c128 *sigma, int *newton_iters, int *dec_iters, double *resid, int *info) {
  SS_TRY(enter(ctx));
  if (batch < 0 || s < 1 || nk < 1 || max_newton < 0 || smith_steps < 0)
    return fail(ctx, SS_ERR_ARG, "ss_lead_selfenergy_warm: size out of range");
  if (s > SS_MAX_S) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_lead_selfenergy_warm: s > SS_MAX_S");
  if (batch > 32767) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_lead_selfenergy_warm: batch > 32767");
  if (batch == 0) return SS_OK;
  if (!H00 || !H01 || !S00 || !S01 || !E || !sigma_init || !sigma)
    return fail(ctx, SS_ERR_ARG, "ss_lead_selfenergy_warm: null pointer");
  if (sigma_init == sigma) return fail(ctx, SS_ERR_ARG, "ss_lead_selfenergy_warm: sigma_init must not alias sigma");
  if (ctx->sync_free) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_lead_selfenergy_warm: needs host polls");
  return lead_selfenergy_warm(ctx, batch, s, nk, H00, H01, S00, S01, kidx, E, eta, sigma_init, tol, max_newton,
                              smith_steps, sigma, newton_iters, dec_iters, resid, info);
}

}  // extern "C"
