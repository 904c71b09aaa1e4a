// Internal entry points behind the C ABI (argument checks happen in api.hip).
#pragma once

#include "common.hpp"

namespace ss {

// A batch of instances of one block size s whose block counts differ, sorted by block count (largest
// first).  Device arrays: tab (4 per instance: H_diag, H_upper, S_diag, S_upper), nbv, boff (first
// block of each instance in packed per-block stores), xoff (per recursion system: X offset in
// elements), E.  Host: act[t] = number of instances with more than t blocks.
struct RaggedBatch {
  int s = 0, batch = 0, nb_max = 0;
  long total_blocks = 0;
  const ss_c128 *const *tab = nullptr;
  const int *nbv = nullptr;
  const long *boff = nullptr;
  const long *xoff = nullptr;
  const double *E = nullptr;
  std::vector<int> act;
};

ss_status precompute_ragged(ss_ctx *ctx, const RaggedBatch &rb, int prec, ss_c128 *Q, int *info);

ss_status precompute_columns(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E, int prec,
                             int flags, ss_c128 *Q, int *info);

ss_status lead_selfenergy(ss_ctx *ctx, int batch, int s, int nk, const ss_c128 *H00, const ss_c128 *H01,
                          const ss_c128 *S00, const ss_c128 *S01, const int *kidx, const double *E,
                          double eta, double tol, int max_iter, ss_c128 *sigma, int *iters,
                          double *resid, int *info, const ss_c128 *const *tab = nullptr);

ss_status apply_obc(ss_ctx *ctx, int batch, int nb, int s, const ss_c128 *Q, const ss_c128 *sigma, int m,
                    const ss_c128 *inj, ss_c128 *psi, ss_c128 *gc, int *info);
// The same for a ragged batch (Q packed as by precompute_ragged); psi_tab: per-instance destinations
// [nb(i)][s][m] of psi (null entries or a null table: psi is not formed).
ss_status apply_obc_ragged(ss_ctx *ctx, const RaggedBatch &rb, const ss_c128 *Q, const ss_c128 *sigma, int m,
                           const ss_c128 *inj, ss_c128 *const *psi_tab, ss_c128 *gc, int *info);

ss_status transmission(ss_ctx *ctx, int batch, int s, const ss_c128 *gc, const ss_c128 *sigma, double *T);

ss_status injection_left(ss_ctx *ctx, int batch, int s, const ss_c128 *sigma, double tol, int mmax, ss_c128 *inj,
                         int *rank);

ss_status refine_psi(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E, const ss_c128 *Q,
                     const ss_c128 *sigma, int m, const ss_c128 *inj, ss_c128 *psi, double tol, int max_iter,
                     int *iters, double *resid);

ss_status transmission_psi(ss_ctx *ctx, int batch, int nb, int s, int m, const ss_c128 *psi, const ss_c128 *sigma,
                           double *T);

}  // namespace ss
