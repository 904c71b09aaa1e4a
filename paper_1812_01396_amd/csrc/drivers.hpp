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

ss_status precompute_ragged(ss_ctx *ctx, const RaggedBatch &rb, double absorb, int prec, ss_c128 *Q, int *info);

ss_status precompute_columns(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E,
                             double absorb, int prec, int flags, ss_c128 *Q, int *info);
// Step 1 through nparts partitions per instance and the recursive SPIKE merge of their columns.
ss_status precompute_spike(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E, double absorb,
                           int prec, int nparts, ss_c128 *Q, int *info);

ss_status lead_selfenergy(ss_ctx *ctx, int batch, int s, int nk, const ss_c128 *H00, const ss_c128 *H01,
                          const ss_c128 *S00, const ss_c128 *S01, const int *kidx, const double *E,
                          double eta, double tol, int max_iter, ss_c128 *sigma, int *iters,
                          double *resid, int *info, const ss_c128 *const *tab = nullptr);

ss_status apply_obc(ss_ctx *ctx, int batch, int nb, int s, const ss_c128 *Q, const ss_c128 *sigma, double absorb,
                    int m, const ss_c128 *inj, ss_c128 *psi, ss_c128 *gc, int *info);
// The same for a ragged batch (Q packed as by precompute_ragged); psi_tab: per-instance destinations
// [nb(i)][s][m] of psi (null entries or a null table: psi is not formed).
ss_status apply_obc_ragged(ss_ctx *ctx, const RaggedBatch &rb, const ss_c128 *Q, const ss_c128 *sigma, double absorb,
                           int m, const ss_c128 *inj, ss_c128 *const *psi_tab, ss_c128 *gc, int *info);

ss_status transmission(ss_ctx *ctx, int batch, int s, const ss_c128 *gc, const ss_c128 *sigma, double *T);
// The same with the partial sums in the library's fixed per-device scratch (no allocation); the scratch
// address of `device` (current) is looked up by transmission_scratch_init, called from ss_create.
ss_status transmission_noalloc(ss_ctx *ctx, int batch, int s, const ss_c128 *gc, const ss_c128 *sigma, double *T);
ss_status transmission_scratch_init(int device);
size_t transmission_partials(int batch, int s);

ss_status injection_left(ss_ctx *ctx, int batch, int s, const ss_c128 *sigma, double tol, int mmax, ss_c128 *inj,
                         int *rank);

ss_status refine_psi(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E, const ss_c128 *Q,
                     const ss_c128 *sigma, int m, const ss_c128 *inj, ss_c128 *psi, double tol, int max_iter,
                     int *iters, double *resid);

ss_status lead_selfenergy_warm(ss_ctx *ctx, int batch, int s, int nk, const ss_c128 *H00, const ss_c128 *H01,
                               const ss_c128 *S00, const ss_c128 *S01, const int *kidx, const double *E, double eta,
                               const ss_c128 *sigma_init, double tol, int max_newton, int smith_steps,
                               ss_c128 *sigma, int *newton_iters, int *dec_iters, double *resid, int *info);

ss_status sgemm(ss_ctx *ctx, bool ta, bool tb, int epi, const float *A, int lda, const float *B, int ldb, float *C,
                int ldc, int M, int N, int K, const float *bias, const float *aux, int ldaux);
size_t mlp_param_count(int nlayer, const int *dims);
ss_status mlp_forward(ss_ctx *ctx, int nlayer, const int *dims, const float *params, int n, const float *X,
                      float *acts);
ss_status mlp_backward(ss_ctx *ctx, int nlayer, const int *dims, const float *params, int n, const float *X,
                       const float *acts, const float *target, float *grads, double *loss);
ss_status mlp_adam(ss_ctx *ctx, size_t count, float *params, const float *grads, float *m, float *v, float lr,
                   float b1, float b2, float eps, int step);
ss_status warm_features(ss_ctx *ctx, int n, const double *E, const double *k, int nfreq, double e_scale, float *X);
ss_status sigma_moments(ss_ctx *ctx, int n, int s, const ss_c128 *sigma, float std_floor, float *mean, float *std);
ss_status sigma_encode(ss_ctx *ctx, int n, int s, const ss_c128 *sigma, const float *mean, const float *std, float *y);
ss_status sigma_decode(ss_ctx *ctx, int n, int s, const float *y, const float *mean, const float *std, ss_c128 *sigma);

ss_status transmission_psi(ss_ctx *ctx, int batch, int nb, int s, int m, const ss_c128 *psi, const ss_c128 *sigma,
                           const ss_c128 *psi0, const ss_c128 *gc, double *T);
// Per-tile partial sums of the Caroli T_RL = Re Tr[Gamma_R G_n1 Gamma_L G_n1^H] from the corner gc:
// caroli_rl_tiles(s) per instance at partial[inst * caroli_rl_tiles(s) + tile].
int caroli_rl_tiles(int s);
void launch_caroli_rl_partials(ss_ctx *ctx, int batch, int s, const ss_c128 *gc, const ss_c128 *sigma,
                               double *partial);

ss_status observables(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E, int m,
                      const ss_c128 *psi, double *density, double *current);
ss_status energy_integral(ss_ctx *ctx, int batch, int n, const double *w, const double *x, double *out);

// Rates of plain MFMA, vector-FMA and copy kernels (see ss_measure_ceilings).
ss_status measure_ceilings(ss_ctx *ctx, double *ceil);

}  // namespace ss
