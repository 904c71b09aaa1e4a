/* splitsolve.h — C ABI of the SplitSolve hot path for one AMD MI355X (gfx950).
 *
 * Problem (Sec. 2B, Eq. (wf)): for a block-tridiagonal Hamiltonian H and overlap S with n_B = nb
 * diagonal blocks of size s, at real energy E, solve
 *
 *     (E*S - H - Sigma_L - Sigma_R) psi = Inj
 *
 * where Sigma_L acts on the first and Sigma_R on the last diagonal block.  SplitSolve (Sec. 3B)
 * splits this into a pre-processing step that needs only A = E*S - H (the first and last block
 * columns Q of A^{-1}, Step 1 / Alg. 1) and a post-processing step that folds the boundary
 * self-energies in through a 2s x 2s correction (Sherman-Morrison-Woodbury, Eq. (x), Steps 2-4).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Complex numbers are ss_c128 = {double re, im} (the layout of C99 double complex and of
 *    torch.complex128).  Matrices are ROW-MAJOR and contiguous; a "[a][b][c]" shape lists the
 *    dimensions from slowest to fastest.
 *  - ALL array pointers are DEVICE pointers, owned by the caller.  The library never frees or keeps
 *    caller memory beyond the call; it owns only its context's workspaces.
 *  - Calls are asynchronous on the context's HIP stream: they return once the work is enqueued.
 *    Read outputs after synchronizing that stream (or ss_synchronize).
 *  - Host-detectable problems (null pointers, sizes out of range, a failed HIP call) are returned as
 *    ss_status; the context keeps a message for ss_last_error.  Nothing is printed, nothing thrown.
 *  - Numerical outcomes are written per instance to a caller-owned device int array `info`
 *    (LAPACK style, see each call).  NaN/Inf inputs propagate to the outputs.
 *  - H and S are Hermitian: only the diagonal blocks H_{i,i} and the upper blocks H_{i,i+1} are
 *    passed; the lower blocks are H_{i+1,i} = H_{i,i+1}^H (likewise for S).
 *  - Many (E, k) instances run in one call ("batch").  `nk` (H, S) sets are stored back to back;
 *    instance b uses set kidx[b] (kidx == NULL means set b % nk) and energy E[b].
 *  - One context serves one host thread; calls on one context are ordered on its stream.
 */
#ifndef SPLITSOLVE_H
#define SPLITSOLVE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ss_ctx ss_ctx;

typedef struct {
  double re, im;
} ss_c128;

typedef enum {
  SS_OK = 0,
  SS_ERR_ARG = 1,         /* invalid argument (null pointer, size out of range)            */
  SS_ERR_NOMEM = 2,       /* device workspace allocation failed                             */
  SS_ERR_DEVICE = 3,      /* a HIP runtime call failed (launch, copy, synchronization)      */
  SS_ERR_UNSUPPORTED = 4  /* a well-formed request outside what the library implements     */
} ss_status;

/* Largest block size accepted (the 2s x 2s corner system needs 2s <= 2048). */
#define SS_MAX_S 1024

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` that enqueues on `hip_stream` (a hipStream_t; NULL means
 * the device's default stream).  Workspaces are allocated lazily and grow as needed. */
ss_status ss_create(ss_ctx **ctx, int device, void *hip_stream);
/* Release the context and its workspaces (waits for its stream first).  NULL is a no-op. */
void ss_destroy(ss_ctx *ctx);
/* Redirect later calls to another stream of the same device. */
ss_status ss_set_stream(ss_ctx *ctx, void *hip_stream);
/* on != 0: calls never wait for the stream (required inside stream/graph capture).  Iterative loops
 * then enqueue all of their passes (max_iter) and converged instances skip the work of later passes.
 * Workspaces must already be large enough (run the same calls once eagerly first): growing a
 * workspace waits for the stream, and the call then fails with SS_ERR_ARG instead. */
ss_status ss_set_sync_free(ss_ctx *ctx, int on);
/* Panel width of this context's batched LU factorizations (the recursion of Sec. 3B bottoms out in
 * panels of `width` columns): 0 restores the default by order (32 up to n = 1024, 8 up to 2048); 32 or
 * 16 apply up to n = 1024 and 8 up to n = 2048, and an order outside a width's range uses the default.
 * Results agree to rounding for every width.  SS_ERR_ARG for any other value.  A plan sets the width of
 * each of its groups itself. */
ss_status ss_set_lu_width(ss_ctx *ctx, int width);
/* Tile of the LU's general block products on this context: 0 (default) 64 x 64, 1 32 x 64 (twice the
 * workgroups per product, for batches too small to fill the chip).  SS_ERR_ARG for other values. */
ss_status ss_set_lu_tile(ss_ctx *ctx, int tile);
/* Block the host until the context's stream has drained. */
ss_status ss_synchronize(ss_ctx *ctx);
/* Static text for a status code, and the detail of the context's last failure ("" if none). */
const char *ss_status_string(ss_status st);
const char *ss_last_error(const ss_ctx *ctx);
/* Bytes of device workspace the context currently holds. */
size_t ss_workspace_bytes(const ss_ctx *ctx);
/* Bytes of device workspace a fresh context holds after one pass of the four steps in their order
 * (ss_lead_selfenergy, ss_precompute_columns with `flags`, ss_apply_obc with m columns of psi,
 * ss_transmission) for `batch` instances of nb blocks of size s, with the default LU panel widths; the
 * same calls with these sizes or smaller then run without growing any workspace (for instance in
 * sync-free mode, under stream capture).  Refinement, plans, SPIKE partitions and the warm start need
 * more.  prec is accepted for completeness (the products' precision does not change the workspace).
 * SS_ERR_ARG for sizes out of range or a NULL `bytes`. */
ss_status ss_workspace_size(int batch, int nb, int s, int m, int prec, int flags, size_t *bytes);

/* Kernel timing probe (a profiling aid).  ss_kernel_timer(ctx, family) waits for the stream, clears
 * the accumulated time and from then on brackets every launch of that kernel family on this context
 * with a pair of HIP events on the context's stream (NULL or "" switches the probe off; a list of
 * families enclosed in commas, such as ",form,chain,", times all of them).
 * ss_kernel_timer_read waits for the stream and returns the summed event time in milliseconds, the
 * number of timed launches, (flops, may be NULL) the algorithmic flops of those launches where the
 * launch site states them (8 m n k per complex product; "lu_gemm" only, else 0) and (bytes, may be
 * NULL) their algorithmic HBM bytes (each operand read once and the result written once: 16 (m k +
 * k n + 2 m n) per complex m x n x k update; "lu_gemm" only, else 0) since the last read, then clears
 * them.  Families: "form" (diagonal block formation and product of the recursion),
 * "chain" (Q_i = -X_i Q_{i-1}), "panel" (LU panel factorization), "lu_gemm" (LU trailing and
 * triangular-solve products), "trsm" (triangular-solve leaves), "dec_update" (decimation pass
 * products), "obc" (corner system and psi products), "trans" (transmission), "obs" (observables). */
ss_status ss_kernel_timer(ss_ctx *ctx, const char *family);
/* Measured ceilings of this GPU (a profiling aid, the denominators the roofline fractions are checked
 * against): ceil (HOST pointer, 4 doubles) receives the FP64 matrix-core rate (TFLOP/s,
 * v_mfma_f64_16x16x4 on independent accumulators), the FP32 matrix-core rate (v_mfma_f32_16x16x4), the
 * FP64 vector FMA rate (TFLOP/s) and the rate of a 512 MiB device copy (GB/s, bytes read + written).
 * Waits for the stream; uses and overwrites the context's workspace (~1 GiB). */
ss_status ss_measure_ceilings(ss_ctx *ctx, double *ceil);
ss_status ss_kernel_timer_read(ss_ctx *ctx, double *total_ms, long long *launches, double *flops,
                               double *bytes);

/* ---------------------------------------------------------------- inputs */

typedef struct {
  int nb;                 /* number of diagonal blocks n_B >= 1                                */
  int s;                  /* block size, 1 <= s <= SS_MAX_S                                    */
  int nk;                 /* number of (H, S) sets stored back to back, >= 1                   */
  const ss_c128 *H_diag;  /* [nk][nb][s][s]    H_{i,i}                                          */
  const ss_c128 *H_upper; /* [nk][nb-1][s][s]  H_{i,i+1}  (ignored when nb == 1)                */
  const ss_c128 *S_diag;  /* [nk][nb][s][s]    S_{i,i}   (S is required; pass I for S = 1)      */
  const ss_c128 *S_upper; /* [nk][nb-1][s][s]  S_{i,i+1}                                        */
} ss_btd;

/* ---------------------------------------------------------------- the four steps */

/* Boundary self-energies of a periodic lead (Sec. 3A: the OBCs; computed here by the iterative
 * decimation technique the section names as the standard alternative to FEAST).
 *
 * The lead cell (H00, H01, S00, S01), each [nk][s][s], repeats to infinity on both sides.  With
 * a0 = (E + i*eta) S00 - H00, a1 = E S01 - H01, am1 = a1^H (eta enters the diagonal cell only):
 *     Sigma_L = am1 g_L a1,  g_L = (a0 - am1 g_L a1)^{-1}   (lead on the left of block 1)
 *     Sigma_R = a1 g_R am1,  g_R = (a0 - a1 g_R am1)^{-1}   (lead on the right of block n_B)
 * Decimation doubles the eliminated chain each pass and stops once
 * max|alpha| + max|beta| <= tol * max|a0| (tol <= 0 means 1e-14), or after max_iter passes
 * (max_iter <= 0 means 200).
 *
 * Outputs: sigma [batch][2][s][s] (Sigma_L then Sigma_R); optional (may be NULL): iters [batch]
 * (passes used), resid [batch][2] (relative Frobenius residual of the fixed-point equation,
 * ||Sigma - a (a0 - Sigma)^{-1} a'|| / ||Sigma||, left then right), info [batch]:
 *   0 converged;  -1 not converged within max_iter (last iterate returned);
 *   k > 0: an exactly zero pivot at column k-1 of a factorization. */
ss_status ss_lead_selfenergy(ss_ctx *ctx, int batch, int s, int nk, const ss_c128 *H00,
                             const ss_c128 *H01, const ss_c128 *S00, const ss_c128 *S01,
                             const int *kidx, const double *E, double eta, double tol,
                             int max_iter, ss_c128 *sigma, int *iters, double *resid, int *info);

/* Precision of the recursion's block products in ss_precompute_columns.  Storage is always FP64; the
 * LU panels (pivot search and elimination inside a panel), the triangular leaves, the corner system
 * and every residual are always FP64. */
#define SS_PREC_FP64 0    /* complex FP64 products (FP64 matrix cores)                        */
#define SS_PREC_FP32 1    /* complex FP32 products with FP32 accumulation in the block          */
                          /* formations and the chain; the LU stays FP64                        */
#define SS_PREC_FP32_LU 2 /* as SS_PREC_FP32, and the LU's trailing and triangular-solve        */
                          /* updates in FP32 too (less accurate factors: more refinement passes) */
#define SS_PREC_BF16 3    /* the products of SS_PREC_FP32 on the BF16 matrix cores: every operand  */
                          /* split into three BF16 terms, the six term products of FP32 order,  */
                          /* FP32 accumulation; the LU stays FP64                               */

/* flags of ss_precompute_columns */
#define SS_KEEP_FACTORS 1 /* keep the first-column recursion's factors in the context for     */
                          /* ss_refine_psi (valid until the next ss_precompute_columns call):   */
                          /* per block the LU (16 s^2 bytes) and row map, and with 32-column    */
                          /* panels their diagonal-block inverses (1024 s bytes), with which    */
                          /* the refinement's block solves run as matrix-core products          */

/* Step 1 (Sec. 3B, Alg. 1): Q = [A^{-1}_{:,1}, A^{-1}_{:,n_B}] for A = E*S - H.
 *
 * Backward recursion X_{n_B+1} = 0, (A_{i,i} - A_{i,i+1} X_{i+1}) X_i = A_{i,i-1} with A_{1,0} := I,
 * then Q_i = -X_i Q_{i-1} from Q_0 = -I, gives the first block column; the mirrored recursion (from
 * block 1 upwards with A_{n_B,n_B+1} := I) gives the last one.  Each diagonal system is solved by LU
 * with partial pivoting on the GPU.  prec: SS_PREC_FP64, SS_PREC_FP32, SS_PREC_FP32_LU or SS_PREC_BF16
 * (see above; SS_PREC_BF16 also holds the next step's coupling blocks in FP32, 8 s^2 bytes per
 * system); flags: 0 or SS_KEEP_FACTORS.
 *
 * absorb (>= 0, finite): absorbing boundary.  The open system is T = A - B C with B the identity blocks
 * at the top and bottom and C holding the self-energies (Sec. 3B, Eq. (x)); the section leaves the
 * choice of B and C free.  With absorb > 0 the constant part -i*absorb*I of both self-energies is
 * moved from C into A: the first and last diagonal blocks are formed as E*S - H + i*absorb*I (the
 * single block gets 2i*absorb*I when nb == 1), Q is the first and last block columns of that A'^{-1},
 * and ss_apply_obc must be given the same absorb (it then uses C' = Sigma + i*absorb*I, so that
 * A' - B C' = T).  The pre-processing still needs no self-energy.  Alg. 1 pivots only inside blocks;
 * its pivot blocks are Schur complements of closed sub-chains of the device, nearly singular wherever
 * E approaches one of their eigenvalues, and the closed A itself is singular at the device's
 * eigenvalues; the absorber broadens all of these resonances, which keeps the digits that the closed
 * recursion and the correction otherwise lose.  absorb = 0 is the paper's A = E*S - H.
 *
 * Output Q [batch][nb][s][2s]: block row i holds (A'^{-1})_{i,1} in columns [0, s) and
 * (A'^{-1})_{i,n_B} in columns [s, 2s).  info [batch] (may be NULL): 0, or 1 + (i-1)*s + c for an
 * exactly zero pivot in column c of the i-th diagonal system (1-based i; the smallest such code over
 * both recursions). */
ss_status ss_precompute_columns(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx,
                                const double *E, double absorb, int prec, int flags, ss_c128 *Q,
                                int *info);

/* Step 1 through partitions (Sec. 3B: the partitioned pre-processing and its recursive SPIKE merge,
 * which the paper uses to spread one device over several GPUs; on one GPU it multiplies the systems a
 * small batch offers to the lockstep recursion).  The same Q as ss_precompute_columns (to rounding),
 * computed as follows: the nb blocks are cut into nparts consecutive partitions (a power of two, at
 * most nb; the first nb % nparts partitions are one block longer), Alg. 1 runs on every partition of
 * every instance as one batch (each partition a closed device of its own, with the absorbing shift on
 * both of its end blocks: at a cut it broadens the closed partition's resonances as at the device's
 * ends, and the merge takes it out again), and adjacent partitions are merged level by level
 * (log2 nparts levels): each merge solves one interface system of order 2s per pair (LU with partial
 * pivoting) and updates both halves' columns with products over all their rows.  The merges cost about
 * 16 nb s^3 flops per level and instance, beside the recursion's ~53 nb s^3.  nparts = 1 is the plain
 * recursion.  prec as ss_precompute_columns (no SS_KEEP_FACTORS).  Q [batch][nb][s][2s] as there;
 * info [batch] (may be NULL): 0, or 1 + (i-1)*s + c for an exactly zero pivot in column c of the i-th
 * diagonal system of a partition's recursion (i counted over the whole device), or 1 + la*s + c for one
 * in column c of the interface system after (0-based) block la; the smallest such code.  Workspace: the
 * partitions' recursion as for ss_precompute_columns plus a second Q-sized buffer and the interface
 * systems.  The call uploads small host tables (it is not usable in sync-free mode). */
ss_status ss_precompute_columns_spike(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx,
                                      const double *E, double absorb, int prec, int nparts, ss_c128 *Q,
                                      int *info);

/* The block solver of Step 1 on its own: batched LU with partial pivoting (Alg. 1 solves every
 * D_i X_i = A_{i,i+1} through this factorization).
 *
 * A [nmat][n][n] (row-major complex128) is overwritten with the factors of P A = L U in LAPACK's getrf
 * layout: row i holds row i of L (unit lower, strictly below the diagonal) and of U (on and above it)
 * in the pivoted order.  perm [nmat][n]: row i of P A is row perm[i] of the input.  The pivot of each
 * column is the entry of largest |Re| + |Im| among the remaining rows, the lowest row on ties (the
 * rule of LAPACK's izamax).  info [nmat] (may be NULL): 0, or 1 + c for an exactly zero pivot in
 * column c (elimination continues past it, as getrf does).  1 <= n <= 2048; nmat >= 0. */
ss_status ss_lu_factor(ss_ctx *ctx, int nmat, int n, ss_c128 *A, int *perm, int *info);

/* Steps 2-4 (Sec. 3B, Eq. (x)): fold the boundary self-energies in and recover the wave function.
 *
 * With C Q = [Sigma'_L Q_{1,:}; Sigma'_R Q_{n_B,:}] (2s x 2s), Sigma' = Sigma + i*absorb*I (absorb as
 * given to ss_precompute_columns for this Q; 0: Sigma' = Sigma), R = I - C Q, b' = inj (the non-zero
 * rows of Inj: first block row on top, last block row below) and z = R^{-1} (C Q) b':
 *     psi = Q (b' + z)                      [batch][nb][s][m]
 *     gc  = [Q_{1,:}; Q_{n_B,:}] R^{-1}     [batch][2s][2s]: the corner blocks
 *           [[G_11, G_1n], [G_n1, G_nn]] of G^R = (A - Sigma)^{-1} (Sec. 2B, Eq. (negf)).
 * Q and sigma are the outputs of the two calls above.  m >= 0 (m == 0: inj and psi may be NULL);
 * gc may be NULL.  info [batch] (may be NULL): 0, or 1 + c for an exactly zero pivot in column c
 * of R. */
ss_status ss_apply_obc(ss_ctx *ctx, int batch, int nb, int s, const ss_c128 *Q,
                       const ss_c128 *sigma, double absorb, int m, const ss_c128 *inj, ss_c128 *psi,
                       ss_c128 *gc, int *info);

/* Caroli transmission from the corner of G^R (the product the hot path ends with):
 *     T_LR = Re Tr[Gamma_L G_1n Gamma_R G_1n^H],  T_RL = Re Tr[Gamma_R G_n1 Gamma_L G_n1^H],
 * Gamma = i (Sigma - Sigma^H).  gc [batch][2s][2s] from ss_apply_obc, sigma [batch][2][s][s].
 * Output T [batch][2] = (T_LR, T_RL). */
ss_status ss_transmission(ss_ctx *ctx, int batch, int s, const ss_c128 *gc, const ss_c128 *sigma,
                          double *T);

/* ss_transmission for callers that cannot allocate device memory (code under stream or graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same kernels and the same result, but the
 * per-tile partial sums live in a fixed device array of SS_TRANS_SCRATCH_DOUBLES doubles (8 MiB per GPU,
 * held from library load until the process ends) instead of the context's workspace.  The call
 * allocates nothing and never waits for the stream.  It accepts batch * 2 * ceil(s/32)^2 <=
 * SS_TRANS_SCRATCH_DOUBLES (s = 1024: batch <= 512; s = 512: batch <= 2048) and returns SS_ERR_ARG
 * beyond that.  Every call on one GPU shares that GPU's array and overwrites it (nothing in it needs to
 * start cleared): calls that may overlap on one GPU (other streams, other contexts, other host threads)
 * race and must be ordered by the caller.  Its kernels are not bracketed by ss_kernel_timer. */
#define SS_TRANS_SCRATCH_DOUBLES (1 << 20)
ss_status ss_transmission_noalloc(ss_ctx *ctx, int batch, int s, const ss_c128 *gc, const ss_c128 *sigma,
                                  double *T);

/* Injection from the left lead (Sec. 3A: Inj is built from the lead's modes; here from its
 * broadening).  For each instance, a pivoted Cholesky factorization Gamma_L ~ W_L W_L^H of
 * Gamma_L = i (Sigma_L - Sigma_L^H) stops when the largest remaining diagonal entry falls to
 * tol * max_i Gamma_L[i][i] (tol <= 0 means 1e-12) or after mmax columns; b' = [W_L; 0] is written to
 * inj [batch][2s][mmax] (unused columns are zero) and the number of columns kept to rank [batch]
 * (may be NULL).  Injecting b' gives psi whose last block row carries the transmission:
 * T = Tr[psi_nb^H Gamma_R psi_nb] (ss_transmission_psi). */
ss_status ss_injection_left(ss_ctx *ctx, int batch, int s, const ss_c128 *sigma, double tol, int mmax,
                            ss_c128 *inj, int *rank);

/* Iterative refinement of psi on the full open system (Sec. 3B, Eq. (x) applied to a residual):
 *     r = B b' - (A - B C) psi   (FP64),   psi += A~^{-1} r + Q R^{-1} C A~^{-1} r,
 * where A~^{-1} uses the factors kept by the last ss_precompute_columns(..., SS_KEEP_FACTORS) on this
 * context (the same hs, batch, kidx and E) and R^{-1} the corner factorization of the last
 * ss_apply_obc on this context (no other call may run on the context in between).  With an absorbing
 * boundary both calls must have used the same absorb (SS_ERR_ARG otherwise); A~ and C are then A' and
 * C' = Sigma + i*absorb*I, while the residual is always that of A - Sigma.  Stops per instance
 * when ||r||_F <= tol ||B b'||_F (tol <= 0 means 1e-12) or after max_iter passes (<= 0 means 10).
 * psi [batch][nb][s][m] is updated in place; iters [batch] and resid [batch] (final relative
 * residual) may be NULL. */
ss_status ss_refine_psi(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E,
                        const ss_c128 *Q, const ss_c128 *sigma, int m, const ss_c128 *inj,
                        ss_c128 *psi, double tol, int max_iter, int *iters, double *resid);

/* Transmission carried by a wave function injected from the left lead with b' = [W_L; 0]:
 * T [batch] = Re Tr[psi_nb^H Gamma_R psi_nb] (psi [batch][nb][s][m], sigma [batch][2][s][s]).
 *
 * The injection factor keeps at most m columns of Gamma_L, whose tail (the broadening that eta gives
 * the closed channels, O(eta) per mode, hundreds of modes) then misses from this T.  With psi0 and gc
 * (both, or both NULL) the tail is added back through the corner of G^R:
 *     T = Re Tr[psi_nb^H Gamma_R psi_nb] + (T_RL(gc) - Re Tr[psi0^H Gamma_R psi0]),
 * where gc [batch][2s][2s] is the corner that ss_apply_obc returned together with the unrefined psi and
 * psi0 [batch][s][m] is that psi's last block row.  Since psi0 = G_n1 W_L for the same G_n1 as gc, the
 * bracket is Re Tr[Gamma_R G_n1 (Gamma_L - W_L W_L^H) G_n1^H]: a term as small as the tail, so the
 * error of a low-precision gc enters T only in proportion to it. */
ss_status ss_transmission_psi(ss_ctx *ctx, int batch, int nb, int s, int m, const ss_c128 *psi,
                              const ss_c128 *sigma, const ss_c128 *psi0, const ss_c128 *gc, double *T);

/* ---------------------------------------------------------------- observables
 * Sec. 2B: the charge and current densities follow from the wave function once Eq. (wf) is solved at
 * every energy and momentum (Sec. 5C shows the electron distribution, the current map and the spectral
 * current).  For psi [batch][nb][s][m] injected from the left lead (b' = [W_L; 0], so that
 * psi psi^H = G Gamma_L G^H), with A = E S - H of the instance's (H, S) set (kidx as in the calls above):
 *     density [batch][nb][s]:  n_mu = Re sum_c psi_{mu c} conj((S psi)_{mu c})   (Mulliken: the basis is
 *                              non-orthogonal, n_mu = Re (psi psi^H S)_{mu mu})
 *     current [batch][nb-1]:   J_i = 2 Im Tr[psi_i^H A_{i,i+1} psi_{i+1}]        (units e/h per spin)
 * Either output may be NULL.  Inside the device (E S - H) psi vanishes row block by row block, so J_i
 * is the same at every interface; for b' = [W_L; 0] it equals the transmission T_RL.  Neither depends on
 * the factor W_L chosen.  Only S and the upper blocks of H are read; H_diag may be NULL. */
ss_status ss_observables(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E, int m,
                         const ss_c128 *psi, double *density, double *current);
/* Energy (and momentum) integral as a weighted sum over instances: out[j] = sum_b w[b] x[b][j] for
 * x [batch][n] (for instance the density above with w = quadrature weight x Fermi occupation / (2 pi));
 * summed in instance order. */
ss_status ss_energy_integral(ss_ctx *ctx, int batch, int n, const double *w, const double *x, double *out);

/* ---------------------------------------------------------------- learned warm start
 * The decimation takes no starting iterate; Newton's method on the fixed-point equation of the
 * self-energy does.  For the right lead (the left swaps a1 and am1), with g = (a0 - Sigma)^{-1},
 * M = a1 g, N = g am1 and F = Sigma - a1 N, a Newton step solves the Stein equation D - M D N = -F by
 * Smith's doubling (D += M_j D N_j, M_{j+1} = M_j^2, N_{j+1} = N_j^2, rebalanced) and sets
 * Sigma += D.  The starting iterate comes from a multilayer perceptron trained on self-energies of the
 * decimation.  (Newton on the quadratic and the Stein equation are not in the paper; the self-energies
 * are those of Sec. 3A.) */

/* Parameters of a perceptron with layer sizes dims[0..nlayer] (host array): per layer
 * W [dims[l]][dims[l+1]] row-major, then b [dims[l+1]], FP32.  0 for invalid sizes. */
size_t ss_mlp_param_count(int nlayer, const int *dims);
/* Forward pass on n rows X [n][dims[0]] (FP32, device).  acts (device, FP32) receives every layer's
 * output in order, [n][dims[1]], ..., [n][dims[nlayer]] (hidden layers tanh, the last linear); the
 * network output is the last block.  Products run on the FP32 matrix cores with FP32 accumulation. */
ss_status ss_mlp_forward(ss_ctx *ctx, int nlayer, const int *dims, const float *params, int n, const float *X,
                         float *acts);
/* Gradients (same packing as params) of L = sum (Y - target)^2 / (n dims[nlayer]) by back-propagation
 * through the acts of the forward pass of the same params and X; loss (device double) receives L. */
ss_status ss_mlp_backward(ss_ctx *ctx, int nlayer, const int *dims, const float *params, int n, const float *X,
                          const float *acts, const float *target, float *grads, double *loss);
/* One Adam step (step = 1, 2, ...) on count parameters with moment buffers m, v (device, FP32). */
ss_status ss_mlp_adam(ss_ctx *ctx, size_t count, float *params, const float *grads, float *m, float *v, float lr,
                      float beta1, float beta2, float eps, int step);
/* Features of (E, k) (device doubles [n]): X [n][3 + 4 nfreq] = [E/e_scale, cos k, sin k,
 * sin(j pi E/e_scale), cos(j pi E/e_scale) (j = 1..nfreq), cos(j k), sin(j k) (j = 2..nfreq+1)]. */
ss_status ss_warm_features(ss_ctx *ctx, int n, const double *E, const double *k, int nfreq, double e_scale, float *X);
/* Per component of the encoding [Re Sigma_L, Im Sigma_L, Re Sigma_R, Im Sigma_R] (4 s^2 values) of
 * sigma [n][2][s][s]: mean and standard deviation over the n instances (std at least std_floor). */
ss_status ss_sigma_moments(ss_ctx *ctx, int n, int s, const ss_c128 *sigma, float std_floor, float *mean, float *std);
/* y [n][4 s^2] = (encoding - mean) / std, and back: sigma = mean + std * y. */
ss_status ss_sigma_encode(ss_ctx *ctx, int n, int s, const ss_c128 *sigma, const float *mean, const float *std,
                          float *y);
ss_status ss_sigma_decode(ss_ctx *ctx, int n, int s, const float *y, const float *mean, const float *std,
                          ss_c128 *sigma);
/* Self-energies as ss_lead_selfenergy, starting Newton from sigma_init [batch][2][s][s] (L, R; must not
 * alias sigma).  A side is accepted when its relative residual ||F||_F / ||Sigma||_F <= tol (<= 0:
 * 1e-10) within max_newton steps (<= 0: 8; Smith's doubling with at most smith_steps doublings, <= 0:
 * 40) and its propagator has spectral radius <= 1 + 1e-8 (the retarded root), estimated from 40
 * normalised squarings.  Instances with a rejected side are recomputed by the decimation (tol 1e-14,
 * at most 200 passes).  Outputs (device, any may be NULL except sigma): newton_iters [batch] (largest
 * of the two sides), dec_iters [batch] (decimation passes of the fallback, 0 if accepted), resid
 * [batch][2] (last Newton residuals, L then R), info [batch]: 0 accepted, -2 fallback used, else the
 * decimation's code.  Waits for the stream (host polls); not usable in sync-free mode. */
ss_status ss_lead_selfenergy_warm(ss_ctx *ctx, int batch, int s, int nk, const ss_c128 *H00, const ss_c128 *H01,
                                  const ss_c128 *S00, const ss_c128 *S01, const int *kidx, const double *E,
                                  double eta, const ss_c128 *sigma_init, double tol, int max_newton, int smith_steps,
                                  ss_c128 *sigma, int *newton_iters, int *dec_iters, double *resid, int *info);

/* ---------------------------------------------------------------- uneven batches
 * Many independent (E, k) instances of different block size s and block count nb (the paper solves
 * energy points independently side by side, Sec. 4).  A plan groups the instances by s, sorts each
 * group by nb and splits it into chunks that fit `mem_bytes`; a chunk runs the whole hot path
 * (self-energies, Step 1, Steps 2-4, Caroli T) in lockstep, launching at recursion step t only the
 * instances with more than t blocks.  Groups run on streams of their own.  With use_graph each group's
 * work is captured once at creation, as a sequence of graph segments of about graph_segment_nodes
 * nodes each (cut at launch sites), and every ss_plan_execute replays each group's segments in order on
 * the group's stream (all groups forked from and joined into one origin stream).
 * With autotune, candidate LU panel widths, LU product tiles and chunk sizes are timed per group at
 * creation.
 *
 * Instance blocks are device pointers owned by the caller and must stay valid and unmoved for the
 * plan's life (the plan and its graph keep the addresses; the values are read at every execution).
 * The lead of both sides is the semi-infinite repetition of (H00, H01, S00, S01) as in
 * ss_lead_selfenergy.  psi (optional) receives [nb][s][m] for the injection b' = [W_L; 0] of
 * ss_injection_left with at most m columns (unused columns are zero). */
typedef struct {
  int nb, s;
  double E;
  const ss_c128 *H_diag, *H_upper, *S_diag, *S_upper; /* [nb][s][s], [nb-1][s][s] */
  const ss_c128 *H00, *H01, *S00, *S01;               /* [s][s] each */
  ss_c128 *psi;                                       /* [nb][s][m] or NULL */
} ss_instance;

typedef struct {
  double eta;        /* broadening of the lead's diagonal cell (>= 0) */
  double absorb;     /* absorbing boundary of Step 1 and the corner correction (>= 0; see
                        ss_precompute_columns) */
  double sigma_tol;  /* decimation tolerance (0: 1e-14) */
  int sigma_passes;  /* decimation passes enqueued (0: ceil(log2(1/eta)) + 12, within [16, 200]);
                        converged instances skip later passes, unconverged ones report info -1 */
  int m;             /* columns of psi (0: psi is not formed; then every instance's psi must be NULL) */
  int use_graph;     /* nonzero: capture each size group's work into a graph at creation */
  int autotune;      /* nonzero: time candidate panel widths and chunk sizes per group at creation */
  size_t mem_bytes;  /* device memory for chunk work (0: 32 GiB); a chunk always holds one instance */
  int graph_segment_nodes; /* with use_graph: nodes per captured graph segment (0: 2048; at most 4096) */
} ss_plan_opts;

typedef struct ss_plan ss_plan;

/* Build a plan for n instances (host array, copied).  T [n][2] (T_LR, T_RL) and info [n][4]
 * (self-energy, Step 1 and corner codes as in the single calls, then the decimation passes used) are
 * device outputs in the caller's order, written by every execution.  Creation runs the batch once (the outputs then already hold a
 * result) and waits for it.  The plan runs on ctx's device and is ordered with ctx's stream. */
ss_status ss_plan_create(ss_ctx *ctx, int n, const ss_instance *inst, const ss_plan_opts *opts, double *T,
                         int *info, ss_plan **plan);
/* Enqueue one execution of the whole batch after the work already on ctx's stream; later work on
 * that stream waits for it. */
ss_status ss_plan_execute(ss_plan *plan);
/* Groups of the plan (by block size) and, per group: s, instance count, chunk size, LU panel width,
 * and the autotuner's best probe time in ms (0 without autotune). */
int ss_plan_groups(const ss_plan *plan);
/* The LU product tile (as ss_set_lu_tile) a group of the plan uses; -1 for a bad group index. */
int ss_plan_lu_tile(const ss_plan *plan, int group);
ss_status ss_plan_describe(const ss_plan *plan, int group, int *s, int *count, int *chunk, int *lu_width,
                           double *tune_ms);
/* Nodes of the captured group graphs, summed (0 without use_graph); a negative value -n means that a
 * graph segment came out larger than 8192 nodes (n summed over the groups), and the plan runs as one
 * sync-free enqueue of the same launches instead. */
long long ss_plan_graph_nodes(const ss_plan *plan);
/* Captured graph segments, summed over the groups (0 when the plan does not replay graphs). */
int ss_plan_graph_segments(const ss_plan *plan);
/* Waits for the plan's work and frees it (it does not use the context: a plan may outlive it). */
void ss_plan_destroy(ss_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* SPLITSOLVE_H */
