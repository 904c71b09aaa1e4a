// Batched solve of dense complex systems D X = RHS by LU with partial pivoting (FP64).
#pragma once

#include "common.hpp"

namespace ss {

// Each of the nmat systems lives in an augmented row-major matrix [D | RHS] of n rows and
// ldm >= n + nrhs columns.  Row interchanges are never performed in memory: the factorization keeps
// a logical-to-physical row map `perm` instead, and every kernel addresses rows through it.  After
// the call the physical rows hold L (unit lower, below the diagonal) and U of P D = L U, the RHS
// columns hold L^{-1} P RHS, and X receives U^{-1} L^{-1} P RHS.
struct LuDesc {
  int nmat = 0, n = 0, nrhs = 0;
  double2 *M = nullptr;
  long sM = 0;
  int ldm = 0;
  int *perm = nullptr;  // [nmat][n]
  long sP = 0;
  int *zp = nullptr;  // [nmat]: 1 + first column with an exactly zero pivot, 0 if none
  double2 *X = nullptr;
  long sX = 0;
  const long *xoff = nullptr;  // optional per-system offsets of X (elements) in place of mat * sX
  int ldx = 0;
  // optional: system i is skipped (every kernel returns at once) when skip[i >> skip_shift] != 0
  const int *skip = nullptr;
  int skip_shift = 0;
  // optional: right-hand sides in a separate buffer (rows in physical order, ld ldb) instead of
  // columns [n, n + nrhs) of M
  double2 *B = nullptr;
  long sB = 0;
  int ldb = 0;
  // products of the recursive factorization and of the triangular solves on the FP32 matrix cores
  // (operands rounded to FP32, FP32 accumulation, FP64 storage); panels, pivots and leaves stay FP64
  bool f32 = false;
  // lu_apply only: inverses of the 32 x 32 diagonal blocks of L and U kept from the factorization's
  // panels ([mat][panel][L, U][32][32], system stride sInv); with them (and 32-column panels) the block
  // solves multiply by the inverses instead of substituting
  const double2 *inv = nullptr;
  long sInv = 0;
};

// Default panel width of the factorization for order n (32 up to n = 1024, 8 up to 2048); a context
// may ask for another width (ss_ctx::lu_width) where lu_panel_width_ok allows it.
int lu_panel_width(int n);
bool lu_panel_width_ok(int n, int w);
// The panel width the context's factorizations of order n use (its own width where valid, else the
// default), and the doubles2 per system of the diagonal-block inverses they keep.
int lu_width_of(ss_ctx *ctx, int n);
long lu_inverse_elems(int n, int w);
// Largest order supported.
constexpr int kLuMaxN = 2048;

// Enqueue the factorization and both triangular solves on ctx->stream.  The caller fills the
// augmented matrices and sets perm to the identity (or lets `lu_identity_perm` do it).
ss_status lu_solve(ss_ctx *ctx, const LuDesc &d);
ss_status lu_identity_perm(ss_ctx *ctx, const LuDesc &d);
// Apply factors kept from an earlier lu_solve (M holds L\U in physical rows, perm the row map) to new
// right-hand sides: X = U^{-1} L^{-1} P RHS (no factorization).
ss_status lu_apply(ss_ctx *ctx, const LuDesc &d);
// Factor nmat dense n x n systems in place and return the factors in pivoted row order (getrf layout)
// with the row map perm and the zero-pivot codes info (may be null).
ss_status lu_factor_dense(ss_ctx *ctx, int nmat, int n, double2 *A, int *perm, int *info);

}  // namespace ss
