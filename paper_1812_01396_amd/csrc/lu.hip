// Batched dense complex LU with partial pivoting and the two triangular solves, on gfx950.
//
// Each system is an augmented row-major matrix [D | RHS] (n rows).  Rows are never moved in memory:
// a logical-to-physical row map `perm` records the interchanges and every kernel addresses rows
// through it (row segments stay contiguous, so loads stay coalesced).
//
// Recursive (column-halving) factorization, so that almost all flops are large MFMA products:
//   lu(c0, c1):  if c1 - c0 <= W: factor the panel in registers (pivot search |Re|+|Im| with the
//                lowest row on ties as in LAPACK, interchange in the row map, scale, rank-1 updates)
//                else with cm the midpoint (a multiple of W):
//                  lu(c0, cm);  L11^{-1} on rows [c0, cm) of columns [cm, c1);
//                  A[cm:n, cm:c1] -= L[cm:n, c0:cm] U[c0:cm, cm:c1];  lu(cm, c1)
// then the right-hand sides: Y = L^{-1} P RHS and X = U^{-1} Y by recursive triangular solves whose
// leaves are W-row substitutions inside a tile and whose inner nodes are MFMA products.
#include "lu.hpp"
#include "tile.hpp"
#include "tile32.hpp"

#include <algorithm>
#include <climits>

namespace ss {

int lu_panel_width(int n) { return n <= 1024 ? 32 : 8; }

bool lu_panel_width_ok(int n, int w) {
  // a panel keeps R rows per thread in one workgroup: W 32 and 16 (R 1, up to 1024 threads), 8 (R 2, 1024)
  return (w == 32 && n <= 1024) || (w == 16 && n <= 1024) || (w == 8 && n <= 2048);
}

static int panel_width(const ss_ctx *ctx, int n) {
  return lu_panel_width_ok(n, ctx->lu_width) ? ctx->lu_width : lu_panel_width(n);
}

struct LuArgs {
  double2 *M;
  long sM;
  int ldm;
  int *perm;
  long sP;
  int *zp;
  double2 *X;
  long sX;
  const long *xoff;
  int ldx;
  int n, nrhs;
  const int *skip;
  int skip_shift;
  double2 *B;  // right-hand sides (columns >= n) when non-null
  long sB;
  int ldb;
  // inverses of the W x W diagonal blocks of L and U, written by the panels ([mat][panel][L, U][W][W]);
  // null: the triangular-solve leaves substitute instead
  double2 *inv;
  long sInv;
  int f32;  // products in FP32 (see LuDesc::f32)
};

// Base pointer and leading dimension for columns starting at c of system mat: columns >= n live in the
// separate right-hand-side buffer when one is given (a column range never straddles n).
struct ColView {
  double2 *p;
  long ld;
};
__device__ __forceinline__ ColView col_view(const LuArgs &a, int mat, int c) {
  if (a.B != nullptr && c >= a.n) return ColView{a.B + (long)mat * a.sB - a.n, a.ldb};
  return ColView{a.M + (long)mat * a.sM, a.ldm};
}

__device__ __forceinline__ bool skipped(const LuArgs &a, int mat) {
  return a.skip != nullptr && a.skip[mat >> a.skip_shift] != 0;
}

// Row `row` (logical order) of system mat's solution X, at right-hand-side column 0 (columns >= n of
// the augmented matrix map to X's columns - n).
__device__ __forceinline__ double2 *x_row(const LuArgs &a, int mat, int row) {
  return a.X + (a.xoff ? a.xoff[mat] : (long)mat * a.sX) + (long)row * a.ldx - a.n;
}

static LuArgs make_args(const LuDesc &d) {
  LuArgs a;
  a.M = d.M; a.sM = d.sM; a.ldm = d.ldm; a.perm = d.perm; a.sP = d.sP;
  a.zp = d.zp; a.X = d.X; a.sX = d.sX; a.xoff = d.xoff; a.ldx = d.ldx; a.n = d.n; a.nrhs = d.nrhs;
  a.skip = d.skip; a.skip_shift = d.skip_shift;
  a.B = d.B; a.sB = d.sB; a.ldb = d.ldb;
  a.inv = nullptr; a.sInv = 0;
  a.f32 = d.f32 ? 1 : 0;
  return a;
}

__global__ void k_identity_perm(int *perm, long sP, int n) {
  int *p = perm + (long)blockIdx.y * sP;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
}

// ------------------------------------------------------------------ in-tile triangular solve

// In-tile triangular solve T x = c for the 64 columns of a staged tile, by substitution (LAPACK's
// triangular-solve arithmetic).  Each wave owns 16 columns; 4 lanes share a column and each keeps the
// rows j = part (mod 4), so a row step is a 4-lane partial dot product and two cross-lane additions.
//   rhs(i, col): element (i, col) of c (a staged tile, or generated);  tri: W x W triangle [i][j] (pitch W + 1) holding only the
//   strictly lower (!kUpper) or strictly upper (kUpper) entries, zero elsewhere;  rdiag: reciprocals of
//   the diagonal (kUpper);  kUpper: false = unit lower (forward), true = upper (backward); w <= W rows.
// Unsolved rows hold zero in x and the triangle is zero outside its part, so every row step reads the
// whole row of the triangle unconditionally.  out(i, col, x) receives every solved element (i < w).
template <int W, bool kUpper, class Rhs, class Out>
__device__ __forceinline__ void tile_trsm(Rhs &&rhs, const double2 (*tri)[W + 1], const double2 *rdiag, int w,
                                          Out &&out) {
  constexpr int NX = (W + 3) / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = wave * 16 + (lane >> 2), part = lane & 3;
  double2 x[NX];
#pragma unroll
  for (int t = 0; t < NX; ++t) x[t] = make_double2(0.0, 0.0);
#pragma unroll 1
  for (int step = 0; step < w; ++step) {
    const int i = kUpper ? w - 1 - step : step;
    double ax = 0.0, ay = 0.0;
#pragma unroll
    for (int t = 0; t < NX; ++t) {
      const int j = part + 4 * t;
      const double lx = tri[i][j].x, ly = tri[i][j].y;
      ax += lx * x[t].x - ly * x[t].y;
      ay += lx * x[t].y + ly * x[t].x;
    }
    ax += dpp_double<0xB1>(ax);
    ay += dpp_double<0xB1>(ay);
    ax += dpp_double<0x4E>(ax);
    ay += dpp_double<0x4E>(ay);
    if (part == (i & 3)) {
      const double2 ci = rhs(i, col);
      double2 v = make_double2(ci.x - ax, ci.y - ay);
      if (kUpper) v = cmul(v, ld2(rdiag[i]));
      const int ti = i >> 2;
#pragma unroll
      for (int t = 0; t < NX; ++t) {
        x[t].x = (t == ti) ? v.x : x[t].x;
        x[t].y = (t == ti) ? v.y : x[t].y;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NX; ++t) {
    const int j = part + 4 * t;
    if (j < w) out(j, col, x[t]);
  }
}

// ------------------------------------------------------------------ panel factorization

// One workgroup per system factors logical rows [c0, n) of columns [c0, c0+w).  Each thread keeps R
// rows of the panel in registers.  The column loop runs at run time (a fully unrolled loop would not
// fit the instruction cache) and the registers are only ever addressed with compile-time indices:
// after each column every row is rotated left by one position, so the current column always sits in
// position 0 and the finished entry moves to position W-1; after W rotations the order is restored.
template <int W, int R, int LB>
__global__ void __launch_bounds__(LB) k_panel(LuArgs a, int c0) {
  const int mat = blockIdx.x;
  if (skipped(a, mat)) return;
  const int tid = threadIdx.x, T = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = T >> 6;
  double2 *M = a.M + (long)mat * a.sM;
  int *perm = a.perm + (long)mat * a.sP;
  const int nrows = a.n - c0;
  const int w = min(W, nrows);
  const long ld = a.ldm;

  __shared__ int sperm[LB * R];
  // inversion of the diagonal block: its strict lower and strict upper triangles and the reciprocals of
  // its diagonal (the identity right-hand sides are generated)
  __shared__ double2 tri_l[W][W + 1], tri_u[W][W + 1];
  __shared__ double2 rdiag[W];
  __shared__ double red_v[16];
  __shared__ int red_i[16];
  __shared__ double2 rowbuf[2][W];

  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * T;
    if (lr < nrows) sperm[lr] = perm[c0 + lr];
  }
  __syncthreads();

  double2 v[R * W];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * T;
#pragma unroll
    for (int c = 0; c < W; ++c)
      v[q * W + c] = (lr < nrows && c < w) ? M[(long)sperm[lr] * ld + c0 + c] : make_double2(0.0, 0.0);
  }

  int zero_col = 0;
#pragma unroll 1
  for (int j = 0; j < w; ++j) {
    // ---- pivot search in column j (register position 0) over logical rows >= j
    double bv = -1.0;
    int bi = INT_MAX;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int lr = tid + q * T;
      if (lr >= j && lr < nrows) {
        const double t = cabs1(v[q * W]);
        if (t > bv) { bv = t; bi = lr; }
      }
    }
    // wave arg-max: DPP exchanges inside each row of 16 lanes, then across rows
    auto merge = [&](double ov, int oi) {
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    };
    merge(dpp_double<0xB1>(bv), dpp_int<0xB1>(bi));
    merge(dpp_double<0x4E>(bv), dpp_int<0x4E>(bi));
    merge(dpp_double<0x141>(bv), dpp_int<0x141>(bi));
    merge(dpp_double<0x140>(bv), dpp_int<0x140>(bi));
    merge(__shfl_xor(bv, 16), __shfl_xor(bi, 16));
    merge(__shfl_xor(bv, 32), __shfl_xor(bi, 32));
    if (lane == 0) { red_v[wave] = bv; red_i[wave] = bi; }
    __syncthreads();
    bv = red_v[0];
    bi = red_i[0];
    for (int ww = 1; ww < nw; ++ww) {
      const double ov = red_v[ww];
      const int oi = red_i[ww];
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    // no finite candidate (NaN column): keep the diagonal row so indexing stays in range
    const int piv = (bi >= j && bi < nrows) ? bi : j;
    // ---- interchange logical rows j and piv (data travels between the two owning threads)
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int lr = tid + q * T;
      if (lr == piv) {
#pragma unroll
        for (int c = 0; c < W; ++c) st2(rowbuf[0][c], v[q * W + c]);
      }
      if (lr == j && piv != j) {
#pragma unroll
        for (int c = 0; c < W; ++c) st2(rowbuf[1][c], v[q * W + c]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int lr = tid + q * T;
      if (lr == j) {
#pragma unroll
        for (int c = 0; c < W; ++c) v[q * W + c] = ld2(rowbuf[0][c]);
      } else if (lr == piv) {
#pragma unroll
        for (int c = 0; c < W; ++c) v[q * W + c] = ld2(rowbuf[1][c]);
      }
    }
    if (tid == 0 && piv != j) {
      const int t = sperm[j];
      sperm[j] = sperm[piv];
      sperm[piv] = t;
    }
    // ---- eliminate below the pivot and rotate: l = a_rj / u_jj, a_rc -= l u_jc for columns c > j
    const double2 u = ld2(rowbuf[0][0]);
    const bool live = !(u.x == 0.0 && u.y == 0.0);
    if (!live && zero_col == 0) zero_col = c0 + j + 1;
    const double2 ui = live ? crecip(u) : make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int lr = tid + q * T;
      const bool below = live && lr > j && lr < nrows;
      const double2 v0 = v[q * W];
      const double2 p = cmul(v0, ui);
      const double lx = below ? p.x : v0.x, ly = below ? p.y : v0.y;
      // multiplier: zero leaves rows on and above the pivot (and rows past the end) unchanged
      const double mx = below ? p.x : 0.0, my = below ? p.y : 0.0;
      // position c + 1 holds column j + 1 + c while c < W - 1 - j (later columns); the rest are done and
      // only move.  The bound is uniform over the workgroup: whole groups of 4 positions branch, only the
      // group that straddles it selects per position.
      const int live_pos = W - 1 - j;
#pragma unroll
      for (int g = 0; g < (W - 1 + 3) / 4; ++g) {
        if (4 * g + 4 <= live_pos) {
#pragma unroll
          for (int c = 4 * g; c < 4 * g + 4 && c < W - 1; ++c) {
            const double ux = rowbuf[0][c + 1].x, uy = rowbuf[0][c + 1].y;
            const double vx = v[q * W + c + 1].x, vy = v[q * W + c + 1].y;
            v[q * W + c].x = vx - mx * ux + my * uy;
            v[q * W + c].y = vy - mx * uy - my * ux;
          }
        } else if (4 * g >= live_pos) {
#pragma unroll
          for (int c = 4 * g; c < 4 * g + 4 && c < W - 1; ++c) v[q * W + c] = v[q * W + c + 1];
        } else {
#pragma unroll
          for (int c = 4 * g; c < 4 * g + 4 && c < W - 1; ++c) {
            const double ux = rowbuf[0][c + 1].x, uy = rowbuf[0][c + 1].y;
            const double vx = v[q * W + c + 1].x, vy = v[q * W + c + 1].y;
            const bool upd = c < live_pos;
            v[q * W + c].x = upd ? vx - mx * ux + my * uy : vx;
            v[q * W + c].y = upd ? vy - mx * uy - my * ux : vy;
          }
        }
        __builtin_amdgcn_sched_barrier(0);  // keep each group's pivot-row loads with the group (registers)
      }
      v[q * W + W - 1].x = lx;
      v[q * W + W - 1].y = ly;
    }
  }
  // complete the rotation for a narrow last panel (w < W) so position c holds column c again
#pragma unroll 1
  for (int t = w; t < W; ++t) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const double x0 = v[q * W].x, y0 = v[q * W].y;
#pragma unroll
      for (int c = 0; c < W - 1; ++c) {
        v[q * W + c].x = v[q * W + c + 1].x;
        v[q * W + c].y = v[q * W + c + 1].y;
      }
      v[q * W + W - 1].x = x0;
      v[q * W + W - 1].y = y0;
    }
  }
  __syncthreads();  // sperm final

  if (a.inv != nullptr) {
    // ---- inverses of the diagonal block's unit-lower and upper triangles (the triangular-solve leaves
    // multiply by these on the matrix cores): the in-tile substitution applied to identity columns,
    // by the first four waves (the panel is launched with at least 256 threads)
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int lr = tid + q * T;
      if (lr < W) {
#pragma unroll
        for (int c = 0; c < W; ++c) {
          const bool in = lr < w && c < w;
          st2(tri_l[lr][c], in && c < lr ? v[q * W + c] : make_double2(0.0, 0.0));
          st2(tri_u[lr][c], in && c > lr ? v[q * W + c] : make_double2(0.0, 0.0));
          if (c == lr) st2(rdiag[lr], in ? crecip(v[q * W + c]) : make_double2(0.0, 0.0));
        }
      }
    }
  }

  // ---- write the factored panel back (rows stay in their physical place) and the row map
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * T;
    if (lr < nrows) {
#pragma unroll
      for (int c = 0; c < W; ++c)
        if (c < w) M[(long)sperm[lr] * ld + c0 + c] = v[q * W + c];
      perm[c0 + lr] = sperm[lr];
    }
  }
  if (tid == 0) {
    if (c0 == 0) a.zp[mat] = zero_col;
    else if (zero_col != 0 && a.zp[mat] == 0) a.zp[mat] = zero_col;
  }
  if (a.inv != nullptr) {  // (after the write-back, so the panel's registers are free)
    __syncthreads();
    double2 *dst = a.inv + (long)mat * a.sInv + (long)(c0 / W) * 2 * W * W;
    auto eye = [&](int i, int col) { return make_double2(i == col && i < w ? 1.0 : 0.0, 0.0); };
    if (tid < 256) {
      tile_trsm<W, false>(eye, tri_l, rdiag, w, [&](int i, int col, double2 x) {
        if (col < w) dst[i * W + col] = x;
      });
      tile_trsm<W, true>(eye, tri_u, rdiag, w, [&](int i, int col, double2 x) {
        if (col < w) dst[W * W + i * W + col] = x;
      });
    }
  }
}

// ------------------------------------------------------------------ 32-column panel in quarters

// The 32-column panel (n <= 1024, one logical row per thread) in four quarters of 8 columns.  Quarter q is
// loaded, receives the updates of the 8q columns before it (first the rows of their pivots, in pivot
// order, then every row below them as one product with those rows), and is factored with its columns
// unrolled, then written back.  Every element receives the updates of a one-pass panel in the same
// column order (the compiled rounding may differ in the last bit), while a thread holds 8 complex entries
// of its row instead of 32: the workgroup needs about a quarter of a CU's register file and shares the CU
// with other work, where a whole row per thread needs all of it.  Also leaves the inverses of the
// diagonal block's triangles.
template <int LB>
__global__ void __launch_bounds__(LB) __attribute__((amdgpu_waves_per_eu(6))) k_panel32(LuArgs a, int c0) {
  constexpr int W = 32, H = 8, NQ = W / H;
  const int mat = blockIdx.x;
  if (skipped(a, mat)) return;
  const int lr = threadIdx.x, lane = lr & 63, wave = lr >> 6, nw = blockDim.x >> 6;
  double2 *M = a.M + (long)mat * a.sM;
  int *perm = a.perm + (long)mat * a.sP;
  const int nrows = a.n - c0;
  const int w = min(W, nrows);
  const long ld = a.ldm;

  __shared__ int sperm[LB];
  __shared__ double2 tri_l[W][W + 1], tri_u[W][W + 1];
  __shared__ double2 rdiag[W];
  __shared__ double red_v[LB / 64];
  __shared__ int red_i[LB / 64];
  __shared__ double2 rowbuf[2][H];
  __shared__ double2 ub[W - H][H];          // the quarter's part of the earlier pivot rows (final)
  __shared__ double2 lt[W - H][W - H + 1];  // multipliers among the earlier pivot rows

  if (lr < nrows) sperm[lr] = perm[c0 + lr];
  __syncthreads();
  int zero_col = 0;
  unsigned dead = 0;  // bit k: column k had no nonzero pivot (no update from it)
#pragma unroll 1
  for (int q = 0; q < NQ; ++q) {
    const int j0 = q * H, wh = min(H, w - j0);
    if (wh <= 0) break;  // uniform
    double2 v[H];
#pragma unroll
    for (int c = 0; c < H; ++c)
      v[c] = (lr < nrows && c < wh) ? M[(long)sperm[lr] * ld + c0 + j0 + c] : make_double2(0.0, 0.0);
    if (q > 0) {
      // ---- the earlier columns' updates.  Their multipliers among the first j0 rows, into LDS:
      for (int idx = lr; idx < j0 * j0; idx += blockDim.x) {
        const int i = idx / j0, k = idx % j0;
        if (k < i) lt[i][k] = M[(long)sperm[i] * ld + c0 + k];
      }
      __syncthreads();
      // the pivot rows themselves, in pivot order (row k is final once the columns before k are applied)
#pragma unroll 1
      for (int k = 0; k < j0; ++k) {
        const bool kl = !((dead >> k) & 1u);  // uniform
        if (lr == k) {
#pragma unroll
          for (int c = 0; c < H; ++c) st2(ub[k][c], v[c]);
        }
        __syncthreads();
        if (kl && lr > k && lr < j0) {
          const double mx = lt[lr][k].x, my = lt[lr][k].y;
#pragma unroll
          for (int c = 0; c < H; ++c) {
            const double ux = ub[k][c].x, uy = ub[k][c].y;
            const double vx = v[c].x, vy = v[c].y;
            v[c].x = vx - mx * ux + my * uy;
            v[c].y = vy - mx * uy - my * ux;
          }
        }
      }
      // every row below them: v -= L[lr, 0:j0] U[0:j0, quarter], the columns in order
      if (lr >= j0 && lr < nrows) {
        const double2 *lrow = M + (long)sperm[lr] * ld + c0;
#pragma unroll 1
        for (int kc = 0; kc < j0; kc += 4) {
          double2 lk[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) lk[e] = lrow[kc + e];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int k = kc + e;
            if (!((dead >> k) & 1u)) {  // uniform
              const double mx = lk[e].x, my = lk[e].y;
#pragma unroll
              for (int c = 0; c < H; ++c) {
                const double ux = ub[k][c].x, uy = ub[k][c].y;
                const double vx = v[c].x, vy = v[c].y;
                v[c].x = vx - mx * ux + my * uy;
                v[c].y = vy - mx * uy - my * ux;
              }
            }
          }
        }
      }
    }
    // ---- factor the quarter's columns
#pragma unroll
    for (int j = 0; j < H; ++j) {
      if (j < wh) {  // uniform
        const int p = j0 + j;  // logical row (and panel column) of this pivot
        double bv = -1.0;
        int bi = INT_MAX;
        if (lr >= p && lr < nrows) {
          bv = cabs1(v[j]);
          bi = lr;
        }
        auto merge = [&](double ov, int oi) {
          if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        };
        merge(dpp_double<0xB1>(bv), dpp_int<0xB1>(bi));
        merge(dpp_double<0x4E>(bv), dpp_int<0x4E>(bi));
        merge(dpp_double<0x141>(bv), dpp_int<0x141>(bi));
        merge(dpp_double<0x140>(bv), dpp_int<0x140>(bi));
        merge(__shfl_xor(bv, 16), __shfl_xor(bi, 16));
        merge(__shfl_xor(bv, 32), __shfl_xor(bi, 32));
        if (lane == 0) { red_v[wave] = bv; red_i[wave] = bi; }
        __syncthreads();
        bv = red_v[0];
        bi = red_i[0];
        for (int ww = 1; ww < nw; ++ww) merge(red_v[ww], red_i[ww]);
        const int piv = (bi >= p && bi < nrows) ? bi : p;  // no finite candidate: keep the diagonal row
        // interchange logical rows p and piv (the quarter's entries travel; earlier quarters' entries stay
        // in their physical rows, which the row map follows)
        if (lr == piv) {
#pragma unroll
          for (int c = 0; c < H; ++c) st2(rowbuf[0][c], v[c]);
        }
        if (lr == p && piv != p) {
#pragma unroll
          for (int c = 0; c < H; ++c) st2(rowbuf[1][c], v[c]);
        }
        __syncthreads();
        if (lr == p) {
#pragma unroll
          for (int c = 0; c < H; ++c) v[c] = ld2(rowbuf[0][c]);
        } else if (lr == piv) {
#pragma unroll
          for (int c = 0; c < H; ++c) v[c] = ld2(rowbuf[1][c]);
        }
        if (lr == 0 && piv != p) {
          const int t = sperm[p];
          sperm[p] = sperm[piv];
          sperm[piv] = t;
        }
        const double2 u = ld2(rowbuf[0][j]);
        const bool live = !(u.x == 0.0 && u.y == 0.0);
        if (!live) {
          dead |= 1u << p;
          if (zero_col == 0) zero_col = c0 + p + 1;
        }
        if (live && lr > p && lr < nrows) {
          const double2 m = cmul(v[j], crecip(u));
          v[j] = m;
#pragma unroll
          for (int c = j + 1; c < H; ++c) {
            const double ux = rowbuf[0][c].x, uy = rowbuf[0][c].y;
            const double vx = v[c].x, vy = v[c].y;
            v[c].x = vx - m.x * ux + m.y * uy;
            v[c].y = vy - m.x * uy - m.y * ux;
          }
        }
      }
    }
    __syncthreads();  // row map after this quarter
    if (lr < nrows) {
#pragma unroll
      for (int c = 0; c < H; ++c)
        if (c < wh) M[(long)sperm[lr] * ld + c0 + j0 + c] = v[c];
    }
    __syncthreads();  // the next quarter reads these multipliers (other threads' rows)
  }
  if (lr < nrows) perm[c0 + lr] = sperm[lr];
  if (lr == 0) {
    if (c0 == 0) a.zp[mat] = zero_col;
    else if (zero_col != 0 && a.zp[mat] == 0) a.zp[mat] = zero_col;
  }
  if (a.inv != nullptr) {
    // ---- inverses of the diagonal block's unit-lower and upper triangles (as in k_panel), the block read
    // back from its final rows
    if (lr < W) {
#pragma unroll 4
      for (int c = 0; c < W; ++c) {
        const bool in = lr < w && c < w;
        const double2 x = in ? M[(long)sperm[lr] * ld + c0 + c] : make_double2(0.0, 0.0);
        st2(tri_l[lr][c], c < lr ? x : make_double2(0.0, 0.0));
        st2(tri_u[lr][c], c > lr ? x : make_double2(0.0, 0.0));
        if (c == lr) st2(rdiag[lr], in ? crecip(x) : make_double2(0.0, 0.0));
      }
    }
    __syncthreads();
    double2 *dst = a.inv + (long)mat * a.sInv + (long)(c0 / W) * 2 * W * W;
    auto eye = [&](int i, int col) { return make_double2(i == col && i < w ? 1.0 : 0.0, 0.0); };
    if (lr < 256) {
      tile_trsm<W, false>(eye, tri_l, rdiag, w, [&](int i, int col, double2 x) {
        if (col < w) dst[i * W + col] = x;
      });
      tile_trsm<W, true>(eye, tri_u, rdiag, w, [&](int i, int col, double2 x) {
        if (col < w) dst[W * W + i * W + col] = x;
      });
    }
  }
}

// ------------------------------------------------------------------ products and triangular leaves

using LuTile = TileCfg<64, 64, 16, 2, 2>;
// Products of depth kLuG3Depth or more: the three-product form on the same tile (two waves per SIMD);
// shallower ones keep the four-product form at three waves, where loads and the read-modify-write of
// the result dominate.
using LuTileG3 = TileCfgG3<64, 64, 16, 2, 2>;
constexpr int kLuG3Depth = 128;
// products of at most 32 rows (the deepest levels of the triangular solves): one row of four waves
using LuTileFlat = TileCfg<32, 128, 16, 1, 4>;
// products of at most 32 columns (the depth-32 trailing updates inside a 64-column block): one column
// of four waves, no padded half tile
using LuTileNarrow = TileCfg<64, 32, 16, 4, 1>;
// half-height tile for the general products (ss_ctx::lu_tile = 1): twice the workgroups per product,
// for batches whose products are too few to fill the chip with 64 x 64 tiles
using LuTileHalf = TileCfg<32, 64, 16, 2, 2>;

// the row map into LDS (n <= kLuMaxN, 256 threads): all loads are issued before the first store
__device__ __forceinline__ void load_perm(int *sperm, const int *perm, int n) {
  constexpr int NP = kLuMaxN / 256;
  int v[NP];
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const int i = threadIdx.x + e * 256;
    v[e] = i < n ? perm[i] : 0;
  }
#pragma unroll
  for (int e = 0; e < NP; ++e) {
    const int i = threadIdx.x + e * 256;
    if (i < n) sperm[i] = v[e];
  }
  __syncthreads();
}

static_assert(LuTile::NT == 256, "load_perm assumes 256 threads");

// M[r][c] -= sum_{k in [k_lo, k_hi)} M[r][k] M[k][c] for logical rows [r_lo, r_hi), columns [c_lo, c_hi)
template <class T>
__global__ void __launch_bounds__(T::NT) SS_TILE_WAVES_OF(T) k_lu_gemm(LuArgs a, int r_lo, int r_hi, int c_lo, int c_hi,
                                                                int k_lo, int k_hi) {
  static_assert(T::NT == 256, "load_perm assumes 256 threads");
  __shared__ double lds[T::LDS_DOUBLES];
  __shared__ int sperm[kLuMaxN];
  int tile, mat;
  xcd_tile_order(tile, mat);
  if (skipped(a, mat)) return;
  double2 *M = a.M + (long)mat * a.sM;
  const ColView cv = col_view(a, mat, c_lo);
  load_perm(sperm, a.perm + (long)mat * a.sP, a.n);
  const int tc = cdiv(c_hi - c_lo, T::BN);
  const int m0 = r_lo + (tile / tc) * T::BM, n0 = c_lo + (tile % tc) * T::BN;
  Acc<T> acc;
  acc.zero();
  LdRowPerm la{M, a.ldm, sperm};
  LdRowPerm lb{cv.p, cv.ld, sperm};
  mma_loop<T>(la, lb, m0, r_hi, n0, c_hi, k_lo, k_hi, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 val) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < r_hi && gc < c_hi) {
      double2 *p = cv.p + (long)sperm[gr] * cv.ld + gc;
      *p = csub(*p, val);
    }
  });
}

// The same product with FP32 operands and accumulation on the FP32 matrix cores (the subtraction from
// the FP64 stored value is done in FP64).
using LuTile32 = TileCfg32<64, 64, 16, 2, 2>;
using LuTileFlat32 = TileCfg32<32, 128, 16, 1, 4>;
using LuTileNarrow32 = TileCfg32<64, 32, 16, 4, 1>;

template <class T>
__global__ void __launch_bounds__(T::NT) SS_TILE_WAVES k_lu_gemm32(LuArgs a, int r_lo, int r_hi, int c_lo, int c_hi,
                                                                  int k_lo, int k_hi) {
  static_assert(T::NT == 256, "load_perm assumes 256 threads");
  __shared__ float lds[T::LDS_FLOATS];
  __shared__ int sperm[kLuMaxN];
  int tile, mat;
  xcd_tile_order(tile, mat);
  if (skipped(a, mat)) return;
  double2 *M = a.M + (long)mat * a.sM;
  const ColView cv = col_view(a, mat, c_lo);
  load_perm(sperm, a.perm + (long)mat * a.sP, a.n);
  const int tc = cdiv(c_hi - c_lo, T::BN);
  const int m0 = r_lo + (tile / tc) * T::BM, n0 = c_lo + (tile % tc) * T::BN;
  Acc32<T> acc;
  acc.zero();
  LdRowPerm la{M, a.ldm, sperm};
  LdRowPerm lb{cv.p, cv.ld, sperm};
  mma_loop32<T>(la, lb, m0, r_hi, n0, c_hi, k_lo, k_hi, acc, lds);
  acc_foreach32<T>(acc, [&](int r, int c, double2 val) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < r_hi && gc < c_hi) {
      double2 *p = cv.p + (long)sperm[gr] * cv.ld + gc;
      *p = csub(*p, val);
    }
  });
}

// Leaf of the triangular solves: rows [r0, r0+w) of columns [c_lo, c_hi), in place, with the W x W
// diagonal block at logical rows/columns r0 (unit lower if !kUpper, upper otherwise).
template <int W, bool kUpper>
__global__ void __launch_bounds__(256) k_trsm_leaf(LuArgs a, int r0, int rows, int c_lo, int c_hi) {
  constexpr int CP = 64 + 1;
  __shared__ double cr[W * CP], ci[W * CP];
  __shared__ double2 tri[W][W + 1];
  __shared__ double2 rdiag[W];
  __shared__ int sp[W];
  const int mat = blockIdx.y;
  if (skipped(a, mat)) return;
  double2 *M = a.M + (long)mat * a.sM;
  const ColView cv = col_view(a, mat, c_lo);
  const int *perm = a.perm + (long)mat * a.sP;
  const int w = min(min(W, rows), a.n - r0);
  const int c0 = c_lo + blockIdx.x * 64;
  if (threadIdx.x < W) sp[threadIdx.x] = threadIdx.x < w ? perm[r0 + threadIdx.x] : 0;
  __syncthreads();
  {
    // every global load is issued before the first LDS store: the loads overlap instead of each paying
    // the full memory latency in turn
    constexpr int NV = (W * 64 + 255) / 256, NTR = (W * W + 255) / 256;
    double2 v[NV], tv[NTR];
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int idx = threadIdx.x + e * 256, i = idx / 64, c = idx % 64;
      v[e] = (idx < W * 64 && i < w && c0 + c < c_hi) ? cv.p[(long)sp[i] * cv.ld + c0 + c] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int e = 0; e < NTR; ++e) {
      const int idx = threadIdx.x + e * 256, i = idx / W, j = idx % W;
      tv[e] = (idx < W * W && i < w && j < w && (kUpper ? j >= i : j < i)) ? M[(long)sp[i] * a.ldm + r0 + j]
                                                                          : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      const int idx = threadIdx.x + e * 256, i = idx / 64, c = idx % 64;
      if (idx < W * 64) {
        cr[i * CP + c] = v[e].x;
        ci[i * CP + c] = v[e].y;
      }
    }
#pragma unroll
    for (int e = 0; e < NTR; ++e) {
      const int idx = threadIdx.x + e * 256, i = idx / W, j = idx % W;
      if (idx < W * W) {
        if (kUpper && i == j) {  // the diagonal leaves the triangle for its scaled reciprocal
          st2(rdiag[i], i < w ? crecip(tv[e]) : make_double2(0.0, 0.0));
          st2(tri[i][j], make_double2(0.0, 0.0));
        } else {
          st2(tri[i][j], tv[e]);
        }
      }
    }
  }
  __syncthreads();
  tile_trsm<W, kUpper>([&](int i, int col) { return make_double2(cr[i * CP + col], ci[i * CP + col]); }, tri, rdiag, w,
                       [&](int i, int col, double2 v) {
    if (c0 + col < c_hi) cv.p[(long)sp[i] * cv.ld + c0 + col] = v;
  });
}

// Leaf of the triangular solves on the matrix cores: rows [r0, r0+w) of columns [c_lo, c_hi) are
// replaced by T^{-1} times themselves, with T^{-1} the inverse of the W x W diagonal block at logical
// row/column r0 (unit lower if !kUpper, upper otherwise) kept by its panel; r0 is a multiple of W.
// Every workgroup reads all w rows of its columns before it writes them, so the update is in place.
template <bool kUpper, class T>
__global__ void __launch_bounds__(T::NT) SS_TILE_WAVES k_lu_leaf(LuArgs a, int W, int r0, int rows, int c_lo,
                                                                  int c_hi, int to_x) {
  static_assert(T::BM == 32 && T::NT >= T::BM, "leaf tile: up to 32 rows");
  __shared__ double lds[T::LDS_DOUBLES];
  __shared__ int sp[T::BM];
  const int mat = blockIdx.y;
  if (skipped(a, mat)) return;
  const ColView cv = col_view(a, mat, c_lo);
  const int w = min(min(W, rows), a.n - r0);
  if (threadIdx.x < T::BM) sp[threadIdx.x] = threadIdx.x < w ? a.perm[(long)mat * a.sP + r0 + threadIdx.x] : 0;
  __syncthreads();
  const int n0 = c_lo + blockIdx.x * T::BN;
  const double2 *inv = a.inv + (long)mat * a.sInv + ((long)(r0 / W) * 2 + (kUpper ? 1 : 0)) * W * W;
  Acc<T> acc;
  acc.zero();
  LdRow la{inv, W};
  LdRowPerm lb{cv.p, cv.ld, sp};
  mma_loop<T>(la, lb, 0, w, n0, c_hi, 0, w, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 val) {
    const int gc = n0 + c;
    if (r < w && gc < c_hi) {
      cv.p[(long)sp[r] * cv.ld + gc] = val;
      if (to_x) x_row(a, mat, r0 + r)[gc] = val;  // final rows of the upper solve: also the solution
    }
  });
}

// 64-row leaf of the triangular solves from two 32-column panels, in place, for 32 columns:
//   unit lower:  X1 = A^{-1} C1,  X2 = B^{-1} (C2 - L21 X1)
//   upper:       X2 = B^{-1} C2,  X1 = A^{-1} (C1 - U12 X2)
// with A^{-1}, B^{-1} the panels' inverses of their diagonal blocks (rows r0 and r0 + 32) and the
// coupling block read from the factors.  With p0 >= 0 the block first takes the update from the
// 64-row block already solved at rows p0 (C -= F X_p, F the factors' block at rows r0, columns p0),
// so the 64-deep product between two such leaves needs no launch (and no pass over C) of its own.
// Each 32 x 32 x 32 product stages both operands in LDS once (four waves, one 16 x 16 block each, on
// the matrix cores); partial results stay in the accumulators or in LDS.  Requires W = 32, r0 + 64 <= n.
using LuTileLeaf = TileCfgG3<32, 32, 32, 2, 2>;

template <bool kUpper>
__global__ void __launch_bounds__(LuTileLeaf::NT) SS_TILE_WAVES k_lu_leaf2x(LuArgs a, int r0, int p0, int c_lo,
                                                                             int c_hi, int to_x) {
  using T = LuTileLeaf;
  constexpr int H = 32;
  static_assert(T::BM == H && T::BK == H && H * H % T::NT == 0 && H * T::BN % T::NT == 0, "leaf tile");
  __shared__ double lds[T::LDS_DOUBLES];
  __shared__ int sp[2 * H], spp[2 * H];
  const int mat = blockIdx.y;
  if (skipped(a, mat)) return;
  const ColView cv = col_view(a, mat, c_lo);
  const double2 *M = a.M + (long)mat * a.sM;
  const int tid = threadIdx.x;
  const int *perm = a.perm + (long)mat * a.sP;
  if (tid < 2 * H) {
    sp[tid] = perm[r0 + tid];
    if (p0 >= 0) spp[tid] = perm[p0 + tid];
  }
  __syncthreads();
  const int n0 = c_lo + blockIdx.x * T::BN;
  const double2 *inv = a.inv + (long)mat * a.sInv;
  const int kind = kUpper ? 1 : 0;
  const int f = kUpper ? H : 0, g = kUpper ? 0 : H;  // the half solved first, and the other
  const double2 *inv_f = inv + ((long)(r0 + f) / H * 2 + kind) * H * H;
  const double2 *inv_g = inv + ((long)(r0 + g) / H * 2 + kind) * H * H;
  Lds<T> L(lds);
  constexpr int E = H * H / T::NT;         // elements per thread of a 32 x 32 operand
  constexpr int EB = H * T::BN / T::NT;   // elements per thread of 32 right-hand-side rows
  // A operand (r, k) -> planes [k][r];  B operand (k, c) -> planes [k][c].  Every operand that does not
  // depend on this workgroup's results is fetched into registers one stage ahead, while the matrix cores
  // work on the current stage, and stored to LDS after the next barrier.
  double2 pa[E], pb[EB], pc[4 * T::FM * T::FN];
  auto fetch_a = [&](auto load) {
#pragma unroll
    for (int e = 0; e < E; ++e) pa[e] = load((tid + e * T::NT) / H, (tid + e * T::NT) % H);
  };
  auto put_a = [&]() {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int r = (tid + e * T::NT) / H, k = (tid + e * T::NT) % H;
      L.ar[k * T::PA + r] = pa[e].x;
      L.ai[k * T::PA + r] = pa[e].y;
    }
  };
  auto fetch_b_rows = [&](const int *rowmap) {  // 32 right-hand-side rows (columns n0 .. n0 + BN - 1)
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int k = (tid + e * T::NT) / T::BN, c = (tid + e * T::NT) % T::BN;
      pb[e] = n0 + c < c_hi ? cv.p[(long)rowmap[k] * cv.ld + n0 + c] : make_double2(0.0, 0.0);
    }
  };
  auto put_b = [&]() {
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int k = (tid + e * T::NT) / T::BN, c = (tid + e * T::NT) % T::BN;
      L.br[k * T::PB + c] = pb[e].x;
      L.bi[k * T::PB + c] = pb[e].y;
    }
  };
  // C of a half (its right-hand-side rows), in the accumulator's element order
  auto fetch_c = [&](int half) {
    Acc<T> shape;  // only its element positions are used
    shape.zero();
    int i = 0;
    acc_foreach<T>(shape, [&](int r, int c, double2) {
      pc[i++] = n0 + c < c_hi ? cv.p[(long)sp[half + r] * cv.ld + n0 + c] : make_double2(0.0, 0.0);
    });
  };
  // B planes <- C - acc
  auto publish_diff = [&](const Acc<T> &acc) {
    int i = 0;
    acc_foreach<T>(acc, [&](int r, int c, double2 x) {
      L.br[r * T::PB + c] = pc[i].x - x.x;
      L.bi[r * T::PB + c] = pc[i].y - x.y;
      ++i;
    });
  };
  auto coupling = [&](int half, int col0) {  // factors' block at rows r0 + half, columns col0
    return [=](int r, int k) { return M[(long)sp[half + r] * a.ldm + col0 + k]; };
  };
  auto inv_of = [&](const double2 *iv) {
    return [=](int r, int k) { return iv[r * H + k]; };
  };
  Acc<T> acc_f, acc_g;
  acc_f.zero();
  acc_g.zero();
  if (p0 >= 0) {  // F X_p for both halves, in two 32-deep steps
    fetch_b_rows(spp);
    fetch_a(coupling(f, p0));
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      put_b();
      put_a();
      __syncthreads();
      fetch_a(coupling(g, p0 + kk * H));
      mma_stage<T>(L, acc_f);
      __syncthreads();
      put_a();
      __syncthreads();
      if (kk == 0) {
        fetch_b_rows(spp + H);
        fetch_a(coupling(f, p0 + H));
      } else {
        fetch_c(f);
        fetch_a(inv_of(inv_f));
      }
      mma_stage<T>(L, acc_g);
      __syncthreads();
    }
  } else {
    fetch_c(f);
    fetch_a(inv_of(inv_f));
  }
  // ---- X_f = inv_f (C_f - acc_f)
  publish_diff(acc_f);
  put_a();
  __syncthreads();
  fetch_a(coupling(g, r0 + f));
  Acc<T> acc;
  acc.zero();
  mma_stage<T>(L, acc);
  __syncthreads();  // operands consumed
  acc_foreach<T>(acc, [&](int r, int c, double2 x) {
    if (n0 + c < c_hi) {
      cv.p[(long)sp[f + r] * cv.ld + n0 + c] = x;
      if (to_x) x_row(a, mat, r0 + f + r)[n0 + c] = x;
    }
    L.br[r * T::PB + c] = x.x;  // X_f is the next product's right operand
    L.bi[r * T::PB + c] = x.y;
  });
  // ---- Y = C_g - acc_g - coupling X_f   (coupling: L21 below the first half, U12 right of the second)
  put_a();
  __syncthreads();
  fetch_c(g);
  fetch_a(inv_of(inv_g));
  mma_stage<T>(L, acc_g);
  __syncthreads();
  publish_diff(acc_g);
  // ---- X_g = inv_g Y
  put_a();
  __syncthreads();
  acc.zero();
  mma_stage<T>(L, acc);
  acc_foreach<T>(acc, [&](int r, int c, double2 x) {
    if (n0 + c < c_hi) {
      cv.p[(long)sp[g + r] * cv.ld + n0 + c] = x;
      if (to_x) x_row(a, mat, r0 + g + r)[n0 + c] = x;
    }
  });
}

// X[r][c] = M[perm[r]][n + c]: the solution rows in natural order
__global__ void k_copy_out(LuArgs a) {
  const int mat = blockIdx.y;
  if (skipped(a, mat)) return;
  const ColView cv = col_view(a, mat, a.n);
  const int *perm = a.perm + (long)mat * a.sP;
  double2 *X = a.X + (a.xoff ? a.xoff[mat] : (long)mat * a.sX);
  const long total = (long)a.n * a.nrhs;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int r = idx / a.nrhs, c = idx % a.nrhs;
    X[(long)r * a.ldx + c] = cv.p[(long)perm[r] * cv.ld + a.n + c];
  }
}

// ------------------------------------------------------------------ narrow solves with kept factors
//
// The refinement applies kept factors to a few right-hand-side columns (m, typically 32).  The recursive
// solve would issue about two launches per 32 rows and triangle, each far too small to fill the chip.
// Here a diagonal block of up to kTrsmBlock rows is solved by ONE launch: a workgroup owns one system
// and NarrowTile::BN columns and walks the block in panels of 32 rows (the rows of the right-hand sides
// minus the product with the block's already solved rows, a matrix-core product whose depth grows with
// the panel, then the 32 x 32 triangle by substitution, in place); the products between blocks are the
// factorization's own batched products, so a triangle of order n takes n / kTrsmBlock block launches and
// one fewer products.
using NarrowTile = TileCfg<32, 32, 32, 2, 2>;
constexpr int kTrsmBlock = 256;

// the staged right-hand sides of k_trsm_block as the right operand of a product: element (k, c)
struct LdLds {
  const double *re, *im;
  int pitch;
  static constexpr bool kFastSecond = true;
  __device__ __forceinline__ double2 operator()(int k, int c) const {
    return make_double2(re[k * pitch + c], im[k * pitch + c]);
  }
};

template <bool kUpper>
__global__ void __launch_bounds__(NarrowTile::NT) k_trsm_block(LuArgs a, int r0, int rows, int c_lo, int c_hi) {
  using T = NarrowTile;
  constexpr int P = 32;   // panel rows
  constexpr int CP = 33;  // LDS pitch of the staged right-hand sides (32 columns)
  __shared__ double lds[T::LDS_DOUBLES];
  __shared__ double cr[P * CP], ci[P * CP];
  __shared__ double2 tri[P][P + 1];
  __shared__ double2 rdiag[P];
  __shared__ int sperm[kTrsmBlock];
  const int mat = blockIdx.y;
  if (skipped(a, mat)) return;
  const int n = a.n, rb = min(rows, n - r0);
  const int c0 = c_lo + blockIdx.x * T::BN, cw = min(T::BN, c_hi - c0);
  double2 *M = a.M + (long)mat * a.sM;
  const ColView cv = col_view(a, mat, c_lo);  // right-hand sides: element (physical row, column c >= n)
  const int *perm = a.perm + (long)mat * a.sP;
  for (int i = threadIdx.x; i < rb; i += T::NT) sperm[i] = perm[r0 + i];  // block-local rows
  __syncthreads();
  const int npanel = cdiv(rb, P);
  // operands in block-local coordinates: the factor's rows r0 + r, columns r0 + k; the right-hand sides'
  // rows r0 + k (physical through the row map), columns c0 + c
  LdRowPerm la{M + r0, a.ldm, sperm};
  LdRowPerm lb{cv.p + c0, cv.ld, sperm};
  for (int q = 0; q < npanel; ++q) {
    const int pidx = kUpper ? npanel - 1 - q : q;
    const int p0 = pidx * P, w = min(P, rb - p0);
    Acc<T> acc;
    acc.zero();
    if (kUpper) mma_loop<T>(la, lb, p0, rb, 0, cw, p0 + P, rb, acc, lds);  // U[panel][p0+P : rb] X
    else mma_loop<T>(la, lb, p0, rb, 0, cw, 0, p0, acc, lds);              // L[panel][0 : p0] Y
    acc_foreach<T>(acc, [&](int r, int c, double2 v) {
      double2 b = make_double2(0.0, 0.0);
      if (r < w && c < cw) b = csub(cv.p[(long)sperm[p0 + r] * cv.ld + c0 + c], v);
      cr[r * CP + c] = b.x;
      ci[r * CP + c] = b.y;
    });
    if (a.inv != nullptr) {
      // the kept inverse of the panel's diagonal block times the staged rows, on the matrix cores
      __syncthreads();
      const double2 *tinv = a.inv + (long)mat * a.sInv + ((long)((r0 + p0) / P) * 2 + (kUpper ? 1 : 0)) * P * P;
      Acc<T> acc2;
      acc2.zero();
      mma_loop<T>(LdRow{tinv, P}, LdLds{cr, ci, CP}, 0, w, 0, cw, 0, w, acc2, lds);
      acc_foreach<T>(acc2, [&](int r, int c, double2 x) {
        if (r < w && c < cw) cv.p[(long)sperm[p0 + r] * cv.ld + c0 + c] = x;
      });
    } else {
      for (int idx = threadIdx.x; idx < P * P; idx += T::NT) {
        const int i = idx / P, j = idx % P;
        const bool in = i < w && j < w && (kUpper ? j > i : j < i);
        st2(tri[i][j], in ? M[(long)sperm[p0 + i] * a.ldm + r0 + p0 + j] : make_double2(0.0, 0.0));
        if (kUpper && j == i)
          st2(rdiag[i], i < w ? crecip(M[(long)sperm[p0 + i] * a.ldm + r0 + p0 + i]) : make_double2(0.0, 0.0));
      }
      __syncthreads();
      tile_trsm<P, kUpper>(
          [&](int i, int col) { return col < P ? make_double2(cr[i * CP + col], ci[i * CP + col]) : make_double2(0.0, 0.0); },
          tri, rdiag, w, [&](int i, int col, double2 x) {
            if (col < cw) cv.p[(long)sperm[p0 + i] * cv.ld + c0 + col] = x;
          });
    }
    __syncthreads();  // the panel's rows are stored before the next panel's product reads them
  }
}

// ------------------------------------------------------------------ driver

template <int W, int R, int LB>
struct LuRun {
  ss_ctx *ctx;
  const LuDesc &d;
  LuArgs a;

  // split point: a multiple of W strictly inside (lo, hi)
  int mid(int lo, int hi) const { return lo + std::max(W, ((hi - lo) / 2 + W - 1) / W * W); }

  void gemm(int r_lo, int r_hi, int c_lo, int c_hi, int k_lo, int k_hi) {
    if (r_lo >= r_hi || c_lo >= c_hi || k_lo >= k_hi) return;
    const double m_ = r_hi - r_lo, n_ = c_hi - c_lo, k_ = k_hi - k_lo;
    KernelScope ks_(ctx, "lu_gemm", 8.0 * m_ * n_ * k_ * d.nmat, 16.0 * (m_ * k_ + k_ * n_ + 2.0 * m_ * n_) * d.nmat);
    if (a.f32) {
      if (r_hi - r_lo <= LuTileFlat32::BM && c_hi - c_lo > LuTileFlat32::BN / 2) {
        const int tiles = cdiv(c_hi - c_lo, LuTileFlat32::BN);
        hipLaunchKernelGGL(k_lu_gemm32<LuTileFlat32>, dim3(tiles, d.nmat), dim3(LuTileFlat32::NT), 0, ctx->stream, a,
                           r_lo, r_hi, c_lo, c_hi, k_lo, k_hi);
      } else if (c_hi - c_lo <= LuTileNarrow32::BN && r_hi - r_lo > LuTileNarrow32::BM) {
        const int tiles = cdiv(r_hi - r_lo, LuTileNarrow32::BM);
        hipLaunchKernelGGL(k_lu_gemm32<LuTileNarrow32>, dim3(tiles, d.nmat), dim3(LuTileNarrow32::NT), 0, ctx->stream,
                           a, r_lo, r_hi, c_lo, c_hi, k_lo, k_hi);
      } else {
        const int tiles = cdiv(r_hi - r_lo, LuTile32::BM) * cdiv(c_hi - c_lo, LuTile32::BN);
        hipLaunchKernelGGL(k_lu_gemm32<LuTile32>, dim3(tiles, d.nmat), dim3(LuTile32::NT), 0, ctx->stream, a, r_lo,
                           r_hi, c_lo, c_hi, k_lo, k_hi);
      }
      return;
    }
    if (r_hi - r_lo <= LuTileFlat::BM && c_hi - c_lo > LuTileFlat::BN / 2) {
      const int tiles = cdiv(c_hi - c_lo, LuTileFlat::BN);
      hipLaunchKernelGGL(k_lu_gemm<LuTileFlat>, dim3(tiles, d.nmat), dim3(LuTileFlat::NT), 0, ctx->stream, a, r_lo,
                         r_hi, c_lo, c_hi, k_lo, k_hi);
    } else if (c_hi - c_lo <= LuTileNarrow::BN && r_hi - r_lo > LuTileNarrow::BM) {
      const int tiles = cdiv(r_hi - r_lo, LuTileNarrow::BM);
      hipLaunchKernelGGL(k_lu_gemm<LuTileNarrow>, dim3(tiles, d.nmat), dim3(LuTileNarrow::NT), 0, ctx->stream, a,
                         r_lo, r_hi, c_lo, c_hi, k_lo, k_hi);
    } else if (ctx->lu_tile == 1) {
      const int tiles = cdiv(r_hi - r_lo, LuTileHalf::BM) * cdiv(c_hi - c_lo, LuTileHalf::BN);
      hipLaunchKernelGGL(k_lu_gemm<LuTileHalf>, dim3(tiles, d.nmat), dim3(LuTileHalf::NT), 0, ctx->stream, a, r_lo,
                         r_hi, c_lo, c_hi, k_lo, k_hi);
    } else if (k_hi - k_lo >= kLuG3Depth) {
      const int tiles = cdiv(r_hi - r_lo, LuTileG3::BM) * cdiv(c_hi - c_lo, LuTileG3::BN);
      hipLaunchKernelGGL(k_lu_gemm<LuTileG3>, dim3(tiles, d.nmat), dim3(LuTileG3::NT), 0, ctx->stream, a, r_lo,
                         r_hi, c_lo, c_hi, k_lo, k_hi);
    } else {
      const int tiles = cdiv(r_hi - r_lo, LuTile::BM) * cdiv(c_hi - c_lo, LuTile::BN);
      hipLaunchKernelGGL(k_lu_gemm<LuTile>, dim3(tiles, d.nmat), dim3(LuTile::NT), 0, ctx->stream, a, r_lo, r_hi,
                         c_lo, c_hi, k_lo, k_hi);
    }
  }
  // triangular-solve leaves cover up to TL rows
  static constexpr int TL = W;
  // set during the upper right-hand-side solve when its leaves also write the solution X (no copy)
  int to_x = 0;
  template <bool kUpper>
  void leaf(int r0, int rows, int c_lo, int c_hi) {
    if (c_lo >= c_hi) return;
    KernelScope ks_(ctx, "trsm");
    if (a.inv != nullptr && c_hi - c_lo <= LuTileLeaf::BN)  // a narrow range: no padded 128-wide tile
      hipLaunchKernelGGL((k_lu_leaf<kUpper, LuTileLeaf>), dim3(cdiv(c_hi - c_lo, LuTileLeaf::BN), d.nmat),
                         dim3(LuTileLeaf::NT), 0, ctx->stream, a, W, r0, rows, c_lo, c_hi, kUpper ? to_x : 0);
    else if (a.inv != nullptr)
      hipLaunchKernelGGL((k_lu_leaf<kUpper, LuTileFlat>), dim3(cdiv(c_hi - c_lo, LuTileFlat::BN), d.nmat),
                         dim3(LuTileFlat::NT), 0, ctx->stream, a, W, r0, rows, c_lo, c_hi, kUpper ? to_x : 0);
    else
      hipLaunchKernelGGL((k_trsm_leaf<TL, kUpper>), dim3(cdiv(c_hi - c_lo, 64), d.nmat), dim3(256), 0, ctx->stream,
                         a, r0, rows, c_lo, c_hi);
  }
  // the fused 64-row leaf at rows r0 (p0 >= 0: with the update from the solved block at rows p0)
  void leaf2x(bool upper, int r0, int p0, int c_lo, int c_hi) {
    if (c_lo >= c_hi) return;
    KernelScope ks_(ctx, "trsm");
    const dim3 grid(cdiv(c_hi - c_lo, LuTileLeaf::BN), d.nmat);
    if (upper)
      hipLaunchKernelGGL(k_lu_leaf2x<true>, grid, dim3(LuTileLeaf::NT), 0, ctx->stream, a, r0, p0, c_lo, c_hi,
                         to_x);
    else
      hipLaunchKernelGGL(k_lu_leaf2x<false>, grid, dim3(LuTileLeaf::NT), 0, ctx->stream, a, r0, p0, c_lo, c_hi, 0);
  }
  bool fused_ok(int lo, int hi, int rows) const {
    return W == 32 && a.inv != nullptr && hi - lo == rows && lo % 32 == 0;
  }
  // a full 64-row block of two 32-column panels: one fused leaf; a full 128-row block: two fused leaves,
  // the second also applying the 64-deep update from the first
  bool leaf64(bool upper, int lo, int hi, int c_lo, int c_hi) {
    if (fused_ok(lo, hi, 128)) {
      if (upper) {
        leaf2x(true, lo + 64, -1, c_lo, c_hi);
        leaf2x(true, lo, lo + 64, c_lo, c_hi);
      } else {
        leaf2x(false, lo, -1, c_lo, c_hi);
        leaf2x(false, lo + 64, lo, c_lo, c_hi);
      }
      return true;
    }
    if (!fused_ok(lo, hi, 64)) return false;
    leaf2x(upper, lo, -1, c_lo, c_hi);
    return true;
  }
  // unit lower solve on rows [lo, hi) of columns [c_lo, c_hi)
  void trsm_lower(int lo, int hi, int c_lo, int c_hi) {
    if (hi - lo <= TL) return leaf<false>(lo, hi - lo, c_lo, c_hi);
    if (leaf64(false, lo, hi, c_lo, c_hi)) return;
    const int m = mid(lo, hi);
    trsm_lower(lo, m, c_lo, c_hi);
    gemm(m, hi, c_lo, c_hi, lo, m);
    trsm_lower(m, hi, c_lo, c_hi);
  }
  // upper solve on rows [lo, hi) of columns [c_lo, c_hi)
  void trsm_upper(int lo, int hi, int c_lo, int c_hi) {
    if (hi - lo <= TL) return leaf<true>(lo, hi - lo, c_lo, c_hi);
    if (leaf64(true, lo, hi, c_lo, c_hi)) return;
    const int m = mid(lo, hi);
    trsm_upper(m, hi, c_lo, c_hi);
    gemm(lo, m, c_lo, c_hi, m, hi);
    trsm_upper(lo, m, c_lo, c_hi);
  }
  void factor(int c0, int c1) {
    if (c1 - c0 <= W) {
      const int rows = cdiv(d.n - c0, R);
      // at least four waves: they invert the panel's diagonal block at the end
      const int threads = std::min(LB, std::max(256, cdiv(rows, 64) * 64));
      KernelScope ks_(ctx, "panel");
      if constexpr (W == 32 && R == 1) {
        if (threads <= 512)
          hipLaunchKernelGGL(k_panel32<512>, dim3(d.nmat), dim3(threads), 0, ctx->stream, a, c0);
        else
          hipLaunchKernelGGL(k_panel32<1024>, dim3(d.nmat), dim3(threads), 0, ctx->stream, a, c0);
      } else {
        hipLaunchKernelGGL((k_panel<W, R, LB>), dim3(d.nmat), dim3(threads), 0, ctx->stream, a, c0);
      }
      return;
    }
    const int cm = mid(c0, c1);
    factor(c0, cm);
    trsm_lower(c0, cm, cm, c1);
    gemm(cm, d.n, cm, c1, c0, cm);
    factor(cm, c1);
  }
  // the two triangles for a few right-hand-side columns: blocks of kTrsmBlock rows by k_trsm_block,
  // the products between blocks by gemm, then the solution rows to X in natural order
  void narrow(bool upper, int lo, int hi) {
    const int c_lo = d.n, c_hi = d.n + d.nrhs;
    if (hi - lo <= kTrsmBlock) {
      const dim3 grid(cdiv(c_hi - c_lo, NarrowTile::BN), d.nmat);
      KernelScope ks_(ctx, "trsm");
      if (upper) hipLaunchKernelGGL(k_trsm_block<true>, grid, dim3(NarrowTile::NT), 0, ctx->stream, a, lo, hi - lo, c_lo, c_hi);
      else hipLaunchKernelGGL(k_trsm_block<false>, grid, dim3(NarrowTile::NT), 0, ctx->stream, a, lo, hi - lo, c_lo, c_hi);
      return;
    }
    const int m = lo + std::max(kTrsmBlock, ((hi - lo) / 2 + kTrsmBlock - 1) / kTrsmBlock * kTrsmBlock);
    if (!upper) {
      narrow(false, lo, m);
      gemm(m, hi, c_lo, c_hi, lo, m);
      narrow(false, m, hi);
    } else {
      narrow(true, m, hi);
      gemm(lo, m, c_lo, c_hi, m, hi);
      narrow(true, lo, m);
    }
  }
  ss_status apply_narrow() {
    narrow(false, 0, d.n);
    narrow(true, 0, d.n);
    const long total = (long)d.n * d.nrhs;
    const int blocks = (int)std::min<long>((total + 255) / 256, 256);
    hipLaunchKernelGGL(k_copy_out, dim3(blocks, d.nmat), dim3(256), 0, ctx->stream, a);
    return check_launch(ctx, "lu_apply");
  }
  ss_status run(bool do_factor = true) {
    if (do_factor) factor(0, d.n);
    if (d.nrhs > 0) {
      trsm_lower(0, d.n, d.n, d.n + d.nrhs);
      // with matrix-core leaves every row of the upper solve is final when its leaf writes it: the
      // leaves also write X, and no copy pass is needed
      to_x = a.inv != nullptr ? 1 : 0;
      trsm_upper(0, d.n, d.n, d.n + d.nrhs);
      to_x = 0;
      if (a.inv == nullptr) {
        const long total = (long)d.n * d.nrhs;
        const int blocks = (int)std::min<long>((total + 255) / 256, 256);
        hipLaunchKernelGGL(k_copy_out, dim3(blocks, d.nmat), dim3(256), 0, ctx->stream, a);
      }
    }
    return check_launch(ctx, "lu_solve");
  }
};

int lu_width_of(ss_ctx *ctx, int n) { return panel_width(ctx, n); }
long lu_inverse_elems(int n, int w) { return (long)cdiv(n, w) * 2 * w * w; }

ss_status lu_solve(ss_ctx *ctx, const LuDesc &d) {
  if (d.nmat <= 0) return SS_OK;
  if (d.n < 1 || d.n > kLuMaxN) return fail(ctx, SS_ERR_UNSUPPORTED, "lu_solve: order out of range");
  const int W = panel_width(ctx, d.n);
  LuArgs a = make_args(d);
  // the panels keep the inverses of their diagonal blocks for the triangular-solve leaves
  a.sInv = (long)cdiv(d.n, W) * 2 * W * W;
  SS_TRY(workspace(ctx, kSlotLuInv, sizeof(double2) * (size_t)d.nmat * a.sInv, (void **)&a.inv));
  if (W == 32) return LuRun<32, 1, 1024>{ctx, d, a}.run();
  if (W == 16) return LuRun<16, 1, 1024>{ctx, d, a}.run();
  return LuRun<8, 2, 1024>{ctx, d, a}.run();
}

ss_status lu_apply(ss_ctx *ctx, const LuDesc &d) {
  if (d.nmat <= 0) return SS_OK;
  if (d.n < 1 || d.n > kLuMaxN) return fail(ctx, SS_ERR_UNSUPPORTED, "lu_apply: order out of range");
  const int W = panel_width(ctx, d.n);
  if (d.nrhs <= 2 * NarrowTile::BN) {  // a few columns: diagonal blocks of kTrsmBlock rows, one launch each
    if (W == 32) {
      LuArgs a = make_args(d);
      if (d.inv != nullptr) {  // kept inverses of the 32 x 32 diagonal blocks
        a.inv = const_cast<double2 *>(d.inv);
        a.sInv = d.sInv;
      }
      return LuRun<32, 1, 1024>{ctx, d, a}.apply_narrow();
    }
    if (W == 16) return LuRun<16, 1, 1024>{ctx, d, make_args(d)}.apply_narrow();
    return LuRun<8, 2, 1024>{ctx, d, make_args(d)}.apply_narrow();
  }
  if (W == 32) return LuRun<32, 1, 1024>{ctx, d, make_args(d)}.run(false);
  if (W == 16) return LuRun<16, 1, 1024>{ctx, d, make_args(d)}.run(false);
  return LuRun<8, 2, 1024>{ctx, d, make_args(d)}.run(false);
}

// rows of every system in the factorization's logical order: dst[i] = src[perm[i]] (n x n, ld n)
__global__ void k_gather_rows(const double2 *src, double2 *dst, const int *perm, int n) {
  const long base = (long)blockIdx.y * n * n;
  const int *p = perm + (long)blockIdx.y * n;
  const long total = (long)n * n;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int r = idx / n, c = idx % n;
    dst[base + idx] = src[base + (long)p[r] * n + c];
  }
}

ss_status lu_factor_dense(ss_ctx *ctx, int nmat, int n, double2 *A, int *perm, int *info) {
  if (nmat <= 0) return SS_OK;
  if (n < 1 || n > kLuMaxN) return fail(ctx, SS_ERR_UNSUPPORTED, "lu_factor: order out of range");
  int *zp = info;
  if (!zp) SS_TRY(workspace(ctx, kSlotZp, sizeof(int) * (size_t)nmat, (void **)&zp));
  LuDesc d;
  d.nmat = nmat;
  d.n = n;
  d.nrhs = 0;
  d.M = A;
  d.sM = (long)n * n;
  d.ldm = n;
  d.perm = perm;
  d.sP = n;
  d.zp = zp;
  SS_TRY(lu_identity_perm(ctx, d));
  SS_TRY(lu_solve(ctx, d));
  void *tmp;
  const size_t bytes = sizeof(double2) * (size_t)nmat * n * n;
  SS_TRY(workspace(ctx, kSlotM, bytes, &tmp));
  const int blocks = (int)std::min<long>(((long)n * n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_gather_rows, dim3(blocks, nmat), dim3(256), 0, ctx->stream, A, (double2 *)tmp, perm, n);
  if (hipMemcpyAsync(A, tmp, bytes, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess)
    return fail(ctx, SS_ERR_DEVICE, "lu_factor: copy failed");
  return check_launch(ctx, "lu_factor");
}

ss_status lu_identity_perm(ss_ctx *ctx, const LuDesc &d) {
  if (d.nmat <= 0) return SS_OK;
  hipLaunchKernelGGL(k_identity_perm, dim3(cdiv(d.n, 256), d.nmat), dim3(256), 0, ctx->stream, d.perm, d.sP,
                     d.n);
  return check_launch(ctx, "lu_identity_perm");
}

}  // namespace ss
