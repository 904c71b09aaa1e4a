// Batched dense complex LU with partial pivoting and the two triangular solves, on gfx950.
//
// Left-looking (Crout) blocked factorization of the augmented matrix [D | RHS], panel width W:
//   for each panel p (columns [r0, r0+w)):
//     1. panel update   A[r0:, panel] -= L[r0:, :r0] U[:r0, panel]                (MFMA tiles)
//     2. panel factor   pivot search (|Re|+|Im|, lowest row on ties, as LAPACK), row
//                       interchange in the logical row map, scaling and rank-1 updates, all in
//                       registers of one workgroup per system; inverts the W x W diagonal blocks
//                       of L and U for the later tile solves
//     3. row block      U[panel rows, r0+w:] = L11^{-1} (A[panel rows, r0+w:] - L[rows, :r0] U[:r0, r0+w:])
//                       over the remaining D columns and all RHS columns (MFMA tiles, then the
//                       inverted L11 applied inside the tile)
//   back substitution, block rows from the bottom:
//     X[rows] = U11^{-1} (Y[rows] - U[rows, r0+w:n] X[r0+w:n])                    (MFMA tiles)
// Rows are never moved in memory; `perm` maps logical rows to physical rows.
#include "lu.hpp"
#include "tile.hpp"

#include <climits>
#include <utility>

namespace ss {

int lu_panel_width(int n) { return n <= 512 ? 32 : (n <= 1024 ? 16 : 8); }

long lu_tri_elems(int n) {
  const int w = lu_panel_width(n);
  return (long)cdiv(n, w) * 2 * w * w;
}

struct LuArgs {
  double2 *M;
  long sM;
  int ldm;
  int *perm;
  long sP;
  double2 *tri;
  long sT;
  int *zp;
  double2 *X;
  long sX;
  int ldx;
  int n, nrhs;
  const int *skip;
  int skip_shift;
};

__device__ __forceinline__ bool skipped(const LuArgs &a, int mat) {
  return a.skip != nullptr && a.skip[mat >> a.skip_shift] != 0;
}

static LuArgs make_args(const LuDesc &d) {
  LuArgs a;
  a.M = d.M; a.sM = d.sM; a.ldm = d.ldm; a.perm = d.perm; a.sP = d.sP; a.tri = d.tri; a.sT = d.sT;
  a.zp = d.zp; a.X = d.X; a.sX = d.sX; a.ldx = d.ldx; a.n = d.n; a.nrhs = d.nrhs;
  a.skip = d.skip; a.skip_shift = d.skip_shift;
  return a;
}

__global__ void k_identity_perm(int *perm, long sP, int n) {
  int *p = perm + (long)blockIdx.y * sP;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
}

// ------------------------------------------------------------------ panel factorization

struct PanelShared {
  double red_v[16];
  int red_i[16];
};

// One column step of the panel factorization for compile-time column J (keeps v in registers).
template <int J, int W, int R>
__device__ __forceinline__ void panel_column(double2 (&v)[R * W], double2 (*rowbuf)[W], int *sperm, PanelShared &ps,
                                             int T, int nrows, int w, int r0, int &zero_col) {
  if (J >= w) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = T >> 6;
  // ---- pivot search: largest |Re|+|Im| in column J among logical rows >= J, lowest row on ties
  double bv = -1.0;
  int bi = INT_MAX;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * T;
    if (lr >= J && lr < nrows) {
      const double t = cabs1(v[q * W + J]);
      if (t > bv) { bv = t; bi = lr; }
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(bv, off);
    const int oi = __shfl_xor(bi, off);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  if (lane == 0) { ps.red_v[wave] = bv; ps.red_i[wave] = bi; }
  __syncthreads();
  bv = ps.red_v[0];
  bi = ps.red_i[0];
  for (int ww = 1; ww < nw; ++ww) {
    const double ov = ps.red_v[ww];
    const int oi = ps.red_i[ww];
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  // no finite candidate (NaN column): keep the diagonal row so indexing stays in range
  const int piv = (bi >= J && bi < nrows) ? bi : J;
  // ---- interchange logical rows J and piv (data travels between the two owning threads)
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * T;
    if (lr == piv) {
#pragma unroll
      for (int c = 0; c < W; ++c) st2(rowbuf[0][c], v[q * W + c]);
    }
    if (lr == J && piv != J) {
#pragma unroll
      for (int c = 0; c < W; ++c) st2(rowbuf[1][c], v[q * W + c]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * T;
    if (lr == J) {
#pragma unroll
      for (int c = 0; c < W; ++c) v[q * W + c] = ld2(rowbuf[0][c]);
    } else if (lr == piv) {
#pragma unroll
      for (int c = 0; c < W; ++c) v[q * W + c] = ld2(rowbuf[1][c]);
    }
  }
  if (tid == 0 && piv != J) {
    const int t = sperm[J];
    sperm[J] = sperm[piv];
    sperm[piv] = t;
  }
  // ---- eliminate below the pivot
  const double2 u = ld2(rowbuf[0][J]);
  if (u.x == 0.0 && u.y == 0.0) {
    if (zero_col == 0) zero_col = r0 + J + 1;
  } else {
    const double2 ui = crecip(u);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int lr = tid + q * T;
      if (lr > J && lr < nrows) {
        const double2 l = cmul(v[q * W + J], ui);
        v[q * W + J] = l;
#pragma unroll
        for (int c = J + 1; c < W; ++c) v[q * W + c] = cfnms(v[q * W + c], l, ld2(rowbuf[0][c]));
      }
    }
  }
}

template <int W, int R, int... J>
__device__ __forceinline__ void panel_columns(std::integer_sequence<int, J...>, double2 (&v)[R * W],
                                              double2 (*rowbuf)[W], int *sperm, PanelShared &ps, int T, int nrows,
                                              int w, int r0, int &zero_col) {
  (panel_column<J, W, R>(v, rowbuf, sperm, ps, T, nrows, w, r0, zero_col), ...);
}

template <int W, int R, int LB>
__global__ void __launch_bounds__(LB) k_panel(LuArgs a, int r0, int p) {
  const int mat = blockIdx.x;
  if (skipped(a, mat)) return;
  const int tid = threadIdx.x, T = blockDim.x;
  double2 *M = a.M + (long)mat * a.sM;
  int *perm = a.perm + (long)mat * a.sP;
  const int nrows = a.n - r0;
  const int w = min(W, nrows);
  const long ld = a.ldm;

  __shared__ int sperm[LB * R];
  __shared__ PanelShared ps;
  __shared__ double2 rowbuf[2][W];
  __shared__ double2 blk[W][W + 1];
  __shared__ double2 inv[W][W + 1];

  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * T;
    if (lr < nrows) sperm[lr] = perm[r0 + lr];
  }
  __syncthreads();

  double2 v[R * W];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * T;
#pragma unroll
    for (int c = 0; c < W; ++c)
      v[q * W + c] = (lr < nrows && c < w) ? M[(long)sperm[lr] * ld + r0 + c] : make_double2(0.0, 0.0);
  }

  int zero_col = 0;
  panel_columns<W, R>(std::make_integer_sequence<int, W>{}, v, rowbuf, sperm, ps, T, nrows, w, r0, zero_col);
  __syncthreads();  // sperm final

  // ---- write the factored panel back (rows stay in their physical place) and the row map
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int lr = tid + q * T;
    if (lr < nrows) {
#pragma unroll
      for (int c = 0; c < W; ++c)
        if (c < w) M[(long)sperm[lr] * ld + r0 + c] = v[q * W + c];
      perm[r0 + lr] = sperm[lr];
    }
  }
  if (tid == 0) {
    if (p == 0) a.zp[mat] = zero_col;
    else if (zero_col != 0 && a.zp[mat] == 0) a.zp[mat] = zero_col;
  }

  // ---- invert the diagonal blocks: L11 (unit lower) and U11 (upper), padded with the identity
  if (tid < W) {
#pragma unroll
    for (int c = 0; c < W; ++c) {
      double2 e = make_double2(tid == c ? 1.0 : 0.0, 0.0);
      st2(blk[tid][c], (tid < w && c < w) ? v[c] : e);
    }
  }
  __syncthreads();
  if (tid < W) {
    const int c = tid;
    // column c of L11^{-1}
    for (int i = 0; i < W; ++i) {
      double2 x;
      if (i < c) x = make_double2(0.0, 0.0);
      else if (i == c) x = make_double2(1.0, 0.0);
      else {
        x = make_double2(0.0, 0.0);
        for (int k = c; k < i; ++k) x = cfnms(x, ld2(blk[i][k]), ld2(inv[k][c]));
      }
      st2(inv[i][c], x);
    }
  }
  __syncthreads();
  double2 *tL = a.tri + (long)mat * a.sT + (long)p * 2 * W * W;
  double2 *tU = tL + W * W;
  for (int idx = tid; idx < W * W; idx += T) tL[idx] = ld2(inv[idx / W][idx % W]);
  __syncthreads();
  if (tid < W) {
    const int c = tid;
    // column c of U11^{-1}: x_c = 1/U_cc, x_i = -(sum_{k=i+1..c} U_ik x_k) / U_ii
    for (int i = W - 1; i >= 0; --i) {
      double2 x = make_double2(0.0, 0.0);
      if (i == c) x = crecip(ld2(blk[c][c]));
      else if (i < c) {
        double2 s = make_double2(0.0, 0.0);
        for (int k = i + 1; k <= c; ++k) s = cfnms(s, ld2(blk[i][k]), ld2(inv[k][c]));
        x = cmul(s, crecip(ld2(blk[i][i])));
      }
      st2(inv[i][c], x);
    }
  }
  __syncthreads();
  for (int idx = tid; idx < W * W; idx += T) tU[idx] = ld2(inv[idx / W][idx % W]);
}

// ------------------------------------------------------------------ tile kernels

template <int W>
struct LuTiles {
  static constexpr int TB = W < 16 ? 16 : W;  // rows of a row-block tile (MFMA needs 16)
  // tall tile of the panel update: 64 rows x TB columns
  using Upd = TileCfg<64, TB, 16, (TB == 32 ? 2 : 4), (TB == 32 ? 2 : 1)>;
  // wide tile of the row block / back substitution: TB rows x 64 columns
  using Row = TileCfg<TB, 64, 16, (TB == 32 ? 2 : 1), (TB == 32 ? 2 : 4)>;
};

template <class T>
constexpr int lds_need() {
  return T::LDS_DOUBLES > tri_lds_doubles<T>() ? T::LDS_DOUBLES : tri_lds_doubles<T>();
}

__device__ __forceinline__ void load_perm(int *sperm, const int *perm, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) sperm[i] = perm[i];
  __syncthreads();
}

// A[r0:n, r0:r0+w] -= L[r0:n, 0:r0] * U[0:r0, r0:r0+w]
template <int W>
__global__ void __launch_bounds__(LuTiles<W>::Upd::NT) k_panel_update(LuArgs a, int r0) {
  using T = typename LuTiles<W>::Upd;
  __shared__ double lds[T::LDS_DOUBLES];
  __shared__ int sperm[kLuMaxN];
  const int mat = blockIdx.y;
  if (skipped(a, mat)) return;
  double2 *M = a.M + (long)mat * a.sM;
  load_perm(sperm, a.perm + (long)mat * a.sP, a.n);
  const int w = min(W, a.n - r0);
  const int m0 = r0 + blockIdx.x * T::BM;
  Acc<T> acc;
  acc.zero();
  LdRowPerm la{M, a.ldm, sperm};
  LdRowPerm lb{M, a.ldm, sperm};
  mma_loop<T>(la, lb, m0, a.n, r0, r0 + w, 0, r0, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 val) {
    const int gr = m0 + r, gc = r0 + c;
    if (gr < a.n && c < w) {
      double2 *p = M + (long)sperm[gr] * a.ldm + gc;
      *p = csub(*p, val);
    }
  });
}

// Row block of panel p: rows [r0, r0+w), columns [r0+w, n+nrhs)
template <int W>
__global__ void __launch_bounds__(LuTiles<W>::Row::NT) k_row_block(LuArgs a, int r0, int p) {
  using T = typename LuTiles<W>::Row;
  __shared__ double lds[lds_need<T>()];
  __shared__ int sperm[kLuMaxN];
  const int mat = blockIdx.y;
  if (skipped(a, mat)) return;
  double2 *M = a.M + (long)mat * a.sM;
  load_perm(sperm, a.perm + (long)mat * a.sP, a.n);
  const int w = min(W, a.n - r0);
  const int ncol = a.n + a.nrhs;
  const int c0 = r0 + w + blockIdx.x * T::BN;
  Acc<T> acc;
  acc.zero();
  LdRowPerm la{M, a.ldm, sperm};
  LdRowPerm lb{M, a.ldm, sperm};
  mma_loop<T>(la, lb, r0, r0 + w, c0, ncol, 0, r0, acc, lds);
  const double2 *tL = a.tri + (long)mat * a.sT + (long)p * 2 * W * W;
  LdRow lt{tL, W};
  tri_apply<T>(lt, W, acc,
               [&](int r, int c, double2 val) {
                 if (r < w && c0 + c < ncol) return csub(M[(long)sperm[r0 + r] * a.ldm + c0 + c], val);
                 return make_double2(0.0, 0.0);
               },
               lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 val) {
    if (r < w && c0 + c < ncol) M[(long)sperm[r0 + r] * a.ldm + c0 + c] = val;
  });
}

// Back substitution of block row p: X[r0:r0+w, :] = U11^{-1} (Y[r0:r0+w, :] - U[r0:r0+w, r0+w:n] X[r0+w:n, :])
template <int W>
__global__ void __launch_bounds__(LuTiles<W>::Row::NT) k_back_sub(LuArgs a, int r0, int p) {
  using T = typename LuTiles<W>::Row;
  __shared__ double lds[lds_need<T>()];
  __shared__ int sperm[kLuMaxN];
  const int mat = blockIdx.y;
  if (skipped(a, mat)) return;
  double2 *M = a.M + (long)mat * a.sM;
  double2 *X = a.X + (long)mat * a.sX;
  load_perm(sperm, a.perm + (long)mat * a.sP, a.n);
  const int w = min(W, a.n - r0);
  const int c0 = blockIdx.x * T::BN;
  Acc<T> acc;
  acc.zero();
  LdRowPerm la{M, a.ldm, sperm};
  LdRow lb{X, a.ldx};
  mma_loop<T>(la, lb, r0, r0 + w, c0, a.nrhs, r0 + w, a.n, acc, lds);
  const double2 *tU = a.tri + (long)mat * a.sT + (long)p * 2 * W * W + W * W;
  LdRow lt{tU, W};
  tri_apply<T>(lt, W, acc,
               [&](int r, int c, double2 val) {
                 if (r < w && c0 + c < a.nrhs)
                   return csub(M[(long)sperm[r0 + r] * a.ldm + a.n + c0 + c], val);
                 return make_double2(0.0, 0.0);
               },
               lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 val) {
    if (r < w && c0 + c < a.nrhs) X[(long)(r0 + r) * a.ldx + c0 + c] = val;
  });
}

// ------------------------------------------------------------------ driver

template <int W, int R, int LB>
static ss_status lu_run(ss_ctx *ctx, const LuDesc &d) {
  const LuArgs a = make_args(d);
  const int n = d.n, np = cdiv(n, W), ncol = d.n + d.nrhs;
  for (int p = 0; p < np; ++p) {
    const int r0 = p * W, w = std::min(W, n - r0);
    if (p > 0) {
      dim3 g(cdiv(n - r0, LuTiles<W>::Upd::BM), d.nmat);
      {
        KernelScope ks_(ctx, "panel_update");
        hipLaunchKernelGGL(k_panel_update<W>, g, dim3(LuTiles<W>::Upd::NT), 0, ctx->stream, a, r0);
      }
    }
    const int rows = cdiv(n - r0, R);
    const int threads = std::min(LB, std::max(64, cdiv(rows, 64) * 64));
    {
      KernelScope ks_(ctx, "panel");
      hipLaunchKernelGGL((k_panel<W, R, LB>), dim3(d.nmat), dim3(threads), 0, ctx->stream, a, r0, p);
    }
    const int right = ncol - (r0 + w);
    if (right > 0) {
      dim3 g(cdiv(right, LuTiles<W>::Row::BN), d.nmat);
      {
        KernelScope ks_(ctx, "row_block");
        hipLaunchKernelGGL(k_row_block<W>, g, dim3(LuTiles<W>::Row::NT), 0, ctx->stream, a, r0, p);
      }
    }
  }
  if (d.nrhs > 0) {
    for (int p = np - 1; p >= 0; --p) {
      const int r0 = p * W;
      dim3 g(cdiv(d.nrhs, LuTiles<W>::Row::BN), d.nmat);
      {
        KernelScope ks_(ctx, "back_sub");
        hipLaunchKernelGGL(k_back_sub<W>, g, dim3(LuTiles<W>::Row::NT), 0, ctx->stream, a, r0, p);
      }
    }
  }
  return check_launch(ctx, "lu_solve");
}

ss_status lu_solve(ss_ctx *ctx, const LuDesc &d) {
  if (d.nmat <= 0) return SS_OK;
  if (d.n < 1 || d.n > kLuMaxN) return fail(ctx, SS_ERR_UNSUPPORTED, "lu_solve: order out of range");
  const int W = lu_panel_width(d.n);
  if (W == 32) return lu_run<32, 1, 512>(ctx, d);
  if (W == 16) return lu_run<16, 1, 1024>(ctx, d);
  return lu_run<8, 2, 1024>(ctx, d);
}

ss_status lu_identity_perm(ss_ctx *ctx, const LuDesc &d) {
  if (d.nmat <= 0) return SS_OK;
  hipLaunchKernelGGL(k_identity_perm, dim3(cdiv(d.n, 256), d.nmat), dim3(256), 0, ctx->stream, d.perm, d.sP,
                     d.n);
  return check_launch(ctx, "lu_identity_perm");
}

}  // namespace ss
