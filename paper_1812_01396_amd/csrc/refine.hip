// Injection from the left lead, iterative refinement of psi on the full open system, and the
// transmission carried by psi.
//
// Refinement (Sec. 3B, Eq. (x) applied to a residual): with T = A - B C,
//     r = B b' - T psi                    (FP64, the blocks of A formed as E*S - H)
//     y = A~^{-1} r                       (kept factors of the first-column recursion, below)
//     z = R^{-1} (C y),  psi += y + Q z   (corner factorization of ss_apply_obc)
// A~^{-1} r from the recursion D_i = A_ii - A_{i,i+1} X_{i+1}, X_i = D_i^{-1} A_{i,i-1}:
//     backward  g_n = D_n^{-1} r_n,  g_i = D_i^{-1} (r_i - A_{i,i+1} g_{i+1})
//     forward   y_1 = g_1,           y_i = g_i - X_i y_{i-1}
// which is exact for the factors it is given: with factors from lower-precision products the loop
// converges to the FP64 solution at a rate set by their accuracy.  With an absorbing boundary
// (absorb > 0, see sweep.hip) the factors are those of A' = A + i*absorb*[boundary blocks] and the
// correction uses C' = Sigma + i*absorb*I; the residual is always that of T = A - Sigma itself.
#include <algorithm>
#include <cmath>

#include "drivers.hpp"
#include "lu.hpp"
#include "tile.hpp"

namespace ss {

// the products of the refinement have m (the injected modes, typically 32) columns: 64 x 32 tiles, no
// padded half tile
using RefTile = TileCfgG3<64, 32, 16, 4, 1>;

struct LdRowNeg {  // -p[r * ld + c]
  const double2 *p;
  long ld;
  static constexpr bool kFastSecond = true;
  __device__ __forceinline__ double2 operator()(int r, int c) const { return cneg(p[(long)r * ld + c]); }
};

struct LdGammaR {  // element (r, c) of Gamma = i (Sigma - Sigma^H)
  const double2 *sig;
  int s;
  static constexpr bool kFastSecond = true;
  __device__ __forceinline__ double2 operator()(int r, int c) const {
    const double2 a = sig[(long)r * s + c], b = sig[(long)c * s + r];
    return make_double2(-(a.y + b.y), a.x - b.x);
  }
};

struct RefArgs {
  const double2 *Hd, *Hu, *Sd, *Su;
  long kstride_d, kstride_u;
  const int *kidx;
  const double *E;
  int nk, nb, s, m, batch;
  const double2 *Q, *sigma, *inj;
  double2 *x;    // psi [batch][nb][s][m]
  double2 *r;    // residual, then r~ [batch][nb][s][m]
  double2 *g;    // g, then y [batch][nb][s][m]
  double2 *cy;   // C y [batch][2s][m]
  double2 *z;    // [batch][2s][m]
  const double2 *X;  // kept X_i: [2 batch][nb][s][s], first-column systems are the even ones
  double *nrm;   // [batch][2]: ||r||^2, ||b||^2
  int *done;     // [batch]
  double tol;
  double absorb;  // C' = Sigma + i*absorb*I
};

__device__ __forceinline__ int ref_set(const RefArgs &a, int inst) {
  const int k = a.kidx ? a.kidx[inst] : inst % a.nk;
  return min(max(k, 0), a.nk - 1);
}

// Instance-major order for a grid of (work items, instances): linear workgroup ids go to the eight XCDs
// round-robin, so the ids are remapped such that XCD x runs the instances [x b/8, (x+1) b/8) and takes
// them work item by work item: the instances that share a momentum (consecutive ones, as the callers
// order them) then read each (H, S) block panel together through one L2 instead of once per energy.
// A bijection of the grid; batches that are not a multiple of 8 keep the plain order.
__device__ __forceinline__ void xcd_inst_order(int &work, int &inst) {
  const int nw = gridDim.x, nbat = gridDim.y;
  if (nbat % 8 != 0) {
    work = blockIdx.x;
    inst = blockIdx.y;
    return;
  }
  const long lin = blockIdx.x + (long)nw * blockIdx.y;
  const long slot = lin >> 3;
  const int per = nbat >> 3;
  inst = (int)(lin & 7) * per + (int)(slot % per);
  work = (int)(slot / per);
}

// r = B b' - T x for every block, with ||r||^2 and ||B b'||^2; grid (nb * tiles(s) * tiles(m), batch)
__global__ void __launch_bounds__(RefTile::NT) SS_TILE_WAVES_OF(RefTile) k_ref_resid(RefArgs a) {
  using T = RefTile;
  __shared__ double lds[T::LDS_DOUBLES];
  __shared__ double red[2][T::NT / 64];
  int work, inst;
  xcd_inst_order(work, inst);
  if (a.done[inst]) return;
  const int s = a.s, m = a.m, nb = a.nb;
  const int tr = cdiv(s, T::BM), tc = cdiv(m, T::BN);
  const int i = work / (tr * tc), rem = work % (tr * tc);
  const int m0 = (rem / tc) * T::BM, n0 = (rem % tc) * T::BN;
  const int ks = ref_set(a, inst);
  const double e = a.E[inst];
  const long ss2 = (long)s * s, sm = (long)s * m;
  const double2 *x = a.x + (long)inst * nb * sm;
  Acc<T> acc;
  acc.zero();
  {
    LdForm<false> la{a.Hd + ks * a.kstride_d + i * ss2, a.Sd + ks * a.kstride_d + i * ss2, s, e};
    LdRow lb{x + i * sm, m};
    mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  }
  if (i < nb - 1) {  // A_{i,i+1} x_{i+1}
    LdForm<false> la{a.Hu + ks * a.kstride_u + i * ss2, a.Su + ks * a.kstride_u + i * ss2, s, e};
    LdRow lb{x + (i + 1) * sm, m};
    mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  }
  if (i > 0) {  // A_{i,i-1} x_{i-1} = (E S_u[i-1] - H_u[i-1])^H x_{i-1}
    LdForm<true> la{a.Hu + ks * a.kstride_u + (i - 1) * ss2, a.Su + ks * a.kstride_u + (i - 1) * ss2, s, e};
    LdRow lb{x + (i - 1) * sm, m};
    mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  }
  if (i == 0) {  // - Sigma_L x_0
    LdRowNeg la{a.sigma + (long)inst * 2 * ss2, s};
    LdRow lb{x, m};
    mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  }
  if (i == nb - 1) {  // - Sigma_R x_{nb-1}
    LdRowNeg la{a.sigma + ((long)inst * 2 + 1) * ss2, s};
    LdRow lb{x + (long)(nb - 1) * sm, m};
    mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  }
  const double2 *inj = a.inj + (long)inst * 2 * sm;
  double2 *r = a.r + (long)inst * nb * sm + i * sm;
  double rr = 0.0, bb = 0.0;
  acc_foreach<T>(acc, [&](int rl, int cl, double2 v) {
    const int gr = m0 + rl, gc = n0 + cl;
    if (gr < s && gc < m) {
      double2 b = make_double2(0.0, 0.0);
      if (i == 0) b = cadd(b, inj[(long)gr * m + gc]);
      if (i == nb - 1) b = cadd(b, inj[(long)(s + gr) * m + gc]);
      const double2 res = csub(b, v);
      r[(long)gr * m + gc] = res;
      rr += res.x * res.x + res.y * res.y;
      bb += b.x * b.x + b.y * b.y;
    }
  });
  for (int off = 32; off >= 1; off >>= 1) {
    rr += __shfl_xor(rr, off);
    bb += __shfl_xor(bb, off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { red[0][wave] = rr; red[1][wave] = bb; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0, t1 = 0.0;
    for (int w = 0; w < T::NT / 64; ++w) { t0 += red[0][w]; t1 += red[1][w]; }
    atomicAdd(a.nrm + 2 * inst, t0);
    atomicAdd(a.nrm + 2 * inst + 1, t1);
  }
}

// convergence test: done when ||r|| <= tol ||b|| (the norms are cleared for the next pass)
__global__ void k_ref_check(RefArgs a, int it, int *iters, double *resid) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= a.batch || a.done[inst]) return;
  const double rr = a.nrm[2 * inst], bb = a.nrm[2 * inst + 1];
  a.nrm[2 * inst] = 0.0;
  a.nrm[2 * inst + 1] = 0.0;
  const double rel = sqrt(rr) / fmax(sqrt(bb), 1e-300);
  if (resid) resid[inst] = rel;
  if (iters) iters[inst] = it;
  if (rel <= a.tol) a.done[inst] = 1;
}

// r_i -= A_{i,i+1} g_{i+1}
__global__ void __launch_bounds__(RefTile::NT) SS_TILE_WAVES_OF(RefTile) k_ref_couple(RefArgs a, int i) {
  using T = RefTile;
  __shared__ double lds[T::LDS_DOUBLES];
  int tile, inst;
  xcd_inst_order(tile, inst);
  if (a.done[inst]) return;
  const int s = a.s, m = a.m, nb = a.nb;
  const int tc = cdiv(m, T::BN);
  const int m0 = (tile / tc) * T::BM, n0 = (tile % tc) * T::BN;
  const int ks = ref_set(a, inst);
  const double e = a.E[inst];
  const long ss2 = (long)s * s, sm = (long)s * m;
  Acc<T> acc;
  acc.zero();
  LdForm<false> la{a.Hu + ks * a.kstride_u + i * ss2, a.Su + ks * a.kstride_u + i * ss2, s, e};
  LdRow lb{a.g + (long)inst * nb * sm + (i + 1) * sm, m};
  mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  double2 *r = a.r + (long)inst * nb * sm + i * sm;
  acc_foreach<T>(acc, [&](int rl, int cl, double2 v) {
    const int gr = m0 + rl, gc = n0 + cl;
    if (gr < s && gc < m) r[(long)gr * m + gc] = csub(r[(long)gr * m + gc], v);
  });
}

// y_i = g_i - X_i y_{i-1} (in place in g); X_i of block i was kept at slot nb-1-i of the even system
__global__ void __launch_bounds__(RefTile::NT) SS_TILE_WAVES_OF(RefTile) k_ref_chain(RefArgs a, int i) {
  using T = RefTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int inst = blockIdx.y;
  if (a.done[inst]) return;
  const int s = a.s, m = a.m, nb = a.nb;
  const int tc = cdiv(m, T::BN);
  const int m0 = (blockIdx.x / tc) * T::BM, n0 = (blockIdx.x % tc) * T::BN;
  const long ss2 = (long)s * s, sm = (long)s * m;
  Acc<T> acc;
  acc.zero();
  LdRow la{a.X + ((long)(2 * inst) * nb + (nb - 1 - i)) * ss2, s};
  LdRow lb{a.g + (long)inst * nb * sm + (i - 1) * sm, m};
  mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  double2 *y = a.g + (long)inst * nb * sm + i * sm;
  acc_foreach<T>(acc, [&](int rl, int cl, double2 v) {
    const int gr = m0 + rl, gc = n0 + cl;
    if (gr < s && gc < m) y[(long)gr * m + gc] = csub(y[(long)gr * m + gc], v);
  });
}

// C y = [Sigma_L y_1; Sigma_R y_nb]; grid (2 * tiles(s) * tiles(m), batch)
__global__ void __launch_bounds__(RefTile::NT) SS_TILE_WAVES_OF(RefTile) k_ref_cy(RefArgs a) {
  using T = RefTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int inst = blockIdx.y;
  if (a.done[inst]) return;
  const int s = a.s, m = a.m, nb = a.nb;
  const int tr = cdiv(s, T::BM), tc = cdiv(m, T::BN);
  const int half = blockIdx.x / (tr * tc), rem = blockIdx.x % (tr * tc);
  const int m0 = (rem / tc) * T::BM, n0 = (rem % tc) * T::BN;
  const long ss2 = (long)s * s, sm = (long)s * m;
  Acc<T> acc;
  acc.zero();
  LdRow la{a.sigma + ((long)inst * 2 + half) * ss2, s};
  LdRow lb{a.g + (long)inst * nb * sm + (half ? (long)(nb - 1) * sm : 0), m};
  mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  double2 *cy = a.cy + (long)inst * 2 * sm + half * sm;
  const double2 *yb = a.g + (long)inst * nb * sm + (half ? (long)(nb - 1) * sm : 0);
  acc_foreach<T>(acc, [&](int rl, int cl, double2 v) {
    const int gr = m0 + rl, gc = n0 + cl;
    if (gr < s && gc < m) {
      if (a.absorb != 0.0) {  // + i*absorb*y
        const double2 y = yb[(long)gr * m + gc];
        v = make_double2(v.x - a.absorb * y.y, v.y + a.absorb * y.x);
      }
      cy[(long)gr * m + gc] = v;
    }
  });
}

// x += y + Q z; grid (tiles(nb s) * tiles(m), batch)
__global__ void __launch_bounds__(RefTile::NT) SS_TILE_WAVES_OF(RefTile) k_ref_update(RefArgs a) {
  using T = RefTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int inst = blockIdx.y;
  if (a.done[inst]) return;
  const int s = a.s, m = a.m, nb = a.nb, rows = nb * s;
  const int tc = cdiv(m, T::BN);
  const int m0 = (blockIdx.x / tc) * T::BM, n0 = (blockIdx.x % tc) * T::BN;
  Acc<T> acc;
  acc.zero();
  LdRow la{a.Q + (long)inst * rows * 2 * s, 2 * s};
  LdRow lb{a.z + (long)inst * 2 * s * m, m};
  mma_loop<T>(la, lb, m0, rows, n0, m, 0, 2 * s, acc, lds);
  double2 *x = a.x + (long)inst * rows * m;
  const double2 *y = a.g + (long)inst * rows * m;
  acc_foreach<T>(acc, [&](int rl, int cl, double2 v) {
    const int gr = m0 + rl, gc = n0 + cl;
    if (gr < rows && gc < m) {
      const long o = (long)gr * m + gc;
      x[o] = cadd(x[o], cadd(y[o], v));
    }
  });
}

__global__ void k_ref_reset(RefArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.batch) return;
  a.done[i] = 0;
  a.nrm[2 * i] = 0.0;
  a.nrm[2 * i + 1] = 0.0;
}

__global__ void k_count_done(const int *done, int batch, int *count) {
  __shared__ int c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  int mine = 0;
  for (int i = threadIdx.x; i < batch; i += blockDim.x) mine += done[i] != 0;
  atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) *count = c;
}

ss_status refine_psi(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E, const ss_c128 *Q,
                     const ss_c128 *sigma, int m, const ss_c128 *inj, ss_c128 *psi, double tol, int max_iter,
                     int *iters, double *resid) {
  const int s = hs->s, nb = hs->nb;
  if (!ctx->fact_valid || ctx->fact_batch != batch || ctx->fact_nb != nb || ctx->fact_s != s)
    return fail(ctx, SS_ERR_ARG, "ss_refine_psi: no kept factors for this batch (ss_precompute_columns with "
                                 "SS_KEEP_FACTORS must run first on this context)");
  if (!ctx->corner_valid || ctx->corner_batch != batch || ctx->corner_s != s)
    return fail(ctx, SS_ERR_ARG, "ss_refine_psi: no corner factorization for this batch (ss_apply_obc must run "
                                 "last on this context)");
  if (ctx->fact_absorb != ctx->corner_absorb)
    return fail(ctx, SS_ERR_ARG, "ss_refine_psi: the kept factors and the corner system were formed with different "
                                 "absorbing shifts");
  if (tol <= 0) tol = 1e-12;
  if (max_iter <= 0) max_iter = 10;
  const long ss2 = (long)s * s, sm = (long)s * m;
  void *wR, *wMisc;
  SS_TRY(workspace(ctx, kSlotRef, sizeof(double2) * (size_t)batch * (2 * nb * sm + 4 * sm), &wR));
  SS_TRY(workspace(ctx, kSlotMisc, (size_t)batch * (16 + 4) + 64, &wMisc));
  int *count = nullptr;
  SS_TRY(host_word(ctx, &count));

  RefArgs a;
  a.Hd = (const double2 *)hs->H_diag;
  a.Hu = (const double2 *)hs->H_upper;
  a.Sd = (const double2 *)hs->S_diag;
  a.Su = (const double2 *)hs->S_upper;
  a.kstride_d = (long)nb * ss2;
  a.kstride_u = (long)std::max(nb - 1, 0) * ss2;
  a.kidx = kidx;
  a.E = E;
  a.nk = hs->nk;
  a.nb = nb;
  a.s = s;
  a.m = m;
  a.batch = batch;
  a.Q = (const double2 *)Q;
  a.sigma = (const double2 *)sigma;
  a.inj = (const double2 *)inj;
  a.x = (double2 *)psi;
  a.r = (double2 *)wR;
  a.g = a.r + (size_t)batch * nb * sm;
  a.cy = a.g + (size_t)batch * nb * sm;
  a.z = a.cy + (size_t)batch * 2 * sm;
  void *wX, *wF, *wP, *wMc, *wPc;
  SS_TRY(workspace(ctx, kSlotX, 0, &wX));
  SS_TRY(workspace(ctx, kSlotFact, 0, &wF));
  SS_TRY(workspace(ctx, kSlotFactPerm, 0, &wP));
  SS_TRY(workspace(ctx, kSlotM, 0, &wMc));
  SS_TRY(workspace(ctx, kSlotPerm, 0, &wPc));
  a.X = (const double2 *)wX;
  a.nrm = (double *)wMisc;
  a.done = (int *)((char *)wMisc + (size_t)batch * 16);
  int *dcount = a.done + batch;
  a.tol = tol;
  a.absorb = ctx->fact_absorb;

  // block solves with the kept diagonal factorizations: D_i of block i was factored at step nb-1-i
  LuDesc dd;
  dd.nmat = batch;
  dd.n = s;
  dd.nrhs = m;
  dd.sM = (long)nb * ss2;
  dd.ldm = s;
  dd.sP = (long)nb * s;
  dd.zp = nullptr;
  dd.sB = (long)nb * sm;
  dd.ldb = m;
  dd.sX = (long)nb * sm;
  dd.ldx = m;
  dd.skip = a.done;
  void *wFI = nullptr;
  if (ctx->fact_inv) {  // the kept inverses of the 32 x 32 diagonal blocks, laid out like the factors
    SS_TRY(workspace(ctx, kSlotFactInv, 0, &wFI));
    dd.sInv = (long)nb * lu_inverse_elems(s, 32);
  }
  // the corner solve with R
  LuDesc dc;
  dc.nmat = batch;
  dc.n = 2 * s;
  dc.nrhs = m;
  dc.M = (double2 *)wMc;
  dc.sM = (long)2 * s * ctx->corner_ldm;
  dc.ldm = ctx->corner_ldm;
  dc.perm = (int *)wPc;
  dc.sP = 2 * s;
  dc.B = a.cy;
  dc.sB = 2 * sm;
  dc.ldb = m;
  dc.X = a.z;
  dc.sX = 2 * sm;
  dc.ldx = m;
  dc.skip = a.done;

  using T = RefTile;
  const int tr = cdiv(s, T::BM), tc = cdiv(m, T::BN);
  hipLaunchKernelGGL(k_ref_reset, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, a);
  for (int it = 0; it <= max_iter; ++it) {
    hipLaunchKernelGGL(k_ref_resid, dim3(nb * tr * tc, batch), dim3(T::NT), 0, ctx->stream, a);
    hipLaunchKernelGGL(k_ref_check, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, a, it, iters, resid);
    if (it == max_iter) break;
    if (!ctx->sync_free) {  // stop once every instance has converged
      hipLaunchKernelGGL(k_count_done, dim3(1), dim3(256), 0, ctx->stream, (const int *)a.done, batch, dcount);
      if (hipMemcpyAsync(count, dcount, sizeof(int), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
          hipStreamSynchronize(ctx->stream) != hipSuccess)
        return fail(ctx, SS_ERR_DEVICE, "ss_refine_psi: convergence poll");
      if (*count >= batch) break;
    }
    // backward: g_i = D_i^{-1} (r_i - A_{i,i+1} g_{i+1})
    for (int i = nb - 1; i >= 0; --i) {
      if (i < nb - 1)
        hipLaunchKernelGGL(k_ref_couple, dim3(tr * tc, batch), dim3(T::NT), 0, ctx->stream, a, i);
      const int t = nb - 1 - i;
      dd.M = (double2 *)wF + (long)t * ss2;
      dd.perm = (int *)wP + (long)t * s;
      if (ctx->fact_inv) dd.inv = (const double2 *)wFI + (long)t * lu_inverse_elems(s, 32);
      dd.B = a.r + (long)i * sm;
      dd.X = a.g + (long)i * sm;
      SS_TRY(lu_apply(ctx, dd));
    }
    // forward: y_i = g_i - X_i y_{i-1}
    for (int i = 1; i < nb; ++i)
      hipLaunchKernelGGL(k_ref_chain, dim3(tr * tc, batch), dim3(T::NT), 0, ctx->stream, a, i);
    hipLaunchKernelGGL(k_ref_cy, dim3(2 * tr * tc, batch), dim3(T::NT), 0, ctx->stream, a);
    SS_TRY(lu_apply(ctx, dc));
    hipLaunchKernelGGL(k_ref_update, dim3(cdiv(nb * s, T::BM) * tc, batch), dim3(T::NT), 0, ctx->stream, a);
  }
  return check_launch(ctx, "refine_psi");
}

// ------------------------------------------------------------------ injection and T from psi

// Pivoted Cholesky of Gamma_L = i (Sigma_L - Sigma_L^H): one workgroup per instance, thread i owns row i.
__global__ void __launch_bounds__(1024) k_inject_left(const double2 *sigma, int s, double tol, int mmax,
                                                      double2 *inj, int *rank) {
  const int inst = blockIdx.x, tid = threadIdx.x, T = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = T >> 6;
  __shared__ double red_v[16];
  __shared__ int red_i[16];
  __shared__ double dmax0;
  const double2 *sig = sigma + (long)inst * 2 * s * s;  // Sigma_L
  double2 *w = inj + (long)inst * 2 * s * mmax;
  for (long idx = tid; idx < (long)2 * s * mmax; idx += T) w[idx] = make_double2(0.0, 0.0);
  // diagonal of Gamma: i (S_ii - conj(S_ii)) = -2 Im S_ii
  double d = tid < s ? -2.0 * sig[(long)tid * s + tid].y : -1.0;
  bool taken = false;
  int k = 0;
  __syncthreads();
  for (; k < mmax; ++k) {
    double bv = (tid < s && !taken) ? d : -1.0;
    int bi = tid < s ? tid : INT_MAX;
    for (int off = 32; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { red_v[wave] = bv; red_i[wave] = bi; }
    __syncthreads();
    bv = red_v[0];
    bi = red_i[0];
    for (int ww = 1; ww < nw; ++ww)
      if (red_v[ww] > bv || (red_v[ww] == bv && red_i[ww] < bi)) { bv = red_v[ww]; bi = red_i[ww]; }
    if (k == 0 && tid == 0) dmax0 = bv;
    __syncthreads();
    if (!(bv > 0.0) || bv <= tol * dmax0 || bi >= s) break;
    const int p = bi;
    const double sq = sqrt(bv);
    if (tid < s) {
      // Gamma[tid][p] - sum_{j<k} W[tid][j] conj(W[p][j])
      const double2 a = sig[(long)tid * s + p], b = sig[(long)p * s + tid];
      double2 g = make_double2(-(a.y + b.y), a.x - b.x);
      for (int j = 0; j < k; ++j) {
        const double2 wi = w[(long)tid * mmax + j], wp = w[(long)p * mmax + j];
        g = make_double2(g.x - (wi.x * wp.x + wi.y * wp.y), g.y - (wi.y * wp.x - wi.x * wp.y));
      }
      double2 col = make_double2(g.x / sq, g.y / sq);
      if (tid == p) col = make_double2(sq, 0.0);
      if (taken) col = make_double2(0.0, 0.0);
      w[(long)tid * mmax + k] = col;
      d -= col.x * col.x + col.y * col.y;
      if (tid == p) taken = true;
    }
    __syncthreads();  // column k visible to every thread before the next pivot row is read
  }
  if (tid == 0 && rank) rank[inst] = k;
}

using TpTile = TileCfg<64, 32, 16, 4, 1>;

// partial sums of Re sum_{a,c} conj(psi[a][c]) (Gamma_R psi)[a][c] over tiles of the last block row
__global__ void __launch_bounds__(TpTile::NT) SS_TILE_WAVES k_trans_psi(const double2 *psi, const double2 *sigma, int nb, int s,
                                                           int m, double *partial) {
  using T = TpTile;
  __shared__ double lds[T::LDS_DOUBLES];
  __shared__ double red[T::NT / 64];
  const int inst = blockIdx.y;
  const int tc = cdiv(m, T::BN);
  const int m0 = (blockIdx.x / tc) * T::BM, n0 = (blockIdx.x % tc) * T::BN;
  const long ss2 = (long)s * s, sm = (long)s * m;
  const double2 *pn = psi + (long)inst * nb * sm + (long)(nb - 1) * sm;
  Acc<T> acc;
  acc.zero();
  LdGammaR la{sigma + ((long)inst * 2 + 1) * ss2, s};
  LdRow lb{pn, m};
  mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  double t = 0.0;
  acc_foreach<T>(acc, [&](int rl, int cl, double2 v) {
    const int gr = m0 + rl, gc = n0 + cl;
    if (gr < s && gc < m) {
      const double2 p = pn[(long)gr * m + gc];
      t += p.x * v.x + p.y * v.y;
    }
  });
  for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < T::NT / 64; ++w) sum += red[w];
    partial[(long)inst * gridDim.x + blockIdx.x] = sum;
  }
}

__global__ void k_sum_rows(const double *partial, int ntile, double *out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double t = 0.0;
  for (int k = 0; k < ntile; ++k) t += partial[(long)i * ntile + k];
  out[i] = t;
}

ss_status injection_left(ss_ctx *ctx, int batch, int s, const ss_c128 *sigma, double tol, int mmax, ss_c128 *inj,
                         int *rank) {
  if (tol <= 0) tol = 1e-12;
  const int threads = std::min(1024, std::max(64, cdiv(s, 64) * 64));
  hipLaunchKernelGGL(k_inject_left, dim3(batch), dim3(threads), 0, ctx->stream, (const double2 *)sigma, s, tol,
                     mmax, (double2 *)inj, rank);
  return check_launch(ctx, "injection_left");
}

// T[i] = sum of the psi partials + (sum of the Caroli partials - sum of the psi0 partials)
__global__ void k_sum_tail(const double *pp, int np, const double *pc, int nc, const double *p0, double *out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double t = 0.0, c = 0.0, t0 = 0.0;
  for (int k = 0; k < np; ++k) t += pp[(long)i * np + k];
  for (int k = 0; k < nc; ++k) c += pc[(long)i * nc + k];
  for (int k = 0; k < np; ++k) t0 += p0[(long)i * np + k];
  out[i] = t + (c - t0);
}

ss_status transmission_psi(ss_ctx *ctx, int batch, int nb, int s, int m, const ss_c128 *psi, const ss_c128 *sigma,
                           const ss_c128 *psi0, const ss_c128 *gc, double *T) {
  const int ntile = cdiv(s, TpTile::BM) * cdiv(m, TpTile::BN);
  const bool tail = psi0 != nullptr && gc != nullptr;
  const int nc = tail ? caroli_rl_tiles(s) : 0;
  void *wP;
  SS_TRY(workspace(ctx, kSlotMisc, sizeof(double) * (size_t)batch * (tail ? 2 * ntile + nc : ntile), &wP));
  double *pp = (double *)wP, *p0 = pp + (size_t)batch * ntile, *pc = p0 + (size_t)batch * ntile;
  hipLaunchKernelGGL(k_trans_psi, dim3(ntile, batch), dim3(TpTile::NT), 0, ctx->stream, (const double2 *)psi,
                     (const double2 *)sigma, nb, s, m, pp);
  if (!tail) {
    hipLaunchKernelGGL(k_sum_rows, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, (const double *)pp, ntile, T,
                       batch);
    return check_launch(ctx, "transmission_psi");
  }
  // psi0 holds one block row per instance: the last block row of the unrefined psi
  hipLaunchKernelGGL(k_trans_psi, dim3(ntile, batch), dim3(TpTile::NT), 0, ctx->stream, (const double2 *)psi0,
                     (const double2 *)sigma, 1, s, m, p0);
  launch_caroli_rl_partials(ctx, batch, s, gc, sigma, pc);
  hipLaunchKernelGGL(k_sum_tail, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, (const double *)pp, ntile,
                     (const double *)pc, nc, (const double *)p0, T, batch);
  return check_launch(ctx, "transmission_psi");
}

}  // namespace ss
