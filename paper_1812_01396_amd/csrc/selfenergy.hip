// Boundary self-energies of a periodic lead by iterative decimation (the standard technique named in
// Sec. 3A as the alternative to the FEAST mode solver), batched over (E, k) instances.
//
// Lead blocks: a0 = (E + i eta) S00 - H00, a1 = E S01 - H01, am1 = a1^H.  One pass of decimation
// eliminates every other cell of the chain; with G = eps^{-1}:
//     eps_s  -= alpha G beta        eps_sL -= beta G alpha        eps -= alpha G beta + beta G alpha
//     alpha <- -alpha G alpha       beta  <- -beta G beta
// from eps = eps_s = eps_sL = a0, alpha = a1, beta = am1.  G beta and G alpha come from one LU solve
// of [eps | beta | alpha]; the four products share one tile kernel which also writes the next
// augmented matrix and the max-norms of the new alpha and beta.  After convergence
//     Sigma_R = a1 eps_s^{-1} am1,   Sigma_L = am1 eps_sL^{-1} a1,
// and the fixed-point residuals ||Sigma - a (a0 - Sigma)^{-1} a'||_F / ||Sigma||_F are evaluated.
#include <algorithm>
#include <climits>

#include "drivers.hpp"
#include "lu.hpp"
#include "tile.hpp"

namespace ss {

struct DecArgs {
  const double2 *H00, *H01, *S00, *S01;  // [nk][s][s]
  const double2 *const *tab;             // or per lead cell {H00, H01, S00, S01} pointers (null: stacked)
  const int *kidx;
  const double *E;
  double eta;
  int nk, s, batch;
  double2 *st;  // per instance: eps, eps_s, eps_sL, alpha[2], beta[2]  (7 s^2)
  double2 *M;   // per instance: [s][3s] augmented matrix
  double2 *Y;   // per instance: [s][2s] = [G beta | G alpha]
  unsigned long long *nrm;  // per instance: [2] max|alpha|, max|beta| bit patterns of the newest pass
  double *scale;            // per instance: max|a0|
  int *done;                // per instance: 1 once converged
  int *iters;               // per instance: passes used
  int *zp;                  // per system: zero pivot of the last factorization
  int *code;                // per instance: first zero pivot code seen
  int *ndone;               // converged-instance counter
  double tol;
};

// lead cell of an instance, clamped into [0, nk) (the binding rejects out-of-range indices)
__device__ __forceinline__ int dec_set(const DecArgs &a, int inst) {
  const int k = a.kidx ? a.kidx[inst] : inst % a.nk;
  return min(max(k, 0), a.nk - 1);
}

// block j (0 H00, 1 H01, 2 S00, 3 S01) of lead cell k
__device__ __forceinline__ const double2 *dec_cell(const DecArgs &a, int k, int j) {
  if (a.tab) return a.tab[4 * k + j];
  const double2 *base = j == 0 ? a.H00 : j == 1 ? a.H01 : j == 2 ? a.S00 : a.S01;
  return base + (long)k * a.s * a.s;
}

enum { kEps = 0, kEpsS = 1, kEpsL = 2, kAlpha0 = 3, kBeta0 = 5 };

__device__ __forceinline__ double2 *dec_mat(const DecArgs &a, int inst, int which) {
  return a.st + ((long)inst * 7 + which) * a.s * a.s;
}

// Maximum of non-negative doubles through their bit patterns (monotone for v >= 0); a NaN is stored as
// the positive quiet NaN, whose pattern lies above every finite value and +Inf, so it survives.
__device__ __forceinline__ void atomic_max_pos(unsigned long long *p, double v) {
  if (v != v) v = __longlong_as_double(0x7ff8000000000000LL);
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// Initial state and the first augmented matrix [a0 | am1 | a1].
__global__ void k_dec_init(DecArgs a) {
  const int inst = blockIdx.y, s = a.s;
  const int ks = dec_set(a, inst);
  const double e = a.E[inst];
  const long ss2 = (long)s * s;
  const double2 *h00 = dec_cell(a, ks, 0), *s00 = dec_cell(a, ks, 2);
  const double2 *h01 = dec_cell(a, ks, 1), *s01 = dec_cell(a, ks, 3);
  double2 *M = a.M + (long)inst * 3 * ss2;
  double lmax = 0.0;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < ss2; idx += (long)gridDim.x * blockDim.x) {
    const int r = idx / s, c = idx % s;
    const double2 hv = h00[idx], sv = s00[idx];
    const double2 a0 = make_double2(e * sv.x - a.eta * sv.y - hv.x, e * sv.y + a.eta * sv.x - hv.y);
    const double2 a1 = make_double2(e * s01[idx].x - h01[idx].x, e * s01[idx].y - h01[idx].y);
    const long t = (long)c * s + r;  // am1(r, c) = conj(a1(c, r))
    const double2 am1 = make_double2(e * s01[t].x - h01[t].x, -(e * s01[t].y - h01[t].y));
    dec_mat(a, inst, kEps)[idx] = a0;
    dec_mat(a, inst, kEpsS)[idx] = a0;
    dec_mat(a, inst, kEpsL)[idx] = a0;
    dec_mat(a, inst, kAlpha0)[idx] = a1;
    dec_mat(a, inst, kBeta0)[idx] = am1;
    M[(long)r * 3 * s + c] = a0;
    M[(long)r * 3 * s + s + c] = am1;
    M[(long)r * 3 * s + 2 * s + c] = a1;
    lmax = nanmax(lmax, hypot(a0.x, a0.y));
  }
  for (int off = 32; off >= 1; off >>= 1) lmax = nanmax(lmax, __shfl_xor(lmax, off));
  if ((threadIdx.x & 63) == 0) atomic_max_pos((unsigned long long *)(a.scale + inst), lmax);
}

__global__ void k_dec_reset(DecArgs a) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= a.batch) return;
  a.done[inst] = 0;
  a.iters[inst] = 0;
  a.code[inst] = 0;
  a.scale[inst] = 0.0;
  a.nrm[2 * inst] = 0;
  a.nrm[2 * inst + 1] = 0;
  if (inst == 0) *a.ndone = 0;
}

using DecTile = TileCfg<64, 64, 16, 2, 2>;
using DecTileG3 = TileCfgG3<64, 64, 16, 2, 2>;

// One decimation pass for tile (m0, n0) of every s x s block, from Y = [G beta | G alpha].
__global__ void __launch_bounds__(DecTile::NT) SS_TILE_WAVES_OF(DecTileG3) k_dec_update(DecArgs a, int par) {
  using T = DecTileG3;
  __shared__ double lds[T::LDS_DOUBLES];
  int tile, inst;
  xcd_tile_order(tile, inst);
  const int s = a.s;
  if (a.done[inst]) return;
  const long ss2 = (long)s * s;
  const int tiles = cdiv(s, T::BM);
  const int m0 = (tile / tiles) * T::BM, n0 = (tile % tiles) * T::BN;
  const double2 *alpha = dec_mat(a, inst, kAlpha0 + par);
  const double2 *beta = dec_mat(a, inst, kBeta0 + par);
  double2 *alpha_n = dec_mat(a, inst, kAlpha0 + (par ^ 1));
  double2 *beta_n = dec_mat(a, inst, kBeta0 + (par ^ 1));
  double2 *eps = dec_mat(a, inst, kEps), *eps_s = dec_mat(a, inst, kEpsS), *eps_l = dec_mat(a, inst, kEpsL);
  const double2 *Y = a.Y + (long)inst * 2 * ss2;
  double2 *M = a.M + (long)inst * 3 * ss2;
  LdRow la_alpha{alpha, s}, la_beta{beta, s};
  LdRow lb_gb{Y, 2 * s}, lb_ga{Y + s, 2 * s};
  Acc<T> acc;

  // alpha G beta: right surface and bulk
  acc.zero();
  mma_loop<T>(la_alpha, lb_gb, m0, s, n0, s, 0, s, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) {
      const long o = (long)gr * s + gc;
      eps_s[o] = csub(eps_s[o], v);
      eps[o] = csub(eps[o], v);
    }
  });
  // beta G alpha: left surface and bulk
  acc.zero();
  mma_loop<T>(la_beta, lb_ga, m0, s, n0, s, 0, s, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) {
      const long o = (long)gr * s + gc;
      eps_l[o] = csub(eps_l[o], v);
      const double2 ne = csub(eps[o], v);
      eps[o] = ne;
      M[(long)gr * 3 * s + gc] = ne;
    }
  });
  // alpha <- -alpha G alpha
  double amax = 0.0;
  acc.zero();
  mma_loop<T>(la_alpha, lb_ga, m0, s, n0, s, 0, s, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) {
      const double2 nv = cneg(v);
      alpha_n[(long)gr * s + gc] = nv;
      M[(long)gr * 3 * s + 2 * s + gc] = nv;
      amax = nanmax(amax, hypot(nv.x, nv.y));
    }
  });
  // beta <- -beta G beta
  double bmax = 0.0;
  acc.zero();
  mma_loop<T>(la_beta, lb_gb, m0, s, n0, s, 0, s, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) {
      const double2 nv = cneg(v);
      beta_n[(long)gr * s + gc] = nv;
      M[(long)gr * 3 * s + s + gc] = nv;
      bmax = nanmax(bmax, hypot(nv.x, nv.y));
    }
  });
  for (int off = 32; off >= 1; off >>= 1) {
    amax = nanmax(amax, __shfl_xor(amax, off));
    bmax = nanmax(bmax, __shfl_xor(bmax, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomic_max_pos(a.nrm + 2 * inst, amax);
    atomic_max_pos(a.nrm + 2 * inst + 1, bmax);
  }
}

// Convergence test after pass `it` (0-based); clears the norms for the next pass.
__global__ void k_dec_check(DecArgs a, int it) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= a.batch || a.done[inst]) return;
  const double na = __longlong_as_double((long long)a.nrm[2 * inst]);
  const double nb = __longlong_as_double((long long)a.nrm[2 * inst + 1]);
  a.nrm[2 * inst] = 0;
  a.nrm[2 * inst + 1] = 0;
  if (a.code[inst] == 0 && a.zp[inst] != 0) a.code[inst] = a.zp[inst];
  a.iters[inst] = it + 1;
  if (na + nb <= a.tol * a.scale[inst]) {
    a.done[inst] = 1;
    atomicAdd(a.ndone, 1);
  }
}

// [eps_s | am1] (system 2i, right) and [eps_sL | a1] (system 2i+1, left); optionally subtract from
// a0 instead (residual check): [a0 - Sigma_R | am1], [a0 - Sigma_L | a1].
__global__ void k_dec_final_form(DecArgs a, double2 *M2, const double2 *sigma, int residual) {
  const int sys = blockIdx.y, inst = sys >> 1, side = sys & 1;  // side 0 = right, 1 = left
  const int s = a.s;
  const int ks = dec_set(a, inst);
  const double e = a.E[inst];
  const long ss2 = (long)s * s;
  const double2 *h00 = dec_cell(a, ks, 0), *s00 = dec_cell(a, ks, 2);
  const double2 *h01 = dec_cell(a, ks, 1), *s01 = dec_cell(a, ks, 3);
  const double2 *src = dec_mat(a, inst, side == 0 ? kEpsS : kEpsL);
  const double2 *sig = sigma + ((long)inst * 2 + (side == 0 ? 1 : 0)) * ss2;
  double2 *M = M2 + (long)sys * 2 * ss2;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < ss2; idx += (long)gridDim.x * blockDim.x) {
    const int r = idx / s, c = idx % s;
    double2 left;
    if (residual) {
      const double2 hv = h00[idx], sv = s00[idx];
      const double2 a0 = make_double2(e * sv.x - a.eta * sv.y - hv.x, e * sv.y + a.eta * sv.x - hv.y);
      left = csub(a0, sig[idx]);
    } else {
      left = src[idx];
    }
    double2 rhs;
    if (side == 0) {  // am1(r, c) = conj(a1(c, r))
      const long t = (long)c * s + r;
      rhs = make_double2(e * s01[t].x - h01[t].x, -(e * s01[t].y - h01[t].y));
    } else {
      rhs = make_double2(e * s01[idx].x - h01[idx].x, e * s01[idx].y - h01[idx].y);
    }
    M[(long)r * 2 * s + c] = left;
    M[(long)r * 2 * s + s + c] = rhs;
  }
}

// Sigma_R = a1 W_R (system 2i), Sigma_L = am1 W_L (system 2i+1).  residual != 0: instead accumulate
// ||Sigma - a W||_F^2 and ||Sigma||_F^2 into acc2[sys][2].
__global__ void __launch_bounds__(DecTile::NT) SS_TILE_WAVES k_dec_sigma(DecArgs a, const double2 *Wsol, double2 *sigma,
                                                           double *acc2, int residual) {
  using T = DecTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int sys = blockIdx.y, inst = sys >> 1, side = sys & 1;
  const int s = a.s;
  const int ks = dec_set(a, inst);
  const double e = a.E[inst];
  const long ss2 = (long)s * s;
  const int tiles = cdiv(s, T::BM);
  const int m0 = (blockIdx.x / tiles) * T::BM, n0 = (blockIdx.x % tiles) * T::BN;
  const double2 *w = Wsol + (long)sys * ss2;
  double2 *sig = sigma + ((long)inst * 2 + (side == 0 ? 1 : 0)) * ss2;
  LdRow lb{w, s};
  Acc<T> acc;
  acc.zero();
  if (side == 0) {
    LdForm<false> la{dec_cell(a, ks, 1), dec_cell(a, ks, 3), s, e};
    mma_loop<T>(la, lb, m0, s, n0, s, 0, s, acc, lds);
  } else {
    LdForm<true> la{dec_cell(a, ks, 1), dec_cell(a, ks, 3), s, e};
    mma_loop<T>(la, lb, m0, s, n0, s, 0, s, acc, lds);
  }
  double d2 = 0.0, n2 = 0.0;
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) {
      const long o = (long)gr * s + gc;
      if (residual) {
        const double2 sv = sig[o];
        const double2 df = csub(sv, v);
        d2 += df.x * df.x + df.y * df.y;
        n2 += sv.x * sv.x + sv.y * sv.y;
      } else {
        sig[o] = v;
      }
    }
  });
  if (residual) {
    for (int off = 32; off >= 1; off >>= 1) {
      d2 += __shfl_xor(d2, off);
      n2 += __shfl_xor(n2, off);
    }
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(acc2 + 2 * sys, d2);
      atomicAdd(acc2 + 2 * sys + 1, n2);
    }
  }
}

__global__ void k_zero_d(double *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void k_dec_finish(DecArgs a, const double *acc2, int *iters, double *resid, int *info) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= a.batch) return;
  if (iters) iters[inst] = a.iters[inst];
  if (resid) {
    // acc2 rows: system 2i = right, 2i+1 = left; output order (left, right)
    const double dr = acc2[4 * inst], nr = acc2[4 * inst + 1];
    const double dl = acc2[4 * inst + 2], nl = acc2[4 * inst + 3];
    resid[2 * inst] = sqrt(dl) / fmax(sqrt(nl), 1e-300);
    resid[2 * inst + 1] = sqrt(dr) / fmax(sqrt(nr), 1e-300);
  }
  if (info) info[inst] = a.done[inst] ? a.code[inst] : -1;
}

ss_status lead_selfenergy(ss_ctx *ctx, int batch, int s, int nk, const ss_c128 *H00, const ss_c128 *H01,
                          const ss_c128 *S00, const ss_c128 *S01, const int *kidx, const double *E,
                          double eta, double tol, int max_iter, ss_c128 *sigma, int *iters, double *resid,
                          int *info, const ss_c128 *const *tab) {
  const long ss2 = (long)s * s;
  if (tol <= 0) tol = 1e-14;
  if (max_iter <= 0) max_iter = 200;
  // workspace: state 7 s^2 + M 3 s^2 + Y 2 s^2 per instance; final solves reuse M/Y (2 x 2 s^2 each)
  void *wD, *wP, *wZ, *wMisc;
  const size_t per = (size_t)12 * ss2;
  SS_TRY(workspace(ctx, kSlotDec, sizeof(double2) * per * batch, &wD));
  SS_TRY(workspace(ctx, kSlotPerm, sizeof(int) * (size_t)2 * batch * s, &wP));
  SS_TRY(workspace(ctx, kSlotZp, sizeof(int) * (size_t)2 * batch, &wZ));
  const size_t misc_bytes = (size_t)batch * (2 * 8 + 8 + 4 + 4 + 4) + 64 + (size_t)batch * 4 * 8;
  SS_TRY(workspace(ctx, kSlotMisc, misc_bytes, &wMisc));

  DecArgs a;
  a.H00 = (const double2 *)H00;
  a.H01 = (const double2 *)H01;
  a.S00 = (const double2 *)S00;
  a.S01 = (const double2 *)S01;
  a.tab = (const double2 *const *)tab;
  a.kidx = kidx;
  a.E = E;
  a.eta = eta;
  a.nk = nk;
  a.s = s;
  a.batch = batch;
  a.st = (double2 *)wD;
  a.M = a.st + (size_t)7 * ss2 * batch;
  a.Y = a.M + (size_t)3 * ss2 * batch;
  char *mp = (char *)wMisc;
  a.nrm = (unsigned long long *)mp;
  mp += (size_t)batch * 16;
  a.scale = (double *)mp;
  mp += (size_t)batch * 8;
  double *acc2 = (double *)mp;
  mp += (size_t)batch * 32;
  a.done = (int *)mp;
  mp += (size_t)batch * 4;
  a.iters = (int *)mp;
  mp += (size_t)batch * 4;
  a.code = (int *)mp;
  mp += (size_t)batch * 4;
  a.ndone = (int *)mp;
  a.zp = (int *)wZ;
  a.tol = tol;

  hipLaunchKernelGGL(k_dec_reset, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, a);
  const int eblocks = std::min(cdiv((int)std::min<long>(ss2, 1 << 30), 256), 64);
  hipLaunchKernelGGL(k_dec_init, dim3(eblocks, batch), dim3(256), 0, ctx->stream, a);

  LuDesc d;
  d.nmat = batch;
  d.n = s;
  d.nrhs = 2 * s;
  d.M = a.M;
  d.sM = 3 * ss2;
  d.ldm = 3 * s;
  d.perm = (int *)wP;
  d.sP = s;
  d.zp = a.zp;
  d.X = a.Y;
  d.sX = 2 * ss2;
  d.ldx = 2 * s;
  d.skip = a.done;
  d.skip_shift = 0;

  const int tiles = cdiv(s, DecTile::BM);
  int *hostDone = nullptr;
  SS_TRY(host_word(ctx, &hostDone));
  ss_status st = SS_OK;
  for (int it = 0; it < max_iter; ++it) {
    if ((st = lu_identity_perm(ctx, d)) != SS_OK) break;
    if ((st = lu_solve(ctx, d)) != SS_OK) break;
    {
      KernelScope ks_(ctx, "dec_update");
      hipLaunchKernelGGL(k_dec_update, dim3(tiles * tiles, batch), dim3(DecTile::NT), 0, ctx->stream, a, it & 1);
    }
    hipLaunchKernelGGL(k_dec_check, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, a, it);
    // every few passes, stop early once every instance has converged (unless the context must not
    // wait for its stream: then all max_iter passes are enqueued and converged instances skip them)
    if (!ctx->sync_free && it >= 3 && (it % 4 == 3)) {
      if (hipMemcpyAsync(hostDone, a.ndone, sizeof(int), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
          hipStreamSynchronize(ctx->stream) != hipSuccess) {
        st = fail(ctx, SS_ERR_DEVICE, "lead_selfenergy: convergence poll");
        break;
      }
      if (*hostDone >= batch) break;
    }
  }
  SS_TRY(st);

  // Sigma from the converged surfaces, then the fixed-point residuals.  The 2 systems per instance
  // ([s][2s] each) fit in the contiguous (M, Y) region of 5 s^2 per instance.
  double2 *Wsol;
  SS_TRY(workspace(ctx, kSlotObc, sizeof(double2) * (size_t)2 * batch * ss2, (void **)&Wsol));
  LuDesc f = d;
  f.nmat = 2 * batch;
  f.nrhs = s;
  f.M = a.M;
  f.sM = 2 * ss2;
  f.ldm = 2 * s;
  f.X = Wsol;
  f.sX = ss2;
  f.ldx = s;
  f.skip = nullptr;
  hipLaunchKernelGGL(k_dec_final_form, dim3(eblocks, 2 * batch), dim3(256), 0, ctx->stream, a, a.M,
                     (const double2 *)sigma, 0);
  SS_TRY(lu_identity_perm(ctx, f));
  SS_TRY(lu_solve(ctx, f));
  hipLaunchKernelGGL(k_dec_sigma, dim3(tiles * tiles, 2 * batch), dim3(DecTile::NT), 0, ctx->stream, a, Wsol,
                     (double2 *)sigma, acc2, 0);
  if (resid) {
    hipLaunchKernelGGL(k_zero_d, dim3(cdiv(4 * batch, 256)), dim3(256), 0, ctx->stream, acc2, 4 * batch);
    hipLaunchKernelGGL(k_dec_final_form, dim3(eblocks, 2 * batch), dim3(256), 0, ctx->stream, a, a.M,
                       (const double2 *)sigma, 1);
    SS_TRY(lu_identity_perm(ctx, f));
    SS_TRY(lu_solve(ctx, f));
    hipLaunchKernelGGL(k_dec_sigma, dim3(tiles * tiles, 2 * batch), dim3(DecTile::NT), 0, ctx->stream, a, Wsol,
                       (double2 *)sigma, acc2, 1);
  }
  hipLaunchKernelGGL(k_dec_finish, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, a, acc2, iters, resid, info);
  return check_launch(ctx, "lead_selfenergy");
}

}  // namespace ss
