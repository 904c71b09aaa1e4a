// Warm-started self-energies: Newton's method on the fixed-point equation from a given starting iterate,
// judged by its residual and by retardedness, with the decimation as fallback.
//
// For the left lead (c = am1, c' = a1) and the right lead (c = a1, c' = am1) of every instance:
//     g = (a0 - Sigma)^{-1},  N = g c',  M = c g,  F = Sigma - c N
//     Newton step: D - M D N = -F (Stein equation), Sigma <- Sigma + D
// The Stein equation is solved by Smith's doubling, D = sum_k M^k (-F) N^k summed in 2^j terms:
//     D += M_j D N_j,  M_{j+1} = (c_j M_j)^2,  N_{j+1} = (N_j / c_j)^2
// with c_j = sqrt(|N_j| / |M_j|) keeping the two powers balanced (every term M_j X N_j is unchanged).
// A side is accepted when ||F||_F <= tol ||Sigma||_F and its propagator -N has spectral radius below
// 1 + 1e-8 (the retarded root; other roots of the quadratic have a growing mode).  The radius is read
// from J normalised squarings: log ||N^(2^J)|| / 2^J.  Instances with a side that fails either test are
// recomputed by the decimation.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "drivers.hpp"
#include "lu.hpp"
#include "tile.hpp"

namespace ss {

namespace {

using WTile = TileCfg<64, 64, 16, 2, 2>;

struct WarmArgs {
  const double2 *H00, *H01, *S00, *S01;  // [nk][s][s]
  const int *kidx;
  const double *E;
  double eta;
  int nk, s, nsys;
  double2 *sig;  // [nsys][s][s] = the output sigma [batch][2][s][s] (L, R)
  double2 *aug;  // [nsys][s][3s]
  double2 *X;    // [nsys][s][2s]: [N | g]
  double2 *Mm, *D, *T;
  double2 *Mp[2], *Np[2];
  double *nrm;   // [nsys][8]: |F|^2, |Sigma|^2, |term|^2, |D|^2, |M|^2, |N|^2, log-norm, spare
  double *bal;   // [nsys] balance factor c_j^2 of the current doubling
  int *state;    // [nsys]: 0 Newton running, 1 converged, 2 failed
  int *sstate;   // [nsys]: 0 Smith running, 1 done, 2 diverged
  int *iters;    // [nsys]
  double tol;
};

__device__ __forceinline__ int wset(const WarmArgs &a, int inst) {
  const int k = a.kidx ? a.kidx[inst] : inst % a.nk;
  return min(max(k, 0), a.nk - 1);
}
__device__ __forceinline__ double2 *wmat(double2 *base, const WarmArgs &a, int sys) {
  return base + (long)sys * a.s * a.s;
}

__device__ __forceinline__ void wave_sum_add(double *dst, double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(dst, v);
}

// [a0 - Sigma | c' | I] for every running system
__global__ void k_warm_form(WarmArgs a) {
  const int sys = blockIdx.y, inst = sys >> 1, right = sys & 1;
  if (a.state[sys] != 0) return;
  const int s = a.s, ks = wset(a, inst);
  const double e = a.E[inst];
  const long ss2 = (long)s * s;
  const double2 *h00 = a.H00 + ks * ss2, *s00 = a.S00 + ks * ss2, *h01 = a.H01 + ks * ss2, *s01 = a.S01 + ks * ss2;
  const double2 *sg = wmat(a.sig, a, sys);
  double2 *M = a.aug + (long)sys * 3 * ss2;
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // norms of the Smith start are accumulated afresh
    a.nrm[8 * sys + 4] = 0.0;
    a.nrm[8 * sys + 5] = 0.0;
  }
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < ss2; idx += (long)gridDim.x * blockDim.x) {
    const int r = idx / s, c = idx % s;
    const double2 hv = h00[idx], sv = s00[idx];
    const double2 a0 = make_double2(e * sv.x - a.eta * sv.y - hv.x, e * sv.y + a.eta * sv.x - hv.y);
    double2 cp;
    if (right) {  // c' = am1 = a1^H
      const long t = (long)c * s + r;
      cp = make_double2(e * s01[t].x - h01[t].x, -(e * s01[t].y - h01[t].y));
    } else {  // c' = a1
      cp = make_double2(e * s01[idx].x - h01[idx].x, e * s01[idx].y - h01[idx].y);
    }
    M[(long)r * 3 * s + c] = csub(a0, sg[idx]);
    M[(long)r * 3 * s + s + c] = cp;
    M[(long)r * 3 * s + 2 * s + c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
}

// D = c N - Sigma (= -F), |F|^2, |Sigma|^2; Mm = c g; Smith start M_0 = Mm, N_0 = N with their norms
__global__ void __launch_bounds__(WTile::NT) k_warm_mf(WarmArgs a) {
  using T = WTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int sys = blockIdx.y, inst = sys >> 1, right = sys & 1;
  if (a.state[sys] != 0) return;
  const int s = a.s, ks = wset(a, inst);
  const double e = a.E[inst];
  const long ss2 = (long)s * s;
  const int tiles = cdiv(s, T::BM);
  const int m0 = (blockIdx.x / tiles) * T::BM, n0 = (blockIdx.x % tiles) * T::BN;
  const double2 *X = a.X + (long)sys * 2 * ss2;
  const double2 *sg = wmat(a.sig, a, sys);
  double2 *D = wmat(a.D, a, sys), *Mm = wmat(a.Mm, a, sys), *M0 = wmat(a.Mp[0], a, sys), *N0 = wmat(a.Np[0], a, sys);
  double *nr = a.nrm + 8 * sys;
  const double2 *h01 = a.H01 + ks * ss2, *s01 = a.S01 + ks * ss2;
  LdRow lbN{X, 2 * s}, lbG{X + s, 2 * s};
  Acc<T> acc;
  double f2 = 0.0, s2 = 0.0, n2 = 0.0, m2 = 0.0;
  // c N
  acc.zero();
  if (right) mma_loop<T>(LdForm<false>{h01, s01, s, e}, lbN, m0, s, n0, s, 0, s, acc, lds);
  else mma_loop<T>(LdForm<true>{h01, s01, s, e}, lbN, m0, s, n0, s, 0, s, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) {
      const long o = (long)gr * s + gc;
      const double2 sv = sg[o], d = csub(v, sv), nv = X[(long)gr * 2 * s + gc];
      D[o] = d;
      N0[o] = nv;
      f2 += d.x * d.x + d.y * d.y;
      s2 += sv.x * sv.x + sv.y * sv.y;
      n2 += nv.x * nv.x + nv.y * nv.y;
    }
  });
  // c g
  acc.zero();
  if (right) mma_loop<T>(LdForm<false>{h01, s01, s, e}, lbG, m0, s, n0, s, 0, s, acc, lds);
  else mma_loop<T>(LdForm<true>{h01, s01, s, e}, lbG, m0, s, n0, s, 0, s, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) {
      const long o = (long)gr * s + gc;
      Mm[o] = v;
      M0[o] = v;
      m2 += v.x * v.x + v.y * v.y;
    }
  });
  wave_sum_add(nr + 0, f2);
  wave_sum_add(nr + 1, s2);
  wave_sum_add(nr + 4, m2);
  wave_sum_add(nr + 5, n2);
}

// residual test after the products; starts Smith for the systems that go on
__global__ void k_warm_check(WarmArgs a, int it, int max_newton) {
  const int sys = blockIdx.x * blockDim.x + threadIdx.x;
  if (sys >= a.nsys || a.state[sys] != 0) return;
  double *nr = a.nrm + 8 * sys;
  const double f = sqrt(nr[0]), sn = sqrt(nr[1]);
  const double rel = f / fmax(sn, 1e-300);
  a.iters[sys] = it;
  nr[6] = rel;  // kept for the caller
  nr[0] = nr[1] = nr[2] = nr[3] = 0.0;
  if (!(rel == rel) || rel > 1e30) {
    a.state[sys] = 2;
  } else if (rel <= a.tol) {
    a.state[sys] = 1;
  } else if (it >= max_newton) {
    a.state[sys] = 2;
  } else {
    a.sstate[sys] = 0;
  }
}

// T = D N_j
__global__ void __launch_bounds__(WTile::NT) SS_TILE_WAVES k_smith_t(WarmArgs a, int par) {
  using T = WTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int sys = blockIdx.y;
  if (a.state[sys] != 0 || a.sstate[sys] != 0) return;
  const int s = a.s, tiles = cdiv(s, T::BM);
  const int m0 = (blockIdx.x / tiles) * T::BM, n0 = (blockIdx.x % tiles) * T::BN;
  Acc<T> acc;
  acc.zero();
  mma_loop<T>(LdRow{wmat(a.D, a, sys), s}, LdRow{wmat(a.Np[par], a, sys), s}, m0, s, n0, s, 0, s, acc, lds);
  double2 *Tm = wmat(a.T, a, sys);
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) Tm[(long)gr * s + gc] = v;
  });
}

// D += M_j T with |term|^2 and |D|^2
__global__ void __launch_bounds__(WTile::NT) SS_TILE_WAVES k_smith_term(WarmArgs a, int par) {
  using T = WTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int sys = blockIdx.y;
  if (a.state[sys] != 0 || a.sstate[sys] != 0) return;
  const int s = a.s, tiles = cdiv(s, T::BM);
  const int m0 = (blockIdx.x / tiles) * T::BM, n0 = (blockIdx.x % tiles) * T::BN;
  Acc<T> acc;
  acc.zero();
  mma_loop<T>(LdRow{wmat(a.Mp[par], a, sys), s}, LdRow{wmat(a.T, a, sys), s}, m0, s, n0, s, 0, s, acc, lds);
  double2 *D = wmat(a.D, a, sys);
  double t2 = 0.0, d2 = 0.0;
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) {
      const long o = (long)gr * s + gc;
      const double2 nd = cadd(D[o], v);
      D[o] = nd;
      t2 += v.x * v.x + v.y * v.y;
      d2 += nd.x * nd.x + nd.y * nd.y;
    }
  });
  double *nr = a.nrm + 8 * sys;
  wave_sum_add(nr + 2, t2);
  wave_sum_add(nr + 3, d2);
}

// Smith bookkeeping after a doubling: done when the block of terms is negligible, diverged when it blows
// up; otherwise the balance factor for the squaring
__global__ void k_smith_check(WarmArgs a, int last) {
  const int sys = blockIdx.x * blockDim.x + threadIdx.x;
  if (sys >= a.nsys || a.state[sys] != 0 || a.sstate[sys] != 0) return;
  double *nr = a.nrm + 8 * sys;
  const double t = sqrt(nr[2]), d = sqrt(nr[3]);
  nr[2] = nr[3] = 0.0;
  if (!(t == t) || !(d == d) || t > 1e10 * d) {
    a.sstate[sys] = 2;
    a.state[sys] = 2;
    return;
  }
  if (t <= 1e-16 * d || last) {
    a.sstate[sys] = 1;
    return;
  }
  const double mn = sqrt(nr[4]), nn = sqrt(nr[5]);
  a.bal[sys] = (mn > 0.0 && nn > 0.0) ? nn / mn : 1.0;  // c^2
  nr[4] = nr[5] = 0.0;
}

// M_{j+1} = c^2 M_j^2, N_{j+1} = N_j^2 / c^2 with their norms
__global__ void __launch_bounds__(WTile::NT) SS_TILE_WAVES k_smith_square(WarmArgs a, int par) {
  using T = WTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int sys = blockIdx.y;
  if (a.state[sys] != 0 || a.sstate[sys] != 0) return;
  const int s = a.s, tiles = cdiv(s, T::BM);
  const int m0 = (blockIdx.x / tiles) * T::BM, n0 = (blockIdx.x % tiles) * T::BN;
  const double c2 = a.bal[sys];
  double *nr = a.nrm + 8 * sys;
  Acc<T> acc;
  double m2 = 0.0, n2 = 0.0;
  acc.zero();
  const double2 *Mj = wmat(a.Mp[par], a, sys), *Nj = wmat(a.Np[par], a, sys);
  double2 *Mn = wmat(a.Mp[par ^ 1], a, sys), *Nn = wmat(a.Np[par ^ 1], a, sys);
  mma_loop<T>(LdRow{Mj, s}, LdRow{Mj, s}, m0, s, n0, s, 0, s, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) {
      const double2 w = make_double2(v.x * c2, v.y * c2);
      Mn[(long)gr * s + gc] = w;
      m2 += w.x * w.x + w.y * w.y;
    }
  });
  acc.zero();
  mma_loop<T>(LdRow{Nj, s}, LdRow{Nj, s}, m0, s, n0, s, 0, s, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) {
      const double2 w = make_double2(v.x / c2, v.y / c2);
      Nn[(long)gr * s + gc] = w;
      n2 += w.x * w.x + w.y * w.y;
    }
  });
  wave_sum_add(nr + 4, m2);
  wave_sum_add(nr + 5, n2);
}

// Newton update for the systems whose Stein solve finished
__global__ void k_warm_update(WarmArgs a) {
  const int sys = blockIdx.y;
  if (a.state[sys] != 0 || a.sstate[sys] != 1) return;
  const long ss2 = (long)a.s * a.s;
  double2 *sg = wmat(a.sig, a, sys);
  const double2 *D = wmat(a.D, a, sys);
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < ss2; idx += (long)gridDim.x * blockDim.x)
    sg[idx] = cadd(sg[idx], D[idx]);
}

// ---- retardedness: spectral radius of N from normalised squarings

// P_0 = N / |N|, logn = log |N| (N of the converged iterate is the left block of X)
__global__ void k_pow_init(WarmArgs a) {
  const int sys = blockIdx.y;
  if (a.state[sys] != 1) return;
  const int s = a.s;
  const long ss2 = (long)s * s;
  const double2 *X = a.X + (long)sys * 2 * ss2;
  double2 *P = wmat(a.Np[0], a, sys);
  const double inv = 1.0 / fmax(sqrt(a.nrm[8 * sys + 5]), 1e-300);
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < ss2; idx += (long)gridDim.x * blockDim.x) {
    const double2 v = X[(idx / s) * 2 * s + idx % s];
    P[idx] = make_double2(v.x * inv, v.y * inv);
  }
}

__global__ void k_pow_norm_init(WarmArgs a) {
  const int sys = blockIdx.x * blockDim.x + threadIdx.x;
  if (sys >= a.nsys || a.state[sys] != 1) return;
  a.nrm[8 * sys + 7] = log(fmax(sqrt(a.nrm[8 * sys + 5]), 1e-300));  // log |N|
  a.nrm[8 * sys + 4] = 0.0;
}

// Q = P^2 (unnormalised), |Q|^2
__global__ void __launch_bounds__(WTile::NT) SS_TILE_WAVES k_pow_square(WarmArgs a, int par) {
  using T = WTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int sys = blockIdx.y;
  if (a.state[sys] != 1) return;
  const int s = a.s, tiles = cdiv(s, T::BM);
  const int m0 = (blockIdx.x / tiles) * T::BM, n0 = (blockIdx.x % tiles) * T::BN;
  const double2 *P = wmat(a.Np[par], a, sys);
  double2 *Q = wmat(a.Np[par ^ 1], a, sys);
  Acc<T> acc;
  acc.zero();
  mma_loop<T>(LdRow{P, s}, LdRow{P, s}, m0, s, n0, s, 0, s, acc, lds);
  double q2 = 0.0;
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) {
      Q[(long)gr * s + gc] = v;
      q2 += v.x * v.x + v.y * v.y;
    }
  });
  wave_sum_add(a.nrm + 8 * sys + 4, q2);
}

// logn <- 2 logn + log |Q|; P <- Q / |Q|
__global__ void k_pow_normalise(WarmArgs a, int par) {
  const int sys = blockIdx.y;
  if (a.state[sys] != 1) return;
  const long ss2 = (long)a.s * a.s;
  const double q = sqrt(a.nrm[8 * sys + 4]);
  const double inv = 1.0 / fmax(q, 1e-300);
  double2 *Q = wmat(a.Np[par ^ 1], a, sys);
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < ss2; idx += (long)gridDim.x * blockDim.x)
    Q[idx] = make_double2(Q[idx].x * inv, Q[idx].y * inv);
}

__global__ void k_pow_log(WarmArgs a) {
  const int sys = blockIdx.x * blockDim.x + threadIdx.x;
  if (sys >= a.nsys || a.state[sys] != 1) return;
  double *nr = a.nrm + 8 * sys;
  nr[7] = 2.0 * nr[7] + log(fmax(sqrt(nr[4]), 1e-300));
  nr[4] = 0.0;
}

// accept or reject each instance; ok[inst] = 1 when both sides converged to a retarded root
__global__ void k_warm_judge(WarmArgs a, int J, int *ok, int *newton_iters, double *resid) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * inst >= a.nsys) return;
  bool good = true;
  int its = 0;
  for (int h = 0; h < 2; ++h) {
    const int sys = 2 * inst + h;
    const double *nr = a.nrm + 8 * sys;
    const double logrho = nr[7] / ldexp(1.0, J);
    good = good && a.state[sys] == 1 && logrho <= log1p(1e-8);
    its = max(its, a.iters[sys]);
    if (resid) resid[2 * inst + h] = nr[6];
  }
  ok[inst] = good ? 1 : 0;
  if (newton_iters) newton_iters[inst] = its;
}

__global__ void k_warm_init(WarmArgs a, const double2 *init) {
  const int sys = blockIdx.y;
  const long ss2 = (long)a.s * a.s;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < ss2; idx += (long)gridDim.x * blockDim.x)
    a.sig[(long)sys * ss2 + idx] = init[(long)sys * ss2 + idx];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.state[sys] = 0;
    a.sstate[sys] = 0;
    a.iters[sys] = 0;
    for (int q = 0; q < 8; ++q) a.nrm[8 * sys + q] = 0.0;
    a.bal[sys] = 1.0;
  }
}

__global__ void k_count_state(const int *state, int n, int *count) {
  __shared__ int c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (state[i] == 0) atomicAdd(&c, 1);
  __syncthreads();
  if (threadIdx.x == 0) *count = c;
}

// compact the rejected instances for the fallback
__global__ void k_gather_rejected(const int *ok, int batch, const int *kidx, const double *E, int *list, int *kk,
                                  double *ee, int *count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int c = 0;
  for (int i = 0; i < batch; ++i)
    if (!ok[i]) {
      list[c] = i;
      kk[c] = kidx ? kidx[i] : i;
      ee[c] = E[i];
      ++c;
    }
  *count = c;
}

__global__ void k_scatter_fallback(const int *list, int count, long ss2, const double2 *sig_fb, const int *info_fb,
                                   const int *iters_fb, double2 *sigma, int *info, int *iters) {
  const int j = blockIdx.y;
  if (j >= count) return;
  const int inst = list[j];
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < 2 * ss2; idx += (long)gridDim.x * blockDim.x)
    sigma[(long)inst * 2 * ss2 + idx] = sig_fb[(long)j * 2 * ss2 + idx];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (info) info[inst] = info_fb[j] == 0 ? -2 : info_fb[j];
    if (iters) iters[inst] = iters_fb[j];
  }
}

__global__ void k_accept_info(const int *ok, int batch, int *info, int *dec_iters) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch || !ok[i]) return;
  if (info) info[i] = 0;
  if (dec_iters) dec_iters[i] = 0;
}

}  // namespace

ss_status lead_selfenergy_warm(ss_ctx *ctx, int batch, int s, int nk, const ss_c128 *H00, const ss_c128 *H01,
                               const ss_c128 *S00, const ss_c128 *S01, const int *kidx, const double *E, double eta,
                               const ss_c128 *sigma_init, double tol, int max_newton, int smith_steps,
                               ss_c128 *sigma, int *newton_iters, int *dec_iters, double *resid, int *info) {
  if (tol <= 0) tol = 1e-10;
  if (max_newton <= 0) max_newton = 8;
  if (smith_steps <= 0) smith_steps = 40;
  const int nsys = 2 * batch;
  const long ss2 = (long)s * s;
  constexpr int J = 40;  // squarings of the retardedness test
  void *wW, *wP, *wZ, *wMisc;
  // aug 3, X 2, Mm, D, T, M 2, N 2  = 12 s^2 per system
  SS_TRY(workspace(ctx, kSlotWarm, sizeof(double2) * (size_t)nsys * 12 * ss2, &wW));
  SS_TRY(workspace(ctx, kSlotPerm, sizeof(int) * (size_t)nsys * s, &wP));
  SS_TRY(workspace(ctx, kSlotZp, sizeof(int) * (size_t)nsys, &wZ));
  const size_t misc = sizeof(double) * (size_t)nsys * 9 + sizeof(int) * (size_t)nsys * 3 + 64 +
                      sizeof(int) * (size_t)batch * 4 + sizeof(double) * (size_t)batch + 64;
  SS_TRY(workspace(ctx, kSlotWarmMisc, misc, &wMisc));
  WarmArgs a;
  a.H00 = (const double2 *)H00;
  a.H01 = (const double2 *)H01;
  a.S00 = (const double2 *)S00;
  a.S01 = (const double2 *)S01;
  a.kidx = kidx;
  a.E = E;
  a.eta = eta;
  a.nk = nk;
  a.s = s;
  a.nsys = nsys;
  a.sig = (double2 *)sigma;
  double2 *w = (double2 *)wW;
  a.aug = w;
  a.X = a.aug + (size_t)nsys * 3 * ss2;
  a.Mm = a.X + (size_t)nsys * 2 * ss2;
  a.D = a.Mm + (size_t)nsys * ss2;
  a.T = a.D + (size_t)nsys * ss2;
  a.Mp[0] = a.T + (size_t)nsys * ss2;
  a.Mp[1] = a.Mp[0] + (size_t)nsys * ss2;
  a.Np[0] = a.Mp[1] + (size_t)nsys * ss2;
  a.Np[1] = a.Np[0] + (size_t)nsys * ss2;
  char *mp = (char *)wMisc;
  a.nrm = (double *)mp;
  mp += sizeof(double) * (size_t)nsys * 8;
  a.bal = (double *)mp;
  mp += sizeof(double) * (size_t)nsys;
  a.state = (int *)mp;
  a.sstate = a.state + nsys;
  a.iters = a.sstate + nsys;
  int *dcount = a.iters + nsys;
  int *ok = dcount + 16;
  int *list = ok + batch;
  int *kk = list + batch;
  double *ee = (double *)(((uintptr_t)(kk + batch) + 7) & ~(uintptr_t)7);
  a.tol = tol;

  const int eblocks = std::min(cdiv((int)std::min<long>(ss2, 1 << 30), 256), 64);
  const int tiles = cdiv(s, WTile::BM);
  hipLaunchKernelGGL(k_warm_init, dim3(eblocks, nsys), dim3(256), 0, ctx->stream, a, (const double2 *)sigma_init);

  LuDesc d;
  d.nmat = nsys;
  d.n = s;
  d.nrhs = 2 * s;
  d.M = a.aug;
  d.sM = 3 * ss2;
  d.ldm = 3 * s;
  d.perm = (int *)wP;
  d.sP = s;
  d.zp = (int *)wZ;
  d.X = a.X;
  d.sX = 2 * ss2;
  d.ldx = 2 * s;
  d.skip = a.state;  // converged and failed systems skip the factorization
  d.skip_shift = 0;

  int *host = nullptr;
  SS_TRY(host_word(ctx, &host));
  for (int it = 0; it <= max_newton; ++it) {
    hipLaunchKernelGGL(k_warm_form, dim3(eblocks, nsys), dim3(256), 0, ctx->stream, a);
    SS_TRY(lu_identity_perm(ctx, d));
    SS_TRY(lu_solve(ctx, d));
    hipLaunchKernelGGL(k_warm_mf, dim3(tiles * tiles, nsys), dim3(WTile::NT), 0, ctx->stream, a);
    hipLaunchKernelGGL(k_warm_check, dim3(cdiv(nsys, 256)), dim3(256), 0, ctx->stream, a, it, max_newton);
    for (int j = 0; j < smith_steps; ++j) {
      const int par = j & 1;
      hipLaunchKernelGGL(k_smith_t, dim3(tiles * tiles, nsys), dim3(WTile::NT), 0, ctx->stream, a, par);
      hipLaunchKernelGGL(k_smith_term, dim3(tiles * tiles, nsys), dim3(WTile::NT), 0, ctx->stream, a, par);
      hipLaunchKernelGGL(k_smith_check, dim3(cdiv(nsys, 256)), dim3(256), 0, ctx->stream, a,
                         (int)(j == smith_steps - 1));
      if (j < smith_steps - 1)
        hipLaunchKernelGGL(k_smith_square, dim3(tiles * tiles, nsys), dim3(WTile::NT), 0, ctx->stream, a, par);
    }
    hipLaunchKernelGGL(k_warm_update, dim3(eblocks, nsys), dim3(256), 0, ctx->stream, a);
    // stop once no system is still running
    hipLaunchKernelGGL(k_count_state, dim3(1), dim3(256), 0, ctx->stream, (const int *)a.state, nsys, dcount);
    if (hipMemcpyAsync(host, dcount, sizeof(int), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      return fail(ctx, SS_ERR_DEVICE, "lead_selfenergy_warm: poll");
    if (*host == 0) break;
  }
  // retardedness of the converged sides
  hipLaunchKernelGGL(k_pow_norm_init, dim3(cdiv(nsys, 256)), dim3(256), 0, ctx->stream, a);
  hipLaunchKernelGGL(k_pow_init, dim3(eblocks, nsys), dim3(256), 0, ctx->stream, a);
  for (int j = 0; j < J; ++j) {
    const int par = j & 1;
    hipLaunchKernelGGL(k_pow_square, dim3(tiles * tiles, nsys), dim3(WTile::NT), 0, ctx->stream, a, par);
    hipLaunchKernelGGL(k_pow_normalise, dim3(eblocks, nsys), dim3(256), 0, ctx->stream, a, par);
    hipLaunchKernelGGL(k_pow_log, dim3(cdiv(nsys, 256)), dim3(256), 0, ctx->stream, a);
  }
  hipLaunchKernelGGL(k_warm_judge, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, a, J, ok, newton_iters, resid);
  hipLaunchKernelGGL(k_accept_info, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, (const int *)ok, batch, info,
                     dec_iters);
  // fallback: the decimation for every rejected instance
  hipLaunchKernelGGL(k_gather_rejected, dim3(1), dim3(64), 0, ctx->stream, (const int *)ok, batch, kidx, E, list, kk,
                     ee, dcount);
  if (hipMemcpyAsync(host, dcount, sizeof(int), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    return fail(ctx, SS_ERR_DEVICE, "lead_selfenergy_warm: rejected count");
  const int nrej = *host;
  if (nrej > 0) {
    // the rejected sigmas, infos and pass counts go to the (now free) Newton work area
    double2 *sig_fb = a.aug;
    int *info_fb = (int *)(a.X);
    int *iters_fb = info_fb + batch;
    SS_TRY(lead_selfenergy(ctx, nrej, s, nk, H00, H01, S00, S01, kk, ee, eta, 0.0, 0, (ss_c128 *)sig_fb, iters_fb,
                           nullptr, info_fb));
    hipLaunchKernelGGL(k_scatter_fallback, dim3(eblocks, nrej), dim3(256), 0, ctx->stream, (const int *)list, nrej, ss2,
                       (const double2 *)sig_fb, (const int *)info_fb, (const int *)iters_fb, (double2 *)sigma, info,
                       dec_iters);
  }
  return check_launch(ctx, "lead_selfenergy_warm");
}

}  // namespace ss
