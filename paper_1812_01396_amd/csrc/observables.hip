// Observables from the wave function over the (E, k) grid (Sec. 2B: the charge and current densities
// follow from c(E) once Eq. (wf) is solved at every energy and momentum; Sec. 5C shows the electron
// distribution, the current map and the spectral current).
//
// For psi injected from the left lead (psi psi^H = G Gamma_L G^H), per instance:
//     density  n_mu = Re sum_c psi_{mu c} conj((S psi)_{mu c})       (Mulliken: Re (psi psi^H S)_{mu mu})
//     current  J_i  = 2 Im Tr[psi_i^H A_{i,i+1} psi_{i+1}],  A_{i,i+1} = E S_{i,i+1} - H_{i,i+1}
// (S psi)_i = S_{i,i-1} psi_{i-1} + S_ii psi_i + S_{i,i+1} psi_{i+1} and A_{i,i+1} psi_{i+1} are products of
// an s x s block with the s x m block of psi on the FP64 matrix cores; the epilogues reduce them against
// psi_i in registers, so nothing of size s x m is written back.  Inside the device the rows of
// (E S - H) psi vanish, so J_i is the same at every interface (current conservation) and, for b' = [W_L; 0],
// equals T_RL.  The energy integral is a weighted sum over instances with the caller's quadrature weights.
#include "drivers.hpp"
#include "tile.hpp"

namespace ss {

// psi has as many columns as injected modes (typically 32): 64 x 32 tiles of four waves
using ObsTile = TileCfgG3<64, 32, 16, 4, 1>;

struct LdHerm {  // element (r, c) of P^H for row-major P: conj(p[c * ld + r])
  const double2 *p;
  long ld;
  static constexpr bool kFastSecond = false;
  __device__ __forceinline__ double2 operator()(int r, int c) const { return cconj(p[(long)c * ld + r]); }
};

struct ObsArgs {
  const double2 *Hd, *Hu, *Sd, *Su;
  long kstride_d, kstride_u;
  const int *kidx;
  const double *E;
  int nk, nb, s, m, batch;
  const double2 *psi;  // [batch][nb][s][m]
  double *density;     // [batch][nb][s]
  double *current;     // [batch][nb - 1]
};

__device__ __forceinline__ int obs_set(const ObsArgs &a, int inst) {
  const int k = a.kidx ? a.kidx[inst] : inst % a.nk;
  return min(max(k, 0), a.nk - 1);
}

__global__ void k_obs_zero(double *p, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0.0;
}

// grid (tiles(s) * tiles(m), nb, batch)
__global__ void __launch_bounds__(ObsTile::NT) SS_TILE_WAVES_OF(ObsTile) k_obs_density(ObsArgs a) {
  using T = ObsTile;
  __shared__ double lds[T::LDS_DOUBLES];
  __shared__ double rowsum[T::BM];
  const int inst = blockIdx.z, i = blockIdx.y;
  const int s = a.s, m = a.m, nb = a.nb;
  const int tc = cdiv(m, T::BN);
  const int m0 = (blockIdx.x / tc) * T::BM, n0 = (blockIdx.x % tc) * T::BN;
  const int ks = obs_set(a, inst);
  const long ss2 = (long)s * s, sm = (long)s * m;
  const double2 *x = a.psi + (long)inst * nb * sm;
  for (int r = threadIdx.x; r < T::BM; r += T::NT) rowsum[r] = 0.0;
  Acc<T> acc;
  acc.zero();
  {
    LdRow la{a.Sd + ks * a.kstride_d + i * ss2, s};
    LdRow lb{x + i * sm, m};
    mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  }
  if (i < nb - 1) {  // S_{i,i+1} psi_{i+1}
    LdRow la{a.Su + ks * a.kstride_u + i * ss2, s};
    LdRow lb{x + (i + 1) * sm, m};
    mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  }
  if (i > 0) {  // S_{i,i-1} psi_{i-1} = S_u[i-1]^H psi_{i-1}
    LdHerm la{a.Su + ks * a.kstride_u + (i - 1) * ss2, s};
    LdRow lb{x + (i - 1) * sm, m};
    mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  }
  __syncthreads();  // rowsum cleared before any lane adds to it
  const double2 *xi = x + i * sm;
  acc_foreach<T>(acc, [&](int rl, int cl, double2 v) {
    const int gr = m0 + rl, gc = n0 + cl;
    if (gr < s && gc < m) {
      const double2 p = xi[(long)gr * m + gc];
      atomicAdd(&rowsum[rl], p.x * v.x + p.y * v.y);
    }
  });
  __syncthreads();
  double *dn = a.density + ((long)inst * nb + i) * s;
  for (int r = threadIdx.x; r < T::BM; r += T::NT)
    if (m0 + r < s) {
      if (tc == 1) dn[m0 + r] = rowsum[r];
      else atomicAdd(dn + m0 + r, rowsum[r]);
    }
}

// grid (tiles(s) * tiles(m), nb - 1, batch)
__global__ void __launch_bounds__(ObsTile::NT) SS_TILE_WAVES_OF(ObsTile) k_obs_current(ObsArgs a) {
  using T = ObsTile;
  __shared__ double lds[T::LDS_DOUBLES];
  __shared__ double red[T::NT / 64];
  const int inst = blockIdx.z, i = blockIdx.y;
  const int s = a.s, m = a.m, nb = a.nb;
  const int tc = cdiv(m, T::BN);
  const int m0 = (blockIdx.x / tc) * T::BM, n0 = (blockIdx.x % tc) * T::BN;
  const int ks = obs_set(a, inst);
  const double e = a.E[inst];
  const long ss2 = (long)s * s, sm = (long)s * m;
  const double2 *x = a.psi + (long)inst * nb * sm;
  Acc<T> acc;
  acc.zero();
  LdForm<false> la{a.Hu + ks * a.kstride_u + i * ss2, a.Su + ks * a.kstride_u + i * ss2, s, e};
  LdRow lb{x + (i + 1) * sm, m};
  mma_loop<T>(la, lb, m0, s, n0, m, 0, s, acc, lds);
  const double2 *xi = x + i * sm;
  double t = 0.0;
  acc_foreach<T>(acc, [&](int rl, int cl, double2 v) {
    const int gr = m0 + rl, gc = n0 + cl;
    if (gr < s && gc < m) {
      const double2 p = xi[(long)gr * m + gc];
      t += p.x * v.y - p.y * v.x;  // Im(conj(p) v)
    }
  });
  for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < T::NT / 64; ++w) sum += red[w];
    atomicAdd(a.current + (long)inst * (nb - 1) + i, 2.0 * sum);
  }
}

// out[j] = sum_b w[b] x[b][j], in instance order (one thread per j)
__global__ void k_energy_integral(int batch, int n, const double *w, const double *x, double *out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double t = 0.0;
  for (int b = 0; b < batch; ++b) t += w[b] * x[(long)b * n + j];
  out[j] = t;
}

ss_status observables(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E, int m,
                      const ss_c128 *psi, double *density, double *current) {
  const int s = hs->s, nb = hs->nb;
  const long ss2 = (long)s * s;
  ObsArgs a;
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
  a.psi = (const double2 *)psi;
  a.density = density;
  a.current = current;
  using T = ObsTile;
  const int tiles = cdiv(s, T::BM) * cdiv(m, T::BN);
  if (density) {
    const long n = (long)batch * nb * s;
    if (cdiv(m, T::BN) > 1)  // several column tiles add into one row
      hipLaunchKernelGGL(k_obs_zero, dim3((int)std::min<long>(cdiv((int)std::min<long>(n, 1L << 30), 256), 4096)),
                         dim3(256), 0, ctx->stream, density, n);
    KernelScope ks_(ctx, "obs");
    hipLaunchKernelGGL(k_obs_density, dim3(tiles, nb, batch), dim3(T::NT), 0, ctx->stream, a);
  }
  if (current && nb > 1) {
    const long n = (long)batch * (nb - 1);
    hipLaunchKernelGGL(k_obs_zero, dim3((int)std::min<long>(cdiv((int)std::min<long>(n, 1L << 30), 256), 4096)),
                       dim3(256), 0, ctx->stream, current, n);
    KernelScope ks_(ctx, "obs");
    hipLaunchKernelGGL(k_obs_current, dim3(tiles, nb - 1, batch), dim3(T::NT), 0, ctx->stream, a);
  }
  return check_launch(ctx, "observables");
}

ss_status energy_integral(ss_ctx *ctx, int batch, int n, const double *w, const double *x, double *out) {
  hipLaunchKernelGGL(k_energy_integral, dim3(cdiv(n, 256)), dim3(256), 0, ctx->stream, batch, n, w, x, out);
  return check_launch(ctx, "energy_integral");
}

}  // namespace ss
