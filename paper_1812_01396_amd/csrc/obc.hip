// Post-processing of SplitSolve (Sec. 3B, Eq. (x) and Steps 2-4) and the Caroli transmission.
//
// With B = [I 0 ... 0; 0 ... 0 I]^T (N x 2s), C = [Sigma_L 0 ...; ... 0 Sigma_R] (2s x N) and Q = A^{-1} B:
//     C Q = [Sigma_L Q_{1,:}; Sigma_R Q_{nb,:}]                 (2s x 2s)
//     R   = I - C Q,   [V | z] = R^{-1} [I | C Q b']           (one LU solve, 2s + m right-hand sides)
//     gc  = [Q_{1,:}; Q_{nb,:}] V                               (corner of G^R = (A - B C)^{-1} = Q R^{-1})
//     psi = Q (b' + z)                                          (y + Q z with y = Q b')
// With an absorbing boundary (absorb > 0, see sweep.hip) Q = A'^{-1} B for A' = A + i*absorb*[boundary
// blocks], and every C above is C' = C + i*absorb*I (T = A - B C = A' - B C'), so C Q gains
// i*absorb*[Q_{1,:}; Q_{nb,:}].
// The transmission uses only the off-diagonal corner blocks:
//     T_LR = Re Tr[Gamma_L G_1n Gamma_R G_1n^H] = Re sum_ij (Gamma_L G_1n)_ij conj((G_1n Gamma_R)_ij)
// (Gamma Hermitian), and likewise T_RL with G_n1 and the leads exchanged.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>

#include "drivers.hpp"
#include "lu.hpp"
#include "tile.hpp"

namespace ss {

using ObcTile = TileCfgG3<64, 64, 16, 2, 2>;
// psi = Q (b' + z) has as many columns as injected modes (typically 32): a 64 x 32 tile of four waves
using PsiTile = TileCfgG3<64, 32, 16, 4, 1>;

// element (r, k) of Q_c = [Q_{1,:}; Q_{nb,:}] (2s x 2s) from Q [nb*s][2s]
struct LdCorner {
  const double2 *q;
  int s, nb;
  static constexpr bool kFastSecond = true;
  __device__ __forceinline__ double2 operator()(int r, int k) const {
    const long row = r < s ? r : (long)(nb - 1) * s + (r - s);
    return q[row * 2 * s + k];
  }
};

// element (k, c) of b' + z
struct LdSum {
  const double2 *b, *z;
  long ldb, ldz;
  static constexpr bool kFastSecond = true;
  __device__ __forceinline__ double2 operator()(int k, int c) const {
    return cadd(b[(long)k * ldb + c], z[(long)k * ldz + c]);
  }
};

// element (r, c) of Gamma = i (Sigma - Sigma^H)
struct LdGamma {
  const double2 *sig;
  int s;
  static constexpr bool kFastSecond = true;
  __device__ __forceinline__ double2 operator()(int r, int c) const {
    const double2 a = sig[(long)r * s + c], b = sig[(long)c * s + r];
    // i * (a - conj(b)) = i*((a.x - b.x) + i (a.y + b.y)) = -(a.y + b.y) + i (a.x - b.x)
    return make_double2(-(a.y + b.y), a.x - b.x);
  }
};

struct ObcArgs {
  const double2 *Q, *sigma, *inj;
  double2 *psi, *gc;
  double absorb;  // C' = Sigma + i*absorb*I
  int nb, s, m, batch;
  const int *nbv;               // per-instance block counts (null: nb)
  const long *boff;             // first block of each instance in the packed Q (null: inst * nb)
  double2 *const *psi_tab;      // per-instance psi destinations (null: psi packed like Q)
  double2 *M;   // [batch][2s][4s+m]
  double2 *CQ;  // [batch][2s][2s]
  double2 *X;   // [batch][2s][2s+m]
};

// C Q, R = I - C Q and the identity block: grid (2 halves * tiles(s) * tiles(2s), batch)
__device__ __forceinline__ int obc_nb(const ObcArgs &a, int inst) { return a.nbv ? a.nbv[inst] : a.nb; }
__device__ __forceinline__ const double2 *obc_q(const ObcArgs &a, int inst) {
  return a.Q + (a.boff ? a.boff[inst] : (long)inst * a.nb) * 2 * (long)a.s * a.s;
}

__global__ void __launch_bounds__(ObcTile::NT) SS_TILE_WAVES_OF(ObcTile) k_obc_cq(ObcArgs a) {
  using T = ObcTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int inst = blockIdx.y, s = a.s, nb = obc_nb(a, inst);
  const int tr = cdiv(s, T::BM), tc = cdiv(2 * s, T::BN);
  int t = blockIdx.x;
  const int half = t / (tr * tc);
  t %= tr * tc;
  const int m0 = (t / tc) * T::BM, n0 = (t % tc) * T::BN;
  const long ss2 = (long)s * s;
  const double2 *sig = a.sigma + ((long)inst * 2 + half) * ss2;  // half 0: Sigma_L, 1: Sigma_R
  const double2 *qrow = obc_q(a, inst) + (half ? (long)(nb - 1) * 2 * ss2 : 0);
  Acc<T> acc;
  acc.zero();
  LdRow la{sig, s};
  LdRow lb{qrow, 2 * s};
  mma_loop<T>(la, lb, m0, s, n0, 2 * s, 0, s, acc, lds);
  const int ldm = 4 * s + a.m;
  double2 *M = a.M + (long)inst * 2 * s * ldm;
  double2 *cq = a.CQ + (long)inst * 4 * ss2;
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < 2 * s) {
      if (a.absorb != 0.0) {  // + i*absorb*Q_row
        const double2 q = qrow[(long)gr * 2 * s + gc];
        v = make_double2(v.x - a.absorb * q.y, v.y + a.absorb * q.x);
      }
      const int row = half * s + gr;
      const double d = row == gc ? 1.0 : 0.0;
      cq[(long)row * 2 * s + gc] = v;
      M[(long)row * ldm + gc] = make_double2(d - v.x, -v.y);
      M[(long)row * ldm + 2 * s + gc] = make_double2(d, 0.0);
    }
  });
}

// C Q b' into the last m columns of the augmented matrix (m columns: 64 x 32 tiles)
__global__ void __launch_bounds__(PsiTile::NT) SS_TILE_WAVES_OF(PsiTile) k_obc_cqb(ObcArgs a) {
  using T = PsiTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int inst = blockIdx.y, s = a.s, m = a.m;
  const int tc = cdiv(m, T::BN);
  const int m0 = (blockIdx.x / tc) * T::BM, n0 = (blockIdx.x % tc) * T::BN;
  Acc<T> acc;
  acc.zero();
  LdRow la{a.CQ + (long)inst * 4 * s * s, 2 * s};
  LdRow lb{a.inj + (long)inst * 2 * s * m, m};
  mma_loop<T>(la, lb, m0, 2 * s, n0, m, 0, 2 * s, acc, lds);
  const int ldm = 4 * s + m;
  double2 *M = a.M + (long)inst * 2 * s * ldm;
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < 2 * s && gc < m) M[(long)gr * ldm + 4 * s + gc] = v;
  });
}

// gc = Q_c V
__global__ void __launch_bounds__(ObcTile::NT) SS_TILE_WAVES_OF(ObcTile) k_obc_gc(ObcArgs a) {
  using T = ObcTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int inst = blockIdx.y, s = a.s;
  const int tc = cdiv(2 * s, T::BN);
  const int m0 = (blockIdx.x / tc) * T::BM, n0 = (blockIdx.x % tc) * T::BN;
  const int ldx = 2 * s + a.m;
  Acc<T> acc;
  acc.zero();
  LdCorner la{obc_q(a, inst), s, obc_nb(a, inst)};
  LdRow lb{a.X + (long)inst * 2 * s * ldx, ldx};
  mma_loop<T>(la, lb, m0, 2 * s, n0, 2 * s, 0, 2 * s, acc, lds);
  double2 *g = a.gc + (long)inst * 4 * s * s;
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gcl = n0 + c;
    if (gr < 2 * s && gcl < 2 * s) g[(long)gr * 2 * s + gcl] = v;
  });
}

// psi = Q (b' + z): rows nb*s, columns m, depth 2s
__global__ void __launch_bounds__(PsiTile::NT) SS_TILE_WAVES_OF(PsiTile) k_obc_psi(ObcArgs a) {
  using T = PsiTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int inst = blockIdx.y, s = a.s, m = a.m;
  const int rows = obc_nb(a, inst) * s;
  const int tc = cdiv(m, T::BN);
  const int m0 = (blockIdx.x / tc) * T::BM, n0 = (blockIdx.x % tc) * T::BN;
  if (m0 >= rows) return;  // the grid covers the largest instance
  double2 *p = a.psi_tab ? a.psi_tab[inst]
                         : a.psi + (a.boff ? a.boff[inst] : (long)inst * a.nb) * (long)s * m;
  if (p == nullptr) return;
  const int ldx = 2 * s + m;
  Acc<T> acc;
  acc.zero();
  LdRow la{obc_q(a, inst), 2 * s};
  LdSum lb{a.inj + (long)inst * 2 * s * m, a.X + (long)inst * 2 * s * ldx + 2 * s, m, ldx};
  mma_loop<T>(la, lb, m0, rows, n0, m, 0, 2 * s, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < rows && gc < m) p[(long)gr * m + gc] = v;
  });
}

__global__ void k_obc_info(const int *zp, int *info, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < batch && info) info[i] = zp[i];
}

static ss_status obc_run(ss_ctx *ctx, ObcArgs &a, int nb_max, bool want_psi, int *info) {
  const int batch = a.batch, s = a.s, m = a.m;
  const long ss2 = (long)s * s;
  const int n = 2 * s, nrhs = 2 * s + m, ldm = 4 * s + m;
  void *wM, *wP, *wZ, *wO;
  SS_TRY(workspace(ctx, kSlotM, sizeof(double2) * (size_t)batch * n * ldm, &wM));
  SS_TRY(workspace(ctx, kSlotPerm, sizeof(int) * (size_t)batch * n, &wP));
  SS_TRY(workspace(ctx, kSlotZp, sizeof(int) * (size_t)batch, &wZ));
  SS_TRY(workspace(ctx, kSlotObc, sizeof(double2) * (size_t)batch * (4 * ss2 + (long)n * nrhs), &wO));
  a.M = (double2 *)wM;
  a.CQ = (double2 *)wO;
  a.X = a.CQ + (size_t)batch * 4 * ss2;

  using T = ObcTile;
  const int tr = cdiv(s, T::BM), tc2 = cdiv(2 * s, T::BN);
  {
    KernelScope ks_(ctx, "obc");
    hipLaunchKernelGGL(k_obc_cq, dim3(2 * tr * tc2, batch), dim3(T::NT), 0, ctx->stream, a);
  }
  if (m > 0) {
    KernelScope ks_(ctx, "obc");
    hipLaunchKernelGGL(k_obc_cqb, dim3(cdiv(2 * s, PsiTile::BM) * cdiv(m, PsiTile::BN), batch), dim3(PsiTile::NT), 0,
                       ctx->stream, a);
  }
  LuDesc d;
  d.nmat = batch;
  d.n = n;
  d.nrhs = nrhs;
  d.M = a.M;
  d.sM = (long)n * ldm;
  d.ldm = ldm;
  d.perm = (int *)wP;
  d.sP = n;
  d.zp = (int *)wZ;
  d.X = a.X;
  d.sX = (long)n * nrhs;
  d.ldx = nrhs;
  SS_TRY(lu_identity_perm(ctx, d));
  SS_TRY(lu_solve(ctx, d));
  if (a.gc) {
    KernelScope ks_(ctx, "obc");
    hipLaunchKernelGGL(k_obc_gc, dim3(cdiv(2 * s, T::BM) * tc2, batch), dim3(T::NT), 0, ctx->stream, a);
  }
  if (m > 0 && want_psi) {
    KernelScope ks_(ctx, "obc");
    hipLaunchKernelGGL(k_obc_psi, dim3(cdiv(nb_max * s, PsiTile::BM) * cdiv(m, PsiTile::BN), batch),
                       dim3(PsiTile::NT), 0, ctx->stream, a);
  }
  hipLaunchKernelGGL(k_obc_info, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, (const int *)wZ, info, batch);
  return check_launch(ctx, "apply_obc");
}

ss_status apply_obc(ss_ctx *ctx, int batch, int nb, int s, const ss_c128 *Q, const ss_c128 *sigma, double absorb,
                    int m, const ss_c128 *inj, ss_c128 *psi, ss_c128 *gc, int *info) {
  ObcArgs a{};
  a.Q = (const double2 *)Q;
  a.sigma = (const double2 *)sigma;
  a.absorb = absorb;
  a.inj = (const double2 *)inj;
  a.psi = (double2 *)psi;
  a.gc = (double2 *)gc;
  a.nb = nb;
  a.s = s;
  a.m = m;
  a.batch = batch;
  a.nbv = nullptr;
  a.boff = nullptr;
  a.psi_tab = nullptr;
  return obc_run(ctx, a, nb, psi != nullptr, info);
}

ss_status apply_obc_ragged(ss_ctx *ctx, const RaggedBatch &rb, const ss_c128 *Q, const ss_c128 *sigma, double absorb,
                           int m, const ss_c128 *inj, ss_c128 *const *psi_tab, ss_c128 *gc, int *info) {
  ObcArgs a{};
  a.Q = (const double2 *)Q;
  a.sigma = (const double2 *)sigma;
  a.absorb = absorb;
  a.inj = (const double2 *)inj;
  a.psi = nullptr;
  a.gc = (double2 *)gc;
  a.nb = rb.nb_max;
  a.s = rb.s;
  a.m = m;
  a.batch = rb.batch;
  a.nbv = rb.nbv;
  a.boff = rb.boff;
  a.psi_tab = (double2 *const *)psi_tab;
  return obc_run(ctx, a, rb.nb_max, psi_tab != nullptr, info);
}

// ------------------------------------------------------------------ transmission

using TrTile = TileCfg<32, 32, 16, 2, 2>;

// per (instance, direction, tile): partial sum of Re[(Gam_a G)_ij conj((G Gam_b)_ij)]
// Directions dir0 + blockIdx.y; partial sums at [inst][blockIdx.y][tile].
__global__ void __launch_bounds__(TrTile::NT) k_trans(const double2 *gcp, const double2 *sigma, int s, int dir0,
                                                       double *partial) {
  using T = TrTile;
  __shared__ double lds[T::LDS_DOUBLES];
  __shared__ double red[T::NT / 64];
  const int inst = blockIdx.z, dir = dir0 + blockIdx.y;  // dir 0: T_LR with G_1n; dir 1: T_RL with G_n1
  const int tiles = cdiv(s, T::BM);
  const int m0 = (blockIdx.x / tiles) * T::BM, n0 = (blockIdx.x % tiles) * T::BN;
  const long ss2 = (long)s * s;
  const double2 *g = gcp + (long)inst * 4 * ss2 + (dir == 0 ? s : (long)s * 2 * s);  // G_1n or G_n1
  const double2 *sig_a = sigma + ((long)inst * 2 + (dir == 0 ? 0 : 1)) * ss2;  // left factor's lead
  const double2 *sig_b = sigma + ((long)inst * 2 + (dir == 0 ? 1 : 0)) * ss2;
  Acc<T> p1, p2;
  p1.zero();
  p2.zero();
  LdGamma ga{sig_a, s}, gb{sig_b, s};
  LdRow lg{g, 2 * s};
  mma_loop<T>(ga, lg, m0, s, n0, s, 0, s, p1, lds);
  mma_loop<T>(lg, gb, m0, s, n0, s, 0, s, p2, lds);
  double acc = 0.0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = m0 + wm * T::FM * 16 + i * 16 + 4 * q + (lane >> 4);
        const int c = n0 + wn * T::FN * 16 + j * 16 + (lane & 15);
        if (r < s && c < s) acc += p1.re[i][j][q] * p2.re[i][j][q] + p1.im[i][j][q] * p2.im[i][j][q];
      }
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < T::NT / 64; ++w) t += red[w];
    partial[((long)inst * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = t;
  }
}

__global__ void k_trans_sum(const double *partial, int ntile, double *T, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double t = 0.0;
  for (int k = 0; k < ntile; ++k) t += partial[(long)i * ntile + k];
  T[i] = t;
}

// Per-tile partial sums of one transmission call: batch * 2 * (tiles per direction) doubles.
size_t transmission_partials(int batch, int s) {
  const size_t tiles = (size_t)cdiv(s, TrTile::BM);
  return (size_t)batch * 2 * tiles * tiles;
}

// Both kernels of a transmission call; `partial` holds transmission_partials(batch, s) doubles.  Every
// partial is written by k_trans before k_trans_sum reads it (same stream), so nothing needs clearing.
static void launch_transmission(ss_ctx *ctx, int batch, int s, const ss_c128 *gc, const ss_c128 *sigma, double *T,
                                double *partial) {
  const int tiles = cdiv(s, TrTile::BM);
  const int ntile = tiles * tiles;
  hipLaunchKernelGGL(k_trans, dim3(ntile, 2, batch), dim3(TrTile::NT), 0, ctx->stream, (const double2 *)gc,
                     (const double2 *)sigma, s, 0, partial);
  hipLaunchKernelGGL(k_trans_sum, dim3(cdiv(2 * batch, 256)), dim3(256), 0, ctx->stream, (const double *)partial,
                     ntile, T, 2 * batch);
}

int caroli_rl_tiles(int s) { return cdiv(s, TrTile::BM) * cdiv(s, TrTile::BM); }

void launch_caroli_rl_partials(ss_ctx *ctx, int batch, int s, const ss_c128 *gc, const ss_c128 *sigma,
                               double *partial) {
  hipLaunchKernelGGL(k_trans, dim3(caroli_rl_tiles(s), 1, batch), dim3(TrTile::NT), 0, ctx->stream,
                     (const double2 *)gc, (const double2 *)sigma, s, 1, partial);
}

ss_status transmission(ss_ctx *ctx, int batch, int s, const ss_c128 *gc, const ss_c128 *sigma, double *T) {
  void *wP;
  SS_TRY(workspace(ctx, kSlotMisc, sizeof(double) * transmission_partials(batch, s), &wP));
  {
    KernelScope ks_(ctx, "trans");
    launch_transmission(ctx, batch, s, gc, sigma, T, (double *)wP);
  }
  return check_launch(ctx, "transmission");
}

// ------------------------------------------------------------------ transmission without allocation
//
// The partial sums live in a fixed device array instead of the context's workspace.  Host code never
// uses the array's name as an address (it stands for a host-side shadow there): its device address is
// looked up once per device with hipGetSymbolAddress and kept in g_trans_scratch.  Every call on one
// device shares that device's copy; calls that overlap on one device race.

static __device__ __align__(256) double scratch[SS_TRANS_SCRATCH_DOUBLES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_trans_scratch_mu;
std::atomic<double *> g_trans_scratch[kScratchDevices];
}  // namespace

ss_status transmission_scratch_init(int device) {
  if (device < 0 || device >= kScratchDevices) return SS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_trans_scratch_mu);
  if (g_trans_scratch[device].load()) return SS_OK;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != device) return SS_ERR_DEVICE;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return SS_ERR_DEVICE;
  }
  g_trans_scratch[device].store((double *)p);
  return SS_OK;
}

ss_status transmission_noalloc(ss_ctx *ctx, int batch, int s, const ss_c128 *gc, const ss_c128 *sigma, double *T) {
  if (transmission_partials(batch, s) > (size_t)SS_TRANS_SCRATCH_DOUBLES)
    return fail(ctx, SS_ERR_ARG,
                "ss_transmission_noalloc: batch * 2 * ceil(s/32)^2 = " + std::to_string(transmission_partials(batch, s)) +
                    " partial sums exceed the fixed scratch of " + std::to_string(SS_TRANS_SCRATCH_DOUBLES));
  double *partial = (ctx->device >= 0 && ctx->device < kScratchDevices) ? g_trans_scratch[ctx->device].load() : nullptr;
  if (!partial) return fail(ctx, SS_ERR_DEVICE, "ss_transmission_noalloc: scratch address of this device unknown");
  launch_transmission(ctx, batch, s, gc, sigma, T, partial);
  return check_launch(ctx, "transmission_noalloc");
}

}  // namespace ss
