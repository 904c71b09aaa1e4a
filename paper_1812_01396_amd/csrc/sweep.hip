// Step 1 of SplitSolve (Sec. 3B, Alg. 1): first and last block columns Q of A^{-1}, A = E*S - H.
//
// Optional absorbing boundary (Sec. 3B: the split T = A - B C of the open system leaves the choice of B
// and C free): with absorb > 0 the first and last diagonal blocks are formed as E*S - H + i*absorb*I,
// i.e. the constant part -i*absorb*I of the boundary self-energies is moved from C into A.  Q is then
// A'^{-1} B for that A', and the post-processing uses C' = Sigma + i*absorb*I.  absorb = 0 is the
// paper's A = E*S - H.
//
// Every instance runs two independent recursions ("directions") in lockstep, as separate systems of
// one batch:
//   direction 0 (first column), 0-based block ib = nb-1-t at step t:
//     D = A_{ib,ib} - A_{ib,ib+1} X_{ib+1},   X_{ib} = D^{-1} A_{ib,ib-1},   A_{0,-1} := I
//   direction 1 (last column), block ib = t:
//     D = A_{ib,ib} - A_{ib,ib-1} Y_{ib-1},   Y_{ib} = D^{-1} A_{ib,ib+1},   A_{nb-1,nb} := I
// A is never stored: its blocks are formed as E*S - H inside the tile loads.  The per-step
// solutions go to slot t of a per-system store, so both directions address slot t at step t.
// Then the chains Q_{ib} = -X_{ib} Q_{ib-1} (from Q_0 = X_0) and Q'_{ib} = -Y_{ib} Q'_{ib+1} (from
// Q'_{nb-1} = Y_{nb-1}) both read slot nb-1-u at chain step u and write into the caller's Q.
#include <algorithm>
#include <climits>

#include "lu.hpp"
#include "drivers.hpp"
#include "tile.hpp"
#include "tile32.hpp"
#include "tilebf.hpp"

namespace ss {

struct SweepArgs {
  const double2 *Hd, *Hu, *Sd, *Su;
  long kstride_d, kstride_u;   // elements between consecutive (H, S) sets
  const double2 *const *tab;   // or per set {H_diag, H_upper, S_diag, S_upper} pointers (null: strided)
  const int *kidx;
  const double *E;
  double absorb;     // i*absorb*I added to the first and last diagonal blocks
  int nk, nb, s;
  const int *nbv;    // per-instance block counts (null: every instance has nb blocks)
  const long *boff;  // per-instance first block in the packed per-block stores (null: inst * nb)
  double2 *M;  // [nmat][s][2s]
  int *perm;   // [nmat][s]
  int *zp;     // [nmat]
  int *code;   // [batch] smallest zero-pivot code, INT_MAX if none
  double2 *X;  // per system: one s x s slot per block, packed (system 2i+d at block 2 boff(i) + d nb(i))
  double2 *Q;  // per instance [nb][s][2s], packed at block boff(i)
  float2 *cpl;  // per system [s][s]: the next step's coupling block in FP32 (BF16-term products only)
  int *info;   // [batch] or null
  int batch;
};

// (H, S) set of an instance; out-of-range indices are clamped so a bad index cannot address
// outside the caller's arrays (the binding rejects them before the call).
__device__ __forceinline__ int set_of(const SweepArgs &a, int inst) {
  const int k = a.kidx ? a.kidx[inst] : inst % a.nk;
  return min(max(k, 0), a.nk - 1);
}
__device__ __forceinline__ int nb_of(const SweepArgs &a, int inst) { return a.nbv ? a.nbv[inst] : a.nb; }
__device__ __forceinline__ long boff_of(const SweepArgs &a, int inst) {
  return a.boff ? a.boff[inst] : (long)inst * a.nb;
}
// block b of array j (0 H_diag, 1 H_upper, 2 S_diag, 3 S_upper) of set k
__device__ __forceinline__ const double2 *blk(const SweepArgs &a, int k, int j, int b) {
  const long ss2 = (long)a.s * a.s;
  if (a.tab) return a.tab[4 * k + j] + b * ss2;
  const double2 *base = j == 0 ? a.Hd : j == 1 ? a.Hu : j == 2 ? a.Sd : a.Su;
  return base + k * ((j & 1) ? a.kstride_u : a.kstride_d) + b * ss2;
}
// slot t of system mat
__device__ __forceinline__ double2 *xslot(const SweepArgs &a, int mat, int t) {
  const int inst = mat >> 1, dir = mat & 1;
  return a.X + (2 * boff_of(a, inst) + (long)dir * nb_of(a, inst) + t) * ((long)a.s * a.s);
}

// element (r, c) of an FP32 complex row-major block
struct LdRowF32 {
  const float2 *p;
  long ld;
  static constexpr bool kFastSecond = true;
  __device__ __forceinline__ double2 operator()(int r, int c) const {
    const float2 v = p[(long)r * ld + c];
    return make_double2(v.x, v.y);
  }
};

using FormTile = TileCfg<64, 64, 16, 2, 2>;
using FormTileG3 = TileCfgG3<64, 64, 16, 2, 2>;
using FormTile32 = TileCfg32G3<64, 64, 16, 2, 2>;
using FormTileB = TileCfgB<64, 64, 32, 2, 2, 3>;
static_assert(FormTile32::LDS_FLOATS <= 2 * FormTile::LDS_DOUBLES, "shared staging buffer too small");
static_assert(FormTileB::NT == FormTile::NT, "one workgroup shape for every precision");

// precision of the block products: FP64, FP32, or BF16 terms (three per operand) with FP32 accumulation
enum { kProdF64 = 0, kProdF32 = 1, kProdBF16 = 2 };

// acc(r, c) = sum_k A(r, k) B(k, c) over one 64 x 64 tile in the precision kP; f(r, c, value) receives
// every element of the tile.  FP64 and FP32 products take the three-product form (two waves per SIMD for
// FP64, three for FP32); the BF16-term products keep four real products.
template <int kP, class LA, class LB, class F>
__device__ __forceinline__ void tile_product(const LA &la, const LB &lb, int m0, int M, int n0, int N, int kbeg,
                                             int kend, double *lds, F &&f) {
  if constexpr (kP == kProdF32) {
    Acc32<FormTile32> acc;
    acc.zero();
    mma_loop32<FormTile32>(la, lb, m0, M, n0, N, kbeg, kend, acc, reinterpret_cast<float *>(lds));
    acc_foreach32<FormTile32>(acc, f);
  } else if constexpr (kP == kProdBF16) {
    AccB<FormTileB> acc;
    acc.zero();
    mma_loop_bf<FormTileB>(la, lb, m0, M, n0, N, kbeg, kend, acc, reinterpret_cast<unsigned short *>(lds));
    acc_foreach_bf<FormTileB>(acc, f);
  } else {
    Acc<FormTileG3> acc;
    acc.zero();
    mma_loop<FormTileG3>(la, lb, m0, M, n0, N, kbeg, kend, acc, lds);
    acc_foreach<FormTileG3>(acc, f);
  }
}

// Forms [D | RHS] of step t for every system; fold the previous step's zero pivot into `code`.
// kPart 0: the grid covers the D tiles and then the RHS tiles; 1: the D tiles only; 2: the RHS tiles only.
template <int kP, int kPart>
__device__ __forceinline__ void form_body(const SweepArgs &a, int t, double *lds) {
  using T = FormTile;
  int tile, mat;
  xcd_tile_order(tile, mat);
  const int inst = mat >> 1, dir = mat & 1;
  const int s = a.s, nb = nb_of(a, inst);
  if (t >= nb) return;
  const int ks = set_of(a, inst);
  const double e = a.E[inst];
  const int ib = dir == 0 ? nb - 1 - t : t;
  const long ss2 = (long)s * s;
  const double2 *hd = blk(a, ks, 0, ib);
  const double2 *sd = blk(a, ks, 2, ib);
  double2 *M = a.M + (long)mat * 2 * ss2;
  const int tiles = cdiv(s, T::BM);
  const int ntile = tiles * tiles;
  if (kPart == 2) tile += ntile;

  if (tile == 0 && threadIdx.x == 0 && t > 0) {
    const int z = a.zp[mat];
    if (z != 0) {
      const int pib = dir == 0 ? nb - t : t - 1;  // block of the previous step
      atomicMin(a.code + inst, pib * s + z);
    }
  }

  if (tile < ntile) {
    if constexpr (kPart != 2) {
    // D tile: D = A_ib,ib - coupling * previous solution
    const int m0 = (tile / tiles) * T::BM, n0 = (tile % tiles) * T::BN;
    // absorbing shift of the boundary blocks (both of them when nb == 1)
    const double shift = a.absorb * ((ib == 0 ? 1 : 0) + (ib == nb - 1 ? 1 : 0));
    auto store = [&](int r, int c, double2 v) {
      const int gr = m0 + r, gc = n0 + c;
      if (gr < s && gc < s) {
        const long o = (long)gr * s + gc;
        const double2 av = make_double2(e * sd[o].x - hd[o].x, e * sd[o].y - hd[o].y + (gr == gc ? shift : 0.0));
        M[(long)gr * 2 * s + gc] = csub(av, v);
      }
    };
    if (t > 0) {
      const double2 *xp = xslot(a, mat, t - 1);
      LdRow lb{xp, s};
      if constexpr (kP == kProdBF16) {  // the coupling block, formed in FP32 by the previous step
        using TB = FormTileB;
        LdRowF32 la{a.cpl + (long)mat * ss2, s};
        AccB<TB> acc;
        acc.zero();
        mma_loop_bf<TB>(la, lb, m0, s, n0, s, 0, s, acc, reinterpret_cast<unsigned short *>(lds));
        // the epilogue reads every A_ii element of this thread before it writes any of D, so the
        // loads are in flight together (two waves per SIMD hide little latency)
        double2 av[TB::FM * TB::FN * 4];
        int i = 0;
        acc_foreach_bf<TB>(acc, [&](int r, int c, double2) {
          const int gr = m0 + r, gc = n0 + c;
          const long o = (long)min(gr, s - 1) * s + min(gc, s - 1);
          const double2 hv = hd[o], sv = sd[o];
          av[i++] = make_double2(e * sv.x - hv.x, e * sv.y - hv.y + (gr == gc ? shift : 0.0));
        });
        i = 0;
        acc_foreach_bf<TB>(acc, [&](int r, int c, double2 v) {
          const int gr = m0 + r, gc = n0 + c;
          const double2 w = av[i++];
          if (gr < s && gc < s) M[(long)gr * 2 * s + gc] = csub(w, v);
        });
      } else if (dir == 0) {  // A_{ib,ib+1} = E S_u[ib] - H_u[ib]
        LdForm<false> la{blk(a, ks, 1, ib), blk(a, ks, 3, ib), s, e};
        tile_product<kP>(la, lb, m0, s, n0, s, 0, s, lds, store);
      } else {  // A_{ib,ib-1} = (E S_u[ib-1] - H_u[ib-1])^H
        LdForm<true> la{blk(a, ks, 1, ib - 1), blk(a, ks, 3, ib - 1), s, e};
        tile_product<kP>(la, lb, m0, s, n0, s, 0, s, lds, store);
      }
    } else {
      for (int idx = threadIdx.x; idx < T::BM * T::BN; idx += T::NT)
        store(idx / T::BN, idx % T::BN, make_double2(0.0, 0.0));
    }
    if (n0 == 0) {
      for (int r = threadIdx.x; r < T::BM; r += T::NT)
        if (m0 + r < s) a.perm[(long)mat * s + m0 + r] = m0 + r;
    }
    }
  } else if constexpr (kPart != 1) {
    // RHS tile: the coupling to the already-eliminated side, or the identity at the boundary
    tile -= ntile;
    const int m0 = (tile / tiles) * T::BM, n0 = (tile % tiles) * T::BN;
    const bool ident = dir == 0 ? ib == 0 : ib == nb - 1;
    const int ub = dir == 0 ? ib - 1 : ib;
    const double2 *hu = blk(a, ks, 1, std::max(ub, 0));
    const double2 *su = blk(a, ks, 3, std::max(ub, 0));
    // with BF16-term products, the next step's coupling block (the conjugate transpose of this RHS)
    // is also written, in FP32: A_{ib-1,ib} = E S_u - H_u (direction 0), A_{ib+1,ib} = its transpose
    // conjugate (direction 1)
    float2 *cp = (kPart == 2 && !ident) ? a.cpl + (long)mat * ss2 : nullptr;
    for (int idx = threadIdx.x; idx < T::BM * T::BN; idx += T::NT) {
      const int r = idx / T::BN, c = idx % T::BN;
      const int gr = m0 + r, gc = n0 + c;
      if (gr >= s || gc >= s) continue;
      double2 v;
      if (ident) v = make_double2(gr == gc ? 1.0 : 0.0, 0.0);
      else if (dir == 0) {  // (E S_u - H_u)^H element (gr, gc) = conj(E S_u[gc][gr] - H_u[gc][gr])
        const long o = (long)gc * s + gr;
        v = make_double2(e * su[o].x - hu[o].x, -(e * su[o].y - hu[o].y));
      } else {
        const long o = (long)gr * s + gc;
        v = make_double2(e * su[o].x - hu[o].x, e * su[o].y - hu[o].y);
      }
      M[(long)gr * 2 * s + s + gc] = v;
      if (cp) {
        double2 w;
        if (dir == 0) {
          const long o = (long)gr * s + gc;
          w = make_double2(e * su[o].x - hu[o].x, e * su[o].y - hu[o].y);
        } else {
          const long o = (long)gc * s + gr;
          w = make_double2(e * su[o].x - hu[o].x, -(e * su[o].y - hu[o].y));
        }
        cp[(long)gr * s + gc] = make_float2((float)w.x, (float)w.y);
      }
    }
  }
}

// Fold the last step's zero pivot and publish info.
__global__ void k_sweep_finish(SweepArgs a) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= a.batch) return;
  int c = a.code[inst];
  for (int dir = 0; dir < 2; ++dir) {
    const int z = a.zp[2 * inst + dir];
    if (z != 0) {
      const int pib = dir == 0 ? 0 : nb_of(a, inst) - 1;
      c = min(c, pib * a.s + z);
    }
  }
  if (a.info) a.info[inst] = c == INT_MAX ? 0 : c;
}

__global__ void k_code_init(int *code, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) code[i] = INT_MAX;
}

template <bool kF32>
__global__ void __launch_bounds__(FormTile::NT) __attribute__((amdgpu_waves_per_eu(kF32 ? 3 : FormTileG3::WAVES))) k_form(SweepArgs a, int t) {
  __shared__ double lds[FormTile::LDS_DOUBLES];
  form_body<kF32 ? kProdF32 : kProdF64, 0>(a, t, lds);
}

// The BF16-term products need 60 KB of staging: two workgroups per CU, so two waves' registers per SIMD.
// The RHS tiles, plain element-wise formation, go to k_form_rhs, which runs at full occupancy.
__global__ void __launch_bounds__(FormTile::NT) __attribute__((amdgpu_waves_per_eu(2))) k_form_bf(SweepArgs a, int t) {
  __shared__ double lds[FormTileB::LDS_BYTES / 8];
  form_body<kProdBF16, 1>(a, t, lds);
}

__global__ void __launch_bounds__(FormTile::NT) k_form_rhs(SweepArgs a, int t) {
  form_body<kProdF64, 2>(a, t, nullptr);
}

// Chain step u: Q_ib = -X(slot nb-1-u) Q_prev (u > 0), or a copy of the slot (u == 0).
template <int kP>
__device__ __forceinline__ void chain_body(const SweepArgs &a, int u, double *lds) {
  using T = FormTile;
  int tile, mat;
  xcd_tile_order(tile, mat);
  const int inst = mat >> 1, dir = mat & 1;
  const int s = a.s, nb = nb_of(a, inst);
  if (u >= nb) return;
  const long ss2 = (long)s * s;
  const int tiles = cdiv(s, T::BM);
  const int m0 = (tile / tiles) * T::BM, n0 = (tile % tiles) * T::BN;
  const int ib = dir == 0 ? u : nb - 1 - u;
  const double2 *x = xslot(a, mat, nb - 1 - u);
  double2 *q0 = a.Q + boff_of(a, inst) * 2 * ss2 + (dir ? s : 0);
  double2 *qi = q0 + (long)ib * 2 * ss2;
  if (u == 0) {
    for (int idx = threadIdx.x; idx < T::BM * T::BN; idx += T::NT) {
      const int gr = m0 + idx / T::BN, gc = n0 + idx % T::BN;
      if (gr < s && gc < s) qi[(long)gr * 2 * s + gc] = x[(long)gr * s + gc];
    }
    return;
  }
  const int pb = dir == 0 ? ib - 1 : ib + 1;
  const double2 *qp = q0 + (long)pb * 2 * ss2;
  LdRow la{x, s};
  LdRow lb{qp, 2 * s};
  tile_product<kP>(la, lb, m0, s, n0, s, 0, s, lds, [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) qi[(long)gr * 2 * s + gc] = cneg(v);
  });
}

template <bool kF32>
__global__ void __launch_bounds__(FormTile::NT) __attribute__((amdgpu_waves_per_eu(kF32 ? 3 : FormTileG3::WAVES))) k_chain(SweepArgs a, int u) {
  __shared__ double lds[FormTile::LDS_DOUBLES];
  chain_body<kF32 ? kProdF32 : kProdF64>(a, u, lds);
}

__global__ void __launch_bounds__(FormTile::NT) __attribute__((amdgpu_waves_per_eu(2))) k_chain_bf(SweepArgs a, int u) {
  __shared__ double lds[FormTileB::LDS_BYTES / 8];
  chain_body<kProdBF16>(a, u, lds);
}

// Keep the factorization of the first-column recursion's step t (L\U in physical rows and the row
// map, and, when inv is given, its panels' inverses of their 32 x 32 diagonal blocks: sInv per system)
// for later solves with the same diagonal systems.
__global__ void k_save_factors(SweepArgs a, double2 *F, int *P, int t, const double2 *inv, long sInv, double2 *FI) {
  const int inst = blockIdx.y, s = a.s;
  if (t >= nb_of(a, inst)) return;
  const long ss2 = (long)s * s;
  const double2 *M = a.M + (long)(2 * inst) * 2 * ss2;
  const long blk_t = boff_of(a, inst) + t;
  double2 *f = F + blk_t * ss2;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < ss2; idx += (long)gridDim.x * blockDim.x) {
    const int r = idx / s, c = idx % s;
    f[idx] = M[(long)r * 2 * s + c];
  }
  if (inv != nullptr) {
    const double2 *src = inv + (long)(2 * inst) * sInv;
    double2 *dst = FI + blk_t * sInv;
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < sInv; idx += (long)gridDim.x * blockDim.x)
      dst[idx] = src[idx];
  }
  if (blockIdx.x == 0)
    for (int r = threadIdx.x; r < s; r += blockDim.x) P[blk_t * s + r] = a.perm[(long)(2 * inst) * s + r];
}

// Enqueue both recursions and chains.  act[t] is the number of leading instances with more than t
// blocks (instances come sorted by block count, largest first), so step t runs on that prefix only.
// xoff: per-system X offsets for ragged batches (null when every instance has a.nb blocks).
static ss_status sweep_run(ss_ctx *ctx, SweepArgs &a, const std::vector<int> &act, long total_blocks,
                           const long *xoff, int prec, bool keep) {
  const int s = a.s, batch = a.batch, nmat = 2 * batch, nsteps = (int)act.size();
  const long ss2 = (long)s * s;
  const int n = s, nrhs = s, ldm = 2 * s;
  void *wM, *wP, *wZ, *wX;
  SS_TRY(workspace(ctx, kSlotM, sizeof(double2) * nmat * (size_t)n * ldm, &wM));
  SS_TRY(workspace(ctx, kSlotPerm, sizeof(int) * nmat * (size_t)n, &wP));
  SS_TRY(workspace(ctx, kSlotZp, sizeof(int) * (size_t)(nmat + batch), &wZ));
  SS_TRY(workspace(ctx, kSlotX, sizeof(double2) * 2 * (size_t)total_blocks * ss2, &wX));
  a.M = (double2 *)wM;
  a.perm = (int *)wP;
  a.zp = (int *)wZ;
  a.code = (int *)wZ + nmat;
  a.X = (double2 *)wX;
  a.cpl = nullptr;
  if (prec == SS_PREC_BF16) {
    void *wC;
    SS_TRY(workspace(ctx, kSlotCpl, sizeof(float2) * nmat * (size_t)ss2, &wC));
    a.cpl = (float2 *)wC;
  }

  LuDesc d;
  d.n = n;
  d.nrhs = nrhs;
  d.M = a.M;
  d.sM = (long)n * ldm;
  d.ldm = ldm;
  d.perm = a.perm;
  d.sP = n;
  d.zp = a.zp;
  d.sX = (long)a.nb * ss2;
  d.xoff = xoff;
  d.ldx = s;
  d.f32 = prec == SS_PREC_FP32_LU;

  double2 *F = nullptr, *FI = nullptr;
  int *P = nullptr;
  // with 32-column panels the kept factors also keep their panels' diagonal-block inverses
  const bool keep_inv = keep && lu_width_of(ctx, n) == 32;
  const long sInv = lu_inverse_elems(n, 32);
  if (keep) {
    SS_TRY(workspace(ctx, kSlotFact, sizeof(double2) * (size_t)total_blocks * ss2, (void **)&F));
    SS_TRY(workspace(ctx, kSlotFactPerm, sizeof(int) * (size_t)total_blocks * s, (void **)&P));
    if (keep_inv)
      SS_TRY(workspace(ctx, kSlotFactInv, sizeof(double2) * (size_t)total_blocks * sInv, (void **)&FI));
  }
  ctx->fact_valid = false;
  const bool f32 = prec == SS_PREC_FP32 || prec == SS_PREC_FP32_LU;
  hipLaunchKernelGGL(k_code_init, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, a.code, batch);
  const int tiles = cdiv(s, FormTile::BM);
  for (int t = 0; t < nsteps; ++t) {
    const int na = act[t];
    if (na <= 0) break;
    {
      KernelScope ks_(ctx, "form");
      if (prec == SS_PREC_BF16) {  // the product reads the coupling block before the RHS kernel replaces it
        hipLaunchKernelGGL(k_form_bf, dim3(tiles * tiles, 2 * na), dim3(FormTile::NT), 0, ctx->stream, a, t);
        hipLaunchKernelGGL(k_form_rhs, dim3(tiles * tiles, 2 * na), dim3(FormTile::NT), 0, ctx->stream, a, t);
      } else if (f32)
        hipLaunchKernelGGL(k_form<true>, dim3(2 * tiles * tiles, 2 * na), dim3(FormTile::NT), 0, ctx->stream, a, t);
      else
        hipLaunchKernelGGL(k_form<false>, dim3(2 * tiles * tiles, 2 * na), dim3(FormTile::NT), 0, ctx->stream, a,
                           t);
    }
    d.nmat = 2 * na;
    d.X = a.X + (long)t * ss2;
    SS_TRY(lu_solve(ctx, d));
    if (keep) {
      double2 *inv = nullptr;  // the inverses this step's factorization left in the LU's workspace
      if (keep_inv) SS_TRY(workspace(ctx, kSlotLuInv, sizeof(double2) * (size_t)d.nmat * sInv, (void **)&inv));
      hipLaunchKernelGGL(k_save_factors, dim3(std::min(cdiv((int)std::min<long>(ss2, 1 << 30), 256), 64), na),
                         dim3(256), 0, ctx->stream, a, F, P, t, (const double2 *)inv, sInv, FI);
    }
  }
  hipLaunchKernelGGL(k_sweep_finish, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, a);
  for (int u = 0; u < nsteps; ++u) {
    const int na = act[u];
    if (na <= 0) break;
    KernelScope ks_(ctx, "chain");
    if (prec == SS_PREC_BF16)
      hipLaunchKernelGGL(k_chain_bf, dim3(tiles * tiles, 2 * na), dim3(FormTile::NT), 0, ctx->stream, a, u);
    else if (f32)
      hipLaunchKernelGGL(k_chain<true>, dim3(tiles * tiles, 2 * na), dim3(FormTile::NT), 0, ctx->stream, a, u);
    else
      hipLaunchKernelGGL(k_chain<false>, dim3(tiles * tiles, 2 * na), dim3(FormTile::NT), 0, ctx->stream, a, u);
  }
  return check_launch(ctx, "precompute_columns");
}

ss_status precompute_columns(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E,
                             double absorb, int prec, int flags, ss_c128 *Q, int *info) {
  const int s = hs->s, nb = hs->nb;
  const long ss2 = (long)s * s;
  SweepArgs a{};
  a.Hd = (const double2 *)hs->H_diag;
  a.Hu = (const double2 *)hs->H_upper;
  a.Sd = (const double2 *)hs->S_diag;
  a.Su = (const double2 *)hs->S_upper;
  a.kstride_d = (long)nb * ss2;
  a.kstride_u = (long)std::max(nb - 1, 0) * ss2;
  a.tab = nullptr;
  a.kidx = kidx;
  a.E = E;
  a.absorb = absorb;
  a.nk = hs->nk;
  a.nb = nb;
  a.s = s;
  a.nbv = nullptr;
  a.boff = nullptr;
  a.Q = (double2 *)Q;
  a.info = info;
  a.batch = batch;
  const bool keep = (flags & SS_KEEP_FACTORS) != 0;
  SS_TRY(sweep_run(ctx, a, std::vector<int>(nb, batch), (long)batch * nb, nullptr, prec, keep));
  if (keep) {
    ctx->fact_valid = true;
    ctx->fact_inv = lu_width_of(ctx, s) == 32;
    ctx->fact_batch = batch;
    ctx->fact_nb = nb;
    ctx->fact_s = s;
    ctx->fact_absorb = absorb;
  }
  return SS_OK;
}

ss_status precompute_ragged(ss_ctx *ctx, const RaggedBatch &rb, double absorb, int prec, ss_c128 *Q, int *info) {
  SweepArgs a{};
  a.tab = (const double2 *const *)rb.tab;
  a.kidx = nullptr;
  a.E = rb.E;
  a.absorb = absorb;
  a.nk = rb.batch;
  a.nb = rb.nb_max;
  a.s = rb.s;
  a.nbv = rb.nbv;
  a.boff = rb.boff;
  a.Q = (double2 *)Q;
  a.info = info;
  a.batch = rb.batch;
  return sweep_run(ctx, a, rb.act, rb.total_blocks, rb.xoff, prec, false);
}

}  // namespace ss
