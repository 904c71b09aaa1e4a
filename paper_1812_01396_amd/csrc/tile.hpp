// Complex FP64 tile engine on the gfx950 matrix cores (v_mfma_f64_16x16x4_f64).
//
// A workgroup of WM x WN wavefronts computes a BM x BN tile of complex outputs
//     acc(r, c) = sum_k A(r, k) * B(k, c)
// with A and B fetched through loader functors (plain row-major, row-permuted, conjugate-transposed,
// or formed on the fly as E*S - H).  Operands are staged through LDS as separate real and imaginary
// planes laid out [k][m] and [k][n], so each MFMA operand read is 16 consecutive doubles per k row.
// A complex product is four real MFMAs (re*re - im*im, re*im + im*re), or, for tile configurations of
// type TileCfgG3, three (Gauss's method: ArBr, AiBi and (Ar+Ai)(Br+Bi) summed separately, the real part
// the first minus the second, the imaginary part the third minus both); the next stage's global loads
// are issued before the current stage's MFMAs so their latency hides behind the matrix work.
//
// Register layout of v_mfma_f64_16x16x4_f64 (wave64), measured on gfx950:
//   A (16x4):  lane l holds A[l % 16][l / 16]
//   B (4x16):  lane l holds B[l / 16][l % 16]
//   D (16x16): lane l, element j holds D[4*j + l / 16][l % 16]
#pragma once

#include "common.hpp"

// Register budget of the 4-wave tile kernels: at most 168 registers per lane so that three waves fit
// on each SIMD.  Left alone the compiler keeps the accumulators in AGPRs beside ~150 VGPRs (two waves
// per SIMD); measured on batched 64 x 64 x k products, three waves are 12-20 % faster, four spill.
// (Kernels whose budget would spill at 168, such as the FP32-product variants, keep the default.)
#define SS_TILE_WAVES __attribute__((amdgpu_waves_per_eu(3)))
// The same for a kernel whose budget follows its tile configuration (T::WAVES waves per SIMD).
#define SS_TILE_WAVES_OF(T) __attribute__((amdgpu_waves_per_eu(T::WAVES)))

namespace ss {

template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct TileCfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
  static constexpr int NT = 64 * WM * WN;
  static constexpr int FM = BM / (16 * WM);
  static constexpr int FN = BN / (16 * WN);
  static constexpr int PA = BM + 1;  // odd row pitch (doubles): conflict-free transposing stores
  static constexpr int PB = BN + 1;
  static constexpr int LDS_DOUBLES = 2 * BK * PA + 2 * BK * PB;
  static constexpr int EA = (BM * BK + NT - 1) / NT;
  static constexpr int EB = (BK * BN + NT - 1) / NT;
  static constexpr bool G3 = false;  // three-product complex multiply (TileCfgG3)
  static constexpr int WAVES = 3;    // waves per SIMD the register budget is set for
  static_assert(FM >= 1 && FN >= 1, "tile smaller than one MFMA block per wave");
  static_assert(FM * 16 * WM == BM && FN * 16 * WN == BN, "tile not a multiple of the wave grid");
  static_assert(BK % 4 == 0, "BK must be a multiple of the MFMA depth");
};

// Gauss's three-product complex multiply: the same tile with 3/4 of the matrix-core work, at the cost
// of a third accumulator set (8 FM FN more registers per lane) and FM + FN additions per k step.  Its
// rounding error is bounded normwise like the four-product form's, with (|Ar| + |Ai|)(|Br| + |Bi|) in
// place of the products of the parts in the imaginary part's bound.  With four or more MFMA blocks per
// wave the accumulators (96 registers) leave too little of a 168-register budget: two waves per SIMD.
template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct TileCfgG3 : TileCfg<BM_, BN_, BK_, WM_, WN_> {
  using Base = TileCfg<BM_, BN_, BK_, WM_, WN_>;
  static constexpr bool G3 = true;
  static constexpr int WAVES = Base::FM * Base::FN >= 4 ? 2 : 3;
};

// Accumulators.  Four-product form: re and im are the real and imaginary parts.  Three-product form:
// re = sum Ar Br, im = sum (Ar + Ai)(Br + Bi), x = sum Ai Bi (acc_foreach and value() combine them).
template <class T>
struct Acc {
  static constexpr int XM = T::G3 ? T::FM : 1, XN = T::G3 ? T::FN : 1;
  v4d re[T::FM][T::FN];
  v4d im[T::FM][T::FN];
  v4d x[XM][XN];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < T::FM; ++i)
#pragma unroll
      for (int j = 0; j < T::FN; ++j) {
        re[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
        im[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      }
    if constexpr (T::G3) {
#pragma unroll
      for (int i = 0; i < XM; ++i)
#pragma unroll
        for (int j = 0; j < XN; ++j) x[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  }
  // the complex value of element q of block (i, j)
  __device__ __forceinline__ double2 value(int i, int j, int q) const {
    if constexpr (T::G3) {
      const double t1 = re[i][j][q], t2 = x[i][j][q];
      return make_double2(t1 - t2, im[i][j][q] - t1 - t2);
    } else {
      return make_double2(re[i][j][q], im[i][j][q]);
    }
  }
};

// ------------------------------------------------------------------ XCD-aware tile order
// Workgroups go to the eight XCDs (each with its own L2) round-robin by linear id.  For a grid of
// (tiles, systems) this remaps the ids so that every tile of a system runs on one XCD, in tile order,
// and that XCD's L2 serves the operand panels the tiles share.  A bijection of the grid; grids whose
// system count is not a multiple of 8 keep the plain order.
__device__ __forceinline__ void xcd_tile_order(int &tile, int &sys) {
  const int nt = gridDim.x, ns = gridDim.y;
  if (ns % 8 != 0) {
    tile = blockIdx.x;
    sys = blockIdx.y;
    return;
  }
  const long lin = blockIdx.x + (long)nt * blockIdx.y;
  const long slot = lin >> 3;
  sys = (int)(lin & 7) + 8 * (int)(slot / nt);
  tile = (int)(slot % nt);
}

// ------------------------------------------------------------------ loaders
// A loader returns element (r, k) of the left operand, a B loader element (k, c) of the right one.
// kFastSecond: consecutive values of the second index are contiguous in memory (row-major).

struct LdRow {  // p[r * ld + c]
  const double2 *p;
  long ld;
  static constexpr bool kFastSecond = true;
  __device__ __forceinline__ double2 operator()(int r, int c) const { return p[(long)r * ld + c]; }
};

struct LdRowPerm {  // p[perm[r] * ld + c]; perm usually lives in LDS
  const double2 *p;
  long ld;
  const int *perm;
  static constexpr bool kFastSecond = true;
  __device__ __forceinline__ double2 operator()(int r, int c) const { return p[(long)perm[r] * ld + c]; }
};

// element (r, c) of E*S - H (kConj == false) or of (E*S - H)^H (kConj == true) for row-major
// blocks H, S with leading dimension ld; E is real.
template <bool kConj>
struct LdForm {
  const double2 *h, *s;
  long ld;
  double e;
  static constexpr bool kFastSecond = !kConj;
  __device__ __forceinline__ double2 operator()(int r, int c) const {
    long o = kConj ? (long)c * ld + r : (long)r * ld + c;
    double2 hv = h[o], sv = s[o];
    double2 v = make_double2(e * sv.x - hv.x, e * sv.y - hv.y);
    return kConj ? cconj(v) : v;
  }
};

// ------------------------------------------------------------------ engine

template <class T>
struct Lds {
  double *ar, *ai, *br, *bi;
  __device__ __forceinline__ explicit Lds(double *base) {
    ar = base;
    ai = ar + T::BK * T::PA;
    br = ai + T::BK * T::PA;
    bi = br + T::BK * T::PB;
  }
};

// One BK-deep stage of MFMAs from LDS into the accumulators.
template <class T, int KSTEPS = T::BK / 4>
__device__ __forceinline__ void mma_stage(const Lds<T> &L, Acc<T> &acc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  const int mbase = wm * T::FM * 16 + (lane & 15);
  const int nbase = wn * T::FN * 16 + (lane & 15);
#pragma unroll
  for (int ks = 0; ks < KSTEPS; ++ks) {
    const int kr = ks * 4 + (lane >> 4);
    if constexpr (T::G3) {
      double ar[T::FM], ai[T::FM], as[T::FM], br[T::FN], bi[T::FN], bs[T::FN];
#pragma unroll
      for (int i = 0; i < T::FM; ++i) {
        ar[i] = L.ar[kr * T::PA + mbase + i * 16];
        ai[i] = L.ai[kr * T::PA + mbase + i * 16];
        as[i] = ar[i] + ai[i];
      }
#pragma unroll
      for (int j = 0; j < T::FN; ++j) {
        br[j] = L.br[kr * T::PB + nbase + j * 16];
        bi[j] = L.bi[kr * T::PB + nbase + j * 16];
        bs[j] = br[j] + bi[j];
      }
#pragma unroll
      for (int i = 0; i < T::FM; ++i)
#pragma unroll
        for (int j = 0; j < T::FN; ++j) {
          acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], acc.re[i][j], 0, 0, 0);
          acc.x[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bi[j], acc.x[i][j], 0, 0, 0);
          acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[i], bs[j], acc.im[i][j], 0, 0, 0);
        }
    } else {
      double ar[T::FM], ai[T::FM], an[T::FM], br[T::FN], bi[T::FN];
#pragma unroll
      for (int i = 0; i < T::FM; ++i) {
        ar[i] = L.ar[kr * T::PA + mbase + i * 16];
        ai[i] = L.ai[kr * T::PA + mbase + i * 16];
        an[i] = -ai[i];
      }
#pragma unroll
      for (int j = 0; j < T::FN; ++j) {
        br[j] = L.br[kr * T::PB + nbase + j * 16];
        bi[j] = L.bi[kr * T::PB + nbase + j * 16];
      }
#pragma unroll
      for (int i = 0; i < T::FM; ++i)
#pragma unroll
        for (int j = 0; j < T::FN; ++j) {
          acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], acc.re[i][j], 0, 0, 0);
          acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], acc.im[i][j], 0, 0, 0);
          acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(an[i], bi[j], acc.re[i][j], 0, 0, 0);
          acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], acc.im[i][j], 0, 0, 0);
        }
    }
  }
}

// acc += A[m0:m0+BM, kbeg:kend] * B[kbeg:kend, n0:n0+BN]; rows >= M and columns >= N read as zero.
// All threads of the workgroup must call this (it synchronizes).  `lds` holds T::LDS_DOUBLES.
template <class T, class LA, class LB>
__device__ __forceinline__ void mma_loop(const LA &la, const LB &lb, int m0, int M, int n0, int N,
                                         int kbeg, int kend, Acc<T> &acc, double *lds) {
  if (kbeg >= kend) return;
  const int tid = threadIdx.x;
  Lds<T> L(lds);
  double2 ra[T::EA], rb[T::EB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < T::EA; ++e) {
      const int idx = tid + e * T::NT;
      int r, k;
      if (LA::kFastSecond) { r = idx / T::BK; k = idx % T::BK; }
      else { r = idx % T::BM; k = idx / T::BM; }
      const bool ok = (idx < T::BM * T::BK) && (m0 + r < M) && (k0 + k < kend);
      ra[e] = ok ? la(m0 + r, k0 + k) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int e = 0; e < T::EB; ++e) {
      const int idx = tid + e * T::NT;
      int k, c;
      if (LB::kFastSecond) { k = idx / T::BN; c = idx % T::BN; }
      else { k = idx % T::BK; c = idx / T::BK; }
      const bool ok = (idx < T::BK * T::BN) && (n0 + c < N) && (k0 + k < kend);
      rb[e] = ok ? lb(k0 + k, n0 + c) : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int e = 0; e < T::EA; ++e) {
      const int idx = tid + e * T::NT;
      if (idx < T::BM * T::BK) {
        int r, k;
        if (LA::kFastSecond) { r = idx / T::BK; k = idx % T::BK; }
        else { r = idx % T::BM; k = idx / T::BM; }
        L.ar[k * T::PA + r] = ra[e].x;
        L.ai[k * T::PA + r] = ra[e].y;
      }
    }
#pragma unroll
    for (int e = 0; e < T::EB; ++e) {
      const int idx = tid + e * T::NT;
      if (idx < T::BK * T::BN) {
        int k, c;
        if (LB::kFastSecond) { k = idx / T::BN; c = idx % T::BN; }
        else { k = idx % T::BK; c = idx / T::BK; }
        L.br[k * T::PB + c] = rb[e].x;
        L.bi[k * T::PB + c] = rb[e].y;
      }
    }
  };
  gload(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += T::BK) {
    __syncthreads();  // the previous stage's MFMAs have read their operands
    sstore();
    __syncthreads();
    if (k0 + T::BK < kend) gload(k0 + T::BK);
    mma_stage<T>(L, acc);
  }
}

// Visit every accumulator element with its (row, col) inside the BM x BN tile.
template <class T, class F>
__device__ __forceinline__ void acc_foreach(const Acc<T> &acc, F &&f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wm * T::FM * 16 + i * 16 + 4 * q + (lane >> 4);
        const int c = wn * T::FN * 16 + j * 16 + (lane & 15);
        f(r, c, acc.value(i, j, q));
      }
}

}  // namespace ss
