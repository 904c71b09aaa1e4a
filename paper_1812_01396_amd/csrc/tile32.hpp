// Complex tile engine in FP32 on the gfx950 matrix cores (v_mfma_f32_16x16x4_f32), FP32 accumulation.
//
// Same structure as the FP64 engine in tile.hpp (complex = four real MFMAs, operands staged in LDS as
// real and imaginary planes [k][m] / [k][n]); the loaders still read FP64 operands, which are rounded
// to FP32 when they are staged, and results leave the engine as FP64 values for the caller's epilogue.
// Used for the recursion products of the mixed-precision path; the LU, the corner system and all
// residuals stay FP64.
//
// Register layout of v_mfma_f32_16x16x4_f32 (wave64), measured: A (16x4): lane l holds A[l % 16][l / 16];
// B (4x16): lane l holds B[l / 16][l % 16]; D (16x16): lane l, element j holds D[4*(l / 16) + j][l % 16]
// (the inputs are arranged as for the FP64 instruction, the output rows are not).
#pragma once

#include "tile.hpp"

typedef float v4f __attribute__((ext_vector_type(4)));

namespace ss {

template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct TileCfg32 {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
  static constexpr int NT = 64 * WM * WN;
  static constexpr int FM = BM / (16 * WM);
  static constexpr int FN = BN / (16 * WN);
  static constexpr int PA = BM + 1;
  static constexpr int PB = BN + 1;
  static constexpr int LDS_FLOATS = 2 * BK * PA + 2 * BK * PB;
  static constexpr int EA = (BM * BK + NT - 1) / NT;
  static constexpr int EB = (BK * BN + NT - 1) / NT;
  static constexpr bool G3 = false;  // three-product complex multiply (TileCfg32G3)
  static_assert(FM >= 1 && FN >= 1, "tile smaller than one MFMA block per wave");
  static_assert(FM * 16 * WM == BM && FN * 16 * WN == BN, "tile not a multiple of the wave grid");
  static_assert(BK % 4 == 0, "BK must be a multiple of the MFMA depth");
};

// Gauss's three-product complex multiply, as for the FP64 engine: re = sum Ar Br, im = sum (Ar + Ai)(Br + Bi),
// x = sum Ai Bi; the parts are combined in FP32 before the result leaves the engine.
template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct TileCfg32G3 : TileCfg32<BM_, BN_, BK_, WM_, WN_> {
  static constexpr bool G3 = true;
};

template <class T>
struct Acc32 {
  static constexpr int XM = T::G3 ? T::FM : 1, XN = T::G3 ? T::FN : 1;
  v4f re[T::FM][T::FN];
  v4f im[T::FM][T::FN];
  v4f x[XM][XN];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < T::FM; ++i)
#pragma unroll
      for (int j = 0; j < T::FN; ++j) {
        re[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
        im[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
      }
    if constexpr (T::G3) {
#pragma unroll
      for (int i = 0; i < XM; ++i)
#pragma unroll
        for (int j = 0; j < XN; ++j) x[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  }
  __device__ __forceinline__ double2 value(int i, int j, int q) const {
    if constexpr (T::G3) {
      const float t1 = re[i][j][q], t2 = x[i][j][q];
      return make_double2((double)(t1 - t2), (double)(im[i][j][q] - t1 - t2));
    } else {
      return make_double2((double)re[i][j][q], (double)im[i][j][q]);
    }
  }
};

template <class T, class LA, class LB>
__device__ __forceinline__ void mma_loop32(const LA &la, const LB &lb, int m0, int M, int n0, int N, int kbeg,
                                           int kend, Acc32<T> &acc, float *lds) {
  if (kbeg >= kend) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  float *sar = lds, *sai = sar + T::BK * T::PA, *sbr = sai + T::BK * T::PA, *sbi = sbr + T::BK * T::PB;
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
        sar[k * T::PA + r] = (float)ra[e].x;
        sai[k * T::PA + r] = (float)ra[e].y;
      }
    }
#pragma unroll
    for (int e = 0; e < T::EB; ++e) {
      const int idx = tid + e * T::NT;
      if (idx < T::BK * T::BN) {
        int k, c;
        if (LB::kFastSecond) { k = idx / T::BN; c = idx % T::BN; }
        else { k = idx % T::BK; c = idx / T::BK; }
        sbr[k * T::PB + c] = (float)rb[e].x;
        sbi[k * T::PB + c] = (float)rb[e].y;
      }
    }
  };
  const int mbase = wm * T::FM * 16 + (lane & 15);
  const int nbase = wn * T::FN * 16 + (lane & 15);
  gload(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += T::BK) {
    __syncthreads();
    sstore();
    __syncthreads();
    if (k0 + T::BK < kend) gload(k0 + T::BK);
#pragma unroll
    for (int ks = 0; ks < T::BK / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      if constexpr (T::G3) {
        float ar[T::FM], ai[T::FM], as[T::FM], br[T::FN], bi[T::FN], bs[T::FN];
#pragma unroll
        for (int i = 0; i < T::FM; ++i) {
          ar[i] = sar[kr * T::PA + mbase + i * 16];
          ai[i] = sai[kr * T::PA + mbase + i * 16];
          as[i] = ar[i] + ai[i];
        }
#pragma unroll
        for (int j = 0; j < T::FN; ++j) {
          br[j] = sbr[kr * T::PB + nbase + j * 16];
          bi[j] = sbi[kr * T::PB + nbase + j * 16];
          bs[j] = br[j] + bi[j];
        }
#pragma unroll
        for (int i = 0; i < T::FM; ++i)
#pragma unroll
          for (int j = 0; j < T::FN; ++j) {
            acc.re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], br[j], acc.re[i][j], 0, 0, 0);
            acc.x[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], bi[j], acc.x[i][j], 0, 0, 0);
            acc.im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[i], bs[j], acc.im[i][j], 0, 0, 0);
          }
      } else {
        float ar[T::FM], ai[T::FM], an[T::FM], br[T::FN], bi[T::FN];
#pragma unroll
        for (int i = 0; i < T::FM; ++i) {
          ar[i] = sar[kr * T::PA + mbase + i * 16];
          ai[i] = sai[kr * T::PA + mbase + i * 16];
          an[i] = -ai[i];
        }
#pragma unroll
        for (int j = 0; j < T::FN; ++j) {
          br[j] = sbr[kr * T::PB + nbase + j * 16];
          bi[j] = sbi[kr * T::PB + nbase + j * 16];
        }
#pragma unroll
        for (int i = 0; i < T::FM; ++i)
#pragma unroll
          for (int j = 0; j < T::FN; ++j) {
            acc.re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], br[j], acc.re[i][j], 0, 0, 0);
            acc.im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bi[j], acc.im[i][j], 0, 0, 0);
            acc.re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(an[i], bi[j], acc.re[i][j], 0, 0, 0);
            acc.im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], br[j], acc.im[i][j], 0, 0, 0);
          }
      }
    }
  }
}

template <class T, class F>
__device__ __forceinline__ void acc_foreach32(const Acc32<T> &acc, F &&f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
#pragma unroll
  for (int i = 0; i < T::FM; ++i)
#pragma unroll
    for (int j = 0; j < T::FN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wm * T::FM * 16 + i * 16 + 4 * (lane >> 4) + q;
        const int c = wn * T::FN * 16 + j * 16 + (lane & 15);
        f(r, c, acc.value(i, j, q));
      }
}

}  // namespace ss
