// Complex tile engine on the gfx950 BF16 matrix cores (v_mfma_f32_16x16x32_bf16) with operands split
// into BF16 terms and FP32 accumulation.
//
// Every real operand value x (read as FP64, rounded once to FP32) is split into NS BF16 terms,
// x ~ x_0 + x_1 + ... with x_0 = bf16(x) and x_t = bf16(x - x_0 - ... - x_{t-1}), each rounded to
// nearest; with NS = 3 the terms carry the FP32 value to within about 2^-24 of itself.  A real product
// x y is accumulated as the sum of the term products x_i y_j with i + j < NS (the dropped ones are of
// order 2^-8NS relative), so NS = 3 gives six BF16 products per real product at FP32-level accuracy.
// A complex product takes four real ones: Re += Ar Br - Ai Bi (the two kept in separate accumulators
// and subtracted at the end), Im += Ar Bi + Ai Br.
//
// Operands are staged in LDS as BF16 planes [component][term][row][p] with the stage's k positions p
// contiguous (A as rows of the left operand, B as columns of the right one), pitch BK + 8 elements
// (16-byte rows that walk the banks), so a fragment of eight positions is one 16-byte LDS read.  A
// product does not depend on the order of its k terms, so A and B share one order: position 8c + i holds
// k = c + (BK/8) i.  A thread that reads eight values along a row of memory then reads them BK/8 apart,
// and the threads of one load instruction cover whole runs of the row instead of single elements.
//
// Register layout of v_mfma_f32_16x16x32_bf16 (wave64), measured: lane l supplies row l % 16 of A and
// column l % 16 of B, each with eight k values (any assignment of k to the lane groups l / 16 that A
// and B share gives the same product; here the stage position 8 (l / 16) + i); D lane l, element j holds
// D[4 (l / 16) + j][l % 16], as for v_mfma_f32_16x16x4_f32.
#pragma once

#include "tile.hpp"

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

namespace ss {

template <int BM_, int BN_, int BK_, int WM_, int WN_, int NS_>
struct TileCfgB {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_, NS = NS_;
  static constexpr int NT = 64 * WM * WN;
  static constexpr int FM = BM / (16 * WM);
  static constexpr int FN = BN / (16 * WN);
  static constexpr int PK = BK + 8;       // LDS row pitch in BF16 elements
  static constexpr int KC = BK / 8;       // 8-value chunks per row and stage
  static constexpr int PLANE_A = BM * PK, PLANE_B = BN * PK;
  static constexpr int LDS_BYTES = 2 * (2 * NS * (PLANE_A + PLANE_B));
  static constexpr int CA = (BM * KC + NT - 1) / NT;  // A chunks per thread and stage
  static constexpr int CB = (BN * KC + NT - 1) / NT;
  static_assert(FM >= 1 && FN >= 1, "tile smaller than one MFMA block per wave");
  static_assert(FM * 16 * WM == BM && FN * 16 * WN == BN, "tile not a multiple of the wave grid");
  static_assert(BK % 32 == 0, "BK must be a multiple of the MFMA depth");
  static_assert(NS >= 1 && NS <= 3, "one to three BF16 terms");
};

template <class T>
struct AccB {
  v4f rp[T::FM][T::FN];  // sum Ar Br
  v4f rn[T::FM][T::FN];  // sum Ai Bi
  v4f im[T::FM][T::FN];  // sum Ar Bi + Ai Br
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < T::FM; ++i)
#pragma unroll
      for (int j = 0; j < T::FN; ++j) {
        rp[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
        rn[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
        im[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
      }
  }
};

// Two FP32 values to a packed pair of BF16 (round to nearest even): element 0 in the low half.
__device__ __forceinline__ unsigned bf16_pair(float a, float b) {
  const v2bf h = __builtin_convertvector((v2f){a, b}, v2bf);
  return __builtin_bit_cast(unsigned, h);
}

// Split eight FP32 values into NS planes of eight BF16 terms (one uint4 per plane).
template <int NS>
__device__ __forceinline__ void split8(float (&r)[8], uint4 (&out)[NS]) {
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    unsigned w[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      w[p] = bf16_pair(r[2 * p], r[2 * p + 1]);
      if (t + 1 < NS) {  // the remainders are exact in FP32
        r[2 * p] -= __uint_as_float(w[p] << 16);
        r[2 * p + 1] -= __uint_as_float(w[p] & 0xffff0000u);
      }
    }
    out[t] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// acc(r, c) += sum_k A(r, k) B(k, c) over rows [m0, min(m0+BM, M)), columns [n0, min(n0+BN, N)) and
// k in [kbeg, kend); loaders as for mma_loop (la(r, k), lb(k, c) return FP64 complex values; kFastSecond
// tells which index is contiguous in memory).  lds: T::LDS_BYTES bytes.
template <class T, class LA, class LB>
__device__ __forceinline__ void mma_loop_bf(const LA &la, const LB &lb, int m0, int M, int n0, int N, int kbeg,
                                            int kend, AccB<T> &acc, unsigned short *lds) {
  if (kbeg >= kend) return;
  constexpr int NS = T::NS;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  // planes: A [comp][term][BM][PK], then B [comp][term][BN][PK]
  unsigned short *sa = lds, *sb = lds + 2 * NS * T::PLANE_A;
  double2 ra[T::CA][8], rb[T::CB][8];
  auto a_chunk = [&](int idx, int &r, int &c) {
    if (LA::kFastSecond) { r = idx / T::KC; c = idx % T::KC; }
    else { r = idx % T::BM; c = idx / T::BM; }
  };
  auto b_chunk = [&](int idx, int &n, int &c) {
    if (LB::kFastSecond) { n = idx % T::BN; c = idx / T::BN; }
    else { n = idx / T::KC; c = idx % T::KC; }
  };
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < T::CA; ++e) {
      const int idx = tid + e * T::NT;
      int r, c;
      a_chunk(idx, r, c);
      const bool row_ok = idx < T::BM * T::KC && m0 + r < M;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + c + T::KC * i;
        ra[e][i] = (row_ok && k < kend) ? la(m0 + r, k) : make_double2(0.0, 0.0);
      }
    }
#pragma unroll
    for (int e = 0; e < T::CB; ++e) {
      const int idx = tid + e * T::NT;
      int n, c;
      b_chunk(idx, n, c);
      const bool col_ok = idx < T::BN * T::KC && n0 + n < N;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + c + T::KC * i;
        rb[e][i] = (col_ok && k < kend) ? lb(k, n0 + n) : make_double2(0.0, 0.0);
      }
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int e = 0; e < T::CA; ++e) {
      const int idx = tid + e * T::NT;
      if (idx < T::BM * T::KC) {
        int r, c;
        a_chunk(idx, r, c);
        float fr[8], fi[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          fr[i] = (float)ra[e][i].x;
          fi[i] = (float)ra[e][i].y;
        }
        uint4 tr[NS], ti[NS];
        split8<NS>(fr, tr);
        split8<NS>(fi, ti);
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          *reinterpret_cast<uint4 *>(sa + (0 * NS + t) * T::PLANE_A + r * T::PK + 8 * c) = tr[t];
          *reinterpret_cast<uint4 *>(sa + (1 * NS + t) * T::PLANE_A + r * T::PK + 8 * c) = ti[t];
        }
      }
    }
#pragma unroll
    for (int e = 0; e < T::CB; ++e) {
      const int idx = tid + e * T::NT;
      if (idx < T::BN * T::KC) {
        int n, c;
        b_chunk(idx, n, c);
        float fr[8], fi[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          fr[i] = (float)rb[e][i].x;
          fi[i] = (float)rb[e][i].y;
        }
        uint4 tr[NS], ti[NS];
        split8<NS>(fr, tr);
        split8<NS>(fi, ti);
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          *reinterpret_cast<uint4 *>(sb + (0 * NS + t) * T::PLANE_B + n * T::PK + 8 * c) = tr[t];
          *reinterpret_cast<uint4 *>(sb + (1 * NS + t) * T::PLANE_B + n * T::PK + 8 * c) = ti[t];
        }
      }
    }
  };
  const int arow = wm * T::FM * 16 + (lane & 15);
  const int bcol = wn * T::FN * 16 + (lane & 15);
  const int koff = 8 * (lane >> 4);
  gload(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += T::BK) {
    __syncthreads();
    sstore();
    __syncthreads();
    if (k0 + T::BK < kend) gload(k0 + T::BK);
#pragma unroll
    for (int kc = 0; kc < T::BK / 32; ++kc) {
      const int kk = kc * 32 + koff;
      v8bf ar[T::FM][NS], ai[T::FM][NS];
#pragma unroll
      for (int i = 0; i < T::FM; ++i)
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const int o = (arow + i * 16) * T::PK + kk;
          ar[i][t] = *reinterpret_cast<const v8bf *>(sa + (0 * NS + t) * T::PLANE_A + o);
          ai[i][t] = *reinterpret_cast<const v8bf *>(sa + (1 * NS + t) * T::PLANE_A + o);
        }
#pragma unroll
      for (int j = 0; j < T::FN; ++j) {
        v8bf br[NS], bi[NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const int o = (bcol + j * 16) * T::PK + kk;
          br[t] = *reinterpret_cast<const v8bf *>(sb + (0 * NS + t) * T::PLANE_B + o);
          bi[t] = *reinterpret_cast<const v8bf *>(sb + (1 * NS + t) * T::PLANE_B + o);
        }
#pragma unroll
        for (int i = 0; i < T::FM; ++i)
#pragma unroll
          for (int ta = 0; ta < NS; ++ta)
#pragma unroll
            for (int tb = 0; ta + tb < NS; ++tb) {
              acc.rp[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar[i][ta], br[tb], acc.rp[i][j], 0, 0, 0);
              acc.rn[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[i][ta], bi[tb], acc.rn[i][j], 0, 0, 0);
              acc.im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar[i][ta], bi[tb], acc.im[i][j], 0, 0, 0);
              acc.im[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai[i][ta], br[tb], acc.im[i][j], 0, 0, 0);
            }
      }
    }
  }
}

template <class T, class F>
__device__ __forceinline__ void acc_foreach_bf(const AccB<T> &acc, F &&f) {
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
        f(r, c, make_double2((double)acc.rp[i][j][q] - (double)acc.rn[i][j][q], (double)acc.im[i][j][q]));
      }
}

}  // namespace ss
