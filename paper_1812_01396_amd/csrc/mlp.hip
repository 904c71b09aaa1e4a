// Multilayer perceptron of the learned warm start: training and inference kernels in FP32.
//
// The network maps features of (E, k) to a starting iterate for Sigma_L and Sigma_R: tanh hidden layers,
// a linear output layer, mean squared error against standardized targets, Adam updates.  Every product
// is one FP32 matrix-core GEMM (v_mfma_f32_16x16x4_f32, FP32 accumulation) with its epilogue fused:
//     forward          A_{l+1} = tanh(A_l W_l + b_l)            (linear for the last layer)
//     weight gradient  dW_l = A_l^T dZ_l,  db_l = column sums of dZ_l
//     back-propagation dZ_{l-1} = (dZ_l W_l^T) * (1 - A_l^2)
// Products with a long inner dimension and few output tiles are split over the inner dimension and the
// partial tiles are summed (with the epilogue) by a second kernel.
// Parameters are packed layer by layer: W_l [d_l][d_{l+1}] row-major, then b_l [d_{l+1}].
#include <algorithm>
#include <cmath>

#include "drivers.hpp"

typedef float v4f __attribute__((ext_vector_type(4)));

namespace ss {

namespace {

constexpr int SBM = 64, SBN = 64, SBK = 16, SNT = 256;
constexpr int SPA = SBM + 1, SPB = SBN + 1;

enum Epi { kStore = 0, kBiasTanh = 1, kBias = 2, kTanhGrad = 3 };

__device__ __forceinline__ float epilogue(int epi, float v, int r, int c, const float *bias, const float *aux,
                                          int ldaux) {
  if (epi == kBiasTanh) return tanhf(v + bias[c]);
  if (epi == kBias) return v + bias[c];
  if (epi == kTanhGrad) {
    const float a = aux[(long)r * ldaux + c];
    return v * (1.0f - a * a);
  }
  return v;
}

// C (or the z-th partial of C) = op(A)[M x K-range] * op(B)[K-range x N]; op(A) = A or A^T as stored
// row-major ([M][K] or [K][M]), likewise op(B) ([K][N] or [N][K]).
template <bool TA, bool TB>
__global__ void __launch_bounds__(SNT) k_sgemm(const float *A, int lda, const float *B, int ldb, float *C, int ldc,
                                                int M, int N, int K, int kchunk, long zstride, int epi,
                                                const float *bias, const float *aux, int ldaux) {
  __shared__ float sa[SBK * SPA], sb[SBK * SPB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int m0 = blockIdx.y * SBM, n0 = blockIdx.x * SBN;
  const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  constexpr int EL = SBM * SBK / SNT;  // 4 elements of each operand per thread and stage
  float ra[EL], rb[EL];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      const int idx = tid + e * SNT;
      int r, k;
      if (TA) { r = idx % SBM; k = idx / SBM; } else { r = idx / SBK; k = idx % SBK; }
      const int gr = m0 + r, gk = k0 + k;
      ra[e] = (gr < M && gk < kend) ? (TA ? A[(long)gk * lda + gr] : A[(long)gr * lda + gk]) : 0.f;
      int c, kb;
      if (TB) { c = idx / SBK; kb = idx % SBK; } else { c = idx % SBN; kb = idx / SBN; }
      const int gc = n0 + c, gkb = k0 + kb;
      rb[e] = (gc < N && gkb < kend) ? (TB ? B[(long)gc * ldb + gkb] : B[(long)gkb * ldb + gc]) : 0.f;
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      const int idx = tid + e * SNT;
      int r, k;
      if (TA) { r = idx % SBM; k = idx / SBM; } else { r = idx / SBK; k = idx % SBK; }
      sa[k * SPA + r] = ra[e];
      int c, kb;
      if (TB) { c = idx / SBK; kb = idx % SBK; } else { c = idx % SBN; kb = idx / SBN; }
      sb[kb * SPB + c] = rb[e];
    }
  };
  if (kbeg < kend) gload(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += SBK) {
    __syncthreads();
    sstore();
    __syncthreads();
    if (k0 + SBK < kend) gload(k0 + SBK);
#pragma unroll
    for (int ks = 0; ks < SBK / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      float av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = sa[kr * SPA + wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = sb[kr * SPB + wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
  }
  float *Cz = C + (long)blockIdx.z * zstride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // FP32 16x16x4 output: lane l, element q holds row 4 (l / 16) + q, column l % 16
        const int r = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + q;
        const int c = n0 + wn * 32 + j * 16 + (lane & 15);
        if (r < M && c < N) Cz[(long)r * ldc + c] = epilogue(epi, acc[i][j][q], r, c, bias, aux, ldaux);
      }
}

__global__ void k_splitk_sum(const float *part, int nsplit, long zstride, int M, int N, float *C, int ldc, int epi,
                             const float *bias, const float *aux, int ldaux) {
  const long total = (long)M * N;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int r = idx / N, c = idx % N;
    float v = 0.f;
    for (int z = 0; z < nsplit; ++z) v += part[z * zstride + (long)r * N + c];
    C[(long)r * ldc + c] = epilogue(epi, v, r, c, bias, aux, ldaux);
  }
}

// db[c] = sum_r dz[r][c]
__global__ void k_colsum(const float *dz, int n, int d, float *db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d) return;
  float s = 0.f;
  for (int r = 0; r < n; ++r) s += dz[(long)r * d + c];
  db[c] = s;
}

// dY = 2 (Y - T) / (n d); loss += sum (Y - T)^2 / (n d)
__global__ void k_mse(const float *Y, const float *T, long count, float *dY, double *loss) {
  __shared__ double red[4];
  double s = 0.0;
  const float scale = 2.0f / (float)count;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
    const float r = Y[i] - T[i];
    dY[i] = scale * r;
    s += (double)r * r;
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, (red[0] + red[1] + red[2] + red[3]) / (double)count);
}

__global__ void k_zero_d1(double *p) { *p = 0.0; }

__global__ void k_adam(float *p, const float *g, float *m, float *v, long count, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

// features of (E, k): [E/es, cos k, sin k, sin(j pi E/es), cos(j pi E/es) (j = 1..nf), cos(j k), sin(j k)
// (j = 2..nf+1)]
__global__ void k_features(const double *E, const double *kz, int n, int nf, double es, float *X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int F = 3 + 4 * nf;
  const double e = E[i], k = kz[i];
  float *x = X + (long)i * F;
  x[0] = (float)(e / es);
  x[1] = (float)cos(k);
  x[2] = (float)sin(k);
  for (int j = 1; j <= nf; ++j) {
    x[1 + 2 * j] = (float)sin(j * M_PI * e / es);
    x[2 + 2 * j] = (float)cos(j * M_PI * e / es);
  }
  for (int j = 2; j <= nf + 1; ++j) {
    x[3 + 2 * nf + 2 * (j - 2)] = (float)cos(j * k);
    x[4 + 2 * nf + 2 * (j - 2)] = (float)sin(j * k);
  }
}

// component q of the encoding [Re S_L, Im S_L, Re S_R, Im S_R] of instance i (sigma [n][2][s][s])
__device__ __forceinline__ double enc_at(const double2 *sigma, long ss2, int i, long q) {
  const int part = (int)(q / ss2);
  const long o = q % ss2;
  const double2 v = sigma[((long)i * 2 + (part >> 1)) * ss2 + o];
  return (part & 1) ? v.y : v.x;
}

// per component: mean and standard deviation over n instances (std floored at floor * max std)
__global__ void k_moments(const double2 *sigma, int n, long ss2, float *mean, float *std) {
  const long D = 4 * ss2;
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < D; q += (long)gridDim.x * blockDim.x) {
    double s = 0.0, s2 = 0.0;
    for (int i = 0; i < n; ++i) {
      const double v = enc_at(sigma, ss2, i, q);
      s += v;
      s2 += v * v;
    }
    const double mu = s / n;
    mean[q] = (float)mu;
    std[q] = (float)sqrt(fmax(s2 / n - mu * mu, 0.0));
  }
}

__global__ void k_std_floor(float *std, long D, float floor_abs) {
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < D; q += (long)gridDim.x * blockDim.x)
    std[q] = fmaxf(std[q], floor_abs);
}

__global__ void k_encode(const double2 *sigma, int n, long ss2, const float *mean, const float *std, float *y) {
  const long D = 4 * ss2, total = (long)n * D;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / D);
    const long q = idx % D;
    y[idx] = (float)((enc_at(sigma, ss2, i, q) - mean[q]) / std[q]);
  }
}

__global__ void k_decode(const float *y, int n, long ss2, const float *mean, const float *std, double2 *sigma) {
  const long total = (long)n * 2 * ss2;
  const long D = 4 * ss2;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / (2 * ss2));
    const long rem = idx % (2 * ss2);
    const int side = (int)(rem / ss2);
    const long o = rem % ss2;
    const long qr = (2 * side) * ss2 + o, qi = (2 * side + 1) * ss2 + o;
    const float *yi = y + (long)i * D;
    sigma[idx] = make_double2((double)yi[qr] * std[qr] + mean[qr], (double)yi[qi] * std[qi] + mean[qi]);
  }
}

int grid1(long n) { return (int)std::min<long>((n + 255) / 256, 8192); }

}  // namespace

ss_status sgemm(ss_ctx *ctx, bool ta, bool tb, int epi, const float *A, int lda, const float *B, int ldb, float *C,
                int ldc, int M, int N, int K, const float *bias, const float *aux, int ldaux) {
  if (M <= 0 || N <= 0) return SS_OK;
  const int tiles = cdiv(N, SBN) * cdiv(M, SBM);
  int nsplit = 1;
  if (tiles < 512 && K > 2048) nsplit = std::min(64, std::max(1, std::min(cdiv(K, 2048), cdiv(1024, tiles))));
  const int kchunk = cdiv(cdiv(K, nsplit), SBK) * SBK;
  nsplit = cdiv(K, kchunk);
  float *out = C;
  long zstride = 0;
  int ldo = ldc;
  if (nsplit > 1) {
    void *w;
    SS_TRY(workspace(ctx, kSlotMlp, sizeof(float) * (size_t)nsplit * M * N, &w));
    out = (float *)w;
    zstride = (long)M * N;
    ldo = N;
  }
  dim3 grid(cdiv(N, SBN), cdiv(M, SBM), nsplit);
  const int e0 = nsplit > 1 ? kStore : epi;
  if (ta && tb) hipLaunchKernelGGL((k_sgemm<true, true>), grid, dim3(SNT), 0, ctx->stream, A, lda, B, ldb, out, ldo, M, N, K, kchunk, zstride, e0, bias, aux, ldaux);
  else if (ta) hipLaunchKernelGGL((k_sgemm<true, false>), grid, dim3(SNT), 0, ctx->stream, A, lda, B, ldb, out, ldo, M, N, K, kchunk, zstride, e0, bias, aux, ldaux);
  else if (tb) hipLaunchKernelGGL((k_sgemm<false, true>), grid, dim3(SNT), 0, ctx->stream, A, lda, B, ldb, out, ldo, M, N, K, kchunk, zstride, e0, bias, aux, ldaux);
  else hipLaunchKernelGGL((k_sgemm<false, false>), grid, dim3(SNT), 0, ctx->stream, A, lda, B, ldb, out, ldo, M, N, K, kchunk, zstride, e0, bias, aux, ldaux);
  if (nsplit > 1)
    hipLaunchKernelGGL(k_splitk_sum, dim3(grid1((long)M * N)), dim3(256), 0, ctx->stream, (const float *)out, nsplit,
                       zstride, M, N, C, ldc, epi, bias, aux, ldaux);
  return check_launch(ctx, "sgemm");
}

size_t mlp_param_count(int nlayer, const int *dims) {
  size_t t = 0;
  for (int l = 0; l < nlayer; ++l) t += (size_t)dims[l] * dims[l + 1] + dims[l + 1];
  return t;
}

static size_t w_off(const int *dims, int l) {
  size_t t = 0;
  for (int i = 0; i < l; ++i) t += (size_t)dims[i] * dims[i + 1] + dims[i + 1];
  return t;
}

static size_t act_off(const int *dims, int l, int n) {  // output of layer l (1-based) in the acts buffer
  size_t t = 0;
  for (int i = 1; i < l; ++i) t += (size_t)n * dims[i];
  return t;
}

ss_status mlp_forward(ss_ctx *ctx, int nlayer, const int *dims, const float *params, int n, const float *X,
                      float *acts) {
  for (int l = 0; l < nlayer; ++l) {
    const float *in = l == 0 ? X : acts + act_off(dims, l, n);
    float *out = acts + act_off(dims, l + 1, n);
    const float *W = params + w_off(dims, l);
    const float *b = W + (size_t)dims[l] * dims[l + 1];
    SS_TRY(sgemm(ctx, false, false, l < nlayer - 1 ? kBiasTanh : kBias, in, dims[l], W, dims[l + 1], out,
                 dims[l + 1], n, dims[l + 1], dims[l], b, nullptr, 0));
  }
  return SS_OK;
}

ss_status mlp_backward(ss_ctx *ctx, int nlayer, const int *dims, const float *params, int n, const float *X,
                       const float *acts, const float *target, float *grads, double *loss) {
  int dmax = 0;
  for (int l = 1; l <= nlayer; ++l) dmax = std::max(dmax, dims[l]);
  void *w;
  SS_TRY(workspace(ctx, kSlotMlpDz, sizeof(float) * (size_t)2 * n * dmax, &w));
  float *dz = (float *)w, *dz2 = dz + (size_t)n * dmax;
  const long cnt = (long)n * dims[nlayer];
  hipLaunchKernelGGL(k_zero_d1, dim3(1), dim3(1), 0, ctx->stream, loss);
  hipLaunchKernelGGL(k_mse, dim3(grid1(cnt)), dim3(256), 0, ctx->stream, acts + act_off(dims, nlayer, n), target, cnt,
                     dz, loss);
  for (int l = nlayer - 1; l >= 0; --l) {
    const float *in = l == 0 ? X : acts + act_off(dims, l, n);
    float *gW = grads + w_off(dims, l);
    float *gb = gW + (size_t)dims[l] * dims[l + 1];
    SS_TRY(sgemm(ctx, true, false, kStore, in, dims[l], dz, dims[l + 1], gW, dims[l + 1], dims[l], dims[l + 1], n,
                 nullptr, nullptr, 0));
    hipLaunchKernelGGL(k_colsum, dim3(cdiv(dims[l + 1], 256)), dim3(256), 0, ctx->stream, (const float *)dz, n,
                       dims[l + 1], gb);
    if (l > 0) {
      const float *W = params + w_off(dims, l);
      SS_TRY(sgemm(ctx, false, true, kTanhGrad, dz, dims[l + 1], W, dims[l + 1], dz2, dims[l], n, dims[l],
                   dims[l + 1], nullptr, in, dims[l]));
      std::swap(dz, dz2);
    }
  }
  return check_launch(ctx, "mlp_backward");
}

ss_status mlp_adam(ss_ctx *ctx, size_t count, float *params, const float *grads, float *m, float *v, float lr,
                   float b1, float b2, float eps, int step) {
  const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid1((long)count)), dim3(256), 0, ctx->stream, params, grads, m, v, (long)count, lr,
                     b1, b2, eps, bc1, bc2);
  return check_launch(ctx, "mlp_adam");
}

ss_status warm_features(ss_ctx *ctx, int n, const double *E, const double *k, int nfreq, double e_scale, float *X) {
  hipLaunchKernelGGL(k_features, dim3(cdiv(n, 256)), dim3(256), 0, ctx->stream, E, k, n, nfreq, e_scale, X);
  return check_launch(ctx, "warm_features");
}

ss_status sigma_moments(ss_ctx *ctx, int n, int s, const ss_c128 *sigma, float std_floor, float *mean, float *std) {
  const long ss2 = (long)s * s;
  hipLaunchKernelGGL(k_moments, dim3(grid1(4 * ss2)), dim3(256), 0, ctx->stream, (const double2 *)sigma, n, ss2, mean,
                     std);
  hipLaunchKernelGGL(k_std_floor, dim3(grid1(4 * ss2)), dim3(256), 0, ctx->stream, std, 4 * ss2, std_floor);
  return check_launch(ctx, "sigma_moments");
}

ss_status sigma_encode(ss_ctx *ctx, int n, int s, const ss_c128 *sigma, const float *mean, const float *std, float *y) {
  const long ss2 = (long)s * s;
  hipLaunchKernelGGL(k_encode, dim3(grid1((long)n * 4 * ss2)), dim3(256), 0, ctx->stream, (const double2 *)sigma, n, ss2,
                     mean, std, y);
  return check_launch(ctx, "sigma_encode");
}

ss_status sigma_decode(ss_ctx *ctx, int n, int s, const float *y, const float *mean, const float *std, ss_c128 *sigma) {
  const long ss2 = (long)s * s;
  hipLaunchKernelGGL(k_decode, dim3(grid1((long)n * 2 * ss2)), dim3(256), 0, ctx->stream, y, n, ss2, mean, std,
                     (double2 *)sigma);
  return check_launch(ctx, "sigma_decode");
}

}  // namespace ss
