// Measured ceilings of the GPU the context runs on: the denominators that the roofline fractions are
// checked against (the datasheet peaks are FP64 matrix and vector 78.6 TF/s, FP32 matrix 157.3 TF/s,
// HBM 8 TB/s).  Each figure is the rate of a kernel that does nothing but that one thing:
//   FP64 / FP32 matrix: v_mfma_f64_16x16x4_f64 / v_mfma_f32_16x16x4_f32 on independent accumulators
//   (2048 flops per wave instruction), operands in registers (512-thread workgroups: with 256 the
//   compiler shuttles the accumulators between VGPRs and AGPRs every iteration);
//   FP64 vector: independent fused multiply-add chains;
//   copy: a grid-stride copy of 512 MiB (bytes read + bytes written per second).
#include "common.hpp"
#include "drivers.hpp"

namespace ss {

typedef float v4f_c __attribute__((ext_vector_type(4)));

template <int NACC>
__global__ void __launch_bounds__(512) k_ceil_mfma64(double *out, int iters, double seed) {
  v4d acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
  const double a = seed + threadIdx.x * 1e-3, b = seed * 0.5 + threadIdx.x * 1e-4;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NACC; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;  // keeps the loop alive
}

template <int NACC>
__global__ void __launch_bounds__(512) k_ceil_mfma32(double *out, int iters, float seed) {
  v4f_c acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = v4f_c{0.f, 0.f, 0.f, 0.f};
  const float a = seed + threadIdx.x * 1e-3f, b = seed * 0.5f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < NACC; ++i) s += acc[i][0] + acc[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int NACC>
__global__ void __launch_bounds__(512) k_ceil_valu64(double *out, int iters, double seed) {
  double acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = i * 1e-3;
  const double a = seed + threadIdx.x * 1e-3, b = 0.999999;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = fma(acc[i], b, a);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NACC; ++i) s += acc[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_ceil_copy(const double2 *__restrict__ src, double2 *__restrict__ dst, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

ss_status measure_ceilings(ss_ctx *ctx, double *ceil) {
  constexpr int kBlocks = 2048, kThreads = 512, kAcc = 8;
  constexpr long kCopy = (512L << 20) / sizeof(double2);  // elements of 512 MiB
  void *wOut, *wCopy;
  SS_TRY(workspace(ctx, kSlotMisc, sizeof(double) * kBlocks * kThreads, &wOut));
  SS_TRY(workspace(ctx, kSlotM, sizeof(double2) * 2 * (size_t)kCopy, &wCopy));
  double *out = (double *)wOut;
  double2 *src = (double2 *)wCopy, *dst = src + kCopy;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(ctx, SS_ERR_DEVICE, "ss_measure_ceilings: event creation failed");
  // best of five timed launches after two untimed ones (the clocks ramp up under load)
  auto timed = [&](auto launch) -> double {
    launch();
    launch();
    double best = -1.0;
    for (int rep = 0; rep < 5; ++rep) {
      (void)hipEventRecord(e0, ctx->stream);
      launch();
      (void)hipEventRecord(e1, ctx->stream);
      float ms = 0.f;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
      if (best < 0 || ms * 1e-3 < best) best = ms * 1e-3;
    }
    return best;
  };
  const int iters = 4096;
  const double mfma_flops = (double)kBlocks * (kThreads / 64) * iters * kAcc * 2048.0;
  // a first pass over every kernel brings the clocks up before anything is timed
  hipLaunchKernelGGL(k_ceil_valu64<16>, dim3(kBlocks), dim3(kThreads), 0, ctx->stream, out, 8192, 1.0);
  const double t64 = timed([&] {
    hipLaunchKernelGGL(k_ceil_mfma64<kAcc>, dim3(kBlocks), dim3(kThreads), 0, ctx->stream, out, iters, 1.0);
  });
  const double t32 = timed([&] {
    hipLaunchKernelGGL(k_ceil_mfma32<kAcc>, dim3(kBlocks), dim3(kThreads), 0, ctx->stream, out, iters, 1.0f);
  });
  const int viters = 8192;
  const double valu_flops = (double)kBlocks * kThreads * viters * 16 * 2.0;
  const double tv = timed([&] {
    hipLaunchKernelGGL(k_ceil_valu64<16>, dim3(kBlocks), dim3(kThreads), 0, ctx->stream, out, viters, 1.0);
  });
  const double tc = timed([&] {
    hipLaunchKernelGGL(k_ceil_copy, dim3(8192), dim3(256), 0, ctx->stream, src, dst, kCopy);
  });
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (t64 <= 0 || t32 <= 0 || tv <= 0 || tc <= 0) return fail(ctx, SS_ERR_DEVICE, "ss_measure_ceilings: timing failed");
  ceil[0] = mfma_flops / t64 * 1e-12;
  ceil[1] = mfma_flops / t32 * 1e-12;
  ceil[2] = valu_flops / tv * 1e-12;
  ceil[3] = 2.0 * sizeof(double2) * kCopy / tc * 1e-9;
  return check_launch(ctx, "ss_measure_ceilings");
}

}  // namespace ss
