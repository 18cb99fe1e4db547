// probe.hip -- sustained matrix-core rate on this device (measurement aid).
//
// Every wave of n_cu workgroups of 8 waves (two per SIMD, as the BF16 MLP
// kernel runs) issues `iters` blocks of 16 dependent 32x32x16 BF16 MFMAs.
// Kind 0 takes both operands from registers: the matrix pipe's own ceiling.
// Kind 1 reads the A operand of every MFMA from LDS (one 16-byte read per lane,
// three steps ahead), which is the operand traffic of one point block in the
// MLP layers: the ceiling of that data flow, LDS bandwidth included.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dinr.h"
#include "dinr_dev.h"

namespace dinr {

template <int KIND>
__global__ __launch_bounds__(512, 1) void k_probe(int64_t iters, float* __restrict__ sink) {
  constexpr int KC = 16, D = 3;
  __shared__ __align__(16) bf16x8 sA[2 * KC * 64];
  const int lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < 2 * KC * 64; i += blockDim.x) {
    const float v = (float)((i * 37) % 101) * (1.f / 1024.f);
    f32x8 t = {v, -v, v, -v, v, -v, v, -v};
    sA[i] = __builtin_convertvector(t, bf16x8);
  }
  __syncthreads();
  bf16x8 b[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const float v = (float)(lane + c) * (1.f / 4096.f);
    f32x8 t = {v, v, -v, v, v, -v, v, v};
    b[c] = __builtin_convertvector(t, bf16x8);
  }
  f32x16 acc = {};
  for (int64_t it = 0; it < iters; ++it) {
    if (KIND == 0) {
#pragma unroll
      for (int c = 0; c < KC; ++c)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[c], b[KC - 1 - c], acc, 0, 0, 0);
    } else {
      int z = 0;
      asm volatile("" : "+v"(z));  // keeps the reads inside the loop
      const bf16x8* Wp = sA + (it & 1) * KC * 64 + z;
      bf16x8 a[D + 1];
#pragma unroll
      for (int c = 0; c < D; ++c) a[c] = Wp[c * 64 + lane];
      __builtin_amdgcn_sched_group_barrier(0x100, D, 0);
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        if (c + D < KC) a[(c + D) % (D + 1)] = Wp[(c + D) * 64 + lane];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[c % (D + 1)], b[c], acc, 0, 0, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if (c + D < KC) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) s += acc[r];
  if (s == 1234.5f) sink[0] = s;  // keeps the chain alive; never true in practice
}

}  // namespace dinr

extern "C" int dinr_probe_mfma(int kind, int64_t iters, void* stream, double* tflops) {
  using namespace dinr;
  if ((kind != 0 && kind != 1) || iters <= 0 || !tflops) return DINR_EINVAL;
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return DINR_EHIP;
  hipStream_t st = (hipStream_t)stream;
  float* sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = DINR_EHIP;
  if (hipMalloc(&sink, sizeof(float)) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
      hipEventCreate(&e1) == hipSuccess && hipEventRecord(e0, st) == hipSuccess) {
    if (kind == 0) hipLaunchKernelGGL(k_probe<0>, dim3(n_cu), dim3(512), 0, st, iters, sink);
    else hipLaunchKernelGGL(k_probe<1>, dim3(n_cu), dim3(512), 0, st, iters, sink);
    float ms = 0.f;
    if (hipGetLastError() == hipSuccess && hipEventRecord(e1, st) == hipSuccess &&
        hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
        ms > 0.f) {
      const double flop = (double)n_cu * 8 * (double)iters * 16 * (2.0 * 32 * 32 * 16);
      *tflops = flop / (ms * 1e-3) / 1e12;
      rc = DINR_OK;
    }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (sink) hipFree(sink);
  return rc;
}
