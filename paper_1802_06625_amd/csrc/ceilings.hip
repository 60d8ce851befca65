// Ceiling probes: what one device sustains, measured rather than read from a
// datasheet, so that a kernel's roofline fraction can be stated against both.
//
// * copy: float4 grid-stride copy between two buffers of `bytes` each
//   (HBM read + write bandwidth), `waves` workgroups per CU;
// * fma32: independent chains of unpacked fp32 FMAs (v_fma_f32; the build
//   disables packed fp32) in every lane, `waves` waves per SIMD;
// * fmac32: 16 accumulators per lane, acc += a * b with all operands in
//   registers (the accumulate form the filter-bank kernels use);
// * fma3v / fmamix: 8 chains v = v * a + b with every operand in a register
//   (three-operand v_fma_f32), or 4 of those beside 4 accumulators;
// * mfma32: independent chains of the 16x16x4 fp32 matrix-core instruction
//   the block-Toeplitz kernels use, `waves` waves per SIMD.
//
// Each launch also measures the shader clock it ran at: the first lane of
// every workgroup reads the core cycle counter (s_memtime) and the constant
// rate real-time counter (s_memrealtime) at its start and end, and the clock
// is the ratio of the summed deltas, scaled by the real-time counter's rate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "prune_internal.h"

namespace prune {

namespace {

constexpr int kProbeWG = 256;

struct ClockAcc {
  unsigned long long cycles, ticks;
};

__device__ __forceinline__ void clock_mark(unsigned long long *c0, unsigned long long *w0) {
  *c0 = __builtin_amdgcn_s_memtime();
  *w0 = __builtin_amdgcn_s_memrealtime();
}

__device__ __forceinline__ void clock_add(ClockAcc *acc, unsigned long long c0,
                                          unsigned long long w0) {
  const unsigned long long c1 = __builtin_amdgcn_s_memtime();
  const unsigned long long w1 = __builtin_amdgcn_s_memrealtime();
  atomicAdd(&acc->cycles, c1 - c0);
  atomicAdd(&acc->ticks, w1 - w0);
}

// Grid-stride float4 copy with four loads in flight per lane before their
// stores, then a plain tail.
__global__ __launch_bounds__(kProbeWG) void k_probe_copy(const float4 *__restrict__ a,
                                                         float4 *__restrict__ b, size_t n,
                                                         ClockAcc *acc) {
  unsigned long long c0 = 0, w0 = 0;
  if (threadIdx.x == 0) clock_mark(&c0, &w0);
  const size_t stride = (size_t)gridDim.x * kProbeWG;
  size_t i = (size_t)blockIdx.x * kProbeWG + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const float4 v0 = a[i], v1 = a[i + stride], v2 = a[i + 2 * stride], v3 = a[i + 3 * stride];
    b[i] = v0;
    b[i + stride] = v1;
    b[i + 2 * stride] = v2;
    b[i + 3 * stride] = v3;
  }
  for (; i < n; i += stride) b[i] = a[i];
  if (threadIdx.x == 0) clock_add(acc, c0, w0);
}

// kCh independent FMA chains per lane; the multiplier and addend come from
// the arguments so nothing folds.  Every chain feeds the store at the end.
template <int kCh>
__global__ __launch_bounds__(kProbeWG) void k_probe_fma(float *__restrict__ out, uint32_t iters,
                                                        float m, float c, ClockAcc *acc) {
  float v[kCh];
#pragma unroll
  for (int k = 0; k < kCh; ++k) v[k] = (float)(threadIdx.x + k) * 1e-3f;
  unsigned long long c0 = 0, w0 = 0;
  if (threadIdx.x == 0) clock_mark(&c0, &w0);
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int k = 0; k < kCh; ++k) v[k] = fmaf(v[k], m, c);
    }
  }
  if (threadIdx.x == 0) clock_add(acc, c0, w0);
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kCh; ++k) s += v[k];
  out[(size_t)blockIdx.x * kProbeWG + threadIdx.x] = s;
}

// The accumulate form of the filter-bank kernels: 16 accumulators per lane,
// each taking acc += a_k * b with a_k and b in registers (the two-operand
// v_fmac_f32 encoding), 64 FMAs per trip.
__global__ __launch_bounds__(kProbeWG) void k_probe_fmac(float *__restrict__ out, uint32_t iters,
                                                         float m, float c, ClockAcc *acc) {
  float a[16], v[16];
  const float b = m + (float)threadIdx.x * 1e-9f;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    a[k] = c * (float)(k + 1);
    v[k] = (float)(threadIdx.x + k) * 1e-3f;
  }
  unsigned long long c0 = 0, w0 = 0;
  if (threadIdx.x == 0) clock_mark(&c0, &w0);
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = fmaf(a[k], b, v[k]);
    }
  }
  if (threadIdx.x == 0) clock_add(acc, c0, w0);
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += v[k];
  out[(size_t)blockIdx.x * kProbeWG + threadIdx.x] = s;
}

// Instruction-form mix: kV3 chains v = v * a + b (the multiplicand is the
// destination, so the three-operand v_fma_f32 encoding, every operand in a
// register) beside kV2 accumulators u += c * d (two-operand v_fmac_f32), per
// lane, 8 trips of each per loop trip.
template <int kV3, int kV2>
__global__ __launch_bounds__(kProbeWG) void k_probe_mix(float *__restrict__ out, uint32_t iters,
                                                        float m, float c, ClockAcc *acc) {
  float v[kV3 ? kV3 : 1], a[kV3 ? kV3 : 1], b[kV3 ? kV3 : 1];
  float u[kV2 ? kV2 : 1], e[kV2 ? kV2 : 1];
  const float f = m + (float)threadIdx.x * 1e-9f;
#pragma unroll
  for (int k = 0; k < kV3; ++k) {
    v[k] = (float)(threadIdx.x + k) * 1e-3f;
    a[k] = 0.999999f - (float)k * 1e-8f + (float)threadIdx.x * 1e-10f;
    b[k] = c * (float)(k + 1);
  }
#pragma unroll
  for (int k = 0; k < kV2; ++k) {
    u[k] = (float)(threadIdx.x + k) * 1e-3f;
    e[k] = c * (float)(k + 2);
  }
  unsigned long long c0 = 0, w0 = 0;
  if (threadIdx.x == 0) clock_mark(&c0, &w0);
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
#pragma unroll
      for (int k = 0; k < kV3; ++k) v[k] = fmaf(v[k], a[k], b[k]);
#pragma unroll
      for (int k = 0; k < kV2; ++k) u[k] = fmaf(e[k], f, u[k]);
    }
  }
  if (threadIdx.x == 0) clock_add(acc, c0, w0);
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kV3; ++k) s += v[k];
#pragma unroll
  for (int k = 0; k < kV2; ++k) s += u[k];
  out[(size_t)blockIdx.x * kProbeWG + threadIdx.x] = s;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// kCh independent accumulators per wave, each a 16x16 fp32 tile.
template <int kCh>
__global__ __launch_bounds__(kProbeWG) void k_probe_mfma(float *__restrict__ out, uint32_t iters,
                                                         float av, float bv, ClockAcc *acc) {
  f32x4 d[kCh];
#pragma unroll
  for (int k = 0; k < kCh; ++k) d[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float a = av * (float)(threadIdx.x & 63), b = bv;
  unsigned long long c0 = 0, w0 = 0;
  if (threadIdx.x == 0) clock_mark(&c0, &w0);
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kCh; ++k) d[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d[k], 0, 0, 0);
  }
  if (threadIdx.x == 0) clock_add(acc, c0, w0);
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kCh; ++k) s += d[k][0] + d[k][1] + d[k][2] + d[k][3];
  out[(size_t)blockIdx.x * kProbeWG + threadIdx.x] = s;
}

}  // namespace

}  // namespace prune

using namespace prune;

extern "C" prune_status prune_probe_ceiling(int kind, uint32_t waves, uint64_t size, uint32_t reps,
                                            prune_probe_result *out) {
  if (!out || reps == 0 || (kind != PRUNE_PROBE_COPY && (waves < 1 || waves > 8)) ||
      (kind == PRUNE_PROBE_COPY && waves > 32))
    return PRUNE_E_ARG;
  if (kind != PRUNE_PROBE_COPY && kind != PRUNE_PROBE_FMA32 && kind != PRUNE_PROBE_MFMA32 &&
      kind != PRUNE_PROBE_FMAC32 && kind != PRUNE_PROBE_FMA3V && kind != PRUNE_PROBE_FMAMIX)
    return PRUNE_E_ARG;
  int dev = 0, ncu = 0, wall_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      ncu <= 0 || wall_khz <= 0)
    return PRUNE_E_HIP;
  // copy: `size` bytes per buffer; compute probes: `size` loop trips
  const size_t bytes = kind == PRUNE_PROBE_COPY ? (size_t)size / 16 * 16 : 0;
  if (kind == PRUNE_PROBE_COPY && bytes < 16) return PRUNE_E_ARG;
  if (kind != PRUNE_PROBE_COPY && (size < 1 || size > (1u << 30))) return PRUNE_E_ARG;
  // compute probes: 4 SIMDs per CU, 4 waves per 256-thread workgroup
  // copy: `waves` workgroups per CU (0: 8)
  const uint32_t grid = kind == PRUNE_PROBE_COPY ? (uint32_t)ncu * (waves ? waves : 8)
                                                 : (uint32_t)ncu * waves;
  char *a = nullptr, *b = nullptr;
  ClockAcc *acc = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  prune_status st = PRUNE_OK;
  const size_t abytes = kind == PRUNE_PROBE_COPY ? bytes : (size_t)grid * kProbeWG * sizeof(float);
  if (hipMalloc((void **)&a, abytes) != hipSuccess ||
      (kind == PRUNE_PROBE_COPY && hipMalloc((void **)&b, bytes) != hipSuccess) ||
      hipMalloc((void **)&acc, sizeof(ClockAcc)) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    st = PRUNE_E_HIP;
  }
  double work = 0.0;
  if (st == PRUNE_OK) {
    if (kind == PRUNE_PROBE_COPY) (void)hipMemset(a, 0, bytes);
    auto launch = [&]() {
      if (kind == PRUNE_PROBE_COPY) {
        hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(kProbeWG), 0, nullptr, (const float4 *)a,
                           (float4 *)b, bytes / 16, acc);
      } else if (kind == PRUNE_PROBE_FMA32) {
        hipLaunchKernelGGL(k_probe_fma<8>, dim3(grid), dim3(kProbeWG), 0, nullptr, (float *)a,
                           (uint32_t)size, 0.999999f, 1e-7f, acc);
      } else if (kind == PRUNE_PROBE_FMA3V) {
        hipLaunchKernelGGL((k_probe_mix<8, 0>), dim3(grid), dim3(kProbeWG), 0, nullptr, (float *)a,
                           (uint32_t)size, 1e-7f, 1e-3f, acc);
      } else if (kind == PRUNE_PROBE_FMAMIX) {
        hipLaunchKernelGGL((k_probe_mix<4, 4>), dim3(grid), dim3(kProbeWG), 0, nullptr, (float *)a,
                           (uint32_t)size, 1e-7f, 1e-3f, acc);
      } else if (kind == PRUNE_PROBE_FMAC32) {
        hipLaunchKernelGGL(k_probe_fmac, dim3(grid), dim3(kProbeWG), 0, nullptr, (float *)a,
                           (uint32_t)size, 1e-7f, 1e-3f, acc);
      } else {
        hipLaunchKernelGGL(k_probe_mfma<4>, dim3(grid), dim3(kProbeWG), 0, nullptr, (float *)a,
                           (uint32_t)size, 1e-6f, 1e-6f, acc);
      }
    };
    launch();   // warm-up (clock ramp, page mapping)
    (void)hipMemset(acc, 0, sizeof(ClockAcc));
    (void)hipEventRecord(e0, nullptr);
    for (uint32_t r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess) st = PRUNE_E_HIP;
    float ms = 0.f;
    ClockAcc h{};
    if (st == PRUNE_OK && (hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
                           hipMemcpy(&h, acc, sizeof h, hipMemcpyDeviceToHost) != hipSuccess))
      st = PRUNE_E_HIP;
    if (st == PRUNE_OK) {
      const double threads = (double)grid * kProbeWG;
      if (kind == PRUNE_PROBE_COPY)
        work = 2.0 * (double)bytes * reps;                       // bytes read + written
      else if (kind == PRUNE_PROBE_FMA32 || kind == PRUNE_PROBE_FMAC32 ||
               kind == PRUNE_PROBE_FMA3V || kind == PRUNE_PROBE_FMAMIX)
        work = threads * 64.0 * (double)size * reps;             // fp32 FMAs
      else
        work = (double)grid * 4.0 * 4.0 * (double)size * reps * 2048.0;   // flops
      out->seconds = ms * 1e-3 / reps;
      out->work = work / reps;
      out->rate = work / (ms * 1e-3);
      out->clock_ghz = h.ticks ? (double)h.cycles / (double)h.ticks * (double)wall_khz * 1e-6 : 0.0;
      out->grid = grid;
      out->block = kProbeWG;
      out->n_cu = (uint32_t)ncu;
    }
  }
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  if (acc) (void)hipFree(acc);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return st;
}
