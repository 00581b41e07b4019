// gsb_probe.hip -- this device's ceilings, measured (libgsb_probe.so, apart from the
// product library): the issue rate of each MFMA form the step kernels use, how matrix-core
// and vector-ALU waves share a SIMD, read bandwidth at L2-, MALL- and HBM-sized
// footprints, write bandwidth, and the shader clock during a busy kernel.  The roofline fractions of the
// step kernels are stated against the published peaks; these figures say how close to
// them the chip itself gets.
#include "gsb_internal.h"
#include "gsb_device.h"

#include <hip/hip_runtime.h>

namespace gsb {
namespace {

typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kChains = 8;  // independent accumulators per wave: enough to hide MFMA latency

// KIND 0: FP8 x FP8 16x16x128, 1: FP4 x FP8 16x16x128, 2: int8 16x16x64, 3: bf16 16x16x32,
// 4: binary32 16x16x4, 5: FP8 x FP8 32x32x64, 6: int8 32x32x32, 7: bf16 32x32x16.  Every wave runs `iters` rounds of kChains MFMAs on operands that
// depend on the lane (so nothing folds) and keeps the result alive through `sink`.
template <int KIND>
__global__ void __launch_bounds__(256) k_mfma_rate(int iters, float* sink) {
  const int lane = threadIdx.x & 63;
  const int v = lane * 0x01010101;
  // the 32x32 shapes have 16-register accumulators: half as many chains keep the
  // registers (and 4 waves per SIMD) the same
  constexpr int CH = KIND >= 5 ? kChains / 2 : kChains;
  v4f acc[CH];
  v4i iacc[CH];
  v16f acc16[CH];
  v16i iacc16[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
    iacc[j] = v4i{0, 0, 0, 0};
    acc16[j] = v16f{};
    iacc16[j] = v16i{};
  }
  const v8i a8 = v8i{v, v + 1, v + 2, v + 3, v + 4, v + 5, v + 6, v + 7} & 0x37373737;  // small E4M3 values
  const v4i a4 = v4i{v, v + 1, v + 2, v + 3} & 0x77777777;
  const float f = (float)lane * 0.001f;
  const v8bf bf = v8bf{(__bf16)f, (__bf16)f, (__bf16)f, (__bf16)f, (__bf16)f, (__bf16)f, (__bf16)f, (__bf16)f};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if constexpr (KIND == 0)
        acc[j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, a8, acc[j], 0, 0, 0, 127, 0, 127);
      else if constexpr (KIND == 1)
        acc[j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(v8i{a4[0], a4[1], a4[2], a4[3], a4[0], a4[1], a4[2], a4[3]},
                                                                  a8, acc[j], 4, 0, 0, 127, 0, 127);
      else if constexpr (KIND == 2)
        iacc[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a4, a4, iacc[j], 0, 0, 0);
      else if constexpr (KIND == 3)
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf, bf, acc[j], 0, 0, 0);
      else if constexpr (KIND == 4)
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(f, f, acc[j], 0, 0, 0);
      else if constexpr (KIND == 5)
        acc16[j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, a8, acc16[j], 0, 0, 0, 127, 0, 127);
      else if constexpr (KIND == 6)
        iacc16[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a4, a4, iacc16[j], 0, 0, 0);
      else
        acc16[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bf, bf, acc16[j], 0, 0, 0);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < CH; ++j)
    s += acc[j][0] + acc[j][3] + (float)iacc[j][0] + acc16[j][0] + acc16[j][15] + (float)iacc16[j][0];
  if (s == 1.2345e-30f) sink[blockIdx.x] = s;  // never true in practice; keeps the chains
}

// operations per MFMA x chains per wave
constexpr double kMfmaOps[8] = {2.0 * 16 * 16 * 128 * kChains, 2.0 * 16 * 16 * 128 * kChains,
                                2.0 * 16 * 16 * 64 * kChains,  2.0 * 16 * 16 * 32 * kChains,
                                2.0 * 16 * 16 * 4 * kChains,   2.0 * 32 * 32 * 64 * (kChains / 2),
                                2.0 * 32 * 32 * 32 * (kChains / 2), 2.0 * 32 * 32 * 16 * (kChains / 2)};

__global__ void __launch_bounds__(256) k_stream_read(const v4f* p, size_t n4, int passes, float* sink) {
  v4f s = v4f{0.f, 0.f, 0.f, 0.f};
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (int pass = 0; pass < passes; ++pass)
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) s += p[i];
  if (s[0] + s[1] + s[2] + s[3] == 1.2345e-30f) sink[blockIdx.x] = s[0];
}

// L2 read rate: device-scope 16-byte loads (they skip L1, as the step kernels' operand
// loads do), four independent ones in flight per thread, at offsets that move by a
// different amount on every round so that no CU reads its own lines again.  `mask` + 1
// is the buffer's size, a power of two; every offset is a multiple of 16 within it.
__global__ void __launch_bounds__(256) k_l2_read(const float* base, unsigned mask, int rounds, float* sink) {
  const __amdgpu_buffer_rsrc_t r = make_rsrc(base, (size_t)mask + 1);
  const unsigned t = (blockIdx.x * blockDim.x + threadIdx.x) * 16u;
  v4f s0 = v4f{0.f, 0.f, 0.f, 0.f}, s1 = s0, s2 = s0, s3 = s0;
  for (int k = 0; k < 4 * rounds; k += 4) {
    const unsigned o0 = (t + (unsigned)(k + 0) * 0x9E3779B0u) & mask;
    const unsigned o1 = (t + (unsigned)(k + 1) * 0x9E3779B0u) & mask;
    const unsigned o2 = (t + (unsigned)(k + 2) * 0x9E3779B0u) & mask;
    const unsigned o3 = (t + (unsigned)(k + 3) * 0x9E3779B0u) & mask;
    s0 += __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, o0, 0, kPolicySc1));
    s1 += __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, o1, 0, kPolicySc1));
    s2 += __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, o2, 0, kPolicySc1));
    s3 += __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, o3, 0, kPolicySc1));
  }
  const v4f s = s0 + s1 + s2 + s3;
  if (s[0] + s[1] + s[2] + s[3] == 1.2345e-30f) sink[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(256) k_stream_write(v4f* p, size_t n4, int passes) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (int pass = 0; pass < passes; ++pass)
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
      p[i] = v4f{(float)pass, 0.f, 0.f, 0.f};
}

// Shader-clock ticks (s_memtime) against the constant-rate wall clock over a busy loop.
__global__ void k_clock(int iters, unsigned long long* out, float* sink) {
  const unsigned long long c0 = __builtin_amdgcn_s_memtime(), w0 = wall_clock64();
  float x = (float)threadIdx.x;
  for (int i = 0; i < iters; ++i) x = x * 1.0000001f + 1e-7f;
  const unsigned long long c1 = __builtin_amdgcn_s_memtime(), w1 = wall_clock64();
  if (threadIdx.x == 0 && blockIdx.x == 0) { out[0] = c1 - c0; out[1] = w1 - w0; }
  if (x == 1.2345e-30f) sink[0] = x;
}

// Co-issue of the matrix cores and the vector ALU, in the headline kernel's arrangement:
// 8 waves per workgroup, one workgroup per CU, so each SIMD runs one wave of each kind.
// Waves 0-3 issue rounds of four independent FP4 x FP8 16x16x128 MFMAs (the product
// wave's k-step); waves 4-7 issue rounds of 20 binary32 multiplies and adds over ten
// independent chains (about the update's share of vector instructions per k-step).
// mode 1: MFMA waves only; 2: VALU waves only; 3: both.
__global__ void __launch_bounds__(512) k_coissue(int mode, int iters, float* sink) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float s = 0.0f;
  if (wave < 4) {
    if (!(mode & 1)) return;
    const int v = lane * 0x01010101;
    const v8i b = v8i{v, v + 1, v + 2, v + 3, v + 4, v + 5, v + 6, v + 7} & 0x37373737;
    const v4i a = v4i{v, v + 1, v + 2, v + 3} & 0x77777777;
    v4f acc[4] = {};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(v8i{a[0], a[1], a[2], a[3], a[0], a[1], a[2], a[3]},
                                                                  b, acc[j], 4, 0, 0, 127, 0, 127);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) s += acc[j][0];
  } else {
    if (!(mode & 2)) return;
    float x[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) x[j] = (float)(lane + j) * 1e-3f;
    const float m = 0.9999f, c = 1e-4f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int j = 0; j < 10; ++j) x[j] = x[j] * m + c;  // contraction off: a multiply and an add
    }
#pragma unroll
    for (int j = 0; j < 10; ++j) s += x[j];
  }
  if (s == 1.2345e-30f) sink[blockIdx.x] = s;
}

hipError_t time_coissue(int cus, int iters, float* sink, hipEvent_t e0, hipEvent_t e1, double* ms_out) {
  for (int mode = 1; mode <= 3; ++mode) {
    hipLaunchKernelGGL(k_coissue, dim3(cus), dim3(512), 0, 0, mode, 1, sink);  // warm-up
    hipError_t e = hipEventRecord(e0, 0);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_coissue, dim3(cus), dim3(512), 0, 0, mode, iters, sink);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipEventRecord(e1, 0)) != hipSuccess) return e;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
    float ms = 0;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
    ms_out[mode - 1] = ms;
  }
  return hipSuccess;
}

template <int KIND>
hipError_t time_mfma(int blocks, int iters, float* sink, hipEvent_t e0, hipEvent_t e1, double* rate) {
  hipLaunchKernelGGL(k_mfma_rate<KIND>, dim3(blocks), dim3(256), 0, 0, 1, sink);  // warm-up
  hipError_t e = hipEventRecord(e0, 0);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mfma_rate<KIND>, dim3(blocks), dim3(256), 0, 0, iters, sink);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipEventRecord(e1, 0)) != hipSuccess) return e;
  if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
  float ms = 0;
  if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
  const double ops = kMfmaOps[KIND] * (double)iters * blocks * 4.0;  // 4 waves per block
  *rate = ops / (ms * 1e-3);
  return hipSuccess;
}

}  // namespace

hipError_t measure_ceilings(double* out, int count) {
  int dev = 0, cus = 0, rate_khz = 0;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess) return e;
  const size_t big = (size_t)2 << 30;  // 2 GiB: well beyond the 256 MiB MALL
  void* buf = nullptr;
  // sink: one float per workgroup of any probe (at most 8 per CU), then the clock ticks
  const size_t sink_floats = (size_t)cus * 8 + 64;
  if ((e = hipMalloc(&buf, big + sink_floats * 4 + 64)) != hipSuccess) return e;
  float* sink = reinterpret_cast<float*>(static_cast<char*>(buf) + big);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double v[16] = {0};
  auto run = [&]() -> hipError_t {
    hipError_t r;
    if ((r = hipEventCreate(&e0)) != hipSuccess) return r;
    if ((r = hipEventCreate(&e1)) != hipSuccess) return r;
    const int blocks = cus * 4;  // four 4-wave workgroups per CU: 4 waves per SIMD
    if ((r = time_mfma<0>(blocks, 2000, sink, e0, e1, &v[0])) != hipSuccess) return r;
    if ((r = time_mfma<1>(blocks, 2000, sink, e0, e1, &v[1])) != hipSuccess) return r;
    if ((r = time_mfma<2>(blocks, 2000, sink, e0, e1, &v[2])) != hipSuccess) return r;
    if ((r = time_mfma<3>(blocks, 2000, sink, e0, e1, &v[3])) != hipSuccess) return r;
    if ((r = time_mfma<4>(blocks, 2000, sink, e0, e1, &v[4])) != hipSuccess) return r;
    if ((r = time_mfma<5>(blocks, 1000, sink, e0, e1, &v[10])) != hipSuccess) return r;
    if ((r = time_mfma<6>(blocks, 1000, sink, e0, e1, &v[11])) != hipSuccess) return r;
    if ((r = time_mfma<7>(blocks, 1000, sink, e0, e1, &v[12])) != hipSuccess) return r;
    if ((r = time_coissue(cus, 20000, sink, e0, e1, &v[13])) != hipSuccess) return r;
    // reads: 2 MiB (each XCD's L2 holds a copy; scattered device-scope loads, above),
    // then streaming over 64 MiB (MALL) and 2 GiB (HBM)
    const v4f* p = static_cast<const v4f*>(buf);
    if ((r = hipMemset(buf, 0, big)) != hipSuccess) return r;
    {
      const unsigned grid = (unsigned)(cus * 8);  // sink holds more than cus * 8 floats
      const unsigned mask = (2u << 20) - 1u;
      const int rounds = 256;
      hipLaunchKernelGGL(k_l2_read, dim3(grid), dim3(256), 0, 0, static_cast<const float*>(buf), mask, 4, sink);
      if ((r = hipEventRecord(e0, 0)) != hipSuccess) return r;
      hipLaunchKernelGGL(k_l2_read, dim3(grid), dim3(256), 0, 0, static_cast<const float*>(buf), mask, rounds, sink);
      if ((r = hipGetLastError()) != hipSuccess) return r;
      if ((r = hipEventRecord(e1, 0)) != hipSuccess) return r;
      if ((r = hipEventSynchronize(e1)) != hipSuccess) return r;
      float ms = 0;
      if ((r = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return r;
      v[5] = (double)grid * 256 * 16 * 4 * rounds / (ms * 1e-3);
    }
    const size_t sizes[3] = {(size_t)2 << 20, (size_t)64 << 20, big};
    const int passes[3] = {400, 20, 2};
    for (int k = 1; k < 3; ++k) {
      const size_t n4 = sizes[k] / 16;
      const unsigned grid = (unsigned)(cus * 8);
      hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, 0, p, n4, 1, sink);
      if ((r = hipEventRecord(e0, 0)) != hipSuccess) return r;
      hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, 0, p, n4, passes[k], sink);
      if ((r = hipGetLastError()) != hipSuccess) return r;
      if ((r = hipEventRecord(e1, 0)) != hipSuccess) return r;
      if ((r = hipEventSynchronize(e1)) != hipSuccess) return r;
      float ms = 0;
      if ((r = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return r;
      v[5 + k] = (double)sizes[k] * passes[k] / (ms * 1e-3);
    }
    {
      const size_t n4 = big / 16;
      const unsigned grid = (unsigned)(cus * 8);
      hipLaunchKernelGGL(k_stream_write, dim3(grid), dim3(256), 0, 0, static_cast<v4f*>(buf), n4, 1);
      if ((r = hipEventRecord(e0, 0)) != hipSuccess) return r;
      hipLaunchKernelGGL(k_stream_write, dim3(grid), dim3(256), 0, 0, static_cast<v4f*>(buf), n4, 2);
      if ((r = hipGetLastError()) != hipSuccess) return r;
      if ((r = hipEventRecord(e1, 0)) != hipSuccess) return r;
      if ((r = hipEventSynchronize(e1)) != hipSuccess) return r;
      float ms = 0;
      if ((r = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return r;
      v[8] = (double)big * 2 / (ms * 1e-3);
    }
    {
      unsigned long long* ticks = reinterpret_cast<unsigned long long*>(sink + (size_t)cus * 8 + 16);
      hipLaunchKernelGGL(k_clock, dim3(cus * 4), dim3(256), 0, 0, 200000, ticks, sink);
      if ((r = hipGetLastError()) != hipSuccess) return r;
      unsigned long long t[2] = {0, 0};
      if ((r = hipMemcpy(t, ticks, sizeof(t), hipMemcpyDeviceToHost)) != hipSuccess) return r;
      const double wall_hz = rate_khz > 0 ? rate_khz * 1e3 : 1e8;
      v[9] = t[1] ? (double)t[0] / ((double)t[1] / wall_hz) : 0.0;
    }
    return hipSuccess;
  };
  e = run();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  const hipError_t ef = hipFree(buf);
  if (e == hipSuccess) e = ef;
  if (e == hipSuccess)
    for (int k = 0; k < count && k < 16; ++k) out[k] = v[k];
  return e;
}

}  // namespace gsb

extern "C" int32_t gsb_probe_ceilings(double* out, int32_t count) {
  if (!out || count < 0) return (int32_t)hipErrorInvalidValue;
  return (int32_t)gsb::measure_ceilings(out, count);
}
