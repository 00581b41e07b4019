// gsb_device.h -- device code shared by the step kernels of libgsb (gfx950): vector
// types, buffer resources, the replica-group barrier and the fragment-major operand
// encodings.  Included by the kernel translation units only.
#pragma once
#include "gsb_types.h"

#pragma clang fp contract(off)

namespace gsb {
namespace {


typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Cache policies of loads.  Operand (Q) loads use device scope, which skips L1: the
// operand buffers are rewritten every step by other CUs, and a workgroup-scope L1
// invalidate does not reliably drop such lines on gfx950 (measured: stale operands when
// the buffers fit in L1), while an agent-scope invalidate costs microseconds.  Plain
// loads (J, read-only for a launch) may hit L1.
constexpr int kPolicySc1 = 16;
constexpr unsigned kSpinLimit = 1u << 22;  // polls before a barrier gives up (seconds)
constexpr int kHwRegXccId = 20 | (0 << 6) | ((4 - 1) << 11);  // hwreg(HW_REG_XCC_ID, 0, 4)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ v8i cat(v4i a, v4i b) {
  return v8i{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
}

__device__ __forceinline__ unsigned ld_dev(const unsigned* p) {
  return __hip_atomic_load(const_cast<unsigned*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier over the `nb` workgroups that share a replica group.  Every wave first waits
// until its own stores are acknowledged (they are then in L2), then one thread counts
// the workgroup in and polls the counter with device-scope loads.  When all members sit
// on one XCD (`local`) they share that XCD's L2, which the operand loads read directly
// (they bypass L1), so no cache maintenance is needed; otherwise the agent-scope
// release/acquire fences write back and invalidate the caches between XCDs.
__device__ __forceinline__ bool group_sync(unsigned* ctr, unsigned target, int local,
                                           unsigned* abort_flag, unsigned* status, int* s_flag) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!local) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    unsigned spins = 0;
    while (ld_dev(ctr) < target) {
      ++spins;
      if ((spins & 63u) == 0 && ld_dev(abort_flag)) { ok = 0; break; }
      if (spins > kSpinLimit) { st_dev(abort_flag, 1u); st_dev(status, 1u); ok = 0; break; }
    }
    if (!local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_flag = ok;
  }
  __syncthreads();
  return *s_flag != 0;
}

// ---------------------------------------------------------------------------------------
// Operand encodings and their fragment-major placement.
//
// Q holds, per (16-replica block rb, 128-spin k-step kc), the operand bytes in exactly the
// order the MFMA B operand is held in a wavefront's lanes, so a fragment is one coalesced
// 1 KiB load per VGPR quad:
//   FP8   : 2048 B = [half 2][lane 64][16 B];  lane = r%16 + 16*((kk/4)%4),
//           half kk/64, byte 4*((kk/16)%4) + kk%4                            (16x16x128;
//           a permutation of the spins within the k-step, see fp8_elem_offset)
//   BF16  : 32x32x16 bf16 MFMA.  Per (32-replica block, k-step): 8 KiB per plane =
//           [sixteenth 8][lane 64][8 bf16]; lane = r%32 + 32*((kk%16)/8),
//           kk = 16*sixteenth + 8*(lane/32) + e; plane 0 holds hi, plane 1 lo.
//   FP32  : 8192 B = [grp 8][lane 64][4 f32];  kk = 16*grp + 4*(lane/16) + t, where
//           element t feeds the t-th of four 16x16x4 MFMAs of that group.
//   FIX16 : 32x32x32 int8 MFMA.  Per (32-replica block, k-step): 4 KiB per plane =
//           [quarter 4][lane 64][16 x int8]; lane = r%32 + 32*((kk%32)/16),
//           kk = 32*quarter + 16*(lane/32) + b; plane 0 holds hi, plane 1 lo of
//           q = rint(x 2^14) = 256 hi + lo, hi in [-64, 64], lo in [-128, 127].  J: the same
//           per (32-row tile, k-step), rows in place of replicas.
// (kk = k mod 128.)  J uses the same layouts with the row i in place of the replica r
// (FP4 J of the FP8 product: see fp4_pair_kk).
// store_operand receives the 16x16 tile origin (ibase, rcol) of the lane's elements, or
// for the 32x32 layouts (BF16, FIX16) the lane's own first element (row ibase,
// ibase % 4 == 0, column rcol).
// ---------------------------------------------------------------------------------------
// Encodings of four operand values (one lane's four rows), shared by the step kernels'
// operand stores and by the standalone encoder.  `discrete` replaces each value by its
// sign, s(x) = +1 for x >= 0 (including -0.0).
__device__ __forceinline__ float operand_value(float x, bool discrete) {
  return discrete ? (x < 0.0f ? -1.0f : 1.0f) : x;
}
// FP8: OCP E4M3 bytes, value v in byte v (round to nearest even, the hardware conversion),
// with `orin` ORed into the word (the step tag of the step kernels).
template <bool DISC>
__device__ __forceinline__ unsigned encode_fp8x4(const float xv[4], unsigned orin = 0u) {
  if constexpr (DISC) {
    // +1.0 in E4M3 (0x38) in every byte, with the sign bit of the E4M3 conversion of
    // x + 0: adding +0 turns -0.0 into +0.0 and leaves every other value as it is, and the
    // conversion keeps the sign (a value that rounds to zero gives a signed zero), so the
    // bit is set exactly where x < 0.  bitop3 0xEA: (a & b) | c.  The first conversion
    // writes the low half of a register that starts as any value at hand (here n0, which
    // it reads first; the second conversion replaces the high half).
    const float n0 = xv[0] + 0.0f;
    const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(n0, xv[1] + 0.0f, __builtin_bit_cast(int, n0), false);
    const int w = __builtin_amdgcn_cvt_pk_fp8_f32(xv[2] + 0.0f, xv[3] + 0.0f, lo, true);
    return __builtin_amdgcn_bitop3_b32((unsigned)w, 0x80808080u, 0x38383838u | orin, 0xEA);
  } else {
    const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(xv[0], xv[1], 0, false);
    return (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(xv[2], xv[3], lo, true) | orin;
  }
}
// BF16X2: hi = bf16(q), lo = bf16(q - hi) (q - hi is exact in binary32); two bf16 per word.
template <bool DISC>
__device__ __forceinline__ void encode_bf16x4(const float xv[4], v2u& wh, v2u& wl) {
  unsigned short hi[4], lo[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float q = operand_value(xv[v], DISC);
    const __bf16 h = (__bf16)q;
    const float hf = (float)h;
    const __bf16 l = (__bf16)(q - hf);
    hi[v] = __builtin_bit_cast(unsigned short, h);
    lo[v] = __builtin_bit_cast(unsigned short, l);
  }
  wh = v2u{(unsigned)hi[0] | ((unsigned)hi[1] << 16), (unsigned)hi[2] | ((unsigned)hi[3] << 16)};
  wl = v2u{(unsigned)lo[0] | ((unsigned)lo[1] << 16), (unsigned)lo[2] | ((unsigned)lo[3] << 16)};
}
// FIX16: q = rint(x 2^14) (exact scaling, round half to even) = 256 hi + lo with
// hi = (q + 128) >> 8 in [-64, 64] and lo in [-128, 127]; int8 value v in byte v.
template <bool DISC>
__device__ __forceinline__ void encode_fix16x4(const float xv[4], unsigned& wh, unsigned& wl) {
  wh = 0;
  wl = 0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int qi = (int)__builtin_rintf(operand_value(xv[v], DISC) * 16384.0f);
    const int hi = (qi + 128) >> 8;
    const int lo = qi - 256 * hi;
    wh |= (unsigned)(hi & 0xFF) << (8 * v);
    wl |= (unsigned)(lo & 0xFF) << (8 * v);
  }
}

// FP8 operand placement.  A fragment (16 replicas x one 128-spin k-step) is two 1 KiB
// halves of 64 lanes x 16 bytes, the B operand of the 16x16x128 MFMA: lane p of a half
// holds replica p mod 16 and lane group g = p / 16, byte j of the lane's 32 (16 h + b for
// half h) is MFMA k index 16 g + b + 64 h.  Which spin feeds which k index is free as long
// as J (below) uses the same map; this one puts spin kk = k mod 128 at
//   half kk / 64, lane group (kk / 4) mod 4, byte 4 ((kk / 16) mod 4) + kk mod 4,
// so that the sixteen spins 64 h + 16 t + 4 L + v (t, v < 4) of one replica -- the four
// row tiles t of lane L of a 16x16 MFMA result, rows 4 L + v -- are one lane's 16
// contiguous bytes, which the lane that computed them can store with wide stores.
__host__ __device__ __forceinline__ size_t fp8_elem_offset(int nks, int r, int k) {
  const int kk = k & 127;
  const int lanep = (r & 15) + 16 * ((kk >> 2) & 3);
  return ((size_t)((r >> 4) * nks + (k >> 7)) * 2 + (kk >> 6)) * 1024 + lanep * 16 + (((kk >> 4) & 3) << 2) +
         (kk & 3);
}
// Offset of the FP8 word of a lane's four rows (16x16 tile origin ibase, rcol; rows
// ibase + 4 (lane / 16) + v, replica rcol + lane mod 16): bytes v of one word.
__host__ __device__ __forceinline__ size_t fp8_operand_offset(int nks, int ibase, int rcol, int lane) {
  return fp8_elem_offset(nks, rcol + (lane & 15), ibase + 4 * (lane >> 4));
}

// fp8_tag (FP8 only) is ORed into the stored word: a step tag in bit 6 of its first byte,
// which the E4M3 code of any |x| <= 1 leaves clear (exponent field at most 7).
template <int FORM, bool DISC>
__device__ __forceinline__ void store_operand(uint8_t* qbuf, size_t plane_bytes, int nks,
                                              int ibase, int rcol, int lane, const float xv[4],
                                              unsigned fp8_tag = 0u) {
  const int rb = rcol >> 4;
  const int kc = ibase >> 7;
  const int kk0 = (ibase & 127) + 4 * (lane >> 4);  // first of this lane's 4 rows
  if constexpr (FORM == kFormFP8) {
    const unsigned w = encode_fp8x4<DISC>(xv, fp8_tag);
    (void)kk0;
    (void)rb;
    (void)kc;
    *reinterpret_cast<unsigned*>(qbuf + fp8_operand_offset(nks, ibase, rcol, lane)) = w;
  } else if constexpr (FORM == kFormBF16X2) {
    v2u wh, wl;
    encode_bf16x4<DISC>(xv, wh, wl);
    (void)kk0;
    (void)rb;
    const int lanep = (rcol & 31) + 32 * ((ibase & 15) >> 3);
    const size_t off =
        ((size_t)((rcol >> 5) * nks + kc) * 8 + ((ibase & 127) >> 4)) * 1024 + lanep * 16 + (ibase & 7) * 2;
    *reinterpret_cast<v2u*>(qbuf + off) = wh;
    *reinterpret_cast<v2u*>(qbuf + plane_bytes + off) = wl;
  } else if constexpr (FORM == kFormFIX16) {
    unsigned wh, wl;
    encode_fix16x4<DISC>(xv, wh, wl);
    (void)kk0;
    (void)rb;
    const int lanep = (rcol & 31) + 32 * ((ibase & 31) >> 4);
    const size_t off =
        ((size_t)((rcol >> 5) * nks + kc) * 4 + ((ibase & 127) >> 5)) * 1024 + lanep * 16 + (ibase & 15);
    *reinterpret_cast<unsigned*>(qbuf + off) = wh;
    *reinterpret_cast<unsigned*>(qbuf + plane_bytes + off) = wl;
  } else {
    v4f q;
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = operand_value(xv[v], DISC);
    const int grp = kk0 >> 4;
    const int lanep = (lane & 15) + 16 * ((kk0 & 15) >> 2);
    const size_t off = ((size_t)(rb * nks + kc) * 8 + grp) * 1024 + lanep * 16;
    *reinterpret_cast<v4f*>(qbuf + off) = q;
  }
}

// J (zero padded, entries in {0, +-1}) -> FP4 (E2M1) fragment-major layout of the FP8
// product: [row tile][k-step][lane 64][16 bytes], two values per byte, low nibble first.
// In the mixed FP4 x FP8 MFMA (16x16x128), FP4 nibble p (0..127 over the four lane groups
// of a row tile, 32 per group) multiplies MFMA k index p of the operand, which is FP8 byte
// j = p mod 16 of lane group (p mod 64) / 16 in half p / 64; the spin there is the one the
// operand placement (fp8_elem_offset) puts at that byte.
__host__ __device__ __forceinline__ int fp4_pair_kk(int p) {
  return 64 * (p >> 6) + 16 * ((p >> 2) & 3) + 4 * ((p >> 4) & 3) + (p & 3);
}
__device__ __forceinline__ unsigned fp4_code(float v) {  // exact for 0 and +-1
  return (v < 0.0f ? 0x8u : 0u) | (__builtin_fabsf(v) == 1.0f ? 0x2u : 0u);
}

}  // namespace
}  // namespace gsb
