// gsb_types.h -- tile geometry, product forms and the step-kernel argument block shared
// by the host code and the gfx950 step kernels of libgsb.  Not installed.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gsb {

// Tile geometry of the persistent step kernels: one workgroup of 4 waves per tile, each
// wave a 64-spin x 32-replica tile (see Kind for the workgroup shapes).
constexpr int kWaveRows = 64;
constexpr int kWaveCols = 32;
constexpr int kRepPad = 128;   // replica counts are padded to a multiple of this
constexpr int kKS = 128;       // K (spins j) per k-step
constexpr int kThreads = 256;
constexpr int kKStepsUnroll = 4;  // k-steps per software-pipeline round
constexpr int kRowPad = kKS * kKStepsUnroll;  // np is a multiple of this (512)
// batched instances pad to two k-steps (256 spins): the generic tile's rounds are two
// k-steps at two workgroups per CU, and a remainder of two k-steps runs unpipelined at one
constexpr int kBatchRowPad = 2 * kKS;

// FIX16: 16-bit fixed point, q = rint(x 2^14) split into int8 hi/lo planes
// (q = 256 hi + lo), J in int8, two int8 MFMA passes with exact int32 accumulation.
enum Form { kFormFP32 = 0, kFormBF16X2 = 1, kFormFP8 = 2, kFormFIX16 = 3 };

// Step-kernel variants.
//   kKindRegJ : FP8 product, np <= 2048: J rows in registers (FP4), 256 spins x 32 replicas
//               per workgroup, two half-step-offset column sub-groups.
//   kKindGeneric : J fragments from L2 (any form; FP4 J for the FP8 product), 64 spins x
//               128 replicas per workgroup (the batched kernel also runs 128 x 64 and
//               256 x 32 tiles).
//   kKindWaveSpec : FP8 product, np <= 2048, the kKindRegJ tile with two waves per SIMD:
//               one computes the product (J in registers and LDS), the other the update.
enum Kind { kKindGeneric = 0, kKindRegJ = 2, kKindWaveSpec = 3 };

__host__ __device__ constexpr int tile_rows_kind(int kind) {
  return (kind == kKindRegJ || kind == kKindWaveSpec) ? 256 : 64;
}
__host__ __device__ constexpr int tile_cols_kind(int kind) { return 8192 / tile_rows_kind(kind); }
__host__ __device__ constexpr int threads_kind(int kind) { return kind == kKindWaveSpec ? 2 * kThreads : kThreads; }

// Bytes of one operand plane per (16-replica block, k-step) and of one J block per
// (16-row tile, k-step), in the fragment-major layouts.  (The register-resident FP8 path
// stores J as FP4 (E2M1), 1 KiB per block, which holds 0 and +-1 exactly.)
__host__ __device__ constexpr size_t operand_block_bytes(int form) {
  return (form == kFormFP8 || form == kFormFIX16) ? 2048 : (form == kFormBF16X2 ? 4096 : 8192);
}

__host__ __device__ constexpr int operand_planes(int form) {
  return (form == kFormBF16X2 || form == kFormFIX16) ? 2 : 1;
}

struct StepArgs {
  int n;          // spins carried by the dynamics (including an ancilla)
  int np;         // padded spins (multiple of kRowPad)
  int rp;         // replicas of this launch (multiple of kBN)
  int groups;     // rp / tile_cols
  int nb;         // np / tile_rows  (workgroups per replica group)
  int discrete;   // 1: operand is sgn(x) (dSB, GdSB)
  int m_begin, m_end;
  float A, dt, cdt;
  const float* acol;      // per-replica control strength (tangent mode), or nullptr
  const float* rtab;      // r_m, m = 0..M-1
  const void* jf;         // J in the fragment-major layout of `form`
  uint8_t* q;             // operand ping-pong buffers of this launch
  size_t q_buf_bytes;     // bytes of one ping-pong buffer (all planes)
  float* x; float* y; float* p;  // state of this launch's replicas, [rp][np]
  unsigned* sync;         // zeroed before the launch; see sync_words()
  unsigned* status;       // set nonzero on a device-side timeout
  float* tape = nullptr;  // binary32 form: per-step input states (reverse pass), or nullptr
  size_t tape_arr = 0;    // floats between the x, y, p planes of one tape entry
  // Workgroups per row block in the grid: 0 (= groups), or groups rounded up to a
  // multiple of 8 so that workgroup b, which runs on XCD b mod 8, belongs to a group whose
  // workgroups all share that XCD; workgroups of the padding groups exit at once.
  int gpad = 0;
};

__host__ __device__ inline int grid_groups(const StepArgs& a) { return a.gpad > 0 ? a.gpad : a.groups; }

inline size_t sync_words(int groups) { return (size_t)(4 * groups + 1) * 64; }

}  // namespace gsb
