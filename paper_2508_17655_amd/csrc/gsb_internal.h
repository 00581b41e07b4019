// Internal interface between the C ABI (gsb_api.cpp) and the gfx950 kernels
// (gsb_kernels.hip).  Not installed; not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gsb {

// Tile geometry of the persistent step kernel: one workgroup of 4 waves per tile, each
// wave a 64-spin x 32-replica tile.  With J resident in LDS (FP8 product, J stored as
// FP4) a workgroup is 128 spins x 64 replicas; otherwise 64 spins x 128 replicas.
constexpr int kWaveRows = 64;
constexpr int kWaveCols = 32;
constexpr int kRepPad = 128;   // replica counts are padded to a multiple of this
constexpr int kKS = 128;       // K (spins j) per k-step
constexpr int kThreads = 256;
constexpr int kKStepsUnroll = 4;  // k-steps per software-pipeline round
constexpr int kRowPad = kKS * kKStepsUnroll;  // np is a multiple of this (512)

// FIX16: 16-bit fixed point, q = rint(x 2^14) split into int8 hi/lo planes
// (q = 256 hi + lo), J in int8, two int8 MFMA passes with exact int32 accumulation.
enum Form { kFormFP32 = 0, kFormBF16X2 = 1, kFormFP8 = 2, kFormFIX16 = 3 };

// Step-kernel variants.
//   kKindRegJ : FP8 product, np <= 2048: J rows in registers (FP4), 256 spins x 32 replicas
//               per workgroup, two half-step-offset column sub-groups.
//   kKindGeneric : J fragments from L2 (any form), 64 spins x 128 replicas per workgroup.
enum Kind { kKindGeneric = 0, kKindRegJ = 2 };

__host__ __device__ constexpr int tile_rows_kind(int kind) { return kind == kKindRegJ ? 256 : 64; }
__host__ __device__ constexpr int tile_cols_kind(int kind) { return 8192 / tile_rows_kind(kind); }

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
};

inline size_t sync_words(int groups) { return (size_t)(4 * groups + 1) * 64; }

// ---- launchers (all asynchronous on `stream`) ----
hipError_t launch_fill_u32(unsigned* p, size_t count, unsigned v, hipStream_t stream);
hipError_t launch_encode_j(int form, bool fp4, const float* j32, int np, void* jf, hipStream_t stream);
hipError_t launch_init_state(int n, int np, int rp, uint64_t seed, int mode, float* x, float* y,
                             float* p, hipStream_t stream);
// Persistent step kernel of variant `kind` (see Kind).  With `tangent` (binary32 form,
// generic kind, continuous variants) the launch's columns are the tangent-mode layout:
// blocks of 32 = 16 replicas followed by their 16 tangents.
hipError_t launch_steps(int form, int kind, const StepArgs& a, hipStream_t stream, bool tangent = false);
int max_coresident_workgroups(int form, int kind, int np, bool tangent = false);
// Reverse pass of the binary32 dynamics over a recorded tape (see k_adjoint); a.x, a.y,
// a.p carry the cotangents in and out.  Occupancy limit of that kernel.
hipError_t launch_adjoint(const StepArgs& a, hipStream_t stream);
int max_coresident_adjoint();
// Tangent mode: starting state (as launch_init_state for each replica) and tangent
// dx = +-1 from `tseed` (dy = dp = 0) for rp replicas in 2 rp columns.
hipError_t launch_init_tangent(int n, int np, int rp, uint64_t seed, int mode, uint64_t tseed, float* x, float* y,
                               float* p, hipStream_t stream);
// Scale every replica's tangent to unit norm; with `accumulate`, lg[r] += ln(norm).
hipError_t launch_tangent_renorm(int n, int np, int rp, float* x, float* y, float* p, double* lg, bool accumulate,
                                 hipStream_t stream);
// Tangent-mode state of the first R replicas -> [6][R][n] (x, y, p, dx, dy, dp).
hipError_t launch_tangent_extract(int n, int np, int R, const float* x, const float* y, const float* p, float* out,
                                  hipStream_t stream);
// eq. (8) for pairs (2k, 2k + 1), k < pairs, over spins < n.
hipError_t launch_delta(int n, int np, int pairs, const float* x, double* out, hipStream_t stream);
int choose_kind(int form, int np);
hipError_t launch_energy(const float* j32, int n, int np, int rp, int r_count, const float* x,
                         double* partial, double* energies, hipStream_t stream);
size_t energy_partial_doubles(int np, int rp);
// Exact energies for J in {0, +-1} from the FP4 J of the register-resident FP8 path
// (np a multiple of 256, rp of 32): E = -1/2 s^T J s on MFMA with integer accumulation.
// `scratch` holds energy_fp4_scratch_bytes(np, rp) bytes.
hipError_t launch_energy_fp4(const void* jf4, int np, int rp, int r_count, const float* x, void* scratch,
                             double* energies, hipStream_t stream);
size_t energy_fp4_scratch_bytes(int np, int rp);
hipError_t launch_best(const double* energies, int r_count, int* best_idx, double* best_e,
                       hipStream_t stream);
hipError_t launch_spins(const float* x, int n_out, int np, int r_first, int r_count, int anc,
                        const int* r_index, int8_t* spins, hipStream_t stream);

}  // namespace gsb
