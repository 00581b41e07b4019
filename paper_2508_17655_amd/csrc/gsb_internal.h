// Internal interface between the C ABI (gsb_api.cpp, gsb_batch.cpp) and the gfx950
// kernels (gsb_kernels.hip, gsb_steps_rj.hip).  Not installed; not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gsb_types.h"

namespace gsb {

// ---- batched instances (one persistent launch over many instances of different n) ----
// Slot of a queue: workgroup mb of replica group g of instance `inst`, in tiles of `bm`
// spin rows (64, 128 or 256) x 8192 / bm replicas.  The nb = np / bm slots of one
// (instance, group) pair form a gang: they run together and synchronise every step.
struct BatchSlot { int inst, g, mb, bm; };
// Per-instance buffers beside the instance's StepArgs (FP8 product; a.jf is FP4 J).
struct BatchInst {
  uint64_t seed;    // initial state: the single-instance generator with this seed
  uint8_t* s8;      // sign operand of the energy product, rp x np bytes
  int* eacc;        // integer energy sums, rp ints (zeroed before the energy kernels)
  double* E;        // energies, rp doubles
  int* best_idx;    // lowest-energy replica (ties to the lowest index)
  double* best_e;
};
constexpr int kBatchXcds = 8;        // per-XCD queues 0..7; queue 8 spans the device
constexpr int kBatchCtlWords = 256;  // control words of a batched launch (zeroed before it)
struct BatchArgs {
  const StepArgs* inst;       // per-instance step arguments (device array)
  const BatchSlot* slots;     // queue d holds slots [qoff[d], qoff[d + 1]), d = 0..8
  const int* qoff;            // kBatchXcds + 2 offsets
  const int* need;            // per XCD queue: workgroups its widest gang needs
  unsigned* ctl;              // kBatchCtlWords words, zero at launch
  unsigned* status;           // 1: a gang barrier timed out; 2: the start-up count did
  unsigned long long* clk;    // per slot: wall-clock ticks at start and end, or nullptr
  int grid;                   // workgroups of the launch (all co-resident)
  int lds_bytes;              // dynamic LDS per workgroup for J rows (0: J from L2 / MALL)
};

// ---- launchers (all asynchronous on `stream`) ----
hipError_t launch_fill_u32(unsigned* p, size_t count, unsigned v, hipStream_t stream);
// *flag = 0, then bit 0 set for a non-finite entry of x, y or p and bit 1 for |x| > 1
// among `count` elements of each (device arrays).
hipError_t launch_check_state(const float* x, const float* y, const float* p, size_t count, unsigned* flag,
                              hipStream_t stream);
hipError_t launch_encode_j(int form, bool fp4, const float* j32, int np, void* jf, hipStream_t stream);
// r_m = fl32(1 / (M - m)) for m < steps (linear schedule), else 0, computed on the device.
hipError_t launch_rtab(float* rtab, int steps, bool linear, hipStream_t stream);
hipError_t launch_encode_operand(int form, bool discrete, const float* x, size_t count, void* out,
                                 hipStream_t stream);
hipError_t launch_init_state(int n, int np, int rp, uint64_t seed, int mode, float* x, float* y,
                             float* p, hipStream_t stream);
// Persistent step kernel of variant `kind` (see Kind).  With `tangent` (binary32 form,
// generic kind, continuous variants) the launch's columns are the tangent-mode layout:
// blocks of 32 = 16 replicas followed by their 16 tangents.
hipError_t launch_steps(int form, int kind, const StepArgs& a, hipStream_t stream, bool tangent = false);
int max_coresident_workgroups(int form, int kind, int np, bool tangent = false);
// The register-resident FP8 kernel for nks = np / 128 in {4, 8, 12, 16}, else nullptr.
const void* steps_kernel_rj(int nks, bool discrete);
const void* steps_kernel_ws(int nks, bool discrete);
size_t steps_ws_lds_bytes(int np, bool discrete);
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
int choose_kind(int form, int np, int pref = 0);
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

// Batched instances (FP8 product, variants by `discrete`): the persistent queue kernel,
// its co-resident workgroups per CU, and the per-instance start, energy and best kernels
// over `count` instances (np_max: the largest np; rp replicas each, r_count of them real).
// occ: workgroups per CU the kernel variant is built for (1 or 2).
hipError_t launch_steps_batch(bool discrete, int occ, const BatchArgs& b, hipStream_t stream, bool cooperative);
int batch_workgroups_per_cu(bool discrete, int occ, int lds_bytes);
hipError_t launch_init_batch(const StepArgs* inst, const BatchInst* bi, int count, int np_max, int rp, int mode,
                             hipStream_t stream);
hipError_t launch_energy_batch(const StepArgs* inst, const BatchInst* bi, int count, int np_max, int rp,
                               int r_count, hipStream_t stream);
// This device's measured ceilings (gsb_probe.hip, built as its own library); synchronous,
// null stream.
hipError_t measure_ceilings(double* out, int count);
// Message of the last failed C ABI call on this thread (read by gsb_last_error).
void set_last_error(const char* msg);
// Lanczos estimate of the extreme eigenvalues of the symmetric n x n matrix J (host,
// binary64; a sparse J is multiplied in compressed-row form).
void extreme_eigenvalues(const float* J, int n, double* lmax, double* lmin);

}  // namespace gsb
