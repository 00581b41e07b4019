// gsb_steps_rj.hip -- the register-resident step kernel of libgsb (gfx950): FP8 product,
// J held as FP4 in the register files of the CUs for the whole launch (np <= 2048).
//
// The dynamics, eqs. (3)-(7) of Goto, Hidaka, Tatsumura (arXiv 2508.17655), are the ones
// of the generic step kernel; only the placement of J and the schedule of the K loop and
// barrier differ.  Contraction is off: the update is one binary32 rounding per operator.
#include "gsb_device.h"

#pragma clang fp contract(off)

namespace gsb {
namespace {

constexpr int kAccKSteps = 14;  // k-steps of J held in AGPRs (the rest in VGPRs)

// ---------------------------------------------------------------------------------------
// Register-resident step kernel for the FP8 product with np <= 2048 (NKS = np/128 k-steps).
//
// Workgroup (g, mb) owns spins [256 mb, 256 mb + 256) of replicas [32 g, 32 g + 32); wave
// w owns the 64 spins [256 mb + 64 w, +64) and keeps its 64 rows of J, as FP4 (exact for
// 0 and +-1), in registers for the whole launch: 4 row tiles x NKS fragments of 16 bytes
// per lane, k-steps [0, kAccKSteps) in accumulation registers (AGPRs, which the MFMA reads
// directly as its A operand) and the rest in VGPRs; at np = 2048 that is 224 AGPRs of J
// beside the 16 of the accumulators.  The four waves read the same Q fragments, from L2.
//
// The 32 replica columns form two independent sub-groups of 16 (column tiles 0 and 1),
// each with its own barrier counter, processed half a step apart:
//   K loop (sub 0) | wait (sub 1) + first Q loads of sub 1 | update (sub 0), publish, arrive
//   K loop (sub 1) | wait (sub 0, next step) + first loads | update (sub 1), publish, arrive
// so every wait comes half a step after the arrivals it needs, and the first operand loads
// of each K loop are in flight during the preceding update.
// ---------------------------------------------------------------------------------------
template <int NKS, bool DISC>
__global__ void __launch_bounds__(kThreads, 1) __attribute__((amdgpu_waves_per_eu(1, 1))) k_steps_rj(StepArgs a) {
  __shared__ int s_flag;
  __shared__ int s_local;
  constexpr int kPF = kKStepsUnroll;
  static_assert(NKS % kPF == 0 && NKS >= kPF, "k-steps must be a multiple of the prefetch depth");
  // k-steps [0, NACC) of J in AGPRs, [NACC, NKS) in VGPRs
  constexpr int NACC = NKS > kAccKSteps ? kAccKSteps : NKS;
  constexpr int NVJ = NKS - NACC;

  // the wave index is uniform within a wave; readfirstlane tells the compiler so
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = blockIdx.x % grid_groups(a);
  const int mb = blockIdx.x / grid_groups(a);
  if (g >= a.groups) return;  // a padding workgroup (see StepArgs::gpad)
  const int row0 = mb * 256 + wave * kWaveRows;
  const int col0 = g * kWaveCols;
  unsigned* ctr0 = a.sync + (size_t)(2 * g) * 64;
  unsigned* ctr1 = a.sync + (size_t)(2 * g + 1) * 64;
  unsigned* hs = a.sync + (size_t)(2 * a.groups + g) * 64;
  unsigned* msk = a.sync + (size_t)(3 * a.groups + g) * 64;
  unsigned* abort_flag = a.sync + (size_t)(4 * a.groups) * 64;

  // J rows of this wave (FP4 fragment-major, 1 KiB per (row tile, k-step)).
  v4i jr[4][NACC];
  v4i jv[4][NVJ > 0 ? NVJ : 1];
  {
    const uint8_t* jw = static_cast<const uint8_t*>(a.jf) + (size_t)(row0 >> 4) * NKS * 1024 + lane * 16;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        v4i f = *reinterpret_cast<const v4i*>(jw + (size_t)(rt * NKS + ks) * 1024);
        if (ks < NACC) {
          asm volatile("" : "+a"(f));  // place it in AGPRs
          jr[rt][ks < NACC ? ks : 0] = f;
        } else {
          jv[rt][ks < NACC ? 0 : ks - NACC] = f;
        }
      }
  }

  // State: [sub-group = column tile][row tile][v]; lane holds rows 4*(lane/16)+v of column
  // lane%16 of each 16 x 16 tile.
  float xs[2][4][4], ys[2][4][4], ps[2][4][4];
#pragma unroll
  for (int sub = 0; sub < 2; ++sub)
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int i = row0 + rt * 16 + 4 * (lane >> 4);
      const int r = col0 + sub * 16 + (lane & 15);
      const size_t o = (size_t)r * a.np + i;
      const v4f vx = *reinterpret_cast<const v4f*>(a.x + o);
      const v4f vy = *reinterpret_cast<const v4f*>(a.y + o);
      const v4f vp = *reinterpret_cast<const v4f*>(a.p + o);
#pragma unroll
      for (int v = 0; v < 4; ++v) { xs[sub][rt][v] = vx[v]; ys[sub][rt][v] = vy[v]; ps[sub][rt][v] = vp[v]; }
    }

  // Handshake: learn whether all members of this group run on one XCD.
  if (tid == 0) {
    const unsigned xcc = (unsigned)__builtin_amdgcn_s_getreg(kHwRegXccId) & 15u;
    __hip_atomic_fetch_or(msk, 1u << xcc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(hs, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    unsigned spins = 0;
    while (ld_dev(hs) < (unsigned)a.nb) {
      ++spins;
      if ((spins & 63u) == 0 && ld_dev(abort_flag)) { ok = 0; break; }
      if (spins > kSpinLimit) { st_dev(abort_flag, 1u); st_dev(a.status, 1u); ok = 0; break; }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_local = (__builtin_popcount(ld_dev(msk)) == 1) ? 1 : 0;
    s_flag = ok;
  }
  __syncthreads();
  bool alive = s_flag != 0;
  const int local = s_local;

  // arrive: this workgroup's operand stores for `ctr` are complete and counted.
  auto arrive = [&](unsigned* ctr) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      if (!local) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  // wait: every member has arrived `target` times on `ctr` (across XCDs, behind an
  // agent-scope acquire fence).  The operand loads bypass L1, so no L1 line can be stale
  // (a workgroup-scope invalidate does not reliably drop lines other CUs have rewritten).
  // `seen` is a count read earlier (mid K loop); when it already reaches the target the
  // poll round trip is skipped.
  auto wait = [&](unsigned* ctr, unsigned target, unsigned seen) -> bool {
    if (tid == 0) {
      int ok = 1;
      unsigned spins = 0;
      unsigned v = seen;
      while (v < target) {
        v = ld_dev(ctr);
        ++spins;
        if ((spins & 63u) == 0 && ld_dev(abort_flag)) { ok = 0; break; }
        if (spins > kSpinLimit) { st_dev(abort_flag, 1u); st_dev(a.status, 1u); ok = 0; break; }
      }
      if (!local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_flag = ok;
    }
    __syncthreads();
    return s_flag != 0;
  };

  const __amdgpu_buffer_rsrc_t qr = make_rsrc(a.q, 2 * a.q_buf_bytes);
  v8i bq[kPF];
  // Q fragment of column tile `sub`, k-step ks, in ping-pong buffer `buf`.
  auto load_b = [&](int sub, int buf, int ks, v8i& dst) {
    const unsigned base = (unsigned)((size_t)buf * a.q_buf_bytes) +
                          (unsigned)(((2 * g + sub) * NKS + ks) * 2048 + lane * 16);
    const v4i lo = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(qr, base, 0, kPolicySc1));
    const v4i hi = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(qr, base + 1024, 0, kPolicySc1));
    dst = cat(lo, hi);
  };
  auto prefetch = [&](int sub, int buf) {
#pragma unroll
    for (int u = 0; u < kPF; ++u) load_b(sub, buf, u, bq[u]);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  };

  const float A = a.A, dt = a.dt, cdt = a.cdt;
  // Update of column tile `sub` with the product in acc (eqs. (7), (3), (4), (5), binary32,
  // one rounding per operator), then its operand for the next step.  Written stage by
  // stage over the 16 elements of the tile so that each stage is 16 independent operations.
  auto update = [&](int sub, const v4f* acc, float rm, uint8_t* qnext) {
    float t[16], u[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) { const float x = xs[sub][e >> 2][e & 3]; t[e] = x * x; }
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = A * t[e];
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = 1.0f - t[e];
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = t[e] * ps[sub][e >> 2][e & 3];
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = t[e] * rm;
#pragma unroll
    for (int e = 0; e < 16; ++e) ps[sub][e >> 2][e & 3] = ps[sub][e >> 2][e & 3] - t[e];  // p(t_{m+1})
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = ps[sub][e >> 2][e & 3] * xs[sub][e >> 2][e & 3];
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = t[e] * dt;
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = ys[sub][e >> 2][e & 3] - t[e];            // y + dy
#pragma unroll
    for (int e = 0; e < 16; ++e) u[e] = cdt * acc[e >> 2][e & 3];                 // Dy
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = t[e] + u[e];                              // eq. (3)
#pragma unroll
    for (int e = 0; e < 16; ++e) u[e] = t[e] * dt;
#pragma unroll
    for (int e = 0; e < 16; ++e) u[e] = xs[sub][e >> 2][e & 3] + u[e];            // eq. (4)
#pragma unroll
    for (int e = 0; e < 16; ++e) {                                                // eq. (5)
      ys[sub][e >> 2][e & 3] = __builtin_fabsf(u[e]) > 1.0f ? 0.0f : t[e];
      xs[sub][e >> 2][e & 3] = __builtin_amdgcn_fmed3f(u[e], -1.0f, 1.0f);
    }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
      store_operand<kFormFP8, DISC>(qnext, a.q_buf_bytes, NKS, row0 + rt * 16, col0 + sub * 16, lane,
                                    xs[sub][rt]);
  };

  // Operand of the starting state for both column tiles, then the first arrivals.
  if (alive) {
#pragma unroll
    for (int sub = 0; sub < 2; ++sub)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
        store_operand<kFormFP8, DISC>(a.q, a.q_buf_bytes, NKS, row0 + rt * 16, col0 + sub * 16, lane,
                                      xs[sub][rt]);
    arrive(ctr0);
    arrive(ctr1);
    alive = wait(ctr0, (unsigned)a.nb, 0u);
    if (alive) prefetch(0, 0);
  }

  const int steps = a.m_end - a.m_begin;
  for (int s = 0; alive && s < steps; ++s) {
    const int m = a.m_begin + s;
    const int cur = s & 1;
    uint8_t* qnext = a.q + (size_t)(cur ^ 1) * a.q_buf_bytes;
    const float rm = a.rtab[m];
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) {
      unsigned seen = 0;  // count of the other column tile's counter, read mid K loop
      unsigned* const other = sub == 0 ? ctr1 : ctr0;
      v4f acc[4];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) acc[rt] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
          const v4i f = ks < NACC ? jr[rt][ks < NACC ? ks : 0] : jv[rt][ks < NACC ? 0 : ks - NACC];
          acc[rt] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(cat(f, f), bq[ks % kPF], acc[rt], 4, 0, 0,
                                                                     127, 0, 127);
        }
        // Pin this k-step's MFMAs here: the empty asm reads and redefines the accumulators
        // and, being volatile, keeps its place relative to the memory fences around the
        // prefetches, so loads and MFMAs stay interleaved as written.
        asm volatile("" : "+a"(acc[0]), "+a"(acc[1]), "+a"(acc[2]), "+a"(acc[3]));
        if (ks + kPF < NKS) load_b(sub, cur, ks + kPF, bq[ks % kPF]);
        if (ks == NKS / 2 && tid == 0) seen = ld_dev(other);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
      }
      // wait for the other column tile's data and start its first loads
      if (sub == 0) {
        alive = wait(ctr1, (unsigned)((s + 1) * a.nb), seen);
        if (alive) prefetch(1, cur);
      } else if (s + 1 < steps) {
        alive = wait(ctr0, (unsigned)((s + 2) * a.nb), seen);
        if (alive) prefetch(0, cur ^ 1);
      }
      if (!alive) break;
      update(sub, acc, rm, qnext);
      arrive(sub == 0 ? ctr0 : ctr1);
    }
  }

#pragma unroll
  for (int sub = 0; sub < 2; ++sub)
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int i = row0 + rt * 16 + 4 * (lane >> 4);
      const int r = col0 + sub * 16 + (lane & 15);
      const size_t o = (size_t)r * a.np + i;
      *reinterpret_cast<v4f*>(a.x + o) = v4f{xs[sub][rt][0], xs[sub][rt][1], xs[sub][rt][2], xs[sub][rt][3]};
      *reinterpret_cast<v4f*>(a.y + o) = v4f{ys[sub][rt][0], ys[sub][rt][1], ys[sub][rt][2], ys[sub][rt][3]};
      *reinterpret_cast<v4f*>(a.p + o) = v4f{ps[sub][rt][0], ps[sub][rt][1], ps[sub][rt][2], ps[sub][rt][3]};
    }
}

}  // namespace

const void* steps_kernel_rj(int nks, bool discrete) {
  if (discrete) {
    switch (nks) {
      case 4: return reinterpret_cast<const void*>(&k_steps_rj<4, true>);
      case 8: return reinterpret_cast<const void*>(&k_steps_rj<8, true>);
      case 12: return reinterpret_cast<const void*>(&k_steps_rj<12, true>);
      case 16: return reinterpret_cast<const void*>(&k_steps_rj<16, true>);
      default: return nullptr;
    }
  }
  switch (nks) {
    case 4: return reinterpret_cast<const void*>(&k_steps_rj<4, false>);
    case 8: return reinterpret_cast<const void*>(&k_steps_rj<8, false>);
    case 12: return reinterpret_cast<const void*>(&k_steps_rj<12, false>);
    case 16: return reinterpret_cast<const void*>(&k_steps_rj<16, false>);
    default: return nullptr;
  }
}

}  // namespace gsb
