// gsb_kernels.hip -- gfx950 kernels of libgsb.
//
// Simulated bifurcation (Goto, Hidaka, Tatsumura, arXiv 2508.17655): every step is
//   p_i <- p_i - [1 - A x_i^2] p_i / (M - m)                    eq. (7) (eq. (6) at A = 0)
//   y_i <- y_i - p_i(t_{m+1}) x_i dt + c dt sum_j J_ij q_j      eq. (3), q = x or sgn(x)
//   x_i <- x_i + y_i dt                                         eq. (4)
//   |x_i| > 1  =>  x_i <- sgn(x_i), y_i <- 0                    eq. (5)
// for R independent replicas at once (batch processing, Sec. VI).  The coupling product
// of all replicas is one GEMM, G = J Q, with replicas as columns; it runs on MFMA and the
// update above is fused into its epilogue, which also writes the next step's operand Q.
//
// Floating-point contraction is disabled for this file: the update is evaluated as one
// binary32 operation per arithmetic operator, in the order written, so the sign and E4M3
// forms reproduce a strict binary32 evaluation bit for bit.
#include "gsb_device.h"
#include "gsb_internal.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#pragma clang fp contract(off)

namespace gsb {
namespace {

// One wave's 64 x 32 tile of G = J Q in the binary32 form: 4 row tiles (J rows, `jrows`)
// x 2 column tiles (Q blocks rb0, rb0 + 1 of the buffer behind `qr`) of 16x16x4 MFMAs.
__device__ __forceinline__ void gemm_tile_fp32(const uint8_t* jrows, __amdgpu_buffer_rsrc_t qr, int rb0, int nks,
                                               int lane, v4f (&acc)[4][2]) {
  for (int ks = 0; ks < nks; ++ks) {
    for (int grp = 0; grp < 8; ++grp) {
      v4f aj[4], bq[2];
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        const size_t o = ((size_t)(rt * nks + ks) * 8 + grp) * 1024 + lane * 16;
        aj[rt] = *reinterpret_cast<const v4f*>(jrows + o);
      }
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        const unsigned base = (unsigned)(((size_t)((rb0 + ct) * nks + ks) * 8 + grp) * 1024 + lane * 16);
        bq[ct] = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(qr, base, 0, kPolicySc1));
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct)
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(aj[rt][t], bq[ct][t], acc[rt][ct], 0, 0, 0);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Generic persistent step tile (any product form; J fragments read from L2 or MALL).
// Workgroup (g, mb) owns spins [BM mb, BM mb + BM) of replicas [BN g, BN g + BN), with
// BM x BN = 64 x 128, 128 x 64 or 256 x 32; each of its 4 waves computes a 64 x 32 tile
// of G = J Q (4 x 2 MFMA tiles of 16 x 16) and keeps x, y, p of those 2048 elements in
// registers for the whole launch.  The nb = np / BM workgroups of one replica group
// synchronise every step.  For the FP8 product J is read as FP4 (E2M1, exact for 0 and
// +-1; the FP8 form requires J in {0, +-1}), half the bytes of FP8.
//
// With `lds_j` (FP8 product) the workgroup first copies the leading k-steps of its J rows
// into LDS, as many as `lds_bytes` holds (all of them for 64 rows up to np = 4096 in
// 128 KiB), and reads those from LDS every step: J then costs no L2, MALL or HBM traffic.
//
// k_steps runs one tile per workgroup, b = (g, mb) = (b mod groups, b div groups): with
// 8 or 16 groups, round-robin dispatch puts each group on one XCD.
//
// TANG (binary32 product, continuous variants): the launch's columns come in blocks of
// 32 whose first 16 are replicas and whose last 16 carry the forward derivative (the
// tangent) of the same 16 replicas, so one lane holds an element's state and its
// tangent, and one GEMM forms both J x and J dx.  The tangent follows the derivative of
// eqs. (7), (3), (4), (5) (see the update below); the control strength may differ per
// replica (a.acol).
// ---------------------------------------------------------------------------------------
template <int FORM, bool DISC, bool TANG, int BM, bool LJ = false, int QD = kKStepsUnroll>
__device__ __forceinline__ void steps_tile(const StepArgs& a, int g, int mb, int& s_flag, int& s_local,
                                           uint8_t* lds_j = nullptr, int lds_bytes = 0) {
  static_assert(!LJ || FORM == kFormFP8 || FORM == kFormFIX16, "J rows in LDS: FP8 (FP4 J) or FIX16 (int8 J)");
  static_assert(!TANG || (FORM == kFormFP32 && !DISC), "the tangent needs the continuous binary32 product");
  static_assert(BM == 64 || BM == 128 || BM == 256, "tile rows");
  constexpr int BN = 8192 / BM;
  constexpr int WCOLS = BN / kWaveCols;  // waves across the replica columns
  // operand loads bypass L1 (see kPolicySc1)
  constexpr int kQPolicy = kPolicySc1;

  // the wave index is uniform within a wave; readfirstlane tells the compiler so
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wrow = wave / WCOLS;             // 64-row slice of the workgroup's rows
  const int row0 = mb * BM + wrow * kWaveRows;
  const int col0 = g * BN + (wave % WCOLS) * kWaveCols;
  const int nks = a.np / kKS;
  unsigned* ctr = a.sync + (size_t)g * 64;
  unsigned* hs = a.sync + (size_t)(a.groups + g) * 64;
  unsigned* msk = a.sync + (size_t)(2 * a.groups + g) * 64;
  unsigned* abort_flag = a.sync + (size_t)(3 * a.groups) * 64;
  const size_t jblk = FORM == kFormFP8 ? 1024 : operand_block_bytes(FORM);  // FP8 product: FP4 J
  const size_t plane_bytes = a.q_buf_bytes / operand_planes(FORM);

  // J rows of this wave: 4 row tiles x nks k-steps, contiguous in the layout (FIX16: 2
  // row tiles of 32, the same bytes).
  const uint8_t* jrows = static_cast<const uint8_t*>(a.jf) + (size_t)(mb * BM / 16 + 4 * wrow) * nks * jblk;

  // Elements of the wave's 64 x 32 tile held by this lane: rows row0 + er(rt, ct) + v
  // (v < 4) of column col0 + ec(ct).  With 16x16 MFMA tiles (4 x 2 of them) that is rows
  // 16 rt + 4 (lane/16) + v of column 16 ct + lane%16; BF16X2 and FIX16 use 32x32 tiles
  // (2 x 1), whose lane holds rows 32 (g/4) + 8 (g%4) + 4 (lane/32) + v of column lane%32
  // for register group g = 2 rt + ct.
  constexpr bool T32 = FORM == kFormFIX16 || FORM == kFormBF16X2;
  auto er = [&](int rt, int ct) {
    return T32 ? 32 * (rt >> 1) + 8 * ((2 * rt + ct) & 3) + 4 * (lane >> 5) : rt * 16 + 4 * (lane >> 4);
  };
  auto ec = [&](int ct) { return T32 ? (lane & 31) : ct * 16 + (lane & 15); };
  // operand of the lane's elements (store_operand takes the 16x16 tile origin, or for
  // FIX16 the lane's own first element)
  auto store_q = [&](uint8_t* buf, int rt, int ct, const float* xv) {
    store_operand<FORM, DISC>(buf, plane_bytes, nks, row0 + (T32 ? er(rt, ct) : rt * 16),
                              col0 + (T32 ? ec(ct) : ct * 16), lane, xv);
  };

  float xs[4][2][4], ys[4][2][4], ps[4][2][4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int i = row0 + er(rt, ct);
      const int r = col0 + ec(ct);
      const size_t o = (size_t)r * a.np + i;
      v4f vx = *reinterpret_cast<const v4f*>(a.x + o);
      v4f vy = *reinterpret_cast<const v4f*>(a.y + o);
      v4f vp = *reinterpret_cast<const v4f*>(a.p + o);
#pragma unroll
      for (int v = 0; v < 4; ++v) { xs[rt][ct][v] = vx[v]; ys[rt][ct][v] = vy[v]; ps[rt][ct][v] = vp[v]; }
    }

  // Leading k-steps of this workgroup's J rows into LDS: [row tile][k-step][lane][16 B].
  int nks_l = 0;
  if constexpr (LJ && FORM == kFormFIX16) {
    // int8 J: the workgroup's BM rows are one contiguous BM * np byte range; all of it or
    // none (the launch gives BM * np bytes of LDS when it fits)
    const size_t bytes = (size_t)BM * a.np;
    nks_l = bytes <= (size_t)lds_bytes ? nks : 0;
    if (nks_l) {
      const uint8_t* jwg = static_cast<const uint8_t*>(a.jf) + (size_t)mb * BM * a.np;
      for (size_t c = tid; c < bytes / 16; c += kThreads)
        *reinterpret_cast<v4i*>(lds_j + c * 16) = *reinterpret_cast<const v4i*>(jwg + c * 16);
    }
    __syncthreads();
  } else if constexpr (LJ) {
    {
      constexpr int kTilesWG = BM / 16;
      nks_l = min(nks, lds_bytes / (kTilesWG * 1024)) / QD * QD;  // whole pipeline rounds
      const uint8_t* jwg = static_cast<const uint8_t*>(a.jf) + (size_t)(mb * kTilesWG) * nks * 1024;
      const int chunks = kTilesWG * nks_l * 64;
      for (int c = tid; c < chunks; c += kThreads) {
        const int t = c / (nks_l * 64), rem = c - t * (nks_l * 64);
        const int ks = rem >> 6, l = rem & 63;
        *reinterpret_cast<v4i*>(lds_j + (size_t)c * 16) =
            *reinterpret_cast<const v4i*>(jwg + ((size_t)t * nks + ks) * 1024 + l * 16);
      }
      __syncthreads();
    }
  }
  // this wave's row tiles in LDS
  const uint8_t* jlds = !LJ ? nullptr
                        : FORM == kFormFIX16 ? lds_j + (size_t)(2 * wrow) * nks * 4096 + lane * 16
                                             : lds_j + (size_t)(4 * wrow) * nks_l * 1024 + lane * 16;

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

  // Operand of the starting state, then the first group barrier.
  if (alive) {
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
        store_q(a.q, rt, ct, xs[rt][ct]);
    alive = group_sync(ctr, (unsigned)a.nb, local, abort_flag, a.status, &s_flag);
  }

  const float A = a.A, dt = a.dt, cdt = a.cdt;
  const int steps = a.m_end - a.m_begin;
  for (int s = 0; alive && s < steps; ++s) {
    const int m = a.m_begin + s;
    const uint8_t* qcur = a.q + (size_t)(s & 1) * a.q_buf_bytes;
    uint8_t* qnext = a.q + (size_t)((s + 1) & 1) * a.q_buf_bytes;
    const __amdgpu_buffer_rsrc_t qr = make_rsrc(qcur, a.q_buf_bytes);
    const int rb0 = col0 >> 4;

    v4f acc[4][2];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = v4f{0.0f, 0.0f, 0.0f, 0.0f};

    if constexpr (FORM == kFormFP8) {
      // Software pipeline: Q fragments are fetched kPF k-steps ahead, FP4 J fragments one
      // k-step ahead from LDS or kPF - 1 ahead from L2/MALL, so no latency stalls the
      // MFMA stream.  The k-steps run in two segments, [0, nks_l) with J from LDS and
      // [nks_l, nks) with J from L2, each a pipeline of its own: J registers are then
      // never written by an LDS read while a global load to them may be in flight (which
      // would force a full wait).  The pipelined part of a segment is a multiple of kPF
      // k-steps (any remainder runs first, unpipelined); its last kPF k-steps are peeled
      // without Q loads.
      constexpr int kPF = QD;
      static_assert(kKStepsUnroll % kPF == 0, "a pipeline round divides the single-instance padding");
      v8i bq[kPF][2];
      auto load_b = [&](int ks, v8i* dst) {
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const unsigned base = (unsigned)(((rb0 + ct) * nks + ks) * 2048 + lane * 16);
          v4i lo = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(qr, base, 0, kQPolicy));
          v4i hi = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(qr, base + 1024, 0, kQPolicy));
          dst[ct] = cat(lo, hi);
        }
      };
      auto load_a_glb = [&](int ks, v4i* dst) {
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
          dst[rt] = *reinterpret_cast<const v4i*>(jrows + (size_t)(rt * nks + ks) * 1024 + lane * 16);
      };
      auto load_a_lds = [&](int ks, v4i* dst) {
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) dst[rt] = *reinterpret_cast<const v4i*>(jlds + (size_t)(rt * nks_l + ks) * 1024);
      };
      auto mfmas = [&](const v4i* aa, const v8i* bb) {
        // A: FP4 (format code 4, the upper four registers unused), B: FP8 E4M3, unit scales
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct)
            acc[rt][ct] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(cat(aa[rt], aa[rt]), bb[ct], acc[rt][ct],
                                                                           4, 0, 0, 127, 0, 127);
      };
      // JD: J prefetch distance (1 or kPF - 1), in a ring of JD + 1 register sets that
      // divides kPF, so every ring index is a compile-time constant
      auto segment = [&](int k0, int k1, auto load_a, auto jd) {
        constexpr int JD = decltype(jd)::value;
        constexpr int RING = JD + 1;
        static_assert(kPF % RING == 0, "J ring must divide the unroll");
        v4i aj[RING][4];
#pragma unroll
        for (int u = 0; u < kPF; ++u) load_b(k0 + u, bq[u]);
#pragma unroll
        for (int d = 0; d < JD; ++d) load_a(k0 + d, aj[d]);  // segments hold >= kPF > JD k-steps
        int ks0 = k0;
        for (; ks0 < k1 - kPF; ks0 += kPF) {
#pragma unroll
          for (int u = 0; u < kPF; ++u) {
            load_a(ks0 + u + JD, aj[(u + JD) % RING]);  // < k1: ks0 + kPF <= k1 - kPF
            __builtin_amdgcn_sched_barrier(0);          // keep each prefetch ahead of the MFMAs
            mfmas(aj[u % RING], bq[u]);
            load_b(ks0 + u + kPF, bq[u]);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
#pragma unroll
        for (int u = 0; u < kPF; ++u) {
          if (u + JD < kPF) load_a(ks0 + u + JD, aj[(u + JD) % RING]);
          __builtin_amdgcn_sched_barrier(0);
          mfmas(aj[u % RING], bq[u]);
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      // A segment whose length is not a multiple of kPF (a batched instance padded to two
      // k-steps, in the one-workgroup-per-CU variant) runs its first (k1 - k0) mod kPF
      // k-steps without a pipeline, before the pipeline's prologue.
      auto run_segment = [&](int k0, int k1, auto load_a, auto jd) {
        const int r = (k1 - k0) % kPF;
        for (int ks = k0; ks < k0 + r; ++ks) {
          v4i aa[4];
          load_b(ks, bq[0]);
          load_a(ks, aa);
          mfmas(aa, bq[0]);
        }
        if (k1 - k0 - r > 0) segment(k0 + r, k1, load_a, jd);
      };
      if constexpr (LJ) {
        if (nks_l > 0) run_segment(0, nks_l, load_a_lds, std::integral_constant<int, 1>{});
      }
      if (nks_l < nks) run_segment(nks_l, nks, load_a_glb, std::integral_constant<int, kPF - 1>{});
    } else if constexpr (FORM == kFormBF16X2) {
      // hi and lo planes of x (the sign operand has no low part) against bf16 J on
      // 32x32x16 MFMAs (the 16x16x32 shape runs at ~55% of their rate here), binary32
      // accumulation, one accumulator per plane and 32-row tile; G = G_hi + G_lo.
      // Software pipeline over sixteenth k-steps (16 spins, 2 or 4 MFMAs each): Q
      // fragments kQS sixteenths ahead and J fragments kJS ahead, in register rings whose
      // indices are compile-time constants.  8 nks is a multiple of kQS; the last kQS
      // sixteenths are peeled without Q loads.
      constexpr int planes = DISC ? 1 : 2;
      constexpr int kQS = 2 * kKStepsUnroll;  // 8 sixteenths
      constexpr int kJS = 3, kJR = 4;         // J distance and ring (kJR divides kQS)
      typedef float v16f __attribute__((ext_vector_type(16)));
      v16f facc[2][2];  // [plane][32-row tile]
#pragma unroll
      for (int pl = 0; pl < 2; ++pl)
#pragma unroll
        for (int t = 0; t < 2; ++t) facc[pl][t] = v16f{};
      const int nsub = 8 * nks;
      const int cb = col0 >> 5;  // the wave's 32-column block
      v8bf aj[kJR][2];
      v8bf bq[kQS][planes];
      auto load_a = [&](int sb, v8bf* dst) {
#pragma unroll
        for (int t = 0; t < 2; ++t)
          dst[t] = *reinterpret_cast<const v8bf*>(jrows + ((size_t)(t * nks + (sb >> 3)) * 8 + (sb & 7)) * 1024 +
                                                  lane * 16);
      };
      auto load_b = [&](int sb, v8bf* dst) {
#pragma unroll
        for (int pl = 0; pl < planes; ++pl) {
          const unsigned base =
              (unsigned)(pl * plane_bytes + ((size_t)(cb * nks + (sb >> 3)) * 8 + (sb & 7)) * 1024 + lane * 16);
          dst[pl] = __builtin_bit_cast(v8bf, __builtin_amdgcn_raw_buffer_load_b128(qr, base, 0, kQPolicy));
        }
      };
      auto mfmas = [&](const v8bf* aa, const v8bf* bb) {
#pragma unroll
        for (int pl = 0; pl < planes; ++pl)
#pragma unroll
          for (int t = 0; t < 2; ++t)
            facc[pl][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aa[t], bb[pl], facc[pl][t], 0, 0, 0);
      };
#pragma unroll
      for (int u = 0; u < kQS; ++u) load_b(u, bq[u]);
#pragma unroll
      for (int d = 0; d < kJS; ++d) load_a(d, aj[d]);
      int s0 = 0;
      for (; s0 < nsub - kQS; s0 += kQS) {
#pragma unroll
        for (int u = 0; u < kQS; ++u) {
          load_a(s0 + u + kJS, aj[(u + kJS) % kJR]);  // < nsub: s0 <= nsub - 2 kQS
          __builtin_amdgcn_sched_barrier(0);
          mfmas(aj[u % kJR], bq[u]);
          load_b(s0 + u + kQS, bq[u]);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (int u = 0; u < kQS; ++u) {
        if (u + kJS < kQS) load_a(s0 + u + kJS, aj[(u + kJS) % kJR]);
        __builtin_amdgcn_sched_barrier(0);
        mfmas(aj[u % kJR], bq[u]);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int j = 4 * ((2 * rt + ct) & 3) + v;
            acc[rt][ct][v] = planes == 2 ? facc[0][rt >> 1][j] + facc[planes - 1][rt >> 1][j] : facc[0][rt >> 1][j];
          }
    } else if constexpr (FORM == kFormFIX16) {
      // two int8 passes (hi, lo planes; the sign operand has lo = 0) on 32x32x32 MFMAs
      // (the 16x16x64 shape runs at ~58% of their rate here), exact int32 sums;
      // G = 256 G_hi + G_lo is exact in int32 and rounded to binary32 once, then scaled.
      // Software pipeline over quarter k-steps (32 spins, 4 MFMAs each): Q fragments of
      // both planes are fetched kQS quarters ahead and J fragments kJS ahead, in register
      // rings whose indices are compile-time constants.  4 nks is a multiple of kQS; the
      // last kQS quarters are peeled without Q loads.
      constexpr int planes = DISC ? 1 : 2;
      constexpr int kQS = 2 * kKStepsUnroll;  // 8 quarters
      constexpr int kJS = 3, kJR = 4;         // J distance and ring (kJR divides kQS)
      typedef int v16i __attribute__((ext_vector_type(16)));
      v16i iacc[2][2];  // [plane][32-row tile]
#pragma unroll
      for (int pl = 0; pl < 2; ++pl)
#pragma unroll
        for (int t = 0; t < 2; ++t) iacc[pl][t] = v16i{};
      const int nsub = 4 * nks;  // a multiple of 16
      const int cb = col0 >> 5;  // the wave's 32-column block
      v4i aj[kJR][2];
      v4i bq[kQS][planes];
      auto load_a_glb = [&](int sb, v4i* dst) {
#pragma unroll
        for (int t = 0; t < 2; ++t)
          dst[t] = *reinterpret_cast<const v4i*>(jrows + ((size_t)(t * nks + (sb >> 2)) * 4 + (sb & 3)) * 1024 +
                                                 lane * 16);
      };
      auto load_a_lds = [&](int sb, v4i* dst) {
#pragma unroll
        for (int t = 0; t < 2; ++t)
          dst[t] = *reinterpret_cast<const v4i*>(jlds + ((size_t)(t * nks + (sb >> 2)) * 4 + (sb & 3)) * 1024);
      };
      auto load_b = [&](int sb, v4i* dst) {
#pragma unroll
        for (int pl = 0; pl < planes; ++pl) {
          const unsigned base =
              (unsigned)(pl * plane_bytes + ((size_t)(cb * nks + (sb >> 2)) * 4 + (sb & 3)) * 1024 + lane * 16);
          dst[pl] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(qr, base, 0, kQPolicy));
        }
      };
      auto mfmas = [&](const v4i* aa, const v4i* bb) {
#pragma unroll
        for (int pl = 0; pl < planes; ++pl)
#pragma unroll
          for (int t = 0; t < 2; ++t)
            iacc[pl][t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(aa[t], bb[pl], iacc[pl][t], 0, 0, 0);
      };
      // one pipeline per J source (LDS or L2), so no register is written by both kinds
      // of load
      auto pipeline = [&](auto load_a) {
#pragma unroll
        for (int u = 0; u < kQS; ++u) load_b(u, bq[u]);
#pragma unroll
        for (int d = 0; d < kJS; ++d) load_a(d, aj[d]);
        int s0 = 0;
        for (; s0 < nsub - kQS; s0 += kQS) {
#pragma unroll
          for (int u = 0; u < kQS; ++u) {
            load_a(s0 + u + kJS, aj[(u + kJS) % kJR]);  // < nsub: s0 <= nsub - 2 kQS
            __builtin_amdgcn_sched_barrier(0);
            mfmas(aj[u % kJR], bq[u]);
            load_b(s0 + u + kQS, bq[u]);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
#pragma unroll
        for (int u = 0; u < kQS; ++u) {
          if (u + kJS < kQS) load_a(s0 + u + kJS, aj[(u + kJS) % kJR]);
          __builtin_amdgcn_sched_barrier(0);
          mfmas(aj[u % kJR], bq[u]);
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      if (LJ && nks_l == nks)
        pipeline(load_a_lds);
      else
        pipeline(load_a_glb);
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int j = 4 * ((2 * rt + ct) & 3) + v;
            acc[rt][ct][v] = (float)(iacc[0][rt >> 1][j] * 256 + iacc[1][rt >> 1][j]) * 0x1p-14f;
          }
    } else {  // FP32
      gemm_tile_fp32(jrows, qr, rb0, nks, lane, acc);
    }

    // Fused update, eqs. (7), (3), (4), (5), in binary32, one rounding per operator.
    const float rm = a.rtab[m];
    if constexpr (TANG) {
      // Column tile 0: the replicas; column tile 1: their tangents (dx, dy, dp).  With
      // f = 1 - A x^2:  dp' = dp (1 - f r) + 2 A x dx p r,
      // dy' = dy - (dp' x + p' dx) dt + c dt (J dx),  dx' = dx + dy' dt,
      // and both dx' and dy' are 0 where the wall acts.
      const float Ar = a.acol ? a.acol[(col0 >> 1) + (lane & 15)] : A;
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float x = xs[rt][0][v], y = ys[rt][0][v], p = ps[rt][0][v];
          const float tx = xs[rt][1][v], ty = ys[rt][1][v], tp = ps[rt][1][v];
          const float xx = x * x;
          const float ax = Ar * xx;
          const float f = 1.0f - ax;
          const float fp = f * p;
          const float dp = fp * rm;
          const float pn = p - dp;
          const float px = pn * x;
          const float pxdt = px * dt;
          const float y1 = y - pxdt;
          const float gy = cdt * acc[rt][0][v];
          const float yn = y1 + gy;
          const float dxs = yn * dt;
          const float xn = x + dxs;
          const bool hit = __builtin_fabsf(xn) > 1.0f;
          const float fr = f * rm;
          const float keep = 1.0f - fr;
          const float ctl = (((2.0f * Ar) * x) * tx) * p;
          const float tpn = tp * keep + ctl * rm;
          const float dyp = (tpn * x + pn * tx) * dt;
          const float tyn = (ty - dyp) + cdt * acc[rt][1][v];
          const float txn = tx + tyn * dt;
          xs[rt][0][v] = __builtin_amdgcn_fmed3f(xn, -1.0f, 1.0f);
          ys[rt][0][v] = hit ? 0.0f : yn;
          ps[rt][0][v] = pn;
          xs[rt][1][v] = hit ? 0.0f : txn;
          ys[rt][1][v] = hit ? 0.0f : tyn;
          ps[rt][1][v] = tpn;
        }
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
          store_q(qnext, rt, ct, xs[rt][ct]);
      }
    } else {
    if (a.tape) {  // record this step's input state (reverse pass)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const size_t o = (size_t)(col0 + ct * 16 + (lane & 15)) * a.np + row0 + rt * 16 + 4 * (lane >> 4);
          float* t = a.tape + (size_t)3 * s * a.tape_arr + o;
          *reinterpret_cast<v4f*>(t) = v4f{xs[rt][ct][0], xs[rt][ct][1], xs[rt][ct][2], xs[rt][ct][3]};
          *reinterpret_cast<v4f*>(t + a.tape_arr) = v4f{ys[rt][ct][0], ys[rt][ct][1], ys[rt][ct][2], ys[rt][ct][3]};
          *reinterpret_cast<v4f*>(t + 2 * a.tape_arr) = v4f{ps[rt][ct][0], ps[rt][ct][1], ps[rt][ct][2], ps[rt][ct][3]};
        }
    }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float x = xs[rt][ct][v], y = ys[rt][ct][v], p = ps[rt][ct][v];
          const float gsum = acc[rt][ct][v];
          const float xx = x * x;
          const float ax = A * xx;
          const float f = 1.0f - ax;
          const float fp = f * p;
          const float dp = fp * rm;
          const float pn = p - dp;        // p_i(t_{m+1}), eq. (7)
          const float px = pn * x;
          const float pxdt = px * dt;
          const float y1 = y - pxdt;      // y + dy
          const float gy = cdt * gsum;    // Dy = c dt sum_j J_ij q_j
          const float yn = y1 + gy;       // eq. (3)
          const float dx = yn * dt;
          const float xn = x + dx;        // eq. (4)
          // eq. (5): beyond a wall x becomes sgn(x) (a clamp to [-1, 1]) and y becomes 0
          const bool hit = __builtin_fabsf(xn) > 1.0f;
          xs[rt][ct][v] = __builtin_amdgcn_fmed3f(xn, -1.0f, 1.0f);
          ys[rt][ct][v] = hit ? 0.0f : yn;
          ps[rt][ct][v] = pn;
        }
        if constexpr (FORM != kFormFP8) store_q(qnext, rt, ct, xs[rt][ct]);
      }
    if constexpr (FORM == kFormFP8) {
      // the FP8 placement keeps a lane's four row tiles of a column tile in 16 contiguous,
      // aligned bytes (row0 is a multiple of 64): one 16-byte store per column tile
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        const v4u w{encode_fp8x4<DISC>(xs[0][ct]), encode_fp8x4<DISC>(xs[1][ct]), encode_fp8x4<DISC>(xs[2][ct]),
                    encode_fp8x4<DISC>(xs[3][ct])};
        *reinterpret_cast<v4u*>(qnext + fp8_operand_offset(nks, row0, col0 + ct * 16, lane)) = w;
      }
    }
    }
    alive = group_sync(ctr, (unsigned)((s + 2) * a.nb), local, abort_flag, a.status, &s_flag);
  }

#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int i = row0 + er(rt, ct);
      const int r = col0 + ec(ct);
      const size_t o = (size_t)r * a.np + i;
      *reinterpret_cast<v4f*>(a.x + o) = v4f{xs[rt][ct][0], xs[rt][ct][1], xs[rt][ct][2], xs[rt][ct][3]};
      *reinterpret_cast<v4f*>(a.y + o) = v4f{ys[rt][ct][0], ys[rt][ct][1], ys[rt][ct][2], ys[rt][ct][3]};
      *reinterpret_cast<v4f*>(a.p + o) = v4f{ps[rt][ct][0], ps[rt][ct][1], ps[rt][ct][2], ps[rt][ct][3]};
    }
}

template <int FORM, bool DISC, bool TANG = false, bool LJ = false>
__global__ void __launch_bounds__(kThreads, 1) k_steps(StepArgs a) {
  __shared__ int s_flag;
  __shared__ int s_local;
  // LJ: the workgroup's 64 rows of J in LDS, 64 np bytes (int8, FIX16) or 32 np (FP4, FP8)
  extern __shared__ __attribute__((aligned(16))) uint8_t lds_j[];
  const int gg = grid_groups(a);
  if ((int)(blockIdx.x % gg) >= a.groups) return;  // a padding workgroup (see StepArgs::gpad)
  steps_tile<FORM, DISC, TANG, 64, LJ>(a, (int)(blockIdx.x % gg), (int)(blockIdx.x / gg), s_flag,
                                       s_local, LJ ? lds_j : nullptr,
                                       LJ ? (FORM == kFormFIX16 ? 64 : 32) * a.np : 0);
}

// ---------------------------------------------------------------------------------------
// Batched instances in one persistent launch.  Batch processing (Sec. VI) runs several
// problems side by side; here the problems may differ in size.  Every replica group of
// every instance is a gang of nb = np / BM workgroups that must run together and meet
// at every step's barrier.  The gangs wait in queues: one per XCD, which the host fills
// so that each carries about the same work, and one spanning the device.  A workgroup
// takes the next slot of its queue (an atomic counter), runs that tile for all steps,
// then takes the next; a gang starts when all of its slots are taken.  Slots are taken
// in queue order and no gang waits on a later one, so a queue drains whenever each of
// its gangs fits in the workgroups serving it.  The host sizes the XCD queues for a grid
// spread evenly over the XCDs (round-robin dispatch); the kernel counts the workgroups
// on each XCD at start-up and, if any queue lacks workers, every workgroup serves the
// device-wide queue instead (whose gangs all fit in the grid).
// ---------------------------------------------------------------------------------------
// Table entries are read with vector loads (the tables are not provably read-only), so
// the compiler takes every field as per-lane; the fields are the same in all lanes, and
// reading them through readfirstlane keeps arguments, descriptors and branches scalar.
__device__ __forceinline__ int ufirst(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float ufirst(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ uint64_t ufirst64(uint64_t v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
// Every pointer of the table points to device memory.  Rebuilt from an integer, a pointer
// is generic to the compiler, and generic (flat) accesses count against the LDS counter as
// well as the memory counter and may complete out of order with other memory accesses, so
// every wait for one drains all outstanding loads; a global-address-space pointer cast to
// a generic one lets the compiler's address-space inference make them global accesses.
template <class T>
__device__ __forceinline__ T* ufirst(T* p) {
  typedef __attribute__((address_space(1))) T GT;
  GT* g = (GT*)ufirst64(reinterpret_cast<uint64_t>(p));
  return (T*)g;
}

__device__ __forceinline__ StepArgs uniform_args(const StepArgs& a) {
  StepArgs u;
  u.n = ufirst(a.n); u.np = ufirst(a.np); u.rp = ufirst(a.rp); u.groups = ufirst(a.groups); u.nb = ufirst(a.nb);
  u.discrete = ufirst(a.discrete); u.m_begin = ufirst(a.m_begin); u.m_end = ufirst(a.m_end);
  u.A = ufirst(a.A); u.dt = ufirst(a.dt); u.cdt = ufirst(a.cdt);
  u.acol = ufirst(a.acol); u.rtab = ufirst(a.rtab); u.jf = ufirst(a.jf); u.q = ufirst(a.q);
  u.q_buf_bytes = (size_t)ufirst64(a.q_buf_bytes);
  u.x = ufirst(a.x); u.y = ufirst(a.y); u.p = ufirst(a.p);
  u.sync = ufirst(a.sync); u.status = ufirst(a.status);
  u.tape = ufirst(a.tape); u.tape_arr = (size_t)ufirst64(a.tape_arr);
  return u;
}

// OCC workgroups per CU: with 2, one workgroup's update and barrier overlap the other's
// K loop; registers then allow a Q prefetch depth of 2 and LDS half as many J rows.
template <bool DISC, int OCC>
__global__ void __launch_bounds__(kThreads, OCC) k_steps_batch(BatchArgs b) {
  constexpr int QD = OCC == 1 ? kKStepsUnroll : kKStepsUnroll / 2;
  __shared__ int s_flag;
  __shared__ int s_local;
  __shared__ int s_slot;
  extern __shared__ __attribute__((aligned(16))) uint8_t lds_dyn[];  // b.lds_bytes: J rows of the current tile
  const int tid = threadIdx.x;
  unsigned* workers = b.ctl + 160;  // [kBatchXcds + 1]: per XCD, then any other XCC id
  unsigned* arrived = b.ctl + 192;
  if (tid == 0) {
    const unsigned xcc = (unsigned)__builtin_amdgcn_s_getreg(kHwRegXccId) & 15u;
    const unsigned mine = xcc < (unsigned)kBatchXcds ? xcc : (unsigned)kBatchXcds;
    __hip_atomic_fetch_add(workers + mine, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(arrived, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int dom = kBatchXcds;
    unsigned spins = 0;
    while (ld_dev(arrived) < (unsigned)b.grid) {
      if (++spins > kSpinLimit) { st_dev(b.status, 2u); dom = -1; break; }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (dom >= 0) {
      bool per_xcd = mine < (unsigned)kBatchXcds && ld_dev(workers + kBatchXcds) == 0u;
      for (int d = 0; d < kBatchXcds; ++d) per_xcd = per_xcd && ld_dev(workers + d) >= (unsigned)b.need[d];
      dom = per_xcd ? (int)mine : kBatchXcds;
    }
    s_slot = dom;
  }
  __syncthreads();
  // values read from LDS are per-lane to the compiler: make them uniform (scalar), so the
  // tile's arguments, buffer descriptors and branches stay scalar
  const int dom = __builtin_amdgcn_readfirstlane(s_slot);
  __syncthreads();
  if (dom < 0) return;
  const int q0 = b.qoff[dom], q1 = b.qoff[dom + 1];
  unsigned* qctr = b.ctl + 16 * dom;
  for (;;) {
    if (tid == 0) {
      const int k = (int)__hip_atomic_fetch_add(qctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_slot = k < q1 - q0 ? q0 + k : -1;
    }
    __syncthreads();
    const int slot = __builtin_amdgcn_readfirstlane(s_slot);
    __syncthreads();
    if (slot < 0) break;
    const BatchSlot tv = b.slots[slot];
    const BatchSlot t{ufirst(tv.inst), ufirst(tv.g), ufirst(tv.mb), ufirst(tv.bm)};
    const StepArgs a = uniform_args(b.inst[t.inst]);
    if (b.clk && tid == 0) b.clk[2 * slot] = wall_clock64();
    if (t.bm == 64)
      steps_tile<kFormFP8, DISC, false, 64, true, QD>(a, t.g, t.mb, s_flag, s_local, lds_dyn, b.lds_bytes);
    else if (t.bm == 128)
      steps_tile<kFormFP8, DISC, false, 128, true, QD>(a, t.g, t.mb, s_flag, s_local, lds_dyn, b.lds_bytes);
    else
      steps_tile<kFormFP8, DISC, false, 256, true, QD>(a, t.g, t.mb, s_flag, s_local, lds_dyn, b.lds_bytes);
    __syncthreads();  // the next tile overwrites the LDS copy of J
    if (b.clk && tid == 0) b.clk[2 * slot + 1] = wall_clock64();
  }
}

// ---------------------------------------------------------------------------------------
// Reverse pass (vector-Jacobian product) of the binary32 dynamics, bSB / GbSB.
//
// Same tiling and barrier as k_steps.  The registers hold the cotangents (xb, yb, pb) of
// the wave's 64 x 32 elements; a.x, a.y, a.p bring them in (cotangents of the state
// after the last step) and take them out (of the state before the first).  tape entry s
// (0 <= s <= steps) holds x, y, p at the input of step m_begin + s, entry `steps` the
// state after the last step.  Step s, from the last one down (J symmetric, so the
// transposed product is the same GEMM), with k the step's wall mask (the next state has
// |x| = 1 and y = 0), f = 1 - A x^2, r = r_m and p' the next state's p:
//   w   = (1 - k) (yb + dt xb)          -- the product operand, G = J w
//   pb' = pb - dt x w
//   xb  = (1 - k) xb - dt p' w + c dt G + 2 A x p r pb'
//   yb  = w,   pb = pb' (1 - f r).
// This is the transpose of the forward derivative of eqs. (7), (3), (4), (5).
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads, 1) k_adjoint(StepArgs a) {
  __shared__ int s_flag;
  __shared__ int s_local;
  constexpr int BM = tile_rows_kind(kKindGeneric);
  constexpr int BN = tile_cols_kind(kKindGeneric);
  constexpr int WCOLS = BN / kWaveCols;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x % a.groups;
  const int mb = blockIdx.x / a.groups;
  const int wrow = wave / WCOLS;
  const int row0 = mb * BM + wrow * kWaveRows;
  const int col0 = g * BN + (wave % WCOLS) * kWaveCols;
  const int nks = a.np / kKS;
  unsigned* ctr = a.sync + (size_t)g * 64;
  unsigned* hs = a.sync + (size_t)(a.groups + g) * 64;
  unsigned* msk = a.sync + (size_t)(2 * a.groups + g) * 64;
  unsigned* abort_flag = a.sync + (size_t)(3 * a.groups) * 64;
  const uint8_t* jrows = static_cast<const uint8_t*>(a.jf) + (size_t)(mb * BM / 16 + 4 * wrow) * nks * 8192;
  auto off = [&](int rt, int ct) {
    return (size_t)(col0 + ct * 16 + (lane & 15)) * a.np + row0 + rt * 16 + 4 * (lane >> 4);
  };
  auto tape = [&](int s, int k, int rt, int ct) {
    return *reinterpret_cast<const v4f*>(a.tape + (size_t)(3 * s + k) * a.tape_arr + off(rt, ct));
  };

  float xb[4][2][4], yb[4][2][4], pb[4][2][4], w[4][2][4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const v4f vx = *reinterpret_cast<const v4f*>(a.x + off(rt, ct));
      const v4f vy = *reinterpret_cast<const v4f*>(a.y + off(rt, ct));
      const v4f vp = *reinterpret_cast<const v4f*>(a.p + off(rt, ct));
#pragma unroll
      for (int v = 0; v < 4; ++v) { xb[rt][ct][v] = vx[v]; yb[rt][ct][v] = vy[v]; pb[rt][ct][v] = vp[v]; }
    }

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
  const float A = a.A, dt = a.dt, cdt = a.cdt;
  const int steps = a.m_end - a.m_begin;

  // w of step s from the current cotangents and the state after step s, published as
  // the product operand in ping-pong buffer `buf`
  auto publish_w = [&](int s, int buf) {
    uint8_t* q = a.q + (size_t)buf * a.q_buf_bytes;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        const v4f xn = tape(s + 1, 0, rt, ct), yn = tape(s + 1, 1, rt, ct);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool k = __builtin_fabsf(xn[v]) == 1.0f && yn[v] == 0.0f;
          w[rt][ct][v] = k ? 0.0f : yb[rt][ct][v] + dt * xb[rt][ct][v];
        }
        store_operand<kFormFP32, false>(q, a.q_buf_bytes, nks, row0 + rt * 16, col0 + ct * 16, lane, w[rt][ct]);
      }
  };

  if (alive && steps > 0) {
    publish_w(steps - 1, 0);
    alive = group_sync(ctr, (unsigned)a.nb, local, abort_flag, a.status, &s_flag);
  }
  for (int it = 0; alive && it < steps; ++it) {
    const int s = steps - 1 - it;
    const uint8_t* qcur = a.q + (size_t)(it & 1) * a.q_buf_bytes;
    const __amdgpu_buffer_rsrc_t qr = make_rsrc(qcur, a.q_buf_bytes);
    v4f acc[4][2];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    gemm_tile_fp32(jrows, qr, col0 >> 4, nks, lane, acc);
    const float rm = a.rtab[a.m_begin + s];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        const v4f x = tape(s, 0, rt, ct), p = tape(s, 2, rt, ct), xn = tape(s + 1, 0, rt, ct);
        const v4f yn = tape(s + 1, 1, rt, ct), pn = tape(s + 1, 2, rt, ct);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool k = __builtin_fabsf(xn[v]) == 1.0f && yn[v] == 0.0f;
          const float wv = w[rt][ct][v];
          const float f = 1.0f - A * (x[v] * x[v]);
          const float pbn = pb[rt][ct][v] - (dt * x[v]) * wv;
          const float ctl = (((2.0f * A) * x[v]) * p[v]) * rm;
          const float xk = k ? 0.0f : xb[rt][ct][v];
          xb[rt][ct][v] = ((xk - (dt * pn[v]) * wv) + cdt * acc[rt][ct][v]) + ctl * pbn;
          yb[rt][ct][v] = wv;
          pb[rt][ct][v] = pbn * (1.0f - f * rm);
        }
      }
    if (s > 0) {
      publish_w(s - 1, (it + 1) & 1);
      alive = group_sync(ctr, (unsigned)((it + 2) * a.nb), local, abort_flag, a.status, &s_flag);
    }
  }

#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      *reinterpret_cast<v4f*>(a.x + off(rt, ct)) = v4f{xb[rt][ct][0], xb[rt][ct][1], xb[rt][ct][2], xb[rt][ct][3]};
      *reinterpret_cast<v4f*>(a.y + off(rt, ct)) = v4f{yb[rt][ct][0], yb[rt][ct][1], yb[rt][ct][2], yb[rt][ct][3]};
      *reinterpret_cast<v4f*>(a.p + off(rt, ct)) = v4f{pb[rt][ct][0], pb[rt][ct][1], pb[rt][ct][2], pb[rt][ct][3]};
    }
}

// ---------------------------------------------------------------------------------------
// Small kernels.
// ---------------------------------------------------------------------------------------
__global__ void k_fill_u32(unsigned* p, size_t count, unsigned v) {
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (size_t)gridDim.x * blockDim.x)
    p[t] = v;
}

// Validity of a caller's state on the device (the checks gsb_set_state makes on the host):
// bit 0 of *flag for a non-finite entry of x, y or p, bit 1 for |x| > 1 (eq. (5) keeps
// |x| <= 1).  One atomic per wave that found something.
__global__ void k_check_state(const float* x, const float* y, const float* p, size_t count, unsigned* flag) {
  unsigned bad = 0;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (size_t)gridDim.x * blockDim.x) {
    const float xv = x[t], yv = y[t], pv = p[t];
    if (!__builtin_isfinite(xv) || !__builtin_isfinite(yv) || !__builtin_isfinite(pv)) bad |= 1u;
    else if (__builtin_fabsf(xv) > 1.0f) bad |= 2u;
  }
  const unsigned long long any1 = __builtin_amdgcn_ballot_w64((bad & 1u) != 0);
  const unsigned long long any2 = __builtin_amdgcn_ballot_w64((bad & 2u) != 0);
  if ((any1 | any2) != 0 && (threadIdx.x & 63) == 0)
    __hip_atomic_fetch_or(flag, (any1 ? 1u : 0u) | (any2 ? 2u : 0u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Schedule table r_m = 1 / (M - m) of eqs. (6), (7), the binary64 quotient rounded to
// binary32 once (the same bits as the host table: both divisions are correctly rounded);
// all zero for the constant schedule.
__global__ void k_rtab(float* rtab, int steps, int linear) {
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < steps; m += gridDim.x * blockDim.x)
    rtab[m] = linear ? (float)(1.0 / (double)(steps - m)) : 0.0f;
}

// J (row-major np x np binary32, zero padded) -> fragment-major layout of `FORM`.
template <int FORM>
__global__ void k_encode_j(const float* j32, int np, uint8_t* jf) {
  const size_t total = (size_t)np * np;
  const int nks = np / kKS;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(t / np), k = (int)(t % np);
    const float v = j32[t];
    const int rt = i >> 4, kc = k >> 7, kk = k & 127;
    if constexpr (FORM == kFormFP8) {  // E4M3 J: the operand's placement, row i for replica r
      jf[fp8_elem_offset(nks, i, k)] = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xFF);
    } else if constexpr (FORM == kFormFIX16) {  // int8 J (entries in {0, +-1}), 32x32x32 A layout
      const int lanep = (i & 31) + 32 * ((kk & 31) >> 4);
      const size_t off = ((size_t)((i >> 5) * nks + kc) * 4 + (kk >> 5)) * 1024 + lanep * 16 + (kk & 15);
      jf[off] = (uint8_t)(int8_t)(int)v;
    } else if constexpr (FORM == kFormBF16X2) {  // bf16 J, 32x32x16 A layout
      const int lanep = (i & 31) + 32 * ((kk & 15) >> 3);
      const size_t off = ((size_t)((i >> 5) * nks + kc) * 8 + (kk >> 4)) * 1024 + lanep * 16 + (kk & 7) * 2;
      *reinterpret_cast<__bf16*>(jf + off) = (__bf16)v;
    } else {
      const int lanep = (i & 15) + 16 * ((kk & 15) >> 2);
      const size_t off = ((size_t)(rt * nks + kc) * 8 + (kk >> 4)) * 1024 + lanep * 16 + (kk & 3) * 4;
      *reinterpret_cast<float*>(jf + off) = v;
    }
  }
}

__global__ void k_encode_j4(const float* j32, int np, uint8_t* jf) {
  const size_t total = (size_t)np * np / 2;
  const int nks = np / kKS;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const size_t blk = t >> 10;
    const int lane = (int)((t >> 4) & 63), b = (int)(t & 15);
    const int rt = (int)(blk / nks), kc = (int)(blk % nks);
    const int i = rt * 16 + (lane & 15);
    const int p0 = 32 * (lane >> 4) + 2 * b;
    const float v0 = j32[(size_t)i * np + kc * kKS + fp4_pair_kk(p0)];
    const float v1 = j32[(size_t)i * np + kc * kKS + fp4_pair_kk(p0 + 1)];
    jf[t] = (uint8_t)(fp4_code(v0) | (fp4_code(v1) << 4));
  }
}

// x (count binary32 values) -> the operand encoding of FORM, value-major planes:
//   FP8    : count E4M3 bytes
//   BF16X2 : count bf16 hi, then count bf16 lo
//   FIX16  : count int8 hi, then count int8 lo (rint(x 2^14) = 256 hi + lo)
//   FP32   : count binary32 values
// Four values per thread through the encoders of the step kernels' operand stores; the
// values past `count` in the last group are zeros and are not stored.
template <int FORM, bool DISC>
__global__ void k_encode_operand(const float* x, size_t count, uint8_t* out) {
  const size_t groups = (count + 3) / 4;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < groups; t += (size_t)gridDim.x * blockDim.x) {
    const size_t e0 = 4 * t;
    const int nv = count - e0 >= 4 ? 4 : (int)(count - e0);
    float xv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) xv[v] = v < nv ? x[e0 + v] : 0.0f;
    if constexpr (FORM == kFormFP8) {
      const unsigned w = encode_fp8x4<DISC>(xv);
      for (int v = 0; v < nv; ++v) out[e0 + v] = (uint8_t)(w >> (8 * v));
    } else if constexpr (FORM == kFormBF16X2) {
      v2u wh, wl;
      encode_bf16x4<DISC>(xv, wh, wl);
      unsigned short* hi = reinterpret_cast<unsigned short*>(out);
      unsigned short* lo = hi + count;
      for (int v = 0; v < nv; ++v) {
        hi[e0 + v] = (unsigned short)(wh[v >> 1] >> (16 * (v & 1)));
        lo[e0 + v] = (unsigned short)(wl[v >> 1] >> (16 * (v & 1)));
      }
    } else if constexpr (FORM == kFormFIX16) {
      unsigned wh, wl;
      encode_fix16x4<DISC>(xv, wh, wl);
      for (int v = 0; v < nv; ++v) {
        out[e0 + v] = (uint8_t)(wh >> (8 * v));
        out[count + e0 + v] = (uint8_t)(wl >> (8 * v));
      }
    } else {
      float* q = reinterpret_cast<float*>(out);
      for (int v = 0; v < nv; ++v) q[e0 + v] = operand_value(xv[v], DISC);
    }
  }
}

// SplitMix64 (Steele, Lea, Flood 2014): output k (k >= 1) of the generator seeded with s
// is mix(s + k * 0x9E3779B97F4A7C15).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ float uniform_pm01(uint64_t z) {
  const double u = (double)(z >> 11) * 0x1.0p-53;  // [0, 1)
  const double t = 0.2 * u;
  return (float)(-0.1 + t);                          // U(-0.1, 0.1), App. A
}

// Initial state: counter (2 r + stream) n + i, draw number counter + 1.
// Starting x, y of spin i < n of replica r.  Draw counter (2 r + s) n + i for stream s.
//   mode 0: x ~ U(-0.1, 0.1), y = 0 (App. A);  mode 1: x, y ~ U(-0.1, 0.1);
//   mode 2: x = +-0.1, y = 0 (Sec. IV);
//   mode 3: the trajectory pairs of Sec. IV: replica 2k starts at x1 = +-0.1 (counter
//           (2k) n + i), replica 2k + 1 at x1 +- 2e-6 (sign from counter (2k + 1) n + i),
//           evaluated in binary64 and rounded once; y = 0.
__device__ __forceinline__ void init_elem(int n, int r, int i, uint64_t seed, int mode, float& xv, float& yv) {
  yv = 0.0f;
  if (mode == 3) {
    const int k = r >> 1;
    const uint64_t c0 = (uint64_t)(2 * (int64_t)k) * (uint64_t)n + (uint64_t)i;
    const float x1 = (splitmix64(seed, c0 + 1) >> 63) ? -0.1f : 0.1f;
    if (r & 1) {
      const double d = (splitmix64(seed, c0 + (uint64_t)n + 1) >> 63) ? -2e-6 : 2e-6;
      xv = (float)((double)x1 + d);
    } else {
      xv = x1;
    }
    return;
  }
  const uint64_t c0 = (uint64_t)(2 * (int64_t)r) * (uint64_t)n + (uint64_t)i;
  const uint64_t z0 = splitmix64(seed, c0 + 1);
  if (mode == 2) {
    xv = (z0 >> 63) ? -0.1f : 0.1f;  // the chaos start of Sec. IV
  } else {
    xv = uniform_pm01(z0);
    if (mode == 1) yv = uniform_pm01(splitmix64(seed, c0 + (uint64_t)n + 1));
  }
}

__global__ void k_init_state(int n, int np, int rp, uint64_t seed, int mode, float* x, float* y, float* p) {
  const size_t total = (size_t)rp * np;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(t / np), i = (int)(t % np);
    float xv = 0.0f, yv = 0.0f;
    if (i < n) init_elem(n, r, i, seed, mode, xv, yv);
    x[t] = xv;
    y[t] = yv;
    p[t] = 1.0f;  // p_i(0) = 1
  }
}

// Starting state of every instance of a batch (blockIdx.y = instance), as k_init_state.
__global__ void k_init_batch(const StepArgs* inst, const BatchInst* bi, int mode) {
  const StepArgs& a = inst[blockIdx.y];
  const int n = a.n, np = a.np;
  const uint64_t seed = bi[blockIdx.y].seed;
  const size_t total = (size_t)a.rp * np;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(t / np), i = (int)(t % np);
    float xv = 0.0f, yv = 0.0f;
    if (i < n) init_elem(n, r, i, seed, mode, xv, yv);
    a.x[t] = xv;
    a.y[t] = yv;
    a.p[t] = 1.0f;
  }
}

// Tangent-mode layout (2 rp columns, blocks of 32: 16 replicas, then their tangents).
// Replica r starts as k_init_state would start it; its tangent is dx_i = +-1 (bit 63 of
// draw r n + i + 1 of `tseed`), dy = dp = 0, to be scaled to unit norm.
__global__ void k_init_tangent(int n, int np, int rp, uint64_t seed, int mode, uint64_t tseed, float* x, float* y,
                               float* p) {
  const size_t total = (size_t)2 * rp * np;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(t / np), i = (int)(t % np);
    const int r = (col >> 5) * 16 + (col & 15);
    float xv = 0.0f, yv = 0.0f, pv = 1.0f;
    if ((col & 31) < 16) {
      if (i < n) init_elem(n, r, i, seed, mode, xv, yv);
    } else {
      pv = 0.0f;
      if (i < n) xv = (splitmix64(tseed, (uint64_t)r * (uint64_t)n + (uint64_t)i + 1) >> 63) ? -1.0f : 1.0f;
    }
    x[t] = xv;
    y[t] = yv;
    p[t] = pv;
  }
}

// Scale each replica's tangent (dx, dy, dp over spins < n) to unit norm; with
// `accumulate`, add ln of the norm it had to lg[r] (binary64, fixed summation order).
__global__ void __launch_bounds__(256) k_tangent_renorm(int n, int np, float* x, float* y, float* p, double* lg,
                                                        int accumulate) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  const size_t o = (size_t)((r >> 4) * 32 + 16 + (r & 15)) * np;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double a = x[o + i], b = y[o + i], c = p[o + i];
    s += (a * a + b * b) + c * c;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  s = ((red[0] + red[1]) + red[2]) + red[3];
  if (s > 0.0) {
    if (accumulate && threadIdx.x == 0) lg[r] += 0.5 * log(s);
    const float k = (float)(1.0 / sqrt(s));
    for (int i = threadIdx.x; i < n; i += 256) {
      x[o + i] *= k;
      y[o + i] *= k;
      p[o + i] *= k;
    }
  } else if (accumulate && threadIdx.x == 0) {
    lg[r] = -INFINITY;  // every component reached a wall: the tangent vanished
  }
}

// Tangent-mode state -> [6][R][n] (x, y, p, dx, dy, dp).
__global__ void k_tangent_extract(int n, int np, int R, const float* x, const float* y, const float* p, float* out) {
  const size_t total = (size_t)R * n;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(t / n), i = (int)(t % n);
    const size_t op = (size_t)((r >> 4) * 32 + (r & 15)) * np + i, ot = op + (size_t)16 * np;
    out[t] = x[op];
    out[total + t] = y[op];
    out[2 * total + t] = p[op];
    out[3 * total + t] = x[ot];
    out[4 * total + t] = y[ot];
    out[5 * total + t] = p[ot];
  }
}

// Normalised distance of the trajectory pairs (replicas 2k, 2k + 1) over spins < n, eq. (8).
__global__ void __launch_bounds__(256) k_delta(int n, int np, const float* x, double* out) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  const float* a = x + (size_t)(2 * k) * np;
  const float* b = a + np;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double d = (double)a[i] - (double)b[i];
    s += d * d;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[k] = sqrt((((red[0] + red[1]) + red[2]) + red[3]) / (4.0 * n));
}

// Energy, eq. (1): E_r = -1/2 sum_i s_i h_i with h_i = sum_j J_ij s_j, s = sgn(x).
// Block (bx, by): replicas 16 bx .. 16 bx + 15, rows i = 256 by + threadIdx.x.  J is read
// as J_ji (= J_ij) so a wavefront's loads are contiguous.  Partial sums per row block
// are reduced in a fixed order (deterministic, exact for integer J).
constexpr int kERep = 16;
constexpr int kEChunk = 2048;
__global__ void __launch_bounds__(256) k_energy_partial(const float* j32, int n, int np, int rp,
                                                        const float* x, double* partial) {
  __shared__ int8_t s[kERep][kEChunk];
  __shared__ double red[4][kERep];
  const int i = blockIdx.y * 256 + threadIdx.x;
  const int r0 = blockIdx.x * kERep;
  double h[kERep];
#pragma unroll
  for (int rr = 0; rr < kERep; ++rr) h[rr] = 0.0;
  for (int j0 = 0; j0 < n; j0 += kEChunk) {
    const int jn = min(kEChunk, n - j0);
    __syncthreads();
    for (int t = threadIdx.x; t < kERep * kEChunk; t += 256) {
      const int rr = t / kEChunk, jj = t % kEChunk;
      s[rr][jj] = (jj < jn) ? (x[(size_t)(r0 + rr) * np + j0 + jj] >= 0.0f ? 1 : -1) : 0;
    }
    __syncthreads();
    if (i < n) {
      for (int jj = 0; jj < jn; ++jj) {
        const double jv = (double)j32[(size_t)(j0 + jj) * np + i];
#pragma unroll
        for (int rr = 0; rr < kERep; ++rr) h[rr] += jv * (double)s[rr][jj];
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int rr = 0; rr < kERep; ++rr) {
    double v = 0.0;
    if (i < n) v = (x[(size_t)(r0 + rr) * np + i] >= 0.0f) ? h[rr] : -h[rr];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wave][rr] = v;
  }
  __syncthreads();
  if (threadIdx.x < kERep) {
    const int rr = threadIdx.x;
    partial[(size_t)blockIdx.y * rp + r0 + rr] = ((red[0][rr] + red[1][rr]) + red[2][rr]) + red[3][rr];
  }
}

__global__ void k_energy_final(const double* partial, int nyb, int rp, int r_count, double* E) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= r_count) return;
  double acc = 0.0;
  for (int b = 0; b < nyb; ++b) acc += partial[(size_t)b * rp + r];
  E[r] = -0.5 * acc;
}

// Exact energies on MFMA for J in {0, +-1} (eq. (1)): E_r = -1/2 sum_i s_i (J s)_i with
// s = sgn x.  The spins go into the FP8 operand layout of the step kernels (+-1 exactly),
// J is the FP4 copy of the register-resident path; every partial sum is an integer of
// magnitude below 2^24, so the binary32 accumulators are exact, and the per-replica
// totals are integer atomics, hence independent of order.
__device__ __forceinline__ void sign_fp8_elems(const float* x, int np, int nks, int rp, uint8_t* s8, size_t t0,
                                               size_t stride) {
  const size_t quads = (size_t)rp * np / 4;
  for (size_t t = t0; t < quads; t += stride) {
    const int r = (int)((t * 4) / np), k = (int)((t * 4) % np);
    const v4f v = *reinterpret_cast<const v4f*>(x + (size_t)r * np + k);
    const float xv[4] = {v[0], v[1], v[2], v[3]};
    // spins k..k+3 (k a multiple of 4) are four consecutive bytes of the placement
    *reinterpret_cast<unsigned*>(s8 + fp8_elem_offset(nks, r, k)) = encode_fp8x4<true>(xv);
  }
}

__global__ void k_sign_fp8(const float* x, int np, int nks, int rp, uint8_t* s8) {
  sign_fp8_elems(x, np, nks, rp, s8, (size_t)blockIdx.x * blockDim.x + threadIdx.x, (size_t)gridDim.x * blockDim.x);
}

// Workgroup (cg, mb): spins [256 mb, +256) (64 per wave, 4 row tiles) x replicas
// [32 cg, +32) (2 column tiles).  G = J S over all k-steps, then sum_i s_i G_ir.
__device__ __forceinline__ void energy_tile(const uint8_t* jf4, const uint8_t* s8, const float* x, int np, int nks,
                                            int* eacc, int cg, int mb) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = mb * 256 + wave * 64;
  v4f acc[4][2];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  for (int ks = 0; ks < nks; ++ks) {
    v4i a[4];
    v8i b[2];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
      a[rt] = *reinterpret_cast<const v4i*>(jf4 + ((size_t)((row0 >> 4) + rt) * nks + ks) * 1024 + lane * 16);
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const uint8_t* f = s8 + ((size_t)(2 * cg + ct) * nks + ks) * 2048 + lane * 16;
      b[ct] = cat(*reinterpret_cast<const v4i*>(f), *reinterpret_cast<const v4i*>(f + 1024));
    }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
        acc[rt][ct] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(cat(a[rt], a[rt]), b[ct], acc[rt][ct], 4, 0, 0,
                                                                       127, 0, 127);
  }
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int r = 32 * cg + 16 * ct + (lane & 15);
    float part = 0.0f;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const v4f xv = *reinterpret_cast<const v4f*>(x + (size_t)r * np + row0 + rt * 16 + 4 * (lane >> 4));
#pragma unroll
      for (int v = 0; v < 4; ++v) part += xv[v] < 0.0f ? -acc[rt][ct][v] : acc[rt][ct][v];
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (lane < 16) atomicAdd(eacc + r, (int)part);
  }
}

__global__ void __launch_bounds__(256) k_energy_mfma(const uint8_t* jf4, const uint8_t* s8, const float* x, int np,
                                                     int nks, int* eacc) {
  energy_tile(jf4, s8, x, np, nks, eacc, blockIdx.x, blockIdx.y);
}

__global__ void k_energy_final_int(const int* eacc, int r_count, double* E) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < r_count) E[r] = -0.5 * (double)eacc[r];
}

// argmin_r E_r, ties to the lowest r (one workgroup of 256 threads): a strided scan per
// thread, then a butterfly over the wavefront's 64 lanes with cross-lane shuffles (every
// lane ends with the wave's minimum), and the four waves' results through LDS.  The
// order (e, r) is total, so the result does not depend on the reduction order.
__device__ __forceinline__ bool before_in_order(double e1, int i1, double e2, int i2) {
  return e1 < e2 || (e1 == e2 && i1 < i2);
}
__device__ __forceinline__ void best_of(const double* E, int r_count, int* best_idx, double* best_e, double* se,
                                        int* si) {
  double be = __builtin_inf();
  int bi = 0x7FFFFFFF;
  for (int r = threadIdx.x; r < r_count; r += 256) {
    const double e = E[r];
    if (before_in_order(e, r, be, bi)) { be = e; bi = r; }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double e2 = __shfl_xor(be, off, 64);
    const int i2 = __shfl_xor(bi, off, 64);
    if (before_in_order(e2, i2, be, bi)) { be = e2; bi = i2; }
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { se[wave] = be; si[wave] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < 4; ++w)
      if (before_in_order(se[w], si[w], be, bi)) { be = se[w]; bi = si[w]; }
    *best_idx = bi;
    *best_e = be;
  }
}

__global__ void __launch_bounds__(256) k_best(const double* E, int r_count, int* best_idx, double* best_e) {
  __shared__ double se[4];
  __shared__ int si[4];
  best_of(E, r_count, best_idx, best_e, se, si);
}

// Energies and best replica of every instance of a batch (the instance is the last grid
// dimension), from the FP4 J each instance keeps for its FP8 product.
__global__ void k_sign_batch(const StepArgs* inst, const BatchInst* bi) {
  const StepArgs& a = inst[blockIdx.y];
  sign_fp8_elems(a.x, a.np, a.np / kKS, a.rp, bi[blockIdx.y].s8, (size_t)blockIdx.x * blockDim.x + threadIdx.x,
                 (size_t)gridDim.x * blockDim.x);
}

__global__ void __launch_bounds__(256) k_energy_batch(const StepArgs* inst, const BatchInst* bi) {
  const StepArgs& a = inst[blockIdx.z];
  if ((int)blockIdx.y >= a.np / 256 || (int)blockIdx.x >= a.rp / 32) return;
  const BatchInst& b = bi[blockIdx.z];
  energy_tile(static_cast<const uint8_t*>(a.jf), b.s8, a.x, a.np, a.np / kKS, b.eacc, blockIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(256) k_energy_best_batch(const BatchInst* bi, int r_count) {
  __shared__ double se[4];
  __shared__ int si[4];
  const BatchInst& b = bi[blockIdx.x];
  for (int r = threadIdx.x; r < r_count; r += 256) b.E[r] = -0.5 * (double)b.eacc[r];
  __syncthreads();
  best_of(b.E, r_count, b.best_idx, b.best_e, se, si);
}

// s = sgn(x) for replicas r_first .. r_first + r_count - 1 (or the single replica
// *r_index when given).  With an ancilla spin `anc` (>= 0) the configuration is flipped
// so that the ancilla reads +1.
__global__ void k_spins(const float* x, int n_out, int np, int r_first, int r_count, int anc,
                        const int* r_index, int8_t* spins) {
  const size_t total = (size_t)r_count * n_out;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(t / n_out), i = (int)(t % n_out);
    const int r = r_index ? *r_index : r_first + k;
    const float* xr = x + (size_t)r * np;
    const bool flip = anc >= 0 && xr[anc] < 0.0f;
    const bool up = xr[i] >= 0.0f;
    spins[t] = (up != flip) ? 1 : -1;
  }
}

inline int grid_for(size_t total, int block) {
  size_t g = (total + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

template <int FORM, bool DISC>
const void* steps_kernel() {
  return reinterpret_cast<const void*>(&k_steps<FORM, DISC>);
}

// The generic tile keeps its 64 rows of J in LDS when they fit beside the kernel's few
// static bytes: int8 J (FIX16, 64 np bytes) or FP4 J (FP8, 32 np bytes).
constexpr size_t kJLdsMax = 159 * 1024;
size_t steps_lds_bytes(int form, int kind, int np, bool discrete) {
  if (kind == kKindWaveSpec) return steps_ws_lds_bytes(np, discrete);
  if (kind != kKindGeneric) return 0;
  const size_t bytes = form == kFormFIX16 ? (size_t)64 * np : (form == kFormFP8 ? (size_t)32 * np : 0);
  return bytes <= kJLdsMax ? bytes : 0;
}

template <bool DISC>
const void* steps_kernel_disc(int form, int kind, int np) {
  if (kind == kKindRegJ) return steps_kernel_rj(np / kKS, DISC);
  if (kind == kKindWaveSpec) return steps_kernel_ws(np / kKS, DISC);
  switch (form) {
    case kFormFP8:
      return steps_lds_bytes(form, kind, np, DISC) ? reinterpret_cast<const void*>(&k_steps<kFormFP8, DISC, false, true>)
                                             : steps_kernel<kFormFP8, DISC>();
    case kFormBF16X2: return steps_kernel<kFormBF16X2, DISC>();
    case kFormFIX16:
      return steps_lds_bytes(form, kind, np, DISC) ? reinterpret_cast<const void*>(&k_steps<kFormFIX16, DISC, false, true>)
                                             : steps_kernel<kFormFIX16, DISC>();
    default: return steps_kernel<kFormFP32, DISC>();
  }
}

const void* steps_kernel_tangent() { return reinterpret_cast<const void*>(&k_steps<kFormFP32, false, true>); }

const void* steps_kernel_for(int form, int kind, int np, bool discrete) {
  return discrete ? steps_kernel_disc<true>(form, kind, np) : steps_kernel_disc<false>(form, kind, np);
}


}  // namespace

// ---------------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------------
hipError_t launch_fill_u32(unsigned* p, size_t count, unsigned v, hipStream_t stream) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, 256)), dim3(256), 0, stream, p, count, v);
  return hipGetLastError();
}

hipError_t launch_check_state(const float* x, const float* y, const float* p, size_t count, unsigned* flag,
                              hipStream_t stream) {
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, flag, (size_t)1, 0u);
  if (count == 0) return hipGetLastError();
  const int grid = std::min(grid_for(count, 256), 1024);
  hipLaunchKernelGGL(k_check_state, dim3(grid), dim3(256), 0, stream, x, y, p, count, flag);
  return hipGetLastError();
}

hipError_t launch_rtab(float* rtab, int steps, bool linear, hipStream_t stream) {
  hipLaunchKernelGGL(k_rtab, dim3(grid_for((size_t)steps, 256)), dim3(256), 0, stream, rtab, steps, linear ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_encode_j(int form, bool fp4, const float* j32, int np, void* jf, hipStream_t stream) {
  const size_t total = (size_t)np * np;
  const dim3 grid(grid_for(total, 256)), block(256);
  uint8_t* out = static_cast<uint8_t*>(jf);
  if (form == kFormFP8 && fp4)
    hipLaunchKernelGGL(k_encode_j4, dim3(grid_for(total / 2, 256)), block, 0, stream, j32, np, out);
  else if (form == kFormFP8) hipLaunchKernelGGL(k_encode_j<kFormFP8>, grid, block, 0, stream, j32, np, out);
  else if (form == kFormBF16X2) hipLaunchKernelGGL(k_encode_j<kFormBF16X2>, grid, block, 0, stream, j32, np, out);
  else if (form == kFormFIX16) hipLaunchKernelGGL(k_encode_j<kFormFIX16>, grid, block, 0, stream, j32, np, out);
  else hipLaunchKernelGGL(k_encode_j<kFormFP32>, grid, block, 0, stream, j32, np, out);
  return hipGetLastError();
}

hipError_t launch_encode_operand(int form, bool discrete, const float* x, size_t count, void* out,
                                 hipStream_t stream) {
  const dim3 grid(grid_for((count + 3) / 4, 256)), block(256);
  uint8_t* o = static_cast<uint8_t*>(out);
  if (form == kFormFP8 && discrete) hipLaunchKernelGGL((k_encode_operand<kFormFP8, true>), grid, block, 0, stream, x, count, o);
  else if (form == kFormFP8) hipLaunchKernelGGL((k_encode_operand<kFormFP8, false>), grid, block, 0, stream, x, count, o);
  else if (form == kFormBF16X2 && discrete) hipLaunchKernelGGL((k_encode_operand<kFormBF16X2, true>), grid, block, 0, stream, x, count, o);
  else if (form == kFormBF16X2) hipLaunchKernelGGL((k_encode_operand<kFormBF16X2, false>), grid, block, 0, stream, x, count, o);
  else if (form == kFormFIX16 && discrete) hipLaunchKernelGGL((k_encode_operand<kFormFIX16, true>), grid, block, 0, stream, x, count, o);
  else if (form == kFormFIX16) hipLaunchKernelGGL((k_encode_operand<kFormFIX16, false>), grid, block, 0, stream, x, count, o);
  else if (discrete) hipLaunchKernelGGL((k_encode_operand<kFormFP32, true>), grid, block, 0, stream, x, count, o);
  else hipLaunchKernelGGL((k_encode_operand<kFormFP32, false>), grid, block, 0, stream, x, count, o);
  return hipGetLastError();
}

hipError_t launch_init_state(int n, int np, int rp, uint64_t seed, int mode, float* x, float* y,
                             float* p, hipStream_t stream) {
  hipLaunchKernelGGL(k_init_state, dim3(grid_for((size_t)rp * np, 256)), dim3(256), 0, stream, n, np,
                     rp, seed, mode, x, y, p);
  return hipGetLastError();
}

int choose_kind(int form, int np, int pref) {
  if (form != kFormFP8 || np > 2048) return kKindGeneric;
  return pref == 1 ? kKindRegJ : kKindWaveSpec;
}

// Host-side facts that do not change while the process runs, looked up once: the dynamic
// LDS attribute of a step kernel on a device, and its co-resident workgroups.
namespace {
std::mutex g_host_cache_mu;
std::map<std::pair<int, const void*>, size_t> g_lds_attr;  // largest dynamic LDS set per kernel
std::map<std::tuple<int, int, int, int, bool>, int> g_coresident;

// The attribute is a maximum: it is raised when a launch needs more and never lowered, so
// one kernel launched with several LDS sizes (the generic tiles' J rows scale with n)
// keeps a setting that covers all of them.
hipError_t set_lds_attribute_once(const void* k, size_t lds) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_host_cache_mu);
  const auto key = std::make_pair(dev, k);
  const auto it = g_lds_attr.find(key);
  if (it != g_lds_attr.end() && it->second >= lds) return hipSuccess;
  e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) g_lds_attr[key] = lds;
  return e;
}
}  // namespace

static int coresident_uncached(int form, int kind, int np, bool tangent);

int max_coresident_workgroups(int form, int kind, int np, bool tangent) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  const auto key = std::make_tuple(dev, form, kind, np, tangent);
  {
    std::lock_guard<std::mutex> lock(g_host_cache_mu);
    const auto it = g_coresident.find(key);
    if (it != g_coresident.end()) return it->second;
  }
  const int v = coresident_uncached(form, kind, np, tangent);
  if (v > 0) {
    std::lock_guard<std::mutex> lock(g_host_cache_mu);
    g_coresident[key] = v;
  }
  return v;
}

static int coresident_uncached(int form, int kind, int np, bool tangent) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (tangent) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, steps_kernel_tangent(), kThreads, 0) != hipSuccess)
      return 0;
    return per_cu * cus;
  }
  int best = 0;
  for (int disc = 0; disc < 2; ++disc) {
    const void* k = steps_kernel_for(form, kind, np, disc != 0);
    if (!k) return 0;
    const size_t lds = steps_lds_bytes(form, kind, np, disc != 0);
    if (lds > 0 && set_lds_attribute_once(k, lds) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads_kind(kind), lds) != hipSuccess) return 0;
    best = disc == 0 ? per_cu * cus : std::min(best, per_cu * cus);
  }
  return best;
}

hipError_t launch_adjoint(const StepArgs& a, hipStream_t stream) {
  if (!a.tape) return hipErrorInvalidValue;
  StepArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_adjoint), dim3(a.groups * a.nb), dim3(kThreads),
                                    args, 0u, stream);
}

int max_coresident_adjoint() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_adjoint), kThreads, 0) !=
      hipSuccess)
    return 0;
  return per_cu * cus;
}

hipError_t launch_steps(int form, int kind, const StepArgs& a, hipStream_t stream, bool tangent) {
  if (tangent && (form != kFormFP32 || kind != kKindGeneric || a.discrete)) return hipErrorInvalidValue;
  const void* k = tangent ? steps_kernel_tangent() : steps_kernel_for(form, kind, a.np, a.discrete != 0);
  if (!k) return hipErrorInvalidValue;
  const size_t lds = steps_lds_bytes(form, kind, a.np, a.discrete != 0);
  if (lds > 0) {
    const hipError_t e = set_lds_attribute_once(k, lds);
    if (e != hipSuccess) return e;
  }
  StepArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(k, dim3(grid_groups(a) * a.nb), dim3(threads_kind(kind)), args, (unsigned)lds,
                                    stream);
}

hipError_t launch_init_tangent(int n, int np, int rp, uint64_t seed, int mode, uint64_t tseed, float* x, float* y,
                               float* p, hipStream_t stream) {
  hipLaunchKernelGGL(k_init_tangent, dim3(grid_for((size_t)2 * rp * np, 256)), dim3(256), 0, stream, n, np, rp, seed,
                     mode, tseed, x, y, p);
  return hipGetLastError();
}

hipError_t launch_tangent_renorm(int n, int np, int rp, float* x, float* y, float* p, double* lg, bool accumulate,
                                 hipStream_t stream) {
  hipLaunchKernelGGL(k_tangent_renorm, dim3(rp), dim3(256), 0, stream, n, np, x, y, p, lg, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_tangent_extract(int n, int np, int R, const float* x, const float* y, const float* p, float* out,
                                  hipStream_t stream) {
  hipLaunchKernelGGL(k_tangent_extract, dim3(grid_for((size_t)R * n, 256)), dim3(256), 0, stream, n, np, R, x, y, p,
                     out);
  return hipGetLastError();
}

hipError_t launch_delta(int n, int np, int pairs, const float* x, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_delta, dim3(pairs), dim3(256), 0, stream, n, np, x, out);
  return hipGetLastError();
}

size_t energy_partial_doubles(int np, int rp) { return (size_t)(np / 256 + 1) * rp; }

hipError_t launch_energy(const float* j32, int n, int np, int rp, int r_count, const float* x,
                         double* partial, double* energies, hipStream_t stream) {
  const int nyb = (n + 255) / 256;
  hipLaunchKernelGGL(k_energy_partial, dim3(rp / kERep, nyb), dim3(256), 0, stream, j32, n, np, rp, x, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_final, dim3((r_count + 255) / 256), dim3(256), 0, stream, partial, nyb, rp,
                     r_count, energies);
  return hipGetLastError();
}

size_t energy_fp4_scratch_bytes(int np, int rp) { return (size_t)rp * np + (size_t)rp * 4 + 256; }

hipError_t launch_energy_fp4(const void* jf4, int np, int rp, int r_count, const float* x, void* scratch,
                             double* energies, hipStream_t stream) {
  if (np % 256 != 0 || rp % 32 != 0) return hipErrorInvalidValue;
  const int nks = np / kKS;
  uint8_t* s8 = static_cast<uint8_t*>(scratch);
  int* eacc = reinterpret_cast<int*>(s8 + (size_t)rp * np);
  hipError_t e = launch_fill_u32(reinterpret_cast<unsigned*>(eacc), (size_t)rp, 0u, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sign_fp8, dim3(grid_for((size_t)rp * np / 4, 256)), dim3(256), 0, stream, x, np, nks, rp, s8);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_mfma, dim3(rp / 32, np / 256), dim3(256), 0, stream, static_cast<const uint8_t*>(jf4),
                     s8, x, np, nks, eacc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_final_int, dim3((r_count + 255) / 256), dim3(256), 0, stream, eacc, r_count, energies);
  return hipGetLastError();
}

hipError_t launch_best(const double* energies, int r_count, int* best_idx, double* best_e, hipStream_t stream) {
  hipLaunchKernelGGL(k_best, dim3(1), dim3(256), 0, stream, energies, r_count, best_idx, best_e);
  return hipGetLastError();
}

const void* batch_kernel(bool discrete, int occ) {
  if (occ == 2)
    return discrete ? reinterpret_cast<const void*>(&k_steps_batch<true, 2>)
                    : reinterpret_cast<const void*>(&k_steps_batch<false, 2>);
  return discrete ? reinterpret_cast<const void*>(&k_steps_batch<true, 1>)
                  : reinterpret_cast<const void*>(&k_steps_batch<false, 1>);
}

hipError_t launch_steps_batch(bool discrete, int occ, const BatchArgs& b, hipStream_t stream, bool cooperative) {
  const void* k = batch_kernel(discrete, occ);
  if (b.lds_bytes > 0) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, b.lds_bytes);
    if (e != hipSuccess) return e;
  }
  BatchArgs copy = b;
  void* args[] = {&copy};
  if (cooperative) return hipLaunchCooperativeKernel(k, dim3(b.grid), dim3(kThreads), args, (unsigned)b.lds_bytes, stream);
  return hipLaunchKernel(k, dim3(b.grid), dim3(kThreads), args, (size_t)b.lds_bytes, stream);
}

int batch_workgroups_per_cu(bool discrete, int occ, int lds_bytes) {
  const void* k = batch_kernel(discrete, occ);
  if (lds_bytes > 0 && hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes) != hipSuccess)
    return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kThreads, (size_t)lds_bytes) != hipSuccess) return 0;
  return per_cu;
}

hipError_t launch_init_batch(const StepArgs* inst, const BatchInst* bi, int count, int np_max, int rp, int mode,
                             hipStream_t stream) {
  const unsigned gx = (unsigned)std::min<size_t>(grid_for((size_t)rp * np_max, 256), 1024);
  hipLaunchKernelGGL(k_init_batch, dim3(gx, count), dim3(256), 0, stream, inst, bi, mode);
  return hipGetLastError();
}

hipError_t launch_energy_batch(const StepArgs* inst, const BatchInst* bi, int count, int np_max, int rp, int r_count,
                               hipStream_t stream) {
  if (np_max % 256 != 0 || rp % 32 != 0) return hipErrorInvalidValue;
  const unsigned gx = (unsigned)std::min<size_t>(grid_for((size_t)rp * np_max / 4, 256), 1024);
  hipLaunchKernelGGL(k_sign_batch, dim3(gx, count), dim3(256), 0, stream, inst, bi);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_batch, dim3(rp / 32, np_max / 256, count), dim3(256), 0, stream, inst, bi);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_best_batch, dim3(count), dim3(256), 0, stream, bi, r_count);
  return hipGetLastError();
}

hipError_t launch_spins(const float* x, int n_out, int np, int r_first, int r_count, int anc,
                        const int* r_index, int8_t* spins, hipStream_t stream) {
  hipLaunchKernelGGL(k_spins, dim3(grid_for((size_t)r_count * n_out, 256)), dim3(256), 0, stream, x, n_out,
                     np, r_first, r_count, anc, r_index, spins);
  return hipGetLastError();
}

}  // namespace gsb
