// gsb_steps_ws.hip -- the wave-specialised step kernel of libgsb (gfx950): FP8 product,
// J held as FP4 in the register files and LDS of the CUs for the whole launch
// (np <= 2048), with the product and the update of eqs. (3)-(7) in different waves.
//
// Same tile as the register-resident kernel: workgroup (g, mb) owns spins
// [256 mb, 256 mb + 256) of replicas [32 g, 32 g + 32), and row slice w (64 spins) of it
// belongs to SIMD w.  Each SIMD runs two waves of the workgroup:
//   - product wave w (waves 0-3): keeps its 64 rows of J (k-steps [0, NR) in registers,
//     the rest in LDS), runs the K loops of both 16-replica column tiles, alternately,
//     and leaves each 64 x 16 product in an LDS slot;
//   - update wave w (waves 4-7): takes the product from the slot, applies eqs. (7), (3),
//     (4), (5) in binary32 (one rounding per operator) and writes the next operand.
// The matrix cores and the vector ALU of a SIMD execute instructions of different waves
// at the same time, so the update of one column tile runs under the K loop of the other.
//
// Operand exchange.  The update waves write the operand in aligned 64-bit units, two
// words of one lane per store (the operand placement keeps a lane's rows together), and
// an aligned 64-bit store is seen whole or not at all.  The first word of every unit
// carries a tag of the step that wrote it, in bit 6 of its first byte (the E4M3 code of a
// value in [-1, 1] never sets that bit; the wall of eq. (5) keeps x there).  Operand k
// (k = 0 at the launch's first step) sits in buffer k % 2 with tag (k / 2) % 2, so a
// buffer holds either the operand a product wave wants or the one two steps older, whose
// tag differs.  Each product wave strips and checks the tagged word of every unit it
// loads and loads again while any is stale (the sign operand of dSB and GdSB carries the
// tag in every byte of every word and is not stripped: tagged, its bytes are +-256
// instead of +-1, which the MFMA's E8M0 block scale of 2^-8 undoes exactly), and no group
// counter is needed between steps.  The launch's first operand is behind the group counter (buffer 1 is cleared to
// the stale tag under the same counter).  Where the group spans XCDs, whose L2 caches are
// not coherent with each other, every step also goes through the group counter with
// agent-scope fences, and the product waves meet in LDS where one of them polls it.
#include "gsb_device.h"

#pragma clang fp contract(off)

namespace gsb {
namespace {

constexpr int kWsThreads = 512;
// k-steps of J per product wave in VGPRs; the rest sit in LDS.  The register budget of a
// wave at two waves per SIMD is 256 VGPRs and AGPRs together, shared by both roles (the
// compiler splits it evenly as soon as a kernel uses AGPRs), so all of it stays in VGPRs.
// The sign product hands its product over in f16 (integers of magnitude <= 2048, exact),
// which leaves the LDS room for one more k-step of J; the registers that frees hold one
// more operand fragment in flight (a second one made the J registers spill).
constexpr int ws_reg_ksteps(bool disc) { return disc ? 7 : 8; }
constexpr int ws_prefetch(bool disc) { return disc ? 6 : 5; }
// bytes of one product wave's slot: 4 row tiles x 64 lanes x 4 values (f16 or f32)
constexpr int ws_slot_bytes(bool disc) { return 4 * 64 * (disc ? 8 : 16); }
constexpr unsigned kLdsSpinLimit = 1u << 27;  // LDS polls before giving up (seconds)
constexpr int kPwAbandoned = -1000000;        // s_pw_go when the poller gave up

// Poll bookkeeping shared by the waits: false when the launch is being abandoned.
__device__ __forceinline__ bool keep_polling(unsigned spins, unsigned limit, unsigned* abort_flag,
                                             unsigned* status) {
  if ((spins & 255u) == 0 && ld_dev(abort_flag)) return false;
  if (spins > limit) {
    st_dev(abort_flag, 1u);
    st_dev(status, 1u);
    return false;
  }
  return true;
}

// c * h for the f16 h in the low (HI false) or high half of word hw, in one instruction:
// a fused multiply-add with addend -0.0 (the product of a binary32 and an f16 is exact
// before its one rounding, and x + -0.0 = x for every x, zeros included) gives the
// binary32 product c * (float)h bit for bit, without converting h first.  The compiler
// folds a written fmaf(c, h, -0.0f) into a multiply after the conversion, hence the asm
// (register operands only, no memory access).
template <bool HI>
__device__ __forceinline__ float mul_f16(float c, unsigned hw, float nz) {
  float d;
  if constexpr (HI)
    asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[0,1,0] op_sel_hi:[0,1,0]" : "=v"(d) : "s"(c), "v"(hw), "v"(nz));
  else
    asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[0,0,0] op_sel_hi:[0,1,0]" : "=v"(d) : "s"(c), "v"(hw), "v"(nz));
  return d;
}

template <int NKS, bool DISC>
__global__ void __launch_bounds__(kWsThreads, 1) k_steps_ws(StepArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ int s_flag;
  __shared__ int s_local;
  __shared__ int s_ready[4];  // sequence number of the product in slot w (2 m + sub + 1)
  __shared__ int s_taken[4];  // sequence number of the last product update wave w read
  __shared__ int s_pw_arrived;  // product waves that have handed over their product
  __shared__ int s_pw_go;       // product waves may load the operand of this sequence number
  // operand fragments in flight per product wave (the K loop is fully unrolled, so the
  // depth need not divide the k-steps): what the registers hold without spills
  constexpr int kPF = NKS < ws_prefetch(DISC) ? NKS : ws_prefetch(DISC);
  constexpr int NR = NKS < ws_reg_ksteps(DISC) ? NKS : ws_reg_ksteps(DISC);  // J k-steps in registers
  constexpr int NL = NKS - NR;                                 // J k-steps in LDS

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int w = wave & 3;
  const bool product_wave = wave < 4;
  const int g = blockIdx.x % grid_groups(a);
  const int mb = blockIdx.x / grid_groups(a);
  if (g >= a.groups) return;  // a padding workgroup (see StepArgs::gpad)
  const int row0 = mb * 256 + w * kWaveRows;
  const int col0 = g * kWaveCols;
  unsigned* ctr0 = a.sync + (size_t)(2 * g) * 64;
  unsigned* ctr1 = a.sync + (size_t)(2 * g + 1) * 64;
  unsigned* hs = a.sync + (size_t)(2 * a.groups + g) * 64;
  unsigned* msk = a.sync + (size_t)(3 * a.groups + g) * 64;
  unsigned* abort_flag = a.sync + (size_t)(4 * a.groups) * 64;
  // per generation every update wave of the group arrives once
  const unsigned gen = 4u * (unsigned)a.nb;

  // LDS: J tails [w][row tile][NL][1 KiB], then the product slots [w][row tile][lane][4 values]
  uint8_t* jtail = lds;
  uint8_t* slot = lds + (size_t)16 * NL * 1024 + (size_t)w * ws_slot_bytes(DISC);

  v4i jr[4][NR];
  if (product_wave) {
    const uint8_t* jw = static_cast<const uint8_t*>(a.jf) + (size_t)(row0 >> 4) * NKS * 1024 + lane * 16;
    // the LDS part one row tile at a time (so that no more than one tile's fragments are
    // in flight: registers are scarce at two waves per SIMD), then the register part,
    // and no load of it left outstanding when the step loop begins
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
#pragma unroll
      for (int ks = NR; ks < NKS; ++ks)
        *reinterpret_cast<v4i*>(jtail + ((size_t)((w * 4 + rt) * NL + (ks - NR)) * 1024 + lane * 16)) =
            *reinterpret_cast<const v4i*>(jw + (size_t)(rt * NKS + ks) * 1024);
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ks = 0; ks < NR; ++ks) jr[rt][ks] = *reinterpret_cast<const v4i*>(jw + (size_t)(rt * NKS + ks) * 1024);
    __builtin_amdgcn_s_waitcnt(0);
  }
  if (tid < 4) {
    s_ready[tid] = 0;
    s_taken[tid] = 0;
  }
  if (tid == 0) { s_pw_arrived = 0; s_pw_go = -1; }

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
      if (!keep_polling(spins, kSpinLimit, abort_flag, a.status)) { ok = 0; break; }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_local = (__builtin_popcount(ld_dev(msk)) == 1) ? 1 : 0;
    s_flag = ok;
  }
  __syncthreads();  // the last workgroup-wide barrier: the two roles run apart from here
  const bool alive0 = s_flag != 0;
  const int local = s_local;
  const int steps = a.m_end - a.m_begin;

  if (product_wave) {
    // ---- product wave ----
    // the two roles share the register file; a full wait here keeps the compiler's
    // count of outstanding loads from carrying the update role's loads into this loop
    __builtin_amdgcn_s_waitcnt(0);
    const __amdgpu_buffer_rsrc_t qr = make_rsrc(a.q, 2 * a.q_buf_bytes);
    v8i bq[kPF];
    // Operand loads bypass L1 (device scope) and need no cache maintenance: a workgroup-
    // scope invalidate does not reliably drop L1 lines that other CUs have rewritten (a
    // race that shows when the operand fits in L1), and an agent-scope one costs
    // microseconds.  The fragment's offset is uniform (a scalar register); only lane * 16
    // is per lane.
    const unsigned qbuf = (unsigned)__builtin_amdgcn_readfirstlane((int)a.q_buf_bytes);
    auto load_b = [&](int sub, int buf, int ks, v8i& dst) {
      const int soff = __builtin_amdgcn_readfirstlane((int)((unsigned)buf * qbuf +
                                                            (unsigned)(((2 * g + sub) * NKS + ks) * 2048)));
      const v4i lo = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(qr, lane * 16, soff, kPolicySc1));
      const v4i hi = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(qr, lane * 16 + 1024, soff, kPolicySc1));
      dst = cat(lo, hi);
    };
    auto prefetch = [&](int sub, int buf) {
#pragma unroll
      for (int u = 0; u < kPF; ++u) load_b(sub, buf, u, bq[u]);
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
    };
    // operand data of a column tile: every update wave of the group has arrived `target`
    // times (across XCDs, behind an agent-scope acquire fence)
    auto wait_q = [&](unsigned* ctr, unsigned target) -> bool {
      unsigned spins = 0;
      while (ld_dev(ctr) < target) {
        ++spins;
        if (!keep_polling(spins, kSpinLimit, abort_flag, a.status)) return false;
      }
      if (!local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      return true;
    };
    // strip the step tag from fragments and report (for the whole wave) whether any of
    // their units was stale: pat is the expected tag, cmask 0x40 (or 0: no check).  The
    // update waves write the operand in aligned 64-bit units (two words of one lane, one
    // store), so the first word of each unit tells its step: words 0, 2, 4, 6.
    // The sign product keeps its tags: there the tag is in every byte of a word, a tagged
    // +-1 byte is +-256 exactly, and the MFMA's block scale of the operand (2^-8 for a
    // tagged operand) takes the factor back exactly, so the words are only checked.
    auto strip = [&](v8i& b, unsigned pat) -> unsigned {
      unsigned o = 0;
      if constexpr (DISC) {
        // (b0 ^ pat) | (b2 ^ pat), (b4 ^ pat) | (b6 ^ pat): one bitop3 each (table 0x7E)
        o = __builtin_amdgcn_bitop3_b32((unsigned)b[0], (unsigned)b[2], pat, 0x7E) |
            __builtin_amdgcn_bitop3_b32((unsigned)b[4], (unsigned)b[6], pat, 0x7E);
      } else {
        // the E4M3 operand's tag is in the first word of each unit only
#pragma unroll
        for (int d = 0; d < 8; d += 2) {
          b[d] ^= (int)pat;
          o |= (unsigned)b[d];
        }
      }
      return o;
    };
    auto any_stale = [&](unsigned o, unsigned cmask) -> bool {
      return __builtin_amdgcn_ballot_w64((o & cmask) != 0u) != 0;
    };
    // the first kPF fragments of a K loop, loaded before it: checked together, and all
    // loaded again while any word is stale (the common wait for the operand)
    auto gate = [&](int sub, int buf, unsigned pat, unsigned cmask) -> bool {
      unsigned o = 0;
#pragma unroll
      for (int u = 0; u < kPF; ++u) o |= strip(bq[u], pat);
      if (__builtin_expect(!any_stale(o, cmask), 1)) return true;
      unsigned spins = 0;
      do {
        if (!keep_polling(++spins, kSpinLimit, abort_flag, a.status)) return false;
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int u = 0; u < kPF; ++u) load_b(sub, buf, u, bq[u]);
        __builtin_amdgcn_s_waitcnt(0);
        o = 0;
#pragma unroll
        for (int u = 0; u < kPF; ++u) o |= strip(bq[u], pat);
      } while (any_stale(o, cmask));
      return true;
    };
    // a later fragment: loaded again on its own while stale (other fragments in flight
    // are left alone, so that their registers and the load counter stay as they are)
    auto recheck = [&](int sub, int buf, int ks, unsigned pat, unsigned cmask) -> bool {
      if (__builtin_expect(!any_stale(strip(bq[ks % kPF], pat), cmask), 1)) return true;
      unsigned spins = 0;
      do {
        if (!keep_polling(++spins, kSpinLimit, abort_flag, a.status)) return false;
        __builtin_amdgcn_s_sleep(1);
        load_b(sub, buf, ks, bq[ks % kPF]);
        __builtin_amdgcn_s_waitcnt(0);
      } while (any_stale(strip(bq[ks % kPF], pat), cmask));
      return true;
    };
    auto load_jl = [&](int ks, v4i* dst) {
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
        dst[rt] = *reinterpret_cast<const v4i*>(jtail + ((size_t)((w * 4 + rt) * NL + (ks - NR)) * 1024 + lane * 16));
    };

    // the slot flag is read half way through the K loop (it has returned by its end)
    constexpr int kTakenAt = NKS / 2;
    // Where the group counter is needed (the launch's first operand; every operand switch
    // when the group spans XCDs) the four product waves meet: wave 0 polls the counter once
    // all four have handed over their product, then all load (one poller per workgroup
    // instead of four, and the four load the same fragments together).
    auto pw_sync = [&](int seqv, unsigned* ctr, unsigned target) -> bool {
      bool ok = true;
      if (w == 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(&s_pw_arrived, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < 4 * seqv) {
          if (!keep_polling(++spins, kLdsSpinLimit, abort_flag, a.status)) { ok = false; break; }
        }
        if (ok) ok = wait_q(ctr, target);
        __hip_atomic_store(&s_pw_go, ok ? seqv : kPwAbandoned, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        return ok;
      }
      unsigned spins = 0;
      int gv;
      while ((gv = __hip_atomic_load(&s_pw_go, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) < seqv) {
        if (gv == kPwAbandoned) return false;
        if (!keep_polling(++spins, kLdsSpinLimit, abort_flag, a.status)) return false;
      }
      return true;
    };
    bool alive = alive0 && pw_sync(0, ctr0, gen);
    if (alive) prefetch(0, 0);
    for (int s = 0; alive && s < steps; ++s) {
      const int cur = s & 1;
      // the launch's first operand is behind the group counter and carries no tag
      const unsigned cmask = s > 0 ? 0x40u : 0u;
      const unsigned pat = ((s >> 1) & 1) ? cmask : 0u;
      // E8M0 block scale of the operand: 2^0, or 2^-8 for a tagged sign operand
      const int scale_q = DISC && pat ? 127 - 8 : 127;
#pragma unroll
      for (int sub = 0; sub < 2; ++sub) {
        const int seq = 2 * s + sub + 1;
        // the operand of the next K loop: tile 1 of this step, or tile 0 of the next
        const bool has_next = sub == 0 || s + 1 < steps;
        unsigned* const nctr = sub == 0 ? ctr1 : ctr0;
        const unsigned ntarget = gen * (unsigned)(sub == 0 ? s + 1 : s + 2);
        const int nbuf = sub == 0 ? cur : cur ^ 1;
        int taken = 0;
        v4f acc[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) acc[rt] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        // the scale in a vector register of its own for the whole K loop (as a scalar the
        // compiler copies it into a free vector register before every k-step)
        int scale_v;
        asm volatile("v_mov_b32 %0, %1" : "=v"(scale_v) : "s"(scale_q));
        v4i jl[2][4];
        if constexpr (NL > 0) load_jl(NR, jl[0]);
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
          __builtin_amdgcn_sched_barrier(0);
          if (ks == 0) {
            if (alive) alive = gate(sub, cur, pat, cmask);
          } else if (ks >= kPF) {
            if (alive) alive = recheck(sub, cur, ks, pat, cmask);
          }
          if constexpr (NL > 0) {
            if (ks >= NR && ks + 1 < NKS) load_jl(ks + 1, jl[(ks + 1 - NR) & 1]);
          }
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) {
            const v4i f = ks < NR ? jr[rt][ks < NR ? ks : 0] : jl[(ks - NR) & 1][rt];
            acc[rt] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(cat(f, f), bq[ks % kPF], acc[rt], 4, 0, 0,
                                                                       127, 0, scale_v);
          }
          asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]));
          if (ks + kPF < NKS) load_b(sub, cur, ks + kPF, bq[ks % kPF]);
          if (ks == kTakenAt) taken = __hip_atomic_load(&s_taken[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          asm volatile("" ::: "memory");
          __builtin_amdgcn_sched_barrier(0);
        }
        if (!alive) break;
        // within one XCD the next operand's first fragments travel during the hand-over
        if (local && has_next) prefetch(sub ^ 1, nbuf);
        // hand the product to the update wave once it has read the previous one (the
        // update wave publishes its read count with a release after reading the slot;
        // LDS operations execute in order, so the relaxed reads here suffice)
        {
          unsigned spins = 0;
          while (taken < seq - 1 &&
                 (taken = __hip_atomic_load(&s_taken[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) < seq - 1) {
            __builtin_amdgcn_s_sleep(1);
            if (!keep_polling(++spins, kLdsSpinLimit, abort_flag, a.status)) { alive = false; break; }
          }
          if (!alive) break;
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) {
            if constexpr (DISC) {
              // integers of magnitude <= 2048: f16 holds them exactly (round toward zero
              // leaves them unchanged)
              const v2u h{__builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(acc[rt][0], acc[rt][1])),
                          __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(acc[rt][2], acc[rt][3]))};
              *reinterpret_cast<v2u*>(slot + (size_t)(rt * 64 + lane) * 8) = h;
            } else {
              *reinterpret_cast<v4f*>(slot + (size_t)(rt * 64 + lane) * 16) = acc[rt];
            }
          }
          // LDS operations of one wave execute in order, so the flag, written after the
          // slot, is seen after it; a release here would only wait for the slot writes
          asm volatile("" ::: "memory");
          __hip_atomic_store(&s_ready[w], seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        // across XCDs, the operand of the next K loop is loaded behind the group counter
        if (!local) {
          __hip_atomic_fetch_add(&s_pw_arrived, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (has_next) {
            alive = pw_sync(seq, nctr, ntarget);
            if (alive) prefetch(sub ^ 1, nbuf);
          }
          if (!alive) break;
        }
      }
    }
    return;
  }

  // ---- update wave ----
  __builtin_amdgcn_s_waitcnt(0);
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
  // count this wave in at `ctr` once its operand stores are acknowledged (then in L2)
  auto arrive = [&](unsigned* ctr) {
    __builtin_amdgcn_s_waitcnt(0);
    if (lane == 0) {
      if (!local) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  const float A = a.A, dt = a.dt, cdt = a.cdt;
  // eqs. (7), (3), (4), (5) for column tile `sub`, in two parts: `before` needs only the
  // state and runs while the product wave computes the tile's product; `after` adds the
  // product (acc), applies the wall and writes the operand.  t carries y + dy between them.
  float t[16];
  auto before = [&](int sub, float rm) {
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
  };
  // the operand buffers as one buffer resource; this lane's words of column tile sub sit
  // at qoff[sub] in either buffer, those of row tiles 0..3 one after the other (the
  // placement keeps a lane's sixteen spins of a k-step together; row0 is a multiple of 64)
  const __amdgpu_buffer_rsrc_t qw = make_rsrc(a.q, 2 * a.q_buf_bytes);
  unsigned qoff[2];
#pragma unroll
  for (int sub = 0; sub < 2; ++sub) qoff[sub] = (unsigned)fp8_operand_offset(NKS, row0, col0 + sub * 16, lane);
  // u holds Dy = c dt (J q)_i of the lane's 16 elements on entry
  auto after = [&](int sub, float* u, int qbase, unsigned tag) {
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
    // row tiles 2 h and 2 h + 1 in one 64-bit store: the product waves check one word of
    // each aligned 64-bit unit (an aligned 64-bit store is seen whole or not at all)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      // the E4M3 operand carries the tag in the unit's first word only (the product waves
      // strip and check that word); the sign operand in every byte (its block scale)
      const v2u wd{encode_fp8x4<DISC>(xs[sub][2 * h], tag), encode_fp8x4<DISC>(xs[sub][2 * h + 1], DISC ? tag : 0u)};
      __builtin_amdgcn_raw_buffer_store_b64(wd, qw, qoff[sub] + 8 * h, qbase, 0);
    }
  };

  // the step tag: bit 6 of the word's first byte, or of every byte for the sign operand
  constexpr unsigned kTag = DISC ? 0x40404040u : 0x40u;
  bool alive = alive0;
  if (alive) {
#pragma unroll
    for (int sub = 0; sub < 2; ++sub)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        // operand 0 untagged in buffer 0; buffer 1 holds the tag that operand 1 does not carry
        store_operand<kFormFP8, DISC>(a.q, a.q_buf_bytes, NKS, row0 + rt * 16, col0 + sub * 16, lane,
                                      xs[sub][rt]);
        store_operand<kFormFP8, DISC>(a.q + a.q_buf_bytes, a.q_buf_bytes, NKS, row0 + rt * 16, col0 + sub * 16,
                                      lane, xs[sub][rt], DISC || rt % 2 == 0 ? kTag : 0u);
      }
    arrive(ctr0);
    arrive(ctr1);
  }
  for (int s = 0; alive && s < steps; ++s) {
    const int m = a.m_begin + s;
    const int qbase = ((s + 1) & 1) * (int)a.q_buf_bytes;  // operand s + 1 in buffer (s + 1) % 2
    const unsigned tag = ((s + 1) >> 1) & 1 ? kTag : 0u;  // operand s + 1
    const float rm = a.rtab[m];
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) {
      const int seq = 2 * s + sub + 1;
      before(sub, rm);
      unsigned spins = 0;
      while (__hip_atomic_load(&s_ready[w], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < seq) {
        if (!keep_polling(++spins, kLdsSpinLimit, abort_flag, a.status)) { alive = false; break; }
      }
      if (!alive) break;
      float u[16];  // Dy = c dt (J q)_i, eq. (3)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        if constexpr (DISC) {
          const v2u h = *reinterpret_cast<const v2u*>(slot + (size_t)(rt * 64 + lane) * 8);
          // the words go through scalars: a bit cast of a vector element expression is
          // compiled as a cast of element 0 by this compiler
          const unsigned w0 = h[0], w1 = h[1];
          u[4 * rt + 0] = mul_f16<false>(cdt, w0, -0.0f);
          u[4 * rt + 1] = mul_f16<true>(cdt, w0, -0.0f);
          u[4 * rt + 2] = mul_f16<false>(cdt, w1, -0.0f);
          u[4 * rt + 3] = mul_f16<true>(cdt, w1, -0.0f);
        } else {
          const v4f acc = *reinterpret_cast<const v4f*>(slot + (size_t)(rt * 64 + lane) * 16);
#pragma unroll
          for (int v = 0; v < 4; ++v) u[4 * rt + v] = cdt * acc[v];
        }
      }
      __hip_atomic_store(&s_taken[w], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      after(sub, u, qbase, tag);
      if (!local) arrive(sub == 0 ? ctr0 : ctr1);
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

const void* steps_kernel_ws(int nks, bool discrete) {
  if (discrete) {
    switch (nks) {
      case 4: return reinterpret_cast<const void*>(&k_steps_ws<4, true>);
      case 8: return reinterpret_cast<const void*>(&k_steps_ws<8, true>);
      case 12: return reinterpret_cast<const void*>(&k_steps_ws<12, true>);
      case 16: return reinterpret_cast<const void*>(&k_steps_ws<16, true>);
      default: return nullptr;
    }
  }
  switch (nks) {
    case 4: return reinterpret_cast<const void*>(&k_steps_ws<4, false>);
    case 8: return reinterpret_cast<const void*>(&k_steps_ws<8, false>);
    case 12: return reinterpret_cast<const void*>(&k_steps_ws<12, false>);
    case 16: return reinterpret_cast<const void*>(&k_steps_ws<16, false>);
    default: return nullptr;
  }
}

size_t steps_ws_lds_bytes(int np, bool discrete) {
  const int nks = np / kKS;
  const int nl = nks > ws_reg_ksteps(discrete) ? nks - ws_reg_ksteps(discrete) : 0;
  return (size_t)16 * nl * 1024 + (size_t)4 * ws_slot_bytes(discrete);
}

}  // namespace gsb
