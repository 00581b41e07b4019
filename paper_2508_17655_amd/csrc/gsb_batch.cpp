// gsb_batch.cpp -- batched instances of different sizes (C ABI, include/gsb.h): argument
// checking, device layout, the queue plan, the tile autotuner and HIP-graph replay of
// the persistent batched launch.
#include "../../include/gsb.h"
#include "gsb_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

using namespace gsb;

namespace {

gsb_status bfail(gsb_status s, const std::string& msg) {
  set_last_error(msg.c_str());
  return s;
}

gsb_status bhip(hipError_t e, const char* what) {
  return bfail(GSB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define BHIP(expr, what)                          \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return bhip(e_, what);  \
  } while (0)

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr int kTiles[3] = {64, 128, 256};
int tile_index(int bm) { return bm == 64 ? 0 : (bm == 128 ? 1 : (bm == 256 ? 2 : -1)); }

// Longest processing time first: units (all gangs of one instance) in decreasing order of
// work = gangs x width x cost, each to the queue with the least work so far; within a
// queue, units run in decreasing order of cost (then width, then index).
gsb_status plan_queues(int units, const int* width, const int* gangs, const double* cost, int queues, int workers,
                       int* queue, int* rank) {
  if (units < 0 || queues < 1 || workers < 1) return bfail(GSB_EINVAL, "plan: bad sizes");
  for (int u = 0; u < units; ++u) {
    if (width[u] < 1 || gangs[u] < 1 || !(cost[u] >= 0) || !std::isfinite(cost[u]))
      return bfail(GSB_EINVAL, "plan: unit " + std::to_string(u) + " has a bad width, gang count or cost");
    if (width[u] > workers)
      return bfail(GSB_EUNSUPPORTED, "plan: a gang of " + std::to_string(width[u]) + " workgroups exceeds the " +
                                         std::to_string(workers) + " workgroups of a queue");
  }
  std::vector<int> idx(units);
  std::iota(idx.begin(), idx.end(), 0);
  auto work = [&](int u) { return (double)gangs[u] * width[u] * cost[u]; };
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return work(a) > work(b); });
  std::vector<double> load(queues, 0.0);
  for (int u : idx) {
    const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    queue[u] = q;
    load[q] += work(u);
  }
  std::vector<int> ord(units);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (cost[a] != cost[b]) return cost[a] > cost[b];
    return width[a] > width[b];
  });
  std::vector<int> next(queues, 0);
  for (int u : ord) rank[u] = next[queue[u]]++;
  return GSB_OK;
}

}  // namespace

struct gsb_batch {
  int count = 0, R = 0, rp = 0, np_max = 0;
  std::vector<int> n, np;
  std::vector<double> c, dt, lmax, lmin;
  std::vector<char> have_j, have_eig;
  std::vector<int> tile_fixed;             // 0: automatic
  std::vector<double> us[2][3];            // measured us per step of one gang, per occupancy and tile
  int occ = 1;                             // workgroups per CU of the runs (1 or 2)
  int occ_fixed = 0;                       // caller's choice, 0 = automatic
  int init_mode = GSB_INIT_X;
  bool use_graph = false;
  hipStream_t stream = nullptr;
  std::mutex upload_mu;                    // gsb_batch_set_coupling may run on several threads
  // workspace
  void* ws_user = nullptr;
  size_t ws_user_bytes = 0;
  void* ws_own = nullptr;
  size_t ws_own_bytes = 0;
  uint8_t* ws = nullptr;
  std::vector<size_t> off_j, off_x, off_y, off_p, off_q, off_s8, off_sync;
  size_t off_eacc = 0, off_E = 0, off_bidx = 0, off_be = 0, off_ctl = 0, off_status = 0, off_stage = 0;
  size_t sync_bytes_each = 0, total = 0;
  // tables of the current run (device copies in `aux`)
  std::vector<StepArgs> h_inst;
  std::vector<BatchInst> h_bi;
  std::vector<BatchSlot> h_slots;
  std::vector<int> h_qoff, h_need, h_tile;
  std::vector<float> h_rtab;
  void* aux = nullptr;
  size_t aux_bytes = 0;
  StepArgs* d_inst = nullptr;
  BatchInst* d_bi = nullptr;
  BatchSlot* d_slots = nullptr;
  int* d_qoff = nullptr;
  int* d_need = nullptr;
  float* d_rtab = nullptr;
  unsigned long long* d_clk = nullptr;
  // device facts
  // per occupancy (index occ - 1): workgroups of the launch, per XCD queue, LDS for J rows
  int grid[2] = {0, 0}, cap[2] = {0, 0}, lds_bytes[2] = {0, 0};
  bool facts = false;
  double wall_hz = 0;
  // run
  bool ran = false;
  int variant = 0, M = 0;
  double A = 0;
  uint64_t seed = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  hipStream_t capture_stream = nullptr;  // library-owned: the caller's may be the null stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<double> graph_key;
};

namespace {

gsb_status device_facts(gsb_batch* b) {
  if (b->facts) return GSB_OK;
  int dev = 0, cus = 0, rate_khz = 0, lds_max = 0;
  BHIP(hipGetDevice(&dev), "hipGetDevice");
  BHIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device attribute");
  BHIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev), "device attribute");
  BHIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "device attribute");
  // the step kernel runs one workgroup per CU (registers), so J rows may fill the LDS
  // beside the kernel's own few bytes
  for (int occ = 1; occ <= 2; ++occ) {
    const int lds = std::max(0, std::min(lds_max, 160 * 1024) / occ - 1024) / 1024 * 1024;
    const int a = batch_workgroups_per_cu(false, occ, lds), d = batch_workgroups_per_cu(true, occ, lds);
    const int per_cu = std::min(std::min(a, d), occ);
    if (per_cu < 1) return bfail(GSB_EDEVICE, "occupancy query failed for the batched step kernel");
    b->lds_bytes[occ - 1] = lds;
    b->grid[occ - 1] = per_cu * cus;
    b->cap[occ - 1] = b->grid[occ - 1] / kBatchXcds;
  }
  // occupancy 2 only where the hardware gives it
  if (b->grid[1] < 2 * b->grid[0]) b->grid[1] = 0;
  b->facts = true;
  b->wall_hz = rate_khz > 0 ? rate_khz * 1e3 : 1e8;
  return GSB_OK;
}

void layout(gsb_batch* b) {
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += al256(bytes); return o; };
  const size_t rp = (size_t)b->rp;
  b->sync_bytes_each = sync_words(b->rp / 32) * 4;
  for (int k = 0; k < b->count; ++k) {
    const size_t np = (size_t)b->np[k];
    b->off_j[k] = take(np * np / 2);
    b->off_x[k] = take(rp * np * 4);
    b->off_y[k] = take(rp * np * 4);
    b->off_p[k] = take(rp * np * 4);
    b->off_q[k] = take(2 * rp * np);
    b->off_s8[k] = take(rp * np);
  }
  const size_t sync0 = off;
  for (int k = 0; k < b->count; ++k) b->off_sync[k] = sync0 + (size_t)k * b->sync_bytes_each;
  off = sync0 + al256((size_t)b->count * b->sync_bytes_each);
  b->off_eacc = take((size_t)b->count * rp * 4);
  b->off_ctl = take(kBatchCtlWords * 4);
  b->off_status = take(256);
  b->off_E = take((size_t)b->count * rp * 8);
  b->off_bidx = take((size_t)b->count * 4);
  b->off_be = take((size_t)b->count * 8);
  b->off_stage = take((size_t)b->np_max * b->np_max * 4);
  b->total = off;
}

gsb_status ensure_ws(gsb_batch* b) {
  if (b->ws) return GSB_OK;
  if (b->ws_user) {
    if (b->ws_user_bytes < b->total)
      return bfail(GSB_ENOMEM, "bound workspace has " + std::to_string(b->ws_user_bytes) + " bytes, the batch needs " +
                                   std::to_string(b->total));
    b->ws = static_cast<uint8_t*>(b->ws_user);
    return GSB_OK;
  }
  void* p = nullptr;
  if (hipMalloc(&p, b->total) != hipSuccess)
    return bfail(GSB_ENOMEM, "device allocation of " + std::to_string(b->total) + " bytes failed");
  b->ws_own = p;
  b->ws_own_bytes = b->total;
  b->ws = static_cast<uint8_t*>(p);
  return GSB_OK;
}

void drop_graph(gsb_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->graph_key.clear();
}

// Tile rows of instance k: the caller's choice, else the fastest measured tile, else the
// smallest tile whose gang fits in one XCD queue.
int choose_tile(const gsb_batch* b, int k, int occ) {
  const int cap = b->cap[occ - 1];
  if (b->tile_fixed[k]) return b->tile_fixed[k];
  int best = 0;
  double best_us = 0;
  for (int t = 0; t < 3; ++t) {
    const double u = b->us[occ - 1][t][k];
    if (u > 0 && b->np[k] / kTiles[t] <= cap && (best == 0 || u < best_us)) { best = kTiles[t]; best_us = u; }
  }
  if (best) return best;
  for (int t = 0; t < 3; ++t)
    if (b->np[k] / kTiles[t] <= cap) return kTiles[t];
  return 0;
}

gsb_status ensure_aux(gsb_batch* b, size_t need) {
  if (b->aux_bytes >= need) return GSB_OK;
  if (b->aux) {
    BHIP(hipStreamSynchronize(b->stream), "stream synchronise");
    drop_graph(b);  // the graph refers to the old tables
    BHIP(hipFree(b->aux), "free");
    b->aux = nullptr;
    b->aux_bytes = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, need) != hipSuccess) return bfail(GSB_ENOMEM, "device allocation of the batch tables failed");
  b->aux = p;
  b->aux_bytes = need;
  return GSB_OK;
}

// Build the tables of a run (tiles, step arguments, queue plan) and upload them.
gsb_status prepare(gsb_batch* b, int variant, double A, int steps, uint64_t seed, const int* tile_override,
                   bool with_clock) {
  gsb_status s = device_facts(b);
  if (s != GSB_OK) return s;
  for (int k = 0; k < b->count; ++k)
    if (!b->have_j[k]) return bfail(GSB_ESTATE, "instance " + std::to_string(k) + " has no coupling yet");
  // the host tables of a previous run may still be in flight to the device
  BHIP(hipStreamSynchronize(b->stream), "stream synchronise");
  const bool discrete = variant == GSB_DSB || variant == GSB_GDSB;
  const float Aeff = (variant == GSB_GBSB || variant == GSB_GDSB) ? (float)A : 0.0f;
  b->h_tile.assign(b->count, 0);
  std::vector<int> width(b->count), gangs(b->count), queue(b->count), rank(b->count);
  std::vector<double> cost(b->count);
  for (int k = 0; k < b->count; ++k) {
    const int bm = tile_override ? tile_override[k] : choose_tile(b, k, b->occ);
    if (bm == 0 || b->np[k] / bm > b->cap[b->occ - 1])
      return bfail(GSB_EUNSUPPORTED, "instance " + std::to_string(k) + " (n = " + std::to_string(b->n[k]) +
                                         ") does not fit in the workgroups of one XCD");
    b->h_tile[k] = bm;
    width[k] = b->np[k] / bm;
    gangs[k] = b->rp / (8192 / bm);
    const double u = b->us[b->occ - 1][tile_index(bm)][k];
    cost[k] = u > 0 ? u : 1.0 + 1.2e-3 * b->np[k];  // unmeasured: a model of us per step
  }
  s = plan_queues(b->count, width.data(), gangs.data(), cost.data(), kBatchXcds, b->cap[b->occ - 1], queue.data(),
                  rank.data());
  if (s != GSB_OK) return s;
  // slots: per XCD queue in rank order, then the device-wide queue in decreasing cost
  b->h_slots.clear();
  b->h_qoff.assign(kBatchXcds + 2, 0);
  b->h_need.assign(kBatchXcds, 0);
  auto push_unit = [&](int k) {
    for (int g = 0; g < gangs[k]; ++g)
      for (int mb = 0; mb < width[k]; ++mb) b->h_slots.push_back(BatchSlot{k, g, mb, b->h_tile[k]});
  };
  for (int q = 0; q < kBatchXcds; ++q) {
    b->h_qoff[q] = (int)b->h_slots.size();
    std::vector<int> mine;
    for (int k = 0; k < b->count; ++k)
      if (queue[k] == q) mine.push_back(k);
    std::sort(mine.begin(), mine.end(), [&](int a, int c) { return rank[a] < rank[c]; });
    for (int k : mine) {
      push_unit(k);
      b->h_need[q] = std::max(b->h_need[q], width[k]);
    }
  }
  b->h_qoff[kBatchXcds] = (int)b->h_slots.size();
  {
    std::vector<int> all(b->count);
    std::iota(all.begin(), all.end(), 0);
    std::stable_sort(all.begin(), all.end(), [&](int a, int c) { return cost[a] > cost[c]; });
    for (int k : all) push_unit(k);
  }
  b->h_qoff[kBatchXcds + 1] = (int)b->h_slots.size();
  // schedule table r_m = 1 / (M - m) (eqs. (6), (7)), binary64 rounded once
  b->h_rtab.assign(steps, 0.0f);
  for (int m = 0; m < steps; ++m) b->h_rtab[m] = (float)(1.0 / (double)(steps - m));
  // step arguments and per-instance buffers
  uint8_t* w = b->ws;
  b->h_inst.assign(b->count, StepArgs{});
  b->h_bi.assign(b->count, BatchInst{});
  const size_t nslots = b->h_slots.size();
  size_t aoff = 0;
  auto atake = [&](size_t bytes) { size_t o = aoff; aoff += al256(bytes); return o; };
  const size_t o_inst = atake(sizeof(StepArgs) * b->count), o_bi = atake(sizeof(BatchInst) * b->count);
  const size_t o_slots = atake(sizeof(BatchSlot) * nslots), o_qoff = atake(sizeof(int) * (kBatchXcds + 2));
  const size_t o_need = atake(sizeof(int) * kBatchXcds), o_rtab = atake(sizeof(float) * steps);
  const size_t o_clk = atake(sizeof(unsigned long long) * 2 * nslots);
  s = ensure_aux(b, aoff);
  if (s != GSB_OK) return s;
  uint8_t* x = static_cast<uint8_t*>(b->aux);
  b->d_inst = reinterpret_cast<StepArgs*>(x + o_inst);
  b->d_bi = reinterpret_cast<BatchInst*>(x + o_bi);
  b->d_slots = reinterpret_cast<BatchSlot*>(x + o_slots);
  b->d_qoff = reinterpret_cast<int*>(x + o_qoff);
  b->d_need = reinterpret_cast<int*>(x + o_need);
  b->d_rtab = reinterpret_cast<float*>(x + o_rtab);
  b->d_clk = with_clock ? reinterpret_cast<unsigned long long*>(x + o_clk) : nullptr;
  if (b->d_clk)  // slots the launch does not take keep a zero end time
    BHIP(launch_fill_u32(reinterpret_cast<unsigned*>(b->d_clk), 4 * nslots, 0u, b->stream), "clear clocks");
  for (int k = 0; k < b->count; ++k) {
    StepArgs& a = b->h_inst[k];
    a.n = b->n[k];
    a.np = b->np[k];
    a.rp = b->rp;
    a.groups = gangs[k];
    a.nb = width[k];
    a.discrete = discrete ? 1 : 0;
    a.m_begin = 0;
    a.m_end = steps;
    a.A = Aeff;
    a.dt = (float)b->dt[k];
    a.cdt = (float)(b->c[k] * b->dt[k]);
    a.acol = nullptr;
    a.rtab = b->d_rtab;
    a.jf = w + b->off_j[k];
    a.q = w + b->off_q[k];
    a.q_buf_bytes = (size_t)b->rp * b->np[k];
    a.x = reinterpret_cast<float*>(w + b->off_x[k]);
    a.y = reinterpret_cast<float*>(w + b->off_y[k]);
    a.p = reinterpret_cast<float*>(w + b->off_p[k]);
    a.sync = reinterpret_cast<unsigned*>(w + b->off_sync[k]);
    a.status = reinterpret_cast<unsigned*>(w + b->off_status);
    BatchInst& bi = b->h_bi[k];
    bi.seed = seed + (uint64_t)k;
    bi.s8 = w + b->off_s8[k];
    bi.eacc = reinterpret_cast<int*>(w + b->off_eacc) + (size_t)k * b->rp;
    bi.E = reinterpret_cast<double*>(w + b->off_E) + (size_t)k * b->rp;
    bi.best_idx = reinterpret_cast<int*>(w + b->off_bidx) + k;
    bi.best_e = reinterpret_cast<double*>(w + b->off_be) + k;
  }
  BHIP(hipMemcpyAsync(b->d_inst, b->h_inst.data(), sizeof(StepArgs) * b->count, hipMemcpyHostToDevice, b->stream),
       "upload tables");
  BHIP(hipMemcpyAsync(b->d_bi, b->h_bi.data(), sizeof(BatchInst) * b->count, hipMemcpyHostToDevice, b->stream),
       "upload tables");
  BHIP(hipMemcpyAsync(b->d_slots, b->h_slots.data(), sizeof(BatchSlot) * nslots, hipMemcpyHostToDevice, b->stream),
       "upload tables");
  BHIP(hipMemcpyAsync(b->d_qoff, b->h_qoff.data(), sizeof(int) * (kBatchXcds + 2), hipMemcpyHostToDevice, b->stream),
       "upload tables");
  BHIP(hipMemcpyAsync(b->d_need, b->h_need.data(), sizeof(int) * kBatchXcds, hipMemcpyHostToDevice, b->stream),
       "upload tables");
  BHIP(hipMemcpyAsync(b->d_rtab, b->h_rtab.data(), sizeof(float) * steps, hipMemcpyHostToDevice, b->stream),
       "upload tables");
  BHIP(hipStreamSynchronize(b->stream), "stream synchronise");
  return GSB_OK;
}

// The launch sequence of a run: starting states, cleared barriers and queues, the
// persistent batched step kernel, energies and the best replica of every instance.
gsb_status enqueue_run(gsb_batch* b, bool discrete, bool cooperative, bool timed, hipStream_t st) {
  uint8_t* w = b->ws;
  BHIP(launch_init_batch(b->d_inst, b->d_bi, b->count, b->np_max, b->rp, b->init_mode, st), "init kernel");
  BHIP(launch_fill_u32(reinterpret_cast<unsigned*>(w + b->off_sync[0]), b->count * b->sync_bytes_each / 4, 0u,
                       st),
       "clear barriers");
  BHIP(launch_fill_u32(reinterpret_cast<unsigned*>(w + b->off_ctl), kBatchCtlWords, 0u, st), "clear queues");
  BHIP(launch_fill_u32(reinterpret_cast<unsigned*>(w + b->off_status), 64, 0u, st), "clear status");
  BatchArgs a;
  a.inst = b->d_inst;
  a.slots = b->d_slots;
  a.qoff = b->d_qoff;
  a.need = b->d_need;
  a.ctl = reinterpret_cast<unsigned*>(w + b->off_ctl);
  a.status = reinterpret_cast<unsigned*>(w + b->off_status);
  a.clk = b->d_clk;
  a.grid = b->grid[b->occ - 1];
  a.lds_bytes = b->lds_bytes[b->occ - 1];
  if (timed) BHIP(hipEventRecord(b->ev0, st), "event record");
  BHIP(launch_steps_batch(discrete, b->occ, a, st, cooperative), "batched step kernel launch");
  if (timed) BHIP(hipEventRecord(b->ev1, st), "event record");
  BHIP(launch_fill_u32(reinterpret_cast<unsigned*>(w + b->off_eacc), (size_t)b->count * b->rp, 0u, st),
       "clear energies");
  BHIP(launch_energy_batch(b->d_inst, b->d_bi, b->count, b->np_max, b->rp, b->R, st), "energy kernels");
  return GSB_OK;
}

gsb_status check_status(gsb_batch* b) {
  unsigned st = 0;
  BHIP(hipMemcpyAsync(&st, b->ws + b->off_status, 4, hipMemcpyDeviceToHost, b->stream), "status read");
  BHIP(hipStreamSynchronize(b->stream), "stream synchronise");
  if (st == 2) return bfail(GSB_EDEVICE, "batched step kernel: not all workgroups became co-resident");
  if (st != 0) return bfail(GSB_EDEVICE, "batched step kernel: a replica-group barrier timed out");
  return GSB_OK;
}

gsb_status check_run_args(gsb_batch* b, int variant, double A, int steps) {
  if (!b) return bfail(GSB_EINVAL, "batch is NULL");
  if (variant < GSB_BSB || variant > GSB_GDSB) return bfail(GSB_EINVAL, "unknown variant");
  if (!std::isfinite(A) || A < 0) return bfail(GSB_EINVAL, "control strength must be finite and >= 0");
  if (steps < 1 || steps > (1 << 24)) return bfail(GSB_EINVAL, "steps must be in [1, 2^24]");
  return GSB_OK;
}

}  // namespace

extern "C" {

gsb_status gsb_batch_plan(int32_t units, const int32_t* width, const int32_t* gangs, const double* cost,
                          int32_t queues, int32_t workers, int32_t* queue, int32_t* rank) {
  set_last_error("");
  if (units > 0 && (!width || !gangs || !cost || !queue || !rank)) return bfail(GSB_EINVAL, "NULL argument");
  return plan_queues(units, width, gangs, cost, queues, workers, queue, rank);
}

gsb_status gsb_batch_create(int32_t count, const int32_t* n, int32_t replicas, gsb_batch** out) {
  set_last_error("");
  if (!out) return bfail(GSB_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1 || count > (1 << 16)) return bfail(GSB_EINVAL, "count must be in [1, 65536]");
  if (!n) return bfail(GSB_EINVAL, "n is NULL");
  if (replicas < 1 || replicas > (1 << 16)) return bfail(GSB_EINVAL, "replicas must be in [1, 65536]");
  for (int k = 0; k < count; ++k)
    if (n[k] < 1 || n[k] > 8192) return bfail(GSB_EINVAL, "n[" + std::to_string(k) + "] must be in [1, 8192]");
  gsb_batch* b = new (std::nothrow) gsb_batch;
  if (!b) return bfail(GSB_ENOMEM, "host allocation failed");
  try {
    b->count = count;
    b->R = replicas;
    b->rp = (replicas + kRepPad - 1) / kRepPad * kRepPad;
    b->n.assign(n, n + count);
    b->np.resize(count);
    for (int k = 0; k < count; ++k) {
      b->np[k] = (n[k] + kBatchRowPad - 1) / kBatchRowPad * kBatchRowPad;
      b->np_max = std::max(b->np_max, b->np[k]);
    }
    b->c.assign(count, 0.0);
    b->dt.assign(count, 0.0);
    b->lmax.assign(count, 0.0);
    b->lmin.assign(count, 0.0);
    b->have_j.assign(count, 0);
    b->have_eig.assign(count, 0);
    b->tile_fixed.assign(count, 0);
    for (auto& per_occ : b->us)
      for (auto& u : per_occ) u.assign(count, 0.0);
    for (auto* v : {&b->off_j, &b->off_x, &b->off_y, &b->off_p, &b->off_q, &b->off_s8, &b->off_sync})
      v->assign(count, 0);
  } catch (...) {
    delete b;
    return bfail(GSB_ENOMEM, "host allocation failed");
  }
  layout(b);
  *out = b;
  return GSB_OK;
}

void gsb_batch_destroy(gsb_batch* b) {
  if (!b) return;
  // Teardown cannot report errors; a failed synchronisation or free is ignored here.
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  if (b->ws_own) (void)hipFree(b->ws_own);
  if (b->aux) (void)hipFree(b->aux);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  delete b;
}

gsb_status gsb_batch_set_stream(gsb_batch* b, void* stream) {
  set_last_error("");
  if (!b) return bfail(GSB_EINVAL, "batch is NULL");
  if (static_cast<hipStream_t>(stream) != b->stream) drop_graph(b);
  b->stream = static_cast<hipStream_t>(stream);
  return GSB_OK;
}

gsb_status gsb_batch_workspace_size(gsb_batch* b, size_t* bytes) {
  set_last_error("");
  if (!b || !bytes) return bfail(GSB_EINVAL, "NULL argument");
  *bytes = b->total;
  return GSB_OK;
}

gsb_status gsb_batch_bind_workspace(gsb_batch* b, void* ptr, size_t bytes) {
  set_last_error("");
  if (!b) return bfail(GSB_EINVAL, "batch is NULL");
  if (b->ws) return bfail(GSB_ESTATE, "the batch already holds couplings in its workspace");
  if (!ptr || ((uintptr_t)ptr & 255)) return bfail(GSB_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  if (bytes < b->total)
    return bfail(GSB_ENOMEM, "workspace has " + std::to_string(bytes) + " bytes, the batch needs " +
                                 std::to_string(b->total));
  b->ws_user = ptr;
  b->ws_user_bytes = bytes;
  return GSB_OK;
}

gsb_status gsb_batch_set_coupling(gsb_batch* b, int32_t k, const float* J, double c, double dt) {
  set_last_error("");
  if (!b || !J) return bfail(GSB_EINVAL, "NULL argument");
  if (k < 0 || k >= b->count) return bfail(GSB_EINVAL, "instance index out of range");
  if (!(std::isfinite(c) && std::isfinite(dt))) return bfail(GSB_EINVAL, "c and dt must be finite");
  const int n = b->n[k];
  for (int i = 0; i < n; ++i) {
    if (J[(size_t)i * n + i] != 0.0f) return bfail(GSB_EDIAG, "J_ii != 0 at i = " + std::to_string(i));
    for (int j = 0; j < n; ++j) {
      const float v = J[(size_t)i * n + j];
      if (!std::isfinite(v)) return bfail(GSB_ENONFINITE, "J has a non-finite entry");
      if (!(v == 0.0f || v == 1.0f || v == -1.0f))
        return bfail(GSB_EUNSUPPORTED, "batched instances need J entries in {0, +1, -1} (FP8 product)");
      if (j > i && v != J[(size_t)j * n + i])
        return bfail(GSB_ENOTSYM, "J_ij != J_ji at (" + std::to_string(i) + ", " + std::to_string(j) + ")");
    }
  }
  // App. A: c = 1 / lambda_max, and eq. (13) dt = D_t sqrt(2 / (1 - lambda_min / lambda_max)),
  // D_t = 1.25, unless given (> 0)
  double lmax = 0, lmin = 0;
  const bool eig = !(c > 0 && dt > 0);
  if (eig) extreme_eigenvalues(J, n, &lmax, &lmin);
  const double cc = c > 0 ? c : (lmax > 0 ? 1.0 / lmax : 1.0);
  const double dd = dt > 0 ? dt : (lmax > 0 ? 1.25 * std::sqrt(2.0 / (1.0 - lmin / lmax)) : 1.25);
  std::lock_guard<std::mutex> lock(b->upload_mu);
  gsb_status s = ensure_ws(b);
  if (s != GSB_OK) return s;
  const int np = b->np[k];
  float* stage = reinterpret_cast<float*>(b->ws + b->off_stage);
  BHIP(hipStreamSynchronize(b->stream), "stream synchronise");
  BHIP(launch_fill_u32(reinterpret_cast<unsigned*>(stage), (size_t)np * np, 0u, b->stream), "clear staging");
  BHIP(hipMemcpy2DAsync(stage, (size_t)np * 4, J, (size_t)n * 4, (size_t)n * 4, n, hipMemcpyHostToDevice, b->stream),
       "upload J");
  BHIP(launch_encode_j(kFormFP8, true, stage, np, b->ws + b->off_j[k], b->stream), "encode J");
  BHIP(hipStreamSynchronize(b->stream), "stream synchronise");
  b->c[k] = cc;
  b->dt[k] = dd;
  b->lmax[k] = lmax;
  b->lmin[k] = lmin;
  b->have_eig[k] = eig ? 1 : 0;
  b->have_j[k] = 1;
  b->ran = false;
  drop_graph(b);
  return GSB_OK;
}

// An option value that must be an integer in [lo, hi]: false for anything else, NaN and
// infinities included (checked before the conversion, which is undefined out of range).
static bool int_option(double v, int lo, int hi, int* out) {
  if (!(v >= (double)lo && v <= (double)hi)) return false;
  const int iv = (int)v;
  if ((double)iv != v) return false;
  *out = iv;
  return true;
}

gsb_status gsb_batch_set(gsb_batch* b, int32_t k, int32_t option, double v) {
  set_last_error("");
  if (!b) return bfail(GSB_EINVAL, "batch is NULL");
  if (option == GSB_BATCH_OCCUPANCY) {
    if (k != -1) return bfail(GSB_EINVAL, "batch-wide option: pass k = -1");
    int iv = 0;
    if (!int_option(v, 0, 2, &iv)) return bfail(GSB_EINVAL, "GSB_BATCH_OCCUPANCY is 0, 1 or 2");
    if (iv) {
      gsb_status s = device_facts(b);
      if (s != GSB_OK) return s;
      if (b->grid[iv - 1] == 0) return bfail(GSB_EUNSUPPORTED, "this device does not run the kernel at that occupancy");
      b->occ = iv;
    }
    b->occ_fixed = iv;
    drop_graph(b);
    return GSB_OK;
  }
  if (option == GSB_BATCH_GRAPH || option == GSB_BATCH_INIT_MODE) {
    if (k != -1) return bfail(GSB_EINVAL, "batch-wide option: pass k = -1");
    int iv = 0;
    if (!int_option(v, -1, 1 << 20, &iv)) return bfail(GSB_EINVAL, "integer option");
    if (option == GSB_BATCH_GRAPH) {
      if (iv != 0 && iv != 1) return bfail(GSB_EINVAL, "GSB_BATCH_GRAPH is 0 or 1");
      b->use_graph = iv == 1;
    } else {
      if (iv < GSB_INIT_X || iv > GSB_INIT_PAIRS) return bfail(GSB_EINVAL, "unknown init mode");
      b->init_mode = iv;
    }
    drop_graph(b);
    return GSB_OK;
  }
  if (k < 0 || k >= b->count) return bfail(GSB_EINVAL, "instance index out of range");
  switch (option) {
    case GSB_BATCH_C:
    case GSB_BATCH_DT:
      if (!b->have_j[k]) return bfail(GSB_ESTATE, "set the coupling of the instance first");
      if (!std::isfinite(v) || v <= 0) return bfail(GSB_EINVAL, "value must be finite and > 0");
      (option == GSB_BATCH_C ? b->c : b->dt)[k] = v;
      drop_graph(b);
      return GSB_OK;
    case GSB_BATCH_TILE_ROWS: {
      int iv = 0;
      if (!int_option(v, 0, 256, &iv) || (iv != 0 && tile_index(iv) < 0))
        return bfail(GSB_EINVAL, "tile rows: 0, 64, 128 or 256");
      b->tile_fixed[k] = iv;
      drop_graph(b);
      return GSB_OK;
    }
    default:
      return bfail(GSB_EINVAL, "unknown or read-only option " + std::to_string(option));
  }
}

gsb_status gsb_batch_get(gsb_batch* b, int32_t k, int32_t option, double* v) {
  set_last_error("");
  if (!b || !v) return bfail(GSB_EINVAL, "NULL argument");
  if (option == GSB_BATCH_GRAPH) { *v = b->use_graph ? 1 : 0; return GSB_OK; }
  if (option == GSB_BATCH_INIT_MODE) { *v = b->init_mode; return GSB_OK; }
  if (option == GSB_BATCH_COUNT) { *v = b->count; return GSB_OK; }
  if (option == GSB_BATCH_REPLICAS) { *v = b->R; return GSB_OK; }
  if (option == GSB_BATCH_GRID) {
    gsb_status s = device_facts(b);
    if (s != GSB_OK) return s;
    *v = b->grid[b->occ - 1];
    return GSB_OK;
  }
  if (option == GSB_BATCH_OCCUPANCY) { *v = b->occ; return GSB_OK; }
  if (k < 0 || k >= b->count) return bfail(GSB_EINVAL, "instance index out of range");
  switch (option) {
    case GSB_BATCH_N: *v = b->n[k]; return GSB_OK;
    case GSB_BATCH_C:
    case GSB_BATCH_DT:
      if (!b->have_j[k]) return bfail(GSB_ESTATE, "the instance has no coupling yet");
      *v = (option == GSB_BATCH_C ? b->c : b->dt)[k];
      return GSB_OK;
    case GSB_BATCH_LAMBDA_MAX:
    case GSB_BATCH_LAMBDA_MIN:
      if (!b->have_eig[k]) return bfail(GSB_ESTATE, "eigenvalues not computed (c and dt were given)");
      *v = option == GSB_BATCH_LAMBDA_MAX ? b->lmax[k] : b->lmin[k];
      return GSB_OK;
    case GSB_BATCH_TILE_ROWS: {
      gsb_status s = device_facts(b);
      if (s != GSB_OK) return s;
      *v = choose_tile(b, k, b->occ);
      return GSB_OK;
    }
    case GSB_BATCH_STEP_US: {
      gsb_status s = device_facts(b);
      if (s != GSB_OK) return s;
      const int t = tile_index(choose_tile(b, k, b->occ));
      *v = t >= 0 ? b->us[b->occ - 1][t][k] : 0.0;
      return GSB_OK;
    }
    default:
      return bfail(GSB_EINVAL, "unknown option " + std::to_string(option));
  }
}

gsb_status gsb_batch_autotune(gsb_batch* b, int32_t variant, double A, int32_t trial_steps, uint64_t seed) {
  set_last_error("");
  gsb_status s = check_run_args(b, variant, A, trial_steps);
  if (s != GSB_OK) return s;
  s = device_facts(b);
  if (s != GSB_OK) return s;
  const bool discrete = variant == GSB_DSB || variant == GSB_GDSB;
  if (!b->ev0) {
    BHIP(hipEventCreate(&b->ev0), "event create");
    BHIP(hipEventCreate(&b->ev1), "event create");
  }
  std::vector<int> tiles(b->count);
  double best_ms = -1.0;
  int best_occ = b->occ;
  for (int occ = 1; occ <= 2; ++occ) {
    if ((b->occ_fixed && occ != b->occ_fixed) || b->grid[occ - 1] == 0) continue;
    b->occ = occ;
    const int cap = b->cap[occ - 1];
    for (int t = 0; t < 3; ++t) {
      bool any = false;
      for (int k = 0; k < b->count; ++k) {
        int bm = b->tile_fixed[k] ? b->tile_fixed[k] : kTiles[t];
        if (b->np[k] / bm > cap || b->np[k] < bm) bm = choose_tile(b, k, occ);  // keep the queue runnable
        tiles[k] = bm;
        any = any || bm == kTiles[t];
      }
      if (!any) continue;
      s = prepare(b, variant, A, trial_steps, seed, tiles.data(), true);
      if (s != GSB_OK) return s;
      s = enqueue_run(b, discrete, true, false, b->stream);
      if (s != GSB_OK) return s;
      s = check_status(b);
      if (s != GSB_OK) return s;
      const size_t nslots = (size_t)b->h_qoff[kBatchXcds + 1];
      std::vector<unsigned long long> clk(2 * nslots);
      BHIP(hipMemcpy(clk.data(), b->d_clk, clk.size() * 8, hipMemcpyDeviceToHost), "read clocks");
      // a gang runs from its last member's start to its last member's end; every slot
      // of the queue that served it was taken exactly once
      std::vector<double> worst(b->count, 0.0);
      for (size_t i = 0; i < nslots;) {
        const BatchSlot& sl = b->h_slots[i];
        const int k = sl.inst, w = b->h_inst[k].nb;
        unsigned long long s0 = 0, e0 = 0;
        bool served = true;
        for (int j = 0; j < w; ++j) {
          const unsigned long long a0 = clk[2 * (i + j)], a1 = clk[2 * (i + j) + 1];
          if (a1 == 0) served = false;
          s0 = std::max(s0, a0);
          e0 = std::max(e0, a1);
        }
        if (served && e0 > s0) worst[k] = std::max(worst[k], (double)(e0 - s0) / b->wall_hz * 1e6 / trial_steps);
        i += w;
      }
      for (int k = 0; k < b->count; ++k)
        if (tiles[k] == kTiles[t] && worst[k] > 0) b->us[occ - 1][t][k] = worst[k];
    }
    // the whole batch with this occupancy's fastest tiles, timed
    s = prepare(b, variant, A, trial_steps, seed, nullptr, false);
    if (s != GSB_OK) return s;
    s = enqueue_run(b, discrete, true, true, b->stream);
    if (s != GSB_OK) return s;
    s = check_status(b);
    if (s != GSB_OK) return s;
    float ms = 0;
    BHIP(hipEventElapsedTime(&ms, b->ev0, b->ev1), "event elapsed time");
    if (best_ms < 0 || ms < best_ms) { best_ms = ms; best_occ = occ; }
  }
  b->occ = best_occ;
  b->timed = false;
  b->ran = false;
  drop_graph(b);
  return GSB_OK;
}

gsb_status gsb_batch_run(gsb_batch* b, int32_t variant, double A, int32_t steps, uint64_t seed) {
  set_last_error("");
  gsb_status s = check_run_args(b, variant, A, steps);
  if (s != GSB_OK) return s;
  const bool discrete = variant == GSB_DSB || variant == GSB_GDSB;
  if (!b->ev0) {
    BHIP(hipEventCreate(&b->ev0), "event create");
    BHIP(hipEventCreate(&b->ev1), "event create");
  }
  const std::vector<double> key = {(double)variant, A, (double)steps, (double)(seed >> 32), (double)(seed & 0xFFFFFFFFu)};
  if (b->use_graph && b->gexec && key == b->graph_key) {
    BHIP(hipEventRecord(b->ev0, b->stream), "event record");
    BHIP(hipGraphLaunch(b->gexec, b->stream), "graph launch");
    BHIP(hipEventRecord(b->ev1, b->stream), "event record");
  } else {
    drop_graph(b);
    s = prepare(b, variant, A, steps, seed, nullptr, false);
    if (s != GSB_OK) return s;
    if (b->use_graph) {
      // One graph: starting states, cleared barriers, the persistent kernel (a plain
      // launch: the kernel itself checks that its grid is co-resident), energies.  The
      // barrier words are cleared by a fill kernel inside the graph.
      if (!b->capture_stream)
        BHIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking), "create capture stream");
      BHIP(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
      s = enqueue_run(b, discrete, false, false, b->capture_stream);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(b->capture_stream, &g);
      if (s != GSB_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
      }
      if (ec != hipSuccess) return bhip(ec, "end capture");
      b->graph = g;
      BHIP(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0), "graph instantiate");
      b->graph_key = key;
      BHIP(hipEventRecord(b->ev0, b->stream), "event record");
      BHIP(hipGraphLaunch(b->gexec, b->stream), "graph launch");
      BHIP(hipEventRecord(b->ev1, b->stream), "event record");
    } else {
      s = enqueue_run(b, discrete, true, true, b->stream);
      if (s != GSB_OK) return s;
    }
  }
  b->variant = variant;
  b->A = A;
  b->M = steps;
  b->seed = seed;
  b->ran = true;
  b->timed = true;
  return GSB_OK;
}

gsb_status gsb_batch_energy(gsb_batch* b, int32_t k, double* energies) {
  set_last_error("");
  if (!b || !energies) return bfail(GSB_EINVAL, "NULL argument");
  if (k < 0 || k >= b->count) return bfail(GSB_EINVAL, "instance index out of range");
  if (!b->ran) return bfail(GSB_ESTATE, "no run");
  BHIP(hipMemcpyAsync(energies, b->ws + b->off_E + (size_t)k * b->rp * 8, (size_t)b->R * 8, hipMemcpyDeviceToHost,
                      b->stream),
       "copy energies");
  return check_status(b);
}

gsb_status gsb_batch_best(gsb_batch* b, double* energy, int32_t* replica) {
  set_last_error("");
  if (!b) return bfail(GSB_EINVAL, "batch is NULL");
  if (!b->ran) return bfail(GSB_ESTATE, "no run");
  if (energy)
    BHIP(hipMemcpyAsync(energy, b->ws + b->off_be, (size_t)b->count * 8, hipMemcpyDeviceToHost, b->stream),
         "copy best");
  if (replica)
    BHIP(hipMemcpyAsync(replica, b->ws + b->off_bidx, (size_t)b->count * 4, hipMemcpyDeviceToHost, b->stream),
         "copy best");
  return check_status(b);
}

gsb_status gsb_batch_state(gsb_batch* b, int32_t k, float* x, float* y, float* p) {
  set_last_error("");
  if (!b) return bfail(GSB_EINVAL, "batch is NULL");
  if (k < 0 || k >= b->count) return bfail(GSB_EINVAL, "instance index out of range");
  if (!b->ran) return bfail(GSB_ESTATE, "no run");
  const size_t offs[3] = {b->off_x[k], b->off_y[k], b->off_p[k]};
  float* dst[3] = {x, y, p};
  const int n = b->n[k], np = b->np[k];
  for (int i = 0; i < 3; ++i)
    if (dst[i])
      BHIP(hipMemcpy2DAsync(dst[i], (size_t)n * 4, b->ws + offs[i], (size_t)np * 4, (size_t)n * 4, b->R,
                            hipMemcpyDeviceToHost, b->stream),
           "copy state");
  return check_status(b);
}

gsb_status gsb_batch_last_ms(gsb_batch* b, double* ms) {
  set_last_error("");
  if (!b || !ms) return bfail(GSB_EINVAL, "NULL argument");
  if (!b->timed) return bfail(GSB_ESTATE, "no timed run");
  BHIP(hipEventSynchronize(b->ev1), "event synchronise");
  float f = 0;
  BHIP(hipEventElapsedTime(&f, b->ev0, b->ev1), "event elapsed time");
  *ms = f;
  return GSB_OK;
}

}  // extern "C"
