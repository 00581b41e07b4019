// gsb_api.cpp -- the C ABI of libgsb (include/gsb.h): argument checking, instance
// set-up, workspace management and the launch sequence of the gfx950 kernels.
#include "../../include/gsb.h"
#include "gsb_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace gsb;

namespace {

thread_local std::string g_err;

gsb_status fail(gsb_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

gsb_status hip_fail(hipError_t e, const char* what) {
  return fail(GSB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                      \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// The status block of a run is 64 words: word 0 is the step kernels' barrier status, word
// kStateFlagWord the result of the device-side check of a state given by the caller.
constexpr int kStateFlagWord = 32;

int form_of(int precision) {
  switch (precision) {
    case GSB_PREC_FP8: return kFormFP8;
    case GSB_PREC_BF16X2: return kFormBF16X2;
    case GSB_PREC_FIX16: return kFormFIX16;
    default: return kFormFP32;
  }
}
size_t operand_elem_bytes(int form) {
  return (form == kFormFP8 || form == kFormFIX16) ? 1 : (form == kFormBF16X2 ? 2 : 4);
}

// ---- eigenvalue bounds of a symmetric matrix (App. A needs lambda_max and lambda_min) ----
// Lanczos with full reorthogonalisation, binary64; extreme Ritz values of the tridiagonal
// matrix by Sturm-sequence bisection.
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, int k, double x) {
  // number of eigenvalues of T_k smaller than x
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < k; ++i) {
    const double bb = (i > 0) ? b[i - 1] * b[i - 1] : 0.0;
    d = (a[i] - x) - (i > 0 ? bb / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0) ++cnt;
  }
  return cnt;
}

double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, int k, int idx) {
  double lo = 0, hi = 0;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(a, b, k, mid) > idx) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

void gsb::set_last_error(const char* msg) { g_err = msg; }

void gsb::extreme_eigenvalues(const float* J, int n, double* lmax, double* lmin) {
  if (n == 1) { *lmax = 0.0; *lmin = 0.0; return; }
  // a sparse J (at most a quarter of the entries nonzero) is multiplied in compressed rows
  size_t nnz = 0;
  for (size_t k = 0; k < (size_t)n * n; ++k) nnz += J[k] != 0.0f;
  const bool sparse = nnz * 4 <= (size_t)n * n;
  std::vector<size_t> row_ptr;
  std::vector<int> col;
  std::vector<float> val;
  if (sparse) {
    row_ptr.assign(n + 1, 0);
    col.reserve(nnz);
    val.reserve(nnz);
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < n; ++j) {
        const float v = J[(size_t)i * n + j];
        if (v != 0.0f) { col.push_back(j); val.push_back(v); }
      }
      row_ptr[i + 1] = col.size();
    }
  }
  const int kmax = std::min(n, 400);
  std::vector<std::vector<double>> V;
  std::vector<double> alpha, beta;
  std::vector<double> v(n), w(n);
  uint64_t s = 0x243F6A8885A308D3ull;  // fixed start vector
  double nrm = 0;
  for (int i = 0; i < n; ++i) {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    v[i] = (double)(z >> 11) * 0x1.0p-53 - 0.5;
    nrm += v[i] * v[i];
  }
  nrm = std::sqrt(nrm);
  for (auto& e : v) e /= nrm;
  double prev_max = 0, prev_min = 0;
  for (int k = 0; k < kmax; ++k) {
    V.push_back(v);
    for (int i = 0; i < n; ++i) {
      double acc = 0;
      if (sparse) {
        for (size_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) acc += (double)val[e] * v[col[e]];
      } else {
        const float* Ji = J + (size_t)i * n;
        for (int j = 0; j < n; ++j) acc += (double)Ji[j] * v[j];
      }
      w[i] = acc;
    }
    double a = 0;
    for (int i = 0; i < n; ++i) a += w[i] * v[i];
    alpha.push_back(a);
    for (int pass = 0; pass < 2; ++pass)
      for (const auto& u : V) {
        double d = 0;
        for (int i = 0; i < n; ++i) d += w[i] * u[i];
        for (int i = 0; i < n; ++i) w[i] -= d * u[i];
      }
    double bnorm = 0;
    for (int i = 0; i < n; ++i) bnorm += w[i] * w[i];
    bnorm = std::sqrt(bnorm);
    const int kk = k + 1;
    if ((kk % 10 == 0) || kk == kmax || bnorm < 1e-12) {
      const double emax = tridiag_eig(alpha, beta, kk, kk - 1);
      const double emin = tridiag_eig(alpha, beta, kk, 0);
      const double scale = std::max(std::fabs(emax), std::fabs(emin)) + 1e-300;
      if (bnorm < 1e-12 || (kk >= 20 && std::fabs(emax - prev_max) < 1e-13 * scale &&
                            std::fabs(emin - prev_min) < 1e-13 * scale) || kk == kmax) {
        *lmax = emax;
        *lmin = emin;
        return;
      }
      prev_max = emax;
      prev_min = emin;
    }
    beta.push_back(bnorm);
    for (int i = 0; i < n; ++i) v[i] = w[i] / bnorm;
  }
  *lmax = prev_max;
  *lmin = prev_min;
}

struct gsb_ctx {
  // instance
  uint64_t uid = 0;  // unique per context of the process (never reused)
  int n_user = 0, n = 0, np = 0, anc = -1;
  std::vector<float> J;  // n x n, row-major (with the ancilla row/column if any)
  bool pm1 = false;
  double c = 0;
  bool c_set = false;
  double lmax = 0, lmin = 0;
  bool eig_done = false;
  int precision = GSB_PREC_FP32;
  int init_mode = GSB_INIT_X;
  int kernel_pref = 0;  // GSB_OPT_STEP_KERNEL
  int grid_pad = 1;     // GSB_OPT_GRID_PAD
  int lle_from = 0;     // GSB_OPT_LLE_FROM
  hipStream_t stream = nullptr;
  // run
  bool inited = false;
  int variant = 0, schedule = 0, R = 0, rp = 0, M = 0, m = 0;
  double A = 0, dt = 0;
  uint64_t seed = 0;
  int chunk_rp = 0;
  int max_wg = 0;  // co-resident workgroups of the step kernel
  int kind = 0;
  // device memory
  void* ws_user = nullptr;
  size_t ws_user_bytes = 0;
  void* ws_own = nullptr;
  void* vjp_buf = nullptr;   // reverse pass: tape and cotangents (library-owned)
  size_t vjp_bytes = 0;
  size_t ws_own_bytes = 0;
  uint8_t* ws = nullptr;   // current workspace base
  size_t ws_bytes = 0;
  // carved buffers (valid for the current workspace and shape)
  float* j32 = nullptr;
  uint8_t* jf = nullptr;
  float* rtab = nullptr;
  float *X = nullptr, *Y = nullptr, *P = nullptr;
  uint8_t* Q = nullptr;
  size_t q_buf_bytes = 0;
  unsigned* sync = nullptr;
  unsigned* status = nullptr;
  double* partial = nullptr;
  double* E = nullptr;
  int* best_idx = nullptr;
  double* best_e = nullptr;
  int8_t* spins = nullptr;
  // bookkeeping of what the workspace holds
  bool j32_ready = false;
  int jf_form = -1;
  bool energy_valid = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  // pinned host staging for gsb_best's small results (copies into pageable memory would
  // each wait for the device)
  uint8_t* pinned = nullptr;
  size_t pinned_bytes = 0;
};

namespace {

struct Layout {
  size_t j32, jf, rtab, X, Y, P, Q, sync, status, partial, E, best, spins, total;
  size_t acol = 0, lg = 0, ext = 0;  // tangent mode only
  size_t q_buf_bytes;
  int chunk_rp;  // columns per launch
  int max_wg;    // co-resident workgroups of the step kernel
};

// Workspace of a run of R replicas over M steps.  Tangent mode (gsb_lle): binary32 form,
// generic kernel, two columns per replica (replica + tangent), plus the per-replica
// control strengths, log-norm sums and the extraction buffer.
gsb_status plan(gsb_ctx* c, int R, int M, Layout* L, int* kind_out, bool tangent = false) {
  const int form = tangent ? (int)kFormFP32 : form_of(c->precision);
  const int np = c->np;
  const int rp = (R + kRepPad - 1) / kRepPad * kRepPad;
  const int cols = tangent ? 2 * rp : rp;
  const int kind = tangent ? (int)kKindGeneric : choose_kind(form, np, c->kernel_pref);
  const int bm = tile_rows_kind(kind), bn = tile_cols_kind(kind);
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1)
    return fail(GSB_EDEVICE, "no HIP device");
  const int max_wg = max_coresident_workgroups(form, kind, np, tangent);
  if (max_wg < 1) return fail(GSB_EDEVICE, "occupancy query failed for the step kernel");
  const int nb = np / bm;
  const int max_groups = max_wg / nb;
  if (max_groups < 1)
    return fail(GSB_EUNSUPPORTED, "n too large for one co-resident replica group on this device");
  const int chunk_rp = std::min(cols, max_groups * bn / kRepPad * kRepPad);
  if (chunk_rp < kRepPad)
    return fail(GSB_EUNSUPPORTED, "n too large for one co-resident replica block on this device");
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L->j32 = take((size_t)np * np * 4);
  L->jf = take((size_t)np * np * operand_elem_bytes(form));  // FP4 J uses half of it
  L->rtab = take((size_t)M * 4);
  L->X = take((size_t)cols * np * 4);
  L->Y = take((size_t)cols * np * 4);
  L->P = take((size_t)cols * np * 4);
  L->q_buf_bytes = (size_t)chunk_rp * np * operand_elem_bytes(form) * operand_planes(form);
  L->Q = take(2 * L->q_buf_bytes);
  L->sync = take(sync_words(chunk_rp / bn) * 4);
  L->status = take(256);
  L->partial = take(std::max(energy_partial_doubles(np, rp) * 8, energy_fp4_scratch_bytes(np, rp)));
  L->E = take((size_t)rp * 8);
  L->best = take(256);
  L->spins = take((size_t)std::max(rp, 1) * c->n_user + 256);
  if (tangent) {
    L->acol = take((size_t)rp * 4);
    L->lg = take((size_t)rp * 8);
    L->ext = take((size_t)6 * R * c->n * 4);
  }
  L->total = off;
  L->chunk_rp = chunk_rp;
  L->max_wg = max_wg;
  *kind_out = kind;
  return GSB_OK;
}

gsb_status ensure_workspace(gsb_ctx* c, size_t need) {
  uint8_t* base = nullptr;
  size_t bytes = 0;
  if (c->ws_user) {
    if (c->ws_user_bytes < need)
      return fail(GSB_ENOMEM, "bound workspace has " + std::to_string(c->ws_user_bytes) + " bytes, run needs " +
                                  std::to_string(need));
    base = static_cast<uint8_t*>(c->ws_user);
    bytes = c->ws_user_bytes;
  } else {
    if (c->ws_own_bytes < need) {
      if (c->ws_own) {
        const hipError_t es = hipStreamSynchronize(c->stream);
        const hipError_t ef = hipFree(c->ws_own);
        c->ws_own = nullptr;
        c->ws_own_bytes = 0;
        if (es != hipSuccess || ef != hipSuccess)
          return fail(GSB_EDEVICE, std::string("releasing the old workspace: ") +
                                       hipGetErrorString(es != hipSuccess ? es : ef));
      }
      void* p = nullptr;
      if (hipMalloc(&p, need) != hipSuccess)
        return fail(GSB_ENOMEM, "device allocation of " + std::to_string(need) + " bytes failed");
      c->ws_own = p;
      c->ws_own_bytes = need;
    }
    base = static_cast<uint8_t*>(c->ws_own);
    bytes = c->ws_own_bytes;
  }
  if (base != c->ws || bytes != c->ws_bytes) {
    c->ws = base;
    c->ws_bytes = bytes;
    c->j32_ready = false;
    c->jf_form = -1;
  }
  return GSB_OK;
}

gsb_status ensure_eig(gsb_ctx* c) {
  if (!c->eig_done) {
    extreme_eigenvalues(c->J.data(), c->n, &c->lmax, &c->lmin);
    c->eig_done = true;
  }
  return GSB_OK;
}

gsb_status check_status_word(gsb_ctx* c) {
  unsigned st = 0;
  HIP_TRY(hipMemcpyAsync(&st, c->status, 4, hipMemcpyDeviceToHost, c->stream), "status read");
  HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronise");
  if (st != 0) return fail(GSB_EDEVICE, "step kernel: a replica-group barrier timed out");
  return GSB_OK;
}

gsb_status compute_energy(gsb_ctx* c) {
  if (c->energy_valid) return GSB_OK;
  if (c->pm1 && c->jf_form == kFormFP8 * 2 + 1) {
    // J in {0, +-1} is on the device as FP4: the exact integer energy runs on MFMA
    HIP_TRY(launch_energy_fp4(c->jf, c->np, c->rp, c->R, c->X, c->partial, c->E, c->stream), "energy kernel");
  } else {
    HIP_TRY(launch_energy(c->j32, c->n, c->np, c->rp, c->R, c->X, c->partial, c->E, c->stream), "energy kernel");
  }
  c->energy_valid = true;
  return GSB_OK;
}

}  // namespace

extern "C" {

const char* gsb_last_error(void) { return g_err.c_str(); }

gsb_status gsb_encode_operand(int32_t precision, int32_t discrete, const float* x, int64_t count, void* out,
                              void* stream) {
  g_err.clear();
  if (precision < GSB_PREC_FP32 || precision > GSB_PREC_FIX16) return fail(GSB_EINVAL, "unknown precision");
  if (count < 0) return fail(GSB_EINVAL, "count must be >= 0");
  if (count == 0) return GSB_OK;
  if (!x || !out) return fail(GSB_EINVAL, "x and out must be device pointers");
  if (((uintptr_t)x & 3u) != 0 || ((uintptr_t)out & 3u) != 0) return fail(GSB_EINVAL, "x and out must be 4-byte aligned");
  const size_t bytes = (size_t)count * (size_t)(precision == GSB_PREC_FP8 ? 1 : precision == GSB_PREC_FIX16 ? 2 : 4);
  const uintptr_t xb = (uintptr_t)x, xe = xb + (size_t)count * 4, ob = (uintptr_t)out, oe = ob + bytes;
  if (xb < oe && ob < xe) return fail(GSB_EINVAL, "x and out overlap");
  HIP_TRY(launch_encode_operand(form_of(precision), discrete != 0, x, (size_t)count, out,
                                static_cast<hipStream_t>(stream)),
          "operand encoder launch");
  return GSB_OK;
}
const char* gsb_version(void) { return "gsb-mi355x 0.1 (gfx950)"; }

gsb_status gsb_create(const float* J, const float* h, int32_t n, gsb_ctx** out) {
  g_err.clear();
  if (!out) return fail(GSB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!J) return fail(GSB_EINVAL, "J is NULL");
  if (n < 1 || n > 16384) return fail(GSB_EINVAL, "n must be in [1, 16384]");
  for (size_t k = 0; k < (size_t)n * n; ++k)
    if (!std::isfinite(J[k])) return fail(GSB_ENONFINITE, "J has a non-finite entry");
  for (int i = 0; i < n; ++i) {
    if (J[(size_t)i * n + i] != 0.0f) return fail(GSB_EDIAG, "J_ii != 0 at i = " + std::to_string(i));
    for (int j = i + 1; j < n; ++j)
      if (J[(size_t)i * n + j] != J[(size_t)j * n + i])
        return fail(GSB_ENOTSYM, "J_ij != J_ji at (" + std::to_string(i) + ", " + std::to_string(j) + ")");
  }
  bool field = false;
  if (h) {
    for (int i = 0; i < n; ++i) {
      if (!std::isfinite(h[i])) return fail(GSB_ENONFINITE, "h has a non-finite entry");
      if (h[i] != 0.0f) field = true;
    }
  }
  gsb_ctx* c = new (std::nothrow) gsb_ctx;
  if (!c) return fail(GSB_ENOMEM, "host allocation failed");
  static std::atomic<uint64_t> next_uid{1};
  c->uid = next_uid.fetch_add(1);
  c->n_user = n;
  c->n = field ? n + 1 : n;
  c->anc = field ? n : -1;
  c->np = (c->n + kRowPad - 1) / kRowPad * kRowPad;
  try {
    c->J.assign((size_t)c->n * c->n, 0.0f);
  } catch (...) {
    delete c;
    return fail(GSB_ENOMEM, "host allocation failed");
  }
  for (int i = 0; i < n; ++i) std::memcpy(&c->J[(size_t)i * c->n], &J[(size_t)i * n], sizeof(float) * n);
  if (field)
    for (int i = 0; i < n; ++i) {
      c->J[(size_t)i * c->n + n] = h[i];
      c->J[(size_t)n * c->n + i] = h[i];
    }
  c->pm1 = true;
  for (float v : c->J)
    if (!(v == 0.0f || v == 1.0f || v == -1.0f)) { c->pm1 = false; break; }
  c->precision = c->pm1 ? GSB_PREC_FP8 : GSB_PREC_BF16X2;
  *out = c;
  return GSB_OK;
}

void gsb_destroy(gsb_ctx* c) {
  if (!c) return;
  // Teardown cannot report errors; a failed synchronisation or free is ignored here.
  (void)hipStreamSynchronize(c->stream);  // also for copies still reading the context's J
  if (c->ws_own) (void)hipFree(c->ws_own);
  if (c->vjp_buf) (void)hipFree(c->vjp_buf);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}

gsb_status gsb_set(gsb_ctx* c, int32_t option, double v) {
  g_err.clear();
  if (!c) return fail(GSB_EINVAL, "ctx is NULL");
  switch (option) {
    case GSB_OPT_C:
      if (!std::isfinite(v) || v <= 0) return fail(GSB_EINVAL, "c must be finite and > 0");
      c->c = v;
      c->c_set = true;
      return GSB_OK;
    case GSB_OPT_PRECISION: {
      if (!(v >= -1.0 && v <= 64.0)) return fail(GSB_EINVAL, "unknown precision");  // also NaN
      const int p = (int)v;
      if ((double)p != v || p < GSB_PREC_FP32 || p > GSB_PREC_FIX16) return fail(GSB_EINVAL, "unknown precision");
      if ((p == GSB_PREC_FP8 || p == GSB_PREC_FIX16) && !c->pm1)
        return fail(GSB_EUNSUPPORTED, "FP8 and FIX16 precisions need J entries in {0, +1, -1}");
      if (p != c->precision) {
        c->precision = p;
        c->inited = false;  // operand buffers change shape
      }
      return GSB_OK;
    }
    case GSB_OPT_INIT_MODE: {
      if (!(v >= -1.0 && v <= 64.0)) return fail(GSB_EINVAL, "unknown init mode");  // also NaN
      const int mm = (int)v;
      if ((double)mm != v || mm < GSB_INIT_X || mm > GSB_INIT_PAIRS) return fail(GSB_EINVAL, "unknown init mode");
      c->init_mode = mm;
      return GSB_OK;
    }
    case GSB_OPT_STEP_KERNEL: {
      if (!(v >= 0.0 && v <= 2.0)) return fail(GSB_EINVAL, "step kernel must be 0, 1 or 2");  // also NaN
      const int k = (int)v;
      if ((double)k != v || k < 0 || k > 2) return fail(GSB_EINVAL, "step kernel must be 0, 1 or 2");
      if (k != c->kernel_pref) {
        c->kernel_pref = k;
        c->inited = false;  // the workspace layout follows the kernel
      }
      return GSB_OK;
    }
    case GSB_OPT_GRID_PAD: {
      if (!(v == 0.0 || v == 1.0)) return fail(GSB_EINVAL, "grid padding must be 0 or 1");  // also NaN
      c->grid_pad = (int)v;
      return GSB_OK;
    }
    case GSB_OPT_LLE_FROM: {
      if (!(v >= 0.0 && v <= (double)(1 << 24)) || v != std::floor(v))  // also NaN
        return fail(GSB_EINVAL, "the LLE window start must be an integer step in [0, 2^24]");
      c->lle_from = (int)v;
      return GSB_OK;
    }
    default:
      return fail(GSB_EINVAL, "unknown or read-only option " + std::to_string(option));
  }
}

gsb_status gsb_get(gsb_ctx* c, int32_t option, double* v) {
  g_err.clear();
  if (!c || !v) return fail(GSB_EINVAL, "NULL argument");
  switch (option) {
    case GSB_OPT_C:
      if (!c->c_set) {
        ensure_eig(c);
        *v = c->lmax > 0 ? 1.0 / c->lmax : 1.0;
      } else {
        *v = c->c;
      }
      return GSB_OK;
    case GSB_OPT_PRECISION: *v = c->precision; return GSB_OK;
    case GSB_OPT_INIT_MODE: *v = c->init_mode; return GSB_OK;
    case GSB_OPT_STEP_KERNEL: *v = c->kernel_pref; return GSB_OK;
    case GSB_OPT_GRID_PAD: *v = c->grid_pad; return GSB_OK;
    case GSB_OPT_LLE_FROM: *v = c->lle_from; return GSB_OK;
    case GSB_OPT_LAMBDA_MAX: ensure_eig(c); *v = c->lmax; return GSB_OK;
    case GSB_OPT_LAMBDA_MIN: ensure_eig(c); *v = c->lmin; return GSB_OK;
    case GSB_OPT_N: *v = c->n_user; return GSB_OK;
    case GSB_OPT_N_DYN: *v = c->n; return GSB_OK;
    case GSB_OPT_STEP: *v = c->inited ? c->m : 0; return GSB_OK;
    case GSB_OPT_REPLICAS: *v = c->inited ? c->R : 0; return GSB_OK;
    case GSB_OPT_DT_STABLE:
      ensure_eig(c);
      // eq. (13): dt = D_t sqrt(2 / (1 - lambda_min / lambda_max)), D_t = 1.25
      *v = (c->lmax > 0) ? 1.25 * std::sqrt(2.0 / (1.0 - c->lmin / c->lmax)) : 1.25;
      return GSB_OK;
    default:
      return fail(GSB_EINVAL, "unknown option " + std::to_string(option));
  }
}

gsb_status gsb_set_stream(gsb_ctx* c, void* stream) {
  g_err.clear();
  if (!c) return fail(GSB_EINVAL, "ctx is NULL");
  c->stream = static_cast<hipStream_t>(stream);
  return GSB_OK;
}

gsb_status gsb_workspace_size(gsb_ctx* c, int32_t replicas, int32_t steps, size_t* bytes) {
  g_err.clear();
  if (!c || !bytes) return fail(GSB_EINVAL, "NULL argument");
  if (replicas < 1 || steps < 1) return fail(GSB_EINVAL, "replicas and steps must be >= 1");
  Layout L;
  int kind;
  gsb_status s = plan(c, replicas, steps, &L, &kind);
  if (s != GSB_OK) return s;
  *bytes = L.total;
  return GSB_OK;
}

gsb_status gsb_bind_workspace(gsb_ctx* c, void* ptr, size_t bytes) {
  g_err.clear();
  if (!c) return fail(GSB_EINVAL, "ctx is NULL");
  if (ptr && ((uintptr_t)ptr & 255)) return fail(GSB_EINVAL, "workspace must be 256-byte aligned");
  c->ws_user = ptr;
  c->ws_user_bytes = ptr ? bytes : 0;
  c->inited = false;
  c->ws = nullptr;
  c->ws_bytes = 0;
  c->j32_ready = false;
  c->jf_form = -1;
  return GSB_OK;
}

namespace {

// Point the context's buffers into the workspace laid out by `L`, upload and encode J
// for product form `form` if the workspace does not hold it yet, and write the schedule
// table r_m = 1 / (M - m) (eqs. (6), (7)), binary64 rounded once.
gsb_status carve_and_prepare(gsb_ctx* c, const Layout& L, int kind, int form, int schedule, int steps) {
  uint8_t* b = c->ws;
  const bool j32_moved = reinterpret_cast<float*>(b + L.j32) != c->j32;
  c->j32 = reinterpret_cast<float*>(b + L.j32);
  if (reinterpret_cast<uint8_t*>(b + L.jf) != c->jf) c->jf_form = -1;
  c->jf = b + L.jf;
  if (j32_moved) { c->j32_ready = false; c->jf_form = -1; }
  c->rtab = reinterpret_cast<float*>(b + L.rtab);
  c->X = reinterpret_cast<float*>(b + L.X);
  c->Y = reinterpret_cast<float*>(b + L.Y);
  c->P = reinterpret_cast<float*>(b + L.P);
  c->Q = b + L.Q;
  c->q_buf_bytes = L.q_buf_bytes;
  c->sync = reinterpret_cast<unsigned*>(b + L.sync);
  c->status = reinterpret_cast<unsigned*>(b + L.status);
  c->partial = reinterpret_cast<double*>(b + L.partial);
  c->E = reinterpret_cast<double*>(b + L.E);
  c->best_idx = reinterpret_cast<int*>(b + L.best);
  c->best_e = reinterpret_cast<double*>(b + L.best + 8);
  c->spins = reinterpret_cast<int8_t*>(b + L.spins);
  c->chunk_rp = L.chunk_rp;
  c->max_wg = L.max_wg;
  c->kind = kind;
  if (!c->j32_ready) {
    HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(c->j32), (size_t)c->np * c->np, 0u, c->stream), "clear J");
    HIP_TRY(hipMemcpy2DAsync(c->j32, (size_t)c->np * 4, c->J.data(), (size_t)c->n * 4, (size_t)c->n * 4, c->n,
                             hipMemcpyHostToDevice, c->stream),
            "upload J");
    c->j32_ready = true;
    c->jf_form = -1;
  }
  const bool j_fp4 = form == kFormFP8;  // the FP8 product reads J as FP4 (exact for 0, +-1)
  const int jcode = form * 2 + (j_fp4 ? 1 : 0);
  if (c->jf_form != jcode) {
    HIP_TRY(launch_encode_j(form, j_fp4, c->j32, c->np, c->jf, c->stream), "encode J");
    c->jf_form = jcode;
  }
  // the schedule table is computed on the device (no host source to keep alive, so a run
  // needs no synchronisation before its step kernels are queued)
  HIP_TRY(launch_rtab(c->rtab, steps, schedule == GSB_SCHED_LINEAR, c->stream), "schedule table");
  HIP_TRY(launch_fill_u32(c->status, 64, 0u, c->stream), "clear status");
  return GSB_OK;
}

// Persistent step launches for steps [m0, m1) over `cols` columns of the current
// buffers, in chunks of c->chunk_rp columns.
gsb_status launch_chunks(gsb_ctx* c, int form, int cols, bool discrete, float A, const float* acol, int m0, int m1,
                         bool tangent, float* X = nullptr, float* Y = nullptr, float* P = nullptr,
                         float* tape = nullptr, bool adjoint = false, int chunk = 0) {
  if (!X) { X = c->X; Y = c->Y; P = c->P; }
  if (chunk <= 0) chunk = c->chunk_rp;
  for (int r0 = 0; r0 < cols; r0 += chunk) {
    const int rcount = std::min(chunk, cols - r0);
    StepArgs a;
    a.n = c->n;
    a.np = c->np;
    a.rp = rcount;
    a.groups = rcount / tile_cols_kind(c->kind);
    a.nb = c->np / tile_rows_kind(c->kind);
    a.discrete = discrete ? 1 : 0;
    a.m_begin = m0;
    a.m_end = m1;
    a.A = A;
    a.dt = (float)c->dt;
    a.cdt = (float)(c->c * c->dt);
    a.acol = acol ? acol + r0 / 2 : nullptr;  // tangent mode: 2 columns per replica
    a.rtab = c->rtab;
    a.jf = c->jf;
    a.q = c->Q;
    a.q_buf_bytes = (size_t)rcount * c->np * operand_elem_bytes(form) * operand_planes(form);
    a.x = X + (size_t)r0 * c->np;
    a.y = Y + (size_t)r0 * c->np;
    a.p = P + (size_t)r0 * c->np;
    a.sync = c->sync;
    a.status = c->status;
    a.tape = tape ? tape + (size_t)r0 * c->np : nullptr;
    a.tape_arr = (size_t)cols * c->np;
    // pad the grid to whole XCD rounds of groups when that still fits (kernel launches only)
    if (!adjoint) {
      const int gp = (a.groups + 7) / 8 * 8;
      a.gpad = (c->grid_pad && c->max_wg > 0 && gp * a.nb <= c->max_wg) ? gp : a.groups;
    }
    HIP_TRY(launch_fill_u32(c->sync, sync_words(a.groups), 0u, c->stream), "clear sync");
    if (adjoint) {
      HIP_TRY(launch_adjoint(a, c->stream), "adjoint kernel launch");
    } else {
      HIP_TRY(launch_steps(form, c->kind, a, c->stream, tangent), "step kernel launch");
    }
  }
  return GSB_OK;
}

}  // namespace

namespace {

// Arguments of a run (gsb_init, gsb_run_noalloc); sets c = 1/lambda_max (App. A) if unset.
gsb_status check_run_args(gsb_ctx* c, int32_t variant, int32_t schedule, double A, double dt, int32_t replicas,
                          int32_t steps) {
  if (!c) return fail(GSB_EINVAL, "ctx is NULL");
  if (variant < GSB_BSB || variant > GSB_GDSB) return fail(GSB_EINVAL, "unknown variant");
  if (schedule < GSB_SCHED_LINEAR || schedule > GSB_SCHED_CONSTANT) return fail(GSB_EINVAL, "unknown schedule");
  if (!std::isfinite(A) || A < 0) return fail(GSB_EINVAL, "control strength must be finite and >= 0");
  if (!std::isfinite(dt) || dt <= 0) return fail(GSB_EINVAL, "dt must be finite and > 0");
  if (replicas < 1 || replicas > (1 << 20)) return fail(GSB_EINVAL, "replicas must be in [1, 2^20]");
  if (steps < 1 || steps > (1 << 24)) return fail(GSB_EINVAL, "steps must be in [1, 2^24]");
  if ((c->precision == GSB_PREC_FP8 || c->precision == GSB_PREC_FIX16) && !c->pm1)
    return fail(GSB_EUNSUPPORTED, "FP8 and FIX16 precisions need J in {0, +-1}");
  if (!c->c_set) {
    ensure_eig(c);
    c->c = c->lmax > 0 ? 1.0 / c->lmax : 1.0;  // App. A: c = 1 / lambda_max
  }
  return GSB_OK;
}

}  // namespace

gsb_status gsb_init(gsb_ctx* c, int32_t variant, int32_t schedule, double A, double dt, int32_t replicas,
                    int32_t steps, uint64_t seed) {
  g_err.clear();
  gsb_status s0 = check_run_args(c, variant, schedule, A, dt, replicas, steps);
  if (s0 != GSB_OK) return s0;
  Layout L;
  int kind;
  gsb_status s = plan(c, replicas, steps, &L, &kind);
  if (s != GSB_OK) return s;
  s = ensure_workspace(c, L.total);
  if (s != GSB_OK) return s;
  const int form = form_of(c->precision);
  const int rp = (replicas + kRepPad - 1) / kRepPad * kRepPad;
  s = carve_and_prepare(c, L, kind, form, schedule, steps);
  if (s != GSB_OK) return s;
  // the only host source of these copies is the context's own J, which lives as long as
  // the context (gsb_destroy synchronises), so nothing here waits for the device
  HIP_TRY(launch_init_state(c->n, c->np, rp, seed, c->init_mode, c->X, c->Y, c->P, c->stream), "init state");
  c->variant = variant;
  c->schedule = schedule;
  c->A = (variant == GSB_GBSB || variant == GSB_GDSB) ? A : 0.0;
  c->dt = dt;
  c->R = replicas;
  c->rp = rp;
  c->M = steps;
  c->m = 0;
  c->seed = seed;
  c->inited = true;
  c->energy_valid = false;
  c->timed = false;
  return GSB_OK;
}

gsb_status gsb_step(gsb_ctx* c, int32_t count) {
  g_err.clear();
  if (!c) return fail(GSB_EINVAL, "ctx is NULL");
  if (!c->inited) return fail(GSB_ESTATE, "no run: call gsb_init or gsb_run first");
  if (count < 0 || c->m + count > c->M) return fail(GSB_EINVAL, "step count beyond the schedule length M");
  if (count == 0) return GSB_OK;
  const int form = form_of(c->precision);
  if (!c->ev0) {
    HIP_TRY(hipEventCreate(&c->ev0), "event create");
    HIP_TRY(hipEventCreate(&c->ev1), "event create");
  }
  HIP_TRY(hipEventRecord(c->ev0, c->stream), "event record");
  gsb_status st = launch_chunks(c, form, c->rp, c->variant == GSB_DSB || c->variant == GSB_GDSB, (float)c->A,
                                nullptr, c->m, c->m + count, false);
  if (st != GSB_OK) return st;
  HIP_TRY(hipEventRecord(c->ev1, c->stream), "event record");
  c->timed = true;
  c->m += count;
  c->energy_valid = false;
  return GSB_OK;
}

gsb_status gsb_run(gsb_ctx* c, int32_t variant, int32_t schedule, double A, double dt, int32_t replicas,
                   int32_t steps, uint64_t seed) {
  gsb_status s = gsb_init(c, variant, schedule, A, dt, replicas, steps, seed);
  if (s != GSB_OK) return s;
  s = gsb_step(c, steps);
  if (s != GSB_OK) return s;
  return compute_energy(c);
}

// ---- allocation-free run ---------------------------------------------------------------
// Every device buffer of a gsb_run_noalloc call lives in `scratch`: one copy per device,
// which the library holds from its load onto that device until the process ends.  Host
// code never passes the array's name as an address: each device's copy is located once,
// at the entry point's first call on that device (with that device current), and that
// address is what the kernels and copies receive.
namespace {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kNoAllocMaxDevices = 64;

struct ScratchSlot {
  uint8_t* ptr = nullptr;  // this device's copy of `scratch`
  uint64_t j_owner = 0;    // uid of the context whose J the array holds (0: none)
  int j_form = -1;         // jf_form code of that context's encoded J there
};
std::mutex g_scratch_mu;
ScratchSlot g_scratch[kNoAllocMaxDevices];

}  // namespace

static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

gsb_status gsb_run_noalloc(gsb_ctx* c, int32_t variant, int32_t schedule, double A, double dt, int32_t replicas,
                           int32_t steps, uint64_t seed, float* x, double* energies) {
  g_err.clear();
  gsb_status s = check_run_args(c, variant, schedule, A, dt, replicas, steps);
  if (s != GSB_OK) return s;
  if (!x || !energies) return fail(GSB_EINVAL, "x and energies must be device pointers");
  if (((uintptr_t)x & 3u) != 0 || ((uintptr_t)energies & 7u) != 0)
    return fail(GSB_EINVAL, "x must be 4-byte and energies 8-byte aligned");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "current device");
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return fail(GSB_EUNSUPPORTED, "device index beyond the " + std::to_string(kNoAllocMaxDevices) +
                                      " the allocation-free entry point tracks");
  uint8_t* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev].ptr) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "locating the scratch array");
      g_scratch[dev].ptr = static_cast<uint8_t*>(p);
    }
    base = g_scratch[dev].ptr;
  }
  Layout L;
  int kind;
  s = plan(c, replicas, steps, &L, &kind);
  if (s != GSB_OK) return s;
  if (L.total > kNoAllocBytes)
    return fail(GSB_EINVAL, "the run needs " + std::to_string(L.total) + " bytes of device memory; an allocation-free "
                            "run has " + std::to_string(kNoAllocBytes) + " (use fewer replicas or steps, or gsb_run)");
  // The context's own workspace stays as it is; for this call its buffers point into the
  // array.  J is uploaded and encoded unless this context's J is still there.
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    const bool mine = g_scratch[dev].j_owner == c->uid;
    c->j32_ready = mine;
    c->jf_form = mine ? g_scratch[dev].j_form : -1;
    g_scratch[dev].j_owner = 0;  // rewritten below
  }
  c->ws = base;
  c->ws_bytes = kNoAllocBytes;
  c->j32 = reinterpret_cast<float*>(base + L.j32);
  c->jf = base + L.jf;
  c->inited = false;
  auto detach = [&](gsb_status st) {
    {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      if (st == GSB_OK && c->j32_ready) {
        g_scratch[dev].j_owner = c->uid;
        g_scratch[dev].j_form = c->jf_form;
      }
    }
    c->ws = nullptr;
    c->ws_bytes = 0;
    c->j32_ready = false;
    c->jf_form = -1;
    c->inited = false;
    c->energy_valid = false;
    c->timed = false;
    return st;
  };
#define NOALLOC_TRY(expr, what)                              \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return detach(hip_fail(e_, what)); \
  } while (0)
  const int form = form_of(c->precision);
  const int rp = (replicas + kRepPad - 1) / kRepPad * kRepPad;
  s = carve_and_prepare(c, L, kind, form, schedule, steps);
  if (s != GSB_OK) return detach(s);
  c->variant = variant;
  c->schedule = schedule;
  c->A = (variant == GSB_GBSB || variant == GSB_GDSB) ? A : 0.0;
  c->dt = dt;
  c->R = replicas;
  c->rp = rp;
  c->M = steps;
  c->m = 0;
  c->seed = seed;
  c->energy_valid = false;
  NOALLOC_TRY(launch_init_state(c->n, c->np, rp, seed, c->init_mode, c->X, c->Y, c->P, c->stream), "init state");
  s = launch_chunks(c, form, rp, variant == GSB_DSB || variant == GSB_GDSB, (float)c->A, nullptr, 0, steps, false);
  if (s != GSB_OK) return detach(s);
  s = compute_energy(c);
  if (s != GSB_OK) return detach(s);
  NOALLOC_TRY(hipMemcpy2DAsync(x, (size_t)c->n * 4, c->X, (size_t)c->np * 4, (size_t)c->n * 4, replicas,
                               hipMemcpyDeviceToDevice, c->stream),
              "copy x");
  NOALLOC_TRY(hipMemcpyAsync(energies, c->E, (size_t)replicas * 8, hipMemcpyDeviceToDevice, c->stream),
              "copy energies");
#undef NOALLOC_TRY
  return detach(check_status_word(c));
}

gsb_status gsb_energy(gsb_ctx* c, double* energies) {
  g_err.clear();
  if (!c || !energies) return fail(GSB_EINVAL, "NULL argument");
  if (!c->inited) return fail(GSB_ESTATE, "no run");
  gsb_status s = compute_energy(c);
  if (s != GSB_OK) return s;
  HIP_TRY(hipMemcpyAsync(energies, c->E, (size_t)c->R * 8, hipMemcpyDeviceToHost, c->stream), "copy energies");
  return check_status_word(c);
}

gsb_status gsb_best(gsb_ctx* c, int8_t* spins, double* energy, int32_t* replica) {
  g_err.clear();
  if (!c) return fail(GSB_EINVAL, "ctx is NULL");
  if (!c->inited) return fail(GSB_ESTATE, "no run");
  gsb_status s = compute_energy(c);
  if (s != GSB_OK) return s;
  HIP_TRY(launch_best(c->E, c->R, c->best_idx, c->best_e, c->stream), "best kernel");
  HIP_TRY(launch_spins(c->X, c->n_user, c->np, 0, 1, c->anc, c->best_idx, c->spins, c->stream), "spins kernel");
  // index and energy (adjacent on the device), the status word and the spins go to pinned
  // staging in one batch of copies and one synchronisation
  const size_t need = 64 + (size_t)c->n_user;
  if (c->pinned_bytes < need) {
    if (c->pinned) {
      HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronise");
      HIP_TRY(hipHostFree(c->pinned), "release staging");
      c->pinned = nullptr;
      c->pinned_bytes = 0;
    }
    void* h = nullptr;
    if (hipHostMalloc(&h, need, hipHostMallocDefault) != hipSuccess) return fail(GSB_ENOMEM, "pinned staging");
    c->pinned = static_cast<uint8_t*>(h);
    c->pinned_bytes = need;
  }
  uint8_t* h = c->pinned;
  HIP_TRY(hipMemcpyAsync(h, c->best_idx, 16, hipMemcpyDeviceToHost, c->stream), "copy best");
  HIP_TRY(hipMemcpyAsync(h + 16, c->status, 4, hipMemcpyDeviceToHost, c->stream), "status read");
  if (spins) HIP_TRY(hipMemcpyAsync(h + 64, c->spins, (size_t)c->n_user, hipMemcpyDeviceToHost, c->stream), "copy spins");
  HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronise");
  unsigned st = 0;
  std::memcpy(&st, h + 16, 4);
  if (st != 0) return fail(GSB_EDEVICE, "step kernel: a replica-group barrier timed out");
  int bi = 0;
  double be = 0;
  std::memcpy(&bi, h, 4);
  std::memcpy(&be, h + 8, 8);
  if (spins) std::memcpy(spins, h + 64, (size_t)c->n_user);
  if (energy) *energy = be;
  if (replica) *replica = bi;
  return GSB_OK;
}

gsb_status gsb_spins(gsb_ctx* c, int8_t* spins) {
  g_err.clear();
  if (!c || !spins) return fail(GSB_EINVAL, "NULL argument");
  if (!c->inited) return fail(GSB_ESTATE, "no run");
  HIP_TRY(launch_spins(c->X, c->n_user, c->np, 0, c->R, c->anc, nullptr, c->spins, c->stream), "spins kernel");
  HIP_TRY(hipMemcpyAsync(spins, c->spins, (size_t)c->R * c->n_user, hipMemcpyDeviceToHost, c->stream),
          "copy spins");
  return check_status_word(c);
}

namespace {

// The state of the current run into caller arrays [R][n] (host or device, by `kind`).
gsb_status state_out(gsb_ctx* c, float* x, float* y, float* p, int32_t* m, hipMemcpyKind kind) {
  if (!c) return fail(GSB_EINVAL, "ctx is NULL");
  if (!c->inited) return fail(GSB_ESTATE, "no run");
  float* src[3] = {c->X, c->Y, c->P};
  float* dst[3] = {x, y, p};
  for (int k = 0; k < 3; ++k)
    if (dst[k])
      HIP_TRY(hipMemcpy2DAsync(dst[k], (size_t)c->n * 4, src[k], (size_t)c->np * 4, (size_t)c->n * 4, c->R, kind,
                               c->stream),
              "copy state");
  gsb_status s = check_status_word(c);
  if (s != GSB_OK) return s;
  if (m) *m = c->m;
  return GSB_OK;
}

// Replace the state of the current run from caller arrays [R][n]: validated on the host
// (host arrays) or by a kernel whose flag is read back (device arrays).
gsb_status state_in(gsb_ctx* c, const float* x, const float* y, const float* p, int32_t m, bool device) {
  if (!c) return fail(GSB_EINVAL, "ctx is NULL");
  if (!c->inited) return fail(GSB_ESTATE, "no run");
  if (!x || !y || !p) return fail(GSB_EINVAL, "x, y and p are required");
  if (m < 0 || m > c->M) return fail(GSB_EINVAL, "m outside [0, M]");
  const size_t cnt = (size_t)c->R * c->n;
  if (device) {
    unsigned* flag = c->status + kStateFlagWord;
    unsigned bad = 0;
    HIP_TRY(launch_check_state(x, y, p, cnt, flag, c->stream), "state check kernel");
    HIP_TRY(hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, c->stream), "read state check");
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronise");
    if (bad & 1u) return fail(GSB_ENONFINITE, "state has a non-finite entry");
    if (bad & 2u) return fail(GSB_EINVAL, "|x| > 1 in the state (eq. (5) keeps |x| <= 1)");
  } else {
    for (size_t k = 0; k < cnt; ++k) {
      if (!std::isfinite(x[k]) || !std::isfinite(y[k]) || !std::isfinite(p[k]))
        return fail(GSB_ENONFINITE, "state has a non-finite entry");
      if (std::fabs(x[k]) > 1.0f) return fail(GSB_EINVAL, "|x| > 1 in the state (eq. (5) keeps |x| <= 1)");
    }
    HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronise");
  }
  const float* src[3] = {x, y, p};
  float* dst[3] = {c->X, c->Y, c->P};
  for (int k = 0; k < 3; ++k)
    HIP_TRY(hipMemcpy2DAsync(dst[k], (size_t)c->np * 4, src[k], (size_t)c->n * 4, (size_t)c->n * 4, c->R,
                             device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream),
            "copy state");
  HIP_TRY(hipStreamSynchronize(c->stream), "stream synchronise");
  c->m = m;
  c->energy_valid = false;
  return GSB_OK;
}

}  // namespace

gsb_status gsb_state(gsb_ctx* c, float* x, float* y, float* p, int32_t* m) {
  g_err.clear();
  return state_out(c, x, y, p, m, hipMemcpyDeviceToHost);
}

gsb_status gsb_state_device(gsb_ctx* c, float* x, float* y, float* p, int32_t* m) {
  g_err.clear();
  return state_out(c, x, y, p, m, hipMemcpyDeviceToDevice);
}

gsb_status gsb_set_state(gsb_ctx* c, const float* x, const float* y, const float* p, int32_t m) {
  g_err.clear();
  return state_in(c, x, y, p, m, false);
}

gsb_status gsb_set_state_device(gsb_ctx* c, const float* x, const float* y, const float* p, int32_t m) {
  g_err.clear();
  return state_in(c, x, y, p, m, true);
}

gsb_status gsb_delta(gsb_ctx* c, double* out) {
  g_err.clear();
  if (!c || !out) return fail(GSB_EINVAL, "NULL argument");
  if (!c->inited) return fail(GSB_ESTATE, "no run");
  if (c->R < 2) return fail(GSB_EINVAL, "delta needs at least one pair of replicas");
  const int pairs = c->R / 2;
  HIP_TRY(launch_delta(c->n_user, c->np, pairs, c->X, c->partial, c->stream), "delta kernel");
  HIP_TRY(hipMemcpyAsync(out, c->partial, (size_t)pairs * 8, hipMemcpyDeviceToHost, c->stream), "copy delta");
  return check_status_word(c);
}

gsb_status gsb_lle_workspace_size(gsb_ctx* c, int32_t replicas, int32_t steps, size_t* bytes) {
  g_err.clear();
  if (!c || !bytes) return fail(GSB_EINVAL, "NULL argument");
  if (replicas < 1 || steps < 1) return fail(GSB_EINVAL, "replicas and steps must be >= 1");
  Layout L;
  int kind;
  gsb_status s = plan(c, replicas, steps, &L, &kind, true);
  if (s != GSB_OK) return s;
  *bytes = L.total;
  return GSB_OK;
}

gsb_status gsb_lle(gsb_ctx* c, int32_t variant, int32_t schedule, double A, const double* A_per_replica, double dt,
                   int32_t replicas, int32_t steps, uint64_t seed, uint64_t tangent_seed, int32_t renorm_every,
                   double* lle, float* state_out) {
  g_err.clear();
  if (!c || !lle) return fail(GSB_EINVAL, "NULL argument");
  if (variant != GSB_BSB && variant != GSB_GBSB)
    return fail(GSB_EINVAL, "the tangent needs a continuous product: variant must be GSB_BSB or GSB_GBSB");
  if (schedule < GSB_SCHED_LINEAR || schedule > GSB_SCHED_CONSTANT) return fail(GSB_EINVAL, "unknown schedule");
  if (!std::isfinite(dt) || dt <= 0) return fail(GSB_EINVAL, "dt must be finite and > 0");
  if (replicas < 1 || replicas > (1 << 20)) return fail(GSB_EINVAL, "replicas must be in [1, 2^20]");
  if (steps < 1 || steps > (1 << 24)) return fail(GSB_EINVAL, "steps must be in [1, 2^24]");
  if (renorm_every < 1) return fail(GSB_EINVAL, "renorm_every must be >= 1");
  const int m_w = c->lle_from;
  if (m_w >= steps) return fail(GSB_EINVAL, "GSB_OPT_LLE_FROM must be below steps");
  std::vector<float> acol_host;
  try {
    acol_host.assign((size_t)(replicas + kRepPad - 1) / kRepPad * kRepPad, 0.0f);
  } catch (...) {
    return fail(GSB_ENOMEM, "host allocation failed");
  }
  for (int r = 0; r < replicas; ++r) {
    const double a = A_per_replica ? A_per_replica[r] : A;
    if (!std::isfinite(a) || a < 0) return fail(GSB_EINVAL, "control strengths must be finite and >= 0");
    acol_host[r] = variant == GSB_GBSB ? (float)a : 0.0f;
  }
  if (!c->c_set) {
    ensure_eig(c);
    c->c = c->lmax > 0 ? 1.0 / c->lmax : 1.0;  // App. A: c = 1 / lambda_max
  }
  Layout L;
  int kind;
  gsb_status s = plan(c, replicas, steps, &L, &kind, true);
  if (s != GSB_OK) return s;
  s = ensure_workspace(c, L.total);
  if (s != GSB_OK) return s;
  c->inited = false;  // the workspace now holds the tangent-mode layout
  c->energy_valid = false;
  c->timed = false;
  const int rp = (int)acol_host.size();
  s = carve_and_prepare(c, L, kind, kFormFP32, schedule, steps);
  if (s != GSB_OK) return s;
  float* acol = reinterpret_cast<float*>(c->ws + L.acol);
  double* lg = reinterpret_cast<double*>(c->ws + L.lg);
  float* ext = reinterpret_cast<float*>(c->ws + L.ext);
  c->dt = dt;
  HIP_TRY(hipMemcpyAsync(acol, acol_host.data(), (size_t)rp * 4, hipMemcpyHostToDevice, c->stream), "upload A");
  HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(lg), (size_t)rp * 2, 0u, c->stream), "clear log sums");
  HIP_TRY(launch_init_tangent(c->n, c->np, rp, seed, c->init_mode, tangent_seed, c->X, c->Y, c->P, c->stream),
          "init state and tangent");
  HIP_TRY(launch_tangent_renorm(c->n, c->np, rp, c->X, c->Y, c->P, lg, false, c->stream), "normalise tangent");
  if (!c->ev0) {
    HIP_TRY(hipEventCreate(&c->ev0), "event create");
    HIP_TRY(hipEventCreate(&c->ev1), "event create");
  }
  HIP_TRY(hipEventRecord(c->ev0, c->stream), "event record");
  // renormalise every renorm_every steps and at the window start m_w, where the log sums
  // start again from 0 (the tangent there has unit norm)
  for (int m0 = 0; m0 < steps;) {
    int m1 = std::min(steps, m0 + renorm_every);
    if (m0 < m_w && m1 > m_w) m1 = m_w;
    s = launch_chunks(c, kFormFP32, 2 * rp, false, 0.0f, acol, m0, m1, true);
    if (s != GSB_OK) return s;
    HIP_TRY(launch_tangent_renorm(c->n, c->np, rp, c->X, c->Y, c->P, lg, true, c->stream), "renormalise tangent");
    if (m1 == m_w)
      HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(lg), (size_t)rp * 2, 0u, c->stream), "restart log sums");
    m0 = m1;
  }
  HIP_TRY(hipEventRecord(c->ev1, c->stream), "event record");
  c->timed = true;
  std::vector<double> lg_host((size_t)replicas);
  HIP_TRY(hipMemcpyAsync(lg_host.data(), lg, (size_t)replicas * 8, hipMemcpyDeviceToHost, c->stream), "copy logs");
  if (state_out) {
    HIP_TRY(launch_tangent_extract(c->n, c->np, replicas, c->X, c->Y, c->P, ext, c->stream), "extract state");
    HIP_TRY(hipMemcpyAsync(state_out, ext, (size_t)6 * replicas * c->n * 4, hipMemcpyDeviceToHost, c->stream),
            "copy state");
  }
  s = check_status_word(c);
  if (s != GSB_OK) return s;
  for (int r = 0; r < replicas; ++r) lle[r] = lg_host[r] / ((double)(steps - m_w) * dt);
  return GSB_OK;
}

namespace {

// The reverse pass; cotangents in and out of caller arrays [R][n] on the host or the device.
gsb_status vjp_impl(gsb_ctx* c, int32_t count, float* xb, float* yb, float* pb, bool device) {
  if (!c || !xb || !yb || !pb) return fail(GSB_EINVAL, "NULL argument");
  if (!c->inited) return fail(GSB_ESTATE, "no run");
  if (c->variant != GSB_BSB && c->variant != GSB_GBSB)
    return fail(GSB_EINVAL, "the reverse pass needs a continuous product (bSB or GbSB)");
  if (c->precision != GSB_PREC_FP32 || c->kind != kKindGeneric)
    return fail(GSB_EUNSUPPORTED, "the reverse pass runs in the FP32 form (set GSB_OPT_PRECISION before the run)");
  if (count < 1 || c->m + count > c->M) return fail(GSB_EINVAL, "count must be >= 1 and stay within the schedule");
  const size_t arr = (size_t)c->rp * c->np;
  const size_t need = ((size_t)3 * (count + 1) + 3) * arr * 4;
  if (need > c->vjp_bytes) {
    if (c->vjp_buf) {
      const hipError_t es = hipStreamSynchronize(c->stream);
      const hipError_t ef = hipFree(c->vjp_buf);
      c->vjp_buf = nullptr;
      c->vjp_bytes = 0;
      if (es != hipSuccess || ef != hipSuccess) return fail(GSB_EDEVICE, "releasing the reverse-pass buffer");
    }
    void* p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) return fail(GSB_ENOMEM, "reverse-pass buffer of " + std::to_string(need) + " bytes");
    c->vjp_buf = p;
    c->vjp_bytes = need;
  }
  float* tape = static_cast<float*>(c->vjp_buf);
  float* last = tape + (size_t)3 * count * arr;  // entry `count`: the state after the segment
  float* cot = tape + (size_t)3 * (count + 1) * arr;
  // forward again from the current state, recording every step's input
  HIP_TRY(hipMemcpyAsync(last, c->X, arr * 4, hipMemcpyDeviceToDevice, c->stream), "copy state");
  HIP_TRY(hipMemcpyAsync(last + arr, c->Y, arr * 4, hipMemcpyDeviceToDevice, c->stream), "copy state");
  HIP_TRY(hipMemcpyAsync(last + 2 * arr, c->P, arr * 4, hipMemcpyDeviceToDevice, c->stream), "copy state");
  gsb_status s = launch_chunks(c, kFormFP32, c->rp, false, (float)c->A, nullptr, c->m, c->m + count, false, last,
                               last + arr, last + 2 * arr, tape);
  if (s != GSB_OK) return s;
  // cotangents in, reverse pass, cotangents out
  const int nd = c->n;
  HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(cot), 3 * arr, 0u, c->stream), "clear cotangents");
  const float* src[3] = {xb, yb, pb};
  for (int k = 0; k < 3; ++k)
    HIP_TRY(hipMemcpy2DAsync(cot + k * arr, (size_t)c->np * 4, src[k], (size_t)nd * 4, (size_t)nd * 4, c->R,
                             device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream),
            "upload cotangents");
  const int max_wg = max_coresident_adjoint();
  const int nb = c->np / tile_rows_kind(kKindGeneric);
  const int chunk = std::min(c->rp, std::max(max_wg / nb, 0) * tile_cols_kind(kKindGeneric) / kRepPad * kRepPad);
  if (chunk < kRepPad) return fail(GSB_EUNSUPPORTED, "n too large for one co-resident replica block (reverse pass)");
  s = launch_chunks(c, kFormFP32, c->rp, false, (float)c->A, nullptr, c->m, c->m + count, false, cot, cot + arr,
                    cot + 2 * arr, tape, true, chunk);
  if (s != GSB_OK) return s;
  float* dst[3] = {xb, yb, pb};
  for (int k = 0; k < 3; ++k)
    HIP_TRY(hipMemcpy2DAsync(dst[k], (size_t)nd * 4, cot + k * arr, (size_t)c->np * 4, (size_t)nd * 4, c->R,
                             device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream),
            "download cotangents");
  return check_status_word(c);
}

}  // namespace

gsb_status gsb_vjp(gsb_ctx* c, int32_t count, float* xb, float* yb, float* pb) {
  g_err.clear();
  return vjp_impl(c, count, xb, yb, pb, false);
}

gsb_status gsb_vjp_device(gsb_ctx* c, int32_t count, float* xb, float* yb, float* pb) {
  g_err.clear();
  return vjp_impl(c, count, xb, yb, pb, true);
}

gsb_status gsb_last_step_ms(gsb_ctx* c, double* ms) {
  g_err.clear();
  if (!c || !ms) return fail(GSB_EINVAL, "NULL argument");
  if (!c->timed) return fail(GSB_ESTATE, "no timed step yet");
  HIP_TRY(hipEventSynchronize(c->ev1), "event synchronise");
  float f = 0;
  HIP_TRY(hipEventElapsedTime(&f, c->ev0, c->ev1), "event elapsed");
  *ms = f;
  return GSB_OK;
}

}  // extern "C"
