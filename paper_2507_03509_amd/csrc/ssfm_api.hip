// Host side of libssfm: link validation, FP64 operator tables, launch
// orchestration and the C ABI declared in include/ssfm.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ssfm.h"
#include "host_common.hpp"
#include "launch_log.hpp"
#include "ssfm_internal.hpp"

using ssfm::cd;

namespace ssfm {

namespace {
thread_local std::string g_last_error;
}  // namespace

int api_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int api_fail_hip(hipError_t e, const char* what) {
  return api_fail(SSFM_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

const std::string& api_last_error() { return g_last_error; }
void api_clear_error() { g_last_error.clear(); }

}  // namespace ssfm

namespace {

using ssfm::DeviceGuard;
using ssfm::api_fail;
using ssfm::api_fail_hip;

constexpr double kPlanck = 6.62607015e-34;      // J s
constexpr double kDefaultCarrier = 193.4145e12;  // Hz (1550 nm)
constexpr double kPi = 3.14159265358979323846;

bool finite(double v) { return isfinite(v) != 0; }
}  // namespace

// Device scratch of ssfm_adjoint_noalloc: the adjoint's work fields and span
// checkpoints for callers that cannot allocate.  One array per device (each
// device that loads the library holds it until the process ends).  In host
// code its name is only a stand-in: kernels and copies take the device
// address resolved per device by resolve_scratch.
constexpr size_t kNoallocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
struct ScratchAddrs {
  std::mutex mu;
  void* ptr[kMaxDevices] = {};
  hipError_t status[kMaxDevices] = {};
  bool tried[kMaxDevices] = {};
};
ScratchAddrs& scratch_addrs() {
  static ScratchAddrs* a = new ScratchAddrs();  // never destroyed
  return *a;
}

// Once per device, with that device current: the device address of
// `scratch` (called from ssfm_plan).
void resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  ScratchAddrs& a = scratch_addrs();
  std::lock_guard<std::mutex> lock(a.mu);
  if (a.tried[device]) return;
  a.tried[device] = true;
  void* ptr = nullptr;
  a.status[device] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  a.ptr[device] = a.status[device] == hipSuccess ? ptr : nullptr;
}

// The resolved address for `device`, or nullptr with the reason in *why.
void* scratch_ptr(int device, hipError_t* why) {
  *why = hipErrorInvalidDevice;
  if (device < 0 || device >= kMaxDevices) return nullptr;
  ScratchAddrs& a = scratch_addrs();
  std::lock_guard<std::mutex> lock(a.mu);
  *why = a.tried[device] ? a.status[device] : hipErrorNotInitialized;
  return a.ptr[device];
}
}  // namespace

struct ssfm_plan_s {
  ssfm_link link{};
  int device = 0;
  ssfm::KernelSet ks;
  int n_pol = 1;
  int64_t n = 0;
  int steps = 0, spans = 0;
  double gspan = 1.0, sigma_h = 0.0;
  std::vector<double> kappa;
  // device tables
  cd* h_half = nullptr;
  cd* h_full = nullptr;
  cd* tw_n = nullptr;  // path 1: W_N
  cd* tw1 = nullptr;   // path 2: W_N1
  cd* tw2 = nullptr;   // path 2: W_N2
  cd* twA = nullptr;   // path 2: W_N^{a N2}
  cd* twB = nullptr;   // path 2: W_N^{b}
  double* d_kappa = nullptr;
  size_t table_bytes = 0;
  std::vector<void*> allocations;
  // profiling window: event pairs around each launch
  bool profiling = false;
  ssfm::LaunchLog<hipEvent_t> prof;
  // launch-sequence replay: the last forward call's key and, once the same
  // call repeats, its captured graph
  struct GraphKey {
    void* field = nullptr;
    int64_t batch = 0;
    uint64_t seed = 0, real0 = 0;
    int s0 = 0, s1 = 0;
    void* stream = nullptr;
    bool operator==(const GraphKey& o) const {
      return field == o.field && batch == o.batch && seed == o.seed && real0 == o.real0 &&
             s0 == o.s0 && s1 == o.s1 && stream == o.stream;
    }
  };
  // launch shapes chosen by ssfm_plan_autotune, per batch size
  struct Shape {
    bool wide_cols = false, wide_rows = false;
  };
  std::mutex tune_mu;
  std::map<int64_t, Shape> tuned;
  std::mutex graph_mu;
  GraphKey last_key;
  bool have_last = false;
  hipGraphExec_t graph_exec = nullptr;
  bool graph_valid = false;
  hipStream_t capture_stream = nullptr;
  // adjoint workspace (grown on demand): span checkpoints and the
  // [state; cotangent] work buffer
  float2* adj_ckpt = nullptr;
  float2* adj_work = nullptr;
  size_t adj_ckpt_bytes = 0, adj_work_bytes = 0;
  // the adjoint's stored nonlinear-step inputs (ssfm_plan_set_state_memory)
  uint64_t state_budget = 0;
  float2* adj_states = nullptr;
  size_t adj_states_bytes = 0;
  // concurrent parts of a four-step call's chunks: 0 (the library's
  // choice, forward_parts) or 1..5 (ssfm_plan_set_forward_streams)
  int forward_streams = 0;
  // working-set target of a four-step call's sequential chunks (bytes; 0:
  // the whole batch at once)
  size_t chunk_bytes = 0;
  // adjoint calls share the workspace above, so they are serialised: on the
  // host by adj_mu, on the device by adj_done (each call's stream waits for
  // the last work of the previous call, whatever stream that ran on)
  std::mutex adj_mu;
  hipEvent_t adj_done = nullptr;
  bool adj_pending = false;
  // device table allocations made so far (fault injection, SSFM_FAIL_ALLOC)
  int table_allocs = 0;

  ~ssfm_plan_s() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    for (hipEvent_t e : prof.pool()) (void)hipEventDestroy(e);
    for (void* p : allocations) (void)hipFree(p);
    if (adj_ckpt) (void)hipFree(adj_ckpt);
    if (adj_work) (void)hipFree(adj_work);
    if (adj_states) (void)hipFree(adj_states);
    if (adj_done) (void)hipEventDestroy(adj_done);
  }
};

namespace {

int validate_link(const ssfm_link* l) {
  if (!l) return api_fail(SSFM_EINVAL, "link is NULL");
  if (l->n_pol != 1 && l->n_pol != 2) return api_fail(SSFM_EINVAL, "n_pol must be 1 or 2, got %d", l->n_pol);
  const int64_t n = l->n_samples;
  if (n < 64 || n > (int64_t(1) << 18) || (n & (n - 1)) != 0)
    return api_fail(SSFM_EINVAL, "n_samples must be a power of two in [2^6, 2^18], got %lld",
                (long long)n);
  if (l->n_spans < 1 || l->n_spans > 65535)
    return api_fail(SSFM_EINVAL, "n_spans must be in [1, 65535], got %d", l->n_spans);
  if (l->steps_per_span < 1 || l->steps_per_span > (1 << 24))
    return api_fail(SSFM_EINVAL, "steps_per_span must be in [1, 2^24], got %d", l->steps_per_span);
  if (l->ase != 0 && l->ase != 1) return api_fail(SSFM_EINVAL, "ase must be 0 or 1");
  if (!finite(l->sample_rate_hz) || l->sample_rate_hz <= 0)
    return api_fail(SSFM_EINVAL, "sample_rate_hz must be finite and > 0");
  if (!finite(l->span_km) || l->span_km <= 0) return api_fail(SSFM_EINVAL, "span_km must be finite and > 0");
  if (!finite(l->alpha_db_per_km) || !finite(l->beta2_ps2_per_km) || !finite(l->gamma_per_w_km))
    return api_fail(SSFM_EINVAL, "alpha, beta2 and gamma must be finite");
  if (!finite(l->nl_factor) && !isnan(l->nl_factor))
    return api_fail(SSFM_EINVAL, "nl_factor must be finite or NaN");
  if (!finite(l->edfa_gain_db)) return api_fail(SSFM_EINVAL, "edfa_gain_db must be finite");
  if (l->ase && !finite(l->edfa_nf_db)) return api_fail(SSFM_EINVAL, "edfa_nf_db must be finite");
  if (!isnan(l->carrier_hz) && (!finite(l->carrier_hz) || l->carrier_hz <= 0))
    return api_fail(SSFM_EINVAL, "carrier_hz must be NaN or finite and > 0");
  if ((l->flags & ~SSFM_FLAG_FP32_ARITHMETIC) != 0 || l->reserved != 0)
    return api_fail(SSFM_EINVAL, "flags may only hold SSFM_FLAG_FP32_ARITHMETIC; reserved must be 0");
  return SSFM_OK;
}

// Stockham pass twiddles of a length-M transform: for each pass p >= 1, rows
// k < ns(p) of radix(p) entries W_{ns R}^{k r} (the layout the kernels read).
std::vector<cd> pass_twiddles(int M) {
  int l = 0;
  while ((1 << l) < M) ++l;
  const int passes = ssfm::fft_passes(l);
  std::vector<cd> t((size_t)ssfm::fft_tw_offset(l, passes));
  for (int p = 1; p < passes; ++p) {
    const int ns = ssfm::fft_ns(l, p), R = ssfm::fft_radix(l, p);
    const int base = ssfm::fft_tw_offset(l, p);
    for (int k = 0; k < ns; ++k)
      for (int r = 0; r < R; ++r) {
        const double ang = -2.0 * kPi * (double)((k * r) % (ns * R)) / (double)(ns * R);
        t[(size_t)(base + k * R + r)] = {cos(ang), sin(ang)};
      }
  }
  if (t.empty()) t.push_back({1.0, 0.0});
  return t;
}

// W_M^m = exp(-2 pi i m / M) for m < count.
std::vector<cd> twiddles(int64_t M, int64_t count, int64_t stride) {
  std::vector<cd> t((size_t)count);
  for (int64_t m = 0; m < count; ++m) {
    const double ang = -2.0 * kPi * (double)((m * stride) % M) / (double)M;
    t[(size_t)m] = {cos(ang), sin(ang)};
  }
  return t;
}

// Fault injection for tests: the value of environment variable `name` as a
// positive integer, else 0.
int env_count(const char* name) {
  const char* v = getenv(name);
  return v ? std::max(0, atoi(v)) : 0;
}

// Realisations per sequential chunk of a four-step call whose kernels carry
// `fields` fields of each realisation.  A chunk of about 256 MiB keeps much
// of the field in the MI355X's 256 MB Infinity Cache from one pass to the
// next (measured on the 2^16 dual-polarisation link: 7.2e10 sample-steps/s
// at 256 realisations against 6.4e10 at 512); larger batches run as equal
// chunks, one after the other.
int64_t chunk_max(const ssfm_plan_s* p, int fields) {
  if (p->ks.path != 2 || p->chunk_bytes == 0) return 0;
  const size_t per = (size_t)fields * p->n_pol * p->n * sizeof(float2);
  return std::max<int64_t>(1, (int64_t)(p->chunk_bytes / per));
}

int64_t chunk_batch(const ssfm_plan_s* p, int64_t batch, int fields) {
  const int64_t cmax = chunk_max(p, fields);
  if (cmax == 0 || batch <= cmax) return batch;
  const int64_t parts = (batch + cmax - 1) / cmax;
  return (batch + parts - 1) / parts;
}

template <typename T>
int upload(ssfm_plan_s* p, T** dst, const std::vector<T>& src) {
  const size_t bytes = src.size() * sizeof(T);
  void* d = nullptr;
  // SSFM_FAIL_ALLOC=k: the plan's k-th table allocation fails
  const int fail_at = env_count("SSFM_FAIL_ALLOC");
  if (++p->table_allocs == fail_at)
    return api_fail(SSFM_ENOMEM, "allocation %d failed (injected by SSFM_FAIL_ALLOC)", fail_at);
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return api_fail(SSFM_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  p->allocations.push_back(d);
  e = hipMemcpy(d, src.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return api_fail_hip(e, "hipMemcpy (plan tables)");
  *dst = static_cast<T*>(d);
  p->table_bytes += bytes;
  return SSFM_OK;
}

int build_tables(ssfm_plan_s* p) {
  const ssfm_link& l = p->link;
  const int64_t n = p->n;
  const double fs = l.sample_rate_hz;
  const double alpha = l.alpha_db_per_km * log(10.0) / 10.0 / 1e3;  // 1/m, power
  const double beta2 = l.beta2_ps2_per_km * 1e-27;                   // s^2/m
  const double gamma = l.gamma_per_w_km * 1e-3;                      // 1/(W m)
  const double c_nl = isnan(l.nl_factor) ? (l.n_pol == 1 ? 1.0 : 8.0 / 9.0) : l.nl_factor;
  const double span_m = l.span_km * 1e3;
  const double h = span_m / l.steps_per_span;
  const double h_nl = alpha == 0.0 ? h : 2.0 * sinh(alpha * h / 2.0) / alpha;
  const double gain = pow(10.0, l.edfa_gain_db / 10.0);
  const double carrier = isnan(l.carrier_hz) ? kDefaultCarrier : l.carrier_hz;

  p->kappa.resize((size_t)p->steps);
  for (int j = 0; j < p->steps; ++j)
    p->kappa[(size_t)j] = c_nl * gamma * h_nl * exp(-alpha * (j + 0.5) * h);
  p->gspan = sqrt(gain) * exp(-alpha * span_m / 2.0);
  p->sigma_h = 0.0;
  if (l.ase && gain > 1.0) {
    const double nf = pow(10.0, l.edfa_nf_db / 10.0);
    const double var = (nf / 2.0) * (gain - 1.0) * kPlanck * carrier * fs;  // per pol
    p->sigma_h = sqrt(var / 2.0);
  }

  // dispersion operator, 1/N of the unnormalised inverse FFT folded in
  auto omega = [&](int64_t k) {
    const int64_t kk = k < (n + 1) / 2 ? k : k - n;  // fftfreq order
    return 2.0 * kPi * (double)kk * fs / (double)n;
  };
  std::vector<cd> hh((size_t)n), hf((size_t)n);
  const int n1 = p->ks.n1, n2 = p->ks.n2;
  for (int64_t k = 0; k < n; ++k) {
    const double w = omega(k);
    const double th_full = 0.5 * beta2 * w * w * h;
    const double th_half = 0.5 * th_full;
    // storage position: natural order (path 1) or [k1][k2] with k = k1 + N1 k2
    const int64_t pos = p->ks.path == 1 ? k : (k % n1) * n2 + k / n1;
    hh[(size_t)pos] = {cos(th_half) / (double)n, sin(th_half) / (double)n};
    hf[(size_t)pos] = {cos(th_full) / (double)n, sin(th_full) / (double)n};
  }
  int rc;
  if ((rc = upload(p, &p->h_half, hh)) != SSFM_OK) return rc;
  if ((rc = upload(p, &p->h_full, hf)) != SSFM_OK) return rc;
  if ((rc = upload(p, &p->d_kappa, p->kappa)) != SSFM_OK) return rc;
  if (p->ks.path == 1) {
    if ((rc = upload(p, &p->tw_n, pass_twiddles((int)n))) != SSFM_OK) return rc;
  } else {
    if ((rc = upload(p, &p->tw1, pass_twiddles(n1))) != SSFM_OK) return rc;
    if ((rc = upload(p, &p->tw2, pass_twiddles(n2))) != SSFM_OK) return rc;
    if ((rc = upload(p, &p->twA, twiddles(n, n1, n2))) != SSFM_OK) return rc;
    if ((rc = upload(p, &p->twB, twiddles(n, n2, 1))) != SSFM_OK) return rc;
  }
  return SSFM_OK;
}

enum { KIND_LDS = 0, KIND_ROW = 1, KIND_COL = 2, KIND_ADJ = 3, KIND_COUNT = 4 };
const char* const kKindName[KIND_COUNT] = {"k1_lds", "k2_rows", "k3_cols", "k3_adj"};

// Launch through `fn`, bracketed by events when the plan is profiling.  A
// launch that fails leaves no record (and frees its event pair).
template <typename F>
hipError_t launch(ssfm_plan_s* p, int kind, double bytes, hipStream_t st, F&& fn) {
  if (!p->profiling) return fn();
  hipError_t e = hipSuccess;
  size_t pair = 0;
  if (!p->prof.reserve([&](hipEvent_t* ev) { return (e = hipEventCreate(ev)) == hipSuccess; },
                       &pair))
    return e;
  ssfm::LaunchLog<hipEvent_t>::Record r{kind, bytes, pair};
  e = hipEventRecord(p->prof.before(r), st);
  if (e == hipSuccess) e = fn();
  if (e == hipSuccess) e = hipEventRecord(p->prof.after(r), st);
  if (e != hipSuccess) {
    p->prof.release(pair);
    return e;
  }
  p->prof.record(pair, kind, bytes);
  return hipSuccess;
}

int64_t launches_per_call(const ssfm_plan_s* p) {
  if (p->ks.path == 1) return 1;
  return 1 + (int64_t)p->spans * (p->steps + 1) * 2;
}

// Launch shape of a four-step call: SSFM_COLUMNS override (the width of the
// wide or the narrow column tile, with the matching row workgroup), else the shape
// ssfm_plan_autotune recorded for this batch, else wide column tiles once the
// batch gives at least 512 column workgroups, and 256-lane row workgroups
// below 2^16 rows (64-lane ones from there on: measured faster on the 2^16 and
// 2^18 links at large batches, where the grid holds several waves per SIMD).
struct Shape4 {
  const ssfm::FourStepKernels* cols;
  ssfm::RowLaunch row;
  bool wide_cols, wide_rows;
};

Shape4 pick_shape(ssfm_plan_s* p, int64_t batch) {
  const char* env = getenv("SSFM_COLUMNS");
  if (env) {
    const int c = atoi(env);
    for (const ssfm::FourStepKernels* k : {&p->ks.wide, &p->ks.narrow})
      if (k->columns == c) {
        const bool w = k == &p->ks.wide;
        return {k, w ? p->ks.row_wide : p->ks.row_narrow, w, w};
      }
  }
  {
    std::lock_guard<std::mutex> lock(p->tune_mu);
    auto it = p->tuned.find(batch);
    if (it != p->tuned.end()) {
      const auto& t = it->second;
      return {t.wide_cols ? &p->ks.wide : &p->ks.narrow,
              t.wide_rows ? p->ks.row_wide : p->ks.row_narrow, t.wide_cols, t.wide_rows};
    }
  }
  const bool w = batch * (p->ks.n2 / p->ks.wide.columns) >= 512;
  const bool wr = w && batch * p->n_pol * p->ks.n1 < 65536;
  return {w ? &p->ks.wide : &p->ks.narrow, wr ? p->ks.row_wide : p->ks.row_narrow, w, wr};
}

// Graph replay for the four-step path (many launches per call); not while a
// profiling window records per-launch events.  SSFM_GRAPH=0 disables it.
bool use_graphs(const ssfm_plan_s* p) {
  if (p->ks.path != 2 || p->profiling) return false;
  const char* env = getenv("SSFM_GRAPH");
  return !(env && strcmp(env, "0") == 0);
}

// states (four-step path): for spans s >= state_span0, the input of each
// nonlinear step i is stored at states + ((s - state_span0) steps + i) slice,
// slice = batch * n_pol * n elements.
int run_forward(ssfm_plan_s* p, float2* field, int64_t batch, uint64_t seed, uint64_t real0,
                int s0, int s1, hipStream_t st, float2* ckpt = nullptr,
                const uint64_t* seeds = nullptr, float2* states = nullptr,
                int state_span0 = 0, size_t ckpt_stride = 0) {
  const ssfm::KernelSet& ks = p->ks;
  hipError_t e;
  if (s0 == s1) return SSFM_OK;
  // algorithmic HBM traffic of one launch: the field read once and written once
  const double field_bytes = 2.0 * (double)batch * p->n_pol * (double)p->n * sizeof(float2);
  if (ks.path == 1) {
    ssfm::LdsArgs a{};
    a.field = field;
    a.h_half = p->h_half;
    a.h_full = p->h_full;
    a.tw = p->tw_n;
    a.kappa = p->d_kappa;
    a.steps = p->steps;
    a.span_begin = s0;
    a.span_end = s1;
    a.gspan = p->gspan;
    a.sigma_h = p->sigma_h;
    a.seed = seed;
    a.realization0 = real0;
    a.seeds = seeds;
    if ((e = launch(p, KIND_LDS, field_bytes, st, [&] { return ks.lds(a, batch, st); })) != hipSuccess)
      return api_fail_hip(e, "k1_lds launch");
    return SSFM_OK;
  }
  const Shape4 shape = pick_shape(p, batch);
  const ssfm::FourStepKernels& cols = *shape.cols;
  const ssfm::RowLaunch row = shape.row;
  const int64_t rows = batch * p->n_pol * ks.n1;
  int log2_n2 = 0;
  while ((1 << log2_n2) < ks.n2) ++log2_n2;
  ssfm::RowArgs ra{};
  ra.field = field;
  ra.tw = p->tw2;
  ra.twA = p->twA;
  ra.twB = p->twB;
  ra.n1 = ks.n1;
  ra.log2_n2 = log2_n2;
  ra.conj_h = 0;
  ssfm::ColArgs a{};
  a.field = field;
  a.tw1 = p->tw1;
  a.n2 = ks.n2;
  a.n = p->n;
  a.gspan = p->gspan;
  a.sigma_h = p->sigma_h;
  a.seed = seed;
  a.realization0 = real0;
  a.seeds = seeds;
  if ((e = launch(p, KIND_COL, field_bytes, st,
                  [&] { return cols.col[ssfm::MODE_FIRST](a, batch, st); })) != hipSuccess)
    return api_fail_hip(e, "k3 launch");
  for (int s = s0; s < s1; ++s) {
    a.span = s;
    for (int i = 0; i <= p->steps; ++i) {
      ra.H = (i == 0 || i == p->steps) ? p->h_half : p->h_full;
      if ((e = launch(p, KIND_ROW, field_bytes, st,
                      [&] { return row(ra, rows, st); })) != hipSuccess)
        return api_fail_hip(e, "k2 launch");
      int mode;
      if (i < p->steps) {
        mode = ssfm::MODE_NL;
        a.kappa = p->kappa[(size_t)i];
        if (states && s >= state_span0) {
          mode = ssfm::MODE_NL_STORE;
          a.states = states + ((size_t)(s - state_span0) * p->steps + (size_t)i) *
                                  ((size_t)batch * p->n_pol * p->n);
        }
      } else {
        mode = s + 1 < s1 ? ssfm::MODE_EDFA : ssfm::MODE_LAST;
        // span s's checkpoints: ckpt_stride elements apart (default: the batch)
        a.ckpt = ckpt ? ckpt + (size_t)s * (ckpt_stride ? ckpt_stride
                                                        : (size_t)batch * p->n_pol * p->n)
                      : nullptr;
      }
      // a stored nonlinear-step input is one more write of the field
      const double bytes = mode == ssfm::MODE_NL_STORE ? 1.5 * field_bytes : field_bytes;
      if ((e = launch(p, KIND_COL, bytes, st,
                      [&] { return cols.col[mode](a, batch, st); })) != hipSuccess)
        return api_fail_hip(e, "k3 launch");
    }
  }
  return SSFM_OK;
}


int check_call(ssfm_plan_t plan, const void* field, int64_t batch) {
  if (!plan) return api_fail(SSFM_EINVAL, "plan is NULL");
  if (!field) return api_fail(SSFM_EINVAL, "field is NULL");
  if (((uintptr_t)field & 7u) != 0) return api_fail(SSFM_EINVAL, "field must be 8-byte aligned");
  if (batch < 1) return api_fail(SSFM_EINVAL, "batch must be >= 1, got %lld", (long long)batch);
  const int64_t n2 = plan->ks.path == 2 ? plan->ks.n2 : 1;
  const int64_t cols = plan->ks.path == 2 ? plan->ks.narrow.columns : 1;
  if (batch * (n2 / cols) > 0x7fffffff || batch * plan->n_pol * plan->ks.n1 > (int64_t(1) << 40))
    return api_fail(SSFM_EINVAL, "batch %lld exceeds the launch grid", (long long)batch);
  return SSFM_OK;
}

constexpr int kMaxSpans = 65535;

bool same_double(double a, double b) {
  return (isnan(a) && isnan(b)) || memcmp(&a, &b, sizeof a) == 0;
}

bool same_link(const ssfm_link& a, const ssfm_link& b) {
  return a.n_pol == b.n_pol && a.n_spans == b.n_spans && a.steps_per_span == b.steps_per_span &&
         a.ase == b.ase && a.n_samples == b.n_samples &&
         same_double(a.sample_rate_hz, b.sample_rate_hz) && same_double(a.span_km, b.span_km) &&
         same_double(a.alpha_db_per_km, b.alpha_db_per_km) &&
         same_double(a.beta2_ps2_per_km, b.beta2_ps2_per_km) &&
         same_double(a.gamma_per_w_km, b.gamma_per_w_km) &&
         same_double(a.nl_factor, b.nl_factor) && same_double(a.edfa_gain_db, b.edfa_gain_db) &&
         same_double(a.edfa_nf_db, b.edfa_nf_db) && same_double(a.carrier_hz, b.carrier_hz) &&
         a.flags == b.flags && a.reserved == b.reserved;
}

// Plans built by ssfm_batch, kept for the life of the process (one per
// distinct link and device).
struct PlanCache {
  std::mutex mu;
  std::vector<std::pair<std::pair<ssfm_link, int>, ssfm_plan_t>> plans;
};
PlanCache& plan_cache() {
  static PlanCache* c = new PlanCache();  // never destroyed: plans outlive static teardown
  return *c;
}

// Worker streams of ssfm_batch, per device, created on first use and kept
// for the life of the process (default priority, not blocking on the null
// stream; every use is ordered against the caller's stream by events).
constexpr int kBatchStreams = 4;
struct BatchStreams {
  hipStream_t s[kBatchStreams] = {};
};
int batch_streams(int device, hipStream_t (&out)[kBatchStreams]) {
  static std::mutex mu;
  static std::map<int, BatchStreams>* per = new std::map<int, BatchStreams>();
  std::lock_guard<std::mutex> lock(mu);
  BatchStreams& b = (*per)[device];
  for (int k = 0; k < kBatchStreams; ++k) {
    if (!b.s[k]) {
      const hipError_t e = hipStreamCreateWithFlags(&b.s[k], hipStreamNonBlocking);
      if (e != hipSuccess) {
        b.s[k] = nullptr;
        return api_fail_hip(e, "ssfm_batch worker stream");
      }
    }
    out[k] = b.s[k];
  }
  return SSFM_OK;
}

}  // namespace

extern "C" int ssfm_plan(const ssfm_link* link, int hip_device, ssfm_plan_t* out);
extern "C" int ssfm_plan_autotune(ssfm_plan_t plan, int64_t batch, void* stream,
                                  ssfm_tune_info* info);


namespace {
int cached_plan(const ssfm_link& key, int device, ssfm_plan_t* out) {
  PlanCache& c = plan_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  for (auto& e : c.plans)
    if (e.first.second == device && same_link(e.first.first, key)) {
      *out = e.second;
      return SSFM_OK;
    }
  ssfm_plan_t p = nullptr;
  const int rc = ssfm_plan(&key, device, &p);
  if (rc != SSFM_OK) return rc;
  c.plans.push_back({{key, device}, p});
  *out = p;
  return SSFM_OK;
}
}  // namespace

namespace {

// The schedule of one ssfm_batch call: entries grouped by physical link (the
// span count is per entry: plans do not depend on it), each group's entries
// ordered most spans first (the entries still propagating are a prefix),
// groups placed, largest estimated time first, on the least-loaded of the
// worker streams.  An LDS-resident group keeps one workgroup per realisation
// busy for the whole link and fills only as many CUs as it has realisations,
// so the four-step groups use the rest of the chip meanwhile.
struct BatchSchedule {
  std::vector<std::vector<int64_t>> groups;
  std::vector<ssfm_plan_t> plans;
  std::vector<std::vector<int64_t>> active_counts;  // per group: entries per span segment
  std::vector<size_t> order;                        // groups by decreasing cost
  std::vector<int> stream;                          // worker stream of each group
  int nstreams = 0;
};

int make_batch_schedule(const ssfm_link* links, int64_t count, int device, BatchSchedule* bs) {
  std::vector<ssfm_link> keys;
  for (int64_t i = 0; i < count; ++i) {
    ssfm_link k = links[i];
    k.n_spans = kMaxSpans;
    size_t gi = 0;
    while (gi < keys.size() && !same_link(keys[gi], k)) ++gi;
    if (gi == keys.size()) {
      keys.push_back(k);
      bs->groups.emplace_back();
    }
    bs->groups[gi].push_back(i);
  }
  const size_t ng = bs->groups.size();
  bs->plans.resize(ng);
  bs->active_counts.resize(ng);
  std::vector<double> cost(ng);
  for (size_t gi = 0; gi < ng; ++gi) {
    const int rc = cached_plan(keys[gi], device, &bs->plans[gi]);
    if (rc != SSFM_OK) return rc;
    const ssfm_plan_s* pl = bs->plans[gi];
    std::vector<int64_t>& idx = bs->groups[gi];
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
      return links[a].n_spans > links[b].n_spans;
    });
    double span_sum = 0.0;
    for (int64_t i : idx) span_sum += links[i].n_spans;
    const int max_spans = links[idx[0]].n_spans;
    // LDS path: latency of the longest realisation; four-step: total work
    cost[gi] = pl->ks.path == 1 ? 4.0 * max_spans * pl->steps * (double)pl->n * pl->n_pol
                                : span_sum * pl->steps * (double)pl->n * pl->n_pol / 16.0;
    const int64_t m = (int64_t)idx.size();
    int s0 = 0;
    for (;;) {
      int64_t active = 0;
      while (active < m && links[idx[(size_t)active]].n_spans > s0) ++active;
      if (active == 0) break;
      bs->active_counts[gi].push_back(active);
      s0 = links[idx[(size_t)(active - 1)]].n_spans;
    }
  }
  bs->order.resize(ng);
  for (size_t gi = 0; gi < ng; ++gi) bs->order[gi] = gi;
  std::stable_sort(bs->order.begin(), bs->order.end(),
                   [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  bs->nstreams = (int)std::min<size_t>(kBatchStreams, ng);
  bs->stream.assign(ng, 0);
  std::vector<double> load((size_t)bs->nstreams, 0.0);
  for (size_t gi : bs->order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[(size_t)k] += cost[gi];
    bs->stream[gi] = k;
  }
  return SSFM_OK;
}

// Staging of a captured call: one field array and one seed array per group,
// allocated before the capture and owned by the graph.
struct BatchStaging {
  std::vector<float2*> fields;
  std::vector<uint64_t*> seeds;
  void release() {
    for (float2* f : fields) (void)hipFree(f);
    for (uint64_t* s : seeds) (void)hipFree(s);
    fields.clear();
    seeds.clear();
  }
};

// Enqueue a call on `st`: fork to the worker streams, per group gather the
// entries into one staging field (most spans first), propagate it over span
// segments on the shrinking prefix still active, scatter back; join.  With
// `stage` (capture) the staging and device seeds are the given arrays;
// without, they come from stream-ordered hipMallocAsync on the group's stream.
int enqueue_batch(const BatchSchedule& bs, const ssfm_link* links, void* const* fields,
                  const uint64_t* seeds, hipStream_t st, hipStream_t (&ws)[kBatchStreams],
                  const BatchStaging* stage) {
  const int nstreams = bs.nstreams;
  hipEvent_t ev[kBatchStreams + 1] = {};
  hipError_t e = hipSuccess;
  for (int k = 0; k <= nstreams && e == hipSuccess; ++k)
    e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ev[nstreams], st);  // fork
  for (int k = 0; k < nstreams && e == hipSuccess; ++k) e = hipStreamWaitEvent(ws[k], ev[nstreams], 0);
  if (e != hipSuccess) {
    for (hipEvent_t x : ev)
      if (x) (void)hipEventDestroy(x);
    return api_fail_hip(e, "ssfm_batch fork");
  }
  int rc = SSFM_OK;
  for (size_t oi = 0; oi < bs.order.size() && rc == SSFM_OK && e == hipSuccess; ++oi) {
    const size_t gi = bs.order[oi];
    hipStream_t gs = ws[bs.stream[gi]];
    ssfm_plan_t plan = bs.plans[gi];
    const std::vector<int64_t>& idx = bs.groups[gi];
    const int64_t m = (int64_t)idx.size();
    const size_t elems = (size_t)plan->n_pol * plan->n;
    const size_t fbytes = elems * sizeof(float2);
    void* buf = nullptr;
    void* dseeds = nullptr;
    if (stage) {
      buf = stage->fields[gi];
      dseeds = stage->seeds[gi];
    } else {
      if ((e = hipMallocAsync(&buf, (size_t)m * fbytes, gs)) != hipSuccess) {
        rc = api_fail(SSFM_ENOMEM, "staging buffer of %zu bytes: %s", (size_t)m * fbytes,
                      hipGetErrorString(e));
        break;
      }
      if ((e = hipMallocAsync(&dseeds, (size_t)m * sizeof(uint64_t), gs)) != hipSuccess) {
        (void)hipFreeAsync(buf, gs);
        rc = api_fail(SSFM_ENOMEM, "seed buffer: %s", hipGetErrorString(e));
        break;
      }
    }
    std::vector<uint64_t> hseeds((size_t)m);
    for (int64_t r = 0; r < m; ++r) {
      hseeds[(size_t)r] = seeds[idx[(size_t)r]];
      if (e == hipSuccess)
        e = hipMemcpyAsync(static_cast<float2*>(buf) + (size_t)r * elems, fields[idx[(size_t)r]],
                           fbytes, hipMemcpyDeviceToDevice, gs);
    }
    if (e == hipSuccess && !stage)
      e = hipMemcpyAsync(dseeds, hseeds.data(), (size_t)m * sizeof(uint64_t),
                         hipMemcpyHostToDevice, gs);
    int s0 = 0;
    for (int64_t active : bs.active_counts[gi]) {
      if (rc != SSFM_OK || e != hipSuccess) break;
      const int s1 = links[idx[(size_t)(active - 1)]].n_spans;
      rc = run_forward(plan, static_cast<float2*>(buf), active, 0, 0, s0, s1, gs, nullptr,
                       static_cast<const uint64_t*>(dseeds));
      s0 = s1;
    }
    for (int64_t r = 0; r < m && rc == SSFM_OK && e == hipSuccess; ++r)
      e = hipMemcpyAsync(fields[idx[(size_t)r]], static_cast<float2*>(buf) + (size_t)r * elems,
                         fbytes, hipMemcpyDeviceToDevice, gs);
    if (!stage) {
      (void)hipFreeAsync(buf, gs);
      (void)hipFreeAsync(dseeds, gs);
    }
  }
  // join: the caller's stream waits for every worker stream (also after an
  // error, so that no work of this call is left unordered)
  hipError_t ej = hipSuccess;
  for (int k = 0; k < nstreams; ++k) {
    if (ej == hipSuccess) ej = hipEventRecord(ev[k], ws[k]);
    if (ej == hipSuccess) ej = hipStreamWaitEvent(st, ev[k], 0);
  }
  for (int k = 0; k <= nstreams; ++k) (void)hipEventDestroy(ev[k]);
  if (rc != SSFM_OK) return rc;
  if (e != hipSuccess) return api_fail_hip(e, "ssfm_batch copies");
  if (ej != hipSuccess) return api_fail_hip(ej, "ssfm_batch join");
  return SSFM_OK;
}

// Replay state of ssfm_batch (one per process): the last call's signature
// and, once it repeats, its captured graph with the staging that graph uses.
struct BatchReplay {
  std::mutex mu;
  bool have_last = false;
  int device = -1;
  void* stream = nullptr;
  std::vector<ssfm_link> links;
  std::vector<void*> fields;
  std::vector<uint64_t> seeds;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
  BatchStaging stage;
  hipEvent_t done = nullptr;  // after the graph's last launch
  bool pending = false;

  bool matches(const ssfm_link* l, void* const* f, int64_t count, const uint64_t* sd, int dev,
               void* strm) const {
    if (!have_last || dev != device || strm != stream || (size_t)count != links.size())
      return false;
    for (int64_t i = 0; i < count; ++i)
      if (!same_link(links[(size_t)i], l[i]) || fields[(size_t)i] != f[i] || seeds[(size_t)i] != sd[i])
        return false;
    return true;
  }
  void remember(const ssfm_link* l, void* const* f, int64_t count, const uint64_t* sd, int dev,
                void* strm) {
    links.assign(l, l + count);
    fields.assign(f, f + count);
    seeds.assign(sd, sd + count);
    device = dev;
    stream = strm;
    have_last = true;
  }
  // drop the graph and its staging, once its last launch has finished
  int release() {
    if (pending && done) {
      const hipError_t e = hipEventSynchronize(done);
      if (e != hipSuccess) return api_fail_hip(e, "hipEventSynchronize (batch replay)");
    }
    pending = false;
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    stage.release();
    have_last = false;
    return SSFM_OK;
  }
};
BatchReplay& batch_replay() {
  static BatchReplay* r = new BatchReplay();  // never destroyed (process lifetime)
  return *r;
}

// Parts a four-step chunk of `batch` realisations runs as concurrently: the
// plan's setting (ssfm_plan_set_forward_streams), at most one per
// realisation; by default two when each part still holds at least 256
// column tiles (measured on 2^16 dual-polarisation fields: from 16
// realisations on two parts are 2-20 % faster, at 2 realisations 15 %
// slower), else one.
// Parts of a chunk on separate streams fill the tail of each pass (its last,
// partly occupied round of workgroups) with the other parts' work, when the
// streams reach the GPU through different hardware queues (which the
// streams' creation order decides, not this library); together they keep
// the chunk's working set.
constexpr int64_t kPartTiles = 256;
int forward_parts(const ssfm_plan_s* p, int64_t batch) {
  if (p->ks.path != 2) return 1;
  int parts = p->forward_streams;
  if (parts == 0) parts = batch * (p->ks.n2 / p->ks.wide.columns) >= 2 * kPartTiles ? 2 : 1;
  return (int)std::max<int64_t>(1, std::min<int64_t>(parts, batch));
}

// Run part(0, st) on the caller's stream and part(k, w_k), k = 1..parts-1,
// on worker streams forked from st and joined back into it (also after an
// error, so that no work is left unordered).
template <typename F>
int run_split(ssfm_plan_s* p, hipStream_t st, int parts, F&& part) {
  hipStream_t ws[kBatchStreams];
  int rc = batch_streams(p->device, ws);
  if (rc != SSFM_OK) return rc;
  parts = std::min(parts, kBatchStreams + 1);
  hipEvent_t fork = nullptr, join[kBatchStreams] = {};
  auto destroy = [&] {
    if (fork) (void)hipEventDestroy(fork);
    for (hipEvent_t x : join)
      if (x) (void)hipEventDestroy(x);
  };
  hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  for (int k = 1; k < parts && e == hipSuccess; ++k)
    e = hipEventCreateWithFlags(&join[k - 1], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(fork, st);
  for (int k = 1; k < parts && e == hipSuccess; ++k) e = hipStreamWaitEvent(ws[k - 1], fork, 0);
  if (e != hipSuccess) {
    destroy();
    return api_fail_hip(e, "sub-batch fork");
  }
  for (int k = parts - 1; k >= 1 && rc == SSFM_OK; --k) rc = part(k, ws[k - 1]);
  if (rc == SSFM_OK) rc = part(0, st);
  hipError_t ej = hipSuccess;
  for (int k = 1; k < parts; ++k) {
    hipError_t x = hipEventRecord(join[k - 1], ws[k - 1]);
    if (x == hipSuccess) x = hipStreamWaitEvent(st, join[k - 1], 0);
    if (ej == hipSuccess) ej = x;
  }
  destroy();
  if (rc != SSFM_OK) return rc;
  if (ej != hipSuccess) return api_fail_hip(ej, "sub-batch join");
  return SSFM_OK;
}

// part(off, count, stream) over the realisations [0, nb) of a chunk: as one
// part on st, or as forward_parts() consecutive parts of nearly equal size,
// the first on st and the others on worker streams.
template <typename F>
int run_parts(ssfm_plan_s* p, int64_t nb, hipStream_t st, F&& part) {
  const int parts = std::min(forward_parts(p, nb), kBatchStreams + 1);
  if (parts < 2) return part(int64_t{0}, nb, st);
  return run_split(p, st, parts, [&](int k, hipStream_t ws) {
    const int64_t o0 = nb * k / parts, o1 = nb * (k + 1) / parts;
    return part(o0, o1 - o0, ws);
  });
}

// run_forward over the batch in the sequential chunks of chunk_batch (plain
// forward calls: no checkpoints or stored states), each chunk as one or two
// concurrent parts; realisation b keeps its noise index real0 + b, so the
// bits are those of one whole-batch pass.
int run_forward_chunked(ssfm_plan_s* p, float2* field, int64_t batch, uint64_t seed,
                        uint64_t real0, int s0, int s1, hipStream_t st) {
  const int64_t cb = chunk_batch(p, batch, 1);
  const size_t elems = (size_t)p->n_pol * p->n;
  for (int64_t b0 = 0; b0 < batch; b0 += cb) {
    const int rc = run_parts(p, std::min(cb, batch - b0), st,
                             [&](int64_t off, int64_t nb, hipStream_t ws) {
                               return run_forward(p, field + (size_t)(b0 + off) * elems, nb, seed,
                                                  real0 + (uint64_t)(b0 + off), s0, s1, ws);
                             });
    if (rc != SSFM_OK) return rc;
  }
  return SSFM_OK;
}

// The adjoint's forward pass over `batch` realisations: the input copied
// into work, run through the link, keeping the span-end states at ckpt
// (span s at ckpt + s * ckpt_stride elements; 0: the batch's own slice) and
// the nonlinear-step inputs of the kept spans.
int adjoint_forward(ssfm_plan_s* plan, const void* field_in, int64_t batch, uint64_t seed,
                    uint64_t real0, hipStream_t st, float2* work, float2* ckpt,
                    size_t ckpt_stride, float2* states, int kept) {
  const size_t slice = (size_t)batch * plan->n_pol * plan->n;  // elements
  const hipError_t e =
      hipMemcpyAsync(work, field_in, slice * sizeof(float2), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return api_fail_hip(e, "hipMemcpyAsync (adjoint input)");
  return run_forward(plan, work, batch, seed, real0, 0, plan->spans, st, ckpt, nullptr,
                     kept > 0 ? states : nullptr, plan->spans - kept, ckpt_stride);
}

// The adjoint's reverse sweep over `batch` realisations: the cotangent taken
// from grad and returned there, the state rebuilt from the span checkpoints
// at ckpt (stride as for adjoint_forward), the kept spans' stored inputs.
int adjoint_reverse(ssfm_plan_s* plan, void* grad, int64_t batch, hipStream_t st,
                    float2* work, float2* ckpt, size_t ckpt_stride, float2* states, int kept) {
  const ssfm::KernelSet& ks = plan->ks;
  const size_t slice = (size_t)batch * plan->n_pol * plan->n;  // elements
  if (!ckpt_stride) ckpt_stride = slice;
  const int kept_span0 = plan->spans - kept;
  float2* cot = work + slice;
  hipError_t e;
  if ((e = hipMemcpyAsync(cot, grad, slice * sizeof(float2), hipMemcpyDeviceToDevice, st)) !=
      hipSuccess)
    return api_fail_hip(e, "hipMemcpyAsync (cotangent)");

  // reverse sweep: state and cotangent together, span by span
  const int64_t batch2 = 2 * batch;
  const ssfm::RowLaunch row = pick_shape(plan, batch2).row;
  const int64_t rows = batch2 * plan->n_pol * ks.n1;
  const double row_bytes = 2.0 * (double)batch2 * plan->n_pol * (double)plan->n * sizeof(float2);
  int log2_n2 = 0;
  while ((1 << log2_n2) < ks.n2) ++log2_n2;
  ssfm::RowArgs ra{};
  ra.field = work;
  ra.tw = plan->tw2;
  ra.twA = plan->twA;
  ra.twB = plan->twB;
  ra.n1 = ks.n1;
  ra.log2_n2 = log2_n2;
  ra.conj_h = 1;
  ssfm::AdjArgs aa{};
  aa.work = work;
  aa.tw1 = plan->tw1;
  aa.n2 = ks.n2;
  aa.n = plan->n;
  aa.batch = batch;
  aa.gspan = plan->gspan;
  // cotangent-only reverse sweep of a kept span: the forward column pass's
  // transforms, the conjugate row pass and the stored-state pullback
  const Shape4 shape1 = pick_shape(plan, batch);
  const int64_t rows1 = batch * plan->n_pol * ks.n1;
  const double bytes1 = 2.0 * (double)slice * sizeof(float2);
  ssfm::RowArgs rc1 = ra;
  rc1.field = cot;
  ssfm::ColArgs ca{};
  ca.field = cot;
  ca.tw1 = plan->tw1;
  ca.n2 = ks.n2;
  ca.n = plan->n;
  ca.gspan = plan->gspan;
  ca.sigma_h = 0.0;  // the pullback of the amplifier is the gain alone
  ssfm::AdjStoredArgs sa{};
  sa.cot = cot;
  sa.tw1 = plan->tw1;
  sa.n2 = ks.n2;
  sa.n = plan->n;
  for (int s = plan->spans - 1; s >= kept_span0; --s) {
    if ((e = launch(plan, KIND_COL, bytes1, st,
                    [&] { return shape1.cols->col[ssfm::MODE_FIRST](ca, batch, st); })) != hipSuccess)
      return api_fail_hip(e, "k3 launch (adjoint)");
    for (int i = plan->steps; i >= 0; --i) {
      rc1.H = (i == 0 || i == plan->steps) ? plan->h_half : plan->h_full;
      if ((e = launch(plan, KIND_ROW, bytes1, st, [&] { return shape1.row(rc1, rows1, st); })) !=
          hipSuccess)
        return api_fail_hip(e, "k2 launch (adjoint)");
      if (i > 0) {
        sa.kappa = plan->kappa[(size_t)(i - 1)];
        sa.state = states + ((size_t)(s - kept_span0) * plan->steps + (size_t)(i - 1)) * slice;
        if ((e = launch(plan, KIND_ADJ, 1.5 * bytes1, st,
                        [&] { return ks.adj_stored(sa, batch, st); })) != hipSuccess)
          return api_fail_hip(e, "k3_adj_stored launch");
      }
    }
    if ((e = launch(plan, KIND_COL, bytes1, st,
                    [&] { return shape1.cols->col[ssfm::MODE_LAST](ca, batch, st); })) != hipSuccess)
      return api_fail_hip(e, "k3 launch (adjoint)");
  }
  for (int s = kept_span0 - 1; s >= 0; --s) {
    aa.ckpt = ckpt + (size_t)s * ckpt_stride;
    if ((e = launch(plan, KIND_ADJ, row_bytes, st,
                    [&] { return ks.adj[ssfm::AMODE_FIRST](aa, st); })) != hipSuccess)
      return api_fail_hip(e, "k3_adj launch");
    for (int i = plan->steps; i >= 0; --i) {
      ra.H = (i == 0 || i == plan->steps) ? plan->h_half : plan->h_full;
      if ((e = launch(plan, KIND_ROW, row_bytes, st, [&] { return row(ra, rows, st); })) !=
          hipSuccess)
        return api_fail_hip(e, "k2 launch");
      if (i > 0) {
        aa.kappa = plan->kappa[(size_t)(i - 1)];
        if ((e = launch(plan, KIND_ADJ, row_bytes, st,
                        [&] { return ks.adj[ssfm::AMODE_NL](aa, st); })) != hipSuccess)
          return api_fail_hip(e, "k3_adj launch");
      }
    }
    if ((e = launch(plan, KIND_ADJ, row_bytes, st,
                    [&] { return ks.adj[ssfm::AMODE_LAST](aa, st); })) != hipSuccess)
      return api_fail_hip(e, "k3_adj launch");
  }
  if ((e = hipMemcpyAsync(grad, cot, slice * sizeof(float2), hipMemcpyDeviceToDevice, st)) !=
      hipSuccess)
    return api_fail_hip(e, "hipMemcpyAsync (gradient)");
  return SSFM_OK;
}

// The whole adjoint of `batch` realisations (noise indices real0 + b) on
// stream st, with the workspace regions of this (sub-)batch: work [2 batch]
// fields, ckpt [spans][batch], states [kept][steps][batch].
int run_adjoint(ssfm_plan_s* plan, const void* field_in, void* grad, int64_t batch, uint64_t seed,
                uint64_t real0, hipStream_t st, float2* work, float2* ckpt, float2* states,
                int kept) {
  const int rc = adjoint_forward(plan, field_in, batch, seed, real0, st, work, ckpt, 0, states, kept);
  if (rc != SSFM_OK) return rc;
  return adjoint_reverse(plan, grad, batch, st, work, ckpt, 0, states, kept);
}


// The adjoint on the LDS-resident path: one launch (k1_adj) over the batch,
// with the span inputs in ckpt ([batch][spans] fields) and one span's
// nonlinear-step inputs per realisation in states ([batch][steps] fields).
int run_adjoint_lds(ssfm_plan_s* plan, const void* field_in, void* grad, int64_t batch,
                    uint64_t seed, hipStream_t st, float2* ckpt, float2* states) {
  ssfm::LdsArgs a{};
  a.h_half = plan->h_half;
  a.h_full = plan->h_full;
  a.tw = plan->tw_n;
  a.kappa = plan->d_kappa;
  a.steps = plan->steps;
  a.span_begin = 0;
  a.span_end = plan->spans;
  a.gspan = plan->gspan;
  a.sigma_h = plan->sigma_h;
  a.seed = seed;
  a.realization0 = 0;
  a.field_in = static_cast<const float2*>(field_in);
  a.grad = static_cast<float2*>(grad);
  a.ckpt = ckpt;
  a.states = states;
  // the forward pass, the recomputation and the reverse sweep of every span
  const double bytes = 2.0 * (double)batch * plan->n_pol * (double)plan->n * sizeof(float2);
  const hipError_t e =
      launch(plan, KIND_LDS, bytes, st, [&] { return plan->ks.lds_adj(a, batch, st); });
  if (e != hipSuccess) return api_fail_hip(e, "k1_adj launch");
  return SSFM_OK;
}

// Workspace of an adjoint call, in elements: the four-step path's work
// fields (state and cotangent) and span checkpoints; the LDS-resident path's
// span inputs and one span's nonlinear-step inputs.
void adjoint_workspace(const ssfm_plan_s* plan, int64_t batch, size_t* work, size_t* ckpt) {
  const size_t slice = (size_t)batch * plan->n_pol * plan->n;
  if (plan->ks.path == 1) {
    *work = (size_t)plan->steps * slice;
    *ckpt = (size_t)plan->spans * slice;
  } else {
    *work = 2 * slice;
    *ckpt = (size_t)plan->spans * slice;
  }
}

// ssfm_adjoint with the plan's adjoint lock held and the stream ordered after
// the previous adjoint call.
int adjoint_serialised(ssfm_plan_s* plan, const void* field_in, void* grad, int64_t batch,
                       uint64_t seed, hipStream_t st) {
  // The batch in sequential chunks sized for two fields (state and
  // cotangent), each chunk as one or two concurrent parts (run_parts, each
  // part on its own share of the chunk's workspace).  Without kept spans the
  // forward pass first runs over the whole batch in the forward's one-field
  // chunks, keeping every realisation's span checkpoints, then the reverse
  // sweep runs chunk by chunk; with kept spans each chunk's whole adjoint
  // runs on the workspace of one chunk, the state budget applied per chunk.
  const int64_t cb = chunk_batch(plan, batch, 2);
  const int64_t fb = chunk_batch(plan, batch, 1);
  const size_t elems = (size_t)plan->n_pol * plan->n;
  const size_t slice = (size_t)cb * elems;
  const size_t span_state_bytes = (size_t)plan->steps * slice * sizeof(float2);
  const bool two_phase = plan->ks.path == 2 && cb < batch &&
                         plan->state_budget < span_state_bytes;
  size_t work_elems, ckpt_elems;
  adjoint_workspace(plan, cb, &work_elems, &ckpt_elems);
  if (two_phase) {
    work_elems = std::max(work_elems, (size_t)fb * elems);
    ckpt_elems = (size_t)plan->spans * batch * elems;
  }
  const size_t ckpt_bytes = ckpt_elems * sizeof(float2);
  const size_t work_bytes = work_elems * sizeof(float2);
  if (ckpt_bytes > plan->adj_ckpt_bytes || work_bytes > plan->adj_work_bytes) {
    // grow the workspace, once the previous call's work is done with it
    if (plan->adj_pending) {
      const hipError_t e = hipEventSynchronize(plan->adj_done);
      if (e != hipSuccess) return api_fail_hip(e, "hipEventSynchronize (adjoint workspace)");
    }
    if (plan->adj_ckpt) (void)hipFree(plan->adj_ckpt);
    if (plan->adj_work) (void)hipFree(plan->adj_work);
    plan->adj_ckpt = plan->adj_work = nullptr;
    plan->adj_ckpt_bytes = plan->adj_work_bytes = 0;
    if (hipMalloc(&plan->adj_ckpt, ckpt_bytes) != hipSuccess ||
        hipMalloc(&plan->adj_work, work_bytes) != hipSuccess) {
      if (plan->adj_ckpt) (void)hipFree(plan->adj_ckpt);
      plan->adj_ckpt = nullptr;
      return api_fail(SSFM_ENOMEM, "adjoint workspace of %zu bytes", ckpt_bytes + work_bytes);
    }
    plan->adj_ckpt_bytes = ckpt_bytes;
    plan->adj_work_bytes = work_bytes;
  }
  if (plan->ks.path == 1)
    return run_adjoint_lds(plan, field_in, grad, batch, seed, st, plan->adj_ckpt, plan->adj_work);
  if (two_phase) {
    const size_t stride = (size_t)batch * elems;  // between spans' checkpoints
    // a part at offset off of a chunk: its realisations' slice of the work
    // buffer (one field in the forward pass, state and cotangent in the
    // reverse sweep) and of every span's checkpoints
    for (int64_t b0 = 0; b0 < batch; b0 += fb) {
      const int rc = run_parts(plan, std::min(fb, batch - b0), st,
                               [&](int64_t off, int64_t nb, hipStream_t ws) {
                                 const size_t o = (size_t)(b0 + off) * elems;
                                 return adjoint_forward(
                                     plan, static_cast<const float2*>(field_in) + o, nb, seed,
                                     (uint64_t)(b0 + off), ws, plan->adj_work + (size_t)off * elems,
                                     plan->adj_ckpt + o, stride, nullptr, 0);
                               });
      if (rc != SSFM_OK) return rc;
    }
    for (int64_t b0 = 0; b0 < batch; b0 += cb) {
      const int rc = run_parts(plan, std::min(cb, batch - b0), st,
                               [&](int64_t off, int64_t nb, hipStream_t ws) {
                                 const size_t o = (size_t)(b0 + off) * elems;
                                 return adjoint_reverse(
                                     plan, static_cast<float2*>(grad) + o, nb, ws,
                                     plan->adj_work + 2 * (size_t)off * elems, plan->adj_ckpt + o,
                                     stride, nullptr, 0);
                               });
      if (rc != SSFM_OK) return rc;
    }
    return SSFM_OK;
  }
  // trailing spans whose nonlinear-step inputs the forward pass keeps, as
  // many as the plan's state budget holds (grown on demand; an allocation
  // the device refuses lowers the count)
  int kept = (int)std::min<uint64_t>((uint64_t)plan->spans, plan->state_budget / span_state_bytes);
  if ((size_t)kept * span_state_bytes > plan->adj_states_bytes) {
    if (plan->adj_pending) {
      const hipError_t e = hipEventSynchronize(plan->adj_done);
      if (e != hipSuccess) return api_fail_hip(e, "hipEventSynchronize (adjoint states)");
    }
    if (plan->adj_states) (void)hipFree(plan->adj_states);
    plan->adj_states = nullptr;
    plan->adj_states_bytes = 0;
    // SSFM_FAIL_STATE_ALLOC=k (tests): a store of more than k spans is refused
    const int fail_above = env_count("SSFM_FAIL_STATE_ALLOC");
    while (kept > 0 && ((fail_above > 0 && kept > fail_above) ||
                        hipMalloc(&plan->adj_states, (size_t)kept * span_state_bytes) != hipSuccess)) {
      (void)hipGetLastError();
      plan->adj_states = nullptr;
      --kept;
    }
    if (kept > 0) plan->adj_states_bytes = (size_t)kept * span_state_bytes;
  }
  // the chunks one after the other, a part at offset off of a chunk on its
  // realisations' share of the chunk's work, checkpoints and stored states
  for (int64_t b0 = 0; b0 < batch; b0 += cb) {
    const int rc = run_parts(
        plan, std::min(cb, batch - b0), st, [&](int64_t off, int64_t nb, hipStream_t ws) {
          const size_t o = (size_t)(b0 + off) * elems, oc = (size_t)off * elems;
          return run_adjoint(plan, static_cast<const float2*>(field_in) + o,
                             static_cast<float2*>(grad) + o, nb, seed, (uint64_t)(b0 + off), ws,
                             plan->adj_work + 2 * oc, plan->adj_ckpt + (size_t)plan->spans * oc,
                             plan->adj_states ? plan->adj_states + (size_t)kept * plan->steps * oc
                                              : nullptr,
                             kept);
        });
    if (rc != SSFM_OK) return rc;
  }
  return SSFM_OK;
}


}  // namespace

extern "C" {

int ssfm_plan(const ssfm_link* link, int hip_device, ssfm_plan_t* out) {
  ssfm::api_clear_error();
  if (!out) return api_fail(SSFM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_link(link);
  if (rc != SSFM_OK) return rc;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return api_fail_hip(e, "hipGetDeviceCount");
  if (hip_device < 0 || hip_device >= count)
    return api_fail(SSFM_EINVAL, "hip_device %d out of range (%d devices)", hip_device, count);
  DeviceGuard guard(hip_device);
  if (guard.status != hipSuccess) return api_fail_hip(guard.status, "hipSetDevice");
  // set-up of ssfm_adjoint_noalloc's device scratch (once per device); a
  // failure is reported by that call, not here
  resolve_scratch(hip_device);

  ssfm_plan_s* p = new (std::nothrow) ssfm_plan_s();
  if (!p) return api_fail(SSFM_ENOMEM, "host allocation of the plan failed");
  p->link = *link;
  p->device = hip_device;
  p->n_pol = link->n_pol;
  p->n = link->n_samples;
  p->steps = link->steps_per_span;
  p->spans = link->n_spans;
  // sequential chunks of about 256 MiB (the Infinity Cache); SSFM_CHUNK_MIB
  // sets another size in MiB, 0 turns chunking off
  {
    const char* env = getenv("SSFM_CHUNK_MIB");
    p->chunk_bytes = (size_t)(env ? std::max(0, atoi(env)) : 256) << 20;
  }
  // concurrent parts per chunk: SSFM_FORWARD_STREAMS (0..5) sets the plan's
  // initial setting, as ssfm_plan_set_forward_streams would
  {
    const char* env = getenv("SSFM_FORWARD_STREAMS");
    if (env) p->forward_streams = std::min(std::max(0, atoi(env)), kBatchStreams + 1);
  }
  if (!ssfm::select_kernels(p->n, p->n_pol, (link->flags & SSFM_FLAG_FP32_ARITHMETIC) != 0, p->ks)) {
    delete p;
    return api_fail(SSFM_EUNSUPPORTED, "no kernel for n_samples = %lld", (long long)link->n_samples);
  }
  if (p->ks.prepare != hipSuccess) {
    const hipError_t pe = p->ks.prepare;
    delete p;
    return api_fail_hip(pe, "hipFuncSetAttribute (LDS size)");
  }
  rc = build_tables(p);
  if (rc != SSFM_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return SSFM_OK;
}

int ssfm_plan_destroy(ssfm_plan_t plan) {
  if (!plan) return SSFM_OK;
  DeviceGuard guard(plan->device);
  delete plan;
  return SSFM_OK;
}

int ssfm_plan_get_info(ssfm_plan_t plan, ssfm_plan_info* info) {
  if (!plan || !info) return api_fail(SSFM_EINVAL, "plan and info must be non-NULL");
  info->path = plan->ks.path;
  info->n1 = plan->ks.path == 2 ? plan->ks.n1 : 0;
  info->n2 = plan->ks.path == 2 ? plan->ks.n2 : 0;
  info->columns_per_tile = plan->ks.path == 2 ? plan->ks.wide.columns : 0;
  info->launches_per_call = launches_per_call(plan);
  info->table_bytes = (int64_t)plan->table_bytes;
  info->chunk_realisations = chunk_max(plan, 1);
  return SSFM_OK;
}

int ssfm_forward_spans(ssfm_plan_t plan, void* field, int64_t batch, uint64_t seed,
                       uint64_t realization0, int32_t span_begin, int32_t span_end,
                       void* stream) {
  ssfm::api_clear_error();
  int rc = check_call(plan, field, batch);
  if (rc != SSFM_OK) return rc;
  if (span_begin < 0 || span_end < span_begin || span_end > plan->spans)
    return api_fail(SSFM_EINVAL, "span range [%d, %d) outside [0, %d]", span_begin, span_end,
                plan->spans);
  DeviceGuard guard(plan->device);
  if (guard.status != hipSuccess) return api_fail_hip(guard.status, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  // two concurrent parts per chunk: no graph replay (the two streams'
  // launches interleave)
  if (forward_parts(plan, batch) > 1 || !use_graphs(plan))
    return run_forward_chunked(plan, static_cast<float2*>(field), batch, seed, realization0,
                               span_begin, span_end, st);
  // A call repeating the previous one (same buffer, batch, seed, spans and
  // stream) replays its captured launch sequence: one graph launch instead of
  // thousands of kernel launches.  The first occurrence runs directly.
  ssfm_plan_s::GraphKey key;
  key.field = field;
  key.batch = batch;
  key.seed = seed;
  key.real0 = realization0;
  key.s0 = span_begin;
  key.s1 = span_end;
  key.stream = stream;
  std::lock_guard<std::mutex> lock(plan->graph_mu);
  const bool repeat = plan->have_last && plan->last_key == key;
  if (!repeat) {
    plan->last_key = key;
    plan->have_last = true;
    if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
    plan->graph_exec = nullptr;
    plan->graph_valid = false;
    return run_forward_chunked(plan, static_cast<float2*>(field), batch, seed, realization0,
                               span_begin, span_end, st);
  }
  if (!plan->graph_valid) {
    hipError_t e;
    if (!plan->capture_stream &&
        (e = hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking)) != hipSuccess)
      return api_fail_hip(e, "hipStreamCreate (capture)");
    if ((e = hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeThreadLocal)) !=
        hipSuccess)
      return api_fail_hip(e, "hipStreamBeginCapture");
    const int rc2 = run_forward_chunked(plan, static_cast<float2*>(field), batch, seed,
                                        realization0, span_begin, span_end, plan->capture_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(plan->capture_stream, &graph);
    if (rc2 != SSFM_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc2;
    }
    if (e != hipSuccess) return api_fail_hip(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&plan->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      plan->graph_exec = nullptr;
      return api_fail_hip(e, "hipGraphInstantiate");
    }
    plan->graph_valid = true;
  }
  const hipError_t e = hipGraphLaunch(plan->graph_exec, st);
  if (e != hipSuccess) return api_fail_hip(e, "hipGraphLaunch");
  return SSFM_OK;
}

int ssfm_forward(ssfm_plan_t plan, void* field, int64_t batch, uint64_t seed, void* stream) {
  if (!plan) return api_fail(SSFM_EINVAL, "plan is NULL");
  return ssfm_forward_spans(plan, field, batch, seed, 0, 0, plan->spans, stream);
}

int ssfm_dft(ssfm_plan_t plan, void* field, int64_t batch, int32_t inverse, void* stream) {
  ssfm::api_clear_error();
  int rc = check_call(plan, field, batch);
  if (rc != SSFM_OK) return rc;
  if (inverse != 0 && inverse != 1) return api_fail(SSFM_EINVAL, "inverse must be 0 or 1");
  DeviceGuard guard(plan->device);
  if (guard.status != hipSuccess) return api_fail_hip(guard.status, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  float2* f = static_cast<float2*>(field);
  const ssfm::KernelSet& ks = plan->ks;
  const double bytes = 2.0 * (double)batch * plan->n_pol * (double)plan->n * sizeof(float2);
  hipError_t e;
  if (ks.path == 1) {
    if ((e = launch(plan, KIND_LDS, bytes, st,
                    [&] { return ks.lds_dft[inverse](f, plan->tw_n, batch, st); })) != hipSuccess)
      return api_fail_hip(e, "k1_dft launch");
    return SSFM_OK;
  }
  const Shape4 shape = pick_shape(plan, batch);
  int log2_n2 = 0;
  while ((1 << log2_n2) < ks.n2) ++log2_n2;
  ssfm::RowArgs ra{};
  ra.field = f;
  ra.H = plan->h_full;  // not read by the transform-only row passes
  ra.tw = plan->tw2;
  ra.twA = plan->twA;
  ra.twB = plan->twB;
  ra.n1 = ks.n1;
  ra.log2_n2 = log2_n2;
  ra.part = inverse ? ssfm::ROW_IFFT : ssfm::ROW_FFT;
  ssfm::ColArgs ca{};
  ca.field = f;
  ca.tw1 = plan->tw1;
  ca.n2 = ks.n2;
  ca.n = plan->n;
  const int64_t rows = batch * plan->n_pol * ks.n1;
  auto col = [&](int mode) {
    return launch(plan, KIND_COL, bytes, st, [&] { return shape.cols->col[mode](ca, batch, st); });
  };
  auto row = [&] { return launch(plan, KIND_ROW, bytes, st, [&] { return shape.row(ra, rows, st); }); };
  if (!inverse) {
    if ((e = col(ssfm::MODE_FIRST)) != hipSuccess) return api_fail_hip(e, "k3 launch (dft)");
    if ((e = row()) != hipSuccess) return api_fail_hip(e, "k2 launch (dft)");
  } else {
    if ((e = row()) != hipSuccess) return api_fail_hip(e, "k2 launch (dft)");
    if ((e = col(ssfm::MODE_IFFT)) != hipSuccess) return api_fail_hip(e, "k3 launch (dft)");
  }
  return SSFM_OK;
}

int ssfm_adjoint(ssfm_plan_t plan, const void* field_in, void* grad, int64_t batch,
                 uint64_t seed, void* stream) {
  ssfm::api_clear_error();
  int rc = check_call(plan, field_in, batch);
  if (rc != SSFM_OK) return rc;
  if (!grad) return api_fail(SSFM_EINVAL, "grad is NULL");
  if (((uintptr_t)grad & 7u) != 0) return api_fail(SSFM_EINVAL, "grad must be 8-byte aligned");
  if (plan->ks.fp32)
    return api_fail(SSFM_EUNSUPPORTED, "ssfm_adjoint: no adjoint for the FP32-arithmetic variant");
  DeviceGuard guard(plan->device);
  if (guard.status != hipSuccess) return api_fail_hip(guard.status, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(plan->adj_mu);
  hipError_t e;
  if (!plan->adj_done &&
      (e = hipEventCreateWithFlags(&plan->adj_done, hipEventDisableTiming)) != hipSuccess) {
    plan->adj_done = nullptr;
    return api_fail_hip(e, "hipEventCreate (adjoint order)");
  }
  // this call starts after the previous adjoint call's work, on any stream
  if (plan->adj_pending && (e = hipStreamWaitEvent(st, plan->adj_done, 0)) != hipSuccess)
    return api_fail_hip(e, "hipStreamWaitEvent (adjoint order)");
  rc = adjoint_serialised(plan, field_in, grad, batch, seed, st);
  if ((e = hipEventRecord(plan->adj_done, st)) != hipSuccess) {
    plan->adj_pending = false;
    return rc != SSFM_OK ? rc : api_fail_hip(e, "hipEventRecord (adjoint order)");
  }
  plan->adj_pending = true;
  return rc;
}

int ssfm_adjoint_noalloc(ssfm_plan_t plan, const void* field_in, void* grad, int64_t batch,
                         uint64_t seed, void* stream) {
  ssfm::api_clear_error();
  int rc = check_call(plan, field_in, batch);
  if (rc != SSFM_OK) return rc;
  if (!grad) return api_fail(SSFM_EINVAL, "grad is NULL");
  if (((uintptr_t)grad & 7u) != 0) return api_fail(SSFM_EINVAL, "grad must be 8-byte aligned");
  if (plan->ks.fp32)
    return api_fail(SSFM_EUNSUPPORTED, "ssfm_adjoint_noalloc: no adjoint for the FP32-arithmetic variant");
  if (plan->profiling)
    return api_fail(SSFM_EINVAL, "ssfm_adjoint_noalloc: a profiling window is open on the plan "
                                 "(its per-launch events would be created here)");
  // four-step path: work [2][batch] fields, then checkpoints [spans][batch];
  // LDS-resident path: [batch][steps] step inputs, then [batch][spans] span inputs
  size_t work_elems, ckpt_elems;
  adjoint_workspace(plan, batch, &work_elems, &ckpt_elems);
  const uint64_t need = (uint64_t)(work_elems + ckpt_elems) * sizeof(float2);
  if (need > kNoallocScratchBytes)
    return api_fail(SSFM_EINVAL,
                    "ssfm_adjoint_noalloc: the workspace of %llu bytes exceeds the %llu-byte "
                    "device scratch; use ssfm_adjoint or a smaller batch",
                    (unsigned long long)need, (unsigned long long)kNoallocScratchBytes);
  hipError_t why;
  float2* base = static_cast<float2*>(scratch_ptr(plan->device, &why));
  if (!base) return api_fail_hip(why, "ssfm_adjoint_noalloc: device scratch address");
  DeviceGuard guard(plan->device);
  if (guard.status != hipSuccess) return api_fail_hip(guard.status, "hipSetDevice");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  if (plan->ks.path == 1)
    return run_adjoint_lds(plan, field_in, grad, batch, seed, st, base + work_elems, base);
  return run_adjoint(plan, field_in, grad, batch, seed, 0, st, base, base + work_elems, nullptr, 0);
}


int ssfm_plan_set_forward_streams(ssfm_plan_t plan, int32_t streams) {
  ssfm::api_clear_error();
  if (!plan) return api_fail(SSFM_EINVAL, "plan is NULL");
  if (streams < 0 || streams > kBatchStreams + 1)
    return api_fail(SSFM_EINVAL, "streams must be 0 (default) .. %d, got %d", kBatchStreams + 1,
                    streams);
  plan->forward_streams = streams;
  return SSFM_OK;
}

int ssfm_plan_set_state_memory(ssfm_plan_t plan, uint64_t bytes) {
  ssfm::api_clear_error();
  if (!plan) return api_fail(SSFM_EINVAL, "plan is NULL");
  std::lock_guard<std::mutex> lock(plan->adj_mu);
  plan->state_budget = bytes;
  if (plan->adj_states && plan->adj_states_bytes > bytes) {
    DeviceGuard guard(plan->device);
    if (guard.status != hipSuccess) return api_fail_hip(guard.status, "hipSetDevice");
    if (plan->adj_pending) {  // the last adjoint call's work may still read it
      const hipError_t e = hipEventSynchronize(plan->adj_done);
      if (e != hipSuccess) return api_fail_hip(e, "hipEventSynchronize (adjoint states)");
    }
    (void)hipFree(plan->adj_states);
    plan->adj_states = nullptr;
    plan->adj_states_bytes = 0;
  }
  return SSFM_OK;
}

int ssfm_batch(const ssfm_link* links, void* const* fields, int64_t count,
               const uint64_t* seeds, int hip_device, void* stream) {
  ssfm::api_clear_error();
  if (!links || !fields || !seeds) return api_fail(SSFM_EINVAL, "links, fields and seeds must be non-NULL");
  if (count < 1) return api_fail(SSFM_EINVAL, "count must be >= 1");
  for (int64_t i = 0; i < count; ++i) {
    int rc = validate_link(&links[i]);
    if (rc != SSFM_OK) return rc;
    if (!fields[i]) return api_fail(SSFM_EINVAL, "fields[%lld] is NULL", (long long)i);
    if (((uintptr_t)fields[i] & 7u) != 0)
      return api_fail(SSFM_EINVAL, "fields[%lld] must be 8-byte aligned", (long long)i);
  }
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return api_fail_hip(e, "hipGetDeviceCount");
  if (hip_device < 0 || hip_device >= ndev)
    return api_fail(SSFM_EINVAL, "hip_device %d out of range (%d devices)", hip_device, ndev);
  DeviceGuard guard(hip_device);
  if (guard.status != hipSuccess) return api_fail_hip(guard.status, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  BatchSchedule bs;
  int rc = make_batch_schedule(links, count, hip_device, &bs);
  if (rc != SSFM_OK) return rc;
  hipStream_t ws[kBatchStreams];
  if ((rc = batch_streams(hip_device, ws)) != SSFM_OK) return rc;

  const char* genv = getenv("SSFM_GRAPH");
  if (genv && strcmp(genv, "0") == 0)
    return enqueue_batch(bs, links, fields, seeds, st, ws, nullptr);
  // A call repeating the previous one (same entries, fields, seeds, device
  // and stream) replays the launch sequence captured on its first repeat;
  // other calls run directly.
  BatchReplay& rp = batch_replay();
  std::lock_guard<std::mutex> lock(rp.mu);
  const bool repeat = rp.matches(links, fields, count, seeds, hip_device, stream);
  if (!repeat) {
    if ((rc = rp.release()) != SSFM_OK) return rc;
    rp.remember(links, fields, count, seeds, hip_device, stream);
    return enqueue_batch(bs, links, fields, seeds, st, ws, nullptr);
  }
  if (!rp.exec) {
    // launch shapes measured for every active count of every four-step group
    for (size_t gi = 0; gi < bs.groups.size(); ++gi) {
      ssfm_plan_t pl = bs.plans[gi];
      if (pl->ks.path != 2) continue;
      for (int64_t active : bs.active_counts[gi]) {
        bool have;
        {
          std::lock_guard<std::mutex> tl(pl->tune_mu);
          have = pl->tuned.count(active) != 0;
        }
        ssfm_tune_info info;
        if (!have && (rc = ssfm_plan_autotune(pl, active, stream, &info)) != SSFM_OK) return rc;
      }
    }
    // staging fields and device seeds owned by the graph
    BatchStaging stage;
    for (size_t gi = 0; gi < bs.groups.size(); ++gi) {
      const ssfm_plan_s* pl = bs.plans[gi];
      const size_t m = bs.groups[gi].size();
      float2* f = nullptr;
      uint64_t* sd = nullptr;
      if (hipMalloc(&f, m * (size_t)pl->n_pol * (size_t)pl->n * sizeof(float2)) != hipSuccess) {
        stage.release();
        return api_fail(SSFM_ENOMEM, "ssfm_batch replay staging");
      }
      stage.fields.push_back(f);
      if (hipMalloc(&sd, m * sizeof(uint64_t)) != hipSuccess) {
        stage.release();
        return api_fail(SSFM_ENOMEM, "ssfm_batch replay seeds");
      }
      stage.seeds.push_back(sd);
      std::vector<uint64_t> hs(m);
      for (size_t r = 0; r < m; ++r) hs[r] = seeds[bs.groups[gi][r]];
      if ((e = hipMemcpy(sd, hs.data(), m * sizeof(uint64_t), hipMemcpyHostToDevice)) != hipSuccess) {
        stage.release();
        return api_fail_hip(e, "ssfm_batch replay seeds");
      }
    }
    if (!rp.capture &&
        (e = hipStreamCreateWithFlags(&rp.capture, hipStreamNonBlocking)) != hipSuccess) {
      rp.capture = nullptr;
      stage.release();
      return api_fail_hip(e, "hipStreamCreate (batch capture)");
    }
    if ((e = hipStreamBeginCapture(rp.capture, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
      stage.release();
      return api_fail_hip(e, "hipStreamBeginCapture (batch)");
    }
    rc = enqueue_batch(bs, links, fields, seeds, rp.capture, ws, &stage);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(rp.capture, &graph);
    if (rc == SSFM_OK && e != hipSuccess) rc = api_fail_hip(e, "hipStreamEndCapture (batch)");
    if (rc == SSFM_OK) {
      e = hipGraphInstantiate(&rp.exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        rp.exec = nullptr;
        rc = api_fail_hip(e, "hipGraphInstantiate (batch)");
      }
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (rc != SSFM_OK) {
      stage.release();
      rp.have_last = false;
      return rc;
    }
    rp.stage = std::move(stage);
  }
  if ((e = hipGraphLaunch(rp.exec, st)) != hipSuccess) return api_fail_hip(e, "hipGraphLaunch (batch)");
  if (!rp.done && (e = hipEventCreateWithFlags(&rp.done, hipEventDisableTiming)) != hipSuccess) {
    rp.done = nullptr;
    return api_fail_hip(e, "hipEventCreate (batch replay)");
  }
  if ((e = hipEventRecord(rp.done, st)) != hipSuccess) return api_fail_hip(e, "hipEventRecord (batch replay)");
  rp.pending = true;
  return SSFM_OK;
}

int ssfm_plan_autotune(ssfm_plan_t plan, int64_t batch, void* stream, ssfm_tune_info* info) {
  ssfm::api_clear_error();
  if (!plan || !info) return api_fail(SSFM_EINVAL, "NULL plan or info");
  if (batch < 1) return api_fail(SSFM_EINVAL, "batch must be >= 1 (got %lld)", (long long)batch);
  *info = ssfm_tune_info{};
  const ssfm::KernelSet& ks = plan->ks;
  if (ks.path != 2) return SSFM_OK;
  DeviceGuard guard(plan->device);
  if (guard.status != hipSuccess) return api_fail_hip(guard.status, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  // a forward call runs larger batches in chunks, each as one or more
  // concurrent parts: tune the shape of the largest part
  const int64_t chunk = chunk_batch(plan, batch, 1);
  const int parts = forward_parts(plan, chunk);
  batch = (chunk + parts - 1) / parts;
  const size_t bytes = (size_t)batch * plan->n_pol * plan->n * sizeof(float2);
  float2* f = nullptr;
  if (hipMalloc(&f, bytes) != hipSuccess)
    return api_fail(SSFM_ENOMEM, "autotune scratch field of %zu bytes", bytes);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // a nonzero field (0.01 + 0.01i everywhere): the kernels run measurably
  // faster on an all-zero one
  hipError_t e = hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(f), 0x3c23d70au, bytes / 4, st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int log2_n2 = 0;
  while ((1 << log2_n2) < ks.n2) ++log2_n2;
  ssfm::RowArgs ra{};
  ra.field = f;
  ra.H = plan->h_full;
  ra.tw = plan->tw2;
  ra.twA = plan->twA;
  ra.twB = plan->twB;
  ra.n1 = ks.n1;
  ra.log2_n2 = log2_n2;
  ssfm::ColArgs a{};
  a.field = f;
  a.tw1 = plan->tw1;
  a.n2 = ks.n2;
  a.n = plan->n;
  a.kappa = plan->kappa.empty() ? 0.0 : plan->kappa[0];
  const int64_t rows = batch * plan->n_pol * ks.n1;
  double best = 0.0;
  int best_idx = -1;
  for (int idx = 0; idx < 4 && e == hipSuccess; ++idx) {
    const ssfm::FourStepKernels& cols = (idx >> 1) ? ks.wide : ks.narrow;
    const ssfm::RowLaunch row = (idx & 1) ? ks.row_wide : ks.row_narrow;
    // one split step: row pass, nonlinear column pass
    auto step = [&]() -> hipError_t {
      hipError_t r = row(ra, rows, st);
      return r == hipSuccess ? cols.col[ssfm::MODE_NL](a, batch, st) : r;
    };
    if ((e = step()) != hipSuccess) break;  // warm-up
    int reps = 3, timed = 0;
    float ms = 0.0f;
    for (int round = 0; round < 3 && e == hipSuccess; ++round) {
      if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = step();
      if (e != hipSuccess || (e = hipEventRecord(e1, st)) != hipSuccess) break;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      timed = reps;
      // at least ~2 ms of work in the measured round
      if (ms >= 2.0f || reps >= 4000) break;
      reps = (int)std::min<double>(4000.0, std::ceil(reps * 2.5 / std::max(ms, 1e-3f)));
    }
    if (e != hipSuccess) break;
    info->us_per_step[idx] = 1e3 * (double)ms / timed;
    if (best_idx < 0 || info->us_per_step[idx] < best) {
      best = info->us_per_step[idx];
      best_idx = idx;
    }
  }
  const hipError_t es = hipStreamSynchronize(st);
  (void)hipFree(f);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return api_fail_hip(e, "autotune");
  if (es != hipSuccess) return api_fail_hip(es, "autotune synchronise");
  ssfm_plan_s::Shape sh;
  sh.wide_cols = (best_idx >> 1) != 0;
  sh.wide_rows = (best_idx & 1) != 0;
  {
    // both part sizes of the chunk (they differ by at most one)
    std::lock_guard<std::mutex> lock(plan->tune_mu);
    plan->tuned[batch] = sh;
    plan->tuned[chunk / parts] = sh;
  }
  {
    // the replay graph may hold the previous shape
    std::lock_guard<std::mutex> lock(plan->graph_mu);
    plan->have_last = false;
    plan->graph_valid = false;
    if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
    plan->graph_exec = nullptr;
  }
  info->columns = sh.wide_cols ? ks.wide.columns : ks.narrow.columns;
  info->row_lanes = sh.wide_rows ? ks.rows_wide * (ks.n2 / 16) : ks.rows_narrow * (ks.n2 / 16);
  info->candidates = 4;
  return SSFM_OK;
}

int ssfm_profile_begin(ssfm_plan_t plan) {
  if (!plan) return api_fail(SSFM_EINVAL, "plan is NULL");
  plan->profiling = true;
  plan->prof.clear();
  return SSFM_OK;
}

int ssfm_profile_end(ssfm_plan_t plan, ssfm_kernel_stats* out, int capacity, int* count) {
  if (!plan || !out || !count) return api_fail(SSFM_EINVAL, "plan, out and count must be non-NULL");
  plan->profiling = false;
  DeviceGuard guard(plan->device);
  double ms[KIND_COUNT] = {0, 0, 0, 0}, bytes[KIND_COUNT] = {0, 0, 0, 0};
  int64_t n[KIND_COUNT] = {0, 0, 0, 0};
  // launches may have run on several streams: wait for each closing event
  for (const auto& r : plan->prof.records()) {
    hipError_t e = hipEventSynchronize(plan->prof.after(r));
    if (e != hipSuccess) return api_fail_hip(e, "hipEventSynchronize");
    float t = 0.0f;
    e = hipEventElapsedTime(&t, plan->prof.before(r), plan->prof.after(r));
    if (e != hipSuccess) return api_fail_hip(e, "hipEventElapsedTime");
    ms[r.kind] += t;
    bytes[r.kind] += r.bytes;
    n[r.kind] += 1;
  }
  int w = 0;
  for (int k = 0; k < KIND_COUNT && w < capacity; ++k) {
    if (!n[k]) continue;
    memset(&out[w], 0, sizeof out[w]);
    snprintf(out[w].name, sizeof out[w].name, "%s", kKindName[k]);
    out[w].launches = n[k];
    out[w].total_ms = ms[k];
    out[w].field_bytes = bytes[k];
    ++w;
  }
  *count = w;
  plan->prof.clear();
  return SSFM_OK;
}

const char* ssfm_status_string(int status) {
  switch (status) {
    case SSFM_OK: return "success";
    case SSFM_EINVAL: return "invalid argument";
    case SSFM_ENOMEM: return "out of memory";
    case SSFM_EHIP: return "HIP runtime error";
    case SSFM_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* ssfm_last_error(void) { return ssfm::api_last_error().c_str(); }

int ssfm_version(void) { return 100; }

}  // extern "C"
