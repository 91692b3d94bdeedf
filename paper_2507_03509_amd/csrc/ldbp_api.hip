// Host side of learned digital back-propagation: description checks, tile
// geometry, workspace and the C ABI declared in include/ssfm_ldbp.h.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "host_common.hpp"
#include "ldbp_internal.hpp"
#include "ssfm_ldbp.h"

using ssfm::cd;
using ssfm::api_fail;
using ssfm::api_fail_hip;
namespace L = ssfm::ldbp;

namespace {

// Tile geometry.  Forward: tiles of up to 1024 samples, up to 10 fused steps
// per launch (halo 7 per step).  Backward: one span per launch over regions
// of 1024 samples (tile plus halo: four whole waves of R samples per lane).
// SSFM_LDBP_FWD_TILE / SSFM_LDBP_FWD_STEPS / SSFM_LDBP_BWD_REGION override
// them (powers of two; for tuning).
constexpr int kFwdTile = 1024;
constexpr int kFwdSteps = 10;
constexpr int kBwdRegion = 1024;
constexpr int kFwdMaxRegion = 512 * L::R;  // forward workgroup <= 512 lanes
constexpr int kBwdMaxRegion = 256 * L::R;  // backward workgroup <= 256 lanes
constexpr int kLossSymbols = 256;          // symbols per loss workgroup
constexpr int kMfSamples = 1024;           // samples per matched-filter-adjoint workgroup

int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  if (!v || !*v) return dflt;
  const int x = atoi(v);
  return x > 0 ? x : dflt;
}

bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct Geometry {
  int w = 0, halo = 0, region = 0, ls = 0, tiles = 0, threads = 0;
  size_t lds = 0;
};

// slot: bytes of one LDS sample slot (FP64 complex in the forward, FP32
// complex in the backward)
Geometry make_geometry(int64_t n, int tile, int halo, int arrays, int n_pol, size_t slot) {
  Geometry g;
  g.w = (int)std::min<int64_t>(n, tile);
  g.halo = halo;
  g.region = round_up(g.w + 2 * halo, L::R);
  g.ls = L::region_stride(g.region);
  g.tiles = (int)((n + g.w - 1) / g.w);  // the last tile of a row may be shorter
  g.threads = round_up(g.region / L::R, 64);
  g.lds = (size_t)arrays * n_pol * g.ls * slot;
  return g;
}

int validate(const ssfm_ldbp_desc* d) {
  if (!d) return api_fail(SSFM_EINVAL, "NULL ldbp description");
  if (d->n_pol != 1 && d->n_pol != 2) return api_fail(SSFM_EINVAL, "n_pol must be 1 or 2 (got %d)", d->n_pol);
  if (d->n_steps < 1 || d->n_steps > 4096)
    return api_fail(SSFM_EINVAL, "n_steps must be in [1, 4096] (got %d)", d->n_steps);
  if (d->n_taps < 1 || d->n_taps > L::TAPS || d->n_taps % 2 == 0)
    return api_fail(SSFM_EINVAL, "n_taps must be odd and in [1, %d] (got %d)", L::TAPS, d->n_taps);
  if (d->steps_per_span < 1 || d->steps_per_span > 4 || d->n_steps % d->steps_per_span != 0)
    return api_fail(SSFM_EINVAL, "steps_per_span must be in [1, 4] and divide n_steps (got %d, %d)",
                    d->steps_per_span, d->n_steps);
  if (!pow2(d->n_samples) || d->n_samples < 64 || d->n_samples > (int64_t(1) << 22))
    return api_fail(SSFM_EINVAL, "n_samples must be a power of two in [2^6, 2^22] (got %lld)",
                    (long long)d->n_samples);
  if (d->sps < 1 || d->sps > 64 || d->n_samples % d->sps != 0)
    return api_fail(SSFM_EINVAL, "sps must be in [1, 64] and divide n_samples (got %d)", d->sps);
  if (d->mf_taps < 1 || d->mf_taps > 257 || d->mf_taps % 2 == 0)
    return api_fail(SSFM_EINVAL, "mf_taps must be odd and in [1, 257] (got %d)", d->mf_taps);
  return SSFM_OK;
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7) == 0; }

}  // namespace

struct ssfm_ldbp_s {
  ssfm_ldbp_desc d{};
  int device = 0;
  int fwd_tile = kFwdTile, fwd_steps = kFwdSteps, bwd_region = kBwdRegion;
  // parts of a call's batch run concurrently on the caller's stream and
  // the workers (forked and joined with the events): 0 two in the backward
  // by its launch size (run_halves), 1 none, 2..4 that many parts in the
  // forward and the backward; SSFM_LDBP_STREAMS
  int streams = 0;
  hipStream_t worker[3] = {};
  hipEvent_t fork_ev = nullptr, join_ev[3] = {};
  // workspace: padded taps [K][15], then a region sized for the largest call
  cd* taps15 = nullptr;
  unsigned char* ws = nullptr;
  size_t ws_bytes = 0;

  int64_t field_elems(int64_t batch) const { return batch * d.n_pol * d.n_samples; }
  int spans() const { return d.n_steps / d.steps_per_span; }
  int fwd_chunk() const {
    // fused steps per forward launch: whole spans, at most fwd_steps
    const int s = d.steps_per_span;
    return std::max(s, fwd_steps / s * s);
  }
  Geometry fwd_geom(int steps) const {
    // every polarisation of R samples per lane
    return make_geometry(d.n_samples, fwd_tile, L::HC * steps, 1, d.n_pol, sizeof(cd));
  }
  Geometry bwd_geom() const {
    const int s = d.steps_per_span;
    const int halo = L::HC * std::max(s, 2 * (s - 1));
    // tiles of bwd_region - 2 halo samples, so a region fills whole waves
    Geometry g = make_geometry(d.n_samples, bwd_region - 2 * halo, halo, s + 1, d.n_pol,
                               sizeof(float2));
    g.lds += (size_t)(g.threads / 64) * sizeof(double);  // reduction scratch
    return g;
  }
};

namespace {

// Grow the workspace to `bytes` (stream-ordered free of the old one is not
// needed: the caller serialises calls on one handle).
int ensure_ws(ssfm_ldbp_s* h, size_t bytes, hipStream_t st) {
  if (!h->taps15) {
    hipError_t e = hipMalloc(&h->taps15, (size_t)h->d.n_steps * L::TAPS * sizeof(cd));
    if (e != hipSuccess) return api_fail(SSFM_ENOMEM, "ldbp: cannot allocate %zu bytes of taps",
                                         (size_t)h->d.n_steps * L::TAPS * sizeof(cd));
  }
  if (bytes <= h->ws_bytes) return SSFM_OK;
  if (h->ws) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return api_fail_hip(e, "ldbp: synchronise before growing the workspace");
    (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  hipError_t e = hipMalloc(&h->ws, bytes);
  if (e != hipSuccess) return api_fail(SSFM_ENOMEM, "ldbp: cannot allocate %zu bytes of workspace", bytes);
  h->ws_bytes = bytes;
  return SSFM_OK;
}

// part(b0, count, stream) over the realisations [0, batch) of a call: as one
// part on st, or as consecutive parts of nearly equal size, the first on st
// and the others on the handle's worker streams, forked from st and joined
// back into it (also after an error, so no work is left unordered).  A
// launch of `blocks` workgroups per realisation ends in a partly filled
// round of workgroups; the other parts' launches fill it.  By default
// (streams 0) two halves run when by_size is set and each half still has
// 512 or more workgroups per launch (the backward: 1088 workgroups at two
// per CU, 2.1 rounds per launch; at 64 x 2 x 2^14 the training step went
// from 1.00 to 0.87 ms); the forward (1024 workgroups at three per CU,
// measured 13 % slower as halves) runs as one part unless the handle asks.
// streams 2..4: that many parts in both (three or four were no faster than
// two).  Every workgroup computes what it computes in one launch over the
// batch, so the results are the same bits.
template <typename F>
int run_halves(ssfm_ldbp_s* h, int64_t batch, int64_t blocks, bool by_size, hipStream_t st,
               F&& part) {
  int parts = h->streams >= 2 ? h->streams : (h->streams == 0 && by_size && batch * blocks >= 1024) ? 2 : 1;
  parts = (int)std::min<int64_t>(parts, batch);
  if (parts < 2) return part(int64_t{0}, batch, st);
  hipError_t e = hipSuccess;
  for (int k = 0; k < parts - 1 && e == hipSuccess; ++k) {
    if (!h->worker[k]) e = hipStreamCreateWithFlags(&h->worker[k], hipStreamNonBlocking);
    if (e == hipSuccess && !h->join_ev[k])
      e = hipEventCreateWithFlags(&h->join_ev[k], hipEventDisableTiming);
  }
  if (e == hipSuccess && !h->fork_ev) e = hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(h->fork_ev, st);
  for (int k = 0; k < parts - 1 && e == hipSuccess; ++k) e = hipStreamWaitEvent(h->worker[k], h->fork_ev, 0);
  if (e != hipSuccess) return api_fail_hip(e, "ldbp: fork onto the worker streams");
  int rc = SSFM_OK;
  for (int k = parts - 1; k >= 0 && rc == SSFM_OK; --k) {
    const int64_t o0 = batch * k / parts, o1 = batch * (k + 1) / parts;
    rc = part(o0, o1 - o0, k == 0 ? st : h->worker[k - 1]);
  }
  hipError_t ej = hipSuccess;
  for (int k = 0; k < parts - 1; ++k) {
    hipError_t x = hipEventRecord(h->join_ev[k], h->worker[k]);
    if (x == hipSuccess) x = hipStreamWaitEvent(st, h->join_ev[k], 0);
    if (ej == hipSuccess) ej = x;
  }
  if (rc != SSFM_OK) return rc;
  if (ej != hipSuccess) return api_fail_hip(ej, "ldbp: join the worker streams");
  return SSFM_OK;
}

// The dynamic-LDS limit is a property of the kernel (process-wide): only
// ever raise it, so that no handle lowers it below another's need.
std::mutex g_lds_mutex;
size_t g_lds_fwd[3] = {0, 0, 0}, g_lds_bwd[3] = {0, 0, 0};

int prepare(int n_pol, size_t fwd_lds, size_t bwd_lds) {
  if (fwd_lds > 160 * 1024 || bwd_lds > 160 * 1024)
    return api_fail(SSFM_EINVAL, "ldbp: tile needs %zu / %zu bytes of LDS (> 160 KiB)", fwd_lds, bwd_lds);
  std::lock_guard<std::mutex> lock(g_lds_mutex);
  const size_t f = std::max(fwd_lds, g_lds_fwd[n_pol]);
  const size_t b = std::max(bwd_lds, g_lds_bwd[n_pol]);
  if (f == g_lds_fwd[n_pol] && b == g_lds_bwd[n_pol]) return SSFM_OK;
  hipError_t e = L::prepare(n_pol, f, b);
  if (e != hipSuccess) return api_fail_hip(e, "ldbp: raise the LDS limit");
  g_lds_fwd[n_pol] = f;
  g_lds_bwd[n_pol] = b;
  return SSFM_OK;
}

int check_handle(ssfm_ldbp_t h, int64_t batch) {
  if (!h) return api_fail(SSFM_EINVAL, "NULL ldbp handle");
  if (batch < 1) return api_fail(SSFM_EINVAL, "batch must be >= 1 (got %lld)", (long long)batch);
  return SSFM_OK;
}

int check_ptr(const void* p, const char* what) {
  if (!p) return api_fail(SSFM_EINVAL, "NULL %s", what);
  if (!aligned8(p)) return api_fail(SSFM_EINVAL, "%s is not 8-byte aligned", what);
  return SSFM_OK;
}

// Forward over all steps of the realisations [b0, b0 + count) of a call of
// `batch`: src -> dst with checkpoints (or temporary ping-pong states in tmp
// when ckpt is NULL and more than one launch runs); every array holds the
// whole call's batch.
int run_forward(ssfm_ldbp_s* h, const float2* src, float2* dst, const double* xi, int64_t batch,
                int64_t b0, int64_t count, float2* ckpt, float2* tmp, hipStream_t st) {
  const int K = h->d.n_steps, S = h->d.steps_per_span;
  const int chunk = h->fwd_chunk();
  const int64_t elems = h->field_elems(batch);
  const float2* cur = src;
  int flip = 0;
  for (int k0 = 0; k0 < K; k0 += chunk) {
    const int k1 = std::min(K, k0 + chunk);
    const Geometry g = h->fwd_geom(k1 - k0);
    float2* out;
    if (k1 == K) out = dst;
    else if (ckpt) out = ckpt + (int64_t)(k1 / S - 1) * elems;
    else out = tmp + (flip++ & 1) * elems;
    L::FwdArgs a{};
    a.src = cur;
    a.dst = out;
    a.ckpt = ckpt;
    a.taps15 = h->taps15;
    a.xi = xi;
    a.n = h->d.n_samples;
    a.batch = batch;
    a.b0 = b0;
    a.count = count;
    a.k0 = k0;
    a.k1 = k1;
    a.spans_steps = S;
    a.w = g.w;
    a.halo = g.halo;
    a.region = g.region;
    a.ls = g.ls;
    a.tiles = g.tiles;
    hipError_t e = L::launch_fwd(h->d.n_pol, a, g.threads, g.lds, st);
    if (e != hipSuccess) return api_fail_hip(e, "ldbp forward launch");
    cur = out;
  }
  return SSFM_OK;
}

}  // namespace

extern "C" {

int ssfm_ldbp_init_params(const ssfm_link* link, int32_t n_taps, int32_t steps_per_span,
                          double* taps, double* xi) {
  ssfm::api_clear_error();
  if (!link || !taps || !xi) return api_fail(SSFM_EINVAL, "link, taps and xi must be non-NULL");
  const int64_t n = link->n_samples;
  if (link->n_pol != 1 && link->n_pol != 2) return api_fail(SSFM_EINVAL, "n_pol must be 1 or 2");
  if (n < 64 || n > (int64_t(1) << 22) || (n & (n - 1)) != 0)
    return api_fail(SSFM_EINVAL, "n_samples must be a power of two in [2^6, 2^22]");
  if (n_taps < 1 || n_taps > 15 || n_taps % 2 == 0)
    return api_fail(SSFM_EINVAL, "n_taps must be odd, 1..15 (got %d)", n_taps);
  if (steps_per_span < 1 || steps_per_span > 4)
    return api_fail(SSFM_EINVAL, "steps_per_span must be 1..4 (got %d)", steps_per_span);
  if (link->n_spans < 1 || (int64_t)link->n_spans * steps_per_span > 4096)
    return api_fail(SSFM_EINVAL, "n_spans * steps_per_span must be 1..4096");
  const double vals[] = {link->sample_rate_hz, link->span_km, link->alpha_db_per_km,
                         link->beta2_ps2_per_km, link->gamma_per_w_km, link->edfa_gain_db};
  for (double v : vals)
    if (!std::isfinite(v)) return api_fail(SSFM_EINVAL, "link parameters must be finite");
  if (link->sample_rate_hz <= 0 || link->span_km <= 0)
    return api_fail(SSFM_EINVAL, "sample_rate_hz and span_km must be > 0");
  const double kPi = 3.14159265358979323846;
  const double fs = link->sample_rate_hz;
  const double span = link->span_km * 1e3;
  const double alpha = link->alpha_db_per_km * std::log(10.0) / 10.0 / 1e3;
  const double beta2 = link->beta2_ps2_per_km * 1e-27;
  const double gamma = link->gamma_per_w_km * 1e-3;
  const double cnl = std::isnan(link->nl_factor) ? (link->n_pol == 1 ? 1.0 : 8.0 / 9.0)
                                                 : link->nl_factor;
  const double gain = std::pow(10.0, link->edfa_gain_db / 10.0);
  const int S = steps_per_span, T = n_taps, c = (T - 1) / 2;
  const double step = span / S;
  // response of the inverse dispersion over one step, exp(-i (beta2/2) w^2 step),
  // w the angular frequency of DFT bin k (bins above n/2 are negative)
  std::vector<double> ph((size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    const double w = 2.0 * kPi * (double)(k < n / 2 ? k : k - n) * fs / (double)n;
    ph[(size_t)k] = -0.5 * beta2 * w * w * step;
  }
  // the impulse response at the T centred offsets m = t - c (mod n): the
  // inverse DFT by its direct sum, exponents k m reduced mod n
  std::vector<double> hre((size_t)T), him((size_t)T);
  std::vector<int64_t> m((size_t)T);
  for (int t = 0; t < T; ++t) {
    m[(size_t)t] = ((int64_t)(t - c) % n + n) % n;
    double sr = 0.0, si = 0.0;
    for (int64_t k = 0; k < n; ++k) {
      const double a = ph[(size_t)k] + 2.0 * kPi * (double)((k * m[(size_t)t]) % n) / (double)n;
      sr += std::cos(a);
      si += std::sin(a);
    }
    hre[(size_t)t] = sr / (double)n;
    him[(size_t)t] = si / (double)n;
  }
  // peak gain of the truncated filter on the n-point grid
  double peak = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    double sr = 0.0, si = 0.0;
    for (int t = 0; t < T; ++t) {
      const double a = -2.0 * kPi * (double)((k * m[(size_t)t]) % n) / (double)n;
      const double ca = std::cos(a), sa = std::sin(a);
      sr += hre[(size_t)t] * ca - him[(size_t)t] * sa;
      si += hre[(size_t)t] * sa + him[(size_t)t] * ca;
    }
    peak = std::max(peak, std::sqrt(sr * sr + si * si));
  }
  const double gspan = std::sqrt(gain) * std::exp(-0.5 * alpha * span);
  const double hnl = alpha == 0.0 ? step : 2.0 * std::sinh(0.5 * alpha * step) / alpha;
  const int64_t K = (int64_t)link->n_spans * S;
  for (int64_t k = 0; k < K; ++k) {
    const int j = (int)(k % S);  // sub-step within its span, from the span's end
    const double scale = peak * (j == 0 ? gspan : 1.0);
    for (int t = 0; t < T; ++t) {
      taps[2 * (k * T + t)] = hre[(size_t)t] / scale;
      taps[2 * (k * T + t) + 1] = him[(size_t)t] / scale;
    }
    xi[k] = -cnl * gamma * hnl * std::exp(-alpha * (span - (j + 0.5) * step));
  }
  return SSFM_OK;
}

int ssfm_ldbp_create(const ssfm_ldbp_desc* desc, int hip_device, ssfm_ldbp_t* out) {
  ssfm::api_clear_error();
  if (!out) return api_fail(SSFM_EINVAL, "NULL output handle pointer");
  *out = nullptr;
  int rc = validate(desc);
  if (rc != SSFM_OK) return rc;
  ssfm::DeviceGuard guard(hip_device);
  if (guard.status != hipSuccess) return api_fail_hip(guard.status, "select device");
  auto* h = new (std::nothrow) ssfm_ldbp_s;
  if (!h) return api_fail(SSFM_ENOMEM, "ldbp handle");
  h->d = *desc;
  h->device = hip_device;
  h->fwd_tile = env_int("SSFM_LDBP_FWD_TILE", kFwdTile);
  h->fwd_steps = env_int("SSFM_LDBP_FWD_STEPS", kFwdSteps);
  h->bwd_region = env_int("SSFM_LDBP_BWD_REGION", kBwdRegion);
  h->streams = std::min(4, env_int("SSFM_LDBP_STREAMS", 0));
  if (!pow2(h->fwd_tile) || !pow2(h->bwd_region) || h->bwd_region < 256) {
    delete h;
    return api_fail(SSFM_EINVAL, "ldbp tile overrides must be powers of two (region >= 256)");
  }
  // the largest forward launch and the backward launch must fit a workgroup
  const Geometry gf = h->fwd_geom(h->fwd_chunk());
  const Geometry gb = h->bwd_geom();
  if (gf.region > kFwdMaxRegion || gb.region > kBwdMaxRegion) {
    delete h;
    return api_fail(SSFM_EINVAL, "ldbp tile geometry too large (forward region %d, backward %d)",
                    gf.region, gb.region);
  }
  rc = prepare(h->d.n_pol, gf.lds, gb.lds);
  if (rc != SSFM_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return SSFM_OK;
}

int ssfm_ldbp_destroy(ssfm_ldbp_t h) {
  ssfm::api_clear_error();
  if (!h) return SSFM_OK;
  ssfm::DeviceGuard guard(h->device);
  if (h->ws) (void)hipFree(h->ws);
  if (h->taps15) (void)hipFree(h->taps15);
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  for (int k = 0; k < 3; ++k) {
    if (h->join_ev[k]) (void)hipEventDestroy(h->join_ev[k]);
    if (h->worker[k]) (void)hipStreamDestroy(h->worker[k]);
  }
  delete h;
  return SSFM_OK;
}

int ssfm_ldbp_checkpoint_bytes(ssfm_ldbp_t h, int64_t batch, int64_t* bytes) {
  ssfm::api_clear_error();
  int rc = check_handle(h, batch);
  if (rc != SSFM_OK) return rc;
  if (!bytes) return api_fail(SSFM_EINVAL, "NULL bytes");
  *bytes = (int64_t)(h->spans() - 1) * h->field_elems(batch) * (int64_t)sizeof(float2);
  return SSFM_OK;
}

int ssfm_ldbp_forward(ssfm_ldbp_t h, const void* field_in, void* field_out, const void* taps,
                      const double* xi, int64_t batch, void* checkpoints, void* stream) {
  ssfm::api_clear_error();
  int rc = check_handle(h, batch);
  if (rc == SSFM_OK) rc = check_ptr(field_in, "field_in");
  if (rc == SSFM_OK) rc = check_ptr(field_out, "field_out");
  if (rc == SSFM_OK) rc = check_ptr(taps, "taps");
  if (rc == SSFM_OK) rc = check_ptr(xi, "xi");
  if (rc == SSFM_OK && checkpoints) rc = check_ptr(checkpoints, "checkpoints");
  if (rc != SSFM_OK) return rc;
  if (field_in == field_out) return api_fail(SSFM_EINVAL, "field_in and field_out must differ");
  ssfm::DeviceGuard guard(h->device);
  if (guard.status != hipSuccess) return api_fail_hip(guard.status, "select device");
  hipStream_t st = (hipStream_t)stream;
  const bool several = h->d.n_steps > h->fwd_chunk();
  rc = ensure_ws(h, (several && !checkpoints) ? 2 * h->field_elems(batch) * sizeof(float2) : 0, st);
  if (rc != SSFM_OK) return rc;
  hipError_t e = L::launch_pad_taps((const cd*)taps, h->d.n_steps, h->d.n_taps, h->taps15, st);
  if (e != hipSuccess) return api_fail_hip(e, "ldbp tap padding launch");
  return run_halves(h, batch, h->fwd_geom(h->fwd_chunk()).tiles, false, st,
                    [&](int64_t b0, int64_t count, hipStream_t s) {
                      return run_forward(h, (const float2*)field_in, (float2*)field_out, xi, batch,
                                         b0, count, (float2*)checkpoints, (float2*)h->ws, s);
                    });
}

int ssfm_ldbp_loss(ssfm_ldbp_t h, const void* field_out, const void* symbols, const double* mf,
                   int64_t batch, double* loss, void* grad_out, void* stream) {
  ssfm::api_clear_error();
  int rc = check_handle(h, batch);
  if (rc == SSFM_OK) rc = check_ptr(field_out, "field_out");
  if (rc == SSFM_OK) rc = check_ptr(symbols, "symbols");
  if (rc == SSFM_OK) rc = check_ptr(mf, "mf");
  if (rc == SSFM_OK) rc = check_ptr(loss, "loss");
  if (rc == SSFM_OK && grad_out) rc = check_ptr(grad_out, "grad_out");
  if (rc != SSFM_OK) return rc;
  ssfm::DeviceGuard guard(h->device);
  if (guard.status != hipSuccess) return api_fail_hip(guard.status, "select device");
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = h->d.n_samples, m = n / h->d.sps;
  const int64_t rows = batch * h->d.n_pol;
  const int mf_half = (h->d.mf_taps - 1) / 2;
  // symbols per workgroup: a power of two dividing m whose staged samples fit 32 KiB of LDS
  int ms = (int)std::min<int64_t>(m, kLossSymbols);
  while (ms > 1 && (size_t)(h->d.sps * (ms - 1) + 2 * mf_half + 1) * sizeof(float2) > 32768) ms /= 2;
  const int tiles = (int)(m / ms);
  const int64_t nblk = rows * tiles;
  const size_t ubar_bytes = (size_t)(rows * m) * sizeof(cd);
  const size_t part_bytes = (size_t)nblk * sizeof(double);
  rc = ensure_ws(h, ubar_bytes + part_bytes, st);
  if (rc != SSFM_OK) return rc;
  cd* ubar = (cd*)h->ws;
  double* partial = (double*)(h->ws + ubar_bytes);
  L::LossArgs a{};
  a.z = (const float2*)field_out;
  a.sym = (const float2*)symbols;
  a.mf = mf;
  a.ubar = ubar;
  a.partial = partial;
  a.n = n;
  a.m = m;
  a.mf_half = mf_half;
  a.sps = h->d.sps;
  a.ms = ms;
  a.tiles = tiles;
  a.scale = 2.0 / (double)(rows * m);
  hipError_t e = L::launch_loss(a, rows, st);
  if (e != hipSuccess) return api_fail_hip(e, "ldbp loss launch");
  e = L::launch_loss_total(partial, (int)nblk, 1.0 / (double)(rows * m), loss, st);
  if (e != hipSuccess) return api_fail_hip(e, "ldbp loss total launch");
  if (grad_out) {
    L::MfAdjArgs b{};
    b.ubar = ubar;
    b.mf = mf;
    b.grad = (float2*)grad_out;
    b.n = n;
    b.m = m;
    b.mf_half = mf_half;
    b.sps = h->d.sps;
    b.ns = (int)std::min<int64_t>(n, kMfSamples);
    b.tiles = (int)(n / b.ns);
    e = L::launch_mf_adjoint(b, rows, st);
    if (e != hipSuccess) return api_fail_hip(e, "ldbp matched-filter adjoint launch");
  }
  return SSFM_OK;
}

int ssfm_ldbp_backward(ssfm_ldbp_t h, const void* field_in, const void* field_out, const void* taps,
                       const double* xi, int64_t batch, const void* checkpoints, void* grad,
                       void* grad_taps, double* grad_xi, void* stream) {
  ssfm::api_clear_error();
  int rc = check_handle(h, batch);
  if (rc == SSFM_OK) rc = check_ptr(field_in, "field_in");
  if (rc == SSFM_OK) rc = check_ptr(field_out, "field_out");
  if (rc == SSFM_OK) rc = check_ptr(taps, "taps");
  if (rc == SSFM_OK) rc = check_ptr(xi, "xi");
  if (rc == SSFM_OK) rc = check_ptr(grad, "grad");
  if (rc == SSFM_OK) rc = check_ptr(grad_taps, "grad_taps");
  if (rc == SSFM_OK) rc = check_ptr(grad_xi, "grad_xi");
  if (rc == SSFM_OK && h->spans() > 1) rc = check_ptr(checkpoints, "checkpoints");
  if (rc != SSFM_OK) return rc;
  ssfm::DeviceGuard guard(h->device);
  if (guard.status != hipSuccess) return api_fail_hip(guard.status, "select device");
  hipStream_t st = (hipStream_t)stream;
  const Geometry g = h->bwd_geom();
  const int64_t nblk = batch * g.tiles;
  const int64_t elems = h->field_elems(batch);
  const size_t gbytes = (size_t)elems * sizeof(float2);
  const size_t pbytes = (size_t)h->d.n_steps * nblk * L::NRED * sizeof(double);
  rc = ensure_ws(h, gbytes + pbytes, st);
  if (rc != SSFM_OK) return rc;
  hipError_t e = L::launch_pad_taps((const cd*)taps, h->d.n_steps, h->d.n_taps, h->taps15, st);
  if (e != hipSuccess) return api_fail_hip(e, "ldbp tap padding launch");
  float2* other = (float2*)h->ws;
  double* partial = (double*)(h->ws + gbytes);
  const int spans = h->spans(), S = h->d.steps_per_span;
  // the gradient alternates between grad and the workspace; start so that
  // the last span's output lands in grad
  float2* bufs[2] = {(float2*)grad, other};
  int cur = 0;
  if (spans % 2 == 1) {
    e = hipMemcpyAsync(other, grad, gbytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return api_fail_hip(e, "ldbp gradient staging copy");
    cur = 1;
  }
  const float2* ck = (const float2*)checkpoints;
  const int cur0 = cur;
  rc = run_halves(h, batch, g.tiles, true, st, [&](int64_t b0, int64_t count, hipStream_t hs) {
    int c = cur0;
    for (int s = spans - 1; s >= 0; --s) {
      L::BwdArgs a{};
      a.x0 = s == 0 ? (const float2*)field_in : ck + (int64_t)(s - 1) * elems;
      a.xs = s == spans - 1 ? (const float2*)field_out : ck + (int64_t)s * elems;
      a.g_in = bufs[c];
      a.g_out = bufs[c ^ 1];
      a.taps15 = h->taps15;
      a.xi = xi;
      a.partial = partial;
      a.n = h->d.n_samples;
      a.batch = batch;
      a.b0 = b0;
      a.count = count;
      a.k0 = s * S;
      a.s_steps = S;
      a.w = g.w;
      a.halo = g.halo;
      a.region = g.region;
      a.ls = g.ls;
      a.tiles = g.tiles;
      const hipError_t el = L::launch_bwd(h->d.n_pol, a, g.threads, g.lds, hs);
      if (el != hipSuccess) return api_fail_hip(el, "ldbp backward launch");
      c ^= 1;
    }
    return SSFM_OK;
  });
  if (rc != SSFM_OK) return rc;
  e = L::launch_reduce(partial, (int)nblk, h->d.n_steps, h->d.n_taps, (cd*)grad_taps, grad_xi, st);
  if (e != hipSuccess) return api_fail_hip(e, "ldbp gradient reduction launch");
  return SSFM_OK;
}

}  // extern "C"
