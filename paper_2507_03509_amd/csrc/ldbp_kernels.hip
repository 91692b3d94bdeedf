// Learned digital back-propagation kernels (gfx950).
//
// The model alternates a short complex FIR filter (circular, both
// polarisations) with a Kerr phase rotation.  A workgroup owns a tile of w
// samples of one realisation plus a halo on each side: one step needs 7
// neighbours per side, so a launch fusing q steps carries a halo of 7 q and
// never exchanges data with other workgroups.  Each lane owns R = 4
// consecutive samples of every polarisation and reads the 18-sample window of
// its 4 outputs from LDS into registers (4.5 LDS reads per output instead of
// 15).  HBM sees the state once per launch.  The forward keeps the tile's
// state in LDS in FP64; the backward keeps its recomputed states and the
// gradient in FP32 (each rounding of the size of the complex64 field store),
// which halves its LDS and doubles the workgroups a CU holds.
//
// LDS slot of sample i: j + floor(j / 4), j = i + 8 -- one pad slot per 4
// samples.  For the lane owning samples 4 l .. 4 l + 3 the slot of window
// sample d is 5 l + (a constant of d), so a window is one base address plus
// immediate offsets, and the lanes of one LDS access fall on distinct banks
// for every d (a lane stride of 80 bytes in FP64, 40 in FP32).
//
// Backward: one launch per span (steps [k0, k0 + S)).  The span's inner
// states are recomputed from its start checkpoint with the forward code
// (bitwise the forward's values: the forward rounds to complex64 only at
// span boundaries), then each step is pulled back in reverse: the Kerr step
// pointwise from its output z (y = z e^{-i phi}, |y| = |z|), the FIR step as
// the correlation with conj(h) through an LDS window.  The tap gradient is
// a separate phase with its own lane map (wave = group of 5 taps, lane = run
// of interior samples, sliding 5-sample window), so that its 10 accumulators
// never share a lane with the pullback's window; each wave reduces its group
// by recursive halving.  dL/dxi is summed over the workgroup.  Both are
// written as per-workgroup partials that a last kernel sums in a fixed order.
#include "kernel_common.hpp"
#include "ldbp_internal.hpp"

namespace ssfm {
namespace ldbp {

// Sample i of a region lives at slot lslot(i) of its LDS array, for
// -GUARD <= i < region + GUARD; the guard slots hold zeros, so the windows
// of the edge lanes need no bounds check.
__device__ __forceinline__ int lslot(int i) {
  const int j = i + GUARD;
  return j + (j >> 2);
}

__device__ __forceinline__ double norm2(cd v) { return fma(v.re, v.re, v.im * v.im); }

// acc + a b
__device__ __forceinline__ cd cmac(cd acc, cd a, cd b) {
  return {fma(a.re, b.re, fma(-a.im, b.im, acc.re)), fma(a.re, b.im, fma(a.im, b.re, acc.im))};
}

// exp(i phi) to FP64 accuracy for |phi| < 2^20: Cody-Waite reduction
// r = phi - q pi/2 with pi/2 split in two parts (the product q * PIO2_HI is
// exact for |q| < 2^20), Taylor series of sin (to r^15) and cos (to r^16) on
// |r| <= pi/4, whose next terms are below 5e-17, and the quadrant rotation
// by i^q.  Register-light, with no data-dependent branch.
__device__ __forceinline__ cd phasor64(double phi) {
  constexpr double TWO_OVER_PI = 0.63661977236758134308;
  constexpr double PIO2_HI = 1.5707963267341256141;   // 33 significant bits
  constexpr double PIO2_LO = 6.0771005065061922e-11;  // pi/2 - PIO2_HI
  const double q = rint(phi * TWO_OVER_PI);
  const double r = fma(-q, PIO2_LO, fma(-q, PIO2_HI, phi));
  const double r2 = r * r;
  double ps = fma(r2, -1.0 / 1307674368000.0, 1.0 / 6227020800.0);
  ps = fma(ps, r2, -1.0 / 39916800.0);
  ps = fma(ps, r2, 1.0 / 362880.0);
  ps = fma(ps, r2, -1.0 / 5040.0);
  ps = fma(ps, r2, 1.0 / 120.0);
  ps = fma(ps, r2, -1.0 / 6.0);
  const double sn = fma(ps * r2, r, r);
  double pc = fma(r2, 1.0 / 20922789888000.0, -1.0 / 87178291200.0);
  pc = fma(pc, r2, 1.0 / 479001600.0);
  pc = fma(pc, r2, -1.0 / 3628800.0);
  pc = fma(pc, r2, 1.0 / 40320.0);
  pc = fma(pc, r2, -1.0 / 720.0);
  pc = fma(pc, r2, 1.0 / 24.0);
  pc = fma(pc, r2, -0.5);
  const double cs = fma(pc, r2, 1.0);
  const int quad = (int)(((long long)q) & 3);
  // e^{i(r + quad pi/2)} = i^quad e^{ir}: (cs, sn), (-sn, cs), (-cs, -sn),
  // (sn, -cs) for quad = 0..3, formed with selects (no branch)
  const double re = (quad & 1) ? sn : cs;
  const double im = (quad & 1) ? cs : sn;
  return {((quad + 1) & 2) ? -re : re, (quad & 2) ? -im : im};
}

// Step k's filter from the padded [K][15] copy (uniform loads: the taps
// sit in scalar registers).
__device__ __forceinline__ void load_taps(const cd* __restrict__ taps15, int k, cd (&h)[TAPS]) {
#pragma unroll
  for (int t = 0; t < TAPS; ++t) h[t] = taps15[k * TAPS + t];
}

// The lane owning samples 4 l .. 4 l + 3 addresses its
// window and its own samples from slot 5 l with compile-time offsets (the
// slot map is affine there), so every LDS access is one base register plus
// an immediate.
static_assert(R == 4 && GUARD % 4 == 0, "affine lane addressing needs R = 4");
template <typename L>
__device__ __forceinline__ const L* lane_base(const L* a, int q) { return a + 5 * q; }
template <typename L>
__device__ __forceinline__ L* lane_base(L* a, int q) { return a + 5 * q; }
// window sample d (= sample 4 l - HC + d)
constexpr int win_off(int d) { return (d + GUARD - HC) + ((d + GUARD - HC) >> 2); }
// own sample r (= sample 4 l + r)
constexpr int own_off(int r) { return (r + GUARD) + ((r + GUARD) >> 2); }

// Window sample d of the lane owning samples base = 4 q ..: a[base - HC + d].
template <typename L>
__device__ __forceinline__ cd window_at(const L* a, int q, int d) {
  return lds_get<cd>(lane_base(a, q) + win_off(d));
}

// y[r] = sum_t h[t] a[base + r + HC - t]: the FIR step at the lane's samples.
// The window is streamed: each of its R + 14 samples updates the outputs that
// use it and is dropped, so only the outputs stay live.
template <typename L>
__device__ __forceinline__ void fir_own(const L* a, int q, const cd (&h)[TAPS], cd (&y)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) y[r] = cd{0.0, 0.0};
#pragma unroll
  for (int d = 0; d < R + 2 * HC; ++d) {
    const cd v = window_at(a, q, d);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int t = r + 2 * HC - d;
      if (t >= 0 && t < TAPS) y[r] = cmac(y[r], h[t], v);
    }
  }
}

// Kerr step in place: y_p <- y_p exp(i xi sum_q |y_q|^2).  The power is one
// add of per-polarisation terms (commutative: every lane forms the same sum).
template <int P>
__device__ __forceinline__ void kerr(cd (&y)[P][R], double xi) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double pw = norm2(y[0][r]);
    if constexpr (P == 2) pw = pw + norm2(y[1][r]);
    const cd e = phasor64(xi * pw);
#pragma unroll
    for (int p = 0; p < P; ++p) y[p][r] = cmul(y[p][r], e);
  }
}

// One forward step at the lane's samples (both polarisations), reading state
// array st: the forward kernel's arithmetic, bit for bit (the power is the
// same single add of the two per-polarisation terms).
template <int P, typename L>
__device__ __forceinline__ void step_own(const L* st, int ls, int q,
                                         const cd* __restrict__ taps15, const double* __restrict__ xi,
                                         int k, cd (&y)[P][R]) {
  cd h[TAPS];
  load_taps(taps15, k, h);
#pragma unroll
  for (int p = 0; p < P; ++p) {
    fir_own(st + p * ls, q, h, y[p]);
    // keep the next polarisation's window loads behind this one's FMAs: the
    // two windows together would not fit the register budget
    __builtin_amdgcn_sched_barrier(0);
  }
  kerr<P>(y, xi[k]);
}

// Zero the guard slots of `arrays` consecutive LDS arrays of stride ls
// holding a region of `region` samples.
template <typename L>
__device__ __forceinline__ void zero_guards(L* a, int arrays, int ls, int region) {
  for (int q = threadIdx.x; q < arrays * 2 * GUARD; q += blockDim.x) {
    const int arr = q / (2 * GUARD), e = q % (2 * GUARD);
    const int i = e < GUARD ? e - GUARD : region + (e - GUARD);
    lds_put(a + arr * ls + lslot(i), cd{0.0, 0.0});
  }
}

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------
// Every lane carries its R samples of all polarisations (the backward's
// step_own, so a recomputed state is bitwise the forward's): the Kerr phase
// is formed once per sample, in the lane, and the polarisations need no
// exchange.
template <int P>
__global__ __launch_bounds__(512) void ldbp_fwd(FwdArgs a, const cd* __restrict__ taps15,
                                                 const double* __restrict__ xi) {
  extern __shared__ __align__(16) unsigned char smem_f[];
  cd* st = reinterpret_cast<cd*>(smem_f);  // [P][ls]
  const int tid = threadIdx.x;
  const int64_t b = a.b0 + blockIdx.x / a.tiles;  // realisation
  const int tile = (int)(blockIdx.x % a.tiles);
  const int64_t n0 = (int64_t)tile * a.w - a.halo;
  const int64_t nm = a.n - 1;
  const int wt = (int)min((int64_t)a.w, a.n - (int64_t)tile * a.w);  // interior samples
  const float2* src = a.src + b * P * a.n;
  zero_guards(st, P, a.ls, a.region);
  for (int i = tid; i < a.region; i += blockDim.x) {
#pragma unroll
    for (int pp = 0; pp < P; ++pp)
      st[pp * a.ls + lslot(i)] = load_c64(src + pp * a.n + ((n0 + i) & nm));
  }
  __syncthreads();
  const bool active = tid * R < a.region;
  for (int k = a.k0; k < a.k1; ++k) {
    cd y[P][R];
    if (active) step_own<P>(st, a.ls, tid, taps15, xi, k, y);
    __syncthreads();  // every window of this step is read
    // the state at a span boundary is the complex64 field
    const bool span_end = (k + 1) % a.spans_steps == 0;
    if (active) {
      if (span_end) {  // uniform over the workgroup
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
          for (int r = 0; r < R; ++r) lane_base(st + p * a.ls, tid)[own_off(r)] = round_c64(y[p][r]);
      } else {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
          for (int r = 0; r < R; ++r) lane_base(st + p * a.ls, tid)[own_off(r)] = y[p][r];
      }
    }
    __syncthreads();
    if (a.ckpt && span_end && k + 1 < a.k1) {
      float2* cp = a.ckpt + ((int64_t)((k + 1) / a.spans_steps - 1) * a.batch + b) * P * a.n +
                   (int64_t)tile * a.w;
      for (int i = tid; i < wt; i += blockDim.x) {
#pragma unroll
        for (int pp = 0; pp < P; ++pp)
          store_c64(cp + pp * a.n + i, st[pp * a.ls + lslot(a.halo + i)]);
      }
    }
  }
  float2* dst = a.dst + b * P * a.n + (int64_t)tile * a.w;
  for (int i = tid; i < wt; i += blockDim.x) {
#pragma unroll
    for (int pp = 0; pp < P; ++pp) store_c64(dst + pp * a.n + i, st[pp * a.ls + lslot(a.halo + i)]);
  }
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------

// Sum v[0..15] over the 64 lanes of the wave by recursive halving: in round
// r lanes exchange with lane ^ (1 << r) the half of their values they do not
// keep, so each round halves the values per lane (15 shuffle-adds, then two
// for the last value).  Returns on lane l the wave sum of value
// bitrev4(l & 15).
__device__ __forceinline__ double wave_sum16(double (&v)[16]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int half = 16 >> (r + 1);
    const bool upper = (lane >> r) & 1;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const double lo = v[i], hi = v[i + half];
      const double send = upper ? lo : hi;
      const double keep = upper ? hi : lo;
      v[i] = keep + __shfl_xor(send, 1 << r, 64);
    }
  }
  double x = v[0] + __shfl_xor(v[0], 16, 64);
  return x + __shfl_xor(x, 32, 64);
}

__device__ __forceinline__ int bitrev4(int l) {
  return ((l & 1) << 3) | ((l & 2) << 1) | ((l & 4) >> 1) | ((l & 8) >> 3);
}

// Sum one value over the workgroup into *out (thread 0 writes).  red: at
// least nwaves doubles of LDS.  Contains barriers.
__device__ __forceinline__ void block_sum1(double v, double* red, double* out) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    *out = t;
  }
  __syncthreads();
}

// Tap gradient of one step over the tile's interior samples n:
//   dL/dh[t] = sum_{p, n} gy_p[n] conj(x_p[n + c - t]),
// gy in G and x in X (LDS, both polarisations).  Wave w handles the taps
// 5 g .. 5 g + 4 of the groups g = w, w + nwaves, ...; its lane l sums a
// contiguous chunk of samples with a sliding 5-sample window of x (two LDS
// reads per sample for five complex multiply-adds), and the wave reduces
// its 10 values and writes them to part[10 g ..] (lanes 0..9).
template <int P, typename L>
__device__ __forceinline__ void tap_gradient(const L* G, const L* X, int ls, int halo, int w,
                                             double* part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int chunk = (w + 63) >> 6;
  const int n0 = halo + min(lane * chunk, w), n1 = halo + min(lane * chunk + chunk, w);
  for (int grp = wave; grp < 3; grp += nw) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = 0.0;
    const int t0 = 5 * grp;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const L* Gp = G + p * ls;
      const L* Xp = X + p * ls;
      // xw[u] = x[n + c - t0 - u]
      cd xw[5];
#pragma unroll
      for (int u = 0; u < 5; ++u) xw[u] = lds_get<cd>(Xp + lslot(n0 - 1 + HC - t0 - u));
      for (int n = n0; n < n1; ++n) {
#pragma unroll
        for (int u = 4; u > 0; --u) xw[u] = xw[u - 1];
        xw[0] = lds_get<cd>(Xp + lslot(n + HC - t0));
        const cd gv = lds_get<cd>(Gp + lslot(n));
#pragma unroll
        for (int u = 0; u < 5; ++u) {
          v[2 * u] = fma(gv.re, xw[u].re, fma(gv.im, xw[u].im, v[2 * u]));
          v[2 * u + 1] = fma(gv.im, xw[u].re, fma(-gv.re, xw[u].im, v[2 * u + 1]));
        }
      }
    }
    const double sum = wave_sum16(v);
    const int idx = bitrev4(lane & 15);
    if (lane < 16 && idx < 10) part[2 * t0 + idx] = sum;
  }
}

// ---------------------------------------------------------------------------
// Backward of one span
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void ldbp_bwd(BwdArgs a, const cd* __restrict__ taps15,
                                                 const double* __restrict__ xis) {
  extern __shared__ __align__(16) unsigned char smem_b[];
  // [X_0 .. X_{S-1}][G] states and gradient, P * ls each, then the reduction
  float2* xs_lds = reinterpret_cast<float2*>(smem_b);
  const int plane = P * a.ls;
  float2* G = xs_lds + a.s_steps * plane;
  double* red = reinterpret_cast<double*>(G + plane);
  const int tid = threadIdx.x;
  const int64_t b = a.b0 + blockIdx.x / a.tiles;  // realisation
  const int tile = (int)(blockIdx.x % a.tiles);
  const int64_t n0 = (int64_t)tile * a.w - a.halo;
  const int64_t nm = a.n - 1;
  const int64_t row0 = b * P * a.n;
  // interior samples of this tile (the row's last tile may be shorter)
  const int wt = (int)min((int64_t)a.w, a.n - (int64_t)tile * a.w);
  zero_guards(xs_lds, P * (a.s_steps + 1), a.ls, a.region);
  for (int i = tid; i < a.region; i += blockDim.x) {
#pragma unroll
    for (int p = 0; p < P; ++p)
      xs_lds[p * a.ls + lslot(i)] = a.x0[row0 + p * a.n + ((n0 + i) & nm)];
  }
  const int base = tid * R;
  const bool active = base < a.region;
  __syncthreads();
  // inner states X_1 .. X_{S-1} (no rounding inside a span, as in the forward)
  for (int j = 1; j < a.s_steps; ++j) {
    cd y[P][R];
    if (active) {
      step_own<P>(xs_lds + (j - 1) * plane, a.ls, tid, taps15, xis, a.k0 + j - 1, y);
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int r = 0; r < R; ++r) lds_put(lane_base(xs_lds + j * plane + p * a.ls, tid) + own_off(r), y[p][r]);
    }
    __syncthreads();
  }
  // the lane's samples of the span-end state and of its gradient (loaded
  // after the recompute, which needs the registers)
  cd z[P][R], g[P][R];
  if (active) {
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int64_t idx = row0 + p * a.n + ((n0 + base + r) & nm);
        z[p][r] = load_c64(a.xs + idx);
        g[p][r] = load_c64(a.g_in + idx);
      }
  }
  for (int j = a.s_steps - 1; j >= 0; --j) {
    const int k = a.k0 + j;
    const double xi = xis[k];
    const float2* X = xs_lds + j * plane;
    if (j < a.s_steps - 1 && active) {
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int r = 0; r < R; ++r)
          z[p][r] = lds_get<cd>(lane_base(xs_lds + (j + 1) * plane + p * a.ls, tid) + own_off(r));
    }
    // Kerr pullback at the lane's samples (z = output, g = its gradient)
    double xi_part = 0.0;
    cd gy[P][R];
    // e^{-i phi} by the short series when every phase of the wave is within
    // 1/32 (the common case), else per sample by the series or the reduced
    // form: a sample's rotation depends on its own phase only
    bool wide = false;
    if (active) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double pw = norm2(z[0][r]);
        if constexpr (P == 2) pw = pw + norm2(z[1][r]);
        wide |= !(fabs(xi * pw) <= kShortPhase);
      }
    }
    const bool any_wide = __any(wide);
    if (active) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double pw = norm2(z[0][r]);
        if constexpr (P == 2) pw = pw + norm2(z[1][r]);
        const double phi = -xi * pw;
        const cd e = !any_wide ? phasor_short(phi)
                               : (fabs(phi) <= kShortPhase ? phasor_short(phi) : phasor64(phi));
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) s = fma(g[p][r].im, z[p][r].re, fma(-g[p][r].re, z[p][r].im, s));
        const double w2 = 2.0 * xi * s;
#pragma unroll
        for (int p = 0; p < P; ++p) {
          const cd y = cmul(z[p][r], e);
          const cd ge = cmul(g[p][r], e);
          gy[p][r] = {fma(w2, y.re, ge.re), fma(w2, y.im, ge.im)};
        }
        const int i = base + r;
        if (i >= a.halo && i < a.halo + wt) xi_part = fma(pw, s, xi_part);
      }
    }
    __syncthreads();  // earlier readers of G are done
    if (active) {
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int r = 0; r < R; ++r) lds_put(lane_base(G + p * a.ls, tid) + own_off(r), gy[p][r]);
    }
    __syncthreads();
    // the tap gradient first: nothing else is live in the registers then
    // the partials of workgroup (b, tile) of the whole call, whichever
    // launch ran it: [k][b tiles + tile]
    double* part = a.partial + ((int64_t)k * a.batch * a.tiles + a.b0 * a.tiles + blockIdx.x) * NRED;
    tap_gradient<P>(G, X, a.ls, a.halo, wt, part);
    // FIR pullback at the lane's samples: gx[m] = sum_t conj(h[t]) gy[m - c + t]
    if (active) {
      cd h[TAPS];
      load_taps(taps15, k, h);
#pragma unroll
      for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int r = 0; r < R; ++r) g[p][r] = cd{0.0, 0.0};
        // window sample d = gy[base - c + d] meets output r through t = d - r
#pragma unroll
        for (int d = 0; d < R + 2 * HC; ++d) {
          const cd v = window_at(G + p * a.ls, tid, d);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int t = d - r;
            if (t >= 0 && t < TAPS) g[p][r] = cmac(g[p][r], cd{h[t].re, -h[t].im}, v);
          }
        }
      }
    }
    // dL/dxi: one value, summed over the workgroup
    block_sum1(xi_part, red, part + 2 * TAPS);
  }
  if (active) {
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = base + r;
        if (i >= a.halo && i < a.halo + wt) store_c64(a.g_out + row0 + p * a.n + (n0 + i), g[p][r]);
      }
  }
}

// taps15[k][t] = the caller's taps[k][t - off] (zero outside), off = 7 - (T-1)/2
__global__ __launch_bounds__(256) void ldbp_pad_taps(const cd* __restrict__ taps, int n_steps,
                                                     int n_taps, cd* taps15) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_steps * TAPS) return;
  const int k = q / TAPS, t = q % TAPS, s = t - (HC - (n_taps - 1) / 2);
  taps15[q] = (s >= 0 && s < n_taps) ? taps[(int64_t)k * n_taps + s] : cd{0.0, 0.0};
}

// Parameter gradients: sum the per-workgroup partials of every step in a
// fixed order.  One workgroup of 1024 lanes per step: lane (g, v) sums value v
// of the partials g, g + 32, ... in two interleaved accumulators; the 32
// groups are then added in order.
__global__ __launch_bounds__(1024) void ldbp_reduce(const double* __restrict__ partial, int blocks,
                                                    int n_taps, cd* grad_taps, double* grad_xi) {
  __shared__ double red[32][NRED + 1];
  const int k = blockIdx.x;
  const int v = threadIdx.x & 31, grp = threadIdx.x >> 5;
  const double* src = partial + (int64_t)k * blocks * NRED + v;
  double s0 = 0.0, s1 = 0.0;
  int i = grp;
  for (; i + 32 < blocks; i += 64) {
    s0 += src[(int64_t)i * NRED];
    s1 += src[(int64_t)(i + 32) * NRED];
  }
  if (i < blocks) s0 += src[(int64_t)i * NRED];
  red[grp][v] = s0 + s1;
  __syncthreads();
  if (threadIdx.x < NRED) {
    double t = 0.0;
    for (int q = 0; q < 32; ++q) t += red[q][v];
    red[0][v] = t;
  }
  __syncthreads();
  if (threadIdx.x < n_taps) {
    const int tt = threadIdx.x + HC - (n_taps - 1) / 2;
    grad_taps[(int64_t)k * n_taps + threadIdx.x] = cd{red[0][2 * tt], red[0][2 * tt + 1]};
  }
  if (threadIdx.x == 0) grad_xi[k] = red[0][2 * TAPS];
}

// ---------------------------------------------------------------------------
// Loss: matched filter at the symbol instants
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ldbp_loss(LossArgs a) {
  extern __shared__ __align__(16) unsigned char smem_l[];
  double* g = reinterpret_cast<double*>(smem_l);            // 2R + 1 taps
  float2* zs = reinterpret_cast<float2*>(g + 2 * a.mf_half + 2);
  __shared__ double red[4];
  const int64_t row = blockIdx.x / a.tiles;
  const int tile = (int)(blockIdx.x % a.tiles);
  const int64_t m0 = (int64_t)tile * a.ms;
  // samples sps m0 - R .. sps (m0 + ms - 1) + R
  const int span = a.sps * (a.ms - 1) + 2 * a.mf_half + 1;
  const int64_t s0 = a.sps * m0 - a.mf_half;
  const int64_t nm = a.n - 1;
  const float2* zr = a.z + row * a.n;
  for (int i = threadIdx.x; i <= 2 * a.mf_half; i += blockDim.x) g[i] = a.mf[i];
  for (int i = threadIdx.x; i < span; i += blockDim.x) zs[i] = zr[(s0 + i) & nm];
  __syncthreads();
  double part = 0.0;
  if (threadIdx.x < a.ms) {
    // u = sum_j g[j + R] z[sps m - j]: local sample index c - j, c = sps t + R
    const float2* zc = zs + a.sps * threadIdx.x + 2 * a.mf_half;
    cd u{0.0, 0.0};
#pragma unroll 4
    for (int q = 0; q <= 2 * a.mf_half; ++q) {   // q = j + R
      const float2 v = zc[-q];
      u.re = fma(g[q], (double)v.x, u.re);
      u.im = fma(g[q], (double)v.y, u.im);
    }
    const int64_t m = m0 + threadIdx.x;
    const float2 sv = a.sym[row * a.m + m];
    const cd e{u.re - (double)sv.x, u.im - (double)sv.y};
    part = norm2(e);
    a.ubar[row * a.m + m] = cscale(e, a.scale);
  }
  // workgroup sum in a fixed order
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) t += red[w];
    a.partial[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(256) void ldbp_loss_total(const double* __restrict__ partial, int count,
                                                       double inv_count, double* loss) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) s += partial[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *loss = (red[0] + red[1] + red[2] + red[3]) * inv_count;
}

// grad[n] = sum_m mf[sps m - n + R] ubar[m] over the symbols within R of n.
// For a sample n the taps that meet a symbol are k = k0 + sps j (k0 the
// least k >= 0 with sps | n + k - R), meeting symbols m0(n) + j in order, so
// the B samples n, n + sps, .., n + (B - 1) sps of one lane share k0 and see
// the same symbols shifted by one: the lane streams its symbols through a B
// value window in registers (one LDS read per tap for B outputs) and sums
// each output over increasing m, as the direct sum does.  Lanes: sps phases
// x (ns / sps) / B groups of B consecutive samples of one phase.
template <int B>
__global__ __launch_bounds__(256) void ldbp_mf_adjoint(MfAdjArgs a) {
  extern __shared__ __align__(16) unsigned char smem_m[];
  double* g = reinterpret_cast<double*>(smem_m);            // 2R + 1 taps
  cd* us = reinterpret_cast<cd*>(g + 2 * a.mf_half + 2);
  const int64_t row = blockIdx.x / a.tiles;
  const int tile = (int)(blockIdx.x % a.tiles);
  const int64_t nb = (int64_t)tile * a.ns;
  // symbols m in [floor((nb - R) / sps), floor((nb + ns - 1 + R) / sps)]
  const int64_t mlo = (nb - a.mf_half >= 0) ? (nb - a.mf_half) / a.sps
                                            : -((a.mf_half - nb + a.sps - 1) / a.sps);
  const int64_t mhi = (nb + a.ns - 1 + a.mf_half) / a.sps;
  const int cnt = (int)(mhi - mlo + 1);
  const int64_t mm = a.m - 1;
  const cd* ur = a.ubar + row * a.m;
  for (int i = threadIdx.x; i <= 2 * a.mf_half; i += blockDim.x) g[i] = a.mf[i];
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) us[i] = ur[(mlo + i) & mm];
  __syncthreads();
  const int groups = a.ns / a.sps / B;  // lanes per phase
  const int t = threadIdx.x;
  if (t >= a.sps * groups) return;
  const int rho = t / groups;
  const int64_t n0 = nb + rho + (int64_t)a.sps * ((t % groups) * B);
  const int k0 = (int)(((a.mf_half - n0) % a.sps + a.sps) % a.sps);
  const int J = k0 <= 2 * a.mf_half ? (2 * a.mf_half - k0) / a.sps + 1 : 0;
  // symbol of tap k0 for sample n0, relative to the staged range
  const cd* uw = us + ((n0 + k0 - a.mf_half) / a.sps - mlo);
  const int last = J + B - 2;  // the window's last symbol index
  cd acc[B], w[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    acc[b] = cd{0.0, 0.0};
    w[b] = cd{0.0, 0.0};
    if (J > 0 && b <= last) w[b] = uw[b];
  }
  // w[(s + b) % B] holds uw[j + s + b] at step j + s (j a multiple of B)
  int j = 0;
  for (; j + B <= J; j += B) {
#pragma unroll
    for (int s2 = 0; s2 < B; ++s2) {
      const double gj = g[k0 + a.sps * (j + s2)];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const cd u = w[(s2 + b) % B];
        acc[b].re = fma(gj, u.re, acc[b].re);
        acc[b].im = fma(gj, u.im, acc[b].im);
      }
      if (j + s2 + B <= last) w[s2] = uw[j + s2 + B];
    }
  }
#pragma unroll
  for (int s2 = 0; s2 < B; ++s2) {
    if (j + s2 < J) {
      const double gj = g[k0 + a.sps * (j + s2)];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const cd u = w[(s2 + b) % B];
        acc[b].re = fma(gj, u.re, acc[b].re);
        acc[b].im = fma(gj, u.im, acc[b].im);
      }
      if (j + s2 + B <= last) w[s2] = uw[j + s2 + B];
    }
  }
#pragma unroll
  for (int b = 0; b < B; ++b) store_c64(a.grad + row * a.n + n0 + (int64_t)a.sps * b, acc[b]);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_fwd(int n_pol, const FwdArgs& a, int threads, size_t lds, hipStream_t st) {
  const unsigned blocks = (unsigned)(a.count * a.tiles);
  if (n_pol == 1)
    hipLaunchKernelGGL(ldbp_fwd<1>, dim3(blocks), dim3(threads), lds, st, a, a.taps15, a.xi);
  else
    hipLaunchKernelGGL(ldbp_fwd<2>, dim3(blocks), dim3(threads), lds, st, a, a.taps15, a.xi);
  return hipGetLastError();
}

hipError_t launch_bwd(int n_pol, const BwdArgs& a, int threads, size_t lds, hipStream_t st) {
  const unsigned blocks = (unsigned)(a.count * a.tiles);
  if (n_pol == 1)
    hipLaunchKernelGGL(ldbp_bwd<1>, dim3(blocks), dim3(threads), lds, st, a, a.taps15, a.xi);
  else
    hipLaunchKernelGGL(ldbp_bwd<2>, dim3(blocks), dim3(threads), lds, st, a, a.taps15, a.xi);
  return hipGetLastError();
}

hipError_t launch_loss(const LossArgs& a, int64_t rows, hipStream_t st) {
  const size_t lds = (size_t)(2 * a.mf_half + 2) * sizeof(double) +
                     (size_t)(a.sps * (a.ms - 1) + 2 * a.mf_half + 1) * sizeof(float2);
  hipLaunchKernelGGL(ldbp_loss, dim3((unsigned)(rows * a.tiles)), dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_loss_total(const double* partial, int count, double inv_count, double* loss,
                             hipStream_t st) {
  hipLaunchKernelGGL(ldbp_loss_total, dim3(1), dim3(256), 0, st, partial, count, inv_count, loss);
  return hipGetLastError();
}

hipError_t launch_mf_adjoint(const MfAdjArgs& a, int64_t rows, hipStream_t st) {
  const size_t lds = (size_t)(2 * a.mf_half + 2) * sizeof(double) +
                     (size_t)((a.ns + 2 * a.mf_half) / a.sps + 3) * sizeof(cd);
  // B samples per lane, ns / B <= 256 lanes; ns / sps (a power of two) a
  // multiple of B
  const int per_phase = a.ns / a.sps;
  const int B = (a.ns >= 1024 && per_phase % 4 == 0) ? 4 : (a.ns >= 512 && per_phase % 2 == 0) ? 2 : 1;
  const dim3 grid((unsigned)(rows * a.tiles)), block((unsigned)(a.ns / B));
  if (B == 4) hipLaunchKernelGGL(ldbp_mf_adjoint<4>, grid, block, lds, st, a);
  else if (B == 2) hipLaunchKernelGGL(ldbp_mf_adjoint<2>, grid, block, lds, st, a);
  else hipLaunchKernelGGL(ldbp_mf_adjoint<1>, grid, block, lds, st, a);
  return hipGetLastError();
}

hipError_t launch_pad_taps(const cd* taps, int n_steps, int n_taps, cd* taps15, hipStream_t st) {
  const int total = n_steps * TAPS;
  hipLaunchKernelGGL(ldbp_pad_taps, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, taps,
                     n_steps, n_taps, taps15);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int blocks, int n_steps, int n_taps,
                         cd* grad_taps, double* grad_xi, hipStream_t st) {
  hipLaunchKernelGGL(ldbp_reduce, dim3((unsigned)n_steps), dim3(1024), 0, st, partial, blocks,
                     n_taps, grad_taps, grad_xi);
  return hipGetLastError();
}

hipError_t prepare(int n_pol, size_t fwd_lds, size_t bwd_lds) {
  hipError_t e = hipSuccess;
  const void* f = n_pol == 1 ? reinterpret_cast<const void*>(&ldbp_fwd<1>)
                             : reinterpret_cast<const void*>(&ldbp_fwd<2>);
  const void* b = n_pol == 1 ? reinterpret_cast<const void*>(&ldbp_bwd<1>)
                             : reinterpret_cast<const void*>(&ldbp_bwd<2>);
  if (fwd_lds > 65536) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fwd_lds);
  if (e == hipSuccess && bwd_lds > 65536)
    e = hipFuncSetAttribute(b, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bwd_lds);
  return e;
}

}  // namespace ldbp
}  // namespace ssfm
