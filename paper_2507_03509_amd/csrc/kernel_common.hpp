// Device helpers shared by the forward and adjoint kernels of libssfm:
// complex64 <-> FP64 conversion at the HBM boundary, the unit phasors of the
// nonlinear step and the four-step twiddle lookup.
#pragma once

#include "fft_dev.hpp"

namespace ssfm {

template <typename CT = cd>
__device__ __forceinline__ CT load_c64(const float2* p) {
  float2 v = *p;
  return cconv<CT>(cf{v.x, v.y});
}
template <typename R>
__device__ __forceinline__ void store_c64(float2* p, cplx<R> v) {
  *p = make_float2((float)v.re, (float)v.im);
}
// Strided access to the elements j + T r (r < 16) of a lane's column through
// a buffer resource: a wave-uniform base address in scalar registers, one
// 32-bit lane offset, and a wave-uniform byte step per element, so the 16
// loads and stores of a lane share one address register (64-bit addresses
// would take 32).  `bytes` is the resource's range (the hardware's bounds
// check applies to the lane offset); every caller keeps each access inside
// its tile, which lies within the range.  Word 3 of the resource selects the
// 32-bit data format (field 15..18 = 4) that untyped buffer loads need on
// this chip family.
struct col_buf {
  __amdgpu_buffer_rsrc_t rs;
  uint32_t lane, step;
};
__device__ __forceinline__ col_buf make_col_buf(const float2* base, uint32_t bytes, uint32_t lane,
                                                uint32_t step) {
  return {__builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(base), (short)0, (int)bytes,
                                            0x00020000),
          lane, step};
}
__device__ __forceinline__ float2 col_load_f2(const col_buf& b, int r) {
  return __builtin_bit_cast(
      float2, __builtin_amdgcn_raw_buffer_load_b64(b.rs, b.lane, (uint32_t)r * b.step, 0));
}
template <typename CT = cd>
__device__ __forceinline__ CT col_load(const col_buf& b, int r) {
  const float2 v = col_load_f2(b, r);
  return cconv<CT>(cf{v.x, v.y});
}
template <typename R>
__device__ __forceinline__ void col_store(const col_buf& b, int r, cplx<R> v) {
  using raw64 = decltype(__builtin_amdgcn_raw_buffer_load_b64(b.rs, 0, 0, 0));
  const float2 f = make_float2((float)v.re, (float)v.im);
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(raw64, f), b.rs, b.lane,
                                        (uint32_t)r * b.step, 0);
}

// A pointer that the caller knows to be equal on every lane of the wave, moved
// to scalar registers (a buffer resource must be).
__device__ __forceinline__ const float2* wave_uniform(const float2* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<const float2*>(((uint64_t)hi << 32) | lo);
}

// The state at a span boundary is the complex64 field: rounding to it there
// makes a run split at span boundaries identical, bit for bit, to one call.
__device__ __forceinline__ cd round_c64(cd v) {
  return {(double)(float)v.re, (double)(float)v.im};
}

// exp(i phi) in FP64.  For |phi| <= 1/4 (the nonlinear phase of one split
// step is ~1e-2 rad on the workloads here) the Taylor series of sin to phi^11
// and cos to phi^10, truncation below 1e-15 relative, so the rotation is
// unit-modulus to FP64 rounding.
__device__ __forceinline__ cd phasor_series(double phi) {
  const double x2 = phi * phi;
  double ps = fma(x2, -1.0 / 39916800.0, 1.0 / 362880.0);
  ps = fma(ps, x2, -1.0 / 5040.0);
  ps = fma(ps, x2, 1.0 / 120.0);
  ps = fma(ps, x2, -1.0 / 6.0);
  double pc = fma(x2, -1.0 / 3628800.0, 1.0 / 40320.0);
  pc = fma(pc, x2, -1.0 / 720.0);
  pc = fma(pc, x2, 1.0 / 24.0);
  pc = fma(pc, x2, -0.5);
  return {fma(pc, x2, 1.0), fma(ps * x2, phi, phi)};
}

// exp(i phi) for |phi| <= 1/32, the common case by far (one split step's
// nonlinear phase is ~1e-3..1e-2 rad here): sin to phi^7 and cos to phi^6,
// whose truncation (phi^9/9! and phi^8/8!, at most 2.2e-17) is below FP64
// rounding, in 7 FP64 operations instead of 13.
constexpr double kShortPhase = 1.0 / 32.0;
__device__ __forceinline__ cd phasor_short(double phi) {
  const double x2 = phi * phi;
  double ps = fma(x2, -1.0 / 5040.0, 1.0 / 120.0);
  ps = fma(ps, x2, -1.0 / 6.0);
  double pc = fma(x2, -1.0 / 720.0, 1.0 / 24.0);
  pc = fma(pc, x2, -0.5);
  return {fma(pc, x2, 1.0), fma(ps * x2, phi, phi)};
}

// Any angle: the series at phi / 2^k (halved until |phi / 2^k| <= 1/4),
// squared k times, then one Newton step on the modulus (k squarings double
// the relative rounding error k times).  Angles within 1/32 get the short
// series, those within 1/4 the long one.  Reads no memory.
__device__ __forceinline__ cd unit_phasor_any(double phi) {
  int k = 0;
#pragma unroll 1
  while (fabs(phi) > 0.25 && k < 1100) {  // any finite angle needs < 1030
    phi *= 0.5;
    ++k;
  }
  if (k == 0) return fabs(phi) <= kShortPhase ? phasor_short(phi) : phasor_series(phi);
  cd z = phasor_series(phi);
#pragma unroll 1
  for (int i = 0; i < k; ++i) z = {(z.re - z.im) * (z.re + z.im), 2.0 * z.re * z.im};
  const double m = fma(z.re, z.re, z.im * z.im);
  const double f = fma(-0.5, m, 1.5);
  return {z.re * f, z.im * f};
}

// rot[r] = exp(i phi[r]), r < 16, out of line: only waves holding an angle
// above 1/32 call it, and its registers do not count against the callers'.
__device__ __noinline__ void unit_phasors_any16(const double* phi, cd* rot) {
#pragma unroll 1
  for (int r = 0; r < 16; ++r) rot[r] = unit_phasor_any(phi[r]);
}

// f(r, exp(i phi[r])) for the 16 angles of a lane.  The branch is uniform
// over the wave: the short series when every angle of the wave is within
// 1/32, else the general routine, which gives the short series' bits to the
// angles within 1/32 -- so a result never depends on its neighbours.  (A
// per-element branch makes the compiler keep registers for both paths across
// 16 divergent regions.)
template <typename F>
__device__ __forceinline__ void for_each_phasor16(const double (&phi)[16], F&& f) {
  bool wide = false;
#pragma unroll
  for (int r = 0; r < 16; ++r) wide |= !(fabs(phi[r]) <= kShortPhase);
  if (__any(wide)) {
    double ph[16];
    cd rot[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) ph[r] = phi[r];
    unit_phasors_any16(ph, rot);
#pragma unroll
    for (int r = 0; r < 16; ++r) f(r, rot[r]);
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r) f(r, phasor_short(phi[r]));
  }
}

// Sum of x over the lane pair (l, l ^ 32) of a wave, the same bits on both
// lanes: v_permlane32_swap exchanges the upper half of one operand with the
// lower half of the other, so with x in both operands every lane receives
// the lower lane's x in the first result and the upper lane's in the second,
// and adds them in that order.
__device__ __forceinline__ double pair32_sum(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
  const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double lower = __builtin_bit_cast(double, ((uint64_t)rh[0] << 32) | rl[0]);
  const double upper = __builtin_bit_cast(double, ((uint64_t)rh[1] << 32) | rl[1]);
  return lower + upper;
}
// FP32 operand: through the FP64 sum (exact for two floats of similar size),
// rounded once.  (A 32-bit v_permlane32_swap of one value was compiled as the
// first result added to itself.)
__device__ __forceinline__ float pair32_sum(float x) { return (float)pair32_sum((double)x); }

// The FP32-arithmetic variant's nonlinear rotation: f(r, exp(i phi[r])) with
// the FP32 sine and cosine of HIP's device library.
template <typename F>
__device__ __forceinline__ void for_each_phasor16(const float (&phi)[16], F&& f) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float sn, cs;
    sincosf(phi[r], &sn, &cs);
    f(r, cf{cs, sn});
  }
}

// |v|^2 in the arithmetic of v
template <typename R>
__device__ __forceinline__ R cnorm2(cplx<R> v) {
  return fma(v.re, v.re, v.im * v.im);
}

// twiddle W_N^m from the two-level table (m < N): twA[a] = W_N^{a N2},
// twB[b] = W_N^b
__device__ __forceinline__ cd four_step_twiddle(const cd* __restrict__ twA,
                                                const cd* __restrict__ twB, int m, int log2_n2,
                                                int n2) {
  return cmul(twA[m >> log2_n2], twB[m & (n2 - 1)]);
}

}  // namespace ssfm
