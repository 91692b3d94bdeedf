// Device helpers shared by the forward and adjoint kernels of libssfm:
// complex64 <-> FP64 conversion at the HBM boundary, the unit phasor of the
// nonlinear step and the four-step twiddle lookup.
#pragma once

#include "fft_dev.hpp"

namespace ssfm {

__device__ __forceinline__ cd load_c64(const float2* p) {
  float2 v = *p;
  return {(double)v.x, (double)v.y};
}
__device__ __forceinline__ void store_c64(float2* p, cd v) {
  *p = make_float2((float)v.re, (float)v.im);
}
// The state at a span boundary is the complex64 field: rounding to it there
// makes a run split at span boundaries identical, bit for bit, to one call.
__device__ __forceinline__ cd round_c64(cd v) {
  return {(double)(float)v.re, (double)(float)v.im};
}

// exp(i phi) in FP64.  For |phi| <= 1/4 (the nonlinear phase of one split
// step is ~1e-2 rad on the workloads here) the Taylor series of sin to phi^11
// and cos to phi^10, truncation below 1e-15 relative, so the rotation is
// unit-modulus to FP64 rounding.  Larger angles: single-precision sine and
// cosine, then one Newton step on the modulus in FP64 (a rotation whose
// modulus carries a single-precision rounding would bias the power at every
// step).
__device__ __forceinline__ cd unit_phasor(double phi) {
  if (fabs(phi) <= 0.25) {
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
  float s, c;
  sincosf((float)phi, &s, &c);
  const double cr = c, sr = s;
  const double m = fma(cr, cr, sr * sr);
  const double f = fma(-0.5, m, 1.5);
  return {cr * f, sr * f};
}

// twiddle W_N^m from the two-level table (m < N): twA[a] = W_N^{a N2},
// twB[b] = W_N^b
__device__ __forceinline__ cd four_step_twiddle(const cd* __restrict__ twA,
                                                const cd* __restrict__ twB, int m, int log2_n2,
                                                int n2) {
  return cmul(twA[m >> log2_n2], twB[m & (n2 - 1)]);
}

}  // namespace ssfm
