// Radix-16 DFT stage on the FP64 matrix cores against the FP64 vector
// butterfly that the FFT passes use: the measured prototype behind keeping the
// FFT stages on the vector units.
//
// A transform is 16 complex FP64 values x[n]; one round replaces it by
// y[k] = (1/4) sum_n x[n] exp(-2 pi i n k / 16) (the 1/4 keeps the norm).
// Between rounds the values go through LDS, as between the passes of an FFT.
//   method 0  one transform per lane: the 4 x 4 Cooley-Tukey radix-16
//             butterfly of the FFTs, FP64 VALU.
//   method 1  16 transforms per wave as the matrix product Y = F X on the
//             matrix cores (v_mfma_f64_16x16x4): in real form
//             [Yr; Yi] = [[Fr, -Fi], [Fi, Fr]] [Xr; Xi], two accumulations of
//             eight K = 4 products per 16 transforms.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_dev.hpp"
#include "host_common.hpp"
#include "ssfm.h"

namespace {

using ssfm::cd;

typedef double v4d __attribute__((ext_vector_type(4)));

// exp(-2 pi i m / 16), m mod 16, from the radix-16 constants of the FFTs
__device__ __forceinline__ cd w16_any(int m) {
  const cd tab[16] = {ssfm::w16<false, 0>(),  ssfm::w16<false, 1>(),  ssfm::w16<false, 2>(),
                      ssfm::w16<false, 3>(),  ssfm::w16<false, 4>(),  ssfm::w16<false, 5>(),
                      ssfm::w16<false, 6>(),  ssfm::w16<false, 7>(),  ssfm::w16<false, 8>(),
                      ssfm::w16<false, 9>(),  ssfm::w16<false, 10>(), ssfm::w16<false, 11>(),
                      ssfm::w16<false, 12>(), ssfm::w16<false, 13>(), ssfm::w16<false, 14>(),
                      ssfm::w16<false, 15>()};
  return tab[m & 15];
}

// method 0: lane = transform; LDS rows of 17 slots (one pad) per lane
__global__ __launch_bounds__(64) void dft16_valu(cd* __restrict__ data, int rounds) {
  __shared__ cd x[64 * 17];
  const int l = threadIdx.x;
  cd* row = data + ((int64_t)blockIdx.x * 64 + l) * 16;
  cd v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = row[r];
  for (int it = 0; it < rounds; ++it) {
    ssfm::dft<16, false>(v);
#pragma unroll
    for (int r = 0; r < 16; ++r) x[l * 17 + r] = ssfm::cscale(v[r], 0.25);
    ssfm::wave_sync();
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = x[l * 17 + r];
    ssfm::wave_sync();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) row[r] = v[r];
}

// method 1: a wave holds 16 transforms; lane l = j + 16 k (j = transform,
// k = 0..3).  Operand layouts of v_mfma_f64_16x16x4 (measured with an
// in-bounds probe of the instruction): A[i][kk] at lane i + 16 kk, B[kk][jj]
// at lane jj + 16 kk, D[i][jj] at lane jj + 16 (i mod 4), register i / 4.
// Step s (0..7) covers columns c = 4 s + kk of the 16 x 32 real operator,
// i.e. input x[c mod 16] (real part for c < 16, imaginary part above).  The
// result rows of a lane, k + 4 v, are the input rows it holds, so a round
// leaves every value in the lane that needs it next; the LDS round trip
// stands for the exchange between FFT passes, as in method 0.
__global__ __launch_bounds__(64) void dft16_mfma(cd* __restrict__ data, int rounds) {
  __shared__ cd x[16 * 17];
  const int l = threadIdx.x, j = l & 15, k = l >> 4;
  cd* tr = data + ((int64_t)blockIdx.x * 16 + j) * 16;  // this lane's transform
  // A operands (row i = j): [Fr | -Fi] for the real part of Y, [Fi | Fr] for
  // the imaginary part, F[i][n] = exp(-2 pi i i n / 16)
  double ar[8], ai[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int c = 4 * s + k;
    const cd f = w16_any(j * (c & 15));
    ar[s] = c < 16 ? f.re : -f.im;
    ai[s] = c < 16 ? f.im : f.re;
  }
  // B operands: x[k + 4 s] of transform j, s = 0..3
  double br[4], bi[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const cd v = tr[k + 4 * s];
    br[s] = v.re;
    bi[s] = v.im;
  }
  for (int it = 0; it < rounds; ++it) {
    v4d dr = {0.0, 0.0, 0.0, 0.0}, di = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const double b = s < 4 ? br[s] : bi[s - 4];
      dr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[s], b, dr, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[s], b, di, 0, 0, 0);
    }
    // lane (j, k) holds y[k + 4 v] of transform j, v = 0..3
#pragma unroll
    for (int v = 0; v < 4; ++v) x[j * 17 + k + 4 * v] = cd{0.25 * dr[v], 0.25 * di[v]};
    ssfm::wave_sync();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const cd v = x[j * 17 + k + 4 * s];
      br[s] = v.re;
      bi[s] = v.im;
    }
    ssfm::wave_sync();
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) tr[k + 4 * s] = cd{br[s], bi[s]};
}

}  // namespace

extern "C" int ssfm_dft16_rounds(int method, void* data, int64_t count, int rounds, void* stream) {
  ssfm::api_clear_error();
  if (method != 0 && method != 1) return ssfm::api_fail(SSFM_EINVAL, "method must be 0 or 1 (got %d)", method);
  if (!data) return ssfm::api_fail(SSFM_EINVAL, "NULL data");
  if (((uintptr_t)data & 15) != 0) return ssfm::api_fail(SSFM_EINVAL, "data must be 16-byte aligned");
  if (count < 0 || count % 64 != 0 || count / 16 > 0x7fffffff)
    return ssfm::api_fail(SSFM_EINVAL, "count must be a non-negative multiple of 64 (got %lld)",
                          (long long)count);
  if (rounds < 0 || rounds > (1 << 20))
    return ssfm::api_fail(SSFM_EINVAL, "rounds must be in [0, 2^20] (got %d)", rounds);
  if (count == 0) return SSFM_OK;
  hipStream_t st = (hipStream_t)stream;
  if (method == 0)
    hipLaunchKernelGGL(dft16_valu, dim3((unsigned)(count / 64)), dim3(64), 0, st,
                       static_cast<cd*>(data), rounds);
  else
    hipLaunchKernelGGL(dft16_mfma, dim3((unsigned)(count / 16)), dim3(64), 0, st,
                       static_cast<cd*>(data), rounds);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SSFM_OK : ssfm::api_fail_hip(e, "dft16 launch");
}
