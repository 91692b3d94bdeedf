// SSFM kernels for gfx950.
//
// Every kernel reads and writes the field as complex64 in HBM and computes in
// FP64 registers.  The propagated variable is the loss-free field
// a(z) = A(z) exp(alpha z / 2): the linear step on it is a pure phase
// exp(i (beta2/2) omega^2 h), the loss moves into the coefficient of the
// nonlinear phase (exp(-alpha z_j) at the step midpoint z_j) and into one
// field factor exp(-alpha L / 2) at the span end, where it meets the
// amplifier gain sqrt(G).  This is the same discrete scheme as applying the
// loss inside every linear step (every factor is a scalar that commutes with
// the rest), without a per-step loss factor whose rounding would repeat at
// every step.
//
// Kernels:
//   k1_lds   whole field of one realisation resident in one workgroup
//            (n <= 8192 per polarisation): every span and step in one launch.
//   k2_rows  four-step row pass: row FFT -> dispersion multiply -> row IFFT.
//   k3_cols  four-step column pass: twiddle* -> column IFFT -> nonlinear
//            phase or amplifier + ASE -> column FFT -> twiddle.
//
// Four-step indexing (N = N1 * N2, time index n = n1 N2 + n2, frequency index
// k = k1 + N1 k2): the column FFT over n1 gives k1, the twiddle W_N^{n2 k1}
// couples the two, the row FFT over n2 gives k2, and bin k is held at storage
// position k1 N2 + k2 (transposed), where the dispersion table is laid out in
// the same order.  Between passes the field sits in HBM in the mixed
// (k1, n2) domain, so a split step costs exactly two read+write sweeps.
#include "fft_dev.hpp"
#include "philox_dev.hpp"
#include "ssfm_internal.hpp"

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

// exp(i phi) with phi given in FP64: FP32 sine/cosine, then one Newton step
// on the modulus in FP64 so the rotation is unit-modulus to ~1e-15 (a rotation
// whose modulus is off by an FP32 rounding would bias the power every step).
__device__ __forceinline__ cd unit_phasor(double phi) {
  float s, c;
  sincosf((float)phi, &s, &c);
  const double cr = c, sr = s;
  const double m = fma(cr, cr, sr * sr);
  const double f = fma(-0.5, m, 1.5);
  return {cr * f, sr * f};
}

// ---------------------------------------------------------------------------
// K2: rows of length N2 (contiguous), WG lanes, FP32 LDS exchange.
// ---------------------------------------------------------------------------
template <int N2, int WG>
__global__ __launch_bounds__(WG) void k2_rows(float2* __restrict__ field,
                                              const cd* __restrict__ H, const cd* __restrict__ tw,
                                              int n1) {
  constexpr int T = N2 / 16;
  constexpr int RPW = WG / T;
  extern __shared__ float2 lds2[];
  const int lr = threadIdx.x / T;
  const int j = threadIdx.x % T;
  const int64_t row = (int64_t)blockIdx.x * RPW + lr;
  const int k1 = (int)(row % n1);
  float2* rp = field + row * N2;
  float2* mylds = lds2 + lr * N2;
  cd reg[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) reg[r] = load_c64(rp + j + T * r);
  fft<N2, false>(reg, mylds, 1, j, tw);
  const cd* hp = H + (int64_t)k1 * N2;
#pragma unroll
  for (int r = 0; r < 16; ++r) reg[r] = cmul(reg[r], hp[j + T * r]);
  fft<N2, true>(reg, mylds, 1, j, tw);
#pragma unroll
  for (int r = 0; r < 16; ++r) store_c64(rp + j + T * r, reg[r]);
}

// ---------------------------------------------------------------------------
// K3: column tiles of C adjacent columns x N1 rows x P polarisations.
// ---------------------------------------------------------------------------


// twiddle W_N^{n2 k1} from the two-level table (n2 k1 < N, no reduction)
__device__ __forceinline__ cd four_step_twiddle(const ColArgs& a, int n2, int k1) {
  const int m = n2 * k1;
  return cmul(a.twA[m >> a.log2_n2], a.twB[m & (a.n2 - 1)]);
}

template <int N1, int C, int P, int MODE>
__global__ __launch_bounds__(P * C * (N1 / 16)) void k3_cols(ColArgs a) {
  constexpr int T = N1 / 16;
  extern __shared__ float2 lds3[];
  const int tid = threadIdx.x;
  const int p = tid / (C * T);
  const int rem = tid % (C * T);
  const int c = rem % C;
  const int j = rem / C;
  const int tiles = a.n2 / C;
  const int64_t b = blockIdx.x / tiles;
  const int n2 = (int)(blockIdx.x % tiles) * C + c;
  float2* fp = a.field + (b * P + p) * a.n + n2;
  float2* mylds = lds3 + p * (N1 * C) + c;
  cd reg[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) reg[r] = load_c64(fp + (int64_t)(j + T * r) * a.n2);

  if constexpr (MODE != MODE_FIRST) {
    // mixed (k1, n2) domain -> time: conjugate twiddle, inverse column FFT
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[r] = cmulc(reg[r], four_step_twiddle(a, n2, j + T * r));
    fft<N1, true>(reg, mylds, C, j, a.tw1);
    if constexpr (MODE == MODE_NL) {
      double pw[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) pw[r] = fma(reg[r].re, reg[r].re, reg[r].im * reg[r].im);
      if constexpr (P == 2) {
        // exchange |a_p|^2 with the lane of the other polarisation
        double* pbuf = reinterpret_cast<double*>(lds3);
        __syncthreads();  // the inverse FFT's LDS reads are done
#pragma unroll
        for (int r = 0; r < 16; ++r) pbuf[p * (N1 * C) + (j + T * r) * C + c] = pw[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const double other = pbuf[(1 - p) * (N1 * C) + (j + T * r) * C + c];
          pw[r] = p == 0 ? pw[r] + other : other + pw[r];
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) reg[r] = cmul(reg[r], unit_phasor(a.kappa * pw[r]));
    } else {
      // amplifier: a <- gspan a + ASE(t), t = n1 N2 + n2.  The noise is drawn
      // in a rolled loop into this lane's own LDS slots and added back in an
      // unrolled one, so the field registers are never indexed at run time.
      const uint64_t key1 = (a.realization0 + (uint64_t)b) * 65536ull + (uint64_t)a.span;
      const bool noisy = a.sigma_h != 0.0;
      if (noisy) {
        __syncthreads();  // the inverse FFT's LDS reads are done
#pragma unroll 1
        for (int r = 0; r < 16; ++r) {
          const uint64_t t = (uint64_t)(j + T * r) * (uint64_t)a.n2 + (uint64_t)n2;
          const u64x4 w = philox4x64_10(t, 0, 0, 0, a.seed, key1);
          mylds[(j + T * r) * C] = p == 0 ? box_muller(w.w[0], w.w[1]) : box_muller(w.w[2], w.w[3]);
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        cd v = cscale(reg[r], a.gspan);
        if (noisy) {
          const float2 g = mylds[(j + T * r) * C];
          v.re = fma(a.sigma_h, (double)g.x, v.re);
          v.im = fma(a.sigma_h, (double)g.y, v.im);
        }
        reg[r] = round_c64(v);
      }
    }
  }
  if constexpr (MODE != MODE_LAST) {
    // time -> mixed domain: column FFT, twiddle
    fft<N1, false>(reg, mylds, C, j, a.tw1);
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[r] = cmul(reg[r], four_step_twiddle(a, n2, j + T * r));
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) store_c64(fp + (int64_t)(j + T * r) * a.n2, reg[r]);
}

// ---------------------------------------------------------------------------
// K1: one realisation per workgroup, field resident in registers, FFT
// exchanges through LDS, every span and step in one launch.
// ---------------------------------------------------------------------------


template <int N, int P>
__global__ __launch_bounds__(N / 16) void k1_lds(LdsArgs a) {
  constexpr int T = N / 16;
  extern __shared__ float2 lds1[];
  const int jj = threadIdx.x;  // the block is exactly T lanes
  const int64_t b = blockIdx.x;
  float2* fp = a.field + b * P * N;
  cd reg[P][16];
#pragma unroll
  for (int q = 0; q < P; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[q][r] = load_c64(fp + q * N + jj + T * r);

  const uint64_t rkey = (a.realization0 + (uint64_t)b) * 65536ull;
  for (int s = a.span_begin; s < a.span_end; ++s) {
    for (int i = 0; i <= a.steps; ++i) {
      if (i > 0) {
        // nonlinear phase of step i-1
        const double kap = a.kappa[i - 1];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          double pw = 0.0;
#pragma unroll
          for (int q = 0; q < P; ++q) pw = fma(reg[q][r].re, reg[q][r].re, fma(reg[q][r].im, reg[q][r].im, pw));
          const cd rot = unit_phasor(kap * pw);
#pragma unroll
          for (int q = 0; q < P; ++q) reg[q][r] = cmul(reg[q][r], rot);
        }
      }
      const cd* h = (i == 0 || i == a.steps) ? a.h_half : a.h_full;
      fft_multi<N, false, P>(reg, lds1, N, 1, jj, a.tw);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const cd hv = h[jj + T * r];
#pragma unroll
        for (int q = 0; q < P; ++q) reg[q][r] = cmul(reg[q][r], hv);
      }
      fft_multi<N, true, P>(reg, lds1, N, 1, jj, a.tw);
    }
    // span end: loss factor, amplifier gain, ASE (drawn into this lane's own
    // LDS slots in a rolled loop, then added in an unrolled one)
    const bool noisy = a.sigma_h != 0.0;
    if (noisy) {
      __syncthreads();  // the inverse FFT's LDS reads are done
#pragma unroll 1
      for (int r = 0; r < 16; ++r) {
        const u64x4 w = philox4x64_10((uint64_t)(jj + T * r), 0, 0, 0, a.seed, rkey + (uint64_t)s);
        lds1[jj + T * r] = box_muller(w.w[0], w.w[1]);
        if (P == 2) lds1[N + jj + T * r] = box_muller(w.w[2], w.w[3]);
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
#pragma unroll
      for (int q = 0; q < P; ++q) {
        reg[q][r] = cscale(reg[q][r], a.gspan);
        if (noisy) {
          const float2 g = lds1[q * N + jj + T * r];
          reg[q][r].re = fma(a.sigma_h, (double)g.x, reg[q][r].re);
          reg[q][r].im = fma(a.sigma_h, (double)g.y, reg[q][r].im);
        }
        reg[q][r] = round_c64(reg[q][r]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < P; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) store_c64(fp + q * N + jj + T * r, reg[q][r]);
}

// ---------------------------------------------------------------------------
// Launchers (host side): one function per instantiation, selected at plan time.
// ---------------------------------------------------------------------------
template <int N2, int WG>
static hipError_t launch_k2(float2* field, const cd* H, const cd* tw, int n1, int64_t rows,
                            hipStream_t st) {
  constexpr int T = N2 / 16;
  constexpr int RPW = WG / T;
  const size_t lds = (size_t)RPW * N2 * sizeof(float2);
  hipLaunchKernelGGL((k2_rows<N2, WG>), dim3((unsigned)(rows / RPW)), dim3(WG), lds, st, field,
                     H, tw, n1);
  return hipGetLastError();
}

template <int N1, int C, int P, int MODE>
static hipError_t launch_k3(const ColArgs& a, int64_t batch, hipStream_t st) {
  constexpr int T = N1 / 16;
  const size_t lds = (size_t)P * C * N1 * sizeof(double);  // power exchange needs 8 B/elem
  const unsigned blocks = (unsigned)(batch * (a.n2 / C));
  hipLaunchKernelGGL((k3_cols<N1, C, P, MODE>), dim3(blocks), dim3(P * C * T), lds, st, a);
  return hipGetLastError();
}

template <int N, int P>
static hipError_t launch_k1(const LdsArgs& a, int64_t batch, hipStream_t st) {
  constexpr int T = N / 16;
  const size_t lds = (size_t)P * N * sizeof(float2);
  hipLaunchKernelGGL((k1_lds<N, P>), dim3((unsigned)batch), dim3(T), lds, st, a);
  return hipGetLastError();
}

template <int N, int P>
static hipError_t prepare_k1() {
  const size_t lds = (size_t)P * N * sizeof(float2);
  if (lds > 65536)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k1_lds<N, P>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

template <int N1, int C, int P, int MODE>
static hipError_t prepare_k3_one() {
  const size_t lds = (size_t)P * C * N1 * sizeof(double);
  if (lds > 65536)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k3_cols<N1, C, P, MODE>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

// ---- dispatch tables ------------------------------------------------------

static int log2i(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

template <int N1, int C, int P>
static void fill_k3(FourStepKernels& k) {
  k.col[MODE_FIRST] = &launch_k3<N1, C, P, MODE_FIRST>;
  k.col[MODE_NL] = &launch_k3<N1, C, P, MODE_NL>;
  k.col[MODE_EDFA] = &launch_k3<N1, C, P, MODE_EDFA>;
  k.col[MODE_LAST] = &launch_k3<N1, C, P, MODE_LAST>;
  k.columns = C;
  k.prepare_status = prepare_k3_one<N1, C, P, MODE_FIRST>();
  if (k.prepare_status == hipSuccess) k.prepare_status = prepare_k3_one<N1, C, P, MODE_NL>();
  if (k.prepare_status == hipSuccess) k.prepare_status = prepare_k3_one<N1, C, P, MODE_EDFA>();
  if (k.prepare_status == hipSuccess) k.prepare_status = prepare_k3_one<N1, C, P, MODE_LAST>();
}

template <int N1, int P>
static void fill_cols(FourStepKernels& wide, FourStepKernels& narrow) {
  // wide tiles: 16 (8 at N1 = 512) adjacent columns, 128/64-byte row segments;
  // narrow tiles: 2 columns, for batches too small to fill the chip
  if constexpr (N1 == 512) fill_k3<N1, 8, P>(wide);
  else fill_k3<N1, 16, P>(wide);
  fill_k3<N1, 2, P>(narrow);
}

bool select_kernels(int64_t n, int n_pol, KernelSet& ks) {
  const int l = log2i(n);
  ks = KernelSet{};
  if (l <= 13) {
    ks.path = 1;
#define K1CASE(LN)                                                           \
  case LN:                                                                   \
    if (n_pol == 1) { ks.lds = &launch_k1<(1 << LN), 1>; ks.prepare = prepare_k1<(1 << LN), 1>(); } \
    else { ks.lds = &launch_k1<(1 << LN), 2>; ks.prepare = prepare_k1<(1 << LN), 2>(); } \
    return true;
    switch (l) {
      K1CASE(6) K1CASE(7) K1CASE(8) K1CASE(9) K1CASE(10) K1CASE(11) K1CASE(12) K1CASE(13)
      default: return false;
    }
#undef K1CASE
  }
  ks.path = 2;
  const int l1 = l / 2;
  ks.n1 = 1 << l1;
  ks.n2 = (int)(n >> l1);
  switch (ks.n2) {
    case 128: ks.row_wide = &launch_k2<128, 256>; ks.row_narrow = &launch_k2<128, 64>; ks.rows_narrow = 64 / 8; ks.rows_wide = 256 / 8; break;
    case 256: ks.row_wide = &launch_k2<256, 256>; ks.row_narrow = &launch_k2<256, 64>; ks.rows_narrow = 64 / 16; ks.rows_wide = 256 / 16; break;
    case 512: ks.row_wide = &launch_k2<512, 256>; ks.row_narrow = &launch_k2<512, 64>; ks.rows_narrow = 64 / 32; ks.rows_wide = 256 / 32; break;
    default: return false;
  }
  switch (ks.n1) {
    case 128: if (n_pol == 1) fill_cols<128, 1>(ks.wide, ks.narrow); else fill_cols<128, 2>(ks.wide, ks.narrow); break;
    case 256: if (n_pol == 1) fill_cols<256, 1>(ks.wide, ks.narrow); else fill_cols<256, 2>(ks.wide, ks.narrow); break;
    case 512: if (n_pol == 1) fill_cols<512, 1>(ks.wide, ks.narrow); else fill_cols<512, 2>(ks.wide, ks.narrow); break;
    default: return false;
  }
  ks.prepare = ks.wide.prepare_status != hipSuccess ? ks.wide.prepare_status : ks.narrow.prepare_status;
  return true;
}

}  // namespace ssfm
