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
// The adjoint's column pass (k3_adj) is in its own translation unit; its row
// pass is k2_rows with the conjugate dispersion operator.
//
// Four-step indexing (N = N1 * N2, time index n = n1 N2 + n2, frequency index
// k = k1 + N1 k2): the column FFT over n1 gives k1, the twiddle W_N^{n2 k1}
// couples the two, the row FFT over n2 gives k2, and bin k is held at storage
// position k1 N2 + k2 (transposed), where the dispersion table is laid out in
// the same order.  Between passes the field sits in HBM in the mixed
// (k1, n2) domain, so a split step costs exactly two read+write sweeps.
#include <type_traits>

#include "fft_dev.hpp"
#include "kernel_common.hpp"
#include "philox_dev.hpp"
#include "ssfm_internal.hpp"

namespace ssfm {

// ---------------------------------------------------------------------------
// K2: rows of length N2 (contiguous), WG lanes, FP32 LDS exchange.
// ---------------------------------------------------------------------------
template <int N2, int WG, typename L, bool CONJ, typename R, int PART = ROW_STEP>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2, 2))) void k2_rows(float2* __restrict__ field, const cd* __restrict__ H,
                                              const cd* __restrict__ tw,
                                              const cd* __restrict__ twA,
                                              const cd* __restrict__ twB, int n1, int log2_n2) {
  constexpr int T = N2 / 16;
  constexpr int RPW = WG / T;
  extern __shared__ __align__(16) unsigned char lds2_raw[];
  L* lds2 = reinterpret_cast<L*>(lds2_raw);
  const int lr = threadIdx.x / T;
  const int j = threadIdx.x % T;
  const int64_t row = (int64_t)blockIdx.x * RPW + lr;
  const int k1 = (int)(row & (n1 - 1));  // n1 is a power of two
  float2* rp = field + row * N2;
  L* mylds = lds2 + lr * (N2 + N2 / 16);  // padded row: stride = 16 mod 32 slots
  using CT = cplx<R>;
  CT reg[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) reg[r] = load_c64<CT>(rp + j + T * r);
  const lane_twiddles<N2, CT> ltw(tw, j);
  // four-step twiddle W_N^{n2 k1} on n2 = j + T r: W_N^{k1 j} (W_N^{k1 T})^r
  const CT w0 = cconv<CT>(four_step_twiddle(twA, twB, k1 * j, log2_n2, N2));
  const CT wstep = cconv<CT>(four_step_twiddle(twA, twB, k1 * T, log2_n2, N2));
  if constexpr (PART != ROW_IFFT) {
    CT w = w0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      reg[r] = cmul(reg[r], w);
      if (r < 15) w = cmul(w, wstep);
    }
    fft<N2, false, true, true>(reg, mylds, 1, j, ltw);  // one wave per row
  }
  if constexpr (PART == ROW_STEP) {
    const cd* hp = H + (int64_t)k1 * N2;
    // CONJ: conj(H), the adjoint (and inverse) of the unitary linear step.
    // The dispersion multiply is FP64 in both arithmetic variants.
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[r] = cconv<CT>(cmul_t<CONJ>(cconv<cd>(reg[r]), hp[j + T * r]));
  }
  if constexpr (PART != ROW_FFT) {
    fft<N2, true, true, true>(reg, mylds, 1, j, ltw);
    CT w = w0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      reg[r] = cmulc(reg[r], w);
      if (r < 15) w = cmul(w, wstep);
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) store_c64(rp + j + T * r, reg[r]);
}

// ---------------------------------------------------------------------------
// K3: column tiles of C adjacent columns x N1 rows x P polarisations.
// ---------------------------------------------------------------------------


template <int N1, int C, int P, int MODE, typename L, typename R>
__global__ __launch_bounds__(P * C * (N1 / 16)) __attribute__((amdgpu_waves_per_eu(2, 2))) void k3_cols(ColArgs a) {
  using CT = cplx<R>;
  constexpr int T = N1 / 16;
  extern __shared__ __align__(16) unsigned char lds3_raw[];
  L* lds3 = reinterpret_cast<L*>(lds3_raw);
  const int tid = threadIdx.x;
  // Lane -> (polarisation p, column c, row j).  Two polarisations with at
  // least 32 lanes each: the two halves of every wave hold the same (c, j)
  // for p = 0 and p = 1, so the nonlinear step sums the powers across the
  // lane pair in registers; otherwise the polarisations are consecutive
  // blocks of C T lanes.
  constexpr bool PAIR = P == 2 && C * T >= 32;
  int p, c, j;
  if constexpr (PAIR) {
    const int l = tid & 63;
    const int q = (tid >> 6) * 32 + (l & 31);
    p = l >> 5;
    c = q % C;
    j = q / C;
  } else {
    p = tid / (C * T);
    const int rem = tid % (C * T);
    c = rem % C;
    j = rem / C;
  }
  const int tiles = a.n2 / C;
  // Adjacent column tiles share 128-byte lines.  Workgroups are dispatched
  // round-robin over the 8 XCDs (each with its own L2), so XCD x runs blocks
  // x, x + 8, ...: give it the contiguous tile range [x G/8, (x + 1) G/8) so a
  // line is fetched into one L2 only.
  const unsigned G = gridDim.x;
  const unsigned id = (G % 8 == 0) ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  const int64_t b = id / tiles;
  const int col0 = (int)(id % tiles) * C;
  const int n2 = col0 + c;
  // this tile's realisation from column col0 on; lane element r at
  // (p n + c + (j + T r) n2) complex64 slots
  const uint32_t tile_bytes = (uint32_t)((P * a.n - col0) * 8);
  const uint32_t lane_off = (uint32_t)(p * a.n + c + (int64_t)j * a.n2) * 8u;
  const uint32_t step = (uint32_t)(T * a.n2) * 8u;
  const col_buf fb = make_col_buf(a.field + b * P * a.n + col0, tile_bytes, lane_off, step);
  L* mylds = lds3 + p * (N1 * C) + c;
  CT reg[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) reg[r] = col_load<CT>(fb, r);
  const lane_twiddles<N1, CT> ltw(a.tw1, j);

  if constexpr (MODE != MODE_FIRST) {
    // mixed (k1, n2) domain -> time: inverse column FFT
    fft<N1, true, false, false>(reg, mylds, C, j, ltw);
    if constexpr (MODE == MODE_NL_STORE) {
      // the nonlinear step's input, kept for the adjoint's reverse sweep
      const col_buf sb = make_col_buf(a.states + b * P * a.n + col0, tile_bytes, lane_off, step);
#pragma unroll
      for (int r = 0; r < 16; ++r) col_store(sb, r, reg[r]);
    }
    if constexpr (MODE == MODE_NL || MODE == MODE_NL_STORE) {
      const R kappa = (R)a.kappa;
      if constexpr (PAIR) {
        // |a_x|^2 + |a_y|^2 from the lane pair, added x + y on both lanes,
        // so both rotate by the same phase
        R phi[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) phi[r] = kappa * pair32_sum(cnorm2(reg[r]));
        for_each_phasor16(phi, [&](int r, CT e) { reg[r] = cmul(reg[r], e); });
      } else if constexpr (P == 2) {
        // exchange |a_p|^2 with the lane of the other polarisation (the sum
        // is formed x + y on both lanes, so both rotate by the same phase)
        R* pbuf = reinterpret_cast<R*>(lds3_raw);
        __syncthreads();  // the inverse FFT's LDS reads are done
#pragma unroll
        for (int r = 0; r < 16; ++r) pbuf[p * (N1 * C) + (j + T * r) * C + c] = cnorm2(reg[r]);
        __syncthreads();
        R phi[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = (j + T * r) * C + c;
          phi[r] = kappa * (pbuf[i] + pbuf[N1 * C + i]);
        }
        for_each_phasor16(phi, [&](int r, CT e) { reg[r] = cmul(reg[r], e); });
      } else {
        R phi[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) phi[r] = kappa * cnorm2(reg[r]);
        for_each_phasor16(phi, [&](int r, CT e) { reg[r] = cmul(reg[r], e); });
      }
    } else if constexpr (MODE == MODE_EDFA || MODE == MODE_LAST) {
      // amplifier: a <- gspan a + ASE(t), t = n1 N2 + n2.  The noise is drawn
      // in a rolled loop into this lane's own LDS slots and added back in an
      // unrolled one, so the field registers are never indexed at run time.
      const uint64_t key0 = a.seeds ? a.seeds[b] : a.seed;
      const uint64_t key1 = a.seeds ? (uint64_t)a.span
                                    : (a.realization0 + (uint64_t)b) * 65536ull + (uint64_t)a.span;
      const bool noisy = a.sigma_h != 0.0;
      if (a.ckpt) {
        // span-end state before the amplifier, for the adjoint
        const col_buf cb = make_col_buf(a.ckpt + b * P * a.n + col0, tile_bytes, lane_off, step);
#pragma unroll
        for (int r = 0; r < 16; ++r) col_store(cb, r, reg[r]);
      }
      float2* nbuf = reinterpret_cast<float2*>(lds3_raw) + p * (N1 * C) + c;
      if (noisy) {
        __syncthreads();  // the inverse FFT's LDS reads are done
        if constexpr (PAIR) {
          // one draw of a time sample gives both polarisations' noise: the
          // lane pair splits the rows, lane p drawing rows j + T (8 p + r)
          // for both, then each reads its own polarisation's 16 values
          float2* nb0 = reinterpret_cast<float2*>(lds3_raw) + c;
#pragma unroll 1
          for (int r = 8 * p; r < 8 * p + 8; ++r) {
            const int row = j + T * r;
            const uint64_t t = (uint64_t)row * (uint64_t)a.n2 + (uint64_t)n2;
            const u64x4 w = philox4x64_10(t, 0, 0, 0, key0, key1);
            nb0[row * C] = box_muller(w.w[0], w.w[1]);
            nb0[N1 * C + row * C] = box_muller(w.w[2], w.w[3]);
          }
          wave_sync();  // the pair lanes are in one wave
        } else {
#pragma unroll 1
          for (int r = 0; r < 16; ++r) {
            const uint64_t t = (uint64_t)(j + T * r) * (uint64_t)a.n2 + (uint64_t)n2;
            const u64x4 w = philox4x64_10(t, 0, 0, 0, key0, key1);
            nbuf[(j + T * r) * C] = p == 0 ? box_muller(w.w[0], w.w[1]) : box_muller(w.w[2], w.w[3]);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        cd v = cscale(cconv<cd>(reg[r]), a.gspan);
        if (noisy) {
          const float2 g = nbuf[(j + T * r) * C];
          v.re = fma(a.sigma_h, (double)g.x, v.re);
          v.im = fma(a.sigma_h, (double)g.y, v.im);
        }
        reg[r] = cconv<CT>(round_c64(v));
      }
    }
  }
  if constexpr (MODE != MODE_LAST && MODE != MODE_IFFT) {
    // time -> mixed domain: column FFT
    fft<N1, false, false, false>(reg, mylds, C, j, ltw);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) col_store(fb, r, reg[r]);
}

// ---------------------------------------------------------------------------
// K1: one realisation per workgroup, field resident in registers, FFT
// exchanges through LDS, every span and step in one launch.
// ---------------------------------------------------------------------------


// The adjoint's copy of k1_lds's span (the same operations in the same
// order, so a span recomputed from its checkpoint repeats the forward's
// states): for i = 0..steps, the nonlinear step i-1 (i > 0) then the linear
// step with the half (i = 0, steps) or full operator; lane jj holds samples
// jj + T r of every polarisation.  STORE: the input of nonlinear step i-1 is
// also written, rounded to complex64, to states + (i-1) P N.
template <int N, int P, bool STORE, typename L, typename CT>
__device__ __forceinline__ void k1_span(CT (&reg)[P][16], L* lds1, const cd* __restrict__ h_half,
                                        const cd* __restrict__ h_full,
                                        const cd* __restrict__ tw,
                                        const double* __restrict__ kappa, int steps, int jj,
                                        float2* states) {
  using R = decltype(CT{}.re);
  constexpr int T = N / 16;
  for (int i = 0; i <= steps; ++i) {
    if (i > 0) {
      if constexpr (STORE) {
        float2* sp = states + (int64_t)(i - 1) * P * N;
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
          for (int r = 0; r < 16; ++r) store_c64(sp + q * N + jj + T * r, reg[q][r]);
      }
      // nonlinear phase of step i-1
      const R kap = (R)kappa[i - 1];
      R phi[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        R pw = 0;
#pragma unroll
        for (int q = 0; q < P; ++q) pw = fma(reg[q][r].re, reg[q][r].re, fma(reg[q][r].im, reg[q][r].im, pw));
        phi[r] = kap * pw;
      }
      for_each_phasor16(phi, [&](int r, CT rot) {
#pragma unroll
        for (int q = 0; q < P; ++q) reg[q][r] = cmul(reg[q][r], rot);
      });
    }
    const cd* h = (i == 0 || i == steps) ? h_half : h_full;
    fft_multi<N, false, P, true, false>(reg, lds1, N + N / 16, 1, jj, tw);
    // the dispersion multiply is FP64 in both arithmetic variants
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const cd hv = h[jj + T * r];
#pragma unroll
      for (int q = 0; q < P; ++q) reg[q][r] = cconv<CT>(cmul(cconv<cd>(reg[q][r]), hv));
    }
    fft_multi<N, true, P, true, false>(reg, lds1, N + N / 16, 1, jj, tw);
  }
}

// The adjoint's copy of k1_lds's span end: loss factor, amplifier gain, ASE
// (drawn into this lane's own LDS slots in a rolled loop, then added in an
// unrolled one); the state is then the complex64 field.
template <int N, int P, typename CT>
__device__ __forceinline__ void k1_amplifier(CT (&reg)[P][16], unsigned char* lds1_raw,
                                             double gspan, double sigma_h, int jj,
                                             uint64_t key0, uint64_t key1) {
  constexpr int T = N / 16;
  float2* nbuf = reinterpret_cast<float2*>(lds1_raw);
  const bool noisy = sigma_h != 0.0;
  if (noisy) {
    __syncthreads();  // the inverse FFT's LDS reads are done
#pragma unroll 1
    for (int r = 0; r < 16; ++r) {
      const u64x4 w = philox4x64_10((uint64_t)(jj + T * r), 0, 0, 0, key0, key1);
      nbuf[jj + T * r] = box_muller(w.w[0], w.w[1]);
      if (P == 2) nbuf[N + jj + T * r] = box_muller(w.w[2], w.w[3]);
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      cd v = cscale(cconv<cd>(reg[q][r]), gspan);
      if (noisy) {
        const float2 g = nbuf[q * N + jj + T * r];
        v.re = fma(sigma_h, (double)g.x, v.re);
        v.im = fma(sigma_h, (double)g.y, v.im);
      }
      reg[q][r] = cconv<CT>(round_c64(v));
    }
  }
}

template <int N, int P, typename L, typename R>
__global__ __launch_bounds__(N / 16) void k1_lds(LdsArgs a) {
  using CT = cplx<R>;
  constexpr int T = N / 16;
  extern __shared__ __align__(16) unsigned char lds1_raw[];
  L* lds1 = reinterpret_cast<L*>(lds1_raw);
  float2* nbuf = reinterpret_cast<float2*>(lds1_raw);
  const int jj = threadIdx.x;  // the block is exactly T lanes
  const int64_t b = blockIdx.x;
  float2* fp = a.field + b * P * N;
  CT reg[P][16];
#pragma unroll
  for (int q = 0; q < P; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[q][r] = load_c64<CT>(fp + q * N + jj + T * r);

  const uint64_t key0 = a.seeds ? a.seeds[b] : a.seed;
  const uint64_t rkey = a.seeds ? 0ull : (a.realization0 + (uint64_t)b) * 65536ull;
  for (int s = a.span_begin; s < a.span_end; ++s) {
    for (int i = 0; i <= a.steps; ++i) {
      if (i > 0) {
        // nonlinear phase of step i-1
        const R kap = (R)a.kappa[i - 1];
        R phi[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          R pw = 0;
#pragma unroll
          for (int q = 0; q < P; ++q) pw = fma(reg[q][r].re, reg[q][r].re, fma(reg[q][r].im, reg[q][r].im, pw));
          phi[r] = kap * pw;
        }
        for_each_phasor16(phi, [&](int r, CT rot) {
#pragma unroll
          for (int q = 0; q < P; ++q) reg[q][r] = cmul(reg[q][r], rot);
        });
      }
      const cd* h = (i == 0 || i == a.steps) ? a.h_half : a.h_full;
      fft_multi<N, false, P, true, false>(reg, lds1, N + N / 16, 1, jj, a.tw);
      // the dispersion multiply is FP64 in both arithmetic variants
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const cd hv = h[jj + T * r];
#pragma unroll
        for (int q = 0; q < P; ++q) reg[q][r] = cconv<CT>(cmul(cconv<cd>(reg[q][r]), hv));
      }
      fft_multi<N, true, P, true, false>(reg, lds1, N + N / 16, 1, jj, a.tw);
    }
    // span end: loss factor, amplifier gain, ASE (drawn into this lane's own
    // LDS slots in a rolled loop, then added in an unrolled one)
    const bool noisy = a.sigma_h != 0.0;
    if (noisy) {
      __syncthreads();  // the inverse FFT's LDS reads are done
#pragma unroll 1
      for (int r = 0; r < 16; ++r) {
        const u64x4 w = philox4x64_10((uint64_t)(jj + T * r), 0, 0, 0, key0, rkey + (uint64_t)s);
        nbuf[jj + T * r] = box_muller(w.w[0], w.w[1]);
        if (P == 2) nbuf[N + jj + T * r] = box_muller(w.w[2], w.w[3]);
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
#pragma unroll
      for (int q = 0; q < P; ++q) {
        cd v = cscale(cconv<cd>(reg[q][r]), a.gspan);
        if (noisy) {
          const float2 g = nbuf[q * N + jj + T * r];
          v.re = fma(a.sigma_h, (double)g.x, v.re);
          v.im = fma(a.sigma_h, (double)g.y, v.im);
        }
        reg[q][r] = cconv<CT>(round_c64(v));
      }
    }
  }
#pragma unroll
  for (int q = 0; q < P; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) store_c64(fp + q * N + jj + T * r, reg[q][r]);
}

// Adjoint of the LDS-resident path (FP64), one realisation per workgroup, the
// whole link in one launch, with span checkpoints and in-span recomputation:
//   1. forward pass from field_in, writing the input of every span (complex64,
//      exact: the state at a span boundary is the complex64 field) to ckpt;
//   2. for each span from the last: recompute its split steps from its
//      checkpoint with the forward's arithmetic (the same states, bit for
//      bit), writing each nonlinear step's input x to this realisation's
//      step slices; then pull the cotangent g = dL/dA* back through the
//      span in reverse: amplifier g <- gspan g; per step i = steps..0 the
//      linear step's adjoint (FFT, x conj(H), IFFT) and, for i > 0, the
//      nonlinear step's pullback with its input x (y = x e^{i phi},
//      phi = kappa sum_q |x_q|^2):
//        g' = g e^{-i phi},  s = -Im sum_q conj(g'_q) x_q,  g <- g' + 2 s kappa x.
//      All polarisations of a sample sit in one lane, so the sums are local.
// The cotangent waits in the grad buffer (complex64) while a span is
// recomputed; every lane reads back only the samples it wrote.
template <int N, int P, typename L>
__global__ __launch_bounds__(N / 16) void k1_adj(LdsArgs a) {
  constexpr int T = N / 16;
  extern __shared__ __align__(16) unsigned char lds1_raw[];
  L* lds1 = reinterpret_cast<L*>(lds1_raw);
  const int jj = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int64_t slice = (int64_t)P * N;
  const float2* xin = a.field_in + b * slice;
  float2* gp = a.grad + b * slice;
  float2* ck = a.ckpt + b * a.span_end * slice;        // [spans][P][N]
  float2* st = a.states + b * (int64_t)a.steps * slice;  // [steps][P][N]
  const uint64_t key0 = a.seed;
  const uint64_t rkey = (a.realization0 + (uint64_t)b) * 65536ull;
  cd reg[P][16];
#pragma unroll
  for (int q = 0; q < P; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[q][r] = load_c64(xin + q * N + jj + T * r);
  for (int s = 0; s < a.span_end; ++s) {
    float2* cs = ck + s * slice;
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) store_c64(cs + q * N + jj + T * r, reg[q][r]);
    if (s + 1 == a.span_end) break;  // the last span's output is not needed
    k1_span<N, P, false>(reg, lds1, a.h_half, a.h_full, a.tw, a.kappa, a.steps, jj, nullptr);
    k1_amplifier<N, P>(reg, lds1_raw, a.gspan, a.sigma_h, jj, key0, rkey + (uint64_t)s);
  }
  for (int s = a.span_end - 1; s >= 0; --s) {
    const float2* cs = ck + s * slice;
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) reg[q][r] = load_c64(cs + q * N + jj + T * r);
    k1_span<N, P, true>(reg, lds1, a.h_half, a.h_full, a.tw, a.kappa, a.steps, jj, st);
    // the cotangent, through the amplifier
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) reg[q][r] = cscale(load_c64(gp + q * N + jj + T * r), a.gspan);
    for (int i = a.steps; i >= 0; --i) {
      const cd* h = (i == 0 || i == a.steps) ? a.h_half : a.h_full;
      fft_multi<N, false, P, true, false>(reg, lds1, N + N / 16, 1, jj, a.tw);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const cd hv = h[jj + T * r];
#pragma unroll
        for (int q = 0; q < P; ++q) reg[q][r] = cmulc(reg[q][r], hv);
      }
      fft_multi<N, true, P, true, false>(reg, lds1, N + N / 16, 1, jj, a.tw);
      if (i > 0) {
        const float2* sp = st + (int64_t)(i - 1) * slice;
        const double kap = a.kappa[i - 1];
        double phi[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          double pw = 0.0;
#pragma unroll
          for (int q = 0; q < P; ++q) {
            const cd x = load_c64(sp + q * N + jj + T * r);
            pw = fma(x.re, x.re, fma(x.im, x.im, pw));
          }
          phi[r] = -kap * pw;
        }
        // x is read again below rather than held in registers across the
        // phasors (a compiler barrier, no instruction)
        asm volatile("" ::: "memory");
        for_each_phasor16(phi, [&](int r, cd e) {  // e = e^{-i phi}
          cd x[P];
          double sgn = 0.0;
#pragma unroll
          for (int q = 0; q < P; ++q) {
            x[q] = load_c64(sp + q * N + jj + T * r);
            reg[q][r] = cmul(reg[q][r], e);  // g'
            sgn = fma(reg[q][r].im, x[q].re, fma(-reg[q][r].re, x[q].im, sgn));
          }
          const double w = 2.0 * sgn * kap;  // s = -Im sum conj(g') x = sum (g'.im x.re - g'.re x.im)
#pragma unroll
          for (int q = 0; q < P; ++q) {
            reg[q][r].re = fma(w, x[q].re, reg[q][r].re);
            reg[q][r].im = fma(w, x[q].im, reg[q][r].im);
          }
        });
      }
    }
#pragma unroll
    for (int q = 0; q < P; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) store_c64(gp + q * N + jj + T * r, reg[q][r]);
  }
}

// The LDS-resident transform alone (ssfm_dft): k1_lds's load, one FFT (or
// IFFT) of every polarisation, store.
template <int N, int P, typename L, typename R, bool INV>
__global__ __launch_bounds__(N / 16) void k1_dft(float2* field, const cd* tw) {
  using CT = cplx<R>;
  constexpr int T = N / 16;
  extern __shared__ __align__(16) unsigned char lds1d_raw[];
  L* lds1 = reinterpret_cast<L*>(lds1d_raw);
  const int jj = threadIdx.x;
  float2* fp = field + (int64_t)blockIdx.x * P * N;
  CT reg[P][16];
#pragma unroll
  for (int q = 0; q < P; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[q][r] = load_c64<CT>(fp + q * N + jj + T * r);
  fft_multi<N, INV, P, true, false>(reg, lds1, N + N / 16, 1, jj, tw);
#pragma unroll
  for (int q = 0; q < P; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) store_c64(fp + q * N + jj + T * r, reg[q][r]);
}

// ---------------------------------------------------------------------------
// Launchers (host side): one function per instantiation, selected at plan time.
// ---------------------------------------------------------------------------
template <int N2, int WG, typename L, typename R>
static hipError_t launch_k2(const RowArgs& a, int64_t rows, hipStream_t st) {
  constexpr int T = N2 / 16;
  constexpr int RPW = WG / T;
  const size_t lds = (size_t)RPW * (N2 + N2 / 16) * sizeof(L);
  const dim3 grid((unsigned)(rows / RPW));
  if (a.part == ROW_FFT)
    hipLaunchKernelGGL((k2_rows<N2, WG, L, false, R, ROW_FFT>), grid, dim3(WG), lds, st, a.field,
                       a.H, a.tw, a.twA, a.twB, a.n1, a.log2_n2);
  else if (a.part == ROW_IFFT)
    hipLaunchKernelGGL((k2_rows<N2, WG, L, false, R, ROW_IFFT>), grid, dim3(WG), lds, st,
                       a.field, a.H, a.tw, a.twA, a.twB, a.n1, a.log2_n2);
  else if (a.conj_h)
    hipLaunchKernelGGL((k2_rows<N2, WG, L, true, R>), grid, dim3(WG), lds, st, a.field, a.H, a.tw,
                       a.twA, a.twB, a.n1, a.log2_n2);
  else
    hipLaunchKernelGGL((k2_rows<N2, WG, L, false, R>), grid, dim3(WG), lds, st, a.field, a.H,
                       a.tw, a.twA, a.twB, a.n1, a.log2_n2);
  return hipGetLastError();
}

template <int N2, int WG, typename L, typename R>
static hipError_t prepare_k2() {
  constexpr int T = N2 / 16;
  const size_t lds = (size_t)(WG / T) * (N2 + N2 / 16) * sizeof(L);
  if (lds <= 65536) return hipSuccess;
  for (const void* k : {reinterpret_cast<const void*>(&k2_rows<N2, WG, L, false, R>),
                        reinterpret_cast<const void*>(&k2_rows<N2, WG, L, true, R>),
                        reinterpret_cast<const void*>(&k2_rows<N2, WG, L, false, R, ROW_FFT>),
                        reinterpret_cast<const void*>(&k2_rows<N2, WG, L, false, R, ROW_IFFT>)}) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int N1, int C, int P, int MODE, typename L>
constexpr size_t k3_lds_bytes() {
  // FFT exchange: P*C*N1 elements of L; nonlinear step: P*C*N1 doubles;
  // noise staging: P*C*N1 float2
  return (size_t)P * C * N1 * (sizeof(L) > 8 ? sizeof(L) : 8);
}

template <int N1, int C, int P, int MODE, typename L, typename R>
static hipError_t launch_k3(const ColArgs& a, int64_t batch, hipStream_t st) {
  constexpr int T = N1 / 16;
  const unsigned blocks = (unsigned)(batch * (a.n2 / C));
  const size_t lds = k3_lds_bytes<N1, C, P, MODE, L>();
  hipLaunchKernelGGL((k3_cols<N1, C, P, MODE, L, R>), dim3(blocks), dim3(P * C * T), lds, st, a);
  return hipGetLastError();
}

template <int N, int P, typename L>
constexpr size_t k1_lds_bytes() {
  return (size_t)P * (N + N / 16) * sizeof(L);
}

template <int N, int P, typename L, typename R>
static hipError_t launch_k1(const LdsArgs& a, int64_t batch, hipStream_t st) {
  constexpr int T = N / 16;
  const size_t lds = k1_lds_bytes<N, P, L>();
  hipLaunchKernelGGL((k1_lds<N, P, L, R>), dim3((unsigned)batch), dim3(T), lds, st, a);
  return hipGetLastError();
}

template <int N, int P, typename L, typename R, bool INV>
static hipError_t launch_k1_dft(float2* field, const cd* tw, int64_t batch, hipStream_t st) {
  constexpr int T = N / 16;
  const size_t lds = k1_lds_bytes<N, P, L>();
  hipLaunchKernelGGL((k1_dft<N, P, L, R, INV>), dim3((unsigned)batch), dim3(T), lds, st, field, tw);
  return hipGetLastError();
}

template <int N, int P, typename L>
static hipError_t launch_k1_adj(const LdsArgs& a, int64_t batch, hipStream_t st) {
  constexpr int T = N / 16;
  const size_t lds = k1_lds_bytes<N, P, L>();
  hipLaunchKernelGGL((k1_adj<N, P, L>), dim3((unsigned)batch), dim3(T), lds, st, a);
  return hipGetLastError();
}

template <int N, int P, typename L, typename R>
static hipError_t prepare_k1() {
  const size_t lds = k1_lds_bytes<N, P, L>();
  if (lds <= 65536) return hipSuccess;
  for (const void* k : {reinterpret_cast<const void*>(&k1_lds<N, P, L, R>),
                        reinterpret_cast<const void*>(&k1_dft<N, P, L, R, false>),
                        reinterpret_cast<const void*>(&k1_dft<N, P, L, R, true>)}) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if constexpr (sizeof(R) == 8)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k1_adj<N, P, L>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

template <int N1, int C, int P, int MODE, typename L, typename R>
static hipError_t prepare_k3_one() {
  const size_t lds = k3_lds_bytes<N1, C, P, MODE, L>();
  if (lds > 65536)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k3_cols<N1, C, P, MODE, L, R>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

// ---- dispatch tables ------------------------------------------------------

static int log2i(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

// The FP32-arithmetic variant has no nonlinear-step store (no adjoint).
template <int N1, int C, int P, typename L, typename R>
static void fill_k3(FourStepKernels& k) {
  constexpr bool F64 = sizeof(R) == 8;
  k.col[MODE_FIRST] = &launch_k3<N1, C, P, MODE_FIRST, L, R>;
  k.col[MODE_NL] = &launch_k3<N1, C, P, MODE_NL, L, R>;
  k.col[MODE_EDFA] = &launch_k3<N1, C, P, MODE_EDFA, L, R>;
  k.col[MODE_LAST] = &launch_k3<N1, C, P, MODE_LAST, L, R>;
  k.col[MODE_IFFT] = &launch_k3<N1, C, P, MODE_IFFT, L, R>;
  if constexpr (F64) k.col[MODE_NL_STORE] = &launch_k3<N1, C, P, MODE_NL_STORE, L, R>;
  k.columns = C;
  k.prepare_status = prepare_k3_one<N1, C, P, MODE_FIRST, L, R>();
  if (k.prepare_status == hipSuccess) k.prepare_status = prepare_k3_one<N1, C, P, MODE_NL, L, R>();
  if (k.prepare_status == hipSuccess) k.prepare_status = prepare_k3_one<N1, C, P, MODE_EDFA, L, R>();
  if (k.prepare_status == hipSuccess) k.prepare_status = prepare_k3_one<N1, C, P, MODE_LAST, L, R>();
  if (k.prepare_status == hipSuccess) k.prepare_status = prepare_k3_one<N1, C, P, MODE_IFFT, L, R>();
  if constexpr (F64)
    if (k.prepare_status == hipSuccess) k.prepare_status = prepare_k3_one<N1, C, P, MODE_NL_STORE, L, R>();
}

// FFT exchanges in FP64 LDS (FP32 for the FP32 variant), 64 KB per workgroup
// for the wide FP64 tiles: 8 adjacent columns, 64-byte row segments; narrow
// tiles: 2 columns, for batches too small to fill the chip
template <int N1, int P, typename R>
static void fill_cols(KernelSet& ks) {
  using L = std::conditional_t<sizeof(R) == 8, cd, float2>;
  fill_k3<N1, 8, P, L, R>(ks.wide);
  fill_k3<N1, 2, P, L, R>(ks.narrow);
}

template <int N2, typename R>
static hipError_t fill_rows(KernelSet& ks) {
  using L = std::conditional_t<sizeof(R) == 8, cd, float2>;
  constexpr int T = N2 / 16;
  ks.row_wide = &launch_k2<N2, 256, L, R>;
  ks.row_narrow = &launch_k2<N2, 64, L, R>;
  ks.rows_narrow = 64 / T;
  ks.rows_wide = 256 / T;
  hipError_t e = prepare_k2<N2, 256, L, R>();
  if (e == hipSuccess) e = prepare_k2<N2, 64, L, R>();
  return e;
}

template <int N, typename R>
static void fill_lds(KernelSet& ks, int n_pol) {
  // FP64 LDS exchange where the padded field fits in 160 KB (every one-
  // polarisation length, two polarisations up to 4096), else FP32; the FP32
  // variant always exchanges FP32
  constexpr bool F64 = sizeof(R) == 8;
  using L1 = std::conditional_t<F64, cd, float2>;
  using L2 = std::conditional_t<F64 && N <= 4096, cd, float2>;
  if constexpr (F64) ks.lds_adj = n_pol == 1 ? &launch_k1_adj<N, 1, L1> : &launch_k1_adj<N, 2, L2>;
  if (n_pol == 1) {
    ks.lds = &launch_k1<N, 1, L1, R>;
    ks.lds_dft[0] = &launch_k1_dft<N, 1, L1, R, false>;
    ks.lds_dft[1] = &launch_k1_dft<N, 1, L1, R, true>;
    ks.prepare = prepare_k1<N, 1, L1, R>();
  } else {
    ks.lds = &launch_k1<N, 2, L2, R>;
    ks.lds_dft[0] = &launch_k1_dft<N, 2, L2, R, false>;
    ks.lds_dft[1] = &launch_k1_dft<N, 2, L2, R, true>;
    ks.prepare = prepare_k1<N, 2, L2, R>();
  }
}

template <typename R>
static bool select_kernels_t(int64_t n, int n_pol, KernelSet& ks) {
  const int l = log2i(n);
  if (l <= 13) {
    ks.path = 1;
    switch (l) {
      case 6: fill_lds<64, R>(ks, n_pol); return true;
      case 7: fill_lds<128, R>(ks, n_pol); return true;
      case 8: fill_lds<256, R>(ks, n_pol); return true;
      case 9: fill_lds<512, R>(ks, n_pol); return true;
      case 10: fill_lds<1024, R>(ks, n_pol); return true;
      case 11: fill_lds<2048, R>(ks, n_pol); return true;
      case 12: fill_lds<4096, R>(ks, n_pol); return true;
      case 13: fill_lds<8192, R>(ks, n_pol); return true;
      default: return false;
    }
  }
  ks.path = 2;
  // N1 x N2 with N1 <= N2 and N1 <= 256: 2^18 = 256 x 1024 (the 8-column
  // tiles of the 256-row column pass and its two FFT passes; 512 x 512 with
  // 4-column tiles and three passes measured 18 % slower on workload 3)
  const int l1 = l == 18 ? 8 : l / 2;
  ks.n1 = 1 << l1;
  ks.n2 = (int)(n >> l1);
  hipError_t pr = hipSuccess;
  switch (ks.n2) {
    case 128: pr = fill_rows<128, R>(ks); break;
    case 256: pr = fill_rows<256, R>(ks); break;
    case 512: pr = fill_rows<512, R>(ks); break;
    case 1024: pr = fill_rows<1024, R>(ks); break;
    default: return false;
  }
  if (pr != hipSuccess) ks.prepare = pr;
  switch (ks.n1) {
    case 128:
      if (n_pol == 1) { fill_cols<128, 1, R>(ks); }
      else { fill_cols<128, 2, R>(ks); }
      break;
    case 256:
      if (n_pol == 1) { fill_cols<256, 1, R>(ks); }
      else { fill_cols<256, 2, R>(ks); }
      break;
    default: return false;
  }
  for (const FourStepKernels* k : {&ks.wide, &ks.narrow})
    if (k->prepare_status != hipSuccess) ks.prepare = k->prepare_status;
  if constexpr (sizeof(R) == 8) select_adjoint_kernels(ks.n1, n_pol, ks);
  return true;
}

bool select_kernels(int64_t n, int n_pol, bool fp32, KernelSet& ks) {
  ks = KernelSet{};
  ks.fp32 = fp32;
  return fp32 ? select_kernels_t<float>(n, n_pol, ks) : select_kernels_t<double>(n, n_pol, ks);
}

}  // namespace ssfm
