// Adjoint column pass of the four-step SSFM (gfx950).
//
// The reverse sweep of the vector-Jacobian product runs on a work buffer that
// holds, for each realisation, the forward state reconstructed backwards from
// the span-end checkpoint and the cotangent dL/dA*.  Its row pass is k2_rows
// with the conjugate dispersion operator; this file holds the column pass.
#include "fft_dev.hpp"
#include "kernel_common.hpp"
#include "ssfm_internal.hpp"

namespace ssfm {

__device__ __forceinline__ double norm2(cd v) { return fma(v.re, v.re, v.im * v.im); }

// ---------------------------------------------------------------------------
// K3 adjoint: column tiles of the work buffer holding, for realisation b, the
// reconstructed forward state (at b) and the cotangent dL/dA* (at batch + b).
// Lanes: field f (0 state, 1 cotangent) x polarisation x C columns x T.
//   AMODE_FIRST  state <- span-end checkpoint; both fields time -> mixed
//   AMODE_NL     both mixed -> time; with y the state (output of the forward
//                nonlinear step) and phi = kappa sum_q |y_q|^2:
//                  state     x   = y e^{-i phi}            (inverse step)
//                  cotangent g_x = g_y e^{-i phi} + 2 s kappa x,
//                            s   = -Im sum_q conj(g_y,q) y_q (pullback)
//                then both time -> mixed
//   AMODE_LAST   cotangent mixed -> time, times the span gain (the pullback of
//                the amplifier, applied at the end of the span's reverse sweep
//                because everything in between is linear in the cotangent)
// ---------------------------------------------------------------------------
template <int N1, int C, int P, int AMODE>
__global__ __launch_bounds__(2 * P * C * (N1 / 16)) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k3_adj(AdjArgs a) {
  constexpr int T = N1 / 16;
  extern __shared__ __align__(16) unsigned char lds_adj[];
  cd* lds = reinterpret_cast<cd*>(lds_adj);
  const int tid = threadIdx.x;
  const int f = tid / (P * C * T);
  const int rem0 = tid % (P * C * T);
  const int p = rem0 / (C * T);
  const int rem = rem0 % (C * T);
  const int c = rem % C;
  const int j = rem / C;
  const int tiles = a.n2 / C;
  const unsigned G = gridDim.x;
  const unsigned id = (G % 8 == 0) ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  const int64_t b = id / tiles;
  const int col0 = (int)(id % tiles) * C;
  // FFT regions: one per (field, polarisation), N1 + N1/16 padded rows of C
  constexpr int RS = (N1 + N1 / 16) * C;
  cd* mylds = lds + (f * P + p) * RS + c;
  // Field f of a wave is one value when a field's lanes fill whole waves:
  // then the tile is addressed through buffer resources (wave-uniform base,
  // one lane offset), else through per-element 64-bit addresses.
  constexpr bool WAVE_F = (P * C * T) % 64 == 0;
  const float2* rbase = a.work + (f * a.batch + b) * P * a.n + col0;  // realisation, column col0
  const float2* sbase = rbase;
  if constexpr (AMODE == AMODE_FIRST) {
    if (f == 0) sbase = a.ckpt + b * P * a.n + col0;
  }
  const uint32_t tile_bytes = (uint32_t)((P * a.n - col0) * 8);
  const uint32_t lane_off = (uint32_t)(p * a.n + c + (int64_t)j * a.n2) * 8u;
  const uint32_t step = (uint32_t)(T * a.n2) * 8u;
  col_buf fb{}, sb{};
  if constexpr (WAVE_F) {
    fb = make_col_buf(wave_uniform(rbase), tile_bytes, lane_off, step);
    sb = make_col_buf(wave_uniform(sbase), tile_bytes, lane_off, step);
  }
  float2* fp = const_cast<float2*>(rbase) + p * a.n + c;
  const float2* src = sbase + p * a.n + c;
  cd reg[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if constexpr (WAVE_F) reg[r] = col_load(sb, r);
    else reg[r] = load_c64(src + (int64_t)(j + T * r) * a.n2);
  }
  const lane_twiddles<N1> ltw(a.tw1, j);

  if constexpr (AMODE == AMODE_FIRST) {
    fft<N1, false, 2, false>(reg, mylds, C, j, ltw);
  } else if constexpr (AMODE == AMODE_NL) {
    fft<N1, true, 2, false>(reg, mylds, C, j, ltw);
    // exchange in natural (row, column) order: every lane publishes its
    // value and reads only those it does not hold (state lanes: the other
    // polarisation's state; cotangent lanes: both states and the other
    // polarisation's cotangent)
    __syncthreads();  // the inverse FFT's LDS reads are done
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[((f * P + p) * N1 + j + T * r) * C + c] = reg[r];
    __syncthreads();
    constexpr int F = N1 * C;  // one field-polarisation plane
    double phi[16];
    if (f == 0) {
      // x = y e^{-i phi}; the power is one add of per-polarisation terms
      // (commutative, so every lane of the sample gets the same phase)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = (j + T * r) * C + c;
        double pw = norm2(reg[r]);
        if constexpr (P == 2) pw = pw + norm2(lds[(1 - p) * F + i]);
        phi[r] = -a.kappa * pw;
      }
      for_each_phasor16(phi, [&](int r, cd e) { reg[r] = cmul(reg[r], e); });
    } else {
      // g_x = g_y e^{-i phi} + 2 s kappa x,  s = -Im sum_q conj(g_q) y_q
      // (the states and the other cotangent are read from LDS again in the
      // second loop rather than held in registers)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = (j + T * r) * C + c;
        double pw = norm2(lds[p * F + i]);
        if constexpr (P == 2) pw = pw + norm2(lds[(1 - p) * F + i]);
        phi[r] = -a.kappa * pw;
      }
      for_each_phasor16(phi, [&](int r, cd e) {  // e = e^{-i phi}
        const int i = (j + T * r) * C + c;
        const cd yp = lds[p * F + i];
        double s = fma(reg[r].im, yp.re, -reg[r].re * yp.im);
        if constexpr (P == 2) {
          const cd yo = lds[(1 - p) * F + i];
          const cd go = lds[(P + 1 - p) * F + i];
          s = fma(go.im, yo.re, fma(-go.re, yo.im, s));
        }
        const double w = 2.0 * s * a.kappa;
        const cd x = cmul(yp, e);
        const cd gx = cmul(reg[r], e);
        reg[r] = {fma(w, x.re, gx.re), fma(w, x.im, gx.im)};
      });
    }
    fft<N1, false, 2, false>(reg, mylds, C, j, ltw);
  }
  if constexpr (AMODE == AMODE_LAST) {
    // every lane transforms (the block barriers need all of them); only the
    // cotangent is stored, the state is not needed past the span start
    fft<N1, true, 2, false>(reg, mylds, C, j, ltw);
    if (f == 0) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[r] = round_c64(cscale(reg[r], a.gspan));
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if constexpr (WAVE_F) col_store(fb, r, reg[r]);
    else store_c64(fp + (int64_t)(j + T * r) * a.n2, reg[r]);
  }
}

// ---------------------------------------------------------------------------
// K3 adjoint with stored states: column tiles of the cotangent alone (the
// forward pass stored the nonlinear step's input x in the time domain).
// Lanes: polarisation x C columns x T, as in the forward column pass.
//   cotangent mixed -> time;  phi = kappa sum_q |x_q|^2;
//   g' = g e^{-i phi},  s = -Im sum_q conj(g'_q) x_q  (= -Im sum_q conj(g_q) y_q
//   with y = x e^{i phi});  g_x = g' + 2 s kappa x;  time -> mixed.
// The per-polarisation powers and s terms are exchanged through the two
// halves of the LDS tile (FP64); both lanes of a sample form the sums in the
// same order, so they use the same phase and the same s.
// ---------------------------------------------------------------------------
template <int N1, int C, int P>
__global__ __launch_bounds__(P * C * (N1 / 16)) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k3_adj_stored(AdjStoredArgs a) {
  constexpr int T = N1 / 16;
  extern __shared__ __align__(16) unsigned char lds_as[];
  cd* lds = reinterpret_cast<cd*>(lds_as);
  const int tid = threadIdx.x;
  const int p = tid / (C * T);
  const int rem = tid % (C * T);
  const int c = rem % C;
  const int j = rem / C;
  const int tiles = a.n2 / C;
  const unsigned G = gridDim.x;
  const unsigned id = (G % 8 == 0) ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  const int64_t b = id / tiles;
  const int col0 = (int)(id % tiles) * C;
  const uint32_t tile_bytes = (uint32_t)((P * a.n - col0) * 8);
  const uint32_t lane_off = (uint32_t)(p * a.n + c + (int64_t)j * a.n2) * 8u;
  const uint32_t step = (uint32_t)(T * a.n2) * 8u;
  const col_buf gb = make_col_buf(a.cot + b * P * a.n + col0, tile_bytes, lane_off, step);
  const col_buf xb = make_col_buf(a.state + b * P * a.n + col0, tile_bytes, lane_off, step);
  cd reg[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) reg[r] = col_load(gb, r);
  float2 xs[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) xs[r] = col_load_f2(xb, r);
  // the pass twiddles' powers are formed in each transform (kept from the
  // inverse to the forward transform they would hold 60 registers)
  lane_twiddles<N1> ltw(a.tw1, j);
  ltw.opaque();
  cd* mylds = lds + p * (N1 * C) + c;
  fft<N1, true, false, false>(reg, mylds, C, j, ltw);  // cotangent: mixed -> time
  constexpr int F = N1 * C;  // one polarisation plane of a half
  double* pw = reinterpret_cast<double*>(lds_as);      // powers: first half
  double* sp = pw + P * F;                             // s terms: second half
  double phi[16];
  __syncthreads();  // the inverse FFT's LDS reads are done
  if constexpr (P == 2) {
#pragma unroll
    for (int r = 0; r < 16; ++r)
      pw[p * F + (j + T * r) * C + c] =
          fma((double)xs[r].x, (double)xs[r].x, (double)xs[r].y * (double)xs[r].y);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = (j + T * r) * C + c;
      phi[r] = a.kappa * (pw[i] + pw[F + i]);
    }
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r)
      phi[r] = a.kappa * fma((double)xs[r].x, (double)xs[r].x, (double)xs[r].y * (double)xs[r].y);
  }
  for_each_phasor16(phi, [&](int r, cd e) {  // e = e^{i phi}
    const cd g = cmulc(reg[r], e);
    reg[r] = g;
    sp[p * F + (j + T * r) * C + c] = fma(g.im, (double)xs[r].x, -g.re * (double)xs[r].y);
  });
  if constexpr (P == 2) __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = (j + T * r) * C + c;
    const double sr = P == 2 ? sp[i] + sp[F + i] : sp[i];
    const double w = 2.0 * sr * a.kappa;
    reg[r] = {fma(w, (double)xs[r].x, reg[r].re), fma(w, (double)xs[r].y, reg[r].im)};
  }
  ltw.opaque();
  fft<N1, false, false, false>(reg, mylds, C, j, ltw);  // time -> mixed
#pragma unroll
  for (int r = 0; r < 16; ++r) col_store(gb, r, reg[r]);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// padded FFT regions of both fields; the nonlinear exchange (2 P N1 C values)
// fits in them
template <int N1, int C, int P>
constexpr size_t adj_lds_bytes() {
  return (size_t)2 * P * (N1 + N1 / 16) * C * sizeof(cd);
}

template <int N1, int C, int P, int AMODE>
static hipError_t launch_k3_adj(const AdjArgs& a, hipStream_t st) {
  constexpr int T = N1 / 16;
  const size_t lds = adj_lds_bytes<N1, C, P>();
  const unsigned blocks = (unsigned)(a.batch * (a.n2 / C));
  hipLaunchKernelGGL((k3_adj<N1, C, P, AMODE>), dim3(blocks), dim3(2 * P * C * T), lds, st, a);
  return hipGetLastError();
}

template <int N1, int C, int P, int AMODE>
static hipError_t prepare_k3_adj() {
  const size_t lds = adj_lds_bytes<N1, C, P>();
  if (lds > 65536)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k3_adj<N1, C, P, AMODE>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

template <int N1, int C, int P>
static hipError_t launch_k3_adj_stored(const AdjStoredArgs& a, int64_t batch, hipStream_t st) {
  constexpr int T = N1 / 16;
  const size_t lds = (size_t)P * C * N1 * sizeof(cd);
  const unsigned blocks = (unsigned)(batch * (a.n2 / C));
  hipLaunchKernelGGL((k3_adj_stored<N1, C, P>), dim3(blocks), dim3(P * C * T), lds, st, a);
  return hipGetLastError();
}

template <int N1, int C, int P>
static hipError_t prepare_k3_adj_stored() {
  const size_t lds = (size_t)P * C * N1 * sizeof(cd);
  if (lds > 65536)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k3_adj_stored<N1, C, P>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

// adjoint column tiles: 4 columns (2 at N1 = 512), both fields, FP64 LDS
// (68 KB per workgroup with the padding)
template <int N1, int P>
static void fill_adj(KernelSet& ks) {
  constexpr int C = N1 == 512 ? 2 : 4;
  ks.adj[AMODE_FIRST] = &launch_k3_adj<N1, C, P, AMODE_FIRST>;
  ks.adj[AMODE_NL] = &launch_k3_adj<N1, C, P, AMODE_NL>;
  ks.adj[AMODE_LAST] = &launch_k3_adj<N1, C, P, AMODE_LAST>;
  ks.adj_columns = C;
  for (hipError_t e : {prepare_k3_adj<N1, C, P, AMODE_FIRST>(), prepare_k3_adj<N1, C, P, AMODE_NL>(),
                       prepare_k3_adj<N1, C, P, AMODE_LAST>()})
    if (e != hipSuccess) ks.prepare = e;
  // cotangent-only tiles with stored states: the forward column pass's wide
  // tile (8 columns, 4 at N1 = 512; 64 KB of FP64 LDS)
  constexpr int CS = N1 == 512 ? 4 : 8;
  ks.adj_stored = &launch_k3_adj_stored<N1, CS, P>;
  const hipError_t e = prepare_k3_adj_stored<N1, CS, P>();
  if (e != hipSuccess) ks.prepare = e;
}

void select_adjoint_kernels(int n1, int n_pol, KernelSet& ks) {
  switch (n1) {
    case 128: if (n_pol == 1) fill_adj<128, 1>(ks); else fill_adj<128, 2>(ks); break;
    case 256: if (n_pol == 1) fill_adj<256, 1>(ks); else fill_adj<256, 2>(ks); break;
    case 512: if (n_pol == 1) fill_adj<512, 1>(ks); else fill_adj<512, 2>(ks); break;
    default: break;
  }
}

}  // namespace ssfm
