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

// Sum over the polarisations of a sample: across the lane pair (l, l ^ 32)
// for two, the value itself for one.
template <int P>
__device__ __forceinline__ double pol_sum(double x) {
  if constexpr (P == 2) return pair32_sum(x);
  else return x;
}

// ---------------------------------------------------------------------------
// K3 adjoint: column tiles of the work buffer holding, for realisation b, the
// reconstructed forward state (at b) and the cotangent dL/dA* (at batch + b).
// The tile and lane map are the forward column pass's (C columns x N1 rows x
// P polarisations; 8 columns, so every load and store moves 64-byte runs of
// a row); a workgroup carries the state's tile first, then the cotangent's.
//   AMODE_FIRST  state <- span-end checkpoint; both fields time -> mixed
//   AMODE_NL     both mixed -> time; with y the state (output of the forward
//                nonlinear step), e = e^{-i phi}, phi = kappa sum_q |y_q|^2:
//                  state     x   = y e                       (inverse step)
//                  cotangent g_x = ge + 2 s kappa x,  ge = g_y e,
//                            s   = -Im sum_q conj(g_y,q) y_q = -Im sum_q conj(ge_q) x_q
//                (y = x conj(e)); then both time -> mixed
//   AMODE_LAST   cotangent mixed -> time, times the span gain (the pullback of
//                the amplifier, applied at the end of the span's reverse sweep
//                because everything in between is linear in the cotangent);
//                the state is not needed past the span start
// Between the halves of AMODE_NL the lane keeps its x (rounded to complex64)
// and phi (rounded to FP32) in LDS slots of its own (registers would spill).
// The transforms exchange through LDS in FP32 (the arithmetic stays FP64):
// with x and phi that keeps a workgroup at 80 KB, two per CU.  Each rounding
// is of the size of the complex64 field store between kernels.  Sums over
// the polarisations are formed across the lane pair, lower lane first.
// ---------------------------------------------------------------------------
template <int N1, int C, int P, int AMODE>
__global__ __launch_bounds__(P * C * (N1 / 16)) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k3_adj(AdjArgs a) {
  constexpr int T = N1 / 16;
  static_assert(P == 1 || C * T >= 32, "two polarisations need lane pairs");
  // [P][N1][C] transform exchange, then [16][lanes] the lanes' x and phi
  extern __shared__ __align__(16) unsigned char lds_adj[];
  float2* lds = reinterpret_cast<float2*>(lds_adj);
  float2* xl = lds + P * N1 * C;
  float* pl = reinterpret_cast<float*>(xl + P * N1 * C);  // [16][lanes] the lanes' phase
  const int tid = threadIdx.x;
  int p, c, j;
  if constexpr (P == 2) {
    const int l = tid & 63;
    const int q = (tid >> 6) * 32 + (l & 31);
    p = l >> 5;
    c = q % C;
    j = q / C;
  } else {
    p = 0;
    c = tid % C;
    j = tid / C;
  }
  const int tiles = a.n2 / C;
  const unsigned G = gridDim.x;
  const unsigned id = (G % 8 == 0) ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  const int64_t b = id / tiles;
  const int col0 = (int)(id % tiles) * C;
  const uint32_t tile_bytes = (uint32_t)((P * a.n - col0) * 8);
  const uint32_t lane_off = (uint32_t)(p * a.n + c + (int64_t)j * a.n2) * 8u;
  const uint32_t step = (uint32_t)(T * a.n2) * 8u;
  const col_buf sb = make_col_buf(a.work + b * P * a.n + col0, tile_bytes, lane_off, step);
  const col_buf gb =
      make_col_buf(a.work + (a.batch + b) * P * a.n + col0, tile_bytes, lane_off, step);
  float2* mylds = lds + p * (N1 * C) + c;
  const lane_twiddles<N1> ltw(a.tw1, j);
  cd reg[16];
  if constexpr (AMODE == AMODE_FIRST) {
    // state <- span-end checkpoint; both fields time -> mixed
    const col_buf kb = make_col_buf(a.ckpt + b * P * a.n + col0, tile_bytes, lane_off, step);
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[r] = col_load<cd>(kb, r);
    fft<N1, false, 0, false>(reg, mylds, C, j, ltw);
#pragma unroll
    for (int r = 0; r < 16; ++r) col_store(sb, r, reg[r]);
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[r] = col_load<cd>(gb, r);
    fft<N1, false, 0, false>(reg, mylds, C, j, ltw);
#pragma unroll
    for (int r = 0; r < 16; ++r) col_store(gb, r, reg[r]);
  } else if constexpr (AMODE == AMODE_NL) {
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[r] = col_load<cd>(sb, r);
    fft<N1, true, 0, false>(reg, mylds, C, j, ltw);
    {
      double phi[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        phi[r] = -a.kappa * pol_sum<P>(norm2(reg[r]));
        pl[r * (P * C * T) + tid] = (float)phi[r];
      }
      for_each_phasor16(phi, [&](int r, cd e) { reg[r] = cmul(reg[r], e); });
    }
#pragma unroll
    for (int r = 0; r < 16; ++r)
      xl[r * (P * C * T) + tid] = make_float2((float)reg[r].re, (float)reg[r].im);
    fft<N1, false, 0, false>(reg, mylds, C, j, ltw);
#pragma unroll
    for (int r = 0; r < 16; ++r) col_store(sb, r, reg[r]);
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[r] = col_load<cd>(gb, r);
    fft<N1, true, 0, false>(reg, mylds, C, j, ltw);
    {
      double phi[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) phi[r] = (double)pl[r * (P * C * T) + tid];
      // x is read again below rather than held across the phasor (the
      // fence keeps the compiler from merging the two reads, which would
      // spill)
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      for_each_phasor16(phi, [&](int r, cd e) {
        const float2 v = xl[r * (P * C * T) + tid];
        const cd x{(double)v.x, (double)v.y};
        const cd ge = cmul(reg[r], e);
        const double s = pol_sum<P>(fma(ge.im, x.re, -ge.re * x.im));
        const double w = 2.0 * s * a.kappa;
        reg[r] = {fma(w, x.re, ge.re), fma(w, x.im, ge.im)};
      });
    }
    fft<N1, false, 0, false>(reg, mylds, C, j, ltw);
#pragma unroll
    for (int r = 0; r < 16; ++r) col_store(gb, r, reg[r]);
  } else {
    // the cotangent mixed -> time, times the span gain; the state is not
    // needed past the span start
#pragma unroll
    for (int r = 0; r < 16; ++r) reg[r] = col_load<cd>(gb, r);
    fft<N1, true, 0, false>(reg, mylds, C, j, ltw);
#pragma unroll
    for (int r = 0; r < 16; ++r) col_store(gb, r, round_c64(cscale(reg[r], a.gspan)));
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

template <int N1, int C, int P>
constexpr size_t adj_lds_bytes() {
  // exchange, the lanes' x and phi
  return (size_t)2 * P * N1 * C * sizeof(float2) + (size_t)P * N1 * C * sizeof(float);
}

template <int N1, int C, int P, int AMODE>
static hipError_t launch_k3_adj(const AdjArgs& a, hipStream_t st) {
  constexpr int T = N1 / 16;
  const size_t lds = adj_lds_bytes<N1, C, P>();
  const unsigned blocks = (unsigned)(a.batch * (a.n2 / C));
  hipLaunchKernelGGL((k3_adj<N1, C, P, AMODE>), dim3(blocks), dim3(P * C * T), lds, st, a);
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

// adjoint column tiles: the forward pass's wide tile (8 columns; 80 KB of
// LDS), state then cotangent
template <int N1, int P>
static void fill_adj(KernelSet& ks) {
  constexpr int C = 8;
  ks.adj[AMODE_FIRST] = &launch_k3_adj<N1, C, P, AMODE_FIRST>;
  ks.adj[AMODE_NL] = &launch_k3_adj<N1, C, P, AMODE_NL>;
  ks.adj[AMODE_LAST] = &launch_k3_adj<N1, C, P, AMODE_LAST>;
  ks.adj_columns = C;
  for (hipError_t e : {prepare_k3_adj<N1, C, P, AMODE_FIRST>(), prepare_k3_adj<N1, C, P, AMODE_NL>(),
                       prepare_k3_adj<N1, C, P, AMODE_LAST>()})
    if (e != hipSuccess) ks.prepare = e;
  // cotangent-only tiles with stored states: the forward column pass's wide
  // tile (8 columns; 64 KB of FP64 LDS)
  constexpr int CS = 8;
  ks.adj_stored = &launch_k3_adj_stored<N1, CS, P>;
  const hipError_t e = prepare_k3_adj_stored<N1, CS, P>();
  if (e != hipSuccess) ks.prepare = e;
}

void select_adjoint_kernels(int n1, int n_pol, KernelSet& ks) {
  switch (n1) {
    case 128: if (n_pol == 1) fill_adj<128, 1>(ks); else fill_adj<128, 2>(ks); break;
    case 256: if (n_pol == 1) fill_adj<256, 1>(ks); else fill_adj<256, 2>(ks); break;
    default: break;
  }
}

}  // namespace ssfm
