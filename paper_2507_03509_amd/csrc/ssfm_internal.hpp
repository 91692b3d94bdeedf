// Types shared by the kernel and host translation units of libssfm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_dev.hpp"

namespace ssfm {

// column-pass variants
enum { MODE_FIRST = 0,      // time -> mixed domain (start of the link)
       MODE_NL = 1,         // mixed -> time, nonlinear phase, time -> mixed
       MODE_EDFA = 2,       // mixed -> time, amplifier + ASE, time -> mixed
       MODE_LAST = 3,       // mixed -> time, amplifier + ASE (end of the link)
       MODE_NL_STORE = 4,   // MODE_NL, also storing the nonlinear step's input
       MODE_IFFT = 5,       // mixed -> time only (the transform alone, ssfm_dft)
       N_MODES = 6 };

// row-pass variants: the linear step, or one of its two transforms alone
enum { ROW_STEP = 0,        // twiddle, row FFT, x H, row IFFT, conj twiddle
       ROW_FFT = 1,         // twiddle, row FFT (ssfm_dft forward)
       ROW_IFFT = 2 };      // row IFFT, conj twiddle (ssfm_dft inverse)

struct RowArgs {
  float2* field;
  const cd* H;       // dispersion operator in [k1][k2] order
  const cd* tw;      // W_N2^m, m < N2
  const cd* twA;     // W_N^{a N2}, a < N1
  const cd* twB;     // W_N^{b}, b < N2
  int n1;
  int log2_n2;
  int conj_h;        // 1: multiply by conj(H) (adjoint / inverse linear step)
  int part;          // ROW_STEP, ROW_FFT or ROW_IFFT
};

struct ColArgs {
  float2* field;
  const cd* tw1;     // W_N1^m, m < N1
  int n2;
  int64_t n;         // N = N1 * N2 samples per polarisation
  double kappa;      // nonlinear coefficient of this step (MODE_NL)
  double gspan;      // field factor at the span end (MODE_EDFA, MODE_LAST)
  double sigma_h;    // ASE standard deviation per quadrature, 0 = none
  uint64_t seed;
  uint64_t realization0;
  int span;
  float2* ckpt;      // MODE_EDFA/LAST: if set, the pre-amplifier time-domain
                     // field is stored here ([batch][pol][n]), else unused
  const uint64_t* seeds;  // if set, realisation b's noise key is
                          // (seeds[b], span), else (seed, (realization0 + b) 2^16 + span)
  float2* states;    // MODE_NL_STORE: the time-domain field entering the
                     // nonlinear step, rounded to complex64, [batch][pol][n]
};

// adjoint column-pass variants (state = reconstructed forward field,
// cotangent = dL/dA*), on a work buffer holding both: realisation b's state
// at b, its cotangent at batch + b
enum { AMODE_FIRST = 0,  // state <- checkpoint, both: time -> mixed
       AMODE_NL = 1,     // both: mixed -> time, inverse step + pullback, -> mixed
       AMODE_LAST = 2 }; // cotangent: mixed -> time, times the span gain

struct AdjArgs {
  float2* work;      // [2 batch][pol][n]
  const float2* ckpt;  // AMODE_FIRST: span-end state [batch][pol][n]
  const cd* tw1;
  int n2;
  int64_t n;
  int64_t batch;
  double kappa;      // AMODE_NL
  double gspan;      // AMODE_LAST
};

struct LdsArgs {
  float2* field;
  const cd* h_half;  // exp(i (beta2/2) omega^2 h/2) / N, natural bin order
  const cd* h_full;  // exp(i (beta2/2) omega^2 h) / N
  const cd* tw;      // W_N^m, m < N
  const double* kappa;
  int steps;
  int span_begin, span_end;
  double gspan;
  double sigma_h;
  uint64_t seed;
  uint64_t realization0;
  const uint64_t* seeds;  // as ColArgs::seeds
  // adjoint (k1_adj): spans 0..span_end-1 of realisations realization0 + b
  const float2* field_in;  // forward input [batch][pol][n]
  float2* grad;            // cotangent in and out [batch][pol][n]
  float2* ckpt;            // span inputs [batch][spans][pol][n]
  float2* states;          // nonlinear-step inputs of one span [batch][steps][pol][n]
};

// adjoint column pass over the cotangent alone, with the forward state read
// from the nonlinear-step inputs stored by MODE_NL_STORE
struct AdjStoredArgs {
  float2* cot;         // cotangent [batch][pol][n], mixed domain in and out
  const float2* state; // the step's stored nonlinear-step input, time domain
  const cd* tw1;
  int n2;
  int64_t n;
  double kappa;
};

using RowLaunch = hipError_t (*)(const RowArgs&, int64_t, hipStream_t);
using ColLaunch = hipError_t (*)(const ColArgs&, int64_t, hipStream_t);
using LdsLaunch = hipError_t (*)(const LdsArgs&, int64_t, hipStream_t);
using LdsDftLaunch = hipError_t (*)(float2*, const cd*, int64_t, hipStream_t);
using AdjLaunch = hipError_t (*)(const AdjArgs&, hipStream_t);
using AdjStoredLaunch = hipError_t (*)(const AdjStoredArgs&, int64_t, hipStream_t);

struct FourStepKernels {
  ColLaunch col[N_MODES] = {};
  int columns = 0;
  hipError_t prepare_status = hipSuccess;
};

struct KernelSet {
  int path = 0;  // 1 = LDS-resident, 2 = four-step
  bool fp32 = false;  // FP32-arithmetic variant (no adjoint kernels)
  int n1 = 0, n2 = 0;
  LdsLaunch lds = nullptr;
  LdsLaunch lds_adj = nullptr;  // adjoint of the LDS-resident path (FP64)
  LdsDftLaunch lds_dft[2] = {nullptr, nullptr};  // the LDS-resident transform: forward, inverse
  RowLaunch row_wide = nullptr, row_narrow = nullptr;
  int rows_wide = 0, rows_narrow = 0;  // rows per workgroup
  // column tiles: narrow (2 columns) and wide (8)
  FourStepKernels narrow, wide;
  AdjLaunch adj[3] = {nullptr, nullptr, nullptr};
  int adj_columns = 0;
  AdjStoredLaunch adj_stored = nullptr;
  hipError_t prepare = hipSuccess;
};

// Pick the kernel instantiations for n samples per polarisation, FP64 or
// (fp32) FP32 arithmetic.  Returns false if no instantiation exists for that
// size.
bool select_kernels(int64_t n, int n_pol, bool fp32, KernelSet& ks);

// Fill ks.adj for the four-step column length n1 (leaves it empty if there is
// no adjoint instantiation for that length).
void select_adjoint_kernels(int n1, int n_pol, KernelSet& ks);

}  // namespace ssfm
