// Types shared by the learned digital back-propagation kernels and their
// host side.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_dev.hpp"

namespace ssfm {
namespace ldbp {

constexpr int TAPS = 15;           // compiled filter length; shorter odd
                                   // filters are zero-padded about the centre
constexpr int HC = (TAPS - 1) / 2; // halo one step consumes on each side
constexpr int R = 4;               // consecutive samples per lane
constexpr int NRED = 32;           // reduced values per step: 15 complex tap
                                   // gradients, dL/dxi, one pad
constexpr int GUARD = 8;           // zero LDS slots before and after a region

// LDS stride (in complex FP64 slots) of one region array: guards and the
// pad slot of every 4 samples included, rounded to whole 128-byte lines.
inline int region_stride(int region) {
  const int j = region + 2 * GUARD - 1;
  return (j + (j >> 2) + 1 + 7) & ~7;
}

// Forward: steps [k0, k1) over tiles of w samples with a halo of
// 7 (k1 - k0) on each side.
struct FwdArgs {
  const float2* src;  // state at step k0, [batch][P][n]
  float2* dst;        // state at step k1
  float2* ckpt;       // NULL, or span-start states [K/S - 1][batch][P][n]
  const cd* taps15;   // [K][15], centred and zero-padded
  const double* xi;   // [K]
  int64_t n, batch;   // batch: the call's realisations (array strides)
  int64_t b0, count;  // this launch's realisations [b0, b0 + count)
  int k0, k1, spans_steps;
  int w, halo, region, ls, tiles;  // ls: LDS stride of one polarisation
};

// Backward of one span: steps [k0, k0 + s_steps).
struct BwdArgs {
  const float2* x0;    // state at the span start
  const float2* xs;    // state at the span end
  const float2* g_in;  // gradient w.r.t. the span-end state
  float2* g_out;       // gradient w.r.t. the span-start state
  const cd* taps15;
  const double* xi;
  double* partial;     // [K][blocks][NRED], blocks = batch * tiles
  int64_t n, batch;    // batch: the call's realisations (array strides)
  int64_t b0, count;   // this launch's realisations [b0, b0 + count)
  int k0, s_steps;
  int w, halo, region, ls, tiles;
};

// Loss: rows = batch * P, m symbols per row, ms per workgroup.
struct LossArgs {
  const float2* z;
  const float2* sym;
  const double* mf;
  cd* ubar;          // [rows][m]: dL/dRe u + i dL/dIm u
  double* partial;   // [blocks]: sum |u - s|^2
  int64_t n, m;
  int mf_half, sps, ms, tiles;
  double scale;      // 2 / (rows m)
};

struct MfAdjArgs {
  const cd* ubar;
  const double* mf;
  float2* grad;      // [rows][n]
  int64_t n, m;
  int mf_half, sps, ns, tiles;
};

hipError_t launch_fwd(int n_pol, const FwdArgs& a, int threads, size_t lds, hipStream_t st);
hipError_t launch_bwd(int n_pol, const BwdArgs& a, int threads, size_t lds, hipStream_t st);
hipError_t launch_loss(const LossArgs& a, int64_t rows, hipStream_t st);
hipError_t launch_loss_total(const double* partial, int count, double inv_count, double* loss,
                             hipStream_t st);
hipError_t launch_mf_adjoint(const MfAdjArgs& a, int64_t rows, hipStream_t st);
hipError_t launch_pad_taps(const cd* taps, int n_steps, int n_taps, cd* taps15, hipStream_t st);
hipError_t launch_reduce(const double* partial, int blocks, int n_steps, int n_taps,
                         cd* grad_taps, double* grad_xi, hipStream_t st);
// Raise the dynamic LDS limit of the forward/backward kernels.
hipError_t prepare(int n_pol, size_t fwd_lds, size_t bwd_lds);

}  // namespace ldbp
}  // namespace ssfm
