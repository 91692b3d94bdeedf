// Register/LDS Stockham FFT for gfx950 (FP64 arithmetic, or FP32 for the
// FP32-arithmetic variant).
//
// Layout contract.  A length-M transform is carried by T = M/16 lanes; lane j
// holds the 16 elements j + T*r (r = 0..15) of its transform in registers, in
// both the input and the output order (the Stockham autosort keeps natural
// order).  Between radix passes the elements go through LDS; element i of a
// transform lives at lds[i * ls] (ls = element stride, so several transforms
// can be interleaved column-wise for conflict-free access).
//
// Pass structure (self-sorting Stockham, decimation in time): with Ns the
// product of the radices already applied, butterfly jj reads elements
// jj + r*M/R, multiplies element r by W_{Ns*R}^{(jj mod Ns) r}, applies a
// radix-R DFT and writes element r to (jj / Ns) * Ns * R + (jj mod Ns) + r*Ns.
// Radices are 16 repeated, then one of 8/4/2 for the remainder.  A lane runs
// 16/R butterflies per pass: jj = j + T*q, q = 0..16/R-1, whose element r is
// register q + r*16/R -- which is why the first pass can read the registers
// and the last pass can leave its output there.
//
// Twiddles come from a table built in FP64 on the host: for each pass p >= 1
// a block of ns(p) rows of radix(p) entries, row k holding
// W_{ns R}^{k r} = exp(-2 pi i k r / (ns R)); the inverse transform uses their
// conjugates.  The transforms are templates on the complex type of the
// registers: FP64 (cd) on the production path, so the coefficients of the
// linear operator carry no FP32 rounding (a fixed rounding error in them would
// repeat identically at every split step and grow linearly with the step
// count), or FP32 (cf) for the FP32-arithmetic variant, whose coefficients are
// the FP64 table values rounded to FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssfm {

// Complex value of real type R: FP64 (cd) on the default path, FP32 (cf) on
// the FP32-arithmetic variant.
template <typename R>
struct cplx {
  R re, im;
};
using cd = cplx<double>;
using cf = cplx<float>;

template <typename R>
__device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return {a.re * s, a.im * s}; }
// a * b
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b) {
  return {fma(a.re, b.re, a.im * b.im), fma(a.im, b.re, -a.re * b.im)};
}
template <bool CONJ, typename R>
__device__ __forceinline__ cplx<R> cmul_t(cplx<R> a, cplx<R> b) {
  return CONJ ? cmulc(a, b) : cmul(a, b);
}
// multiply by -i (forward) or +i (inverse): the exp(-+ i pi/2) rotation
template <bool INV, typename R>
__device__ __forceinline__ cplx<R> rot90(cplx<R> a) {
  return INV ? cplx<R>{-a.im, a.re} : cplx<R>{a.im, -a.re};
}
// value conversions between the two precisions (identity for the same type)
template <typename T, typename R>
__device__ __forceinline__ T cconv(cplx<R> v) {
  using U = decltype(T{}.re);
  return {(U)v.re, (U)v.im};
}

// exp(-2 pi i k / 16) for the forward transform, conjugate for the inverse.
template <bool INV, int K>
__device__ __forceinline__ cd w16() {
  constexpr double c1 = 0.92387953251128675613;  // cos(pi/8)
  constexpr double s1 = 0.38268343236508977173;  // sin(pi/8)
  constexpr double r2 = 0.70710678118654752440;  // cos(pi/4)
  constexpr int k = K & 15;
  constexpr double re = k == 0 ? 1.0 : k == 1 ? c1 : k == 2 ? r2 : k == 3 ? s1
                      : k == 4 ? 0.0 : k == 5 ? -s1 : k == 6 ? -r2 : k == 7 ? -c1
                      : k == 8 ? -1.0 : k == 9 ? -c1 : k == 10 ? -r2 : k == 11 ? -s1
                      : k == 12 ? 0.0 : k == 13 ? s1 : k == 14 ? r2 : c1;
  constexpr double sn = k == 0 ? 0.0 : k == 1 ? s1 : k == 2 ? r2 : k == 3 ? c1
                      : k == 4 ? 1.0 : k == 5 ? c1 : k == 6 ? r2 : k == 7 ? s1
                      : k == 8 ? 0.0 : k == 9 ? -s1 : k == 10 ? -r2 : k == 11 ? -c1
                      : k == 12 ? -1.0 : k == 13 ? -c1 : k == 14 ? -r2 : -s1;
  return {re, INV ? sn : -sn};
}

template <bool INV, int K, typename R>
__device__ __forceinline__ cplx<R> mul_w16(cplx<R> a) {
  if constexpr ((K & 15) == 0) return a;
  else if constexpr ((K & 15) == 4) return rot90<INV>(a);
  else if constexpr ((K & 15) == 8) return cplx<R>{-a.re, -a.im};
  else if constexpr ((K & 15) == 12) return rot90<!INV>(a);
  else return cmul(a, cconv<cplx<R>>(w16<INV, K>()));
}

template <bool INV, typename CT>
__device__ __forceinline__ void dft2(CT& a0, CT& a1) {
  CT t = a0;
  a0 = t + a1;
  a1 = t - a1;
}

template <bool INV, typename CT>
__device__ __forceinline__ void dft4(CT& a0, CT& a1, CT& a2, CT& a3) {
  CT t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = rot90<INV>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

// In-place DFT of length R on v[0..R-1], natural order in and out.
// R = 8 and 16 use the 4 x 2 and 4 x 4 Cooley-Tukey splits with the
// internal twiddles W_R^{b c}.
template <int R, bool INV, typename CT>
__device__ __forceinline__ void dft(CT* v) {
  if constexpr (R == 2) {
    dft2<INV>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<INV>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    // n = 2a + b, k = c + 4d
    dft4<INV>(v[0], v[2], v[4], v[6]);  // b = 0 -> Y0[c] at 2c
    dft4<INV>(v[1], v[3], v[5], v[7]);  // b = 1 -> Y1[c] at 2c+1
    v[3] = mul_w16<INV, 2>(v[3]);       // W8^1 = W16^2
    v[5] = mul_w16<INV, 4>(v[5]);       // W8^2
    v[7] = mul_w16<INV, 6>(v[7]);       // W8^3
    CT x[8];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      CT a = v[2 * c], b = v[2 * c + 1];
      dft2<INV>(a, b);
      x[c] = a;
      x[c + 4] = b;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = x[i];
  } else {
    static_assert(R == 16, "radix");
    // n = 4a + b, k = c + 4d
#pragma unroll
    for (int b = 0; b < 4; ++b) dft4<INV>(v[b], v[4 + b], v[8 + b], v[12 + b]);
    // element 4c + b now holds Y_b[c]; apply W16^{b c}
    v[5] = mul_w16<INV, 1>(v[5]);
    v[6] = mul_w16<INV, 2>(v[6]);
    v[7] = mul_w16<INV, 3>(v[7]);
    v[9] = mul_w16<INV, 2>(v[9]);
    v[10] = mul_w16<INV, 4>(v[10]);
    v[11] = mul_w16<INV, 6>(v[11]);
    v[13] = mul_w16<INV, 3>(v[13]);
    v[14] = mul_w16<INV, 6>(v[14]);
    v[15] = mul_w16<INV, 9>(v[15]);
    CT x[16];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      CT a0 = v[4 * c], a1 = v[4 * c + 1], a2 = v[4 * c + 2], a3 = v[4 * c + 3];
      dft4<INV>(a0, a1, a2, a3);
      x[c] = a0;
      x[c + 4] = a1;
      x[c + 8] = a2;
      x[c + 12] = a3;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = x[i];
  }
}

// Pass structure of a length-2^log2m transform: radix 16 repeated, then the
// remainder 2^(log2m mod 4).  Host (twiddle tables) and device share these.
__host__ __device__ constexpr int fft_passes(int log2m) {
  return log2m / 4 + (log2m % 4 ? 1 : 0);
}
__host__ __device__ constexpr int fft_radix(int log2m, int p) {
  return p < log2m / 4 ? 16 : 1 << (log2m % 4);
}
__host__ __device__ constexpr int fft_ns(int log2m, int p) {  // product of radices before pass p
  int s = 1;
  for (int i = 0; i < p; ++i) s *= fft_radix(log2m, i);
  return s;
}
// pass p >= 1 reads its twiddle rows [ns(p)][radix(p)] starting here
__host__ __device__ constexpr int fft_tw_offset(int log2m, int p) {
  int o = 0;
  for (int i = 1; i < p; ++i) o += fft_ns(log2m, i) * fft_radix(log2m, i);
  return o;
}

template <int M>
struct fft_shape {
  static constexpr int log2m = M == 64 ? 6 : M == 128 ? 7 : M == 256 ? 8 : M == 512 ? 9
                             : M == 1024 ? 10 : M == 2048 ? 11 : M == 4096 ? 12
                             : M == 8192 ? 13 : M == 16384 ? 14 : -1;
  static_assert(log2m > 0, "unsupported transform length");
  static constexpr int passes = fft_passes(log2m);
  static constexpr int T = M / 16;
  static constexpr int radix(int p) { return fft_radix(log2m, p); }
  static constexpr int ns(int p) { return fft_ns(log2m, p); }
  static constexpr int tw_offset(int p) { return fft_tw_offset(log2m, p); }
};

// Synchronisation of the LDS exchanges.  A transform carried by one wave
// only needs its own LDS accesses kept in program order (the LDS executes a
// wave's instructions in order), so a wavefront-scope fence pair suffices and
// no block barrier -- which would also wait for every outstanding global->LDS
// copy of the block -- is needed.  Transforms spanning several waves use a
// block barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <bool WAVE>
__device__ __forceinline__ void xsync() {
  if constexpr (WAVE) wave_sync();
  else __syncthreads();
}

// LDS element conversions: values are held as cd or rounded to float2.
template <typename R>
__device__ __forceinline__ void lds_put(cd* p, cplx<R> v) { *p = cconv<cd>(v); }
template <typename R>
__device__ __forceinline__ void lds_put(float2* p, cplx<R> v) {
  *p = make_float2((float)v.re, (float)v.im);
}
template <typename CT>
__device__ __forceinline__ CT lds_get(const cd* p) { return cconv<CT>(*p); }
template <typename CT>
__device__ __forceinline__ CT lds_get(const float2* p) {
  float2 v = *p;
  return cconv<CT>(cf{v.x, v.y});
}

// LDS slot of element i.  The first pass writes with a stride of 16
// elements.  PAD = 1: contiguous transforms (ls = 1) get one pad slot per 16
// elements, else every lane of a row would hit the same bank.  PAD = 2:
// interleaved transforms (element i of transform c at i ls + c) get one pad
// row per 16, for tiles of ls < 8 FP64 columns where the lanes of one LDS
// access group would otherwise span two rows a multiple of 1 KiB apart.
template <int PAD>
__device__ __forceinline__ int lds_slot(int i, int ls) {
  return PAD == 1 ? i + (i >> 4) : PAD == 2 ? (i + (i >> 4)) * ls : i * ls;
}

// The pass twiddles a lane uses, read once: entry 1 of row jj mod ns(p) for
// each butterfly jj = j + T q (q < 16/R) of every pass p >= 1.  A kernel that
// runs many transforms keeps them in registers instead of reading the table
// inside every transform (where the read would wait behind the lane's other
// outstanding global loads).
template <int M, typename CT = cd>
struct fft_twiddles {
  using S = fft_shape<M>;
  static constexpr int first(int P) {
    int c = 0;
    for (int p = 1; p < P; ++p) c += 16 / S::radix(p);
    return c;
  }
  static constexpr int count = first(S::passes);
  CT w[count > 0 ? count : 1];

  __device__ __forceinline__ void load(const cd* __restrict__ tw, int j) {
#pragma unroll
    for (int p = 1; p < S::passes; ++p) {
      const int R = S::radix(p), NS = S::ns(p);
#pragma unroll
      for (int q = 0; q < 16 / R; ++q)
        w[first(p) + q] = cconv<CT>(tw[S::tw_offset(p) + ((j + S::T * q) % NS) * R + 1]);
    }
  }
};

// W_{NS R}^k of butterfly jj (= j + T q) in pass P, from the table or from
// the lane's preloaded set.  (Every level takes the twiddle source as a
// restrict pointer: without it the compiler serialises the row pass's field
// loads.)
template <int M, int P, typename CT>
__device__ __forceinline__ CT pass_twiddle(const cd* __restrict__ tw, int jj, int) {
  using S = fft_shape<M>;
  return cconv<CT>(tw[S::tw_offset(P) + (jj % S::ns(P)) * S::radix(P) + 1]);
}
template <int M, int P, typename CT>
__device__ __forceinline__ CT pass_twiddle(const fft_twiddles<M, CT>* __restrict__ tw, int, int q) {
  return tw->w[fft_twiddles<M, CT>::first(P) + q];
}

// Read the inputs of pass P from LDS into the registers.
template <int M, int P, int PAD, typename L, typename CT>
__device__ __forceinline__ void pass_load(CT (&reg)[16], const L* lds, int ls, int j) {
  using S = fft_shape<M>;
  constexpr int R = S::radix(P);
  constexpr int NB = 16 / R;
  constexpr int T = S::T;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int jj = j + T * q;
#pragma unroll
    for (int r = 0; r < R; ++r) reg[q + r * NB] = lds_get<CT>(lds + lds_slot<PAD>(jj + r * (M / R), ls));
  }
}

// Twiddle, butterfly and write of pass P.  DST_REG: the outputs stay in the
// registers (last pass), otherwise they are written to LDS.
template <int M, int P, bool INV, bool DST_REG, int PAD, typename L, typename TW, typename CT>
__device__ __forceinline__ void pass_compute(CT (&reg)[16], L* lds, int ls, int j,
                                             TW __restrict__ tw) {
  using S = fft_shape<M>;
  constexpr int R = S::radix(P);
  constexpr int NS = S::ns(P);
  constexpr int NB = 16 / R;
  constexpr int T = S::T;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int jj = j + T * q;
    CT v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = reg[q + r * NB];
    if constexpr (NS > 1) {
      // W_{NS R}^{k r}, r = 1..R-1: w = W_{NS R}^k from this pass's table
      // block (row k, entry 1), powers by FP64 products (~r ulps of FP64, far
      // below the single-precision storage of the field; one load per
      // butterfly keeps the register footprint down)
      const CT w = pass_twiddle<M, P, CT>(tw, jj, q);
      CT wr = w;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        v[r] = cmul_t<INV>(v[r], wr);
        if (r + 1 < R) wr = cmul(wr, w);
      }
    }
    dft<R, INV>(v);
    if constexpr (DST_REG) {
#pragma unroll
      for (int r = 0; r < R; ++r) reg[q + r * NB] = v[r];
    } else {
      const int base = (jj / NS) * NS * R + (jj % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) lds_put(lds + lds_slot<PAD>(base + r * NS, ls), v[r]);
    }
  }
}

template <int M, bool INV, int P, int NT, int PAD, bool WAVE, typename L, typename TW, typename CT>
__device__ __forceinline__ void fft_rest(CT (&reg)[NT][16], L* lds, int tstride, int ls,
                                         int j, TW __restrict__ tw) {
  using S = fft_shape<M>;
  if constexpr (P < S::passes) {
    constexpr bool last = P == S::passes - 1;
    xsync<WAVE>();  // writes of the previous pass are visible
#pragma unroll
    for (int t = 0; t < NT; ++t) pass_load<M, P, PAD>(reg[t], lds + t * tstride, ls, j);
    if constexpr (!last) xsync<WAVE>();  // all reads done before overwriting
#pragma unroll
    for (int t = 0; t < NT; ++t)
      pass_compute<M, P, INV, last, PAD>(reg[t], lds + t * tstride, ls, j, tw);
    fft_rest<M, INV, P + 1, NT, PAD, WAVE>(reg, lds, tstride, ls, j, tw);
  }
}

template <int M, bool INV, int NT, int PAD, bool WAVE, typename L, typename TW, typename CT>
__device__ __forceinline__ void fft_multi_impl(CT (&reg)[NT][16], L* lds, int tstride, int ls,
                                               int j, TW __restrict__ tw) {
  using S = fft_shape<M>;
  if constexpr (S::passes == 1) {
#pragma unroll
    for (int t = 0; t < NT; ++t) pass_compute<M, 0, INV, true, PAD>(reg[t], lds, ls, j, tw);
  } else {
    xsync<WAVE>();  // earlier readers of the LDS regions are done
#pragma unroll
    for (int t = 0; t < NT; ++t)
      pass_compute<M, 0, INV, false, PAD>(reg[t], lds + t * tstride, ls, j, tw);
    fft_rest<M, INV, 1, NT, PAD, WAVE>(reg, lds, tstride, ls, j, tw);
  }
}

// NT unnormalised transforms of length M advanced in lockstep (they share the
// barriers); transform t uses the LDS region starting at lds + t * tstride.
// Lane j holds elements j + (M/16) r of each transform on entry and on exit.
// Forward uses exp(-2 pi i nk/M), inverse exp(+2 pi i nk/M).
// PAD selects the slot map (lds_slot); a padded transform occupies M + M/16
// slots (rows of ls slots for PAD = 2).  WAVE: every lane sharing the LDS
// regions is in the calling wave (see xsync); otherwise the whole block must
// call.  The pass twiddles come from the table tw, or from a lane's
// preloaded fft_twiddles<M>.
template <int M, bool INV, int NT, int PAD, bool WAVE, typename L, typename CT>
__device__ __forceinline__ void fft_multi(CT (&reg)[NT][16], L* lds, int tstride, int ls,
                                          int j, const cd* __restrict__ tw) {
  fft_multi_impl<M, INV, NT, PAD, WAVE>(reg, lds, tstride, ls, j, tw);
}

template <int M, bool INV, int PAD, bool WAVE, typename L, typename CT>
__device__ __forceinline__ void fft(CT (&reg)[16], L* lds, int ls, int j,
                                    const cd* __restrict__ tw) {
  fft_multi_impl<M, INV, 1, PAD, WAVE>(*reinterpret_cast<CT(*)[1][16]>(&reg), lds, 0, ls, j, tw);
}

template <int M, bool INV, int PAD, bool WAVE, typename L, typename CT>
__device__ __forceinline__ void fft(CT (&reg)[16], L* lds, int ls, int j,
                                    const fft_twiddles<M, CT>& tw) {
  fft_multi_impl<M, INV, 1, PAD, WAVE>(*reinterpret_cast<CT(*)[1][16]>(&reg), lds, 0, ls, j,
                                       &tw);
}

// The twiddle source of a kernel's transforms: the lane's pass twiddles in
// registers when there are at most two of them (read right after the
// kernel's field loads, so no transform waits on a table read behind other
// loads), else the table.
template <int M, typename CT = cd, bool PRE = (fft_twiddles<M, CT>::count <= 2)>
struct lane_twiddles {
  fft_twiddles<M, CT> t;
  __device__ __forceinline__ lane_twiddles(const cd* __restrict__ tw, int j) { t.load(tw, j); }
  // Hide the values from the optimiser: what a transform computes from them
  // (the powers of the pass twiddle) is then formed again in the next one
  // instead of being kept in registers from the earlier transform.
  __device__ __forceinline__ void opaque() {
#pragma unroll
    for (int i = 0; i < fft_twiddles<M, CT>::count; ++i)
      asm volatile("" : "+v"(t.w[i].re), "+v"(t.w[i].im));
  }
};
template <int M, typename CT>
struct lane_twiddles<M, CT, false> {
  const cd* tw;
  __device__ __forceinline__ lane_twiddles(const cd* __restrict__ table, int) : tw(table) {}
  __device__ __forceinline__ void opaque() {}
};

template <int M, bool INV, int PAD, bool WAVE, typename L, typename CT, bool PRE>
__device__ __forceinline__ void fft(CT (&reg)[16], L* lds, int ls, int j,
                                    const lane_twiddles<M, CT, PRE>& lt) {
  if constexpr (PRE) fft<M, INV, PAD, WAVE>(reg, lds, ls, j, lt.t);
  else fft<M, INV, PAD, WAVE>(reg, lds, ls, j, lt.tw);
}

}  // namespace ssfm
