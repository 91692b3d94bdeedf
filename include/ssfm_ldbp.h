/*
 * ssfm_ldbp.h -- C ABI of learned digital back-propagation (LDBP) in
 * libssfm: forward, loss and reverse-mode gradient of a trainable
 * back-propagation model on the MI355X.
 *
 * Model (learned digital back-propagation: Haeger and Pfister,
 * "Physics-based deep learning for fiber-optic communication systems",
 * IEEE J. Sel. Areas Commun. 39(1), 2021).  Per realisation, a field
 * x in C^{P x N} (P polarisations, N samples, circular time axis) passes K
 * steps k = 0..K-1:
 *
 *   FIR       y_p[n] = sum_{t=0}^{T-1} h_k[t] x_p[(n + c - t) mod N],
 *             c = (T - 1) / 2, one complex filter for both polarisations
 *   Kerr      x_p[n] <- y_p[n] exp(i xi_k sum_q |y_q[n]|^2)
 *
 * with trainable taps h_k (T complex) and a trainable real coefficient
 * xi_k per step.  Steps are grouped in spans of S steps (the back-propagated
 * fibre spans); the state is rounded to complex64 at every span boundary,
 * which is where checkpoints are taken.
 *
 * Loss: a real matched filter g of 2R + 1 taps sampled at the symbol
 * instants, u_p[m] = sum_{j=-R}^{R} g[j + R] z_p[(sps m - j) mod N], and
 * L = mean over (realisation, polarisation, symbol) of |u_p[m] - s_p[m]|^2
 * for the transmitted symbols s.
 *
 * Gradients use PyTorch's complex convention: for a complex quantity w the
 * gradient is dL/dRe(w) + i dL/dIm(w); for the real xi_k it is dL/dxi_k.
 *
 * Layouts (device memory, owned by the caller):
 *   fields      complex64 (float re, im) [batch][P][N]
 *   taps        complex128 (double re, im) [K][T]
 *   xi          double [K]
 *   symbols     complex64 [batch][P][N / sps]
 *   mf          double [2R + 1]
 *   checkpoints complex64 [K/S - 1][batch][P][N]: the state at the start of
 *               spans 1 .. K/S - 1 (span 0 starts from the input itself)
 * Arithmetic is FP64; fields are stored complex64.  Every entry point is
 * asynchronous on `stream` (NULL = default stream) and returns a status
 * code from ssfm.h; ssfm_last_error() describes a failure.  A handle owns
 * device workspace that it grows on first use: calls on one handle must not
 * run concurrently (serialise them on one stream).  ssfm_ldbp_backward runs
 * the two halves of a batch concurrently, one on `stream` and one on a
 * worker stream of the handle (created on first use, default priority)
 * forked from `stream` and joined back into it, when each half still fills
 * 512 workgroups per launch; the results are the same bits either way.
 * SSFM_LDBP_STREAMS in the environment at handle creation sets 1 (one
 * stream) or 2..4 (that many parts, on as many streams, in
 * ssfm_ldbp_forward and ssfm_ldbp_backward whenever the batch has as many
 * realisations).
 */
#ifndef SSFM_LDBP_H_
#define SSFM_LDBP_H_

#include <stdint.h>

#include "ssfm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssfm_ldbp_desc {
  int32_t n_pol;          /* P: 1 or 2                                      */
  int32_t n_steps;        /* K: 1 .. 4096                                   */
  int32_t n_taps;         /* T: odd, 1 .. 15                                */
  int32_t steps_per_span; /* S: 1 .. 4, dividing K                          */
  int64_t n_samples;      /* N per polarisation: power of two, 2^6 .. 2^22  */
  int32_t sps;            /* samples per symbol of the loss: 1 .. 64, | N   */
  int32_t mf_taps;        /* 2R + 1: odd, 1 .. 257                          */
} ssfm_ldbp_desc;

typedef struct ssfm_ldbp_s* ssfm_ldbp_t;

/* Create a handle for `desc` on HIP device `hip_device`.  SSFM_EINVAL for a
 * malformed description or NULL out; SSFM_EHIP if the device cannot be
 * selected.  Allocates nothing on the device yet. */
int ssfm_ldbp_create(const ssfm_ldbp_desc* desc, int hip_device, ssfm_ldbp_t* out);

/* Release a handle and its workspace (NULL accepted); no call using it may
 * still be running. */
int ssfm_ldbp_destroy(ssfm_ldbp_t h);

/* Initial parameters that back-propagate `link` (host function, no device
 * work): K = n_spans * steps_per_span steps, the last span first.  Step k
 * covers 1/S of a span (S = steps_per_span): its filter is the T-tap
 * truncation, centred (offsets t - (T-1)/2), of the impulse response of the
 * inverse dispersion exp(-i (beta2/2) w^2 L/S) on the link's n_samples-point
 * DFT grid (inverse DFT by its direct sum), divided by the truncated filter's
 * peak gain over that grid (so that no frequency is amplified step after
 * step) and, for the first step of each span (k mod S = 0), by the span's
 * field gain sqrt(G) exp(-alpha L/2) (undoing the amplifier); its Kerr
 * coefficient is xi_k = -c_nl gamma h_nl exp(-alpha z), the forward model's
 * nonlinear phase per unit power over the step, with h_nl =
 * 2 sinh(alpha L/(2S))/alpha and z = L - (k mod S + 1/2) L/S the step's
 * midpoint (the model of Haeger and Pfister, initialised from the link).
 *   taps: host complex128 [K][T] (double re, im), written
 *   xi:   host double [K], written
 * The link's n_samples may be up to 2^22 (the LDBP range); its span count,
 * fibre and amplifier parameters are used, the rest ignored.  Errors:
 * SSFM_EINVAL for NULL pointers, T not odd in 1..15, S not in 1..4,
 * K > 4096, n_samples not a power of two in [2^6, 2^22], non-finite
 * parameters. */
int ssfm_ldbp_init_params(const ssfm_link* link, int32_t n_taps, int32_t steps_per_span,
                          double* taps, double* xi);

/* Bytes of the checkpoint buffer for `batch` realisations:
 * (K/S - 1) * batch * P * N * 8 (0 when K = S). */
int ssfm_ldbp_checkpoint_bytes(ssfm_ldbp_t h, int64_t batch, int64_t* bytes);

/* Forward model: field_out = LDBP(field_in).  field_in and field_out may
 * not overlap.  checkpoints: NULL, or a buffer of
 * ssfm_ldbp_checkpoint_bytes that receives the span-start states needed by
 * ssfm_ldbp_backward.  SSFM_EINVAL for NULL or misaligned (8-byte) pointers
 * or batch < 1; SSFM_EHIP on a launch failure. */
int ssfm_ldbp_forward(ssfm_ldbp_t h, const void* field_in, void* field_out,
                      const void* taps, const double* xi, int64_t batch,
                      void* checkpoints, void* stream);

/* Loss of `field_out` against `symbols` (layouts above) into the device
 * double *loss; if grad_out is not NULL it receives the gradient of the loss
 * w.r.t. field_out (complex64, layout of the fields).  Errors as
 * ssfm_ldbp_forward, SSFM_ENOMEM if the workspace cannot grow. */
int ssfm_ldbp_loss(ssfm_ldbp_t h, const void* field_out, const void* symbols,
                   const double* mf, int64_t batch, double* loss, void* grad_out,
                   void* stream);

/* Reverse-mode gradient of ssfm_ldbp_forward (vector-Jacobian product).
 *   field_in, field_out, taps, xi, checkpoints: exactly as passed to and
 *       produced by the forward call (checkpoints required when K > S);
 *   grad: on entry the gradient w.r.t. field_out, on exit the gradient
 *       w.r.t. field_in (complex64, in place);
 *   grad_taps: receives complex128 [K][T]; grad_xi: receives double [K]
 *       (both written, not accumulated).
 * Method: per span, from the last to the first, the span's inner states
 * are recomputed from its checkpoint, then the span's steps are pulled back
 * in reverse: Kerr step gy = gz e^{-i phi} + 2 xi s y with
 * s = -Im sum_q conj(gz_q) z_q and dL/dxi += sum |y|^2 s; FIR step
 * gx[m] = sum_t conj(h[t]) gy[m - c + t] and
 * dL/dh[t] += sum gy[n] conj(x[n + c - t]).  Parameter gradients are summed
 * over the batch in a fixed order (bitwise reproducible).  Errors as
 * ssfm_ldbp_loss. */
int ssfm_ldbp_backward(ssfm_ldbp_t h, const void* field_in, const void* field_out,
                       const void* taps, const double* xi, int64_t batch,
                       const void* checkpoints, void* grad, void* grad_taps,
                       double* grad_xi, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SSFM_LDBP_H_ */
