/*
 * ssfm.h -- C ABI of the MI355X split-step Fourier (SSFM) propagation library.
 *
 * The library propagates sampled optical fields through amplified fibre
 * links.  Per polarisation p the field A_p(z, T) obeys
 *
 *   dA_p/dz = -(alpha/2) A_p - i (beta2/2) d^2A_p/dT^2
 *             + i c_nl gamma (sum_q |A_q|^2) A_p
 *
 * (the nonlinear Schroedinger equation with loss, Agrawal, "Nonlinear Fiber
 * Optics", ch. 2; with two polarisations and c_nl = 8/9 it is the Manakov-PMD
 * equation of Marcuse, Menyuk and Wai, J. Lightwave Technol. 15(9), 1997).
 * The paper accompanying this library does not state a propagation model;
 * the equation, scheme and amplifier model are the textbook ones above.
 *
 * Scheme: symmetric split-step Fourier method with merged half steps.  A
 * span of n steps of length h = span/n is
 *   L(h/2) . [N(h) . L(h)]^(n-1) . N(h) . L(h/2) . EDFA
 * with L(x) the exact linear (dispersion + loss) solution over length x,
 * applied in the frequency domain, and N(h) the exact nonlinear phase
 * rotation with the loss-weighted length h_nl = 2 sinh(alpha h/2)/alpha.
 * The amplifier multiplies the field by sqrt(G) and, when enabled, adds
 * amplified spontaneous emission: a white circular complex Gaussian of
 * variance n_sp (G-1) h_planck nu fs per polarisation (n_sp = NF/2).
 *
 * Noise draws (bitwise contract): Philox4x64-10 (Salmon et al., SC'11) with
 * key (seed, realization * 2^16 + span) and counter (t, 0, 0, 0) for time
 * sample t; words (w0, w1) serve polarisation x and (w2, w3) polarisation
 * y; u = ((w >> 41) + 1/2) 2^-23; Box-Muller g = sqrt(-2 ln u1) e^{2 pi i u2};
 * noise = sqrt(variance / 2) * g.
 *
 * Field layout: complex64 interleaved (re, im) in device memory, shape
 * [batch][n_pol][n_samples], each polarisation contiguous, natural time
 * order.  All entry points return an int status (0 = success, negative =
 * error); nothing is thrown across the ABI.  On error, ssfm_last_error()
 * returns a thread-local message describing it.
 */
#ifndef SSFM_H_
#define SSFM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSFM_OK 0
#define SSFM_EINVAL (-1)       /* an argument is out of range or malformed    */
#define SSFM_ENOMEM (-2)       /* a device or host allocation failed          */
#define SSFM_EHIP (-3)         /* a HIP runtime call or kernel launch failed  */
#define SSFM_EUNSUPPORTED (-4) /* valid request this build does not implement */

/* ssfm_link.flags: FP32 arithmetic (a precision study variant, forward
 * only).  The default path computes every step in FP64 registers and rounds
 * only the stored field to complex64.  With this flag the FFT butterflies,
 * the twiddle multiplications (with the FP64 twiddle tables rounded to FP32)
 * and the nonlinear phase rotation (FP32 sine and cosine) run in FP32, while
 * the dispersion multiply -- the per-step linear operator -- and the span-end
 * gain and noise stay FP64.  Its error against the FP64 reference grows with
 * the step count (a fixed rounding of the transform's coefficients repeats at
 * every step); ssfm_adjoint and ssfm_adjoint_noalloc refuse such plans with
 * SSFM_EUNSUPPORTED. */
#define SSFM_FLAG_FP32_ARITHMETIC 1u

/* One amplified fibre link, in the units such links are quoted in.
 * Every span is identical.  The library converts to SI internally:
 * alpha[1/m] = alpha_db_per_km * ln(10)/10 / 1e3 (power attenuation),
 * beta2[s^2/m] = beta2_ps2_per_km * 1e-27, gamma[1/(W m)] = gamma_per_w_km
 * * 1e-3, h = span_km * 1e3 / steps_per_span. */
typedef struct ssfm_link {
  int32_t n_pol;             /* 1 = scalar NLSE, 2 = Manakov                  */
  int32_t n_spans;           /* >= 1, < 65536                                 */
  int32_t steps_per_span;    /* >= 1                                          */
  int32_t ase;               /* 0 = noiseless amplifier, 1 = add ASE (G > 1)  */
  int64_t n_samples;         /* per polarisation; power of two, 2^6 .. 2^18   */
  double sample_rate_hz;     /* fs > 0; sample spacing 1/fs                   */
  double span_km;            /* > 0                                           */
  double alpha_db_per_km;    /* any finite value (negative = gain)            */
  double beta2_ps2_per_km;   /* any finite value                              */
  double gamma_per_w_km;     /* any finite value                              */
  double nl_factor;          /* c_nl; NaN selects 1 (n_pol 1) or 8/9 (n_pol 2) */
  double edfa_gain_db;       /* power gain per span end; 0 dB = unity gain    */
  double edfa_nf_db;         /* noise figure, used when ase = 1               */
  double carrier_hz;         /* optical carrier; NaN selects 193.4145 THz     */
  uint32_t flags;            /* 0, or SSFM_FLAG_FP32_ARITHMETIC               */
  uint32_t reserved;         /* must be 0                                     */
} ssfm_link;

/* Opaque plan: device tables (dispersion operator, twiddles) for one link on
 * one device.  The tables are immutable after creation, so forward calls
 * (ssfm_forward, ssfm_forward_spans) on one plan may run concurrently on
 * several streams of its device.  ssfm_adjoint calls on one plan share the
 * plan's adjoint workspace and are serialised by the library (see there).
 * ssfm_plan_autotune, ssfm_plan_set_forward_streams and the profiling window
 * change the plan: they must not overlap other calls on it. */
typedef struct ssfm_plan_s* ssfm_plan_t;

/* Plan description, for callers that report what will run. */
typedef struct ssfm_plan_info {
  int32_t path;              /* 1 = LDS-resident field, 2 = four-step passes  */
  int32_t n1;                /* four-step: column FFT length (0 for path 1)   */
  int32_t n2;                /* four-step: row FFT length (0 for path 1)      */
  int32_t columns_per_tile;  /* four-step: column-tile width at batch >= 8    */
  int64_t launches_per_call; /* kernel launches of one ssfm_forward call of  *
                              * at most chunk_realisations realisations       */
  int64_t table_bytes;       /* device memory owned by the plan               */
  int64_t chunk_realisations; /* four-step: the most realisations a forward   *
                              * call carries through the link at a time:     *
                              * larger batches run as equal chunks, one      *
                              * after the other, each about 256 MiB (the     *
                              * Infinity Cache; SSFM_CHUNK_MIB in the        *
                              * environment at plan creation sets another    *
                              * size, 0 none); the adjoint's chunks are half *
                              * as large (two fields).  0 for path 1 or      *
                              * without chunks                               */
} ssfm_plan_info;

/* Build a plan for `link` on HIP device `hip_device`.
 * On success *out receives a plan that the caller releases with
 * ssfm_plan_destroy.  Errors: SSFM_EINVAL for an invalid link or NULL out
 * (no device work is done), SSFM_ENOMEM if the tables cannot be allocated,
 * SSFM_EHIP if the device cannot be selected.  Blocks until the tables are
 * on the device. */
int ssfm_plan(const ssfm_link* link, int hip_device, ssfm_plan_t* out);

/* Release a plan and its device memory.  NULL is accepted.  The caller must
 * ensure no call using the plan is still running on any stream. */
int ssfm_plan_destroy(ssfm_plan_t plan);

/* Fill *info for `plan`.  SSFM_EINVAL if either pointer is NULL. */
int ssfm_plan_get_info(ssfm_plan_t plan, ssfm_plan_info* info);

/* Propagate `batch` independent fields through the whole link, in place.
 *   field:  device pointer to complex64 [batch][n_pol][n_samples], 8-byte
 *           aligned, owned by the caller; overwritten with the output.
 *   batch:  >= 1.  Realisation r of the batch draws its noise with key
 *           (seed, r * 2^16 + span).  On the four-step path a batch above
 *           the plan's chunk_realisations (ssfm_plan_info) runs as equal
 *           chunks through the whole link, one after the other (each as
 *           one or more concurrent parts, ssfm_plan_set_forward_streams),
 *           with the same bits as one pass over the batch.
 *   stream: hipStream_t to order the work on (NULL = default stream).
 * Asynchronous with respect to the host: returns once the kernels are
 * enqueued; a fault inside a kernel surfaces at the caller's next
 * synchronisation.  Errors: SSFM_EINVAL (NULL plan/field, misaligned field,
 * batch < 1), SSFM_EHIP (launch failure). */
int ssfm_forward(ssfm_plan_t plan, void* field, int64_t batch, uint64_t seed,
                 void* stream);

/* The plan's discrete Fourier transform alone, for checking the transform
 * stages of the propagation against the DFT's definition: every polarisation
 * of every realisation of `field` (layout as ssfm_forward) is replaced, in
 * place, by its unnormalised length-n_samples DFT
 *   X[k] = sum_t x[t] exp(-+2 pi i t k / n_samples)   (inverse = 0 / 1),
 * computed by the same FFT stages, in the same arithmetic, as the
 * propagation: the LDS-resident transform for n_samples <= 2^13; on the
 * four-step path the column FFT pass and the twiddle + row FFT pass
 * (inverse: the row IFFT + conjugate twiddle pass, then the column IFFT).
 * Frequency order: natural on the LDS-resident path; on the four-step path
 * the passes' own order, bin k = k1 + n1 k2 (k1 < n1, k2 < n2) at position
 * k1 n2 + k2 (n1, n2 from ssfm_plan_get_info); the inverse takes its input
 * in that order.  Asynchronous.  Errors: those of ssfm_forward, SSFM_EINVAL
 * for inverse not 0 or 1. */
int ssfm_dft(ssfm_plan_t plan, void* field, int64_t batch, int32_t inverse, void* stream);

/* As ssfm_forward, restricted to spans [span_begin, span_end) and with the
 * noise realisation index of batch entry b equal to realization0 + b.  A run
 * split into consecutive span ranges gives the same result, bit for bit, as
 * one call over the union (span-granular checkpoint and resume).
 * SSFM_EINVAL unless 0 <= span_begin <= span_end <= n_spans. */
int ssfm_forward_spans(ssfm_plan_t plan, void* field, int64_t batch,
                       uint64_t seed, uint64_t realization0, int32_t span_begin,
                       int32_t span_end, void* stream);

/* Adjoint (reverse-mode) propagation: the vector-Jacobian product of
 * ssfm_forward (seed, realisations 0..batch-1, all spans) at `field_in`.
 *   field_in: device complex64 [batch][n_pol][n_samples], the forward input;
 *             read only.
 *   grad:     device complex64 of the same shape; on entry the cotangent
 *             dL/dA_out* of a real loss L at the forward output, on exit
 *             dL/dA_in* (any constant factor on the way in, such as the 2 of
 *             PyTorch's complex gradients, carries through: the map is
 *             real-linear in the cotangent).
 * Method: a forward pass keeps the span-end states (span checkpoints); the
 * reverse sweep then rebuilds each span's intermediate states from its
 * checkpoint with the exact inverse steps (in the loss-free variable every
 * linear and nonlinear step is unitary) while pulling the cotangent back
 * through each step (linear: conj(H); nonlinear: g e^{-i phi} +
 * 2 s coef x, s = -Im sum conj(g) y; amplifier: sqrt(G)).  Pullback formulas:
 * chain rule in Wirtinger calculus for y = x exp(i coef sum|x|^2).
 * Kept spans: with a state budget set (ssfm_plan_set_state_memory), the
 * forward pass also stores the input x of every nonlinear step of the last
 * K spans (K = the number of whole spans of steps_per_span * chunk * n_pol *
 * n_samples * 8 bytes that the budget holds, at most n_spans), rounded to
 * complex64; the reverse sweep of those spans carries the cotangent alone
 * and takes x from the store (y = x e^{i phi}, phi = coef sum|x|^2).  The
 * result differs from the reconstructing sweep by rounding only.
 * LDS-resident path (n_samples <= 2^13): one launch, one workgroup per
 * realisation: a forward pass keeps every span's input, then each span, from
 * the last, is recomputed from its input (the forward's arithmetic), keeping
 * the input x of each nonlinear step, and the cotangent is pulled back
 * through it (amplifier, then per step the linear step's adjoint and the
 * nonlinear pullback with x); the state budget does not apply.
 * Chunks: on the four-step path a batch above half the plan's
 * chunk_realisations (ssfm_plan_info) runs as equal chunks of two-field
 * working sets.  Without kept spans, the forward pass runs first over the
 * whole batch (in the forward's chunks), keeping every realisation's span
 * checkpoints, then the reverse sweep runs chunk by chunk; the bits are
 * those of one pass over the batch; every chunk of either phase runs as
 * one or more concurrent parts (ssfm_plan_set_forward_streams), each on its
 * share of the chunk's workspace.  With a state budget each chunk's whole
 * adjoint runs on the workspace of one chunk, the budget applied per chunk
 * (so a chunk may keep more spans than a whole-batch pass would).
 * Workspace: four-step path n_spans * batch * n_pol * n_samples * 8 bytes
 * of checkpoints (n_spans * chunk * ... with a state budget) and a work
 * buffer of two chunks' fields, plus the kept spans' states
 * (steps_per_span * chunk * n_pol * n_samples * 8 bytes per span);
 * LDS-resident path (n_spans + steps_per_span) * batch * n_pol * n_samples *
 * 8 bytes; allocated on first
 * use (and grown) and owned by the plan; if the device refuses the states'
 * allocation, fewer spans are kept.
 * Calls on one plan are serialised, since they share that workspace: on the
 * host by a lock, and on the device by an event, so each call's work starts
 * after the previous call's work has finished, whatever stream each runs on
 * (concurrent calls on several streams give the results of consecutive
 * ones).  Growing the workspace waits for the previous call to finish.
 * Asynchronous like ssfm_forward.  Errors: SSFM_EINVAL (NULL/misaligned
 * pointers, batch < 1), SSFM_EUNSUPPORTED for an FP32-arithmetic plan,
 * SSFM_ENOMEM, SSFM_EHIP. */
int ssfm_adjoint(ssfm_plan_t plan, const void* field_in, void* grad,
                 int64_t batch, uint64_t seed, void* stream);

/* ssfm_adjoint for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments and result as ssfm_adjoint, computed by the same kernels in
 * the same order (span checkpoints, every span rebuilt: no kept states, and
 * one stream whatever ssfm_plan_set_forward_streams says), but the work
 * fields and checkpoints live in a device scratch array of the library
 * (128 MiB per device, held by every device that loads the library until the
 * process ends; its address is resolved per device by ssfm_plan).  The call
 * makes no hipMalloc/hipFree and creates no stream or event.
 *   Limit: the workspace of ssfm_adjoint without kept states must fit in
 *   128 MiB: (n_spans + 2) * batch * n_pol * n_samples * 8 bytes on the
 *   four-step path (e.g. batch <= 10 for 2^16 samples x 2 pol x 10 spans),
 *   (n_spans + steps_per_span) * batch * n_pol * n_samples * 8 bytes on the
 *   LDS-resident path; larger calls return SSFM_EINVAL before any device
 *   work.
 * Every call on a device shares that device's one scratch array, whatever
 * the plan: calls that overlap on one device (two streams, two threads, two
 * plans) race and give wrong results; the caller must order them.  Nothing
 * in the scratch needs to start at zero (each call writes what it reads).
 * Errors: those of ssfm_adjoint, SSFM_EINVAL also for the size limit and
 * while a profiling window is open on the plan, SSFM_EHIP if the scratch
 * address could not be resolved. */
int ssfm_adjoint_noalloc(ssfm_plan_t plan, const void* field_in, void* grad,
                         int64_t batch, uint64_t seed, void* stream);

/* Concurrent parts of a four-step call (n_samples >= 2^14).  ssfm_forward,
 * ssfm_forward_spans and ssfm_adjoint run a large batch as sequential chunks
 * (ssfm_plan_info.chunk_realisations); each chunk may run as consecutive
 * parts of nearly equal size, the first on the caller's stream and the
 * others on worker streams of the device (created on first use, shared with
 * ssfm_batch, default priority) forked from the caller's stream and joined
 * back into it with events, so the call stays ordered on that stream.  Parts
 * on separate streams fill the tail of each pass with the other parts' work.
 *   0      the library's choice (the default): two parts when each still
 *          holds at least 256 column tiles (batch * n2 / 8 >= 512, e.g.
 *          >= 16 realisations of 2^16 samples), else one;
 *   1..5   that many parts (at most one per realisation).
 * Realisation b keeps its noise key and every part runs the same per-tile
 * arithmetic, so results are the same bit for bit whatever the setting.
 * Whether parts are faster depends on the streams reaching the GPU through
 * different hardware queues, which the process's stream creation order
 * decides.  A call with two or more parts does not use graph replay.
 * SSFM_FORWARD_STREAMS (0..5) in the environment at plan creation sets a
 * plan's initial setting.  Not to be changed while a call on the plan runs.  Errors: SSFM_EINVAL (NULL plan,
 * streams outside 0..5). */
int ssfm_plan_set_forward_streams(ssfm_plan_t plan, int32_t streams);

/* Device memory, in bytes, that ssfm_adjoint may hold for the kept spans'
 * nonlinear-step inputs (see ssfm_adjoint); 0 (the default) keeps none.
 * Trading memory for the reverse sweep's work: a kept span's reverse sweep
 * moves one field per pass instead of two.  The store is allocated by the
 * next ssfm_adjoint call that needs it and released by ssfm_plan_destroy,
 * or here when it exceeds the new budget (after the work using it is done).
 * Errors: SSFM_EINVAL (NULL plan), SSFM_EHIP. */
int ssfm_plan_set_state_memory(ssfm_plan_t plan, uint64_t bytes);

/* Independent realisations of different links in one call: entry i (of
 * `count`) propagates the device field fields[i] (complex64
 * [links[i].n_pol][links[i].n_samples], in place) through links[i] with
 * noise key (seeds[i], span) -- the key ssfm_forward uses for seed seeds[i]
 * and realisation 0.  Lengths, span counts, launch powers (the fields'
 * content) and seeds may all differ.  Entries whose links agree in
 * everything but the span count are propagated together: gathered into one
 * stream-ordered staging buffer, most spans first, and run over span
 * segments on the shrinking prefix of entries still propagating; plans are
 * built on first use and cached for the life of the process.  Such groups
 * run concurrently on up to four worker streams of the device (created on
 * first use, kept for the life of the process), forked from `stream` and
 * joined back into it with events.  links, fields and seeds are host
 * arrays; the call is asynchronous on `stream` of device `hip_device`.  Errors: SSFM_EINVAL (invalid link, NULL or misaligned
 * pointer, count < 1), SSFM_ENOMEM, SSFM_EHIP. */
int ssfm_batch(const ssfm_link* links, void* const* fields, int64_t count,
               const uint64_t* seeds, int hip_device, void* stream);

/* Result of ssfm_plan_autotune. */
typedef struct ssfm_tune_info {
  int32_t columns;        /* chosen column-tile width (0: nothing to tune)    */
  int32_t row_lanes;      /* chosen row-pass workgroup size (0: likewise)     */
  int32_t candidates;     /* timed variants: entries of us_per_step           */
  int32_t reserved;
  double us_per_step[4];  /* one split step per variant, in the order
                             (narrow columns, narrow rows), (narrow, wide),
                             (wide, narrow), (wide, wide); microseconds       */
} ssfm_tune_info;

/* Choose the launch shape of the four-step path for `batch` realisations by
 * measurement: each combination of column tile (narrow: 2 columns; wide: 8)
 * and row workgroup (narrow: 64 lanes; wide: 256) runs a
 * few split steps (row pass + nonlinear column pass) on a scratch field on
 * `stream`, timed with HIP events, and the fastest is recorded in the plan
 * for this batch size.  Later forward calls with this batch use it (the
 * SSFM_COLUMNS environment override still takes precedence).  The variants
 * compute every transform with the same FP64 arithmetic, so results do not
 * depend on the choice, bit for bit.  Synchronises `stream`; allocates and
 * frees a batch-sized scratch field; not to be called while another call on
 * the plan runs.  On the LDS-resident path (n_samples <= 8192) there is
 * nothing to tune: *info reports zeros.  Errors: SSFM_EINVAL (NULL plan or
 * info, batch < 1), SSFM_ENOMEM, SSFM_EHIP. */
int ssfm_plan_autotune(ssfm_plan_t plan, int64_t batch, void* stream, ssfm_tune_info* info);

/* Per-kernel timing, for reporting achieved bandwidth.  Between
 * ssfm_profile_begin and ssfm_profile_end every kernel launch of this plan
 * is bracketed by two HIP events recorded on the launch's own stream; the
 * GPU time between them is summed per kernel family.  Not thread-safe: one
 * profiling window per plan at a time. */
typedef struct ssfm_kernel_stats {
  char name[24];      /* "k1_lds", "k2_rows" or "k3_cols"                    */
  int64_t launches;   /* launches recorded in the window                     */
  double total_ms;    /* sum of per-launch GPU durations                     */
  double field_bytes; /* algorithmic HBM bytes: field read + write, summed   */
} ssfm_kernel_stats;

/* Start recording (clears earlier records).  SSFM_EINVAL on NULL plan. */
int ssfm_profile_begin(ssfm_plan_t plan);

/* Wait for the recorded events, stop recording and write up to `capacity`
 * entries (one per kernel family that ran) to `out`; *count receives the
 * number written.  SSFM_EINVAL on NULL arguments, SSFM_EHIP on event errors. */
int ssfm_profile_end(ssfm_plan_t plan, ssfm_kernel_stats* out, int capacity, int* count);

/* Measurement utility (not part of the propagation): copy `bytes` (a
 * multiple of 16) from device buffer src to dst on `stream` with a plain
 * 16-byte-per-lane grid-stride kernel -- the achievable HBM bandwidth the
 * propagation kernels are compared with.  Asynchronous.  SSFM_EINVAL for
 * NULL or 16-byte-misaligned pointers or a size not a multiple of 16,
 * SSFM_EHIP on a launch failure. */
int ssfm_stream_copy(void* dst, const void* src, int64_t bytes, void* stream);

/* Radix-16 DFT stage on the FP64 matrix cores against the FP64 vector
 * butterfly of the FFT passes: the measured prototype of the "DFT as a
 * matrix product" alternative (a radix-16 DFT is the product of the 16 x 16
 * DFT matrix with the transform's values; Cooley and Tukey's 4 x 4 split is
 * the butterfly).  `data` (device, 16-byte aligned) holds `count` transforms
 * of 16 complex FP64 values, [count][16] interleaved (re, im); each is
 * replaced in place by (F / 4)^rounds x with F[k][n] = exp(-2 pi i n k / 16),
 * the values passing through LDS between rounds as between FFT passes.
 * method 0: one transform per lane, the FFTs' butterfly on the vector
 * units; method 1: 16 transforms per wave as real 16 x 32 by 32 x 16
 * products on v_mfma_f64_16x16x4.  Not used by the propagation path.
 * Asynchronous on `stream`.  Errors: SSFM_EINVAL (method not 0/1, NULL or
 * misaligned data, count not a non-negative multiple of 64, rounds outside
 * [0, 2^20]), SSFM_EHIP. */
int ssfm_dft16_rounds(int method, void* data, int64_t count, int rounds, void* stream);

/* Measurement utility (not part of the propagation): the cost of one
 * ordering point between dependent passes of a split-step call, as the
 * four-step path could order them.  method 0: a captured graph of `rounds`
 * dependent launches of an empty kernel of `workgroups` workgroups (256
 * lanes), replayed (how repeated calls run); 1: the same launches issued
 * directly on `stream`; 2: one cooperative kernel of `workgroups` resident
 * workgroups crossing `rounds` device-wide barriers (an atomic arrival
 * counter and generation word, bounded polling) -- the persistent
 * alternative.  *us_per_round receives the GPU time per launch or barrier
 * (HIP events on `stream`).  Synchronous: waits for the work.  Errors:
 * SSFM_EINVAL (NULL us_per_round, method not 0..2, rounds outside
 * [1, 65536], workgroups outside [1, 65536], or for method 2 above the
 * device's resident capacity), SSFM_ENOMEM, SSFM_EHIP (including a barrier
 * wait that ran out). */
int ssfm_orchestration_probe(int method, int32_t workgroups, int32_t rounds, void* stream,
                             double* us_per_round);

/* Static description of a status code (never NULL). */
const char* ssfm_status_string(int status);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* ssfm_last_error(void);

/* ABI version: major * 10000 + minor * 100 + patch. */
int ssfm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SSFM_H_ */
