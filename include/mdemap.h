/*
 * mdemap -- bit-wise soft demapping of labelled multidimensional constellations
 * over AWGN on AMD Instinct MI355X (gfx950).  C ABI.
 *
 * What is computed.  The paper's GPU receiver (section "Experimental setup",
 * DSP-chain paragraph) ends by demapping the equaliser's decisions; its acronym
 * glossary names LLR, GMI, AIR, AWGN, BICM and BRGC but the text defines none of
 * them.  The library computes their standard bit-interleaved-coded-modulation
 * definitions with uniform priors.  For a constellation X (M x D, M = 2^m) with a
 * bijective labelling l_j, received symbols y_n and noise variance sigma2 per
 * real dimension:
 *
 *   q_nj  = -||y_n - x_j||^2 / (2 sigma2)
 *   L_nk  = ln sum_{j: b_k(l_j)=0} e^{q_nj} - ln sum_{j: b_k(l_j)=1} e^{q_nj}
 *           b_k(l) = (l >> (m-1-k)) & 1: column k of the LLR row is label bit
 *           m-1-k (most significant bit first); the sign is ln P(b=0)/P(b=1)
 *   GMI   = m - (1/N) sum_n sum_k log2(1 + e^{-s_nk L_nk}),  s_nk = +1 if the
 *           transmitted label's bit k is 0, else -1     [bits per D-dim symbol]
 *
 * Conventions for every call
 *   - Pointers named d_* are DEVICE memory owned by the caller; the library never
 *     frees them.  Arrays are dense and row-major.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Every call only enqueues work on that stream and returns; results are ready
 *     when the stream has reached them.
 *   - Arguments are checked on the host before anything is enqueued; a negative
 *     status is returned and last_error() describes it.  No call throws.
 *   - The library keeps an internal device workspace per (device, stream) that it
 *     grows on demand and frees in release_cache().  Calls on one stream are
 *     ordered; calls that overlap on different streams use different workspaces.
 *   - Labels are checked to be a permutation of [0, M): on the host the first time
 *     a given label buffer (device, address, M) is seen (a synchronous copy, skipped
 *     while the stream is being captured into a graph), and on the device in every
 *     call (an invalid label set turns every output of that call into NaN).  Labels
 *     rewritten in place at an address already checked are caught by the device check
 *     only; release_cache() forgets the checked addresses.
 *   - Limits: 2 <= M <= 65536 and a power of two; 1 <= D <= 30; N >= 0, and
 *     N <= 2^31 - 1 symbols per llr_exact / llr_maxlog call.
 */
#ifndef MDEMAP_H
#define MDEMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define MD_OK            0
#define MD_EINVAL       -1   /* bad argument (null pointer, N < 0, sigma2 <= 0 ...) */
#define MD_ENOTPOW2     -2   /* M is not a power of two in [2, 65536] */
#define MD_ELABEL       -3   /* labels are not a permutation of [0, M) */
#define MD_EDIM         -4   /* D outside [1, 30] or a shape mismatch */
#define MD_ENOMEM       -5   /* device workspace allocation failed */
#define MD_EHIP         -6   /* a HIP runtime call failed (message in last_error) */
#define MD_ENODEV       -7   /* no GPU visible */
#define MD_EUNSUPPORTED -8   /* combination not implemented */
#define MD_ENONFINITE   -9   /* gmi_status: the last GMI saw non-finite loss terms */

/* Precision of llr_exact.
 *   MD_PREC_FP32: scores by one split-FP16 MFMA contraction whose K dimension holds
 *     the hi*hi, hi*lo and lo*hi partial products side by side (3D+4 slots, FP32
 *     accumulation, error about 2^-21 of sum_k |a_k b_k|); exponentials and all
 *     subset sums in FP32.
 *   MD_PREC_BF16: same scores; the exponentials are rounded to BF16 and the
 *     subset sums are formed by a BF16 MFMA contraction against the label-bit
 *     matrix with FP32 accumulation (LLR relative error about 2^-8).
 *   MD_PREC_FP16: reduced-precision scores -- one unsplit FP16 MFMA pass whose K
 *     dimension holds [a x (D), p_hi, p_lo, a, a] against [(2c/a) y (D), a, a, r_hi,
 *     r_lo] (D + 4 slots, so D <= 12; the per-point and per-symbol biases keep a hi/lo
 *     split), FP32 accumulation: every score carries an error of at most about
 *     2^-10 sum_k |u_k w_k| base-2 units (u = a x, w = (2c/a) y), so each LLR moves by at
 *     most 2 ln 2 times that; half the matrix work of MD_PREC_FP32.  Exponentials and
 *     subset sums in FP32 after the same fixed exponent shift (no running maximum is
 *     needed: every score is measured from -c ||y||^2).  Symbols whose sums leave the
 *     FP32 range are evaluated by the FP64 kernel.
 *   MD_PREC_BF16_SCORES: the same one-pass layout with BF16 operands (score error about
 *     2^-8 sum_k |u_k w_k|).
 * The reduced-precision variants are measured against the FP64 oracle, not pinned. */
#define MD_PREC_FP32 0
#define MD_PREC_FP16 1
#define MD_PREC_BF16 2
#define MD_PREC_BF16_SCORES 3

/* ------------------------------------------------------------------ channel */
/* awgn_sample -- draws N channel uses: a uniform transmitted index u_n in [0, M)
 * and y_n = fl32(x_{u_n} + sigma z_n), z_n ~ N(0, I_D).  The AWGN of the paper's
 * glossary; the generator is fixed bit for bit by this definition, so that any
 * (seed, offset) window is reproducible on any launch geometry and on the CPU:
 *
 *   key = (seed & 0xffffffff, seed >> 32); g = offset + n (64-bit);
 *   Philox4x32-10 (Salmon et al., SC'11) of counter (g_lo, g_hi, j, 1), j = 0, 1, ...,
 *   gives channel use n one stream of words: word 4j + i is output word i of block j.
 *   u_n = word 0 >> (32 - m).
 *   Pair p = 0 .. ceil(D/2)-1 takes the radius word a = word 2p+1 and the angle word
 *   b = word 2p+2 (so 8D draws three blocks, 2D one), in IEEE single precision (every
 *   operation correctly rounded, fma where written):
 *     v = (float)(a | 1) (round to nearest even), U1 = v 2^-32 in [2^-32, 1];
 *     v = f 2^E with f in [1, 2) from its bits, k = E - 32;
 *     if f > SQRT2 (0x1.6a09e6p+0): f = f/2, k = k + 1;
 *     s = (f-1)/(f+1), w = s*s, P = Horner in w of 1/(2i+1), i = 5..0 (fmaf),
 *     ln U1 = fmaf(k, LN2_HI, fmaf(k, LN2_LO, (2s) P)) with LN2_HI = 0x1.62e300p-1,
 *       LN2_LO = 0x1.2fefa2p-17;
 *     R = sqrtf(-2 ln U1);
 *     quadrant Q = b >> 30, T = (b >> 7) mod 2^23 (the angle is
 *       2 pi (Q + (2T+1) 2^-24) / 4);
 *     if T < 2^22: phi = ((2T+1) 2^-24) * PIO2 gives (cos, sin) = (C, S)
 *       else phi' from T' = 2^23 - 1 - T gives (cos, sin) = (S', C'),
 *       with PIO2 = 0x1.921fb6p+0, w = phi^2,
 *       S = phi * Horner_w(+-1/(2i+1)!, i = 5..0), C = Horner_w(+-1/(2i)!, i = 6..0)
 *       (each coefficient the float nearest 1/n!);
 *     rotate by Q quarter turns: (c, s) -> (c, s), (-s, c), (-c, -s), (s, -c);
 *     z_{2p} = R c, z_{2p+1} = R s (the latter dropped when 2p+1 = D);
 *   y_nd = (float) fma(sigma, (double) z_d, (double) X[u_n][d])   (IEEE double fma).
 * Round-to-nearest throughout, no contraction beyond the fmas written above.
 *
 *   d_X    M x D float32 constellation (row u is point u; labels are not used)
 *   sigma  noise standard deviation per real dimension, sigma >= 0 (host FP64)
 *   d_tx   out: N uint32 transmitted point indices (rows of X)
 *   d_y    out: N x D float32 received symbols
 * Returns MD_OK (N = 0 enqueues nothing), MD_EINVAL, MD_ENOTPOW2, MD_EDIM, MD_EHIP. */
int awgn_sample(const float* d_X, int M, int D, uint64_t seed, uint64_t offset, int64_t N,
                double sigma, uint32_t* d_tx, float* d_y, void* stream);

/* ------------------------------------------------------------------ demappers */
/* llr_exact -- exact bit-wise LLRs L_nk above (log-sum-exp over the label-0 and
 * label-1 subsets of every bit).
 *   d_X       M x D float32 constellation
 *   d_labels  M uint32, a permutation of [0, M); l_j is the label of point j
 *   d_y       N x D float32 received symbols
 *   sigma2    noise variance per real dimension (> 0, finite)
 *   prec      MD_PREC_FP32, MD_PREC_FP16, MD_PREC_BF16 or MD_PREC_BF16_SCORES (FP16 and
 *             BF16_SCORES take D <= 12, else MD_EUNSUPPORTED)
 *   d_llr     out: N x m float32
 * Symbols whose subset sums leave the FP32 range in the first pass (a subset's best
 * point more than 196 base-2 units below the bias; high SNR) are evaluated again in
 * two exponent windows (down to 386 units), what those miss in three (576 units), and
 * what is still left by a per-subset-maximum FP64 evaluation, so every finite input
 * gives finite LLRs (llr_path_counts reports how many symbols took each stage).
 * Returns MD_OK (N = 0 enqueues nothing), MD_EINVAL, MD_ENOTPOW2, MD_ELABEL,
 * MD_EDIM, MD_ENOMEM, MD_EHIP. */
int llr_exact(const float* d_X, const uint32_t* d_labels, int M, int D, const float* d_y,
              int64_t N, double sigma2, int prec, float* d_llr, void* stream);

/* llr_exact_noalloc -- llr_exact for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, layout, results (bit for bit) and errors as llr_exact, but it calls no
 * hipMalloc, hipFree or allocating routine: its prep buffers, stage counters and
 * fallback lists live in a 24 MiB file-scope device array, one copy per device, held
 * until the process ends.  Limits: N <= 2^20 symbols per call and at most 24 MiB of
 * prep data (every M and D above fit at that N); beyond them MD_EINVAL, before anything
 * is enqueued.  All calls on one device share its array and each call's prep kernels
 * clear the counters it needs, so calls that overlap on one device (other streams,
 * other threads) race: serialise them.  llr_path_counts does not report these calls.
 * The first call on a device looks up the array's device address (no allocation). */
int llr_exact_noalloc(const float* d_X, const uint32_t* d_labels, int M, int D, const float* d_y,
                      int64_t N, double sigma2, int prec, float* d_llr, void* stream);

/* llr_maxlog -- max-log LLRs: L_nk = max_{b_k=0} q_nj - max_{b_k=1} q_nj.  Same
 * arguments, layout and errors as llr_exact (no precision argument). */
int llr_maxlog(const float* d_X, const uint32_t* d_labels, int M, int D, const float* d_y,
               int64_t N, double sigma2, float* d_llr, void* stream);

/* llr_path_counts -- waits for `stream` and reports, for the last llr_exact or
 * llr_maxlog call enqueued on it from this process, how many symbols the wide-range
 * passes took (*n_wide, the symbols entering the two-window pass; exact only) and how
 * many the FP64 careful kernel took (*n_careful).  Constellations of M <= 16 points take a one-thread-per-symbol kernel and
 * report 0 and 0.  Both are 0 if no call was made on the stream since the last
 * release_cache.  Returns MD_OK, MD_EINVAL, MD_EHIP. */
int llr_path_counts(void* stream, int64_t* n_wide, int64_t* n_careful);

/* ------------------------------------------------------------------ metric */
/* gmi_reduce -- Monte-Carlo GMI (the glossary's generalised mutual information,
 * an achievable information rate of BICM) of N LLR rows against the transmitted
 * labels: T_n = sum_k log2(1 + e^{-s_nk L_nk}) in FP32 per symbol, compensated
 * FP32 partial sums, FP64 final sums in a fixed order (deterministic).
 *   d_llr          N x m float32
 *   d_tx           N uint32 transmitted point indices
 *   d_labels       M = 2^m uint32 labels (d_labels[d_tx[n]] is the sent label)
 *   d_gmi          out: 1 double, bits per D-dimensional symbol
 *   d_gmi_per_bit  out: m doubles (1 - mean loss of column k) or NULL
 *   d_se           out: 1 double, std(T_n)/sqrt(N), or NULL
 * N = 0 is MD_EINVAL (the GMI of an empty sample is undefined).  Non-finite LLRs
 * (or a transmitted index outside [0, M)) give a NaN GMI, and the call records on
 * the device how many symbols had a non-finite loss term: gmi_status reads it. */
int gmi_reduce(const float* d_llr, int64_t N, int m, const uint32_t* d_tx,
               const uint32_t* d_labels, double* d_gmi, double* d_gmi_per_bit, double* d_se,
               void* stream);

/* gmi_status -- waits for `stream` and reports how many symbols had a non-finite loss
 * term in the last gmi_reduce or llr_exact_gmi enqueued on it (0 if none was made):
 * MD_OK when there were none, MD_ENONFINITE (with the count in *n_nonfinite and
 * last_error) otherwise.  The asynchronous calls cannot return this status themselves. */
int gmi_status(void* stream, int64_t* n_nonfinite);

/* llr_exact_gmi -- llr_exact and gmi_reduce in one pass: the exact LLRs are written to
 * d_llr as by llr_exact, and the fast kernel's epilogue forms each finished symbol's loss
 * term T_n = sum_k log2((S0_k + S1_k) / S_sent,k) from the subset sums it already holds,
 * so no separate pass reads the LLRs back; the symbols that the later (wide-range or
 * FP64) passes finish take their term from their final LLRs in the reduction.  The GMI
 * equals gmi_reduce's of the same LLRs up to FP32 rounding of the terms; the reduction is
 * deterministic (fixed order); S0_k + S1_k is the total over all points for every k, so
 * the epilogue takes one logarithm of it.  Arguments as llr_exact, plus d_tx (N transmitted
 * indices), d_gmi (1 double out) and d_se (1 double out, or NULL); no per-bit GMI.
 * M <= 16, MD_PREC_BF16 and D > 9 (FP32 scores) run the two calls in sequence.
 * N = 0 is MD_EINVAL.
 * Workspace: llr_exact's plus 4 N bytes.  Returns as llr_exact. */
int llr_exact_gmi(const float* d_X, const uint32_t* d_labels, int M, int D, const float* d_y, int64_t N,
                  double sigma2, int prec, const uint32_t* d_tx, float* d_llr, double* d_gmi, double* d_se,
                  void* stream);

/* ber_count -- hard decisions and bit errors (the paper's receiver decides hard and
 * reports the Q-factor of the measured bit-error rate, see its Results section): the
 * decided bit of LLR column k is 1 where L_nk < 0 and 0 otherwise (for max-log LLRs
 * this is the label of the nearest point, the ML symbol decision; for exact LLRs the
 * bit-wise MAP decision), counted against the sent label's bit m-1-k.  Integer sums,
 * deterministic.
 *   d_llr          N x m float32
 *   d_tx           N uint32 transmitted point indices; d_labels M = 2^m uint32
 *   d_bit_errors   out: m uint64, errors of column k, or NULL
 *   d_errors       out: 1 uint64, all bit errors (BER = errors / (N m))
 * Returns MD_OK, MD_EINVAL (N <= 0, m outside [1, 16], NULL pointer), MD_EHIP. */
int ber_count(const float* d_llr, int64_t N, int m, const uint32_t* d_tx, const uint32_t* d_labels,
              uint64_t* d_bit_errors, uint64_t* d_errors, void* stream);

/* q_factor_db -- the Q-factor the paper reports for its measured bit-error rates (Results
 * section: Q computed from the BER; the paper does not print the relation), by the
 * Gaussian-tail relation BER = erfc(Q / sqrt 2) / 2:
 *   BER = errors / n_bits,  *d_q_db = 20 log10( sqrt2 erfcinv(2 BER) )
 * evaluated in FP64 on the device.  NaN when BER = 0 or BER >= 1/2 (no finite Q).
 *   d_errors  1 uint64 bit-error count (device; ber_count's d_errors output)
 *   n_bits    number of bits the count is over (> 0), e.g. N m
 *   d_q_db    out: 1 double (device)
 * Returns MD_OK, MD_EINVAL (n_bits <= 0, NULL pointer), MD_EHIP. */
int q_factor_db(const uint64_t* d_errors, int64_t n_bits, double* d_q_db, void* stream);

/* ------------------------------------------------------------------ learned demapper */
/* A small network f: R^D -> R^m approximating the exact LLRs, trained on the GPU by the
 * library's own kernels on (y, exact-LLR) pairs that llr_exact produces; the exact path
 * stays the reference its GMI is measured against (through gmi_reduce).  The glossary's ML entry is
 * the only mention of learning in the paper; the network and its training are this
 * library's design:
 *   f(y) = s_out (W3 g(W2 g(W1 (s_in y) + b1) + b2) + b3),  hidden width H in both
 *          layers, fixed scales s_in, s_out (default 1; mlp_set_scales),
 *   g(a) = a Phi(a), Phi the standard normal distribution function (GELU; the kernels
 *          evaluate Phi by Abramowitz & Stegun 7.1.26, absolute error below 3e-7 in FP32),
 *   loss = mean_b sum_k p_bk softplus(-f_bk) + (1 - p_bk) softplus(f_bk),
 *          p_bk = sigmoid(L_target_bk)   (distillation of the exact bit posteriors),
 *   Adam (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights.
 * Every product runs as a BF16 MFMA with FP32 accumulation.  Parameters form one FP32
 * vector in the order W1 (H x D), b1 (H), W2 (H x H), b2 (H), W3 (m x H), b3 (m), row-major
 * [out][in]; initial values are uniform in +-1/sqrt(fan_in) from Philox4x32-10 (key =
 * seed, counter = (index_lo, index_hi, 0, 3)).  A handle is bound to the device that was
 * current at mlp_create and must be used on that device.  Handles are not thread-safe. */

/* Creates a network (1 <= D <= 30, 1 <= hidden <= 4096, 1 <= m <= 16).  *out receives the
 * handle; release it with mlp_destroy. */
int mlp_create(int D, int hidden, int m, uint64_t seed, void** out);
int mlp_destroy(void* mlp);
/* Number of parameters P, or -1 for a NULL handle. */
int64_t mlp_num_params(const void* mlp);
int mlp_info(const void* mlp, int* D, int* hidden, int* m, int64_t* step);
/* Fixed input and output scales s_in, s_out of f (finite, > 0; not trained; saved in
 * checkpoints).  For a demapper at noise variance sigma2, s_in = s_out = 1/sqrt(sigma2)
 * puts the inputs and the LLRs on the scale of the noise.  Returns MD_OK or MD_EINVAL. */
int mlp_set_scales(void* mlp, float in_scale, float out_scale);
int mlp_get_scales(const void* mlp, float* in_scale, float* out_scale);
/* Copies P floats between host memory and the handle (synchronises the device).
 * which: 0 parameters, 1 last gradient, 2 Adam first moment, 3 Adam second moment. */
int mlp_get(const void* mlp, int which, float* h_out);
int mlp_set(void* mlp, int which, const float* h_in);
/* Forward + backward on a batch: d_y B x D, d_target B x m (exact LLRs); gradients are
 * kept in the handle, the mean loss goes to d_loss (1 double, device) unless NULL. */
int mlp_grad(void* mlp, const float* d_y, const float* d_target, int64_t B, double* d_loss, void* stream);
/* One Adam update with the last gradient. */
int mlp_adam_step(void* mlp, float lr, void* stream);
/* mlp_grad followed by mlp_adam_step. */
int mlp_train_step(void* mlp, const float* d_y, const float* d_target, int64_t B, float lr, double* d_loss,
                   void* stream);
/* `steps` training steps on batches of B rows drawn with replacement from the N pairs
 * (a hash of (shuffle_seed, step, row) picks the rows), learning rate on a cosine
 * schedule from lr_max to lr_min; d_loss_trace receives `steps` doubles or is NULL.
 * Allocates its batch buffers and returns after the stream has drained. */
int mlp_fit(void* mlp, const float* d_y, const float* d_target, int64_t N, int64_t steps, int64_t B,
            float lr_max, float lr_min, uint64_t shuffle_seed, double* d_loss_trace, void* stream);
/* llr_learned -- network LLRs for N symbols: d_y N x D float32 -> d_llr N x m float32,
 * same column order and sign as llr_exact.  N = 0 enqueues nothing. */
int llr_learned(const void* mlp, const float* d_y, int64_t N, float* d_llr, void* stream);
/* Checkpoint: parameters, Adam moments and step count, with a CRC-32 over the data.
 * mlp_load creates a new handle on the current device; a corrupt file is MD_EINVAL. */
int mlp_save(const void* mlp, const char* path);
int mlp_load(const char* path, void** out);

/* ------------------------------------------------------------------ batched sweep */
/* Many constellations (uneven M and D) at many noise levels in one captured hipGraph of
 * persistent kernels, one per constellation class (K steps, label bits), each claiming
 * its work items dynamically: for every (instance i, noise level s) the channel of
 * awgn_sample (seed_i, offset = s * N_i, N_i uses), the exact LLRs and their GMI, without
 * storing received symbols or LLRs.  The GMI equals gmi_reduce(llr_exact(...)) of the
 * same channel draw up to FP32 rounding.  Every class has its own launch shape
 * (wavefronts per block, 32-symbol blocks per wavefront, symbol groups per work item):
 * 0 (8, 2, 1), 1 (8, 2, 4), 2 (16, 1, 1), 3 (16, 1, 4) for the matrix-core kernel, and
 * for classes with M <= 64 also 4, a vector kernel with one thread per symbol (scores
 * from coordinate differences at M = 16 and from the per-point terms of prep at M = 32
 * and 64; each wavefront claims work items of 512 symbols; reported
 * as (4, 1, 4)).  variant 0..3 fixes one shape for all classes, variant 4 gives the classes
 * with M <= 64 the vector kernel and the others shape 0; variant = -1 autotunes: the plan
 * is run once under each shape with its
 * class kernels timed by events, and each class keeps the shape its kernel ran fastest
 * under; the choices are cached per (device, K steps, label bits) for the process, so a
 * later plan whose classes are all known is built without measuring (sweep_tuning_clear
 * forgets them).  The plan snapshots the constellations' fragments at creation; d_X and
 * d_labels must stay valid and unchanged while the plan lives (the channel reads d_X).
 * Limits: M in {16 .. 8192}, 1 <= D <= 8, instances x noise levels <= 2^20; more than
 * 2^20 symbols of one run needing the FP64 fallback makes that run's GMIs NaN. */
typedef struct {
  const float* d_X;           /* M x D float32 constellation (device) */
  const uint32_t* d_labels;   /* M uint32 labels, a permutation of [0, M) (device) */
  int M, D;
  int64_t N;                  /* channel uses per noise level */
  uint64_t seed;              /* channel seed */
} md_sweep_instance;

/* sigma2: host array n_inst x n_snr (row i = instance i).  Synchronous. */
int sweep_plan_create(const md_sweep_instance* inst, int n_inst, const double* sigma2, int n_snr, int variant,
                      void** out);
/* The launch shape of the plan's first (most expensive) class and the number of work items. */
int sweep_plan_info(const void* plan, int* waves, int* blocks_per_wave, int* groups_per_item, int* n_items);
/* Class i of the plan (0 = most expensive): K steps, label bits, launch shape (0..4), work
 * items, and the kernel time the autotuner measured for the class under that shape (ms;
 * -1 when this plan measured nothing: fixed variant or cached choice); any output may be
 * NULL.  MD_EINVAL when i is not a class index (classes are numbered from 0). */
int sweep_plan_class(const void* plan, int i, int* k_steps, int* label_bits, int* shape, int* n_items,
                     float* tuned_ms);
/* Forgets the autotuner's cached shapes (every device). */
int sweep_tuning_clear(void);
/* Runs the sweep (use_graph = 1: one launch of the captured graph; 0: the same kernels
 * enqueued directly) and copies the n_inst x n_snr GMIs (bits per symbol) to d_gmi. */
int sweep_run(void* plan, double* d_gmi, int use_graph, void* stream);
/* After the last sweep_run on `stream` (the call waits for the stream): how many symbols
 * of that run were re-evaluated by the FP64 fallback (their subset sums left the FP32
 * range, or their operands the FP16 split range) and whether the fallback queue
 * overflowed (then the run's GMIs are NaN).  Either pointer may be NULL. */
int sweep_run_stats(const void* plan, int64_t* n_fallback, int* overflowed, void* stream);
int sweep_plan_destroy(void* plan);

/* ------------------------------------------------------------------ streaming receiver */
/* Continuous demapping of a host-resident symbol stream, after the paper's real-time
 * receiver (Experimental setup: ADC buffers moved to the GPU by DMA, several streams
 * working on different buffers in parallel, events for the dependencies between buffers;
 * Results: Q-factors from the BER in short bins over 20 s of continuous operation).
 *
 * The stream of `total` symbols is cut into buffers of buf_symbols symbols, which go
 * round-robin to n_streams HIP streams (default priority).  Per buffer, its stream copies
 * the received symbols (and the sent indices) from host to device, demaps them, counts
 * the bit errors and the GMI of each statistics bin the buffer touches, and copies the
 * decisions or the LLRs back to host memory.  Copies and kernels of different buffers
 * overlap; an event per buffer marks its end: before a stream takes a new buffer the host
 * waits for that stream's previous buffer (at most n_streams buffers in flight), and the
 * events give each buffer's latency from the start of its host-to-device copy to the end
 * of its device-to-host copy.
 *
 * Modes:
 *   MD_RX_HARD   max-log LLRs; the decision is the label whose bit m-1-k is 1 where
 *                column k is negative, i.e. the label of the nearest constellation point
 *                (the paper's receiver decides hard).  Output: total uint32 labels.
 *   MD_RX_EXACT  exact LLRs (llr_exact).  Output: total x m float32 LLRs.
 * Statistics per bin b (symbols [b bin_symbols, (b+1) bin_symbols) of the stream): bit
 * errors of the hard decisions (ber_count of the mode's LLRs) and the GMI of the mode's
 * LLRs (gmi_reduce), each bin's GMI combined from its buffers' pieces in stream order
 * (deterministic).  Bit errors equal ber_count over the bin; the GMI equals gmi_reduce
 * over the bin up to the FP64 rounding of combining the pieces.  A bin spans at least one
 * buffer (bin_symbols >= buf_symbols).
 *
 * The host arrays form a ring of N symbols (a looped capture): stream symbol i is
 * h_y[i mod N] / h_tx[i mod N], and its output goes to h_out[i mod N]; when total > N, N
 * must be a multiple of buf_symbols.  All host arrays must be pinned (hipHostMalloc, or
 * torch's pin_memory): pageable memory cannot overlap copies and is rejected. */
#define MD_RX_HARD  0
#define MD_RX_EXACT 1

typedef struct {
  int mode;               /* MD_RX_HARD or MD_RX_EXACT */
  int n_streams;          /* 1 .. 8 */
  int64_t buf_symbols;    /* symbols per buffer, 1 .. 2^24 */
  int64_t bin_symbols;    /* symbols per statistics bin, >= buf_symbols */
  int eq_instances;       /* 0: the ring holds received symbols; P > 0: equaliser stage below */
  double eq_mu;           /* equaliser step size (finite, >= 0) */
  double eq_h0[8];        /* starting taps h_j, g_j (re, im), shared by the P instances */
  double eq_g0[8];
} md_rx_config;

/* Equaliser stage (eq_instances = P > 0; D = 2, M <= 1024, the constellation's rows are also
 * the equaliser's reference points): the ring holds complex samples at two per symbol of P
 * parallel channels, TIME-MAJOR as in ddlms_equalize: h_y is (2 N/P + 2) rows of P complex
 * float32 (re, im), stream symbol i is symbol i / P of channel i mod P.  buf_symbols, N and
 * total must be multiples of P.  Each buffer (n = buf_symbols / P symbols per channel) is
 * copied in with its two overlapping samples, equalised by ddlms_equalize_chain on its lane
 * after an event from the previous buffer's equaliser (the taps are carried from buffer to
 * buffer, so the equaliser stages run in stream order while copies and demapping of other
 * buffers overlap them), and the equaliser outputs z are demapped in place of received
 * symbols.  The decisions, outputs and taps equal one ddlms_equalize call over the whole
 * stream; every rx_run starts from eq_h0, eq_g0.  When a ring is read more than once, the
 * equaliser continues across the wrap with the ring's first samples. */

/* Copies the constellation (M x D float32, device) and its labels (M uint32 permutation,
 * device) and allocates every device buffer of the pipeline (synchronous).  sigma2 is the
 * noise variance per real dimension that the LLRs assume. */
int rx_create(const float* d_X, const uint32_t* d_labels, int M, int D, double sigma2, const md_rx_config* cfg,
              void** out);
/* Runs `total` stream symbols through the pipeline and returns when all are done.
 *   h_y            N x D float32 received symbols (pinned host ring), or with the
 *                  equaliser stage (2 N/P + 2) x P complex float32 samples
 *   h_tx           N uint32 sent point indices (pinned host ring), or NULL: no statistics
 *   h_out          N uint32 decisions (MD_RX_HARD) or N x m float32 LLRs (MD_RX_EXACT)
 *                  (pinned host ring), or NULL: nothing copied back
 *   h_bin_errors   ceil(total / bin_symbols) uint64 bit errors per bin, or NULL
 *   h_bin_gmi      ceil(total / bin_symbols) doubles, GMI per bin (bits per symbol), or NULL
 *   h_stats        4 doubles, or NULL: wall seconds, symbols per second, mean and maximum
 *                  buffer latency in milliseconds
 * h_bin_errors and h_bin_gmi need h_tx.  Returns MD_OK, MD_EINVAL (NULL or unpinned
 * array, total < 0, N < 1, ring length not a multiple of buf_symbols, equaliser sizes not
 * multiples of P), MD_ENOMEM, MD_EHIP. */
int rx_run(void* rx, const float* h_y, const uint32_t* h_tx, int64_t N, int64_t total, void* h_out,
           uint64_t* h_bin_errors, double* h_bin_gmi, double* h_stats);
int rx_destroy(void* rx);

/* ------------------------------------------------------------------ equaliser */
/* ddlms_equalize -- four-tap widely-linear decision-directed LMS equaliser, the step
 * that feeds the demapper in the paper's receiver (section "Experimental setup": after
 * downsampling to 2 samples per symbol, a four-tap adaptive time-domain DD-LMS
 * widely-linear equaliser whose decisions are demapped; the paper gives no equations).
 * B independent instances (buffers, sub-blocks or channels) run side by side, one
 * sequential recursion each.  Per instance, complex samples u_t, t = 0 .. 2N+1; symbol n
 * sees the window w_j = u_{2n+j}, j = 0..3, and
 *   z_n = sum_j ( h_j w_j + g_j conj(w_j) )        (j ascending, the h term first)
 *   d_n = argmin_i |z_n - C_i|^2                   (the first minimum)
 *   e_n = C_{d_n} - z_n
 *   h_j <- h_j + mu e_n conj(w_j),  g_j <- g_j + mu e_n w_j     (with the old w_j)
 * in IEEE double with complex products (ac - bd) + i(ad + bc) and no contraction, so the
 * results are fixed bit for bit by this definition.
 *   d_x    (2N + 2) x B complex float32 samples, TIME-MAJOR: sample t of instance b at
 *          d_x[2 (t B + b)] (re) and d_x[2 (t B + b) + 1] (im)
 *   d_C    M complex float32 reference points (re, im), 1 <= M <= 1024 (pass the
 *          demapper's 2D constellation to feed llr_* or ber_count with the decisions)
 *   h_h0, h_g0  host, 8 doubles each: starting taps h_j, g_j (re, im), shared by all
 *          instances
 *   mu     step size, finite and >= 0
 *   d_dec  out: N x B uint32 decisions (indices into d_C), time-major (n B + b)
 *   d_z    out: N x B complex float32 equaliser outputs, time-major, or NULL
 *   d_h, d_g  out: B x 8 doubles, the final taps of each instance, or NULL
 * Returns MD_OK (B = 0 enqueues nothing; N = 0 only writes the starting taps), MD_EINVAL,
 * MD_EHIP. */
int ddlms_equalize(const float* d_x, int64_t B, int64_t N, const float* d_C, int M, const double* h_h0,
                   const double* h_g0, double mu, uint32_t* d_dec, float* d_z, double* d_h, double* d_g,
                   void* stream);
/* ddlms_equalize_chain -- the same recursion, continued across consecutive buffers of one
 * stream (the paper's receiver orders such dependent buffers with events): every instance
 * starts from its own taps in d_h, d_g (B x 8 doubles each, device, in/out) and leaves its
 * final taps there.  A call over samples [2S, 2S + 2N + 2) of each instance continues one
 * over [2S - 2N', 2S + 2) exactly (consecutive windows overlap by two samples): chained
 * calls give the decisions, outputs and taps of a single call over the whole window, bit
 * for bit.  The other arguments are those of ddlms_equalize; taps that are not finite
 * propagate.  Returns MD_OK (B = 0 enqueues nothing; N = 0 leaves the taps unchanged),
 * MD_EINVAL, MD_EHIP. */
int ddlms_equalize_chain(const float* d_x, int64_t B, int64_t N, const float* d_C, int M, double mu,
                         uint32_t* d_dec, float* d_z, double* d_h, double* d_g, void* stream);

/* ------------------------------------------------------------------ Kramers-Kronig front end */
/* kk_frontend -- the receiver's first step (section "Experimental setup": square root and
 * logarithm of the detected samples, the phase by a Hilbert transform with 1024-point
 * overlap-save FFTs, the optical field rebuilt from amplitude and phase and downshifted to
 * DC).  For real intensity samples x_t > 0, t < T:
 *   l_t   = 0.5 ln x_t
 *   phi   = Hilbert(l) in blocks: for output samples [512 k, 512 k + 512) the 1024 samples
 *           starting at 512 k - 256 (zero outside the stream) are transformed, multiplied
 *           by the analytic mask (1, 2 .. 2, 1, 0 .. 0), transformed back, and the
 *           imaginary parts of the middle 512 are the phases
 *   s_t   = (exp(l_t) e^{i phi_t} - A) e^{-i 2 pi frac(nu t)}
 * FP32 FFTs and transcendental functions; the downshift phase frac(nu t) in FP64.
 * A detected intensity is positive; a sample below 2^-126 (zero or negative after noise,
 * or NaN) is taken as 2^-126, the smallest normal float, so that one bad sample gives a
 * large negative log-amplitude instead of spreading NaN over the 1024-sample windows
 * around it.
 *   d_x    T float32 intensity samples (T a multiple of 512)
 *   A      carrier amplitude removed from the rebuilt field (finite, >= 0)
 *   nu     downshift frequency in cycles per sample (finite)
 *   d_out  out: T complex float32 samples (re, im)
 * Returns MD_OK (T = 0 enqueues nothing), MD_EINVAL, MD_EHIP. */
int kk_frontend(const float* d_x, int64_t T, float A, double nu, float* d_out, void* stream);

/* ------------------------------------------------------------------ peak calibration */
/* Measured rates of what the kernels above are bound by, on the current device: the
 * roofline denominators.  The datasheet gives no rate for the exponential unit, and code
 * built without packed FP32 instructions issues one FP32 add per lane per instruction,
 * so both are measured here, next to the matrix-core and copy rates.
 *
 * One warm-up and one timed kernel run on `stream`; the call waits for them (it is
 * synchronous) and writes the rate to *h_rate and the timed kernel's milliseconds to
 * *h_ms (either may be NULL).  The compute kernels run 8 blocks of 256 threads per
 * compute unit, each lane with 16 independent chains (or each wavefront with 4
 * independent accumulators), so that instruction issue, not latency, bounds them.
 * `work` is the number of loop iterations per lane for the compute kinds (0: a default
 * of a few milliseconds) and the number of bytes for the copy.
 *   MD_UB_EXP        v_exp_f32                                  -> exponentials/s
 *   MD_UB_ADD_F32    v_add_f32 (non-packed)                     -> adds/s
 *   MD_UB_MFMA_F16   v_mfma_f32_32x32x16_f16                    -> flop/s
 *   MD_UB_MFMA_BF16  v_mfma_f32_32x32x16_bf16                   -> flop/s
 *   MD_UB_MFMA_F32   v_mfma_f32_32x32x2_f32                     -> flop/s
 *   MD_UB_COPY       d_dst[i] = d_src[i] over `work` bytes with 16-byte loads and stores;
 *                    d_src and d_dst are device buffers of at least `work` bytes, 16-byte
 *                    aligned, not overlapping (ignored by the other kinds)
 *                                                               -> bytes read + written /s
 *   MD_UB_EXP_ADD2   one v_exp_f32 and two independent v_add_f32 of its result per step
 *                    (the exact demapper's work per (symbol, point) pair)
 *                                                               -> steps/s
 *   MD_UB_TILE_MIX   the exact demapper's whole per-tile instruction mix at two K steps
 *                    and 11 label bits, without memory traffic: two dependent
 *                    v_mfma_f32_32x32x16_f16 per 32 x 32 tile (A operands from LDS),
 *                    16 exponentials per lane of the previous tile's products, their
 *                    position adds and tile-sum tree, group routing every 8 tiles
 *                                                               -> exponentials/s
 *   MD_UB_TILE_MIX4  the same at four K steps and 16 label bits (four MFMAs per tile,
 *                    8 routed bits)                             -> exponentials/s
 *   MD_UB_TILE_MIX1  the same as MD_UB_TILE_MIX with one K step (one MFMA per tile)
 *                                                               -> exponentials/s
 * Returns MD_OK, MD_EINVAL (unknown kind, work < 0, a copy without buffers, with work not a
 * positive multiple of 16 or with unaligned buffers), MD_ENOMEM, MD_EHIP. */
#define MD_UB_EXP       0
#define MD_UB_ADD_F32   1
#define MD_UB_MFMA_F16  2
#define MD_UB_MFMA_BF16 3
#define MD_UB_MFMA_F32  4
#define MD_UB_COPY      5
#define MD_UB_EXP_ADD2  6
#define MD_UB_TILE_MIX  7
#define MD_UB_TILE_MIX4 8
#define MD_UB_TILE_MIX1 9
int ubench(int kind, int64_t work, const void* d_src, void* d_dst, double* h_rate, double* h_ms, void* stream);

/* ------------------------------------------------------------------ kernel timing */
/* Live timing of the demappers' dominant kernel (the fast pass of llr_exact and
 * llr_maxlog, M > 16), for roofline figures.  kernel_timing(1, stream) makes every later
 * demapping call on `stream` (current device) record a HIP event pair on that stream
 * around its fast kernel (not around prep or the fallback passes; not while the stream
 * is being captured); kernel_timing(0, stream) waits for the stream and stops it.
 * kernel_timing_read waits for the stream, writes the summed milliseconds and the number
 * of timed launches since the last read, and starts a new count.
 * Returns MD_OK, MD_EINVAL (NULL output), MD_ENODEV, MD_EHIP. */
int kernel_timing(int enable, void* stream);
int kernel_timing_read(double* total_ms, int64_t* launches, void* stream);

/* ------------------------------------------------------------------ failure injection */
/* Test hook for the failure paths: the k-th next device allocation the library makes
 * (workspaces, stage counters, plans, networks, receivers; k = 0: the very next one)
 * fails as if the device were out of memory, so that the caller sees MD_ENOMEM and can
 * check that nothing leaked; k < 0 switches it off.  Process-wide.  Returns MD_OK. */
int alloc_fault_inject(int k);

/* The device memory the library holds right now through its own allocations (stream
 * workspaces and counters, sweep plans, networks, receivers; not the fixed per-device
 * arrays of llr_exact_noalloc and kk_frontend): bytes and number of allocations.  After
 * release_cache and the destroy calls of every handle it returns to zero.  Returns MD_OK,
 * MD_EINVAL (NULL output). */
int alloc_stats(int64_t* live_bytes, int64_t* live_allocs);

/* ------------------------------------------------------------------ housekeeping */
/* Frees every internal device workspace (synchronises the device first). */
int release_cache(void);

/* Message for the last non-OK status returned on the calling thread ("" if none). */
const char* last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int mdemap_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MDEMAP_H */
