/*
 * FP64 CPU oracle for bit-wise demapping of labelled constellations over AWGN.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What the method computes is not written out in the paper: the paper's receiver
 * (section "Experimental setup", DSP-chain paragraph) ends with the equaliser
 * decisions being demapped, and its acronym glossary names the quantities used
 * here (LLR, GMI, AIR, AWGN, BICM, BRGC) without defining them.  The oracle is
 * therefore the textbook definition of each quantity for bit-interleaved coded
 * modulation with a bit-metric decoder and uniform priors:
 *
 *   q[n][j]   = -||y_n - x_j||^2 / (2 sigma2)                 (difference form)
 *   L[n][k]   = LSE_{j: bit_k(l_j)=0} q[n][j] - LSE_{j: bit_k(l_j)=1} q[n][j]
 *               bit_k(l) = (l >> (m-1-k)) & 1   (column 0 is the label's MSB)
 *               LSE(S)   = max(S) + ln sum exp(q - max(S))    (max per subset)
 *   Lml[n][k] = max_{bit=0} q - max_{bit=1} q                 (max-log)
 *   T_n       = sum_k softplus(-s_nk L_nk) / ln 2,  s = +1 if the sent bit is 0
 *   GMI       = m - (1/N) sum_n T_n      bits per D-dimensional symbol
 *   SE        = std(T_n) / sqrt(N)
 *
 * plus a re-implementation, from its written definition, of the counter-based
 * AWGN generator that the library's awgn_sample follows (Philox4x32-10, Salmon et
 * al., SC'11, then a Box-Muller transform evaluated with IEEE single +,-,*,/,
 * fma and sqrt only), and an FP64 reference of the small MLP demapper with its
 * analytic backward pass and an Adam step.
 *
 * Everything is plain double precision.  Build with -ffp-contract=off: the AWGN
 * twin depends on every operation being the one written here.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11).  Counter c[4], key k[2]; ten rounds, each round
 *   (hi0,lo0) = mulhilo(0xD2511F53, c0), (hi1,lo1) = mulhilo(0xCD9E8D57, c2)
 *   c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
 * followed by the Weyl key bump k0 += 0x9E3779B9, k1 += 0xBB67AE85 between
 * rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------- */
/* The channel's normal pair, in IEEE single precision exactly as the generator
 * definition fixes it (every operation correctly rounded, fma where written), from a
 * radius word a and an angle word b:
 *   radius: v = (float)(a | 1), rounded to nearest even, and U = v 2^-32, uniform on
 *     [2^-32, 1] with 24 bits inside each binade; v = f 2^E with f in [1, 2) read
 *     from its bits, k = E - 32;
 *     if f > sqrt2: f = f/2, k = k + 1;
 *     s = (f-1)/(f+1), w = s*s, P = Horner over w of 1/(2i+1), i = 5..0;
 *     ln U = fma(k, LN2_HI, fma(k, LN2_LO, (2 s) P))   (ln f = 2 atanh s);
 *     R = sqrt(-2 ln U);
 *   angle: q = b >> 30 quarter turns plus t = (2T+1) 2^-24 of a quarter turn,
 *     T = (b >> 7) mod 2^23; for t <= 1/2 sin and cos of phi = t pi/2 by Taylor
 *     polynomials in phi^2 (sin to phi^11, cos to phi^12), otherwise the complement
 *     t' = 1 - t with the two swapped;
 *   (z0, z1) = R (cos, sin) after q quarter turns. */
static const float GEN_SQRT2 = 0x1.6a09e6p+0f;
static const float GEN_LN2_HI = 0x1.62e300p-1f;
static const float GEN_LN2_LO = 0x1.2fefa2p-17f;
static const float GEN_PIO2 = 0x1.921fb6p+0f;

static float orc_gen_log_u(uint32_t a) {
    float v = (float)(a | 1u);                        /* correctly rounded */
    uint32_t bits;
    memcpy(&bits, &v, sizeof bits);
    int E = (int)(bits >> 23) - 127;                  /* v >= 1: a normal number */
    uint32_t fb = (bits & 0x007FFFFFu) | 0x3F800000u;
    float f;
    memcpy(&f, &fb, sizeof f);
    float k = (float)(E - 32);
    if (f > GEN_SQRT2) {
        f = f * 0.5f;
        k = k + 1.0f;
    }
    float s = (f - 1.0f) / (f + 1.0f);
    float w = s * s;
    float P = 1.0f / 11.0f;
    P = fmaf(P, w, 1.0f / 9.0f);
    P = fmaf(P, w, 1.0f / 7.0f);
    P = fmaf(P, w, 1.0f / 5.0f);
    P = fmaf(P, w, 1.0f / 3.0f);
    P = fmaf(P, w, 1.0f);
    float lnf = (2.0f * s) * P;
    return fmaf(k, GEN_LN2_HI, fmaf(k, GEN_LN2_LO, lnf));
}

static void orc_gen_sincos_quarter(uint32_t T, float* s_out, float* c_out) {
    float t = (float)(2u * T + 1u) * 0x1p-24f;        /* exact */
    float phi = t * GEN_PIO2;
    float w = phi * phi;
    float S = -1.0f / 39916800.0f;                    /* 1/11! */
    S = fmaf(S, w, 1.0f / 362880.0f);                 /* 1/9!  */
    S = fmaf(S, w, -1.0f / 5040.0f);                  /* 1/7!  */
    S = fmaf(S, w, 1.0f / 120.0f);                    /* 1/5!  */
    S = fmaf(S, w, -1.0f / 6.0f);                     /* 1/3!  */
    S = fmaf(S, w, 1.0f);
    float C = 1.0f / 479001600.0f;                    /* 1/12! */
    C = fmaf(C, w, -1.0f / 3628800.0f);               /* 1/10! */
    C = fmaf(C, w, 1.0f / 40320.0f);                  /* 1/8!  */
    C = fmaf(C, w, -1.0f / 720.0f);                   /* 1/6!  */
    C = fmaf(C, w, 1.0f / 24.0f);                     /* 1/4!  */
    C = fmaf(C, w, -1.0f / 2.0f);                     /* 1/2!  */
    C = fmaf(C, w, 1.0f);
    *s_out = phi * S;
    *c_out = C;
}

/* One Box-Muller pair from a radius word a and an angle word b. */
static void orc_gen_normal_pair(uint32_t a, uint32_t b, float* z0, float* z1) {
    float R = sqrtf(-2.0f * orc_gen_log_u(a));
    uint32_t q = b >> 30;
    uint32_t T = (b >> 7) & 0x7FFFFFu;
    float sp, cp, c, s;
    if (T < (1u << 22)) {
        orc_gen_sincos_quarter(T, &sp, &cp);
        c = cp; s = sp;
    } else {
        /* phi = pi/2 - phi' with phi' = (2 T' + 1) 2^-24 pi/2 */
        orc_gen_sincos_quarter((1u << 23) - 1u - T, &sp, &cp);
        c = sp; s = cp;
    }
    float ct, st;
    switch ((int)q) {
        case 0: ct = c;  st = s;  break;
        case 1: ct = -s; st = c;  break;
        case 2: ct = -c; st = -s; break;
        default: ct = s; st = -c; break;
    }
    *z0 = R * ct;
    *z1 = R * st;
}

/* The normal pair for a radius word w[0] and an angle word w[1] (exported so the
 * transform can be checked against libm's log, atan2 and hypot). */
void orc_gen_box_muller(const uint32_t w[2], double z[2]) {
    float z0, z1;
    orc_gen_normal_pair(w[0], w[1], &z0, &z1);
    z[0] = z0;
    z[1] = z1;
}

/* Channel: u_n uniform on {0..M-1}, z_n ~ N(0, I_D), y_n = fl32(x_{u_n} + sigma z_n).
 * Channel use n (g = offset + n, key = (seed_lo, seed_hi)) reads one stream of words:
 * block j of the stream is the Philox output of counter (g_lo, g_hi, j, 1), and word
 * 4j + i is its output word i.  Word 0 gives u_n = word >> (32 - m); pair p takes words
 * 2p + 1 (radius) and 2p + 2 (angle) and feeds dimensions 2p and 2p + 1. */
void orc_awgn(const float* X, int M, int D, uint64_t seed, uint64_t offset, int64_t N,
              double sigma, uint32_t* tx, float* y) {
    int m = 0;
    while ((1 << m) < M) ++m;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int npairs = (D + 1) / 2;
    int nwords = 1 + 2 * npairs;
    int nblocks = (nwords + 3) / 4;
    uint32_t* words = (uint32_t*)malloc(sizeof(uint32_t) * 4 * (size_t)nblocks);
    for (int64_t n = 0; n < N; ++n) {
        uint64_t g = offset + (uint64_t)n;
        for (int j = 0; j < nblocks; ++j) {
            uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(g >> 32), (uint32_t)j, 1u};
            orc_philox4x32_10(ctr, key, words + 4 * j);
        }
        uint32_t u = words[0] >> (32 - m);
        tx[n] = u;
        for (int p = 0; p < npairs; ++p) {
            float z0, z1;
            orc_gen_normal_pair(words[2 * p + 1], words[2 * p + 2], &z0, &z1);
            int d0 = 2 * p, d1 = 2 * p + 1;
            y[n * D + d0] = (float)fma(sigma, (double)z0, (double)X[(int64_t)u * D + d0]);
            if (d1 < D) y[n * D + d1] = (float)fma(sigma, (double)z1, (double)X[(int64_t)u * D + d1]);
        }
    }
    free(words);
}

/* ------------------------------------------------------------------------- */
static int orc_log2_int(int M) {
    int m = 0;
    while ((1 << m) < M) ++m;
    return m;
}

/* Exact bit-wise LLR (definition above), one symbol at a time; q[] is scratch of M doubles. */
static void orc_llr_exact_one(const float* X, const uint32_t* labels, int M, int D, int m,
                              const float* yn, double sigma2, double* q, double* out) {
    for (int j = 0; j < M; ++j) {
        double d2 = 0.0;
        for (int d = 0; d < D; ++d) {
            double diff = (double)yn[d] - (double)X[(int64_t)j * D + d];
            d2 += diff * diff;
        }
        q[j] = -d2 / (2.0 * sigma2);
    }
    for (int k = 0; k < m; ++k) {
        int shift = m - 1 - k;
        double lse[2];
        for (int b = 0; b < 2; ++b) {
            double mx = -INFINITY;
            for (int j = 0; j < M; ++j)
                if ((int)((labels[j] >> shift) & 1u) == b && q[j] > mx) mx = q[j];
            double s = 0.0;
            for (int j = 0; j < M; ++j)
                if ((int)((labels[j] >> shift) & 1u) == b) s += exp(q[j] - mx);
            lse[b] = mx + log(s);
        }
        out[k] = lse[0] - lse[1];
    }
}

void orc_llr_exact(const float* X, const uint32_t* labels, int M, int D, const float* y, int64_t N,
                   double sigma2, double* llr) {
    int m = orc_log2_int(M);
#pragma omp parallel
    {
        double* q = (double*)malloc(sizeof(double) * (size_t)M);
#pragma omp for schedule(static)
        for (int64_t n = 0; n < N; ++n)
            orc_llr_exact_one(X, labels, M, D, m, y + n * D, sigma2, q, llr + n * m);
        free(q);
    }
}

void orc_llr_maxlog(const float* X, const uint32_t* labels, int M, int D, const float* y, int64_t N,
                    double sigma2, double* llr) {
    int m = orc_log2_int(M);
#pragma omp parallel
    {
        double* q = (double*)malloc(sizeof(double) * (size_t)M);
#pragma omp for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            const float* yn = y + n * D;
            for (int j = 0; j < M; ++j) {
                double d2 = 0.0;
                for (int d = 0; d < D; ++d) {
                    double diff = (double)yn[d] - (double)X[(int64_t)j * D + d];
                    d2 += diff * diff;
                }
                q[j] = -d2 / (2.0 * sigma2);
            }
            for (int k = 0; k < m; ++k) {
                int shift = m - 1 - k;
                double mx[2] = {-INFINITY, -INFINITY};
                for (int j = 0; j < M; ++j) {
                    int b = (int)((labels[j] >> shift) & 1u);
                    if (q[j] > mx[b]) mx[b] = q[j];
                }
                llr[n * m + k] = mx[0] - mx[1];
            }
        }
        free(q);
    }
}

/* Hard decision: index of the nearest constellation point (lowest index on ties). */
void orc_hard_decision(const float* X, int M, int D, const float* y, int64_t N, uint32_t* jhat) {
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double best = INFINITY;
        uint32_t arg = 0;
        for (int j = 0; j < M; ++j) {
            double d2 = 0.0;
            for (int d = 0; d < D; ++d) {
                double diff = (double)y[n * D + d] - (double)X[(int64_t)j * D + d];
                d2 += diff * diff;
            }
            if (d2 < best) { best = d2; arg = (uint32_t)j; }
        }
        jhat[n] = arg;
    }
}

/* ------------------------------------------------------------------------- */
static double orc_softplus(double t) {
    return (t > 0.0 ? t : 0.0) + log1p(exp(-fabs(t)));
}

/* Neumaier-compensated running sum. */
typedef struct { double s, c; } orc_ksum;
static void orc_ksum_add(orc_ksum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double orc_ksum_get(const orc_ksum* a) { return a->s + a->c; }

/* Per-symbol T_n = sum_k softplus(-s_nk L_nk)/ln 2 (bits lost by symbol n). */
void orc_gmi_terms(const double* llr, int64_t N, int m, const uint32_t* tx, const uint32_t* labels,
                   double* T, double* per_bit_terms /* N x m or NULL */) {
    for (int64_t n = 0; n < N; ++n) {
        uint32_t lab = labels[tx[n]];
        double acc = 0.0;
        for (int k = 0; k < m; ++k) {
            int bit = (int)((lab >> (m - 1 - k)) & 1u);
            double sgn = bit ? -1.0 : 1.0;
            double t = orc_softplus(-sgn * llr[n * m + k]) / M_LN2;
            if (per_bit_terms) per_bit_terms[n * m + k] = t;
            acc += t;
        }
        T[n] = acc;
    }
}

/* GMI, per-bit GMI and standard error (two-pass variance), all sums compensated. */
void orc_gmi(const double* llr, int64_t N, int m, const uint32_t* tx, const uint32_t* labels,
             double* gmi, double* gmi_per_bit, double* se) {
    double* T = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double* Tb = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N * m : 1));
    orc_gmi_terms(llr, N, m, tx, labels, T, Tb);
    orc_ksum tot = {0.0, 0.0};
    for (int64_t n = 0; n < N; ++n) orc_ksum_add(&tot, T[n]);
    double mean = orc_ksum_get(&tot) / (double)N;
    *gmi = (double)m - mean;
    if (gmi_per_bit) {
        for (int k = 0; k < m; ++k) {
            orc_ksum bk = {0.0, 0.0};
            for (int64_t n = 0; n < N; ++n) orc_ksum_add(&bk, Tb[n * m + k]);
            gmi_per_bit[k] = 1.0 - orc_ksum_get(&bk) / (double)N;
        }
    }
    if (se) {
        orc_ksum v = {0.0, 0.0};
        for (int64_t n = 0; n < N; ++n) orc_ksum_add(&v, (T[n] - mean) * (T[n] - mean));
        *se = N > 1 ? sqrt(orc_ksum_get(&v) / (double)(N - 1)) / sqrt((double)N) : 0.0;
    }
    free(T);
    free(Tb);
}

/* ------------------------------------------------------------------------- */
/* MLP demapper reference: f(y) = s_out (W3 g(W2 g(W1 (s_in y) + b1) + b2) + b3) with fixed
 * (untrained) input and output scales s_in, s_out and the GELU activation (Hendrycks &
 * Gimpel) in its exact form, the input times the standard normal distribution function:
 *   g(a) = a Phi(a),  Phi(a) = erfc(-a / sqrt 2) / 2,
 *   g'(a) = Phi(a) + a phi(a),  phi(a) = exp(-a^2 / 2) / sqrt(2 pi).
 * (erfc rather than 1 + erf keeps Phi accurate in the lower tail.)
 * Weights are row-major [out][in].  Loss per sample:
 * sum_k p_k softplus(-f_k) + (1 - p_k) softplus(f_k) with p_k = sigmoid(L_target_k),
 * averaged over the batch. */
static double orc_gelu(double a) {
    return 0.5 * a * erfc(-a / M_SQRT2);
}
static double orc_gelu_grad(double a) {
    return 0.5 * erfc(-a / M_SQRT2) + a * exp(-0.5 * a * a) / sqrt(2.0 * M_PI);
}
/* The activation and its derivative at n points (exposed for the oracle's own pins). */
void orc_gelu_eval(const double* a, int64_t n, double* g, double* dg) {
    for (int64_t i = 0; i < n; ++i) {
        g[i] = orc_gelu(a[i]);
        dg[i] = orc_gelu_grad(a[i]);
    }
}
static double orc_sigmoid(double t) {
    return t >= 0.0 ? 1.0 / (1.0 + exp(-t)) : exp(t) / (1.0 + exp(t));
}

void orc_mlp_forward(int D, int H1, int H2, int m,
                     const double* W1, const double* b1, const double* W2, const double* b2,
                     const double* W3, const double* b3, double s_in, double s_out,
                     const float* y, int64_t N, double* out) {
#pragma omp parallel
    {
        double* h1 = (double*)malloc(sizeof(double) * (size_t)H1);
        double* h2 = (double*)malloc(sizeof(double) * (size_t)H2);
#pragma omp for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            for (int i = 0; i < H1; ++i) {
                double z = b1[i];
                for (int d = 0; d < D; ++d) z += W1[i * D + d] * (s_in * (double)y[n * D + d]);
                h1[i] = orc_gelu(z);
            }
            for (int i = 0; i < H2; ++i) {
                double z = b2[i];
                for (int d = 0; d < H1; ++d) z += W2[(int64_t)i * H1 + d] * h1[d];
                h2[i] = orc_gelu(z);
            }
            for (int k = 0; k < m; ++k) {
                double z = b3[k];
                for (int d = 0; d < H2; ++d) z += W3[(int64_t)k * H2 + d] * h2[d];
                out[n * m + k] = s_out * z;
            }
        }
        free(h1);
        free(h2);
    }
}

/* Mean distillation loss over the batch and its gradient with respect to every
 * parameter (gradient arrays are overwritten). */
double orc_mlp_loss_grad(int D, int H1, int H2, int m,
                         const double* W1, const double* b1, const double* W2, const double* b2,
                         const double* W3, const double* b3, double s_in, double s_out,
                         const float* y, const float* target, int64_t B,
                         double* gW1, double* gb1, double* gW2, double* gb2, double* gW3, double* gb3) {
    memset(gW1, 0, sizeof(double) * (size_t)H1 * D);
    memset(gb1, 0, sizeof(double) * (size_t)H1);
    memset(gW2, 0, sizeof(double) * (size_t)H2 * H1);
    memset(gb2, 0, sizeof(double) * (size_t)H2);
    memset(gW3, 0, sizeof(double) * (size_t)m * H2);
    memset(gb3, 0, sizeof(double) * (size_t)m);
    double* z1 = (double*)malloc(sizeof(double) * (size_t)H1);
    double* h1 = (double*)malloc(sizeof(double) * (size_t)H1);
    double* z2 = (double*)malloc(sizeof(double) * (size_t)H2);
    double* h2 = (double*)malloc(sizeof(double) * (size_t)H2);
    double* dz2 = (double*)malloc(sizeof(double) * (size_t)H2);
    double* dz1 = (double*)malloc(sizeof(double) * (size_t)H1);
    double* f = (double*)malloc(sizeof(double) * (size_t)m);
    double* df = (double*)malloc(sizeof(double) * (size_t)m);
    double loss = 0.0;
    for (int64_t n = 0; n < B; ++n) {
        const float* yn = y + n * D;
        for (int i = 0; i < H1; ++i) {
            double z = b1[i];
            for (int d = 0; d < D; ++d) z += W1[i * D + d] * (s_in * (double)yn[d]);
            z1[i] = z;
            h1[i] = orc_gelu(z);
        }
        for (int i = 0; i < H2; ++i) {
            double z = b2[i];
            for (int d = 0; d < H1; ++d) z += W2[(int64_t)i * H1 + d] * h1[d];
            z2[i] = z;
            h2[i] = orc_gelu(z);
        }
        for (int k = 0; k < m; ++k) {
            double z = b3[k];
            for (int d = 0; d < H2; ++d) z += W3[(int64_t)k * H2 + d] * h2[d];
            f[k] = s_out * z;                       /* the network output */
            double p = orc_sigmoid((double)target[n * m + k]);
            loss += p * orc_softplus(-f[k]) + (1.0 - p) * orc_softplus(f[k]);
            df[k] = s_out * (orc_sigmoid(f[k]) - p) / (double)B;   /* d loss / d z */
        }
        for (int k = 0; k < m; ++k) {
            gb3[k] += df[k];
            for (int d = 0; d < H2; ++d) gW3[(int64_t)k * H2 + d] += df[k] * h2[d];
        }
        for (int i = 0; i < H2; ++i) {
            double g = 0.0;
            for (int k = 0; k < m; ++k) g += W3[(int64_t)k * H2 + i] * df[k];
            dz2[i] = g * orc_gelu_grad(z2[i]);
            gb2[i] += dz2[i];
            for (int d = 0; d < H1; ++d) gW2[(int64_t)i * H1 + d] += dz2[i] * h1[d];
        }
        for (int i = 0; i < H1; ++i) {
            double g = 0.0;
            for (int k = 0; k < H2; ++k) g += W2[(int64_t)k * H1 + i] * dz2[k];
            dz1[i] = g * orc_gelu_grad(z1[i]);
            gb1[i] += dz1[i];
            for (int d = 0; d < D; ++d) gW1[i * D + d] += dz1[i] * (s_in * (double)yn[d]);
        }
    }
    free(z1); free(h1); free(z2); free(h2); free(dz2); free(dz1); free(f); free(df);
    return loss / (double)B;
}

/* One Adam step (Kingma & Ba, 2015) on P parameters; t is the 1-based step count. */
void orc_adam_step(double* w, const double* g, double* mom1, double* mom2, int64_t P, int t,
                   double lr, double beta1, double beta2, double eps) {
    double c1 = 1.0 - pow(beta1, (double)t);
    double c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < P; ++i) {
        mom1[i] = beta1 * mom1[i] + (1.0 - beta1) * g[i];
        mom2[i] = beta2 * mom2[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = mom1[i] / c1;
        double vh = mom2[i] / c2;
        w[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* Number of OpenMP threads the parallel loops above use. */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------- */
/* Four-tap widely-linear decision-directed LMS equaliser: the step just before the
 * demapper in the paper's receiver (section "Experimental setup", DSP-chain paragraph,
 * which names a four-tap adaptive time-domain DD-LMS widely-linear equaliser after
 * downsampling to 2 samples per symbol, and gives no equations).  Textbook complex LMS
 * with a widely-linear output (a filter on the samples plus one on their conjugates),
 * read as follows.  Per instance b, complex samples u_t (t = 0 .. 2N+1, 2 per symbol);
 * symbol n sees the window w_j = u_{2n+j}, j = 0..3:
 *   z_n = sum_j ( h_j w_j + g_j conj(w_j) )           (j ascending, the h term first)
 *   d_n = argmin_i |z_n - c_i|^2 over the reference points c_i (the first minimum)
 *   e_n = c_{d_n} - z_n
 *   h_j <- h_j + mu e_n conj(w_j),   g_j <- g_j + mu e_n w_j    (with the old w_j)
 * Complex products are (ac - bd) + i(ad + bc), every operation in double precision in
 * the order written below (the file is built without contraction).  Layout: time-major,
 * sample t of instance b is x[2 (t B + b)] (re) and x[2 (t B + b) + 1] (im); symbol n of
 * instance b goes to dec[n B + b] and z[2 (n B + b)], the final taps of instance b to
 * h_out[8 b + 2 j] (re), h_out[8 b + 2 j + 1] (im), likewise g_out.  h0 and g0 hold the
 * starting taps (re, im interleaved) shared by all instances. */
void orc_ddlms(const float* x, int64_t B, int64_t N, const float* C, int M, const double* h0, const double* g0,
               double mu, uint32_t* dec, float* z, double* h_out, double* g_out) {
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < B; ++b) {
        double hr[4], hi[4], gr[4], gi[4];
        for (int j = 0; j < 4; ++j) {
            hr[j] = h0[2 * j];
            hi[j] = h0[2 * j + 1];
            gr[j] = g0[2 * j];
            gi[j] = g0[2 * j + 1];
        }
        for (int64_t n = 0; n < N; ++n) {
            double wr[4], wi[4];
            for (int j = 0; j < 4; ++j) {
                const int64_t t = 2 * n + j;
                wr[j] = (double)x[2 * (t * B + b)];
                wi[j] = (double)x[2 * (t * B + b) + 1];
            }
            double zr = 0.0, zi = 0.0;
            for (int j = 0; j < 4; ++j) {
                zr = zr + (hr[j] * wr[j] - hi[j] * wi[j]);
                zr = zr + (gr[j] * wr[j] + gi[j] * wi[j]);
                zi = zi + (hr[j] * wi[j] + hi[j] * wr[j]);
                zi = zi + (gi[j] * wr[j] - gr[j] * wi[j]);
            }
            double best = INFINITY;
            int arg = 0;
            for (int i = 0; i < M; ++i) {
                const double dr = zr - (double)C[2 * i];
                const double di = zi - (double)C[2 * i + 1];
                const double d2 = dr * dr + di * di;
                if (d2 < best) { best = d2; arg = i; }
            }
            const double er = (double)C[2 * arg] - zr;
            const double ei = (double)C[2 * arg + 1] - zi;
            for (int j = 0; j < 4; ++j) {
                hr[j] = hr[j] + mu * (er * wr[j] + ei * wi[j]);
                hi[j] = hi[j] + mu * (ei * wr[j] - er * wi[j]);
                gr[j] = gr[j] + mu * (er * wr[j] - ei * wi[j]);
                gi[j] = gi[j] + mu * (er * wi[j] + ei * wr[j]);
            }
            dec[n * B + b] = (uint32_t)arg;
            z[2 * (n * B + b)] = (float)zr;
            z[2 * (n * B + b) + 1] = (float)zi;
        }
        for (int j = 0; j < 4; ++j) {
            h_out[8 * b + 2 * j] = hr[j];
            h_out[8 * b + 2 * j + 1] = hi[j];
            g_out[8 * b + 2 * j] = gr[j];
            g_out[8 * b + 2 * j + 1] = gi[j];
        }
    }
}
