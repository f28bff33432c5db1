/*
 * ldpc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, CPU reference for layered normalised min-sum decoding of
 * quasi-cyclic LDPC codes (Ling & Cautereels, "Fast LDPC GPU Decoder for
 * Cloud RAN", §III and §IV). It exists to check the GPU decoder; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it. It shares no source with the GPU path: the graph arrives as data
 * (block row pointers, block columns, shifts), the LLRs as bytes.
 *
 * Notation (paper §III): L_v posterior of variable v, L_b channel LLR,
 * L_{c->v} check-to-variable message (here R), L_{v->c} variable-to-check
 * message (here x), beta the normalisation factor.
 *
 * Graph: M block rows, N block columns, lift Z; block e of row r
 * (row_ptr[r] <= e < row_ptr[r+1], ascending column) has column col[e] and
 * shift shift[e]: check row z of block row r touches variable
 * col[e]*Z + (z + shift[e]) mod Z. The first n_punct block columns are not
 * transmitted: their L_v start at 0 and they are absent from the input.
 *
 * Schedule (§III, horizontal layered): block rows in order 0..M-1, one
 * iteration = all M block rows; inside a block row the Z check rows touch
 * disjoint variables (§II), so their order does not matter.
 *
 * Four number modes:
 *   i8   -- 8-bit saturating fixed point (symmetric +-127), normalisation in
 *           Q1.7: a = min((w*m + 64) >> 7, 127), w = 96 gives beta = 3/4.
 *   f16  -- IEEE binary16 with every operation rounded to nearest-even,
 *           emulated by exact double arithmetic followed by one rounding.
 *   f64  -- double precision, no clamp (beta per (iteration, block row)).
 * The f64 mode also provides the exact gradient of the learned weighted
 * min-sum loss (oracle_nwms_grad_f64), and, for context only, the
 * sum-product check rule and the flooding schedule (oracle_decode_bp_f64).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -2

typedef struct {
    int M, N, Z, n_punct;
    const int32_t *row_ptr;
    const int16_t *col;
    const int16_t *shift;
} graph_t;

static int graph_check(const graph_t *g) {
    if (g->M < 1 || g->N < 1 || g->Z < 1 || g->n_punct < 0 || g->n_punct > g->N) return 0;
    if (!g->row_ptr || !g->col || !g->shift || g->row_ptr[0] != 0) return 0;
    for (int r = 0; r < g->M; ++r) {
        if (g->row_ptr[r + 1] <= g->row_ptr[r]) return 0;
        for (int e = g->row_ptr[r]; e < g->row_ptr[r + 1]; ++e) {
            if (g->col[e] < 0 || g->col[e] >= g->N) return 0;
            if (g->shift[e] < 0 || g->shift[e] >= g->Z) return 0;
            if (e > g->row_ptr[r] && g->col[e] <= g->col[e - 1]) return 0;
        }
    }
    return 1;
}

/* variable index touched by check row z through block e */
static inline int var_of(const graph_t *g, int e, int z) {
    return g->col[e] * g->Z + (z + g->shift[e]) % g->Z;
}

/* Syndrome of hard decisions hd[N*Z] (1 = bit one): 1 if every check holds. */
static int all_checks_hold(const graph_t *g, const uint8_t *hd) {
    for (int r = 0; r < g->M; ++r)
        for (int z = 0; z < g->Z; ++z) {
            int par = 0;
            for (int e = g->row_ptr[r]; e < g->row_ptr[r + 1]; ++e) par ^= hd[var_of(g, e, z)];
            if (par) return 0;
        }
    return 1;
}

static void pack_bits(const uint8_t *hd, int K, uint8_t *out) {
    memset(out, 0, (size_t)(K + 7) / 8);
    for (int j = 0; j < K; ++j)
        if (hd[j]) out[j >> 3] |= (uint8_t)(1u << (j & 7));
}

/* ------------------------------------------------------------------ */
/* int8 saturating mode                                                */
/* ------------------------------------------------------------------ */

static inline int sat127(int v) { return v > 127 ? 127 : (v < -127 ? -127 : v); }

/* Normalised magnitude (§III min-sum with correction factor beta): the
 * offset delta is removed first, then the Q1.7 multiplier w is applied
 * with round-half-up, and the result saturates at 127. */
static inline int norm_i8(int m, int w, int delta) {
    int v = m - delta;
    if (v < 0) v = 0;
    v = (w * v + 64) >> 7;
    return v > 127 ? 127 : v;
}

typedef struct {
    const graph_t *g;
    int kb_bits;          /* K: number of information bits output */
    const int8_t *q;      /* [n_cw][T] */
    int n_cw, max_iter, early_exit, delta;
    const uint8_t *wq;    /* [wq_iters][M] or NULL */
    int wq_iters;
    uint8_t *out_bits;    /* [n_cw][ceil(K/8)] */
    int32_t *out_iters;   /* [n_cw] */
    uint8_t *out_ok;      /* [n_cw] or NULL */
    int8_t *out_llr;      /* [n_cw][N*Z] or NULL */
    int cw_begin, cw_end, status;
} i8_job_t;

static int decode_one_i8(const i8_job_t *jb, int cw, int *L, int *R, int *x, uint8_t *hd) {
    const graph_t *g = jb->g;
    const int Z = g->Z, NZ = g->N * g->Z, E = g->row_ptr[g->M];
    const int T = (g->N - g->n_punct) * Z;
    const int8_t *q = jb->q + (size_t)cw * T;

    /* Initialisation: punctured variables carry no channel information. */
    for (int j = 0; j < g->n_punct * Z; ++j) L[j] = 0;
    for (int i = 0; i < T; ++i) L[g->n_punct * Z + i] = q[i] < -127 ? -127 : q[i];
    memset(R, 0, sizeof(int) * (size_t)E * Z);

    int iters = jb->max_iter, ok = 0;
    for (int t = 1; t <= jb->max_iter; ++t) {
        for (int r = 0; r < g->M; ++r) {
            const int e0 = g->row_ptr[r], w_r = g->row_ptr[r + 1] - e0;
            int w = 96;
            if (jb->wq) {
                int ti = t <= jb->wq_iters ? t : jb->wq_iters;
                w = jb->wq[(size_t)(ti - 1) * g->M + r];
            }
            for (int z = 0; z < Z; ++z) {
                /* variable-to-check messages L_{v->c} = L_v - L_{c->v} */
                int m1 = 1 << 30, m2 = 1 << 30, k1 = -1, S = 0;
                for (int k = 0; k < w_r; ++k) {
                    const int v = var_of(g, e0 + k, z);
                    x[k] = sat127(L[v] - R[(size_t)(e0 + k) * Z + z]);
                    const int a = x[k] < 0 ? -x[k] : x[k];
                    if (a < m1) { m2 = m1; m1 = a; k1 = k; }
                    else if (a < m2) { m2 = a; }
                    S ^= x[k] < 0;
                }
                /* check-to-variable: magnitude of the minimum over the
                 * other edges (m2 for the argmin edge, m1 otherwise), sign
                 * the product of the other edges' signs. */
                const int a1 = norm_i8(m1, w, jb->delta), a2 = norm_i8(m2, w, jb->delta);
                for (int k = 0; k < w_r; ++k) {
                    const int v = var_of(g, e0 + k, z);
                    const int mag = (k == k1) ? a2 : a1;
                    const int neg = S ^ (x[k] < 0);
                    const int rn = neg ? -mag : mag;
                    R[(size_t)(e0 + k) * Z + z] = rn;
                    L[v] = sat127(x[k] + rn); /* posterior L_v = L_{v->c} + L_{c->v} */
                }
            }
        }
        if (jb->early_exit || t == jb->max_iter) {
            for (int j = 0; j < NZ; ++j) hd[j] = L[j] < 0;
            const int holds = all_checks_hold(g, hd);
            if (jb->early_exit && holds) { iters = t; ok = 1; break; }
            if (t == jb->max_iter) ok = holds;
        }
    }
    for (int j = 0; j < NZ; ++j) hd[j] = L[j] < 0;
    pack_bits(hd, jb->kb_bits, jb->out_bits + (size_t)cw * ((jb->kb_bits + 7) / 8));
    jb->out_iters[cw] = iters;
    if (jb->out_ok) jb->out_ok[cw] = (uint8_t)ok;
    if (jb->out_llr)
        for (int j = 0; j < NZ; ++j) jb->out_llr[(size_t)cw * NZ + j] = (int8_t)L[j];
    return ORACLE_OK;
}

static int max_row_weight(const graph_t *g) {
    int w = 0;
    for (int r = 0; r < g->M; ++r)
        if (g->row_ptr[r + 1] - g->row_ptr[r] > w) w = g->row_ptr[r + 1] - g->row_ptr[r];
    return w;
}

static void *i8_worker(void *arg) {
    i8_job_t *jb = (i8_job_t *)arg;
    const graph_t *g = jb->g;
    const size_t NZ = (size_t)g->N * g->Z, EZ = (size_t)g->row_ptr[g->M] * g->Z;
    int *L = malloc(sizeof(int) * NZ), *R = malloc(sizeof(int) * EZ);
    int *x = malloc(sizeof(int) * (size_t)max_row_weight(g));
    uint8_t *hd = malloc(NZ);
    if (!L || !R || !x || !hd) { jb->status = ORACLE_ENOMEM; goto out; }
    for (int cw = jb->cw_begin; cw < jb->cw_end; ++cw) decode_one_i8(jb, cw, L, R, x, hd);
    jb->status = ORACLE_OK;
out:
    free(L); free(R); free(x); free(hd);
    return NULL;
}

/* Runs `worker` on each of n_jobs job records, one POSIX thread per job
 * (the calling thread takes the first); a job whose thread cannot be
 * started runs on the calling thread afterwards. */
static void run_threads(void *jobs, size_t job_size, int n_jobs, void *(*worker)(void *)) {
    pthread_t *th = malloc(sizeof(pthread_t) * (size_t)n_jobs);
    int started = 0;
    if (th)
        for (int i = 1; i < n_jobs; ++i) {
            if (pthread_create(&th[i], NULL, worker, (char *)jobs + job_size * i) != 0) break;
            started = i;
        }
    worker(jobs);
    for (int i = 1; i <= started; ++i) pthread_join(th[i], NULL);
    for (int i = started + 1; i < n_jobs; ++i) worker((char *)jobs + job_size * i);
    free(th);
}

int oracle_decode_i8(int M, int N, int Z, int n_punct, int K,
                     const int32_t *row_ptr, const int16_t *col, const int16_t *shift,
                     int n_cw, const int8_t *q, int max_iter, int early_exit, int delta,
                     const uint8_t *wq, int wq_iters,
                     uint8_t *out_bits, int32_t *out_iters, uint8_t *out_ok, int8_t *out_llr,
                     int n_threads) {
    graph_t g = {M, N, Z, n_punct, row_ptr, col, shift};
    if (!graph_check(&g) || n_cw < 0 || max_iter < 1 || K < 0 || K > N * Z || delta < 0 ||
        delta > 127 || (n_cw > 0 && (!q || !out_bits || !out_iters)) ||
        (wq && wq_iters < 1))
        return ORACLE_EINVAL;
    if (n_cw == 0) return ORACLE_OK;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > n_cw) n_threads = n_cw;
    i8_job_t *jobs = calloc((size_t)n_threads, sizeof(i8_job_t));
    if (!jobs) return ORACLE_ENOMEM;
    for (int i = 0; i < n_threads; ++i) {
        i8_job_t *jb = &jobs[i];
        jb->g = &g; jb->kb_bits = K; jb->q = q; jb->n_cw = n_cw; jb->max_iter = max_iter;
        jb->early_exit = early_exit; jb->delta = delta; jb->wq = wq; jb->wq_iters = wq_iters;
        jb->out_bits = out_bits; jb->out_iters = out_iters; jb->out_ok = out_ok;
        jb->out_llr = out_llr;
        jb->cw_begin = (int)((long long)n_cw * i / n_threads);
        jb->cw_end = (int)((long long)n_cw * (i + 1) / n_threads);
        jb->status = ORACLE_OK;
    }
    run_threads(jobs, sizeof(i8_job_t), n_threads, i8_worker);
    int status = ORACLE_OK;
    for (int i = 0; i < n_threads; ++i)
        if (jobs[i].status != ORACLE_OK) status = jobs[i].status;
    free(jobs);
    return status;
}

/* ------------------------------------------------------------------ */
/* IEEE binary16 emulation                                             */
/* ------------------------------------------------------------------ */

/* binary16 bit pattern -> double (exact). */
static double h2d(uint16_t h) {
    const int s = h >> 15, e = (h >> 10) & 31, m = h & 1023;
    double v;
    if (e == 0) v = ldexp((double)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = ldexp((double)(1024 + m), e - 25);
    return s ? -v : v;
}

/* double -> binary16, round to nearest, ties to even, with subnormals and
 * overflow to infinity (IEEE 754-2008 §4.3.1). */
static uint16_t d2h(double v) {
    const uint16_t sign = signbit(v) ? 0x8000 : 0;
    if (isnan(v)) return 0x7e00;
    const double a = fabs(v);
    if (a >= 65520.0) return sign | 0x7c00; /* at or beyond max + half an ulp */
    if (a == 0.0) return sign;
    int e2;
    frexp(a, &e2); /* a in [2^(e2-1), 2^e2) */
    int E = e2 - 1;
    if (E < -14) E = -14; /* subnormals share the quantum 2^-24 */
    const double quantum = ldexp(1.0, E - 10);
    const double n = a / quantum; /* exact: division by a power of two */
    double fl = floor(n);
    const double fr = n - fl;
    if (fr > 0.5 || (fr == 0.5 && fmod(fl, 2.0) == 1.0)) fl += 1.0;
    unsigned m = (unsigned)fl;
    if (m == 0) return sign;
    if (m >= 2048) { m >>= 1; E += 1; }
    if (m < 1024) return sign | (uint16_t)m; /* subnormal */
    if (E > 15) return sign | 0x7c00;
    return sign | (uint16_t)(((E + 15) << 10) | (m - 1024));
}

void oracle_f64_to_f16(const double *in, uint16_t *out, long n) {
    for (long i = 0; i < n; ++i) out[i] = d2h(in[i]);
}

void oracle_f16_to_f64(const uint16_t *in, double *out, long n) {
    for (long i = 0; i < n; ++i) out[i] = h2d(in[i]);
}

/* Each binary16 operation: exact double result (sums and products of two
 * binary16 values are exact in double), then one rounding. */
static inline uint16_t hsub(uint16_t a, uint16_t b) { return d2h(h2d(a) - h2d(b)); }
static inline uint16_t hadd(uint16_t a, uint16_t b) { return d2h(h2d(a) + h2d(b)); }
static inline uint16_t hmul(uint16_t a, uint16_t b) { return d2h(h2d(a) * h2d(b)); }

typedef struct {
    const graph_t *g;
    int kb_bits;
    const int8_t *q;
    int n_cw, max_iter, early_exit;
    uint16_t beta, delta;     /* binary16 */
    const uint16_t *wh;       /* [wh_iters][M] binary16 or NULL */
    int wh_iters;
    uint8_t *out_bits;
    int32_t *out_iters;
    uint8_t *out_ok;
    uint16_t *out_llr;        /* [n_cw][N*Z] binary16 or NULL */
    int cw_begin, cw_end, status;
} f16_job_t;

/* Normalised magnitude in binary16: m' = max(m - delta, 0), a = w * m'. */
static inline uint16_t norm_f16(uint16_t m, uint16_t w, uint16_t delta) {
    uint16_t v = hsub(m, delta);
    if (h2d(v) < 0.0) v = 0;
    return hmul(w, v);
}

static void decode_one_f16(const f16_job_t *jb, int cw, uint16_t *L, uint16_t *R, uint16_t *x,
                           uint8_t *hd) {
    const graph_t *g = jb->g;
    const int Z = g->Z, NZ = g->N * g->Z, E = g->row_ptr[g->M];
    const int T = (g->N - g->n_punct) * Z;
    const int8_t *q = jb->q + (size_t)cw * T;
    for (int j = 0; j < g->n_punct * Z; ++j) L[j] = 0;
    for (int i = 0; i < T; ++i) L[g->n_punct * Z + i] = d2h((double)(q[i] < -127 ? -127 : q[i]));
    memset(R, 0, sizeof(uint16_t) * (size_t)E * Z);

    int iters = jb->max_iter, ok = 0;
    for (int t = 1; t <= jb->max_iter; ++t) {
        for (int r = 0; r < g->M; ++r) {
            const int e0 = g->row_ptr[r], w_r = g->row_ptr[r + 1] - e0;
            uint16_t w = jb->beta;
            if (jb->wh) {
                int ti = t <= jb->wh_iters ? t : jb->wh_iters;
                w = jb->wh[(size_t)(ti - 1) * g->M + r];
            }
            for (int z = 0; z < Z; ++z) {
                double m1 = INFINITY, m2 = INFINITY;
                int k1 = -1, S = 0;
                for (int k = 0; k < w_r; ++k) {
                    const int v = var_of(g, e0 + k, z);
                    x[k] = hsub(L[v], R[(size_t)(e0 + k) * Z + z]);
                    const double a = fabs(h2d(x[k]));
                    if (a < m1) { m2 = m1; m1 = a; k1 = k; }
                    else if (a < m2) { m2 = a; }
                    S ^= x[k] >> 15; /* IEEE sign bit */
                }
                const uint16_t a1 = norm_f16(d2h(m1), w, jb->delta);
                const uint16_t a2 = norm_f16(d2h(m2), w, jb->delta);
                for (int k = 0; k < w_r; ++k) {
                    const int v = var_of(g, e0 + k, z);
                    const uint16_t mag = (k == k1) ? a2 : a1;
                    const int neg = S ^ (x[k] >> 15);
                    const uint16_t rn = (uint16_t)(neg ? (mag | 0x8000) : mag);
                    R[(size_t)(e0 + k) * Z + z] = rn;
                    L[v] = hadd(x[k], rn);
                }
            }
        }
        if (jb->early_exit || t == jb->max_iter) {
            for (int j = 0; j < NZ; ++j) hd[j] = h2d(L[j]) < 0.0;
            const int holds = all_checks_hold(g, hd);
            if (jb->early_exit && holds) { iters = t; ok = 1; break; }
            if (t == jb->max_iter) ok = holds;
        }
    }
    for (int j = 0; j < NZ; ++j) hd[j] = h2d(L[j]) < 0.0;
    pack_bits(hd, jb->kb_bits, jb->out_bits + (size_t)cw * ((jb->kb_bits + 7) / 8));
    jb->out_iters[cw] = iters;
    if (jb->out_ok) jb->out_ok[cw] = (uint8_t)ok;
    if (jb->out_llr) memcpy(jb->out_llr + (size_t)cw * NZ, L, sizeof(uint16_t) * (size_t)NZ);
}

static void *f16_worker(void *arg) {
    f16_job_t *jb = (f16_job_t *)arg;
    const graph_t *g = jb->g;
    const size_t NZ = (size_t)g->N * g->Z, EZ = (size_t)g->row_ptr[g->M] * g->Z;
    uint16_t *L = malloc(sizeof(uint16_t) * NZ), *R = malloc(sizeof(uint16_t) * EZ);
    uint16_t *x = malloc(sizeof(uint16_t) * (size_t)max_row_weight(g));
    uint8_t *hd = malloc(NZ);
    if (!L || !R || !x || !hd) { jb->status = ORACLE_ENOMEM; goto out; }
    for (int cw = jb->cw_begin; cw < jb->cw_end; ++cw) decode_one_f16(jb, cw, L, R, x, hd);
    jb->status = ORACLE_OK;
out:
    free(L); free(R); free(x); free(hd);
    return NULL;
}

int oracle_decode_f16(int M, int N, int Z, int n_punct, int K,
                      const int32_t *row_ptr, const int16_t *col, const int16_t *shift,
                      int n_cw, const int8_t *q, int max_iter, int early_exit,
                      uint16_t beta, uint16_t delta, const uint16_t *wh, int wh_iters,
                      uint8_t *out_bits, int32_t *out_iters, uint8_t *out_ok, uint16_t *out_llr,
                      int n_threads) {
    graph_t g = {M, N, Z, n_punct, row_ptr, col, shift};
    if (!graph_check(&g) || n_cw < 0 || max_iter < 1 || K < 0 || K > N * Z ||
        (n_cw > 0 && (!q || !out_bits || !out_iters)) || (wh && wh_iters < 1))
        return ORACLE_EINVAL;
    if (n_cw == 0) return ORACLE_OK;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > n_cw) n_threads = n_cw;
    f16_job_t *jobs = calloc((size_t)n_threads, sizeof(f16_job_t));
    if (!jobs) return ORACLE_ENOMEM;
    for (int i = 0; i < n_threads; ++i) {
        f16_job_t *jb = &jobs[i];
        jb->g = &g; jb->kb_bits = K; jb->q = q; jb->n_cw = n_cw; jb->max_iter = max_iter;
        jb->early_exit = early_exit; jb->beta = beta; jb->delta = delta; jb->wh = wh;
        jb->wh_iters = wh_iters; jb->out_bits = out_bits; jb->out_iters = out_iters;
        jb->out_ok = out_ok; jb->out_llr = out_llr;
        jb->cw_begin = (int)((long long)n_cw * i / n_threads);
        jb->cw_end = (int)((long long)n_cw * (i + 1) / n_threads);
        jb->status = ORACLE_OK;
    }
    run_threads(jobs, sizeof(f16_job_t), n_threads, f16_worker);
    int status = ORACLE_OK;
    for (int i = 0; i < n_threads; ++i)
        if (jobs[i].status != ORACLE_OK) status = jobs[i].status;
    free(jobs);
    return status;
}

/* ------------------------------------------------------------------ */
/* double-precision mode (no clamp, no rounding emulation)             */
/* ------------------------------------------------------------------ */

typedef struct {
    const graph_t *g;
    int kb_bits;
    const double *llr;        /* [n_cw][T] channel LLRs */
    int n_cw, max_iter, early_exit;
    double beta, delta;
    const double *w;          /* [w_iters][M] or NULL */
    int w_iters;
    uint8_t *out_bits;
    int32_t *out_iters;
    uint8_t *out_ok;
    double *out_llr;          /* [n_cw][N*Z] or NULL */
    int cw_begin, cw_end, status;
} f64_job_t;

static void decode_one_f64(const f64_job_t *jb, int cw, double *L, double *R, double *x,
                           uint8_t *hd) {
    const graph_t *g = jb->g;
    const int Z = g->Z, NZ = g->N * g->Z, E = g->row_ptr[g->M];
    const int T = (g->N - g->n_punct) * Z;
    const double *b = jb->llr + (size_t)cw * T;
    for (int j = 0; j < g->n_punct * Z; ++j) L[j] = 0.0;
    for (int i = 0; i < T; ++i) L[g->n_punct * Z + i] = b[i];
    for (size_t i = 0; i < (size_t)E * Z; ++i) R[i] = 0.0;

    int iters = jb->max_iter, ok = 0;
    for (int t = 1; t <= jb->max_iter; ++t) {
        for (int r = 0; r < g->M; ++r) {
            const int e0 = g->row_ptr[r], w_r = g->row_ptr[r + 1] - e0;
            double w = jb->beta;
            if (jb->w) {
                int ti = t <= jb->w_iters ? t : jb->w_iters;
                w = jb->w[(size_t)(ti - 1) * g->M + r];
            }
            for (int z = 0; z < Z; ++z) {
                double m1 = INFINITY, m2 = INFINITY;
                int k1 = -1, S = 0;
                for (int k = 0; k < w_r; ++k) {
                    const int v = var_of(g, e0 + k, z);
                    x[k] = L[v] - R[(size_t)(e0 + k) * Z + z];
                    const double a = fabs(x[k]);
                    if (a < m1) { m2 = m1; m1 = a; k1 = k; }
                    else if (a < m2) { m2 = a; }
                    S ^= signbit(x[k]) ? 1 : 0;
                }
                double a1 = m1 - jb->delta, a2 = m2 - jb->delta;
                a1 = w * (a1 > 0.0 ? a1 : 0.0);
                a2 = w * (a2 > 0.0 ? a2 : 0.0);
                for (int k = 0; k < w_r; ++k) {
                    const int v = var_of(g, e0 + k, z);
                    const double mag = (k == k1) ? a2 : a1;
                    const int neg = S ^ (signbit(x[k]) ? 1 : 0);
                    const double rn = neg ? -mag : mag;
                    R[(size_t)(e0 + k) * Z + z] = rn;
                    L[v] = x[k] + rn;
                }
            }
        }
        if (jb->early_exit || t == jb->max_iter) {
            for (int j = 0; j < NZ; ++j) hd[j] = L[j] < 0.0;
            const int holds = all_checks_hold(g, hd);
            if (jb->early_exit && holds) { iters = t; ok = 1; break; }
            if (t == jb->max_iter) ok = holds;
        }
    }
    for (int j = 0; j < NZ; ++j) hd[j] = L[j] < 0.0;
    pack_bits(hd, jb->kb_bits, jb->out_bits + (size_t)cw * ((jb->kb_bits + 7) / 8));
    jb->out_iters[cw] = iters;
    if (jb->out_ok) jb->out_ok[cw] = (uint8_t)ok;
    if (jb->out_llr) memcpy(jb->out_llr + (size_t)cw * NZ, L, sizeof(double) * (size_t)NZ);
}

static void *f64_worker(void *arg) {
    f64_job_t *jb = (f64_job_t *)arg;
    const graph_t *g = jb->g;
    const size_t NZ = (size_t)g->N * g->Z, EZ = (size_t)g->row_ptr[g->M] * g->Z;
    double *L = malloc(sizeof(double) * NZ), *R = malloc(sizeof(double) * EZ);
    double *x = malloc(sizeof(double) * (size_t)max_row_weight(g));
    uint8_t *hd = malloc(NZ);
    if (!L || !R || !x || !hd) { jb->status = ORACLE_ENOMEM; goto out; }
    for (int cw = jb->cw_begin; cw < jb->cw_end; ++cw) decode_one_f64(jb, cw, L, R, x, hd);
    jb->status = ORACLE_OK;
out:
    free(L); free(R); free(x); free(hd);
    return NULL;
}

int oracle_decode_f64(int M, int N, int Z, int n_punct, int K,
                      const int32_t *row_ptr, const int16_t *col, const int16_t *shift,
                      int n_cw, const double *llr, int max_iter, int early_exit,
                      double beta, double delta, const double *w, int w_iters,
                      uint8_t *out_bits, int32_t *out_iters, uint8_t *out_ok, double *out_llr,
                      int n_threads) {
    graph_t g = {M, N, Z, n_punct, row_ptr, col, shift};
    if (!graph_check(&g) || n_cw < 0 || max_iter < 1 || K < 0 || K > N * Z ||
        (n_cw > 0 && (!llr || !out_bits || !out_iters)) || (w && w_iters < 1))
        return ORACLE_EINVAL;
    if (n_cw == 0) return ORACLE_OK;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > n_cw) n_threads = n_cw;
    f64_job_t *jobs = calloc((size_t)n_threads, sizeof(f64_job_t));
    if (!jobs) return ORACLE_ENOMEM;
    for (int i = 0; i < n_threads; ++i) {
        f64_job_t *jb = &jobs[i];
        jb->g = &g; jb->kb_bits = K; jb->llr = llr; jb->n_cw = n_cw; jb->max_iter = max_iter;
        jb->early_exit = early_exit; jb->beta = beta; jb->delta = delta; jb->w = w;
        jb->w_iters = w_iters; jb->out_bits = out_bits; jb->out_iters = out_iters;
        jb->out_ok = out_ok; jb->out_llr = out_llr;
        jb->cw_begin = (int)((long long)n_cw * i / n_threads);
        jb->cw_end = (int)((long long)n_cw * (i + 1) / n_threads);
        jb->status = ORACLE_OK;
    }
    run_threads(jobs, sizeof(f64_job_t), n_threads, f64_worker);
    int status = ORACLE_OK;
    for (int i = 0; i < n_threads; ++i)
        if (jobs[i].status != ORACLE_OK) status = jobs[i].status;
    free(jobs);
    return status;
}

/* ------------------------------------------------------------------ */
/* Check rules and schedules for context (double precision)            */
/* ------------------------------------------------------------------ */
/*
 * The decoder's method is the normalised min-sum approximation of belief
 * propagation on the layered schedule (§III). For context on what those two
 * choices cost, this routine also runs
 *   rule BP_SPA   -- the sum-product check rule of §III: the message to edge
 *                    k is 2 atanh(prod_{j != k} tanh(x_j / 2)), the product
 *                    taken directly (|product| kept at most the largest
 *                    double below 1, so a message is at most about 36.7;
 *                    the true value is then within 1e-15 of a hard decision);
 *   rule BP_MINSUM -- the normalised min-sum of the double mode (beta);
 *   schedule BP_LAYERED  -- block rows in order, each row reading the
 *                    posteriors the previous rows left (§III layered);
 *   schedule BP_FLOODING -- every check row of an iteration reads the
 *                    posteriors of the previous iteration; afterwards each
 *                    posterior is its channel LLR plus all its incoming
 *                    check-to-variable messages (§III flooding).
 * Same stopping rule, outputs and no clamping as the double mode.
 */
#define BP_MINSUM 0
#define BP_SPA 1
#define BP_LAYERED 0
#define BP_FLOODING 1

typedef struct {
    const graph_t *g;
    int kb_bits;
    const double *llr;
    int n_cw, max_iter, early_exit, rule, schedule;
    double beta;
    uint8_t *out_bits;
    int32_t *out_iters;
    uint8_t *out_ok;
    double *out_llr;
    int cw_begin, cw_end, status;
} bp_job_t;

/* New check-to-variable messages rn[0..w) of one check row from its
 * variable-to-check messages x[0..w). */
static void check_rule(int rule, double beta, const double *x, int w, double *rn) {
    if (rule == BP_SPA) {
        const double pmax = nextafter(1.0, 0.0);
        for (int k = 0; k < w; ++k) {
            double p = 1.0;
            for (int j = 0; j < w; ++j)
                if (j != k) p *= tanh(x[j] / 2.0);
            if (p > pmax) p = pmax;
            if (p < -pmax) p = -pmax;
            rn[k] = 2.0 * atanh(p);
        }
        return;
    }
    double m1 = INFINITY, m2 = INFINITY;
    int k1 = -1, S = 0;
    for (int k = 0; k < w; ++k) {
        const double a = fabs(x[k]);
        if (a < m1) { m2 = m1; m1 = a; k1 = k; }
        else if (a < m2) { m2 = a; }
        S ^= signbit(x[k]) ? 1 : 0;
    }
    for (int k = 0; k < w; ++k) {
        const double mag = beta * ((k == k1) ? m2 : m1);
        rn[k] = (S ^ (signbit(x[k]) ? 1 : 0)) ? -mag : mag;
    }
}

static void decode_one_bp(const bp_job_t *jb, int cw, double *L, double *Lch, double *R,
                          double *x, double *rn, uint8_t *hd) {
    const graph_t *g = jb->g;
    const int Z = g->Z, NZ = g->N * g->Z, E = g->row_ptr[g->M];
    const int T = (g->N - g->n_punct) * Z;
    const double *b = jb->llr + (size_t)cw * T;
    for (int j = 0; j < g->n_punct * Z; ++j) Lch[j] = 0.0;
    for (int i = 0; i < T; ++i) Lch[g->n_punct * Z + i] = b[i];
    memcpy(L, Lch, sizeof(double) * (size_t)NZ);
    for (size_t i = 0; i < (size_t)E * Z; ++i) R[i] = 0.0;

    int iters = jb->max_iter, ok = 0;
    for (int t = 1; t <= jb->max_iter; ++t) {
        for (int r = 0; r < g->M; ++r) {
            const int e0 = g->row_ptr[r], w_r = g->row_ptr[r + 1] - e0;
            for (int z = 0; z < Z; ++z) {
                for (int k = 0; k < w_r; ++k)
                    x[k] = L[var_of(g, e0 + k, z)] - R[(size_t)(e0 + k) * Z + z];
                check_rule(jb->rule, jb->beta, x, w_r, rn);
                for (int k = 0; k < w_r; ++k) {
                    R[(size_t)(e0 + k) * Z + z] = rn[k];
                    /* layered: the posterior takes the new message at once */
                    if (jb->schedule == BP_LAYERED) L[var_of(g, e0 + k, z)] = x[k] + rn[k];
                }
            }
        }
        if (jb->schedule == BP_FLOODING) {
            /* every row read the previous iteration's posteriors; now each
             * posterior is its channel LLR plus all its new messages */
            memcpy(L, Lch, sizeof(double) * (size_t)NZ);
            for (int r = 0; r < g->M; ++r)
                for (int e = g->row_ptr[r]; e < g->row_ptr[r + 1]; ++e)
                    for (int z = 0; z < Z; ++z) L[var_of(g, e, z)] += R[(size_t)e * Z + z];
        }
        if (jb->early_exit || t == jb->max_iter) {
            for (int j = 0; j < NZ; ++j) hd[j] = L[j] < 0.0;
            const int holds = all_checks_hold(g, hd);
            if (jb->early_exit && holds) { iters = t; ok = 1; break; }
            if (t == jb->max_iter) ok = holds;
        }
    }
    for (int j = 0; j < NZ; ++j) hd[j] = L[j] < 0.0;
    pack_bits(hd, jb->kb_bits, jb->out_bits + (size_t)cw * ((jb->kb_bits + 7) / 8));
    jb->out_iters[cw] = iters;
    if (jb->out_ok) jb->out_ok[cw] = (uint8_t)ok;
    if (jb->out_llr) memcpy(jb->out_llr + (size_t)cw * NZ, L, sizeof(double) * (size_t)NZ);
}

static void *bp_worker(void *arg) {
    bp_job_t *jb = (bp_job_t *)arg;
    const graph_t *g = jb->g;
    const size_t NZ = (size_t)g->N * g->Z, EZ = (size_t)g->row_ptr[g->M] * g->Z;
    const size_t W = (size_t)max_row_weight(g);
    double *L = malloc(sizeof(double) * NZ), *Lch = malloc(sizeof(double) * NZ);
    double *R = malloc(sizeof(double) * EZ);
    double *x = malloc(sizeof(double) * W), *rn = malloc(sizeof(double) * W);
    uint8_t *hd = malloc(NZ);
    if (!L || !Lch || !R || !x || !rn || !hd) { jb->status = ORACLE_ENOMEM; goto out; }
    for (int cw = jb->cw_begin; cw < jb->cw_end; ++cw) decode_one_bp(jb, cw, L, Lch, R, x, rn, hd);
    jb->status = ORACLE_OK;
out:
    free(L); free(Lch); free(R); free(x); free(rn); free(hd);
    return NULL;
}

int oracle_decode_bp_f64(int M, int N, int Z, int n_punct, int K,
                         const int32_t *row_ptr, const int16_t *col, const int16_t *shift,
                         int n_cw, const double *llr, int max_iter, int early_exit, int rule,
                         int schedule, double beta, uint8_t *out_bits, int32_t *out_iters,
                         uint8_t *out_ok, double *out_llr, int n_threads) {
    graph_t g = {M, N, Z, n_punct, row_ptr, col, shift};
    if (!graph_check(&g) || n_cw < 0 || max_iter < 1 || K < 0 || K > N * Z ||
        (rule != BP_MINSUM && rule != BP_SPA) ||
        (schedule != BP_LAYERED && schedule != BP_FLOODING) ||
        (n_cw > 0 && (!llr || !out_bits || !out_iters)))
        return ORACLE_EINVAL;
    if (n_cw == 0) return ORACLE_OK;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > n_cw) n_threads = n_cw;
    bp_job_t *jobs = calloc((size_t)n_threads, sizeof(bp_job_t));
    if (!jobs) return ORACLE_ENOMEM;
    for (int i = 0; i < n_threads; ++i) {
        bp_job_t *jb = &jobs[i];
        jb->g = &g; jb->kb_bits = K; jb->llr = llr; jb->n_cw = n_cw; jb->max_iter = max_iter;
        jb->early_exit = early_exit; jb->rule = rule; jb->schedule = schedule; jb->beta = beta;
        jb->out_bits = out_bits; jb->out_iters = out_iters; jb->out_ok = out_ok;
        jb->out_llr = out_llr;
        jb->cw_begin = (int)((long long)n_cw * i / n_threads);
        jb->cw_end = (int)((long long)n_cw * (i + 1) / n_threads);
        jb->status = ORACLE_OK;
    }
    run_threads(jobs, sizeof(bp_job_t), n_threads, bp_worker);
    int status = ORACLE_OK;
    for (int i = 0; i < n_threads; ++i)
        if (jobs[i].status != ORACLE_OK) status = jobs[i].status;
    free(jobs);
    return status;
}

/* ------------------------------------------------------------------ */
/* Learned (neural) weighted min-sum: loss and exact gradient, double  */
/* ------------------------------------------------------------------ */
/*
 * Forward: the layered min-sum of the double mode with one multiplier per
 * (iteration t, block row r), w[t][r], no offset, no early exit, n_iter
 * iterations. Posterior after iteration t: L_t. With y = L_t / scale (scale
 * converts the LLR units to natural-log units) and p = sigmoid(-y) =
 * P(bit = 1), the loss of a codeword c is
 *     loss = sum_t lambda_t * (1/(N*Z)) * sum_j BCE(p_tj, c_j),
 * with per-iteration loss weights lambda_t (iter_w; NULL: 1/n_iter each),
 * BCE(p, c) = -(c log p + (1 - c) log(1 - p)); dBCE/dL = (c - p) / scale.
 *
 * Backward (reverse of the layered schedule). Each check-row update
 *     x_k = L_k - R_k,  m1 = |x_k1|, m2 = |x_k2|  (k1 = first argmin,
 *     k2 = first argmin over k != k1),  R'_k = s_k * w * (k == k1 ? m2 : m1)
 *     with s_k the product of sgn(x_j) over j != k,  L'_k = x_k + R'_k
 * is differentiated with the signs and argmins held fixed (they are
 * piecewise constant): with gL' and gR' the gradients of the new L_k and
 * R_k, g_k = (gL'_k + gR'_k) * s_k, then
 *     dw += sum_k g_k * (k == k1 ? m2 : m1),
 *     gx_k = gL'_k + [k == k1] sgn(x_k1) w sum_{j != k1} g_j
 *                  + [k == k2] sgn(x_k2) w g_k1,
 * and the old values get gL_k = gx_k, gR_k = -gx_k. sgn(x) = -1 iff the
 * sign bit of x is set.
 */
static inline double sgn_bit(double v) { return signbit(v) ? -1.0 : 1.0; }

static double softplus(double v) { return v > 0 ? v + log1p(exp(-v)) : log1p(exp(v)); }

int oracle_nwms_grad_f64(int M, int N, int Z, int n_punct,
                         const int32_t *row_ptr, const int16_t *col, const int16_t *shift,
                         int n_cw, const double *llr, const uint8_t *cbits, int n_iter,
                         const double *w, const double *iter_w, double scale, double *loss,
                         double *grad_w) {
    graph_t g = {M, N, Z, n_punct, row_ptr, col, shift};
    if (!graph_check(&g) || n_cw < 1 || n_iter < 1 || !llr || !cbits || !w || !loss ||
        !grad_w || !(scale > 0))
        return ORACLE_EINVAL;
    const int NZ = N * Z, E = row_ptr[M], T = (N - n_punct) * Z;
    const int wmax = max_row_weight(&g);
    double *L = malloc(sizeof(double) * NZ);
    double *R = malloc(sizeof(double) * (size_t)E * Z);
    double *X = malloc(sizeof(double) * (size_t)n_iter * E * Z);  /* tape of x */
    double *Lt = malloc(sizeof(double) * (size_t)n_iter * NZ);    /* posteriors per iteration */
    double *gL = malloc(sizeof(double) * NZ);
    double *gR = malloc(sizeof(double) * (size_t)E * Z);
    double *gk = malloc(sizeof(double) * (size_t)wmax);
    if (!L || !R || !X || !Lt || !gL || !gR || !gk) {
        free(L); free(R); free(X); free(Lt); free(gL); free(gR); free(gk);
        return ORACLE_ENOMEM;
    }
    for (int i = 0; i < n_iter * M; ++i) grad_w[i] = 0.0;
    for (int cw = 0; cw < n_cw; ++cw) {
        const double *b = llr + (size_t)cw * T;
        const uint8_t *c = cbits + (size_t)cw * NZ;
        for (int j = 0; j < n_punct * Z; ++j) L[j] = 0.0;
        for (int i = 0; i < T; ++i) L[n_punct * Z + i] = b[i];
        for (size_t i = 0; i < (size_t)E * Z; ++i) R[i] = 0.0;
        /* forward */
        for (int t = 0; t < n_iter; ++t) {
            for (int r = 0; r < M; ++r) {
                const int e0 = row_ptr[r], wr = row_ptr[r + 1] - e0;
                const double wt = w[(size_t)t * M + r];
                for (int z = 0; z < Z; ++z) {
                    double *x = X + ((size_t)t * E + e0) * Z;  /* x of edge e0+k at x[k*Z+z] */
                    double m1 = INFINITY, m2 = INFINITY;
                    int k1 = -1, S = 0;
                    for (int k = 0; k < wr; ++k) {
                        const double xv = L[var_of(&g, e0 + k, z)] - R[(size_t)(e0 + k) * Z + z];
                        x[(size_t)k * Z + z] = xv;
                        const double a = fabs(xv);
                        if (a < m1) { m2 = m1; m1 = a; k1 = k; }
                        else if (a < m2) { m2 = a; }
                        S ^= signbit(xv) ? 1 : 0;
                    }
                    for (int k = 0; k < wr; ++k) {
                        const double xv = x[(size_t)k * Z + z];
                        const double mag = wt * ((k == k1) ? m2 : m1);
                        const int neg = S ^ (signbit(xv) ? 1 : 0);
                        const double rn = neg ? -mag : mag;
                        R[(size_t)(e0 + k) * Z + z] = rn;
                        L[var_of(&g, e0 + k, z)] = xv + rn;
                    }
                }
            }
            memcpy(Lt + (size_t)t * NZ, L, sizeof(double) * NZ);
        }
        /* loss */
        double lsum = 0.0;
        for (int t = 0; t < n_iter; ++t) {
            const double lam = iter_w ? iter_w[t] : 1.0 / n_iter;
            double st = 0.0;
            for (int j = 0; j < NZ; ++j) {
                const double y = Lt[(size_t)t * NZ + j] / scale;
                st += c[j] ? softplus(y) : softplus(-y);
            }
            lsum += lam * st;
        }
        loss[cw] = lsum / NZ;
        /* backward */
        for (int j = 0; j < NZ; ++j) gL[j] = 0.0;
        for (size_t i = 0; i < (size_t)E * Z; ++i) gR[i] = 0.0;
        for (int t = n_iter - 1; t >= 0; --t) {
            const double coef = (iter_w ? iter_w[t] : 1.0 / n_iter) / ((double)NZ * scale);
            for (int j = 0; j < NZ; ++j) {
                const double y = Lt[(size_t)t * NZ + j] / scale;
                const double p = 1.0 / (1.0 + exp(y)); /* sigmoid(-y) */
                gL[j] += (c[j] - p) * coef;
            }
            for (int r = M - 1; r >= 0; --r) {
                const int e0 = row_ptr[r], wr = row_ptr[r + 1] - e0;
                const double wt = w[(size_t)t * M + r];
                double gw = 0.0;
                for (int z = 0; z < Z; ++z) {
                    const double *x = X + ((size_t)t * E + e0) * Z;
                    double m1 = INFINITY, m2 = INFINITY;
                    int k1 = -1, k2 = -1, S = 0;
                    for (int k = 0; k < wr; ++k) {
                        const double a = fabs(x[(size_t)k * Z + z]);
                        if (a < m1) { m2 = m1; k2 = k1; m1 = a; k1 = k; }
                        else if (a < m2) { m2 = a; k2 = k; }
                        S ^= signbit(x[(size_t)k * Z + z]) ? 1 : 0;
                    }
                    double gsum_not_k1 = 0.0;
                    for (int k = 0; k < wr; ++k) {
                        const double xv = x[(size_t)k * Z + z];
                        const int v = var_of(&g, e0 + k, z);
                        const size_t er = (size_t)(e0 + k) * Z + z;
                        const double sk = (S ^ (signbit(xv) ? 1 : 0)) ? -1.0 : 1.0;
                        gk[k] = (gL[v] + gR[er]) * sk;
                        gw += gk[k] * ((k == k1) ? m2 : m1);
                        if (k != k1) gsum_not_k1 += gk[k];
                    }
                    for (int k = 0; k < wr; ++k) {
                        const double xv = x[(size_t)k * Z + z];
                        const int v = var_of(&g, e0 + k, z);
                        const size_t er = (size_t)(e0 + k) * Z + z;
                        double gx = gL[v];
                        if (k == k1) gx += sgn_bit(xv) * wt * gsum_not_k1;
                        if (k == k2) gx += sgn_bit(xv) * wt * gk[k1];
                        gL[v] = gx;
                        gR[er] = -gx;
                    }
                }
                grad_w[(size_t)t * M + r] += gw;
            }
        }
    }
    free(L); free(R); free(X); free(Lt); free(gL); free(gR); free(gk);
    return ORACLE_OK;
}
