/*
 * CPU oracle of the chain-rule sampler, C tier (TEST INFRASTRUCTURE).
 *
 * Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py
 * load this library.  It shares no code with the GPU library.  The same
 * algorithm as oracle/sampler.py, written out in plain C with OpenMP over
 * samples, for sizes the Python tier cannot reach; it is checked against it.
 *
 * Bits are numbered 1..M in sampling order (bit n is mode n-1).  With
 * gamma_A = kappa(A) chi(A), chi(A) = (-1)^(sum x_i), the joint probability of
 * the first n bits is expanded in the parity cumulants up to order K
 * (Sec. II, Eq. samplecumulant; App. B, Eq. probs_corr_cumulants_3):
 *   single elision, K = 3: Eq. methprob (p), Eq. b (p1), Eq. a (p+);
 *   double elision, K = 5: Eq. probade (p), Eq. probpartialade (p+),
 *                          Eq. probelidedade (p1), Eq. probdoubleelidedade (p2).
 * Marginal tables (all tops): p(a); p1(a, e), e < a; p2(a, e, d), d < e < a;
 * p+(b, a), a <= b.  Traced-out top variables reduce: p1(a, a) = p(a - 1),
 * p2(a, a, d) = p1(a - 1, d); p+(b, a) = 1 for b < a.
 * x_n = 1 iff u_n < p(x_n = 1, x_<n) / p(n - 1) (1/2 when p(n - 1) <= 0).
 * Sums are Neumaier-compensated, FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double s, c; } acc_t;
static void acc_add(acc_t* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double acc_val(const acc_t* a) { return a->s + a->c; }

typedef struct {
    int M, K;
    const double* cum;  /* parity cumulants, library layout */
    int64_t off[7];     /* order offsets */
    int64_t* bin;       /* C(n, k) at bin[k * (M + 1) + n] */
    /* tables of one sample */
    double* P0;
    double* P1;
    double* P2;
    double* PP;
    const uint8_t* x;   /* bits, x[1..M] */
} sctx;

static int64_t C(const sctx* c, int n, int k) {
    if (n < k || n < 0) return 0;
    return c->bin[k * (c->M + 1) + n];
}

/* kappa of the bits given in decreasing order (b[0] > b[1] > ...) */
static double kap(const sctx* c, int d, const int* b) {
    int64_t r = 0;
    for (int j = 0; j < d; ++j) r += C(c, b[d - 1 - j] - 1, j + 1);
    return c->cum[c->off[d] + r];
}

static double chi(const sctx* c, int d, const int* b) {
    int s = 0;
    for (int j = 0; j < d; ++j) s ^= c->x[b[j]];
    return s ? -1.0 : 1.0;
}

static double gam(const sctx* c, int d, const int* b) { return kap(c, d, b) * chi(c, d, b); }

static int64_t i1(int a, int e) { return (int64_t)(a - 1) * (a - 2) / 2 + (e - 1); }
static int64_t i2(const sctx* c, int a, int e, int d) { return C(c, a - 1, 3) + C(c, e - 1, 2) + (d - 1); }
static int64_t ip(int b, int a) { return (int64_t)b * (b - 1) / 2 + (a - 1); }

static double p0(const sctx* c, int a) { return c->P0[a]; }
static double p1(const sctx* c, int a, int e) { return e == a ? p0(c, a - 1) : c->P1[i1(a, e)]; }
static double p2(const sctx* c, int a, int e, int d) {
    return e == a ? p1(c, a - 1, d) : c->P2[i2(c, a, e, d)];
}
static double pp(const sctx* c, int b, int a) { return b < a ? 1.0 : c->PP[ip(b, a)]; }

static void sort3(int* v) {
    for (int i = 1; i < 3; ++i)
        for (int j = i; j > 0 && v[j - 1] < v[j]; --j) { int t = v[j]; v[j] = v[j - 1]; v[j - 1] = t; }
}

/* p(x_n, ..., x_1) with the current bits */
static double single_p(const sctx* c, int n) {
    acc_t a = {0, 0};
    int b[3];
    b[0] = n;
    acc_add(&a, 0.5 * (1.0 + gam(c, 1, b)) * p0(c, n - 1));
    for (int i = 1; i < n; ++i) {
        b[0] = n; b[1] = i;
        acc_add(&a, 0.25 * gam(c, 2, b) * p1(c, n - 1, i));
    }
    for (int i = 1; i < n; ++i)
        for (int j = 1; j < i; ++j) {
            b[0] = n; b[1] = i; b[2] = j;
            acc_add(&a, 0.125 * gam(c, 3, b) * pp(c, n - 1, i + 1) * p1(c, i - 1, j));
        }
    return acc_val(&a);
}

static void single_update(sctx* c, int n, double pn) {
    int b[3];
    b[0] = n;
    const double h = 0.5 * (1.0 + gam(c, 1, b));
    for (int e = 1; e < n; ++e) {
        acc_t a = {0, 0};
        acc_add(&a, h * p1(c, n - 1, e));
        for (int i = 1; i < n; ++i) {
            if (i == e) continue;
            int lo = i < e ? i : e, hi = i < e ? e : i;
            b[0] = n; b[1] = i;
            acc_add(&a, 0.25 * gam(c, 2, b) * pp(c, n - 1, hi + 1) * p1(c, hi - 1, lo));
        }
        c->P1[i1(n, e)] = acc_val(&a);
    }
    for (int l = 1; l <= n; ++l) {
        acc_t a = {0, 0};
        acc_add(&a, h * pp(c, n - 1, l));
        for (int i = l; i < n; ++i) {
            b[0] = n; b[1] = i;
            acc_add(&a, 0.25 * gam(c, 2, b) * pp(c, n - 1, i + 1) * pp(c, i - 1, l));
        }
        c->PP[ip(n, l)] = acc_val(&a);
    }
    c->P0[n] = pn;
}

static double double_p(const sctx* c, int n) {
    acc_t a = {0, 0};
    int b[5];
    b[0] = n;
    acc_add(&a, 0.5 * (1.0 + gam(c, 1, b)) * p0(c, n - 1));
    for (int i = 1; i < n; ++i) {
        b[1] = i;
        acc_add(&a, 0.25 * gam(c, 2, b) * p1(c, n - 1, i));
    }
    for (int i = 2; i < n; ++i)
        for (int j = 1; j < i; ++j) {
            b[1] = i; b[2] = j;
            acc_add(&a, 0.125 * gam(c, 3, b) * p2(c, n - 1, i, j));
        }
    for (int i = 3; i < n; ++i)
        for (int j = 2; j < i; ++j)
            for (int k = 1; k < j; ++k) {
                b[1] = i; b[2] = j; b[3] = k;
                acc_add(&a, gam(c, 4, b) * pp(c, n - 1, i + 1) * p2(c, i - 1, j, k) / 16.0);
            }
    for (int i = 4; i < n; ++i)
        for (int j = 3; j < i; ++j)
            for (int k = 2; k < j; ++k)
                for (int l = 1; l < k; ++l) {
                    b[1] = i; b[2] = j; b[3] = k; b[4] = l;
                    acc_add(&a, gam(c, 5, b) * pp(c, n - 1, i + 1) * pp(c, i - 1, j + 1) *
                                    p2(c, j - 1, k, l) / 32.0);
                }
    return acc_val(&a);
}

static void double_update(sctx* c, int n, double pn) {
    int b[3];
    b[0] = n;
    const double h = 0.5 * (1.0 + gam(c, 1, b));
    for (int l = 1; l <= n; ++l) {
        acc_t a = {0, 0};
        acc_add(&a, h * pp(c, n - 1, l));
        for (int i = l; i < n; ++i) {
            b[0] = n; b[1] = i;
            acc_add(&a, 0.25 * gam(c, 2, b) * pp(c, n - 1, i + 1) * pp(c, i - 1, l));
        }
        for (int i = l + 1; i < n; ++i)
            for (int j = l; j < i; ++j) {
                b[0] = n; b[1] = i; b[2] = j;
                acc_add(&a, 0.125 * gam(c, 3, b) * pp(c, n - 1, i + 1) * pp(c, i - 1, j + 1) *
                                pp(c, j - 1, l));
            }
        c->PP[ip(n, l)] = acc_val(&a);
    }
    for (int e = 1; e < n; ++e) {
        acc_t a = {0, 0};
        acc_add(&a, h * p1(c, n - 1, e));
        for (int i = 1; i < n; ++i) {
            if (i == e) continue;
            int hi = i > e ? i : e, lo = i > e ? e : i;
            b[0] = n; b[1] = i;
            acc_add(&a, 0.25 * gam(c, 2, b) * p2(c, n - 1, hi, lo));
        }
        for (int i = 1; i < n; ++i)
            for (int j = 1; j < i; ++j) {
                if (i == e || j == e) continue;
                int o[3] = {i, j, e};
                sort3(o);
                b[0] = n; b[1] = i; b[2] = j;
                acc_add(&a, 0.125 * gam(c, 3, b) * pp(c, n - 1, o[0] + 1) * p2(c, o[0] - 1, o[1], o[2]));
            }
        c->P1[i1(n, e)] = acc_val(&a);
    }
    for (int e = 2; e < n; ++e)
        for (int d = 1; d < e; ++d) {
            acc_t a = {0, 0};
            acc_add(&a, h * p2(c, n - 1, e, d));
            for (int i = 1; i < n; ++i) {
                if (i == e || i == d) continue;
                int o[3] = {i, e, d};
                sort3(o);
                b[0] = n; b[1] = i;
                acc_add(&a, 0.25 * gam(c, 2, b) * pp(c, n - 1, o[0] + 1) * p2(c, o[0] - 1, o[1], o[2]));
            }
            c->P2[i2(c, n, e, d)] = acc_val(&a);
        }
    c->P0[n] = pn;
}

static int64_t binom_plain(int64_t n, int64_t k) {
    if (k < 0 || n < k) return 0;
    int64_t r = 1;
    for (int64_t i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

/*
 * nsamples samples of M bits.  cum: parity cumulants, orders 1..K (K = 3:
 * single elision, K = 5: double elision), library layout.  u: M x nsamples
 * uniforms, u[n * ldu + s] for bit n + 1 of sample s (ldu >= nsamples).
 * Outputs: bits[s * M + n]; prob[s] = p(x_M, ..., x_1) (may be NULL);
 * cond[n * ldu + s] = p(x_{n+1} = 1 | earlier bits) (may be NULL).  forced:
 * if non-NULL, bits to follow (s * M + n) instead of sampling.
 */
int oracle_sample(int M, const double* cum, int K, int64_t nsamples, const double* u, int64_t ldu,
                  const uint8_t* forced, uint8_t* bits, double* prob, double* cond, int threads) {
    if (M < 1 || M > 512 || (K != 3 && K != 5) || nsamples < 0) return 1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    int64_t* bin = (int64_t*)malloc(sizeof(int64_t) * 7 * (M + 1));
    if (!bin) return 3;
    for (int k = 0; k < 7; ++k)
        for (int n = 0; n <= M; ++n) bin[k * (M + 1) + n] = binom_plain(n, k);
    int64_t off[7] = {0};
    for (int d = 2; d <= 6; ++d) off[d] = off[d - 1] + (d - 1 <= M ? binom_plain(M, d - 1) : 0);
    const int64_t n1 = binom_plain(M, 2) + 1, n2 = binom_plain(M, 3) + 1, npp = binom_plain(M + 1, 2) + 1;
    int err = 0;
#pragma omp parallel reduction(| : err)
    {
        sctx c;
        c.M = M;
        c.K = K;
        c.cum = cum;
        memcpy(c.off, off, sizeof(off));
        c.bin = bin;
        c.P0 = (double*)malloc(sizeof(double) * (M + 1));
        c.P1 = (double*)malloc(sizeof(double) * n1);
        c.PP = (double*)malloc(sizeof(double) * npp);
        c.P2 = K == 5 ? (double*)malloc(sizeof(double) * n2) : NULL;
        uint8_t* x = (uint8_t*)malloc(M + 1);
        c.x = x;
        if (!c.P0 || !c.P1 || !c.PP || (K == 5 && !c.P2) || !x) {
            err |= 3;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t s = 0; s < nsamples; ++s) {
                c.P0[0] = 1.0;
                for (int n = 1; n <= M; ++n) {
                    x[n] = 1;
                    double pone = K == 3 ? single_p(&c, n) : double_p(&c, n);
                    double prev = c.P0[n - 1];
                    double q = prev > 0.0 ? pone / prev : 0.5;
                    if (cond) cond[(int64_t)(n - 1) * ldu + s] = q;
                    int xn = forced ? forced[s * M + (n - 1)] : (u[(int64_t)(n - 1) * ldu + s] < q);
                    x[n] = (uint8_t)xn;
                    bits[s * M + (n - 1)] = (uint8_t)xn;
                    double pn = xn ? pone : (K == 3 ? single_p(&c, n) : double_p(&c, n));
                    if (K == 3) single_update(&c, n, pn);
                    else double_update(&c, n, pn);
                }
                if (prob) prob[s] = c.P0[M];
            }
        }
        free(c.P0); free(c.P1); free(c.PP); free(c.P2); free(x);
    }
    free(bin);
    return err;
}
