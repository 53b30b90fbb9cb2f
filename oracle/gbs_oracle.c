/*
 * CPU oracle, C tier (TEST INFRASTRUCTURE).
 *
 * Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py
 * load this library.  It shares no code with the GPU library.
 *
 * Plain FP64 evaluation of the definitions, one subset at a time:
 *   p(T)  = det(Q_T)^(-1/2), Q = sigma + I/2, Q_T the rows/columns k, k+M for
 *           k in T (App. D.1, Eqs. vacuum_gaussian_prob, correlator_sum_cov,
 *           hbar = 1); the determinant is the squared product of a textbook
 *           Cholesky diagonal.  With first moments mu (the *_mu entry points)
 *           the same equation multiplies by exp(-|z|^2 / 2), z the forward
 *           substitution L z = mu_T with the same Cholesky factor L;
 *   mu(S) = sum_{T subset S} (-1)^|T| p(T)            (App. A.2, joint moments)
 *   c(S)  = (-1)^|S| sum_{T subset S} (-2)^|T| p(T)   (Eq. corre_cov_main)
 *   cumulant(S) = sum over set partitions pi of S of
 *           (-1)^(|pi|-1) (|pi|-1)! prod_{B in pi} moment(B)
 *                                                     (Eq. cumulant_corr_main)
 * Each subset recomputes every p(T), T subset S, from scratch; sums use
 * Neumaier compensation.  OpenMP distributes subsets over threads.
 *
 * Layout: order blocks d = 1..K, colex order inside a block.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KMAX 5
#define NMAX (2 * KMAX)

static int64_t binom(int64_t n, int64_t k) {
    if (k < 0 || n < k) return 0;
    int64_t r = 1;
    for (int64_t i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

/* colex unrank: the d-subset with rank r, ascending */
static void unrank(int d, int64_t r, int* s) {
    for (int j = d; j >= 1; --j) {
        int x = j - 1;
        while (binom(x + 1, j) <= r) ++x;
        s[j - 1] = x;
        r -= binom(x, j);
    }
}

static int64_t rank_of(int d, const int* s) {
    int64_t r = 0;
    for (int j = 0; j < d; ++j) r += binom(s[j], j + 1);
    return r;
}

typedef struct { double s, c; } nsum;
static void nadd(nsum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

/* p(T) for the subset of S selected by mask; Q is 2M x 2M row-major; mu is
 * the 2M first moments (xxpp) or NULL for the zero-mean state */
static int vacuum_prob(const double* Q, const double* mu, int M, const int* S, int d,
                       unsigned mask, double* out) {
    int idx[NMAX];
    int n = 0;
    for (int k = 0; k < d; ++k) if (mask & (1u << k)) idx[n++] = S[k];
    int h = n;
    for (int k = 0; k < h; ++k) idx[n++] = idx[k] + M;
    if (n == 0) { *out = 1.0; return 0; }
    double A[NMAX][NMAX];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[i][j] = Q[(int64_t)idx[i] * 2 * M + idx[j]];
    double prod = 1.0;
    for (int j = 0; j < n; ++j) {
        double s = A[j][j];
        for (int k = 0; k < j; ++k) s -= A[j][k] * A[j][k];
        if (!(s > 0.0)) return 2;
        double l = sqrt(s);
        A[j][j] = l;
        prod *= l;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i][j];
            for (int k = 0; k < j; ++k) t -= A[i][k] * A[j][k];
            A[i][j] = t / l;
        }
    }
    double e = 1.0;
    if (mu) {
        double z[NMAX];
        double q = 0.0;
        for (int i = 0; i < n; ++i) {
            double t = mu[idx[i]];
            for (int k = 0; k < i; ++k) t -= A[i][k] * z[k];
            z[i] = t / A[i][i];
            q += z[i] * z[i];
        }
        e = exp(-0.5 * q);
    }
    *out = e / prod;
    return 0;
}

/* set partitions of {0..d-1}: block label per element (restricted growth) */
typedef struct { int n; int nblocks[64]; unsigned blocks[64][KMAX]; } partitions;
static partitions g_parts[KMAX + 1];
static int g_parts_ready = 0;

static void gen_parts(int d, int i, int* lab, int nb, partitions* P) {
    if (i == d) {
        int id = P->n++;
        P->nblocks[id] = nb;
        for (int b = 0; b < nb; ++b) P->blocks[id][b] = 0;
        for (int k = 0; k < d; ++k) P->blocks[id][lab[k]] |= 1u << k;
        return;
    }
    for (int b = 0; b <= nb; ++b) {
        lab[i] = b;
        gen_parts(d, i + 1, lab, b + 1 > nb ? b + 1 : nb, P);
    }
}

static void init_parts(void) {
    if (g_parts_ready) return;
    for (int d = 1; d <= KMAX; ++d) {
        int lab[KMAX];
        g_parts[d].n = 0;
        gen_parts(d, 0, lab, 0, &g_parts[d]);
    }
    g_parts_ready = 1;
}

static double weight(int nb) {
    double f = 1.0;
    for (int i = 2; i < nb; ++i) f *= i;
    return (nb % 2 == 1) ? f : -f;  /* (-1)^(nb-1) (nb-1)! */
}

static int popc(unsigned x) { int c = 0; while (x) { c += x & 1u; x >>= 1; } return c; }

/* correlator and cumulant of one subset S (ascending, size d).  When smu and
 * skap are not NULL they receive the summand magnitudes of the two sums:
 *   smu  = sum_{T subset S} |w_T| p(T)  (w_T = (-1)^|T| or (-2)^|T|),
 *   skap = sum_pi |w(pi)| prod_{B in pi} |m(B)|,
 * the scales against which the rounding of an FP64 evaluation is measured. */
static int subset_values(const double* Q, const double* mu, int M, const int* S, int d,
                         int convention, double* corr, double* cum, double* smu,
                         double* skap) {
    double p[1 << KMAX];
    double m[1 << KMAX];
    int full = (1 << d) - 1;
    for (unsigned T = 0; T <= (unsigned)full; ++T) {
        int rc = vacuum_prob(Q, mu, M, S, d, T, &p[T]);
        if (rc) return rc;
    }
    double mag = 0.0;
    for (unsigned B = 1; B <= (unsigned)full; ++B) {
        nsum acc = {0.0, 0.0};
        for (unsigned T = 0; T <= B; ++T) {
            if ((T & B) != T) continue;
            int t = popc(T);
            double term;
            if (convention == 0) term = (t % 2 ? -1.0 : 1.0) * p[T];
            else term = ldexp((t % 2 ? -1.0 : 1.0), t) * p[T];
            nadd(&acc, term);
            if (B == (unsigned)full) mag += fabs(term);
        }
        double v = nval(&acc);
        if (convention != 0 && (popc(B) % 2)) v = -v;
        m[B] = v;
    }
    const partitions* P = &g_parts[d];
    nsum acc = {0.0, 0.0};
    double kmag = 0.0;
    for (int i = 0; i < P->n; ++i) {
        double prod = weight(P->nblocks[i]);
        for (int b = 0; b < P->nblocks[i]; ++b) prod *= m[P->blocks[i][b]];
        nadd(&acc, prod);
        kmag += fabs(prod);
    }
    *corr = m[full];
    *cum = nval(&acc);
    if (smu) *smu = mag;
    if (skap) *skap = kmag;
    return 0;
}

static double* make_q(const double* sigma, int M) {
    int64_t n = 2 * (int64_t)M;
    double* Q = (double*)malloc(sizeof(double) * n * n);
    if (!Q) return NULL;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            /* symmetric input; read the lower triangle */
            double v = (i >= j) ? sigma[i * n + j] : sigma[j * n + i];
            Q[i * n + j] = v + (i == j ? 0.5 : 0.0);
        }
    return Q;
}

int oracle_threads(int requested) {
#ifdef _OPENMP
    if (requested > 0) omp_set_num_threads(requested);
    return omp_get_max_threads();
#else
    (void)requested;
    return 1;
#endif
}

/* mu: 2M first moments (xxpp), or NULL for the zero-mean state */
int oracle_forward_sample_mu(int M, const double* sigma, const double* mu, int d,
                             const int64_t* ranks, int64_t n, int convention, double* corr,
                             double* cum, int threads) {
    if (M < 1 || d < 1 || d > KMAX || d > M) return 1;
    init_parts();
    oracle_threads(threads);
    double* Q = make_q(sigma, M);
    if (!Q) return 3;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : err)
    for (int64_t i = 0; i < n; ++i) {
        int S[KMAX];
        unrank(d, ranks[i], S);
        err |= subset_values(Q, mu, M, S, d, convention, &corr[i], &cum[i], NULL, NULL);
    }
    free(Q);
    return err;
}

int oracle_forward_sample(int M, const double* sigma, int d, const int64_t* ranks, int64_t n,
                          int convention, double* corr, double* cum, int threads) {
    return oracle_forward_sample_mu(M, sigma, NULL, d, ranks, n, convention, corr, cum, threads);
}

int oracle_forward_mu(int M, const double* sigma, const double* mu, int K, int convention,
                      double* corr, double* cum, int threads) {
    if (M < 1 || K < 1 || K > KMAX || K > M) return 1;
    init_parts();
    oracle_threads(threads);
    double* Q = make_q(sigma, M);
    if (!Q) return 3;
    int err = 0;
    int64_t off = 0;
    for (int d = 1; d <= K; ++d) {
        int64_t cnt = binom(M, d);
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : err)
        for (int64_t r = 0; r < cnt; ++r) {
            int S[KMAX];
            unrank(d, r, S);
            err |= subset_values(Q, mu, M, S, d, convention, &corr[off + r], &cum[off + r], NULL,
                                 NULL);
        }
        off += cnt;
    }
    free(Q);
    return err;
}

int oracle_forward(int M, const double* sigma, int K, int convention, double* corr,
                   double* cum, int threads) {
    return oracle_forward_mu(M, sigma, NULL, K, convention, corr, cum, threads);
}

/* One contiguous colex rank range of one order: the order-d subsets with ranks
 * rank0 .. rank0 + count - 1, in rank order, so that a full workload can be
 * streamed through bounded host buffers.  smu and skap (either may be NULL)
 * receive the summand magnitudes described at subset_values. */
int oracle_forward_range_mu(int M, const double* sigma, const double* mu, int d, int64_t rank0,
                            int64_t count, int convention, double* corr, double* cum,
                            double* smu, double* skap, int threads) {
    if (M < 1 || d < 1 || d > KMAX || d > M || rank0 < 0 || count < 0 ||
        rank0 + count > binom(M, d))
        return 1;
    init_parts();
    oracle_threads(threads);
    double* Q = make_q(sigma, M);
    if (!Q) return 3;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : err)
    for (int64_t i = 0; i < count; ++i) {
        int S[KMAX];
        unrank(d, rank0 + i, S);
        err |= subset_values(Q, mu, M, S, d, convention, &corr[i], &cum[i], smu ? &smu[i] : NULL,
                             skap ? &skap[i] : NULL);
    }
    free(Q);
    return err;
}

/* Summand magnitudes (see subset_values) of the sampled order-d subsets: the
 * scales of the stated FP64 tolerances. */
int oracle_tolerance_scale_mu(int M, const double* sigma, const double* mu, int d,
                              const int64_t* ranks, int64_t n, int convention, double* smu,
                              double* skap, int threads) {
    if (M < 1 || d < 1 || d > KMAX || d > M) return 1;
    init_parts();
    oracle_threads(threads);
    double* Q = make_q(sigma, M);
    if (!Q) return 3;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : err)
    for (int64_t i = 0; i < n; ++i) {
        int S[KMAX];
        double c, k;
        unrank(d, ranks[i], S);
        err |= subset_values(Q, mu, M, S, d, convention, &c, &k, &smu[i], &skap[i]);
    }
    free(Q);
    return err;
}

/* inverse of the SPD matrix Q_T (n x n) by Gauss-Jordan without pivoting */
static int spd_inverse(double A[NMAX][NMAX], int n, double Inv[NMAX][NMAX]) {
    double W[NMAX][2 * NMAX];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j) W[i][j] = (j < n) ? A[i][j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        double piv = W[c][c];
        if (!(piv > 0.0)) return 2;
        for (int j = 0; j < 2 * n; ++j) W[c][j] /= piv;
        for (int i = 0; i < n; ++i) {
            if (i == c) continue;
            double f = W[i][c];
            for (int j = 0; j < 2 * n; ++j) W[i][j] -= f * W[c][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Inv[i][j] = W[i][n + j];
    return 0;
}

/*
 * L = sum_{|S| <= K} (kappa~(S) - target(S))^2 and dL/dsigma (entries treated as
 * independent, symmetric result), by hand-written reverse mode of the click path:
 *   kbar(S)  = 2 (kappa~(S) - target(S))
 *   mubar(B) += kbar(S) w(pi) prod_{B' in pi, B' != B} mu(B')   for B in pi, pi of S
 *   pbar(T)  = (-1)^|T| sum_{B superset of T} mubar(B)
 *   dL/dQ_T += -pbar(T) p(T) Q_T^{-1} / 2
 */
int oracle_loss_grad(int M, const double* sigma, int K, const double* target, double* loss,
                     double* grad, int threads) {
    if (M < 1 || K < 1 || K > KMAX || K > M) return 1;
    init_parts();
    oracle_threads(threads);
    double* Q = make_q(sigma, M);
    if (!Q) return 3;
    int64_t off[KMAX + 2];
    off[1] = 0;
    for (int d = 1; d <= K; ++d) off[d + 1] = off[d] + binom(M, d);
    int64_t N = off[K + 1];
    double* p = (double*)malloc(sizeof(double) * N);
    double* mu = (double*)malloc(sizeof(double) * N);
    double* kap = (double*)malloc(sizeof(double) * N);
    double* mubar = (double*)calloc(N, sizeof(double));
    double* pbar = (double*)calloc(N, sizeof(double));
    if (!p || !mu || !kap || !mubar || !pbar) return 3;
    int err = 0;
    /* forward: p and mu of every subset (mu from the p of its own subsets) */
    for (int d = 1; d <= K; ++d) {
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : err)
        for (int64_t r = 0; r < binom(M, d); ++r) {
            int S[KMAX];
            unrank(d, r, S);
            double c, k;
            double pv;
            err |= vacuum_prob(Q, NULL, M, S, d, (1u << d) - 1, &pv);
            err |= subset_values(Q, NULL, M, S, d, 0, &c, &k, NULL, NULL);
            p[off[d] + r] = pv;
            mu[off[d] + r] = c;
            kap[off[d] + r] = k;
        }
    }
    if (err) goto done;
    nsum L = {0.0, 0.0};
    for (int64_t i = 0; i < N; ++i) {
        double diff = kap[i] - target[i];
        nadd(&L, diff * diff);
    }
    *loss = nval(&L);
    /* mubar: scatter from every S to the blocks of its partitions (serial, plain) */
    for (int d = 1; d <= K; ++d) {
        const partitions* P = &g_parts[d];
        for (int64_t r = 0; r < binom(M, d); ++r) {
            int S[KMAX];
            unrank(d, r, S);
            double kb = 2.0 * (kap[off[d] + r] - target[off[d] + r]);
            double mloc[1 << KMAX];
            int64_t rloc[1 << KMAX];
            for (unsigned B = 1; B < (1u << d); ++B) {
                int sub[KMAX], nb = 0;
                for (int k = 0; k < d; ++k) if (B & (1u << k)) sub[nb++] = S[k];
                rloc[B] = off[nb] + rank_of(nb, sub);
                mloc[B] = mu[rloc[B]];
            }
            for (int i = 0; i < P->n; ++i) {
                int nb = P->nblocks[i];
                double w = weight(nb);
                for (int b = 0; b < nb; ++b) {
                    double prod = w;
                    for (int b2 = 0; b2 < nb; ++b2)
                        if (b2 != b) prod *= mloc[P->blocks[i][b2]];
                    mubar[rloc[P->blocks[i][b]]] += kb * prod;
                }
            }
        }
    }
    /* pbar: every B passes mubar(B) to each non-empty subset T */
    for (int d = 1; d <= K; ++d) {
        for (int64_t r = 0; r < binom(M, d); ++r) {
            int S[KMAX];
            unrank(d, r, S);
            double mb = mubar[off[d] + r];
            for (unsigned T = 1; T < (1u << d); ++T) {
                int sub[KMAX], nt = 0;
                for (int k = 0; k < d; ++k) if (T & (1u << k)) sub[nt++] = S[k];
                pbar[off[nt] + rank_of(nt, sub)] += (nt % 2 ? -mb : mb);
            }
        }
    }
    /* dL/dQ_T = -pbar p Q_T^{-1} / 2, scattered onto the 2M x 2M gradient */
    int64_t n2 = 2 * (int64_t)M;
    memset(grad, 0, sizeof(double) * n2 * n2);
    for (int d = 1; d <= K; ++d) {
        for (int64_t r = 0; r < binom(M, d); ++r) {
            int S[KMAX];
            unrank(d, r, S);
            int idx[NMAX];
            for (int k = 0; k < d; ++k) { idx[k] = S[k]; idx[k + d] = S[k] + M; }
            int n = 2 * d;
            double A[NMAX][NMAX], Inv[NMAX][NMAX];
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) A[i][j] = Q[(int64_t)idx[i] * n2 + idx[j]];
            if (spd_inverse(A, n, Inv)) { err = 2; goto done; }
            double f = -0.5 * pbar[off[d] + r] * p[off[d] + r];
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) grad[(int64_t)idx[i] * n2 + idx[j]] += f * Inv[i][j];
        }
    }
    for (int64_t i = 0; i < n2; ++i)
        for (int64_t j = 0; j < i; ++j) {
            double v = 0.5 * (grad[i * n2 + j] + grad[j * n2 + i]);
            grad[i * n2 + j] = grad[j * n2 + i] = v;
        }
done:
    free(Q); free(p); free(mu); free(kap); free(mubar); free(pbar);
    return err;
}

/*
 * Magnitudes of the cancelling terms, for stating tolerances:
 *   vmu(S)  = sum_{T subset S} w_T p(T), w_T = 1 (click) or 2^|T| (parity):
 *             FP64 evaluation of the correlator errs by O(u) * vmu(S);
 *   vkap(S) = sum_pi |w(pi)| sum_{B in pi} vmu(B) prod_{B' in pi, B' != B} |m(B')|:
 *             the first-order propagation of those errors into the cumulant.
 */
int oracle_error_floor_mu(int M, const double* sigma, const double* mu, int d,
                          const int64_t* ranks, int64_t n, int convention, double* vmu,
                          double* vkap, int threads) {
    if (M < 1 || d < 1 || d > KMAX || d > M) return 1;
    init_parts();
    oracle_threads(threads);
    double* Q = make_q(sigma, M);
    if (!Q) return 3;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : err)
    for (int64_t i = 0; i < n; ++i) {
        int S[KMAX];
        unrank(d, ranks[i], S);
        double p[1 << KMAX], m[1 << KMAX], v[1 << KMAX];
        int full = (1 << d) - 1;
        for (unsigned T = 0; T <= (unsigned)full; ++T) err |= vacuum_prob(Q, mu, M, S, d, T, &p[T]);
        for (unsigned B = 1; B <= (unsigned)full; ++B) {
            nsum acc = {0.0, 0.0};
            double mag = 0.0;
            for (unsigned T = 0; T <= B; ++T) {
                if ((T & B) != T) continue;
                int t = popc(T);
                double w = convention == 0 ? 1.0 : ldexp(1.0, t);
                nadd(&acc, (t % 2 ? -w : w) * p[T]);
                mag += w * p[T];
            }
            m[B] = nval(&acc);
            v[B] = mag;
        }
        const partitions* P = &g_parts[d];
        double vk = 0.0;
        for (int j = 0; j < P->n; ++j) {
            int nb = P->nblocks[j];
            double w = fabs(weight(nb));
            for (int b = 0; b < nb; ++b) {
                double prod = w * v[P->blocks[j][b]];
                for (int b2 = 0; b2 < nb; ++b2)
                    if (b2 != b) prod *= fabs(m[P->blocks[j][b2]]);
                vk += prod;
            }
        }
        vmu[i] = v[full];
        vkap[i] = vk;
    }
    free(Q);
    return err;
}

int oracle_error_floor(int M, const double* sigma, int d, const int64_t* ranks, int64_t n,
                       int convention, double* vmu, double* vkap, int threads) {
    return oracle_error_floor_mu(M, sigma, NULL, d, ranks, n, convention, vmu, vkap, threads);
}
