/*
 * gbs.h -- click correlators and cumulants of a Gaussian state on MI355X (gfx950).
 *
 * C ABI of libgbs.  Plain pointers and sizes only.  Every compute entry point
 * takes DEVICE pointers and runs its arithmetic in HIP kernels on `stream`
 * (a hipStream_t; NULL means the null stream).  Helpers marked "host" take
 * host pointers and launch nothing.
 *
 * Problem (arXiv 2511.14923, Sec. I.A and App. D.1): sigma is the 2M x 2M
 * quadrature covariance of a zero-mean M-mode Gaussian state measured by
 * threshold detectors, hbar = 1 (vacuum = I/2); gbs_cumulants_displaced adds
 * first moments.  With Q = sigma + I/2 and Q_T
 * the rows/columns k and k+M for k in T, the probability that every mode of T
 * is in vacuum is
 *        p(T) = det(Q_T)^(-1/2)          (Eqs. vacuum_gaussian_prob, correlator_sum_cov)
 * and, for every subset S of the modes with 1 <= |S| <= max_order,
 *   click correlator   mu(S)  = sum_{T subset S} (-1)^|T| p(T)
 *                      (= probability that all of S click; App. A.2, Eq. joint_moments_def)
 *   parity correlator  c(S)   = (-1)^|S| sum_{T subset S} (-2)^|T| p(T)
 *                      (Sec. I.A, Eq. corre_cov_main)
 *   cumulant           sum_{pi partition of S} (-1)^(|pi|-1) (|pi|-1)! prod_{B in pi} m(B)
 *                      with m = mu (click cumulant kappa~, App. A.2, Eq. joint_cumulants_def)
 *                      or m = c (cumulant kappa, Sec. I.A, Eq. cumulant_corr_main).
 *
 * Input layout: sigma is 2M x 2M FP64, row-major, xxpp ordering (index k is
 * x_k, index k+M is p_k).  Only the lower triangle (row >= column) is read.
 *
 * Output layout (all output arrays): N(M, K) = sum_{d=1..K} C(M, d) FP64
 * values; order blocks d = 1, 2, ..., K one after the other (block d starts at
 * gbs_order_offset(M, d)); inside a block, subsets in colexicographic order:
 * the subset {s_0 < s_1 < ... < s_{d-1}} has rank sum_j C(s_j, j+1).
 *
 * Ownership: the caller allocates and owns every argument buffer.  The library
 * allocates its own scratch (stream-ordered, released before the call
 * returns, or at stream completion for GBS_ASYNC calls) and keeps small
 * per-device tables until the process ends.  Entry points are thread safe.
 *
 * Errors: return codes only; nothing aborts or prints.  Arguments are checked
 * on the host before anything is launched.  Outputs are unspecified when the
 * call does not return GBS_OK.
 */
#ifndef GBS_H
#define GBS_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define GBS_API __attribute__((visibility("default")))
#else
#define GBS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gbs_status;

enum {
    GBS_OK = 0,
    GBS_E_INVALID_ARG = 1,   /* bad size, order, flag bit or null pointer            */
    GBS_E_NOT_SPD = 2,       /* a pivot of some Q_T was not positive and finite        */
    GBS_E_OUT_OF_MEMORY = 3, /* scratch allocation failed                              */
    GBS_E_DEVICE = 4,        /* a HIP runtime call failed                              */
    GBS_E_UNSUPPORTED = 5,   /* valid request that this library does not implement     */
    GBS_E_SCRATCH_LIMIT = 6  /* gbs_cumulants_noalloc: the problem needs more scratch than
                                GBS_NOALLOC_SCRATCH_BYTES                               */
};

/* flags (bit set) */
enum {
    GBS_CLICK = 0,   /* bit 0 clear: click correlators mu and click cumulants kappa~ (default) */
    GBS_PARITY = 1,  /* bit 0 set:   parity correlators c and cumulants kappa                  */
    GBS_FP64 = 0,    /* bit 1 clear: every step in FP64 (default)                              */
    GBS_MIXED = 2,   /* bit 1 set:   FP32 determinant work on the normalised Q (deviations from
                        the identity), FP64 probabilities, inclusion-exclusion and partition
                        sums (not for gbs_cumulant_grad); error per order as reported       */
    GBS_ASYNC = 4,   /* bit 2 set:   return right after the launches; a NOT_SPD pivot is then
                        reported only by gbs_last_error after the stream has completed          */
    GBS_TIMING = 8,  /* bit 3 set:   record a HIP event pair around every kernel launch of the
                        call, on `stream`; read them back with gbs_last_timings               */
    GBS_ALL_MINORS = 16 /* bit 4 set: evaluate all 2^d principal minors of every subset from Q
                        (no lower-order tables): the kernel of the batched launch; slower    */
};

/* Kernel stages reported by gbs_last_timings. */
enum {
    GBS_STAGE_BUILD_Q = 0,    /* Q = sigma + I/2 (interleaved copy)                 */
    GBS_STAGE_NORMALISE = 1,  /* per-mode normalisation of Q (GBS_MIXED)            */
    GBS_STAGE_FORWARD = 2,    /* one order's correlator/cumulant kernel             */
    GBS_STAGE_ADJOINT = 3,    /* one kernel of the vector-Jacobian product          */
    GBS_STAGE_BATCHED = 4,    /* the persistent batched kernel                      */
    GBS_STAGE_SAMPLE = 5,     /* one launch of the sampler kernel                   */
    GBS_STAGE_ESTIMATE = 6    /* gbs_sample_cumulants or gbs_pearson (whole call)   */
};

typedef struct {
    int32_t stage;  /* GBS_STAGE_*                                   */
    int32_t order;  /* subset order of a FORWARD stage, else 0        */
    float ms;       /* elapsed time between the launch's event pair   */
} gbs_kernel_time;

#define GBS_MAX_ORDER 5
#define GBS_MAX_MODES 2048

/* host.  C(M, d) for 0 <= d <= M <= GBS_MAX_MODES; -1 otherwise.  The number of
 * order-d correlators (the subsets S with |S| = d of Sec. I.A, counted in the
 * space estimate of Sec. "Cost estimation and scaling"). */
GBS_API int64_t gbs_num_subsets(int32_t M, int32_t d);

/* host.  Start of the order-d block: sum_{e=1..d-1} C(M, e); -1 on bad arguments
 * (1 <= d <= GBS_MAX_ORDER + 1, d <= M + 1).  Output layout of this library
 * (the paper keeps explicit subset lists with auxiliary indices, Sec. III
 * Phase I; here order blocks and colex ranks replace them). */
GBS_API int64_t gbs_order_offset(int32_t M, int32_t d);

/* host.  N(M, K) = total number of outputs for orders 1..K; -1 on bad arguments
 * (all subsets up to the truncation order K of Sec. I.A). */
GBS_API int64_t gbs_total_outputs(int32_t M, int32_t max_order);

/* host.  Colex rank of the d-subset S (host array of d distinct modes in any
 * order, each in [0, GBS_MAX_MODES)); -1 on bad arguments.  The position of S
 * inside its order block (combinatorial number system; replaces the subset
 * lists of Sec. III Phase I). */
GBS_API int64_t gbs_colex_rank(int32_t d, const int32_t* S);

/* host.  Inverse of gbs_colex_rank: writes the d-subset of rank r, ascending,
 * into the host array S (length d).  GBS_E_INVALID_ARG if d is outside
 * [1, GBS_MAX_ORDER], r < 0, or the subset would need a mode >= GBS_MAX_MODES. */
GBS_API gbs_status gbs_colex_unrank(int32_t d, int64_t r, int32_t* S);

/* Correlators only (the cumulant stage is skipped): mu(S) by inclusion-exclusion
 * over the vacuum probabilities of the subsets of S (App. A.2, Eq.
 * joint_moments_def; App. D.1, Eq. correlator_sum_cov), or the parity
 * correlator c(S) (Sec. I.A, Eq. corre_cov_main).
 *   M          number of modes, 1 <= M <= GBS_MAX_MODES
 *   sigma      device, 2M x 2M FP64 (layout above)
 *   max_order  K, 1 <= K <= min(GBS_MAX_ORDER, M)
 *   flags      GBS_CLICK/GBS_PARITY | GBS_FP64/GBS_MIXED | GBS_ASYNC
 *   corr       device, N(M, K) FP64, overwritten with mu (click) or c (parity)
 */
GBS_API gbs_status gbs_correlators(int32_t M, const double* sigma, int32_t max_order, int32_t flags,
                           double* corr, void* stream);

/* Correlators and cumulants.  Orders run in sequence; by default an order-d
 * subset factors one new 2d x 2d block of Q and reads the vacuum probabilities,
 * correlators and cumulants of its lower-order sub-blocks from the previous
 * orders (App. B, Eq. correlators_expanded_2 for the cumulant); with
 * GBS_ALL_MINORS it evaluates all of them itself.
 *   corr   device, N(M, K) FP64, or NULL to skip writing the correlators
 *   cum    device, N(M, K) FP64, overwritten with kappa~ (click) or kappa (parity)
 * Other arguments as gbs_correlators. */
GBS_API gbs_status gbs_cumulants(int32_t M, const double* sigma, int32_t max_order, int32_t flags,
                         double* corr, double* cum, void* stream);

/* Static scratch of gbs_cumulants_noalloc, bytes per device (160 MiB). */
#define GBS_NOALLOC_SCRATCH_BYTES (160u * 1024u * 1024u)

/* gbs_cumulants for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, outputs, kernels and results as gbs_cumulants (bit for bit),
 * but every scratch buffer of the call -- Q, its diagonal blocks, the
 * mixed-precision operands, the status word, the group kernel's tile plans and
 * the lower-order probability tables (and the correlator tables when corr is
 * NULL) -- lives in one static device array of GBS_NOALLOC_SCRATCH_BYTES per
 * device, held from the library's load until the process ends.  The call
 * makes no hipMalloc, hipFree, stream-ordered or pinned-host allocation.
 *   Limit: about 8 (N(M, K-1) [+ N(M, K) if corr is NULL] + 4 M^2) bytes plus
 *   the tile plans (~3.5 MB at M = 144, K = 5) must fit: M = 144, K = 5 fits
 *   with corr given, not with corr NULL.  Larger problems return
 *   GBS_E_SCRATCH_LIMIT before anything is launched.
 *   flags  GBS_CLICK/GBS_PARITY | GBS_MIXED | GBS_ASYNC | GBS_ALL_MINORS
 *          (GBS_TIMING gives GBS_E_UNSUPPORTED: its events are allocations)
 * Set-up: the first call on a device looks up the array's address there and
 * writes a constant binomial table into it (a blocking copy); it must not be
 * captured.  Tile plans are copied in (from host memory, on `stream`) when the
 * previous call on the device had a different (M, max_order).
 * Every call on one device shares that device's array and leaves its contents
 * there: calls that overlap on one device (other threads, other streams, or a
 * second call before the first has completed its kernels on another stream)
 * race and give wrong results; serialise them.  The status word stays on the
 * device: a synchronous call reads it back with a blocking copy, a
 * GBS_ASYNC call leaves it for gbs_last_error (valid once the stream has
 * completed).  Other errors as gbs_cumulants. */
GBS_API gbs_status gbs_cumulants_noalloc(int32_t M, const double* sigma, int32_t max_order,
                                         int32_t flags, double* corr, double* cum, void* stream);

/* Correlators and cumulants of a DISPLACED Gaussian state (first moments
 * mu != 0).  The vacuum probability becomes
 *        p(T) = exp(-mu_T^T Q_T^{-1} mu_T / 2) det(Q_T)^(-1/2)
 * (App. D.1, Eq. vacuum_gaussian_prob, hbar = 1), with mu_T the entries k and
 * k+M of mu for k in T; correlators and cumulants follow from p exactly as in
 * gbs_cumulants.  mu = 0 gives gbs_cumulants' results (through a different
 * kernel, so the last bits may differ).
 *   mu     device, 2M FP64 first moments, xxpp order (index k is <x_k>, k+M is <p_k>)
 *   flags  GBS_CLICK/GBS_PARITY | GBS_ASYNC | GBS_TIMING | GBS_ALL_MINORS;
 *          GBS_MIXED gives GBS_E_UNSUPPORTED (FP64 only)
 * Other arguments, layouts, ownership and errors as gbs_cumulants; the same
 * kernels run, each also carrying the mean through its factorisation (one
 * forward substitution of mu per factor). */
GBS_API gbs_status gbs_cumulants_displaced(int32_t M, const double* sigma, const double* mu,
                                   int32_t max_order, int32_t flags, double* corr, double* cum,
                                   void* stream);

/* One shard of one order: the correlators and cumulants of the order-`order`
 * subsets with colex ranks rank0 .. rank0 + count - 1 (in rank order), each
 * evaluated from Q alone (no lower-order tables), so that disjoint rank ranges
 * are independent work: the unit by which the computation splits across
 * devices for large M (e.g. M = 1152 pseudo-photon-number-resolving detection,
 * C(1152, 5) = 1.7e13 order-5 subsets).  Orders 3..5 run the T-shared kernel
 * (the subsets {a, b_0} + T of one T share the factors of Q_T, of each b_0
 * and of each a against T; App. D.1, Eq. vacuum_gaussian_prob).  Its host
 * side lists the range's T's on the first call of a range and copies the list
 * to the device with a blocking copy (so that first call must not be captured
 * in a graph); the last eight lists stay on the device, and evicting one waits
 * for the device.  A range of more than 2^16 T's runs as consecutive chunks of
 * 2^16 T's, one list and one launch each.  Orders 1, 2 and GBS_ALL_MINORS
 * run the all-minors kernel of gbs_cumulants' GBS_ALL_MINORS, whose shards are
 * bit-identical to slices of that full pass.
 * Same definitions and tolerance as gbs_cumulants.
 *   order        1 <= order <= min(GBS_MAX_ORDER, M)
 *   rank0, count rank0 >= 0, count >= 0, rank0 + count <= C(M, order)
 *   corr, cum    device, count FP64 each (either may be NULL, not both)
 *   flags        GBS_CLICK/GBS_PARITY | GBS_ASYNC | GBS_TIMING | GBS_ALL_MINORS
 *                (GBS_MIXED gives GBS_E_UNSUPPORTED)
 * Other arguments and errors as gbs_cumulants; gbs_last_error reports the
 * global colex rank of a failing subset. */
GBS_API gbs_status gbs_cumulants_shard(int32_t M, const double* sigma, int32_t order, int64_t rank0,
                                       int64_t count, int32_t flags, double* corr, double* cum,
                                       void* stream);

/* Vector-Jacobian product of gbs_cumulants (FP64 only; GBS_MIXED gives
 * GBS_E_UNSUPPORTED).  Not in the paper (it has no gradients): derived from
 * App. D.1, Eq. correlator_sum_cov, with d log det A = tr(A^{-1} dA).  The
 * fifth argument is the upstream gradient of the correlators, not the forward
 * correlators: the forward pass (vacuum probabilities and correlators of every
 * subset) is recomputed inside the call, so one call serves losses on the
 * correlators, the cumulants or both:
 *   grad_sigma[i][j] = sum_S grad_corr[S] d corr[S]/d sigma_ij
 *                    + sum_S grad_cum[S]  d cum[S] /d sigma_ij
 * with the 4M^2 entries of sigma treated as independent variables, so the
 * result is symmetric (d log det A = tr(A^{-1} dA), App. D.1 equations).
 *   grad_corr   device, N(M, K) FP64 upstream gradient of the correlators, or NULL (zero)
 *   grad_cum    device, N(M, K) FP64 upstream gradient of the cumulants, or NULL (zero)
 *   grad_sigma  device, 2M x 2M FP64, overwritten (row-major, xxpp)
 * Work grows like C(M, K) * M^(K-1); intended for K <= 3 at M ~ 100-150.
 * Deterministic: every sum has a fixed order (no atomics). */
GBS_API gbs_status gbs_cumulant_grad(int32_t M, const double* sigma, int32_t max_order, int32_t flags,
                             const double* grad_corr, const double* grad_cum, double* grad_sigma,
                             void* stream);

/* One covariance instance of a batch. */
typedef struct {
    int32_t M;           /* modes of this instance, max_order <= M <= GBS_MAX_MODES           */
    int32_t reserved;    /* must be 0                                                         */
    const double* sigma; /* device, 2M x 2M FP64                                              */
    double* corr;        /* device, N(M, K) FP64, or NULL to skip the correlators             */
    double* cum;         /* device, N(M, K) FP64 (required)                                   */
} gbs_instance;

/* gbs_cumulants for many covariance instances at once (the same definitions:
 * Sec. I.A, Eqs. corre_cov_main and cumulant_corr_main; App. A.2; the batching
 * itself is not in the paper, which computes one ground truth per run).
 * Many instances of uneven M in persistent launches over device work lists
 * (plus the launches that form every instance's Q): one launch over
 * (instance, order, rank range) items evaluated from all the principal minors
 * of Q_S (orders 1 and 2; every order with GBS_ALL_MINORS, and for instances
 * the group kernel does not take), then one launch per order 3..max_order over
 * the (instance, tile) items of the group kernel (FP64 or GBS_MIXED), which
 * reads each instance's lower-order tables.  FP64 results agree with n separate
 * gbs_cumulants calls (same flags) to FP64 rounding; mixed-form results agree
 * with them within the mixed form's error (its orders 1 and 2 come from all
 * minors here, from the order-recursive kernels there, with FP32 roundings
 * taken in other orders).  Library-owned scratch per instance list: Q, its
 * diagonal blocks and (GBS_MIXED) its normalised form, and, for the group
 * launches, the vacuum probabilities of orders 1..max_order-1 (and their
 * correlators when inst.corr is NULL).  The pipeline is captured once into a
 * HIP graph per (instance list, stream, order, flags, tuning) and replayed on
 * later calls with the same list on the same stream (a plan's work-list counter
 * and status word serve one stream: threads calling on one stream are
 * serialised while they enqueue, a list used on two streams gets two plans, and
 * an evicted plan is freed only after its last call has returned); the launch
 * shapes come from gbs_autotune_batched's cached choice when one exists for
 * this device, order and precision, else from a fixed default (the group
 * launches then fill the device).
 *   n      1 <= n <= 4096
 *   inst   HOST array of n descriptors (pointers inside are device pointers)
 */
GBS_API gbs_status gbs_cumulants_batched(int32_t n, const gbs_instance* inst, int32_t max_order,
                                 int32_t flags, void* stream);

/* Launch shape of the batched launches: the all-minors launch (block, unroll,
 * tile, waves_per_cu) and the group launches (group_wpc). */
typedef struct {
    int32_t block;   /* threads per workgroup: 64, 128 or 256               */
    int32_t unroll;  /* subsets per thread and work item: 1, 2 or 4         */
    int32_t tile;    /* subsets per work item (multiple of block * unroll)  */
    int32_t waves_per_cu; /* persistent workgroups per compute unit, 1..8   */
    int32_t group_wpc; /* workgroups per compute unit of the group launches
                          (orders 3..K): 0 = as many as fit, else 1..8    */
} gbs_tuning;

/* Launch-shape autotuner of gbs_cumulants_batched (library plumbing, not in the
 * paper).  Times the whole pipeline on the given batch for every candidate
 * shape of the all-minors launch (81: block x unroll x tile x workgroups per
 * CU), then, with the fastest, for the group launches' workgroups per CU
 * (as many as fit, 2, 1); outputs are overwritten (stream-ordered,
 * synchronising).  Caches the fastest shape for this device, order and
 * precision; writes it to *best (host) when best is non-NULL. */
GBS_API gbs_status gbs_autotune_batched(int32_t n, const gbs_instance* inst, int32_t max_order,
                                int32_t flags, void* stream, gbs_tuning* best);

/* host (library plumbing, not in the paper).  Set (or, with t == NULL, clear)
 * the cached shape used by
 * gbs_cumulants_batched for this device, order and precision. */
GBS_API gbs_status gbs_set_tuning(int32_t max_order, int32_t flags, const gbs_tuning* t);

/* Stage-2 sampler (Sec. II "The sampling algorithm"; Methods; App. C.1):
 * nsamples click patterns x_1 .. x_M (bit n is mode n - 1) drawn one bit at a
 * time by the chain rule, with the joint probability of the first n bits
 * expanded in the parity cumulants kappa up to order max_order (Eq.
 * samplecumulant) and the marginals it needs approximated by tables updated
 * after every bit:
 *   max_order = 3  single elision (Eqs. methprob, b, a), O(M^3) per sample;
 *   max_order = 5  double elision (Eqs. probade, probpartialade, probelidedade,
 *                  probdoubleelidedade), O(M^5) per sample.
 * Bit n of sample s is 1 iff uniforms[(n-1) * nsamples + s] < p(x_n = 1 | x_<n)
 * = (p(x_{n-1}, .., x_1) / 2 - D_n) / p(x_{n-1}, .., x_1), the expansion's value
 * (1/2 when the previous marginal is not positive); all arithmetic is FP64.
 *   M          1 <= M, max_order <= M; M <= 256 (max_order 3) or M <= 200 (5)
 *   kappa      device, N(M, max_order) FP64 parity cumulants in the output layout
 *              above (as written by gbs_cumulants with GBS_PARITY)
 *   nsamples   >= 0 (0: nothing is launched; uniforms and bits may then be NULL)
 *   uniforms   device, M x nsamples FP64 in [0, 1), row n-1 for bit n
 *   bits       device, nsamples x M bytes (0/1), sample-major, overwritten
 *   prob       device, nsamples FP64: the expansion's p(x_M, .., x_1), or NULL
 *   cond       device, M x nsamples FP64: p(x_n = 1 | x_<n) of every step, or NULL
 *   batch      samples per kernel launch (rounded to a multiple of 64); 0 = as
 *              many as fit in a quarter of the free device memory.  The library
 *              allocates the per-sample tables for one batch: 8 x (M + 1 + C(M,2)
 *              + C(M+1,2) [+ C(M,3) for max_order 5]) bytes per sample
 *   flags      GBS_ASYNC | GBS_TIMING (other bits: GBS_E_INVALID_ARG)
 * Errors: GBS_E_INVALID_ARG for bad sizes, orders or null pointers;
 * GBS_E_UNSUPPORTED for max_order other than 3 or 5. */
GBS_API gbs_status gbs_sample(int32_t M, const double* kappa, int32_t max_order, int64_t nsamples,
                              const double* uniforms, uint8_t* bits, double* prob, double* cond,
                              int64_t batch, int32_t flags, void* stream);

/* Click cumulants estimated from samples (App. F, "Click cumulants, Pearson and
 * Spearman coefficients", Eq. cumulants_test_def): for every S with
 * 1 <= |S| <= max_order, the unbiased estimate of kappa~(S) in which each
 * product of |pi| click moments of the partition sum is averaged over ordered
 * tuples of distinct samples (k-statistics).  Computed from the power sums
 * s_B (samples in which every mode of B clicked) of all subsets, as bit-matrix
 * products of per-mode bit columns; FP64 combination.
 *   M          1 <= M <= 256, max_order <= M
 *   nsamples   max_order <= nsamples < 2^32
 *   bits       device, nsamples x M bytes (0/1), sample-major (as gbs_sample writes)
 *   max_order  1..GBS_MAX_ORDER
 *   cum        device, N(M, max_order) FP64, output layout above, overwritten
 *   flags      GBS_ASYNC | GBS_TIMING
 * The library allocates M * ceil(nsamples / 64) * 8 bytes of bit columns plus
 * 4 bytes per subset of counts. */
GBS_API gbs_status gbs_sample_cumulants(int32_t M, int64_t nsamples, const uint8_t* bits,
                                        int32_t max_order, double* cum, int32_t flags,
                                        void* stream);

/* Pearson correlation coefficient of x and y (Eq. pearson_correlation):
 * sum (x - <x>)(y - <y>) / sqrt(sum (x - <x>)^2 sum (y - <y>)^2), two passes
 * of FP64 reductions in a fixed order (deterministic).
 *   n      >= 2
 *   x, y   device, n FP64 each
 *   r      device, one FP64, overwritten
 *   flags  GBS_ASYNC | GBS_TIMING */
GBS_API gbs_status gbs_pearson(int64_t n, const double* x, const double* y, double* r,
                               int32_t flags, void* stream);

/* host (error reporting, not in the paper: a Q_T that is not positive definite
 * has no vacuum probability, App. D.1).  After a call returned GBS_E_NOT_SPD
 * (or after a GBS_ASYNC call's
 * stream completed), the order and colex rank of the first failing subset
 * seen by this thread's last call; GBS_OK if none.  Either pointer may be NULL. */
GBS_API gbs_status gbs_last_error(int32_t* order, int64_t* rank);

/* host (measurement plumbing, not in the paper).  Kernel timings of this
 * thread's last call made with GBS_TIMING: waits
 * for its events, writes up to `capacity` entries (launch order) to `out` and
 * returns the number of entries recorded (-1 on a HIP error). */
GBS_API int32_t gbs_last_timings(int32_t capacity, gbs_kernel_time* out);

/* host (library plumbing, not in the paper).  Static description of a status code. */
GBS_API const char* gbs_status_string(gbs_status s);

#ifdef __cplusplus
}
#endif

#endif /* GBS_H */
