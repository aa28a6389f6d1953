/*
 * qmc.h -- C interface of the MI355X (gfx950) fast QMC matrix-product library.
 *
 * Computes X = Y A and dA = Y^T G, where the N rows of Y are QMC points
 * mapped by one univariate function phi in every coordinate, without ever
 * forming Y: after re-indexing the rows by the discrete logarithm with respect
 * to a primitive element, the nonzero rows of Y are a circulant of length
 * L = N - 1 applied to a selection of A's rows, so every column costs one
 * FFT-based circular convolution (Dick, Kuo, Le Gia, Schwab, "Fast QMC
 * matrix-vector multiplication", Section 2.1, eq. (ZPa), and Remark 1 for
 * polynomial lattice rules).
 *
 * Conventions shared by every entry point
 *   - Matrices are row-major.  A is s x t with row stride lda (elements),
 *     X is N x t with row stride ldx; G is N x t (ldg), dA is s x t (ldda).
 *   - Row n of X is the point with conventional index n: for a lattice rule
 *     x_n = ({n g_1/N + D}, ..., {n g_s/N + D}) (Section 2.1, with the equal
 *     shift D of Remark 2); for a polynomial lattice rule over GF(2) the row
 *     index n is the polynomial whose coefficient of x^i is bit i of n.
 *   - Device pointers (A, X, G, dA, workspace) belong to the caller and must
 *     stay valid until the stream has executed the call.  Host pointers are
 *     read before the call returns.
 *   - All work is enqueued on the HIP stream passed as `stream`
 *     (hipStream_t; NULL = the null stream) and is asynchronous.
 *   - The element type is fixed per plan: QMC_F32 (float) or QMC_F64
 *     (double) for A, X, G and dA and for all arithmetic on them.
 *   - Return value 0 on success, a negative QMC_ERR_* code otherwise.
 *     Arguments are checked before anything is launched; on error nothing is
 *     enqueued and outputs are untouched.  A fault inside a launched kernel
 *     surfaces as QMC_ERR_HIP from a later call or from the caller's own
 *     stream synchronisation.  No C++ exception crosses this interface.
 *   - A plan may be used from one host thread at a time.  Calls on one plan
 *     that share a workspace must be ordered on one stream.
 */
#ifndef QMC_H_
#define QMC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qmc_plan_s* qmc_plan_t;

/* point-set families */
#define QMC_RULE_LATTICE  0   /* rank-1 lattice rule (Section 2.1; prime N, or non-prime N by orbits) */
#define QMC_RULE_POLY_GF2 1   /* polynomial lattice rule over GF(2), N = 2^m, primitive modulus (Remark 1) */

/* the univariate map phi applied to every coordinate (Section 2.1) */
#define QMC_PHI_IDENTITY  0   /* phi(x) = x */
#define QMC_PHI_CENTERED  1   /* phi(x) = x - 1/2 (Experiment 2) */
#define QMC_PHI_INVNORM   2   /* phi(x) = Phi^{-1}(x), inverse standard normal CDF (Section 3.1) */
#define QMC_PHI_TENT      3   /* phi(x) = 1 - |2x - 1| (Section 2.1) */

/* element types */
#define QMC_F32 0
#define QMC_F64 1

/* error codes */
#define QMC_OK                 0
#define QMC_ERR_ARG           -1   /* a size, stride, pointer or enum is invalid */
#define QMC_ERR_NOT_PRIME     -2   /* the union of Korobov rules with K not prime (lattice rules take any N) */
#define QMC_ERR_NOT_PRIMITIVE -3   /* GF(2) modulus not primitive of degree m with 2^m = N */
#define QMC_ERR_GEN_ZERO      -4   /* a generator component is not a unit mod N (0, or a common factor) */
#define QMC_ERR_ALIAS         -5   /* output overlaps an input */
#define QMC_ERR_WORKSPACE     -6   /* workspace missing or smaller than qmc_workspace_size */
#define QMC_ERR_OOM           -7   /* device allocation failed while building a plan */
#define QMC_ERR_HIP           -8   /* a HIP runtime call failed */
#define QMC_ERR_UNSUPPORTED   -9   /* valid request outside what the library handles */

/*
 * qmc_plan_create -- build everything that depends only on the point set.
 *
 * Section 2.1: a primitive element beta of the cyclic group (Z_N^* for prime
 * N, the nonzero residues mod p(x) for a primitive GF(2) modulus -- where the
 * element x is used), the exponents l_j with g_j = beta^{l_j} (the paper's
 * c_j - 1), the generator z_k = phi(point of beta^k) of the circulant Z, and
 * the FFT of z computed in FP64 (rounded once to FP32 for an FP32 plan).
 * The power and logarithm tables are built on the device, bit-exact.
 *
 *   out        receives the plan handle (host pointer)
 *   rule       QMC_RULE_LATTICE or QMC_RULE_POLY_GF2
 *   N          number of points: 2 <= N < 2^31 prime, or non-prime up to
 *              2^25 (lattice); 2^m with 1 <= m <= 30 (GF(2))
 *   s          dimension, s >= 1
 *   gen        host array of s generator components: g_j in [1, N-1]
 *              (lattice, taken mod N; a component that is not a unit mod N
 *              -- 0, or sharing a prime factor with a non-prime N -- is
 *              QMC_ERR_GEN_ZERO) or GF(2) polynomial bitmasks q_j in
 *              [1, 2^m - 1]
 *   modulus    GF(2): the primitive polynomial p with bit m set; lattice: 0
 *   phi_kind   QMC_PHI_*
 *   shift_num, shift_den
 *              the equal shift D = shift_num/shift_den in [0,1) added to
 *              every coordinate before phi (Remark 2); 0/1 for none.
 *              QMC_PHI_INVNORM requires a shift that keeps every coordinate
 *              inside (0,1) (e.g. 1/(2N)): a shift with N D an integer (D = 0,
 *              or any multiple of 1/N) puts the coordinate of one residue at 0
 *              and returns QMC_ERR_ARG.
 *   dtype      QMC_F32 or QMC_F64
 *   stream     HIP stream for the plan-building kernels; the call
 *              synchronises that stream before returning.
 * The convolution length M (N - 1 when that is a power of two, else the
 * shortest power of two, 3 x 2^k or 5 x 2^k >= 2N - 3, see qmc_plan_info; the union
 * of Korobov rules takes powers of two only) must split as M = M1 x M2 with
 * M1 <= 4096 on chip
 * and M2 <= 64 x 64; longer rules (N - 1 > 2^23 when not a power of two, or
 * above 2^24) return QMC_ERR_UNSUPPORTED before any device work.
 *
 * Non-prime N (lattice rules; Section 2.1 defers this case to the fast
 * construction of Nuyens and Cools for non-prime n): with unit generator
 * components the rows split into the orbits n = d m, d | N, m a unit mod
 * N/d, on which the coordinates are those of the rule with N/d points.  Each
 * unit group is a direct product of cyclic groups (one per odd prime power,
 * one for 4, two for 2^k, k >= 3); with its largest cyclic factor of order L
 * and the product H of the others, the rows and columns of an orbit split
 * into |H| x |H| blocks, each a circulant of length L handled like a prime
 * rule (its own spectrum and collapse), the blocks of one row coset adding
 * up (summed on their spectra: one inverse transform and one pass writing
 * the rows per row coset; the adjoint likewise per column coset).  Orbits
 * with L >= 64 and |H| <= 8 take blocks (at most 1024 over all
 * orbits); the others and row 0 are summed directly (phi(N/d) s t
 * multiply-adds for an orbit: fast for 2^k, prime powers and products of
 * few primes, slow for highly composite N with large s t).  Non-prime N above
 * 2^25 return QMC_ERR_UNSUPPORTED.  Such a plan has no single cyclic
 * group: qmc_plan_set_row_order(QMC_ROWS_GROUP), the power/logarithm/exponent
 * tables of qmc_plan_tables and batches return QMC_ERR_UNSUPPORTED.
 * The plan owns its device memory; release it with qmc_plan_destroy.
 */
int qmc_plan_create(qmc_plan_t* out, int rule, int64_t N, int64_t s,
                    const uint64_t* gen, uint64_t modulus, int phi_kind,
                    int64_t shift_num, int64_t shift_den, int dtype, void* stream);

void qmc_plan_destroy(qmc_plan_t plan);

/*
 * Plan facts for callers and tests (host pointer to a filled struct).  The
 * transform factorisation is M = M1 x M2 with M1 = R^3 on chip (three
 * register DFTs of radix R) and the outer length M2 = P2 x Q2 (a split pass of
 * radix P2 when P2 > 1, the back pass of radix Q2).  R and P2 are powers of
 * two; Q2 (and M2) is a power of two, 3 x 2^i or 5 x 2^i, whose register
 * DFTs take one radix-3 or radix-5 stage and then radix-4 and radix-2 stages.  These fields are
 * the whole radix plan, so no separate list of radices is reported.
 */
typedef struct {
    int64_t N, s, L;        /* points, dimension, order L of the unit group (N - 1 for prime N) */
    int64_t M;              /* circular-convolution length used: L, or the shortest power
                               of two >= 2L-1, or 3 x 2^k or 5 x 2^k >= 2L-1 when shorter
                               (M >= 3 x 4096 and M2 no longer than one back pass) */
    int64_t M1, M2;         /* M = M1 * M2 (on-chip transform length, outer length) */
    int64_t rounds;         /* rounds of the sparse collapse schedule */
    uint64_t beta;          /* primitive element (lattice: smallest primitive root; GF(2): x = 2) */
    int rule, phi_kind, dtype, embedded;
    double phi0;            /* phi of the point of row 0 (the constant first row, Section 2.1) */
    int P2, Q2;             /* outer split M2 = P2 x Q2 of the current tuning */
    int64_t blocks;         /* non-prime N: circulant blocks (M, M1, M2, P2, Q2, rounds
                               describe the longest); 0 for prime N and GF(2) */
    int64_t direct_rows;    /* non-prime N: rows summed directly (row 0, small orbits) */
} qmc_plan_info_t;
int qmc_plan_info(qmc_plan_t plan, qmc_plan_info_t* info);

/*
 * qmc_plan_tables -- copy the plan's bit-exact tables to host memory (for
 * verification).  Any pointer may be NULL.
 *   pow_out[e], e < L : conventional row index of group element beta^e
 *   log_out[r], r < N : e with pow[e] = r (log_out[0] = -1)
 *   ell_out[j], j < s : l_j with g_j = beta^{l_j}
 *   phi_out[r], r < N : phi of the one-dimensional point of residue r (FP64)
 */
int qmc_plan_tables(qmc_plan_t plan, int32_t* pow_out, int32_t* log_out,
                    int32_t* ell_out, double* phi_out);

/*
 * qmc_plan_set_row_order -- the order of the rows of X (qmc_matmul,
 * qmc_matmul_epilogue, batches) and of G (qmc_matmul_adjoint):
 *   QMC_ROWS_CONVENTIONAL (default): row n is point n, x_n = {n g / N + D}
 *   QMC_ROWS_GROUP: row 0 is point 0, row 1 + e is the point of group element
 *                   beta^e (pow_out[e] of qmc_plan_tables), e < L
 * A QMC rule does not depend on the order of its points (Section 2.1); the
 * group order is the circulant's own order (eq. (ZPa)), for callers that
 * work in it.  It is not faster: the back pass writes whole row segments in
 * either order (measured 3% slower at N = 65537, t = 4096: consecutive rows
 * spread over fewer HBM channels than the scattered conventional ones).  The
 * first switch to the group order allocates and fills an L-entry row table
 * (synchronous).  QMC_ERR_ARG for an unknown order.
 */
#define QMC_ROWS_CONVENTIONAL 0
#define QMC_ROWS_GROUP        1
int qmc_plan_set_row_order(qmc_plan_t plan, int order);

/*
 * Launch tuning of a plan (chosen by paper_1501_06286_amd/autotune.py):
 *   chunk_pairs  column pairs per chunk of the passes of qmc_matmul and
 *                qmc_matmul_adjoint; the intermediate spectrum buffers then
 *                hold one or two chunks instead of all pairs (0 = one chunk
 *                of all pairs)
 *   streams      1, or 2 to run the back pass of chunk c on a second stream,
 *                overlapping the fused pass of chunk c+1 (needs chunk_pairs > 0)
 *   nt_store     1 = write X with non-temporal stores
 *   front        how qmc_matmul forms the outer DFT of the collapsed columns:
 *                1 = sparse: the fused pass sums the s rows of A directly for
 *                every outer frequency (cost grows with s times M2);
 *                2 = dense: a gather pass collapses A into length-M columns and
 *                transforms the outer index (extra passes over M per pair,
 *                one stream); 3 = sparse with bucket twiddles: as 1, but an
 *                item's slot twiddle W_M^{slot w2} is split into its outer
 *                factor W_{M2}^{e2 w2} (a table of M2 values) and a factor
 *                W_M^{e1 w2} applied once per bucket after the sums (no
 *                per-item twiddle table reads; M2 a power of two, other
 *                outer lengths run 3 as 1); 0 = dense when s > 8 M1,
 *                else sparse
 *   outer_q      the outer radix: the outer inverse DFT of length M2
 *                (qmc_plan_info) is split as M2 = P2 x Q2 with
 *                Q2 = min(outer_q, M2) values of w2 per output column of the
 *                back pass and one extra split pass when P2 > 1; Q2 <= 32 is
 *                held in registers (FP64: up to 24), the larger ones in LDS
 *                (96 and 128: FP32 plans only).
 *                A power of two <= 128, or for M2 = f x 2^j (f = 3, 5) a value
 *                f x 2^i <= 96, with P2 = M2 / Q2 a power of two <= 64; or 0 for the
 *                default: all of M2 when that fits one back pass (M2 <= 128
 *                in FP32, 64 in FP64: no split pass), else 32, or M2/64 when
 *                larger.  The dense fronts' forward split uses Q2 up to 64,
 *                else Q2 / 2
 *   nt_inter     stores of the intermediate spectrum by the fused pass: 1 =
 *                cached, 2 = streaming (non-temporal), 0 = streaming when one
 *                launch's intermediates (with the dense fronts: both
 *                buffers) exceed 128 MiB (they would not stay in the
 *                Infinity Cache for the back pass anyway)
 * The workspace size depends on the tuning: query it after setting it.
 * Returns QMC_ERR_ARG for negative chunks, streams outside {1, 2}, nt_store
 * outside {0, 1}, front outside {0, 1, 2, 3}, an invalid outer_q or nt_inter
 * outside {0, 1, 2}.
 */
typedef struct {
    int64_t chunk_pairs;
    int streams;
    int nt_store;
    int front;
    int outer_q;
    int nt_inter;
} qmc_tuning_t;
int qmc_plan_set_tuning(qmc_plan_t plan, const qmc_tuning_t* tuning);
int qmc_plan_get_tuning(qmc_plan_t plan, qmc_tuning_t* tuning);

/* Bytes of device workspace that qmc_matmul / qmc_matmul_adjoint need for t columns. */
int qmc_workspace_size(qmc_plan_t plan, int64_t t, size_t* bytes);

/*
 * qmc_matmul -- X = Y A (Section 2.1: row 0 is phi(x_0) sum_j a_j, the other
 * rows are Z (P a) by FFT, one circular convolution per pair of columns).
 *   A          device, s x t, row stride lda >= t
 *   t          number of columns, t >= 1
 *   X          device, N x t, row stride ldx >= t; every entry is written
 *   workspace  device, at least qmc_workspace_size(plan, t) bytes
 * Errors: QMC_ERR_ARG (bad sizes/NULL), QMC_ERR_ALIAS (X overlaps A or the
 * workspace), QMC_ERR_WORKSPACE.
 */
int qmc_matmul(qmc_plan_t plan, const void* A, int64_t t, int64_t lda,
               void* X, int64_t ldx, void* workspace, size_t workspace_bytes,
               void* stream);

/*
 * qmc_matmul_epilogue -- X = Y A with an elementwise epilogue fused into the
 * writes of X (the downstream steps of Sections 3.2 and 3.3):
 *   QMC_EPI_AFFINE  X[n,c] = scale[c] * (bias[c] + (Y A)[n,c])
 *                   (the stiffness entries b_{k,l} = a_{0,k,l} + Y a_{k,l},
 *                   eq. (Ya), one column per (k, l));
 *   QMC_EPI_EXP     X[n,c] = scale[c] * exp(bias[c] + (Y A)[n,c])
 *                   (the log-normal coefficient a = exp(theta) with
 *                   Theta = Psi^ + Y Psi, eqs. (fastB), (eq_as); scale may
 *                   carry quadrature weight times basis gradients);
 *   QMC_EPI_NONE    as qmc_matmul.
 *   bias, scale  device vectors of t entries in the plan dtype, or NULL
 *                (bias 0, scale 1); read only; must not overlap X or the
 *                workspace.
 * Other arguments, workspace and errors as qmc_matmul; QMC_ERR_ARG for an
 * unknown epi_kind.
 */
#define QMC_EPI_NONE   0
#define QMC_EPI_AFFINE 1
#define QMC_EPI_EXP    2
int qmc_matmul_epilogue(qmc_plan_t plan, const void* A, int64_t t, int64_t lda, void* X,
                        int64_t ldx, int epi_kind, const void* bias, const void* scale,
                        void* workspace, size_t workspace_bytes, void* stream);

/*
 * qmc_matmul_adjoint -- dA = Y^T G, the transpose product needed to
 * differentiate X = Y A with respect to A.  The nonzero rows of Y in group
 * order form a symmetric (Hankel-circulant) operator, so the same spectrum
 * serves: G's rows are gathered in reflected group order, convolved, and
 * read back at the exponents l_j; the constant row adds phi(x_0) G[0,:].
 *   G   device, N x t (ldg >= t);  dA  device, s x t (ldda >= t), overwritten
 */
int qmc_matmul_adjoint(qmc_plan_t plan, const void* G, int64_t t, int64_t ldg,
                       void* dA, int64_t ldda, void* workspace, size_t workspace_bytes,
                       void* stream);

/*
 * qmc_matmul_noalloc -- X = Y A exactly as qmc_matmul computes it (the same
 * kernels in the same order, so the same bits), for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  The call allocates nothing: no
 * hipMalloc/hipFree, no stream or event creation.  Its workspace is a static
 * device array of QMC_NOALLOC_SCRATCH_BYTES that every GPU the library runs
 * on holds from the first load of the library's code on that device until
 * the process ends.
 *   A, t, lda, X, ldx, stream   as qmc_matmul; X is written, A only read.
 * Every launch goes to `stream`, also when the plan's tuning asks for two
 * streams.  All calls on one GPU share that GPU's one scratch array: calls
 * that can overlap on a GPU (different streams, host threads or plans) race
 * and give undefined results; order them on one stream.  The array keeps the
 * last call's contents; a call reads only scratch bytes it wrote itself.
 * Errors: QMC_ERR_ARG (bad sizes/NULL, or timing instrumentation switched on
 * with qmc_profile_enable, which creates events), QMC_ERR_ALIAS (X overlaps
 * A), QMC_ERR_WORKSPACE (qmc_workspace_size(plan, t) exceeds
 * QMC_NOALLOC_SCRATCH_BYTES: fewer columns, or a smaller chunk_pairs in the
 * plan's tuning, brings it under), QMC_ERR_HIP (the scratch address could not
 * be looked up).
 */
#define QMC_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int qmc_matmul_noalloc(qmc_plan_t plan, const void* A, int64_t t, int64_t lda,
                       void* X, int64_t ldx, void* stream);

/*
 * qmc_explicit_points -- write the N x s matrix Y itself (row stride ldy) in
 * conventional order, Y[n,j] = phi(point of n g_j): the input of the dense
 * baseline.  Y is device memory owned by the caller.
 */
int qmc_explicit_points(qmc_plan_t plan, void* Y, int64_t ldy, void* stream);

/*
 * qmc_dense_matmul -- the standard approach of the paper's experiments: the
 * plain product X = Y A (M x K by K x t, row-major, plan dtype) on the MFMA
 * matrix cores, for an explicit Y from qmc_explicit_points.  Sizes are
 * general (rows = N, K = s).  Used as the baseline the FFT path is compared with.
 */
int qmc_dense_matmul(qmc_plan_t plan, const void* Y, int64_t ldy, const void* A,
                     int64_t t, int64_t lda, void* X, int64_t ldx, void* stream);

/*
 * Batched products X_i = Y_i A_i for many plans of uneven size.
 *
 * qmc_batch_create binds `count` plans (same dtype) to their device
 * matrices A[i] (s_i x t[i], row stride lda[i], or t[i] if lda is NULL) and
 * X[i] (N_i x t[i], ldx[i] or t[i]); it uploads one descriptor per product
 * and synchronises `stream`.  The plans and buffers must outlive the batch.
 * qmc_batch_run enqueues, per run of products (below), one persistent launch
 * of each pass over the run's products: the collapse over all of them, the
 * fused pass once per on-chip transform size, the split once per split
 * radix and the back pass once per outer radix (the kernels are compiled
 * per size and radix).  It makes no host-to-device copies, so it can be
 * captured in a HIP graph and replayed.  Workspace: qmc_batch_workspace_size bytes, caller-owned.
 * Errors: QMC_ERR_ARG (bad arguments or mixed dtypes), QMC_ERR_ALIAS (at
 * create: some X[i] overlaps an A[k] or another X[k]; at run: the workspace
 * overlaps an operand), QMC_ERR_WORKSPACE.
 *
 * qmc_batch_set_chunk cuts the products (ordered by transform size and
 * radix) into runs of consecutive products whose intermediate spectra
 * (pairs x M complex values each) take at most chunk_bytes together, so
 * that the intermediate can stay in the Infinity Cache between the passes
 * that write and read it (a product larger than chunk_bytes runs alone; 0 =
 * one run of all products).  nt_inter chooses the stores of the intermediates as in
 * qmc_tuning_t (0: streaming for runs whose intermediates exceed 128 MiB).  A
 * new batch starts with QMC_BATCH_CHUNK_DEFAULT and nt_inter 0.  The runs
 * share the workspace, whose size changes with the chunk: query it
 * afterwards.  Uploads the new descriptors and synchronises `stream`; the
 * old descriptors are freed, so no run of the batch may be in flight (and a
 * graph that captured a run must be captured again).  QMC_ERR_ARG for a
 * negative chunk or nt_inter outside {0, 1, 2}; after any other failure the
 * batch holds no runs and qmc_batch_run returns QMC_ERR_ARG until a
 * regrouping succeeds.
 */
#define QMC_BATCH_CHUNK_DEFAULT ((int64_t)256 << 20)
typedef struct qmc_batch_s* qmc_batch_t;
int qmc_batch_create(qmc_batch_t* out, int count, const qmc_plan_t* plans, const int64_t* t,
                     const void* const* A, const int64_t* lda, void* const* X,
                     const int64_t* ldx, void* stream);
int qmc_batch_set_chunk(qmc_batch_t batch, int64_t chunk_bytes, int nt_inter, void* stream);

/*
 * qmc_batch_set_epilogue -- the epilogue of qmc_matmul_epilogue (Sections 3.2
 * and 3.3) for every product of the batch: X_i = scale_i * f(bias_i + Y_i A_i)
 * per column, one kind for all (QMC_EPI_*), bias[i] / scale[i] device arrays
 * of t[i] values in the plans' dtype (a NULL array, or a NULL entry, means
 * bias 0 / scale 1).  The vectors must outlive the batch's runs and must not
 * overlap any X of the batch (QMC_ERR_ALIAS; the batch is then unchanged).
 * Re-uploads the descriptors and synchronises `stream`, with the same
 * restrictions as qmc_batch_set_chunk.
 */
int qmc_batch_set_epilogue(qmc_batch_t batch, int kind, const void* const* bias,
                           const void* const* scale, void* stream);
int qmc_batch_workspace_size(qmc_batch_t batch, size_t* bytes);
int qmc_batch_run(qmc_batch_t batch, void* workspace, size_t workspace_bytes, void* stream);
void qmc_batch_destroy(qmc_batch_t batch);

/*
 * qmc_matmul_batched -- one-shot form: create a batch over dense row-major
 * A[i], X[i] (row stride t[i]), run it, synchronise `stream` and release the
 * batch.  Workspace: qmc_batched_workspace_size bytes.
 */
int qmc_batched_workspace_size(int count, const qmc_plan_t* plans, const int64_t* t,
                               size_t* bytes);
int qmc_matmul_batched(int count, const qmc_plan_t* plans, const void* const* A,
                       const int64_t* t, void* const* X, void* workspace,
                       size_t workspace_bytes, void* stream);

/*
 * Union of all Korobov lattice point sets (Section 2.2, after Hua and Wang):
 * for a prime K the N = (K-1)^2 points
 *     x_{b,n} = ({n b^0 / K + D}, {n b^1 / K + D}, ..., {n b^{s-1} / K + D}),
 *     b, n = 1..K-1,
 * in conventional order: row (b-1)(K-1) + (n-1) holds x_{b,n} (block b is
 * the Korobov lattice rule of base b without its point n = 0).  Every block
 * is one rank-1 lattice product sharing the spectrum of z (Section 2.2:
 * Y'_g = Z P_g); block b collapses A through the exponents
 * l_{b,j} = j log_beta(b) mod (K-1), which are c_{g,j} - 1 of the paper's
 * ordering for b = beta^(g-1), taken in [0, K-2].
 *
 * qmc_korobov_create -- tables for K, s, phi (as qmc_plan_create; the shift
 *   D = shift_num / shift_den may be 0 for every phi since no coordinate is 0;
 *   a nonzero shift with K D an integer puts one coordinate at 0, which the
 *   inverse normal CDF refuses with QMC_ERR_ARG), dtype.  Synchronous on `stream`.  Device memory grows as (K-1) times the
 *   collapse schedule of s rows.
 *   Errors: QMC_ERR_ARG (K < 3, s < 1, bad phi/dtype/shift), QMC_ERR_NOT_PRIME,
 *   QMC_ERR_OOM, QMC_ERR_HIP.
 * qmc_korobov_info -- N, s, K, L = K-1, the convolution layout and beta.
 * qmc_korobov_set_chunk -- blocks per run of the passes (0: all blocks);
 *   the workspace holds one run.
 * qmc_korobov_workspace_size -- device bytes qmc_korobov_matmul (and its
 *   epilogue and adjoint variants) need for t.
 * qmc_korobov_plan -- the lattice plan of K points whose spectrum and tables
 *   every block shares (owned by the union: valid until qmc_korobov_destroy;
 *   for qmc_plan_tables and the timing instrumentation, which also covers
 *   qmc_korobov_matmul; its own generating vector is all ones).
 * qmc_korobov_matmul -- X = Y A: A device s x t (row stride lda >= t), X
 *   device N x t (ldx >= t), every entry written; asynchronous on `stream`.
 *   Errors: QMC_ERR_ARG, QMC_ERR_ALIAS (X overlaps A), QMC_ERR_WORKSPACE.
 * qmc_korobov_matmul_epilogue -- the same with the per-column epilogue of
 *   qmc_matmul_epilogue (Sections 3.2, 3.3) in the writes of X.
 * qmc_korobov_matmul_adjoint -- dA = Y^T G: G device N x t (ldg >= t), dA
 *   device s x t (ldda >= t), every entry written; the blocks' parts are
 *   summed in increasing block order (so the result depends on the chunk of
 *   blocks only through rounding).  Same workspace query; QMC_ERR_UNSUPPORTED
 *   when the outer split keeps more than 32 values per back-pass column.
 */
typedef struct qmc_korobov_s* qmc_korobov_t;
typedef struct {
    int64_t K, s, N, L, M, M1, M2;
    int64_t blocks;          /* K - 1 */
    int64_t rounds;          /* collapse rounds per block (common to all blocks) */
    uint64_t beta;           /* primitive root used */
    int phi_kind, dtype;
    int64_t chunk_blocks;
} qmc_korobov_info_t;
int qmc_korobov_create(qmc_korobov_t* out, int64_t K, int64_t s, int phi_kind,
                       int64_t shift_num, int64_t shift_den, int dtype, void* stream);
int qmc_korobov_info(qmc_korobov_t U, qmc_korobov_info_t* info);
int qmc_korobov_set_chunk(qmc_korobov_t U, int64_t chunk_blocks);
int qmc_korobov_workspace_size(qmc_korobov_t U, int64_t t, size_t* bytes);
qmc_plan_t qmc_korobov_plan(qmc_korobov_t U);
int qmc_korobov_matmul(qmc_korobov_t U, const void* A, int64_t t, int64_t lda, void* X,
                       int64_t ldx, void* workspace, size_t workspace_bytes, void* stream);
int qmc_korobov_matmul_epilogue(qmc_korobov_t U, const void* A, int64_t t, int64_t lda,
                                void* X, int64_t ldx, int epi_kind, const void* bias,
                                const void* scale, void* workspace, size_t workspace_bytes,
                                void* stream);
int qmc_korobov_matmul_adjoint(qmc_korobov_t U, const void* G, int64_t t, int64_t ldg, void* dA,
                               int64_t ldda, void* workspace, size_t workspace_bytes,
                               void* stream);
void qmc_korobov_destroy(qmc_korobov_t U);

/*
 * Timing instrumentation for benchmarks.  When enabled, every kernel launch
 * of qmc_matmul / qmc_matmul_adjoint on this plan is bracketed by two HIP
 * events recorded on the launch stream.  qmc_profile_collect waits for the
 * recorded events, writes per kernel slot the summed elapsed milliseconds and
 * the number of launches (arrays of QMC_PROF_SLOTS entries, host memory) and
 * forgets the events.  Slot names: qmc_profile_slot_name.
 */
#define QMC_PROF_SLOTS 10
int qmc_profile_enable(qmc_plan_t plan, int on);
int qmc_profile_collect(qmc_plan_t plan, double* total_ms, int64_t* launches);
const char* qmc_profile_slot_name(int slot);

/* Human-readable name of an error code (static string). */
const char* qmc_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* QMC_H_ */
