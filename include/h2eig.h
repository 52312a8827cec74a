/*
 * h2eig — k-th eigenvalues of a symmetric H^2 matrix on one AMD MI355X (gfx950).
 *
 * The method is "slicing the spectrum" (Algorithm 1 of Apriansyah & Yokota,
 * "Computing the k-th Eigenvalue of Symmetric H^2-Matrices"): bisection on a
 * shift sigma, where each step needs the inertia nu(A - sigma I), the number of
 * eigenvalues below sigma (Sec. 2).  The inertia is read off the block-diagonal
 * factor of the generalized H^2-LDL factorization of Secs. 3.2-3.4 (Sylvester's
 * law of inertia, Sec. 4), computed level by level up the cluster tree on the GPU.
 *
 * Conventions for every call:
 *   - Return value: H2_OK (0) or a negative h2_status; h2_last_error() then
 *     returns a thread-local, NUL-terminated message (valid until the next call
 *     on the same thread).
 *   - Inputs are host arrays and are copied; the caller keeps ownership and may
 *     free them after the call returns.  Outputs are caller-allocated host arrays.
 *   - A handle owns all of its device memory until h2_free.  A handle must not be
 *     used from two threads at once (H2_EBUSY).
 *   - The library always runs its kernels on the GPU; if no usable gfx950 device
 *     is present every call that needs one fails with H2_EDEVICE.
 */
#ifndef H2EIG_H
#define H2EIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct h2_matrix_s* h2_matrix;

typedef enum {
  H2_OK = 0,
  H2_EINVAL = -1,    /* invalid argument (sizes, non-finite input, k out of range) */
  H2_ENOMEM = -2,    /* device or host memory exhausted, or workspace cap exceeded  */
  H2_EDEVICE = -3,   /* no usable GPU, or a HIP runtime error                       */
  H2_ENUMERIC = -4,  /* exactly singular or non-finite pivot block for some shift   */
  H2_EBUSY = -5      /* handle already in use by another thread                     */
} h2_status;

/* Kernel of the matrix: A_ij = f(|x_i - x_j|) for i != j, A_ii = diag.
 * The paper's synthetic test (Sec. 5.1) is H2_K_REG_LAPLACE with p0 = 1e-3. */
typedef enum {
  H2_K_LAPLACE = 0,       /* 1/r                                                */
  H2_K_YUKAWA = 1,        /* exp(-r)/r                                          */
  H2_K_GAUSS_DAMPED = 2,  /* exp(-r^2/p0) / (r + p1)                            */
  H2_K_REG_LAPLACE = 3,   /* 1/(r + p0)                                         */
  H2_K_TRIDIAG_1D = 4     /* -1 if |r - p0| < 1e-9*p0 else 0 (1-D test matrix)  */
} h2_kernel_kind;

typedef struct {
  int32_t kind;   /* h2_kernel_kind */
  double diag;    /* A_ii */
  double p0, p1;  /* kernel parameters (see h2_kernel_kind) */
} h2_kernel;

/* Build options (pass NULL for defaults). */
typedef struct {
  int32_t reserved0;         /* must be 0                                       */
  int32_t reserved1;         /* must be 0                                       */
  int32_t max_shifts;        /* shifts factored together per launch; 0 = auto   */
  int32_t reserved[5];
} h2_opts;

/*
 * Build the H^2 representation of the kernel matrix of n points in `dim`
 * dimensions (Sec. 3.1).
 *   points : host, n*dim doubles, row-major (point i at points[i*dim .. i*dim+dim-1]).
 *   leaf   : maximum cluster size at the leaf level (>= 2 unless n == 1).
 *   eta    : strong admissibility parameter: clusters i != j are admissible when
 *            eta * |c_i - c_j| >= rho_i + rho_j (bounding-box centres / half
 *            diagonals).
 *   eps    : compression tolerance; the absolute truncation threshold is
 *            tau = eps * normA (see h2_norm).  Used for the shared bases
 *            (Eq. shared-bases) and for fill-in recompression (Sec. 3.4).
 * On success *out receives a handle whose bases, couplings and leaf near blocks
 * (in skeleton coordinates, Eq. dense_skeleton) are resident in GPU memory.
 * Errors: H2_EINVAL (n < 1, dim not in 1..3, leaf < 2 with n > 1, eta <= 0,
 * eps <= 0, non-finite points, a singular kernel at coincident points),
 * H2_ENOMEM, H2_EDEVICE.
 * Environment H2EIG_PROGRESS=1: one line per tree level of the basis
 * construction on stderr.
 */
h2_status h2_build(const double* points, int64_t n, int32_t dim, h2_kernel kern,
                   int32_t leaf, double eta, double eps, const h2_opts* opts,
                   h2_matrix* out);

/*
 * Inertia counts nu_s = #{ lambda(A~) < sigma_s } for nshift shifts (Sec. 2,
 * Eq. for nu; Sec. 4), by the generalized H^2-LDL of A~ - sigma_s I.  All shifts
 * are factored on the GPU, batched.
 *   sigma  : host, nshift doubles.
 *   nu     : host output, nshift int64.
 *   status : optional host output (may be NULL), nshift int32: H2_OK or
 *            H2_ENUMERIC for a shift whose factorization met an exactly singular
 *            or non-finite pivot (its nu is then -1).
 * Returns H2_ENUMERIC if any shift failed (the others are still valid).
 * Every count obtained joins the handle's record cache of (sigma, nu) pairs,
 * kept sorted by sigma for the handle's lifetime, from which h2_kth_eig
 * narrows its brackets before factoring anything (Sec. 4.2).  Of a run of
 * records with equal counts only the first and the last can end a bracket, so
 * only those are kept: at most two records (16 bytes each) per distinct count.
 */
h2_status h2_inertia(h2_matrix A, const double* sigma, int64_t nshift,
                     int64_t* nu, int32_t* status);

/*
 * The same counts with the contractions of the basis rotation, elimination,
 * Schur updates and merge (Eqs. blr2-diag-elimination, blr2-diag-schur;
 * Sec. 3.3) multiplied in FP32 on the matrix cores with FP32 accumulation;
 * operands and results stay FP64 in memory, and the recompression (rank
 * decisions, Sec. 3.4) and the pivot-block LDL with its negative count run in
 * FP64.  Recompression truncates at max(eps, 1e-6) * normA instead of
 * eps * normA: rounding noise of the FP32 contractions (about 1e-7 of the
 * fill-in) is not kept as new directions, and the counts are those of a matrix
 * within about 1e-6 * normA of A~.  Meant for shifts far from every eigenvalue (early bisection steps):
 * a count may differ from h2_inertia's when an eigenvalue lies within the
 * FP32 error of sigma.  Arguments and errors as h2_inertia.  The counts do
 * not join the handle's record cache.
 */
h2_status h2_inertia_f32(h2_matrix A, const double* sigma, int64_t nshift,
                         int64_t* nu, int32_t* status);

/*
 * k-th smallest eigenvalues of A~ by Algorithm 1 (bisection), for nk 1-based
 * indices k[j] in [1, n], to absolute tolerance tol > 0:
 *   lambda[j] = midpoint of the final bracket, |lambda - lambda_k| < tol/2 when
 *   every inertia is correct (Eq. error-bound).
 *   ab     : optional [a, b] containing every requested eigenvalue; NULL = the
 *            Gershgorin interval of the kernel matrix widened by 10*eps*normA.
 *   bracket: optional output, 2*nk doubles (final [a_k, b_k]).
 * All active brackets contribute one shift each to a single batched
 * factorization per bisection step; inertia results are reused across the
 * requested indices and across calls through the record cache (Sec. 4.2).
 * A split point whose factorization meets an exactly singular pivot block is
 * moved inside its bracket (by 1/64 of the width, up to 8 times, then
 * H2_ENUMERIC).  With h2_set_mixed, wide brackets use h2_inertia_f32.
 * Environment H2EIG_PROGRESS=1: one line per bisection step on stderr.
 */
h2_status h2_kth_eig(h2_matrix A, const int64_t* k, int64_t nk, double tol,
                     const double* ab, double* lambda, double* bracket);

/*
 * Slicing the spectrum beyond one index (Sec. 2: nu(b) - nu(a) eigenvalues lie
 * in [a, b); Sec. 4.2: several eigenvalues share one interval and its inertia
 * records; Sec. 5.1 computes every eigenvalue this way, Sec. 5.2 the gap
 * between the highest occupied and the lowest unoccupied state).
 * h2_count   : *count = nu(b) - nu(a), the number of eigenvalues of A~ in
 *              [a, b) (two inertia evaluations; finite a <= b).
 * h2_eigs_in : every eigenvalue of A~ in [a, b), ascending, each by
 *              Algorithm 1 to absolute tolerance tol inside [a, b); lambda is a
 *              host array of cap doubles.  *count receives the number of
 *              eigenvalues in [a, b) even when it exceeds cap, in which case
 *              nothing else is computed and H2_EINVAL is returned.
 * h2_gap     : lambda_{k+1} - lambda_k for 1 <= k < n, both to tolerance tol
 *              (starting interval as h2_kth_eig with ab = NULL); lambda2, if
 *              not NULL, receives the two eigenvalues.
 * Errors as h2_inertia and h2_kth_eig.
 */
h2_status h2_count(h2_matrix A, double a, double b, int64_t* count);
h2_status h2_eigs_in(h2_matrix A, double a, double b, double tol, int64_t cap, double* lambda, int64_t* count);
h2_status h2_gap(h2_matrix A, int64_t k, double tol, double* lambda2, double* gap);

/* normA used for tau = eps*normA: max(mean row sum of A over rows i = 0 mod s,
 * |A_ii|), s = max(1, n/16384). */
h2_status h2_norm(h2_matrix A, double* normA);

/* Precision policy of h2_kth_eig (and of nothing else): a bracket is bisected
 * with h2_inertia_f32 while it is at least switch_rel * normA wide, then in
 * FP64.  At the switch its two ends, when FP32 counts set them, are counted in
 * FP64 and the bracket is rebuilt from FP64 counts alone (the largest shift
 * with fewer than k eigenvalues below it, then the smallest larger shift with
 * at least k), so a wrong FP32 decision falls back to the nearest FP64-checked
 * shifts.  0 (the default) = FP64 throughout.  H2_EINVAL for a negative or
 * non-finite value. */
h2_status h2_set_mixed(h2_matrix A, double switch_rel);

/* Default starting interval of Algorithm 1 (Sec. 2) used when h2_kth_eig gets
 * ab = NULL: the Gershgorin interval of the kernel matrix widened by
 * 10*eps*normA on both sides to cover the approximation error of the H^2
 * matrix.  ab: host output, 2 doubles.  Computed once per handle (all n^2
 * kernel entries, summed on the device), then cached.  H2_EDEVICE on a HIP
 * error. */
h2_status h2_interval(h2_matrix A, double* ab);

/* Shifts this handle factors together in one launch, from the free device
 * memory at the time of the call (the admission unit of the serving loop). */
h2_status h2_capacity(h2_matrix A, int32_t* max_shifts);

/* Block capacity (largest cluster dimension, rounded up to 8) of levels
 * 0..nlev-1 in the last factorization, 0 for levels it did not reach; shows
 * the rank growth level by level.  cap: host output, nlev ints. */
h2_status h2_level_dims(h2_matrix A, int32_t nlev, int32_t* cap);

/* Launch parameters of the dense contractions (the batched MFMA GEMM), by
 * operand layout (0 NN, 1 NT, 2 TN, 3 TT), precision (f32 0/1) and capacity
 * bucket (largest block dimension <= 256, 512, 1024, 2048, larger: 0..4):
 * grid = workgroups per shift (0 = built-in default, else a multiple of 8 in
 * [8, 65536]), group_m = tile-order group (tiles taken column by column within
 * groups of group_m tile rows; 0 or 1 = row by row), tile = output tile size
 * (64 or 128; 0 = 64).  The table is process-wide and written by the
 * autotuner's file at load time; set it while no factorization runs.  Results
 * do not depend on it.  H2_EINVAL for values out of range. */
h2_status h2_set_gemm_tuning(int32_t layout, int32_t f32, int32_t bucket, int32_t grid, int32_t group_m,
                             int32_t tile);
h2_status h2_get_gemm_tuning(int32_t layout, int32_t f32, int32_t bucket, int32_t* grid, int32_t* group_m,
                             int32_t* tile);

/* Free the handle's factorization workspace (it is allocated again, at the
 * size the next h2_inertia needs, by that call); the resident H^2 data stays.
 * The serving loop calls it when a matrix has nothing in flight.  H2_EBUSY,
 * H2_EDEVICE. */
h2_status h2_release_workspace(h2_matrix A);

/* Device-memory allocator of the library, process-wide (plumbing: no passage
 * of the paper defines it; the handle owns HBM through this hook, and a
 * framework points it at its own caching allocator).
 * Every device allocation made after the call (resident H^2 data, plans,
 * factorization workspace, construction scratch) calls alloc(bytes, ctx),
 * which returns device memory of the current device aligned to at least 256
 * bytes, or NULL (the call that needed it then fails with H2_ENOMEM).  Each
 * block is returned by release(ptr, ctx) of the allocator that made it, after
 * the device has finished all work queued so far (as hipFree), even if the
 * hook has changed since.  alloc = release = NULL restores hipMalloc/hipFree
 * for new blocks.  The callbacks may be called from any thread that uses the
 * library (the serving loop's workers included) and must be thread-safe.
 * H2_EINVAL if exactly one of alloc and release is NULL. */
h2_status h2_set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* ctx);

/* Cap on the shifts factored together in one launch (0 = automatic, from the
 * free device memory at each call); larger batches are split.  H2_EINVAL for
 * max_shifts < 0. */
h2_status h2_set_max_shifts(h2_matrix A, int32_t max_shifts);

typedef struct {
  int64_t n;
  int32_t levels;           /* depth L of the cluster tree (leaves at level L) */
  int32_t leaf_max;         /* largest leaf cluster                            */
  int32_t rank_max;         /* largest skeleton rank of the construction       */
  int32_t near_max;         /* largest near-list length (incl. self)           */
  int64_t near_blocks;      /* ordered near pairs at the leaf level            */
  int64_t resident_bytes;   /* device bytes held by the handle                 */
  int64_t last_work_bytes;  /* workspace bytes of the last factorization       */
  double last_flops;        /* algorithmic flops of the last factorization,
                               per shift (from the actual ranks)               */
  double last_bytes;        /* algorithmic HBM bytes per shift                 */
  double build_seconds;
  int32_t last_rank_max;    /* largest cluster dimension met in the last
                               factorization (after rank growth)               */
  int32_t evals_f64;        /* shifts factored in FP64 since h2_build          */
  int32_t evals_f32;        /* shifts factored with FP32 contractions          */
  int32_t reserved[3];
} h2_stats_t;

h2_status h2_stats(h2_matrix A, h2_stats_t* out);

/* Run subsequent work of this handle on the given hipStream_t (NULL = the
 * library's own stream). */
h2_status h2_set_stream(h2_matrix A, void* hip_stream);

/* Tree permutation: perm[p] = original index of the p-th point in leaf order
 * (n int64, host output). */
h2_status h2_tree_perm(h2_matrix A, int64_t* perm);

/*
 * Construction diagnostics (Sec. 3.1).
 * h2_basis_ranks: r[i] = rank of the shared basis of cluster i at tree level
 *   `level` (0 = root), i = 0 .. 2^level - 1 (host output).
 * h2_matvec: y = A~ x with the built H^2 matrix (near blocks, nested bases,
 *   couplings), evaluated on the host; x, y host arrays of n doubles in the
 *   original point order.
 * h2_kernel_matvec: y = A x with the exact kernel matrix (A_ii = diag), O(n^2)
 *   kernel evaluations on the GPU; x, y as above.
 * Together they measure the construction error ||A - A~|| at sizes where no
 * dense matrix fits.  Errors: H2_EINVAL (NULL argument, level out of range),
 * H2_EBUSY, H2_EDEVICE.
 */
h2_status h2_basis_ranks(h2_matrix A, int32_t level, int32_t* r);
/* Rank growth of the last factorization (Secs. 3.2-3.4): for shift `shift` of
 * the last h2_inertia call (0-based position in its batch) and every level
 * l < nlev, out[4l .. 4l+3] = (sum over the level's clusters of the directions
 * t added by recompression, sum of the cluster dimensions m, largest m, sum of
 * the pivot block sizes R); zeros for levels the factorization did not reach.
 * out: host, 4*nlev int64.  H2_EINVAL for a shift outside the last batch. */
h2_status h2_level_stats(h2_matrix A, int32_t shift, int32_t nlev, int64_t* out);
h2_status h2_matvec(h2_matrix A, const double* x, double* y);
h2_status h2_kernel_matvec(h2_matrix A, const double* x, double* y);

/*
 * h2_kernel_matvec without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same product y = A x (same kernel, same summation
 * order, hence the same bits), with the points, x and y staged through a
 * static 64 MiB device array held by each GPU the library runs on until the
 * process ends.  x, y: host arrays of n doubles, original point order.
 * n must be at most (8*2^20 - 96) / (dim + 2) points (1677702 in 3-D), else
 * H2_EINVAL.  Every call on one GPU shares that array: calls that overlap on
 * one GPU (several threads, several handles) race and must be serialised by
 * the caller.  Errors: H2_EINVAL, H2_EBUSY, H2_EDEVICE.
 */
h2_status h2_kernel_matvec_noalloc(h2_matrix A, const double* x, double* y);

/*
 * Diagnostic profiling (not needed for results).  When enabled, every kernel
 * launch of h2_inertia is bracketed by HIP events on the handle's stream, and
 * each kernel class accumulates its algorithmic flops (the method's own
 * operation counts from the actual per-shift ranks, e.g. 2*M*N*K per block
 * product, R^3/3 + R^3/3 per pivot LDL and its inverse) in device counters.
 * Enabling resets the totals.  Classes are numbered 0 .. h2_profile_classes()-1:
 * first the roles of the factorization (names such as "rotate", "schur"), then
 * one entry per operand layout of the MFMA GEMM kernel (names starting with
 * "kernel:"), which counts the same GEMM launches by kernel symbol.
 * enable = 2 brackets only the GEMM launches (less instrumentation; the
 * other classes then report flops but no time); 0 disables.
 */
h2_status h2_profile_enable(h2_matrix A, int32_t enable);
int32_t h2_profile_classes(void);
const char* h2_profile_class_name(int32_t cls);
/* launches: events pairs recorded; ms: summed event time; flops: algorithmic flops */
h2_status h2_profile_read(h2_matrix A, int32_t cls, int64_t* launches, double* ms, double* flops);
/* Algorithmic bytes of the GEMM launches of kernel symbol `cls` (a "kernel:"
 * class; 0 for the roles): per product, each operand read once, the per-K
 * weights, the output written (and read when accumulated) and its transposed
 * twin likewise, 8 bytes per element.  H2_EINVAL for a bad class or NULL. */
h2_status h2_profile_bytes(h2_matrix A, int32_t cls, double* bytes);
/* Diagnostic: milliseconds of class `cls` spent at tree level `level` (0 = root)
 * since profiling was enabled.  H2_EINVAL for a bad class, level (>= 32) or NULL. */
h2_status h2_profile_level_ms(h2_matrix A, int32_t cls, int32_t level, double* ms);

void h2_free(h2_matrix A);

/*
 * Serving loop (continuous batching of k-th eigenvalue queries over resident
 * matrices).  Every resident matrix gets a worker thread; each tick the worker
 * admits queued queries, merges the next bisection midpoint of every in-flight
 * query (Algorithm 1, Sec. 2) into one h2_inertia call on the matrix's stream,
 * narrows every bracket with every new inertia record (inertia reuse,
 * Sec. 4.2) and completes queries whose bracket is below their tolerance.
 * Matrices are served concurrently.
 * Admission by memory: the server holds one budget of device bytes for the
 * factorization workspace of all its matrices.  A matrix's workspace per shift
 * is measured when it is added; a worker admits a queued query only while the
 * budget holds one more shift of its matrix, else the query waits in the
 * queue, and a worker with nothing in flight frees its workspace and returns
 * its share to the budget.  The server does not own the matrices: free them
 * after h2s_destroy.  A matrix added to a server must not be used by the
 * caller until h2s_destroy.
 */
typedef struct h2_server_s* h2_server;
/* budget_bytes: device bytes for the workspace of all matrices (0 = 85% of the
 * free device memory now); max_slots: in-flight queries per matrix (0 = 64). */
h2_status h2s_create(int64_t budget_bytes, int32_t max_slots, h2_server* out);
/* Make A resident with at most `slots` queries in flight (0 = the server's
 * max_slots); id: index used by h2s_submit.  Runs one factorization (the
 * midpoint of the starting interval h2_interval, whose count seeds the
 * matrix's records) to measure the workspace of a shift, then frees it.
 * H2_ENOMEM if one shift needs more than the server's budget. */
h2_status h2s_add(h2_server S, h2_matrix A, int32_t slots, int32_t* id);
/* Queue a query for lambda_k (1-based, ascending) of matrix id to absolute
 * tolerance tol; returns immediately with a ticket.  H2_EINVAL for a bad id,
 * k outside [1, n] or tol <= 0. */
h2_status h2s_submit(h2_server S, int32_t id, int64_t k, double tol, int64_t* ticket);
/* done = 1 and lambda set once the query has finished; the status of a failed
 * factorization is returned for its queries.  A finished ticket is read once:
 * the call that reports it done (or failed) forgets it. */
h2_status h2s_poll(h2_server S, int64_t ticket, double* lambda, int32_t* done);
/* Block until the query has finished (H2_EINVAL if the server stops first);
 * forgets the ticket as h2s_poll does.  If another h2s_poll or h2s_wait reads
 * the ticket first, this call returns H2_EINVAL. */
h2_status h2s_wait(h2_server S, int64_t ticket, double* lambda);
/* Latency percentiles (submission to completion, ms) of the finished queries,
 * and the numbers of finished and submitted queries. */
h2_status h2s_stats(h2_server S, double* p50_ms, double* p99_ms, int64_t* served, int64_t* submitted);
/* Censored latency: percentiles over every submitted query, an unfinished one
 * counted at its time since submission (a lower bound of its latency);
 * unfinished = queries queued or in flight now; the budget and the bytes of
 * it held now.  Any output may be NULL. */
h2_status h2s_latency(h2_server S, double* p50_ms, double* p99_ms, int64_t* unfinished, int64_t* budget_bytes,
                      int64_t* used_bytes);
/* Stop the workers (in-flight queries are abandoned; a worker inside a
 * factorization finishes it first), free the factorization workspace of every
 * added matrix and free the server.  No other h2s_ call on S may be running
 * or follow: join the threads that poll or wait first. */
void h2s_destroy(h2_server S);

const char* h2_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* H2EIG_H */
