/*
 * rsm.h — C ABI of librsm, the MI355X (gfx950) implementation of the hot path of the
 * Random SubMatrix method (RSM) for low-rank decomposition with missing entries:
 *
 *   Y. Liu, "A random algorithm for low-rank decomposition of large-scale matrices with
 *   missing entries", arXiv:1411.0814.
 *
 * The problem (eq.(problem)): given Y (m x n) and a mask W (w_ij = 1 where y_ij is known),
 * find U (m x r) and V (n x r) minimising ||W o (Y - U V^T)||.  The library runs the
 * paper's three steps (Section IV-A) with method M1 and the L2 norm:
 *
 *   a1  draw I random l-column subsets C_t (l = r + 1 by default)             [step 1-2, M1]
 *   a2  keep the rows R_t whose entries at C_t are all known                  [M1]
 *   a3  form the l x l Gram G_t = Z_t^T Z_t of Z_t = Y[R_t, C_t]
 *   a4  its nvec = l - r eigenvectors of the smallest eigenvalues, i.e. the minor right
 *       singular vectors zeta of Z_t                                           [Section III]
 *   a5  N += e(zeta) e(zeta)^T, N = Xi Xi^T                     [eq.(get_xi), eq.(XI)]
 *   a6  V-hat = the r eigenvectors of N with the smallest eigenvalues
 *                                                              [eq.(solve.barV_L2_norm)]
 *   a7  U-hat row by row: u_i = argmin_u sum_j w_ij (y_ij - u^T v_j)^2      [eq.(solve.barU)]
 *
 * With RSM_ROWS_FIRST the sub-matrices are drawn by the paper's method M2 instead
 * (Section III): a1 draws k-row subsets S_t of [0, m); a2 keeps the columns C_t whose
 * entries at S_t are all known; a3 forms the k x k Gram H_t = Z_t Z_t^T of
 * Z_t = Y[S_t, C_t]; a4 takes H_t's r largest eigenpairs (u_a, s_a^2), whose vectors
 * q_a = Z_t^T u_a / s_a are Z_t's r leading right singular vectors; a5 adds the projector
 * on all |C_t| - r remaining right singular vectors (null vectors included),
 * I - Q_t Q_t^T, into N[C_t, C_t].  Steps a6 and a7 are shared.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller; the library never allocates
 *     device memory.  Scratch memory is the caller's `workspace` (size from
 *     rsm_workspace_bytes).  Structs themselves (rsm_problem, rsm_input, rsm_output) are
 *     host memory, read during the call only.
 *   - Work is enqueued asynchronously on the caller's HIP stream (`hip_stream`, a
 *     hipStream_t; NULL = the default stream).  Results are valid once the stream has
 *     reached that point.  Inputs must stay valid and unmodified until then.
 *   - Every argument is validated on the host before anything is enqueued: a negative
 *     return (RSM_E_*) means nothing was launched.  RSM_E_DEVICE means a launch failed
 *     part-way; the outputs are then undefined.
 *   - Data-dependent conditions are reported in the device-side rsm_info (`warn` bit
 *     flags RSM_W_*), never as a return value.
 *   - Outputs are FP64, column-major.  V-hat (n x r) has orthonormal columns ordered by
 *     ascending eigenvalue of N; U-hat is m x r with leading dimension m.  Only the
 *     subspace of V-hat (and the product U-hat V-hat^T) is unique.
 *   - Calls on different streams that use different workspaces and outputs may overlap.
 */
#ifndef RSM_H
#define RSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSM_ABI_VERSION 1

/* Size limits of this build. */
#define RSM_MAX_R 16          /* rank r */
#define RSM_MAX_L 17          /* columns per sub-matrix l (r < l <= RSM_MAX_L) */
#define RSM_MAX_N 2048        /* columns of Y */

/* Return values.  Negative: error, nothing (or, for RSM_E_DEVICE, not everything) was
 * enqueued.  Warnings are never returned; they are bits of rsm_info.warn. */
enum {
  RSM_OK = 0,
  RSM_E_ARG = -1,          /* a NULL pointer, a size out of range, an inconsistent field */
  RSM_E_WORKSPACE = -2,    /* ws_bytes below rsm_workspace_bytes(), or workspace misaligned */
  RSM_E_DEVICE = -3,       /* a HIP launch or query failed */
  RSM_E_UNSUPPORTED = -4,  /* valid request outside this build's limits (RSM_MAX_*) */
  RSM_E_SCRATCH = -5       /* rsm_decompose_noalloc: the problem's workspace exceeds
                              RSM_NOALLOC_MAX_BYTES */
};

/* Bits of rsm_info.warn (per problem, written by the device). */
enum {
  RSM_W_NO_CONSTRAINTS = 1,      /* no trial was accepted: N == 0, V-hat arbitrary */
  RSM_W_RANK_DEFICIENT = 2,      /* a column of Y was never sampled (N_jj == 0), or
                                    lambda_{r+1}(N) <= 1e-12 lambda_max(N): V-hat not unique */
  RSM_W_ROWS_UNDERDETERMINED = 4,/* some rows have fewer than r known entries: u_i = 0 */
  RSM_W_NOT_CONVERGED = 8,       /* eigen-solver residual of N above its tolerance */
  RSM_W_BAD_SUBSET = 16,         /* a caller-supplied subset was out of range or unsorted;
                                    that trial was rejected */
  RSM_W_PIVOT = 32               /* a Cholesky pivot of N + mu I was clamped */
};

/* Element type of Y. */
enum { RSM_F32 = 0, RSM_F64 = 1 };

/* Storage order of Y and W.  RSM_COL_MAJOR: element (i, j) at [i + j * ld] (the paper's
 * Matlab order; read in place).  RSM_ROW_MAJOR: at [i * ld + j] (repacked once into the
 * workspace). */
enum { RSM_COL_MAJOR = 0, RSM_ROW_MAJOR = 1 };

/* Arithmetic of the Gram step a3.  The l x l eigen-solves (a4), the n x n eigen-solve
 * (a6) and the r x r solves (a7) are FP64 in every mode. */
enum {
  RSM_GRAM_F64 = 0,        /* FP64 products and sums */
  RSM_GRAM_F32 = 1,        /* FP32 products, FP32 sums over row chunks, FP64 across chunks */
  RSM_GRAM_BF16X2 = 2      /* split-BF16 (hi + lo) products on MFMA, FP32 accumulate */
};

/* rsm_problem.flags */
enum {
  RSM_ACCUMULATE_ONLY = 1u << 0, /* stop after a5: N only (no V-hat, no U-hat) */
  RSM_FINALIZE_ONLY = 1u << 1,   /* skip a1..a5: take N from out->N, run a6 and a7 */
  RSM_N_ACCUMULATE = 1u << 2,    /* add this call's trials onto the N passed in out->N
                                    instead of starting from zero (resume / sharding) */
  RSM_COMPUTE_ERROR = 1u << 3,   /* fill rsm_info.e (eq.(ep)) with an extra pass over Y */
  RSM_PLAIN_GRAM = 1u << 4,      /* use the per-trial column-streaming Gram kernel alone
                                    (the unblocked baseline) instead of the tiled or the
                                    gathering one */
  RSM_DETERMINISTIC = 1u << 5,   /* bitwise-reproducible results, whatever else shares the
                                    launches: N is accumulated in 64-bit fixed point with
                                    2^-40 resolution (integer atomics, order-free) instead
                                    of FP64 atomics.  Needs |N_ij| < 2^23 (at most 2^23
                                    trials per column pair); a caller's N given with
                                    RSM_N_ACCUMULATE is first rounded to that grid.  (The
                                    optional error e is summed in a fixed order with or
                                    without this flag.) */
  RSM_ROWS_FIRST = 1u << 6,      /* method M2 (Section III, rows first; see the top of
                                    this file).  Then `l` is the number k of rows per
                                    sub-matrix (0 => r + 1; r < k <= min(m, RSM_MAX_L),
                                    m <= 2^31 - 1), `nvec` must be 0 (every trial gives
                                    |C_t| - r vectors), `min_rows` is the least |C_t| for a
                                    trial to count (0 => r + 1; must exceed r; the paper
                                    forms a sub-matrix only with more than r columns,
                                    Section IV-A), subsets (drawn or given) are row
                                    indices in [0, m), H_t is formed in FP64 whatever
                                    gram_prec says (RSM_GRAM_BF16X2 and RSM_PLAIN_GRAM are
                                    RSM_E_UNSUPPORTED), and trial_vecs must be NULL.
                                    The workspace then also holds the row bit-planes,
                                    a row-major copy of a column-major Y, and I x n x r
                                    doubles for the rows of every trial's Q_t. */
  RSM_SERIAL_STEPS = 1u << 7     /* rsm_decompose_batched: run each step's launch groups
                                    one after another on the caller's stream.  Without it
                                    a call of at least 64 problems runs the groups of its
                                    Gram, minor-vector and U-hat steps side by side on
                                    streams of the library (made once per device, default
                                    priority), joined back into the caller's stream before
                                    the next step.  For callers that overlap several calls
                                    on streams of their own (lanes shared by those calls
                                    would queue one call's launches behind another's).  Set
                                    on any problem of a call, it holds for the whole call;
                                    results do not depend on it. */
};

typedef struct rsm_problem {
  int64_t m, n;              /* Y is m x n; 1 <= r < min(m, n); n <= RSM_MAX_N */
  int32_t r;                 /* target rank */
  int32_t l;                 /* columns per sub-matrix; 0 => r + 1; r < l <= min(n, RSM_MAX_L) */
  int32_t nvec;              /* minor vectors per accepted sub-matrix; 0 => l - r; 1..l-r */
  int32_t min_rows;          /* accept trial t iff |R_t| >= min_rows; 0 => r */
  int64_t num_submatrices;   /* I: trials drawn (rejected ones included); >= 0 */
  int64_t trial_begin;       /* counter of the first trial (resume / sharding); >= 0 */
  uint64_t seed;             /* key of the subset generator */
  int32_t gram_prec;         /* RSM_GRAM_* */
  uint32_t flags;            /* RSM_* flags above */
  int32_t y_dtype;           /* RSM_F32 | RSM_F64: element type of Y */
  int32_t y_layout;          /* RSM_COL_MAJOR | RSM_ROW_MAJOR: storage order of Y */
  int32_t w_layout;          /* RSM_COL_MAJOR | RSM_ROW_MAJOR: storage order of W */
  int32_t reserved;          /* must be 0 */
} rsm_problem;

/* Subset generator (a1), identical on every implementation: trial t's column subset is
 * Floyd's sampling (Bentley & Floyd, CACM 1987) driven by the 64-bit words of
 * Philox4x64-10 (Salmon et al., SC'11) with key (seed, 0) and counter (b, t, 0, 0), words
 * taken block b = 0, 1, ... in order: for i = 0..l-1, j = n-l+i, x = mulhi64(u_i, j+1);
 * insert j if x is taken, else x.  The subset is sorted ascending. */

typedef struct rsm_input {
  const void* Y;             /* device, m x n of y_dtype in y_layout, leading dimension ldy:
                                col-major ldy >= m, row-major ldy >= n */
  int64_t ldy;
  const uint8_t* W;          /* device, m x n bytes in w_layout, nonzero = known;
                                col-major ldw >= m, row-major ldw >= n */
  int64_t ldw;
  const int32_t* subsets;    /* optional device I x l row-major column indices replacing the
                                generator (each row sorted ascending, in [0, n)); NULL = draw */
} rsm_input;

/* Device-side report, one per problem (device memory, written by the library). */
typedef struct rsm_info {
  uint32_t warn;             /* RSM_W_* bits */
  int32_t uncovered;         /* columns j with N_jj == 0 */
  int64_t accepted;          /* trials with |R_t| >= min_rows */
  int64_t rows_total;        /* sum over all trials of |R_t| */
  int64_t rows_underdetermined; /* rows with fewer than r known entries */
  int64_t known;             /* sum of w_ij (numerator of rho, eq.(def.rho)) */
  int32_t eig_iterations;    /* inverse-iteration steps taken for V-hat */
  int32_t reserved;
  double lambda[RSM_MAX_R + 1]; /* Ritz values of N on the final subspace, ascending:
                                lambda_1..lambda_r (converged with V-hat) and an upper
                                bound on lambda_{r+1} (rest zero) */
  double residual;           /* max_k ||N v_k - lambda_k v_k|| / lambda_max(N) */
  double mu;                 /* shift used for the factorisation of N */
  double e;                  /* eq.(ep) if RSM_COMPUTE_ERROR, else NaN */
} rsm_info;

/* Steps of one decomposition, in launch order (for the optional step events below). */
enum {
  RSM_STEP_PACK = 0,     /* a0: mask bit-planes (and Y repack) */
  RSM_STEP_SUBSETS = 1,  /* a1 */
  RSM_STEP_GRAM = 2,     /* a2 + a3 */
  RSM_STEP_MINOR = 3,    /* a4 + a5 */
  RSM_STEP_EIG = 4,      /* a6 */
  RSM_STEP_USOLVE = 5,   /* a7 */
  RSM_STEP_ERROR = 6,    /* eq.(ep), only with RSM_COMPUTE_ERROR */
  RSM_NUM_STEPS = 7
};

typedef struct rsm_output {
  double* V;                 /* device n x r (ld n); required unless RSM_ACCUMULATE_ONLY */
  double* U;                 /* device m x r (ld m); required unless RSM_ACCUMULATE_ONLY */
  double* N;                 /* device n x n (ld n) or NULL (then kept in the workspace).
                                Written: the lower triangle and the diagonal (the upper
                                triangle is not touched).  Read when RSM_FINALIZE_ONLY or
                                RSM_N_ACCUMULATE is set. */
  rsm_info* info;            /* device, required */
  /* Optional per-trial taps (device, NULL = not written), trial index k = 0..I-1
     (with RSM_ROWS_FIRST: S_t, |C_t|, H_t and its eigenvalues; no vectors): */
  int32_t* trial_cols;       /* I x l: C_t */
  int32_t* trial_rows;       /* I: |R_t| */
  double* trial_gram;        /* I x l x l: G_t (as reduced in FP64) */
  double* trial_vecs;        /* I x nvec x l: minor vectors (zero for rejected trials) */
  double* trial_eigs;        /* I x l: eigenvalues of G_t, ascending */
  /* Optional host array of 2 * RSM_NUM_STEPS hipEvent_t created by the caller (NULL = none):
     element 2k is recorded on the stream just before step k, element 2k + 1 just after
     it.  Events of steps that do not run are left untouched. */
  void* const* step_events;
} rsm_output;

/* Library ABI version (RSM_ABI_VERSION of the build). */
int32_t rsm_abi_version(void);

/* Static text for a return value or a single RSM_W_* bit. */
const char* rsm_status_string(int32_t status);

/* Bytes of workspace rsm_decompose (nprob == 1) or rsm_decompose_batched needs for these
 * problems: each problem's scratch (256-byte aligned) plus one small area per call for the
 * device-side problem descriptors, so a batch needs slightly less than the sum of its
 * problems' single sizes.  Host only: no device call.  Returns RSM_E_ARG /
 * RSM_E_UNSUPPORTED for a problem the decomposition would reject. */
int32_t rsm_workspace_bytes(const rsm_problem* problems, int32_t nprob, size_t* bytes);

/* One decomposition (steps a1..a7, Section IV-A).  `workspace` is device memory of at
 * least rsm_workspace_bytes(p, 1) bytes, 256-byte aligned; its contents on entry do not
 * matter and on exit are undefined.  The call returns after enqueueing. */
int32_t rsm_decompose(const rsm_problem* p, const rsm_input* in, const rsm_output* out,
                      void* workspace, size_t ws_bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): rsm_decompose with its workspace taken
 * from a scratch array built into the library, RSM_NOALLOC_MAX_BYTES per device, held
 * until the process ends (its device address is looked up once per device, on the first
 * call there).  The caller still owns and passes Y, W and the outputs; the call allocates
 * nothing.  Returns RSM_E_SCRATCH, with nothing enqueued, when rsm_workspace_bytes(p, 1)
 * exceeds the limit; otherwise as rsm_decompose.  The device is the stream's (the current
 * device for the NULL stream).  Every call on a device shares that device's array: calls
 * that may overlap on one device (different streams, or host threads) race and must be
 * serialised by the caller; calls in order on one stream are safe. */
#define RSM_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int32_t rsm_decompose_noalloc(const rsm_problem* p, const rsm_input* in, const rsm_output* out,
                              void* hip_stream);

/* Several independent decompositions (uneven sizes allowed) fused into shared launches:
 * every step runs once for all problems that share its kernel instance (the Gram and
 * minor-vector steps per l, the U-hat step per r and element type of Y, the V-hat steps
 * for all problems together), each launch's extent set by its largest problem.
 * problems/inputs/outputs are host arrays of nprob entries; each problem's results equal
 * those of rsm_decompose on it alone, up to the order of floating-point accumulation
 * into N.  workspace: rsm_workspace_bytes(problems, nprob) bytes.  A call of 64 or more
 * problems runs the launch groups of its Gram, minor-vector and U-hat steps side by side
 * on the caller's stream and three streams of the library, joined back into the caller's
 * stream before the next step (see RSM_SERIAL_STEPS); everything the call enqueues is
 * still ordered after the caller's earlier work on hip_stream and before its later work. */
int32_t rsm_decompose_batched(int32_t nprob, const rsm_problem* problems,
                              const rsm_input* inputs, const rsm_output* outputs,
                              void* workspace, size_t ws_bytes, void* hip_stream);

/* ---------------------------------------------------------------------------------------
 * Step 1 (Section IV-A): how many sub-matrices to draw.  Host only: no device call, no
 * allocation, thread-safe.  Every function returns RSM_OK or RSM_E_ARG (a NULL output
 * pointer or an argument outside the stated range; the output is then untouched).
 *
 * Lemma 1: C_{n,rho}(k) = (1 - rho)^n at k = 0, 1 - rho^n at k = n, otherwise the standard
 * normal distribution function at sgn(k/n - rho) sqrt(2 n phi(k/n, rho)), phi the
 * Kullback-Leibler divergence of Bernoulli(k/n) from Bernoulli(rho).  It brackets the
 * binomial distribution function: C(k) <= P(X <= k) <= C(k + 1) for X ~ B(n, rho) (the
 * lemma's sum "up to k" read as inclusive).  Needs n >= 1, 0 <= k <= n, 0 < rho < 1. */
int32_t rsm_lemma1_c(int64_t n, double rho, int64_t k, double* value);

/* Theorem 3: after at most
 *     I = m n rho / (k (r + 1) (1 - C_{n, rho^k}(r + 2))) ln(1 / (1 - eps))
 * trials every known entry of Y has been in some sub-matrix with probability >= eps.
 * rows_first != 0: the theorem as stated, k = l rows per trial (method M2).
 * rows_first == 0: method M1 (l columns per trial), the same bound for Y^T (m and n
 * exchanged).  l = 0 means r + 1.  Needs m, n >= 1, r >= 1, l > r, 0 < rho < 1,
 * 0 < eps < 1 and r + 2 <= (columns kept per trial's side: n for M2, m for M1).  *bound is
 * +inf when a trial is unlikely to keep more than r columns (rows for M1). */
int32_t rsm_trials_bound(int64_t m, int64_t n, double rho, int32_t r, int32_t l, double eps,
                         int32_t rows_first, double* bound);

/* rsm_trials_bound rounded up to a trial count for num_submatrices; RSM_E_ARG as well when
 * the bound is infinite or does not fit an int64_t. */
int32_t rsm_plan_trials(int64_t m, int64_t n, double rho, int32_t r, int32_t l, double eps,
                        int32_t rows_first, int64_t* trials);

/* ---------------------------------------------------------------------------------------
 * Tile table (library-wide, host side).  The fused gather + Gram step (a2 + a3) has three
 * free parameters: how the tiled kernel stages Y (1: through registers, 32-row chunks; 2:
 * straight from global memory into LDS, 16-row chunks, fewer registers per thread; 3: as 2
 * with two chunk buffers, the next chunk's loads overlapping the sums), the
 * trials per workgroup (each thread owns one trial's l(l+1)/2 accumulators, so this is also
 * its thread count) and the number of workgroups a launch aims for (rows are split so that
 * trial groups x row splits reaches it; the row splits' partial Grams are summed in split
 * order afterwards).  The best pair
 * depends on l, precision, Y's element type and on whether the launch serves one problem
 * or a batch, and is found by timing (an autotuner sweeps the candidates on the caller's
 * workload and stores the winners here).  Launches without an entry, and every problem
 * with RSM_DETERMINISTIC, use the built-in shapes, so that a deterministic result never
 * depends on the table or on the other problems of a batch.
 *
 * The table is process-wide and guarded by a lock; a call reads it once while planning.
 * rsm_workspace_bytes and the decomposition must see the same table (the Gram row splits
 * size part of the workspace): change the table only between calls. */
typedef struct {
  int32_t l;             /* columns per sub-matrix, 2..RSM_MAX_L */
  int32_t gram_prec;     /* rsm_gram_prec */
  int32_t y_dtype;       /* rsm_dtype of Y */
  int32_t batched;       /* 0: the launch holds one problem; 1: several */
  int32_t gram_threads;  /* trials per workgroup, one of rsm_tune_threads(); 0 = built-in */
  int32_t gram_wgs;      /* workgroups the launch aims for, 1..1048576; 0 = built-in */
  int32_t gram_kernel;   /* RSM_GRAM_KERNEL_*; 0 = built-in */
} rsm_tune_entry;

#define RSM_GRAM_KERNEL_REGS 1  /* tiled Gram staging Y through registers */
#define RSM_GRAM_KERNEL_DMA 2   /* tiled Gram loading Y straight into LDS (FP32 Y and Gram) */
#define RSM_GRAM_KERNEL_DMA2 3  /* the same with two chunk buffers (loads overlap the sums);
                                   FP32 Y with FP32 or FP64 sums */
#define RSM_GRAM_KERNEL_GATHER 4 /* only the mask words staged in LDS, each trial's
                                    qualifying values loaded straight from Y (for trials
                                    that keep few rows) */
#define RSM_GRAM_KERNEL_AUTO 5  /* GATHER or the staging kernel (DMA2 for FP32 Y, REGS for
                                   FP64 Y) per problem, by the mask's density: the built-in
                                   choice for every precision but split-BF16 */

/* Replaces the table with `count` entries (0 clears it; later duplicates of a key win).
 * RSM_E_ARG, and the table unchanged, for an entry outside the ranges above, a kernel not
 * built for its (l, precision, type) or a thread count not built for that kernel. */
int32_t rsm_tune_set(const rsm_tune_entry* entries, int32_t count);

/* Copies up to `cap` entries of the table into `entries` (may be NULL when cap is 0) and
 * the table's size into *count. */
int32_t rsm_tune_get(rsm_tune_entry* entries, int32_t cap, int32_t* count);

/* The trials-per-workgroup values built for the tiled Gram of (l, gram_prec, y_dtype) with
 * staging `gram_kernel` (RSM_GRAM_KERNEL_*), ascending: up to `cap` into `threads`, their
 * number into *count (0 when that kernel does not run that combination, e.g. the per-trial
 * streaming kernel's cases). */
int32_t rsm_tune_threads(int32_t l, int32_t gram_prec, int32_t y_dtype, int32_t gram_kernel,
                         int32_t* threads, int32_t cap, int32_t* count);

#ifdef __cplusplus
}
#endif

#endif /* RSM_H */
