// Internal declarations of librsm: the execution plan of one problem, the workspace
// layout, and the host-side launchers of every kernel (one source file per step).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include <vector>

#include "rsm.h"

// In the device pass the descriptors' pointers are typed as global memory, so accesses
// through them compile to global (not flat) instructions; the layout is the same.
#if defined(__HIP_DEVICE_COMPILE__)
#define RSM_GLOBAL __attribute__((address_space(1)))
#else
#define RSM_GLOBAL
#endif

namespace rsm {

constexpr int kWave = 64;                 // CDNA wavefront width
constexpr int kCholNB = 64;               // tile of the blocked Cholesky of N
constexpr int kEigPad = 4;                // extra vectors in the subspace iteration for V-hat
constexpr int kEigMaxB = RSM_MAX_R + kEigPad + 1;
constexpr int kEigMaxIters = 600;         // cap of the inverse-iteration steps
constexpr size_t kTileLdsBytes = 148 * 1024;  // LDS budget of the Y tile of the tiled Gram
constexpr int64_t kTileTargetGroups = 256;    // tiled Gram: workgroups to aim for (one per CU)

// Trials per workgroup of the split-BF16 Gram kernel (8 per wavefront, 8 wavefronts).
constexpr int kBfTrialsPerGroup = 64;

// U-hat: ranks from which the per-row normal equations are formed on the FP64 matrix cores
// (one dense product over all columns, 0/1 mask weights) instead of one thread per row.
constexpr int kUMfmaMinR = 6;

// Row of the matrix-core U-hat product's right operand, one per column j of Y:
// [v_ja v_jb for a >= b (r(r+1)/2 entries) | zeros to a multiple of 16 | v_j (r entries) |
// zeros], stored with this many doubles per row.  The stride is 16 mod 32 doubles, so the
// four rows a matrix-core fragment reads from LDS fall on alternate halves of the banks.
__host__ __device__ constexpr int uform_tiles_a(int r) { return (r * (r + 1) / 2 + 15) / 16; }
__host__ __device__ constexpr int uform_stride(int r) {
  return (uform_tiles_a(r) + 1) * 16 + (((uform_tiles_a(r) + 1) % 2 == 0) ? 16 : 0);
}

// Threads (= trials) per workgroup of the tiled Gram kernel: as many as the register file
// allows with l(l+1)/2 accumulators plus the prefetched next tile held per thread.
__host__ __device__ constexpr int tile_threads(int l, int elem_bytes) {
  return elem_bytes == 4 ? (l <= 10 ? 512 : 256) : (l <= 6 ? 512 : 256);
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr int kMaskOnesParts = 64;

// Trials per workgroup of the gathering Gram kernel when it pairs with the per-trial
// streamer (problems whose n-column tile does not fit LDS).
constexpr int kGatherPlainThreads = 256;

// Scalars the device passes between steps of one problem (lives in the workspace).
struct DevScalars {
  double mu;            // shift of the factorisation
  double lam_max;       // Gershgorin bound on lambda_max(N)
  int32_t pivots;       // clamped Cholesky pivots
  uint32_t bar;         // arrival count of the group solver's barrier
  uint32_t ticket;      // workgroup tickets of the group solver (first problem of a launch)
  uint32_t stalled;     // set when a group barrier wait timed out (the launch then stops)
  // known entries of W, counted while packing the mask: 64 partial counts (workgroup k of
  // the packing adds to entry k mod 64, so that no single address takes every atomic)
  unsigned long long mask_ones[kMaskOnesParts];
};

// Group form of the V-hat solver's subspace iteration: rows of the iterate per workgroup,
// and the per-workgroup partial sums it exchanges (doubles): two alternating buffers of
// b x b matrices and one of r squared residual norms, for ceil(n / kSubRows) workgroups,
// summed in workgroup order.
constexpr int kSubRows = 16;
__host__ __device__ constexpr int64_t sub_partials(int64_t n) {
  return (2 * kEigMaxB * kEigMaxB + RSM_MAX_R) * ((n + kSubRows - 1) / kSubRows);
}

// How one problem is executed and where its scratch lives in the workspace.
struct Plan {
  // problem (defaults resolved)
  int64_t m = 0, n = 0;
  int r = 0, l = 0, nvec = 0, min_rows = 0;
  int64_t I = 0, t0 = 0;
  uint64_t seed = 0;
  int prec = RSM_GRAM_F32;
  uint32_t flags = 0;
  int y_dtype = RSM_F32, y_layout = RSM_COL_MAJOR, w_layout = RSM_COL_MAJOR;
  // derived
  int64_t mw = 0;        // 64-row words per column of the mask bit-planes
  int ng = 0;            // l (l + 1) / 2 unique Gram entries
  bool tiled = false;    // tiled (LDS-reuse) Gram kernel instead of the per-trial streamer
  int splits = 1;        // row splits of the Gram step (partial Grams per trial)
  int64_t words_per_split = 0;  // 64-row mask words per split
  int eig_b = 0;         // subspace width of the V-hat iteration
  int nb = 0;            // Cholesky tiles per dimension
  int64_t npad = 0;      // 64 x (nb rounded up to a power of two): size of L^{-1}
  size_t part_elem = 4;  // bytes of one partial-Gram element
  int gram_groups = 0;   // tiled Gram: trial groups (workgroups per row split)
  int gram_threads = 0;  // tiled Gram: trials per workgroup (0: per-trial streamer)
  int gram_kernel = 0;   // tiled Gram staging: RSM_GRAM_KERNEL_REGS or _DMA (0: streamer)
  bool u_mfma = false;   // U-hat normal equations formed on the FP64 matrix cores
  bool minor_inv = false;  // minor vector by inverse iteration (nvec 1, no eigen taps)
  bool rows_first = false; // method M2: k-row subsets, qualifying columns (l holds k)
  int64_t nw = 0;          // 64-column words per row of the row bit-planes (M2)
  int gram_wgs = 0;      // workgroups of the Gram step of this problem
  // workspace offsets (bytes from the workspace base); ~0 = unused
  size_t off_wbits = 0, off_ypack = 0, off_cols = 0, off_part = 0, off_prow = 0, off_G = 0,
         off_rows = 0;
  size_t off_N = 0, off_Nsym = 0, off_L = 0, off_M = 0, off_Mt = 0, off_T = 0, off_X = 0,
         off_Z = 0, off_SP = 0, off_ab = 0, off_abcnt = 0, off_kext = 0, off_errp = 0,
         off_mflag = 0, off_rbits = 0, off_yrow = 0, off_B = 0, off_cmask = 0, off_Qd = 0;
  size_t off_scal = 0;
  size_t total = 0;
};


// Device-side description of one V-hat solve (step a6).  The solver's kernels take an array
// of these and run every problem of a batch in the same launch (problem = blockIdx.y); each
// workgroup reads its problem's sizes and buffers from here.
struct EigProb {
  int64_t n;             // order of N
  int64_t npad;          // order of M = L^{-1}: 64 x (tiles rounded up to a power of two)
  int32_t nb;            // 64 x 64 tiles per dimension of N
  int32_t b;             // subspace width
  int32_t r;             // target rank
  int32_t check_accepted;  // flag "no accepted trial" (off when only finalising a given N)
  int32_t deterministic;   // RSM_DETERMINISTIC: the solve's form may not depend on the batch
  int32_t pad_;
  uint64_t seed;         // start-vector stream
  RSM_GLOBAL const double* N;  // accumulated N (lower triangle, column-major n x n)
  RSM_GLOBAL double* Nsym;     // N with both triangles
  RSM_GLOBAL double* Lf;       // trailing matrix of the factorisation (lower)
  RSM_GLOBAL double* M;        // L^{-1}, npad x npad, lower tiles
  RSM_GLOBAL double* Mt;       // (L^{-1})^T, npad x npad, upper tiles
  RSM_GLOBAL double* T;        // recursion temporary (npad/2 x npad/2); row-sum and residual partials
  RSM_GLOBAL double* X;        // n x b iterate
  RSM_GLOBAL double* Z;        // n x b: L^{-1} X, then N X
  RSM_GLOBAL double* SP;       // sub_partials(n) doubles (group form of the iteration)
  RSM_GLOBAL DevScalars* scal;
  RSM_GLOBAL double* V;        // output n x r
  RSM_GLOBAL rsm_info* info;
};

// Device-side description of one problem for steps a0..a5 and a7 (problem index =
// blockIdx.y or .z of a launch, through an IdxList).
struct ProbDesc {
  int64_t m, n, mw, I, t0;
  int64_t ldw;           // caller's mask leading dimension
  int64_t ldy_in;        // caller's Y leading dimension
  int64_t ldy;           // leading dimension of the column-major Y the kernels read
  int32_t r, l, nvec, min_rows;
  int32_t y_layout, w_layout, splits, gram_groups;
  int64_t words_per_split;
  uint64_t seed;
  int32_t fixed_n;       // N accumulated as 64-bit fixed point (deterministic mode)
  int32_t pad_;
  double gram_unit;      // relative accuracy of the Gram's products and sums
  RSM_GLOBAL const uint8_t* W;
  RSM_GLOBAL const void* Yin;  // caller's Y
  RSM_GLOBAL void* ycm;        // column-major Y (the caller's, or the packed copy)
  RSM_GLOBAL uint64_t* wbits;
  RSM_GLOBAL const int32_t* user_subsets;
  RSM_GLOBAL int32_t* cols;
  RSM_GLOBAL void* part;
  RSM_GLOBAL int32_t* prow;
  RSM_GLOBAL double* G;
  RSM_GLOBAL int32_t* rows;
  RSM_GLOBAL double* N;
  RSM_GLOBAL double* V;
  RSM_GLOBAL double* U;
  RSM_GLOBAL rsm_info* info;
  RSM_GLOBAL DevScalars* scal;
  RSM_GLOBAL int32_t* tap_rows;
  RSM_GLOBAL double* tap_gram;
  RSM_GLOBAL double* tap_vecs;
  RSM_GLOBAL double* tap_eigs;
  RSM_GLOBAL int32_t* mflag;   // per trial: minor vector left to the Jacobi pass (I)
  RSM_GLOBAL double* ab;       // U-hat normal equations on MFMA: (r(r+1)/2 + r) x m, ld m
  RSM_GLOBAL int32_t* abcnt;   // known entries per row (m)
  RSM_GLOBAL double* kext;     // its right operand: ceil(n/32)*32 rows of uform_stride(r)
  RSM_GLOBAL double* errp;     // error of eq.(ep): one partial sum per 256 rows
  // method M2 (rows first)
  int32_t rows_first;
  int32_t nw;                  // 64-column words per row of rbits
  int64_t ldyr;                // leading dimension of the row-major Y in yrow
  RSM_GLOBAL uint64_t* rbits;  // row bit-planes: word w of row i, bit b = (W[i, 64 w + b] != 0)
  RSM_GLOBAL const void* yrow; // row-major Y (the caller's, or the packed copy)
  RSM_GLOBAL double* Bm;       // per trial k x r: u_a / s_a of the r leading pairs of H_t
  RSM_GLOBAL uint64_t* cmask;  // per trial nw words: the qualifying columns C_t
  RSM_GLOBAL double* Qd;       // per trial n x r (row j of Q_t at column j; C_t only)
};

// The problems of one launch: indices into a device ProbDesc array, passed by value.
constexpr int kLaunchMax = 256;
struct IdxList {
  int32_t count = 0;
  int32_t idx[kLaunchMax];
};

// Host launchers.  Each enqueues on `s` one launch (or one per storage layout) for every
// problem in `g`; `d` is the device descriptor array and `h[k]` the plan of problem
// g.idx[k].  Launchers that instantiate a kernel per l or r require the group to share it.
// Errors surface through hipGetLastError.
void launch_init_info(const ProbDesc* d, const IdxList& g, hipStream_t s);
void launch_pack(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s);
void launch_subsets(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s);
void launch_gram(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s);
// N between FP64 and its 64-bit fixed-point form (to_fixed: before accumulating onto a given
// N; otherwise back to FP64 after accumulating).
constexpr double kFixedScale = 1099511627776.0;  // 2^40
void launch_n_fixed(const ProbDesc* d, const IdxList& g, const Plan* const* h, bool to_fixed,
                    hipStream_t s);
void launch_minor(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s);
// Method M2: a0's row bit-planes and row-major Y; a2 + a3 (H_t), a4 + a5 (N update).
void launch_rows_pack(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s);
void launch_rows_gram(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s);
void launch_rows_minor(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s);
void launch_solve_u(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s);
void launch_error(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s);

// Planning (rsm_api.hip): a problem's own plan (validation, sizes, default Gram shape);
// the Gram row splits for `threads` trials per workgroup (splits_hint 0: this problem
// alone); the workspace offsets; all plans of a call, with the tile table applied.
int32_t make_plan(const rsm_problem& p, Plan& P);
int builtin_gram_kernel(int l, int prec, int y_dtype);
int default_gram_kernel(const Plan& P);
bool threads_built(int l, int prec, int y_dtype, int kernel, int threads);
int default_gram_threads(const Plan& P, int kernel);
void set_gram_shape(Plan& P, int threads, int64_t splits_hint);
void set_layout(Plan& P);
int32_t make_plans(const rsm_problem* problems, int32_t nprob, std::vector<Plan>& plans);

// Trials-per-workgroup values built for the tiled Gram of (l, precision, Y type) with the
// given staging kernel, ascending, into out[0..7]; returns their number (0: not built).
int gram_threads_built(int l, int prec, int y_dtype, int kernel, int* out);

// Whether the LDS-tiled Gram kernel can run this problem (its eligibility and matching
// element types).
bool gram_tiled_ok(const Plan& P);

// V-hat of `nprob` problems in the same launches.  `host` holds their descriptors on the
// host; `dev` is device memory for nprob descriptors (filled here, on the stream).
void launch_solve_v(const EigProb* host, int nprob, EigProb* dev, hipStream_t s);

// Copies `count` descriptors from the host to device memory `dev` on the stream (kernel
// arguments carry them; no host-to-device copy engine call).
void put_prob_descs(const ProbDesc* host, int count, ProbDesc* dev, hipStream_t s);

}  // namespace rsm
