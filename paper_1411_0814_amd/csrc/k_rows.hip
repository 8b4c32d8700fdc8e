// Method M2 (Section III, rows first): a k-row subset S_t of [0, m), the columns C_t whose
// entries at S_t are all known, Z_t = Y[S_t, C_t] (k x |C_t|), and the |C_t| - r right
// singular vectors of Z_t past its r leading ones (null vectors included), accumulated
// into N as the projector I - Q_t Q_t^T on C_t x C_t.
//
//  a0  k_pack_rowbits: W -> row bit-planes (word w of row i: bit b = W[i, 64 w + b] != 0);
//      k_transpose_rows: column-major Y -> row-major copy (row-major Y is read in place).
//  a2 + a3  k_m2_gram: one wavefront per trial.  The qualifying-column word of 64 columns
//      is the AND of the k row words; lane b owns column 64 w + b, loads its k entries
//      (a coalesced read of 64 consecutive entries of each chosen row), and the k x k Gram
//      H_t = Z_t Z_t^T is summed in FP64 over the words, one entry per lane.
//  a4  k_m2_eig_reg (k <= 11) / k_m2_eig: one thread per trial, cyclic Jacobi (FP64) on
//      H_t = U diag(s^2) U^T (packed in registers, or in LDS for larger k); the r largest
//      eigenpairs give B_t = [u_a / s_a] (k x r), so that the leading right singular
//      vectors of Z_t are Q_t = Z_t^T B_t.
//  a5  N[C_t, C_t] += I - Q_t Q_t^T (lower triangle) in two passes:
//      k_m2_qform: one wavefront per trial; lane b of word w computes row 64 w + b of Q_t,
//      q = B_t^T z (z: the column's k chosen entries), into a dense trial x column x r
//      array (only qualifying columns are written or read).
//      k_m2_tiles: one workgroup per 64 x 64 block of N (lower blocks) and range of trials.
//      The block stays in LDS; each wavefront takes one trial at a time (the next trial's
//      mask words and rows loading meanwhile), finds the trial's columns inside the block's
//      row and column ranges from two mask words, holds their rows of Q_t in registers (lane
//      b: columns 64 bi + b and 64 bj + b), forms every pair's -q_i . q_j (+1 on the
//      diagonal) with one lane per pair and cross-lane reads, and adds it to the block with
//      LDS atomics.  The block is then added into N with one global atomic per entry.
//      Deterministic mode uses 64-bit fixed point in LDS and in N (integer atomics,
//      order-free).  A trial is skipped by every pass when it has fewer than min_rows
//      qualifying columns (default r + 1; its mask words are then stored empty).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

constexpr int kMaxK = RSM_MAX_L;
constexpr double kJacobiEpsM2 = 2.220446049250313e-16;  // 2^-52
constexpr int kJacobiSweepsM2 = 40;
// An eigenvalue s_a^2 of H_t at or below this fraction of the largest is taken as zero
// (its direction is dropped from Q_t): below it the direction is set by rounding.
constexpr double kRankTolM2 = 1e-13;

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ __forceinline__ double ld_y(RSM_GLOBAL const T* y, int64_t idx) {
  return static_cast<double>(y[idx]);
}

// ------------------------------------------------------------------ a0

// Row bit-planes from W in either storage order: a 64-row x 256-column byte tile through
// LDS (loads coalesced along the storage order, 8-byte aligned rows), then each thread packs
// one 64-column word of one row, 8 bytes at a time.
// Grid (64-row tiles, 256-column tiles, problems).
constexpr int kRbCols = 256;
constexpr int kRbStride = kRbCols + 8;

__global__ __launch_bounds__(256) void k_pack_rowbits(const ProbDesc* __restrict__ probs,
                                                      IdxList list) {
  __shared__ __align__(8) uint8_t tile[64][kRbStride];
  const ProbDesc& P = probs[list.idx[blockIdx.z]];
  const int64_t m = P.m, n = P.n;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int64_t j0 = static_cast<int64_t>(blockIdx.y) * kRbCols;
  if (i0 >= m || j0 >= n) return;
  const bool rowmajor = P.w_layout == RSM_ROW_MAJOR;
  for (int e = threadIdx.x; e < 64 * kRbCols; e += blockDim.x) {
    // row-major: consecutive threads take consecutive columns; column-major: rows
    const int rr = rowmajor ? e / kRbCols : e % 64;
    const int cc = rowmajor ? e % kRbCols : e / 64;
    const int64_t i = i0 + rr, j = j0 + cc;
    uint8_t v = 0;
    if (i < m && j < n) v = rowmajor ? P.W[i * P.ldw + j] : P.W[i + j * P.ldw];
    tile[rr][cc] = v;
  }
  __syncthreads();
  const int rr = threadIdx.x / 4, wd = threadIdx.x % 4;
  const int64_t i = i0 + rr, w = j0 / 64 + wd;
  if (i < m && w < P.nw) {
    const uint64_t* src = reinterpret_cast<const uint64_t*>(&tile[rr][64 * wd]);
    uint64_t word = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) word |= static_cast<uint64_t>(nonzero_bytes_to_bits(src[b])) << (8 * b);
    P.rbits[i * P.nw + w] = word;
  }
}

// Column-major Y -> row-major copy (leading dimension n), 64 x 64 tiles through LDS.
// Grid (row tiles, column tiles, problems).
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_rows(const ProbDesc* __restrict__ probs,
                                                        IdxList list) {
  __shared__ T tile[64][65];
  const ProbDesc& P = probs[list.idx[blockIdx.z]];
  const int64_t m = P.m, n = P.n;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int64_t j0 = static_cast<int64_t>(blockIdx.y) * 64;
  if (i0 >= m || j0 >= n) return;
  auto src = static_cast<RSM_GLOBAL const T*>(P.Yin);
  auto dst = static_cast<RSM_GLOBAL T*>(const_cast<RSM_GLOBAL void*>(P.yrow));
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const int rr = e % 64, cc = e / 64;
    const int64_t i = i0 + rr, j = j0 + cc;
    tile[rr][cc] = (i < m && j < n) ? src[i + j * P.ldy_in] : T(0);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const int rr = e / 64, cc = e % 64;
    const int64_t i = i0 + rr, j = j0 + cc;
    if (i < m && j < n) dst[i * P.ldyr + j] = tile[rr][cc];
  }
}

// ------------------------------------------------------------------ a2 + a3

constexpr int kGramWaves = 4;

// Grid (ceil(I / 4), problems); one wavefront per trial.
template <typename T>
__global__ __launch_bounds__(64 * kGramWaves) void k_m2_gram(const ProbDesc* __restrict__ probs,
                                                            IdxList list) {
  __shared__ double zs[kGramWaves][kMaxK][64];
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kGramWaves + wv;
  if (t >= P.I) return;  // whole wavefront (no workgroup barrier below)
  const int k = P.l, nw = P.nw;
  const int ng = k * (k + 1) / 2;
  auto y = static_cast<RSM_GLOBAL const T*>(P.yrow);
  const int64_t ldyr = P.ldyr;
  int S[kMaxK];
  bool valid = true;
#pragma unroll
  for (int i = 0; i < kMaxK; ++i) {
    S[i] = i < k ? P.cols[t * k + i] : 0;
    valid &= S[i] >= 0;
  }
  // lane w < nw: the qualifying-column word w (AND over the k chosen rows)
  uint64_t myword = 0;
  if (valid && ln < nw) {
    myword = ~0ull;
#pragma unroll
    for (int i = 0; i < kMaxK; ++i)
      if (i < k) myword &= P.rbits[static_cast<int64_t>(S[i]) * nw + ln];
  }
  const int cnt = static_cast<int>(wave_sum(static_cast<int64_t>(__popcll(myword))));
  // entries of H owned by this lane: e = ln, ln + 64, ln + 128 (packed lower, a >= b)
  int ea[3], eb[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int e = ln + 64 * s;
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= e) ++a;
    ea[s] = a;
    eb[s] = e - a * (a + 1) / 2;
  }
  double acc[3] = {0.0, 0.0, 0.0};
  // this lane's entries of the k chosen rows at column 64 w + ln (zero if not qualifying);
  // the next word's are loaded while the current one is summed
  auto load_z = [&](int w, double* z) {
    const uint64_t word = w < nw ? __shfl(myword, w) : 0ull;
    const bool mine = (word >> ln) & 1ull;
    const int64_t col = static_cast<int64_t>(w) * 64 + ln;
#pragma unroll
    for (int i = 0; i < kMaxK; ++i)
      z[i] = (mine && i < k) ? ld_y(y, static_cast<int64_t>(S[i]) * ldyr + col) : 0.0;
  };
  double zc[kMaxK], zn[kMaxK];
  load_z(0, zc);
  for (int w = 0; w < nw; ++w) {
    load_z(w + 1, zn);
    const uint64_t word = __shfl(myword, w);
    if (word != 0) {
#pragma unroll
      for (int i = 0; i < kMaxK; ++i)
        if (i < k) zs[wv][i][ln] = zc[i];
      wave_fence();
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        if (ln + 64 * s < ng) {
          const double* za = zs[wv][ea[s]];
          const double* zb = zs[wv][eb[s]];
          double part = 0.0;
          for (int p = 0; p < 64; ++p) part = fma(za[p], zb[p], part);
          acc[s] += part;
        }
      }
      wave_fence();
    }
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) zc[i] = zn[i];
  }
#pragma unroll
  for (int s = 0; s < 3; ++s)
    if (ln + 64 * s < ng) P.G[static_cast<int64_t>(ln + 64 * s) * P.I + t] = acc[s];
  if (ln == 0) P.rows[t] = valid ? cnt : 0;
  // the mask words of C_t, empty for a rejected trial (the N-update passes skip it)
  if (ln < nw) P.cmask[t * nw + ln] = (cnt >= P.min_rows) ? myword : 0ull;
}

// ------------------------------------------------------------------ a4

// 16 trials per workgroup: enough workgroups to spread a few thousand trials over the CUs
template <int K>
constexpr int eig_tpb() {
  return 16;
}

// Grid (ceil(I / TPB), problems); one thread per trial, H and the rotations in LDS laid out
// [entry][thread] (conflict-free).
template <int K>
__global__ __launch_bounds__(eig_tpb<K>()) void k_m2_eig(const ProbDesc* __restrict__ probs,
                                                        IdxList list) {
  constexpr int TPB = eig_tpb<K>();
  constexpr int NG = K * (K + 1) / 2;
  __shared__ double Hs[NG * TPB];
  __shared__ double Vs[K * K * TPB];
  __shared__ unsigned long long s_acc, s_cols;
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_acc = 0;
    s_cols = 0;
  }
  __syncthreads();
  const int64_t I = P.I;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * TPB + tid;
  const bool active = t < I;
  const int r = P.r;
  auto A = [&](int i, int j) -> double& {
    return i >= j ? Hs[(i * (i + 1) / 2 + j) * TPB + tid] : Hs[(j * (j + 1) / 2 + i) * TPB + tid];
  };
  auto v = [&](int i, int j) -> double& { return Vs[(i * K + j) * TPB + tid]; };
  int cnt = 0;
  bool valid = false;
  if (active) {
    cnt = P.rows[t];
    valid = P.cols[t * K] >= 0;
#pragma unroll
    for (int g = 0; g < NG; ++g) Hs[g * TPB + tid] = P.G[static_cast<int64_t>(g) * I + t];
    if (P.tap_rows) P.tap_rows[t] = cnt;
    if (P.tap_gram)
      for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) P.tap_gram[(t * K + i) * K + j] = A(i, j);
  }
  const bool accept = active && valid && cnt >= P.min_rows;
  if (accept) {
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
      for (int j = 0; j < K; ++j) v(i, j) = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < kJacobiSweepsM2; ++sweep) {
      bool rotated = false;
      for (int p = 0; p < K - 1; ++p) {
        for (int q = p + 1; q < K; ++q) {
          const double apq = A(q, p);
          const double app = A(p, p);
          const double aqq = A(q, q);
          if (fabs(apq) > kJacobiEpsM2 * sqrt(fabs(app * aqq))) {
            rotated = true;
            // t = sign(d) e / (|d| + hypot(d, e)), d = a_qq - a_pp, e = 2 a_pq
            const double d = aqq - app;
            const double e2 = 2.0 * apq;
            const double den = fabs(d) + sqrt(d * d + e2 * e2);
            const double tr = (d >= 0.0 ? e2 : -e2) / den;
            const double cr = rsqrt(1.0 + tr * tr);
            const double sr = tr * cr;
            for (int kk = 0; kk < K; ++kk) {
              if (kk == p || kk == q) continue;
              const double akp = A(kk, p);
              const double akq = A(kk, q);
              A(kk, p) = cr * akp - sr * akq;
              A(kk, q) = sr * akp + cr * akq;
            }
            A(p, p) = app - tr * apq;
            A(q, q) = aqq + tr * apq;
            A(q, p) = 0.0;
            for (int kk = 0; kk < K; ++kk) {
              const double vkp = v(kk, p);
              const double vkq = v(kk, q);
              v(kk, p) = cr * vkp - sr * vkq;
              v(kk, q) = sr * vkp + cr * vkq;
            }
          }
        }
      }
      if (!rotated) break;
    }
    // rank of each eigenvalue, ascending (ties by index)
    int rank[K];
    double dmax = 0.0;
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const double dk = A(kk, kk);
      dmax = fmax(dmax, dk);
      int rk = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const double dj = A(j, j);
        rk += (dj < dk) || (dj == dk && j < kk);
      }
      rank[kk] = rk;
    }
    if (P.tap_eigs)
#pragma unroll
      for (int kk = 0; kk < K; ++kk) P.tap_eigs[t * K + rank[kk]] = A(kk, kk);
    // B_t[i][a] = u_a[i] / s_a for the r largest eigenvalues, a = 0 the largest
    RSM_GLOBAL double* B = P.Bm + t * K * r;
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int a = K - 1 - rank[kk];
      if (a < r) {
        const double dk = A(kk, kk);
        const double inv = (dk > kRankTolM2 * dmax && dk > 0.0) ? rsqrt(dk) : 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) B[i * r + a] = v(i, kk) * inv;
      }
    }
  } else if (active && P.tap_eigs) {
    for (int kk = 0; kk < K; ++kk) P.tap_eigs[t * K + kk] = 0.0;
  }
  if (accept) atomicAdd(&s_acc, 1ull);
  if (active) atomicAdd(&s_cols, static_cast<unsigned long long>(cnt));
  __syncthreads();
  if (tid == 0) {
    atomicAdd((unsigned long long*)&P.info->accepted, s_acc);
    atomicAdd((unsigned long long*)&P.info->rows_total, s_cols);
  }
}

// The same for k <= 11 with H_t packed in registers (static indices throughout) and the
// rotations in LDS: 64 trials per workgroup.
template <int K>
__global__ __launch_bounds__(64) void k_m2_eig_reg(const ProbDesc* __restrict__ probs,
                                                   IdxList list) {
  constexpr int TPB = 64;
  constexpr int NG = K * (K + 1) / 2;
  __shared__ double Vs[K * K * TPB];
  __shared__ unsigned long long s_acc, s_cols;
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_acc = 0;
    s_cols = 0;
  }
  __syncthreads();
  const int64_t I = P.I;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * TPB + tid;
  const bool active = t < I;
  const int r = P.r;
  double h[NG];
  auto A = [&](int i, int j) -> double& { return i >= j ? h[i * (i + 1) / 2 + j] : h[j * (j + 1) / 2 + i]; };
  auto v = [&](int i, int j) -> double& { return Vs[(i * K + j) * TPB + tid]; };
  int cnt = 0;
  bool valid = false;
#pragma unroll
  for (int g = 0; g < NG; ++g) h[g] = active ? P.G[static_cast<int64_t>(g) * I + t] : 0.0;
  if (active) {
    cnt = P.rows[t];
    valid = P.cols[t * K] >= 0;
    if (P.tap_rows) P.tap_rows[t] = cnt;
    if (P.tap_gram)
#pragma unroll
      for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) P.tap_gram[(t * K + i) * K + j] = A(i, j);
  }
  const bool accept = active && valid && cnt >= P.min_rows;
  if (accept) {
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
      for (int j = 0; j < K; ++j) v(i, j) = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < kJacobiSweepsM2; ++sweep) {
      bool rotated = false;
#pragma unroll
      for (int p = 0; p < K - 1; ++p) {
#pragma unroll
        for (int q = p + 1; q < K; ++q) {
          const double apq = A(q, p);
          const double app = A(p, p);
          const double aqq = A(q, q);
          if (fabs(apq) > kJacobiEpsM2 * sqrt(fabs(app * aqq))) {
            rotated = true;
            const double d = aqq - app;
            const double e2 = 2.0 * apq;
            const double den = fabs(d) + sqrt(d * d + e2 * e2);
            const double tr = (d >= 0.0 ? e2 : -e2) / den;
            const double cr = rsqrt(1.0 + tr * tr);
            const double sr = tr * cr;
#pragma unroll
            for (int kk = 0; kk < K; ++kk) {
              if (kk == p || kk == q) continue;
              const double akp = A(kk, p);
              const double akq = A(kk, q);
              A(kk, p) = cr * akp - sr * akq;
              A(kk, q) = sr * akp + cr * akq;
            }
            A(p, p) = app - tr * apq;
            A(q, q) = aqq + tr * apq;
            A(q, p) = 0.0;
#pragma unroll
            for (int kk = 0; kk < K; ++kk) {
              const double vkp = v(kk, p);
              const double vkq = v(kk, q);
              v(kk, p) = cr * vkp - sr * vkq;
              v(kk, q) = sr * vkp + cr * vkq;
            }
          }
        }
      }
      if (!rotated) break;
    }
    int rank[K];
    double dmax = 0.0;
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const double dk = A(kk, kk);
      dmax = fmax(dmax, dk);
      int rk = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const double dj = A(j, j);
        rk += (dj < dk) || (dj == dk && j < kk);
      }
      rank[kk] = rk;
    }
    if (P.tap_eigs)
#pragma unroll
      for (int kk = 0; kk < K; ++kk) P.tap_eigs[t * K + rank[kk]] = A(kk, kk);
    RSM_GLOBAL double* B = P.Bm + t * K * r;
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int a = K - 1 - rank[kk];
      if (a < r) {
        const double dk = A(kk, kk);
        const double inv = (dk > kRankTolM2 * dmax && dk > 0.0) ? rsqrt(dk) : 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) B[i * r + a] = v(i, kk) * inv;
      }
    }
  } else if (active && P.tap_eigs) {
    for (int kk = 0; kk < K; ++kk) P.tap_eigs[t * K + kk] = 0.0;
  }
  if (accept) atomicAdd(&s_acc, 1ull);
  if (active) atomicAdd(&s_cols, static_cast<unsigned long long>(cnt));
  __syncthreads();
  if (tid == 0) {
    atomicAdd((unsigned long long*)&P.info->accepted, s_acc);
    atomicAdd((unsigned long long*)&P.info->rows_total, s_cols);
  }
}

// ------------------------------------------------------------------ a5

// Grid (ceil(I / 4), problems); one wavefront per accepted trial.
template <typename T>
__global__ __launch_bounds__(64 * kGramWaves) void k_m2_qform(const ProbDesc* __restrict__ probs,
                                                             IdxList list) {
  __shared__ double sB[kGramWaves][kMaxK * RSM_MAX_R];
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kGramWaves + wv;
  if (t >= P.I) return;  // whole wavefront (no workgroup barrier below)
  const int k = P.l, r = P.r, nw = P.nw;
  if (P.cols[t * k] < 0 || P.rows[t] < P.min_rows) return;  // rejected
  auto y = static_cast<RSM_GLOBAL const T*>(P.yrow);
  const int64_t ldyr = P.ldyr, n = P.n;
  int S[kMaxK];
#pragma unroll
  for (int i = 0; i < kMaxK; ++i) S[i] = i < k ? P.cols[t * k + i] : 0;
  for (int e = ln; e < k * r; e += 64) sB[wv][e] = P.Bm[t * k * r + e];
  wave_fence();
  const uint64_t myword = ln < nw ? P.cmask[t * nw + ln] : 0ull;
  // the next word's entries load while the current one's Q rows are formed
  auto load_z = [&](int w, double* z) {
    const uint64_t word = w < nw ? __shfl(myword, w) : 0ull;
    const bool mine = (word >> ln) & 1ull;
    const int64_t col = static_cast<int64_t>(w) * 64 + ln;
#pragma unroll
    for (int i = 0; i < kMaxK; ++i)
      z[i] = (mine && i < k) ? ld_y(y, static_cast<int64_t>(S[i]) * ldyr + col) : 0.0;
  };
  double z[kMaxK], zn[kMaxK];
  load_z(0, z);
  for (int w = 0; w < nw; ++w) {
    load_z(w + 1, zn);
    const uint64_t word = __shfl(myword, w);
    const int64_t col = static_cast<int64_t>(w) * 64 + ln;
    if ((word >> ln) & 1ull) {
      RSM_GLOBAL double* q = P.Qd + (t * n + col) * r;
#pragma unroll
      for (int a = 0; a < RSM_MAX_R; ++a) {
        if (a < r) {
          double s = 0.0;
#pragma unroll
          for (int i = 0; i < kMaxK; ++i)
            if (i < k) s = fma(z[i], sB[wv][i * r + a], s);
          q[a] = s;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) z[i] = zn[i];
  }
}

constexpr int kTileWaves = 4;

// Grid (lower 64 x 64 blocks of N, trial ranges, problems); R = r.  Each wavefront walks its
// trials with the next trial's mask words and Q rows loading while the current one is added.
template <bool FIXED, int R>
__global__ __launch_bounds__(64 * kTileWaves) void k_m2_tiles(const ProbDesc* __restrict__ probs,
                                                             IdxList list, int ranges) {
  using Acc = typename std::conditional<FIXED, unsigned long long, double>::type;
  __shared__ Acc acc[64][65];
  __shared__ int li[kTileWaves][64];
  __shared__ int lj[kTileWaves][64];
  const ProbDesc& P = probs[list.idx[blockIdx.z]];
  const int64_t n = P.n, I = P.I;
  const int nb = static_cast<int>(ceil_div(n, 64));
  const int blk = blockIdx.x;
  if (blk >= nb * (nb + 1) / 2) return;  // whole workgroup
  int bi = 0;
  while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
  const int bj = blk - bi * (bi + 1) / 2;
  const int64_t per = ceil_div(I, ranges);
  const int64_t t_begin = static_cast<int64_t>(blockIdx.y) * per;
  const int64_t t_end = t_begin + per < I ? t_begin + per : I;
  if (t_begin >= t_end) return;  // whole workgroup
  const int tid = threadIdx.x, wv = tid / 64, ln = tid % 64;
  for (int e = tid; e < 64 * 65; e += 64 * kTileWaves) (&acc[0][0])[e] = Acc(0);
  __syncthreads();
  const int nw = P.nw;
  const bool diag = bi == bj;
  const uint64_t below = (ln == 0) ? 0ull : (~0ull >> (64 - ln));  // bits under this lane
  RSM_GLOBAL const uint64_t* cm = P.cmask;
  RSM_GLOBAL const double* Qd = P.Qd;
  const int64_t rowi = static_cast<int64_t>(bi) * 64 + ln, rowj = static_cast<int64_t>(bj) * 64 + ln;
  auto words = [&](int64_t t, uint64_t& wi, uint64_t& wj) {
    wi = t < t_end ? cm[t * nw + bi] : 0ull;
    wj = t < t_end ? cm[t * nw + bj] : 0ull;
  };
  auto rows_of = [&](int64_t t, uint64_t wi, uint64_t wj, double* qi, double* qj) {
    const bool hi = (wi >> ln) & 1ull, hj = (wj >> ln) & 1ull;
    RSM_GLOBAL const double* Qt = Qd + t * n * R;
#pragma unroll
    for (int a = 0; a < R; ++a) {
      qi[a] = hi ? Qt[rowi * R + a] : 0.0;
      qj[a] = hj ? Qt[rowj * R + a] : 0.0;
    }
  };
  int64_t t = t_begin + wv;
  uint64_t wi, wj, wi_n, wj_n;
  double qi[R], qj[R], qi_n[R], qj_n[R];
  words(t, wi, wj);
  rows_of(t, wi, wj, qi, qj);
  words(t + kTileWaves, wi_n, wj_n);
  for (; t < t_end; t += kTileWaves) {
    // next trial's rows and the mask words of the one after it, in flight meanwhile
    rows_of(t + kTileWaves, wi_n, wj_n, qi_n, qj_n);
    uint64_t wi_nn, wj_nn;
    words(t + 2 * kTileWaves, wi_nn, wj_nn);
    if (wi != 0 && wj != 0) {
      if ((wi >> ln) & 1ull) li[wv][__popcll(wi & below)] = ln;
      if ((wj >> ln) & 1ull) lj[wv][__popcll(wj & below)] = ln;
      wave_fence();
      const int ni = __popcll(wi), nj = __popcll(wj);
      const int pairs = ni * nj;
      for (int base = 0; base < pairs; base += 64) {
        const int p = base + ln;
        const int ii = p / nj, jj = p - (p / nj) * nj;
        const bool valid = p < pairs && !(diag && jj > ii);
        const int si = p < pairs ? li[wv][ii] : 0;
        const int sj = p < pairs ? lj[wv][jj] : 0;
        double dot = 0.0;
#pragma unroll
        for (int a = 0; a < R; ++a) dot = fma(__shfl(qi[a], si), __shfl(qj[a], sj), dot);
        if (valid) {
          const double v = (diag && si == sj ? 1.0 : 0.0) - dot;
          if constexpr (FIXED)
            atomicAdd(&acc[si][sj], static_cast<unsigned long long>(llrint(v * kFixedScale)));
          else
            atomicAdd(&acc[si][sj], v);
        }
      }
      wave_fence();  // before the next trial overwrites li / lj
    }
    wi = wi_n;
    wj = wj_n;
    wi_n = wi_nn;
    wj_n = wj_nn;
#pragma unroll
    for (int a = 0; a < R; ++a) {
      qi[a] = qi_n[a];
      qj[a] = qj_n[a];
    }
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 64 * kTileWaves) {
    const int i = e / 64, j = e % 64;
    const int64_t row = static_cast<int64_t>(bi) * 64 + i, col = static_cast<int64_t>(bj) * 64 + j;
    if (row >= n || col > row) continue;
    const Acc v = acc[i][j];
    if (v == Acc(0)) continue;
    if constexpr (FIXED)
      atomicAdd((unsigned long long*)&P.N[row + col * n], v);
    else
      atomic_add_f64((double*)&P.N[row + col * n], v);
  }
}

// Members of g whose plan satisfies `pred`, as a new list (plans in `hs`).
template <typename F>
IdxList pick(const IdxList& g, const Plan* const* h, F pred, const Plan** hs) {
  IdxList out;
  for (int k = 0; k < g.count; ++k)
    if (pred(*h[k])) {
      hs[out.count] = h[k];
      out.idx[out.count++] = g.idx[k];
    }
  return out;
}

template <int R>
void tiles_dispatch(bool fixed, int r, dim3 grid, const ProbDesc* d, const IdxList& g, int ranges,
                    hipStream_t s) {
  if (r == R) {
    if (fixed)
      k_m2_tiles<true, R><<<grid, 64 * kTileWaves, 0, s>>>(d, g, ranges);
    else
      k_m2_tiles<false, R><<<grid, 64 * kTileWaves, 0, s>>>(d, g, ranges);
    return;
  }
  if constexpr (R < RSM_MAX_R) tiles_dispatch<R + 1>(fixed, r, grid, d, g, ranges, s);
}

template <int K>
void run_eig(const ProbDesc* d, const IdxList& g, int64_t I, hipStream_t s) {
  if constexpr (K <= 11) {
    k_m2_eig_reg<K><<<dim3(static_cast<unsigned>(ceil_div(I, 64)), g.count), 64, 0, s>>>(d, g);
  } else {
    constexpr int TPB = eig_tpb<K>();
    k_m2_eig<K><<<dim3(static_cast<unsigned>(ceil_div(I, TPB)), g.count), TPB, 0, s>>>(d, g);
  }
}

template <int K>
bool eig_dispatch(int k, const ProbDesc* d, const IdxList& g, int64_t I, hipStream_t s) {
  if (k == K) {
    run_eig<K>(d, g, I, s);
    return true;
  }
  if constexpr (K < kMaxK) return eig_dispatch<K + 1>(k, d, g, I, s);
  return false;
}

}  // namespace

void launch_rows_pack(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  const Plan* hs[kLaunchMax];
  const IdxList rf = pick(g, h, [](const Plan& P) { return P.rows_first; }, hs);
  if (!rf.count) return;
  int64_t mt = 0, ct = 0;
  for (int k = 0; k < rf.count; ++k) {
    mt = std::max<int64_t>(mt, ceil_div(hs[k]->m, 64));
    ct = std::max<int64_t>(ct, ceil_div(hs[k]->n, kRbCols));
  }
  k_pack_rowbits<<<dim3(static_cast<unsigned>(mt), static_cast<unsigned>(ct), rf.count), 256, 0, s>>>(d, rf);
  for (int dt = RSM_F32; dt <= RSM_F64; ++dt) {
    const IdxList yc = pick(g, h, [dt](const Plan& P) {
      return P.rows_first && P.y_layout == RSM_COL_MAJOR && P.y_dtype == dt; }, hs);
    if (!yc.count) continue;
    int64_t rt = 0, ct = 0;
    for (int k = 0; k < yc.count; ++k) {
      rt = std::max<int64_t>(rt, ceil_div(hs[k]->m, 64));
      ct = std::max<int64_t>(ct, ceil_div(hs[k]->n, 64));
    }
    const dim3 grid(static_cast<unsigned>(rt), static_cast<unsigned>(ct), yc.count);
    if (dt == RSM_F32)
      k_transpose_rows<float><<<grid, 256, 0, s>>>(d, yc);
    else
      k_transpose_rows<double><<<grid, 256, 0, s>>>(d, yc);
  }
}

void launch_rows_gram(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  const Plan* hs[kLaunchMax];
  for (int dt = RSM_F32; dt <= RSM_F64; ++dt) {
    const IdxList gd = pick(g, h, [dt](const Plan& P) { return P.y_dtype == dt && P.I > 0; }, hs);
    if (!gd.count) continue;
    int64_t I = 0;
    for (int k = 0; k < gd.count; ++k) I = std::max<int64_t>(I, hs[k]->I);
    const dim3 grid(static_cast<unsigned>(ceil_div(I, kGramWaves)), gd.count);
    if (dt == RSM_F32)
      k_m2_gram<float><<<grid, 64 * kGramWaves, 0, s>>>(d, gd);
    else
      k_m2_gram<double><<<grid, 64 * kGramWaves, 0, s>>>(d, gd);
  }
}

// All members of g share k (= l).
void launch_rows_minor(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  const Plan* hs[kLaunchMax];
  const IdxList ga = pick(g, h, [](const Plan& P) { return P.I > 0; }, hs);
  if (!ga.count) return;
  int64_t I = 0;
  for (int k = 0; k < ga.count; ++k) I = std::max<int64_t>(I, hs[k]->I);
  eig_dispatch<2>(hs[0]->l, d, ga, I, s);
  for (int dt = RSM_F32; dt <= RSM_F64; ++dt) {
    const IdxList gd = pick(g, h, [dt](const Plan& P) { return P.y_dtype == dt && P.I > 0; }, hs);
    if (!gd.count) continue;
    const dim3 grid(static_cast<unsigned>(ceil_div(I, kGramWaves)), gd.count);
    if (dt == RSM_F32)
      k_m2_qform<float><<<grid, 64 * kGramWaves, 0, s>>>(d, gd);
    else
      k_m2_qform<double><<<grid, 64 * kGramWaves, 0, s>>>(d, gd);
  }
  // blocks of N x trial ranges: about four workgroups per CU over the launch
  for (int key = 0; key < 2 * (RSM_MAX_R + 1); ++key) {
    const int fx = key & 1, rr = key >> 1;
    const IdxList gf = pick(g, h, [fx, rr](const Plan& P) {
      return P.I > 0 && P.r == rr && ((P.flags & RSM_DETERMINISTIC) != 0) == (fx == 1); }, hs);
    if (!gf.count) continue;
    int64_t blocks = 0;
    for (int k = 0; k < gf.count; ++k) {
      const int64_t nb = ceil_div(hs[k]->n, 64);
      blocks = std::max<int64_t>(blocks, nb * (nb + 1) / 2);
    }
    int64_t ranges = 1024 / (blocks * gf.count);
    ranges = std::max<int64_t>(1, std::min<int64_t>(ranges, ceil_div(I, 64)));
    const dim3 grid(static_cast<unsigned>(blocks), static_cast<unsigned>(ranges), gf.count);
    tiles_dispatch<1>(fx == 1, rr, grid, d, gf, static_cast<int>(ranges), s);
  }
}

}  // namespace rsm
