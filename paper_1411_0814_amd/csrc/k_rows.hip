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
//  a4  k_m2_eig: one thread per trial, cyclic Jacobi (FP64) on H_t = U diag(s^2) U^T; the
//      r largest eigenpairs give B_t = [u_a / s_a] (k x r), so that the leading right
//      singular vectors of Z_t are Q_t = Z_t^T B_t.
//  a5  k_m2_update: one workgroup per trial.  N[C_t, C_t] += I - Q_t Q_t^T, lower triangle,
//      formed in 64 x 64 blocks of C_t positions: the rows of Q_t for a block are computed
//      into LDS from the k chosen rows of Y, then 256 threads form 4 x 4 entries each and add
//      them with FP64 atomics (64-bit fixed point in deterministic mode).
#include <algorithm>
#include <cmath>

#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

constexpr int kMaxK = RSM_MAX_L;
constexpr int kMaxW = RSM_MAX_N / 64;     // 64-column words per row
constexpr double kJacobiEpsM2 = 2.220446049250313e-16;  // 2^-52
constexpr int kJacobiSweepsM2 = 40;
// An eigenvalue s_a^2 of H_t at or below this fraction of the largest is taken as zero
// (its direction is dropped from Q_t): below it the direction is set by rounding.
constexpr double kRankTolM2 = 1e-13;

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void add_to_N_m2(RSM_GLOBAL double* N, int64_t idx, double v, bool fixed) {
  if (fixed)
    atomicAdd((unsigned long long*)&N[idx],
              static_cast<unsigned long long>(llrint(v * kFixedScale)));
  else
    atomic_add_f64((double*)&N[idx], v);
}

template <typename T>
__device__ __forceinline__ double ld_y(RSM_GLOBAL const T* y, int64_t idx) {
  return static_cast<double>(y[idx]);
}

// ------------------------------------------------------------------ a0

// Row bit-planes from W in either storage order: a 64 x 64 byte tile through LDS (loads
// coalesced along the storage order), one thread per output word.
// Grid (64-row tiles, 64-column words, problems).
__global__ __launch_bounds__(256) void k_pack_rowbits(const ProbDesc* __restrict__ probs,
                                                      IdxList list) {
  __shared__ uint8_t tile[64][65];
  const ProbDesc& P = probs[list.idx[blockIdx.z]];
  const int64_t m = P.m, n = P.n;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int64_t w = blockIdx.y;
  const int64_t j0 = w * 64;
  if (i0 >= m || j0 >= n) return;
  const bool rowmajor = P.w_layout == RSM_ROW_MAJOR;
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    // row-major: consecutive threads take consecutive columns; column-major: rows
    const int rr = rowmajor ? e / 64 : e % 64;
    const int cc = rowmajor ? e % 64 : e / 64;
    const int64_t i = i0 + rr, j = j0 + cc;
    uint8_t v = 0;
    if (i < m && j < n) v = (rowmajor ? P.W[i * P.ldw + j] : P.W[i + j * P.ldw]) != 0;
    tile[rr][cc] = v;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int64_t i = i0 + threadIdx.x;
    if (i < m) {
      uint64_t word = 0;
      for (int cc = 0; cc < 64; ++cc) word |= static_cast<uint64_t>(tile[threadIdx.x][cc]) << cc;
      P.rbits[i * P.nw + w] = word;
    }
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
  for (int w = 0; w < nw; ++w) {
    const uint64_t word = __shfl(myword, w);
    if (word == 0) continue;
    const bool mine = (word >> ln) & 1ull;
    const int64_t col = static_cast<int64_t>(w) * 64 + ln;
#pragma unroll
    for (int i = 0; i < kMaxK; ++i)
      if (i < k) zs[wv][i][ln] = mine ? ld_y(y, static_cast<int64_t>(S[i]) * ldyr + col) : 0.0;
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
  for (int s = 0; s < 3; ++s)
    if (ln + 64 * s < ng) P.G[static_cast<int64_t>(ln + 64 * s) * P.I + t] = acc[s];
  if (ln == 0) P.rows[t] = valid ? cnt : 0;
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

// ------------------------------------------------------------------ a5

constexpr int kQs = RSM_MAX_R + 1;  // LDS row stride of a Q panel

// Grid (I, problems); one workgroup of 256 threads per trial.
template <typename T>
__global__ __launch_bounds__(256) void k_m2_update(const ProbDesc* __restrict__ probs,
                                                   IdxList list) {
  __shared__ int sS[kMaxK];
  __shared__ double sB[kMaxK][RSM_MAX_R];
  __shared__ int sCl[RSM_MAX_N];
  __shared__ int sOff[kMaxW + 1];
  __shared__ double zp[kMaxK][64];
  __shared__ double qA[64][kQs];
  __shared__ double qB[64][kQs];
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t t = blockIdx.x;
  if (t >= P.I) return;
  const int k = P.l, r = P.r, nw = P.nw;
  const int64_t n = P.n;
  const int tid = threadIdx.x;
  const int cnt = P.rows[t];
  if (P.cols[t * k] < 0 || cnt < P.min_rows) return;  // rejected (uniform per workgroup)
  const bool fixed = P.fixed_n != 0;
  auto y = static_cast<RSM_GLOBAL const T*>(P.yrow);
  const int64_t ldyr = P.ldyr;
  if (tid < k) sS[tid] = P.cols[t * k + tid];
  for (int e = tid; e < k * r; e += 256) sB[e / r][e % r] = P.Bm[t * k * r + e];
  __syncthreads();
  // the qualifying-column list C_t (ascending): word offsets by a scan in wavefront 0
  uint64_t word = 0;
  if (tid < 64) {
    if (tid < nw) {
      word = ~0ull;
      for (int i = 0; i < k; ++i) word &= P.rbits[static_cast<int64_t>(sS[i]) * nw + tid];
    }
    int c = __popcll(word);
    int incl = c;
#pragma unroll
    for (int d = 1; d < 64; d *= 2) {
      const int o = __shfl_up(incl, d);
      if (tid >= d) incl += o;
    }
    if (tid < nw) sOff[tid] = incl - c;
    if (tid < nw) {
      int pos = incl - c;
      uint64_t wbits = word;
      while (wbits) {
        const int b = __ffsll(static_cast<long long>(wbits)) - 1;
        sCl[pos++] = tid * 64 + b;
        wbits &= wbits - 1;
      }
    }
  }
  __syncthreads();
  const int np = (cnt + 63) / 64;
  // rows of Q for the positions [64 panel, 64 panel + 64) of C_t into q
  auto panel = [&](int pnl, double (*q)[kQs]) {
    const int base = pnl * 64;
    const int pc = min(64, cnt - base);
    for (int e = tid; e < k * 64; e += 256) {
      const int i = e / 64, p = e % 64;
      zp[i][p] = p < pc ? ld_y(y, static_cast<int64_t>(sS[i]) * ldyr + sCl[base + p]) : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < 64 * r; e += 256) {
      const int p = e % 64, a = e / 64;
      double s = 0.0;
      for (int i = 0; i < k; ++i) s = fma(zp[i][p], sB[i][a], s);
      q[p][a] = s;
    }
    __syncthreads();
  };
  const int ty = tid / 16, tx = tid % 16;
  for (int pa = 0; pa < np; ++pa) {
    panel(pa, qA);
    for (int pb = 0; pb <= pa; ++pb) {
      double (*qb)[kQs] = qA;
      if (pb != pa) {
        panel(pb, qB);
        qb = qB;
      }
      double acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v2 = 0; v2 < 4; ++v2) acc[u][v2] = 0.0;
      for (int a = 0; a < r; ++a) {
        double xa[4], xb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xa[u] = qA[ty + 16 * u][a];
#pragma unroll
        for (int v2 = 0; v2 < 4; ++v2) xb[v2] = qb[tx + 16 * v2][a];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v2 = 0; v2 < 4; ++v2) acc[u][v2] = fma(xa[u], xb[v2], acc[u][v2]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int ia = pa * 64 + ty + 16 * u;
        if (ia >= cnt) continue;
#pragma unroll
        for (int v2 = 0; v2 < 4; ++v2) {
          const int ib = pb * 64 + tx + 16 * v2;
          if (ib >= cnt || ib > ia) continue;
          const double val = (ia == ib ? 1.0 : 0.0) - acc[u][v2];
          add_to_N_m2(P.N, static_cast<int64_t>(sCl[ia]) + static_cast<int64_t>(sCl[ib]) * n,
                      val, fixed);
        }
      }
      __syncthreads();  // before the next panel overwrites qB / qA
    }
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

template <int K>
void run_eig(const ProbDesc* d, const IdxList& g, int64_t I, hipStream_t s) {
  constexpr int TPB = eig_tpb<K>();
  k_m2_eig<K><<<dim3(static_cast<unsigned>(ceil_div(I, TPB)), g.count), TPB, 0, s>>>(d, g);
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
  int64_t mt = 0, nwm = 0;
  for (int k = 0; k < rf.count; ++k) {
    mt = std::max<int64_t>(mt, ceil_div(hs[k]->m, 64));
    nwm = std::max<int64_t>(nwm, hs[k]->nw);
  }
  k_pack_rowbits<<<dim3(static_cast<unsigned>(mt), static_cast<unsigned>(nwm), rf.count), 256, 0, s>>>(d, rf);
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
    int64_t Id = 0;
    for (int k = 0; k < gd.count; ++k) Id = std::max<int64_t>(Id, hs[k]->I);
    const dim3 grid(static_cast<unsigned>(Id), gd.count);
    if (dt == RSM_F32)
      k_m2_update<float><<<grid, 256, 0, s>>>(d, gd);
    else
      k_m2_update<double><<<grid, 256, 0, s>>>(d, gd);
  }
}

}  // namespace rsm
