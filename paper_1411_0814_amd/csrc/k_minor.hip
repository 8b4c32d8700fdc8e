// Steps a4 + a5: minor vectors of every accepted trial and their accumulation into N.
//
//  k_gram_reduce: G_t = sum over row splits of the partial Grams, in FP64, and |R_t|
//    likewise (one thread per Gram entry; coalesced over trials).
//  k_minor_*: one thread per trial.
//   1. Accept iff the subset is valid and |R_t| >= min_rows (Section IV-A, step 2).
//   2. Cyclic Jacobi (FP64) on G_t: G_t = Q diag(d) Q^T.  The columns of Q for the nvec
//      smallest d are the right singular vectors of Z_t for its smallest singular values
//      (G_t = Z_t^T Z_t), i.e. the zeta_j of Section III.  A rotation is applied when
//      |g_pq| > eps sqrt(|g_pp g_qq|) (the relative-accuracy criterion for symmetric
//      positive semidefinite matrices); the sweeps stop when none is.  With d = g_qq - g_pp
//      and e = 2 g_pq the rotation is t = sign(d) e / (|d| + hypot(d, e)),
//      c = 1 / sqrt(1 + t^2), s = t c (the usual tau formula without its first division).
//   3. N[C_t, C_t] += sum_j zeta_j zeta_j^T — the embedding xi = e(zeta) of eq.(get_xi)
//      contributes only on C_t x C_t.  Lower triangle only (c_a >= c_b), FP64 atomics.
//
//  For l <= 11 the matrix lives in registers (static indices) and the rotations are
//  accumulated in a per-thread LDS slice laid out [entry][thread]; for larger l one
//  wavefront works on each trial.  For l > 11, step 2 is replaced by inverse iteration
//  with Rayleigh-quotient refinement (k_minor_inv) when a trial needs only its one minor
//  vector and no eigenvalue taps are requested (the default); trials where that cannot be
//  shown to have found the smallest eigenvalue go through the wavefront Jacobi after it.
#include <algorithm>
#include <cmath>

#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

constexpr double kJacobiEps = 2.220446049250313e-16;  // 2^-52
constexpr int kJacobiMaxSweeps = 40;
constexpr int kRegMaxL = 11;

// Jacobi rotation for the pair (p, q) from g_pp, g_qq, g_pq (g_pq != 0).
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double& c,
                                                double& s, double& t) {
  const double d = aqq - app;
  const double e = 2.0 * apq;
  const double den = fabs(d) + sqrt(d * d + e * e);
  t = (d >= 0.0 ? e : -e) / den;
  c = rsqrt(1.0 + t * t);
  s = t * c;
}

// N[idx] += v: FP64 atomics, or (deterministic mode) 64-bit integer atomics on the
// fixed-point image of N, whose sum does not depend on the order of the updates.
__device__ __forceinline__ void add_to_N(RSM_GLOBAL double* N, int64_t idx, double v, bool fixed) {
  if (fixed)
    atomicAdd((unsigned long long*)&N[idx],
              static_cast<unsigned long long>(llrint(v * kFixedScale)));
  else
    atomic_add_f64((double*)&N[idx], v);
}

// ------------------------------------------------------------------ split reduction

template <typename TA>
__global__ void k_gram_reduce(const ProbDesc* __restrict__ probs, IdxList list) {
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t I = P.I;
  const int ng = P.l * (P.l + 1) / 2, splits = P.splits;
  auto part = static_cast<RSM_GLOBAL const TA*>(P.part);
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < static_cast<int64_t>(ng) * I) {
    double sum = 0.0;
    for (int s = 0; s < splits; ++s) sum += static_cast<double>(part[static_cast<int64_t>(s) * ng * I + e]);
    P.G[e] = sum;
  }
  if (e < I) {
    int r = 0;
    for (int s = 0; s < splits; ++s) r += P.prow[static_cast<int64_t>(s) * I + e];
    P.rows[e] = r;
  }
}

// Common tail of both kernels: taps, N accumulation, counters.  ev(k) is eigenvalue k,
// vv(i, k) entry i of eigenvector k.
template <int L, typename EV, typename VV>
__device__ __forceinline__ void finish_trial(int64_t t, int nvec, int64_t n, const int* c,
                                             EV ev, VV vv, bool fixed,
                                             RSM_GLOBAL double* __restrict__ N,
                                             RSM_GLOBAL double* __restrict__ tap_vecs,
                                             RSM_GLOBAL double* __restrict__ tap_eigs) {
  int rank[L];
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const double dk = ev(k);
    int rk = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const double dj = ev(j);
      rk += (dj < dk) || (dj == dk && j < k);
    }
    rank[k] = rk;
  }
  if (tap_eigs)
#pragma unroll
    for (int k = 0; k < L; ++k) tap_eigs[t * L + rank[k]] = ev(k);
  if (tap_vecs) {
#pragma unroll
    for (int k = 0; k < L; ++k)
      if (rank[k] < nvec)
#pragma unroll
        for (int i = 0; i < L; ++i) tap_vecs[(t * nvec + rank[k]) * L + i] = vv(i, k);
  }
#pragma unroll
  for (int i = 0; i < L; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double pij = 0.0;
#pragma unroll
      for (int k = 0; k < L; ++k)
        if (rank[k] < nvec) pij += vv(i, k) * vv(j, k);
      add_to_N(N, static_cast<int64_t>(c[i]) + static_cast<int64_t>(c[j]) * n, pij, fixed);
    }
  }
}

// ------------------------------------------------------------------ registers + LDS

template <int L>
__global__ __launch_bounds__(64) void k_minor_reg(const ProbDesc* __restrict__ probs,
                                                  IdxList list) {
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t I = P.I, n = P.n;
  const int nvec = P.nvec, min_rows = P.min_rows;
  RSM_GLOBAL const double* __restrict__ G = P.G;
  RSM_GLOBAL const int32_t* __restrict__ rows_in = P.rows;
  RSM_GLOBAL const int32_t* __restrict__ cols = P.cols;
  RSM_GLOBAL double* __restrict__ N = P.N;
  RSM_GLOBAL rsm_info* info = P.info;
  RSM_GLOBAL int32_t* __restrict__ tap_rows = P.tap_rows;
  RSM_GLOBAL double* __restrict__ tap_gram = P.tap_gram;
  RSM_GLOBAL double* __restrict__ tap_vecs = P.tap_vecs;
  RSM_GLOBAL double* __restrict__ tap_eigs = P.tap_eigs;
  constexpr int TPB = 64;
  constexpr int NG = L * (L + 1) / 2;
  __shared__ double Vs[L * L * TPB];
  __shared__ unsigned long long s_acc;
  __shared__ unsigned long long s_rows;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_acc = 0;
    s_rows = 0;
  }
  const int64_t t = static_cast<int64_t>(blockIdx.x) * TPB + tid;
  const bool active = t < I;
  // packed lower triangle, entry (i, j), j <= i, at i (i + 1) / 2 + j
  double a[NG];
  int c[L];
  int rows = 0;
  bool valid = active;
#pragma unroll
  for (int g = 0; g < NG; ++g) a[g] = active ? G[static_cast<int64_t>(g) * I + t] : 0.0;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    c[k] = active ? cols[t * L + k] : 0;
    valid &= c[k] >= 0;
  }
  if (active) rows = rows_in[t];
  const bool accept = valid && rows >= min_rows;
  auto A = [&](int i, int j) -> double& { return i >= j ? a[i * (i + 1) / 2 + j] : a[j * (j + 1) / 2 + i]; };
  double* V = Vs + tid;
  auto v = [&](int i, int j) -> double& { return V[(i * L + j) * TPB]; };
  if (active) {
    if (tap_rows) tap_rows[t] = rows;
    if (tap_gram)
#pragma unroll
      for (int i = 0; i < L; ++i)
#pragma unroll
        for (int j = 0; j < L; ++j) tap_gram[(t * L + i) * L + j] = A(i, j);
  }
  if (accept) {
#pragma unroll
    for (int i = 0; i < L; ++i)
#pragma unroll
      for (int j = 0; j < L; ++j) v(i, j) = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < kJacobiMaxSweeps; ++sweep) {
      bool rotated = false;
#pragma unroll
      for (int p = 0; p < L - 1; ++p) {
#pragma unroll
        for (int q = p + 1; q < L; ++q) {
          const double apq = A(q, p);
          const double app = A(p, p);
          const double aqq = A(q, q);
          if (fabs(apq) > kJacobiEps * sqrt(fabs(app * aqq))) {
            rotated = true;
            double cr, sr, tr;
            jacobi_rotation(app, aqq, apq, cr, sr, tr);
#pragma unroll
            for (int k = 0; k < L; ++k) {
              if (k == p || k == q) continue;
              const double akp = A(k, p);
              const double akq = A(k, q);
              A(k, p) = cr * akp - sr * akq;
              A(k, q) = sr * akp + cr * akq;
            }
            A(p, p) = app - tr * apq;
            A(q, q) = aqq + tr * apq;
            A(q, p) = 0.0;
#pragma unroll
            for (int k = 0; k < L; ++k) {
              const double vkp = v(k, p);
              const double vkq = v(k, q);
              v(k, p) = cr * vkp - sr * vkq;
              v(k, q) = sr * vkp + cr * vkq;
            }
          }
        }
      }
      if (!rotated) break;
    }
    finish_trial<L>(t, nvec, n, c, [&](int k) { return A(k, k); },
                    [&](int i, int k) { return v(i, k); }, P.fixed_n != 0, N, tap_vecs, tap_eigs);
  } else if (active) {
    if (tap_eigs)
      for (int k = 0; k < L; ++k) tap_eigs[t * L + k] = 0.0;
    if (tap_vecs)
      for (int k = 0; k < nvec * L; ++k) tap_vecs[t * nvec * L + k] = 0.0;
  }
  __syncthreads();
  if (accept) atomicAdd(&s_acc, 1ull);
  if (active) atomicAdd(&s_rows, static_cast<unsigned long long>(rows));
  __syncthreads();
  if (tid == 0) {
    atomicAdd((unsigned long long*)&info->accepted, s_acc);
    atomicAdd((unsigned long long*)&info->rows_total, s_rows);
  }
}

// ------------------------------------------------------------------ one wavefront per trial
//
// For large l (12..17) the l x l matrix and the rotations of one trial are held in LDS by
// a wavefront, which runs parallel-ordering (round-robin) Jacobi: each round rotates
// floor(l/2) disjoint pairs at once (rotation angles computed from the same pre-round
// entries, so the result is the product of commuting plane rotations), elements spread
// over the 64 lanes.  The acceptance criterion per pair is the one of the per-thread
// kernel.  Four trials per workgroup.

constexpr int kWaveTrials = 4;

// REDO: only the trials the inverse-iteration kernel left over (flag set), which it has
// already counted; their minor vectors go into N, nothing else is written.
template <int L, bool REDO>
__global__ __launch_bounds__(64 * kWaveTrials) void k_minor_wave(const ProbDesc* __restrict__ probs,
                                                                 IdxList list) {
  constexpr int NG = L * L;
  constexpr int BB = L + (L & 1);  // even number of players (one idle slot if l is odd)
  constexpr int LS = L + 1;        // LDS row stride
  __shared__ double As[kWaveTrials][L][LS];
  __shared__ double Vs[kWaveTrials][L][LS];
  __shared__ double Cs[kWaveTrials][BB];
  __shared__ double Sn[kWaveTrials][BB];
  __shared__ int Pt[kWaveTrials][BB];
  __shared__ int Pm[kWaveTrials][BB];
  __shared__ int Fl[kWaveTrials];
  __shared__ unsigned long long s_acc, s_rows;
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t I = P.I, n = P.n;
  const int nvec = P.nvec, min_rows = P.min_rows;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) {
    s_acc = 0;
    s_rows = 0;
  }
  auto A = As[w];
  auto V = Vs[w];
  double* cs = Cs[w];
  double* sn = Sn[w];
  int* partner = Pt[w];
  int* perm = Pm[w];
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kWaveTrials + w;
  const bool active = t < I;  // wave-uniform
  int c[L];
  bool valid = active;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    c[k] = active ? P.cols[t * L + k] : 0;
    valid &= c[k] >= 0;
  }
  const int rows = active ? P.rows[t] : 0;
  const bool accept = valid && rows >= min_rows && (!REDO || P.mflag[t] != 0);
  if (active) {
    // packed lower triangle of G_t, entry (i, j), j <= i, at i (i + 1) / 2 + j
    for (int i = 0; i < L; ++i)
      for (int j = lane; j <= i; j += 64) {
        const double v = P.G[static_cast<int64_t>(i * (i + 1) / 2 + j) * I + t];
        A[i][j] = v;
        A[j][i] = v;
      }
    for (int e = lane; e < NG; e += 64) V[e / L][e % L] = (e / L == e % L) ? 1.0 : 0.0;
    if (lane < BB) perm[lane] = lane;
  }
  __syncthreads();
  if (!REDO && active && lane == 0) {
    if (P.tap_rows) P.tap_rows[t] = rows;
    if (P.tap_gram)
      for (int e = 0; e < NG; ++e) P.tap_gram[t * NG + e] = A[e / L][e % L];
  }
  if (accept) {
    for (int sweep = 0; sweep < kJacobiMaxSweeps; ++sweep) {
      if (lane == 0) Fl[w] = 0;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      for (int round = 0; round < BB - 1; ++round) {
        if (lane < BB) partner[lane] = -1;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (lane < BB / 2) {
          int p = perm[lane], q = perm[BB - 1 - lane];
          if (p > q) {
            const int tmp = p;
            p = q;
            q = tmp;
          }
          if (q < L) {
            const double apq = A[q][p], app = A[p][p], aqq = A[q][q];
            double cr = 1.0, sr = 0.0;
            if (fabs(apq) > kJacobiEps * sqrt(fabs(app * aqq))) {
              double tr;
              jacobi_rotation(app, aqq, apq, cr, sr, tr);
              Fl[w] = 1;
            }
            partner[p] = q;
            partner[q] = p;
            cs[p] = cr;
            sn[p] = sr;
            cs[q] = cr;
            sn[q] = -sr;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        // A <- J^T A J, V <- V J for the elements of this lane (reads, then writes)
        constexpr int PER = (NG + 63) / 64;
        double an[PER], vn[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int e = lane + 64 * k;
          if (e < NG) {
            const int i = e / L, j = e % L;
            const int pi = partner[i], pj = partner[j];
            const double ci = pi >= 0 ? cs[i] : 1.0, si = pi >= 0 ? sn[i] : 0.0;
            const double cj = pj >= 0 ? cs[j] : 1.0, sj = pj >= 0 ? sn[j] : 0.0;
            const int ii = pi >= 0 ? pi : i, jj = pj >= 0 ? pj : j;
            an[k] = ci * (cj * A[i][j] - sj * A[i][jj]) - si * (cj * A[ii][j] - sj * A[ii][jj]);
            vn[k] = cj * V[i][j] - sj * V[i][jj];
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int e = lane + 64 * k;
          if (e < NG) {
            A[e / L][e % L] = an[k];
            V[e / L][e % L] = vn[k];
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        // exact symmetry; circle method for the next round (player 0 fixed)
        double sym[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int e = lane + 64 * k;
          sym[k] = (e < NG) ? 0.5 * (A[e / L][e % L] + A[e % L][e / L]) : 0.0;
        }
        int nxt = 0;
        if (lane < BB) nxt = lane == 0 ? perm[0] : (lane == 1 ? perm[BB - 1] : perm[lane - 1]);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int e = lane + 64 * k;
          if (e < NG) A[e / L][e % L] = sym[k];
        }
        if (lane < BB) perm[lane] = nxt;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      }
      if (Fl[w] == 0) break;
    }
    // eigenvalue ranks (ascending), taps, N[C_t, C_t] += sum_{rank < nvec} v v^T
    int rank[L];
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const double dk = A[k][k];
      int rk = 0;
#pragma unroll
      for (int j = 0; j < L; ++j) {
        const double dj = A[j][j];
        rk += (dj < dk) || (dj == dk && j < k);
      }
      rank[k] = rk;
    }
    if (P.tap_eigs && lane < L) {
      int rk = 0;
      for (int j = 0; j < L; ++j) rk += (A[j][j] < A[lane][lane]) || (A[j][j] == A[lane][lane] && j < lane);
      P.tap_eigs[t * L + rk] = A[lane][lane];
    }
    if (P.tap_vecs)
      for (int e = lane; e < NG; e += 64) {
        const int i = e % L, k = e / L;  // entry i of eigenvector (column) k
        if (rank[0] >= 0) {
          int rk = 0;
          for (int j = 0; j < L; ++j) rk += (A[j][j] < A[k][k]) || (A[j][j] == A[k][k] && j < k);
          if (rk < nvec) P.tap_vecs[(t * nvec + rk) * L + i] = V[i][k];
        }
      }
    for (int e = lane; e < L * (L + 1) / 2; e += 64) {
      int i = static_cast<int>((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
      while (i * (i + 1) / 2 > e) --i;
      while ((i + 1) * (i + 2) / 2 <= e) ++i;
      const int j = e - i * (i + 1) / 2;
      double pij = 0.0;
#pragma unroll
      for (int k = 0; k < L; ++k)
        if (rank[k] < nvec) pij += V[i][k] * V[j][k];
      int ci = 0, cj = 0;
#pragma unroll
      for (int k = 0; k < L; ++k) {
        ci = (k == i) ? c[k] : ci;
        cj = (k == j) ? c[k] : cj;
      }
      add_to_N(P.N, static_cast<int64_t>(ci) + static_cast<int64_t>(cj) * n, pij, P.fixed_n != 0);
    }
  } else if (!REDO && active) {
    if (P.tap_eigs)
      for (int k = lane; k < L; k += 64) P.tap_eigs[t * L + k] = 0.0;
    if (P.tap_vecs)
      for (int k = lane; k < nvec * L; k += 64) P.tap_vecs[t * nvec * L + k] = 0.0;
  }
  if constexpr (!REDO) {
    __syncthreads();
    if (lane == 0 && accept) atomicAdd(&s_acc, 1ull);
    if (lane == 0 && active) atomicAdd(&s_rows, static_cast<unsigned long long>(rows));
    __syncthreads();
    if (tid == 0) {
      atomicAdd((unsigned long long*)&P.info->accepted, s_acc);
      atomicAdd((unsigned long long*)&P.info->rows_total, s_rows);
    }
  }
}

// ------------------------------------------------------------------ inverse iteration
//
// One minor vector per trial (nvec = 1, the default l = r + 1), no eigen taps, l > 11: the
// eigenvector of G_t's smallest eigenvalue by inverse iteration refined with Rayleigh
// quotient shifts, one thread per trial, instead of a full Jacobi eigen-decomposition in a
// wavefront (for l <= 11 the register-resident Jacobi is cheaper still).
//  1. G_t = L L^T by Cholesky (FP64, packed in registers).  G_t is positive semidefinite,
//     but its rounding can leave the smallest eigenvalue slightly negative; when a pivot
//     comes out non-positive, G_t + mu I is factorised instead, with mu = 4 u trace(G_t)
//     for the relative accuracy u of the Gram's products and sums (2^-53 FP64, 2^-24 FP32,
//     2^-16 split-BF16), which exceeds that rounding (a pivot still below mu is raised to
//     mu).  kInvIters steps x <- (L L^T)^{-1} x / norm from a fixed irregular start shrink
//     the other eigen-directions by (lambda_1 + mu) / (lambda_k + mu) each.
//  2. up to kRqSteps steps, until the residual ||G_t x - rho x|| is below 32 2^-53 trace(G_t),
//     with the shift rho = x^T G_t x (the Rayleigh quotient, just above
//     lambda_1): G_t - rho I = L D L^T without pivoting (a pivot of magnitude below
//     2^-60 trace(G_t) is set to that magnitude), x <- (L D L^T)^{-1} x / norm.  Near
//     convergence the factor is nearly singular in the minor direction only, which the
//     solve amplifies; the convergence is cubic, so trials whose two smallest eigenvalues
//     are close (noisy data: lambda_1 / lambda_2 up to about 0.6 at the paper-scale
//     workload) still reach the accuracy of a full eigen-decomposition.
constexpr int kInvIters = 4;
constexpr int kRqSteps = 8;   // at most; the steps stop once the residual is at rounding level

// In-place Cholesky of the packed lower triangle a + mu I (entry (i, j), j <= i, at
// i (i + 1) / 2 + j); pivots below `floor_d` are raised to it.  The diagonal receives the
// reciprocals 1 / l_jj (the solves multiply by them).  Returns whether every pivot was
// above the floor.
template <int L>
__device__ __forceinline__ bool cholesky_packed(double (&a)[L * (L + 1) / 2], double mu,
                                                double floor_d) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    double d = a[j * (j + 1) / 2 + j] + mu;
#pragma unroll
    for (int p = 0; p < j; ++p) d -= a[j * (j + 1) / 2 + p] * a[j * (j + 1) / 2 + p];
    ok &= d > floor_d;
    const double ljj = sqrt(d > floor_d ? d : floor_d);
    const double inv = 1.0 / ljj;
    a[j * (j + 1) / 2 + j] = inv;
#pragma unroll
    for (int i = j + 1; i < L; ++i) {
      double sum = a[i * (i + 1) / 2 + j];
#pragma unroll
      for (int p = 0; p < j; ++p) sum -= a[i * (i + 1) / 2 + p] * a[j * (j + 1) / 2 + p];
      a[i * (i + 1) / 2 + j] = sum * inv;
    }
  }
  return ok;
}

// In-place L D L^T of the packed lower triangle a - rho I without pivoting: the diagonal
// receives d_j, the entries below it L's (unit diagonal implied).  |d_j| below `tiny` is
// set to `tiny` with its sign.
template <int L>
__device__ __forceinline__ void ldlt_packed(double (&a)[L * (L + 1) / 2], double rho,
                                            double tiny) {
#pragma unroll
  for (int j = 0; j < L; ++j) {
    double d = a[j * (j + 1) / 2 + j] - rho;
#pragma unroll
    for (int p = 0; p < j; ++p) d -= a[j * (j + 1) / 2 + p] * a[j * (j + 1) / 2 + p] * a[p * (p + 1) / 2 + p];
    if (fabs(d) < tiny) d = d < 0.0 ? -tiny : tiny;
    a[j * (j + 1) / 2 + j] = d;
    const double inv = 1.0 / d;
#pragma unroll
    for (int i = j + 1; i < L; ++i) {
      double sum = a[i * (i + 1) / 2 + j];
#pragma unroll
      for (int p = 0; p < j; ++p) sum -= a[i * (i + 1) / 2 + p] * a[j * (j + 1) / 2 + p] * a[p * (p + 1) / 2 + p];
      a[i * (i + 1) / 2 + j] = sum * inv;
    }
  }
}

template <int L>
__global__ __launch_bounds__(64) void k_minor_inv(const ProbDesc* __restrict__ probs,
                                                  IdxList list) {
  constexpr int NG = L * (L + 1) / 2;
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t I = P.I, n = P.n;
  __shared__ unsigned long long s_acc, s_rows;
  __shared__ double xs[L][64];
  __shared__ int cs[L][64];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_acc = 0;
    s_rows = 0;
  }
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 64 + tid;
  const bool active = t < I;
  double a[NG];  // packed lower triangle, entry (i, j), j <= i, at i (i + 1) / 2 + j
  int c[L];
  int rows = 0;
  bool valid = active;
#pragma unroll
  for (int g = 0; g < NG; ++g) a[g] = active ? P.G[static_cast<int64_t>(g) * I + t] : 0.0;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    c[k] = active ? P.cols[t * L + k] : 0;
    valid &= c[k] >= 0;
  }
  if (active) rows = P.rows[t];
  const bool accept = valid && rows >= P.min_rows;
  if (active) {
    if (P.tap_rows) P.tap_rows[t] = rows;
    if (P.tap_gram)
#pragma unroll
      for (int i = 0; i < L; ++i)
#pragma unroll
        for (int j = 0; j < L; ++j)
          P.tap_gram[(t * L + i) * L + j] = a[i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i];
  }
  if (active && !accept) P.mflag[t] = 0;
  if (accept) {
    bool redo = false;
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < L; ++i) tr += a[i * (i + 1) / 2 + i];
    if (!cholesky_packed<L>(a, 0.0, fmax(0x1p-52 * tr, 1e-300))) {
      const double mu = fmax(4.0 * P.gram_unit * tr, 1e-300);
#pragma unroll
      for (int g = 0; g < NG; ++g) a[g] = P.G[static_cast<int64_t>(g) * I + t];
      cholesky_packed<L>(a, mu, mu);
    }
    double x[L];
#pragma unroll
    for (int i = 0; i < L; ++i) x[i] = 1.0 + 0.5 * static_cast<double>((i * 7 + 3) % 11) / 11.0;
#pragma unroll 1
    for (int it = 0; it < kInvIters; ++it) {
      // L z = x, then L^T y = z (both in x)
#pragma unroll
      for (int i = 0; i < L; ++i) {
        double sum = x[i];
#pragma unroll
        for (int p = 0; p < i; ++p) sum -= a[i * (i + 1) / 2 + p] * x[p];
        x[i] = sum * a[i * (i + 1) / 2 + i];
      }
#pragma unroll
      for (int i = L - 1; i >= 0; --i) {
        double sum = x[i];
#pragma unroll
        for (int p = i + 1; p < L; ++p) sum -= a[p * (p + 1) / 2 + i] * x[p];
        x[i] = sum * a[i * (i + 1) / 2 + i];
      }
      double nrm = 0.0;
#pragma unroll
      for (int i = 0; i < L; ++i) nrm += x[i] * x[i];
      const double s = 1.0 / sqrt(nrm);
#pragma unroll
      for (int i = 0; i < L; ++i) x[i] *= s;
    }
    // the solve itself runs in FP64: its residual floor is a few units of 2^-53 trace(G_t),
    // whatever the precision the Gram was accumulated in
    const double res_tol = 32.0 * 0x1p-53 * tr;
#pragma unroll 1
    for (int q = 0; q < kRqSteps; ++q) {
#pragma unroll
      for (int g = 0; g < NG; ++g) a[g] = P.G[static_cast<int64_t>(g) * I + t];
      // y = G x, rho = x^T y, and stop once the residual G x - rho x is at the Gram's
      // rounding level
      double y[L];
#pragma unroll
      for (int i = 0; i < L; ++i) {
        double sum = 0.0;
#pragma unroll
        for (int j = 0; j < L; ++j) sum += a[i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i] * x[j];
        y[i] = sum;
      }
      double rho = 0.0;
#pragma unroll
      for (int i = 0; i < L; ++i) rho += x[i] * y[i];
      double res2 = 0.0;
#pragma unroll
      for (int i = 0; i < L; ++i) res2 += (y[i] - rho * x[i]) * (y[i] - rho * x[i]);
      if (res2 <= res_tol * res_tol) break;
      ldlt_packed<L>(a, rho, fmax(0x1p-60 * tr, 1e-300));
      // L z = x; z <- z / d; L^T y = z (all in x)
#pragma unroll
      for (int i = 0; i < L; ++i) {
        double sum = x[i];
#pragma unroll
        for (int p = 0; p < i; ++p) sum -= a[i * (i + 1) / 2 + p] * x[p];
        x[i] = sum;
      }
#pragma unroll
      for (int i = 0; i < L; ++i) x[i] /= a[i * (i + 1) / 2 + i];
#pragma unroll
      for (int i = L - 1; i >= 0; --i) {
        double sum = x[i];
#pragma unroll
        for (int p = i + 1; p < L; ++p) sum -= a[p * (p + 1) / 2 + i] * x[p];
        x[i] = sum;
      }
      double nrm = 0.0;
#pragma unroll
      for (int i = 0; i < L; ++i) nrm += x[i] * x[i];
      const double s = 1.0 / sqrt(nrm);
#pragma unroll
      for (int i = 0; i < L; ++i) x[i] *= s;
    }
    // the vector must belong to the smallest eigenvalue: then G - (rho - delta) I, delta =
    // 4 u trace(G) (below that, eigenvalues are not told apart by the Gram), has no
    // negative pivot (Sylvester's law of inertia).  Otherwise the trial goes to the Jacobi
    // pass.
    {
#pragma unroll
      for (int g = 0; g < NG; ++g) a[g] = P.G[static_cast<int64_t>(g) * I + t];
      double rho = 0.0;
#pragma unroll
      for (int i = 0; i < L; ++i) {
        double row = 0.0;
#pragma unroll
        for (int j = 0; j < i; ++j) row += a[i * (i + 1) / 2 + j] * x[j];
        rho += x[i] * (2.0 * row + a[i * (i + 1) / 2 + i] * x[i]);
      }
      ldlt_packed<L>(a, rho - 4.0 * P.gram_unit * tr, fmax(0x1p-60 * tr, 1e-300));
      bool neg = false;
#pragma unroll
      for (int j = 0; j < L; ++j) neg |= a[j * (j + 1) / 2 + j] < 0.0;
      P.mflag[t] = neg ? 1 : 0;
      redo = neg;
    }
    // N[C_t, C_t] += x x^T (lower triangle: c is ascending); x and c go through this
    // thread's LDS slice so that the l(l+1)/2 updates run as a loop
#pragma unroll
    for (int i = 0; i < L; ++i) {
      xs[i][tid] = x[i];
      cs[i][tid] = c[i];
    }
    const bool fixed = P.fixed_n != 0;
#pragma unroll 1
    for (int i = 0; i < (redo ? 0 : L); ++i) {
      const double xi = xs[i][tid];
      const int64_t ci = cs[i][tid];
#pragma unroll 1
      for (int j = 0; j <= i; ++j)
        add_to_N(P.N, ci + static_cast<int64_t>(cs[j][tid]) * n, xi * xs[j][tid], fixed);
    }
  }
  __syncthreads();
  if (accept) atomicAdd(&s_acc, 1ull);
  if (active) atomicAdd(&s_rows, static_cast<unsigned long long>(rows));
  __syncthreads();
  if (tid == 0) {
    atomicAdd((unsigned long long*)&P.info->accepted, s_acc);
    atomicAdd((unsigned long long*)&P.info->rows_total, s_rows);
  }
}

template <int L>
void run_minor(const ProbDesc* d, const IdxList& g, int64_t I, bool inv, hipStream_t s) {
  if constexpr (L <= kRegMaxL) {
    // the register Jacobi is cheap and exact here
    (void)inv;
    const unsigned blocks = static_cast<unsigned>(ceil_div(I, 64));
    k_minor_reg<L><<<dim3(blocks, g.count), 64, 0, s>>>(d, g);
  } else {
    const unsigned blocks = static_cast<unsigned>(ceil_div(I, kWaveTrials));
    if (inv) {
      // inverse iteration for every trial, then Jacobi for the few it leaves over
      k_minor_inv<L><<<dim3(static_cast<unsigned>(ceil_div(I, 64)), g.count), 64, 0, s>>>(d, g);
      k_minor_wave<L, true><<<dim3(blocks, g.count), 64 * kWaveTrials, 0, s>>>(d, g);
      return;
    }
    k_minor_wave<L, false><<<dim3(blocks, g.count), 64 * kWaveTrials, 0, s>>>(d, g);
  }
}

}  // namespace

void launch_minor_kernel(const ProbDesc* d, const IdxList& all, int l, int64_t I, bool inv,
                         hipStream_t s);

void launch_minor(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  // the group shares l; the partial-Gram element type follows the precision
  IdxList sub[2];
  int64_t total[2] = {0, 0};
  for (int k = 0; k < g.count; ++k) {
    if (h[k]->I == 0) continue;
    const int f = h[k]->part_elem == sizeof(double) ? 1 : 0;
    sub[f].idx[sub[f].count++] = g.idx[k];
    total[f] = std::max<int64_t>(total[f], static_cast<int64_t>(h[k]->ng) * h[k]->I);
  }
  if (sub[0].count)
    k_gram_reduce<float><<<dim3(static_cast<unsigned>(ceil_div(total[0], 256)), sub[0].count), 256, 0, s>>>(d, sub[0]);
  if (sub[1].count)
    k_gram_reduce<double><<<dim3(static_cast<unsigned>(ceil_div(total[1], 256)), sub[1].count), 256, 0, s>>>(d, sub[1]);
  // inverse iteration for the problems that allow it, Jacobi for the rest
  IdxList part[2];
  int64_t Ip[2] = {0, 0};
  for (int k = 0; k < g.count; ++k) {
    if (h[k]->I == 0) continue;
    const int v = (h[k]->minor_inv && h[0]->l > kRegMaxL) ? 1 : 0;
    part[v].idx[part[v].count++] = g.idx[k];
    Ip[v] = std::max(Ip[v], h[k]->I);
  }
  for (int v = 0; v < 2; ++v) {
    if (!part[v].count) continue;
    launch_minor_kernel(d, part[v], h[0]->l, Ip[v], v == 1, s);
  }
}

void launch_minor_kernel(const ProbDesc* d, const IdxList& all, int l, int64_t I, bool inv,
                         hipStream_t s) {
  switch (l) {
#define RSM_MINOR_CASE(LL) \
  case LL:                 \
    run_minor<LL>(d, all, I, inv, s); \
    break;
    RSM_MINOR_CASE(2) RSM_MINOR_CASE(3) RSM_MINOR_CASE(4) RSM_MINOR_CASE(5)
    RSM_MINOR_CASE(6) RSM_MINOR_CASE(7) RSM_MINOR_CASE(8) RSM_MINOR_CASE(9)
    RSM_MINOR_CASE(10) RSM_MINOR_CASE(11) RSM_MINOR_CASE(12) RSM_MINOR_CASE(13)
    RSM_MINOR_CASE(14) RSM_MINOR_CASE(15) RSM_MINOR_CASE(16) RSM_MINOR_CASE(17)
#undef RSM_MINOR_CASE
    default:
      break;
  }
}

}  // namespace rsm
