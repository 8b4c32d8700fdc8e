// Steps a4 + a5: minor vectors of every accepted trial and their accumulation into N.
//
// One thread per trial:
//  1. G_t = sum over row splits of the partial Grams (FP64), |R_t| likewise.
//  2. Accept iff the subset is valid and |R_t| >= min_rows (Section IV-A, step 2).
//  3. Cyclic Jacobi (FP64) on G_t: G_t = Q diag(d) Q^T.  The columns of Q for the nvec
//     smallest d are the right singular vectors of Z_t for its smallest singular values
//     (G_t = Z_t^T Z_t), i.e. the zeta_j of Section III.  A rotation is applied when
//     |g_pq| > eps sqrt(|g_pp g_qq|) (the relative-accuracy criterion for symmetric
//     positive semidefinite matrices); the sweeps stop when none is.
//  4. N[C_t, C_t] += sum_j zeta_j zeta_j^T — the embedding xi = e(zeta) of eq.(get_xi)
//     contributes only on C_t x C_t.  Lower triangle only (c_a >= c_b), FP64 atomics.
//
// The matrices live in LDS in a per-thread slice laid out [entry][thread] so that a
// wavefront's accesses to one entry hit consecutive addresses.
#include <cmath>

#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

constexpr double kJacobiEps = 2.220446049250313e-16;  // 2^-52
constexpr int kJacobiMaxSweeps = 40;

template <int L>
struct MinorCfg {
  static constexpr int kThreads = (16 * L * L * 64 <= 150 * 1024) ? 64 : 32;
  static constexpr size_t kLds = static_cast<size_t>(16) * L * L * kThreads;
};

// Jacobi on the symmetric L x L matrix A (in place -> eigenvalues on the diagonal),
// accumulating the rotations into V (starts as the identity).  A(i,j) / V(i,j) address the
// thread's LDS slice.
template <int L, int TPB>
__device__ void jacobi_lds(double* A, double* V) {
  auto a = [&](int i, int j) -> double& { return A[(i * L + j) * TPB]; };
  auto v = [&](int i, int j) -> double& { return V[(i * L + j) * TPB]; };
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < L; ++j) v(i, j) = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < kJacobiMaxSweeps; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < L - 1; ++p) {
      for (int q = p + 1; q < L; ++q) {
        const double apq = a(p, q);
        const double app = a(p, p);
        const double aqq = a(q, q);
        if (!(fabs(apq) > kJacobiEps * sqrt(fabs(app * aqq)))) continue;
        rotated = true;
        const double tau = (aqq - app) / (2.0 * apq);
        double t;
        if (fabs(tau) > 1e150) {
          t = 0.5 / tau;
        } else {
          t = 1.0 / (fabs(tau) + sqrt(1.0 + tau * tau));
          if (tau < 0.0) t = -t;
        }
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = t * c;
        for (int k = 0; k < L; ++k) {
          if (k == p || k == q) continue;
          const double akp = a(k, p);
          const double akq = a(k, q);
          const double nkp = c * akp - s * akq;
          const double nkq = s * akp + c * akq;
          a(k, p) = nkp;
          a(p, k) = nkp;
          a(k, q) = nkq;
          a(q, k) = nkq;
        }
        a(p, p) = app - t * apq;
        a(q, q) = aqq + t * apq;
        a(p, q) = 0.0;
        a(q, p) = 0.0;
        for (int k = 0; k < L; ++k) {
          const double vkp = v(k, p);
          const double vkq = v(k, q);
          v(k, p) = c * vkp - s * vkq;
          v(k, q) = s * vkp + c * vkq;
        }
      }
    }
    if (!rotated) break;
  }
}

template <int L, typename TA>
__global__ __launch_bounds__(MinorCfg<L>::kThreads) void k_minor(
    const TA* __restrict__ part, const int32_t* __restrict__ prow,
    const int32_t* __restrict__ cols, int64_t I, int splits, int nvec, int min_rows,
    int64_t n, double* __restrict__ N, rsm_info* info, int32_t* __restrict__ tap_rows,
    double* __restrict__ tap_gram, double* __restrict__ tap_vecs,
    double* __restrict__ tap_eigs) {
  constexpr int TPB = MinorCfg<L>::kThreads;
  constexpr int NG = L * (L + 1) / 2;
  extern __shared__ double smem[];
  __shared__ unsigned long long s_acc;
  __shared__ unsigned long long s_rows;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_acc = 0;
    s_rows = 0;
  }
  double* A = smem + tid;
  double* V = smem + L * L * TPB + tid;
  auto a = [&](int i, int j) -> double& { return A[(i * L + j) * TPB]; };
  auto v = [&](int i, int j) -> double& { return V[(i * L + j) * TPB]; };

  const int64_t t = static_cast<int64_t>(blockIdx.x) * TPB + tid;
  const bool active = t < I;
  int rows = 0;
  bool accept = false;
  int c[L];
  if (active) {
    for (int s = 0; s < splits; ++s) rows += prow[static_cast<int64_t>(s) * I + t];
    int g = 0;
    for (int i = 0; i < L; ++i) {
      for (int j = 0; j <= i; ++j, ++g) {
        double sum = 0.0;
        for (int s = 0; s < splits; ++s)
          sum += static_cast<double>(part[(static_cast<int64_t>(s) * NG + g) * I + t]);
        a(i, j) = sum;
        a(j, i) = sum;
      }
    }
    bool valid = true;
#pragma unroll
    for (int k = 0; k < L; ++k) {
      c[k] = cols[t * L + k];
      valid &= c[k] >= 0;
    }
    accept = valid && rows >= min_rows;
    if (tap_rows) tap_rows[t] = rows;
    if (tap_gram)
      for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) tap_gram[(t * L + i) * L + j] = a(i, j);
  }
  __syncthreads();

  if (accept) {
    jacobi_lds<L, TPB>(A, V);
    // rank of each eigenvalue (ascending, ties broken by index)
    int rank[L];
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const double dk = a(k, k);
      int rk = 0;
      for (int j = 0; j < L; ++j) {
        const double dj = a(j, j);
        rk += (dj < dk) || (dj == dk && j < k);
      }
      rank[k] = rk;
    }
    if (tap_eigs)
#pragma unroll
      for (int k = 0; k < L; ++k) tap_eigs[t * L + rank[k]] = a(k, k);
    if (tap_vecs) {
#pragma unroll
      for (int k = 0; k < L; ++k)
        if (rank[k] < nvec)
          for (int i = 0; i < L; ++i) tap_vecs[(t * nvec + rank[k]) * L + i] = v(i, k);
    }
    // N[c_i, c_j] += sum over the nvec minor vectors of zeta_i zeta_j, for i >= j
    for (int i = 0; i < L; ++i) {
      for (int j = 0; j <= i; ++j) {
        double pij = 0.0;
#pragma unroll
        for (int k = 0; k < L; ++k)
          if (rank[k] < nvec) pij += v(i, k) * v(j, k);
        atomic_add_f64(&N[static_cast<int64_t>(c[i]) + static_cast<int64_t>(c[j]) * n], pij);
      }
    }
  } else if (active) {
    if (tap_eigs)
      for (int k = 0; k < L; ++k) tap_eigs[t * L + k] = 0.0;
    if (tap_vecs)
      for (int k = 0; k < nvec * L; ++k) tap_vecs[t * nvec * L + k] = 0.0;
  }

  // per-block totals in LDS (the block may be narrower than a wavefront), then one
  // global atomic each
  if (accept) atomicAdd(&s_acc, 1ull);
  if (active) atomicAdd(&s_rows, static_cast<unsigned long long>(rows));
  __syncthreads();
  if (tid == 0) {
    atomicAdd(reinterpret_cast<unsigned long long*>(&info->accepted), s_acc);
    atomicAdd(reinterpret_cast<unsigned long long*>(&info->rows_total), s_rows);
  }
}

template <int L, typename TA>
void run_minor(const Plan& P, const void* part, const int32_t* prow, const int32_t* cols,
               double* N, rsm_info* info, const rsm_output& out, hipStream_t s) {
  constexpr int TPB = MinorCfg<L>::kThreads;
  const unsigned blocks = static_cast<unsigned>(ceil_div(P.I, TPB));
  static bool attr_set = false;  // dynamic LDS above 64 KiB must be allowed explicitly
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_minor<L, TA>),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(MinorCfg<L>::kLds));
    attr_set = true;
  }
  k_minor<L, TA><<<blocks, TPB, MinorCfg<L>::kLds, s>>>(
      static_cast<const TA*>(part), prow, cols, P.I, P.splits, P.nvec, P.min_rows, P.n, N,
      info, out.trial_rows, out.trial_gram, out.trial_vecs, out.trial_eigs);
}

template <int L>
void dispatch_minor(const Plan& P, const void* part, const int32_t* prow, const int32_t* cols,
                    double* N, rsm_info* info, const rsm_output& out, hipStream_t s) {
  if (P.part_elem == sizeof(double))
    run_minor<L, double>(P, part, prow, cols, N, info, out, s);
  else
    run_minor<L, float>(P, part, prow, cols, N, info, out, s);
}

}  // namespace

void launch_minor(const Plan& P, const void* part, const int32_t* prow, const int32_t* cols,
                  double* N, rsm_info* info, const rsm_output& out, hipStream_t s) {
  if (P.I == 0) return;
  switch (P.l) {
#define RSM_MINOR_CASE(LL) \
  case LL:                 \
    dispatch_minor<LL>(P, part, prow, cols, N, info, out, s); \
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
