// Step a7: U-hat by eq.(solve.barU) with the L2 norm, row by row:
//   u_i = argmin_u sum_j w_ij (y_ij - u^T v_j)^2  =>  A_i u_i = b_i,
//   A_i = sum_{j known} v_j v_j^T (r x r),  b_i = sum_{j known} y_ij v_j.
// One thread per row; a wavefront covers 64 consecutive rows, i.e. one word of each
// column's mask bit-plane, read once per wavefront.  V-hat is staged through LDS in
// chunks of columns and read as a broadcast.  A_i is factorised by Cholesky in registers
// (FP64).  Rows with fewer than r known entries (or a singular A_i) get u_i = 0 and are
// counted as underdetermined.
//
// Also: the optional error of eq.(ep), e = (sum w)^-1/2 ||W o (Y - U V^T)||_F.
#include <algorithm>
#include <cmath>

#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

constexpr int kUChunk = 256;  // columns of V-hat per LDS stage

// Columns whose loads are issued together: fewer for large r, whose r(r+1)/2 accumulators
// already fill most of the register file.
template <int R>
constexpr int u_unroll() {
  return R <= 8 ? 4 : (R <= 12 ? 2 : 1);
}

template <int R, typename TY>
__global__ __launch_bounds__(256) void k_usolve(const ProbDesc* __restrict__ probs, IdxList list) {
  constexpr int NA = R * (R + 1) / 2;
  __shared__ double Vs[kUChunk * R];
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t m = P.m, n = P.n, mw = P.mw, ldy = P.ldy;
  if (static_cast<int64_t>(blockIdx.x) * 256 >= m) return;
  auto Y = static_cast<RSM_GLOBAL const TY*>(P.ycm);
  RSM_GLOBAL const uint64_t* __restrict__ wbits = P.wbits;
  RSM_GLOBAL const double* __restrict__ V = P.V;
  RSM_GLOBAL double* __restrict__ U = P.U;
  RSM_GLOBAL rsm_info* info = P.info;
  const int tid = threadIdx.x;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + tid;
  const bool active = i < m;
  const int64_t w = uniform_i64((static_cast<int64_t>(blockIdx.x) * 256 + (tid & ~63)) >> 6);
  const int bit = tid & 63;
  double A[NA];
  double bv[R];
#pragma unroll
  for (int g = 0; g < NA; ++g) A[g] = 0.0;
#pragma unroll
  for (int a = 0; a < R; ++a) bv[a] = 0.0;
  int cnt = 0;
  const bool wave_active = w < mw;
  // rows past m (last wavefront only) read row m - 1: valid address, zero weight
  const int64_t iy = active ? i : (m - 1);
  for (int64_t j0 = 0; j0 < n; j0 += kUChunk) {
    const int jn = static_cast<int>((n - j0) < kUChunk ? (n - j0) : kUChunk);
    __syncthreads();
    for (int e = tid; e < jn * R; e += 256) {
      const int jj = e / R, a = e % R;
      Vs[e] = V[(j0 + jj) + static_cast<int64_t>(a) * n];
    }
    __syncthreads();
    if (wave_active) {
      // groups of kUnroll columns: all loads of a group first, then the products; the
      // mask bit is a 0/1 weight, so there is no divergent branch
      constexpr int kUnroll = u_unroll<R>();
      for (int jj = 0; jj < jn; jj += kUnroll) {
        uint64_t word[kUnroll];
        double y[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int64_t j = j0 + jj + u;
          if (jj + u < jn) {
            word[u] = wbits[j * mw + w];
            y[u] = static_cast<double>(Y[j * ldy + iy]);
          } else {
            word[u] = 0;
            y[u] = 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const bool known = ((word[u] >> bit) & 1ull) && active;
          const double yw = known ? y[u] : 0.0;
          double v[R], wv[R];
#pragma unroll
          for (int a = 0; a < R; ++a) {
            v[a] = Vs[(jj + u) * R + a];
            wv[a] = known ? v[a] : 0.0;
          }
          int g = 0;
#pragma unroll
          for (int a = 0; a < R; ++a) {
            bv[a] += yw * v[a];
#pragma unroll
            for (int b = 0; b <= a; ++b) A[g++] += wv[a] * v[b];
          }
          cnt += known ? 1 : 0;
        }
      }
    }
  }
  // Cholesky A = L L^T in place (lower, packed row-major), then L L^T u = b
  bool ok = active && cnt >= R;
  if (ok) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      double d = A[j * (j + 1) / 2 + j];
#pragma unroll
      for (int p = 0; p < j; ++p) d -= A[j * (j + 1) / 2 + p] * A[j * (j + 1) / 2 + p];
      ok &= (d > 0.0);
      const double ljj = sqrt(d > 0.0 ? d : 1.0);
      A[j * (j + 1) / 2 + j] = ljj;
#pragma unroll
      for (int ii = j + 1; ii < R; ++ii) {
        double s = A[ii * (ii + 1) / 2 + j];
#pragma unroll
        for (int p = 0; p < j; ++p) s -= A[ii * (ii + 1) / 2 + p] * A[j * (j + 1) / 2 + p];
        A[ii * (ii + 1) / 2 + j] = s / ljj;
      }
    }
  }
  double u[R];
#pragma unroll
  for (int a = 0; a < R; ++a) u[a] = 0.0;
  if (ok) {
    // forward: L z = b
#pragma unroll
    for (int a = 0; a < R; ++a) {
      double s = bv[a];
#pragma unroll
      for (int p = 0; p < a; ++p) s -= A[a * (a + 1) / 2 + p] * u[p];
      u[a] = s / A[a * (a + 1) / 2 + a];
    }
    // backward: L^T u = z
#pragma unroll
    for (int a = R - 1; a >= 0; --a) {
      double s = u[a];
#pragma unroll
      for (int p = a + 1; p < R; ++p) s -= A[p * (p + 1) / 2 + a] * u[p];
      u[a] = s / A[a * (a + 1) / 2 + a];
    }
  }
  if (active) {
#pragma unroll
    for (int a = 0; a < R; ++a) U[i + static_cast<int64_t>(a) * m] = ok ? u[a] : 0.0;
  }
  const unsigned long long under = wave_sum<unsigned long long>((active && !ok) ? 1ull : 0ull);
  const unsigned long long known = wave_sum<unsigned long long>(active ? static_cast<unsigned long long>(cnt) : 0ull);
  if ((tid & 63) == 0) {
    if (under) {
      atomicAdd((unsigned long long*)&info->rows_underdetermined, under);
      atomicOr((uint32_t*)&info->warn, static_cast<uint32_t>(RSM_W_ROWS_UNDERDETERMINED));
    }
    if (known) atomicAdd((unsigned long long*)&info->known, known);
  }
}

template <int R, typename TY>
__global__ __launch_bounds__(256) void k_error(const ProbDesc* __restrict__ probs, IdxList list) {
  __shared__ double Vs[kUChunk * R];
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t m = P.m, n = P.n, mw = P.mw, ldy = P.ldy;
  if (static_cast<int64_t>(blockIdx.x) * 256 >= m) return;
  auto Y = static_cast<RSM_GLOBAL const TY*>(P.ycm);
  RSM_GLOBAL const uint64_t* __restrict__ wbits = P.wbits;
  RSM_GLOBAL const double* __restrict__ V = P.V;
  RSM_GLOBAL const double* __restrict__ U = P.U;
  const int tid = threadIdx.x;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + tid;
  const bool active = i < m;
  const int64_t w = uniform_i64((static_cast<int64_t>(blockIdx.x) * 256 + (tid & ~63)) >> 6);
  const int bit = tid & 63;
  double u[R];
#pragma unroll
  for (int a = 0; a < R; ++a) u[a] = active ? U[i + static_cast<int64_t>(a) * m] : 0.0;
  double acc = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += kUChunk) {
    const int jn = static_cast<int>((n - j0) < kUChunk ? (n - j0) : kUChunk);
    __syncthreads();
    for (int e = tid; e < jn * R; e += 256) {
      const int jj = e / R, a = e % R;
      Vs[e] = V[(j0 + jj) + static_cast<int64_t>(a) * n];
    }
    __syncthreads();
    if (w < mw) {
      for (int jj = 0; jj < jn; ++jj) {
        const int64_t j = j0 + jj;
        const uint64_t word = wbits[j * mw + w];
        if ((word >> bit) & 1ull) {
          double res = static_cast<double>(Y[j * ldy + i]);
#pragma unroll
          for (int a = 0; a < R; ++a) res -= u[a] * Vs[jj * R + a];
          acc += res * res;
        }
      }
    }
  }
  acc = wave_sum(acc);
  if ((tid & 63) == 0) atomic_add_f64((double*)&P.scal->err_acc, acc);
}

__global__ void k_error_finalize(const ProbDesc* __restrict__ probs, IdxList list) {
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  if (threadIdx.x == 0) {
    const double k = static_cast<double>(P.info->known);
    P.info->e = k > 0.0 ? sqrt(P.scal->err_acc / k) : 0.0;
  }
}

template <int R>
void run_usolve(const ProbDesc* d, const IdxList& g, int64_t m, int y_dtype, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(ceil_div(m, 256)), g.count);
  if (y_dtype == RSM_F32)
    k_usolve<R, float><<<grid, 256, 0, s>>>(d, g);
  else
    k_usolve<R, double><<<grid, 256, 0, s>>>(d, g);
}

template <int R>
void run_error(const ProbDesc* d, const IdxList& g, int64_t m, int y_dtype, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(ceil_div(m, 256)), g.count);
  if (y_dtype == RSM_F32)
    k_error<R, float><<<grid, 256, 0, s>>>(d, g);
  else
    k_error<R, double><<<grid, 256, 0, s>>>(d, g);
  k_error_finalize<<<dim3(1, g.count), 64, 0, s>>>(d, g);
}

}  // namespace

#define RSM_R_CASES(X)                                                                 \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

// The group shares r and the element type of Y.
void launch_solve_u(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  if (!g.count) return;
  int64_t m = 0;
  for (int k = 0; k < g.count; ++k) m = std::max(m, h[k]->m);
  switch (h[0]->r) {
#define RSM_U_CASE(RR) \
  case RR:             \
    run_usolve<RR>(d, g, m, h[0]->y_dtype, s); \
    break;
    RSM_R_CASES(RSM_U_CASE)
#undef RSM_U_CASE
    default:
      break;
  }
}

void launch_error(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  if (!g.count) return;
  int64_t m = 0;
  for (int k = 0; k < g.count; ++k) m = std::max(m, h[k]->m);
  switch (h[0]->r) {
#define RSM_E_CASE(RR) \
  case RR:             \
    run_error<RR>(d, g, m, h[0]->y_dtype, s); \
    break;
    RSM_R_CASES(RSM_E_CASE)
#undef RSM_E_CASE
    default:
      break;
  }
}

}  // namespace rsm
