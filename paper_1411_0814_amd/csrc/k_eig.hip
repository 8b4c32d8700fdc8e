// Step a6: V-hat = the r eigenvectors of N = Xi Xi^T with the smallest eigenvalues
// (eq.(solve.barV_L2_norm); "||V|| = 1" read as V^T V = I_r).  FP64 throughout.
//
// N is symmetric positive semidefinite with (near-)null space of dimension r, so its
// smallest eigenvalues are the dominant ones of (N + mu I)^{-1}:
//   1. N (lower triangle) -> full symmetric copy; Gershgorin bound lam_max; uncovered
//      columns (N_jj == 0).
//   2. mu = 8 n eps lam_max (above the backward error of the factorisation) and the
//      blocked right-looking Cholesky N + mu I = L L^T (64 x 64 tiles).
//   3. Block inverse iteration on b = r + 4 vectors: X <- orth(L^{-T} L^{-1} X), with
//      backward-stable triangular solves and classical Gram-Schmidt applied twice.
//   4. Rayleigh-Ritz: H = X^T N X, H = Q Theta Q^T (Jacobi), V-hat = X Q[:, :r],
//      lambda_1..lambda_{r+1} = Theta, residual max_k ||N v_k - theta_k v_k|| / lam_max.
#include <cmath>

#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

constexpr int NB = kCholNB;
constexpr double kEps = 1.1102230246251565e-16;  // 2^-53

__device__ __forceinline__ void atomic_max_pos_f64(double* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long*>(addr), static_cast<unsigned long long>(__double_as_longlong(v)));
}

// Nsym = N with the upper triangle mirrored from the lower one.
__global__ void k_symmetrize(const double* __restrict__ N, int64_t n, double* __restrict__ Ns) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t j = idx / n, i = idx - j * n;
  Ns[idx] = (i >= j) ? N[i + j * n] : N[j + i * n];
}

// Thread per row: Gershgorin bound max_i sum_j |N_ij| and the count of zero diagonals.
__global__ void k_norm_stats(const double* __restrict__ Ns, int64_t n, DevScalars* scal,
                             rsm_info* info) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double s = 0.0;
  int zero = 0;
  if (i < n) {
    for (int64_t j = 0; j < n; ++j) s += fabs(Ns[i + j * n]);
    zero = (Ns[i + i * n] == 0.0);
  }
  const double smax = [&] {
    double v = s;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
  }();
  const int zsum = wave_sum(zero);
  if ((threadIdx.x & 63) == 0) {
    atomic_max_pos_f64(&scal->lam_max, smax);
    if (zsum) atomicAdd(&info->uncovered, zsum);
  }
}

// L <- lower(Nsym) + mu I.
__global__ void k_chol_init(const double* __restrict__ Ns, int64_t n, double* __restrict__ Lf,
                            DevScalars* scal, rsm_info* info) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const double lam = scal->lam_max;
  // N == 0 (no accepted trial): factor I instead; V-hat is then an arbitrary orthonormal basis
  const double mu = lam > 0.0 ? fmax(8.0 * static_cast<double>(n) * kEps * lam, 1e-290) : 1.0;
  if (idx == 0) {
    scal->mu = mu;
    info->mu = mu;
  }
  if (idx >= n * n) return;
  const int64_t j = idx / n, i = idx - j * n;
  Lf[idx] = (i > j) ? Ns[idx] : (i == j ? Ns[idx] + mu : 0.0);
}

// Unblocked Cholesky of the kb x kb lower block held in LDS (ld NB+1), 256 threads.
__device__ void potrf_lds(double (*A)[NB + 1], int kb, double mu, int* npiv) {
  const int tid = threadIdx.x;
  for (int j = 0; j < kb; ++j) {
    if (tid == 0) {
      double d = A[j][j];
      if (!(d > 0.0) || !isfinite(d)) {
        d = mu;
        ++*npiv;
      }
      A[j][j] = sqrt(d);
    }
    __syncthreads();
    const double ljj = A[j][j];
    for (int i = j + 1 + tid; i < kb; i += blockDim.x) A[i][j] /= ljj;
    __syncthreads();
    const int rem = kb - j - 1;
    for (int e = tid; e < rem * rem; e += blockDim.x) {
      const int ii = j + 1 + e / rem, kk = j + 1 + e % rem;
      if (kk <= ii) A[ii][kk] -= A[ii][j] * A[kk][j];
    }
    __syncthreads();
  }
}

// Panel step k, part 1: factor tile (k, k) in place (one workgroup).
__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ Lf, int64_t n, int k,
                                                   DevScalars* scal) {
  __shared__ double D[NB][NB + 1];
  __shared__ int npiv;
  const int tid = threadIdx.x;
  const int64_t k0 = static_cast<int64_t>(k) * NB;
  const int kb = static_cast<int>((n - k0) < NB ? (n - k0) : NB);
  if (tid == 0) npiv = 0;
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int ii = e % NB, jj = e / NB;
    D[ii][jj] = (ii < kb && jj < kb && jj <= ii) ? Lf[(k0 + ii) + (k0 + jj) * n] : 0.0;
  }
  __syncthreads();
  potrf_lds(D, kb, scal->mu, &npiv);
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int ii = e % NB, jj = e / NB;
    if (ii < kb && jj < kb && jj <= ii) Lf[(k0 + ii) + (k0 + jj) * n] = D[ii][jj];
  }
  if (tid == 0 && npiv) atomicAdd(&scal->pivots, npiv);
}

// Panel step k, part 2: workgroup i solves tile (k+1+i, k): L_ik = A_ik L_kk^{-T}.
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ Lf, int64_t n, int k) {
  __shared__ double D[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  const int tid = threadIdx.x;
  const int64_t k0 = static_cast<int64_t>(k) * NB;
  const int kb = static_cast<int>((n - k0) < NB ? (n - k0) : NB);
  const int64_t i0 = k0 + static_cast<int64_t>(blockIdx.x + 1) * NB;
  if (i0 >= n) return;
  const int ib = static_cast<int>((n - i0) < NB ? (n - i0) : NB);
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int ii = e % NB, jj = e / NB;
    D[ii][jj] = (ii < kb && jj < kb && jj <= ii) ? Lf[(k0 + ii) + (k0 + jj) * n] : 0.0;
    X[ii][jj] = (ii < ib && jj < kb) ? Lf[(i0 + ii) + (k0 + jj) * n] : 0.0;
  }
  __syncthreads();
  // X L^T = A  ->  column j: x_j = (a_j - sum_{p<j} x_p L_jp) / L_jj, column-oriented
  for (int j = 0; j < kb; ++j) {
    const double ljj = D[j][j];
    for (int ii = tid; ii < ib; ii += blockDim.x) X[ii][j] /= ljj;
    __syncthreads();
    const int rem = kb - j - 1;
    for (int e = tid; e < ib * rem; e += blockDim.x) {
      const int ii = e % ib, jj = j + 1 + e / ib;
      X[ii][jj] -= X[ii][j] * D[jj][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int ii = e % NB, jj = e / NB;
    if (ii < ib && jj < kb) Lf[(i0 + ii) + (k0 + jj) * n] = X[ii][jj];
  }
}

// Trailing update after panel k: tile (i, j), k < j <= i:  A_ij -= L_ik L_jk^T.
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ Lf, int64_t n, int k,
                                                     int nb) {
  __shared__ double Li[NB][NB + 1];
  __shared__ double Lj[NB][NB + 1];
  // tile index -> (i, j)
  int b = blockIdx.x;
  int ti = k + 1, tj = k + 1;
  for (int i = k + 1; i < nb; ++i) {
    const int cnt = i - k;
    if (b < cnt) {
      ti = i;
      tj = k + 1 + b;
      break;
    }
    b -= cnt;
  }
  const int64_t k0 = static_cast<int64_t>(k) * NB;
  const int64_t i0 = static_cast<int64_t>(ti) * NB, j0 = static_cast<int64_t>(tj) * NB;
  const int ib = static_cast<int>((n - i0) < NB ? (n - i0) : NB);
  const int jb = static_cast<int>((n - j0) < NB ? (n - j0) : NB);
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int rr = e % NB, pp = e / NB;
    Li[rr][pp] = (rr < ib) ? Lf[(i0 + rr) + (k0 + pp) * n] : 0.0;
    Lj[rr][pp] = (rr < jb) ? Lf[(j0 + rr) + (k0 + pp) * n] : 0.0;
  }
  __syncthreads();
  const int tx = tid % 16, ty = tid / 16;
  double acc[4][4] = {};
  for (int p = 0; p < NB; ++p) {
    double a[4], bb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = Li[ty * 4 + u][p];
      bb[u] = Lj[tx * 4 + u][p];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * bb[v];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = ty * 4 + u, cc = tx * 4 + v;
      if (rr < ib && cc < jb && (ti != tj || cc <= rr)) Lf[(i0 + rr) + (j0 + cc) * n] -= acc[u][v];
    }
  }
}

// Deterministic start block: entries uniform in [-1, 1) from Philox (key = seed, 1).
__global__ void k_start_vectors(double* __restrict__ X, int64_t n, int b, uint64_t seed) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * b) return;
  uint64_t c[4] = {static_cast<uint64_t>(idx), 0x5eedull, 0ull, 0ull};
  Philox4x64::block(c, seed, 1ull);
  X[idx] = static_cast<double>(static_cast<int64_t>(c[0]) >> 11) * (1.0 / 4503599627370496.0);
}

// Transposed copy of the factor: Lt[i + j n] = L[j + i n] (upper triangle = L^T), so that
// the backward solve reads rows of L^T contiguously.
__global__ void k_transpose_lower(const double* __restrict__ Lf, int64_t n,
                                  double* __restrict__ Lt) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t j = idx / n, i = idx - j * n;
  Lt[idx] = (i <= j) ? Lf[j + i * n] : 0.0;
}

// Inverse of every 64 x 64 diagonal tile of L (one workgroup per tile, one thread per
// column of the inverse: L_kk x = e_c by forward substitution).  Dinv[k][i + 64 j].
__global__ __launch_bounds__(64) void k_diag_inverse(const double* __restrict__ Lf, int64_t n,
                                                     double* __restrict__ Dinv) {
  __shared__ double D[NB][NB + 1];
  __shared__ double Xs[NB][NB + 1];
  const int kb = blockIdx.x;
  const int64_t k0 = static_cast<int64_t>(kb) * NB;
  const int kk = static_cast<int>((n - k0) < NB ? (n - k0) : NB);
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int ii = e % NB, jj = e / NB;
    D[ii][jj] = (ii < kk && jj < kk && jj <= ii) ? Lf[(k0 + ii) + (k0 + jj) * n] : (ii == jj ? 1.0 : 0.0);
  }
  __syncthreads();
  const int c = tid;
  for (int i = 0; i < NB; ++i) {
    double v = (i == c) ? 1.0 : 0.0;
    for (int p = c; p < i; ++p) v -= D[i][p] * Xs[p][c];
    Xs[i][c] = (i < c) ? 0.0 : v / D[i][i];
  }
  __syncthreads();
  double* out = Dinv + static_cast<int64_t>(kb) * NB * NB;
  for (int e = tid; e < NB * NB; e += blockDim.x) out[e] = Xs[e % NB][e / NB];
}

// Single-workgroup blocked triangular solve with b right-hand sides (n x b, ld n):
//   upper = 0:  L Z = X with T = L (lower);   upper = 1:  L^T Z = X with T = L^T (upper).
// Per 64-row tile: acc = X_k - sum over solved tiles T_kj Z_j (four wavefronts split the
// inner index), then z = D^{-1} acc followed by one step of iterative refinement
// z += D^{-1} (acc - D z) with the stored tile inverse.  Z may alias X.
__global__ __launch_bounds__(256) void k_trsm(const double* __restrict__ T, int64_t n, int b,
                                              const double* __restrict__ Dinv, const double* X,
                                              double* Z, int upper) {
  __shared__ double acc[NB][kEigMaxB];
  __shared__ double zs[NB][kEigMaxB];
  __shared__ double Dm[NB][NB + 1];
  __shared__ double Di[NB][NB + 1];
  __shared__ double red[3][NB][kEigMaxB];
  const int tid = threadIdx.x;
  const int rr = tid % NB;
  const int g = tid / NB;  // 0..3
  const int nb = static_cast<int>(ceil_div(n, NB));
  for (int s = 0; s < nb; ++s) {
    const int kb = upper ? (nb - 1 - s) : s;
    const int64_t k0 = static_cast<int64_t>(kb) * NB;
    const int kk = static_cast<int>((n - k0) < NB ? (n - k0) : NB);
    const double* dinv = Dinv + static_cast<int64_t>(kb) * NB * NB;
    for (int e = tid; e < NB * NB; e += blockDim.x) {
      const int ii = e % NB, jj = e / NB;
      const bool in = ii < kk && jj < kk;
      Dm[ii][jj] = in ? T[(k0 + ii) + (k0 + jj) * n] : 0.0;
      // inverse of L_kk^T is (L_kk^{-1})^T
      Di[ii][jj] = in ? (upper ? dinv[jj + NB * ii] : dinv[ii + NB * jj]) : 0.0;
    }
    // off-diagonal contribution: rows k0..k0+kk of T times the solved part of Z
    double part[kEigMaxB];
#pragma unroll
    for (int c = 0; c < kEigMaxB; ++c) part[c] = 0.0;
    const int64_t p_begin = upper ? (k0 + kk) : 0;
    const int64_t p_end = upper ? n : k0;
    if (rr < kk) {
      for (int64_t p = p_begin + g; p < p_end; p += 4) {
        const double tv = T[(k0 + rr) + p * n];
#pragma unroll
        for (int c = 0; c < kEigMaxB; ++c)
          if (c < b) part[c] += tv * Z[p + c * n];
      }
    }
    if (g > 0) {
#pragma unroll
      for (int c = 0; c < kEigMaxB; ++c) red[g - 1][rr][c] = part[c];
    }
    __syncthreads();
    if (g == 0) {
#pragma unroll
      for (int c = 0; c < kEigMaxB; ++c) {
        if (c < b) {
          const double x = (rr < kk) ? X[(k0 + rr) + c * n] : 0.0;
          acc[rr][c] = x - (part[c] + red[0][rr][c] + red[1][rr][c] + red[2][rr][c]);
        }
      }
    }
    __syncthreads();
    // z = Dinv acc, then one refinement step
    for (int e = tid; e < NB * b; e += blockDim.x) {
      const int i = e % NB, c = e / NB;
      double v = 0.0;
      for (int p = 0; p < NB; ++p) v += Di[i][p] * acc[p][c];
      zs[i][c] = v;
    }
    __syncthreads();
    for (int e = tid; e < NB * b; e += blockDim.x) {
      const int i = e % NB, c = e / NB;
      double v = acc[i][c];
      for (int p = 0; p < NB; ++p) v -= Dm[i][p] * zs[p][c];
      red[0][i][c] = v;  // residual
    }
    __syncthreads();
    for (int e = tid; e < NB * b; e += blockDim.x) {
      const int i = e % NB, c = e / NB;
      double v = 0.0;
      for (int p = 0; p < NB; ++p) v += Di[i][p] * red[0][p][c];
      if (i < kk) Z[(k0 + i) + c * n] = zs[i][c] + v;
    }
    __threadfence();
    __syncthreads();
  }
}

// Block reduction of `cnt` per-thread values into red[0..cnt) (1024 threads).
__device__ void block_sum(double* vals, int cnt, double* red /* [16][kEigMaxB] */,
                          double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j = 0; j < cnt; ++j) {
    const double s = wave_sum(vals[j]);
    if (lane == 0) red[wid * kEigMaxB + j] = s;
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    double s = 0.0;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) s += red[w * kEigMaxB + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// X = orth(Z): classical Gram-Schmidt applied twice per column (one workgroup).
__global__ __launch_bounds__(1024) void k_orth(const double* __restrict__ Z, int64_t n, int b,
                                               double* __restrict__ X) {
  __shared__ double red[16 * kEigMaxB];
  __shared__ double h[kEigMaxB];
  const int tid = threadIdx.x;
  for (int64_t i = tid; i < n; i += blockDim.x)
    for (int c = 0; c < b; ++c) X[i + c * n] = Z[i + c * n];
  __threadfence();
  __syncthreads();
  for (int k = 0; k < b; ++k) {
    for (int pass = 0; pass < 2; ++pass) {
      double part[kEigMaxB];
      for (int j = 0; j < k; ++j) part[j] = 0.0;
      for (int64_t i = tid; i < n; i += blockDim.x) {
        const double xk = X[i + k * n];
        for (int j = 0; j < k; ++j) part[j] += X[i + j * n] * xk;
      }
      block_sum(part, k, red, h);
      for (int64_t i = tid; i < n; i += blockDim.x) {
        double v = X[i + k * n];
        for (int j = 0; j < k; ++j) v -= h[j] * X[i + j * n];
        X[i + k * n] = v;
      }
      __threadfence();
      __syncthreads();
    }
    double part1[1] = {0.0};
    for (int64_t i = tid; i < n; i += blockDim.x) {
      const double v = X[i + k * n];
      part1[0] += v * v;
    }
    block_sum(part1, 1, red, h);
    const double nrm = sqrt(h[0]);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int64_t i = tid; i < n; i += blockDim.x) X[i + k * n] *= inv;
    __threadfence();
    __syncthreads();
  }
}

// NX = Nsym X (n x b), one 64-row block per workgroup, 256 threads.
__global__ __launch_bounds__(256) void k_symm_mult(const double* __restrict__ Ns, int64_t n,
                                                   int b, const double* __restrict__ X,
                                                   double* __restrict__ NX) {
  const int rr = threadIdx.x % 64;
  const int cg = threadIdx.x / 64;  // 4 column groups
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + rr;
  double acc[6] = {};
  if (i < n) {
    for (int64_t p = 0; p < n; ++p) {
      const double a = Ns[i + p * n];
#pragma unroll
      for (int u = 0; u < 6; ++u) {
        const int c = cg + 4 * u;
        if (c < b) acc[u] += a * X[p + c * n];
      }
    }
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int c = cg + 4 * u;
      if (c < b) NX[i + c * n] = acc[u];
    }
  }
}

// Cyclic Jacobi on the b x b symmetric H (row-major, LDS) by one wavefront; the lanes
// apply each rotation's row/column updates in parallel.  Q accumulates the rotations.
__device__ void jacobi_wave(double* H, double* Q, int b) {
  const int lane = threadIdx.x & 63;
  for (int i = lane; i < b * b; i += 64) Q[i] = ((i / b) == (i % b)) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 40; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < b - 1; ++p) {
      for (int q = p + 1; q < b; ++q) {
        const double apq = H[p * b + q];
        const double app = H[p * b + p];
        const double aqq = H[q * b + q];
        if (!(fabs(apq) > 2.220446049250313e-16 * sqrt(fabs(app * aqq)))) continue;
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
        const int k = lane;
        double akp = 0.0, akq = 0.0, qkp = 0.0, qkq = 0.0;
        if (k < b) {
          akp = H[k * b + p];
          akq = H[k * b + q];
          qkp = Q[k * b + p];
          qkq = Q[k * b + q];
        }
        __builtin_amdgcn_wave_barrier();
        if (k < b) {
          if (k != p && k != q) {
            const double nkp = c * akp - s * akq;
            const double nkq = s * akp + c * akq;
            H[k * b + p] = nkp;
            H[p * b + k] = nkp;
            H[k * b + q] = nkq;
            H[q * b + k] = nkq;
          }
          Q[k * b + p] = c * qkp - s * qkq;
          Q[k * b + q] = s * qkp + c * qkq;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
          H[p * b + p] = app - t * apq;
          H[q * b + q] = aqq + t * apq;
          H[p * b + q] = 0.0;
          H[q * b + p] = 0.0;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (!rotated) break;
  }
}

// Rayleigh-Ritz on span(X), then V-hat, lambda_1..lambda_{r+1}, residual and flags.
__global__ __launch_bounds__(256) void k_rayleigh_ritz(const double* __restrict__ X,
                                                       const double* __restrict__ NX, int64_t n,
                                                       int b, int r, double* __restrict__ V,
                                                       DevScalars* scal, rsm_info* info,
                                                       int check_accepted) {
  __shared__ double H[kEigMaxB * kEigMaxB];
  __shared__ double Q[kEigMaxB * kEigMaxB];
  __shared__ int order[kEigMaxB];
  __shared__ double theta[kEigMaxB];
  __shared__ double resid[RSM_MAX_R];
  const int tid = threadIdx.x;
  // H = X^T NX, one thread per entry (b <= 21 -> at most 441 entries)
  for (int e = tid; e < b * b; e += blockDim.x) {
    const int i = e / b, j = e % b;
    double s = 0.0;
    for (int64_t p = 0; p < n; ++p) s += X[p + i * n] * NX[p + j * n];
    H[e] = s;
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += blockDim.x) {
    const int i = e / b, j = e % b;
    if (i < j) {
      const double avg = 0.5 * (H[i * b + j] + H[j * b + i]);
      H[i * b + j] = avg;
      H[j * b + i] = avg;
    }
  }
  __syncthreads();
  if (tid < 64) jacobi_wave(H, Q, b);
  __syncthreads();
  if (tid < b) {
    const double dk = H[tid * b + tid];
    int rk = 0;
    for (int j = 0; j < b; ++j) {
      const double dj = H[j * b + j];
      rk += (dj < dk) || (dj == dk && j < tid);
    }
    order[rk] = tid;
    theta[rk] = dk;
  }
  __syncthreads();
  // V-hat = X Q[:, order[0..r)]
  for (int64_t e = tid; e < n * r; e += blockDim.x) {
    const int64_t i = e % n;
    const int k = static_cast<int>(e / n);
    const int col = order[k];
    double s = 0.0;
    for (int j = 0; j < b; ++j) s += X[i + j * n] * Q[j * b + col];
    V[i + static_cast<int64_t>(k) * n] = s;
  }
  // residual of each Ritz pair: ||NX q - theta X q||
  if (tid < 64) {
    for (int k = 0; k < r; ++k) {
      const int col = order[k];
      double part = 0.0;
      for (int64_t i = tid; i < n; i += 64) {
        double s = 0.0;
        for (int j = 0; j < b; ++j) s += (NX[i + j * n] - theta[k] * X[i + j * n]) * Q[j * b + col];
        part += s * s;
      }
      part = wave_sum(part);
      if (tid == 0) resid[k] = sqrt(part);
    }
  }
  __syncthreads();
  if (tid == 0) {
    const double lam_max = scal->lam_max;
    double rmax = 0.0;
    for (int k = 0; k < r; ++k) rmax = fmax(rmax, resid[k]);
    const double rel = lam_max > 0.0 ? rmax / lam_max : rmax;
    info->residual = rel;
    for (int k = 0; k <= r && k < b; ++k) info->lambda[k] = theta[k];
    uint32_t warn = 0;
    if (info->uncovered > 0) warn |= RSM_W_RANK_DEFICIENT;
    if (b > r && !(theta[r] > 1e-12 * lam_max)) warn |= RSM_W_RANK_DEFICIENT;
    if (rel > 1e-6) warn |= RSM_W_NOT_CONVERGED;
    if (scal->pivots > 0) warn |= RSM_W_PIVOT;
    if (check_accepted && info->accepted == 0) warn |= RSM_W_NO_CONSTRAINTS;
    atomicOr(&info->warn, warn);
    info->eig_iterations = kEigIters;
  }
}

}  // namespace

void launch_solve_v(const Plan& P, const double* N, double* Nsym, double* Lf, double* Lt,
                    double* Dinv, double* X, double* Z, double* NX, DevScalars* scal, double* V,
                    rsm_info* info, hipStream_t s) {
  const int64_t n = P.n;
  const int b = P.eig_b;
  const unsigned g_nn = static_cast<unsigned>(ceil_div(n * n, 256));
  k_symmetrize<<<g_nn, 256, 0, s>>>(N, n, Nsym);
  k_norm_stats<<<static_cast<unsigned>(ceil_div(n, 256)), 256, 0, s>>>(Nsym, n, scal, info);
  k_chol_init<<<g_nn, 256, 0, s>>>(Nsym, n, Lf, scal, info);
  const int nb = P.nb;
  for (int k = 0; k < nb; ++k) {
    k_chol_diag<<<1, 256, 0, s>>>(Lf, n, k, scal);
    if (nb - k - 1 > 0) k_chol_panel<<<static_cast<unsigned>(nb - k - 1), 256, 0, s>>>(Lf, n, k);
    const int tiles = (nb - k - 1) * (nb - k) / 2;
    if (tiles > 0) k_chol_update<<<static_cast<unsigned>(tiles), 256, 0, s>>>(Lf, n, k, nb);
  }
  // Nsym is not needed past this point except for the Rayleigh-Ritz product; the
  // transposed factor goes to Lt and the tile inverses to Dinv.
  k_transpose_lower<<<g_nn, 256, 0, s>>>(Lf, n, Lt);
  k_diag_inverse<<<static_cast<unsigned>(nb), 64, 0, s>>>(Lf, n, Dinv);
  k_start_vectors<<<static_cast<unsigned>(ceil_div(n * b, 256)), 256, 0, s>>>(X, n, b, P.seed ^ 0x9E3779B97F4A7C15ull);
  for (int it = 0; it < kEigIters; ++it) {
    k_trsm<<<1, 256, 0, s>>>(Lf, n, b, Dinv, X, Z, 0);
    k_trsm<<<1, 256, 0, s>>>(Lt, n, b, Dinv, Z, Z, 1);
    k_orth<<<1, 1024, 0, s>>>(Z, n, b, X);
  }
  k_symm_mult<<<static_cast<unsigned>(ceil_div(n, 64)), 256, 0, s>>>(Nsym, n, b, X, NX);
  k_rayleigh_ritz<<<1, 256, 0, s>>>(X, NX, n, b, P.r, V, scal, info,
                                    (P.flags & RSM_FINALIZE_ONLY) ? 0 : 1);
}

}  // namespace rsm
