// Step a6: V-hat = the r eigenvectors of N = Xi Xi^T with the smallest eigenvalues
// (eq.(solve.barV_L2_norm); "||V|| = 1" read as V^T V = I_r).  FP64 throughout.
//
// N is symmetric positive semidefinite and its wanted eigenvalues are the smallest ones,
// i.e. the dominant ones of (N + mu I)^{-1}.  The solver:
//   1. Nsym = N with the upper triangle mirrored; Gershgorin bound lam_max of lambda_max(N);
//      the count of uncovered columns (N_jj == 0).
//   2. mu = 1e-8 lam_max, so cond(N + mu I) <= 1e8 and cond(L) <= 1e4: the factor and its
//      explicit inverse stay accurate to ~1e-12 relative, while one step of inverse
//      iteration still shrinks the unwanted components by (lambda_r + mu) /
//      (lambda_{b+1} + mu).  Blocked right-looking Cholesky N + mu I = L L^T in 64 x 64
//      tiles; each diagonal tile's inverse is formed with its factor, so the panel solve
//      is a product.
//   3. M = L^{-1} by recursive doubling over the tile structure:
//      [A 0; C B]^{-1} = [A^{-1} 0; -B^{-1} C A^{-1}  B^{-1}], log2(tiles) levels of
//      products (the matrix is padded to a power-of-two number of tiles with identity).
//   4. b = r + 4 vectors: X <- orth(M^T M X), a fixed number of steps, with classical
//      Gram-Schmidt applied twice (rows held in registers of one workgroup).
//   5. Rayleigh-Ritz: H = X^T N X, H = Q Theta Q^T by parallel-ordering Jacobi,
//      V-hat = X Q[:, :r]; lambda_1..lambda_{r+1} = Theta; residual
//      max_k ||N v_k - theta_k v_k|| / lam_max.
#include <cmath>

#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

constexpr int NB = kCholNB;
constexpr double kShiftRel = 1e-8;

__device__ __forceinline__ void atomic_max_pos_f64(double* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long*>(addr),
            static_cast<unsigned long long>(__double_as_longlong(v)));
}

__device__ __forceinline__ double shift_of(const DevScalars* scal) {
  const double lam = scal->lam_max;
  // N == 0 (no accepted trial): factor I instead; V-hat is then an arbitrary basis
  return lam > 0.0 ? kShiftRel * lam : 1.0;
}

// ------------------------------------------------------------------ 1. preparation

// Nsym (full), Lf = lower(N) (the shift is added when a diagonal tile is factored),
// uncovered columns.
__global__ void k_eig_prep(const double* __restrict__ N, int64_t n, double* __restrict__ Ns,
                           double* __restrict__ Lf, double* __restrict__ rowsum, rsm_info* info) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx < n) rowsum[idx] = 0.0;
  if (idx >= n * n) return;
  const int64_t j = idx / n, i = idx - j * n;
  const double v = (i >= j) ? N[i + j * n] : N[j + i * n];
  Ns[idx] = v;
  Lf[idx] = (i >= j) ? v : 0.0;
  if (i == j && v == 0.0) atomicAdd(&info->uncovered, 1);
}

// Row sums of |N| over a column chunk (rows in 64-row blocks, columns split in chunks):
// rowsum_i += sum_{j in chunk} |N_ij|.  max_i rowsum_i >= lambda_max(N) (Gershgorin).
__global__ __launch_bounds__(256) void k_rowsum(const double* __restrict__ Ns, int64_t n,
                                                int64_t cols_per_chunk,
                                                double* __restrict__ rowsum) {
  __shared__ double red[4][64];
  const int rr = threadIdx.x % 64, g = threadIdx.x / 64;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + rr;
  const int64_t j0 = static_cast<int64_t>(blockIdx.y) * cols_per_chunk;
  const int64_t j1 = (j0 + cols_per_chunk < n) ? (j0 + cols_per_chunk) : n;
  double s = 0.0;
  if (i < n)
    for (int64_t j = j0 + g; j < j1; j += 4) s += fabs(Ns[i + j * n]);
  red[g][rr] = s;
  __syncthreads();
  if (g == 0 && i < n) atomic_add_f64(&rowsum[i], red[0][rr] + red[1][rr] + red[2][rr] + red[3][rr]);
}

// ------------------------------------------------------------------ 2. Cholesky

// Factor tile (k, k) of N + mu I and invert the factor, by one wavefront: lane i holds
// row i of the tile in registers (static indices after full unrolling).  Step j of the
// factorisation broadcasts column j through LDS; step j of the inverse (L X = I, rows of
// X finished in order) broadcasts row j of X.  Writes L_kk into Lf and Dinv_kk = L_kk^{-1}.
// A ragged last tile is completed with the identity.
// Step J of the left-looking (Crout) factorisation, lane = row: column J of L is
//   l_iJ = (a_iJ - sum_{p<J} l_ip l_Jp) / l_JJ,   l_JJ = sqrt(a_JJ - sum_{p<J} l_Jp^2),
// with row J of L read from LDS (broadcast) and the lane's own finished entries l[0..J)
// in registers.  The pivot lane stores 1 / l_JJ (from rsqrt) for the other lanes and for
// the inverse.  Four partial sums shorten the dependent chain.  The template recursion
// keeps every index static.
template <int J>
__device__ __forceinline__ void crout_steps(double (&l)[NB], const double (*As)[NB + 1],
                                            double (*Ls)[NB + 1], double* invd, int lane,
                                            double mu, int& npiv) {
  if constexpr (J < NB) {
    double s4[4] = {As[lane][J], 0.0, 0.0, 0.0};
#pragma unroll
    for (int p0 = 0; p0 < J; p0 += 8) {
#pragma unroll
      for (int p = p0; p < p0 + 8 && p < J; ++p) s4[p & 3] -= l[p] * Ls[J][p];
      __builtin_amdgcn_sched_barrier(0);
    }
    double sum = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    if (lane == J) {
      if (!(sum > 0.0) || !isfinite(sum)) {
        sum = mu;
        ++npiv;
      }
      const double inv = rsqrt(sum);
      l[J] = sum * inv;
      Ls[J][J] = l[J];
      invd[J] = inv;
    }
    __syncthreads();
    if (lane > J) {
      l[J] = sum * invd[J];
      Ls[lane][J] = l[J];
    }
    __syncthreads();
    crout_steps<J + 1>(l, As, Ls, invd, lane, mu, npiv);
  }
}

// Step J of X = L^{-1} (lane = row of X): row J of X is final; rows below subtract it.
template <int J>
__device__ __forceinline__ void trinv_steps(double (&x)[NB], double* bc, double (*Ls)[NB + 1],
                                            const double* invd, int lane) {
  if constexpr (J < NB) {
    if (lane == J) {
      const double inv = invd[J];
#pragma unroll
      for (int c = 0; c <= J; ++c) {
        x[c] *= inv;
        bc[c] = x[c];
      }
    }
    __syncthreads();
    if (lane > J) {
      const double lij = Ls[lane][J];
#pragma unroll
      for (int c0 = 0; c0 <= J; c0 += 8) {
#pragma unroll
        for (int c = c0; c < c0 + 8 && c <= J; ++c) x[c] -= lij * bc[c];
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    __syncthreads();
    trinv_steps<J + 1>(x, bc, Ls, invd, lane);
  }
}

__global__ __launch_bounds__(64) void k_chol_diag(double* __restrict__ Lf, int64_t n, int k,
                                                  double* __restrict__ Dinv,
                                                  const double* __restrict__ rowsum,
                                                  DevScalars* scal, rsm_info* info) {
  __shared__ double bc[NB];
  __shared__ double invd[NB];
  __shared__ double As[NB][NB + 1];
  __shared__ double Ls[NB][NB + 1];
  __shared__ double lam;
  const int lane = threadIdx.x;
  const int64_t k0 = static_cast<int64_t>(k) * NB;
  const int kb = static_cast<int>((n - k0) < NB ? (n - k0) : NB);
  if (k == 0) {  // Gershgorin bound from the row sums, once
    double v = 0.0;
    for (int64_t i = lane; i < n; i += NB) v = fmax(v, rowsum[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if (lane == 0) {
      scal->lam_max = v;
      lam = v;
    }
  } else if (lane == 0) {
    lam = scal->lam_max;
  }
  __syncthreads();
  const double mu = lam > 0.0 ? kShiftRel * lam : 1.0;
  if (k == 0 && lane == 0) {
    scal->mu = mu;
    info->mu = mu;
  }
  // stage the tile (coalesced: lane = row), shift on the diagonal, identity past n
  for (int c = 0; c < NB; ++c) {
    double v;
    if (lane < kb && c < kb)
      v = (c <= lane) ? Lf[(k0 + lane) + (k0 + c) * n] + (c == lane ? mu : 0.0) : 0.0;
    else
      v = (lane == c) ? 1.0 : 0.0;
    As[lane][c] = v;
    Ls[lane][c] = 0.0;
  }
  __syncthreads();
  int npiv = 0;
  {
    double l[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) l[c] = 0.0;
    crout_steps<0>(l, As, Ls, invd, lane, mu, npiv);
  }
  for (int c = 0; c < NB; ++c)  // L back to memory (lower part)
    if (lane < kb && c < kb && c <= lane) Lf[(k0 + lane) + (k0 + c) * n] = Ls[lane][c];
  {
    double x[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) x[c] = (c == lane) ? 1.0 : 0.0;
    trinv_steps<0>(x, bc, Ls, invd, lane);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NB; ++c) Ls[lane][c] = (c <= lane) ? x[c] : 0.0;
  }
  __syncthreads();
  double* out = Dinv + static_cast<int64_t>(k) * NB * NB;
  for (int c = 0; c < NB; ++c) out[lane + c * NB] = Ls[lane][c];
  if (npiv) atomicAdd(&scal->pivots, npiv);
}

// Panel: tile (k+1+bid, k) becomes L_ik = A_ik L_kk^{-T} = A_ik Dinv_kk^T.
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ Lf, int64_t n, int k,
                                                    const double* __restrict__ Dinv) {
  __shared__ double Xs[NB][NB + 1];
  __shared__ double Ds[NB][NB + 1];
  const int tid = threadIdx.x;
  const int64_t k0 = static_cast<int64_t>(k) * NB;
  const int kb = static_cast<int>((n - k0) < NB ? (n - k0) : NB);
  const int64_t i0 = k0 + static_cast<int64_t>(blockIdx.x + 1) * NB;
  const int ib = static_cast<int>((n - i0) < NB ? (n - i0) : NB);
  const double* dk = Dinv + static_cast<int64_t>(k) * NB * NB;
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int ii = e % NB, jj = e / NB;
    Xs[ii][jj] = (ii < ib && jj < kb) ? Lf[(i0 + ii) + (k0 + jj) * n] : 0.0;
    Ds[ii][jj] = dk[e];
  }
  __syncthreads();
  const int tx = tid % 16, ty = tid / 16;
  double acc[4][4] = {};
  for (int p = 0; p < NB; ++p) {
    double a[4], d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = Xs[ty * 4 + u][p];
      d[u] = Ds[tx * 4 + u][p];  // (Dinv^T)[p][c] = Dinv[c][p]
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * d[v];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = ty * 4 + u, cc = tx * 4 + v;
      if (rr < ib && cc < kb) Lf[(i0 + rr) + (k0 + cc) * n] = acc[u][v];
    }
}

// Trailing update after panel k: tile (i, j), k < j <= i:  A_ij -= L_ik L_jk^T.
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ Lf, int64_t n, int k,
                                                     int nb) {
  __shared__ double Li[NB][NB + 1];
  __shared__ double Lj[NB][NB + 1];
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

// ------------------------------------------------------------------ 3. M = L^{-1}

// M (npad x npad, ld npad): diagonal tiles = Dinv (identity past the last tile), and the
// strictly lower tiles of L copied in (zero past n) as the blocks C of the recursion.
__global__ void k_inv_init(const double* __restrict__ Lf, const double* __restrict__ Dinv,
                           int64_t n, int nb, int64_t npad, double* __restrict__ M) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= npad * npad) return;
  const int64_t c = idx / npad, rr = idx - c * npad;
  const int64_t ti = rr / NB, tj = c / NB;
  double v = 0.0;
  if (ti == tj) {
    if (ti < nb)
      v = Dinv[ti * NB * NB + (rr - ti * NB) + (c - tj * NB) * NB];
    else
      v = (rr == c) ? 1.0 : 0.0;
  } else if (ti > tj && rr < n && c < n) {
    v = Lf[rr + c * n];
  }
  M[idx] = v;
}

// Level with inverted diagonal blocks of size bs: for every pair of consecutive blocks,
// T = C A^{-1} where C = M[block2, block1] (still the L entries) and A^{-1} = M[block1,
// block1] (lower triangular).  One 64 x 64 output tile per workgroup.
__global__ __launch_bounds__(256) void k_inv_stage1(const double* __restrict__ M, int64_t npad,
                                                    int64_t bs, double* __restrict__ T) {
  __shared__ double As[NB][NB + 1];
  __shared__ double Bs[NB][NB + 1];
  const int64_t tpb = bs / NB;                       // tiles per block side
  const int64_t pair = blockIdx.x / (tpb * tpb);
  const int64_t rem = blockIdx.x - pair * tpb * tpb;
  const int64_t ti = rem / tpb, tj = rem % tpb;      // output tile inside the pair
  const int64_t r1 = pair * 2 * bs;                  // block 1 origin
  const int64_t r2 = r1 + bs;                        // block 2 origin
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  double acc[4][4] = {};
  // T[ti, tj] = sum_q C[ti, q] Ainv[q, tj], q >= tj (Ainv lower)
  for (int64_t q = tj; q < tpb; ++q) {
    for (int e = tid; e < NB * NB; e += blockDim.x) {
      const int a = e % NB, c = e / NB;
      As[a][c] = M[(r2 + ti * NB + a) + (r1 + q * NB + c) * npad];  // C tile
      Bs[a][c] = M[(r1 + q * NB + a) + (r1 + tj * NB + c) * npad];  // Ainv tile
    }
    __syncthreads();
    for (int p = 0; p < NB; ++p) {
      double x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = As[ty * 4 + u][p];
        y[u] = Bs[p][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += x[u] * y[v];
    }
    __syncthreads();
  }
  const int64_t ldt = npad / 2;
  const int64_t base = (pair * bs + ti * NB) + (tj * NB) * ldt;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      T[base + (ty * 4 + u) + static_cast<int64_t>(tx * 4 + v) * ldt] = acc[u][v];
}

// M[block2, block1] = -B^{-1} T with B^{-1} = M[block2, block2] (lower triangular).
__global__ __launch_bounds__(256) void k_inv_stage2(double* __restrict__ M, int64_t npad,
                                                    int64_t bs, const double* __restrict__ T) {
  __shared__ double As[NB][NB + 1];
  __shared__ double Bs[NB][NB + 1];
  const int64_t tpb = bs / NB;
  const int64_t pair = blockIdx.x / (tpb * tpb);
  const int64_t rem = blockIdx.x - pair * tpb * tpb;
  const int64_t ti = rem / tpb, tj = rem % tpb;
  const int64_t r1 = pair * 2 * bs;
  const int64_t r2 = r1 + bs;
  const int64_t ldt = npad / 2;
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  double acc[4][4] = {};
  for (int64_t q = 0; q <= ti; ++q) {
    for (int e = tid; e < NB * NB; e += blockDim.x) {
      const int a = e % NB, c = e / NB;
      As[a][c] = M[(r2 + ti * NB + a) + (r2 + q * NB + c) * npad];      // Binv tile
      Bs[a][c] = T[(pair * bs + q * NB + a) + (tj * NB + c) * ldt];     // T tile
    }
    __syncthreads();
    for (int p = 0; p < NB; ++p) {
      double x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = As[ty * 4 + u][p];
        y[u] = Bs[p][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += x[u] * y[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      M[(r2 + ti * NB + ty * 4 + u) + (r1 + tj * NB + tx * 4 + v) * npad] = -acc[u][v];
}

// ------------------------------------------------------------------ 4. subspace iteration

// Deterministic start block: entries uniform in [-1, 1) from Philox (key = seed, 1).
__global__ void k_start_vectors(double* __restrict__ X, int64_t n, int b, uint64_t seed) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * b) return;
  uint64_t c[4] = {static_cast<uint64_t>(idx), 0x5eedull, 0ull, 0ull};
  Philox4x64::block(c, seed, 1ull);
  X[idx] = static_cast<double>(static_cast<int64_t>(c[0]) >> 11) * (1.0 / 4503599627370496.0);
}

__global__ void k_zero(double* __restrict__ x, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) x[i] = 0.0;
}

// Z += op(M)[row tile, col tile] X[col tile]  (one tile pair per workgroup; FP64 atomics).
// trans = 0: Z = M X with M lower;  trans = 1: Z = M^T X.
__global__ __launch_bounds__(256) void k_trmm(const double* __restrict__ M, int64_t npad,
                                              int64_t n, int b, const double* __restrict__ X,
                                              double* __restrict__ Z, int trans) {
  __shared__ double Ms[NB][NB + 1];
  __shared__ double Xs[NB][kEigMaxB + 1];
  const int nt = static_cast<int>(ceil_div(n, NB));
  // enumerate the tiles (i, k), k <= i, of the lower triangle of M
  int bidx = blockIdx.x;
  int ti = 0, tk = 0;
  for (int i = 0; i < nt; ++i) {
    if (bidx <= i) {
      ti = i;
      tk = bidx;
      break;
    }
    bidx -= i + 1;
  }
  if (trans) {  // M tile (ti, tk) feeds output rows tk of M^T X
    const int t = ti;
    ti = tk;
    tk = t;
  }
  const int tid = threadIdx.x;
  const int64_t r0 = static_cast<int64_t>(ti) * NB, k0 = static_cast<int64_t>(tk) * NB;
  for (int e = tid; e < NB * NB; e += blockDim.x) {
    const int a = e % NB, c = e / NB;
    // element (r0 + a, k0 + c) of op(M); loads run along the first index of M
    double v;
    if (!trans) {
      v = (r0 + a < n && k0 + c < n) ? M[(r0 + a) + (k0 + c) * npad] : 0.0;
      Ms[a][c] = v;
    } else {
      v = (k0 + a < n && r0 + c < n) ? M[(k0 + a) + (r0 + c) * npad] : 0.0;
      Ms[c][a] = v;
    }
  }
  for (int e = tid; e < NB * b; e += blockDim.x) {
    const int a = e % NB, c = e / NB;
    Xs[a][c] = (k0 + a < n) ? X[(k0 + a) + static_cast<int64_t>(c) * n] : 0.0;
  }
  __syncthreads();
  const int rr = tid % NB;
  const int cg = tid / NB;  // 4 column groups
  if (r0 + rr < n) {
    for (int c = cg; c < b; c += 4) {
      double s = 0.0;
#pragma unroll 8
      for (int p = 0; p < NB; ++p) s += Ms[rr][p] * Xs[p][c];
      atomic_add_f64(&Z[(r0 + rr) + static_cast<int64_t>(c) * n], s);
    }
  }
}

// X = orth(Z): classical Gram-Schmidt applied twice per column, one workgroup of 1024
// threads, thread t owning rows t, t + 1024, ... (RPT rows) in registers.
template <int RPT>
__global__ __launch_bounds__(1024) void k_orth(const double* __restrict__ Z, int64_t n, int b,
                                               double* __restrict__ X) {
  __shared__ double red[16][kEigMaxB];
  __shared__ double h[kEigMaxB];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  double x[RPT][kEigMaxB];
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int64_t i = tid + static_cast<int64_t>(s) * 1024;
#pragma unroll
    for (int c = 0; c < kEigMaxB; ++c) x[s][c] = (i < n && c < b) ? Z[i + c * n] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < kEigMaxB; ++k) {
    if (k < b) {
      for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
        for (int j = 0; j < k; ++j) {
          double p = 0.0;
#pragma unroll
          for (int s = 0; s < RPT; ++s) p += x[s][j] * x[s][k];
          p = wave_sum(p);
          if (lane == 0) red[wid][j] = p;
        }
        __syncthreads();
        if (tid < k) {
          double s = 0.0;
          for (int w = 0; w < 16; ++w) s += red[w][tid];
          h[tid] = s;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < k; ++j) {
          const double hj = h[j];
#pragma unroll
          for (int s = 0; s < RPT; ++s) x[s][k] -= hj * x[s][j];
        }
        __syncthreads();
      }
      double p = 0.0;
#pragma unroll
      for (int s = 0; s < RPT; ++s) p += x[s][k] * x[s][k];
      p = wave_sum(p);
      if (lane == 0) red[wid][0] = p;
      __syncthreads();
      if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < 16; ++w) s += red[w][0];
        h[0] = s;
      }
      __syncthreads();
      const double nrm = sqrt(h[0]);
      const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
#pragma unroll
      for (int s = 0; s < RPT; ++s) x[s][k] *= inv;
      __syncthreads();
    }
  }
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int64_t i = tid + static_cast<int64_t>(s) * 1024;
    if (i < n)
#pragma unroll
      for (int c = 0; c < kEigMaxB; ++c)
        if (c < b) X[i + c * n] = x[s][c];
  }
}

// NX += Nsym[row block, column chunk] X[column chunk] (NX zeroed beforehand; FP64
// atomics).  Thread per row, X staged through LDS.
__global__ __launch_bounds__(256) void k_symm_mult(const double* __restrict__ Ns, int64_t n,
                                                   int b, const double* __restrict__ X,
                                                   int64_t cols_per_chunk,
                                                   double* __restrict__ NX) {
  __shared__ double Xs[NB][kEigMaxB + 1];
  const int tid = threadIdx.x;
  const int rr = tid % 64, cg = tid / 64;  // 4 column groups
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + rr;
  const int64_t j0 = static_cast<int64_t>(blockIdx.y) * cols_per_chunk;
  const int64_t j1 = (j0 + cols_per_chunk < n) ? (j0 + cols_per_chunk) : n;
  double acc[6] = {};
  for (int64_t p0 = j0; p0 < j1; p0 += NB) {
    __syncthreads();
    for (int e = tid; e < NB * b; e += blockDim.x) {
      const int a = e % NB, c = e / NB;
      Xs[a][c] = (p0 + a < j1) ? X[(p0 + a) + static_cast<int64_t>(c) * n] : 0.0;
    }
    __syncthreads();
    if (i < n) {
      const int pe = static_cast<int>((j1 - p0) < NB ? (j1 - p0) : NB);
      for (int p = 0; p < pe; ++p) {
        const double a = Ns[i + (p0 + p) * n];
#pragma unroll
        for (int u = 0; u < 6; ++u) {
          const int c = cg + 4 * u;
          if (c < b) acc[u] += a * Xs[p][c];
        }
      }
    }
  }
  if (i < n) {
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int c = cg + 4 * u;
      if (c < b) atomic_add_f64(&NX[i + c * n], acc[u]);
    }
  }
}

// H += X[rows]^T NX[rows] over one 64-row block (H zeroed beforehand).
__global__ __launch_bounds__(256) void k_xtnx(const double* __restrict__ X,
                                              const double* __restrict__ NX, int64_t n, int b,
                                              double* __restrict__ H) {
  __shared__ double xs[NB][kEigMaxB + 1];
  __shared__ double ys[NB][kEigMaxB + 1];
  const int tid = threadIdx.x;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * NB;
  for (int e = tid; e < NB * b; e += blockDim.x) {
    const int a = e % NB, c = e / NB;
    const bool in = r0 + a < n;
    xs[a][c] = in ? X[(r0 + a) + static_cast<int64_t>(c) * n] : 0.0;
    ys[a][c] = in ? NX[(r0 + a) + static_cast<int64_t>(c) * n] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += blockDim.x) {
    const int i = e / b, j = e % b;
    double s = 0.0;
    for (int a = 0; a < NB; ++a) s += xs[a][i] * ys[a][j];
    atomic_add_f64(&H[e], s);
  }
}

// ------------------------------------------------------------------ 5. Rayleigh-Ritz

typedef double SmallMat[kEigMaxB + 1];

// Parallel-ordering (round-robin) Jacobi on the symmetric b x b matrix H (LDS), one
// workgroup.  Each round rotates floor(b/2) disjoint index pairs: the rotations are
// computed in parallel, then applied as H <- J^T H J and Q <- Q J.  For a pair (p, q),
// p < q, with c, s from the usual tau formula, column p becomes c col_p - s col_q and
// column q becomes s col_p + c col_q (rows likewise); storing sn[q] = -s makes both
// "cs[j] col_j - sn[j] col_partner".
__device__ void jacobi_rounds(SmallMat* H, SmallMat* Q, int b, SmallMat* tmp, int* perm,
                              double* cs, double* sn, int* partner, int* flag) {
  const int tid = threadIdx.x;
  const int bb = b + (b & 1);  // even number of players (one idle slot if b is odd)
  for (int e = tid; e < b * b; e += blockDim.x) Q[e / b][e % b] = ((e / b) == (e % b)) ? 1.0 : 0.0;
  if (tid < bb) perm[tid] = tid;
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int round = 0; round < bb - 1; ++round) {
      if (tid < bb) partner[tid] = -1;
      __syncthreads();
      if (tid < bb / 2) {
        int p = perm[tid], q = perm[bb - 1 - tid];
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q < b) {
          double c = 1.0, s = 0.0;
          const double apq = H[p][q], app = H[p][p], aqq = H[q][q];
          if (fabs(apq) > 2.220446049250313e-16 * sqrt(fabs(app * aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            double t;
            if (fabs(tau) > 1e150) {
              t = 0.5 / tau;
            } else {
              t = 1.0 / (fabs(tau) + sqrt(1.0 + tau * tau));
              if (tau < 0.0) t = -t;
            }
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            *flag = 1;
          }
          partner[p] = q;
          partner[q] = p;
          cs[p] = c;
          sn[p] = s;
          cs[q] = c;
          sn[q] = -s;
        }
      }
      __syncthreads();
      for (int e = tid; e < b * b; e += blockDim.x) {  // tmp = H J
        const int i = e / b, j = e % b;
        const int pj = partner[j];
        tmp[i][j] = (pj >= 0) ? cs[j] * H[i][j] - sn[j] * H[i][pj] : H[i][j];
      }
      __syncthreads();
      for (int e = tid; e < b * b; e += blockDim.x) {  // H = J^T tmp
        const int i = e / b, j = e % b;
        const int pi = partner[i];
        H[i][j] = (pi >= 0) ? cs[i] * tmp[i][j] - sn[i] * tmp[pi][j] : tmp[i][j];
      }
      __syncthreads();
      for (int e = tid; e < b * b; e += blockDim.x) {  // tmp = Q J
        const int i = e / b, j = e % b;
        const int pj = partner[j];
        tmp[i][j] = (pj >= 0) ? cs[j] * Q[i][j] - sn[j] * Q[i][pj] : Q[i][j];
      }
      __syncthreads();
      for (int e = tid; e < b * b; e += blockDim.x) {
        const int i = e / b, j = e % b;
        Q[i][j] = tmp[i][j];
        if (i < j) {  // keep H exactly symmetric
          const double avg = 0.5 * (H[i][j] + H[j][i]);
          H[i][j] = avg;
          H[j][i] = avg;
        }
      }
      if (tid == 0) {  // circle method: player 0 fixed, the others rotate
        const int last = perm[bb - 1];
        for (int k = bb - 1; k > 1; --k) perm[k] = perm[k - 1];
        perm[1] = last;
      }
      __syncthreads();
    }
    if (*flag == 0) break;
    __syncthreads();
  }
}

// Small part of Rayleigh-Ritz (one workgroup): Jacobi of H, eigenvalues sorted ascending;
// writes Qs = Q with its columns in that order and theta.
__global__ __launch_bounds__(256) void k_rr_small(const double* __restrict__ Hg, int b,
                                                  double* __restrict__ Qs,
                                                  double* __restrict__ theta_out) {
  __shared__ SmallMat H[kEigMaxB];
  __shared__ SmallMat Q[kEigMaxB];
  __shared__ SmallMat tmp[kEigMaxB];
  __shared__ int perm[kEigMaxB + 1];
  __shared__ double cs[kEigMaxB + 1];
  __shared__ double sn[kEigMaxB + 1];
  __shared__ int partner[kEigMaxB + 1];
  __shared__ int flag;
  __shared__ int order[kEigMaxB];
  const int tid = threadIdx.x;
  for (int e = tid; e < b * b; e += blockDim.x) {
    const int i = e / b, j = e % b;
    H[i][j] = 0.5 * (Hg[i * b + j] + Hg[j * b + i]);
  }
  __syncthreads();
  jacobi_rounds(H, Q, b, tmp, perm, cs, sn, partner, &flag);
  __syncthreads();
  if (tid < b) {
    const double dk = H[tid][tid];
    int rk = 0;
    for (int j = 0; j < b; ++j) {
      const double dj = H[j][j];
      rk += (dj < dk) || (dj == dk && j < tid);
    }
    order[rk] = tid;
    theta_out[rk] = dk;
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += blockDim.x) {
    const int j = e / b, k = e % b;  // Qs[j][k] = Q[j][order[k]]
    Qs[e] = Q[j][order[k]];
  }
}

// V-hat = X Qs[:, :r] and the squared residual norms ||NX q_k - theta_k X q_k||^2 (per
// 64-row block, accumulated into res2[k]).
__global__ __launch_bounds__(256) void k_rr_apply(const double* __restrict__ X,
                                                  const double* __restrict__ NX, int64_t n,
                                                  int b, int r, const double* __restrict__ Qs,
                                                  const double* __restrict__ theta,
                                                  double* __restrict__ V,
                                                  double* __restrict__ res2) {
  __shared__ double q[kEigMaxB * kEigMaxB];
  __shared__ double red[4][RSM_MAX_R];
  const int tid = threadIdx.x;
  for (int e = tid; e < b * b; e += blockDim.x) q[e] = Qs[e];
  __syncthreads();
  const int rr = tid % 64, g = tid / 64;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + rr;
  for (int k = g; k < r; k += 4) {
    double v = 0.0, res = 0.0;
    if (i < n) {
      for (int j = 0; j < b; ++j) {
        const double x = X[i + static_cast<int64_t>(j) * n];
        const double y = NX[i + static_cast<int64_t>(j) * n];
        v += x * q[j * b + k];
        res += (y - theta[k] * x) * q[j * b + k];
      }
      V[i + static_cast<int64_t>(k) * n] = v;
    }
    const double s2 = wave_sum(res * res);
    if (rr == 0) atomic_add_f64(&res2[k], s2);
  }
}

__global__ void k_rr_finish(int b, int r, const double* __restrict__ theta,
                            const double* __restrict__ res2, DevScalars* scal, rsm_info* info,
                            int check_accepted) {
  if (threadIdx.x != 0) return;
  const double lam_max = scal->lam_max;
  double rmax = 0.0;
  for (int k = 0; k < r; ++k) rmax = fmax(rmax, sqrt(res2[k]));
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

}  // namespace

void launch_solve_v(const Plan& P, const double* N, double* Nsym, double* Lf, double* Mi,
                    double* T, double* Dinv, double* X, double* Z, double* NX, DevScalars* scal,
                    double* V, rsm_info* info, hipStream_t s) {
  const int64_t n = P.n;
  const int b = P.eig_b;
  const int nb = P.nb;
  const int64_t npad = P.npad;
  const unsigned g_nn = static_cast<unsigned>(ceil_div(n * n, 256));
  const unsigned g_rows = static_cast<unsigned>(ceil_div(n, 64));
  const int64_t chunk_cols = ceil_div(n, 16);
  // small scratch carved from T (its first use, by the inverse, is over by then)
  double* rowsum = Z;              // n values, before the iteration uses Z
  double* Hb = T;                  // b x b
  double* Qs = T + kEigMaxB * kEigMaxB;
  double* theta = Qs + kEigMaxB * kEigMaxB;
  double* res2 = theta + kEigMaxB;
  k_eig_prep<<<g_nn, 256, 0, s>>>(N, n, Nsym, Lf, rowsum, info);
  k_rowsum<<<dim3(g_rows, 16), 256, 0, s>>>(Nsym, n, chunk_cols, rowsum);
  for (int k = 0; k < nb; ++k) {
    k_chol_diag<<<1, NB, 0, s>>>(Lf, n, k, Dinv, rowsum, scal, info);
    if (nb - k - 1 > 0) {
      k_chol_panel<<<static_cast<unsigned>(nb - k - 1), 256, 0, s>>>(Lf, n, k, Dinv);
      const int tiles = (nb - k - 1) * (nb - k) / 2;
      k_chol_update<<<static_cast<unsigned>(tiles), 256, 0, s>>>(Lf, n, k, nb);
    }
  }
  k_inv_init<<<static_cast<unsigned>(ceil_div(npad * npad, 256)), 256, 0, s>>>(Lf, Dinv, n, nb,
                                                                                npad, Mi);
  for (int64_t bs = NB; bs < npad; bs *= 2) {
    const int64_t tpb = bs / NB;
    const unsigned grid = static_cast<unsigned>((npad / (2 * bs)) * tpb * tpb);
    k_inv_stage1<<<grid, 256, 0, s>>>(Mi, npad, bs, T);
    k_inv_stage2<<<grid, 256, 0, s>>>(Mi, npad, bs, T);
  }
  k_start_vectors<<<static_cast<unsigned>(ceil_div(n * b, 256)), 256, 0, s>>>(
      X, n, b, P.seed ^ 0x9E3779B97F4A7C15ull);
  const int nt = static_cast<int>(ceil_div(n, NB));
  const unsigned tri = static_cast<unsigned>(nt * (nt + 1) / 2);
  const unsigned gz = static_cast<unsigned>(ceil_div(n * b, 256));
  for (int it = 0; it < kEigIters; ++it) {
    k_zero<<<gz, 256, 0, s>>>(Z, n * b);
    k_trmm<<<tri, 256, 0, s>>>(Mi, npad, n, b, X, Z, 0);
    k_zero<<<gz, 256, 0, s>>>(NX, n * b);
    k_trmm<<<tri, 256, 0, s>>>(Mi, npad, n, b, Z, NX, 1);
    if (n <= 1024)
      k_orth<1><<<1, 1024, 0, s>>>(NX, n, b, X);
    else if (n <= 2048)
      k_orth<2><<<1, 1024, 0, s>>>(NX, n, b, X);
    else
      k_orth<4><<<1, 1024, 0, s>>>(NX, n, b, X);
  }
  // Rayleigh-Ritz with the true N
  k_zero<<<gz, 256, 0, s>>>(NX, n * b);
  const int64_t small = kEigMaxB * kEigMaxB * 2 + 2 * kEigMaxB;
  k_zero<<<static_cast<unsigned>(ceil_div(small, 256)), 256, 0, s>>>(Hb, small);
  k_symm_mult<<<dim3(g_rows, 16), 256, 0, s>>>(Nsym, n, b, X, chunk_cols, NX);
  k_xtnx<<<g_rows, 256, 0, s>>>(X, NX, n, b, Hb);
  k_rr_small<<<1, 256, 0, s>>>(Hb, b, Qs, theta);
  k_rr_apply<<<g_rows, 256, 0, s>>>(X, NX, n, b, P.r, Qs, theta, V, res2);
  k_rr_finish<<<1, 64, 0, s>>>(b, P.r, theta, res2, scal, info,
                               (P.flags & RSM_FINALIZE_ONLY) ? 0 : 1);
}

}  // namespace rsm
