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
//      (lambda_{b+1} + mu).  Blocked Cholesky N + mu I = L L^T in 64 x 64 tiles, one launch
//      per tile step: each workgroup of the step solves the two panel tiles it needs with
//      the inverse of the diagonal tile, updates its trailing tile, and the workgroup that
//      owns the next diagonal tile factors it at once (look-ahead).  Factoring a diagonal
//      tile also forms its inverse, which becomes the diagonal tile of M = L^{-1}.  The
//      64 x 64 tile products run on the FP64 matrix cores.
//   3. M = L^{-1} by recursive doubling over the tile structure:
//      [A 0; C B]^{-1} = [A^{-1} 0; -B^{-1} C A^{-1}  B^{-1}], log2(tiles) levels of
//      products (the matrix is padded to a power-of-two number of tiles with identity).
//      M^T is stored as well, so that both products of an iteration read rows.
//   4. b = r + 4 vectors: X <- orth(M^T M X) by inverse subspace iteration until the
//      residual test of the r wanted Ritz pairs passes (one launch, k_subspace);
//   5. Rayleigh-Ritz at check iterations: H = X^T N X, H = Q Theta Q^T by parallel-ordering
//      Jacobi, V-hat = X Q[:, :r]; lambda_1..lambda_{r+1} = Theta; residual
//      max_k ||N v_k - theta_k v_k|| / lam_max, the stopping test.
// Every kernel takes an array of problem descriptors (problem = blockIdx.y), so a batch of
// problems of different sizes runs in the same launches; workgroups past a problem's own
// work return at once.
#include <cmath>

#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

constexpr int NB = kCholNB;     // 64
constexpr int kLd = NB + 4;     // LDS row stride of product operands (16-byte aligned rows)
constexpr int kTr = NB + 1;     // LDS row stride of transposition buffers (odd: no conflicts)
constexpr double kShiftRel = 1e-8;
constexpr int kDescPerLaunch = 16;

typedef RSM_GLOBAL double* gdouble;
typedef RSM_GLOBAL const double* gcdouble;

// Generic-pointer view of a global address, for the atomics.
template <typename T>
__device__ __forceinline__ T* generic(RSM_GLOBAL T* p) {
  return (T*)p;
}

// Global load at a 32-bit element offset from a uniform base: the compiler can then
// use the scalar-base + 32-bit vector-offset addressing form (every matrix here has fewer
// than 2^28 elements).
__device__ __forceinline__ double gld(gcdouble base, uint32_t idx) {
  return *reinterpret_cast<gcdouble>(reinterpret_cast<RSM_GLOBAL const char*>(base) + (idx << 3));
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(u), l);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(u >> 32), l);
  return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

// Orders the LDS accesses of one wavefront around this point (a wavefront's LDS operations
// complete in issue order, so no wait is needed, only no compiler reordering).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------------ 64 x 64 tiles

// Coordinates of element u (0..15) of thread threadIdx.x when 256 threads stage a 64 x 64
// tile.  TR: lanes run down a column (64 rows) and the tile lands transposed in LDS
// (S[c][a]); otherwise 16-lane groups run down a column (S[a][c]).  Both read whole
// 128-byte lines.
template <bool TR>
__device__ __forceinline__ void tile_coord(int u, int& a, int& c) {
  const int t = threadIdx.x;
  if (TR) {
    a = t & 63;
    c = (t >> 6) + 4 * u;
  } else {
    a = (t & 15) + 16 * (u & 3);
    c = ((t >> 4) & 15) + 16 * (u >> 2);
  }
}

// Loads the tile src[a + c * ld], rows a < rv and columns c < cv (zero elsewhere); all 16
// loads are issued before any is used.
template <bool TR>
__device__ __forceinline__ void tile_load(double (&v)[16], gcdouble __restrict__ src, int64_t ld,
                                          int rv, int cv) {
  const uint32_t ld32 = static_cast<uint32_t>(ld);
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    int a, c;
    tile_coord<TR>(u, a, c);
    const bool ok = a < rv && c < cv;
    const double x = gld(src, static_cast<uint32_t>(ok ? a : 0) + static_cast<uint32_t>(ok ? c : 0) * ld32);
    v[u] = ok ? x : 0.0;
  }
}

template <bool TR>
__device__ __forceinline__ void tile_store(double (*S)[kLd], const double (&v)[16]) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    int a, c;
    tile_coord<TR>(u, a, c);
    if (TR)
      S[c][a] = v[u];
    else
      S[a][c] = v[u];
  }
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Output coordinates (row, column of the 64 x 64 tile) of accumulator acc[u][v] of this
// thread in the layout of the FP64 matrix-core product: wavefront w owns the 32 x 32
// quadrant at (32 (w / 2), 32 (w % 2)), u is its 16 x 16 sub-tile (2 ti + tj) and v the
// register: row 16 ti + 4 v + lane / 16, column 16 tj + lane % 16.
__device__ __forceinline__ int acc_row(int u, int v) {
  return 32 * (static_cast<int>(threadIdx.x) >> 7) + 16 * (u >> 1) + 4 * v +
         ((static_cast<int>(threadIdx.x) & 63) >> 4);
}
__device__ __forceinline__ int acc_col(int u, int v) {
  (void)v;
  return 32 * ((static_cast<int>(threadIdx.x) >> 6) & 1) + 16 * (u & 1) +
         (static_cast<int>(threadIdx.x) & 15);
}

// acc[u][v] += sum_p X[p][acc_row(u, v)] Y[p][acc_col(u, v)]: the 64 x 64 product X^T Y of
// two LDS tiles on the FP64 matrix cores (v_mfma_f64_16x16x4f64: A(i, k) from lane
// i + 16 k, B(k, j) from lane j + 16 k, D(i, j) in lane j + 16 (i mod 4), register i / 4).
__device__ __forceinline__ void mm64(double (&acc)[4][4], const double (*X)[kLd],
                                     const double (*Y)[kLd]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  f64x4 c[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) c[u] = f64x4{acc[u][0], acc[u][1], acc[u][2], acc[u][3]};
#pragma unroll 4
  for (int p0 = 0; p0 < NB; p0 += 4) {
    const double a0 = X[p0 + g][r0 + j], a1 = X[p0 + g][r0 + 16 + j];
    const double b0 = Y[p0 + g][c0 + j], b1 = Y[p0 + g][c0 + 16 + j];
    c[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c[0], 0, 0, 0);
    c[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, c[1], 0, 0, 0);
    c[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, c[2], 0, 0, 0);
    c[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c[3], 0, 0, 0);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = c[u][v];
}

// Writes the thread's outputs as the transposed operand layout S[col][row].
__device__ __forceinline__ void acc_store_tr(double (*S)[kLd], const double (&acc)[4][4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) S[acc_col(u, v)][acc_row(u, v)] = acc[u][v];
}

// ------------------------------------------------------------------ diagonal tile

// The 64 x 64 diagonal tile is factored and inverted by the 256 threads of a workgroup in
// 16 x 16 blocks: right-looking block Cholesky (the 16 x 16 diagonal blocks by one
// wavefront in registers, the panel and trailing update by all four wavefronts on the
// matrix cores), then L^{-1} block row by block row: X_ii = L_ii^{-1},
// X_ik = -X_ii sum_{p=k}^{i-1} L_ip X_pk.
constexpr int kFB = 16;        // block of the in-tile factorisation
constexpr int kFBs = kFB + 1;  // its LDS row stride
constexpr int kNFB = NB / kFB;

struct FactorWork {
  double Lt[kFB][kFB];            // the current diagonal block's factor: Lt[p][i] = l_ip
  double invd[kFB];               // 1 / l_jj of the current block
  double D[kNFB][kFB][kFBs];      // inverses of the diagonal blocks' factors
  double S[kNFB - 1][kFB][kFBs];  // partial sums of the inverse
};

// Step J of the left-looking (Crout) factorisation of a 16 x 16 block by one wavefront, lane
// = row i (< 16):  l_iJ = (a_iJ - sum_{p<J} l_ip l_Jp) / l_JJ,  l_JJ = sqrt(a_JJ - sum_{p<J}
// l_Jp^2).  a[] holds the lane's row (finished entries l_ip for p < J); the finished row J
// of L and the pivot are read from lane J's registers (readlane), so a step has no LDS
// round trip.  The recursion keeps every register index static.
template <int J>
__device__ __forceinline__ void crout_steps(double (&a)[kFB], double (&invd)[kFB], int lane,
                                            double mu, int& npiv) {
  if constexpr (J < kFB) {
    double s2[2] = {a[J], 0.0};
#pragma unroll
    for (int p = 0; p < J; ++p) s2[p & 1] -= a[p] * readlane_f64(a[p], J);
    const double sum = s2[0] + s2[1];
    double d = readlane_f64(sum, J);
    if (!(d > 0.0) || !isfinite(d)) {  // uniform: every lane holds the same d
      d = mu;
      ++npiv;
    }
    const double inv = rsqrt(d);
    a[J] = lane < J ? 0.0 : (lane == J ? d * inv : sum * inv);
    invd[J] = inv;
    crout_steps<J + 1>(a, invd, lane, mu, npiv);
  }
}

// Wavefront 0: factor diagonal block KB of As and store the inverse of its factor in W.D[KB]
// (the factor goes to LDS once; lane = column c: x_i = (delta_ic - sum_{p<i} l_ip x_p) /
// l_ii with row i of L read as broadcasts).
template <int KB>
__device__ __forceinline__ void fb_diag(double (*As)[kTr], FactorWork& W, double mu, int& npiv) {
  constexpr int k0 = KB * kFB;
  const int lane = threadIdx.x;
  const int row = lane < kFB ? lane : 0;
  double a[kFB], invd[kFB];
#pragma unroll
  for (int c = 0; c < kFB; ++c) a[c] = c <= row ? As[k0 + row][k0 + c] : 0.0;
  crout_steps<0>(a, invd, lane, mu, npiv);
  if (lane < kFB)
#pragma unroll
    for (int p = 0; p < kFB; ++p) W.Lt[p][lane] = a[p];
  if (lane == 0)
#pragma unroll
    for (int p = 0; p < kFB; ++p) W.invd[p] = invd[p];
  wave_lds_fence();
  double x[kFB];
#pragma unroll
  for (int i = 0; i < kFB; ++i) {
    double s2[2] = {i == lane ? 1.0 : 0.0, 0.0};
#pragma unroll
    for (int p = 0; p < i; ++p) s2[p & 1] -= W.Lt[p][i] * x[p];
    x[i] = (s2[0] + s2[1]) * W.invd[i];
  }
  if (lane < kFB)
#pragma unroll
    for (int i = 0; i < kFB; ++i) W.D[KB][i][lane] = x[i];
}

// All threads: panel L_rk = A_rk D_k^T for the rows below block KB, then the trailing update
// A_rc -= L_rk L_ck^T (lower part), on the FP64 matrix cores one 16 x 16 output tile per
// wavefront at a time.  A panel tile is read and written by the wavefront that owns it, so
// only the trailing update waits for the whole panel.
template <int KB>
__device__ __forceinline__ void fb_panel_update(double (*As)[kTr], FactorWork& W) {
  constexpr int k0 = KB * kFB;
  constexpr int B = (NB - k0 - kFB) / kFB;
  if constexpr (B > 0) {
    constexpr int r0 = k0 + kFB;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // panel: tile u = rows r0 + 16 u .. of L_rk; A(i, k) = A_rk[16 u + i][4 s + k],
    // B(k, j) = D_k[j][4 s + k]
    for (int u = w; u < B; u += 4) {
      f64x4 c = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < kFB; s4 += 4) {
        const double a = As[r0 + 16 * u + li][k0 + s4 + lk];
        const double bb = W.D[KB][li][s4 + lk];
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, c, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) As[r0 + 16 * u + 4 * v + lk][k0 + li] = c[v];
    }
    __syncthreads();
    // trailing tiles (u, v), v <= u: A(i, k) = L[16 u + i][4 s + k], B(k, j) = L[16 v + j][4 s + k]
    constexpr int NT = B * (B + 1) / 2;
    for (int tl = w; tl < NT; tl += 4) {
      int u = 0;
      while ((u + 1) * (u + 2) / 2 <= tl) ++u;
      const int v = tl - u * (u + 1) / 2;
      f64x4 c = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < kFB; s4 += 4) {
        const double a = As[r0 + 16 * u + li][k0 + s4 + lk];
        const double bb = As[r0 + 16 * v + li][k0 + s4 + lk];
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, c, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 4 * q + lk, j = li;
        if (u != v || j <= i) As[r0 + 16 * u + i][r0 + 16 * v + j] -= c[q];
      }
    }
    __syncthreads();
  }
}

// X_Ik for k < I (block row I of L^{-1}), all threads; Xs already holds block rows < I.
template <int I>
__device__ __forceinline__ void fb_inverse_row(double (*As)[kTr], double (*Xs)[kTr],
                                               FactorWork& W) {
  const int t = threadIdx.x, tc = t & 15, tr = t >> 4;
#pragma unroll
  for (int k = 0; k < I; ++k) {
    double s = 0.0;
#pragma unroll
    for (int q = kFB * k; q < kFB * I; ++q) s = fma(As[kFB * I + tr][q], Xs[q][kFB * k + tc], s);
    W.S[k][tr][tc] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < I; ++k) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kFB; ++q) s = fma(W.D[I][tr][q], W.S[k][q][tc], s);
    Xs[kFB * I + tr][kFB * k + tc] = -s;
  }
  __syncthreads();
}

// 256 threads: factor the tile As (64 x kTr in LDS: N + mu I in the lower triangle, identity
// rows and columns past the matrix) and write its inverse factor X = L^{-1} as tile (t0, t0)
// of M and X^T as tile (t0, t0) of Mt (column-major, leading dimension ld).  Xs: 64 x kTr of
// LDS.  Returns the clamped pivots (meaningful in thread 0).
__device__ __forceinline__ int factor_tile(double (*As)[kTr], double (*Xs)[kTr], FactorWork& W,
                                           double mu, gdouble __restrict__ M,
                                           gdouble __restrict__ Mt, int ld, int t0) {
  int npiv = 0;
  const int t = threadIdx.x;
#define RSM_FB_STEP(KB)                                  \
  if (t < 64) fb_diag<KB>(As, W, mu, npiv);              \
  __syncthreads();                                       \
  fb_panel_update<KB>(As, W);
  RSM_FB_STEP(0)
  RSM_FB_STEP(1)
  RSM_FB_STEP(2)
  RSM_FB_STEP(3)
#undef RSM_FB_STEP
  // X: diagonal blocks D, zero above; block rows below the first follow
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int a = t & 63, c = (t >> 6) + 4 * u;
    const int ba = a / kFB, bc = c / kFB;
    Xs[a][c] = ba == bc ? W.D[ba][a % kFB][c % kFB] : 0.0;
  }
  __syncthreads();
  fb_inverse_row<1>(As, Xs, W);
  fb_inverse_row<2>(As, Xs, W);
  fb_inverse_row<3>(As, Xs, W);
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int a = t & 63, c = (t >> 6) + 4 * u;
    M[(t0 + a) + (t0 + c) * ld] = Xs[a][c];
    Mt[(t0 + a) + (t0 + c) * ld] = Xs[c][a];
  }
  return npiv;
}

// ------------------------------------------------------------------ descriptors, prep

struct EigProbPack {
  EigProb p[kDescPerLaunch];
  int count;
};

__global__ void k_put_desc(EigProbPack pack, EigProb* dst) {
  if (static_cast<int>(threadIdx.x) < pack.count) dst[threadIdx.x] = pack.p[threadIdx.x];
}

// Nsym (full), Lf = lower(N) (the shift is added when a diagonal tile is factored), uncovered
// columns, the padding of M and Mt (identity), zeroed small arrays.
__global__ __launch_bounds__(256) void k_eig_prep(const EigProb* __restrict__ probs) {
  const EigProb& P = probs[blockIdx.y];
  const int64_t n = P.n, npad = P.npad;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx == 0) {
    P.scal->bar = 0;
    P.scal->ticket = 0;
    P.scal->stalled = 0;
  }
  if (idx >= npad * npad) return;
  const int64_t c = idx / npad, rr = idx - c * npad;
  if (rr < n && c < n) {
    const double v = (rr >= c) ? P.N[rr + c * n] : P.N[c + rr * n];
    P.Nsym[rr + c * n] = v;
    P.Lf[rr + c * n] = (rr >= c) ? v : 0.0;
    if (rr == c && v == 0.0) atomicAdd(generic(&P.info->uncovered), 1);
  }
  const int64_t nbn = static_cast<int64_t>(P.nb) * NB;
  if (rr >= nbn || c >= nbn) {
    const double v = (rr == c) ? 1.0 : 0.0;
    P.M[idx] = v;
    P.Mt[idx] = v;
  }
}

// Row sums of |N| over a column chunk (rows in 64-row blocks, columns split in 16 chunks):
// T[chunk n + i] = sum_{j in chunk} |N_ij|; max_i sum_chunk T[chunk n + i] >= lambda_max(N)
// (Gershgorin).  Partial sums are stored, not added atomically, so the bound does not depend
// on the order in which workgroups finish.
__global__ __launch_bounds__(256) void k_rowsum(const EigProb* __restrict__ probs) {
  __shared__ double red[4][64];
  const EigProb& P = probs[blockIdx.z];
  const int64_t n = P.n;
  if (static_cast<int64_t>(blockIdx.x) * 64 >= n) return;
  const int64_t chunk = ceil_div(n, 16);
  const int rr = threadIdx.x % 64, g = threadIdx.x / 64;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + rr;
  const int64_t j0 = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t j1 = (j0 + chunk < n) ? (j0 + chunk) : n;
  const int64_t ic = i < n ? i : n - 1;
  double s = 0.0;
  for (int64_t jb = j0 + g; jb < j1; jb += 32) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t j = jb + 4 * u;
      const double x = P.Nsym[ic + (j < j1 ? j : j0) * n];
      v[u] = j < j1 ? fabs(x) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  red[g][rr] = s;
  __syncthreads();
  if (g == 0 && i < n)
    P.T[static_cast<int64_t>(blockIdx.y) * n + i] = (red[0][rr] + red[1][rr]) + (red[2][rr] + red[3][rr]);
}

// ------------------------------------------------------------------ 2. Cholesky

// Gershgorin bound, shift, and the factor + inverse of diagonal tile 0.
__global__ __launch_bounds__(256) void k_chol_first(const EigProb* __restrict__ probs) {
  __shared__ double As[NB][kTr];
  __shared__ double Xs[NB][kTr];
  __shared__ FactorWork W;
  __shared__ double red[4];
  const EigProb& P = probs[blockIdx.y];
  const int t = threadIdx.x, lane = t & 63;
  const int n = static_cast<int>(P.n);
  double v = 0.0;
  for (int i0 = 0; i0 < n; i0 += 4 * 256) {
    double x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * 256 + t;
      const int ic = i < n ? i : 0;
      double sum = 0.0;
#pragma unroll
      for (int c = 0; c < 16; ++c) sum += P.T[static_cast<int64_t>(c) * n + ic];
      x[u] = sum;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u * 256 + t < n) v = fmax(v, x[u]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if (lane == 0) red[t >> 6] = v;
  __syncthreads();
  v = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  // N == 0 (no accepted trial): factor I instead; V-hat is then an arbitrary basis
  const double mu = v > 0.0 ? kShiftRel * v : 1.0;
  if (t == 0) {
    P.scal->lam_max = v;
    P.scal->mu = mu;
    P.info->mu = mu;
  }
  const int kb = n < NB ? n : NB;
  gcdouble Lf = P.Lf;
  double x[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int a = t & 63, c = (t >> 6) + 4 * u;
    const bool ok = a < kb && c < kb;
    x[u] = Lf[(ok ? a : 0) + (ok ? c : 0) * n];
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int a = t & 63, c = (t >> 6) + 4 * u;
    As[a][c] = (a < kb && c < kb) ? (c < a ? x[u] : (c == a ? x[u] + mu : 0.0))
                                  : (a == c ? 1.0 : 0.0);
  }
  __syncthreads();
  const int npiv = factor_tile(As, Xs, W, mu, P.M, P.Mt, static_cast<int>(P.npad), 0);
  if (npiv && t == 0) atomicAdd(generic(&P.scal->pivots), npiv);
}

// Tile step k (k = 0 .. nb - 2).  Workgroup (i, j), k < j <= i < nb, of the trailing lower
// triangle:
//   L_ik = A_ik D_k^T, L_jk = A_jk D_k^T  (D_k = L_kk^{-1}, the diagonal tile k of M),
//   A_ij -= L_ik L_jk^T.
// The workgroup with j = k + 1 stores L_ik as tile (i, k) of M (the block C of the
// recursion); the one with i = j = k + 1 then factors the updated tile (look-ahead).
__global__ __launch_bounds__(256) void k_chol_step(const EigProb* __restrict__ probs, int k) {
  __shared__ __align__(16) double S0[NB][kLd];
  __shared__ __align__(16) double S1[NB][kLd];
  __shared__ __align__(16) double S2[NB][kLd];
  const EigProb& P = probs[blockIdx.y];
  const int rem = P.nb - k - 1;
  const int bid = static_cast<int>(blockIdx.x);
  if (rem <= 0 || bid >= rem * (rem + 1) / 2) return;
  int row = static_cast<int>((sqrtf(8.0f * static_cast<float>(bid) + 1.0f) - 1.0f) * 0.5f);
  while (row * (row + 1) / 2 > bid) --row;
  while ((row + 1) * (row + 2) / 2 <= bid) ++row;
  const int col = bid - row * (row + 1) / 2;
  const int ti = k + 1 + row, tj = k + 1 + col;
  const bool diag = ti == tj;
  const int64_t n = P.n, ld = P.npad;
  const int64_t k0 = static_cast<int64_t>(k) * NB;
  const int64_t i0 = static_cast<int64_t>(ti) * NB, j0 = static_cast<int64_t>(tj) * NB;
  const int ib = static_cast<int>((n - i0) < NB ? (n - i0) : NB);
  const int jb = static_cast<int>((n - j0) < NB ? (n - j0) : NB);
  gdouble __restrict__ Lf = P.Lf;

  double vi[16], vj[16], vd[16];
  tile_load<true>(vi, Lf + i0 + k0 * n, n, ib, NB);
  if (!diag) tile_load<true>(vj, Lf + j0 + k0 * n, n, jb, NB);
  tile_load<true>(vd, P.M + k0 + k0 * ld, ld, NB, NB);
  double cur[4][4];  // A_ij in the output layout
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = acc_row(u, v), cc = acc_col(u, v);
      const bool ok = rr < ib && cc < jb;
      const double x = Lf[(i0 + (ok ? rr : 0)) + (j0 + (ok ? cc : 0)) * n];
      cur[u][v] = ok ? x : 0.0;
    }
  tile_store<true>(S0, vi);  // S0[p][row] = A_ik[row][p]
  if (!diag) tile_store<true>(S2, vj);
  tile_store<true>(S1, vd);  // S1[p][col] = D_k[col][p]
  __syncthreads();
  double li[4][4] = {}, lj[4][4] = {};
  mm64(li, S0, S1);
  if (!diag) mm64(lj, S2, S1);
  __syncthreads();
  acc_store_tr(S0, li);  // S0[p][row] = L_ik[row][p]
  if (!diag) acc_store_tr(S2, lj);
  if (tj == k + 1) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) P.M[(i0 + acc_row(u, v)) + (k0 + acc_col(u, v)) * ld] = li[u][v];
  }
  __syncthreads();
  double upd[4][4] = {};
  mm64(upd, S0, diag ? S0 : S2);
  if (bid != 0) {  // not the next diagonal tile: write the updated tile back
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = acc_row(u, v), cc = acc_col(u, v);
        if (rr < ib && cc < jb && (!diag || cc <= rr))
          Lf[(i0 + rr) + (j0 + cc) * n] = cur[u][v] - upd[u][v];
      }
    return;
  }
  // tile (k + 1, k + 1): factor it now
  __syncthreads();
  auto As = reinterpret_cast<double (*)[kTr]>(&S1[0][0]);
  auto Xs = reinterpret_cast<double (*)[kTr]>(&S0[0][0]);
  FactorWork& W = *reinterpret_cast<FactorWork*>(&S2[0][0]);
  const double mu = P.scal->mu;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = acc_row(u, v), cc = acc_col(u, v);
      As[rr][cc] = (rr < ib && cc < ib) ? cur[u][v] - upd[u][v] + (rr == cc ? mu : 0.0)
                                        : (rr == cc ? 1.0 : 0.0);
    }
  __syncthreads();
  const int npiv = factor_tile(As, Xs, W, mu, P.M, P.Mt, static_cast<int>(ld), static_cast<int>(i0));
  if (npiv && threadIdx.x == 0) atomicAdd(generic(&P.scal->pivots), npiv);
}

// ------------------------------------------------------------------ 3. M = L^{-1}

// Pair (block1, block2) of a level with inverted diagonal blocks of size bs; output tile
// (ti, tj) of the bs x bs block below the diagonal.
struct InvTile {
  int64_t pair, ti, tj, tpb, r1, r2;
};

__device__ __forceinline__ bool inv_tile(const EigProb& P, int64_t bs, InvTile& t) {
  if (bs >= P.npad) return false;
  t.tpb = bs / NB;
  const int64_t tiles = (P.npad / (2 * bs)) * t.tpb * t.tpb;
  if (static_cast<int64_t>(blockIdx.x) >= tiles) return false;
  t.pair = blockIdx.x / (t.tpb * t.tpb);
  const int64_t rem = blockIdx.x - t.pair * t.tpb * t.tpb;
  t.ti = rem / t.tpb;
  t.tj = rem % t.tpb;
  t.r1 = t.pair * 2 * bs;
  t.r2 = t.r1 + bs;
  return true;
}

// T = C A^{-1}: C = M[block2, block1] (still the L tiles), A^{-1} = M[block1, block1] (lower
// triangular), T[ti, tj] = sum_{q >= tj} C[ti, q] A^{-1}[q, tj].  T is column-major with
// leading dimension npad / 2.
__global__ __launch_bounds__(256) void k_inv_stage1(const EigProb* __restrict__ probs, int64_t bs) {
  __shared__ __align__(16) double S0[NB][kLd];
  __shared__ __align__(16) double S1[NB][kLd];
  const EigProb& P = probs[blockIdx.y];
  InvTile t;
  if (!inv_tile(P, bs, t)) return;
  const int64_t npad = P.npad;
  gcdouble __restrict__ M = P.M;
  double acc[4][4] = {};
  double vc[16], va[16];
  tile_load<true>(vc, M + (t.r2 + t.ti * NB) + (t.r1 + t.tj * NB) * npad, npad, NB, NB);
  tile_load<false>(va, M + (t.r1 + t.tj * NB) + (t.r1 + t.tj * NB) * npad, npad, NB, NB);
  for (int64_t q = t.tj; q < t.tpb; ++q) {
    __syncthreads();
    tile_store<true>(S0, vc);   // S0[p][row] = C[row][p]
    tile_store<false>(S1, va);  // S1[p][col] = Ainv[p][col]
    __syncthreads();
    if (q + 1 < t.tpb) {
      tile_load<true>(vc, M + (t.r2 + t.ti * NB) + (t.r1 + (q + 1) * NB) * npad, npad, NB, NB);
      tile_load<false>(va, M + (t.r1 + (q + 1) * NB) + (t.r1 + t.tj * NB) * npad, npad, NB, NB);
    }
    mm64(acc, S0, S1);
  }
  const int64_t ldt = npad / 2;
  const int64_t base = (t.pair * bs + t.ti * NB) + (t.tj * NB) * ldt;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      P.T[base + acc_row(u, v) + static_cast<int64_t>(acc_col(u, v)) * ldt] = acc[u][v];
}

// M[block2, block1] = -B^{-1} T, B^{-1} = M[block2, block2] (lower triangular); the same
// tile goes transposed into Mt.
__global__ __launch_bounds__(256) void k_inv_stage2(const EigProb* __restrict__ probs, int64_t bs) {
  __shared__ __align__(16) double S0[NB][kLd];
  __shared__ __align__(16) double S1[NB][kLd];
  const EigProb& P = probs[blockIdx.y];
  InvTile t;
  if (!inv_tile(P, bs, t)) return;
  const int64_t npad = P.npad, ldt = npad / 2;
  gdouble __restrict__ M = P.M;
  gcdouble __restrict__ T = P.T;
  double acc[4][4] = {};
  double vb[16], vt[16];
  tile_load<true>(vb, M + (t.r2 + t.ti * NB) + (t.r2) * npad, npad, NB, NB);
  tile_load<false>(vt, T + (t.pair * bs) + (t.tj * NB) * ldt, ldt, NB, NB);
  for (int64_t q = 0; q <= t.ti; ++q) {
    __syncthreads();
    tile_store<true>(S0, vb);   // S0[p][row] = Binv[row][p]
    tile_store<false>(S1, vt);  // S1[p][col] = T[p][col]
    __syncthreads();
    if (q + 1 <= t.ti) {
      tile_load<true>(vb, M + (t.r2 + t.ti * NB) + (t.r2 + (q + 1) * NB) * npad, npad, NB, NB);
      tile_load<false>(vt, T + (t.pair * bs + (q + 1) * NB) + (t.tj * NB) * ldt, ldt, NB, NB);
    }
    mm64(acc, S0, S1);
  }
  const int64_t rb = t.r2 + t.ti * NB, cb = t.r1 + t.tj * NB;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t rr = rb + acc_row(u, v), cc = cb + acc_col(u, v);
      M[rr + cc * npad] = -acc[u][v];
      P.Mt[cc + rr * npad] = -acc[u][v];
    }
}

// ------------------------------------------------------------------ 4-5. subspace iteration
//
// Inverse subspace iteration and Rayleigh-Ritz run in one launch (k_subspace), one
// workgroup per problem: a problem's iteration needs no other workgroup, so problems of a
// batch, and calls on other streams, run side by side with no waiting between workgroups.
// Thread t owns rows t and n - 1 - t of the n x b iterate, and t + T and n - 1 - t - T when
// n > 2T (T threads; NR = 2 or 4 rows per thread, one kernel instance each): a short and a
// long row of each triangular product per pair, which balances the wavefronts' work.
// Products stream the operator's column segments of each wavefront's rows and the matching
// rows of the right-hand block straight into that wavefront's own LDS buffers.  One
// iteration:
//   Z = M X, Y = M^T Z                       (M = L^{-1}: Y = (N + mu I)^{-1} X)
//   Y <- Y R^{-1} two or three times, R^T R the Cholesky factorisation of the b x b Gram
//   Y^T Y, the first with a shift: shifted Cholesky QR, orthonormal to rounding even when Y
//   is nearly rank deficient (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, SIAM J. Sci.
//   Comput. 42, 2020);
// and at check iterations (2, 3, 4, 5, 6, 7, 8, 10, 12, 15, ... : about 25% apart) the
// Rayleigh-Ritz step: NX = N X, H = X^T N X = Q Theta Q^T (Jacobi), X <- X Q with Theta
// ascending, and the residuals ||N x_k - theta_k x_k|| of the r wanted pairs.  The
// iteration stops when max_k residual <= kSubTol lam_max, when the residual, already below
// kSubFloor lam_max, stops halving between checks (the rounding level of the factor), or
// after kEigMaxIters steps.  Every sum runs in a fixed order, so results do not depend on
// timing.

constexpr int kSubThreads = 512;
constexpr int kSubWaves = kSubThreads / 64;
constexpr int kStageMax = 1184;                   // doubles of one staging buffer (see below)
constexpr int kSubStride = kEigMaxB + 1;          // LDS row stride of b-wide rows
constexpr int kGramRows = 64;                     // rows per block of the Gram reductions
constexpr double kSubTol = 1e-10;                 // converged: residual / lam_max
constexpr double kSubFloor = 1e-8;                // below this a stalled residual stops
constexpr int kSubMinB = 2, kSubMaxB = RSM_MAX_R + kEigPad;  // subspace widths built
constexpr double kEps = 2.220446049250313e-16;
constexpr double kUnit = 1.1102230246251565e-16;  // unit roundoff of FP64

struct SubShared {
  union {
    double stage[kSubWaves][2][kStageMax];    // each wavefront's two staging buffers
    struct {
      double pb[kGramRows][kSubStride];       // a block of rows of P and C (Gram)
      double cb[kGramRows][kSubStride];
      double part[kSubThreads];               // slice partials of the Gram entries
    } g;
  };
  double wred[kSubWaves][RSM_MAX_R];          // per-wavefront residual sums
  double B[kEigMaxB][kSubStride];             // b x b Gram / Rayleigh-Ritz matrix
  double Q[kEigMaxB][kSubStride];             // rotations of the Jacobi method
  double cs[kEigMaxB + 1], sn[kEigMaxB + 1], th[kEigMaxB + 1], rdiag[kEigMaxB + 1];
  int partner[kEigMaxB + 1], order[kEigMaxB];
};

// Problems of one k_subspace launch (they share the subspace width b and the rows per
// thread).
struct SubList {
  int32_t count;
  int32_t idx[kLaunchMax];
};

// The rows of this thread (NR of them; on[q] false where the row does not exist).
template <int NR>
struct SubRows {
  int row[NR];
  bool on[NR];
};

template <int NR>
__device__ __forceinline__ SubRows<NR> sub_rows(int n) {
  SubRows<NR> R;
  const int t = threadIdx.x, h = (n + 1) / 2;
#pragma unroll
  for (int p = 0; p < NR / 2; ++p) {
    const int tp = t + p * kSubThreads;
    const bool own = tp < h;
    R.row[2 * p] = own ? tp : 0;
    R.row[2 * p + 1] = own ? n - 1 - tp : 0;
    R.on[2 * p] = own;
    R.on[2 * p + 1] = own && n - 1 - tp != tp;
  }
  return R;
}

// n made opaque to the optimiser at each use, so that the row addresses are formed where
// they are used rather than kept live in registers across the whole iteration loop.
__device__ __forceinline__ int opaque(int n) {
  int u = __builtin_amdgcn_readfirstlane(n);
  asm volatile("" : "+s"(u));
  return u;
}

// Staging of the products: NR row segments of 64 rows per wavefront, K columns of the
// operator per stage (8 with two segments, 4 with four), and the stage's K rows of the
// right-hand block (as [column][stage row]); the doubles of one buffer.
template <int NR>
constexpr int stage_cols() { return NR == 2 ? 8 : 4; }
template <int B, int NR>
constexpr int stage_xs() { return (stage_cols<NR>() * B + 31) / 32 * 32; }
template <int B, int NR>
constexpr int stage_doubles() { return NR * stage_cols<NR>() * 64 + stage_xs<B, NR>(); }
static_assert(stage_doubles<kSubMaxB, 2>() <= kStageMax &&
              stage_doubles<kSubMaxB, 4>() <= kStageMax, "staging buffer");

__device__ __forceinline__ void lds_dma_dword(const void* src, double* dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 4, 0, 0);
}

// The thread's rows of A In (A n x n column-major with leading dimension lda, In n x B
// column-major with leading dimension n) into y.  SHAPE 1: A is lower triangular (columns
// i <= row); 2: upper (i >= row); 0: full.  Each wavefront streams the operator's column
// segments of its own rows (64 consecutive rows per segment; the second segment runs down
// from n - 1 - 64 w, so lane l reads it backwards) and the stage's rows of In straight into
// its own two LDS buffers (global_load_lds_dword: lane k writes 4 bytes at base + 4 k), the
// next stage in flight while the current one is summed; no wavefront waits for another.
// A stage no row of a segment needs (the triangle's empty part) is neither loaded nor
// summed.
template <int B, int SHAPE, int NR>
__device__ void rows_times(gcdouble __restrict__ A, uint32_t lda, gcdouble In, int n,
                           const SubRows<NR>& R, SubShared& S, double (&y)[NR][B]) {
  constexpr int K = stage_cols<NR>();
  constexpr int XS = stage_xs<B, NR>();
  constexpr int XI = XS / 32;  // instructions for the right-hand rows
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int c = 0; c < B; ++c) y[q][c] = 0.0;
  if (!__any(R.on[0])) return;
  int sb[NR];  // first row of each segment
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int t0 = 64 * w + (q >> 1) * kSubThreads;
    sb[q] = (q & 1) ? n - t0 - 64 : t0;
  }
  double* const buf0 = &S.stage[w][0][0];
  double* const buf1 = &S.stage[w][1][0];
  auto seg_needed = [&](int q, int i_lo, int i_hi) {
    const int rq = R.row[q];
    const bool nd = R.on[q] && (SHAPE == 1 ? i_lo <= rq : (SHAPE == 2 ? i_hi >= rq : true));
    return __any(nd) != 0;
  };
  auto issue = [&](int i0, double* dst) {
    const int i_hi = (i0 + K - 1 < n - 1) ? (i0 + K - 1) : (n - 1);
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      if (!seg_needed(q, i0, i_hi)) continue;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = (i0 + k < n) ? i0 + k : n - 1;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          int row = sb[q] + 32 * hh + (lane >> 1);
          row = row < 0 ? 0 : (row > n - 1 ? n - 1 : row);
          const uint64_t off =
              (static_cast<uint64_t>(static_cast<uint32_t>(row) + static_cast<uint32_t>(i) * lda) << 3) +
              4 * (lane & 1);
          lds_dma_dword((const void*)(reinterpret_cast<RSM_GLOBAL const char*>(A) + off),
                        dst + (q * K + k) * 64 + 32 * hh);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < XI; ++u) {
      const int d = 64 * u + lane, dd = d >> 1;
      const int c = dd / K, kk = dd % K;
      const int i = (i0 + kk < n) ? i0 + kk : n - 1;
      const int cc = c < B ? c : 0;
      const uint64_t off =
          (static_cast<uint64_t>(static_cast<uint32_t>(i) +
                                 static_cast<uint32_t>(cc) * static_cast<uint32_t>(n)) << 3) +
          4 * (d & 1);
      lds_dma_dword((const void*)(reinterpret_cast<RSM_GLOBAL const char*>(In) + off),
                    dst + NR * K * 64 + 32 * u);
    }
  };
  const int stages = (n + K - 1) / K;
  issue(0, buf0);
  for (int st = 0; st < stages; ++st) {
    __builtin_amdgcn_s_waitcnt(0);  // stage st has landed; the other buffer's reads are done
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
    if (st + 1 < stages) issue((st + 1) * K, (st & 1) ? buf0 : buf1);
    const double* cur = (st & 1) ? buf1 : buf0;
    const double* xs = cur + NR * K * 64;
    const int i0 = st * K;
    const int kn = (n - i0) < K ? (n - i0) : K;
#pragma unroll 1
    for (int k = 0; k < kn; ++k) {
      const int i = i0 + k;
      double xv[B];
#pragma unroll
      for (int c = 0; c < B; ++c) xv[c] = xs[c * K + k];
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const int rq = R.row[q];
        const bool nd = R.on[q] && (SHAPE == 1 ? i <= rq : (SHAPE == 2 ? i >= rq : true));
        if (nd) {
          const double a = cur[(q * K + k) * 64 + ((q & 1) ? 63 - lane : lane)];
#pragma unroll
          for (int c = 0; c < B; ++c) y[q][c] = fma(a, xv[c], y[q][c]);
        }
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
}

// The thread's rows into the n x B column-major array D.
template <int B, int NR>
__device__ __forceinline__ void put_rows(gdouble D, int n, const SubRows<NR>& R,
                                         const double (&y)[NR][B]) {
  const int nn = opaque(n);
#pragma unroll
  for (int q = 0; q < NR; ++q)
    if (R.on[q])
#pragma unroll
      for (int c = 0; c < B; ++c) D[R.row[q] + static_cast<int64_t>(c) * nn] = y[q][c];
}

// The thread's rows of the n x B column-major array D.
template <int B, int NR>
__device__ __forceinline__ void get_rows(gcdouble D, int n, const SubRows<NR>& R,
                                         double (&y)[NR][B]) {
  const int nn = opaque(n);
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int c = 0; c < B; ++c) y[q][c] = R.on[q] ? D[R.row[q] + static_cast<int64_t>(c) * nn] : 0.0;
}

// S.B = P^T C for the n x B column-major arrays P and C written by this workgroup (lower
// triangle formed, upper mirrored; with C != P the two products X^T (N X) and its transpose
// are averaged, so the result is exactly symmetric).  Blocks of kGramRows rows of P and C
// are staged in LDS (coalesced loads down the columns); the NP = B (B + 1) / 2 entries get
// SL slots (a power of two), and entry e (packed index) is summed by the threads
// t = e + SL s over the block's rows j = s mod NS (NS = threads / SL), each slice keeping
// one running sum over the blocks; the slices are added in order at the end.
template <int B>
__device__ __forceinline__ void gram_of(gcdouble P, gcdouble C, int n, SubShared& S) {
  constexpr int NP = B * (B + 1) / 2;
  constexpr int SL = NP <= 64 ? 64 : (NP <= 128 ? 128 : 256);
  constexpr int NS = kSubThreads / SL;
  static_assert(NP <= SL && SL <= kSubThreads, "Gram entries exceed their slots");
  const int t = threadIdx.x, e = t % SL, s = t / SL;
  int c1 = 0, c2 = 0;
  if (e < NP) {
    c1 = static_cast<int>((sqrtf(8.0f * static_cast<float>(e) + 1.0f) - 1.0f) * 0.5f);
    while (c1 * (c1 + 1) / 2 > e) --c1;
    while ((c1 + 1) * (c1 + 2) / 2 <= e) ++c1;
    c2 = e - c1 * (c1 + 1) / 2;
  }
  const bool sym = P == C;
  double acc = 0.0;
  for (int j0 = 0; j0 < n; j0 += kGramRows) {
    __syncthreads();  // the previous block (or other use of this LDS) is done
    for (int x = t; x < kGramRows * B; x += kSubThreads) {
      const int jr = x % kGramRows, c = x / kGramRows;
      const int j = j0 + jr;
      S.g.pb[jr][c] = j < n ? P[j + static_cast<int64_t>(c) * n] : 0.0;
      if (!sym) S.g.cb[jr][c] = j < n ? C[j + static_cast<int64_t>(c) * n] : 0.0;
    }
    __syncthreads();
    if (e < NP) {
      const double (*cb)[kSubStride] = sym ? S.g.pb : S.g.cb;
#pragma unroll 4
      for (int jr = s; jr < kGramRows; jr += NS) {
        acc = fma(S.g.pb[jr][c1], cb[jr][c2], acc);
        if (!sym) acc = fma(S.g.pb[jr][c2], cb[jr][c1], acc);
      }
    }
  }
  __syncthreads();
  S.g.part[t] = acc;
  __syncthreads();
  if (t < NP) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < NS; ++q) v += S.g.part[q * SL + t];
    if (!sym) v *= 0.5;
    int a1 = static_cast<int>((sqrtf(8.0f * static_cast<float>(t) + 1.0f) - 1.0f) * 0.5f);
    while (a1 * (a1 + 1) / 2 > t) --a1;
    while ((a1 + 1) * (a1 + 2) / 2 <= t) ++a1;
    const int a2 = t - a1 * (a1 + 1) / 2;
    S.B[a1][a2] = v;
    S.B[a2][a1] = v;
  }
  __syncthreads();
}

// Wavefront 0: Bm = L L^T in place in LDS (lower triangle; the upper one is left as it
// was), rdiag[k] = 1 / l_kk.  Step k: the pivot, column k scaled by the lanes below it, then
// the trailing lower triangle updated with each lane holding up to four fixed entries (i, j),
// i >= j.  A pivot that is not positive (a numerically rank-deficient Gram despite the
// shift) is replaced by the smallest normal number, which keeps the solve finite.
template <int B>
__device__ void chol_wave(double (*Bm)[kSubStride], double* rdiag) {
  constexpr int NL = B * (B + 1) / 2;
  constexpr int KE = (NL + 63) / 64;
  const int lane = threadIdx.x;
  int ei[KE], ej[KE];
#pragma unroll
  for (int u = 0; u < KE; ++u) {
    const int e = lane + 64 * u;
    int i = static_cast<int>((sqrtf(8.0f * static_cast<float>(e) + 1.0f) - 1.0f) * 0.5f);
    while (i * (i + 1) / 2 > e) --i;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    ei[u] = e < NL ? i : -1;
    ej[u] = e < NL ? e - i * (i + 1) / 2 : -1;
  }
  for (int k = 0; k < B; ++k) {
    double d = Bm[k][k];
    if (!(d > 0.0) || !isfinite(d)) d = 2.2250738585072014e-308;
    const double piv = sqrt(d), inv = 1.0 / piv;
    wave_lds_fence();
    if (lane == k) {
      Bm[k][k] = piv;
      rdiag[k] = inv;
    }
    if (lane > k && lane < B) Bm[lane][k] *= inv;
    wave_lds_fence();
#pragma unroll
    for (int u = 0; u < KE; ++u)
      if (ej[u] > k) Bm[ei[u]][ej[u]] = fma(-Bm[ei[u]][k], Bm[ej[u]][k], Bm[ei[u]][ej[u]]);
    wave_lds_fence();
  }
}

// x L^T = y (R = L^T) for one row held in registers: forward substitution with rdiag[c]
// = 1 / l_cc.
template <int B>
__device__ __forceinline__ void row_solve(double (&y)[B], const double (*L)[kSubStride],
                                          const double* rdiag) {
#pragma unroll
  for (int c = 0; c < B; ++c) {
    double s = y[c];
#pragma unroll
    for (int k = 0; k < c; ++k) s = fma(-y[k], L[c][k], s);
    y[c] = s * rdiag[c];
    __builtin_amdgcn_sched_barrier(0);  // keeps the loads of L in step (register pressure)
  }
}

// Cyclic Jacobi with parallel (round-robin) ordering of the symmetric B x B matrix H in LDS
// by wavefront 0: H_in = Q H_out Q^T with H_out diagonal to rounding.  Round k of a sweep
// pairs the bb = B + (B odd) players by the circle method: pair 0 is (k, bb - 1), pair m > 0 is
// (k + m, k - m) mod (bb - 1), so index i's partner is (2k - i) mod (bb - 1) (bb - 1 for k;
// player B, when B is odd, sits the round out).  Lane m finds pair m's rotation: for
// p < q, with c, s from the usual tau formula, column p becomes c col_p - s col_q and column
// q becomes s col_p + c col_q (rows likewise); index p stores (c, s) and q (c, -s), making
// both "cs[j] col_j - sn[j] col_partner(j)".  An element is rotated away only while it is
// above both eps sqrt(|a_pp a_qq|) and 4 eps ||H||_F.  New entries are formed for the lower
// triangle and mirrored, so H stays exactly symmetric.
template <int B>
__device__ void jacobi_wave(double (*H)[kSubStride], double (*Q)[kSubStride], double* cs,
                            double* sn, int* partner) {
  constexpr int bb = B + (B & 1);
  constexpr int nr = bb - 1;
  constexpr int nl = B * (B + 1) / 2;
  constexpr int kH = (nl + 63) / 64, kQ = (B * B + 63) / 64;
  const int lane = threadIdx.x;
  for (int e = lane; e < B * B; e += 64) Q[e / B][e % B] = (e / B == e % B) ? 1.0 : 0.0;
  double f2 = 0.0;
  for (int e = lane; e < B * B; e += 64) f2 = fma(H[e / B][e % B], H[e / B][e % B], f2);
  f2 = wave_sum(f2);
  const double floor_abs = 4.0 * kEps * sqrt(f2);
  // the lane's lower-triangle elements (i >= j), packed index e = i (i + 1) / 2 + j
  int li[kH], lj[kH];
#pragma unroll
  for (int k = 0; k < kH; ++k) {
    const int e = lane + 64 * k;
    int i = static_cast<int>((sqrtf(8.0f * static_cast<float>(e) + 1.0f) - 1.0f) * 0.5f);
    while (i * (i + 1) / 2 > e) --i;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    li[k] = i;
    lj[k] = e - i * (i + 1) / 2;
  }
  wave_lds_fence();
  for (int sweep = 0; sweep < 40; ++sweep) {
    int rotated = 0;
    for (int k = 0; k < nr; ++k) {
      double c = 1.0, s = 0.0;
      if (lane < bb / 2) {
        int p = lane == 0 ? k : (k + lane) % nr;
        int q = lane == 0 ? nr : (k - lane + nr) % nr;
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        if (q < B) {
          const double apq = H[p][q], app = H[p][p], aqq = H[q][q];
          if (apq * apq > kEps * kEps * fabs(app * aqq) && fabs(apq) > floor_abs) {
            const double tau = (aqq - app) / (2.0 * apq);
            double tt;
            if (fabs(tau) > 1e150) {
              tt = 0.5 / tau;
            } else {
              tt = 1.0 / (fabs(tau) + sqrt(fma(tau, tau, 1.0)));
              if (tau < 0.0) tt = -tt;
            }
            c = 1.0 / sqrt(fma(tt, tt, 1.0));
            s = tt * c;
            rotated = 1;
          }
        }
      }
      // index `lane`'s partner and rotation
      int part = 0, m = 0;
      if (lane == nr || lane == k) {
        part = lane == nr ? k : nr;
      } else {
        part = (2 * k - lane + 2 * nr) % nr;
        const int d = (lane - k + nr) % nr;
        m = d <= (nr - 1) / 2 ? d : nr - d;
      }
      const double cm = __shfl(c, m, 64), sm = __shfl(s, m, 64);
      if (lane < B) {
        const bool on = part < B;
        partner[lane] = on ? part : lane;
        cs[lane] = on ? cm : 1.0;
        sn[lane] = on ? (lane < part ? sm : -sm) : 0.0;
      }
      wave_lds_fence();
      double hn[kH], qn[kQ];
#pragma unroll
      for (int u = 0; u < kH; ++u) {
        hn[u] = 0.0;
        if (lane + 64 * u < nl) {
          const int i = li[u], j = lj[u];
          const int ii = partner[i], jj = partner[j];
          const double ci = cs[i], si = sn[i], cj = cs[j], sj = sn[j];
          hn[u] = ci * (cj * H[i][j] - sj * H[i][jj]) - si * (cj * H[ii][j] - sj * H[ii][jj]);
        }
      }
#pragma unroll
      for (int u = 0; u < kQ; ++u) {
        qn[u] = 0.0;
        const int e = lane + 64 * u;
        if (e < B * B) {
          const int i = e / B, j = e % B;
          qn[u] = cs[j] * Q[i][j] - sn[j] * Q[i][partner[j]];
        }
      }
      wave_lds_fence();
#pragma unroll
      for (int u = 0; u < kH; ++u)
        if (lane + 64 * u < nl) {
          H[li[u]][lj[u]] = hn[u];
          H[lj[u]][li[u]] = hn[u];
        }
#pragma unroll
      for (int u = 0; u < kQ; ++u) {
        const int e = lane + 64 * u;
        if (e < B * B) Q[e / B][e % B] = qn[u];
      }
      wave_lds_fence();
    }
    if (!__any(rotated)) break;
  }
}

template <int B, int NR>
__device__ __forceinline__ void subspace_one(const EigProb& P, SubShared& S) {
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int n = static_cast<int>(P.n), r = P.r;
  const SubRows<NR> R = sub_rows<NR>(n);
  const uint32_t ld = static_cast<uint32_t>(P.npad);
  const double lam_max = P.scal->lam_max;
  double y[NR][B];
  int it = 0, next_check = 2;
  double rel = 0.0, prev_rel = 0.0;
  bool first_check = true;
  while (true) {
    ++it;
    // Z = M X, then Y = M^T Z
    rows_times<B, 1, NR>(P.M, ld, P.X, n, R, S, y);
    put_rows<B, NR>(P.Z, n, R, y);
    __syncthreads();
    rows_times<B, 2, NR>(P.Mt, ld, P.Z, n, R, S, y);
    // shifted Cholesky QR: a second pass always, a third when the first factor's diagonal
    // spans more than 1e4 (cond(Y) beyond about 1e4 leaves the second pass's Gram
    // ill conditioned)
    int passes = 3;
    put_rows<B, NR>(P.X, n, R, y);
    for (int pass = 0; pass < passes; ++pass) {
      gram_of<B>(P.X, P.X, n, S);
      if (pass == 0 && t == 0) {
        double tr = 0.0;
        for (int c = 0; c < B; ++c) tr += S.B[c][c];
        const double shift = 11.0 * (static_cast<double>(n) * B + B * (B + 1.0)) * kUnit * tr;
        for (int c = 0; c < B; ++c) S.B[c][c] += shift;
      }
      __syncthreads();
      if (t < 64) chol_wave<B>(S.B, S.rdiag);
      __syncthreads();
      if (pass == 0) {
        double dmin = S.B[0][0], dmax = S.B[0][0];
        for (int c = 1; c < B; ++c) {
          dmin = fmin(dmin, S.B[c][c]);
          dmax = fmax(dmax, S.B[c][c]);
        }
        if (dmin >= 1e-4 * dmax) passes = 2;
      }
      // the thread's rows, re-read (they are not held across the reduction and the factor)
      get_rows<B, NR>(P.X, n, R, y);
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (R.on[q]) row_solve<B>(y[q], S.B, S.rdiag);
      put_rows<B, NR>(P.X, n, R, y);
    }
    __syncthreads();
    if (it < next_check && it < kEigMaxIters) continue;
    // Rayleigh-Ritz: N X (into Z), H = X^T N X
    rows_times<B, 0, NR>(P.Nsym, static_cast<uint32_t>(n), P.X, n, R, S, y);
    put_rows<B, NR>(P.Z, n, R, y);
    gram_of<B>(P.X, P.Z, n, S);
    if (t < 64) jacobi_wave<B>(S.B, S.Q, S.cs, S.sn, S.partner);
    __syncthreads();
    if (t < B) {
      const double dk = S.B[t][t];
      int rk = 0;
      for (int j = 0; j < B; ++j) {
        const double dj = S.B[j][j];
        rk += (dj < dk) || (dj == dk && j < t);
      }
      S.order[rk] = t;
      S.th[rk] = dk;
    }
    __syncthreads();
    // Ritz vectors (ascending) into the thread's rows of X, and per wavefront the squared
    // residuals ||N x_k - theta_k x_k||^2 of the r wanted pairs over its rows
    get_rows<B, NR>(P.X, n, R, y);
    __syncthreads();  // every row read before any is overwritten
#pragma unroll 1
    for (int k = 0; k < B; ++k) {
      const int ok = S.order[k];
      const int nn = opaque(n);
      double d2 = 0.0;
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        if (R.on[q]) {
          const int rq = R.row[q];
          double xv = 0.0, zv = 0.0;
#pragma unroll
          for (int c = 0; c < B; ++c) {
            const double qc = S.Q[c][ok];
            xv = fma(y[q][c], qc, xv);
            zv = fma(P.Z[rq + static_cast<int64_t>(c) * nn], qc, zv);
          }
          P.X[rq + static_cast<int64_t>(k) * nn] = xv;
          const double d = zv - S.th[k] * xv;
          d2 = fma(d, d, d2);
        }
      }
      if (k < r) {
        const double v = wave_sum(d2);
        if (lane == 0) S.wred[wid][k] = v;
      }
    }
    __syncthreads();
    if (t < r) {
      double s2 = 0.0;
      for (int w = 0; w < kSubThreads / 64; ++w) s2 += S.wred[w][t];
      S.cs[t] = sqrt(s2);
    }
    __syncthreads();
    double rmax = 0.0;
    for (int k = 0; k < r; ++k) rmax = fmax(rmax, S.cs[k]);
    rel = lam_max > 0.0 ? rmax / lam_max : rmax;
    __syncthreads();
    const bool stalled = !first_check && rel <= kSubFloor && rel > 0.5 * prev_rel;
    if (rel <= kSubTol || stalled || it >= kEigMaxIters) break;
    first_check = false;
    prev_rel = rel;
    next_check = it + 1 + it / 4;
  }
  // V-hat = the r leading (smallest) Ritz vectors, from the thread's rows of X
#pragma unroll
  for (int q = 0; q < NR; ++q)
    if (R.on[q])
      for (int c = 0; c < r; ++c)
        P.V[R.row[q] + static_cast<int64_t>(c) * n] = P.X[R.row[q] + static_cast<int64_t>(c) * n];
  if (t == 0) {
    RSM_GLOBAL rsm_info* info = P.info;
    uint32_t warn = 0;
    info->residual = rel;
    for (int k = 0; k <= r && k < B; ++k) info->lambda[k] = S.th[k];
    if (B > r && !(S.th[r] > 1e-12 * lam_max)) warn |= RSM_W_RANK_DEFICIENT;
    if (rel > 1e-6) warn |= RSM_W_NOT_CONVERGED;
    if (info->uncovered > 0) warn |= RSM_W_RANK_DEFICIENT;
    if (P.scal->pivots > 0) warn |= RSM_W_PIVOT;
    if (P.check_accepted && info->accepted == 0) warn |= RSM_W_NO_CONSTRAINTS;
    atomicOr(generic(&info->warn), warn);
    info->eig_iterations = it;
  }
}

// The iteration of problem P with its subspace width as a compile-time constant.
template <int B, int NR>
__device__ __forceinline__ void subspace_dispatch(int b, const EigProb& P, SubShared& S) {
  if constexpr (B <= kSubMaxB) {
    if (b == B)
      subspace_one<B, NR>(P, S);
    else
      subspace_dispatch<B + 1, NR>(b, P, S);
  }
}

// One workgroup per problem of `list`, whatever their subspace widths.
template <int NR>
__global__ __launch_bounds__(kSubThreads) void k_subspace(const EigProb* __restrict__ probs,
                                                          SubList list) {
  __shared__ SubShared S;
  const EigProb& P = probs[list.idx[blockIdx.x]];
  subspace_dispatch<kSubMinB, NR>(P.b, P, S);
}

// Group form of the same iteration, for launches of at most kGroupMaxProblems problems: one
// group of G = ceil(n_max / 16) workgroups takes the problems in turn, workgroup `rank`
// owning rows 16 rank .. 16 rank + 15 of the iterate, so a single large problem is spread
// over up to 128 CUs.  The workgroups meet at group barriers (device-scope release fence,
// an arrival count, device-scope acquire) and take their rank from a ticket counter in the
// order they start, so the group only waits for workgroups that have started.  A wait can
// only fail to end if the waiting workgroups of this and other concurrent group launches
// fill every workgroup slot of the device (two per CU): at G <= 64 (n <= 1024) that takes
// more than seven such launches at once, at n = 2048 more than three; the wait is bounded
// (about 4 s of wall clock), after which the launch stops and flags RSM_W_NOT_CONVERGED.
// Partial sums are formed per workgroup and summed in rank order, so results do not depend
// on timing.
constexpr int kGrpChunk = 128;                    // values of i staged per chunk
constexpr int kGrpThreads = 256;
constexpr long long kSubWaitTicks = 400000000LL;  // bound of one barrier wait (wall clock)
constexpr int kGroupMaxProblems = 4;              // launches up to this size use the group form

struct GrpShared {
  double stage[kGrpChunk][kSubStride];  // staged rows of the right-hand block
  double As[kGrpChunk][kSubRows + 1];   // staged slab of the operator (transposed)
  double red[4][kSubRows][kSubStride];  // per-wavefront partial sums
  double Yr[kSubRows][kSubStride];      // this workgroup's rows of the iterate
  double NYr[kSubRows][kSubStride];     // its rows of N X
  double B[kEigMaxB][kSubStride];       // b x b Gram / Rayleigh-Ritz matrix
  double Q[kEigMaxB][kSubStride];       // rotations of the Jacobi method
  double cs[kEigMaxB + 1], sn[kEigMaxB + 1], th[kEigMaxB + 1], rdiag[kEigMaxB + 1];
  int partner[kEigMaxB + 1], order[kEigMaxB];
  int stop;                             // a barrier wait failed: stop
  int group, rank;
};


// The group barrier.  `arrivals` counts this workgroup's barriers times G (every workgroup
// of a group calls it equally often), so the k-th barrier waits for k G arrivals.
__device__ void group_barrier(RSM_GLOBAL uint32_t* ctr, RSM_GLOBAL uint32_t* stalled,
                              uint32_t& arrivals, uint32_t G, GrpShared& S) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  arrivals += G;
  if (threadIdx.x == 0 && !S.stop) {
    uint32_t* c = (uint32_t*)ctr;
    uint32_t* st = (uint32_t*)stalled;
    __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const long long t0 = wall_clock64();
    while (__hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < arrivals) {
      if (__hip_atomic_load(st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          wall_clock64() - t0 > kSubWaitTicks) {
        __hip_atomic_store(st, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        S.stop = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// dst[jr][c] = sum_{lo <= i < hi} A[row_jr + i lda] In[i + c n] for c < B, row_jr = j0 + jr
// (rows at or past n give zero rows).  Per chunk of kGrpChunk values of i, the operator's
// 16 x kGrpChunk slab and the chunk's rows of In are staged in LDS (all loads of a chunk in
// flight together); thread (jr, kp) = (t % 16, t / 16) sums i = kp mod 16 of the
// chunk for all B columns, and the 16 partial sums of a row are added by two cross-lane
// steps and then over the four wavefronts in order.  All threads.
template <int B>
__device__ void row_product(gcdouble __restrict__ A, uint32_t lda, gcdouble In, int n, int j0,
                            int lo, int hi, GrpShared& S, double (*dst)[kSubStride]) {
  constexpr int kIn = (kGrpChunk * B + kGrpThreads - 1) / kGrpThreads;  // In values per thread
  constexpr int kA = kGrpChunk * kSubRows / kGrpThreads;                 // operator values
  const int t = threadIdx.x, jr = t & 15, kp = t >> 4;
  const uint32_t row = static_cast<uint32_t>(j0 + jr < n ? j0 + jr : n - 1);
  double acc[B];
#pragma unroll
  for (int c = 0; c < B; ++c) acc[c] = 0.0;
  for (int i0 = lo; i0 < hi; i0 += kGrpChunk) {
    const int cnt = (hi - i0) < kGrpChunk ? (hi - i0) : kGrpChunk;
    double xv[kIn], av[kA];
#pragma unroll
    for (int u = 0; u < kIn; ++u) {
      const int e = t + u * kGrpThreads, il = e % kGrpChunk, c = e / kGrpChunk;
      const bool ok = c < B && il < cnt;
      xv[u] = gld(In, static_cast<uint32_t>(i0 + (ok ? il : 0)) +
                          static_cast<uint32_t>(ok ? c : 0) * static_cast<uint32_t>(n));
      if (!ok) xv[u] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < kA; ++u) {
      const int il = kp + 16 * u;
      av[u] = gld(A, row + static_cast<uint32_t>(i0 + (il < cnt ? il : 0)) * lda);
      if (il >= cnt) av[u] = 0.0;
    }
    __syncthreads();  // the previous chunk has been used
#pragma unroll
    for (int u = 0; u < kIn; ++u) {
      const int e = t + u * kGrpThreads, il = e % kGrpChunk, c = e / kGrpChunk;
      if (c < B) S.stage[il][c] = xv[u];
    }
#pragma unroll
    for (int u = 0; u < kA; ++u) S.As[kp + 16 * u][jr] = av[u];
    __syncthreads();
#pragma unroll 2
    for (int il = kp; il < kGrpChunk; il += 16) {
      const double a = S.As[il][jr];
#pragma unroll
      for (int c = 0; c < B; ++c) acc[c] = fma(a, S.stage[il][c], acc[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < B; ++c) {
    acc[c] += __shfl_xor(acc[c], 16, 64);
    acc[c] += __shfl_xor(acc[c], 32, 64);
  }
  if ((t & 63) < 16)
#pragma unroll
    for (int c = 0; c < B; ++c) S.red[t >> 6][jr][c] = acc[c];
  __syncthreads();
  for (int e = t; e < kSubRows * B; e += kGrpThreads) {
    const int r2 = e % kSubRows, c = e / kSubRows;
    const double v = (S.red[0][r2][c] + S.red[1][r2][c]) + (S.red[2][r2][c] + S.red[3][r2][c]);
    dst[r2][c] = j0 + r2 < n ? v : 0.0;
  }
  __syncthreads();
}

// dst[c1 B + c2] = sum_jr X[jr][c1] C[jr][c2]: this workgroup's share of X^T C.
template <int B>
__device__ __forceinline__ void put_partial(const double (*X)[kSubStride],
                                            const double (*C)[kSubStride], gdouble dst) {
  for (int e = threadIdx.x; e < B * B; e += kGrpThreads) {
    const int c1 = e / B, c2 = e % B;
    double s = 0.0;
#pragma unroll
    for (int jr = 0; jr < kSubRows; ++jr) s = fma(X[jr][c1], C[jr][c2], s);
    dst[e] = s;
  }
}

// dst[e / B][e % B] = sum over the gp ranks of src[rank * stride + e], in rank order (rank k
// into running sum k mod 4, the four added pairwise at the end; 16 loads in flight).
template <int B>
__device__ __forceinline__ void sum_partials(gcdouble src, int64_t stride, int gp,
                                             double (*dst)[kSubStride]) {
  for (int e = threadIdx.x; e < B * B; e += kGrpThreads) {
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    int k = 0;
    for (; k + 16 <= gp; k += 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = src[(k + u) * stride + e];
#pragma unroll
      for (int u = 0; u < 16; ++u) s4[u & 3] += v[u];
    }
    for (; k < gp; ++k) s4[k & 3] += src[k * stride + e];
    dst[e / B][e % B] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  }
  __syncthreads();
}

// Rows of the iterate times R^{-1} (R = L^T): x L^T = y by forward substitution, one row per
// thread in registers.
template <int B>
__device__ __forceinline__ void rows_solve(double (*Yr)[kSubStride], const double (*L)[kSubStride],
                                           const double* rdiag) {
  const int t = threadIdx.x;
  if (t < kSubRows) {
    double x[B];
#pragma unroll
    for (int c = 0; c < B; ++c) x[c] = Yr[t][c];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      double s = x[c];
#pragma unroll
      for (int k = 0; k < c; ++k) s = fma(-x[k], L[c][k], s);
      x[c] = s * rdiag[c];
    }
#pragma unroll
    for (int c = 0; c < B; ++c) Yr[t][c] = x[c];
  }
  __syncthreads();
}

template <int B>
__global__ __launch_bounds__(kGrpThreads) void k_subspace_group(const EigProb* __restrict__ probs,
                                                          SubList list, int G, int ngroups) {
  __shared__ GrpShared S;
  const int t = threadIdx.x;
  const EigProb& P0 = probs[list.idx[0]];
  if (t == 0) {
    const uint32_t tk = atomicAdd(generic(&P0.scal->ticket), 1u);
    S.group = static_cast<int>(tk / static_cast<uint32_t>(G));
    S.rank = static_cast<int>(tk % static_cast<uint32_t>(G));
    S.stop = 0;
  }
  __syncthreads();
  const int group = S.group, rank = S.rank;
  if (group >= ngroups) return;  // not reached: the grid is G x ngroups
  RSM_GLOBAL uint32_t* ctr = &probs[list.idx[group]].scal->bar;
  RSM_GLOBAL uint32_t* stalled = &P0.scal->stalled;
  uint32_t arrivals = 0;
  constexpr int64_t mstride = B * B;
  for (int li = group; li < list.count; li += ngroups) {
    const EigProb& P = probs[list.idx[li]];
    const int n = static_cast<int>(P.n), r = P.r;
    const int gp = static_cast<int>(ceil_div(P.n, kSubRows));
    const int j0 = rank * kSubRows;
    const bool act = rank < gp;
    const uint32_t ld = static_cast<uint32_t>(P.npad);
    const double lam_max = P.scal->lam_max;
    gdouble sp_mat = P.SP;                                            // [2][gp][B^2]
    gdouble sp_res = P.SP + 2 * static_cast<int64_t>(gp) * kEigMaxB * kEigMaxB;  // [gp][R]
    int it = 0, next_check = 2;
    double rel = 0.0, prev_rel = 0.0;
    bool first_check = true;
    while (!S.stop) {
      ++it;
      // Z = M X (rows j0.., i <= j0 + 15), then Y = M^T Z (i >= j0)
      if (act) {
        row_product<B>(P.M, ld, P.X, n, j0, 0, (j0 + kSubRows < n ? j0 + kSubRows : n), S, S.Yr);
        for (int e = t; e < kSubRows * B; e += kGrpThreads) {
          const int r2 = e % kSubRows, c = e / kSubRows;
          if (j0 + r2 < n) P.Z[(j0 + r2) + static_cast<int64_t>(c) * n] = S.Yr[r2][c];
        }
      }
      group_barrier(ctr, stalled, arrivals, G, S);
      if (S.stop) break;
      if (act) row_product<B>(P.Mt, ld, P.Z, n, j0, j0, n, S, S.Yr);
      // shifted Cholesky QR: a second pass always, a third when the first factor's diagonal
      // spans more than 1e4 (cond(Y) beyond about 1e4 leaves the second pass's Gram
      // ill conditioned); every workgroup takes the same decision from the same factor
      int passes = 3;
      for (int pass = 0; pass < passes && !S.stop; ++pass) {
        gdouble buf = sp_mat + (pass & 1) * gp * mstride;
        if (act) put_partial<B>(S.Yr, S.Yr, buf + rank * mstride);
        group_barrier(ctr, stalled, arrivals, G, S);
        if (S.stop) break;
        sum_partials<B>(buf, mstride, gp, S.B);
        if (pass == 0 && t == 0) {
          double tr = 0.0;
          for (int c = 0; c < B; ++c) tr += S.B[c][c];
          const double shift = 11.0 * (static_cast<double>(n) * B + B * (B + 1.0)) * kUnit * tr;
          for (int c = 0; c < B; ++c) S.B[c][c] += shift;
        }
        __syncthreads();
        if (t < 64) chol_wave<B>(S.B, S.rdiag);
        __syncthreads();
        if (pass == 0) {
          double dmin = S.B[0][0], dmax = S.B[0][0];
          for (int c = 1; c < B; ++c) {
            dmin = fmin(dmin, S.B[c][c]);
            dmax = fmax(dmax, S.B[c][c]);
          }
          if (dmin >= 1e-4 * dmax) passes = 2;
        }
        rows_solve<B>(S.Yr, S.B, S.rdiag);
      }
      if (S.stop) break;
      if (act)
        for (int e = t; e < kSubRows * B; e += kGrpThreads) {
          const int r2 = e % kSubRows, c = e / kSubRows;
          if (j0 + r2 < n) P.X[(j0 + r2) + static_cast<int64_t>(c) * n] = S.Yr[r2][c];
        }
      const bool check = it >= next_check || it >= kEigMaxIters;
      group_barrier(ctr, stalled, arrivals, G, S);
      if (S.stop || !check) continue;
      // Rayleigh-Ritz: NX = N X, H = X^T N X
      gdouble hbuf = sp_mat + gp * mstride;  // buffer 1 (last read in pass 1)
      if (act) {
        row_product<B>(P.Nsym, static_cast<uint32_t>(n), P.X, n, j0, 0, n, S, S.NYr);
        put_partial<B>(S.Yr, S.NYr, hbuf + rank * mstride);
      }
      group_barrier(ctr, stalled, arrivals, G, S);
      if (S.stop) break;
      sum_partials<B>(hbuf, mstride, gp, S.B);
      double hs[(B * B + kGrpThreads - 1) / kGrpThreads];
#pragma unroll
      for (int k = 0; k < (B * B + kGrpThreads - 1) / kGrpThreads; ++k) {
        const int e = t + k * kGrpThreads;
        hs[k] = e < B * B ? 0.5 * (S.B[e / B][e % B] + S.B[e % B][e / B]) : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < (B * B + kGrpThreads - 1) / kGrpThreads; ++k) {
        const int e = t + k * kGrpThreads;
        if (e < B * B) S.B[e / B][e % B] = hs[k];
      }
      __syncthreads();
      if (t < 64) jacobi_wave<B>(S.B, S.Q, S.cs, S.sn, S.partner);
      __syncthreads();
      if (t < B) {
        const double dk = S.B[t][t];
        int rk = 0;
        for (int j = 0; j < B; ++j) {
          const double dj = S.B[j][j];
          rk += (dj < dk) || (dj == dk && j < t);
        }
        S.order[rk] = t;
        S.th[rk] = dk;
      }
      __syncthreads();
      // Ritz vectors (ascending) in this workgroup's rows, and the residual terms; thread
      // (row, k) forms entry k of the row's rotated X and N X
      for (int e = t; e < kSubRows * B; e += kGrpThreads) {
        const int r2 = e % kSubRows, k = e / kSubRows;
        const int ok = S.order[k];
        double xv = 0.0, yv = 0.0;
#pragma unroll
        for (int c = 0; c < B; ++c) {
          xv = fma(S.Yr[r2][c], S.Q[c][ok], xv);
          yv = fma(S.NYr[r2][c], S.Q[c][ok], yv);
        }
        S.red[1][r2][k] = xv;
        S.red[2][r2][k] = yv;
        const double rk = yv - S.th[k] * xv;
        S.red[0][r2][k] = (j0 + r2 < n && k < r) ? rk * rk : 0.0;
      }
      __syncthreads();
      for (int e = t; e < kSubRows * B; e += kGrpThreads) {
        const int r2 = e % kSubRows, k = e / kSubRows;
        S.Yr[r2][k] = S.red[1][r2][k];
        S.NYr[r2][k] = S.red[2][r2][k];
      }
      __syncthreads();
      if (act) {
        if (t < r) {
          double s = 0.0;
#pragma unroll
          for (int jr = 0; jr < kSubRows; ++jr) s += S.red[0][jr][t];
          sp_res[rank * RSM_MAX_R + t] = s;
        }
        for (int e = t; e < kSubRows * B; e += kGrpThreads) {
          const int r2 = e % kSubRows, c = e / kSubRows;
          if (j0 + r2 < n) P.X[(j0 + r2) + static_cast<int64_t>(c) * n] = S.Yr[r2][c];
        }
      }
      group_barrier(ctr, stalled, arrivals, G, S);
      if (S.stop) break;
      if (t < r) {
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        for (int q = 0; q < gp; ++q) s4[q & 3] += sp_res[q * RSM_MAX_R + t];
        S.cs[t] = sqrt((s4[0] + s4[1]) + (s4[2] + s4[3]));
      }
      __syncthreads();
      double rmax = 0.0;
      for (int k = 0; k < r; ++k) rmax = fmax(rmax, S.cs[k]);
      rel = lam_max > 0.0 ? rmax / lam_max : rmax;
      __syncthreads();
      const bool stalled_near_floor = !first_check && rel <= kSubFloor && rel > 0.5 * prev_rel;
      if (rel <= kSubTol || stalled_near_floor || it >= kEigMaxIters) break;
      first_check = false;
      prev_rel = rel;
      next_check = it + 1 + it / 4;
    }
    // V-hat = the r leading (smallest) Ritz vectors
    if (act && !S.stop)
      for (int e = t; e < kSubRows * r; e += kGrpThreads) {
        const int r2 = e % kSubRows, c = e / kSubRows;
        if (j0 + r2 < n) P.V[(j0 + r2) + static_cast<int64_t>(c) * n] = S.Yr[r2][c];
      }
    if (rank == 0 && t == 0) {
      RSM_GLOBAL rsm_info* info = P.info;
      uint32_t warn = 0;
      if (S.stop) {
        warn |= RSM_W_NOT_CONVERGED;
        info->residual = __builtin_nan("");
      } else {
        info->residual = rel;
        for (int k = 0; k <= r && k < B; ++k) info->lambda[k] = S.th[k];
        if (B > r && !(S.th[r] > 1e-12 * lam_max)) warn |= RSM_W_RANK_DEFICIENT;
        if (rel > 1e-6) warn |= RSM_W_NOT_CONVERGED;
      }
      if (info->uncovered > 0) warn |= RSM_W_RANK_DEFICIENT;
      if (P.scal->pivots > 0) warn |= RSM_W_PIVOT;
      if (P.check_accepted && info->accepted == 0) warn |= RSM_W_NO_CONSTRAINTS;
      atomicOr(generic(&info->warn), warn);
      info->eig_iterations = it;
    }
    __syncthreads();
  }
}

template <int B>
void launch_group(int b, const EigProb* dev, const SubList& list, int64_t n_max, hipStream_t s) {
  if constexpr (B <= kSubMaxB) {
    if (b != B) {
      launch_group<B + 1>(b, dev, list, n_max, s);
      return;
    }
    const int G = static_cast<int>(ceil_div(n_max, kSubRows));
    k_subspace_group<B><<<static_cast<unsigned>(G), kGrpThreads, 0, s>>>(dev, list, G, 1);
  }
}

// Deterministic start block: entries uniform in [-1, 1) from Philox (key = seed, 1).
__global__ void k_start_vectors(const EigProb* __restrict__ probs) {
  const EigProb& P = probs[blockIdx.y];
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= P.n * P.b) return;
  uint64_t c[4] = {static_cast<uint64_t>(idx), 0x5eedull, 0ull, 0ull};
  Philox4x64::block(c, P.seed, 1ull);
  P.X[idx] = static_cast<double>(static_cast<int64_t>(c[0]) >> 11) * (1.0 / 4503599627370496.0);
}


}  // namespace

void launch_solve_v(const EigProb* host, int nprob, EigProb* dev, hipStream_t s) {
  if (nprob < 1) return;
  int64_t n_max = 0, npad_max = 0;
  int nb_max = 0;
  for (int k = 0; k < nprob; ++k) {
    n_max = host[k].n > n_max ? host[k].n : n_max;
    npad_max = host[k].npad > npad_max ? host[k].npad : npad_max;
    nb_max = host[k].nb > nb_max ? host[k].nb : nb_max;
  }
  for (int k0 = 0; k0 < nprob; k0 += kDescPerLaunch) {
    EigProbPack pack;
    pack.count = (nprob - k0) < kDescPerLaunch ? (nprob - k0) : kDescPerLaunch;
    for (int k = 0; k < pack.count; ++k) pack.p[k] = host[k0 + k];
    k_put_desc<<<1, kDescPerLaunch, 0, s>>>(pack, dev + k0);
  }
  const unsigned np = static_cast<unsigned>(nprob);
  const unsigned g_rows64 = static_cast<unsigned>(ceil_div(n_max, 64));
  k_eig_prep<<<dim3(static_cast<unsigned>(ceil_div(npad_max * npad_max, 256)), np), 256, 0, s>>>(dev);
  k_rowsum<<<dim3(g_rows64, 16, np), 256, 0, s>>>(dev);
  k_chol_first<<<dim3(1, np), 256, 0, s>>>(dev);
  for (int k = 0; k + 1 < nb_max; ++k) {
    const int rem = nb_max - k - 1;
    k_chol_step<<<dim3(static_cast<unsigned>(rem * (rem + 1) / 2), np), 256, 0, s>>>(dev, k);
  }
  for (int64_t bs = NB; bs < npad_max; bs *= 2) {
    const int64_t tpb = bs / NB;
    const unsigned grid = static_cast<unsigned>((npad_max / (2 * bs)) * tpb * tpb);
    k_inv_stage1<<<dim3(grid, np), 256, 0, s>>>(dev, bs);
    k_inv_stage2<<<dim3(grid, np), 256, 0, s>>>(dev, bs);
  }
  k_start_vectors<<<dim3(static_cast<unsigned>(ceil_div(n_max * kEigMaxB, 256)), np), 256, 0, s>>>(dev);
  // the subspace iteration.  When at most kGroupMaxProblems problems need it, those that are
  // not deterministic take the group form, one launch per subspace width (one group of
  // ceil(n / 16) <= 128 workgroups taking the launch's problems in turn).  Every other
  // problem - all of a larger call, and deterministic ones always, so that their result
  // never depends on the rest of a batch - takes one workgroup of its own: one launch per
  // rows per thread (and per kLaunchMax problems), all widths together.
  const bool small = nprob <= kGroupMaxProblems;
  auto grouped = [&](int k) { return small && !host[k].deterministic; };
  for (int b = kSubMinB; b <= kSubMaxB; ++b) {
    SubList list;
    list.count = 0;
    int64_t nb_n = 0;
    for (int k = 0; k < nprob; ++k)
      if (grouped(k) && host[k].b == b) {
        list.idx[list.count++] = k;
        nb_n = host[k].n > nb_n ? host[k].n : nb_n;
      }
    if (list.count) launch_group<kSubMinB>(b, dev, list, nb_n, s);
  }
  for (int four = 0; four < 2; ++four) {
    SubList list;
    list.count = 0;
    for (int k = 0; k <= nprob; ++k) {
      if (k < nprob && !grouped(k) && (host[k].n > 2 * kSubThreads) == (four != 0))
        list.idx[list.count++] = k;
      if (list.count == kLaunchMax || (k == nprob && list.count > 0)) {
        if (four)
          k_subspace<4><<<static_cast<unsigned>(list.count), kSubThreads, 0, s>>>(dev, list);
        else
          k_subspace<2><<<static_cast<unsigned>(list.count), kSubThreads, 0, s>>>(dev, list);
        list.count = 0;
      }
    }
  }
}

}  // namespace rsm
