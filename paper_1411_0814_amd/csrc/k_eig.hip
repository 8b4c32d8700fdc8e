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
//   4. b = r + 4 vectors: X <- orth(M^T M X), a fixed number of steps, with classical
//      Gram-Schmidt applied twice (rows held in registers of one workgroup).
//   5. Rayleigh-Ritz: H = X^T N X, H = Q Theta Q^T by parallel-ordering Jacobi,
//      V-hat = X Q[:, :r]; lambda_1..lambda_{r+1} = Theta; residual
//      max_k ||N v_k - theta_k v_k|| / lam_max.
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
constexpr int kRows = 16;       // output rows per workgroup of the thin products
constexpr double kShiftRel = 1e-8;
constexpr int kDescPerLaunch = 16;

typedef RSM_GLOBAL double* gdouble;
typedef RSM_GLOBAL const double* gcdouble;

// Generic-pointer view of a global address, for the atomics.
template <typename T>
__device__ __forceinline__ T* generic(RSM_GLOBAL T* p) {
  return (T*)p;
}

// Global load / store at a 32-bit element offset from a uniform base: the compiler can then
// use the scalar-base + 32-bit vector-offset addressing form (every matrix here has fewer
// than 2^28 elements).
__device__ __forceinline__ double gld(gcdouble base, uint32_t idx) {
  return *reinterpret_cast<gcdouble>(reinterpret_cast<RSM_GLOBAL const char*>(base) + (idx << 3));
}
__device__ __forceinline__ void gst(gdouble base, uint32_t idx, double v) {
  *reinterpret_cast<gdouble>(reinterpret_cast<RSM_GLOBAL char*>(base) + (idx << 3)) = v;
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

// Sum over the wavefront of NV values per lane with about NV exchanges instead of 6 NV: each
// halving step sends one half of the values to the partner lane and keeps the other half.
// Afterwards v[0] of lane l is the full sum of value idx(l); lanes whose low 6 - log2(NV)
// bits are zero hold distinct indices.
template <int NV, int OFF>
__device__ __forceinline__ void sum_many(double* v, int lane, int& idx) {
  if constexpr (NV > 1) {
    constexpr int H = NV / 2;
    const bool up = (lane & OFF) != 0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const double send = up ? v[j] : v[j + H];
      const double keep = up ? v[j + H] : v[j];
      v[j] = keep + __shfl_xor(send, OFF, 64);
    }
    idx += up ? H : 0;
    sum_many<H, OFF / 2>(v, lane, idx);
  } else {
#pragma unroll
    for (int off = OFF; off > 0; off >>= 1) v[0] += __shfl_xor(v[0], off, 64);
  }
}

template <int K>
constexpr int pow2_at_least() {
  int p = 1;
  while (p < K) p *= 2;
  return p;
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
  if (idx < kSmallDoubles) P.small[idx] = 0.0;
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

// ------------------------------------------------------------------ 4. subspace iteration

// Deterministic start block: entries uniform in [-1, 1) from Philox (key = seed, 1).
__global__ void k_start_vectors(const EigProb* __restrict__ probs) {
  const EigProb& P = probs[blockIdx.y];
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= P.n * P.b) return;
  uint64_t c[4] = {static_cast<uint64_t>(idx), 0x5eedull, 0ull, 0ull};
  Philox4x64::block(c, P.seed, 1ull);
  P.X[idx] = static_cast<double>(static_cast<int64_t>(c[0]) >> 11) * (1.0 / 4503599627370496.0);
}

// Out[j, c] = sum_i A[j, i] In[i, c] for all c < b, split over workgroups (j-block of 16
// rows, i-chunk of 256): each workgroup writes its chunk's share to AP[chunk][c][j] and
// k_apply_sum adds the shares in chunk order (no atomics: the sum does not depend on
// timing).  MODE 0: A = M (lower: i < j0 + 16), In = X, Out = Z.  MODE 1: A = Mt (upper:
// i >= j0), In = Z, Out = NX.  MODE 2: A = Nsym (all i), In = X, Out = NX, and the sum also
// forms the block's X[rows]^T NX[rows] share of the Rayleigh-Ritz matrix (into M, which is
// free by then).  Thread (jr, kp) = (t % 16, t / 16) sums over i = kp mod 16; the 16
// partial sums are added through LDS.  A chunk outside the operator's triangle writes
// zeros.
template <int MODE>
__global__ __launch_bounds__(256) void k_apply(const EigProb* __restrict__ probs, int nks) {
  __shared__ double Xs[256][kEigMaxB + 1];
  const EigProb& P = probs[blockIdx.y];
  const int n = static_cast<int>(P.n);
  const int b = P.b;
  const int jb = static_cast<int>(blockIdx.x) / nks, ks = static_cast<int>(blockIdx.x) % nks;
  const int j0 = jb * kRows;
  if (j0 >= n || ks * 256 >= n) return;
  gcdouble __restrict__ A = MODE == 0 ? P.M : (MODE == 1 ? P.Mt : P.Nsym);
  const uint32_t lda = static_cast<uint32_t>(MODE == 2 ? P.n : P.npad);
  gcdouble __restrict__ In = MODE == 1 ? P.Z : P.X;
  const int tid = threadIdx.x;
  const int jr = tid & (kRows - 1), kp = tid / kRows;
  const uint32_t jrow = static_cast<uint32_t>((j0 + jr < n) ? (j0 + jr) : (n - 1));
  int i_lo = MODE == 1 ? j0 : 0;
  int i_hi = MODE == 0 ? ((j0 + kRows < n) ? (j0 + kRows) : n) : n;
  i_lo = i_lo > ks * 256 ? i_lo : ks * 256;
  i_hi = i_hi < ks * 256 + 256 ? i_hi : ks * 256 + 256;
  double acc[kEigMaxB];
#pragma unroll
  for (int c = 0; c < kEigMaxB; ++c) acc[c] = 0.0;
  if (i_lo < i_hi) {
    const int c0 = i_lo;
    const int cnt = i_hi - c0;
    double mv[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int il = kp + 16 * s;
      mv[s] = gld(A, jrow + static_cast<uint32_t>(c0 + (il < cnt ? il : 0)) * lda);
      if (il >= cnt) mv[s] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < kEigMaxB; ++c) {
      const bool ok = tid < cnt && c < b;
      const double x = gld(In, static_cast<uint32_t>(c0 + (ok ? tid : 0)) +
                                   static_cast<uint32_t>(ok ? c : 0) * static_cast<uint32_t>(n));
      Xs[tid][c] = ok ? x : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int il = kp + 16 * s;
#pragma unroll
      for (int c = 0; c < kEigMaxB; ++c)
        if (c < b) acc[c] = fma(mv[s], Xs[il][c], acc[c]);
    }
  }
  __syncthreads();
  auto red = reinterpret_cast<double (*)[kRows][kEigMaxB + 1]>(&Xs[0][0]);  // [kp][jr][c]
#pragma unroll
  for (int c = 0; c < kEigMaxB; ++c) red[kp][jr][c] = acc[c];
  __syncthreads();
  gdouble __restrict__ part = P.AP + static_cast<int64_t>(ks) * b * n;
  for (int e = tid; e < kRows * b; e += 256) {
    const int r2 = e % kRows, c = e / kRows;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) s += red[q][r2][c];
    if (j0 + r2 < n) gst(part, static_cast<uint32_t>(j0 + r2 + c * n), s);
  }
}

// Out = the chunk shares of k_apply summed in chunk order, 16 rows per workgroup; MODE 2
// also forms the block's share of the Rayleigh-Ritz matrix.
template <int MODE>
__global__ __launch_bounds__(256) void k_apply_sum(const EigProb* __restrict__ probs) {
  __shared__ double Ys[kRows][kEigMaxB + 1];
  __shared__ double xr[kRows][kEigMaxB + 1];
  const EigProb& P = probs[blockIdx.y];
  const int n = static_cast<int>(P.n);
  const int b = P.b;
  const int j0 = static_cast<int>(blockIdx.x) * kRows;
  if (j0 >= n) return;
  const int nks = static_cast<int>(ceil_div(P.n, 256));
  gdouble __restrict__ Out = MODE == 0 ? P.Z : P.NX;
  const int tid = threadIdx.x;
  for (int e = tid; e < kRows * b; e += 256) {
    const int r2 = e % kRows, c = e / kRows;
    const int j = j0 + r2;
    double s = 0.0;
    if (j < n) {
      for (int ks = 0; ks < nks; ++ks)
        s += gld(P.AP, static_cast<uint32_t>(ks * b * n + j + c * n));
      gst(Out, static_cast<uint32_t>(j + c * n), s);
    }
    if (MODE == 2) {
      Ys[r2][c] = s;
      xr[r2][c] = (j < n) ? gld(P.X, static_cast<uint32_t>(j + c * n)) : 0.0;
    }
  }
  if (MODE == 2) {
    __syncthreads();
    // this block's share of H, summed over the blocks in order by the Jacobi kernel
    for (int e = tid; e < b * b; e += 256) {
      const int i = e / b, j = e % b;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < kRows; ++q) s += xr[q][i] * Ys[q][j];
      P.M[static_cast<int64_t>(blockIdx.x) * b * b + e] = s;
    }
  }
}

// One orthonormalisation column K: X[:, K] -= X[:, :K] h twice (classical Gram-Schmidt
// applied twice), then normalised.  x[s][c] holds rows tid + s NT.
template <int NT, int RPT, int K>
__device__ __forceinline__ void orth_cols(double (&x)[RPT][kEigMaxB], int b, double (*red)[32],
                                          double* h) {
  if constexpr (K < kEigMaxB) {
    if (K < b) {
      constexpr int NW = NT / 64;
      const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
      if constexpr (K > 0) {
        constexpr int NV = pow2_at_least<K>();
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
          double d[NV];
#pragma unroll
          for (int j = 0; j < NV; ++j) {
            double p = 0.0;
            if (j < K)
#pragma unroll
              for (int s = 0; s < RPT; ++s) p = fma(x[s][j], x[s][K], p);
            d[j] = p;
          }
          int idx = 0;
          sum_many<NV, 32>(d, lane, idx);
          if ((lane & (64 / NV - 1)) == 0) red[wid][idx] = d[0];
          __syncthreads();
          if (tid < K) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) s += red[w][tid];
            h[tid] = s;
          }
          __syncthreads();
#pragma unroll
          for (int j = 0; j < K; ++j) {
            const double hj = h[j];
#pragma unroll
            for (int s = 0; s < RPT; ++s) x[s][K] = fma(-hj, x[s][j], x[s][K]);
          }
        }
      }
      double p = 0.0;
#pragma unroll
      for (int s = 0; s < RPT; ++s) p = fma(x[s][K], x[s][K], p);
      p = wave_sum(p);
      __syncthreads();  // h of the last pass has been read
      if (lane == 0) red[wid][0] = p;
      __syncthreads();
      double nrm2 = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) nrm2 += red[w][0];
      const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
#pragma unroll
      for (int s = 0; s < RPT; ++s) x[s][K] *= inv;
      __syncthreads();  // red is reused by the next column
      orth_cols<NT, RPT, K + 1>(x, b, red, h);
    }
  }
}

// X = orth(NX), one workgroup per problem, NT threads x 4 rows in registers (n <= 4 NT).
template <int NT>
__global__ __launch_bounds__(NT) void k_orth(const EigProb* __restrict__ probs) {
  constexpr int RPT = 4;
  __shared__ double red[NT / 64][32];
  __shared__ double h[32];
  const EigProb& P = probs[blockIdx.y];
  const int64_t n = P.n;
  const int b = P.b;
  if (n > static_cast<int64_t>(NT) * RPT) return;  // the launcher picks NT from n
  const int tid = threadIdx.x;
  double x[RPT][kEigMaxB];
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int64_t i = tid + static_cast<int64_t>(s) * NT;
#pragma unroll
    for (int c = 0; c < kEigMaxB; ++c) {
      const bool ok = i < n && c < b;
      const double v = P.NX[(ok ? i : 0) + static_cast<int64_t>(ok ? c : 0) * n];
      x[s][c] = ok ? v : 0.0;
    }
  }
  orth_cols<NT, RPT, 0>(x, b, red, h);
#pragma unroll
  for (int s = 0; s < RPT; ++s) {
    const int64_t i = tid + static_cast<int64_t>(s) * NT;
    if (i < n)
#pragma unroll
      for (int c = 0; c < kEigMaxB; ++c)
        if (c < b) P.X[i + c * n] = x[s][c];
  }
}

// ------------------------------------------------------------------ 5. Rayleigh-Ritz

typedef double SmallMat[kEigMaxB + 1];

// Parallel-ordering (round-robin) Jacobi on the symmetric b x b matrix H (LDS) by one
// workgroup of 256 threads, thread t owning elements t and t + 256 of the row-major b x b
// array.  Each round rotates floor(b/2) disjoint index pairs: the rotations are computed in
// parallel, then applied as H <- J^T H J and Q <- Q J.  For a pair (p, q), p < q, with c, s
// from the usual tau formula, column p becomes c col_p - s col_q and column q becomes
// s col_p + c col_q (rows likewise); storing sn[q] = -s makes both "cs[j] col_j - sn[j]
// col_partner".  An element is rotated away only while it is above both eps sqrt(|a_pp
// a_qq|) and 4 eps ||H||_F (rounding keeps off-diagonal entries near eps ||H||).
__device__ void jacobi_block(SmallMat* H, SmallMat* Q, int b, int* perm, double* cs, double* sn,
                             int* partner, int* flag, double floor_abs) {
  const int t = threadIdx.x;
  const int bb = b + (b & 1);  // even number of players (one idle slot if b is odd)
  const int nel = b * b;
  const bool own0 = t < nel, own1 = t + 256 < nel;
  const int i0 = t / b, j0 = t % b, i1 = (t + 256) / b, j1 = (t + 256) % b;
  if (own0) Q[i0][j0] = i0 == j0 ? 1.0 : 0.0;
  if (own1) Q[i1][j1] = i1 == j1 ? 1.0 : 0.0;
  if (t < bb) perm[t] = t;
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    if (t == 0) *flag = 0;
    __syncthreads();
    for (int round = 0; round < bb - 1; ++round) {
      if (t < bb) partner[t] = -1;
      __syncthreads();
      if (t < bb / 2) {
        int p = perm[t], q = perm[bb - 1 - t];
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        if (q < b) {
          double c = 1.0, s = 0.0;
          const double apq = H[p][q], app = H[p][p], aqq = H[q][q];
          if (fabs(apq) > 2.220446049250313e-16 * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs) {
            const double tau = (aqq - app) / (2.0 * apq);
            double tt;
            if (fabs(tau) > 1e150) {
              tt = 0.5 / tau;
            } else {
              tt = 1.0 / (fabs(tau) + sqrt(1.0 + tau * tau));
              if (tau < 0.0) tt = -tt;
            }
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
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
      // H <- J^T H J and Q <- Q J for the owned elements (reads first, then writes)
      double h0 = 0.0, h1 = 0.0, q0 = 0.0, q1 = 0.0;
      if (own0) {
        const int pi = partner[i0], pj = partner[j0];
        const double ci = pi >= 0 ? cs[i0] : 1.0, si = pi >= 0 ? sn[i0] : 0.0;
        const double cj = pj >= 0 ? cs[j0] : 1.0, sj = pj >= 0 ? sn[j0] : 0.0;
        const int ii = pi >= 0 ? pi : i0, jj = pj >= 0 ? pj : j0;
        const double hij = H[i0][j0], hip = H[i0][jj], hpj = H[ii][j0], hpp = H[ii][jj];
        h0 = ci * (cj * hij - sj * hip) - si * (cj * hpj - sj * hpp);
        q0 = cj * Q[i0][j0] - sj * Q[i0][jj];
      }
      if (own1) {
        const int pi = partner[i1], pj = partner[j1];
        const double ci = pi >= 0 ? cs[i1] : 1.0, si = pi >= 0 ? sn[i1] : 0.0;
        const double cj = pj >= 0 ? cs[j1] : 1.0, sj = pj >= 0 ? sn[j1] : 0.0;
        const int ii = pi >= 0 ? pi : i1, jj = pj >= 0 ? pj : j1;
        const double hij = H[i1][j1], hip = H[i1][jj], hpj = H[ii][j1], hpp = H[ii][jj];
        h1 = ci * (cj * hij - sj * hip) - si * (cj * hpj - sj * hpp);
        q1 = cj * Q[i1][j1] - sj * Q[i1][jj];
      }
      __syncthreads();
      if (own0) {
        H[i0][j0] = h0;
        Q[i0][j0] = q0;
      }
      if (own1) {
        H[i1][j1] = h1;
        Q[i1][j1] = q1;
      }
      __syncthreads();
      // keep H exactly symmetric; circle method for the next round (player 0 fixed)
      double a0 = 0.0, a1 = 0.0;
      if (own0) a0 = 0.5 * (H[i0][j0] + H[j0][i0]);
      if (own1) a1 = 0.5 * (H[i1][j1] + H[j1][i1]);
      int nxt = 0;
      if (t < bb) nxt = t == 0 ? perm[0] : (t == 1 ? perm[bb - 1] : perm[t - 1]);
      __syncthreads();
      if (own0) H[i0][j0] = a0;
      if (own1) H[i1][j1] = a1;
      if (t < bb) perm[t] = nxt;
      __syncthreads();
    }
    if (*flag == 0) break;
    __syncthreads();
  }
}

// Small part of Rayleigh-Ritz (one workgroup per problem): Jacobi of H, eigenvalues sorted
// ascending; writes Qs = Q with its columns in that order and theta; clears res2.
__global__ __launch_bounds__(256) void k_rr_small(const EigProb* __restrict__ probs) {
  __shared__ SmallMat H[kEigMaxB];
  __shared__ SmallMat Q[kEigMaxB];
  __shared__ int perm[kEigMaxB + 1];
  __shared__ double cs[kEigMaxB + 1];
  __shared__ double sn[kEigMaxB + 1];
  __shared__ int partner[kEigMaxB + 1];
  __shared__ int flag;
  __shared__ int order[kEigMaxB];
  __shared__ double red[4];
  const EigProb& P = probs[blockIdx.y];
  const int b = P.b;
  const int t = threadIdx.x;
  // H = sum of the blocks' shares (in block order), then symmetrised
  const int nblk = static_cast<int>(ceil_div(P.n, kRows));
  for (int e = t; e < b * b; e += 256) {
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < nblk; k0 += 4) {
      double x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = P.M[static_cast<int64_t>(k0 + u < nblk ? k0 + u : 0) * b * b + e];
#pragma unroll
      for (int u = 0; u < 4; ++u) s4[u] += (k0 + u < nblk) ? x[u] : 0.0;
    }
    H[e / b][e % b] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  }
  __syncthreads();
  double f2 = 0.0;
  double hs[2] = {0.0, 0.0};
  for (int e = t, k = 0; e < b * b; e += 256, ++k) {
    const int i = e / b, j = e % b;
    hs[k] = 0.5 * (H[i][j] + H[j][i]);
    f2 += hs[k] * hs[k];
  }
  __syncthreads();
  for (int e = t, k = 0; e < b * b; e += 256, ++k) H[e / b][e % b] = hs[k];
  f2 = wave_sum(f2);
  if ((t & 63) == 0) red[t >> 6] = f2;
  __syncthreads();
  f2 = red[0] + red[1] + red[2] + red[3];
  jacobi_block(H, Q, b, perm, cs, sn, partner, &flag, 4.0 * 2.220446049250313e-16 * sqrt(f2));
  __syncthreads();
  if (t < b) {
    const double dk = H[t][t];
    int rk = 0;
    for (int j = 0; j < b; ++j) {
      const double dj = H[j][j];
      rk += (dj < dk) || (dj == dk && j < t);
    }
    order[rk] = t;
    P.small[kSmallTheta + rk] = dk;
  }
  __syncthreads();
  for (int e = t; e < b * b; e += 256) {
    const int j = e / b, k = e % b;  // Qs[j][k] = Q[j][order[k]]
    P.small[kSmallQs + e] = Q[j][order[k]];
  }
}

// V-hat = X Qs[:, :r] (thread per row) and the squared residual norms
// ||NX q_k - theta_k X q_k||^2, accumulated into res2[k].
__global__ __launch_bounds__(256) void k_rr_apply(const EigProb* __restrict__ probs) {
  __shared__ double q[kEigMaxB * kEigMaxB];
  __shared__ double th[kEigMaxB];
  __shared__ double red[4][RSM_MAX_R];
  const EigProb& P = probs[blockIdx.y];
  const int64_t n = P.n;
  const int b = P.b, r = P.r;
  if (static_cast<int64_t>(blockIdx.x) * 256 >= n) return;
  const int tid = threadIdx.x, lane = tid & 63;
  for (int e = tid; e < b * b; e += 256) q[e] = P.small[kSmallQs + e];
  if (tid < b) th[tid] = P.small[kSmallTheta + tid];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + tid;
  const bool act = i < n;
  double x[kEigMaxB], y[kEigMaxB];
#pragma unroll
  for (int j = 0; j < kEigMaxB; ++j) {
    const bool ok = act && j < b;
    const int64_t at = (ok ? i : 0) + static_cast<int64_t>(ok ? j : 0) * n;
    const double xv = P.X[at], yv = P.NX[at];
    x[j] = ok ? xv : 0.0;
    y[j] = ok ? yv : 0.0;
  }
  __syncthreads();
  double res[RSM_MAX_R];
#pragma unroll
  for (int k = 0; k < RSM_MAX_R; ++k) {
    double v = 0.0, rs = 0.0;
    if (k < r) {
#pragma unroll
      for (int j = 0; j < kEigMaxB; ++j) {
        if (j < b) {
          const double qj = q[j * b + k];
          v = fma(x[j], qj, v);
          rs = fma(y[j] - th[k] * x[j], qj, rs);
        }
      }
      if (act) P.V[i + k * n] = v;
    }
    res[k] = rs * rs;
  }
  int idx = 0;
  sum_many<RSM_MAX_R, 32>(res, lane, idx);
  if ((lane & 3) == 0) red[tid >> 6][idx] = res[0];
  __syncthreads();
  // this block's squared residuals (into T, free by then), summed in block order by k_rr_finish
  if (tid < r)
    P.T[static_cast<int64_t>(blockIdx.x) * RSM_MAX_R + tid] =
        (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

__global__ void k_rr_finish(const EigProb* __restrict__ probs) {
  const EigProb& P = probs[blockIdx.y];
  if (threadIdx.x != 0) return;
  const int b = P.b, r = P.r;
  gcdouble theta = P.small + kSmallTheta;
  const double lam_max = P.scal->lam_max;
  const int nblk = static_cast<int>(ceil_div(P.n, 256));
  double rmax = 0.0;
  for (int k = 0; k < r; ++k) {
    double s = 0.0;
    for (int blk = 0; blk < nblk; ++blk) s += P.T[static_cast<int64_t>(blk) * RSM_MAX_R + k];
    rmax = fmax(rmax, sqrt(s));
  }
  const double rel = lam_max > 0.0 ? rmax / lam_max : rmax;
  RSM_GLOBAL rsm_info* info = P.info;
  info->residual = rel;
  for (int k = 0; k <= r && k < b; ++k) info->lambda[k] = theta[k];
  uint32_t warn = 0;
  if (info->uncovered > 0) warn |= RSM_W_RANK_DEFICIENT;
  if (b > r && !(theta[r] > 1e-12 * lam_max)) warn |= RSM_W_RANK_DEFICIENT;
  if (rel > 1e-6) warn |= RSM_W_NOT_CONVERGED;
  if (P.scal->pivots > 0) warn |= RSM_W_PIVOT;
  if (P.check_accepted && info->accepted == 0) warn |= RSM_W_NO_CONSTRAINTS;
  atomicOr(generic(&info->warn), warn);
  info->eig_iterations = kEigIters;
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
  const unsigned g_rows16 = static_cast<unsigned>(ceil_div(n_max, kRows));
  const int nks = static_cast<int>(ceil_div(n_max, 256));
  const unsigned g_apply = g_rows16 * static_cast<unsigned>(nks);
  for (int it = 0; it < kEigIters; ++it) {
    k_apply<0><<<dim3(g_apply, np), 256, 0, s>>>(dev, nks);
    k_apply_sum<0><<<dim3(g_rows16, np), 256, 0, s>>>(dev);
    k_apply<1><<<dim3(g_apply, np), 256, 0, s>>>(dev, nks);
    k_apply_sum<1><<<dim3(g_rows16, np), 256, 0, s>>>(dev);
    if (n_max <= 4 * 256)
      k_orth<256><<<dim3(1, np), 256, 0, s>>>(dev);
    else
      k_orth<512><<<dim3(1, np), 512, 0, s>>>(dev);
  }
  k_apply<2><<<dim3(g_apply, np), 256, 0, s>>>(dev, nks);
  k_apply_sum<2><<<dim3(g_rows16, np), 256, 0, s>>>(dev);
  k_rr_small<<<dim3(1, np), 256, 0, s>>>(dev);
  k_rr_apply<<<dim3(static_cast<unsigned>(ceil_div(n_max, 256)), np), 256, 0, s>>>(dev);
  k_rr_finish<<<dim3(1, np), 64, 0, s>>>(dev);
}

}  // namespace rsm
