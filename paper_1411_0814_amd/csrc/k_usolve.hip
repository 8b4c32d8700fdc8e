// Step a7: U-hat by eq.(solve.barU) with the L2 norm, row by row:
//   u_i = argmin_u sum_j w_ij (y_ij - u^T v_j)^2  =>  A_i u_i = b_i,
//   A_i = sum_{j known} v_j v_j^T (r x r),  b_i = sum_{j known} y_ij v_j.
// Two ways to form A_i and b_i (both FP64):
//  - k_usolve: one thread per row; a wavefront covers 64 consecutive rows, i.e. one word of
//    each column's mask bit-plane, read once per wavefront.  V-hat is staged through LDS in
//    chunks of columns and read as a broadcast.  Used for small r.
//  - k_uform: for all rows at once, [A | b] = W~ [K | V] as one dense product on the FP64
//    matrix cores, where row j of K holds the products v_ja v_jb (a >= b) of V-hat's row j
//    and W~ is the 0/1 mask (for the A part) or the mask times Y (for the b part).  The
//    r(r+1)/2 + r results per row go to the workspace; k_usolve_ab solves them.
// A_i is factorised by Cholesky in registers, one thread per row.  Rows with fewer than r
// known entries (or a singular A_i) get u_i = 0 and are counted as underdetermined.
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

// Cholesky of A (packed lower triangle, row-major: entry (a, b), b <= a, at a(a+1)/2 + b)
// in place, then A u = b by two triangular solves; u_i = 0 unless the row has at least r
// known entries and every pivot is positive.  Writes U's row, and adds the wavefront's
// underdetermined rows and known entries to the problem's info.
template <int R>
__device__ __forceinline__ void solve_row(const ProbDesc& P, double (&A)[R * (R + 1) / 2],
                                          const double (&bv)[R], int cnt, bool active,
                                          int64_t i) {
  const int64_t m = P.m;
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
  RSM_GLOBAL double* __restrict__ U = P.U;
  if (active) {
#pragma unroll
    for (int a = 0; a < R; ++a) U[i + static_cast<int64_t>(a) * m] = ok ? u[a] : 0.0;
  }
  RSM_GLOBAL rsm_info* info = P.info;
  const unsigned long long under = wave_sum<unsigned long long>((active && !ok) ? 1ull : 0ull);
  const unsigned long long known = wave_sum<unsigned long long>(active ? static_cast<unsigned long long>(cnt) : 0ull);
  if ((threadIdx.x & 63) == 0) {
    if (under) {
      atomicAdd((unsigned long long*)&info->rows_underdetermined, under);
      atomicOr((uint32_t*)&info->warn, static_cast<uint32_t>(RSM_W_ROWS_UNDERDETERMINED));
    }
    if (known) atomicAdd((unsigned long long*)&info->known, known);
  }
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
  constexpr int kUnroll = u_unroll<R>();
  static_assert(kUChunk % kUnroll == 0, "column groups tile a chunk");
  for (int64_t j0 = 0; j0 < n; j0 += kUChunk) {
    const int jn = static_cast<int>((n - j0) < kUChunk ? (n - j0) : kUChunk);
    // the last group of kUnroll columns can run past jn: its slots hold zeros, since a zero
    // weight times whatever LDS held before (possibly a NaN) would not be zero
    const int jpad = (jn + kUnroll - 1) / kUnroll * kUnroll;
    __syncthreads();
    for (int e = tid; e < jpad * R; e += 256) {
      const int jj = e / R, a = e % R;
      Vs[e] = jj < jn ? V[(j0 + jj) + static_cast<int64_t>(a) * n] : 0.0;
    }
    __syncthreads();
    if (wave_active) {
      // groups of kUnroll columns: all loads of a group first, then the products; the
      // mask bit is a 0/1 weight, so there is no divergent branch
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
  solve_row<R>(P, A, bv, cnt, active, i);
}

// Solve of the normal equations that k_uform wrote: one thread per row.
template <int R>
__global__ __launch_bounds__(256) void k_usolve_ab(const ProbDesc* __restrict__ probs, IdxList list) {
  constexpr int NA = R * (R + 1) / 2;
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t m = P.m;
  if (static_cast<int64_t>(blockIdx.x) * 256 >= m) return;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const bool active = i < m;
  const int64_t ic = active ? i : m - 1;
  RSM_GLOBAL const double* __restrict__ ab = P.ab;
  double A[NA];
  double bv[R];
#pragma unroll
  for (int g = 0; g < NA; ++g) A[g] = ab[static_cast<int64_t>(g) * m + ic];
#pragma unroll
  for (int a = 0; a < R; ++a) bv[a] = ab[static_cast<int64_t>(NA + a) * m + ic];
  const int cnt = P.abcnt[ic];
  solve_row<R>(P, A, bv, cnt, active, i);
}

// ---------------------------------------------------------------- normal equations on MFMA
// v_mfma_f64_16x16x4f64: D (16 x 16) += A (16 x 4) B (4 x 16), one double per lane for A
// and B: A(i, k) in lane i + 16 k, B(k, j) in lane j + 16 k; D(i, j) in lane j + 16 (i % 4),
// register i / 4.
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kUfTiles = 2;                  // 16-row tiles per wavefront
constexpr int kUfRows = 4 * 16 * kUfTiles;   // rows per workgroup (4 wavefronts)
constexpr int kUfCols = 32;                  // columns per LDS stage (8 k-steps of 4)

template <int R>
struct UfShape {
  static constexpr int kNA = R * (R + 1) / 2;
  static constexpr int kTA = (kNA + 15) / 16;   // 16-wide output tiles of A entries
  static constexpr int kT = kTA + 1;            // and one of b (r <= 16)
  // doubles per staged column: 16 mod 32, so that the 4 k-rows of a B fragment (128 bytes
  // each) fall on alternate halves of the LDS banks
  static constexpr int kStride = kT * 16 + ((kT % 2 == 0) ? 16 : 0);
};

// Row pair (a, b), b <= a, of packed entry e < r(r+1)/2.
__device__ __forceinline__ void unpack_pair(int e, int& a, int& b) {
  a = static_cast<int>((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
  while (a * (a + 1) / 2 > e) --a;
  while ((a + 1) * (a + 2) / 2 <= e) ++a;
  b = e - a * (a + 1) / 2;
}

// A workgroup barrier that orders LDS only: the global loads of the next stage stay in
// flight across it (__syncthreads also waits for every outstanding global load).  The
// kernel shares nothing but LDS between its threads.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Workgroup: 128 consecutive rows (4 wavefronts x 2 tiles of 16).  Per stage of 32 columns
// the workgroup writes K's and V's rows for those columns to LDS ([K | 0 | V | 0] per
// column, the B operands); each lane loads the mask bit and Y value of its (row, column)
// position of every k-step (the A operands: the bit as 0/1 for the A part, bit times y for
// the b part), the next stage's issued while the current stage's K is staged.  Rows past m
// and columns past n have weight 0.
template <int R, typename TY>
__global__ __launch_bounds__(256) void k_uform(const ProbDesc* __restrict__ probs, IdxList list) {
  using S = UfShape<R>;
  constexpr int NA = S::kNA, TA = S::kTA, T = S::kT, LD = S::kStride;
  __shared__ double Kc[kUfCols * LD];
  __shared__ double Vc[kUfCols * R];
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t m = P.m, n = P.n, ldy = P.ldy, mw32 = 2 * P.mw;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kUfRows;
  if (row0 >= m) return;
  auto Y = static_cast<RSM_GLOBAL const TY*>(P.ycm);
  auto wbits = reinterpret_cast<RSM_GLOBAL const uint32_t*>(P.wbits);
  RSM_GLOBAL const double* __restrict__ V = P.V;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  int64_t ic[kUfTiles];
  bool rok[kUfTiles];
#pragma unroll
  for (int t = 0; t < kUfTiles; ++t) {
    const int64_t i = row0 + wv * 16 * kUfTiles + t * 16 + li;
    rok[t] = i < m;
    ic[t] = rok[t] ? i : m - 1;
  }
  f64x4 acc[kUfTiles][T];
#pragma unroll
  for (int t = 0; t < kUfTiles; ++t)
#pragma unroll
    for (int q = 0; q < T; ++q) acc[t][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  int cnt[kUfTiles] = {};
  // (a, b) of the packed A entry in each column slot q of a staged row, once per workgroup
  __shared__ int8_t pa[T * 16], pb[T * 16];
  for (int q = tid; q < T * 16; q += 256) {
    int a = -1, b = -1;
    if (q < NA) unpack_pair(q, a, b);
    pa[q] = static_cast<int8_t>(a);
    pb[q] = static_cast<int8_t>(b);
  }
  // A operands of a stage: mask words and Y values of (row ic[t], column c0 + 4 ks + lk);
  // the next stage's are loaded while the current one runs on the matrix cores
  uint32_t wreg[kUfCols / 4][kUfTiles], wnext[kUfCols / 4][kUfTiles];
  TY yreg[kUfCols / 4][kUfTiles], ynext[kUfCols / 4][kUfTiles];
  auto load_stage = [&](int64_t cs, uint32_t (&wr)[kUfCols / 4][kUfTiles],
                        TY (&yr)[kUfCols / 4][kUfTiles]) {
#pragma unroll
    for (int ks = 0; ks < kUfCols / 4; ++ks) {
      const int64_t j = cs + 4 * ks + lk;
      const int64_t jc = j < n ? j : n - 1;
#pragma unroll
      for (int t = 0; t < kUfTiles; ++t) {
        wr[ks][t] = wbits[jc * mw32 + (ic[t] >> 5)];
        yr[ks][t] = Y[jc * ldy + ic[t]];
      }
    }
  };
  load_stage(0, wreg, yreg);
  for (int64_t c0 = 0; c0 < n; c0 += kUfCols) {
    lds_barrier();  // the previous stage's B operands are consumed
    for (int e = tid; e < kUfCols * R; e += 256) {
      const int c = e / R, a = e - c * R;
      const int64_t j = c0 + c;
      Vc[e] = j < n ? V[j + static_cast<int64_t>(a) * n] : 0.0;
    }
    lds_barrier();
    // the next stage's A operands: issued after this stage's V-hat loads have landed
    // (loads complete in order, so a wait on those would wait on these too), to land while
    // K is staged and the products run
    if (c0 + kUfCols < n) load_stage(c0 + kUfCols, wnext, ynext);
    for (int e = tid; e < kUfCols * T * 16; e += 256) {
      const int c = e / (T * 16), q = e - c * (T * 16);
      double val = 0.0;
      if (q < NA) {
        val = Vc[c * R + pa[q]] * Vc[c * R + pb[q]];
      } else if (q >= TA * 16 && q - TA * 16 < R) {
        val = Vc[c * R + (q - TA * 16)];
      }
      Kc[c * LD + q] = val;
    }
    lds_barrier();
#pragma unroll
    for (int ks = 0; ks < kUfCols / 4; ++ks) {
      // the mask bit as a 0/1 weight, formed without branches
      const uint32_t jok = (c0 + 4 * ks + lk < n) ? 1u : 0u;
      double aw[kUfTiles], awy[kUfTiles];
#pragma unroll
      for (int t = 0; t < kUfTiles; ++t) {
        const uint32_t kn = (wreg[ks][t] >> (ic[t] & 31)) & jok & (rok[t] ? 1u : 0u);
        aw[t] = static_cast<double>(kn);
        awy[t] = kn ? static_cast<double>(yreg[ks][t]) : 0.0;
        cnt[t] += static_cast<int>(kn);
      }
      const double* brow = Kc + (4 * ks + lk) * LD + li;
#pragma unroll
      for (int q = 0; q < T; ++q) {
        const double b = brow[q * 16];
#pragma unroll
        for (int t = 0; t < kUfTiles; ++t)
          acc[t][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(q < TA ? aw[t] : awy[t], b, acc[t][q], 0, 0, 0);
      }
    }
#pragma unroll
    for (int ks = 0; ks < kUfCols / 4; ++ks)
#pragma unroll
      for (int t = 0; t < kUfTiles; ++t) {
        wreg[ks][t] = wnext[ks][t];
        yreg[ks][t] = ynext[ks][t];
      }
  }
  // D(i, e) of tile (t, q): row i = 4 v + lk of the tile (register v), column e = 16 q + li
  RSM_GLOBAL double* __restrict__ ab = P.ab;
#pragma unroll
  for (int t = 0; t < kUfTiles; ++t) {
    const int64_t base = row0 + wv * 16 * kUfTiles + t * 16;
#pragma unroll
    for (int q = 0; q < T; ++q) {
      const int e = q * 16 + li;
      const bool eok = q < TA ? (e < NA) : (li < R);
      const int64_t col = q < TA ? e : NA + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = base + 4 * v + lk;
        if (eok && i < m) ab[col * m + i] = acc[t][q][v];
      }
    }
    // known entries of row ic[t]: lanes li, li + 16, li + 32, li + 48 hold its columns
    int c = cnt[t];
    c += __shfl_xor(c, 16, 64);
    c += __shfl_xor(c, 32, 64);
    if (lk == 0 && rok[t]) P.abcnt[ic[t]] = c;
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
  // one partial per workgroup, summed in a fixed order: e is reproducible bit for bit
  __shared__ double wsum[4];
  acc = wave_sum(acc);
  if ((tid & 63) == 0) wsum[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) P.errp[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

// e = sqrt(sum / known): each lane sums a strided share of the partials in order, then a
// fixed butterfly over the wavefront.
__global__ void k_error_finalize(const ProbDesc* __restrict__ probs, IdxList list) {
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t parts = ceil_div(P.m, int64_t(256));
  double acc = 0.0;
  for (int64_t q = threadIdx.x; q < parts; q += 64) acc += P.errp[q];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) {
    const double k = static_cast<double>(P.info->known);
    P.info->e = k > 0.0 ? sqrt(acc / k) : 0.0;
  }
}

template <int R>
void run_usolve(const ProbDesc* d, const IdxList& g, int64_t m, int y_dtype, bool mfma,
                hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(ceil_div(m, 256)), g.count);
  if constexpr (R >= kUMfmaMinR) {
    if (mfma) {
      const dim3 gf(static_cast<unsigned>(ceil_div(m, kUfRows)), g.count);
      if (y_dtype == RSM_F32)
        k_uform<R, float><<<gf, 256, 0, s>>>(d, g);
      else
        k_uform<R, double><<<gf, 256, 0, s>>>(d, g);
      k_usolve_ab<R><<<grid, 256, 0, s>>>(d, g);
      return;
    }
  }
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

// The group shares r, the element type of Y and the way A_i and b_i are formed.
void launch_solve_u(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  if (!g.count) return;
  int64_t m = 0;
  for (int k = 0; k < g.count; ++k) m = std::max(m, h[k]->m);
  switch (h[0]->r) {
#define RSM_U_CASE(RR) \
  case RR:             \
    run_usolve<RR>(d, g, m, h[0]->y_dtype, h[0]->u_mfma, s); \
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
