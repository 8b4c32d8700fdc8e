// Step a7: U-hat by eq.(solve.barU) with the L2 norm, row by row:
//   u_i = argmin_u sum_j w_ij (y_ij - u^T v_j)^2  =>  A_i u_i = b_i,
//   A_i = sum_{j known} v_j v_j^T (r x r),  b_i = sum_{j known} y_ij v_j.
// Two ways to form A_i and b_i (both FP64):
//  - k_usolve: one thread per row; a wavefront covers 64 consecutive rows, i.e. one word of
//    each column's mask bit-plane, read once per wavefront.  V-hat is staged through LDS in
//    chunks of columns and read as a broadcast.  Used for small r.
//  - k_uform: for all rows at once, [A | b] = W~ [K | V] as one dense product on the FP64
//    matrix cores, where row j of K holds the products v_ja v_jb (a >= b) of V-hat's row j
//    and W~ is the 0/1 mask (for the A part) or the mask times Y (for the b part); k_ukext
//    writes [K | V] once per problem.  The r(r+1)/2 + r results per row go to the
//    workspace; k_usolve_ab solves them.
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
// known entries and every pivot is positive.  The diagonal slots keep 1 / l_jj, so each
// column costs one FP64 division and the rest are multiplications.  Writes U's row, and
// adds the wavefront's underdetermined rows and known entries to the problem's info.
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
      const double rl = 1.0 / sqrt(d > 0.0 ? d : 1.0);
      A[j * (j + 1) / 2 + j] = rl;
#pragma unroll
      for (int ii = j + 1; ii < R; ++ii) {
        double s = A[ii * (ii + 1) / 2 + j];
#pragma unroll
        for (int p = 0; p < j; ++p) s -= A[ii * (ii + 1) / 2 + p] * A[j * (j + 1) / 2 + p];
        A[ii * (ii + 1) / 2 + j] = s * rl;
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
      u[a] = s * A[a * (a + 1) / 2 + a];
    }
    // backward: L^T u = z
#pragma unroll
    for (int a = R - 1; a >= 0; --a) {
      double s = u[a];
#pragma unroll
      for (int p = a + 1; p < R; ++p) s -= A[p * (p + 1) / 2 + a] * u[p];
      u[a] = s * A[a * (a + 1) / 2 + a];
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

// Solve of the normal equations that k_uform wrote: one thread per row.  From r = 14 the
// r(r+1)/2 + r values of a row fill the register file (one wavefront per SIMD), and a
// workgroup is one wavefront, so that it fits wherever one SIMD's registers are free
// while the U-hat launches of other ranks run beside it.
template <int R>
constexpr int usolve_ab_threads() { return R >= 14 ? 64 : 256; }

template <int R>
__global__ __launch_bounds__(usolve_ab_threads<R>()) void k_usolve_ab(
    const ProbDesc* __restrict__ probs, IdxList list) {
  constexpr int NA = R * (R + 1) / 2;
  constexpr int NT = usolve_ab_threads<R>();
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t m = P.m;
  if (static_cast<int64_t>(blockIdx.x) * NT >= m) return;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
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

constexpr int kUfWaves = 4;                          // wavefronts per workgroup
constexpr int kUfThreads = 64 * kUfWaves;
constexpr int kUfCols = 16;                          // columns per LDS stage (4 k-steps)

template <int R>
struct UfShape {
  static constexpr int kNA = R * (R + 1) / 2;
  static constexpr int kTA = uform_tiles_a(R);  // 16-wide output tiles of A entries
  static constexpr int kT = kTA + 1;            // and one of b (r <= 16)
  static constexpr int kStride = uform_stride(R);
  static_assert(kStride == kT * 16 + ((kT % 2 == 0) ? 16 : 0), "row layout");
  static_assert((kUfCols * kStride * 8) % (4 * kUfThreads) == 0, "a stage is whole rounds");
};

// 16-row tiles per wavefront: four while the accumulators of four tiles and FP32 Y values
// leave room for two wavefronts per SIMD (each right-operand value then feeds four
// products), else two; and the rows of a workgroup.
template <int R, typename TY>
constexpr int uf_tiles() { return (UfShape<R>::kT <= 4 && sizeof(TY) == 4) ? 4 : 2; }
template <int R, typename TY>
constexpr int uf_rows() { return kUfWaves * 16 * uf_tiles<R, TY>(); }

// Row pair (a, b), b <= a, of packed entry e < r(r+1)/2.
__device__ __forceinline__ void unpack_pair(int e, int& a, int& b) {
  a = static_cast<int>((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
  while (a * (a + 1) / 2 > e) --a;
  while ((a + 1) * (a + 2) / 2 <= e) ++a;
  b = e - a * (a + 1) / 2;
}

// The right operand of the product, once per problem: row j of kext (j < ceil(n/32)*32) is
// [v_ja v_jb (a >= b) | 0 | v_j | 0], zero for j >= n.
template <int R>
__global__ __launch_bounds__(256) void k_ukext(const ProbDesc* __restrict__ probs, IdxList list) {
  using S = UfShape<R>;
  constexpr int NA = S::kNA, TA = S::kTA, LD = S::kStride;
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t n = P.n, rows = ceil_div(n, 32) * 32;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= rows * LD) return;
  const int64_t j = e / LD;
  const int q = static_cast<int>(e - j * LD);
  RSM_GLOBAL const double* __restrict__ V = P.V;
  double val = 0.0;
  if (j < n) {
    if (q < NA) {
      int a, b;
      unpack_pair(q, a, b);
      val = V[j + static_cast<int64_t>(a) * n] * V[j + static_cast<int64_t>(b) * n];
    } else if (q >= TA * 16 && q - TA * 16 < R) {
      val = V[j + static_cast<int64_t>(q - TA * 16) * n];
    }
  }
  P.kext[e] = val;
}

__device__ __forceinline__ void lds_dma_dword(const void* src, void* dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 4, 0, 0);
}

// Workgroup: uf_rows consecutive rows (kUfWaves wavefronts x uf_tiles tiles of 16).  The
// right operand's rows for a stage of kUfCols columns travel from kext straight into one of
// two LDS buffers (global_load_lds_dword: lane k of a wavefront writes 4 bytes at base + 4 k;
// the workgroup moves 4 bytes per thread per round), and each lane loads the mask bit and
// Y value of its (row, column) position of every k-step (the left operand: the bit as 0/1
// for the A part, bit times y for the b part).  Stage s + 1's loads are issued right after the barrier that publishes stage
// s and land while stage s runs on the matrix cores: one barrier per stage.  Rows past m and
// columns past n have weight 0.
template <int R, typename TY>
__global__ __launch_bounds__(kUfThreads) void k_uform(const ProbDesc* __restrict__ probs,
                                                      IdxList list) {
  using S = UfShape<R>;
  constexpr int NA = S::kNA, TA = S::kTA, T = S::kT, LD = S::kStride, C = kUfCols;
  constexpr int kUfTiles = uf_tiles<R, TY>(), kUfRows = uf_rows<R, TY>();
  constexpr int KS = C / 4;                               // k-steps of 4 columns per stage
  constexpr int kRound = 4 * kUfThreads;                  // bytes the workgroup moves per round
  constexpr int kRounds = C * LD * 8 / kRound;            // rounds of a stage
  __shared__ __align__(16) double Kb[2 * C * LD];
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t m = P.m, n = P.n, ldy = P.ldy, mw32 = 2 * P.mw;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kUfRows;
  if (row0 >= m) return;
  auto Y = static_cast<RSM_GLOBAL const TY*>(P.ycm);
  auto wbits = reinterpret_cast<RSM_GLOBAL const uint32_t*>(P.wbits);
  auto kext = reinterpret_cast<RSM_GLOBAL const char*>(P.kext);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
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
  // right operand of stage st into `dst` (rows st*C .. st*C + C - 1 of kext, all present)
  auto issue_k = [&](int64_t st, double* dst) {
    const char* src = kext + st * (C * LD * 8) + 4 * tid;
    char* d = reinterpret_cast<char*>(dst) + 256 * wv;
#pragma unroll
    for (int u = 0; u < kRounds; ++u) lds_dma_dword(src + kRound * u, d + kRound * u);
  };
  // left operand of a stage: mask words and Y values of (row ic[t], column cs + 4 ks + lk)
  uint32_t wreg[KS][kUfTiles], wnext[KS][kUfTiles];
  TY yreg[KS][kUfTiles], ynext[KS][kUfTiles];
  auto load_stage = [&](int64_t cs, uint32_t (&wr)[KS][kUfTiles], TY (&yr)[KS][kUfTiles]) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int64_t j = cs + 4 * ks + lk;
      const int64_t jc = j < n ? j : n - 1;
#pragma unroll
      for (int t = 0; t < kUfTiles; ++t) {
        wr[ks][t] = wbits[jc * mw32 + (ic[t] >> 5)];
        yr[ks][t] = Y[jc * ldy + ic[t]];
      }
    }
  };
  const int64_t stages = ceil_div(n, C);
  issue_k(0, Kb);
  load_stage(0, wreg, yreg);
  for (int64_t st = 0; st < stages; ++st) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();  // stage st is in its buffer; every wave is done with the other one
    const double* cur = Kb + (st & 1) * (C * LD);
    if (st + 1 < stages) {
      issue_k(st + 1, Kb + ((st + 1) & 1) * (C * LD));
      load_stage((st + 1) * C, wnext, ynext);
    }
    const int64_t c0 = st * C;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
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
      const double* brow = cur + (4 * ks + lk) * LD + li;
#pragma unroll
      for (int q = 0; q < T; ++q) {
        const double b = brow[q * 16];
#pragma unroll
        for (int t = 0; t < kUfTiles; ++t)
          acc[t][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(q < TA ? aw[t] : awy[t], b, acc[t][q], 0, 0, 0);
      }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
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
void run_usolve(const ProbDesc* d, const IdxList& g, int64_t m, int64_t n, int y_dtype,
                bool mfma, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(ceil_div(m, 256)), g.count);
  if constexpr (R >= kUMfmaMinR) {
    if (mfma) {
      const int64_t kext = ceil_div(n, 32) * 32 * UfShape<R>::kStride;
      k_ukext<R><<<dim3(static_cast<unsigned>(ceil_div(kext, 256)), g.count), 256, 0, s>>>(d, g);
      if (y_dtype == RSM_F32)
        k_uform<R, float><<<dim3(static_cast<unsigned>(ceil_div(m, uf_rows<R, float>())), g.count),
                            kUfThreads, 0, s>>>(d, g);
      else
        k_uform<R, double><<<dim3(static_cast<unsigned>(ceil_div(m, uf_rows<R, double>())), g.count),
                             kUfThreads, 0, s>>>(d, g);
      constexpr int nt = usolve_ab_threads<R>();
      k_usolve_ab<R><<<dim3(static_cast<unsigned>(ceil_div(m, nt)), g.count), nt, 0, s>>>(d, g);
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
  int64_t m = 0, n = 0;
  for (int k = 0; k < g.count; ++k) {
    m = std::max(m, h[k]->m);
    n = std::max(n, h[k]->n);
  }
  switch (h[0]->r) {
#define RSM_U_CASE(RR) \
  case RR:             \
    run_usolve<RR>(d, g, m, n, h[0]->y_dtype, h[0]->u_mfma, s); \
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
