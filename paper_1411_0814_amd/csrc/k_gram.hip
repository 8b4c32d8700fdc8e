// Steps a2 + a3: row qualification and the l x l Gram of every trial.
//
// For trial t with sorted columns C_t = {c_0 < ... < c_{l-1}} (method M1, Section III):
//   R_t = { i : W[i, c] = 1 for every c in C_t }            (logical AND of l mask bit-planes)
//   G_t = sum_{i in R_t} y_{i,C_t} y_{i,C_t}^T                (l(l+1)/2 unique entries)
// The minor right singular vectors of Z_t = Y[R_t, C_t] are the eigenvectors of G_t for its
// smallest eigenvalues (Section III; they are computed in k_minor.hip).
//
// Output: partial Grams over row splits, part[split][trial][g] with g enumerating
// (a, b), b <= a, row-major over the lower triangle, and partial row counts
// prow[split][trial].  k_minor sums the splits in FP64.
//
// Two kernels:
//  * k_gram_plain  — one wavefront per (trial, row split).  Each 64-row word ANDs l mask
//    words (scalar loads) and the lanes whose row qualifies load their l values (column-
//    major, coalesced) and accumulate.  Simple, but every trial streams its l columns
//    from HBM: traffic ~ I * l * m * 4 bytes.
//  * k_gram_tile   — the LDS-reuse kernel: a workgroup stages a 32-row x n-column tile of Y
//    (and the tile's mask words) in LDS once and every thread — one trial each — gathers
//    its qualifying rows from LDS.  HBM/L2 traffic drops to (trial groups) x |Y|.
#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

template <typename TY, typename TA>
__device__ __forceinline__ TA load_as(const TY* p) {
  return static_cast<TA>(*p);
}

// ------------------------------------------------------------------ per-trial streamer

template <int L, typename TY, typename TA>
__global__ __launch_bounds__(256) void k_gram_plain(
    const TY* __restrict__ Y, int64_t ldy, const uint64_t* __restrict__ wbits, int64_t mw,
    const int32_t* __restrict__ cols, int64_t I, int64_t words_per_split,
    TA* __restrict__ part, int32_t* __restrict__ prow) {
  constexpr int NG = L * (L + 1) / 2;
  const int lane = threadIdx.x & 63;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (t >= I) return;  // wave-uniform
  const int split = blockIdx.y;
  const int64_t w0 = static_cast<int64_t>(split) * words_per_split;
  const int64_t w1 = (w0 + words_per_split < mw) ? (w0 + words_per_split) : mw;

  const uint64_t* wcol[L];
  const TY* ycol[L];
  bool valid = true;
#pragma unroll
  for (int a = 0; a < L; ++a) {
    const int c = static_cast<int>(uniform_u32(static_cast<uint32_t>(cols[t * L + a])));
    valid &= (c >= 0);
    const int cc = c < 0 ? 0 : c;
    wcol[a] = wbits + static_cast<int64_t>(cc) * mw;
    ycol[a] = Y + static_cast<int64_t>(cc) * ldy;
  }

  TA acc[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) acc[g] = TA(0);
  int count = 0;

  if (valid) {
    for (int64_t w = w0; w < w1; ++w) {
      uint64_t q = ~0ull;
#pragma unroll
      for (int a = 0; a < L; ++a) q &= wcol[a][w];
      count += __popcll(q);
      if ((q >> lane) & 1ull) {
        const int64_t i = w * 64 + lane;
        TA y[L];
#pragma unroll
        for (int a = 0; a < L; ++a) y[a] = load_as<TY, TA>(ycol[a] + i);
        int g = 0;
#pragma unroll
        for (int a = 0; a < L; ++a)
#pragma unroll
          for (int b = 0; b <= a; ++b) acc[g++] += y[a] * y[b];
      }
    }
  }

  TA* dst = part + (static_cast<int64_t>(split) * I + t) * NG;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const TA v = wave_sum(acc[g]);
    if (lane == 0) dst[g] = v;
  }
  if (lane == 0) prow[static_cast<int64_t>(split) * I + t] = count;
}

template <int L, typename TY, typename TA>
void run_plain(const Plan& P, const void* ycm, int64_t ldy, const uint64_t* wbits,
               const int32_t* cols, void* part, int32_t* prow, hipStream_t s) {
  dim3 grid(static_cast<unsigned>(ceil_div(P.I, 4)), static_cast<unsigned>(P.splits));
  k_gram_plain<L, TY, TA><<<grid, 256, 0, s>>>(static_cast<const TY*>(ycm), ldy, wbits, P.mw,
                                               cols, P.I, P.words_per_split,
                                               static_cast<TA*>(part), prow);
}

template <int L>
void dispatch_types(const Plan& P, const void* ycm, int64_t ldy, int y_dtype,
                    const uint64_t* wbits, const int32_t* cols, void* part, int32_t* prow,
                    hipStream_t s) {
  if (P.prec == RSM_GRAM_F64) {
    if (y_dtype == RSM_F32)
      run_plain<L, float, double>(P, ycm, ldy, wbits, cols, part, prow, s);
    else
      run_plain<L, double, double>(P, ycm, ldy, wbits, cols, part, prow, s);
  } else {
    if (y_dtype == RSM_F32)
      run_plain<L, float, float>(P, ycm, ldy, wbits, cols, part, prow, s);
    else
      run_plain<L, double, float>(P, ycm, ldy, wbits, cols, part, prow, s);
  }
}

}  // namespace

void launch_gram(const Plan& P, const void* ycm, int64_t ldy, int y_dtype,
                 const uint64_t* wbits, const int32_t* cols, void* part, int32_t* prow,
                 hipStream_t s) {
  if (P.I == 0) return;
  switch (P.l) {
#define RSM_GRAM_CASE(LL) \
  case LL:                \
    dispatch_types<LL>(P, ycm, ldy, y_dtype, wbits, cols, part, prow, s); \
    break;
    RSM_GRAM_CASE(2) RSM_GRAM_CASE(3) RSM_GRAM_CASE(4) RSM_GRAM_CASE(5) RSM_GRAM_CASE(6)
    RSM_GRAM_CASE(7) RSM_GRAM_CASE(8) RSM_GRAM_CASE(9) RSM_GRAM_CASE(10) RSM_GRAM_CASE(11)
    RSM_GRAM_CASE(12) RSM_GRAM_CASE(13) RSM_GRAM_CASE(14) RSM_GRAM_CASE(15)
    RSM_GRAM_CASE(16) RSM_GRAM_CASE(17)
#undef RSM_GRAM_CASE
    default:
      break;
  }
}

}  // namespace rsm
