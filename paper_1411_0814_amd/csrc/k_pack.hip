// Step a0 (ingest) and a1 (subset draw).
//  * Mask W (bytes, either storage order) -> column bit-planes: word w of column j holds
//    bit k = (W[64 w + k, j] != 0); rows past m are zero.  This is the "logical
//    comparisons on W" of the paper's Section IV-A done 64 rows per instruction.
//  * Y row-major -> column-major copy (Y is read in place when already column-major).
//  * C_t for every trial: Philox4x64-10 + Floyd (or a caller-supplied list, validated).
#include <algorithm>

#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

// Column-major W: one thread per (column, 64-row word) of problem list.idx[blockIdx.y].
// Each workgroup adds the ones of its words to one of the problem's partial counts of known
// entries.
__global__ __launch_bounds__(256) void k_pack_mask_colmajor(const ProbDesc* __restrict__ probs,
                                                            IdxList list) {
  __shared__ unsigned long long wave_ones[4];
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t m = P.m, n = P.n, mw = P.mw;
  if (static_cast<int64_t>(blockIdx.x) * blockDim.x >= n * mw) return;  // whole workgroup
  const int64_t gid0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool in = gid0 < n * mw;
  const int64_t gid = in ? gid0 : 0;
  const int64_t j = gid / mw;
  const int64_t w = gid - j * mw;
  const int64_t i0 = w * 64;
  RSM_GLOBAL const uint8_t* src = P.W + j * P.ldw + i0;
  const int sh = static_cast<int>(reinterpret_cast<uintptr_t>(src) & 7u);
  uint64_t word = 0;
  const bool full = (i0 + 64 <= m);
  if (full && sh == 0) {
    auto s8 = reinterpret_cast<RSM_GLOBAL const uint64_t*>(src);
    uint64_t x[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) x[b] = s8[b];
#pragma unroll
    for (int b = 0; b < 8; ++b) word |= static_cast<uint64_t>(nonzero_bytes_to_bits(x[b])) << (8 * b);
  } else if (full && i0 >= 8 && i0 + 72 <= m) {
    // unaligned column: the 9 aligned words covering [src, src + 64) lie inside this column
    auto s8 = reinterpret_cast<RSM_GLOBAL const uint64_t*>(src - sh);
    uint64_t x[9];
#pragma unroll
    for (int b = 0; b < 9; ++b) x[b] = s8[b];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t v = (x[b] >> (8 * sh)) | (x[b + 1] << (64 - 8 * sh));
      word |= static_cast<uint64_t>(nonzero_bytes_to_bits(v)) << (8 * b);
    }
  } else {  // first or last word of an unaligned column, or the ragged tail: bytes
    const int cnt = full ? 64 : static_cast<int>(m - i0);
    uint8_t x[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) x[k] = src[k < cnt ? k : 0];
#pragma unroll
    for (int k = 0; k < 64; ++k) word |= static_cast<uint64_t>(k < cnt && x[k] != 0) << k;
  }
  if (in) P.wbits[j * mw + w] = word;
  const unsigned long long ones =
      wave_sum<unsigned long long>(in ? static_cast<unsigned long long>(__popcll(word)) : 0ull);
  if ((threadIdx.x & 63) == 0) wave_ones[threadIdx.x >> 6] = ones;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long tot = wave_ones[0] + wave_ones[1] + wave_ones[2] + wave_ones[3];
    if (tot) atomicAdd(&P.scal->mask_ones[blockIdx.x % kMaskOnesParts], tot);
  }
}

// Row-major W: a 64-row x 64-column byte tile through LDS, one thread per output word.
// Grid (row words, column tiles, problems).
__global__ __launch_bounds__(256) void k_pack_mask_rowmajor(const ProbDesc* __restrict__ probs,
                                                            IdxList list) {
  __shared__ uint8_t tile[64][65];
  const ProbDesc& P = probs[list.idx[blockIdx.z]];
  const int64_t m = P.m, n = P.n, mw = P.mw;
  const int64_t w = blockIdx.x;  // row word
  const int64_t j0 = static_cast<int64_t>(blockIdx.y) * 64;
  if (w >= mw || j0 >= n) return;
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const int rr = e / 64, cc = e % 64;
    const int64_t i = w * 64 + rr, j = j0 + cc;
    tile[rr][cc] = (i < m && j < n) ? (P.W[i * P.ldw + j] != 0) : 0;
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // the first wavefront, whole
    const int64_t j = j0 + threadIdx.x;
    uint64_t word = 0;
    if (j < n) {
      for (int rr = 0; rr < 64; ++rr) word |= static_cast<uint64_t>(tile[rr][threadIdx.x]) << rr;
      P.wbits[j * mw + w] = word;
    }
    const unsigned long long ones =
        wave_sum<unsigned long long>(static_cast<unsigned long long>(__popcll(word)));
    if (threadIdx.x == 0 && ones)
      atomicAdd(&P.scal->mask_ones[(blockIdx.x + blockIdx.y) % kMaskOnesParts], ones);
  }
}

// Row-major Y -> column-major (same element type), 64 x 64 tiles through LDS.
// Grid (row tiles, column tiles, problems).
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const ProbDesc* __restrict__ probs,
                                                   IdxList list) {
  __shared__ T tile[64][65];
  const ProbDesc& P = probs[list.idx[blockIdx.z]];
  const int64_t m = P.m, n = P.n;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int64_t j0 = static_cast<int64_t>(blockIdx.y) * 64;
  if (i0 >= m || j0 >= n) return;
  auto src = static_cast<RSM_GLOBAL const T*>(P.Yin);
  auto dst = static_cast<RSM_GLOBAL T*>(P.ycm);
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const int rr = e / 64, cc = e % 64;
    const int64_t i = i0 + rr, j = j0 + cc;
    tile[rr][cc] = (i < m && j < n) ? src[i * P.ldy_in + j] : T(0);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const int cc = e / 64, rr = e % 64;
    const int64_t i = i0 + rr, j = j0 + cc;
    if (i < m && j < n) dst[j * P.ldy + i] = tile[rr][cc];
  }
}

// C_t for t = t0 + k, k = 0..I-1: one thread per trial (method M2: the row subsets S_t,
// drawn the same way from [0, m)).  Caller-supplied subsets are copied instead; an
// unsorted or out-of-range one is replaced by the marker -1 in its first slot (the trial
// is then rejected) and reported.
__global__ void k_subsets(const ProbDesc* __restrict__ probs, IdxList list) {
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= P.I) return;
  const int n = static_cast<int>(P.rows_first ? P.m : P.n), l = P.l;
  if (P.user_subsets) {
    bool ok = true;
    int prev = -1;
    for (int a = 0; a < l; ++a) {
      const int c = P.user_subsets[k * l + a];
      ok &= (c > prev) && (c < n);
      prev = c;
    }
    for (int a = 0; a < l; ++a) P.cols[k * l + a] = ok ? P.user_subsets[k * l + a] : -1;
    if (!ok) atomicOr((uint32_t*)&P.info->warn, static_cast<uint32_t>(RSM_W_BAD_SUBSET));
    return;
  }
  int c[RSM_MAX_L];
  draw_subset<RSM_MAX_L>(P.seed, static_cast<uint64_t>(P.t0 + k), n, l, c);
#pragma unroll
  for (int a = 0; a < RSM_MAX_L; ++a)
    if (a < l) P.cols[k * l + a] = c[a];
}

// N = 0 (unless the problem accumulates into a given N).  Grid (blocks, problems).
__global__ void k_zero_N(const ProbDesc* __restrict__ probs, IdxList list) {
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t count = P.n * P.n;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += stride)
    P.N[i] = 0.0;
}

// N <-> 64-bit fixed point with 2^-40 resolution, in place.  Grid (blocks, problems).
__global__ void k_n_fixed(const ProbDesc* __restrict__ probs, IdxList list, int to_fixed) {
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int64_t count = P.n * P.n;
  auto bits = reinterpret_cast<RSM_GLOBAL long long*>(P.N);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += stride) {
    if (to_fixed)
      bits[i] = llrint(P.N[i] * kFixedScale);
    else
      P.N[i] = static_cast<double>(bits[i]) * (1.0 / kFixedScale);
  }
}

__global__ void k_init_info(const ProbDesc* __restrict__ probs, IdxList list) {
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  RSM_GLOBAL rsm_info* info = P.info;
  RSM_GLOBAL DevScalars* scal = P.scal;
  if (threadIdx.x == 0) {
    info->warn = 0;
    info->uncovered = 0;
    info->accepted = 0;
    info->rows_total = 0;
    info->rows_underdetermined = 0;
    info->known = 0;
    info->eig_iterations = 0;
    info->reserved = 0;
    info->residual = 0.0;
    info->mu = 0.0;
    info->e = __builtin_nan("");
    scal->mu = 0.0;
    scal->lam_max = 0.0;
    scal->pivots = 0;
    scal->bar = 0;
    scal->ticket = 0;
    scal->stalled = 0;
  }
  for (int k = threadIdx.x; k < kMaskOnesParts; k += blockDim.x) scal->mask_ones[k] = 0;
  if (threadIdx.x < RSM_MAX_R + 1) info->lambda[threadIdx.x] = 0.0;
}

struct ProbDescPack {
  ProbDesc p[8];
  int count;
};

__global__ void k_put_prob_desc(ProbDescPack pack, ProbDesc* dst) {
  if (static_cast<int>(threadIdx.x) < pack.count) dst[threadIdx.x] = pack.p[threadIdx.x];
}

// Members of g whose plan satisfies `pred`, as a new list (plans in `hs`).
template <typename F>
IdxList select(const IdxList& g, const Plan* const* h, F pred, const Plan** hs) {
  IdxList out;
  for (int k = 0; k < g.count; ++k)
    if (pred(*h[k])) {
      hs[out.count] = h[k];
      out.idx[out.count++] = g.idx[k];
    }
  return out;
}

}  // namespace

void put_prob_descs(const ProbDesc* host, int count, ProbDesc* dev, hipStream_t s) {
  for (int k0 = 0; k0 < count; k0 += 8) {
    ProbDescPack pack;
    pack.count = (count - k0) < 8 ? (count - k0) : 8;
    for (int k = 0; k < pack.count; ++k) pack.p[k] = host[k0 + k];
    k_put_prob_desc<<<1, 64, 0, s>>>(pack, dev + k0);
  }
}

void launch_init_info(const ProbDesc* d, const IdxList& g, hipStream_t s) {
  if (g.count) k_init_info<<<dim3(1, g.count), 64, 0, s>>>(d, g);
}

void launch_pack(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  const Plan* hs[kLaunchMax];
  const IdxList wc = select(g, h, [](const Plan& P) { return P.w_layout == RSM_COL_MAJOR; }, hs);
  if (wc.count) {
    int64_t words = 0;
    for (int k = 0; k < wc.count; ++k) words = std::max<int64_t>(words, hs[k]->n * hs[k]->mw);
    k_pack_mask_colmajor<<<dim3(static_cast<unsigned>(ceil_div(words, 256)), wc.count), 256, 0, s>>>(d, wc);
  }
  const IdxList wr = select(g, h, [](const Plan& P) { return P.w_layout == RSM_ROW_MAJOR; }, hs);
  if (wr.count) {
    int64_t mw = 0, nt = 0;
    for (int k = 0; k < wr.count; ++k) {
      mw = std::max<int64_t>(mw, hs[k]->mw);
      nt = std::max<int64_t>(nt, ceil_div(hs[k]->n, 64));
    }
    k_pack_mask_rowmajor<<<dim3(static_cast<unsigned>(mw), static_cast<unsigned>(nt), wr.count), 256, 0, s>>>(d, wr);
  }
  for (int dt = RSM_F32; dt <= RSM_F64; ++dt) {
    const IdxList yr = select(g, h, [dt](const Plan& P) {
      return P.y_layout == RSM_ROW_MAJOR && P.y_dtype == dt; }, hs);
    if (!yr.count) continue;
    int64_t mt = 0, nt = 0;
    for (int k = 0; k < yr.count; ++k) {
      mt = std::max<int64_t>(mt, ceil_div(hs[k]->m, 64));
      nt = std::max<int64_t>(nt, ceil_div(hs[k]->n, 64));
    }
    const dim3 grid(static_cast<unsigned>(mt), static_cast<unsigned>(nt), yr.count);
    if (dt == RSM_F32)
      k_transpose<float><<<grid, 256, 0, s>>>(d, yr);
    else
      k_transpose<double><<<grid, 256, 0, s>>>(d, yr);
  }
}

void launch_n_fixed(const ProbDesc* d, const IdxList& g, const Plan* const* h, bool to_fixed,
                    hipStream_t s) {
  if (!g.count) return;
  int64_t nn = 0;
  for (int k = 0; k < g.count; ++k) nn = std::max<int64_t>(nn, h[k]->n * h[k]->n);
  const int64_t blocks = ceil_div(nn, 256);
  k_n_fixed<<<dim3(static_cast<unsigned>(blocks < 1024 ? blocks : 1024), g.count), 256, 0, s>>>(
      d, g, to_fixed ? 1 : 0);
}

void launch_subsets(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  const Plan* hs[kLaunchMax];
  const IdxList gs = select(g, h, [](const Plan& P) {
    return !(P.flags & RSM_FINALIZE_ONLY) && P.I > 0; }, hs);
  if (gs.count) {
    int64_t I = 0;
    for (int k = 0; k < gs.count; ++k) I = std::max<int64_t>(I, hs[k]->I);
    k_subsets<<<dim3(static_cast<unsigned>(ceil_div(I, 128)), gs.count), 128, 0, s>>>(d, gs);
  }
  const IdxList gz = select(g, h, [](const Plan& P) {
    return !(P.flags & RSM_FINALIZE_ONLY) && !(P.flags & RSM_N_ACCUMULATE); }, hs);
  if (gz.count) {
    int64_t nn = 0;
    for (int k = 0; k < gz.count; ++k) nn = std::max<int64_t>(nn, hs[k]->n * hs[k]->n);
    const int64_t blocks = ceil_div(nn, 256);
    k_zero_N<<<dim3(static_cast<unsigned>(blocks < 1024 ? blocks : 1024), gz.count), 256, 0, s>>>(d, gz);
  }
}

}  // namespace rsm
