// Step a0 (ingest) and a1 (subset draw).
//  * Mask W (bytes, either storage order) -> column bit-planes: word w of column j holds
//    bit k = (W[64 w + k, j] != 0); rows past m are zero.  This is the "logical
//    comparisons on W" of the paper's Section IV-A done 64 rows per instruction.
//  * Y row-major -> column-major copy (Y is read in place when already column-major).
//  * C_t for every trial: Philox4x64-10 + Floyd (or a caller-supplied list, validated).
#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

// 8 bytes -> 8 bits: bit k set iff byte k is nonzero.
__device__ __forceinline__ uint32_t nonzero_bytes_to_bits(uint64_t x) {
  const uint64_t lo7 = 0x7F7F7F7F7F7F7F7Full;
  uint64_t t = ((x & lo7) + lo7) | x;          // high bit of each byte = (byte != 0)
  t = (t >> 7) & 0x0101010101010101ull;        // one bit per byte, at bit 8k
  return static_cast<uint32_t>((t * 0x0102040810204080ull) >> 56);  // gather to bits 0..7
}

// Column-major W: one thread per (column, 64-row word).
__global__ void k_pack_mask_colmajor(const uint8_t* __restrict__ W, int64_t ldw, int64_t m,
                                     int64_t n, uint64_t* __restrict__ wbits, int64_t mw) {
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= n * mw) return;
  const int64_t j = gid / mw;
  const int64_t w = gid - j * mw;
  const int64_t i0 = w * 64;
  const uint8_t* src = W + j * ldw + i0;
  uint64_t word = 0;
  const bool full = (i0 + 64 <= m);
  if (full && ((reinterpret_cast<uintptr_t>(src) & 7u) == 0)) {
    const uint64_t* s8 = reinterpret_cast<const uint64_t*>(src);
#pragma unroll
    for (int b = 0; b < 8; ++b)
      word |= static_cast<uint64_t>(nonzero_bytes_to_bits(s8[b])) << (8 * b);
  } else {
    const int64_t cnt = full ? 64 : (m - i0);
    for (int64_t k = 0; k < cnt; ++k)
      if (src[k]) word |= 1ull << k;
  }
  wbits[j * mw + w] = word;
}

// Row-major W: a 64-row x 64-column byte tile through LDS, one thread per output word.
__global__ __launch_bounds__(256) void k_pack_mask_rowmajor(const uint8_t* __restrict__ W,
                                                            int64_t ldw, int64_t m, int64_t n,
                                                            uint64_t* __restrict__ wbits,
                                                            int64_t mw) {
  __shared__ uint8_t tile[64][65];
  const int64_t w = blockIdx.x;          // row word
  const int64_t j0 = static_cast<int64_t>(blockIdx.y) * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const int rr = e / 64, cc = e % 64;
    const int64_t i = w * 64 + rr, j = j0 + cc;
    tile[rr][cc] = (i < m && j < n) ? (W[i * ldw + j] != 0) : 0;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int64_t j = j0 + threadIdx.x;
    if (j < n) {
      uint64_t word = 0;
      for (int rr = 0; rr < 64; ++rr) word |= static_cast<uint64_t>(tile[rr][threadIdx.x]) << rr;
      wbits[j * mw + w] = word;
    }
  }
}

// Row-major Y -> column-major (same element type), 64 x 64 tiles through LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T* __restrict__ src, int64_t lds_,
                                                   int64_t m, int64_t n, T* __restrict__ dst,
                                                   int64_t ldd) {
  __shared__ T tile[64][65];
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int64_t j0 = static_cast<int64_t>(blockIdx.y) * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const int rr = e / 64, cc = e % 64;
    const int64_t i = i0 + rr, j = j0 + cc;
    tile[rr][cc] = (i < m && j < n) ? src[i * lds_ + j] : T(0);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    const int cc = e / 64, rr = e % 64;
    const int64_t i = i0 + rr, j = j0 + cc;
    if (i < m && j < n) dst[j * ldd + i] = tile[rr][cc];
  }
}

// C_t for t = t0 + k, k = 0..I-1: one thread per trial.
__global__ void k_subsets(uint64_t seed, int64_t t0, int64_t I, int n, int l,
                          int32_t* __restrict__ cols) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= I) return;
  int c[RSM_MAX_L];
  draw_subset<RSM_MAX_L>(seed, static_cast<uint64_t>(t0 + k), n, l, c);
#pragma unroll
  for (int a = 0; a < RSM_MAX_L; ++a)
    if (a < l) cols[k * l + a] = c[a];
}

// Caller-supplied subsets: copied; an unsorted or out-of-range row is replaced by the
// marker -1 in its first slot (the trial is then rejected) and reported.
__global__ void k_subsets_user(const int32_t* __restrict__ user, int64_t I, int n, int l,
                               int32_t* __restrict__ cols, rsm_info* info) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= I) return;
  bool ok = true;
  int prev = -1;
  for (int a = 0; a < l; ++a) {
    const int c = user[k * l + a];
    ok &= (c > prev) && (c < n);
    prev = c;
  }
  for (int a = 0; a < l; ++a) cols[k * l + a] = ok ? user[k * l + a] : -1;
  if (!ok) atomicOr(&info->warn, static_cast<uint32_t>(RSM_W_BAD_SUBSET));
}

__global__ void k_fill_zero(double* __restrict__ x, int64_t count) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += stride)
    x[i] = 0.0;
}

__global__ void k_init_info(rsm_info* info, DevScalars* scal) {
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
    scal->err_acc = 0.0;
    scal->pivots = 0;
    scal->pad = 0;
  }
  if (threadIdx.x < RSM_MAX_R + 1) info->lambda[threadIdx.x] = 0.0;
}

}  // namespace

void launch_init_info(rsm_info* info, DevScalars* scal, hipStream_t s) {
  k_init_info<<<1, 64, 0, s>>>(info, scal);
}

void launch_pack_mask(const uint8_t* W, int layout, int64_t ldw, int64_t m, int64_t n,
                      uint64_t* wbits, int64_t mw, hipStream_t s) {
  if (layout == RSM_COL_MAJOR) {
    const int64_t total = n * mw;
    k_pack_mask_colmajor<<<static_cast<unsigned>(ceil_div(total, 256)), 256, 0, s>>>(
        W, ldw, m, n, wbits, mw);
  } else {
    dim3 grid(static_cast<unsigned>(mw), static_cast<unsigned>(ceil_div(n, 64)));
    k_pack_mask_rowmajor<<<grid, 256, 0, s>>>(W, ldw, m, n, wbits, mw);
  }
}

void launch_pack_y(const void* Y, int dtype, int64_t ldy, int64_t m, int64_t n, void* ycm,
                   int64_t ldc, hipStream_t s) {
  dim3 grid(static_cast<unsigned>(ceil_div(m, 64)), static_cast<unsigned>(ceil_div(n, 64)));
  if (dtype == RSM_F32)
    k_transpose<float><<<grid, 256, 0, s>>>(static_cast<const float*>(Y), ldy, m, n,
                                            static_cast<float*>(ycm), ldc);
  else
    k_transpose<double><<<grid, 256, 0, s>>>(static_cast<const double*>(Y), ldy, m, n,
                                             static_cast<double*>(ycm), ldc);
}

void launch_subsets(const Plan& P, const int32_t* user, int32_t* cols, rsm_info* info,
                    hipStream_t s) {
  if (P.I == 0) return;
  const unsigned blocks = static_cast<unsigned>(ceil_div(P.I, 128));
  if (user)
    k_subsets_user<<<blocks, 128, 0, s>>>(user, P.I, static_cast<int>(P.n), P.l, cols, info);
  else
    k_subsets<<<blocks, 128, 0, s>>>(P.seed, P.t0, P.I, static_cast<int>(P.n), P.l, cols);
}

void launch_fill_zero(double* x, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  const int64_t blocks = ceil_div(count, 256);
  k_fill_zero<<<static_cast<unsigned>(blocks < 4096 ? blocks : 4096), 256, 0, s>>>(x, count);
}

}  // namespace rsm
