// Steps a2 + a3: row qualification and the l x l Gram of every trial.
//
// For trial t with sorted columns C_t = {c_0 < ... < c_{l-1}} (method M1, Section III):
//   R_t = { i : W[i, c] = 1 for every c in C_t }            (logical AND of l mask bit-planes)
//   G_t = sum_{i in R_t} y_{i,C_t} y_{i,C_t}^T                (l(l+1)/2 unique entries)
// The minor right singular vectors of Z_t = Y[R_t, C_t] are the eigenvectors of G_t for its
// smallest eigenvalues (Section III; they are computed in k_minor.hip).
//
// Output: partial Grams over row splits, part[split][g][trial] with g enumerating
// (a, b), b <= a, row-major over the lower triangle, and partial row counts
// prow[split][trial].  k_minor sums the splits in FP64.  A split is a range of 64-row
// mask words [split * words_per_split, ...).
//
// Two kernels:
//  * k_gram_plain  — one wavefront per (trial, row split).  Each 64-row word ANDs l mask
//    words (scalar loads) and the lanes whose row qualifies load their l values (column-
//    major, coalesced) and accumulate.  Simple, but every trial streams its l columns
//    from HBM: traffic ~ I * l * m * 4 bytes.
//  * k_gram_tile   — the LDS-reuse kernel: a workgroup stages a 32-row x n-column tile of Y
//    (and the tile's mask words) in LDS once and every thread — one trial each — gathers
//    its qualifying rows from LDS.  HBM/L2 traffic drops to (trial groups) x |Y|.
//  * k_gram_dma    — the same for FP32 with 16-row chunks loaded straight into LDS (no
//    staging registers: more trials' accumulators fit, two workgroups share a CU), with
//    one chunk buffer or two (the next chunk's loads in flight during the sums).
//  * k_gram_bf16   — the tile kernel's staging with the products on the matrix cores.
#include <algorithm>

#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

// ------------------------------------------------------------------ per-trial streamer

// Staging every column of a chunk pays for all n columns whatever a trial keeps: per trial
// and 64-row word about 64 n 4 / NT bytes (the chunk, shared by the workgroup's NT trials).
// Loading a trial's qualifying values straight from Y pays about a cache line per value:
// 64 f l 64 bytes, f = rho^l the expected fraction of qualifying rows, rho the mask's
// density (its ones counted while packing it).  A problem gathers when that is the smaller:
// f l 16 NT < n.  The choice depends only on the problem, so a deterministic problem takes
// the same path alone and in any batch.  Called by whole wavefronts (lane k reads partial
// count k; their sum is exact).
__device__ __forceinline__ bool gram_gathers(const ProbDesc& P, int nt) {
  static_assert(kMaskOnesParts == 64, "one partial count per lane");
  const unsigned long long part = P.scal->mask_ones[threadIdx.x & 63];
  const double known = static_cast<double>(wave_sum<unsigned long long>(part));
  const double rho = known / (static_cast<double>(P.m) * static_cast<double>(P.n));
  const double f = rho > 0.0 ? exp(static_cast<double>(P.l) * log(rho)) : 0.0;
  return f * P.l * 16.0 * nt < static_cast<double>(P.n);
}

// Launch modes of the gathering kernel and of the kernel it pairs with (staging through
// LDS, through registers, or the per-trial streamer): every problem of the launch, or only
// the problems gram_gathers gives to that kernel (both kernels of a pair run with
// kModeAuto).
constexpr int kModeAll = 0, kModeAuto = 1;

template <int L, typename TY, typename TA>
__global__ __launch_bounds__(256) void k_gram_plain(const ProbDesc* __restrict__ probs,
                                                    IdxList list, int mode) {
  constexpr int NG = L * (L + 1) / 2;
  const ProbDesc& P = probs[list.idx[blockIdx.z]];
  const int64_t I = P.I, mw = P.mw, ldy = P.ldy;
  const int lane = threadIdx.x & 63;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int split = blockIdx.y;
  if (t >= I || split >= P.splits) return;  // wave-uniform
  if (mode == kModeAuto && gram_gathers(P, kGatherPlainThreads)) return;  // gathered instead
  const int64_t w0 = static_cast<int64_t>(split) * P.words_per_split;
  const int64_t w1 = (w0 + P.words_per_split < mw) ? (w0 + P.words_per_split) : mw;
  auto Y = static_cast<RSM_GLOBAL const TY*>(P.ycm);

  RSM_GLOBAL const uint64_t* wcol[L];
  RSM_GLOBAL const TY* ycol[L];
  bool valid = true;
#pragma unroll
  for (int a = 0; a < L; ++a) {
    const int c = static_cast<int>(uniform_u32(static_cast<uint32_t>(P.cols[t * L + a])));
    valid &= (c >= 0);
    const int cc = c < 0 ? 0 : c;
    wcol[a] = P.wbits + static_cast<int64_t>(cc) * mw;
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
        for (int a = 0; a < L; ++a) y[a] = static_cast<TA>(ycol[a][i]);
        int g = 0;
#pragma unroll
        for (int a = 0; a < L; ++a)
#pragma unroll
          for (int b = 0; b <= a; ++b) acc[g++] += y[a] * y[b];
      }
    }
  }

  RSM_GLOBAL TA* dst = static_cast<RSM_GLOBAL TA*>(P.part) + static_cast<int64_t>(split) * NG * I + t;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const TA v = wave_sum(acc[g]);
    if (lane == 0) dst[static_cast<int64_t>(g) * I] = v;
  }
  if (lane == 0) P.prow[static_cast<int64_t>(split) * I + t] = count;
}

// ------------------------------------------------------------------ LDS-tiled kernel
//
// Workgroup (trial group g, row split s): NT threads, thread = trial.  The split's rows are
// walked in chunks of 32: the chunk's Y values for ALL n columns (column-major, 32 per
// column) and its 32-bit mask words (one per column) are staged in LDS; every thread ANDs
// its l mask words and, for each set bit, gathers its l values from LDS and accumulates
// the l(l+1)/2 products.  The next chunk is loaded into registers (16-byte vectors) while
// the current one is processed.  Global traffic is (trial groups) x (m n) elements instead
// of I l m; the rest is LDS traffic proportional to the qualifying rows only.

constexpr int kChunk = 32;

// LDS column stride of the tile, in elements: the chunk's 32 rows plus padding that keeps
// 16-byte alignment and spreads different columns over different LDS banks.
template <typename T>
struct TileStride;
template <>
struct TileStride<float> {
  static constexpr int kValue = 36;
};
template <>
struct TileStride<double> {
  static constexpr int kValue = 34;
};

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int kN = 4;
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int kN = 2;
};

// Stages 32-row chunks of Y (all n columns) and their mask words from global memory into
// registers and from registers into the LDS tile.  The tile holds n_pad >= n columns
// (n_pad a multiple of NT / kVPC) and the mask row m_pad >= n words (a multiple of NT), so
// every thread moves exactly kv vectors and km mask words per chunk: uniform trip counts,
// loads issued back to back.  Columns past n repeat column n - 1 (valid addresses, never
// read back).  Vector k of thread tid is column tid / kVPC + k * (NT / kVPC), rows
// kVN * (tid % kVPC) + [0, kVN).  Elements are loaded one by one (the compiler merges
// them into 16-byte loads, which gfx950 allows at 4-byte alignment), so columns need not
// be 16-byte aligned.
template <typename T, int NT>
struct ChunkStager {
  using V = typename Vec16<T>::type;
  static constexpr int kVN = Vec16<T>::kN;              // elements per 16-byte vector
  static constexpr int kVPC = kChunk / kVN;             // vectors per column of a chunk
  static constexpr int kS = TileStride<T>::kValue;      // LDS elements per column
  static constexpr int kVPS = kS / kVN;                 // 16-byte vectors per column stride
  static constexpr int kMaxCols = static_cast<int>(kTileLdsBytes / (kS * sizeof(T)));
  static constexpr int kMaxV = (kMaxCols * kVPC + NT - 1) / NT;
  static constexpr int kMaxM = (kMaxCols + NT - 1) / NT;
  static_assert(NT % kVPC == 0, "threads must cover whole columns");

  RSM_GLOBAL const T* Y;
  RSM_GLOBAL const uint32_t* mask32;
  int64_t m, ldy, mw32;
  int n, kv, km, c0, vpart, tid;
  V vreg[kMaxV];
  uint32_t mreg[kMaxM];

  __device__ __forceinline__ ChunkStager(const ProbDesc& P, int n_pad, int m_pad)
      : Y(static_cast<RSM_GLOBAL const T*>(P.ycm)),
        mask32(reinterpret_cast<RSM_GLOBAL const uint32_t*>(P.wbits)),
        m(P.m), ldy(P.ldy), mw32(2 * P.mw), n(static_cast<int>(P.n)),
        kv(n_pad * kVPC / NT), km(m_pad / NT), c0(static_cast<int>(threadIdx.x) / kVPC),
        vpart((static_cast<int>(threadIdx.x) % kVPC) * kVN), tid(threadIdx.x) {}

  __device__ __forceinline__ void load(int64_t ch) {
    const int64_t r0 = ch * kChunk;
    if (r0 + kChunk <= m) {
#pragma unroll
      for (int k = 0; k < kMaxV; ++k) {
        if (k < kv) {
          const int c = min(c0 + k * (NT / kVPC), n - 1);
          RSM_GLOBAL const T* src = Y + static_cast<int64_t>(c) * ldy + r0 + vpart;
          T tmp[kVN];
#pragma unroll
          for (int u = 0; u < kVN; ++u) tmp[u] = src[u];
          V v;
          __builtin_memcpy(&v, tmp, sizeof(V));
          vreg[k] = v;
        }
      }
    } else {  // ragged last chunk: rows past m read as zero
#pragma unroll
      for (int k = 0; k < kMaxV; ++k) {
        if (k < kv) {
          const int c = min(c0 + k * (NT / kVPC), n - 1);
          RSM_GLOBAL const T* src = Y + static_cast<int64_t>(c) * ldy + r0 + vpart;
          T tmp[kVN];
#pragma unroll
          for (int u = 0; u < kVN; ++u) tmp[u] = (r0 + vpart + u < m) ? src[u] : T(0);
          V v;
          __builtin_memcpy(&v, tmp, sizeof(V));
          vreg[k] = v;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) {
      if (k < km) {
        const int c = min(tid + k * NT, n - 1);
        mreg[k] = mask32[static_cast<int64_t>(c) * mw32 + ch];
      }
    }
  }

  __device__ __forceinline__ void store(T* tile, uint32_t* msk) const {
    V* tv = reinterpret_cast<V*>(tile) + c0 * kVPS + (tid % kVPC);
#pragma unroll
    for (int k = 0; k < kMaxV; ++k)
      if (k < kv) tv[k * (NT / kVPC) * kVPS] = vreg[k];
#pragma unroll
    for (int k = 0; k < kMaxM; ++k)
      if (k < km) msk[tid + k * NT] = mreg[k];
  }
};

// Workgroup -> (trial group, row split) of the tiled kernels.  Workgroups are dispatched to
// the 8 XCDs round-robin by id (the launch's x extent is a multiple of 8), so when the
// splits are a multiple of 8 the ids id = 8 k + x of XCD x enumerate all trial groups of
// split 8 (k / groups) + x before the next split: the groups reading the same rows share
// that XCD's L2.
__device__ __forceinline__ void tile_work(int groups, int splits, int& group, int& split) {
  const int id = blockIdx.x;
  if (splits % 8 == 0) {
    const int x = id & 7, k = id >> 3;
    const int sl = k / groups;
    group = k - sl * groups;
    split = sl * 8 + x;
  } else {
    group = id % groups;
    split = id / groups;
  }
}


template <int L, typename T, int NT>
__global__ __launch_bounds__(NT) void k_gram_tile(const ProbDesc* __restrict__ probs,
                                                  IdxList list, int mode) {
  constexpr int NG = L * (L + 1) / 2;
  using S = ChunkStager<T, NT>;
  constexpr int kS = S::kS;
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int groups = P.gram_groups, splits = P.splits;
  if (static_cast<int>(blockIdx.x) >= groups * splits) return;  // past this problem's work
  if (mode == kModeAuto && gram_gathers(P, NT)) return;           // k_gram_gather takes it
  const int64_t m = P.m, I = P.I;
  const int n = static_cast<int>(P.n);
  const int n_pad = static_cast<int>(ceil_div(n, NT / S::kVPC) * (NT / S::kVPC));
  const int m_pad = static_cast<int>(ceil_div(n, NT) * NT);
  const int64_t chunks = ceil_div(m, kChunk), chunks_per_split = 2 * P.words_per_split;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);                                   // [n_pad][kS]
  uint32_t* msk = reinterpret_cast<uint32_t*>(tile + static_cast<int64_t>(n_pad) * kS);  // [m_pad]
  int group, split;
  tile_work(groups, splits, group, split);
  const int tid = threadIdx.x;
  const int64_t t = static_cast<int64_t>(group) * NT + tid;
  const bool active = t < I;
  const int64_t ch0 = static_cast<int64_t>(split) * chunks_per_split;
  const int64_t ch1 = (ch0 + chunks_per_split < chunks) ? (ch0 + chunks_per_split) : chunks;

  int mc[L];  // column index; its tile values start at mc * kChunk
  bool valid = active;
#pragma unroll
  for (int a = 0; a < L; ++a) {
    int c = active ? P.cols[t * L + a] : 0;
    valid &= (c >= 0);
    mc[a] = c < 0 ? 0 : c;
  }
  T acc[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) acc[g] = T(0);
  int count = 0;

  S stage(P, n_pad, m_pad);
  if (ch0 < ch1) stage.load(ch0);
  for (int64_t ch = ch0; ch < ch1; ++ch) {
    __syncthreads();
    stage.store(tile, msk);
    __syncthreads();
    if (ch + 1 < ch1) stage.load(ch + 1);
    if (valid) {
      uint32_t q = 0xffffffffu;
#pragma unroll
      for (int a = 0; a < L; ++a) q &= msk[mc[a]];
      count += __popc(q);
      // walk the set bits starting at a lane-dependent row, so that the lanes of a
      // wavefront read different rows (and LDS banks) in the same step
      const int rot = (tid * 13) & (kChunk - 1);
      q = (q >> rot) | (q << ((kChunk - rot) & (kChunk - 1)));
      while (q) {
        const int i = (__ffs(q) - 1 + rot) & (kChunk - 1);
        q &= q - 1;
        T y[L];
#pragma unroll
        for (int a = 0; a < L; ++a) y[a] = tile[mc[a] * kS + i];
        int g = 0;
#pragma unroll
        for (int a = 0; a < L; ++a)
#pragma unroll
          for (int b = 0; b <= a; ++b) acc[g++] += y[a] * y[b];
      }
    }
  }
  if (active) {
    RSM_GLOBAL T* dst = static_cast<RSM_GLOBAL T*>(P.part) + static_cast<int64_t>(split) * NG * I + t;
#pragma unroll
    for (int g = 0; g < NG; ++g) dst[static_cast<int64_t>(g) * I] = acc[g];
    P.prow[static_cast<int64_t>(split) * I + t] = count;
  }
}

// ------------------------------------------------------------------ direct-to-LDS staging
//
// FP32 variant of k_gram_tile whose Y tile and mask words travel from global memory
// straight into LDS (global_load_lds_dword: lane k of a wavefront writes 4 bytes at
// base + 4 k), so no registers hold staged data and a workgroup's LDS holds one 16-row
// chunk of all n columns (n x 16 floats, at most 64 KiB): two workgroups share a CU and
// one's staging overlaps the other's Gram work.  Per chunk a wavefront instruction moves
// 4 columns x 16 rows of Y (column stride 16 floats) or the 32-bit mask words of 64
// columns (the word holds two chunks' bits).

constexpr int kDmaRows = 16;

__device__ __forceinline__ void lds_dma4(const void* src, void* dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 4, 0, 0);
}


// DB: two chunk buffers; the loads of chunk k + 1 are issued right after the barrier that
// publishes chunk k and land while chunk k is summed (one barrier per chunk).
// TA: the type of the sums.  With double, every product of two FP32 values is exact and
// only the FP64 additions round: the FP64 Gram of FP32 data.
template <int L, int NT, bool DB, typename TA>
__global__ __launch_bounds__(NT) void k_gram_dma(const ProbDesc* __restrict__ probs,
                                                 IdxList list, int mode) {
  constexpr int NG = L * (L + 1) / 2;
  constexpr int NW = NT / 64;
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int groups = P.gram_groups, splits = P.splits;
  if (static_cast<int>(blockIdx.x) >= groups * splits) return;  // past this problem's work
  if (mode == kModeAuto && gram_gathers(P, NT)) return;           // k_gram_gather takes it
  const int64_t m = P.m, I = P.I, ldy = P.ldy, mw32 = 2 * P.mw;
  const int n = static_cast<int>(P.n);
  const int n4 = (n + 3) & ~3, n64 = (n + 63) & ~63;
  const int64_t chunks = ceil_div(m, kDmaRows), chunks_per_split = 4 * P.words_per_split;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // per buffer: the tile [n4][16] floats, then the mask words [n64]
  const int buf_floats = n4 * kDmaRows + n64;
  float* const buf0 = reinterpret_cast<float*>(smem_raw);
  int group, split;
  tile_work(groups, splits, group, split);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t t = static_cast<int64_t>(group) * NT + tid;
  const bool active = t < I;
  const int64_t ch0 = static_cast<int64_t>(split) * chunks_per_split;
  const int64_t ch1 = (ch0 + chunks_per_split < chunks) ? (ch0 + chunks_per_split) : chunks;
  auto Y = static_cast<RSM_GLOBAL const float*>(P.ycm);
  auto wbits32 = reinterpret_cast<RSM_GLOBAL const uint32_t*>(P.wbits);

  int mc[L];
  bool valid = active;
#pragma unroll
  for (int a = 0; a < L; ++a) {
    int c = active ? P.cols[t * L + a] : 0;
    valid &= (c >= 0);
    mc[a] = c < 0 ? 0 : c;
  }
  TA acc[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) acc[g] = TA(0);
  int count = 0;
  const int rot = (tid * 13) & (kDmaRows - 1);
  const int colk = lane >> 4, rowk = lane & 15;

  // loads of chunk ch into the buffer at `dst` (tile, then mask words)
  auto issue = [&](int64_t ch, float* dst) {
    const int64_t r0 = ch * kDmaRows;
    const int64_t row = (r0 + rowk < m) ? (r0 + rowk) : (m - 1);  // past m: valid address, bit 0
    for (int g = wu; g < n4 / 4; g += NW) {
      const int c = (4 * g + colk < n) ? (4 * g + colk) : (n - 1);
      lds_dma4((const void*)(Y + static_cast<int64_t>(c) * ldy + row), dst + g * 64);
    }
    const int64_t word = ch >> 1;
    float* mdst = dst + n4 * kDmaRows;
    for (int g = wu; g < n64 / 64; g += NW) {
      const int c = (64 * g + lane < n) ? (64 * g + lane) : (n - 1);
      lds_dma4((const void*)(wbits32 + static_cast<int64_t>(c) * mw32 + word), mdst + g * 64);
    }
  };
  if (DB && ch0 < ch1) issue(ch0, buf0);
  for (int64_t ch = ch0; ch < ch1; ++ch) {
    float* cur = buf0;
    if constexpr (DB) {
      cur = buf0 + ((ch - ch0) & 1) * buf_floats;
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();  // chunk ch is in `cur`; every wave is done with the other buffer
      if (ch + 1 < ch1) issue(ch + 1, buf0 + ((ch + 1 - ch0) & 1) * buf_floats);
    } else {
      __syncthreads();  // the previous chunk's reads are done
      issue(ch, cur);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    const float* tile = cur;
    const uint32_t* msk = reinterpret_cast<const uint32_t*>(cur + n4 * kDmaRows);
    if (valid) {
      uint32_t q = 0xffffffffu;
#pragma unroll
      for (int a = 0; a < L; ++a) q &= msk[mc[a]];
      q = (q >> ((ch & 1) * kDmaRows)) & 0xffffu;
      count += __popc(q);
      q = ((q >> rot) | (q << (kDmaRows - rot))) & 0xffffu;
      while (q) {
        const int i = (__ffs(q) - 1 + rot) & (kDmaRows - 1);
        q &= q - 1;
        TA y[L];
#pragma unroll
        for (int a = 0; a < L; ++a) y[a] = static_cast<TA>(tile[mc[a] * kDmaRows + i]);
        int g = 0;
#pragma unroll
        for (int a = 0; a < L; ++a)
#pragma unroll
          for (int b = 0; b <= a; ++b) acc[g++] += y[a] * y[b];
      }
    }
  }
  if (active) {
    RSM_GLOBAL TA* dst = static_cast<RSM_GLOBAL TA*>(P.part) + static_cast<int64_t>(split) * NG * I + t;
#pragma unroll
    for (int g = 0; g < NG; ++g) dst[static_cast<int64_t>(g) * I] = acc[g];
    P.prow[static_cast<int64_t>(split) * I + t] = count;
  }
}

// ------------------------------------------------------------------ gathering
//
// For problems whose trials keep few rows: only the mask words travel into LDS (per 64-row
// word, the lo and hi 32-bit halves of every column's word as two planes, two buffers, the
// next word's loads in flight while the current one is used); each thread ANDs its trial's
// l words and loads the l values of each qualifying row straight from Y, the loads of the
// next qualifying row issued before the current row's products.  Same work split, partial
// sums and row counts as k_gram_dma.

// One qualifying row's products, summed in TA.
template <int L, typename TA, typename TY>
__device__ __forceinline__ void sum_row(const TY (&y)[L], TA (&acc)[L * (L + 1) / 2]) {
  TA v[L];
#pragma unroll
  for (int a = 0; a < L; ++a) v[a] = static_cast<TA>(y[a]);
  int g = 0;
#pragma unroll
  for (int a = 0; a < L; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) acc[g++] += v[a] * v[b];
}

template <int L, int NT, typename TA, typename TY>
__global__ __launch_bounds__(NT) void k_gram_gather(const ProbDesc* __restrict__ probs,
                                                    IdxList list, int mode) {
  constexpr int NG = L * (L + 1) / 2;
  constexpr int NW = NT / 64;
  // the pipelined loop holds a second row of values; kept only where the registers of
  // NT / 256 wavefronts per SIMD leave room for it (an estimate: the sums, the column
  // addresses and indices, the two rows, 48 for the rest)
  constexpr int kRegs = 512 / (NT / 256);
  constexpr int kYRegs = static_cast<int>(sizeof(TY) / 4);
  constexpr bool kPipe =
      NG * static_cast<int>(sizeof(TA) / 4) + 3 * L + 2 * kYRegs * L + 48 <= kRegs;
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int groups = P.gram_groups, splits = P.splits;
  if (static_cast<int>(blockIdx.x) >= groups * splits) return;  // past this problem's work
  if (mode == kModeAuto && !gram_gathers(P, NT)) return;          // the staging kernel takes it
  const int64_t I = P.I, ldy = P.ldy, mw = P.mw, mw32 = 2 * P.mw;
  const int n = static_cast<int>(P.n);
  const int n64 = (n + 63) & ~63;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // per buffer: lo words [n64], hi words [n64]
  uint32_t* const buf0 = reinterpret_cast<uint32_t*>(smem_raw);
  int group, split;
  tile_work(groups, splits, group, split);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t t = static_cast<int64_t>(group) * NT + tid;
  const bool active = t < I;
  const int64_t w0 = static_cast<int64_t>(split) * P.words_per_split;
  const int64_t w1 = (w0 + P.words_per_split < mw) ? (w0 + P.words_per_split) : mw;
  auto Y = static_cast<RSM_GLOBAL const TY*>(P.ycm);
  auto wbits32 = reinterpret_cast<RSM_GLOBAL const uint32_t*>(P.wbits);

  int mc[L];
  bool valid = active;
#pragma unroll
  for (int a = 0; a < L; ++a) {
    int c = active ? P.cols[t * L + a] : 0;
    valid &= (c >= 0);
    mc[a] = c < 0 ? 0 : c;
  }
  RSM_GLOBAL const TY* col[L];
#pragma unroll
  for (int a = 0; a < L; ++a) col[a] = Y + static_cast<int64_t>(mc[a]) * ldy;
  TA acc[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) acc[g] = TA(0);
  int count = 0;

  auto issue = [&](int64_t w, uint32_t* dst) {
    for (int g = wu; g < n64 / 64; g += NW) {
      const int c = (64 * g + lane < n) ? (64 * g + lane) : (n - 1);
      RSM_GLOBAL const uint32_t* src = wbits32 + static_cast<int64_t>(c) * mw32 + 2 * w;
      lds_dma4((const void*)src, dst + g * 64);
      lds_dma4((const void*)(src + 1), dst + n64 + g * 64);
    }
  };
  const int buf_words = 2 * n64;
  if (w0 < w1) issue(w0, buf0);
  for (int64_t w = w0; w < w1; ++w) {
    const uint32_t* cur = buf0 + ((w - w0) & 1) * buf_words;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();  // word w is in `cur`; every wave is done with the other buffer
    if (w + 1 < w1) issue(w + 1, buf0 + ((w + 1 - w0) & 1) * buf_words);
    if (!valid) continue;
    uint32_t lo = 0xffffffffu, hi = 0xffffffffu;
#pragma unroll
    for (int a = 0; a < L; ++a) {
      lo &= cur[mc[a]];
      hi &= cur[n64 + mc[a]];
    }
    uint64_t q = (static_cast<uint64_t>(hi) << 32) | lo;
    count += __popcll(q);
    if (!q) continue;
    if constexpr (kPipe) {
      // software pipeline over the qualifying rows: the next row's values are loaded while
      // the current row's products are summed
      int64_t row = w * 64 + (__ffsll(static_cast<unsigned long long>(q)) - 1);
      q &= q - 1;
      TY y[L];
#pragma unroll
      for (int a = 0; a < L; ++a) y[a] = col[a][row];
      while (true) {
        const bool more = q != 0;
        TY yn[L];
        if (more) {
          const int64_t rn = w * 64 + (__ffsll(static_cast<unsigned long long>(q)) - 1);
          q &= q - 1;
#pragma unroll
          for (int a = 0; a < L; ++a) yn[a] = col[a][rn];
        }
        sum_row<L, TA, TY>(y, acc);
        if (!more) break;
#pragma unroll
        for (int a = 0; a < L; ++a) y[a] = yn[a];
      }
    } else {
      while (q) {
        const int64_t row = w * 64 + (__ffsll(static_cast<unsigned long long>(q)) - 1);
        q &= q - 1;
        TY y[L];
#pragma unroll
        for (int a = 0; a < L; ++a) y[a] = col[a][row];
        sum_row<L, TA, TY>(y, acc);
      }
    }
  }
  if (active) {
    RSM_GLOBAL TA* dst = static_cast<RSM_GLOBAL TA*>(P.part) + static_cast<int64_t>(split) * NG * I + t;
#pragma unroll
    for (int g = 0; g < NG; ++g) dst[static_cast<int64_t>(g) * I] = acc[g];
    P.prow[static_cast<int64_t>(split) * I + t] = count;
  }
}

// ------------------------------------------------------------------ split-BF16 on MFMA
//
// The same staging, but the Gram products run on the matrix cores: each value x of a
// trial's qualifying rows is split into bf16 hi = rn(x) and lo = rn(x - hi), and
// G += Z_hi^T Z_hi + Z_hi^T Z_lo + Z_lo^T Z_hi with FP32 accumulation (the lo * lo term,
// about 2^-18 relative, is dropped).  One v_mfma_f32_16x16x32_bf16 covers one 32-row chunk
// of one trial (l <= 16 columns padded to 16): lane (i, g) = (lane % 16, lane / 16) holds
// rows 8 g .. 8 g + 7 of column i, which is both its A (Z^T) and its B (Z) operand; row i
// of the 16 x 16 result sits in lanes 16 (i / 4) + j, register i % 4.  Rows that do not
// qualify enter as zeros.  A wavefront owns 8 trials (32 accumulator registers), so a
// workgroup of 8 wavefronts covers 64 trials: with 16 trials the accumulators, the staging
// registers and the operands exceeded the 256 registers of two wavefronts per SIMD and the
// loop spilled to scratch.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBfTrialsPerWave = 8;
constexpr int kBfThreads = 512;
static_assert(kBfThreads / 64 * kBfTrialsPerWave == kBfTrialsPerGroup, "BF16 trial groups");

template <int L>
__global__ __launch_bounds__(kBfThreads) void k_gram_bf16(const ProbDesc* __restrict__ probs,
                                                          IdxList list) {
  static_assert(L <= 16, "one 16 x 16 tile per trial");
  constexpr int NT = kBfThreads;
  constexpr int NG = L * (L + 1) / 2;
  constexpr int TW = kBfTrialsPerWave;
  using S = ChunkStager<float, NT>;
  constexpr int kS = S::kS;
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int groups = P.gram_groups, splits = P.splits;
  if (static_cast<int>(blockIdx.x) >= groups * splits) return;
  const int64_t m = P.m, I = P.I;
  const int n = static_cast<int>(P.n);
  const int n_pad = static_cast<int>(ceil_div(n, NT / S::kVPC) * (NT / S::kVPC));
  const int m_pad = static_cast<int>(ceil_div(n, NT) * NT);
  const int64_t chunks = ceil_div(m, kChunk), chunks_per_split = 2 * P.words_per_split;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* tile = reinterpret_cast<float*>(smem_raw);
  uint32_t* msk = reinterpret_cast<uint32_t*>(tile + static_cast<int64_t>(n_pad) * kS);
  int* cnt = reinterpret_cast<int*>(msk + m_pad);  // [NT]: qualifying rows per trial
  int group, split;
  tile_work(groups, splits, group, split);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ci = lane & 15, kg = lane >> 4;
  const int64_t tb = static_cast<int64_t>(group) * (NT / 64) * TW + w * TW;  // first trial of this wavefront
  const int64_t ch0 = static_cast<int64_t>(split) * chunks_per_split;
  const int64_t ch1 = (ch0 + chunks_per_split < chunks) ? (ch0 + chunks_per_split) : chunks;

  // column of operand row ci for each trial, 16 bits each, two per register: kAbsent when
  // the trial is absent or invalid (it then contributes nothing), kPad on the padding rows
  // ci >= l
  constexpr uint32_t kAbsent = 0xffffu, kPad = 0xfffeu;
  uint32_t colp[TW / 2];
#pragma unroll
  for (int tt = 0; tt < TW; ++tt) {
    const int64_t t = tb + tt;
    int c = -2;
    if (ci < L) c = (t < I) ? P.cols[t * L + ci] : -1;
    int bad = (c == -1) ? 1 : 0;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) bad |= __shfl_xor(bad, off, 16);
    const uint32_t code = ci >= L ? kPad : (bad ? kAbsent : static_cast<uint32_t>(c));
    if (tt & 1)
      colp[tt / 2] |= code << 16;
    else
      colp[tt / 2] = code;
  }
  f32x4 acc[TW];
#pragma unroll
  for (int tt = 0; tt < TW; ++tt) acc[tt] = f32x4{0.f, 0.f, 0.f, 0.f};
  cnt[tid] = 0;

  S stage(P, n_pad, m_pad);
  if (ch0 < ch1) stage.load(ch0);
  for (int64_t ch = ch0; ch < ch1; ++ch) {
    __syncthreads();
    stage.store(tile, msk);
    __syncthreads();
    if (ch + 1 < ch1) stage.load(ch + 1);
#pragma unroll
    for (int tt = 0; tt < TW; ++tt) {
      const uint32_t code = (colp[tt / 2] >> (16 * (tt & 1))) & 0xffffu;
      const int c = code < kPad ? static_cast<int>(code) : -1;
      uint32_t q = c >= 0 ? msk[c] : (code == kPad ? 0xffffffffu : 0u);
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) q &= __shfl_xor(q, off, 16);
      const uint32_t bits = (q >> (8 * kg)) & 0xffu;
      const float* src = tile + (c >= 0 ? c : 0) * kS + 8 * kg;
      const float4 xa = *reinterpret_cast<const float4*>(src);
      const float4 xb = *reinterpret_cast<const float4*>(src + 4);
      const float xv[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
      bf16x8 hi, lo;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float x = (c >= 0 && ((bits >> k) & 1u)) ? xv[k] : 0.0f;
        const __bf16 h = static_cast<__bf16>(x);
        hi[k] = h;
        lo[k] = static_cast<__bf16>(x - static_cast<float>(h));
      }
      acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi, hi, acc[tt], 0, 0, 0);
      acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi, lo, acc[tt], 0, 0, 0);
      acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo, hi, acc[tt], 0, 0, 0);
      if (lane == 0) cnt[w * TW + tt] += __popc(q);
      // at most four trials' operands in flight (the scheduler would otherwise hoist the
      // loads of all of them and spill)
      if ((tt & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();
  RSM_GLOBAL float* part = static_cast<RSM_GLOBAL float*>(P.part) + static_cast<int64_t>(split) * NG * I;
#pragma unroll
  for (int tt = 0; tt < TW; ++tt) {
    const int64_t t = tb + tt;
    if (t >= I) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * kg + v, j = ci;
      if (i < L && j <= i) part[static_cast<int64_t>(i * (i + 1) / 2 + j) * I + t] = acc[tt][v];
    }
    if (lane == 0) P.prow[static_cast<int64_t>(split) * I + t] = cnt[w * TW + tt];
  }
}

template <int L, typename T>
size_t tile_lds(const Plan& P, int NT, size_t extra_per_thread) {
  constexpr int kVPC = kChunk / Vec16<T>::kN;
  const int n = static_cast<int>(P.n);
  const int n_pad = static_cast<int>(ceil_div(n, NT / kVPC) * (NT / kVPC));
  const int m_pad = static_cast<int>(ceil_div(n, NT) * NT);
  return static_cast<size_t>(n_pad) * TileStride<T>::kValue * sizeof(T) +
         static_cast<size_t>(m_pad) * sizeof(uint32_t) + NT * extra_per_thread;
}

// Largest trial count per workgroup built for the tiled kernel: 512 threads leave 128
// registers per thread, enough for the l(l+1)/2 accumulators up to these l; 256 is always
// built.
template <int L, typename T>
constexpr bool tile_has_512() {
  return sizeof(T) == 4 ? L <= 10 : L <= 6;
}

template <int L, typename T, int NT>
void run_tile_nt(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s,
                 int mode = kModeAll) {
  size_t lds = 0;
  int wgs = 0;
  for (int k = 0; k < g.count; ++k) {
    lds = std::max(lds, tile_lds<L, T>(*h[k], NT, 0));
    wgs = std::max(wgs, h[k]->gram_wgs);
  }
  static bool attr_set = false;  // dynamic LDS above 64 KiB must be allowed explicitly
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram_tile<L, T, NT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(kTileLdsBytes + 8192));
    attr_set = true;
  }
  const unsigned grid = static_cast<unsigned>(ceil_div(wgs, 8) * 8);
  k_gram_tile<L, T, NT><<<dim3(grid, g.count), NT, lds, s>>>(d, g, mode);
}

template <int L, int NT, bool DB, typename TA = float>
void run_dma(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s,
             int mode = kModeAll) {
  size_t lds = 0;
  int wgs = 0;
  for (int k = 0; k < g.count; ++k) {
    const size_t n = static_cast<size_t>(h[k]->n);
    const size_t one = ((n + 3) & ~size_t(3)) * kDmaRows * 4 + ((n + 63) & ~size_t(63)) * 4;
    lds = std::max(lds, DB ? 2 * one : one);
    wgs = std::max(wgs, h[k]->gram_wgs);
  }
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram_dma<L, NT, DB, TA>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 156 * 1024);
    attr_set = true;
  }
  const unsigned grid = static_cast<unsigned>(ceil_div(wgs, 8) * 8);
  k_gram_dma<L, NT, DB, TA><<<dim3(grid, g.count), NT, lds, s>>>(d, g, mode);
}

template <int L, int NT, typename TA, typename TY = float>
void run_gather(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s,
                int mode) {
  size_t lds = 0;
  int wgs = 0;
  for (int k = 0; k < g.count; ++k) {
    const size_t n64 = (static_cast<size_t>(h[k]->n) + 63) & ~size_t(63);
    lds = std::max(lds, 2 * 2 * n64 * sizeof(uint32_t));
    wgs = std::max(wgs, h[k]->gram_wgs);
  }
  const unsigned grid = static_cast<unsigned>(ceil_div(wgs, 8) * 8);
  k_gram_gather<L, NT, TA, TY><<<dim3(grid, g.count), NT, lds, s>>>(d, g, mode);
}

// The straight-to-LDS kernels of FP32 data with sums of type TA: kernel DMA2 stages every
// problem, GATHER gathers every problem, AUTO runs both, each taking the problems
// gram_gathers gives it.
template <int L, int NT, typename TA>
void run_fp32_data(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  const int kern = h[0]->gram_kernel;
  if (kern != RSM_GRAM_KERNEL_GATHER)
    run_dma<L, NT, true, TA>(d, g, h, s, kern == RSM_GRAM_KERNEL_AUTO ? kModeAuto : kModeAll);
  if (kern != RSM_GRAM_KERNEL_DMA2)
    run_gather<L, NT, TA>(d, g, h, s, kern == RSM_GRAM_KERNEL_AUTO ? kModeAuto : kModeAll);
}

// Largest trial count per workgroup of the double-buffered kernel: 1024 threads leave 128
// registers, enough for the accumulators up to l = 12.
template <int L>
constexpr bool dma_has_1024() {
  return L <= 12;
}

// The group shares its trials per workgroup (part of the launch key).
template <int L, typename T>
void run_tile(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (h[0]->gram_kernel == RSM_GRAM_KERNEL_DMA) {
      if (h[0]->gram_threads == 512)
        run_dma<L, 512, false>(d, g, h, s);
      else
        run_dma<L, 256, false>(d, g, h, s);
      return;
    }
    const int kern = h[0]->gram_kernel;
    if (kern == RSM_GRAM_KERNEL_DMA2 || kern == RSM_GRAM_KERNEL_GATHER ||
        kern == RSM_GRAM_KERNEL_AUTO) {
      if constexpr (dma_has_1024<L>()) {
        if (h[0]->gram_threads == 1024) {
          run_fp32_data<L, 1024, float>(d, g, h, s);
          return;
        }
      }
      run_fp32_data<L, 512, float>(d, g, h, s);
      return;
    }
  }
  // FP64 data: the register-staged kernel (REGS), the gathering one (GATHER), or both,
  // each taking the problems gram_gathers gives it (AUTO)
  const int kern = h[0]->gram_kernel;
  const int mode = kern == RSM_GRAM_KERNEL_AUTO ? kModeAuto : kModeAll;
  if constexpr (tile_has_512<L, T>()) {
    if (h[0]->gram_threads == 512) {
      if (kern != RSM_GRAM_KERNEL_GATHER) run_tile_nt<L, T, 512>(d, g, h, s, mode);
      if constexpr (sizeof(T) == 8)
        if (kern != RSM_GRAM_KERNEL_REGS) run_gather<L, 512, double, double>(d, g, h, s, mode);
      return;
    }
  }
  if (kern != RSM_GRAM_KERNEL_GATHER) run_tile_nt<L, T, 256>(d, g, h, s, mode);
  if constexpr (sizeof(T) == 8)
    if (kern != RSM_GRAM_KERNEL_REGS) run_gather<L, 256, double, double>(d, g, h, s, mode);
}

// FP32 Y, FP64 sums: the double-buffered direct-to-LDS kernel with FP64 accumulators
// (l(l+1) registers): 512 trials per workgroup while they fit two wavefronts per SIMD.
template <int L>
constexpr bool mixed_has_512() {
  return L <= 14;
}

template <int L>
void run_mixed(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  if constexpr (mixed_has_512<L>()) {
    if (h[0]->gram_threads == 512) {
      run_fp32_data<L, 512, double>(d, g, h, s);
      return;
    }
  }
  run_fp32_data<L, 256, double>(d, g, h, s);
}

template <int L>
void run_bf16(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  if constexpr (L <= 16) {
    size_t lds = 0;
    int wgs = 0;
    for (int k = 0; k < g.count; ++k) {
      lds = std::max(lds, tile_lds<L, float>(*h[k], kBfThreads, sizeof(int)));
      wgs = std::max(wgs, h[k]->gram_wgs);
    }
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram_bf16<L>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                static_cast<int>(kTileLdsBytes + 8192));
      attr_set = true;
    }
    const unsigned grid = static_cast<unsigned>(ceil_div(wgs, 8) * 8);
    k_gram_bf16<L><<<dim3(grid, g.count), kBfThreads, lds, s>>>(d, g);
  }
}

template <int L, typename TY, typename TA>
void run_plain(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  int64_t I = 0;
  int splits = 0;
  for (int k = 0; k < g.count; ++k) {
    I = std::max(I, h[k]->I);
    splits = std::max(splits, h[k]->splits);
  }
  // AUTO: the gathering kernel takes the problems whose trials keep few rows
  const bool pair = h[0]->gram_kernel == RSM_GRAM_KERNEL_AUTO;
  const dim3 grid(static_cast<unsigned>(ceil_div(I, 4)), static_cast<unsigned>(splits), g.count);
  k_gram_plain<L, TY, TA><<<grid, 256, 0, s>>>(d, g, pair ? kModeAuto : kModeAll);
  if (pair) run_gather<L, kGatherPlainThreads, TA, TY>(d, g, h, s, kModeAuto);
}

template <int L>
void dispatch_types(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  const Plan& P = *h[0];  // the group shares l, y_dtype, precision and kernel choice
  if (P.prec == RSM_GRAM_BF16X2) {
    run_bf16<L>(d, g, h, s);  // make_plan admits it only for FP32 Y, l <= 16, tiled
  } else if (P.prec == RSM_GRAM_F64) {
    if (P.y_dtype == RSM_F64 && P.tiled)
      run_tile<L, double>(d, g, h, s);
    else if (P.y_dtype == RSM_F32 && P.tiled)
      run_mixed<L>(d, g, h, s);
    else if (P.y_dtype == RSM_F32)
      run_plain<L, float, double>(d, g, h, s);
    else
      run_plain<L, double, double>(d, g, h, s);
  } else {
    if (P.y_dtype == RSM_F32 && P.tiled)
      run_tile<L, float>(d, g, h, s);
    else if (P.y_dtype == RSM_F32)
      run_plain<L, float, float>(d, g, h, s);
    else
      run_plain<L, double, float>(d, g, h, s);
  }
}

}  // namespace

int gram_threads_built(int l, int prec, int y_dtype, int kernel, int* out) {
  if (prec == RSM_GRAM_BF16X2) {
    if (kernel != RSM_GRAM_KERNEL_REGS || y_dtype != RSM_F32 || l > 16) return 0;
    out[0] = kBfTrialsPerGroup;
    return 1;
  }
  const bool f64 = prec == RSM_GRAM_F64;
  const bool fp32_data_kernel = kernel == RSM_GRAM_KERNEL_DMA2 ||
                                kernel == RSM_GRAM_KERNEL_GATHER || kernel == RSM_GRAM_KERNEL_AUTO;
  if (f64 && y_dtype == RSM_F32) {  // FP64 sums of FP32 data: the straight-to-LDS kernels only
    if (!fp32_data_kernel) return 0;
    out[0] = 256;
    if (l <= 14) {
      out[1] = 512;
      return 2;
    }
    return 1;
  }
  if (f64 != (y_dtype == RSM_F64)) return 0;
  if (f64 && (kernel == RSM_GRAM_KERNEL_GATHER || kernel == RSM_GRAM_KERNEL_AUTO)) {
    out[0] = 256;  // FP64 data: as the register-staged kernel it pairs with
    if (l <= 6) {
      out[1] = 512;
      return 2;
    }
    return 1;
  }
  if (kernel == RSM_GRAM_KERNEL_DMA) {
    if (f64) return 0;
    out[0] = 256;
    out[1] = 512;
    return 2;
  }
  if (fp32_data_kernel) {
    if (f64) return 0;
    out[0] = 512;
    if (l <= 12) {
      out[1] = 1024;
      return 2;
    }
    return 1;
  }
  out[0] = 256;
  if (l <= (f64 ? 6 : 10)) {
    out[1] = 512;
    return 2;
  }
  return 1;
}

bool gram_tiled_ok(const Plan& P) {
  if (!P.tiled) return false;
  const bool f64 = P.y_dtype == RSM_F64;
  if (f64 && P.prec != RSM_GRAM_F64) return false;  // FP64 data has no FP32 Gram kernel
  const size_t elem = f64 ? 8 : 4;
  const size_t stride = f64 ? TileStride<double>::kValue : TileStride<float>::kValue;
  return static_cast<size_t>(ceil_div(P.n, 64) * 64) * stride * elem <= kTileLdsBytes;
}

void launch_gram(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  if (!g.count) return;
  switch (h[0]->l) {
#define RSM_GRAM_CASE(LL) \
  case LL:                \
    dispatch_types<LL>(d, g, h, s); \
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
