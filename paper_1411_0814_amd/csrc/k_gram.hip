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
#include <algorithm>

#include "device_util.hpp"
#include "rsm_internal.hpp"

namespace rsm {

namespace {

// ------------------------------------------------------------------ per-trial streamer

template <int L, typename TY, typename TA>
__global__ __launch_bounds__(256) void k_gram_plain(const ProbDesc* __restrict__ probs,
                                                    IdxList list) {
  constexpr int NG = L * (L + 1) / 2;
  const ProbDesc& P = probs[list.idx[blockIdx.z]];
  const int64_t I = P.I, mw = P.mw, ldy = P.ldy;
  const int lane = threadIdx.x & 63;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int split = blockIdx.y;
  if (t >= I || split >= P.splits) return;  // wave-uniform
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

// VEC: Y and its leading dimension are 16-byte aligned, so a chunk column is moved as
// 16-byte vectors; otherwise element by element (same layout in LDS).
template <int L, typename T, int NT, bool VEC>
__global__ __launch_bounds__(NT) void k_gram_tile(const ProbDesc* __restrict__ probs,
                                                  IdxList list) {
  constexpr int NG = L * (L + 1) / 2;
  using V = typename Vec16<T>::type;
  constexpr int kVN = Vec16<T>::kN;                 // elements per 16-byte vector
  constexpr int kVPC = kChunk / kVN;                // vectors per column of a chunk
  constexpr int kS = TileStride<T>::kValue;           // LDS elements per column
  constexpr int kVPS = kS / kVN;                      // 16-byte vectors per column stride
  constexpr int kMaxCols = static_cast<int>(kTileLdsBytes / (kS * sizeof(T)));
  constexpr int kMaxV = (kMaxCols * kVPC + NT - 1) / NT;
  constexpr int kMaxM = (kMaxCols + NT - 1) / NT;
  const ProbDesc& P = probs[list.idx[blockIdx.y]];
  const int groups = P.gram_groups, splits = P.splits;
  if (static_cast<int>(blockIdx.x) >= groups * splits) return;  // past this problem's work
  const int64_t m = P.m, I = P.I, ldy = P.ldy, mw32 = 2 * P.mw;
  const int n = static_cast<int>(P.n);
  const int n_pad = static_cast<int>(ceil_div(n, NT / kVPC) * (NT / kVPC));
  const int m_pad = static_cast<int>(ceil_div(n, NT) * NT);
  const int64_t chunks = ceil_div(m, kChunk), chunks_per_split = 2 * P.words_per_split;
  const bool xcd_map = splits % 8 == 0;
  auto Y = static_cast<RSM_GLOBAL const T*>(P.ycm);
  auto mask32 = reinterpret_cast<RSM_GLOBAL const uint32_t*>(P.wbits);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);                                   // [n_pad][kS]
  uint32_t* msk = reinterpret_cast<uint32_t*>(tile + static_cast<int64_t>(n_pad) * kS);  // [m_pad]

  // Workgroup -> (trial group, row split).  Workgroups are dispatched to the 8 XCDs
  // round-robin by id (the launch's x extent is a multiple of 8), so with xcd_map the ids
  // id = 8 k + x of XCD x enumerate all trial groups of split 8 (k / groups) + x before the
  // next split: the groups reading the same rows share that XCD's L2.
  const int id = blockIdx.x;
  int group, split;
  if (xcd_map) {
    const int x = id & 7, k = id >> 3;
    const int sl = k / groups;
    group = k - sl * groups;
    split = sl * 8 + x;
  } else {
    group = id % groups;
    split = id / groups;
  }
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

  // Chunk staging.  The tile holds n_pad >= n columns (n_pad a multiple of NT / kVPC) and
  // the mask row m_pad >= n words (a multiple of NT), so every thread moves exactly kv
  // vectors and km mask words per chunk: uniform trip counts, loads issued back to back.
  // Columns past n repeat column n - 1 (valid addresses, never read back).  Vector k of
  // thread tid is column tid / kVPC + k * (NT / kVPC), rows kVN * (tid % kVPC) + [0, kVN).
  static_assert(NT % kVPC == 0, "threads must cover whole columns");
  const int kv = n_pad * kVPC / NT;
  const int km = m_pad / NT;
  const int c0 = tid / kVPC;
  const int vpart = (tid % kVPC) * kVN;
  V vreg[kMaxV];
  uint32_t mreg[kMaxM];
  auto load_chunk = [&](int64_t ch) {
    const int64_t r0 = ch * kChunk;
    if (VEC && r0 + kChunk <= m) {
#pragma unroll
      for (int k = 0; k < kMaxV; ++k) {
        if (k < kv) {
          const int c = min(c0 + k * (NT / kVPC), n - 1);
          vreg[k] = *reinterpret_cast<RSM_GLOBAL const V*>(Y + static_cast<int64_t>(c) * ldy + r0 + vpart);
        }
      }
    } else if (r0 + kChunk <= m) {  // unaligned columns: element loads, all issued first
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
  };
  auto store_chunk = [&]() {
    V* tv = reinterpret_cast<V*>(tile) + c0 * kVPS + (tid % kVPC);
#pragma unroll
    for (int k = 0; k < kMaxV; ++k)
      if (k < kv) tv[k * (NT / kVPC) * kVPS] = vreg[k];
#pragma unroll
    for (int k = 0; k < kMaxM; ++k)
      if (k < km) msk[tid + k * NT] = mreg[k];
  };

  if (ch0 < ch1) load_chunk(ch0);
  for (int64_t ch = ch0; ch < ch1; ++ch) {
    __syncthreads();
    store_chunk();
    __syncthreads();
    if (ch + 1 < ch1) load_chunk(ch + 1);
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

template <int L, typename T, bool VEC>
void run_tile(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  constexpr int NT = tile_threads(L, sizeof(T));
  constexpr int kVPC = kChunk / Vec16<T>::kN;
  size_t lds = 0;
  int wgs = 0;
  for (int k = 0; k < g.count; ++k) {
    const int n = static_cast<int>(h[k]->n);
    const int n_pad = static_cast<int>(ceil_div(n, NT / kVPC) * (NT / kVPC));
    const int m_pad = static_cast<int>(ceil_div(n, NT) * NT);
    lds = std::max(lds, static_cast<size_t>(n_pad) * TileStride<T>::kValue * sizeof(T) +
                            static_cast<size_t>(m_pad) * sizeof(uint32_t));
    wgs = std::max(wgs, h[k]->gram_wgs);
  }
  static bool attr_set = false;  // dynamic LDS above 64 KiB must be allowed explicitly
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram_tile<L, T, NT, VEC>),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(kTileLdsBytes + 8192));
    attr_set = true;
  }
  const unsigned grid = static_cast<unsigned>(ceil_div(wgs, 8) * 8);
  k_gram_tile<L, T, NT, VEC><<<dim3(grid, g.count), NT, lds, s>>>(d, g);
}

template <int L, typename TY, typename TA>
void run_plain(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  int64_t I = 0;
  int splits = 0;
  for (int k = 0; k < g.count; ++k) {
    I = std::max(I, h[k]->I);
    splits = std::max(splits, h[k]->splits);
  }
  const dim3 grid(static_cast<unsigned>(ceil_div(I, 4)), static_cast<unsigned>(splits), g.count);
  k_gram_plain<L, TY, TA><<<grid, 256, 0, s>>>(d, g);
}

template <int L>
void dispatch_types(const ProbDesc* d, const IdxList& g, const Plan* const* h, hipStream_t s) {
  const Plan& P = *h[0];  // the group shares l, y_dtype, precision and kernel choice
  if (P.prec == RSM_GRAM_F64) {
    if (P.y_dtype == RSM_F64 && P.tiled)
      P.gram_vec ? run_tile<L, double, true>(d, g, h, s) : run_tile<L, double, false>(d, g, h, s);
    else if (P.y_dtype == RSM_F32)
      run_plain<L, float, double>(d, g, h, s);
    else
      run_plain<L, double, double>(d, g, h, s);
  } else {
    if (P.y_dtype == RSM_F32 && P.tiled)
      P.gram_vec ? run_tile<L, float, true>(d, g, h, s) : run_tile<L, float, false>(d, g, h, s);
    else if (P.y_dtype == RSM_F32)
      run_plain<L, float, float>(d, g, h, s);
    else
      run_plain<L, double, float>(d, g, h, s);
  }
}

}  // namespace

bool gram_tiled_ok(const Plan& P) {
  if (!P.tiled) return false;
  const bool same = (P.prec == RSM_GRAM_F64) == (P.y_dtype == RSM_F64);
  const size_t elem = (P.y_dtype == RSM_F64) ? 8 : 4;
  if (!same) return false;
  const size_t stride = (P.y_dtype == RSM_F64) ? TileStride<double>::kValue : TileStride<float>::kValue;
  return static_cast<size_t>(ceil_div(P.n, 64) * 64) * stride * elem <= kTileLdsBytes;
}

bool gram_vector_loads(const Plan& P, const void* ycm, int64_t ldy) {
  const size_t elem = (P.y_dtype == RSM_F64) ? 8 : 4;
  return (reinterpret_cast<uintptr_t>(ycm) % 16) == 0 && (static_cast<size_t>(ldy) * elem) % 16 == 0;
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
