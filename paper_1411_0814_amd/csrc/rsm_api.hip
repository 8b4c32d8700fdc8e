// The C ABI of librsm (include/rsm.h): argument validation, the execution plan and
// workspace layout of each problem, and the launch sequence of steps a0..a7.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "rsm_internal.hpp"

namespace rsm {

namespace {

constexpr uint32_t kKnownFlags = RSM_ACCUMULATE_ONLY | RSM_FINALIZE_ONLY | RSM_N_ACCUMULATE |
                                 RSM_COMPUTE_ERROR | RSM_PLAIN_GRAM | RSM_DETERMINISTIC |
                                 RSM_ROWS_FIRST | RSM_SERIAL_STEPS;
constexpr size_t kAlign = 256;

size_t carve(size_t& cursor, size_t bytes) {
  const size_t off = cursor;
  cursor = align_up(cursor + bytes, kAlign);
  return off;
}

}  // namespace

int32_t make_plan(const rsm_problem& p, Plan& P) {
  P = Plan{};
  if (p.m < 1 || p.n < 2 || p.r < 1 || p.num_submatrices < 0 || p.trial_begin < 0 ||
      p.reserved != 0)
    return RSM_E_ARG;
  if ((p.flags & ~kKnownFlags) != 0) return RSM_E_ARG;
  if ((p.flags & RSM_ACCUMULATE_ONLY) && (p.flags & RSM_FINALIZE_ONLY)) return RSM_E_ARG;
  if (p.y_dtype != RSM_F32 && p.y_dtype != RSM_F64) return RSM_E_ARG;
  if (p.y_layout != RSM_COL_MAJOR && p.y_layout != RSM_ROW_MAJOR) return RSM_E_ARG;
  if (p.w_layout != RSM_COL_MAJOR && p.w_layout != RSM_ROW_MAJOR) return RSM_E_ARG;
  if (p.gram_prec != RSM_GRAM_F64 && p.gram_prec != RSM_GRAM_F32 &&
      p.gram_prec != RSM_GRAM_BF16X2)
    return RSM_E_ARG;
  const int64_t mn = p.m < p.n ? p.m : p.n;
  if (p.r >= mn) return RSM_E_ARG;
  const bool rows_first = p.flags & RSM_ROWS_FIRST;
  // l: columns per sub-matrix (M1) or rows per sub-matrix k (M2, rows first)
  const int l = p.l ? p.l : p.r + 1;
  if (l <= p.r || l > (rows_first ? p.m : p.n)) return RSM_E_ARG;
  int nvec = 0, min_rows = 0;
  if (rows_first) {
    // every trial gives |C_t| - r vectors; a trial counts with more than r columns
    if (p.nvec != 0) return RSM_E_ARG;
    min_rows = p.min_rows ? p.min_rows : p.r + 1;
    if (min_rows <= p.r) return RSM_E_ARG;
    if (p.gram_prec == RSM_GRAM_BF16X2 || (p.flags & RSM_PLAIN_GRAM) || p.m > 0x7fffffff)
      return RSM_E_UNSUPPORTED;
  } else {
    nvec = p.nvec ? p.nvec : l - p.r;
    if (nvec < 1 || nvec > l - p.r) return RSM_E_ARG;
    min_rows = p.min_rows ? p.min_rows : p.r;
    if (min_rows < 1) return RSM_E_ARG;
  }
  if (p.r > RSM_MAX_R || l > RSM_MAX_L || p.n > RSM_MAX_N) return RSM_E_UNSUPPORTED;
  // split-BF16 runs on the tiled MFMA kernel only: FP32 Y, l <= 16, the n-column tile in LDS
  if (p.gram_prec == RSM_GRAM_BF16X2 &&
      (p.y_dtype != RSM_F32 || l > 16 || (p.flags & RSM_PLAIN_GRAM) ||
       static_cast<size_t>(ceil_div(p.n, 64) * 64) * 36 * sizeof(float) > kTileLdsBytes))
    return RSM_E_UNSUPPORTED;

  P.m = p.m;
  P.n = p.n;
  P.r = p.r;
  P.l = l;
  P.nvec = nvec;
  P.min_rows = min_rows;
  P.I = p.num_submatrices;
  P.t0 = p.trial_begin;
  P.seed = p.seed;
  P.prec = p.gram_prec;
  P.flags = p.flags;
  P.y_dtype = p.y_dtype;
  P.y_layout = p.y_layout;
  P.w_layout = p.w_layout;
  P.mw = ceil_div(p.m, 64);
  P.rows_first = rows_first;
  P.nw = ceil_div(p.n, 64);
  P.ng = l * (l + 1) / 2;
  P.part_elem = (p.gram_prec == RSM_GRAM_F64) ? sizeof(double) : sizeof(float);
  P.eig_b = static_cast<int>((p.r + kEigPad) < p.n ? (p.r + kEigPad) : p.n);
  P.nb = static_cast<int>(ceil_div(p.n, kCholNB));
  int64_t nbp = 1;
  while (nbp < P.nb) nbp *= 2;
  P.npad = nbp * kCholNB;

  P.u_mfma = !(p.flags & RSM_ACCUMULATE_ONLY) && p.r >= kUMfmaMinR;

  // Gram kernel: LDS-tiled (Y tile shared by a group of trials) when the n-column tile fits
  // and the accumulation type matches Y's (split-BF16: FP32 Y), else the per-trial streamer
  P.tiled = !(p.flags & RSM_PLAIN_GRAM) && !rows_first;
  P.tiled = P.tiled && gram_tiled_ok(P);
  if (rows_first) {
    // the M1 Gram kernels do not run: one (unused) split
    P.gram_kernel = 0;
    P.gram_threads = 0;
    P.splits = 1;
    P.words_per_split = P.mw;
    P.gram_groups = 0;
    P.gram_wgs = 0;
  } else if (P.tiled) {
    P.gram_kernel = default_gram_kernel(P);
    set_gram_shape(P, default_gram_threads(P, P.gram_kernel), 0);
  } else {
    // the per-trial streamer, paired with the gathering kernel (each takes the problems the
    // mask's density gives it) unless the caller asked for the streamer alone
    P.gram_kernel = (p.flags & RSM_PLAIN_GRAM) ? 0 : RSM_GRAM_KERNEL_AUTO;
    set_gram_shape(P, 0, 0);
  }
  return RSM_OK;
}

// Staging of the tiled kernels when the tile table does not say otherwise: FP32 data loads
// straight into LDS with two chunk buffers (no staging registers, loads overlapping the
// sums), FP64 data through registers; for problems whose trials keep few rows, only the
// mask words are staged and the values gathered from Y (chosen per problem on the device).
// Split-BF16 stages through registers.
int builtin_gram_kernel(int l, int prec, int y_dtype) {
  (void)l;
  if (prec == RSM_GRAM_BF16X2) return RSM_GRAM_KERNEL_REGS;
  return RSM_GRAM_KERNEL_AUTO;
}

int default_gram_kernel(const Plan& P) { return builtin_gram_kernel(P.l, P.prec, P.y_dtype); }

// Whether `threads` trials per workgroup are built for this staging kernel.
bool threads_built(int l, int prec, int y_dtype, int kernel, int threads) {
  int built[8];
  const int nb = gram_threads_built(l, prec, y_dtype, kernel, built);
  for (int j = 0; j < nb; ++j)
    if (built[j] == threads) return true;
  return false;
}

// Trials per workgroup of the tiled kernels when the tile table does not say otherwise.
int default_gram_threads(const Plan& P, int kernel) {
  if (P.prec == RSM_GRAM_BF16X2) return kBfTrialsPerGroup;
  if (kernel == RSM_GRAM_KERNEL_DMA) return 256;
  if ((kernel == RSM_GRAM_KERNEL_GATHER || kernel == RSM_GRAM_KERNEL_AUTO) &&
      P.y_dtype == RSM_F64)
    return tile_threads(P.l, 8);  // FP64 data: as the register-staged kernel it pairs with
  if (kernel == RSM_GRAM_KERNEL_DMA2 || kernel == RSM_GRAM_KERNEL_GATHER ||
      kernel == RSM_GRAM_KERNEL_AUTO) {
    if (P.prec == RSM_GRAM_F64) return P.l <= 14 ? 512 : 256;  // FP64 sums of FP32 data
    return P.l <= 12 ? 1024 : 512;
  }
  return tile_threads(P.l, P.prec == RSM_GRAM_F64 ? 8 : 4);
}

// Row splits of the Gram step.  Tiled: `threads` trials per workgroup and `splits_hint`
// splits (chosen for a whole launch), or with splits_hint == 0 enough splits for about one
// workgroup per CU for this problem alone.  Per-trial streamer: enough wavefronts of
// (trial, split).
void set_gram_shape(Plan& P, int threads, int64_t splits_hint) {
  int64_t splits = 1;
  int64_t groups = 1;
  if (P.tiled) {
    P.gram_threads = threads;
    groups = ceil_div(P.I > 0 ? P.I : 1, threads);
    splits = splits_hint > 0 ? splits_hint : kTileTargetGroups / groups;
    if (splits < 1) splits = 1;
    if (splits >= 8) splits -= splits % 8;  // whole XCD rounds (see k_gram_tile)
  } else {
    P.gram_threads = 0;
    if (P.I > 0 && P.I < 8192) splits = ceil_div(8192, P.I);
    // the gathering kernel paired with the streamer takes its trials in groups, with
    // row splits for about four workgroups per CU (at most 16: the partial sums of every
    // split are written and reduced)
    if (P.gram_kernel == RSM_GRAM_KERNEL_AUTO) {
      groups = ceil_div(P.I > 0 ? P.I : 1, kGatherPlainThreads);
      const int64_t want = std::min<int64_t>(16, ceil_div(4 * kTileTargetGroups, groups));
      splits = std::max<int64_t>(splits, want);
    }
  }
  if (splits > P.mw) splits = P.mw;
  P.words_per_split = ceil_div(P.mw, splits);
  // the splits actually needed to cover mw words (never more than requested)
  P.splits = static_cast<int>(ceil_div(P.mw, P.words_per_split));
  P.gram_groups = static_cast<int>(groups);
  P.gram_wgs = P.gram_groups * P.splits;
}

// Workspace offsets of one problem (after its Gram shape is fixed).
void set_layout(Plan& P) {
  size_t cur = 0;
  P.off_scal = carve(cur, sizeof(DevScalars));
  P.off_wbits = carve(cur, static_cast<size_t>(P.n) * P.mw * sizeof(uint64_t));
  const size_t yelem = (P.y_dtype == RSM_F64) ? sizeof(double) : sizeof(float);
  P.off_ypack = (P.y_layout == RSM_ROW_MAJOR)
                    ? carve(cur, static_cast<size_t>(P.n) * P.m * yelem)
                    : ~size_t(0);
  P.off_cols = carve(cur, static_cast<size_t>(P.I) * P.l * sizeof(int32_t));
  P.off_part = carve(cur, static_cast<size_t>(P.splits) * P.I * P.ng * P.part_elem);
  P.off_prow = carve(cur, static_cast<size_t>(P.splits) * P.I * sizeof(int32_t));
  P.off_G = carve(cur, static_cast<size_t>(P.I) * P.ng * sizeof(double));
  P.off_rows = carve(cur, static_cast<size_t>(P.I) * sizeof(int32_t));
  P.off_mflag = carve(cur, static_cast<size_t>(P.I) * sizeof(int32_t));
  const size_t nn = static_cast<size_t>(P.n) * P.n * sizeof(double);
  P.off_N = carve(cur, nn);
  P.off_Nsym = carve(cur, nn);
  P.off_L = carve(cur, nn);
  const size_t pp = static_cast<size_t>(P.npad) * P.npad * sizeof(double);
  P.off_M = carve(cur, pp);
  P.off_Mt = carve(cur, pp);
  P.off_T = carve(cur, pp / 4);
  const size_t nbv = static_cast<size_t>(P.n) * P.eig_b * sizeof(double);
  P.off_X = carve(cur, nbv);
  P.off_Z = carve(cur, nbv);
  P.off_SP = carve(cur, static_cast<size_t>(sub_partials(P.n)) * sizeof(double));
  if (P.u_mfma) {
    P.off_ab = carve(cur, static_cast<size_t>(P.m) * (P.r * (P.r + 1) / 2 + P.r) * sizeof(double));
    P.off_abcnt = carve(cur, static_cast<size_t>(P.m) * sizeof(int32_t));
    P.off_kext = carve(cur, static_cast<size_t>(ceil_div(P.n, 32) * 32) * uform_stride(P.r) *
                                sizeof(double));
  }
  P.off_errp = (P.flags & RSM_COMPUTE_ERROR)
                   ? carve(cur, static_cast<size_t>(ceil_div(P.m, 256)) * sizeof(double))
                   : ~size_t(0);
  P.off_rbits = P.off_yrow = P.off_B = P.off_cmask = P.off_Qd = ~size_t(0);
  if (P.rows_first) {
    P.off_rbits = carve(cur, static_cast<size_t>(P.m) * P.nw * sizeof(uint64_t));
    if (P.y_layout == RSM_COL_MAJOR) P.off_yrow = carve(cur, static_cast<size_t>(P.m) * P.n * yelem);
    P.off_B = carve(cur, static_cast<size_t>(P.I) * P.l * P.r * sizeof(double));
    P.off_cmask = carve(cur, static_cast<size_t>(P.I) * P.nw * sizeof(uint64_t));
    P.off_Qd = carve(cur, static_cast<size_t>(P.I) * P.n * P.r * sizeof(double));
  }
  P.total = cur;
}

namespace {

std::mutex g_tune_mu;
std::vector<rsm_tune_entry> g_tune;  // the tile table (later duplicates of a key win)

std::vector<rsm_tune_entry> tune_snapshot() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return g_tune;
}

const rsm_tune_entry* tune_find(const std::vector<rsm_tune_entry>& t, const Plan& P,
                                bool batched) {
  const rsm_tune_entry* hit = nullptr;
  for (const rsm_tune_entry& e : t)
    if (e.l == P.l && e.gram_prec == P.prec && e.y_dtype == P.y_dtype &&
        e.batched == (batched ? 1 : 0))
      hit = &e;
  return hit;
}

}  // namespace

// Plans of one call's problems: each problem's own plan; then, for every launch group of
// the tiled Gram that the tile table covers (problems sharing l, Y's type and the
// precision, deterministic ones excepted), the table's trials per workgroup and one row
// split count for the group, sized so that the launch reaches the table's workgroup
// target; then the workspace layouts.
int32_t make_plans(const rsm_problem* problems, int32_t nprob, std::vector<Plan>& plans) {
  plans.assign(static_cast<size_t>(nprob), Plan{});
  for (int32_t k = 0; k < nprob; ++k) {
    const int32_t st = make_plan(problems[k], plans[k]);
    if (st != RSM_OK) return st;
  }
  const std::vector<rsm_tune_entry> table = tune_snapshot();
  if (!table.empty()) {
    std::map<int64_t, std::vector<int32_t>> groups;
    for (int32_t k = 0; k < nprob; ++k) {
      const Plan& P = plans[k];
      if (!P.tiled || P.I <= 0 || (P.flags & (RSM_FINALIZE_ONLY | RSM_DETERMINISTIC))) continue;
      groups[(int64_t(P.l) * 4 + P.y_dtype) * 4 + P.prec].push_back(k);
    }
    for (const auto& kv : groups) {
      const std::vector<int32_t>& members = kv.second;
      const Plan& P0 = plans[members[0]];
      const rsm_tune_entry* e = tune_find(table, P0, members.size() > 1);
      if (!e) continue;
      const int kernel = e->gram_kernel ? e->gram_kernel : default_gram_kernel(P0);
      int threads = e->gram_threads ? e->gram_threads : default_gram_threads(P0, kernel);
      if (!threads_built(P0.l, P0.prec, P0.y_dtype, kernel, threads))
        threads = default_gram_threads(P0, kernel);  // (rsm_tune_set admits built ones only)
      int64_t splits = 0;
      if (e->gram_wgs > 0) {
        int64_t total = 0;
        for (int32_t k : members) total += ceil_div(plans[k].I, threads);
        splits = e->gram_wgs / total;
        if (splits < 1) splits = 1;
      }
      for (int32_t k : members) {
        plans[k].gram_kernel = kernel;
        set_gram_shape(plans[k], threads, splits);
      }
    }
  }
  for (Plan& P : plans) set_layout(P);
  return RSM_OK;
}

namespace {

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

int32_t check_io(const Plan& P, const rsm_input& in, const rsm_output& out) {
  if (!out.info) return RSM_E_ARG;
  const bool finalize = P.flags & RSM_FINALIZE_ONLY;
  const bool acc_only = P.flags & RSM_ACCUMULATE_ONLY;
  if ((finalize || acc_only || (P.flags & RSM_N_ACCUMULATE)) && !out.N) return RSM_E_ARG;
  if (!acc_only && (!out.V || !out.U)) return RSM_E_ARG;
  // every mode reads Y and W (a2/a3 or a7)
  if (!in.Y || !in.W) return RSM_E_ARG;
  if (P.y_layout == RSM_COL_MAJOR ? in.ldy < P.m : in.ldy < P.n) return RSM_E_ARG;
  if (P.rows_first && out.trial_vecs) return RSM_E_ARG;
  if (P.w_layout == RSM_COL_MAJOR ? in.ldw < P.m : in.ldw < P.n) return RSM_E_ARG;
  return RSM_OK;
}

// Column-major Y as the kernels read it: the caller's array, or its packed copy.
const void* ycm_of(const Plan& P, const rsm_input& in, void* ws) {
  return P.y_layout == RSM_ROW_MAJOR ? at<void>(ws, P.off_ypack) : in.Y;
}
int64_t ldy_of(const Plan& P, const rsm_input& in) {
  return P.y_layout == RSM_ROW_MAJOR ? P.m : in.ldy;
}

void mark(const rsm_output& out, int step, int end, hipStream_t s) {
  if (out.step_events && out.step_events[2 * step + end])
    (void)hipEventRecord(static_cast<hipEvent_t>(out.step_events[2 * step + end]), s);
}

// Device pointer as the descriptors type it (global memory in the device pass).
template <typename T>
RSM_GLOBAL T* gptr(T* p) {
  return (RSM_GLOBAL T*)p;
}

// Descriptor of steps a0..a5 and a7 of one problem.
ProbDesc prob_desc(const Plan& P, const rsm_input& in, const rsm_output& out, void* ws) {
  ProbDesc d{};
  d.m = P.m;
  d.n = P.n;
  d.mw = P.mw;
  d.I = P.I;
  d.t0 = P.t0;
  d.ldw = in.ldw;
  d.ldy_in = in.ldy;
  d.ldy = ldy_of(P, in);
  d.r = P.r;
  d.l = P.l;
  d.nvec = P.nvec;
  d.min_rows = P.min_rows;
  d.y_layout = P.y_layout;
  d.w_layout = P.w_layout;
  d.splits = P.splits;
  d.gram_groups = P.gram_groups;
  d.words_per_split = P.words_per_split;
  d.seed = P.seed;
  d.fixed_n = (P.flags & RSM_DETERMINISTIC) ? 1 : 0;
  d.gram_unit = P.prec == RSM_GRAM_F64 ? 0x1p-53 : (P.prec == RSM_GRAM_F32 ? 0x1p-24 : 0x1p-16);
  d.W = gptr(in.W);
  d.Yin = gptr(in.Y);
  d.ycm = gptr(const_cast<void*>(ycm_of(P, in, ws)));
  d.wbits = gptr(at<uint64_t>(ws, P.off_wbits));
  d.user_subsets = gptr(in.subsets);
  d.cols = gptr(out.trial_cols ? out.trial_cols : at<int32_t>(ws, P.off_cols));
  d.part = gptr(at<void>(ws, P.off_part));
  d.prow = gptr(at<int32_t>(ws, P.off_prow));
  d.G = gptr(at<double>(ws, P.off_G));
  d.rows = gptr(at<int32_t>(ws, P.off_rows));
  d.mflag = gptr(at<int32_t>(ws, P.off_mflag));
  d.N = gptr(out.N ? out.N : at<double>(ws, P.off_N));
  d.V = gptr(out.V);
  d.U = gptr(out.U);
  d.info = gptr(out.info);
  d.scal = gptr(at<DevScalars>(ws, P.off_scal));
  d.ab = P.u_mfma ? gptr(at<double>(ws, P.off_ab)) : nullptr;
  d.abcnt = P.u_mfma ? gptr(at<int32_t>(ws, P.off_abcnt)) : nullptr;
  d.kext = P.u_mfma ? gptr(at<double>(ws, P.off_kext)) : nullptr;
  d.errp = (P.flags & RSM_COMPUTE_ERROR) ? gptr(at<double>(ws, P.off_errp)) : nullptr;
  d.rows_first = P.rows_first ? 1 : 0;
  d.nw = static_cast<int32_t>(P.nw);
  if (P.rows_first) {
    const bool yrm = P.y_layout == RSM_ROW_MAJOR;
    d.ldyr = yrm ? in.ldy : P.n;
    d.rbits = gptr(at<uint64_t>(ws, P.off_rbits));
    d.yrow = yrm ? gptr(in.Y) : gptr(static_cast<const void*>(at<void>(ws, P.off_yrow)));
    d.Bm = gptr(at<double>(ws, P.off_B));
    d.cmask = gptr(at<uint64_t>(ws, P.off_cmask));
    d.Qd = gptr(at<double>(ws, P.off_Qd));
  }
  d.tap_rows = gptr(out.trial_rows);
  d.tap_gram = gptr(out.trial_gram);
  d.tap_vecs = gptr(out.trial_vecs);
  d.tap_eigs = gptr(out.trial_eigs);
  return d;
}

// Descriptor of the a6 solve of one problem.
EigProb eig_desc(const Plan& P, const rsm_output& out, void* ws) {
  EigProb e{};
  e.n = P.n;
  e.npad = P.npad;
  e.nb = P.nb;
  e.b = P.eig_b;
  e.r = P.r;
  e.check_accepted = (P.flags & RSM_FINALIZE_ONLY) ? 0 : 1;
  e.deterministic = (P.flags & RSM_DETERMINISTIC) ? 1 : 0;
  e.pad_ = 0;
  e.seed = P.seed ^ 0x9E3779B97F4A7C15ull;
  e.N = gptr(out.N ? out.N : at<double>(ws, P.off_N));
  e.Nsym = gptr(at<double>(ws, P.off_Nsym));
  e.Lf = gptr(at<double>(ws, P.off_L));
  e.M = gptr(at<double>(ws, P.off_M));
  e.Mt = gptr(at<double>(ws, P.off_Mt));
  e.T = gptr(at<double>(ws, P.off_T));
  e.X = gptr(at<double>(ws, P.off_X));
  e.Z = gptr(at<double>(ws, P.off_Z));
  e.SP = gptr(at<double>(ws, P.off_SP));
  e.scal = gptr(at<DevScalars>(ws, P.off_scal));
  e.V = gptr(out.V);
  e.info = gptr(out.info);
  return e;
}

// Calls fn(list, plans) for the problems selected by `take`, grouped by `key` (problems
// with equal keys share launches), at most kLaunchMax per launch.
template <typename Take, typename Key, typename Fn>
void for_groups(const std::vector<Plan>& plans, Take take, Key key, Fn fn) {
  std::map<int64_t, std::vector<int32_t>> groups;
  for (int32_t k = 0; k < static_cast<int32_t>(plans.size()); ++k)
    if (take(plans[k])) groups[key(plans[k])].push_back(k);
  for (const auto& kv : groups) {
    const std::vector<int32_t>& members = kv.second;
    for (size_t b = 0; b < members.size(); b += kLaunchMax) {
      IdxList g;
      const Plan* h[kLaunchMax];
      for (size_t k = b; k < members.size() && k < b + kLaunchMax; ++k) {
        h[g.count] = &plans[members[k]];
        g.idx[g.count++] = members[k];
      }
      fn(g, h);
    }
  }
}

void mark_all(const rsm_output* outs, const IdxList& g, int step, int end, hipStream_t s) {
  for (int k = 0; k < g.count; ++k) mark(outs[g.idx[k]], step, end, s);
}

// The launch groups of one step touch disjoint problems, so they may run side by side: on
// up to kForkLanes streams, the caller's and library streams of the same device (default
// priority, created once per device), forked from and joined back into the caller's stream
// by events, so that the caller's stream orders the steps as before.  The last, longest
// workgroups of one launch then overlap the next launch instead of leaving CUs idle.
// g_fork_mu is held while a step's lanes are forked, fed and joined.  Only calls of at
// least kForkMinProblems problems fork (a smaller call has few, short launches per step),
// and none with RSM_SERIAL_STEPS: a caller that overlaps several calls on streams of its
// own gets its overlap from them, and lanes shared by its streams would queue one call's
// launches behind another's.
constexpr int kForkLanes = 4;
constexpr int kForkMinProblems = 64;
constexpr int kForkDevices = 64;

struct ForkLanes {
  hipStream_t aux[kForkLanes - 1] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kForkLanes - 1] = {};
  int state = 0;  // 0: not made yet, 1: ready, -1: could not be made (groups run in order)
};
std::mutex g_fork_mu;
ForkLanes g_fork[kForkDevices];

// The lanes of the device of stream s (caller holds g_fork_mu); null when s is not on the
// current device or the lanes could not be made.
ForkLanes* fork_lanes(hipStream_t s) {
  int cur = -1, dev = -1;
  if (hipGetDevice(&cur) != hipSuccess || hipStreamGetDevice(s, &dev) != hipSuccess ||
      dev != cur || dev < 0 || dev >= kForkDevices)
    return nullptr;
  ForkLanes& L = g_fork[dev];
  if (L.state == 0) {
    bool ok = hipEventCreateWithFlags(&L.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < kForkLanes - 1; ++i)
      ok = hipStreamCreateWithFlags(&L.aux[i], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&L.join[i], hipEventDisableTiming) == hipSuccess;
    L.state = ok ? 1 : -1;
  }
  return L.state == 1 ? &L : nullptr;
}

// for_groups with the groups spread over the fork lanes: largest estimated work first, each
// on the lane with the least work so far.  fn(g, h, stream) enqueues one group.
template <typename Take, typename Key, typename Work, typename Fn>
void for_groups_forked(const std::vector<Plan>& plans, bool may_fork, Take take, Key key,
                       Work work, Fn fn, hipStream_t s) {
  struct Group {
    IdxList g;
    const Plan* h[kLaunchMax];
    double work;
  };
  std::vector<Group> gs;
  for_groups(plans, take, key, [&](const IdxList& g, const Plan* const* h) {
    gs.emplace_back();
    Group& x = gs.back();
    x.g = g;
    x.work = 0.0;
    for (int k = 0; k < g.count; ++k) {
      x.h[k] = h[k];
      x.work += work(*h[k]);
    }
  });
  if (gs.size() <= 1 || !may_fork) {
    for (const Group& x : gs) fn(x.g, x.h, s);
    return;
  }
  std::lock_guard<std::mutex> lock(g_fork_mu);
  ForkLanes* L = fork_lanes(s);
  if (!L) {
    for (const Group& x : gs) fn(x.g, x.h, s);
    return;
  }
  const int lanes = std::min<int>(kForkLanes, static_cast<int>(gs.size()));
  (void)hipEventRecord(L->fork, s);
  for (int i = 0; i + 1 < lanes; ++i) (void)hipStreamWaitEvent(L->aux[i], L->fork, 0);
  std::vector<int> order(gs.size());
  for (size_t i = 0; i < gs.size(); ++i) order[i] = static_cast<int>(i);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return gs[a].work > gs[b].work; });
  double load[kForkLanes] = {};
  for (int i : order) {
    int lane = 0;
    for (int q = 1; q < lanes; ++q)
      if (load[q] < load[lane]) lane = q;
    load[lane] += gs[i].work;
    fn(gs[i].g, gs[i].h, lane == 0 ? s : L->aux[lane - 1]);
  }
  for (int i = 0; i + 1 < lanes; ++i) {
    (void)hipEventRecord(L->join[i], L->aux[i]);
    (void)hipStreamWaitEvent(s, L->join[i], 0);
  }
}

}  // namespace

}  // namespace rsm

// Scratch of rsm_decompose_noalloc: one array per device, in the code object's data,
// held until the process ends.  In host code `scratch` is only a handle for
// hipGetSymbolAddress; kernels are given the device address that call returns.
static __device__ __align__(256) unsigned char scratch[RSM_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, looked up once per device with that device
// current.
int32_t scratch_address(int dev, void** ptr) {
  if (dev < 0 || dev >= kMaxDevices) return RSM_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return RSM_E_DEVICE;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return RSM_E_DEVICE;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return RSM_E_DEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return RSM_OK;
}

}  // namespace

extern "C" {

int32_t rsm_abi_version(void) { return RSM_ABI_VERSION; }

const char* rsm_status_string(int32_t status) {
  switch (status) {
    case RSM_OK: return "ok";
    case RSM_E_ARG: return "invalid argument";
    case RSM_E_WORKSPACE: return "workspace too small or misaligned";
    case RSM_E_DEVICE: return "device launch failed";
    case RSM_E_UNSUPPORTED: return "outside the limits of this build";
    case RSM_E_SCRATCH: return "problem needs more scratch than RSM_NOALLOC_MAX_BYTES";
    case RSM_W_NO_CONSTRAINTS: return "warning: no trial accepted";
    case RSM_W_RANK_DEFICIENT: return "warning: V-hat not unique (uncovered column or no eigen-gap)";
    case RSM_W_ROWS_UNDERDETERMINED: return "warning: rows with fewer than r known entries";
    case RSM_W_NOT_CONVERGED: return "warning: eigen-solver residual above tolerance";
    case RSM_W_BAD_SUBSET: return "warning: invalid caller-supplied subset";
    case RSM_W_PIVOT: return "warning: Cholesky pivot clamped";
    default: return "unknown status";
  }
}

// The workspace of a call: each problem's scratch (256-byte aligned, in order), then the
// device copies of the a6 descriptors of all problems.
static size_t desc_bytes(int32_t nprob) {
  return rsm::align_up(static_cast<size_t>(nprob) * sizeof(rsm::ProbDesc), 256) +
         rsm::align_up(static_cast<size_t>(nprob) * sizeof(rsm::EigProb), 256);
}

int32_t rsm_workspace_bytes(const rsm_problem* problems, int32_t nprob, size_t* bytes) {
  if (!problems || !bytes || nprob < 1) return RSM_E_ARG;
  std::vector<rsm::Plan> plans;
  const int32_t st = rsm::make_plans(problems, nprob, plans);
  if (st != RSM_OK) return st;
  size_t total = 0;
  for (const rsm::Plan& P : plans) total += rsm::align_up(P.total, 256);
  *bytes = total + desc_bytes(nprob);
  return RSM_OK;
}

int32_t rsm_decompose(const rsm_problem* p, const rsm_input* in, const rsm_output* out,
                      void* workspace, size_t ws_bytes, void* hip_stream) {
  return rsm_decompose_batched(1, p, in, out, workspace, ws_bytes, hip_stream);
}

int32_t rsm_decompose_noalloc(const rsm_problem* p, const rsm_input* in, const rsm_output* out,
                              void* hip_stream) {
  if (!p) return RSM_E_ARG;
  size_t need = 0;
  const int32_t st = rsm_workspace_bytes(p, 1, &need);
  if (st != RSM_OK) return st;
  if (need > RSM_NOALLOC_MAX_BYTES) return RSM_E_SCRATCH;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int dev = -1;
  if (s) {
    hipDevice_t d = -1;
    if (hipStreamGetDevice(s, &d) != hipSuccess) return RSM_E_DEVICE;
    dev = static_cast<int>(d);
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return RSM_E_DEVICE;
  }
  void* ws = nullptr;
  const int32_t sa = scratch_address(dev, &ws);
  if (sa != RSM_OK) return sa;
  return rsm_decompose_batched(1, p, in, out, ws, RSM_NOALLOC_MAX_BYTES, hip_stream);
}

int32_t rsm_decompose_batched(int32_t nprob, const rsm_problem* problems,
                              const rsm_input* inputs, const rsm_output* outputs,
                              void* workspace, size_t ws_bytes, void* hip_stream) {
  using namespace rsm;
  if (nprob < 1 || !problems || !inputs || !outputs) return RSM_E_ARG;
  size_t need = 0;
  std::vector<Plan> plans;
  int32_t st = make_plans(problems, nprob, plans);
  if (st != RSM_OK) return st;
  std::vector<size_t> base(static_cast<size_t>(nprob));
  for (int32_t k = 0; k < nprob; ++k) {
    st = check_io(plans[k], inputs[k], outputs[k]);
    if (st != RSM_OK) return st;
    // the full spectrum is computed (Jacobi) only when asked for or for several vectors
    plans[k].minor_inv = plans[k].nvec == 1 && !outputs[k].trial_vecs && !outputs[k].trial_eigs;
    base[k] = need;
    need += align_up(plans[k].total, 256);
  }
  const size_t desc_off = need;
  need += desc_bytes(nprob);
  if (!workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255u))
    return RSM_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  (void)hipGetLastError();  // clear a stale error from unrelated earlier work
  char* ws = static_cast<char*>(workspace);
  auto* dprob = reinterpret_cast<ProbDesc*>(ws + desc_off);
  auto* deig = reinterpret_cast<EigProb*>(ws + desc_off + align_up(static_cast<size_t>(nprob) * sizeof(ProbDesc), 256));

  std::vector<ProbDesc> hp(static_cast<size_t>(nprob));
  for (int32_t k = 0; k < nprob; ++k) hp[k] = prob_desc(plans[k], inputs[k], outputs[k], ws + base[k]);
  put_prob_descs(hp.data(), nprob, dprob, s);

  // the launch groups of a step side by side (large calls, unless a problem asks otherwise)
  bool fork = nprob >= kForkMinProblems;
  for (const Plan& P : plans) fork = fork && !(P.flags & RSM_SERIAL_STEPS);
  auto all = [](const Plan&) { return true; };
  auto front = [](const Plan& P) { return !(P.flags & RSM_FINALIZE_ONLY); };
  auto one_key = [](const Plan&) { return int64_t(0); };
  // a0: info, mask bit-planes, column-major Y
  for_groups(plans, all, one_key, [&](const IdxList& g, const Plan* const* h) {
    launch_init_info(dprob, g, s);
    mark_all(outputs, g, RSM_STEP_PACK, 0, s);
    launch_pack(dprob, g, h, s);
    launch_rows_pack(dprob, g, h, s);
    mark_all(outputs, g, RSM_STEP_PACK, 1, s);
  });
  // a1: subsets, N cleared
  for_groups(plans, front, one_key, [&](const IdxList& g, const Plan* const* h) {
    mark_all(outputs, g, RSM_STEP_SUBSETS, 0, s);
    launch_subsets(dprob, g, h, s);
    mark_all(outputs, g, RSM_STEP_SUBSETS, 1, s);
  });
  // a2 + a3: one launch per (l, element type, precision, kernel, trials per workgroup),
  // the launches side by side on the fork lanes
  for_groups_forked(plans, fork, [](const Plan& P) {
               return !(P.flags & RSM_FINALIZE_ONLY) && P.I > 0 && !P.rows_first; },
             [](const Plan& P) {
               return ((((int64_t(P.l) * 4 + P.y_dtype) * 4 + P.prec) * 2 + (P.tiled ? 1 : 0)) *
                       8 + P.gram_kernel) * 2048 + P.gram_threads;
             },
             [](const Plan& P) { return double(P.m) * double(P.I) * P.l; },
             [&](const IdxList& g, const Plan* const* h, hipStream_t ls) {
               mark_all(outputs, g, RSM_STEP_GRAM, 0, ls);
               launch_gram(dprob, g, h, ls);
               mark_all(outputs, g, RSM_STEP_GRAM, 1, ls);
             }, s);
  // method M2: a2 + a3 for all rows-first problems in shared launches (per element type)
  for_groups(plans, [](const Plan& P) {
               return !(P.flags & RSM_FINALIZE_ONLY) && P.I > 0 && P.rows_first; },
             one_key, [&](const IdxList& g, const Plan* const* h) {
               mark_all(outputs, g, RSM_STEP_GRAM, 0, s);
               launch_rows_gram(dprob, g, h, s);
               mark_all(outputs, g, RSM_STEP_GRAM, 1, s);
             });
  // a4 + a5: one launch per l.  Deterministic problems accumulate N in fixed point: a
  // given N is converted to the grid first and everything back to FP64 afterwards.
  auto fixed = [](const Plan& P) {
    return !(P.flags & RSM_FINALIZE_ONLY) && (P.flags & RSM_DETERMINISTIC);
  };
  for_groups(plans, [&](const Plan& P) { return fixed(P) && (P.flags & RSM_N_ACCUMULATE); },
             one_key, [&](const IdxList& g, const Plan* const* h) {
               launch_n_fixed(dprob, g, h, true, s);
             });
  for_groups_forked(plans, fork, [&](const Plan& P) { return front(P) && !P.rows_first; },
             [](const Plan& P) { return int64_t(P.l); },
             [](const Plan& P) { return double(P.I) * P.l * P.l * P.l; },
             [&](const IdxList& g, const Plan* const* h, hipStream_t ls) {
               mark_all(outputs, g, RSM_STEP_MINOR, 0, ls);
               launch_minor(dprob, g, h, ls);
               mark_all(outputs, g, RSM_STEP_MINOR, 1, ls);
             }, s);
  for_groups(plans, [&](const Plan& P) { return front(P) && P.rows_first; },
             [](const Plan& P) { return int64_t(P.l); },
             [&](const IdxList& g, const Plan* const* h) {
               mark_all(outputs, g, RSM_STEP_MINOR, 0, s);
               launch_rows_minor(dprob, g, h, s);
               mark_all(outputs, g, RSM_STEP_MINOR, 1, s);
             });
  for_groups(plans, fixed, one_key, [&](const IdxList& g, const Plan* const* h) {
    launch_n_fixed(dprob, g, h, false, s);
  });
  // a6 for every problem that finalises, in shared launches
  std::vector<EigProb> eig;
  IdxList fin;
  std::vector<int32_t> who;
  for (int32_t k = 0; k < nprob; ++k) {
    if (plans[k].flags & RSM_ACCUMULATE_ONLY) continue;
    eig.push_back(eig_desc(plans[k], outputs[k], ws + base[k]));
    who.push_back(k);
  }
  if (!eig.empty()) {
    for (int32_t k : who) mark(outputs[k], RSM_STEP_EIG, 0, s);
    launch_solve_v(eig.data(), static_cast<int>(eig.size()), deig, s);
    for (int32_t k : who) mark(outputs[k], RSM_STEP_EIG, 1, s);
  }
  // a7 (and the optional error): one launch per (r, element type); a7's side by side
  auto back = [](const Plan& P) { return !(P.flags & RSM_ACCUMULATE_ONLY); };
  auto ukey = [](const Plan& P) { return int64_t(P.r) * 4 + P.y_dtype; };
  auto ukey_v = [](const Plan& P) { return (int64_t(P.r) * 4 + P.y_dtype) * 2 + (P.u_mfma ? 1 : 0); };
  for_groups_forked(plans, fork, back, ukey_v,
                    [](const Plan& P) { return double(P.m) * double(P.n) * P.r * P.r; },
                    [&](const IdxList& g, const Plan* const* h, hipStream_t ls) {
                      mark_all(outputs, g, RSM_STEP_USOLVE, 0, ls);
                      launch_solve_u(dprob, g, h, ls);
                      mark_all(outputs, g, RSM_STEP_USOLVE, 1, ls);
                    }, s);
  for_groups(plans, [](const Plan& P) {
               return !(P.flags & RSM_ACCUMULATE_ONLY) && (P.flags & RSM_COMPUTE_ERROR);
             }, ukey,
             [&](const IdxList& g, const Plan* const* h) {
               mark_all(outputs, g, RSM_STEP_ERROR, 0, s);
               launch_error(dprob, g, h, s);
               mark_all(outputs, g, RSM_STEP_ERROR, 1, s);
             });
  return hipGetLastError() == hipSuccess ? RSM_OK : RSM_E_DEVICE;
}

int32_t rsm_tune_set(const rsm_tune_entry* entries, int32_t count) {
  using namespace rsm;
  if (count < 0 || (count > 0 && !entries)) return RSM_E_ARG;
  for (int32_t k = 0; k < count; ++k) {
    const rsm_tune_entry& e = entries[k];
    if (e.l < 2 || e.l > RSM_MAX_L || e.gram_prec < RSM_GRAM_F64 ||
        e.gram_prec > RSM_GRAM_BF16X2 || (e.y_dtype != RSM_F32 && e.y_dtype != RSM_F64) ||
        (e.batched != 0 && e.batched != 1) || e.gram_wgs < 0 || e.gram_wgs > (1 << 20) ||
        e.gram_threads < 0 || e.gram_kernel < 0 || e.gram_kernel > RSM_GRAM_KERNEL_AUTO)
      return RSM_E_ARG;
    int built[8];
    if (e.gram_kernel && !gram_threads_built(e.l, e.gram_prec, e.y_dtype, e.gram_kernel, built))
      return RSM_E_ARG;
    // thread counts are checked against the entry's kernel, or the built-in one
    const int kernel = e.gram_kernel ? e.gram_kernel : builtin_gram_kernel(e.l, e.gram_prec, e.y_dtype);
    if (e.gram_threads && !threads_built(e.l, e.gram_prec, e.y_dtype, kernel, e.gram_threads))
      return RSM_E_ARG;
  }
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.assign(entries, entries + count);
  return RSM_OK;
}

int32_t rsm_tune_get(rsm_tune_entry* entries, int32_t cap, int32_t* count) {
  using namespace rsm;
  if (!count || cap < 0 || (cap > 0 && !entries)) return RSM_E_ARG;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const int32_t n = static_cast<int32_t>(g_tune.size());
  for (int32_t k = 0; k < n && k < cap; ++k) entries[k] = g_tune[k];
  *count = n;
  return RSM_OK;
}

int32_t rsm_tune_threads(int32_t l, int32_t gram_prec, int32_t y_dtype, int32_t gram_kernel,
                         int32_t* threads, int32_t cap, int32_t* count) {
  using namespace rsm;
  if (!count || cap < 0 || (cap > 0 && !threads) || l < 2 || l > RSM_MAX_L ||
      gram_kernel < RSM_GRAM_KERNEL_REGS || gram_kernel > RSM_GRAM_KERNEL_AUTO)
    return RSM_E_ARG;
  int built[8];
  const int nb = gram_threads_built(l, gram_prec, y_dtype, gram_kernel, built);
  for (int j = 0; j < nb && j < cap; ++j) threads[j] = built[j];
  *count = nb;
  return RSM_OK;
}

}  // extern "C"
