// The C ABI of librsm (include/rsm.h): argument validation, the execution plan and
// workspace layout of each problem, and the launch sequence of steps a0..a7.
#include <cstring>
#include <vector>

#include "rsm_internal.hpp"

namespace rsm {

namespace {

constexpr uint32_t kKnownFlags = RSM_ACCUMULATE_ONLY | RSM_FINALIZE_ONLY | RSM_N_ACCUMULATE |
                                 RSM_COMPUTE_ERROR | RSM_PLAIN_GRAM;
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
  const int l = p.l ? p.l : p.r + 1;
  if (l <= p.r || l > p.n) return RSM_E_ARG;
  const int nvec = p.nvec ? p.nvec : l - p.r;
  if (nvec < 1 || nvec > l - p.r) return RSM_E_ARG;
  const int min_rows = p.min_rows ? p.min_rows : p.r;
  if (min_rows < 1) return RSM_E_ARG;
  if (p.r > RSM_MAX_R || l > RSM_MAX_L || p.n > RSM_MAX_N) return RSM_E_UNSUPPORTED;
  if (p.gram_prec == RSM_GRAM_BF16X2) return RSM_E_UNSUPPORTED;

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
  P.ng = l * (l + 1) / 2;
  P.part_elem = (p.gram_prec == RSM_GRAM_F64) ? sizeof(double) : sizeof(float);
  P.eig_b = static_cast<int>((p.r + kEigPad) < p.n ? (p.r + kEigPad) : p.n);
  P.nb = static_cast<int>(ceil_div(p.n, kCholNB));
  int64_t nbp = 1;
  while (nbp < P.nb) nbp *= 2;
  P.npad = nbp * kCholNB;

  // Gram step.  Tiled kernel (one trial per thread, a 32-row x n tile of Y in LDS): split
  // the rows so that (trial groups) x (splits) is about one workgroup per CU.  Per-trial
  // streamer: enough wavefronts of (trial, split).
  const size_t acc_elem = (p.gram_prec == RSM_GRAM_F64) ? sizeof(double) : sizeof(float);
  const size_t tile_stride = (acc_elem == sizeof(double)) ? 34 : 36;  // see k_gram_tile
  P.tiled = !(p.flags & RSM_PLAIN_GRAM) &&
            static_cast<size_t>(ceil_div(p.n, 64) * 64) * tile_stride * acc_elem <= kTileLdsBytes;
  int64_t splits = 1;
  if (P.tiled) {
    const int64_t groups =
        ceil_div(P.I > 0 ? P.I : 1, tile_threads(l, static_cast<int>(acc_elem)));
    splits = kTileTargetGroups / groups;
    if (splits < 1) splits = 1;
    if (splits >= 8) splits -= splits % 8;  // whole XCD rounds (see k_gram_tile)
  } else if (P.I > 0 && P.I < 8192) {
    splits = ceil_div(8192, P.I);
  }
  if (splits > P.mw) splits = P.mw;
  P.words_per_split = ceil_div(P.mw, splits);
  // the splits actually needed to cover mw words (never more than requested)
  P.splits = static_cast<int>(ceil_div(P.mw, P.words_per_split));

  // workspace layout
  size_t cur = 0;
  P.off_scal = carve(cur, sizeof(DevScalars));
  P.off_wbits = carve(cur, static_cast<size_t>(P.n) * P.mw * sizeof(uint64_t));
  const size_t yelem = (p.y_dtype == RSM_F64) ? sizeof(double) : sizeof(float);
  P.off_ypack = (p.y_layout == RSM_ROW_MAJOR)
                    ? carve(cur, static_cast<size_t>(P.n) * P.m * yelem)
                    : ~size_t(0);
  P.off_cols = carve(cur, static_cast<size_t>(P.I) * l * sizeof(int32_t));
  P.off_part = carve(cur, static_cast<size_t>(P.splits) * P.I * P.ng * P.part_elem);
  P.off_prow = carve(cur, static_cast<size_t>(P.splits) * P.I * sizeof(int32_t));
  P.off_G = carve(cur, static_cast<size_t>(P.I) * P.ng * sizeof(double));
  P.off_rows = carve(cur, static_cast<size_t>(P.I) * sizeof(int32_t));
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
  P.off_NX = carve(cur, nbv);
  P.off_small = carve(cur, kSmallDoubles * sizeof(double));
  P.total = cur;
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

// Steps a0..a5 of one problem whose scratch starts at `ws`.
void enqueue_front(const Plan& P, const rsm_input& in, const rsm_output& out, void* ws,
                   hipStream_t s) {
  DevScalars* scal = at<DevScalars>(ws, P.off_scal);
  uint64_t* wbits = at<uint64_t>(ws, P.off_wbits);
  rsm_info* info = out.info;
  double* N = out.N ? out.N : at<double>(ws, P.off_N);

  launch_init_info(info, scal, s);

  // a0: mask bit-planes, column-major Y
  mark(out, RSM_STEP_PACK, 0, s);
  launch_pack_mask(in.W, P.w_layout, in.ldw, P.m, P.n, wbits, P.mw, s);
  if (P.y_layout == RSM_ROW_MAJOR)
    launch_pack_y(in.Y, P.y_dtype, in.ldy, P.m, P.n, at<void>(ws, P.off_ypack), P.m, s);
  mark(out, RSM_STEP_PACK, 1, s);

  if (P.flags & RSM_FINALIZE_ONLY) return;
  // a1: subsets
  mark(out, RSM_STEP_SUBSETS, 0, s);
  int32_t* cols = out.trial_cols ? out.trial_cols : at<int32_t>(ws, P.off_cols);
  launch_subsets(P, in.subsets, cols, info, s);
  if (!(P.flags & RSM_N_ACCUMULATE)) launch_fill_zero(N, P.n * P.n, s);
  mark(out, RSM_STEP_SUBSETS, 1, s);
  // a2 + a3: row qualification and Gram partials
  void* part = at<void>(ws, P.off_part);
  int32_t* prow = at<int32_t>(ws, P.off_prow);
  mark(out, RSM_STEP_GRAM, 0, s);
  launch_gram(P, ycm_of(P, in, ws), ldy_of(P, in), P.y_dtype, wbits, cols, part, prow, s);
  mark(out, RSM_STEP_GRAM, 1, s);
  // a4 + a5: minor vectors, N accumulation
  mark(out, RSM_STEP_MINOR, 0, s);
  launch_minor(P, part, prow, cols, at<double>(ws, P.off_G), at<int32_t>(ws, P.off_rows), N,
               info, out, s);
  mark(out, RSM_STEP_MINOR, 1, s);
}

// Device pointer as the descriptor types it (global memory in the device pass).
template <typename T>
RSM_GLOBAL T* gptr(T* p) {
  return (RSM_GLOBAL T*)p;
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
  e.seed = P.seed ^ 0x9E3779B97F4A7C15ull;
  e.N = gptr(out.N ? out.N : at<double>(ws, P.off_N));
  e.Nsym = gptr(at<double>(ws, P.off_Nsym));
  e.Lf = gptr(at<double>(ws, P.off_L));
  e.M = gptr(at<double>(ws, P.off_M));
  e.Mt = gptr(at<double>(ws, P.off_Mt));
  e.T = gptr(at<double>(ws, P.off_T));
  e.X = gptr(at<double>(ws, P.off_X));
  e.Z = gptr(at<double>(ws, P.off_Z));
  e.NX = gptr(at<double>(ws, P.off_NX));
  e.small = gptr(at<double>(ws, P.off_small));
  e.scal = gptr(at<DevScalars>(ws, P.off_scal));
  e.V = gptr(out.V);
  e.info = gptr(out.info);
  return e;
}

// Step a7 (and the optional error) of one problem.
void enqueue_back(const Plan& P, const rsm_input& in, const rsm_output& out, void* ws,
                  hipStream_t s) {
  const uint64_t* wbits = at<uint64_t>(ws, P.off_wbits);
  const void* ycm = ycm_of(P, in, ws);
  const int64_t ldy = ldy_of(P, in);
  mark(out, RSM_STEP_USOLVE, 0, s);
  launch_solve_u(P, ycm, ldy, P.y_dtype, wbits, out.V, out.U, out.info, s);
  mark(out, RSM_STEP_USOLVE, 1, s);
  if (P.flags & RSM_COMPUTE_ERROR) {
    mark(out, RSM_STEP_ERROR, 0, s);
    launch_error(P, ycm, ldy, P.y_dtype, wbits, out.U, out.V, at<DevScalars>(ws, P.off_scal),
                 out.info, s);
    mark(out, RSM_STEP_ERROR, 1, s);
  }
}

}  // namespace

}  // namespace rsm

extern "C" {

int32_t rsm_abi_version(void) { return RSM_ABI_VERSION; }

const char* rsm_status_string(int32_t status) {
  switch (status) {
    case RSM_OK: return "ok";
    case RSM_E_ARG: return "invalid argument";
    case RSM_E_WORKSPACE: return "workspace too small or misaligned";
    case RSM_E_DEVICE: return "device launch failed";
    case RSM_E_UNSUPPORTED: return "outside the limits of this build";
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
  return rsm::align_up(static_cast<size_t>(nprob) * sizeof(rsm::EigProb), 256);
}

int32_t rsm_workspace_bytes(const rsm_problem* problems, int32_t nprob, size_t* bytes) {
  if (!problems || !bytes || nprob < 1) return RSM_E_ARG;
  size_t total = 0;
  for (int32_t k = 0; k < nprob; ++k) {
    rsm::Plan P;
    const int32_t st = rsm::make_plan(problems[k], P);
    if (st != RSM_OK) return st;
    total += rsm::align_up(P.total, 256);
  }
  *bytes = total + desc_bytes(nprob);
  return RSM_OK;
}

int32_t rsm_decompose(const rsm_problem* p, const rsm_input* in, const rsm_output* out,
                      void* workspace, size_t ws_bytes, void* hip_stream) {
  return rsm_decompose_batched(1, p, in, out, workspace, ws_bytes, hip_stream);
}

int32_t rsm_decompose_batched(int32_t nprob, const rsm_problem* problems,
                              const rsm_input* inputs, const rsm_output* outputs,
                              void* workspace, size_t ws_bytes, void* hip_stream) {
  if (nprob < 1 || !problems || !inputs || !outputs) return RSM_E_ARG;
  size_t need = 0;
  std::vector<rsm::Plan> plans(static_cast<size_t>(nprob));
  std::vector<size_t> base(static_cast<size_t>(nprob));
  for (int32_t k = 0; k < nprob; ++k) {
    int32_t st = rsm::make_plan(problems[k], plans[k]);
    if (st == RSM_OK) st = rsm::check_io(plans[k], inputs[k], outputs[k]);
    if (st != RSM_OK) return st;
    base[k] = need;
    need += rsm::align_up(plans[k].total, 256);
  }
  const size_t desc_off = need;
  need += desc_bytes(nprob);
  if (!workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255u))
    return RSM_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  (void)hipGetLastError();  // clear a stale error from unrelated earlier work
  char* ws = static_cast<char*>(workspace);
  for (int32_t k = 0; k < nprob; ++k)
    rsm::enqueue_front(plans[k], inputs[k], outputs[k], ws + base[k], s);
  // a6 for every problem that finalises, in shared launches
  std::vector<rsm::EigProb> eig;
  std::vector<int32_t> who;
  for (int32_t k = 0; k < nprob; ++k) {
    if (plans[k].flags & RSM_ACCUMULATE_ONLY) continue;
    eig.push_back(rsm::eig_desc(plans[k], outputs[k], ws + base[k]));
    who.push_back(k);
  }
  if (!eig.empty()) {
    for (int32_t k : who) rsm::mark(outputs[k], RSM_STEP_EIG, 0, s);
    rsm::launch_solve_v(eig.data(), static_cast<int>(eig.size()),
                        reinterpret_cast<rsm::EigProb*>(ws + desc_off), s);
    for (int32_t k : who) rsm::mark(outputs[k], RSM_STEP_EIG, 1, s);
    for (int32_t k : who) rsm::enqueue_back(plans[k], inputs[k], outputs[k], ws + base[k], s);
  }
  return hipGetLastError() == hipSuccess ? RSM_OK : RSM_E_DEVICE;
}

}  // extern "C"
