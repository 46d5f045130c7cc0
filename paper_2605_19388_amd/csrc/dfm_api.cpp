// C ABI of distributed FastMNMF: validation, workspace layout, launch sequencing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "dfm_internal.h"
#include "dfmnmf.h"

using dfm::Buffers;
using dfm::Dims;

struct dfm_plan {
  Dims d;
  Buffers b;
  int dtype;
  // Event timing of one kernel during ordinary launches (dfm_profile_kernel).
  int prof_kid = -1;
  std::vector<hipEvent_t> prof_events;  // pairs (start, stop)
  size_t prof_used = 0;
  // HIP graphs of dfm_step's iterations, captured on first use on the plan's own stream:
  // [0] the first iteration of a call, [1] a later one, [2] kGraphBatch later ones.
  hipStream_t cap = nullptr;
  hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};
  bool graph_off = false;  // DFM_F_NO_GRAPH, or a capture failed (plain launches from then on)
};

namespace dfm {

static size_t real_size(int dtype) { return dtype == DFM_C64 ? 4 : 8; }
static size_t al(size_t x) { return (x + 255) / 256 * 256; }

// Specialised path: uniform partition with a compiled (N, K, M_l) set.  Frames per slice:
// the largest of max_slice(), ..., 16 whose LDS needs fit 64 KB in every kernel.
// Compute units of the current device (the balanced covariance kernel sizes its grid to it).
static int compute_units() {
  int dev = 0, cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cu <= 0)
    return 256;
  return cu;
}

static bool choose_fast(Dims& d, int dtype) {
  int ml = d.mics[0];
  for (int l = 1; l < d.L; ++l)
    if (d.mics[l] != ml) return false;
  const int set = fast_set_index(d.N, d.K, ml, d.L);
  if (set < 0 || (dtype == DFM_C128 && !fast_fp64_ok(set))) return false;
  d.fast = set;
  d.ML = ml;
  for (int sl = d.tile; sl >= 16; sl /= 2) {
    d.S = (d.T + sl - 1) / sl;
    d.SL = (d.T + d.S - 1) / d.S;
    d.SLP = ((d.SL + 3) & ~3) + 4;
    d.TB = 16;
    d.TBN = (d.T + 15) / 16;
    d.TP = (d.T + 15) & ~15;
    // k_gramd_f: as many workgroups as fit on the chip at once share the F*T frames equally:
    // the same number per bin (Dims::GSB) when that is at least two, else equal flattened
    // ranges; a bin then has one partial-sum slot per workgroup that touched it.
    if (dtype == DFM_C64 && (ml == 2 || ml == 4)) {
      const long long total = (long long)d.F * d.T;
      const int per_cu = fast_gramd_blocks_per_cu(d);
      const long long want = (long long)(per_cu > 0 ? per_cu : 2) * compute_units();
      d.GR = (int)std::max<long long>((total + want - 1) / want, 32);
      d.GW = (int)((total + d.GR - 1) / d.GR);
      d.SG = (d.T + d.GR - 1) / d.GR + 1;
      d.GSB = 0;
      const int per_bin = (int)std::min<long long>(want / d.F, d.T / 32);  // parts of >= 32 frames
      if (per_bin >= 2) {
        d.GSB = per_bin;
        d.GW = d.F * d.GSB;
        d.SG = d.GSB;
      }
    } else {
      d.GR = 0;
      d.GW = 0;
      d.SG = d.S;
    }
    // k_g_f: four workgroups per CU share the F*T frames equally.
    {
      const long long total = (long long)d.F * d.T, want = 4LL * compute_units();
      d.GGR = (int)std::max<long long>((total + want - 1) / want, 16);
      d.GGW = (int)((total + d.GGR - 1) / d.GGR);
      d.GGS = (d.T + d.GGR - 1) / d.GGR + 1;
    }
    d.HC = fast_hgemm_windows(d, dtype);
    if (fast_max_smem(d, dtype) <= 64 * 1024) return true;
  }
  d.fast = -1;
  d.ML = 0;
  return false;
}

// Frames per streaming slice: as many as fit the LDS budget of every tile kernel, at most 128.
static void choose_tiles(Dims& d, int dtype) {
  const size_t r = real_size(dtype), c = 2 * r;
  const size_t budget = 48 * 1024;
  int sl = d.tile;
  for (; sl > 8; sl /= 2) {
    const size_t gram = r * (d.N * d.K + d.N * d.M + sl * d.M) + 16 + c * sl * d.M;
    const size_t pw = c * d.QF + 16 + r * (d.N * d.K + d.N * d.M + sl * (3 * d.N + 2 * d.M));
    const size_t gg = r * (d.N * d.K + d.N * d.M + sl * d.N + sl * d.M * 2);
    if (gram <= budget && pw <= budget && gg <= budget) break;
  }
  d.S = (d.T + sl - 1) / sl;
  d.SL = (d.T + d.S - 1) / d.S;
  d.TB = 16;
  d.FB = 16;
  while (d.FB > 1 && r * d.FB * d.TB * d.N * 2 > budget) d.FB /= 2;
  d.FS = (d.F + d.FB - 1) / d.FB;
  d.TBN = (d.T + d.TB - 1) / d.TB;
  d.SG = d.S;
  d.GR = 0;
  d.GW = 0;
}

static dfm_status make_dims(const dfm_problem* p, Dims& d) {
  if (!p) return DFM_E_ARG;
  if (p->dtype != DFM_C64 && p->dtype != DFM_C128) return DFM_E_ARG;
  constexpr uint32_t known = DFM_F_CHECK_FINITE | DFM_F_TRACE_NLL | DFM_F_GRAM_BF16 | DFM_F_NO_GRAPH;
  if (!(p->eps > 0.0) || !std::isfinite(p->eps) || (p->flags & ~known) != 0) return DFM_E_ARG;
  if (p->F < 1 || p->T < 1 || p->N < 1 || p->N > kMaxN || p->K < 1 || p->K > kMaxK || p->L < 1 || p->L > kMaxL)
    return DFM_E_SHAPE;
  std::memset(&d, 0, sizeof(d));
  d.F = p->F;
  d.T = p->T;
  d.N = p->N;
  d.K = p->K;
  d.L = p->L;
  d.eps = p->eps;
  d.flags = (int)p->flags;
  if (p->tile != 0 && p->tile != 16 && p->tile != 32 && p->tile != 64 && p->tile != 128) return DFM_E_ARG;
  d.tile = p->tile ? p->tile : 128;
  d.check = (p->flags & DFM_F_CHECK_FINITE) != 0;
  int m = 0, q = 0, v = 0;
  for (int l = 0; l < p->L; ++l) {
    const int ml = p->mics[l];
    if (ml < 1 || ml > kMaxMl || m + ml > kMaxM) return DFM_E_SHAPE;
    d.mics[l] = ml;
    d.moff[l] = m;
    d.qoff[l] = q;
    d.voff[l] = v;
    for (int i = 0; i < ml; ++i) d.msub[m + i] = l;
    m += ml;
    q += ml * ml;
    v += ml * ml * ml;
  }
  d.M = m;
  d.MLX = 0;
  for (int l = 0; l < p->L; ++l) d.MLX = std::max(d.MLX, (int)p->mics[l]);
  d.QF = q;
  d.VF = v;
  d.VC = v;
  d.fast = -1;
  // 32-bit indexing inside kernels: keep every per-buffer element count below 2^31.
  const double big = (double)d.F * d.T * d.M * 2 * (p->N > 1 ? p->N : 1);
  if (big >= 2147483647.0) return DFM_E_SHAPE;
  if (!choose_fast(d, p->dtype)) choose_tiles(d, p->dtype);
  // BF16 covariances: only where the shape-specialised path has the kernel (k_gramb_f).
  if ((p->flags & DFM_F_GRAM_BF16) &&
      (p->dtype != DFM_C64 || d.fast < 0 || d.GR <= 0 || !fast_gram_bf16(d.N, d.K, d.ML, d.L)))
    return DFM_E_ARG;
  return DFM_OK;
}

size_t workspace_bytes(const Dims& d, int dtype) {
  const size_t r = real_size(dtype);
  size_t n = 0;
  n += al(r * d.F * d.T * d.M);                        // P
  n += al(8 * (size_t)d.F * d.SG * d.VF);              // Vpart (FP64 sums)
  const bool fast = d.fast >= 0;
  n += al(fast ? 0 : r * d.F * d.S * d.N * d.K * 2);    // Wpart
  const size_t kp16 = 16 * 4 * (size_t)((d.K + 3) / 4);
  n += al(fast ? (d.HC > 1 ? r * d.N * d.TBN * d.HC * 2 * kp16 : 0) : r * (size_t)d.FS * d.N * d.K * d.T * 2);  // Hpart
  n += al(fast && d.HC > 1 ? r * d.N * d.K * d.T : 0);  // Hsnap
  n += al(fast ? r * d.F * d.GGS * d.N * d.M * 2 : r * d.F * d.S * d.N * d.M * 2);  // gpart
  n += al(fast ? r * d.F * d.N * d.M : 0);              // gsnap
  n += al(8 * d.F * d.L);                              // logdet
  n += al(8 * d.F * d.S);                              // nllpart
  n += al(16 * d.F * d.QF);                            // Qinv
  n += al(64);                                         // status
  n += al(8);                                          // cost total
  n += al(d.flags & DFM_F_TRACE_NLL ? 8 * DFM_TRACE_CAPACITY : 0);  // cost trace
  n += al(fast ? r * d.F * d.T * d.N : 0);             // lambda
  n += al(fast ? r * 2 * d.N * (size_t)d.F * d.TP : 0);  // coefficient planes [2N][TBN][F][16]
  return n;
}

void carve(const Dims& d, int dtype, char* ws, Buffers& b) {
  const size_t r = real_size(dtype);
  char* p = ws;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += al(bytes);
    return q;
  };
  b.P = take(r * d.F * d.T * d.M);
  b.Vpart = take(8 * (size_t)d.F * d.SG * d.VF);
  const bool fast = d.fast >= 0;
  b.Wpart = take(fast ? 0 : r * d.F * d.S * d.N * d.K * 2);
  const size_t kp16 = 16 * 4 * (size_t)((d.K + 3) / 4);
  b.Hpart = take(fast ? (d.HC > 1 ? r * d.N * d.TBN * d.HC * 2 * kp16 : 0) : r * (size_t)d.FS * d.N * d.K * d.T * 2);
  b.Hsnap = fast && d.HC > 1 ? take(r * d.N * d.K * d.T) : nullptr;
  b.gpart = take(fast ? r * d.F * d.GGS * d.N * d.M * 2 : r * d.F * d.S * d.N * d.M * 2);
  b.gsnap = fast ? take(r * d.F * d.N * d.M) : nullptr;
  b.logdet = reinterpret_cast<double*>(take(8 * d.F * d.L));
  b.nllpart = reinterpret_cast<double*>(take(8 * d.F * d.S));
  b.Qinv = take(16 * d.F * d.QF);
  b.status = reinterpret_cast<int*>(take(64));
  b.nlltot = reinterpret_cast<double*>(take(8));
  b.trace = d.flags & DFM_F_TRACE_NLL ? reinterpret_cast<double*>(take(8 * DFM_TRACE_CAPACITY)) : nullptr;
  b.lam = fast ? take(r * d.F * d.T * d.N) : nullptr;
  b.AB = fast ? take(r * 2 * d.N * (size_t)d.F * d.TP) : nullptr;
}

static hipError_t run_kernel(dfm_plan* plan, int kid, hipStream_t s) {
  const bool prof = plan->prof_kid == kid && plan->prof_used + 2 <= plan->prof_events.size();
  if (prof && hipEventRecord(plan->prof_events[plan->prof_used], s) != hipSuccess) return hipErrorUnknown;
  const hipError_t e = launch_kernel(plan->d, plan->b, plan->dtype, kid, s);
  if (e != hipSuccess) return e;
  if (prof) {
    if (hipEventRecord(plan->prof_events[plan->prof_used + 1], s) != hipSuccess) return hipErrorUnknown;
    plan->prof_used += 2;
  }
  return hipSuccess;
}

static hipError_t run_stage(dfm_plan* plan, int stage, hipStream_t s) {
  int kids[8];
  const int n = stage_kernels(plan->d, stage, kids);
  for (int i = 0; i < n; ++i) {
    const hipError_t e = run_kernel(plan, kids[i], s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Kernels of one dfm_step iteration on stream s.  `first`: no g update is pending from a
// previous iteration of the same call.  With the cost trace, every iteration finishes its own g
// update and records the cost (13) of the new state.
static hipError_t enqueue_iteration(dfm_plan* plan, bool first, hipStream_t s) {
  Dims& d = plan->d;
  const bool trace = (d.flags & DFM_F_TRACE_NLL) != 0;
  d.gpend = g_update_deferred(d) && !trace && !first;
  hipError_t e = hipSuccess;
  for (int stage = DFM_STAGE_IP; stage <= DFM_STAGE_G && e == hipSuccess; ++stage) e = run_stage(plan, stage, s);
  d.gpend = 0;
  if (e == hipSuccess && trace) {
    if (g_update_deferred(d)) e = run_kernel(plan, kFGFin, s);
    if (e == hipSuccess) e = launch_nll(d, plan->b, plan->dtype, s);
    if (e == hipSuccess) e = launch_nll_total(d, plan->b, plan->b.nlltot, true, s);
  }
  return e;
}

constexpr int kGraphBatch = 8;  // iterations in the batch graph

// Capture graph `which` (0: first iteration, 1: a later iteration, 2: kGraphBatch later ones)
// on the plan's own stream.  Only kernel launches are recorded (no memset or copy nodes).
static hipError_t capture_graph(dfm_plan* plan, int which) {
  if (!plan->cap && hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking) != hipSuccess) return hipErrorUnknown;
  hipError_t e = hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const int reps = which == 2 ? kGraphBatch : 1;
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = enqueue_iteration(plan, which == 0, plan->cap);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(plan->cap, &g);
  if (e == hipSuccess) e = ee;
  if (e == hipSuccess && g) e = hipGraphInstantiate(&plan->graph[which], g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) plan->graph[which] = nullptr;
  return e;
}

static void free_graphs(dfm_plan* plan) {
  for (hipGraphExec_t& g : plan->graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  if (plan->cap) (void)hipStreamDestroy(plan->cap);
  plan->cap = nullptr;
}

// Replay graph `which` on s, capturing it first if needed.  False if graphs are off for this plan
// (then the caller launches plainly); a capture failure turns them off for good.
static bool replay(dfm_plan* plan, int which, hipStream_t s, hipError_t& e) {
  if (plan->graph_off) return false;
  if (!plan->graph[which] && capture_graph(plan, which) != hipSuccess) {
    (void)hipGetLastError();
    free_graphs(plan);
    plan->graph_off = true;
    return false;
  }
  e = hipGraphLaunch(plan->graph[which], s);
  return true;
}

static void free_profile(dfm_plan* plan) {
  for (hipEvent_t e : plan->prof_events) (void)hipEventDestroy(e);
  plan->prof_events.clear();
  plan->prof_used = 0;
  plan->prof_kid = -1;
}

static dfm_status read_status(dfm_plan* plan, hipStream_t s, bool clear) {
  int st = 0;
  if (hipMemcpyAsync(&st, plan->b.status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return DFM_E_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return DFM_E_HIP;
  if (clear && st != 0 && launch_clear_status(plan->b, s) != hipSuccess) return DFM_E_HIP;
  if (st & kStSingular) return DFM_E_SINGULAR;
  if (st & kStNonFinite) return DFM_E_NONFINITE;
  return DFM_OK;
}

}  // namespace dfm

extern "C" {

dfm_status dfm_workspace_size(const dfm_problem* p, size_t* bytes) {
  if (!bytes) return DFM_E_ARG;
  Dims d;
  const dfm_status st = dfm::make_dims(p, d);
  if (st != DFM_OK) return st;
  *bytes = dfm::workspace_bytes(d, p->dtype);
  return DFM_OK;
}

dfm_status dfm_init(dfm_plan** out, const dfm_problem* p, const void* X, void* Q, void* g, void* W, void* H,
                    void* workspace, size_t workspace_bytes, void* stream) {
  if (!out) return DFM_E_ARG;
  *out = nullptr;
  Dims d;
  const dfm_status st = dfm::make_dims(p, d);
  if (st != DFM_OK) return st;
  if (!X || !Q || !g || !W || !H || !workspace) return DFM_E_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return DFM_E_WORKSPACE;
  if (workspace_bytes < dfm::workspace_bytes(d, p->dtype)) return DFM_E_WORKSPACE;
  dfm_plan* plan = new (std::nothrow) dfm_plan;
  if (!plan) return DFM_E_ARG;
  plan->d = d;
  plan->dtype = p->dtype;
  plan->graph_off = (p->flags & DFM_F_NO_GRAPH) != 0;
  std::memset(&plan->b, 0, sizeof(plan->b));
  plan->b.X = X;
  plan->b.Q = Q;
  plan->b.g = g;
  plan->b.W = W;
  plan->b.H = H;
  dfm::carve(d, p->dtype, static_cast<char*>(workspace), plan->b);
  if (dfm::launch_init(d, plan->b, static_cast<hipStream_t>(stream)) != hipSuccess) {
    delete plan;
    return DFM_E_HIP;
  }
  *out = plan;
  return DFM_OK;
}

dfm_status dfm_step(dfm_plan* plan, int32_t n_iter, void* stream) {
  if (!plan || n_iter < 0) return DFM_E_ARG;
  if (n_iter == 0) return DFM_OK;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // The specialised kernels read lambda = W H, which the W and H updates then keep
  // current; seed it from the caller's state.
  if (plan->d.fast >= 0 && dfm::run_kernel(plan, dfm::kFLam, s) != hipSuccess) return DFM_E_HIP;
  // Where the g update ends in k_g_f's partial sums (dfm::g_update_deferred), the next
  // iteration's covariance kernel finishes it, and k_gfin_f after the last one.
  hipError_t e = hipSuccess;
  const bool graphs = plan->prof_kid < 0;  // event-profiled launches stay plain
  int left = n_iter;
  if (!(graphs && dfm::replay(plan, 0, s, e))) e = dfm::enqueue_iteration(plan, true, s);
  --left;
  while (e == hipSuccess && left > 0) {
    const int which = left >= dfm::kGraphBatch ? 2 : 1;
    if (graphs && dfm::replay(plan, which, s, e)) {
      left -= which == 2 ? dfm::kGraphBatch : 1;
    } else {
      e = dfm::enqueue_iteration(plan, false, s);
      --left;
    }
  }
  const bool defer = dfm::g_update_deferred(plan->d) && !(plan->d.flags & DFM_F_TRACE_NLL);
  if (e == hipSuccess && defer) e = dfm::run_kernel(plan, dfm::kFGFin, s);
  return e == hipSuccess ? DFM_OK : DFM_E_HIP;
}

dfm_status dfm_substep(dfm_plan* plan, int32_t stage, void* stream) {
  if (!plan || stage < DFM_STAGE_IP || stage > DFM_STAGE_G) return DFM_E_ARG;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // A sub-step may follow a change of the state by the caller: refresh lambda = W H, which
  // the specialised kernels read.
  if (plan->d.fast >= 0 && dfm::run_kernel(plan, dfm::kFLam, s) != hipSuccess) return DFM_E_HIP;
  if (dfm::run_stage(plan, stage, s) != hipSuccess) return DFM_E_HIP;
  if (stage == DFM_STAGE_G && dfm::g_update_deferred(plan->d) && dfm::run_kernel(plan, dfm::kFGFin, s) != hipSuccess)
    return DFM_E_HIP;
  return DFM_OK;
}

dfm_status dfm_nll(dfm_plan* plan, double* out, void* stream) {
  if (!plan || !out) return DFM_E_ARG;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const Dims& d = plan->d;
  if (dfm::launch_nll(d, plan->b, plan->dtype, s) != hipSuccess ||
      dfm::launch_nll_total(d, plan->b, plan->b.nlltot, false, s) != hipSuccess)
    return DFM_E_HIP;
  double v = 0.0;
  if (hipMemcpyAsync(&v, plan->b.nlltot, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return DFM_E_HIP;
  const dfm_status st = dfm::read_status(plan, s, false);  // synchronises s
  if (st == DFM_E_HIP) return st;
  *out = v;
  return st;
}

dfm_status dfm_nll_trace(dfm_plan* plan, double* out, int32_t capacity, int32_t* count, void* stream) {
  if (!plan || !count || capacity < 0 || (capacity > 0 && !out) || !(plan->d.flags & DFM_F_TRACE_NLL))
    return DFM_E_ARG;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  int n = 0;
  if (hipMemcpyAsync(&n, plan->b.status + dfm::kTraceSlot, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return DFM_E_HIP;
  const int k = std::min(std::min(n, (int)capacity), DFM_TRACE_CAPACITY);
  if (k > 0 && (hipMemcpyAsync(out, plan->b.trace, sizeof(double) * k, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess))
    return DFM_E_HIP;
  *count = n;
  return DFM_OK;
}

dfm_status dfm_separate(dfm_plan* plan, void* S, void* stream) {
  if (!plan || !S) return DFM_E_ARG;
  if (dfm::launch_separate(plan->d, plan->b, plan->dtype, S, static_cast<hipStream_t>(stream)) != hipSuccess)
    return DFM_E_HIP;
  return DFM_OK;
}

dfm_status dfm_covariances(dfm_plan* plan, void* V, void* stream) {
  if (!plan || !V) return DFM_E_ARG;
  if (dfm::launch_covariances(plan->d, plan->b, plan->dtype, V, static_cast<hipStream_t>(stream)) != hipSuccess)
    return DFM_E_HIP;
  return DFM_OK;
}

dfm_status dfm_sync_status(dfm_plan* plan, void* stream) {
  if (!plan) return DFM_E_ARG;
  return dfm::read_status(plan, static_cast<hipStream_t>(stream), true);
}

int32_t dfm_kernel_count(const dfm_plan* plan) {
  if (!plan) return 0;
  int kids[16];
  return dfm::iteration_kernels(plan->d, kids);
}

const char* dfm_kernel_name(const dfm_plan* plan, int32_t kernel) {
  if (!plan) return nullptr;
  int kids[16];
  const int n = dfm::iteration_kernels(plan->d, kids);
  if (kernel < 0 || kernel >= n) return nullptr;
  return plan->d.fast >= 0 ? dfm::fast_kernel_name(plan->d, plan->dtype, kids[kernel]) : dfm::kernel_name(kids[kernel]);
}

dfm_status dfm_kernel_times(dfm_plan* plan, int32_t reps, double* avg_ms, void* stream) {
  if (!plan || !avg_ms || reps < 1) return DFM_E_ARG;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess) return DFM_E_HIP;
  if (hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DFM_E_HIP;
  }
  dfm_status st = DFM_OK;
  int kids[16];
  const int nk = dfm::iteration_kernels(plan->d, kids);
  for (int k = 0; k < nk && st == DFM_OK; ++k) {
    float ms = 0.f;
    if (hipEventRecord(e0, s) != hipSuccess) st = DFM_E_HIP;
    for (int r = 0; r < reps && st == DFM_OK; ++r)
      if (dfm::launch_kernel(plan->d, plan->b, plan->dtype, kids[k], s) != hipSuccess) st = DFM_E_HIP;
    if (st == DFM_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = DFM_E_HIP;
    avg_ms[k] = ms / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Timing events skip the system-scope fence at record time: they only order work on the
// stream, and a fence per launch would slow the run being measured.
dfm_status dfm_profile_kernel(dfm_plan* plan, int32_t kernel, int32_t max_launches) {
  if (!plan || kernel >= dfm_kernel_count(plan) || (kernel >= 0 && max_launches < 1)) return DFM_E_ARG;
  dfm::free_profile(plan);
  if (kernel < 0) return DFM_OK;
  int kids[16];
  dfm::iteration_kernels(plan->d, kids);
  kernel = kids[kernel];
  plan->prof_events.resize(2 * (size_t)max_launches);
  for (size_t i = 0; i < plan->prof_events.size(); ++i)
    if (hipEventCreateWithFlags(&plan->prof_events[i], hipEventDisableSystemFence) != hipSuccess) {
      plan->prof_events.resize(i);
      dfm::free_profile(plan);
      return DFM_E_HIP;
    }
  plan->prof_kid = kernel;
  return DFM_OK;
}

dfm_status dfm_profile_read(dfm_plan* plan, double* avg_ms, int64_t* launches, void* stream) {
  if (!plan || !avg_ms || !launches) return DFM_E_ARG;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return DFM_E_HIP;
  double total = 0.0;
  const size_t n = plan->prof_used / 2;
  for (size_t i = 0; i < n; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, plan->prof_events[2 * i], plan->prof_events[2 * i + 1]) != hipSuccess)
      return DFM_E_HIP;
    total += ms;
  }
  *launches = (int64_t)n;
  *avg_ms = n ? total / n : 0.0;
  plan->prof_used = 0;
  return DFM_OK;
}

namespace {

dfm_status grad_tape_size(const dfm_plan* plan, int32_t n_iter, bool full, size_t* bytes) {
  if (!plan || !bytes || n_iter < 0) return DFM_E_ARG;
  if (full && plan->d.MLX > 16) return DFM_E_SHAPE;
  *bytes = dfm::grad_tape_bytes(plan->d, plan->dtype, n_iter, full);
  return DFM_OK;
}

dfm_status grad_tape_ok(const dfm_plan* plan, int32_t n_iter, bool full, const void* tape, size_t tape_bytes) {
  if (full && plan->d.MLX > 16) return DFM_E_SHAPE;
  if (reinterpret_cast<uintptr_t>(tape) % 256 != 0 ||
      tape_bytes < dfm::grad_tape_bytes(plan->d, plan->dtype, n_iter, full))
    return DFM_E_WORKSPACE;
  return DFM_OK;
}

// n_iter iterations on the plan's kernels, each after storing the state it starts from in the tape;
// full: every stage (eqs. (14)-(16), then (8)-(10)), else the MM stages with Q fixed.
dfm_status grad_forward(dfm_plan* plan, int32_t n_iter, bool full, void* tape, size_t tape_bytes, void* stream) {
  if (!plan || n_iter < 0 || (n_iter > 0 && !tape)) return DFM_E_ARG;
  if (n_iter > 0) {
    const dfm_status st = grad_tape_ok(plan, n_iter, full, tape, tape_bytes);
    if (st != DFM_OK) return st;
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const Dims& d = plan->d;
  const size_t r = plan->dtype == DFM_C64 ? 4 : 8;
  if (n_iter > 0 && d.fast >= 0 && dfm::run_kernel(plan, dfm::kFLam, s) != hipSuccess) return DFM_E_HIP;
  for (int it = 0; it < n_iter; ++it) {
    void *cQ, *cg, *cW, *cH;
    dfm::grad_checkpoints(d, plan->dtype, n_iter, full, tape, it, &cQ, &cg, &cW, &cH);
    if (hipMemcpyAsync(cg, plan->b.g, r * d.F * d.N * d.M, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(cW, plan->b.W, r * d.N * d.F * d.K, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(cH, plan->b.H, r * d.N * d.K * d.T, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return DFM_E_HIP;
    if (full && hipMemcpyAsync(cQ, plan->b.Q, 2 * r * d.F * d.QF, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return DFM_E_HIP;
    for (int stage = full ? DFM_STAGE_IP : DFM_STAGE_W; stage <= DFM_STAGE_G; ++stage)
      if (dfm::run_stage(plan, stage, s) != hipSuccess) return DFM_E_HIP;
    if (dfm::g_update_deferred(d) && dfm::run_kernel(plan, dfm::kFGFin, s) != hipSuccess) return DFM_E_HIP;
  }
  return DFM_OK;
}

dfm_status grad_backward(dfm_plan* plan, int32_t n_iter, bool full, void* tape, size_t tape_bytes, void* dQ,
                         void* dg, void* dW, void* dH, void* stream) {
  if (!plan || n_iter < 0 || !tape || !dQ || !dg || !dW || !dH) return DFM_E_ARG;
  const dfm_status st = grad_tape_ok(plan, n_iter, full, tape, tape_bytes);
  if (st != DFM_OK) return st;
  if (dfm::launch_grad_backward(plan->d, plan->b, plan->dtype, n_iter, full, tape, dQ, dg, dW, dH,
                                static_cast<hipStream_t>(stream)) != hipSuccess)
    return DFM_E_HIP;
  return DFM_OK;
}

}  // namespace

dfm_status dfm_mm_tape_size(const dfm_plan* plan, int32_t n_iter, size_t* bytes) {
  return grad_tape_size(plan, n_iter, false, bytes);
}

dfm_status dfm_mm_forward(dfm_plan* plan, int32_t n_iter, void* tape, size_t tape_bytes, void* stream) {
  return grad_forward(plan, n_iter, false, tape, tape_bytes, stream);
}

dfm_status dfm_mm_backward(dfm_plan* plan, int32_t n_iter, void* tape, size_t tape_bytes, void* dQ, void* dg,
                           void* dW, void* dH, void* stream) {
  return grad_backward(plan, n_iter, false, tape, tape_bytes, dQ, dg, dW, dH, stream);
}

dfm_status dfm_iter_tape_size(const dfm_plan* plan, int32_t n_iter, size_t* bytes) {
  return grad_tape_size(plan, n_iter, true, bytes);
}

dfm_status dfm_iter_forward(dfm_plan* plan, int32_t n_iter, void* tape, size_t tape_bytes, void* stream) {
  return grad_forward(plan, n_iter, true, tape, tape_bytes, stream);
}

dfm_status dfm_iter_backward(dfm_plan* plan, int32_t n_iter, void* tape, size_t tape_bytes, void* dQ, void* dg,
                             void* dW, void* dH, void* stream) {
  return grad_backward(plan, n_iter, true, tape, tape_bytes, dQ, dg, dW, dH, stream);
}

dfm_status dfm_initialise_workspace_size(const dfm_problem* p, size_t* bytes) {
  if (!bytes) return DFM_E_ARG;
  Dims d;
  const dfm_status st = dfm::make_dims(p, d);
  if (st != DFM_OK) return st;
  if (d.N < 2) return DFM_E_SHAPE;
  *bytes = dfm::initialise_workspace_bytes(d);
  return DFM_OK;
}

dfm_status dfm_initialise(const dfm_problem* p, const void* C, void* Q, void* g, void* h, void* workspace,
                          size_t workspace_bytes, void* stream) {
  Dims d;
  const dfm_status st = dfm::make_dims(p, d);
  if (st != DFM_OK) return st;
  if (d.N < 2) return DFM_E_SHAPE;
  if (!C || !Q || !g || !workspace) return DFM_E_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0 || workspace_bytes < dfm::initialise_workspace_bytes(d))
    return DFM_E_WORKSPACE;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (dfm::launch_initialise(d, p->dtype, C, Q, g, h, workspace, s) != hipSuccess) return DFM_E_HIP;
  int status = 0;
  if (hipMemcpyAsync(&status, dfm::initialise_status(d, workspace), sizeof(int), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return DFM_E_HIP;
  return status & dfm::kStSingular ? DFM_E_SINGULAR : DFM_OK;
}

}  // extern "C"

// ---- The workspace of dfm_run_noalloc: a static device array, one per GPU.  In host code
// `scratch` names a host-side stand-in, not the array: its device address on the current GPU
// comes from hipGetSymbolAddress, taken once per device and kept in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[DFM_NOALLOC_SCRATCH_BYTES];

namespace dfm {

constexpr int kMaxDevices = 64;
static void* scratch_ptr[kMaxDevices];
static std::mutex scratch_mu;

// Device address of `scratch` on the current GPU (looked up on the first call per device), or
// nullptr on a HIP error.
static void* scratch_address() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    scratch_ptr[dev] = ptr;
  }
  return scratch_ptr[dev];
}

}  // namespace dfm

extern "C" {

dfm_status dfm_run_noalloc(const dfm_problem* p, const void* X, void* Q, void* g, void* W, void* H,
                           int32_t n_iter, double* cost, int32_t* status, void* stream) {
  Dims d;
  const dfm_status st = dfm::make_dims(p, d);
  if (st != DFM_OK) return st;
  if (!X || !Q || !g || !W || !H || n_iter < 0 || (p->flags & DFM_F_TRACE_NLL)) return DFM_E_ARG;
  if (dfm::workspace_bytes(d, p->dtype) > DFM_NOALLOC_SCRATCH_BYTES) return DFM_E_WORKSPACE;
  void* ws = dfm::scratch_address();
  if (!ws) return DFM_E_HIP;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // A plan on the stack (its vector of profiling events stays empty: nothing is allocated),
  // plain launches only.
  dfm_plan plan;
  plan.d = d;
  plan.dtype = p->dtype;
  plan.graph_off = true;
  std::memset(&plan.b, 0, sizeof(plan.b));
  plan.b.X = X;
  plan.b.Q = Q;
  plan.b.g = g;
  plan.b.W = W;
  plan.b.H = H;
  dfm::carve(d, p->dtype, static_cast<char*>(ws), plan.b);
  if (dfm::launch_init(d, plan.b, s) != hipSuccess) return DFM_E_HIP;  // status and trace counter
  const dfm_status r = dfm_step(&plan, n_iter, stream);
  if (r != DFM_OK) return r;
  if (cost && (dfm::launch_nll(d, plan.b, plan.dtype, s) != hipSuccess ||
               dfm::launch_nll_total(d, plan.b, cost, false, s) != hipSuccess))
    return DFM_E_HIP;
  if (status && dfm::launch_copy_status(plan.b, status, s) != hipSuccess) return DFM_E_HIP;
  return DFM_OK;
}

}  // extern "C"

// ---- Batches: all plans' iterations captured into one graph per phase, each plan a branch
// forked from and joined into the capture's origin stream.
struct dfm_batch {
  std::vector<dfm_plan*> plans;
  std::vector<hipStream_t> streams;  // one capture branch per plan
  hipStream_t origin = nullptr;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
  // [0] lambda seeds + first iteration, [1] one later iteration, [2] kGraphBatch later ones,
  // [3] the final g updates (plans whose g update is finished by the next covariance kernel).
  hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace dfm {

static void free_batch(dfm_batch* b) {
  for (hipGraphExec_t& g : b->graph)
    if (g) (void)hipGraphExecDestroy(g);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->joins) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->origin) (void)hipStreamDestroy(b->origin);
  delete b;
}

// What plan p enqueues in phase `which` on stream s.
static hipError_t batch_phase(dfm_plan* p, int which, hipStream_t s) {
  const bool trace = (p->d.flags & DFM_F_TRACE_NLL) != 0;
  hipError_t e = hipSuccess;
  switch (which) {
    case 0:
      if (p->d.fast >= 0) e = run_kernel(p, kFLam, s);
      if (e == hipSuccess) e = enqueue_iteration(p, true, s);
      return e;
    case 1: return enqueue_iteration(p, false, s);
    case 2:
      for (int r = 0; r < kGraphBatch && e == hipSuccess; ++r) e = enqueue_iteration(p, false, s);
      return e;
    default:
      if (g_update_deferred(p->d) && !trace) e = run_kernel(p, kFGFin, s);
      return e;
  }
}

static hipError_t capture_batch(dfm_batch* b, int which) {
  hipError_t e = hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  e = hipEventRecord(b->fork, b->origin);
  for (size_t i = 0; i < b->plans.size() && e == hipSuccess; ++i) {
    e = hipStreamWaitEvent(b->streams[i], b->fork, 0);
    if (e == hipSuccess) e = batch_phase(b->plans[i], which, b->streams[i]);
    if (e == hipSuccess) e = hipEventRecord(b->joins[i], b->streams[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->origin, b->joins[i], 0);
  }
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(b->origin, &g);
  if (e == hipSuccess) e = ee;
  if (e == hipSuccess && g) e = hipGraphInstantiate(&b->graph[which], g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) b->graph[which] = nullptr;
  return e;
}

}  // namespace dfm

extern "C" {

dfm_status dfm_batch_create(dfm_batch** out, dfm_plan* const* plans, int32_t count) {
  if (!out || !plans || count < 1 || count > 4096) return DFM_E_ARG;
  *out = nullptr;
  for (int32_t i = 0; i < count; ++i) {
    if (!plans[i]) return DFM_E_ARG;
    for (int32_t j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return DFM_E_ARG;
  }
  dfm_batch* b = new (std::nothrow) dfm_batch;
  if (!b) return DFM_E_ARG;
  b->plans.assign(plans, plans + count);
  bool ok = hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
  for (int32_t i = 0; i < count && ok; ++i) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    if (ok) b->streams.push_back(s);
    ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    if (ok) b->joins.push_back(e);
  }
  if (!ok) {
    dfm::free_batch(b);
    return DFM_E_HIP;
  }
  *out = b;
  return DFM_OK;
}

dfm_status dfm_batch_step(dfm_batch* batch, int32_t n_iter, void* stream) {
  if (!batch || n_iter < 0) return DFM_E_ARG;
  if (n_iter == 0) return DFM_OK;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  auto launch = [&](int which) -> bool {
    if (!batch->graph[which] && dfm::capture_batch(batch, which) != hipSuccess) return false;
    return hipGraphLaunch(batch->graph[which], s) == hipSuccess;
  };
  if (!launch(0)) return DFM_E_HIP;
  int left = n_iter - 1;
  while (left > 0) {
    const int which = left >= dfm::kGraphBatch ? 2 : 1;
    if (!launch(which)) return DFM_E_HIP;
    left -= which == 2 ? dfm::kGraphBatch : 1;
  }
  return launch(3) ? DFM_OK : DFM_E_HIP;
}

void dfm_batch_destroy(dfm_batch* batch) {
  if (batch) dfm::free_batch(batch);
}

void dfm_destroy(dfm_plan* plan) {
  if (!plan) return;
  dfm::free_profile(plan);
  dfm::free_graphs(plan);
  delete plan;
}

const char* dfm_status_string(dfm_status s) {
  switch (s) {
    case DFM_OK: return "ok";
    case DFM_E_ARG: return "invalid argument";
    case DFM_E_SHAPE: return "shape or partition out of range";
    case DFM_E_WORKSPACE: return "workspace too small or misaligned";
    case DFM_E_HIP: return "HIP runtime error";
    case DFM_E_NONFINITE: return "a parameter became non-finite";
    case DFM_E_SINGULAR: return "singular iterative-projection system";
  }
  return "unknown status";
}

}  // extern "C"
