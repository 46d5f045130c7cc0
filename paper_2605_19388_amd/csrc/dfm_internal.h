// Internal interface between the C ABI (dfm_api.cpp) and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "dfmnmf.h"

namespace dfm {

constexpr int kMaxL = DFM_MAX_SUBARRAYS;
constexpr int kMaxM = DFM_MAX_MICS;
constexpr int kMaxMl = DFM_MAX_SUBARRAY_MICS;
constexpr int kMaxN = DFM_MAX_SOURCES;
constexpr int kMaxK = DFM_MAX_BASES;
constexpr int kBlock = 256;  // threads per workgroup of the streaming kernels

// Sticky device status bits (workspace word).
constexpr int kStSingular = 1;
constexpr int kStNonFinite = 2;
constexpr int kTraceSlot = 4;  // int index of the cost-trace counter in the status area

// Problem geometry, passed by value to every kernel.
struct Dims {
  int F, T, N, K, L, M;
  int QF;  // complex entries of Q per frequency: sum_l M_l^2
  int VF;  // reals of the packed covariances per frequency: sum_l M_l^3
  int VC;  // complex entries of the full covariances per frequency: sum_l M_l^3
  int S, SL;    // time slices per frequency and frames per slice (streaming tiles)
  int FB, FS;   // frequencies per tile and number of frequency tiles (activation update)
  int TB, TBN;  // frames per tile and number of frame tiles (activation update)
  double eps;
  int fast;  // index of the shape-specialised kernel set, or -1 for the generic kernels
  int ML;    // common subarray size when the partition is uniform, else 0
  int MLX;   // largest subarray size
  int SLP;   // LDS row stride (elements) of per-frame arrays in the specialised kernels
  int TP;    // frames rounded up to 16: row length of the coefficient planes (specialised kernels)
  int SG;    // partial-sum slots per bin of the covariances (S slices, or balanced ranges, below)
  int GR;    // k_gramd_f: flattened (f, t) frames per workgroup (0: per-slice partials)
  int GSB;   // covariance workgroups per bin when every bin gets the same number (0: equal flat ranges)
  int GW;    // k_gramd_f: workgroups
  int GGR;   // k_g_f: flattened (f, t) frames per workgroup
  int GGW;   // k_g_f: workgroups
  int GGS;   // k_g_f: partial-sum slots per bin
  int HC;    // LDS windows of W[n] in the H update: above 1, k_hsum_f / k_hlam_f replace k_hgemm_f
  int gpend;  // k_gramd_f finishes the previous iteration's g update (set inside dfm_step only)
  int check;  // DFM_F_CHECK_FINITE: updated W, H, g are checked for NaN / Inf
  int flags;  // dfm_problem.flags
  int tile;   // largest frames per slice (16, 32, 64 or 128)
  int mics[kMaxL];  // M_l
  int moff[kMaxL];  // first mic of subarray l
  int qoff[kMaxL];  // offset of block l in a frequency's packed Q (complex units)
  int voff[kMaxL];  // offset of block l in a frequency's covariances (sum_{l'<l} M_l'^3)
  int msub[kMaxM];  // subarray of each mic
};

// Device buffers of one plan (all carved from the caller's workspace except the state).
struct Buffers {
  const void* X;
  void* Q;
  void* g;
  void* W;
  void* H;
  void* P;       // [F][T][M] real: |Q x|^2 of the latest W sub-step
  void* Vpart;   // [F][SG][VF] double: packed covariance sums (FP64 on every path)
  void* Wpart;   // [F][S][N][K][2] real (generic kernels)
  void* Hpart;   // generic: [FS][N][K][T][2] real; specialised with HC > 1: [N][TBN][HC][2][KP][16] real
  void* Hsnap;   // [N][K][T] real (specialised with HC > 1): the H that the H update multiplies
  void* gpart;   // generic: [F][S][N][M][2] real; specialised: [F][GGS][2][N][M] real
  void* gsnap;   // [F][N][M] real (specialised): the g that a pending g update multiplies
  double* logdet;   // [F][L]
  double* nllpart;  // [F][S]
  void* Qinv;       // [F][QF] complex double
  int* status;      // [0] sticky status word, [kTraceSlot] iterations recorded in the cost trace
  double* nlltot;   // cost (13) total of the latest dfm_nll
  double* trace;    // [DFM_TRACE_CAPACITY] costs after each iteration (DFM_F_TRACE_NLL)
  void* lam;           // [F][N][T] real: lambda = W H of the specialised kernels
  void* AB;            // [2N][TBN][F][16] real: per-bin MM coefficients of the specialised kernels
};

size_t workspace_bytes(const Dims& d, int dtype);
void carve(const Dims& d, int dtype, char* ws, Buffers& b);

// Kernels.  Generic path: eight per iteration; specialised path: seven (kFLam seeds
// lambda = W H).
enum KernelId {
  kKGram = 0, kKIp, kKPw, kKWApply, kKH, kKHApply, kKG, kKGApply,
  kFGram, kFIp, kFPw, kFWGemm, kFH, kFHGemm, kFG, kFLam, kFGFin, kFHLam, kNumKernels
};

// Launchers (return hipSuccess or the first launch error).
hipError_t launch_init(const Dims& d, const Buffers& b, hipStream_t s);
hipError_t launch_kernel(const Dims& d, const Buffers& b, int dtype, int kid, hipStream_t s);
const char* kernel_name(int kid);
int stage_kernels(const Dims& d, int stage, int* kids);  // fills kids, returns count
// Specialised sets whose covariance kernel is k_gramd_f: the G stage ends with k_g_f's partial
// sums, and the g update is finished by the next k_gramd_f (Dims::gpend) or by k_gfin_f.
inline bool g_update_deferred(const Dims& d) { return d.fast >= 0 && d.GR > 0; }
int iteration_kernels(const Dims& d, int* kids);         // fills kids, returns count

// Shape-specialised kernel sets (dfm_fast.hip).
int fast_set_index(int N, int K, int ML, int L);
bool fast_fp64_ok(int set);  // the set also runs FP64 plans
size_t fast_max_smem(const Dims& d, int dtype);
int fast_hgemm_windows(const Dims& d, int dtype);  // LDS windows of W[n] in the H update
int fast_gramd_blocks_per_cu(const Dims& d);  // resident k_gramd_f / k_gramb_f workgroups per CU (0: unknown)
bool fast_gram_bf16(int N, int K, int ML, int L);  // the set has the BF16 covariance kernel
hipError_t fast_launch(const Dims& d, const Buffers& b, int dtype, int kid, hipStream_t s);
const char* fast_kernel_name(const Dims& d, int dtype, int kid);  // symbol family a kernel id runs
// Cost (13) partials or the Wiener filter with the specialised kernels (M_l <= 4).
hipError_t fast_finish(const Dims& d, const Buffers& b, int dtype, bool separate, void* S, hipStream_t s);
hipError_t launch_nll(const Dims& d, const Buffers& b, int dtype, hipStream_t s);
// Total of the cost (13) from the partials of launch_nll, in a fixed order, to *out; with
// `trace`, also appended to b.trace at the counter status[kTraceSlot] (then incremented).
hipError_t launch_nll_total(const Dims& d, const Buffers& b, double* out, bool trace, hipStream_t s);
hipError_t launch_clear_status(const Buffers& b, hipStream_t s);  // sticky word only
hipError_t launch_copy_status(const Buffers& b, int* out, hipStream_t s);  // sticky word -> out
hipError_t launch_separate(const Dims& d, const Buffers& b, int dtype, void* S, hipStream_t s);
hipError_t launch_covariances(const Dims& d, const Buffers& b, int dtype, void* V, hipStream_t s);

hipError_t launch_qinv(const Dims& d, const Buffers& b, int dtype, hipStream_t s);  // Q^-1 -> b.Qinv (generic)

// Gradient of the cost after unrolled MM iterations (full = false) or full iterations
// (dfm_grad.hip).  Q's checkpoint exists for full iterations only (*Q = nullptr otherwise).
size_t grad_tape_bytes(const Dims& d, int dtype, int n_iter, bool full);
void grad_checkpoints(const Dims& d, int dtype, int n_iter, bool full, void* tape, int it, void** Q, void** g,
                      void** W, void** H);
hipError_t launch_grad_backward(const Dims& d, const Buffers& b, int dtype, int n_iter, bool full, void* tape,
                                void* dQ, void* dg, void* dW, void* dH, hipStream_t s);

// Initial parameters from source-image estimates (dfm_init.hip).
size_t initialise_workspace_bytes(const Dims& d);
hipError_t launch_initialise(const Dims& d, int dtype, const void* C, void* Q, void* g, void* h, void* ws,
                             hipStream_t s);
int* initialise_status(const Dims& d, void* ws);  // sticky word inside the workspace

}  // namespace dfm
