/*
 * dfmnmf.h -- C ABI of distributed FastMNMF on AMD MI355X (gfx950).
 *
 * Distributed FastMNMF (Sec. III-B of the paper) separates N sources from a
 * multichannel STFT observed by L subarrays.  The source spatial covariances
 * are block-diagonal over the subarray partition (eq. (11)) and jointly
 * diagonalised within each block (eq. (12)); the source power spectrograms
 * are an NMF with K bases per source (eq. (2)), shared by all subarrays.
 * One iteration updates, in this order (Sec. III-B):
 *   - every subarray's transformation Q_fl by iterative projection,
 *     eqs. (14)-(16), rows in ascending order;
 *   - the bases W (eq. (8)), activations H (eq. (9)) and diagonal SCMs g
 *     (eq. (10)), the model variance refreshed after each.
 *
 * Symbols (paper -> this ABI): frequency i -> f (F bins), frame j -> t
 * (T frames), W_i^(l)H -> Q_fl (row mu is w_mu^H), t_ikn -> W[n][f][k],
 * v_kjn -> H[n][k][t], [Lambda_in]_mm -> g[f][n][m].
 *
 * Every device buffer is owned by the caller.  The library never allocates
 * device memory: its temporaries live in the caller's workspace.  All
 * pointers below are device pointers unless stated otherwise; "stream" is a
 * hipStream_t passed as void* (NULL = the default stream).  Calls are
 * asynchronous on that stream unless stated otherwise.  A plan is used by one
 * stream at a time; plans are independent of each other.
 *
 * Errors: every call returns a dfm_status; nothing else crosses the ABI.
 * Argument and shape errors are found on the host before anything is
 * launched.  Conditions found on the device (a singular IP system, a
 * non-finite parameter) are recorded in a sticky word in the workspace and
 * returned by the next synchronising call (dfm_nll, dfm_sync_status).
 */
#ifndef DFMNMF_H
#define DFMNMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DFM_MAX_SUBARRAYS 64   /* L <= 64 */
#define DFM_MAX_MICS 64        /* M = sum_l M_l <= 64 */
#define DFM_MAX_SUBARRAY_MICS 32 /* M_l <= 32 */
#define DFM_MAX_SOURCES 16     /* N <= 16 */
#define DFM_MAX_BASES 64       /* K <= 64 */

typedef enum {
  DFM_C64 = 0,   /* complex64 observations and Q; float32 g, W, H */
  DFM_C128 = 1   /* complex128 observations and Q; float64 g, W, H */
} dfm_dtype;

typedef enum {
  DFM_OK = 0,
  DFM_E_ARG = 1,        /* null pointer, bad enum, n_iter < 0, eps <= 0 */
  DFM_E_SHAPE = 2,      /* F, T, N, K, L or a subarray size out of range */
  DFM_E_WORKSPACE = 3,  /* workspace smaller than dfm_workspace_size() */
  DFM_E_HIP = 4,        /* a HIP runtime call or kernel launch failed */
  DFM_E_NONFINITE = 5,  /* a parameter became NaN or Inf on the device */
  DFM_E_SINGULAR = 6    /* an IP system (Q_fl V_flmu) had a zero pivot */
} dfm_status;

/* Bits of dfm_problem.flags. */
#define DFM_F_CHECK_FINITE 1u  /* check every updated W, H, g for NaN/Inf on the device; a
                                  non-finite value sets DFM_E_NONFINITE in the sticky status */
#define DFM_F_TRACE_NLL 2u     /* evaluate the cost (13) after every iteration of dfm_step on
                                  the device into a trace read by dfm_nll_trace (costs one extra
                                  pass over X per iteration) */
#define DFM_F_GRAM_BF16 4u     /* weighted covariances of eq. (14) from BF16 operands on the
                                  matrix cores with FP32 sums (the IP solves, the eq. (16)
                                  normalisation and ln|det Q| stay FP64); complex64 plans of a
                                  uniform partition into 2- or 4-mic subarrays with a compiled
                                  (N, K, M_l, L) set, else DFM_E_ARG */
#define DFM_F_NO_GRAPH 8u      /* dfm_step issues plain kernel launches instead of replaying
                                  HIP graphs of its iterations (same kernels, same results) */
#define DFM_TRACE_CAPACITY 4096 /* entries of the cost trace; later iterations are counted
                                   but not stored */

/* Sub-steps of one iteration, for dfm_substep (in this order). */
typedef enum {
  DFM_STAGE_IP = 0,  /* V by eq. (14) from the current W,H,g; IP sweep, eqs. (15)-(16) */
  DFM_STAGE_W = 1,   /* P = |Q x|^2 for the current Q; bases update, eq. (8) */
  DFM_STAGE_H = 2,   /* activations update, eq. (9) (uses P from DFM_STAGE_W) */
  DFM_STAGE_G = 3    /* diagonal SCM update, eq. (10) (uses P from DFM_STAGE_W) */
} dfm_stage;

typedef struct {
  int32_t F;                        /* frequency bins, >= 1 */
  int32_t T;                        /* frames, >= 1 */
  int32_t N;                        /* sources, 1..DFM_MAX_SOURCES */
  int32_t K;                        /* NMF bases per source, 1..DFM_MAX_BASES */
  int32_t L;                        /* subarrays, 1..DFM_MAX_SUBARRAYS */
  int32_t mics[DFM_MAX_SUBARRAYS];  /* M_l in 1..DFM_MAX_SUBARRAY_MICS (sum <= DFM_MAX_MICS); subarray l
                                       owns X columns o_l .. o_l+M_l-1, o_l = sum_{l'<l} M_l' */
  int32_t dtype;                    /* dfm_dtype */
  double eps;                       /* floor on the model variance, the MM denominators
                                       and the IP normaliser (1e-6 in Sec. IV-A); > 0 */
  uint32_t flags;                   /* DFM_F_* bits; unknown bits are DFM_E_ARG */
  int32_t tile;                     /* largest frames per slice of the streaming kernels:
                                       0 (= 128), 16, 32, 64 or 128, else DFM_E_ARG (a
                                       performance choice; results stay within rounding) */
} dfm_problem;

typedef struct dfm_plan dfm_plan;   /* opaque host-side handle */

/* Bytes of device workspace a plan for *p needs (host-only call).
 * Returns DFM_E_ARG / DFM_E_SHAPE for an invalid problem. */
dfm_status dfm_workspace_size(const dfm_problem* p, size_t* bytes);

/* Create a plan bound to caller-owned device buffers (all borrowed for the
 * plan's lifetime, none copied):
 *   X [F][T][M] complex, interleaved (re, im); read-only.  The STFT x_ft of
 *     Sec. II-A with the mics of one subarray contiguous (Sec. III-B).
 *   Q [F][sum_l M_l^2] complex; block l is M_l x M_l row-major at offset
 *     sum_{l'<l} M_l'^2; row mu is w_mu^H.  Must be nonsingular (Sec. IV-A).
 *   g [F][N][M] real > 0;  W [N][F][K] real > 0;  H [N][K][T] real > 0.
 *   Q, g, W, H are the state: read and updated in place by dfm_step.
 *   workspace: >= dfm_workspace_size() bytes, 256-byte aligned.
 * Launches a small initialisation kernel on `stream`.
 * On success *out receives the plan; release it with dfm_destroy. */
dfm_status dfm_init(dfm_plan** out, const dfm_problem* p,
                    const void* X, void* Q, void* g, void* W, void* H,
                    void* workspace, size_t workspace_bytes, void* stream);

/* Run n_iter >= 0 full iterations (IP sweep, then eqs. (8), (9), (10)),
 * updating Q, g, W, H in place.  Asynchronous.  Unless DFM_F_NO_GRAPH is set,
 * the kernels of one iteration (and of a batch of eight) are captured once per
 * plan, on a stream the plan owns, into HIP graphs that are then replayed on
 * `stream`; the plan's buffers are fixed, so a replay runs exactly the kernels
 * and arguments of a plain launch.  While dfm_profile_kernel is active the
 * launches are plain. */
dfm_status dfm_step(dfm_plan* plan, int32_t n_iter, void* stream);

/* Run one sub-step of an iteration (dfm_stage).  Asynchronous.  A full
 * iteration is exactly IP, W, H, G in this order; H and G read the powers
 * computed by the latest W sub-step. */
dfm_status dfm_substep(dfm_plan* plan, int32_t stage, void* stream);

/* Cost (13) of the current state: sum_{f,t,m} (|Q x|^2 / y + ln y)
 * - 2T sum_{f,l} ln|det Q_fl|, terms in the plan's precision, the sums and
 * the total in FP64 on the device (fixed order); only the 8-byte total is
 * copied to the host.  Synchronises `stream`; *out is a host pointer.  Also
 * returns any sticky device error. */
dfm_status dfm_nll(dfm_plan* plan, double* out, void* stream);

/* With DFM_F_TRACE_NLL: copy the costs (13) recorded after each iteration of
 * dfm_step since dfm_init (the first min(count, capacity, DFM_TRACE_CAPACITY)
 * of them) to the host array out[capacity], and the number of iterations
 * recorded to *count.  Synchronises `stream`.  DFM_E_ARG without the flag. */
dfm_status dfm_nll_trace(dfm_plan* plan, double* out, int32_t capacity, int32_t* count, void* stream);

/* Source images at every subarray by the multichannel Wiener filter
 * (Sec. III-B, last paragraph): for each subarray l,
 *   S_n^(l)[f][t] = Q_fl^{-1} diag(lambda_ftn g_fn / y_ft) Q_fl x_ft^(l)
 * with lambda = W_n H_n (eq. (2)) and y = max(sum_n lambda g, eps).
 * S [N][F][T][M] complex, caller-owned, written entirely.  Asynchronous. */
dfm_status dfm_separate(dfm_plan* plan, void* S, void* stream);

/* Weighted covariances of eq. (14) for the current W, H, g, written as
 * V [F][sum_l M_l^3] complex: block l at offset sum_{l'<l} M_l'^3, laid out
 * [mu][a][b] = V_flmu[a][b] (full Hermitian matrices).  Diagnostic; does
 * not change the state.  Asynchronous. */
dfm_status dfm_covariances(dfm_plan* plan, void* V, void* stream);

/* Wait for `stream` and return the sticky device status (DFM_OK,
 * DFM_E_SINGULAR or DFM_E_NONFINITE); clears it. */
dfm_status dfm_sync_status(dfm_plan* plan, void* stream);

/* ---- Measurement (not part of the method; used to price kernels against the roofline).
 * The kernels of one iteration of a plan are numbered 0 .. dfm_kernel_count(plan)-1 in
 * launch order (seven or eight; the streaming kernels are shape-specialised for
 * uniform partitions with a compiled (N, K, M_l, L) set).  Where the covariance
 * kernel of the next iteration finishes the g update, the kernel that finishes
 * the last one runs once per dfm_step call and is not among them. */
int32_t dfm_kernel_count(const dfm_plan* plan);
/* Static name of kernel i of the plan's iteration, or NULL if out of range. */
const char* dfm_kernel_name(const dfm_plan* plan, int32_t kernel);
/* Launch each kernel `reps` >= 1 times back to back between two HIP events on
 * `stream` and write its average duration in ms to avg_ms[i] (host array of
 * dfm_kernel_count(plan) doubles).  Synchronises.  Repeated launches of the
 * update kernels change Q, g, W, H: save and restore the state around it. */
dfm_status dfm_kernel_times(dfm_plan* plan, int32_t reps, double* avg_ms, void* stream);
/* From now on bracket every launch of kernel `kernel` made by dfm_step /
 * dfm_substep with a pair of HIP events on the launch stream, for at most
 * max_launches launches; kernel = -1 stops and frees the events. */
dfm_status dfm_profile_kernel(dfm_plan* plan, int32_t kernel, int32_t max_launches);
/* Synchronise `stream`, return the average event-measured duration (ms) and
 * the number of profiled launches since the last read, and reset the count. */
dfm_status dfm_profile_read(dfm_plan* plan, double* avg_ms, int64_t* launches, void* stream);

/* ---- Gradient of the cost after unrolled MM iterations.
 * The map: from the plan's state (Q, g, W, H), n_iter iterations of the MM updates
 * (8), (9), (10) in that order with Q held fixed (P = |Q x|^2 fixed, y refreshed
 * after each update, every Sec. IV-A floor in place), then the cost (13).
 * dfm_mm_forward runs those iterations on the plan's kernels (updating g, W, H in
 * place) and stores the state (g, W, H) before each iteration in `tape` (per-
 * iteration checkpoints).  dfm_mm_backward, called after it with the same n_iter
 * and tape and with the state it left, computes by hand-written reverse-mode
 * kernels (FP64 internally) the gradient of that cost with respect to the state
 * before the forward: dQ [F][sum_l M_l^2] complex = dL/dRe Q + i dL/dIm Q, dg
 * [F][N][M], dW [N][F][K], dH [N][K][T] real (plan precision, caller-owned,
 * written entirely).  A floored quantity has zero derivative where its floor is
 * active.  n_iter = 0 gives the gradient of the cost at the current state (at a
 * fixed point of (8)-(10), dg = dW = dH = 0).  The tape (caller-owned, 256-byte
 * aligned, >= dfm_mm_tape_size bytes) also holds the reverse pass's FP64 work
 * arrays.  Asynchronous; the IP sweep (14)-(16) is not part of the map. */
dfm_status dfm_mm_tape_size(const dfm_plan* plan, int32_t n_iter, size_t* bytes);
dfm_status dfm_mm_forward(dfm_plan* plan, int32_t n_iter, void* tape, size_t tape_bytes, void* stream);
dfm_status dfm_mm_backward(dfm_plan* plan, int32_t n_iter, void* tape, size_t tape_bytes, void* dQ, void* dg,
                           void* dW, void* dH, void* stream);

/* ---- Gradient of the cost after unrolled full iterations.
 * The map: from the plan's state (Q, g, W, H), n_iter iterations of dfm_step's
 * schedule -- the covariances (14) from the current model, the IP sweep (15)-(16)
 * of every subarray's rows in ascending order, P = |Q x|^2 for the new Q, then the
 * MM updates (8), (9), (10) -- and the cost (13) of the final state, every Sec.
 * IV-A floor in place (the IP normaliser of (16) floored at eps too).
 * dfm_iter_forward runs the iterations on the plan's kernels and stores the state
 * (Q, g, W, H) before each in `tape`; dfm_iter_backward, called after it with the
 * same n_iter and tape and with the state it left, computes by hand-written
 * reverse-mode kernels (FP64 internally) the gradient with respect to the state
 * before the forward, in the layouts and conventions of dfm_mm_backward.  Each
 * iteration's sweep is recomputed in FP64 from its checkpoint and differentiated
 * row by row; through (14) the gradient reaches g, W and H a second way.  After
 * one or more iterations the gradient with respect to the first row of each
 * block of Q is zero (the sweep overwrites that row first, fixed up to a phase
 * by the other rows).  Subarrays of up to 16 mics (DFM_E_SHAPE beyond); tape
 * caller-owned, 256-byte aligned, >= dfm_iter_tape_size bytes.  Asynchronous. */
dfm_status dfm_iter_tape_size(const dfm_plan* plan, int32_t n_iter, size_t* bytes);
dfm_status dfm_iter_forward(dfm_plan* plan, int32_t n_iter, void* tape, size_t tape_bytes, void* stream);
dfm_status dfm_iter_backward(dfm_plan* plan, int32_t n_iter, void* tape, size_t tape_bytes, void* dQ, void* dg,
                             void* dW, void* dH, void* stream);

/* ---- Initial parameters from estimates of the source images (Sec. IV-A, steps 3, 5, 6).
 * The paper initialises from source images estimated by time-frequency masking
 * (its steps 1-2) and factorises the initial spectrograms by IS-NMF (step 4);
 * those are separate methods and the caller's.  From the image estimates
 *   C [N][F][T][M] complex (c_ftn, the dtype of *p), read-only,
 * dfm_initialise computes, all in FP64:
 *   R_fn = (1/T) sum_t c_ftn c_ftn^H (M x M, across subarrays) and
 *   h [N][F][T] real = c_ftn^H R_fn^{-1} c_ftn / M (step 3; h may be NULL);
 *   Q [F][sum_l M_l^2] complex: per (f, l) the columns w_mu of W solve the generalized
 *     eigenproblem R_f,N-1^(l) w = lambda R_f,N^(l) w on the l-th diagonal blocks of
 *     the last two sources (step 5), with W^H R_f,N^(l) W = I, lambda ascending and
 *     each w's largest entry (the first on a tie) real positive; row mu of Q_fl is
 *     w_mu^H;
 *   g [F][N][M] real: g[f][n][o_l + mu] = w_mu^H R_fn^(l) w_mu (step 6, the diagonal
 *     of W^H R_fn^(l) W).
 * Q, g and h are written, caller-owned.  N >= 2 (step 5 needs two sources), else
 * DFM_E_SHAPE.  The workspace (>= dfm_initialise_workspace_size bytes, 256-byte
 * aligned) holds the R_fn.  Synchronises `stream`; returns DFM_E_SINGULAR if an
 * image covariance is not positive definite (that block's outputs are then
 * unspecified). */
dfm_status dfm_initialise_workspace_size(const dfm_problem* p, size_t* bytes);
dfm_status dfm_initialise(const dfm_problem* p, const void* C, void* Q, void* g, void* h,
                          void* workspace, size_t workspace_bytes, void* stream);

/* ---- Entry point that allocates nothing.
 * For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  One call does what
 * dfm_init, dfm_step(n_iter) and (if cost != NULL) the cost of dfm_nll do, with the
 * same kernels and the same results, but its workspace is a static device array
 * of DFM_NOALLOC_SCRATCH_BYTES owned by the library (one per GPU, held until the
 * process ends) instead of a caller's buffer, its launches are plain (no graphs),
 * and it calls no hipMalloc, hipFree or other allocating routine and makes no host
 * copy.  Asynchronous on `stream`.
 *   p, X, Q, g, W, H: as for dfm_init (Q, g, W, H updated in place).
 *   cost: device pointer to one double receiving the cost (13) after the last
 *     iteration, or NULL.
 *   status: device pointer to one int32 receiving the sticky device status bits
 *     after the run (1: singular IP system, 2: non-finite parameter with
 *     DFM_F_CHECK_FINITE), or NULL.
 * Returns DFM_E_WORKSPACE if the problem needs more than DFM_NOALLOC_SCRATCH_BYTES
 * (dfm_workspace_size), DFM_E_ARG for DFM_F_TRACE_NLL (its trace is read through a
 * plan), and the errors of dfm_init / dfm_step otherwise.  Every call on a GPU
 * uses that GPU's one array: calls that overlap on one GPU (on different streams,
 * or from different host threads) race and give wrong results; the array keeps
 * the last call's contents (each call clears what it reads before writing). */
#define DFM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
dfm_status dfm_run_noalloc(const dfm_problem* p, const void* X, void* Q, void* g, void* W, void* H,
                           int32_t n_iter, double* cost, int32_t* status, void* stream);

/* ---- Many mixtures at once.
 * A batch steps several independent plans (any shapes, precisions and tiles; one
 * device) together: dfm_batch_step captures, once per batch, the kernels of all
 * plans' iterations into HIP graphs in which each plan is its own branch (so the
 * mixtures' kernels may run concurrently and fill the chip), and replays them on
 * `stream`: the first iteration (with each plan's lambda seed), later iterations
 * singly and in groups of eight, and the plans' final g updates.  Each plan's
 * result is bit for bit what dfm_step(plan, n_iter) gives.  The batch borrows the
 * plans (they must outlive it, each in at most one batch at a time, and not be
 * stepped otherwise while the batch runs).  dfm_batch_create copies the plan
 * pointers; count in 1..4096. */
typedef struct dfm_batch dfm_batch;
dfm_status dfm_batch_create(dfm_batch** out, dfm_plan* const* plans, int32_t count);
dfm_status dfm_batch_step(dfm_batch* batch, int32_t n_iter, void* stream);
void dfm_batch_destroy(dfm_batch* batch);

/* Free the host-side plan.  Does not touch the caller's device buffers. */
void dfm_destroy(dfm_plan* plan);

/* Static English description of a status code. */
const char* dfm_status_string(dfm_status s);

#ifdef __cplusplus
}
#endif
#endif /* DFMNMF_H */
