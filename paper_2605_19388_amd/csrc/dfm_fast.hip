// Shape-specialised kernels of distributed FastMNMF for gfx950.
//
// Used when every subarray has the same size ML and (N, K, ML, L) is one of the compiled
// sets (DFM_FAST_SETS below).  All four are compile-time constants, so every per-frame
// array (lambda_n, y_m, |Qx|^2, x) lives in registers with a compile-time size and every
// loop over sources, bases and mics is unrolled.  Global loads that feed a computation
// are issued as one batch behind a scheduling barrier (left alone, the scheduler trades
// them for occupancy and waits on each load in turn).
//
// One iteration is seven kernels, each a plain launch on the caller's stream:
//
//   k_gramd_f  covariances V of eq. (14) for M_l <= 4 in FP32 (FP64 sums), a fixed grid
//              sharing the flattened (f, t) frames; k_gram_f (matrix cores) otherwise.
//   k_ip_f     FP64 IP sweep of eqs. (15)-(16), M_l lanes per (f, subarray) block (M_l <= 4;
//              larger blocks use the cooperative generic kernel).
//   k_pw_f     P = |Q x|^2 and the per-frame coefficient planes of eq. (8), one frame per thread.
//   k_wgemm_f  sums over frames of eq. (8) on the matrix cores, the W update and lambda = W H.
//   k_h_f      per-frame coefficient planes of eq. (9) with the new lambda.
//   k_hgemm_f  sums over bins of eq. (9) on the matrix cores, the H update and lambda = W H.
//   k_g_f      equal ranges of the F*T frames per workgroup: partial sums over frames of eq. (10);
//   k_gfin_f   the g update from each bin's partials.
//
// Every reduction finishes in a fixed order inside one kernel (wave sums added in wave
// order in LDS, partial-sum slots added in slot order), so results are identical run to
// run; no floating-point atomics.  Finishing a reduction split over workgroups with a
// last-arriving workgroup instead was measured slower on gfx950: the device-scope
// release/acquire it needs writes back and invalidates L2 in every workgroup.  k_lam_f
// forms lambda for the caller's W and H before a run; the cost (13) and the Wiener filter
// have their own kernels at the end of the file.
#include <hip/hip_runtime.h>

#include "dfm_device.h"

namespace dfm {
namespace fast {

constexpr int kT = 128;   // threads of the (f, time slice) kernels: one frame per thread
constexpr int kHTB = 16;  // frames per activation tile

__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// Element i of an array whose start is the same for the whole workgroup, through a 32-bit byte
// offset: the access then takes the scalar-base-plus-vector-offset form instead of 64-bit
// address arithmetic per lane.  Callers index within one bin's data (far below 4 GB).
template <typename T>
__device__ __forceinline__ T* at(T* base, uint32_t i) {
  typedef typename std::conditional<std::is_const<T>::value, const char, char>::type C;
  return reinterpret_cast<T*>(reinterpret_cast<C*>(base) + i * (uint32_t)sizeof(T));
}

// Reciprocal of a model variance (always >= eps > 0): the hardware estimate in FP32,
// the correctly rounded quotient in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

// 16-byte vectors for batched loads and stores.
template <typename R>
struct V16 {
  static constexpr int E = 16 / sizeof(R);
  typedef R type __attribute__((ext_vector_type(E)));
};

template <typename R, int C>
__device__ __forceinline__ void load16(R (&dst)[C], const R* src) {
  constexpr int E = V16<R>::E;
  static_assert(C % E == 0, "length must fill 16-byte vectors");
#pragma unroll
  for (int i = 0; i < C / E; ++i) {
    const typename V16<R>::type v = reinterpret_cast<const typename V16<R>::type*>(src)[i];
#pragma unroll
    for (int e = 0; e < E; ++e) dst[i * E + e] = v[e];
  }
}

// Plain 16-byte stores (not non-temporal: a wave's partial-line stores must merge in L2).
template <typename R, int C>
__device__ __forceinline__ void store16(R* dst, const R (&src)[C]) {
  constexpr int E = V16<R>::E;
  static_assert(C % E == 0, "length must fill 16-byte vectors");
#pragma unroll
  for (int i = 0; i < C / E; ++i) {
    typename V16<R>::type v;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = src[i * E + e];
    reinterpret_cast<typename V16<R>::type*>(dst)[i] = v;
  }
}

// ------------------------------------------------------------------------------------
// FP64 IP sweep (eqs. (15)-(16)) for subarrays of M_l <= 4 mics, M_l lanes per (f, l) block.
//
// (Q V_mu) b = e_mu is solved as V_mu b = c with c = Q^{-1} e_mu (the same system, since Q is
// nonsingular), so the M_l factorisations of V_mu (Hermitian positive definite: no
// pivoting) do not depend on the sweep and run on the block's lanes side by side; lane r
// factorises V_r and owns column r of Q^{-1}.  Row mu
// then takes one solve on lane mu, the normalisation s = b^H V b = d^H c (eq. (16)), and a
// rank-1 update of Q^{-1} on every lane: with row mu of Q replaced by b^H,
//   Q^{-1} <- Q^{-1} - c (b^H Q^{-1} - e_mu^T) / (b^H c),
// where b^H c = det(Q_new) / det(Q_old), so ln|det Q_fl| for the cost (13) is the log of
// the pivots of Q plus the sum of ln|b^H c| over the rows.  A zero pivot (V_mu or Q
// singular) keeps the row and sets the sticky singular flag.

// 1 / x and 1 / sqrt(x) in FP64 for the small solves: the hardware estimate refined by two
// Newton steps (each squares the relative error, so an estimate good to 2^-14 ends below
// 2^-53).  Shorter dependency chains than the IEEE division and square-root sequences, for
// finite nonzero x (zero pivots are caught before).
__device__ __forceinline__ double nr_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int i = 0; i < 2; ++i) r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double nr_rsqrt(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
#pragma unroll
  for (int i = 0; i < 2; ++i) r = fma(r, fma(-h * r, r, 0.5), r);
  return r;
}
__device__ __forceinline__ cd nr_cinv(cd a) {
  const double s = nr_rcp(cabs2(a));
  return {a.re * s, -a.im * s};
}

// LU factorisation without pivoting of a Hermitian positive (semi)definite n x n matrix in
// registers (L unit lower, U upper; inverse pivots of U in dinv).  Elimination without
// row exchanges is stable for such matrices; a zero pivot (a singular covariance, e.g. a
// silent mic) returns false.
template <int n>
__device__ __forceinline__ bool hpd_factor(cd (&A)[n][n], cd (&dinv)[n]) {
  bool ok = true;
#pragma unroll
  for (int p = 0; p < n; ++p) {
    const bool zero = cabs2(A[p][p]) == 0.0;
    if (zero) ok = false;
    dinv[p] = zero ? cd{0.0, 0.0} : nr_cinv(A[p][p]);
#pragma unroll
    for (int r = p + 1; r < n; ++r) {
      const cd fac = cmul(A[r][p], dinv[p]);
      A[r][p] = fac;
#pragma unroll
      for (int c = p + 1; c < n; ++c) A[r][c] = cfms(A[r][c], fac, A[p][c]);
    }
  }
  return ok;
}

// x <- A^{-1} x for the factors of hpd_factor.
template <int n>
__device__ __forceinline__ void hpd_solve(const cd (&A)[n][n], const cd (&dinv)[n], cd (&x)[n]) {
#pragma unroll
  for (int r = 1; r < n; ++r)
#pragma unroll
    for (int c = 0; c < r; ++c) x[r] = cfms(x[r], A[r][c], x[c]);
#pragma unroll
  for (int r = n - 1; r >= 0; --r) {
#pragma unroll
    for (int c = r + 1; c < n; ++c) x[r] = cfms(x[r], A[r][c], x[c]);
    x[r] = cmul(x[r], dinv[r]);
  }
}

// Column `col` of A^{-1} and ln|det A| by elimination of [A | e_col] with partial pivoting
// (rows exchanged over the active columns only).  Returns false on a zero pivot.
template <int n>
__device__ __forceinline__ bool inverse_column(cd (&A)[n][n + 1], int col, cd (&x)[n], double& logabs) {
  bool ok = true;
  double pivprod = 1.0;  // product of the |pivot|^2 (one log at the end)
  cd pinv[n];            // pivot inverses, reused by the back substitution
#pragma unroll
  for (int r = 0; r < n; ++r) A[r][n] = {r == col ? 1.0 : 0.0, 0.0};
#pragma unroll
  for (int p = 0; p < n; ++p) {
    int pr = p;
    double best = cabs2(A[p][p]);
#pragma unroll
    for (int r = p + 1; r < n; ++r) {
      const double v = cabs2(A[r][p]);
      if (v > best) {
        best = v;
        pr = r;
      }
    }
#pragma unroll
    for (int r = p + 1; r < n; ++r) {
      const bool sw = pr == r;
#pragma unroll
      for (int c = p; c <= n; ++c) {
        const cd tp = A[p][c], tr = A[r][c];
        A[p][c] = sw ? tr : tp;
        A[r][c] = sw ? tp : tr;
      }
    }
    if (best == 0.0) ok = false;
    pivprod *= best == 0.0 ? 1.0 : best;
    pinv[p] = best == 0.0 ? cd{0.0, 0.0} : nr_cinv(A[p][p]);
#pragma unroll
    for (int r = p + 1; r < n; ++r) {
      const cd fac = cmul(A[r][p], pinv[p]);
#pragma unroll
      for (int c = p + 1; c <= n; ++c) A[r][c] = cfms(A[r][c], fac, A[p][c]);
    }
  }
  logabs = 0.5 * log(pivprod);
#pragma unroll
  for (int r = n - 1; r >= 0; --r) {
    cd acc = A[r][n];
#pragma unroll
    for (int c = r + 1; c < n; ++c) acc = cfms(acc, A[r][c], x[c]);
    x[r] = cmul(acc, pinv[r]);
  }
  return ok;
}

template <typename R, int ML>
__global__ __launch_bounds__(64) void k_ip_f(Dims d, const double* __restrict__ Vpart, cx<R>* __restrict__ Q,
                                             double* __restrict__ logdet, int* __restrict__ status) {
  constexpr int ML2 = ML * ML, BPW = 64 / ML;  // blocks per wave
  static_assert(ML >= 1 && ML <= 4 && 64 % ML == 0, "lanes per block");
  __shared__ cd sB[BPW][ML], sC[BPW][ML], sW[BPW];
  __shared__ int sOk[BPW];
  const int lane = threadIdx.x, blk = lane / ML, r = lane - blk * ML;
  const int idx = blockIdx.x * BPW + blk;
  const bool live = idx < d.F * d.L;
  const int f = live ? idx / d.L : 0, l = live ? idx - f * d.L : 0;

  // Q_fl (every lane of the block) and this lane's row of it, loaded with the covariance
  // slots so that both arrive in one round trip.
  // Every load is 16 bytes wide: the block of Q and the slots are 16-byte aligned (and gfx950
  // keeps at most 63 loads in flight per wave, so narrower loads would take two round trips).
  cx<R>* qb = Q + (size_t)f * d.QF + l * ML2;
  R qv[2 * ML2], qr[2 * ML];  // interleaved (re, im)
  load16<R, 2 * ML2>(qv, reinterpret_cast<const R*>(qb));
  load16<R, 2 * ML>(qr, reinterpret_cast<const R*>(qb + r * ML));  // r is not a compile-time index
  // This lane's covariance slots (V_r packed, FP64), in flight while Q^{-1} is formed below.
  const double* vp = Vpart + (size_t)f * d.SG * d.VF + (size_t)l * ML * ML2 + r * ML2;
  const int ns = cov_slots(d, f);
  constexpr int SU = 3;  // slots loaded together (the covariance kernel's grid touches at most 3)
  double part[SU][ML2];
#pragma unroll
  for (int s = 0; s < SU; ++s) load16<double, ML2>(part[s], vp + (size_t)(s < ns ? s : 0) * d.VF);
  sched_fence();  // every load above in flight before the first use

  // Column r of Q_fl^{-1} and ln|det Q_fl| (every sweep from Q itself, so a run resumed from
  // the state is bitwise identical to an uninterrupted one).
  cd A[ML][ML + 1], row[ML], ci[ML];
#pragma unroll
  for (int a = 0; a < ML; ++a)
#pragma unroll
    for (int c = 0; c < ML; ++c) A[a][c] = {(double)qv[2 * (a * ML + c)], (double)qv[2 * (a * ML + c) + 1]};
#pragma unroll
  for (int c = 0; c < ML; ++c) row[c] = {(double)qr[2 * c], (double)qr[2 * c + 1]};
  double ld;
  const bool qok = inverse_column<ML>(A, r, ci, ld);
  // V_r = (sum over slices) / T, Hermitian from its packed entries.
  cd V[ML][ML];
  {
    double vs[ML2];
#pragma unroll
    for (int j = 0; j < ML2; ++j) vs[j] = 0.0;
#pragma unroll
    for (int s = 0; s < SU; ++s)
#pragma unroll
      for (int j = 0; j < ML2; ++j) vs[j] += s < ns ? part[s][j] : 0.0;
    for (int s = SU; s < ns; ++s)
#pragma unroll
      for (int j = 0; j < ML2; ++j) vs[j] += vp[(size_t)s * d.VF + j];
    // Packed order: the M_l diagonal entries, then (Re, Im) of V[a][b], a < b, row-major.
    const double invT = 1.0 / d.T;
#pragma unroll
    for (int a = 0; a < ML; ++a) {
      V[a][a] = {vs[a] * invT, 0.0};
#pragma unroll
      for (int b = a + 1; b < ML; ++b) {
        const int j = ML + 2 * (a * ML - a * (a + 1) / 2 + (b - a - 1));
        V[a][b] = {vs[j] * invT, vs[j + 1] * invT};
        V[b][a] = {vs[j] * invT, -vs[j + 1] * invT};
      }
    }
  }
  cd vdinv[ML];
  const bool vok = hpd_factor<ML>(V, vdinv);

  double wprod = 1.0;

#pragma unroll
  for (int mu = 0; mu < ML; ++mu) {
    if (r == mu) {
      const bool ok = vok && qok;
      cd dv[ML];
#pragma unroll
      for (int k = 0; k < ML; ++k) dv[k] = ci[k];
      hpd_solve<ML>(V, vdinv, dv);
      cd dc = {0.0, 0.0};  // d^H c = d^H V d
#pragma unroll
      for (int k = 0; k < ML; ++k) dc = cfmac(dc, dv[k], ci[k]);
      const double sc = nr_rsqrt(dc.re > d.eps ? dc.re : d.eps);
#pragma unroll
      for (int k = 0; k < ML; ++k) {
        const cd b = {dv[k].re * sc, dv[k].im * sc};
        sB[blk][k] = b;
        sC[blk][k] = ci[k];
        if (ok) row[k] = cconj(b);
      }
      sW[blk] = {dc.re * sc, dc.im * sc};  // b^H c
      sOk[blk] = ok;
      if (live && !ok) atomicOr(status, kStSingular);  // row kept; reported as DFM_E_SINGULAR
    }
    __syncthreads();
    if (sOk[blk]) {
      cd bq = {r == mu ? -1.0 : 0.0, 0.0};  // b^H Q^{-1}[:, r] - delta_{mu r}
#pragma unroll
      for (int k = 0; k < ML; ++k) bq = cfmac(bq, sB[blk][k], ci[k]);
      const cd w = sW[blk];
      const cd fac = cmul(bq, nr_cinv(w));
#pragma unroll
      for (int k = 0; k < ML; ++k) ci[k] = cfms(ci[k], sC[blk][k], fac);
      wprod *= cabs2(w);
    }
    __syncthreads();
  }
  ld += 0.5 * log(wprod);  // one log for the M_l factors |b^H c|^2 (each O(1) after eq. (16))
  if (!live) return;
#pragma unroll
  for (int c = 0; c < ML; ++c) qb[r * ML + c] = {(R)row[c].re, (R)row[c].im};

  if (r == 0) logdet[idx] = qok ? ld : -INFINITY;
}

// ------------------------------------------------------------------------------------
// Weighted covariances (eq. (14)) on the matrix cores.
//
// Per-frame operand rows live in LDS, frame-major, with row strides padded so that the
// 16-byte row writes of one frame per thread are free of bank conflicts: sInv[t][m] =
// 1 / y_ftm, and either the x tile (x_ft itself) or, for FP64 with M_l <= 4, the packed
// entries of every x^(l) x^(l)H formed once per frame.
// FP32 with M_l <= 4: one v_mfma_f32_4x4x1 (16 independent 4x4 blocks) per frame, block
// b = (subarray, group of 4 packed entries), rows = mu, each lane forming its packed entry
// from two staged x values; the frames of a slice are split over the two waves and their
// sums combined through LDS.  Staging x (2 M reals per frame) instead of the products
// (L M_l^2) keeps the LDS per workgroup small enough for five workgroups per CU.
// Otherwise: v_mfma 16x16x4 per subarray and 16 packed entries, K = 4 frames.

// Row stride (elements) >= n whose 16-byte row segments start in distinct bank groups.
template <typename R>
constexpr int padded(int n) {
  return sizeof(R) == 4 ? n + ((4 - n % 8) + 8) % 8 : n + ((2 - n % 4) + 4) % 4;
}

template <typename R, int N, int K, int ML, int L>
struct GramShape {
  static constexpr int M = ML * L, ML2 = ML * ML, OF = L * ML2;
  static constexpr bool kPre = ML <= 4;  // packed products staged per frame
  static constexpr int MP = padded<R>(M);
  static constexpr int OP = kPre ? padded<R>(OF) : padded<R>(2 * M);
};

template <typename R, typename RI, int N, int K, int ML, int L>
__global__ __launch_bounds__(kT) void k_gram_f(Dims d, const cx<RI>* __restrict__ X,
                                               const RI* __restrict__ lamin, const RI* __restrict__ g,
                                               R* __restrict__ Vpart) {
  typedef GramShape<R, N, K, ML, L> G;
  constexpr int M = G::M, ML2 = G::ML2, OF = G::OF, MP = G::MP, OP = G::OP;
  constexpr int JT = (ML2 + 15) / 16;
  constexpr int E = V16<R>::E;
  static_assert((2 * M) % E == 0 && M % E == 0 && OF % E == 0, "rows must fill 16-byte vectors");
  static_assert(N * M <= kT, "g of one frequency is staged one value per thread");
  typedef typename Mma<R>::v4 v4;
  typedef typename V16<R>::type vt;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int T = d.T;
  const int f = blockIdx.x / d.S, s = blockIdx.x - f * d.S;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, T - t0);
  const int ntp = (nt + 3) & ~3;
  extern __shared__ __align__(16) unsigned char smem[];
  R* sg = reinterpret_cast<R*>(smem);
  R* sInv = reinterpret_cast<R*>(smem + align_up(sizeof(R) * N * M, 16));  // [SLP][MP]
  R* sOp = sInv + (size_t)d.SLP * MP;                                       // [SLP][OP]

  // One batch of loads: x and lambda at this thread's frame, one value of g.
  R xv[2 * M], lam[N], gv = 0;
  if (tid < nt) {
    RI xin[2 * M];
    load16<RI, 2 * M>(xin, reinterpret_cast<const RI*>(X + ((size_t)f * T + t0 + tid) * M));
#pragma unroll
    for (int i = 0; i < 2 * M; ++i) xv[i] = (R)xin[i];
#pragma unroll
    for (int n = 0; n < N; ++n) lam[n] = (R)lamin[((size_t)f * N + n) * T + t0 + tid];
  } else {  // padding frames contribute zero products
#pragma unroll
    for (int i = 0; i < 2 * M; ++i) xv[i] = 0;
#pragma unroll
    for (int n = 0; n < N; ++n) lam[n] = 0;
  }
  if (tid < N * M) gv = (R)g[(size_t)f * N * M + tid];
  sched_fence();
  if (tid < N * M) sg[tid] = gv;
  __syncthreads();
  {
    const int tl = tid;  // one frame per thread (slices hold at most kT frames)
    if (tl < ntp) {
      R inv[M];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        R y = 0;
#pragma unroll
        for (int n = 0; n < N; ++n) y += lam[n] * sg[n * M + m];
        inv[m] = tl < nt ? rcp(rmax(y, (R)d.eps)) : (R)0;
      }
#pragma unroll
      for (int i = 0; i < M / E; ++i) {
        vt v;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = inv[i * E + e];
        reinterpret_cast<vt*>(sInv + (size_t)tl * MP)[i] = v;
      }
      if constexpr (G::kPre) {
        R op[OF];
#pragma unroll
        for (int l = 0; l < L; ++l)
#pragma unroll
          for (int a = 0; a < ML; ++a) {
            const R ar = xv[2 * (l * ML + a)], ai = xv[2 * (l * ML + a) + 1];
            op[l * ML2 + a] = ar * ar + ai * ai;
#pragma unroll
            for (int b = a + 1; b < ML; ++b) {
              const int jj = l * ML2 + ML + 2 * (a * ML - a * (a + 1) / 2 + (b - a - 1));
              const R br = xv[2 * (l * ML + b)], bi = xv[2 * (l * ML + b) + 1];
              op[jj] = ar * br + ai * bi;
              op[jj + 1] = ai * br - ar * bi;
            }
          }
#pragma unroll
        for (int i = 0; i < OF / E; ++i) {
          vt v;
#pragma unroll
          for (int e = 0; e < E; ++e) v[e] = op[i * E + e];
          reinterpret_cast<vt*>(sOp + (size_t)tl * OP)[i] = v;
        }
      } else {
#pragma unroll
        for (int i = 0; i < 2 * M / E; ++i) {
          vt v;
#pragma unroll
          for (int e = 0; e < E; ++e) v[e] = xv[i * E + e];
          reinterpret_cast<vt*>(sOp + (size_t)tl * OP)[i] = v;
        }
      }
    }
  }
  __syncthreads();

  // C[mu][j] += sum over 4 frames of (1/y)[frame][mu] * O[frame][j] per (subarray, 16
  // packed entries); four steps of operand loads ahead of their matrix-core ops.
  const int col = lane & 15, kk = lane >> 4;
  for (int item = wave; item < L * JT; item += kT / 64) {
    const int l = item / JT, jt = item - l * JT;
    const int o = l * ML;
    const int j = jt * 16 + col;
    const bool jv = j < ML2;
    const bool rv = col < ML;
    v4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    const int nsteps = ntp >> 2;
    int a = 0, b = 0, part = 0;
    if (jv) packed_pair(ML, j, a, b, part);
    const R* ip = sInv + (size_t)kk * MP + o + (rv ? col : 0);
    for (int q0 = 0; q0 < nsteps; q0 += 4) {
      R av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = min(q0 + u, nsteps - 1);
        const int tq = 4 * q + kk;
        const R ai = ip[(size_t)q * 4 * MP];
        R bo;
        if constexpr (G::kPre) {
          bo = sOp[(size_t)tq * OP + l * ML2 + (jv ? j : 0)];
        } else {
          const R* xr = sOp + (size_t)tq * OP;
          const R xar = xr[2 * (o + a)], xai = xr[2 * (o + a) + 1];
          const R xbr = xr[2 * (o + b)], xbi = xr[2 * (o + b) + 1];
          bo = part == 0 ? xar * xbr + xai * xbi : xai * xbr - xar * xbi;
        }
        const bool ok = q0 + u < nsteps;
        av[u] = (ok && rv) ? ai : (R)0;
        bv[u] = (ok && jv) ? bo : (R)0;
      }
#pragma unroll
      for (int u = 0; u < 4; u += 2) {
        acc0 = Mma<R>::run(av[u], bv[u], acc0);
        acc1 = Mma<R>::run(av[u + 1], bv[u + 1], acc1);
      }
    }
    R* out = Vpart + ((size_t)f * d.S + s) * d.VF + (size_t)l * ML * ML2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mu = Mma<R>::row(lane, r);
      if (mu < ML && jv) out[mu * ML2 + j] = acc0[r] + acc1[r];
    }
  }
}

// g <- g sqrt(num / max(den, eps)) of eq. (10) for one (f, n, m): num and den are the sums of
// the bin's `need` partials of k_g_f (stride 2 N M, den at offset N M), added in slot order with
// four slots' loads in flight at a time.  Every kernel that finishes the g update calls this, so
// they agree bit for bit.
template <typename R>
__device__ __forceinline__ R g_updated(const R* __restrict__ part, int need, int NM, R gv, R eps) {
  R nu = 0, de = 0;
  for (int s0 = 0; s0 < need; s0 += 4) {
    R pn[4], pd[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int sl = min(s0 + u, need - 1);
      pn[u] = part[(size_t)sl * 2 * NM];
      pd[u] = part[(size_t)sl * 2 * NM + NM];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (s0 + u < need) {
        nu += pn[u];
        de += pd[u];
      }
  }
  return gv * sqrt(nu / rmax(de, eps));
}

// Partial-sum slots of bin f in k_g_f's equal ranges of Dims::GGR frames.
__device__ __forceinline__ int g_slots(const Dims& d, int f) {
  return (f * d.T + d.T - 1) / d.GGR - (f * d.T) / d.GGR + 1;
}

// A pending g update split in two: g_preload asks for the first four partial-sum slots (and the
// copy of g) ahead of other loads, g_finish adds them, and any further slots, in the order of
// g_updated, so both give bitwise the same g.
template <typename R>
struct GPre {
  R pn[4], pd[4], gv;
};
template <typename R>
__device__ __forceinline__ void g_preload(GPre<R>& q, const R* __restrict__ part, int need, int NM, R gv) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int sl = min(u, need - 1);
    q.pn[u] = part[(size_t)sl * 2 * NM];
    q.pd[u] = part[(size_t)sl * 2 * NM + NM];
  }
  q.gv = gv;
}
template <typename R>
__device__ __forceinline__ R g_finish(const GPre<R>& q, const R* __restrict__ part, int need, int NM, R eps) {
  R nu = 0, de = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (u < need) {
      nu += q.pn[u];
      de += q.pd[u];
    }
  for (int s0 = 4; s0 < need; s0 += 4) {
    R pn[4], pd[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int sl = min(s0 + u, need - 1);
      pn[u] = part[(size_t)sl * 2 * NM];
      pd[u] = part[(size_t)sl * 2 * NM + NM];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (s0 + u < need) {
        nu += pn[u];
        de += pd[u];
      }
  }
  return q.gv * sqrt(nu / rmax(de, eps));
}

// ------------------------------------------------------------------------------------
// Weighted covariances (eq. (14)) for subarrays of M_l <= 4 mics, FP32 inputs, FP64 sums.
// A workgroup is one wave, and as many as fit on the chip at once share the frames equally:
// when there are at least two per bin, every bin gets the same number (Dims::GSB), each taking
// an equal part of its frames; otherwise they share the flattened (f, t) frames in equal ranges,
// which may cross bins (a range that does is summed as one segment per bin, each with its own
// start-up and reduction -- the reason for the bin-aligned parts).  kGDL lanes per subarray:
// lane j takes frames j, j + kGDL, ... of each segment.  Per frame it forms 1/y for the
// subarray's mics (FP32), the packed entries of x^(l) x^(l)H in FP64 (exact: products of
// FP32 values) and adds (1/y_mu) x x^H into M_l x M_l^2 FP64 registers; the lanes' sums are
// then added through LDS in a fixed order, one slot per (bin, workgroup).  (One-wave
// workgroups of 16 lanes per subarray and bin-aligned parts took the kernel from 16.0 to
// 13.7 us at 513 x 625 frames, against two-wave ones with flattened ranges.)  FP32 sums over
// frames would leave rounding errors outside the dominant directions of V, which the solve
// of eq. (15) amplifies by cond(V) -- large at the lowest bins, where the mixing is nearly
// rank-deficient; FP64 sums keep the solve's input at the precision of the FP64 reference.
// Output: V[f][slot][packed entries], FP64, /T not applied.
constexpr int kGDL = 16;  // lanes per subarray
constexpr int kGDH = 1;   // lanes per frame (each sums ML / kGDH of the rows mu)

template <int L>
constexpr int gramd_threads() {
  return (kGDH * L * kGDL + 63) / 64 * 64;
}

template <int N, int K, int ML, int L>
__global__ __launch_bounds__(gramd_threads<L>()) void k_gramd_f(Dims d, const cx<float>* __restrict__ X,
                                                               const float* __restrict__ lamin,
                                                               float* __restrict__ g,
                                                               const float* __restrict__ gpart,
                                                               const float* __restrict__ gsnap,
                                                               double* __restrict__ V) {
  constexpr int M = ML * L, ML2 = ML * ML, MH = ML / kGDH, NO = MH * ML2;  // outputs per lane
  constexpr int FB = 2;  // frames per load batch; the next batch is in flight during the current one
  constexpr int RH = NO < kGDL ? NO : kGDL, RS = RH + 2;  // outputs per reduction pass, LDS row stride
  static_assert(ML == 2 || ML == 4, "M_l of 2 or 4");
  static_assert(kGDH == 1 && NO % RH == 0 && RH % 2 == 0 && (RS / 2) % 2 == 1, "reduction passes");
  __shared__ __align__(16) double red[gramd_threads<L>() * RS];
  __shared__ float sg[N * M];  // the bin's g when a g update is pending
  const int tid = threadIdx.x;
  const int h = tid / (L * kGDL), l = min(tid / kGDL % L, L - 1), j = tid % kGDL;  // row half, subarray, lane
  const bool live = tid < kGDH * L * kGDL;
  const int T = d.T;
  // This workgroup's share of the flattened (f, t) frames: part p of bin fb, or an equal range
  // that may span several bins, each summed as one segment into slot (workgroup - first
  // workgroup of the bin).
  const long long total = (long long)d.F * T;
  long long a0 = (long long)blockIdx.x * d.GR, a1 = min(total, a0 + d.GR);
  if (d.GSB > 0) {  // part p of bin fb
    const int fb = blockIdx.x / d.GSB, p = blockIdx.x - fb * d.GSB;
    a0 = (long long)fb * T + (long long)p * T / d.GSB;
    a1 = (long long)fb * T + (long long)(p + 1) * T / d.GSB;
  }
  for (long long i0 = a0; i0 < a1;) {
    const int f = (int)(i0 / T);
    const long long fend = min(a1, (long long)(f + 1) * T);
    const int ts = (int)(i0 - (long long)f * T), te = (int)(fend - (long long)f * T);
    const int slot = d.GSB > 0 ? blockIdx.x - f * d.GSB : blockIdx.x - (int)(((long long)f * T) / d.GR);
    i0 = fend;

    const float* xb = reinterpret_cast<const float*>(X + (size_t)f * T * M + l * ML);
    const float* lb = lamin + (size_t)f * N * T;
    float xv[FB][2 * ML], lam[FB][N], xn[FB][2 * ML], ln[FB][N];
    auto fetch = [&](int t0, float (&x)[FB][2 * ML], float (&la)[FB][N]) {
#pragma unroll
      for (int u = 0; u < FB; ++u) {
        const int t = min(t0 + u * kGDL, te - 1);
        load16<float, 2 * ML>(x[u], xb + (size_t)t * 2 * M);
#pragma unroll
        for (int n = 0; n < N; ++n) la[u][n] = lb[(size_t)n * T + t];
      }
    };
    // g of the bin.  With an update pending (Dims::gpend), each workgroup finishes it from the
    // previous g update's partials and copy of g, neither of which this kernel writes; the
    // workgroup holding the bin's first frame stores the result.  The partials are asked for
    // first and the first frames next, so the finish waits for the partials only.
    constexpr int NM = N * M, GE = (NM + gramd_threads<L>() - 1) / gramd_threads<L>();
    GPre<float> gq[GE];
    const float* gp = gpart + (size_t)f * d.GGS * 2 * NM;
    const int gneed = g_slots(d, f);
    if (d.gpend)
#pragma unroll
      for (int e = 0; e < GE; ++e) {
        const int i = tid + e * gramd_threads<L>();
        if (i < NM) g_preload<float>(gq[e], gp + i, gneed, NM, gsnap[(size_t)f * NM + i]);
      }
    if (ts + j < te) fetch(ts + j, xv, lam);  // the first frames' loads fly during the g below
    const float* gsrc = g + (size_t)f * N * M;
    if (d.gpend) {
#pragma unroll
      for (int e = 0; e < GE; ++e) {
        const int i = tid + e * gramd_threads<L>();
        if (i >= NM) break;
        const float v = g_finish<float>(gq[e], gp + i, gneed, NM, (float)d.eps);
        sg[i] = v;
        if (ts == 0) g[(size_t)f * NM + i] = v;
      }
      __syncthreads();
      gsrc = sg;
    }
    float gl[N][MH];
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
      for (int mu = 0; mu < MH; ++mu) gl[n][mu] = gsrc[n * M + l * ML + min(h, kGDH - 1) * MH + mu];
    double acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = 0.0;

    for (int t0 = ts + j; t0 < te; t0 += FB * kGDL) {
      fetch(t0 + FB * kGDL, xn, ln);  // unconditional (clamped to the segment), so the waits count it
      sched_fence();
#pragma unroll
      for (int u = 0; u < FB; ++u) {
        if (t0 + u * kGDL >= te) break;
        double w[MH];
#pragma unroll
        for (int mu = 0; mu < MH; ++mu) {
          float y = 0.0f;
#pragma unroll
          for (int n = 0; n < N; ++n) y += lam[u][n] * gl[n][mu];
          w[mu] = (double)rcp(rmax(y, (float)d.eps));
        }
        double xd[2 * ML];
#pragma unroll
        for (int i = 0; i < 2 * ML; ++i) xd[i] = (double)xv[u][i];
        // Each packed entry goes into the M_l accumulators as soon as it is formed.
        auto add = [&](int e, double v) {
#pragma unroll
          for (int mu = 0; mu < MH; ++mu) acc[mu * ML2 + e] += w[mu] * v;
        };
#pragma unroll
        for (int a = 0; a < ML; ++a) {
          add(a, xd[2 * a] * xd[2 * a] + xd[2 * a + 1] * xd[2 * a + 1]);
#pragma unroll
          for (int b = a + 1; b < ML; ++b) {
            const int e = ML + 2 * (a * ML - a * (a + 1) / 2 + (b - a - 1));
            add(e, xd[2 * a] * xd[2 * b] + xd[2 * a + 1] * xd[2 * b + 1]);
            add(e + 1, xd[2 * a + 1] * xd[2 * b] - xd[2 * a] * xd[2 * b + 1]);
          }
        }
      }
      sched_fence();
#pragma unroll
      for (int u = 0; u < FB; ++u) {
#pragma unroll
        for (int i = 0; i < 2 * ML; ++i) xv[u][i] = xn[u][i];
#pragma unroll
        for (int n = 0; n < N; ++n) lam[u][n] = ln[u][n];
      }
    }

    // Totals over the subarray's lanes, RH outputs per pass: every lane writes its partial
    // sums as one padded LDS row, then lane j of the subarray adds column j over the
    // subarray's rows in lane order (a fixed order, so the sums are reproducible).
#pragma unroll
    for (int ps = 0; ps < NO / RH; ++ps) {
      __syncthreads();  // the previous pass's rows are consumed
#pragma unroll
      for (int i = 0; i < RH; i += 2)
        *reinterpret_cast<double2*>(red + tid * RS + i) = double2{acc[ps * RH + i], acc[ps * RH + i + 1]};
      __syncthreads();
      if (live && j < RH) {
        double sum = 0.0;
        for (int q = 0; q < kGDL; ++q) sum += red[(l * kGDL + q) * RS + j];
        V[((size_t)f * d.SG + slot) * d.VF + (size_t)l * NO + ps * RH + j] = sum;
      }
    }
  }
}

// ------------------------------------------------------------------------------------
// Weighted covariances (eq. (14)) with BF16 operands on the matrix cores and FP32 sums
// (DFM_F_GRAM_BF16), for subarrays of M_l = 2 or 4 mics.  The IP solves that follow stay FP64.
//
// V_flmu = (1/T) sum_t z_t z_t^H with z_t = x^(l)_ft / sqrt(y_{f,t,o_l+mu}): each z is rounded to
// BF16 once and used on both sides, so the computed V is the exact Gram matrix of the rounded
// vectors -- Hermitian positive semidefinite like eq. (14) itself.  (Rounding w x_a and x_b
// separately breaks that: at the lowest bins, where the mixing is nearly rank-1, V then has
// negative eigenvalues and the IP normaliser of eq. (16) loses its meaning.)  As a real matrix
// product with the frames and their (re, im) parts along the contraction,
//   Re V[a][b] = sum_t (Re z_a, Im z_a) . (Re z_b, Im z_b),  Im V[a][b] = sum_t (Im z_a, -Re z_a) . (Re z_b, Im z_b).
// One v_mfma_f32_16x16x32_bf16 contracts 16 frames for a 16 x 16 tile whose rows and columns
// are (subarray, mu, mic) triples of 16 / M_l^2 subarrays; the (l, mu) diagonal blocks are the
// wanted V_flmu.  Lane l supplies row l % 16 of the left operand and column l % 16 of the right
// one for the four frames of lane group l / 16 -- the same z values for both -- and holds column
// l % 16, rows 4 (l / 16) .. + 3 of the sum.  The flattened (f, t) frames are shared out as for
// k_gramd_f (ranges of Dims::GR per workgroup, one partial-sum slot per bin segment) and the
// slots are written in FP64 in its packed layout, so k_ip_f reads either kernel's output.
constexpr int kGBW = 4;  // waves per workgroup of k_gramb_f

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int ML, int L>
struct GramB {
  static constexpr int ML2 = ML * ML;
  static constexpr int SPT = 16 / ML2;                 // subarrays per 16 x 16 tile
  static constexpr int NT = (L + SPT - 1) / SPT;       // tiles
  static_assert(ML == 2 || ML == 4, "M_l of 2 or 4");
};

// Per chunk of 16 frames each wave stages the frames' x (16 M complex, contiguous in X) with
// 16-byte loads and their weights 1 / sqrt(y) (lane (t, mic group) forms y from lambda and g) in
// its own LDS area, then every lane gathers the x and weights of its rows from there.
template <int N, int K, int ML, int L>
__global__ __launch_bounds__(64 * kGBW) void k_gramb_f(Dims d, const cx<float>* __restrict__ X,
                                                      const float* __restrict__ lamin, float* __restrict__ g,
                                                      const float* __restrict__ gpart,
                                                      const float* __restrict__ gsnap, double* __restrict__ V) {
  typedef GramB<ML, L> G;
  constexpr int M = ML * L, ML2 = ML * ML, SPT = G::SPT, NT = G::NT, NM = N * M;
  constexpr int XS = 2 * M + 4;          // LDS row of one frame's x (reals), padded
  constexpr int XV = 2 * M / 4;          // 16-byte vectors of one frame's x
  constexpr int MG = 64 / 16;            // mic groups of the weight stage (lane = (frame, group))
  constexpr int MPG = (M + MG - 1) / MG; // mics per group
  static_assert(NM <= 64 * kGBW, "one thread per g entry");
  static_assert((2 * M) % 4 == 0 && 16 * XV <= 64 * 4, "x staging");
  __shared__ float red[kGBW][L][ML2][ML][2];   // [wave][l][mu * ML + a][b][re, im]
  __shared__ __align__(16) float sx[kGBW][16][XS];  // per wave: the chunk's x, frame-major
  __shared__ float sw[kGBW][16][M + 1];        // per wave: 1 / sqrt(y) of the chunk
  __shared__ float sg[NM];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, kg = lane >> 4;                    // row / column of the tile, lane group
  const int rl = r / ML2, rmu = (r % ML2) / ML, ra = r % ML;  // (subarray in the tile, mu, mic)
  const int wt = lane & 15, wg = lane >> 4;                   // weight stage: frame, mic group
  const int T = d.T;
  const long long total = (long long)d.F * T;
  long long a0 = (long long)blockIdx.x * d.GR, a1 = min(total, a0 + d.GR);
  if (d.GSB > 0) {  // part p of bin fb
    const int fb = blockIdx.x / d.GSB, p = blockIdx.x - fb * d.GSB;
    a0 = (long long)fb * T + (long long)p * T / d.GSB;
    a1 = (long long)fb * T + (long long)(p + 1) * T / d.GSB;
  }
  for (long long i0 = a0; i0 < a1;) {
    const int f = (int)(i0 / T);
    const long long fend = min(a1, (long long)(f + 1) * T);
    const int ts = (int)(i0 - (long long)f * T), te = (int)(fend - (long long)f * T);
    const int slot = d.GSB > 0 ? blockIdx.x - f * d.GSB : blockIdx.x - (int)(((long long)f * T) / d.GR);
    i0 = fend;
    // g of the bin, finishing a pending g update exactly as k_gramd_f does.
    const float* gsrc = g + (size_t)f * NM;
    if (d.gpend) {
      if (tid < NM) {
        const float v = g_updated<float>(gpart + (size_t)f * d.GGS * 2 * NM + tid, g_slots(d, f), NM,
                                         gsnap[(size_t)f * NM + tid], (float)d.eps);
        sg[tid] = v;
        if (ts == 0) g[(size_t)f * NM + tid] = v;
      }
      __syncthreads();
      gsrc = sg;
    }
    float gm[MPG][N];  // g of this lane's weight-stage mics
#pragma unroll
    for (int k = 0; k < MPG; ++k)
#pragma unroll
      for (int n = 0; n < N; ++n) gm[k][n] = wg * MPG + k < M ? gsrc[n * M + wg * MPG + k] : 1.0f;
    const float* xf = reinterpret_cast<const float*>(X + (size_t)f * T * M);
    const float* lb = lamin + (size_t)f * N * T;
    f32x4 cre[NT], cim[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      cre[q] = f32x4{0, 0, 0, 0};
      cim[q] = f32x4{0, 0, 0, 0};
    }
    // Global loads of one chunk: lane v < 16 XV takes 16-byte vector v of the chunk's x (frames
    // past the segment are not read), and lambda at its weight-stage frame (clamped).
    typedef float f4 __attribute__((ext_vector_type(4)));
    auto fetch = [&](int c0, f4 (&xv)[(16 * XV + 63) / 64], float (&la)[N]) {
#pragma unroll
      for (int u = 0; u < (16 * XV + 63) / 64; ++u) {
        const int v = lane + 64 * u, fr = v / XV;
        const bool ok = v < 16 * XV && c0 + fr < te;
        xv[u] = ok ? *reinterpret_cast<const f4*>(xf + (size_t)c0 * 2 * M + 4 * v) : f4{0, 0, 0, 0};
      }
      const int t = min(c0 + wt, te - 1);
#pragma unroll
      for (int n = 0; n < N; ++n) la[n] = lb[(size_t)n * T + t];
    };
    constexpr int XU = (16 * XV + 63) / 64;
    f4 xv[XU], xn[XU];
    float la[N], ln[N];
    int c0 = ts + wave * 16;
    fetch(c0, xv, la);
    for (; c0 < te; c0 += 16 * kGBW) {
      fetch(c0 + 16 * kGBW, xn, ln);  // the next chunk in flight during this one
      // Stage: x rows, and the weights of frame wt at this lane's mic group.
#pragma unroll
      for (int u = 0; u < XU; ++u) {
        const int v = lane + 64 * u;
        if (v < 16 * XV) *reinterpret_cast<f4*>(&sx[wave][v / XV][4 * (v % XV)]) = xv[u];
      }
      const bool tlive = c0 + wt < te;
#pragma unroll
      for (int k = 0; k < MPG; ++k) {
        float y = 0.0f;
#pragma unroll
        for (int n = 0; n < N; ++n) y += la[n] * gm[k][n];
        if (wg * MPG + k < M) sw[wave][wt][wg * MPG + k] = tlive ? __builtin_amdgcn_rsqf(rmax(y, (float)d.eps)) : 0.0f;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int l = min(q * SPT + rl, L - 1);
        const bool rowv = q * SPT + rl < L;
        bf16x8 az, ai;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int fr = 4 * kg + j;
          const float s = rowv ? sw[wave][fr][l * ML + rmu] : 0.0f;
          const float2 x = *reinterpret_cast<const float2*>(&sx[wave][fr][2 * (l * ML + ra)]);
          const __bf16 zr = (__bf16)(s * x.x), zi = (__bf16)(s * x.y);
          az[2 * j] = zr;
          az[2 * j + 1] = zi;
          ai[2 * j] = zi;
          ai[2 * j + 1] = -zr;
        }
        cre[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(az, az, cre[q], 0, 0, 0);
        cim[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, az, cim[q], 0, 0, 0);
      }
      // The staging area is rewritten by the next chunk: every lane's gathers come first.
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int u = 0; u < XU; ++u) xv[u] = xn[u];
#pragma unroll
      for (int n = 0; n < N; ++n) la[n] = ln[n];
    }
    // Lane (column r, group kg) holds rows 4 kg + e of each tile; the (l, mu) diagonal blocks are
    // V_lmu.  Every (l, mu, a, b) sits in exactly one lane of each wave.
    __syncthreads();  // the previous segment's readers of red are done
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = 4 * kg + e;
        const int l = q * SPT + row / ML2, mu = (row % ML2) / ML, a = row % ML;
        if (l < L && row / ML2 == rl && mu == rmu) {
          red[wave][l][mu * ML + a][ra][0] = cre[q][e];
          red[wave][l][mu * ML + a][ra][1] = cim[q][e];
        }
      }
    __syncthreads();
    for (int o = tid; o < L * ML * ML2; o += 64 * kGBW) {
      const int l = o / (ML * ML2), rem = o - l * ML * ML2, mu = rem / ML2, jj = rem - mu * ML2;
      int a, b, part;
      packed_pair(ML, jj, a, b, part);
      float sum = 0.0f;
      for (int w = 0; w < kGBW; ++w) sum += red[w][l][mu * ML + a][b][part];
      V[((size_t)f * d.SG + slot) * d.VF + o] = (double)sum;
    }
  }
}

// lambda[f][n][t] = sum_k W[n][f][k] H[n][k][t] (eq. (2)) on the matrix cores: one 16 x 16
// tile (rows f, columns t) per wave, contraction over the bases four at a time.
// Hn: the activations of source n for the tile's 16 frames, [4 * ceil(K/4)][16] in LDS,
// zero beyond K and T.
template <typename R, int N, int K>
__device__ __forceinline__ void lambda_tile(const Dims& d, const R* __restrict__ W, const R* Hn, int n, int f0,
                                            int t0, int lane, R* __restrict__ lam) {
  constexpr int KS = (K + 3) / 4;
  typedef typename Mma<R>::v4 v4;
  const int i = lane & 15, kk = lane >> 4;
  const int fr = f0 + i;
  R av[KS], bv[KS];
#pragma unroll
  for (int st = 0; st < KS; ++st) {
    const int k = 4 * st + kk;
    av[st] = (fr < d.F && k < K) ? W[((size_t)n * d.F + fr) * K + k] : (R)0;
    bv[st] = Hn[(4 * st + kk) * 16 + i];
  }
  v4 acc = {0, 0, 0, 0};
#pragma unroll
  for (int st = 0; st < KS; ++st) acc = Mma<R>::run(av[st], bv[st], acc);
  const int t = t0 + i;
  if (t < d.T)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = f0 + Mma<R>::row(lane, r);
      if (f < d.F) lam[((size_t)f * N + n) * d.T + t] = acc[r];
    }
}

constexpr int kLamWaves = 8;  // waves of the activation-apply workgroup

// lambda for the caller's W and H (before the first iteration); grid (N, tiles of 16 frames).
template <typename R, int N, int K>
__global__ __launch_bounds__(64 * kLamWaves) void k_lam_f(Dims d, const R* __restrict__ W, const R* __restrict__ H,
                                                          R* __restrict__ lam) {
  constexpr int KS = (K + 3) / 4;
  __shared__ R sHn[4 * KS * 16];
  const int n = blockIdx.x, t0 = blockIdx.y * 16, tid = threadIdx.x;
  const int tl = tid & 15, t = t0 + tl;
  for (int k = tid >> 4; k < 4 * KS; k += 4 * kLamWaves)
    sHn[k * 16 + tl] = (k < K && t < d.T) ? H[((size_t)n * K + k) * d.T + t] : (R)0;
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  for (int f0 = wave * 16; f0 < d.F; f0 += 16 * kLamWaves) lambda_tile<R, N, K>(d, W, sHn, n, f0, t0, lane, lam);
}


// Coefficient planes AB[p][tt][f][16]: value p (a_n for p = n, b_n for p = N + n) of bin f
// and frame t = 16 tt + (t % 16).  The sums over frames and over bins read them as 16 x 16
// tiles, each a contiguous 1 KB block.
__device__ __forceinline__ size_t ab_index(const Dims& d, int p, int f, int t) {
  return (((size_t)p * d.TBN + (t >> 4)) * d.F + f) * 16 + (t & 15);
}

// ------------------------------------------------------------------------------------
// P = |Q x|^2 and the per-bin coefficients of eq. (8) for every (f, t) of two slices:
// a_n = sum_m g_nm P_m / y_m^2 and b_n = sum_m g_nm / y_m, written to the coefficient
// planes (values n and N + n) for the sums over frames in k_wgemm_f.  Each thread takes
// one frame of each slice (grid (F, ceil(S / 2))); the loads of both frames are issued up
// front, so the second frame's data arrives while the first is processed (a thread per
// frame would run every wave's loads and then every wave's arithmetic in lockstep).
template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(kT) void k_pw_f(Dims d, const cx<R>* __restrict__ X, const cx<R>* __restrict__ Q,
                                             const R* __restrict__ lamin, const R* __restrict__ g,
                                             R* __restrict__ P, R* __restrict__ AB) {
  constexpr int M = ML * L, ML2 = ML * ML, QF = L * ML2;
  constexpr int QPT = (QF + kT - 1) / kT, GPT = (N * M + kT - 1) / kT;
  static_assert((2 * M) % V16<R>::E == 0 && M % V16<R>::E == 0, "rows must fill 16-byte vectors");
  const int f = blockIdx.x, tid = threadIdx.x;
  const int T = d.T;
  constexpr int E = V16<R>::E, PS = M + E;  // sP row stride: 16-byte rows in distinct bank groups
  __shared__ cx<R> sQ[QF];
  __shared__ R sg[N * M];
  __shared__ __align__(16) R sP[kT * PS];  // P of the workgroup's frames, staged for contiguous stores

  // Q and g of the bin first (the LDS writes wait for them only), then both frames.
  cx<R> qv[QPT];
  R gv[GPT];
#pragma unroll
  for (int j = 0; j < QPT; ++j) {
    const int i = tid + j * kT;
    if (i < QF) qv[j] = Q[(size_t)f * QF + i];
  }
#pragma unroll
  for (int j = 0; j < GPT; ++j) {
    const int i = tid + j * kT;
    if (i < N * M) gv[j] = g[(size_t)f * N * M + i];
  }
  const R* xf = reinterpret_cast<const R*>(X + (size_t)f * T * M);  // the bin's frames
  const R* lf[N];
#pragma unroll
  for (int n = 0; n < N; ++n) lf[n] = lamin + ((size_t)f * N + n) * T;
  R xv[2][2 * M], lam[2][N];
  int tf[2];
  bool live[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int s = 2 * blockIdx.y + u, t0 = s * d.SL;
    live[u] = s < d.S && tid < min(d.SL, T - t0);
    tf[u] = live[u] ? t0 + tid : T - 1;  // dead lanes load a valid frame and store nothing
    load16<R, 2 * M>(xv[u], at(xf, (uint32_t)tf[u] * (2 * M)));
#pragma unroll
    for (int n = 0; n < N; ++n) lam[u][n] = *at(lf[n], (uint32_t)tf[u]);
  }
  sched_fence();
#pragma unroll
  for (int j = 0; j < QPT; ++j) {
    const int i = tid + j * kT;
    if (i < QF) sQ[i] = qv[j];
  }
#pragma unroll
  for (int j = 0; j < GPT; ++j) {
    const int i = tid + j * kT;
    if (i < N * M) sg[i] = gv[j];
  }
  __syncthreads();

  typedef typename V16<R>::type vt;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int s = 2 * blockIdx.y + u, t0 = s * d.SL, nt = s < d.S ? min(d.SL, T - t0) : 0;
    if (nt <= 0) break;
    if (live[u]) {  // (a branch per frame also keeps the two frames' arithmetic apart)
    R a[N], b[N], pv[M];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      a[n] = 0;
      b[n] = 0;
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
#pragma unroll
      for (int mu = 0; mu < ML; ++mu) {
        R zr = 0, zi = 0;
#pragma unroll
        for (int c = 0; c < ML; ++c) {  // two fused multiply-adds per part
          const cx<R> q = sQ[l * ML2 + mu * ML + c];
          const R xr = xv[u][2 * (l * ML + c)], xi = xv[u][2 * (l * ML + c) + 1];
          zr = fma(q.re, xr, zr);
          zr = fma(-q.im, xi, zr);
          zi = fma(q.re, xi, zi);
          zi = fma(q.im, xr, zi);
        }
        const int m = l * ML + mu;
        const R p = zr * zr + zi * zi;
        pv[m] = p;
        R y = 0;
#pragma unroll
        for (int n = 0; n < N; ++n) y += lam[u][n] * sg[n * M + m];
        const R iy = rcp(rmax(y, (R)d.eps));
        const R piy2 = p * iy * iy;
#pragma unroll
        for (int n = 0; n < N; ++n) {
          a[n] += sg[n * M + m] * piy2;
          b[n] += sg[n * M + m] * iy;
        }
      }
    }
    const int t = tf[u];
    {
      const uint32_t o = (uint32_t)ab_index(d, 0, 0, t);  // the frame's place in a bin row
#pragma unroll
      for (int n = 0; n < N; ++n) {
        *at(AB + ab_index(d, n, f, 0), o) = a[n];
        *at(AB + ab_index(d, N + n, f, 0), o) = b[n];
      }
#pragma unroll
      for (int i = 0; i < M / E; ++i) {
        vt v;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = pv[i * E + e];
        *reinterpret_cast<vt*>(sP + tid * PS + i * E) = v;
      }
    }
    }
    // P rows of the slice's frames are contiguous in memory: store them through LDS so that
    // each wave writes whole 1 KB runs (per-frame 16-byte stores would reach L2 as separate
    // partial-line writes).
    __syncthreads();
    R* pout = P + ((size_t)f * T + t0) * M;
    for (int c = tid; c < nt * (M / E); c += kT) {
      const int fr = c / (M / E), part = c - fr * (M / E);
      *reinterpret_cast<vt*>(at(pout, (uint32_t)c * E)) = *reinterpret_cast<const vt*>(sP + fr * PS + part * E);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------
// Sums over frames or frequencies of the coefficient planes on the 16x16x4 matrix cores,
// with the multiplicative update applied in the same kernel.  A workgroup has kGW waves and
// owns one source and 16 bins (W update) or 16 frames (H update); the contraction range is
// dealt out to the waves in chunks of 16 (four 4-deep steps).
//
// Plane layout AB[p][tt][f][16] (p = n for a_n, N + n for b_n): every 16 bins x 16 frames
// tile is a contiguous 1 KB block, so a wave reads one tile with one 16-byte-per-lane load
// (W update), and a 16-frame column of all bins is one contiguous run (H update).  The
// operand that all chunks share (H[n] for the W update, W[n] for the H update) is staged in
// LDS once per workgroup with contiguous loads (in windows when it does not fit) and read
// from there both by the sums and by the lambda tiles after the update.  The waves'
// accumulators are summed in LDS in wave order.
constexpr int kGW = 8;  // waves per workgroup
constexpr int kGB = 6;  // chunks per wave and load batch

// LDS of the two GEMM kernels: a fixed part (wave sums, the 16 updated rows) and a window of
// the shared operand that fits in the rest of 64 KB.
template <typename R, int K>
struct GemmLds {
  static constexpr int KT = (K + 15) / 16, KP = 4 * ((K + 3) / 4);
  static constexpr size_t fixed = sizeof(R) * (kGW * 2 * KT * 256 + 16 * KP);
  static constexpr size_t budget = 64 * 1024 - fixed - 256;
  // W update: H window of TW frames, rows k < KP, row stride TW + 4.
  static constexpr int TWMAX = ((int)(budget / (sizeof(R) * KP)) - 4) / 16 * 16;
  static constexpr int HRW = (KP + kGW - 1) / kGW, HRC = (TWMAX + 63) / 64;  // per-lane staging
  // H update: W window of FW bins, row stride WS.
  static constexpr int WS = KP + 4;
  static constexpr int FWMAX = (int)(budget / (sizeof(R) * WS)) / 16 * 16;
  static constexpr int WNE = (FWMAX * KP + 64 * kGW - 1) / (64 * kGW);  // per-thread staging
  __host__ __device__ static int tw(const Dims& d) { return d.TP < TWMAX ? d.TP : TWMAX; }
  __host__ __device__ static int fw(const Dims& d) {
    const int fp = (d.F + 15) & ~15;
    return fp < FWMAX ? fp : FWMAX;
  }
  static size_t wgemm_smem(const Dims& d) { return sizeof(R) * KP * (size_t)(tw(d) + 4); }
  static size_t hgemm_smem(const Dims& d) { return sizeof(R) * WS * (size_t)fw(d); }
};

// Wave sums -> LDS as red[wave][which][tile][row][col], rows/cols of the 16 x 16 tiles.
template <typename R, int NT>
__device__ __forceinline__ void spill_tiles(R* red, int wave, int lane, const typename Mma<R>::v4 (&accN)[NT],
                                            const typename Mma<R>::v4 (&accD)[NT]) {
#pragma unroll
  for (int kt = 0; kt < NT; ++kt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = Mma<R>::row(lane, r), col = lane & 15;
      red[(((wave * 2 + 0) * NT + kt) * 16 + row) * 16 + col] = accN[kt][r];
      red[(((wave * 2 + 1) * NT + kt) * 16 + row) * 16 + col] = accD[kt][r];
    }
}

template <typename R, int NT>
__device__ __forceinline__ void sum_tiles(const R* red, int kt, int row, int col, R& num, R& den) {
  num = 0;
  den = 0;
#pragma unroll
  for (int w = 0; w < kGW; ++w) {
    num += red[(((w * 2 + 0) * NT + kt) * 16 + row) * 16 + col];
    den += red[(((w * 2 + 1) * NT + kt) * 16 + row) * 16 + col];
  }
}

// Bases update, eq. (8), for one source n and 16 bins: num/den[f][k] = sum_t (a, b)[f][t] H[k][t]
// (rows f, columns k, contraction over frames), W <- W sqrt(num / max(den, eps)); then
// lambda = W H for the new W at these bins and every frame (the H sums read it).
// LDS window: sH[k][t - w0] = H[n][k][t] for w0 <= t < w0 + TW, row stride TW + 4 (16-byte
// rows in distinct bank groups), zero beyond T and K.
template <typename R, int N, int K>
__global__ __launch_bounds__(64 * kGW) void k_wgemm_f(Dims d, const R* __restrict__ AB, const R* __restrict__ H,
                                                      R* __restrict__ W, R* __restrict__ lam,
                                                      int* __restrict__ status) {
  typedef GemmLds<R, K> G;
  constexpr int KT = G::KT, KP = G::KP, KS = KP / 4;
  static_assert(KT <= 2, "bases per source");
  typedef typename Mma<R>::v4 v4;
  typedef R v4r __attribute__((ext_vector_type(4)));
  __shared__ R red[kGW * 2 * KT * 256];
  __shared__ R sWn[16 * KP];  // new W of the 16 bins, [f][k], zero beyond K and F
  extern __shared__ __align__(16) unsigned char dyn[];
  R* sH = reinterpret_cast<R*>(dyn);
  const int n = blockIdx.x, f0 = blockIdx.y * 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 15, kk = lane >> 4;
  const int T = d.T, F = d.F, TP = d.TP;
  const int TW = G::tw(d), TS = TW + 4;
  const int fr = min(f0 + i, F - 1);  // rows beyond F are computed on a valid row and dropped
  const R* an = AB + ((size_t)n * d.TBN * F + fr) * 16 + 4 * kk;
  const R* bn = AB + ((size_t)(N + n) * d.TBN * F + fr) * 16 + 4 * kk;
  const R* hn = H + (size_t)n * K * T;
  const size_t tstride = (size_t)F * 16;  // one 16-frame tile further
  // The entry of W this thread updates (at most one), asked for now so that the update does not
  // wait for it.
  static_assert(16 * KP <= 64 * kGW, "one updated entry per thread");
  R wold = 0;
  {
    const int fi = tid / KP, k = tid - fi * KP, f = f0 + fi;
    if (tid < 16 * KP && k < K && f < F) wold = W[((size_t)n * F + f) * K + k];
  }

  // Window [w0, w0 + nw) of H[n] -> sH: wave w stages rows w, w + kGW, ...; every load is
  // issued before the first LDS write.
  auto stage = [&](int w0, int nw) {
    R v[G::HRW][G::HRC];
#pragma unroll
    for (int q = 0; q < G::HRW; ++q)
#pragma unroll
      for (int r = 0; r < G::HRC; ++r) {
        const int k = wave + q * kGW, tl = lane + 64 * r, t = w0 + tl;
        v[q][r] = (k < K && tl < nw && t < T) ? hn[(size_t)k * T + t] : (R)0;
      }
#pragma unroll
    for (int q = 0; q < G::HRW; ++q)
#pragma unroll
      for (int r = 0; r < G::HRC; ++r) {
        const int k = wave + q * kGW, tl = lane + 64 * r;
        if (k < KP && tl < nw) sH[k * TS + tl] = v[q][r];
      }
  };

  v4 accN[KT], accD[KT];
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) {
    accN[kt] = v4{0, 0, 0, 0};
    accD[kt] = v4{0, 0, 0, 0};
  }
  for (int w0 = 0; w0 < TP; w0 += TW) {
    const int nw = min(TW, TP - w0), cb = w0 / 16, ce = cb + nw / 16;
    if (w0 > 0) __syncthreads();  // the previous window is consumed
    v4r av[kGB], bv[kGB];
    auto load = [&](int c0) {
#pragma unroll
      for (int u = 0; u < kGB; ++u) {
        const int cc = min(c0 + u * kGW, ce - 1);
        av[u] = *reinterpret_cast<const v4r*>(an + cc * tstride);
        bv[u] = *reinterpret_cast<const v4r*>(bn + cc * tstride);
      }
    };
    load(cb + wave);  // first batch in flight while the window is staged
    stage(w0, nw);
    __syncthreads();
    for (int c0 = cb + wave; c0 < ce; c0 += kGW * kGB) {
      if (c0 != cb + wave) {
        load(c0);
        sched_fence();
      }
#pragma unroll
      for (int u = 0; u < kGB; ++u) {
        const int c = c0 + u * kGW;
        const int tl = (min(c, ce - 1) - cb) * 16 + 4 * kk;  // this lane's frames w0 + tl .. + 3
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          const int k = kt * 16 + i;
          const v4r h4 = *reinterpret_cast<const v4r*>(sH + (k < KP ? k : 0) * TS + tl);
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            const bool ok = c < ce && w0 + tl + st < T;
            const R a = ok ? av[u][st] : (R)0, b = ok ? bv[u][st] : (R)0;
            const R h = k < K ? h4[st] : (R)0;
            accN[kt] = Mma<R>::run(a, h, accN[kt]);
            accD[kt] = Mma<R>::run(b, h, accD[kt]);
          }
        }
      }
    }
  }
  spill_tiles<R, KT>(red, wave, lane, accN, accD);
  __syncthreads();
  if (tid < 16 * KP) {
    const int e = tid, fi = e / KP, k = e - fi * KP, f = f0 + fi;
    R w = 0;
    if (k < K && f < F) {
      R num, den;
      sum_tiles<R, KT>(red, k >> 4, fi, k & 15, num, den);
      const size_t idx = ((size_t)n * F + f) * K + k;
      w = wold * sqrt(num / rmax(den, (R)d.eps));
      if (d.check && !isfinite(w)) atomicOr(status, kStNonFinite);
      W[idx] = w;
    }
    sWn[e] = w;
  }
  __syncthreads();

  // lambda[f][n][t] for the 16 bins: rows f (A = new W from LDS), columns t (B = H from the
  // window), over k.  With one window, H is still staged.
  R wa[KS];
#pragma unroll
  for (int st = 0; st < KS; ++st) wa[st] = sWn[i * KP + 4 * st + kk];
  for (int w0 = 0; w0 < TP; w0 += TW) {
    const int nw = min(TW, TP - w0), cb = w0 / 16, ce = cb + nw / 16;
    if (TW < TP) {
      __syncthreads();
      stage(w0, nw);
      __syncthreads();
    }
    for (int c = cb + wave; c < ce; c += kGW) {
      v4 acc = {0, 0, 0, 0};
#pragma unroll
      for (int st = 0; st < KS; ++st) acc = Mma<R>::run(wa[st], sH[(4 * st + kk) * TS + (c - cb) * 16 + i], acc);
      const int t = c * 16 + i;
      if (t < T)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int f = f0 + Mma<R>::row(lane, r);
          if (f < F) lam[((size_t)f * N + n) * T + t] = acc[r];
        }
    }
  }
}

// Per-bin coefficients of eq. (9) with lambda for the new W: a'_n = sum_m g_nm P_m / y_m^2,
// b'_n = sum_m g_nm / y_m, written to the coefficient planes for the sums over frequencies
// in k_hgemm_f.  Two frames per thread, as in k_pw_f.
template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(kT) void k_h_f(Dims d, const R* __restrict__ lamin, const R* __restrict__ g,
                                            const R* __restrict__ P, R* __restrict__ AB) {
  constexpr int M = ML * L, GPT = (N * M + kT - 1) / kT;
  static_assert(M % V16<R>::E == 0, "rows must fill 16-byte vectors");
  const int f = blockIdx.x, tid = threadIdx.x;
  const int T = d.T;
  __shared__ R sg[N * M];
  R gv[GPT];
#pragma unroll
  for (int j = 0; j < GPT; ++j) {
    const int i = tid + j * kT;
    if (i < N * M) gv[j] = g[(size_t)f * N * M + i];
  }
  const R* pf = P + (size_t)f * T * M;  // the bin's frames
  const R* lf[N];
#pragma unroll
  for (int n = 0; n < N; ++n) lf[n] = lamin + ((size_t)f * N + n) * T;
  R pv[2][M], lam[2][N];
  int tf[2];
  bool live[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int s = 2 * blockIdx.y + u, t0 = s * d.SL;
    live[u] = s < d.S && tid < min(d.SL, T - t0);
    tf[u] = live[u] ? t0 + tid : T - 1;
    load16<R, M>(pv[u], at(pf, (uint32_t)tf[u] * M));
#pragma unroll
    for (int n = 0; n < N; ++n) lam[u][n] = *at(lf[n], (uint32_t)tf[u]);
  }
  sched_fence();
#pragma unroll
  for (int j = 0; j < GPT; ++j) {
    const int i = tid + j * kT;
    if (i < N * M) sg[i] = gv[j];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    if (!live[u]) continue;
    R a[N], b[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      a[n] = 0;
      b[n] = 0;
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      R y = 0;
#pragma unroll
      for (int n = 0; n < N; ++n) y += lam[u][n] * sg[n * M + m];
      const R iy = rcp(rmax(y, (R)d.eps));
      const R piy2 = pv[u][m] * iy * iy;
#pragma unroll
      for (int n = 0; n < N; ++n) {
        a[n] += sg[n * M + m] * piy2;
        b[n] += sg[n * M + m] * iy;
      }
    }
    const uint32_t o = (uint32_t)ab_index(d, 0, 0, tf[u]);  // the frame's place in a bin row
#pragma unroll
    for (int n = 0; n < N; ++n) {
      *at(AB + ab_index(d, n, f, 0), o) = a[n];
      *at(AB + ab_index(d, N + n, f, 0), o) = b[n];
    }
  }
}

// Activation update, eq. (9), for one source n and 16 frames: num/den[k][t] = sum_f W[f][k]
// (a', b')[f][t] (rows k, columns t, contraction over bins), H <- H sqrt(num / max(den, eps));
// then lambda = W H for the new H at these frames and every bin (the g sums and the next
// iteration read it).  Step st of chunk c takes bins c * 16 + 4 st + kk, so each 4-byte
// plane load of a wave is one contiguous 256-byte run.  LDS window: sW[f - f0][k] =
// W[n][f][k] for f0 <= f < f0 + FW, row stride KP + 4, zero beyond F and K.
// Window [f0, f0 + nf) of W[n] -> sW, flat over (bin, basis) with row stride GemmLds::WS; every
// load is issued before the first LDS write.
template <typename R, int K>
__device__ __forceinline__ void stage_w(R* sW, const R* wn, int F, int f0, int nf, int tid) {
  typedef GemmLds<R, K> G;
  constexpr int KP = G::KP, WS = G::WS;
  R v[G::WNE];
#pragma unroll
  for (int q = 0; q < G::WNE; ++q) {
    const int e = tid + q * 64 * kGW, fl = e / KP, k = e - fl * KP, f = f0 + fl;
    v[q] = (fl < nf && f < F && k < K) ? wn[(size_t)f * K + k] : (R)0;
  }
#pragma unroll
  for (int q = 0; q < G::WNE; ++q) {
    const int e = tid + q * 64 * kGW, fl = e / KP, k = e - fl * KP;
    if (fl < nf) sW[fl * WS + k] = v[q];
  }
}

template <typename R, int N, int K>
__global__ __launch_bounds__(64 * kGW) void k_hgemm_f(Dims d, const R* __restrict__ W, const R* __restrict__ AB,
                                                      R* __restrict__ H, R* __restrict__ lam,
                                                      int* __restrict__ status) {
  typedef GemmLds<R, K> G;
  constexpr int KT = G::KT, KP = G::KP, KS = KP / 4, WS = G::WS;
  static_assert(KT <= 2, "bases per source");
  typedef typename Mma<R>::v4 v4;
  __shared__ R red[kGW * 2 * KT * 256];
  __shared__ R sHn[KP * 16];  // new H of the 16 frames, [k][t], zero beyond K and T
  extern __shared__ __align__(16) unsigned char dyn[];
  R* sW = reinterpret_cast<R*>(dyn);
  const int n = blockIdx.x, tt = blockIdx.y, t0 = tt * 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 15, kk = lane >> 4;
  const int T = d.T, F = d.F;
  const int FP = (F + 15) & ~15, FW = G::fw(d);
  const R* ap = AB + ((size_t)n * d.TBN + tt) * F * 16 + i;
  const R* bp = AB + ((size_t)(N + n) * d.TBN + tt) * F * 16 + i;
  const R* wn = W + (size_t)n * F * K;
  const bool tok = t0 + i < T;
  // The entry of H this thread updates (at most one), asked for now so that the update does not
  // wait for it.
  static_assert(KP * 16 <= 64 * kGW, "one updated entry per thread");
  R hold = 0;
  if (tid < KP * 16 && (tid >> 4) < K && t0 + (tid & 15) < T) hold = H[((size_t)n * K + (tid >> 4)) * T + t0 + (tid & 15)];

  auto stage = [&](int f0, int nf) { stage_w<R, K>(sW, wn, F, f0, nf, tid); };

  v4 accN[KT], accD[KT];
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) {
    accN[kt] = v4{0, 0, 0, 0};
    accD[kt] = v4{0, 0, 0, 0};
  }
  for (int f0 = 0; f0 < FP; f0 += FW) {
    const int nf = min(FW, FP - f0), cb = f0 / 16, ce = cb + nf / 16;
    if (f0 > 0) __syncthreads();  // the previous window is consumed
    R av[kGB][4], bv[kGB][4];
    auto load = [&](int c0) {
#pragma unroll
      for (int u = 0; u < kGB; ++u) {
        const int cc = min(c0 + u * kGW, ce - 1);
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int f = min(cc * 16 + 4 * st + kk, F - 1);
          av[u][st] = ap[(size_t)f * 16];
          bv[u][st] = bp[(size_t)f * 16];
        }
      }
    };
    load(cb + wave);  // first batch in flight while the window is staged
    stage(f0, nf);
    __syncthreads();
    for (int c0 = cb + wave; c0 < ce; c0 += kGW * kGB) {
      if (c0 != cb + wave) {
        load(c0);
        sched_fence();
      }
#pragma unroll
      for (int u = 0; u < kGB; ++u) {
        const int c = c0 + u * kGW;
        const int fl = (min(c, ce - 1) - cb) * 16;
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int f = c * 16 + 4 * st + kk;
          const bool ok = c < ce && f < F && tok;
          const R a = ok ? av[u][st] : (R)0, b = ok ? bv[u][st] : (R)0;
#pragma unroll
          for (int kt = 0; kt < KT; ++kt) {
            const int k = kt * 16 + i;
            const R w = k < K ? sW[(fl + 4 * st + kk) * WS + (k < K ? k : 0)] : (R)0;
            accN[kt] = Mma<R>::run(w, a, accN[kt]);
            accD[kt] = Mma<R>::run(w, b, accD[kt]);
          }
        }
      }
    }
  }
  spill_tiles<R, KT>(red, wave, lane, accN, accD);
  __syncthreads();
  if (tid < KP * 16) {
    const int e = tid, k = e >> 4, tl = e & 15, t = t0 + tl;
    R h = 0;
    if (k < K && t < T) {
      R num, den;
      sum_tiles<R, KT>(red, k >> 4, k & 15, tl, num, den);
      const size_t idx = ((size_t)n * K + k) * T + t;
      h = hold * sqrt(num / rmax(den, (R)d.eps));
      if (d.check && !isfinite(h)) atomicOr(status, kStNonFinite);
      H[idx] = h;
    }
    sHn[e] = h;
  }
  __syncthreads();

  // lambda[f][n][t] for the 16 frames: rows f (A = W from the window), columns t (B = new H
  // from LDS), over k.  With one window, W is still staged.
  R hb[KS];
#pragma unroll
  for (int st = 0; st < KS; ++st) hb[st] = sHn[(4 * st + kk) * 16 + i];
  for (int f0 = 0; f0 < FP; f0 += FW) {
    const int nf = min(FW, FP - f0), cb = f0 / 16, ce = cb + nf / 16;
    if (FW < FP) {
      __syncthreads();
      stage(f0, nf);
      __syncthreads();
    }
    for (int c = cb + wave; c < ce; c += kGW) {
      v4 acc = {0, 0, 0, 0};
#pragma unroll
      for (int st = 0; st < KS; ++st) acc = Mma<R>::run(sW[((c - cb) * 16 + i) * WS + 4 * st + kk], hb[st], acc);
      const int t = t0 + i;
      if (t < T)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int f = c * 16 + Mma<R>::row(lane, r);
          if (f < F) lam[((size_t)f * N + n) * T + t] = acc[r];
        }
    }
  }
}

// H update split along the bins, for shapes where W[n] takes more than one LDS window (F above
// about 600 bins in FP32 with K = 16): window c of k_hgemm_f goes to workgroup (n, tt, c) of
// k_hsum_f, which writes its partial sums and (c = 0) a copy of the H it updates; k_hlam_f adds
// a 16-frame block's partials in window order, applies the update (every workgroup the same way,
// the c = 0 workgroup storing H) and writes lambda = W H for its window of bins.  The copy is
// what k_hlam_f multiplies, so no workgroup reads H while another writes it.
template <typename R, int N, int K>
__global__ __launch_bounds__(64 * kGW) void k_hsum_f(Dims d, const R* __restrict__ W, const R* __restrict__ AB,
                                                     const R* __restrict__ H, R* __restrict__ Hpart,
                                                     R* __restrict__ Hsnap) {
  typedef GemmLds<R, K> G;
  constexpr int KT = G::KT, KP = G::KP, WS = G::WS;
  static_assert(KT <= 2, "bases per source");
  typedef typename Mma<R>::v4 v4;
  __shared__ R red[kGW * 2 * KT * 256];
  extern __shared__ __align__(16) unsigned char dyn[];
  R* sW = reinterpret_cast<R*>(dyn);
  const int n = blockIdx.x, tt = blockIdx.y, t0 = tt * 16, c = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 15, kk = lane >> 4;
  const int T = d.T, F = d.F;
  const int FP = (F + 15) & ~15, FW = G::fw(d);
  const int f0 = c * FW, nf = min(FW, FP - f0), cb = f0 / 16, ce = cb + nf / 16;
  const R* ap = AB + ((size_t)n * d.TBN + tt) * F * 16 + i;
  const R* bp = AB + ((size_t)(N + n) * d.TBN + tt) * F * 16 + i;
  const R* wn = W + (size_t)n * F * K;
  const bool tok = t0 + i < T;

  v4 accN[KT], accD[KT];
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) {
    accN[kt] = v4{0, 0, 0, 0};
    accD[kt] = v4{0, 0, 0, 0};
  }
  R av[kGB][4], bv[kGB][4];
  auto load = [&](int c0) {
#pragma unroll
    for (int u = 0; u < kGB; ++u) {
      const int cc = min(c0 + u * kGW, ce - 1);
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int f = min(cc * 16 + 4 * st + kk, F - 1);
        av[u][st] = ap[(size_t)f * 16];
        bv[u][st] = bp[(size_t)f * 16];
      }
    }
  };
  load(cb + wave);  // first batch in flight while the window is staged
  stage_w<R, K>(sW, wn, F, f0, nf, tid);
  __syncthreads();
  for (int c0 = cb + wave; c0 < ce; c0 += kGW * kGB) {
    if (c0 != cb + wave) {
      load(c0);
      sched_fence();
    }
#pragma unroll
    for (int u = 0; u < kGB; ++u) {
      const int cc = c0 + u * kGW;
      const int fl = (min(cc, ce - 1) - cb) * 16;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int f = cc * 16 + 4 * st + kk;
        const bool ok = cc < ce && f < F && tok;
        const R a = ok ? av[u][st] : (R)0, b = ok ? bv[u][st] : (R)0;
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          const int k = kt * 16 + i;
          const R w = k < K ? sW[(fl + 4 * st + kk) * WS + (k < K ? k : 0)] : (R)0;
          accN[kt] = Mma<R>::run(w, a, accN[kt]);
          accD[kt] = Mma<R>::run(w, b, accD[kt]);
        }
      }
    }
  }
  spill_tiles<R, KT>(red, wave, lane, accN, accD);
  __syncthreads();
  R* part = Hpart + (((size_t)n * d.TBN + tt) * d.HC + c) * 2 * KP * 16;
  for (int e = tid; e < KP * 16; e += 64 * kGW) {
    const int k = e >> 4, tl = e & 15, t = t0 + tl;
    R num, den;
    sum_tiles<R, KT>(red, k >> 4, k & 15, tl, num, den);
    part[e] = num;
    part[KP * 16 + e] = den;
    if (c == 0 && k < K && t < T) Hsnap[((size_t)n * K + k) * T + t] = H[((size_t)n * K + k) * T + t];
  }
}

template <typename R, int N, int K>
__global__ __launch_bounds__(64 * kGW) void k_hlam_f(Dims d, const R* __restrict__ Hpart, const R* __restrict__ Hsnap,
                                                     const R* __restrict__ W, R* __restrict__ H, R* __restrict__ lam,
                                                     int* __restrict__ status) {
  typedef GemmLds<R, K> G;
  constexpr int KP = G::KP, KS = KP / 4, WS = G::WS;
  typedef typename Mma<R>::v4 v4;
  __shared__ R sHn[KP * 16];  // new H of the 16 frames, [k][t], zero beyond K and T
  extern __shared__ __align__(16) unsigned char dyn[];
  R* sW = reinterpret_cast<R*>(dyn);
  const int n = blockIdx.x, tt = blockIdx.y, t0 = tt * 16, c = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 15, kk = lane >> 4;
  const int T = d.T, F = d.F;
  const int FP = (F + 15) & ~15, FW = G::fw(d);
  const int f0 = c * FW, nf = min(FW, FP - f0), cb = f0 / 16, ce = cb + nf / 16;
  stage_w<R, K>(sW, W + (size_t)n * F * K, F, f0, nf, tid);  // loads fly during the update
  const R* part = Hpart + ((size_t)n * d.TBN + tt) * d.HC * 2 * KP * 16;
  for (int e = tid; e < KP * 16; e += 64 * kGW) {
    const int k = e >> 4, tl = e & 15, t = t0 + tl;
    R h = 0;
    if (k < K && t < T) {
      R num = 0, den = 0;
      for (int cc = 0; cc < d.HC; ++cc) {
        num += part[(size_t)cc * 2 * KP * 16 + e];
        den += part[(size_t)cc * 2 * KP * 16 + KP * 16 + e];
      }
      const size_t idx = ((size_t)n * K + k) * T + t;
      h = Hsnap[idx] * sqrt(num / rmax(den, (R)d.eps));
      if (c == 0) {
        if (d.check && !isfinite(h)) atomicOr(status, kStNonFinite);
        H[idx] = h;
      }
    }
    sHn[e] = h;
  }
  __syncthreads();
  R hb[KS];
#pragma unroll
  for (int st = 0; st < KS; ++st) hb[st] = sHn[(4 * st + kk) * 16 + i];
  for (int cc = cb + wave; cc < ce; cc += kGW) {
    v4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int st = 0; st < KS; ++st) acc = Mma<R>::run(sW[((cc - cb) * 16 + i) * WS + 4 * st + kk], hb[st], acc);
    const int t = t0 + i;
    if (t < T)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = cc * 16 + Mma<R>::row(lane, r);
        if (f < F) lam[((size_t)f * N + n) * T + t] = acc[r];
      }
  }
}

// ------------------------------------------------------------------------------------
// Diagonal SCM update, eq. (10): num/den[n][m] = sum_t lambda_n (P_m / y_m^2, 1 / y_m) over
// every frame, then g <- g sqrt(num / max(den, eps)).  The F*T frames are dealt out in equal
// contiguous ranges of Dims::GGR to Dims::GGW workgroups (a range may run into the next bins).
// A lane owns one mic of one frame per step (64 / M frames per wave) and keeps the 2N sums of
// its mic in registers; the source asks for the next batch's P and lambda before the current
// batch's arithmetic (the compiler keeps the P loads a batch ahead and moves the lambda loads to
// their batch).  A workgroup adds its lanes' sums in a fixed order through LDS into one partial
// per bin it touched (slot = its rank among the bin's workgroups).  The g update itself (each
// bin's partials added in slot order) is finished by k_gfin_f or, inside a run of iterations,
// by the next iteration's k_gramd_f, which applies it to the copy of g kept here.  (Finishing a
// bin in the last workgroup to reach it would need a device-scope fence per workgroup, which on
// this chip writes back and invalidates the L2 of the workgroup's XCD; that made the kernel ten
// times slower.)
constexpr int kGT = 256;  // threads of a g-update workgroup
constexpr int kGU = 2;    // steps per batch of loads

template <typename R, int N, int M>
struct GShape {
  static constexpr int FPW = 64 / M;              // frames per wave and step
  static constexpr int FS = (kGT / 64) * FPW;     // frames per workgroup and step
  static constexpr int RED = (kGT / 64) * 2 * N * 64;  // LDS: the lanes' sums
};

template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(kGT) void k_g_f(Dims d, const R* __restrict__ lamin, const R* __restrict__ g,
                                             const R* __restrict__ P, R* __restrict__ gpart, R* __restrict__ gsnap) {
  constexpr int M = ML * L;
  typedef GShape<R, N, M> G;
  constexpr int FPW = G::FPW, FS = G::FS, NM = N * M;
  static_assert(FPW >= 1, "shape");
  __shared__ R red[G::RED];  // [wave][2N][64]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = lane / M, m = lane - j * M;  // frame within the wave's step, mic
  const bool lane_ok = j < FPW;
  const int me = wave * FPW + j;  // frame offset within a workgroup step
  const int T = d.T;
  const R eps = (R)d.eps;
  const int a = blockIdx.x * d.GGR, b = min(a + d.GGR, d.F * T);
  for (int s0 = a; s0 < b;) {
    const int f = s0 / T, e = min(b, (f + 1) * T);
    const int t0 = s0 - f * T, t1 = e - f * T;
    s0 = e;
    // The workgroup holding the bin's first frame keeps a copy of the g this update multiplies.
    if (t0 == 0 && tid < NM) gsnap[(size_t)f * NM + tid] = g[(size_t)f * NM + tid];
    R gm[N], num[N], den[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      gm[n] = g[((size_t)f * N + n) * M + m];
      num[n] = 0;
      den[n] = 0;
    }
    const R* Pf = P + (size_t)f * T * M;  // the bin's frames
    const R* Lf[N];
#pragma unroll
    for (int n = 0; n < N; ++n) Lf[n] = lamin + ((size_t)f * N + n) * T;
    // Loads of one batch (kGU steps); frames past the range read the range's last frame.
    auto fetch = [&](int tb, R(&pv)[kGU], R(&lv)[kGU][N]) {
#pragma unroll
      for (int u = 0; u < kGU; ++u) {
        const uint32_t t = (uint32_t)min(tb + u * FS + me, t1 - 1);
        pv[u] = *at(Pf, t * M + m);
#pragma unroll
        for (int n = 0; n < N; ++n) lv[u][n] = *at(Lf[n], t);
      }
    };
    R pa[kGU], la[kGU][N], pb[kGU], lb[kGU][N];
    fetch(t0, pa, la);
    for (int tb = t0; tb < t1; tb += kGU * FS) {
      fetch(tb + kGU * FS, pb, lb);
#pragma unroll
      for (int u = 0; u < kGU; ++u) {
        const bool live = lane_ok && tb + u * FS + me < t1;
        R y = 0;
#pragma unroll
        for (int n = 0; n < N; ++n) y += la[u][n] * gm[n];
        const R iy = live ? rcp(rmax(y, eps)) : (R)0;
        const R w = pa[u] * iy * iy;
#pragma unroll
        for (int n = 0; n < N; ++n) {
          num[n] += la[u][n] * w;
          den[n] += la[u][n] * iy;
        }
      }
#pragma unroll
      for (int u = 0; u < kGU; ++u) {
        pa[u] = pb[u];
#pragma unroll
        for (int n = 0; n < N; ++n) la[u][n] = lb[u][n];
      }
    }
    // Lane sums -> this workgroup's partial for bin f (index q * M + m, q < N: numerators).
    __syncthreads();  // the previous segment's readers of red are done
#pragma unroll
    for (int n = 0; n < N; ++n) {
      red[(wave * 2 * N + n) * 64 + lane] = num[n];
      red[(wave * 2 * N + N + n) * 64 + lane] = den[n];
    }
    __syncthreads();
    const int first = (f * T) / d.GGR;
    for (int o = tid; o < 2 * NM; o += kGT) {
      const int q = o / M, mm = o - q * M;
      R v = 0;
#pragma unroll
      for (int w = 0; w < kGT / 64; ++w)
#pragma unroll
        for (int jj = 0; jj < FPW; ++jj) v += red[(w * 2 * N + q) * 64 + jj * M + mm];
      gpart[((size_t)f * d.GGS + blockIdx.x - first) * 2 * NM + o] = v;
    }
  }
}

// g <- g sqrt(num / max(den, eps)) of eq. (10), one thread per (f, n, m): the bin's partials of
// k_g_f added in slot order.
template <typename R, int N, int M>
__global__ __launch_bounds__(256) void k_gfin_f(Dims d, const R* __restrict__ gpart, R* __restrict__ g,
                                               int* __restrict__ status) {
  constexpr int NM = N * M;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= d.F * NM) return;
  const int f = i / NM, o = i - f * NM;
  const R v = g_updated<R>(gpart + (size_t)f * d.GGS * 2 * NM + o, g_slots(d, f), NM, g[i], (R)d.eps);
  if (d.check && !isfinite(v)) atomicOr(status, kStNonFinite);
  g[i] = v;
}

// ------------------------------------------------------------------------------------
// Cost (13) and the per-subarray Wiener filter for the specialised sets (M_l <= 4).

// Q_fl^{-1} (FP64, for the Wiener filter) and ln|det Q_fl| (for the cost) with M_l lanes per
// (f, l) block: lane r eliminates [Q_fl | e_r] (partial pivoting) for column r.
template <typename R, int ML>
__global__ __launch_bounds__(64) void k_qinv_f(Dims d, const cx<R>* __restrict__ Q, cd* __restrict__ Qinv,
                                               double* __restrict__ logdet, int* __restrict__ status) {
  constexpr int ML2 = ML * ML, BPW = 64 / ML;
  const int lane = threadIdx.x, blk = lane / ML, r = lane - blk * ML;
  const int idx = blockIdx.x * BPW + blk;
  if (idx >= d.F * d.L) return;
  const int f = idx / d.L, l = idx - f * d.L;
  const cx<R>* qb = Q + (size_t)f * d.QF + l * ML2;
  cd A[ML][ML + 1], x[ML];
#pragma unroll
  for (int a = 0; a < ML; ++a)
#pragma unroll
    for (int c = 0; c < ML; ++c) A[a][c] = {(double)qb[a * ML + c].re, (double)qb[a * ML + c].im};
  double ld;
  const bool ok = inverse_column<ML>(A, r, x, ld);
  cd* out = Qinv + (size_t)f * d.QF + l * ML2;
#pragma unroll
  for (int a = 0; a < ML; ++a) out[a * ML + r] = x[a];
  if (r == 0) logdet[idx] = ok ? ld : -INFINITY;
  if (!ok && r == 0) atomicOr(status, kStSingular);
}

// Data part of the cost (13) per (f, slice): sum over frames and mics of |Q x|^2 / y + ln y,
// one frame per thread; each term in the working precision (its rounding error, relative
// 1e-7 in FP32, averages out over the F T M terms), the sums in FP64.
template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(kT) void k_nll_f(Dims d, const cx<R>* __restrict__ X, const cx<R>* __restrict__ Q,
                                              const R* __restrict__ lamin, const R* __restrict__ g,
                                              double* __restrict__ nllpart) {
  constexpr int M = ML * L, ML2 = ML * ML, QF = L * ML2;
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int T = d.T, t0 = s * d.SL, nt = min(d.SL, T - t0);
  __shared__ cx<R> sQ[QF];
  __shared__ R sg[N * M];
  __shared__ double red[kT / 64];
  R xv[2 * M], lam[N];
  const bool live = tid < nt;
  if (live) {
    load16<R, 2 * M>(xv, reinterpret_cast<const R*>(X + ((size_t)f * T + t0 + tid) * M));
#pragma unroll
    for (int n = 0; n < N; ++n) lam[n] = lamin[((size_t)f * N + n) * T + t0 + tid];
  }
  for (int i = tid; i < QF; i += kT) sQ[i] = Q[(size_t)f * QF + i];
  for (int i = tid; i < N * M; i += kT) sg[i] = g[(size_t)f * N * M + i];
  sched_fence();
  __syncthreads();
  double acc = 0.0;
  if (live) {
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int mu = 0; mu < ML; ++mu) {
        R zr = 0, zi = 0;
#pragma unroll
        for (int c = 0; c < ML; ++c) {
          const cx<R> q = sQ[l * ML2 + mu * ML + c];
          const R xr = xv[2 * (l * ML + c)], xi = xv[2 * (l * ML + c) + 1];
          zr += q.re * xr - q.im * xi;
          zi += q.re * xi + q.im * xr;
        }
        R y = 0;
#pragma unroll
        for (int n = 0; n < N; ++n) y += lam[n] * sg[n * M + l * ML + mu];
        y = rmax(y, (R)d.eps);
        acc += (double)((zr * zr + zi * zi) / y) + (double)log(y);
      }
  }
  // Workgroup sum in a fixed order: wave sums by shuffles, then the waves in order.
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 64);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kT / 64; ++w) sum += red[w];
    nllpart[(size_t)f * d.S + s] = sum;
  }
}

// Source images at every subarray, S_n = Q^{-1} diag(lambda_n g_n / y) Q x, one frame per thread.
template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(kT) void k_sep_f(Dims d, const cx<R>* __restrict__ X, const cx<R>* __restrict__ Q,
                                              const cd* __restrict__ Qinv, const R* __restrict__ lamin,
                                              const R* __restrict__ g, cx<R>* __restrict__ S) {
  constexpr int M = ML * L, ML2 = ML * ML, QF = L * ML2;
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int T = d.T, t0 = s * d.SL, nt = min(d.SL, T - t0);
  __shared__ cx<R> sQ[QF], sQi[QF];
  __shared__ R sg[N * M];
  __shared__ __align__(16) unsigned char sOraw[sizeof(R) * kT * (2 * M + V16<R>::E)];  // output rows
  R xv[2 * M], lam[N];
  const bool live = tid < nt;
  if (live) {
    load16<R, 2 * M>(xv, reinterpret_cast<const R*>(X + ((size_t)f * T + t0 + tid) * M));
#pragma unroll
    for (int n = 0; n < N; ++n) lam[n] = lamin[((size_t)f * N + n) * T + t0 + tid];
  }
  for (int i = tid; i < QF; i += kT) {
    sQ[i] = Q[(size_t)f * QF + i];
    const cd qi = Qinv[(size_t)f * QF + i];
    sQi[i] = {(R)qi.re, (R)qi.im};
  }
  for (int i = tid; i < N * M; i += kT) sg[i] = g[(size_t)f * N * M + i];
  sched_fence();
  __syncthreads();
  // Q x and 1/y of this frame, every mic.
  R zr[M], zi[M], iy[M];
  if (live) {
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int mu = 0; mu < ML; ++mu) {
        R ar = 0, ai = 0;
#pragma unroll
        for (int c = 0; c < ML; ++c) {
          const cx<R> q = sQ[l * ML2 + mu * ML + c];
          const R xr = xv[2 * (l * ML + c)], xi = xv[2 * (l * ML + c) + 1];
          ar += q.re * xr - q.im * xi;
          ai += q.re * xi + q.im * xr;
        }
        const int m = l * ML + mu;
        zr[m] = ar;
        zi[m] = ai;
        R y = 0;
#pragma unroll
        for (int n = 0; n < N; ++n) y += lam[n] * sg[n * M + m];
        iy[m] = (R)1 / rmax(y, (R)d.eps);
      }
  }
  // Per source: the frame's row of M complex outputs goes to LDS, then the workgroup stores
  // its frames' rows, contiguous in S, as whole 16-byte-per-lane runs (per-frame stores at the
  // row stride would reach L2 as one partial-line request per lane).
  typedef typename V16<R>::type vt;
  constexpr int E = V16<R>::E, RW = 2 * M, OS = RW + E;  // row length and padded LDS stride (reals)
  R* sO = reinterpret_cast<R*>(sOraw);
#pragma unroll
  for (int n = 0; n < N; ++n) {
    if (live) {
#pragma unroll
      for (int l = 0; l < L; ++l) {
        R out[2 * ML];
#pragma unroll
        for (int a = 0; a < ML; ++a) {
          R vr = 0, vi = 0;
#pragma unroll
          for (int mu = 0; mu < ML; ++mu) {
            const int m = l * ML + mu;
            const R gain = lam[n] * sg[n * M + m] * iy[m];
            const cx<R> q = sQi[l * ML2 + a * ML + mu];
            const R ur = gain * zr[m], ui = gain * zi[m];
            vr += q.re * ur - q.im * ui;
            vi += q.re * ui + q.im * ur;
          }
          out[2 * a] = vr;
          out[2 * a + 1] = vi;
        }
#pragma unroll
        for (int i = 0; i < 2 * ML / E; ++i) {
          vt v;
#pragma unroll
          for (int e = 0; e < E; ++e) v[e] = out[i * E + e];
          *reinterpret_cast<vt*>(sO + tid * OS + l * 2 * ML + i * E) = v;
        }
      }
    }
    __syncthreads();
    R* dst = reinterpret_cast<R*>(S + (((size_t)n * d.F + f) * T + t0) * M);
    for (int c = tid; c < nt * (RW / E); c += kT) {
      const int fr = c / (RW / E), part = c - fr * (RW / E);
      *reinterpret_cast<vt*>(dst + (size_t)c * E) = *reinterpret_cast<const vt*>(sO + fr * OS + part * E);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------
// LDS budgets (bytes) and launches of one compiled set.
template <typename R, int N, int K, int ML, int L>
struct Set {
  static constexpr int M = ML * L;
  // FP32 sets with M_l <= 4 sum the covariances with k_gramd_f (no dynamic LDS); every other
  // set runs k_gram_f in FP64 on the plan's inputs.
  static constexpr bool kGramD = sizeof(R) == 4 && (ML == 2 || ML == 4);
  // k_gram_f stages a bin's g one value per thread: sets above that run in FP32 only.
  static constexpr bool kGramOk = N * M <= kT;
  static size_t smem_gram(const Dims& d) {
    typedef GramShape<double, N, K, ML, L> G;
    return align_up(sizeof(double) * N * M, 16) + sizeof(double) * (size_t)d.SLP * (G::MP + G::OP);
  }
  static size_t max_smem(const Dims& d) { return kGramD ? 0 : smem_gram(d); }
  // LDS windows of W[n] in the H update (k_hgemm_f, or k_hsum_f / k_hlam_f when above one).
  static int hgemm_windows(const Dims& d) {
    const int fp = (d.F + 15) & ~15, fw = GemmLds<R, K>::fw(d);
    return (fp + fw - 1) / fw;
  }
  // BF16 covariances on the matrix cores (DFM_F_GRAM_BF16) exist for the FP32 sets with M_l <= 4.
  static constexpr bool kGramB = kGramD;
  // Workgroups of k_gramd_f (or k_gramb_f) resident per CU (registers and LDS), or 0 if unknown.
  static int gramd_blocks_per_cu(bool bf16) {
    if constexpr (kGramD) {
      int n = 0;
      hipError_t e;
      if constexpr (kGramB) {
        if (bf16)
          e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gramb_f<N, K, ML, L>, 64 * kGBW, 0);
        else
          e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gramd_f<N, K, ML, L>, gramd_threads<L>(), 0);
      } else {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gramd_f<N, K, ML, L>, gramd_threads<L>(), 0);
      }
      return e == hipSuccess ? n : 0;
    } else {
      return 0;
    }
  }

  // Cost or Wiener filter at the end of a run: lambda for the current W, H, then Q^{-1} and
  // ln|det Q|, then the per-frame kernel.
  static hipError_t finish(const Dims& d, const Buffers& b, bool separate, void* S, hipStream_t s) {
    if constexpr (ML <= 4) {
      hipError_t e = launch(d, b, kFLam, s);
      if (e != hipSuccess) return e;
      const cx<R>* X = static_cast<const cx<R>*>(b.X);
      const cx<R>* Q = static_cast<const cx<R>*>(b.Q);
      hipLaunchKernelGGL((k_qinv_f<R, ML>), dim3((d.F * L + 64 / ML - 1) / (64 / ML)), dim3(64), 0, s, d, Q,
                         static_cast<cd*>(b.Qinv), b.logdet, b.status);
      if (separate)
        hipLaunchKernelGGL((k_sep_f<R, N, K, ML, L>), dim3(d.F, d.S), dim3(kT), 0, s, d, X, Q,
                           static_cast<const cd*>(b.Qinv), static_cast<const R*>(b.lam), static_cast<const R*>(b.g),
                           static_cast<cx<R>*>(S));
      else
        hipLaunchKernelGGL((k_nll_f<R, N, K, ML, L>), dim3(d.F, d.S), dim3(kT), 0, s, d, X, Q,
                           static_cast<const R*>(b.lam), static_cast<const R*>(b.g), b.nllpart);
      return hipGetLastError();
    } else {
      return hipErrorNotSupported;
    }
  }

  static hipError_t launch(const Dims& d, const Buffers& b, int kid, hipStream_t s) {
    const cx<R>* X = static_cast<const cx<R>*>(b.X);
    cx<R>* Q = static_cast<cx<R>*>(b.Q);
    R* g = static_cast<R*>(b.g);
    R* W = static_cast<R*>(b.W);
    R* H = static_cast<R*>(b.H);
    R* P = static_cast<R*>(b.P);
    switch (kid) {
      case kFLam:
        hipLaunchKernelGGL((k_lam_f<R, N, K>), dim3(N, (d.T + 15) / 16), dim3(64 * kLamWaves), 0, s, d, W, H,
                           static_cast<R*>(b.lam));
        break;
      case kFGram:
        if constexpr (kGramB) {
          if (d.flags & DFM_F_GRAM_BF16) {
            hipLaunchKernelGGL((k_gramb_f<N, K, ML, L>), dim3(d.GW), dim3(64 * kGBW), 0, s, d, X,
                               static_cast<const R*>(b.lam), g, static_cast<const R*>(b.gpart),
                               static_cast<const R*>(b.gsnap), static_cast<double*>(b.Vpart));
            break;
          }
        }
        if constexpr (kGramD) {
          hipLaunchKernelGGL((k_gramd_f<N, K, ML, L>), dim3(d.GW), dim3(gramd_threads<L>()), 0, s, d, X,
                             static_cast<const R*>(b.lam), g, static_cast<const R*>(b.gpart),
                             static_cast<const R*>(b.gsnap), static_cast<double*>(b.Vpart));
        } else if constexpr (!kGramOk) {
          return hipErrorNotSupported;
        } else {
          hipLaunchKernelGGL((k_gram_f<double, R, N, K, ML, L>), dim3(d.F * d.S), dim3(kT), smem_gram(d), s, d,
                             X, static_cast<const R*>(b.lam), g, static_cast<double*>(b.Vpart));
        }
        break;
      case kFIp:
        if constexpr (ML <= 4) {
          hipLaunchKernelGGL((k_ip_f<R, ML>), dim3((d.F * L + 64 / ML - 1) / (64 / ML)), dim3(64), 0, s, d,
                             static_cast<const double*>(b.Vpart), Q, b.logdet, b.status);
        } else {
          return launch_kernel(d, b, sizeof(R) == 4 ? DFM_C64 : DFM_C128, kKIp, s);
        }
        break;
      case kFPw:
        hipLaunchKernelGGL((k_pw_f<R, N, K, ML, L>), dim3(d.F, (d.S + 1) / 2), dim3(kT), 0, s, d, X, Q,
                           static_cast<const R*>(b.lam), g, P, static_cast<R*>(b.AB));
        break;
      case kFWGemm:
        hipLaunchKernelGGL((k_wgemm_f<R, N, K>), dim3(N, (d.F + 15) / 16), dim3(64 * kGW),
                           (GemmLds<R, K>::wgemm_smem(d)), s, d, static_cast<const R*>(b.AB), H, W,
                           static_cast<R*>(b.lam), b.status);
        break;
      case kFH:
        hipLaunchKernelGGL((k_h_f<R, N, K, ML, L>), dim3(d.F, (d.S + 1) / 2), dim3(kT), 0, s, d,
                           static_cast<const R*>(b.lam), g, P, static_cast<R*>(b.AB));
        break;
      case kFHGemm:
        if (d.HC > 1)
          hipLaunchKernelGGL((k_hsum_f<R, N, K>), dim3(N, d.TBN, d.HC), dim3(64 * kGW),
                             (GemmLds<R, K>::hgemm_smem(d)), s, d, W, static_cast<const R*>(b.AB), H,
                             static_cast<R*>(b.Hpart), static_cast<R*>(b.Hsnap));
        else
          hipLaunchKernelGGL((k_hgemm_f<R, N, K>), dim3(N, (d.T + 15) / 16), dim3(64 * kGW),
                             (GemmLds<R, K>::hgemm_smem(d)), s, d, W, static_cast<const R*>(b.AB), H,
                             static_cast<R*>(b.lam), b.status);
        break;
      case kFHLam:
        hipLaunchKernelGGL((k_hlam_f<R, N, K>), dim3(N, d.TBN, d.HC), dim3(64 * kGW),
                           (GemmLds<R, K>::hgemm_smem(d)), s, d, static_cast<const R*>(b.Hpart),
                           static_cast<const R*>(b.Hsnap), W, H, static_cast<R*>(b.lam), b.status);
        break;
      case kFG:
        hipLaunchKernelGGL((k_g_f<R, N, K, ML, L>), dim3(d.GGW), dim3(kGT), 0, s, d, static_cast<const R*>(b.lam), g,
                           P, static_cast<R*>(b.gpart), static_cast<R*>(b.gsnap));
        break;
      case kFGFin:
        hipLaunchKernelGGL((k_gfin_f<R, N, M>), dim3((d.F * N * M + 255) / 256), dim3(256), 0, s, d,
                           static_cast<const R*>(b.gpart), g, b.status);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
};

}  // namespace fast

// Compiled sets (index, N, K, M_l, L); index = Dims::fast.
#define DFM_FAST_SETS(X)                                                                            \
  X(0, 2, 4, 2, 2) X(1, 5, 16, 4, 4) X(2, 5, 16, 16, 1) X(3, 3, 16, 4, 2) X(4, 8, 16, 4, 3) X(5, 3, 16, 4, 3) \
  X(6, 5, 16, 4, 2) X(7, 8, 16, 4, 2) X(8, 5, 16, 4, 3) X(9, 3, 16, 4, 4) X(10, 8, 16, 4, 4)          \
  X(11, 3, 16, 4, 5) X(12, 5, 16, 4, 5) X(13, 8, 16, 4, 5) X(14, 3, 16, 4, 6) X(15, 5, 16, 4, 6)       \
  X(16, 8, 16, 4, 6) X(17, 3, 16, 4, 7) X(18, 5, 16, 4, 7) X(19, 8, 16, 4, 7) X(20, 3, 16, 4, 8)       \
  X(21, 5, 16, 4, 8) X(22, 8, 16, 4, 8)

hipError_t fast_finish(const Dims& d, const Buffers& b, int dtype, bool separate, void* S, hipStream_t s) {
  switch (d.fast) {
#define DFM_FINISH(i, n, k, ml, l)                                                          \
  case i:                                                                                   \
    return dtype == DFM_C64 ? fast::Set<float, n, k, ml, l>::finish(d, b, separate, S, s)   \
                            : fast::Set<double, n, k, ml, l>::finish(d, b, separate, S, s);
    DFM_FAST_SETS(DFM_FINISH)
#undef DFM_FINISH
  }
  return hipErrorInvalidValue;
}

int fast_set_index(int N, int K, int ML, int L) {
#define DFM_MATCH(i, n, k, ml, l) \
  if (N == n && K == k && ML == ml && L == l) return i;
  DFM_FAST_SETS(DFM_MATCH)
#undef DFM_MATCH
  return -1;
}

bool fast_fp64_ok(int set) {
  switch (set) {
#define DFM_F64(i, n, k, ml, l) \
  case i:                      \
    return fast::Set<double, n, k, ml, l>::kGramOk;
    DFM_FAST_SETS(DFM_F64)
#undef DFM_F64
  }
  return false;
}

int fast_gramd_blocks_per_cu(const Dims& d) {
  const bool bf16 = (d.flags & DFM_F_GRAM_BF16) != 0;
  switch (d.fast) {
#define DFM_OCC(i, n, k, ml, l) \
  case i:                      \
    return fast::Set<float, n, k, ml, l>::gramd_blocks_per_cu(bf16);
    DFM_FAST_SETS(DFM_OCC)
#undef DFM_OCC
  }
  return 0;
}

int fast_hgemm_windows(const Dims& d, int dtype) {
  switch (d.fast) {
#define DFM_HW(i, n, k, ml, l)                                                       \
  case i:                                                                            \
    return dtype == DFM_C64 ? fast::Set<float, n, k, ml, l>::hgemm_windows(d)        \
                            : fast::Set<double, n, k, ml, l>::hgemm_windows(d);
    DFM_FAST_SETS(DFM_HW)
#undef DFM_HW
  }
  return 1;
}

size_t fast_max_smem(const Dims& d, int dtype) {
  switch (d.fast) {
#define DFM_SMEM(i, n, k, ml, l)                                                     \
  case i:                                                                            \
    return dtype == DFM_C64 ? fast::Set<float, n, k, ml, l>::max_smem(d)             \
                            : fast::Set<double, n, k, ml, l>::max_smem(d);
    DFM_FAST_SETS(DFM_SMEM)
#undef DFM_SMEM
  }
  return 0;
}

bool fast_gram_bf16(int N, int K, int ML, int L) {
#define DFM_GB(i, n, k, ml, l) \
  if (N == n && K == k && ML == ml && L == l) return fast::Set<float, n, k, ml, l>::kGramB;
  DFM_FAST_SETS(DFM_GB)
#undef DFM_GB
  return false;
}

const char* fast_kernel_name(const Dims& d, int dtype, int kid) {
  if (kid == kFGram && dtype == DFM_C64 && (d.flags & DFM_F_GRAM_BF16)) return "k_gramb_f";
  if (kid == kFGram && dtype == DFM_C64 && (d.ML == 2 || d.ML == 4)) return "k_gramd_f";
  if (kid == kFIp && d.ML > 4) return kernel_name(kKIp);
  if (kid == kFHGemm && d.HC > 1) return "k_hsum_f";
  return kernel_name(kid);
}

hipError_t fast_launch(const Dims& d, const Buffers& b, int dtype, int kid, hipStream_t s) {
  switch (d.fast) {
#define DFM_LAUNCH(i, n, k, ml, l)                                                   \
  case i:                                                                            \
    return dtype == DFM_C64 ? fast::Set<float, n, k, ml, l>::launch(d, b, kid, s)    \
                            : fast::Set<double, n, k, ml, l>::launch(d, b, kid, s);
    DFM_FAST_SETS(DFM_LAUNCH)
#undef DFM_LAUNCH
  }
  return hipErrorInvalidValue;
}

}  // namespace dfm
