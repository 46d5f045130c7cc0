// Shape-specialised kernels of distributed FastMNMF for gfx950.
//
// Used when every subarray has the same size ML and (N, K, ML, L) is one of the compiled
// sets (DFM_FAST_SETS below).  All four are compile-time constants, so every per-frame
// array (lambda_n, y_m, |Qx|^2, x) lives in registers with a compile-time size and every
// loop over sources, bases and mics is unrolled.  Global loads that feed a computation
// are issued as one batch behind a scheduling barrier (left alone, the scheduler trades
// them for occupancy and waits on each load in turn).
//
// One iteration is these five kernels plus the three small apply kernels of the generic
// path, which sum the per-tile partials in a fixed order (so every result is
// deterministic run to run) and update W, H and g.  Finishing the reductions inside the
// streaming kernels with a last-arriving workgroup was measured slower on gfx950: the
// device-scope release/acquire it needs writes back and invalidates L2 in every
// workgroup.
//
//   k_gram_f  tile (f, time slice), 128 threads.  1/y per frame on the vector units,
//             then the weighted covariances of eq. (14) as a real contraction over
//             frames on the matrix cores (v_mfma 16x16x4: rows = mu, columns = packed
//             Hermitian entries of x x^H, K = 4 frames).
//   k_ip_f    one lane per (f, subarray): FP64 IP sweep of eqs. (15)-(16) (M_l <= 4;
//             larger blocks use the cooperative generic kernel).
//   k_pw_f    tile (f, time slice), 128 threads.  P = |Q x|^2 and the per-frame sums of
//             eq. (8); the contraction with H over frames reads H staged in LDS.
//   k_h_f     16 bins per wave x 16 frames.  lambda = W H and the sum over frequencies
//             of eq. (9) are both 16x16x4 matrix-core contractions.
//   k_g_f     tile (f, time slice), 128 threads.  Sums of eq. (10).
#include <hip/hip_runtime.h>

#include "dfm_device.h"

namespace dfm {
namespace fast {

constexpr int kT = 128;   // threads of the (f, time slice) kernels: one frame per thread
constexpr int kHTB = 16;  // frames per activation tile

__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

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

template <typename R, int C>
__device__ __forceinline__ void store16_nt(R* dst, const R (&src)[C]) {
  constexpr int E = V16<R>::E;
  static_assert(C % E == 0, "length must fill 16-byte vectors");
#pragma unroll
  for (int i = 0; i < C / E; ++i) {
    typename V16<R>::type v;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = src[i * E + e];
    __builtin_nontemporal_store(v, reinterpret_cast<typename V16<R>::type*>(dst) + i);
  }
}

// H[n][k][t] for every (n, k) at one frame, as one batch of loads.
template <typename R, int NK>
__device__ __forceinline__ void load_h_column(R (&hv)[NK], const R* __restrict__ H, int T, int t) {
#pragma unroll
  for (int i = 0; i < NK; ++i) hv[i] = H[(size_t)i * T + t];
}

// ------------------------------------------------------------------------------------
// FP64 IP sweep of one subarray block (M_l <= 4), eqs. (15)-(16).  Q in registers; the
// covariance of the current row in the lane's private LDS slot sV (M_l x M_l complex).
// vp: packed slice sums of the block, [slice (stride vstride)][mu][M_l^2]; V = sum / T.
template <typename R, int ML>
__device__ void ip_sweep_lane(const R* vp, size_t vstride, int S, double invT, cd (&Qm)[ML][ML], cd* sV,
                              double eps, int* status) {
  constexpr int ML2 = ML * ML;
  for (int mu = 0; mu < ML; ++mu) {
    double vs[ML2];
#pragma unroll
    for (int j = 0; j < ML2; ++j) vs[j] = 0.0;
    for (int q = 0; q < S; ++q) {
      R part[ML2];
#pragma unroll
      for (int j = 0; j < ML2; ++j) part[j] = vp[q * vstride + mu * ML2 + j];
#pragma unroll
      for (int j = 0; j < ML2; ++j) vs[j] += (double)part[j];
    }
#pragma unroll
    for (int j = 0; j < ML2; ++j) {
      int a, b, part;
      packed_pair(ML, j, a, b, part);
      const double v = vs[j] * invT;
      if (a == b) {
        sV[a * ML + a] = {v, 0.0};
      } else if (part == 0) {
        sV[a * ML + b].re = v;
        sV[b * ML + a].re = v;
      } else {
        sV[a * ML + b].im = v;
        sV[b * ML + a].im = -v;
      }
    }
    cd A[ML][ML + 1];
#pragma unroll
    for (int r = 0; r < ML; ++r) {
#pragma unroll
      for (int c = 0; c < ML; ++c) {
        cd acc = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < ML; ++j) acc = cadd(acc, cmul(Qm[r][j], sV[j * ML + c]));
        A[r][c] = acc;
      }
      A[r][ML] = {r == mu ? 1.0 : 0.0, 0.0};
    }
    bool sing = false;
#pragma unroll
    for (int p = 0; p < ML; ++p) {
      int piv = p;
      double best = cabs2(A[p][p]);
#pragma unroll
      for (int r = p + 1; r < ML; ++r) {
        const double v = cabs2(A[r][p]);
        if (v > best) {
          best = v;
          piv = r;
        }
      }
#pragma unroll
      for (int r = p + 1; r < ML; ++r) {
        const bool sw = piv == r;
#pragma unroll
        for (int c = p; c <= ML; ++c) {
          const cd tp = A[p][c], tr = A[r][c];
          A[p][c] = sw ? tr : tp;
          A[r][c] = sw ? tp : tr;
        }
      }
      if (best == 0.0) sing = true;
      const cd inv = best == 0.0 ? cd{0.0, 0.0} : cinv(A[p][p]);
#pragma unroll
      for (int r = p + 1; r < ML; ++r) {
        const cd fac = cmul(A[r][p], inv);
#pragma unroll
        for (int c = p + 1; c <= ML; ++c) A[r][c] = csub(A[r][c], cmul(fac, A[p][c]));
      }
    }
    if (sing) {
      atomicOr(status, kStSingular);  // row kept; reported as DFM_E_SINGULAR
      continue;
    }
    cd bsol[ML];
#pragma unroll
    for (int r = ML - 1; r >= 0; --r) {
      cd acc = A[r][ML];
#pragma unroll
      for (int c = r + 1; c < ML; ++c) acc = csub(acc, cmul(A[r][c], bsol[c]));
      bsol[r] = cmul(acc, cinv(A[r][r]));
    }
    double sv = 0.0;
#pragma unroll
    for (int a = 0; a < ML; ++a) {
      cd vb = {0.0, 0.0};
#pragma unroll
      for (int b = 0; b < ML; ++b) vb = cadd(vb, cmul(sV[a * ML + b], bsol[b]));
      sv += bsol[a].re * vb.re + bsol[a].im * vb.im;
    }
    const double sc = 1.0 / sqrt(sv > eps ? sv : eps);
#pragma unroll
    for (int c = 0; c < ML; ++c) Qm[mu][c] = {bsol[c].re * sc, -bsol[c].im * sc};
  }
}

// ln|det| of an M_l x M_l complex matrix by elimination with partial pivoting, in registers.
template <int ML>
__device__ double logabsdet_lane(cd (&A)[ML][ML]) {
  double acc = 0.0;
#pragma unroll
  for (int p = 0; p < ML; ++p) {
    int piv = p;
    double best = cabs2(A[p][p]);
#pragma unroll
    for (int r = p + 1; r < ML; ++r) {
      const double v = cabs2(A[r][p]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
#pragma unroll
    for (int r = p + 1; r < ML; ++r) {
      const bool sw = piv == r;
#pragma unroll
      for (int c = p; c < ML; ++c) {
        const cd tp = A[p][c], tr = A[r][c];
        A[p][c] = sw ? tr : tp;
        A[r][c] = sw ? tp : tr;
      }
    }
    if (best == 0.0) return -INFINITY;
    acc += 0.5 * log(best);
    const cd inv = cinv(A[p][p]);
#pragma unroll
    for (int r = p + 1; r < ML; ++r) {
      const cd fac = cmul(A[r][p], inv);
#pragma unroll
      for (int c = p + 1; c < ML; ++c) A[r][c] = csub(A[r][c], cmul(fac, A[p][c]));
    }
  }
  return acc;
}

// ------------------------------------------------------------------------------------
// Weighted covariances (eq. (14)) on the matrix cores.
template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(kT) void k_gram_f(Dims d, const cx<R>* __restrict__ X, const R* __restrict__ W,
                                               const R* __restrict__ H, const R* __restrict__ g,
                                               R* __restrict__ Vpart) {
  constexpr int M = ML * L, NK = N * K, ML2 = ML * ML;
  constexpr int JT = (ML2 + 15) / 16;
  constexpr int E = V16<R>::E;
  static_assert((2 * M) % E == 0 && M % E == 0, "rows must fill 16-byte vectors");
  typedef typename Mma<R>::v4 v4;
  typedef typename V16<R>::type vt;
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int T = d.T;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, T - t0);
  const int ntp = (nt + 3) & ~3;
  extern __shared__ __align__(16) unsigned char smem[];
  R* sW = reinterpret_cast<R*>(smem);
  R* sg = sW + NK;
  R* sInv = reinterpret_cast<R*>(smem + align_up(sizeof(R) * (NK + N * M), 16));  // [SLP][M]
  R* sX = sInv + (size_t)d.SLP * M;                                                // [SLP][2M]

  for (int i = tid; i < NK; i += kT) sW[i] = W[((size_t)(i / K) * d.F + f) * K + i % K];
  for (int i = tid; i < N * M; i += kT) sg[i] = g[(size_t)f * N * M + i];
  {  // X tile -> LDS in 16-byte vectors, one batch of loads per thread
    constexpr int PER = (128 * 2 * M / E + kT - 1) / kT;  // vectors per thread for a 128-frame slice
    const vt* src = reinterpret_cast<const vt*>(X + ((size_t)f * T + t0) * M);
    vt* dst = reinterpret_cast<vt*>(sX);
    const int nv = nt * 2 * M / E, nvp = ntp * 2 * M / E;
    for (int base = 0; base < nvp; base += PER * kT) {
      vt buf[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int i = base + tid + u * kT;
        buf[u] = i < nv ? src[i] : vt{};
      }
      sched_fence();
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int i = base + tid + u * kT;
        if (i < nvp) dst[i] = buf[u];
      }
    }
  }
  __syncthreads();

  for (int tl = tid; tl < ntp; tl += kT) {
    R inv[M];
    if (tl < nt) {
      R hv[NK];
      load_h_column<R, NK>(hv, H, T, t0 + tl);
      sched_fence();
      R lam[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        R acc = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) acc += sW[n * K + k] * hv[n * K + k];
        lam[n] = acc;
      }
#pragma unroll
      for (int m = 0; m < M; ++m) {
        R y = 0;
#pragma unroll
        for (int n = 0; n < N; ++n) y += lam[n] * sg[n * M + m];
        inv[m] = rcp(rmax(y, (R)d.eps));
      }
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) inv[m] = 0;
    }
#pragma unroll
    for (int i = 0; i < M / E; ++i) {
      vt v;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = inv[i * E + e];
      reinterpret_cast<vt*>(sInv + (size_t)tl * M)[i] = v;
    }
  }
  __syncthreads();

  // C[mu][j] += sum over 4 frames of (1/y)[frame][mu] * O[frame][j], O = packed x x^H;
  // two accumulators alternate so consecutive matrix-core ops are independent.
  const int col = lane & 15, kk = lane >> 4;
  const cx<R>* sXc = reinterpret_cast<const cx<R>*>(sX);
  for (int item = wave; item < L * JT; item += kT / 64) {
    const int l = item / JT, jt = item - l * JT;
    const int o = l * ML;
    const int j = jt * 16 + col;
    const bool jv = j < ML2;
    int a = 0, b = 0, part = 0;
    if (jv) packed_pair(ML, j, a, b, part);
    const bool rv = col < ML;
    v4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    for (int step = 0; step < ntp; step += 8) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int tl = step + 4 * h + kk;
        R av = 0, bv = 0;
        if (tl < ntp) {
          av = rv ? sInv[tl * M + o + col] : (R)0;
          if (jv) {
            const cx<R> xa = sXc[tl * M + o + a], xb = sXc[tl * M + o + b];
            bv = part == 0 ? xa.re * xb.re + xa.im * xb.im : xa.im * xb.re - xa.re * xb.im;
          }
        }
        if (h == 0)
          acc0 = Mma<R>::run(av, bv, acc0);
        else
          acc1 = Mma<R>::run(av, bv, acc1);
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

// IP sweep, eqs. (15)-(16), one lane per (f, subarray) block of size M_l <= 4, in FP64;
// then ln|det Q_fl| for the cost (13).
template <typename R, int ML>
__global__ __launch_bounds__(64) void k_ip_f(Dims d, const R* __restrict__ Vpart, cx<R>* __restrict__ Q,
                                             double* __restrict__ logdet, int* __restrict__ status) {
  constexpr int ML2 = ML * ML;
  __shared__ cd sV[64 * ML2];
  const int idx = blockIdx.x * 64 + threadIdx.x;
  if (idx >= d.F * d.L) return;
  const int f = idx / d.L, l = idx - f * d.L;
  cx<R>* qb = Q + (size_t)f * d.QF + l * ML2;
  cd Qm[ML][ML];
#pragma unroll
  for (int r = 0; r < ML; ++r)
#pragma unroll
    for (int c = 0; c < ML; ++c) Qm[r][c] = {(double)qb[r * ML + c].re, (double)qb[r * ML + c].im};
  ip_sweep_lane<R, ML>(Vpart + (size_t)f * d.S * d.VF + (size_t)l * ML * ML2, d.VF, d.S, 1.0 / d.T, Qm,
                       sV + threadIdx.x * ML2, d.eps, status);
#pragma unroll
  for (int r = 0; r < ML; ++r)
#pragma unroll
    for (int c = 0; c < ML; ++c) {
      const cx<R> q = {(R)Qm[r][c].re, (R)Qm[r][c].im};
      qb[r * ML + c] = q;
      Qm[r][c] = {(double)q.re, (double)q.im};
    }
  logdet[idx] = logabsdet_lane<ML>(Qm);
}

// ------------------------------------------------------------------------------------
// P = |Q x|^2 and the eq. (8) sums per (f, slice).
template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(kT) void k_pw_f(Dims d, const cx<R>* __restrict__ X, const cx<R>* __restrict__ Q,
                                             const R* __restrict__ W, const R* __restrict__ H, const R* __restrict__ g,
                                             R* __restrict__ P, R* __restrict__ Wpart) {
  constexpr int M = ML * L, NK = N * K, ML2 = ML * ML, QF = L * ML2;
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int T = d.T, SLP = d.SLP;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, T - t0);
  const int ntp = (nt + 3) & ~3;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<R>* sQ = reinterpret_cast<cx<R>*>(smem);
  R* sW = reinterpret_cast<R*>(smem + align_up(sizeof(cx<R>) * QF, 16));
  R* sg = sW + NK;
  R* sH = reinterpret_cast<R*>(smem + align_up(sizeof(cx<R>) * QF, 16) + align_up(sizeof(R) * (NK + N * M), 16));
  R* sab = sH + (size_t)NK * SLP;  // [2N][SLP]

  for (int i = tid; i < QF; i += kT) sQ[i] = Q[(size_t)f * QF + i];
  for (int i = tid; i < NK; i += kT) sW[i] = W[((size_t)(i / K) * d.F + f) * K + i % K];
  for (int i = tid; i < N * M; i += kT) sg[i] = g[(size_t)f * N * M + i];
  __syncthreads();

  for (int tl = tid; tl < ntp; tl += kT) {
    if (tl < nt) {
      const int t = t0 + tl;
      R hv[NK], xv[2 * M];
      load_h_column<R, NK>(hv, H, T, t);
      load16<R, 2 * M>(xv, reinterpret_cast<const R*>(X + ((size_t)f * T + t) * M));
      sched_fence();
      R lam[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        R acc = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          sH[(n * K + k) * SLP + tl] = hv[n * K + k];
          acc += sW[n * K + k] * hv[n * K + k];
        }
        lam[n] = acc;
      }
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
          for (int c = 0; c < ML; ++c) {
            const cx<R> q = sQ[l * ML2 + mu * ML + c];
            const R xr = xv[2 * (l * ML + c)], xi = xv[2 * (l * ML + c) + 1];
            zr += q.re * xr - q.im * xi;
            zi += q.re * xi + q.im * xr;
          }
          const int m = l * ML + mu;
          const R p = zr * zr + zi * zi;
          pv[m] = p;
          R y = 0;
#pragma unroll
          for (int n = 0; n < N; ++n) y += lam[n] * sg[n * M + m];
          const R iy = rcp(rmax(y, (R)d.eps));
          const R piy2 = p * iy * iy;
#pragma unroll
          for (int n = 0; n < N; ++n) {
            a[n] += sg[n * M + m] * piy2;
            b[n] += sg[n * M + m] * iy;
          }
        }
      }
      store16_nt<R, M>(P + ((size_t)f * T + t) * M, pv);
#pragma unroll
      for (int n = 0; n < N; ++n) {
        sab[n * SLP + tl] = a[n];
        sab[(N + n) * SLP + tl] = b[n];
      }
    } else {
#pragma unroll
      for (int i = 0; i < NK; ++i) sH[i * SLP + tl] = 0;
#pragma unroll
      for (int i = 0; i < 2 * N; ++i) sab[i * SLP + tl] = 0;
    }
  }
  __syncthreads();

  R* out = Wpart + ((size_t)f * d.S + s) * NK * 2;
  for (int o = tid; o < NK; o += kT) {
    const int n = o / K;
    const R* hr = sH + o * SLP;
    const R* ar = sab + n * SLP;
    const R* br = sab + (N + n) * SLP;
    R num0 = 0, den0 = 0, num1 = 0, den1 = 0;
    for (int tl = 0; tl < ntp; tl += 4) {
      num0 += hr[tl] * ar[tl] + hr[tl + 2] * ar[tl + 2];
      den0 += hr[tl] * br[tl] + hr[tl + 2] * br[tl + 2];
      num1 += hr[tl + 1] * ar[tl + 1] + hr[tl + 3] * ar[tl + 3];
      den1 += hr[tl + 1] * br[tl + 1] + hr[tl + 3] * br[tl + 3];
    }
    out[o * 2 + 0] = num0 + num1;
    out[o * 2 + 1] = den0 + den1;
  }

}

// ------------------------------------------------------------------------------------
// Activation update, eq. (9).  Workgroup = HW waves; wave w owns 16 bins, all waves share
// one block of 16 frames.
template <typename R>
constexpr int h_waves() { return sizeof(R) == 4 ? 4 : 2; }

template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(64 * h_waves<R>()) void k_h_f(Dims d, const R* __restrict__ W, const R* __restrict__ H,
                                                           const R* __restrict__ g, const R* __restrict__ P,
                                                           R* __restrict__ Hpart) {
  constexpr int HW = h_waves<R>();
  constexpr int NT = 64 * HW;
  constexpr int M = ML * L, NK = N * K;
  constexpr int KS = (K + 3) / 4;    // 4-deep steps over bases for lambda = W H
  constexpr int KT = (K + 15) / 16;  // 16-row tiles of bases for the sum over frequencies
  typedef typename Mma<R>::v4 v4;
  const int fg = blockIdx.x, tb = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int T = d.T, F = d.F;
  const int t0 = tb * kHTB;
  const int ntb = min(kHTB, T - t0);
  const int f0 = (fg * HW + wave) * 16;
  const int nf = max(0, min(16, F - f0));
  extern __shared__ __align__(16) unsigned char smem[];
  R* sHt = reinterpret_cast<R*>(smem);                            // [NK][16]
  R* sgc = sHt + NK * kHTB + wave * (16 * N * M);                // per wave [16 f][N*M]
  R* sAB = sHt + NK * kHTB + HW * 16 * N * M + wave * (2 * 256); // per wave [2][16 f][16 t]

  const int cl = lane & 15, ck = lane >> 4;
  // Matrix-core A operands (W) of both contractions, as one batch of loads.
  R wl[N][KS], wh[N][KT][4];
#pragma unroll
  for (int n = 0; n < N; ++n) {
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      const int k = 4 * st + ck;
      wl[n][st] = (k < K && cl < nf) ? W[((size_t)n * F + f0 + cl) * K + k] : (R)0;
    }
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int fl = 4 * st + ck, k = kt * 16 + cl;
        wh[n][kt][st] = (k < K && fl < nf) ? W[((size_t)n * F + f0 + fl) * K + k] : (R)0;
      }
  }
  for (int i = tid; i < NK * kHTB; i += NT) {
    const int nk = i / kHTB, tl = i % kHTB;
    sHt[i] = tl < ntb ? H[(size_t)nk * T + t0 + tl] : (R)0;
  }
  for (int i = lane; i < 16 * N * M; i += 64) {
    const int fl = i / (N * M);
    sgc[i] = fl < nf ? g[(size_t)(f0 + fl) * N * M + i % (N * M)] : (R)0;
  }
  __syncthreads();

  // lambda_n[f][t] = sum_k W[n][f][k] H[n][k][t]: A = W (rows f), B = H (columns t).
  R lam[N][4];
#pragma unroll
  for (int n = 0; n < N; ++n) {
    v4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      const int k = 4 * st + ck;
      const R bv = k < K ? sHt[(n * K + k) * kHTB + cl] : (R)0;
      acc = Mma<R>::run(wl[n][st], bv, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) lam[n][r] = acc[r];
  }
  // a' and b' of eq. (9) for the four (f, t) pairs this lane holds (column t = cl).
  R pv[4][M];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int fl = Mma<R>::row(lane, r);
    if (fl < nf && cl < ntb) {
      load16<R, M>(pv[r], P + ((size_t)(f0 + fl) * T + t0 + cl) * M);
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) pv[r][m] = 0;
    }
  }
  sched_fence();
  R a[N][4], b[N][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int fl = Mma<R>::row(lane, r);
    const R* gf = sgc + fl * N * M;
#pragma unroll
    for (int n = 0; n < N; ++n) {
      a[n][r] = 0;
      b[n][r] = 0;
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      R y = 0;
#pragma unroll
      for (int n = 0; n < N; ++n) y += lam[n][r] * gf[n * M + m];
      const R iy = rcp(rmax(y, (R)d.eps));
      const R piy2 = pv[r][m] * iy * iy;
#pragma unroll
      for (int n = 0; n < N; ++n) {
        a[n][r] += gf[n * M + m] * piy2;
        b[n][r] += gf[n * M + m] * iy;
      }
    }
  }
  // num/den[n][k][t] = sum_f W[n][f][k] (a', b')[n][f][t]: A = W^T (rows k), B = a'/b' (columns t).
  v4 accN[N][KT], accD[N][KT];
#pragma unroll
  for (int n = 0; n < N; ++n) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int fl = Mma<R>::row(lane, r);
      sAB[fl * 16 + cl] = a[n][r];
      sAB[256 + fl * 16 + cl] = b[n][r];
    }
    __syncthreads();
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      accN[n][kt] = v4{0, 0, 0, 0};
      accD[n][kt] = v4{0, 0, 0, 0};
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int fl = 4 * st + ck;
        accN[n][kt] = Mma<R>::run(wh[n][kt][st], sAB[fl * 16 + cl], accN[n][kt]);
        accD[n][kt] = Mma<R>::run(wh[n][kt][st], sAB[256 + fl * 16 + cl], accD[n][kt]);
      }
    }
    __syncthreads();
  }
  // Sum the waves in order through LDS, then write this frequency group's partial.
  R* sRed = reinterpret_cast<R*>(smem);  // [N][KT*16][16][2]
  for (int w = 0; w < HW; ++w) {
    if (wave == w) {
#pragma unroll
      for (int n = 0; n < N; ++n)
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k = kt * 16 + Mma<R>::row(lane, r);
            R* dst = sRed + ((n * KT * 16 + k) * 16 + cl) * 2;
            dst[0] = (w == 0 ? (R)0 : dst[0]) + accN[n][kt][r];
            dst[1] = (w == 0 ? (R)0 : dst[1]) + accD[n][kt][r];
          }
    }
    __syncthreads();
  }
  for (int i = tid; i < NK * ntb * 2; i += NT) {
    const int w = i & 1, rest = i >> 1;
    const int tl = rest % ntb, nk = rest / ntb;
    const int n = nk / K, k = nk % K;
    Hpart[(((size_t)fg * NK + nk) * T + t0 + tl) * 2 + w] = sRed[((n * KT * 16 + k) * 16 + tl) * 2 + w];
  }

}

// ------------------------------------------------------------------------------------
// Eq. (10) sums per (f, slice).
template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(kT) void k_g_f(Dims d, const R* __restrict__ W, const R* __restrict__ H,
                                            const R* __restrict__ g, const R* __restrict__ P,
                                            R* __restrict__ gpart) {
  constexpr int M = ML * L, NK = N * K;
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int T = d.T, SLP = d.SLP;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, T - t0);
  const int ntp = (nt + 3) & ~3;
  extern __shared__ __align__(16) unsigned char smem[];
  R* sW = reinterpret_cast<R*>(smem);
  R* sg = sW + NK;
  R* sLam = sg + N * M;    // [N][SLP]
  R* sR = sLam + N * SLP;  // [2M][SLP]

  for (int i = tid; i < NK; i += kT) sW[i] = W[((size_t)(i / K) * d.F + f) * K + i % K];
  for (int i = tid; i < N * M; i += kT) sg[i] = g[(size_t)f * N * M + i];
  __syncthreads();

  for (int tl = tid; tl < ntp; tl += kT) {
    if (tl < nt) {
      const int t = t0 + tl;
      R hv[NK], pv[M];
      load_h_column<R, NK>(hv, H, T, t);
      load16<R, M>(pv, P + ((size_t)f * T + t) * M);
      sched_fence();
      R lam[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        R acc = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) acc += sW[n * K + k] * hv[n * K + k];
        lam[n] = acc;
        sLam[n * SLP + tl] = acc;
      }
#pragma unroll
      for (int m = 0; m < M; ++m) {
        R y = 0;
#pragma unroll
        for (int n = 0; n < N; ++n) y += lam[n] * sg[n * M + m];
        const R iy = rcp(rmax(y, (R)d.eps));
        sR[m * SLP + tl] = pv[m] * iy * iy;
        sR[(M + m) * SLP + tl] = iy;
      }
    } else {
#pragma unroll
      for (int n = 0; n < N; ++n) sLam[n * SLP + tl] = 0;
#pragma unroll
      for (int m = 0; m < 2 * M; ++m) sR[m * SLP + tl] = 0;
    }
  }
  __syncthreads();

  R* out = gpart + ((size_t)f * d.S + s) * N * M * 2;
  for (int o = tid; o < N * M; o += kT) {
    const int n = o / M, m = o % M;
    const R* lr = sLam + n * SLP;
    const R* r1 = sR + m * SLP;
    const R* r2 = sR + (M + m) * SLP;
    R num0 = 0, den0 = 0, num1 = 0, den1 = 0;
    for (int tl = 0; tl < ntp; tl += 4) {
      num0 += lr[tl] * r1[tl] + lr[tl + 2] * r1[tl + 2];
      den0 += lr[tl] * r2[tl] + lr[tl + 2] * r2[tl + 2];
      num1 += lr[tl + 1] * r1[tl + 1] + lr[tl + 3] * r1[tl + 3];
      den1 += lr[tl + 1] * r2[tl + 1] + lr[tl + 3] * r2[tl + 3];
    }
    out[o * 2 + 0] = num0 + num1;
    out[o * 2 + 1] = den0 + den1;
  }

}

// ------------------------------------------------------------------------------------
// LDS budgets (bytes) and launches of one compiled set.
template <typename R, int N, int K, int ML, int L>
struct Set {
  static constexpr int M = ML * L;
  static size_t smem_gram(const Dims& d) {
    return align_up(sizeof(R) * (N * K + N * M), 16) + sizeof(R) * d.SLP * 3 * M;
  }
  static size_t smem_pw(const Dims& d) {
    return align_up(sizeof(cx<R>) * L * ML * ML, 16) + align_up(sizeof(R) * (N * K + N * M), 16) +
           sizeof(R) * (N * K + 2 * N) * d.SLP;
  }
  static size_t smem_h(const Dims&) {
    constexpr int KT = (K + 15) / 16;
    constexpr int HW = h_waves<R>();
    const size_t stage = sizeof(R) * (N * K * kHTB + HW * 16 * N * M + HW * 2 * 256);
    const size_t red = sizeof(R) * N * KT * 16 * 16 * 2;
    return stage > red ? stage : red;
  }
  static size_t smem_g(const Dims& d) { return sizeof(R) * (N * K + N * M + (N + 2 * M) * d.SLP); }
  static size_t max_smem(const Dims& d) {
    size_t m = smem_gram(d);
    m = smem_pw(d) > m ? smem_pw(d) : m;
    m = smem_h(d) > m ? smem_h(d) : m;
    return smem_g(d) > m ? smem_g(d) : m;
  }

  static hipError_t launch(const Dims& d, const Buffers& b, int kid, hipStream_t s) {
    const cx<R>* X = static_cast<const cx<R>*>(b.X);
    cx<R>* Q = static_cast<cx<R>*>(b.Q);
    R* g = static_cast<R*>(b.g);
    R* W = static_cast<R*>(b.W);
    R* H = static_cast<R*>(b.H);
    R* P = static_cast<R*>(b.P);
    switch (kid) {
      case kFGram:
        hipLaunchKernelGGL((k_gram_f<R, N, K, ML, L>), dim3(d.F, d.S), dim3(kT), smem_gram(d), s, d, X, W, H, g,
                           static_cast<R*>(b.Vpart));
        break;
      case kFIp:
        if constexpr (ML <= 4) {
          hipLaunchKernelGGL((k_ip_f<R, ML>), dim3((d.F * L + 63) / 64), dim3(64), 0, s, d,
                             static_cast<const R*>(b.Vpart), Q, b.logdet, b.status);
        } else {
          return launch_kernel(d, b, sizeof(R) == 4 ? DFM_C64 : DFM_C128, kKIp, s);
        }
        break;
      case kFPw:
        hipLaunchKernelGGL((k_pw_f<R, N, K, ML, L>), dim3(d.F, d.S), dim3(kT), smem_pw(d), s, d, X, Q, W, H, g,
                           P, static_cast<R*>(b.Wpart));
        break;
      case kFH:
        hipLaunchKernelGGL((k_h_f<R, N, K, ML, L>), dim3(d.FG, d.TBN), dim3(64 * h_waves<R>()), smem_h(d), s, d,
                           W, H, g, P, static_cast<R*>(b.Hpart));
        break;
      case kFG:
        hipLaunchKernelGGL((k_g_f<R, N, K, ML, L>), dim3(d.F, d.S), dim3(kT), smem_g(d), s, d, W, H, g, P,
                           static_cast<R*>(b.gpart));
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
};

}  // namespace fast

// Compiled sets (index, N, K, M_l, L); index = Dims::fast.
#define DFM_FAST_SETS(X) \
  X(0, 2, 4, 2, 2) X(1, 5, 16, 4, 4) X(2, 5, 16, 16, 1) X(3, 3, 16, 4, 2) X(4, 8, 16, 4, 3)

int fast_set_index(int N, int K, int ML, int L) {
#define DFM_MATCH(i, n, k, ml, l) \
  if (N == n && K == k && ML == ml && L == l) return i;
  DFM_FAST_SETS(DFM_MATCH)
#undef DFM_MATCH
  return -1;
}

int fast_h_waves(int dtype) { return dtype == DFM_C64 ? fast::h_waves<float>() : fast::h_waves<double>(); }

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
