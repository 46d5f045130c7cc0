// Shape-specialised kernels of distributed FastMNMF for gfx950.
//
// Used when every subarray has the same size ML and (N, K, ML) is one of the compiled
// sets (see kFastSets).  N, K and ML are compile-time constants, so the per-frame model
// arrays live in registers and every loop over sources, bases and in-subarray mics is
// unrolled.  One iteration is four streaming kernels, each finishing its own reduction with a
// last-arriving workgroup (fixed summation order, so results are deterministic), plus
// the small IP kernel:
//
//   k_gram_f  tile (f, time slice), 128 threads.  1/y per frame on the vector units,
//             then the weighted covariances of eq. (14) as a real contraction over
//             frames on the matrix cores (v_mfma 16x16x4: rows = mu, columns = packed
//             Hermitian entries, K = 4 frames).
//   k_ip_f    one lane per (f, subarray): FP64 IP sweep of eqs. (15)-(16) in registers
//             (M_l <= 4; larger blocks use the cooperative generic kernel).
//   k_pw_f    tile (f, time slice), 128 threads.  P = |Q x|^2 and the per-frame sums of
//             eq. (8); the contraction with H over frames reads H staged in LDS.  The
//             last slice applies the update of W for its frequency.
//   k_h_f     tile (16 bins per wave, 16 frames), 4 waves (2 in FP64).  lambda = W H and the sum over
//             frequencies of eq. (9) are both 16x16x4 matrix-core contractions; the
//             last frequency group of a frame block applies the update of H.
//   k_g_f     tile (f, time slice), 128 threads.  Sums of eq. (10); the last slice
//             applies the update of g for its frequency.
#include <hip/hip_runtime.h>

#include "dfm_device.h"

namespace dfm {
namespace fast {

constexpr int kT = 128;   // threads of the (f, time slice) kernels: one frame per thread
constexpr int kHTB = 16;  // frames per activation tile

// Packed Hermitian index -> (a, b, part), as packed_pair but for compile-time M_l.
template <int ML>
__device__ __forceinline__ void pair_of(int j, int& a, int& b, int& part) { packed_pair(ML, j, a, b, part); }

// ------------------------------------------------------------------------------------
// FP64 IP sweep of one subarray block in registers (M_l <= 4), eqs. (15)-(16).
// vp: packed covariance slice sums of the block, [slice (stride vstride)][mu][M_l^2];
// V_mu = (sum over the S slices) / T.
template <typename R, int ML>
__device__ void ip_sweep_lane(const R* vp, size_t vstride, int S, double invT, cd (&Qm)[ML][ML], double eps,
                              int* status) {
  constexpr int ML2 = ML * ML;
#pragma unroll
  for (int mu = 0; mu < ML; ++mu) {
    cd V[ML][ML];
#pragma unroll
    for (int j = 0; j < ML2; ++j) {
      int a, b, part;
      pair_of<ML>(j, a, b, part);
      double v = 0.0;
      for (int q = 0; q < S; ++q) v += (double)vp[q * vstride + mu * ML2 + j];
      v *= invT;
      if (a == b) {
        V[a][a] = {v, 0.0};
      } else if (part == 0) {
        V[a][b].re = v;
        V[b][a].re = v;
      } else {
        V[a][b].im = v;
        V[b][a].im = -v;
      }
    }
    cd A[ML][ML + 1];
#pragma unroll
    for (int r = 0; r < ML; ++r) {
#pragma unroll
      for (int c = 0; c < ML; ++c) {
        cd acc = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < ML; ++j) acc = cadd(acc, cmul(Qm[r][j], V[j][c]));
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
      for (int b = 0; b < ML; ++b) vb = cadd(vb, cmul(V[a][b], bsol[b]));
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
template <typename R, int N, int K, int ML>
__global__ __launch_bounds__(kT) void k_gram_f(Dims d, const cx<R>* __restrict__ X, const R* __restrict__ W,
                                               const R* __restrict__ H, const R* __restrict__ g,
                                               R* __restrict__ Vpart) {
  constexpr int ML2 = ML * ML;
  constexpr int JT = (ML2 + 15) / 16;
  typedef typename Mma<R>::v4 v4;
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int L = d.L, M = d.M, T = d.T, SLP = d.SLP;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, T - t0);
  const int ntp = (nt + 3) & ~3;
  extern __shared__ __align__(16) unsigned char smem[];
  R* sW = reinterpret_cast<R*>(smem);
  R* sg = sW + N * K;
  R* sInv = sg + N * M;  // [SLP][M]
  cx<R>* sX = reinterpret_cast<cx<R>*>(smem + align_up(sizeof(R) * (N * K + N * M + SLP * M), 16));  // [SLP][M]

  for (int i = tid; i < N * K; i += kT) sW[i] = W[((size_t)(i / K) * d.F + f) * K + i % K];
  for (int i = tid; i < N * M; i += kT) sg[i] = g[(size_t)f * N * M + i];
  const cx<R>* xf = X + ((size_t)f * T + t0) * M;
  for (int i = tid; i < ntp * M; i += kT) sX[i] = i < nt * M ? xf[i] : cx<R>{(R)0, (R)0};
  __syncthreads();

  for (int tl = tid; tl < ntp; tl += kT) {
    if (tl < nt) {
      const int t = t0 + tl;
      R lam[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        R acc = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) acc += sW[n * K + k] * H[(size_t)(n * K + k) * T + t];
        lam[n] = acc;
      }
      for (int m = 0; m < M; ++m) {
        R y = 0;
#pragma unroll
        for (int n = 0; n < N; ++n) y += lam[n] * sg[n * M + m];
        sInv[tl * M + m] = (R)1 / rmax(y, (R)d.eps);
      }
    } else {
      for (int m = 0; m < M; ++m) sInv[tl * M + m] = 0;
    }
  }
  __syncthreads();

  // C[mu][j] += sum over 4 frames of (1/y)[frame][mu] * O[frame][j], with O the packed x x^H.
  const int col = lane & 15, kk = lane >> 4;
  for (int item = wave; item < L * JT; item += kT / 64) {
    const int l = item / JT, jt = item - l * JT;
    const int o = l * ML;
    const int j = jt * 16 + col;
    const bool jv = j < ML2;
    int a = 0, b = 0, part = 0;
    if (jv) pair_of<ML>(j, a, b, part);
    const bool rv = col < ML;
    v4 acc = {0, 0, 0, 0};
    for (int step = 0; step < ntp; step += 4) {
      const int tl = step + kk;
      const R av = rv ? sInv[tl * M + o + col] : (R)0;
      R bv = 0;
      if (jv) {
        const cx<R> xa = sX[tl * M + o + a], xb = sX[tl * M + o + b];
        bv = part == 0 ? xa.re * xb.re + xa.im * xb.im : xa.im * xb.re - xa.re * xb.im;
      }
      acc = Mma<R>::run(av, bv, acc);
    }
    R* out = Vpart + ((size_t)f * d.S + s) * d.VF + (size_t)l * ML * ML2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mu = Mma<R>::row(lane, r);
      if (mu < ML && jv) out[mu * ML2 + j] = acc[r];
    }
  }

}

// IP sweep, eqs. (15)-(16), one lane per (f, subarray) block of size M_l <= 4, in FP64
// registers; then ln|det Q_fl| for the cost (13).
template <typename R, int ML>
__global__ __launch_bounds__(64) void k_ip_f(Dims d, const R* __restrict__ Vpart, cx<R>* __restrict__ Q,
                                             double* __restrict__ logdet, int* __restrict__ status) {
  constexpr int ML2 = ML * ML;
  const int idx = blockIdx.x * 64 + threadIdx.x;
  if (idx >= d.F * d.L) return;
  const int f = idx / d.L, l = idx - f * d.L;
  cx<R>* qb = Q + (size_t)f * d.QF + l * ML2;
  cd Qm[ML][ML];
#pragma unroll
  for (int r = 0; r < ML; ++r)
#pragma unroll
    for (int c = 0; c < ML; ++c) Qm[r][c] = {(double)qb[r * ML + c].re, (double)qb[r * ML + c].im};
  ip_sweep_lane<R, ML>(Vpart + (size_t)f * d.S * d.VF + (size_t)l * ML * ML2, d.VF, d.S, 1.0 / d.T, Qm, d.eps,
                       status);
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
// P = |Q x|^2 and the eq. (8) sums; the last slice of a frequency updates W.
template <typename R, int N, int K, int ML>
__global__ __launch_bounds__(kT) void k_pw_f(Dims d, const cx<R>* __restrict__ X, const cx<R>* __restrict__ Q,
                                             R* __restrict__ W, const R* __restrict__ H, const R* __restrict__ g,
                                             R* __restrict__ P, R* __restrict__ Wpart,
                                             unsigned* __restrict__ counters, int* __restrict__ status) {
  constexpr int ML2 = ML * ML;
  constexpr int NK = N * K;
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int L = d.L, M = d.M, T = d.T, SLP = d.SLP;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, T - t0);
  const int ntp = (nt + 3) & ~3;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<R>* sQ = reinterpret_cast<cx<R>*>(smem);
  R* sW = reinterpret_cast<R*>(smem + align_up(sizeof(cx<R>) * d.QF, 16));
  R* sg = sW + NK;
  R* sH = sg + N * M;      // [NK][SLP]
  R* sab = sH + NK * SLP;  // [2N][SLP]
  __shared__ int s_flag;

  for (int i = tid; i < d.QF; i += kT) sQ[i] = Q[(size_t)f * d.QF + i];
  for (int i = tid; i < NK; i += kT) sW[i] = W[((size_t)(i / K) * d.F + f) * K + i % K];
  for (int i = tid; i < N * M; i += kT) sg[i] = g[(size_t)f * N * M + i];
  __syncthreads();

  for (int tl = tid; tl < ntp; tl += kT) {
    if (tl < nt) {
      const int t = t0 + tl;
      R lam[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        R acc = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const R h = H[(size_t)(n * K + k) * T + t];
          sH[(n * K + k) * SLP + tl] = h;
          acc += sW[n * K + k] * h;
        }
        lam[n] = acc;
      }
      R a[N], b[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        a[n] = 0;
        b[n] = 0;
      }
      const cx<R>* xr = X + ((size_t)f * T + t) * M;
      R* pr = P + ((size_t)f * T + t) * M;
      for (int l = 0; l < L; ++l) {
        cx<R> x[ML];
#pragma unroll
        for (int c = 0; c < ML; ++c) x[c] = xr[l * ML + c];
        const cx<R>* qb = sQ + l * ML2;
#pragma unroll
        for (int mu = 0; mu < ML; ++mu) {
          R zr = 0, zi = 0;
#pragma unroll
          for (int c = 0; c < ML; ++c) {
            const cx<R> q = qb[mu * ML + c];
            zr += q.re * x[c].re - q.im * x[c].im;
            zi += q.re * x[c].im + q.im * x[c].re;
          }
          const R p = zr * zr + zi * zi;
          const int m = l * ML + mu;
          pr[m] = p;
          R y = 0;
#pragma unroll
          for (int n = 0; n < N; ++n) y += lam[n] * sg[n * M + m];
          const R iy = (R)1 / rmax(y, (R)d.eps);
          const R piy2 = p * iy * iy;
#pragma unroll
          for (int n = 0; n < N; ++n) {
            a[n] += sg[n * M + m] * piy2;
            b[n] += sg[n * M + m] * iy;
          }
        }
      }
#pragma unroll
      for (int n = 0; n < N; ++n) {
        sab[n * SLP + tl] = a[n];
        sab[(N + n) * SLP + tl] = b[n];
      }
    } else {
      for (int i = 0; i < NK; ++i) sH[i * SLP + tl] = 0;
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
    R num = 0, den = 0;
    for (int tl = 0; tl < ntp; tl += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        num += hr[tl + u] * ar[tl + u];
        den += hr[tl + u] * br[tl + u];
      }
    }
    out[o * 2 + 0] = num;
    out[o * 2 + 1] = den;
  }

  if (!last_arrival(&counters[f], (unsigned)d.S, &s_flag)) return;
  for (int o = tid; o < NK; o += kT) {
    R num = 0, den = 0;
    for (int q = 0; q < d.S; ++q) {
      const R* pp = Wpart + ((size_t)f * d.S + q) * NK * 2 + o * 2;
      num += pp[0];
      den += pp[1];
    }
    R* wp = W + ((size_t)(o / K) * d.F + f) * K + o % K;
    const R v = *wp * sqrt(num / rmax(den, (R)d.eps));
    if (!isfinite(v)) atomicOr(status, kStNonFinite);
    *wp = v;
  }
  if (tid == 0) atomicExch(&counters[f], 0u);
}

// ------------------------------------------------------------------------------------
// Activation update, eq. (9).  Workgroup = HW waves; wave w owns 16 bins, all waves share
// one block of 16 frames.  W is read by the matrix-core operand loads straight from L2.
template <typename R>
constexpr int h_waves() { return sizeof(R) == 4 ? 4 : 2; }

template <typename R, int N, int K, int ML>
__global__ __launch_bounds__(64 * h_waves<R>()) void k_h_f(Dims d, const R* __restrict__ W, R* __restrict__ H,
                                                           const R* __restrict__ g, const R* __restrict__ P,
                                                           R* __restrict__ Hpart, unsigned* __restrict__ counters,
                                                           int* __restrict__ status) {
  constexpr int HW = h_waves<R>();
  constexpr int NT = 64 * HW;
  constexpr int NK = N * K;
  constexpr int KS = (K + 3) / 4;    // 4-deep steps over bases for lambda = W H
  constexpr int KT = (K + 15) / 16;  // 16-row tiles of bases for the sum over frequencies
  typedef typename Mma<R>::v4 v4;
  const int fg = blockIdx.x, tb = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int M = d.M, T = d.T, F = d.F, L = d.L;
  const int t0 = tb * kHTB;
  const int ntb = min(kHTB, T - t0);
  const int f0 = (fg * HW + wave) * 16;
  const int nf = max(0, min(16, F - f0));
  extern __shared__ __align__(16) unsigned char smem[];
  R* sHt = reinterpret_cast<R*>(smem);                           // [NK][16]
  R* sgc = sHt + NK * kHTB + wave * (16 * N * M);                // per wave [16 f][N*M]
  R* sAB = sHt + NK * kHTB + HW * 16 * N * M + wave * (2 * 256); // per wave [2][16 f][16 t]
  __shared__ int s_flag;

  for (int i = tid; i < NK * kHTB; i += NT) {
    const int nk = i / kHTB, tl = i % kHTB;
    sHt[i] = tl < ntb ? H[(size_t)nk * T + t0 + tl] : (R)0;
  }
  for (int i = lane; i < 16 * N * M; i += 64) {
    const int fl = i / (N * M);
    sgc[i] = fl < nf ? g[(size_t)(f0 + fl) * N * M + i % (N * M)] : (R)0;
  }
  __syncthreads();

  const int cl = lane & 15, ck = lane >> 4;
  const bool frow = cl < nf;  // this lane's A-operand row (bin f0 + cl) exists
  // lambda_n[f][t] = sum_k W[n][f][k] H[n][k][t]: A = W (rows f), B = H (columns t).
  R lam[N][4];
#pragma unroll
  for (int n = 0; n < N; ++n) {
    v4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      const int k = 4 * st + ck;
      const R av = (k < K && frow) ? W[((size_t)n * F + f0 + cl) * K + k] : (R)0;
      const R bv = k < K ? sHt[(n * K + k) * kHTB + cl] : (R)0;
      acc = Mma<R>::run(av, bv, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) lam[n][r] = acc[r];
  }
  // a' and b' of eq. (9) for the four (f, t) pairs this lane holds.
  R a[N][4], b[N][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int fl = Mma<R>::row(lane, r), tl = cl;
#pragma unroll
    for (int n = 0; n < N; ++n) {
      a[n][r] = 0;
      b[n][r] = 0;
    }
    if (fl < nf && tl < ntb) {
      const R* pr = P + ((size_t)(f0 + fl) * T + t0 + tl) * M;
      const R* gf = sgc + fl * N * M;
      for (int l = 0; l < L; ++l) {
#pragma unroll
        for (int mu = 0; mu < ML; ++mu) {
          const int m = l * ML + mu;
          R y = 0;
#pragma unroll
          for (int n = 0; n < N; ++n) y += lam[n][r] * gf[n * M + m];
          const R iy = (R)1 / rmax(y, (R)d.eps);
          const R piy2 = pr[m] * iy * iy;
#pragma unroll
          for (int n = 0; n < N; ++n) {
            a[n][r] += gf[n * M + m] * piy2;
            b[n][r] += gf[n * M + m] * iy;
          }
        }
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
      const int k = kt * 16 + cl;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int fl = 4 * st + ck;
        const R av = (k < K && fl < nf) ? W[((size_t)n * F + f0 + fl) * K + k] : (R)0;
        accN[n][kt] = Mma<R>::run(av, sAB[fl * 16 + cl], accN[n][kt]);
        accD[n][kt] = Mma<R>::run(av, sAB[256 + fl * 16 + cl], accD[n][kt]);
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

  if (!last_arrival(&counters[tb], (unsigned)d.FG, &s_flag)) return;
  for (int i = tid; i < NK * ntb; i += NT) {
    const int tl = i % ntb, nk = i / ntb;
    R num = 0, den = 0;
    for (int q = 0; q < d.FG; ++q) {
      const R* pp = Hpart + (((size_t)q * NK + nk) * T + t0 + tl) * 2;
      num += pp[0];
      den += pp[1];
    }
    R* hp = H + (size_t)nk * T + t0 + tl;
    const R v = *hp * sqrt(num / rmax(den, (R)d.eps));
    if (!isfinite(v)) atomicOr(status, kStNonFinite);
    *hp = v;
  }
  if (tid == 0) atomicExch(&counters[tb], 0u);
}

// ------------------------------------------------------------------------------------
// Eq. (10) sums per (f, slice); the last slice of a frequency updates g.
template <typename R, int N, int K, int ML>
__global__ __launch_bounds__(kT) void k_g_f(Dims d, const R* __restrict__ W, const R* __restrict__ H,
                                            R* __restrict__ g, const R* __restrict__ P, R* __restrict__ gpart,
                                            unsigned* __restrict__ counters, int* __restrict__ status) {
  constexpr int NK = N * K;
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int L = d.L, M = d.M, T = d.T, SLP = d.SLP;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, T - t0);
  const int ntp = (nt + 3) & ~3;
  extern __shared__ __align__(16) unsigned char smem[];
  R* sW = reinterpret_cast<R*>(smem);
  R* sg = sW + NK;
  R* sLam = sg + N * M;     // [N][SLP]
  R* sR = sLam + N * SLP;   // [2M][SLP]
  __shared__ int s_flag;

  for (int i = tid; i < NK; i += kT) sW[i] = W[((size_t)(i / K) * d.F + f) * K + i % K];
  for (int i = tid; i < N * M; i += kT) sg[i] = g[(size_t)f * N * M + i];
  __syncthreads();

  for (int tl = tid; tl < ntp; tl += kT) {
    if (tl < nt) {
      const int t = t0 + tl;
      R lam[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        R acc = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) acc += sW[n * K + k] * H[(size_t)(n * K + k) * T + t];
        lam[n] = acc;
        sLam[n * SLP + tl] = acc;
      }
      const R* pr = P + ((size_t)f * T + t) * M;
      for (int l = 0; l < L; ++l) {
#pragma unroll
        for (int mu = 0; mu < ML; ++mu) {
          const int m = l * ML + mu;
          R y = 0;
#pragma unroll
          for (int n = 0; n < N; ++n) y += lam[n] * sg[n * M + m];
          const R iy = (R)1 / rmax(y, (R)d.eps);
          sR[m * SLP + tl] = pr[m] * iy * iy;
          sR[(M + m) * SLP + tl] = iy;
        }
      }
    } else {
      for (int n = 0; n < N; ++n) sLam[n * SLP + tl] = 0;
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
    R num = 0, den = 0;
    for (int tl = 0; tl < ntp; tl += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        num += lr[tl + u] * r1[tl + u];
        den += lr[tl + u] * r2[tl + u];
      }
    }
    out[o * 2 + 0] = num;
    out[o * 2 + 1] = den;
  }

  if (!last_arrival(&counters[f], (unsigned)d.S, &s_flag)) return;
  for (int o = tid; o < N * M; o += kT) {
    R num = 0, den = 0;
    for (int q = 0; q < d.S; ++q) {
      const R* pp = gpart + ((size_t)f * d.S + q) * N * M * 2 + o * 2;
      num += pp[0];
      den += pp[1];
    }
    R* gp = g + (size_t)f * N * M + o;
    const R v = *gp * sqrt(num / rmax(den, (R)d.eps));
    if (!isfinite(v)) atomicOr(status, kStNonFinite);
    *gp = v;
  }
  if (tid == 0) atomicExch(&counters[f], 0u);
}

// ------------------------------------------------------------------------------------
// LDS budgets (bytes) of each kernel for a given slice stride.
template <typename R, int N, int K, int ML>
struct Set {
  static size_t smem_gram(const Dims& d) {
    return align_up(sizeof(R) * (N * K + N * d.M + d.SLP * d.M), 16) + sizeof(cx<R>) * d.SLP * d.M;
  }
  static size_t smem_pw(const Dims& d) {
    return align_up(sizeof(cx<R>) * d.QF, 16) + sizeof(R) * (N * K + N * d.M + N * K * d.SLP + 2 * N * d.SLP);
  }
  static size_t smem_h(const Dims& d) {
    constexpr int KT = (K + 15) / 16;
    constexpr int HW = h_waves<R>();
    const size_t stage = sizeof(R) * (N * K * kHTB + HW * 16 * N * d.M + HW * 2 * 256);
    const size_t red = sizeof(R) * N * KT * 16 * 16 * 2;
    return stage > red ? stage : red;
  }
  static size_t smem_g(const Dims& d) { return sizeof(R) * (N * K + N * d.M + N * d.SLP + 2 * d.M * d.SLP); }
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
    unsigned* cnt = b.counters;
    switch (kid) {
      case kFGram:
        hipLaunchKernelGGL((k_gram_f<R, N, K, ML>), dim3(d.F, d.S), dim3(kT), smem_gram(d), s, d, X, W, H, g,
                           static_cast<R*>(b.Vpart));
        break;
      case kFIp:
        if constexpr (ML <= 4) {
          hipLaunchKernelGGL((k_ip_f<R, ML>), dim3((d.F * d.L + 63) / 64), dim3(64), 0, s, d,
                             static_cast<const R*>(b.Vpart), Q, b.logdet, b.status);
        } else {
          return launch_kernel(d, b, sizeof(R) == 4 ? DFM_C64 : DFM_C128, kKIp, s);
        }
        break;
      case kFPw:
        hipLaunchKernelGGL((k_pw_f<R, N, K, ML>), dim3(d.F, d.S), dim3(kT), smem_pw(d), s, d, X, Q, W, H, g, P,
                           static_cast<R*>(b.Wpart), cnt + d.F, b.status);
        break;
      case kFH:
        hipLaunchKernelGGL((k_h_f<R, N, K, ML>), dim3(d.FG, d.TBN), dim3(64 * h_waves<R>()), smem_h(d), s, d, W, H, g, P,
                           static_cast<R*>(b.Hpart), cnt + 2 * d.F, b.status);
        break;
      case kFG:
        hipLaunchKernelGGL((k_g_f<R, N, K, ML>), dim3(d.F, d.S), dim3(kT), smem_g(d), s, d, W, H, g, P,
                           static_cast<R*>(b.gpart), cnt + 2 * d.F + d.TBN, b.status);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
};

}  // namespace fast

// Compiled shape sets (N, K, M_l); index = Dims::fast.
#define DFM_FAST_SETS(X) X(0, 2, 4, 2) X(1, 5, 16, 4) X(2, 5, 16, 16) X(3, 3, 16, 4) X(4, 8, 16, 4)

int fast_set_index(int N, int K, int ML) {
#define DFM_MATCH(i, n, k, ml) \
  if (N == n && K == k && ML == ml) return i;
  DFM_FAST_SETS(DFM_MATCH)
#undef DFM_MATCH
  return -1;
}

int fast_h_waves(int dtype) { return dtype == DFM_C64 ? fast::h_waves<float>() : fast::h_waves<double>(); }

size_t fast_max_smem(const Dims& d, int dtype) {
  switch (d.fast) {
#define DFM_SMEM(i, n, k, ml)                                                                      \
  case i:                                                                                          \
    return dtype == DFM_C64 ? fast::Set<float, n, k, ml>::max_smem(d) : fast::Set<double, n, k, ml>::max_smem(d);
    DFM_FAST_SETS(DFM_SMEM)
#undef DFM_SMEM
  }
  return 0;
}

hipError_t fast_launch(const Dims& d, const Buffers& b, int dtype, int kid, hipStream_t s) {
  switch (d.fast) {
#define DFM_LAUNCH(i, n, k, ml)                                                                   \
  case i:                                                                                         \
    return dtype == DFM_C64 ? fast::Set<float, n, k, ml>::launch(d, b, kid, s)                    \
                            : fast::Set<double, n, k, ml>::launch(d, b, kid, s);
    DFM_FAST_SETS(DFM_LAUNCH)
#undef DFM_LAUNCH
  }
  return hipErrorInvalidValue;
}

}  // namespace dfm
