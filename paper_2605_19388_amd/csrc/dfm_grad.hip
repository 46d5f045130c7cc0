// Gradient of the cost (13) after n unrolled iterations with respect to the state the iterations
// started from: reverse-mode, hand-written, in FP64 whatever the plan's precision, with the Sec.
// IV-A floors in place.  Two maps: MM iterations (eqs. (8), (9), (10) in that order, Q held fixed)
// and full iterations (eq. (14) and the IP sweep of eqs. (15)-(16), then (8)-(10)).
//
// The forward iterations run on the plan's own kernels and store the state (g, W, H; and Q for
// full iterations) before each iteration in the caller's tape (per-iteration checkpoints).  The reverse pass then starts from
// the cost's gradient at the final state and walks the iterations backwards; for each it
// recomputes, from that iteration's checkpoint, the intermediate sums of (8)-(10) and goes back
// through the g, H and W updates in turn.  With theta' = theta sqrt(a / max(b, eps)) (a, b the
// numerator and denominator sums of the update) and theta'bar the adjoint of the updated value:
//   abar = theta'bar theta' / (2 a),  bbar = -theta'bar theta' / (2 max(b, eps)) [b > eps],
//   thetabar (direct) = theta'bar sqrt(a / max(b, eps)),
// and the sums carry abar, bbar back to the per-frame quantities: y (through P / y^2 and 1 / y;
// y = max(u, eps), u = sum_n lambda g, has zero derivative where floored), P, lambda = W H and g.
// For MM iterations the adjoint of P accumulates over all iterations (Q is fixed, so P is one
// quantity), and the gradient with respect to Q comes last:
//   dL/dRe Q + i dL/dIm Q = 2 sum_t Pbar z conj(x) - 2T Q^-H  (per block, z = Q x).
//
// Kernels (one workgroup per bin where a bin's frames are reduced, so every sum has a fixed
// order and the result is reproducible):
//   kb_powers  P = |Q x|^2 in FP64;
//   kb_coef    c = sum_m g P / y^2, d = sum_m g / y per (f, t, n) (the W and H sums' planes);
//   kb_sum_t   out[n][f][k] (+)= sum_t A1[n][k][t] C1[f][t][n] + A2 C2;
//   kb_sum_f   out[n][k][t] (+)= sum_f A1[n][f][k] C1[f][t][n] + A2 C2;
//   kb_cbar    out[f][t][n] = sum_k A1[n][f][k] B1[n][k][t] (and a second pair);
//   kb_apply / kb_mmback  the update theta' and its adjoint split (elementwise);
//   kb_frame   per (bin, slice of frames): the per-frame adjoints of one update (or of the cost),
//              Pbar += ..., lambdabar, and the slice's sums over frames for g's adjoint, which
//              kb_gsum adds in slice order;
//   kb_qgrad   the gradient with respect to Q.
//
// Full iterations.  Iteration i maps (Q_i, g_i, W_i, H_i) to Q_{i+1} = IP(Q_i, V(y_i)), then runs
// the MM updates against P_{i+1} = |Q_{i+1} x|^2.  Going back through iteration i: the MM part as
// above, with the adjoint of P_{i+1} gathered afresh; Qbar_{i+1} += 2 sum_t Pbar z conj(x); then
// the sweep in reverse row order; then the covariances back to y_i and on to (g_i, W_i, H_i).  For
// one row (A = Q V_mu with the rows before mu already updated, b = A^-1 e_mu, s = b^H V_mu b,
// c = max(s, eps)^-1/2, row mu <- conj(c b)), with bhbar = conj(row mu of Qbar):
//   cbar = Re(bhbar^H b),  sbar = -cbar c^3 / 2 [s > eps],  bbar = c bhbar + 2 sbar V_mu b,
//   gamma = A^-H bbar,  Qbar <- Qbar (row mu zeroed) - gamma (V_mu b)^H,
//   Vbar_mu = sbar b b^H - (Q^H gamma) b^H,
// and from V_mu = (1/T) sum_t x x^H / y_mu:  ybar_mu(t) = -Re(x^H Vbar_mu x) / (T y_mu^2).
// Kernels: kb_y (u = sum_n lambda g), kb_cov (V by eq. (14)), kb_ipfwd (the sweep, kept for
// P_{i+1}), kb_ipbwd (the sweep's adjoint; both one thread per block, in registers for blocks of
// up to 4 mics: kb_ipfwd4, kb_ipbwd4), kb_vbar (ybar), and kb_frame's kBackY mode (ybar on to g,
// lambda).
#include <hip/hip_runtime.h>

#include "dfm_device.h"

namespace dfm {
namespace grad {

constexpr int kB = 256;

__device__ __forceinline__ double dsqrt_ratio(double a, double b, double eps) { return sqrt(a / (b > eps ? b : eps)); }

// P[f][t][m] = |(Q x)_m|^2 in FP64; one thread per (t, m) of bin f (grid (F, T M / kB)), so that
// the threads of one frame share its x and write P coalesced.
template <typename R, typename RQ>
__global__ __launch_bounds__(kB) void kb_powers(Dims d, const cx<R>* __restrict__ X, const cx<RQ>* __restrict__ Q,
                                                double* __restrict__ P) {
  const int f = blockIdx.x, i = blockIdx.y * kB + threadIdx.x;
  if (i >= d.T * d.M) return;
  const int t = i / d.M, m = i - t * d.M, l = d.msub[m], ml = d.mics[l], o = d.moff[l], mu = m - o;
  const cx<R>* x = X + ((size_t)f * d.T + t) * d.M + o;
  const cx<RQ>* q = Q + (size_t)f * d.QF + d.qoff[l] + mu * ml;
  double zr = 0.0, zi = 0.0;
  for (int c = 0; c < ml; ++c) {
    const double qr = q[c].re, qi = q[c].im, xr = x[c].re, xi = x[c].im;
    zr += qr * xr - qi * xi;
    zi += qr * xi + qi * xr;
  }
  P[((size_t)f * d.T + t) * d.M + m] = zr * zr + zi * zi;
}

// lambda_n at (f, t) from W (row of bin f staged in sW [N][K]) and H [N][K][T].
template <typename RH>
__device__ __forceinline__ double lam_at(const Dims& d, const double* sW, const RH* __restrict__ H, int n, int t) {
  double acc = 0.0;
  const RH* hn = H + (size_t)n * d.K * d.T + t;
  for (int k = 0; k < d.K; ++k) acc += sW[n * d.K + k] * (double)hn[(size_t)k * d.T];
  return acc;
}

template <typename RW, typename RG>
__device__ __forceinline__ void stage_bin(const Dims& d, const RW* __restrict__ W, const RG* __restrict__ g, int f,
                                          double* sW, double* sg) {
  for (int i = threadIdx.x; i < d.N * d.K; i += blockDim.x) {
    const int n = i / d.K, k = i - n * d.K;
    sW[i] = (double)W[((size_t)n * d.F + f) * d.K + k];
  }
  for (int i = threadIdx.x; i < d.N * d.M; i += blockDim.x) sg[i] = (double)g[(size_t)f * d.N * d.M + i];
}

// c[f][t][n] = sum_m g P / y^2, d[f][t][n] = sum_m g / y for the state (W, H, g); grid (F, T / kB).
template <typename RW, typename RH, typename RG>
__global__ __launch_bounds__(kB) void kb_coef(Dims d, const RW* __restrict__ W, const RH* __restrict__ H,
                                              const RG* __restrict__ g, const double* __restrict__ P,
                                              double* __restrict__ c, double* __restrict__ dd) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* sW = reinterpret_cast<double*>(smem);
  double* sg = sW + d.N * d.K;
  const int f = blockIdx.x, t = blockIdx.y * kB + threadIdx.x;
  stage_bin(d, W, g, f, sW, sg);
  __syncthreads();
  if (t >= d.T) return;
  double lam[kMaxN];
  for (int n = 0; n < d.N; ++n) lam[n] = lam_at(d, sW, H, n, t);
  double cn[kMaxN], dn[kMaxN];
  for (int n = 0; n < d.N; ++n) cn[n] = dn[n] = 0.0;
  const double* p = P + ((size_t)f * d.T + t) * d.M;
  for (int m = 0; m < d.M; ++m) {
    double u = 0.0;
    for (int n = 0; n < d.N; ++n) u += lam[n] * sg[n * d.M + m];
    const double y = u > d.eps ? u : d.eps, iy = 1.0 / y, w = p[m] * iy * iy;
    for (int n = 0; n < d.N; ++n) {
      cn[n] += sg[n * d.M + m] * w;
      dn[n] += sg[n * d.M + m] * iy;
    }
  }
  for (int n = 0; n < d.N; ++n) {
    c[((size_t)f * d.T + t) * d.N + n] = cn[n];
    dd[((size_t)f * d.T + t) * d.N + n] = dn[n];
  }
}

__device__ __forceinline__ double wave_sum(double v) {  // butterfly: every lane gets the sum, same order
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// out[n][f][k] (+)= sum_t A1[n][k][t] C1[f][t][n] + A2[n][k][t] C2[f][t][n]; A of type RA.  One
// workgroup per (n, f), one wave per k, lanes over frames (coalesced rows of A), a butterfly sum.
template <typename RA>
__global__ __launch_bounds__(kB) void kb_sum_t(Dims d, const RA* __restrict__ A1, const double* __restrict__ C1,
                                               const RA* __restrict__ A2, const double* __restrict__ C2,
                                               double* __restrict__ out, int accumulate) {
  const int n = blockIdx.x / d.F, f = blockIdx.x - n * d.F, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* c1 = C1 + (size_t)f * d.T * d.N + n;
  const double* c2 = C2 ? C2 + (size_t)f * d.T * d.N + n : nullptr;
  for (int k = w; k < d.K; k += kB / 64) {
    const RA* a1 = A1 + ((size_t)n * d.K + k) * d.T;
    const RA* a2 = A2 ? A2 + ((size_t)n * d.K + k) * d.T : nullptr;
    double acc = 0.0;
    for (int t = lane; t < d.T; t += 64) {
      acc += (double)a1[t] * c1[(size_t)t * d.N];
      if (a2) acc += (double)a2[t] * c2[(size_t)t * d.N];
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      double& o = out[((size_t)n * d.F + f) * d.K + k];
      o = accumulate ? o + acc : acc;
    }
  }
}

// out[n][k][t] (+)= sum_f A1[n][f][k] C1[f][t][n] + A2[n][f][k] C2[f][t][n].  Grid (N K, T / 64):
// lanes over frames, the four waves over interleaved bins, their partials added in wave order.
template <typename RA>
__global__ __launch_bounds__(kB) void kb_sum_f(Dims d, const RA* __restrict__ A1, const double* __restrict__ C1,
                                               const RA* __restrict__ A2, const double* __restrict__ C2,
                                               double* __restrict__ out, int accumulate) {
  __shared__ double part[kB];
  const int n = blockIdx.x / d.K, k = blockIdx.x - n * d.K, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t = blockIdx.y * 64 + lane;
  double acc = 0.0;
  if (t < d.T)
    for (int f = w; f < d.F; f += kB / 64) {
      const size_t ai = ((size_t)n * d.F + f) * d.K + k, ci = ((size_t)f * d.T + t) * d.N + n;
      acc += (double)A1[ai] * C1[ci];
      if (A2) acc += (double)A2[ai] * C2[ci];
    }
  part[threadIdx.x] = acc;
  __syncthreads();
  if (w == 0 && t < d.T) {
    double s = part[lane];
    for (int j = 1; j < kB / 64; ++j) s += part[j * 64 + lane];
    double& o = out[((size_t)n * d.K + k) * d.T + t];
    o = accumulate ? o + s : s;
  }
}

// out[f][t][n] = sum_k A[n][f][k] B[n][k][t] for (A1, B1) -> out1 and (A2, B2) -> out2; threads
// ordered (f, n, t) so that rows of B are read coalesced.
template <typename RA, typename RB>
__global__ __launch_bounds__(kB) void kb_cbar(Dims d, const RA* __restrict__ A1, const RB* __restrict__ B1,
                                              const RA* __restrict__ A2, const RB* __restrict__ B2,
                                              double* __restrict__ out1, double* __restrict__ out2) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= d.F * d.T * d.N) return;
  const int f = i / (d.N * d.T), r = i - f * d.N * d.T, n = r / d.T, t = r - n * d.T;
  double s1 = 0.0, s2 = 0.0;
  for (int k = 0; k < d.K; ++k) {
    const size_t ai = ((size_t)n * d.F + f) * d.K + k, bi = ((size_t)n * d.K + k) * d.T + t;
    s1 += (double)A1[ai] * (double)B1[bi];
    s2 += (double)A2[ai] * (double)B2[bi];
  }
  const size_t o = ((size_t)f * d.T + t) * d.N + n;
  out1[o] = s1;
  out2[o] = s2;
}

// theta1 = theta sqrt(a / max(b, eps)).
template <typename R>
__global__ __launch_bounds__(kB) void kb_apply(int n, const R* __restrict__ th, const double* __restrict__ a,
                                               const double* __restrict__ b, double eps, double* __restrict__ th1) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i < n) th1[i] = (double)th[i] * dsqrt_ratio(a[i], b[i], eps);
}

// Adjoint of theta1 = theta sqrt(a / max(b, eps)) with theta1bar in acc: abar, bbar, and
// acc <- the direct part of thetabar.
template <typename R>
__global__ __launch_bounds__(kB) void kb_mmback(int n, const R* __restrict__ th, const double* __restrict__ a,
                                                const double* __restrict__ b, double eps, double* __restrict__ acc,
                                                double* __restrict__ abar, double* __restrict__ bbar) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const double bb = b[i] > eps ? b[i] : eps, r = sqrt(a[i] / bb), t1 = (double)th[i] * r, tb = acc[i];
  abar[i] = a[i] > 0.0 ? tb * t1 / (2.0 * a[i]) : 0.0;
  bbar[i] = b[i] > eps ? -tb * t1 / (2.0 * bb) : 0.0;
  acc[i] = tb * r;
}

// Modes of kb_frame.
enum { kCost = 0, kFwdG = 1, kBackG = 2, kBackWH = 3, kBackY = 4 };

// One workgroup per (bin, slice of CH frames) (grid (F, ceil(T / CH))): phase 1 one thread per
// frame (per-frame adjoints, Pbar, lambdabar; the terms that sum over frames go to LDS), phase 2
// one thread per (n, m) adding the slice's terms in frame order into part[f][slice][2][N][M];
// kb_gsum then adds the slices in order into gout (and gout2).
//   kCost:   L's own gradient: ybar = 1/y - P/y^2, Pbar = 1/y (written), lambdabar, gout = g's.
//   kFwdG:   the sums of eq. (10): gout = sum_t lambda P / y^2, gout2 = sum_t lambda / y.
//   kBackG:  coefficients abar, bbar [F][N][M] of eq. (10): ybar, Pbar +=, lambdabar, gout +=.
//   kBackWH: coefficients cbar, dbar [F][T][N] of eq. (8) or (9): ybar, Pbar +=, lambdabar, gout +=.
//   kBackY:  ybar [F][T][M] given in c1 (from the covariances): lambdabar, gout +=; P, Pbar unused.
template <typename RW, typename RH, typename RG, int MODE, int NX>
__global__ __launch_bounds__(kB) void kb_frame(Dims d, const RW* __restrict__ W, const RH* __restrict__ H,
                                               const RG* __restrict__ g, const double* __restrict__ P,
                                               const double* __restrict__ c1, const double* __restrict__ c2,
                                               double* __restrict__ Pbar, double* __restrict__ lbar,
                                               double* __restrict__ part, int CH) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = d.N, M = d.M, f = blockIdx.x, tid = threadIdx.x;
  double* sW = reinterpret_cast<double*>(smem);  // [N][K]
  double* sg = sW + N * d.K;                      // [N][M]
  double* sa = sg + N * M;                        // kBackG: abar [N][M]
  double* sb = sa + N * M;                        // kBackG: bbar [N][M]
  double* sl = sb + N * M;                        // [CH][N]: lambda
  double* su = sl + CH * N;                       // [CH][M]: ubar (floored y: 0)
  double* sy = su + CH * M;                       // [CH][M]: 1 / y
  double* sp = sy + CH * M;                       // [CH][M]: P / y^2
  double* sc = sp + CH * M;                       // [CH][N]: cbar (kBackWH)
  double* sd = sc + CH * N;                       // [CH][N]: dbar (kBackWH)
  for (int i = tid; i < N * d.K; i += kB) {
    const int n = i / d.K, k = i - n * d.K;
    sW[i] = (double)W[((size_t)n * d.F + f) * d.K + k];
  }
  for (int i = tid; i < N * M; i += kB) {
    sg[i] = (double)g[(size_t)f * N * M + i];
    if (MODE == kBackG) {
      sa[i] = c1[(size_t)f * N * M + i];
      sb[i] = c2[(size_t)f * N * M + i];
    }
  }
  __shared__ double gpart2[2 * kB];  // phase 2: the thread groups' partial sums
  double acc1[4] = {0, 0, 0, 0}, acc2[4] = {0, 0, 0, 0};  // phase 2: this thread's (n, m) entries
  __syncthreads();
  {
    const int t0 = blockIdx.y * CH, nt = min(CH, d.T - t0);
    if (tid < nt) {
      const int t = t0 + tid;
      const size_t ft = (size_t)f * d.T + t;
      double lam[NX], lb[NX], cb[NX], db[NX];  // N <= NX
      for (int n = 0; n < N; ++n) {
        lam[n] = lam_at(d, sW, H, n, t);
        lb[n] = 0.0;
        if (MODE == kBackWH) {
          cb[n] = c1[ft * N + n];
          db[n] = c2[ft * N + n];
        }
      }
      for (int m = 0; m < M; ++m) {
        double u = 0.0;
        for (int n = 0; n < N; ++n) u += lam[n] * sg[n * M + m];
        const bool live = u > d.eps;
        const double y = live ? u : d.eps, iy = 1.0 / y, pm = MODE == kBackY ? 0.0 : P[ft * M + m],
                     py2 = pm * iy * iy;
        double ybar = 0.0, pbar = 0.0;
        if (MODE == kCost) {
          ybar = iy - py2;
          pbar = iy;
        } else if (MODE == kBackG) {
          for (int n = 0; n < N; ++n) {
            const double a = sa[n * M + m], b = sb[n * M + m];
            ybar += lam[n] * (a * (-2.0 * py2 * iy) - b * iy * iy);
            pbar += a * lam[n] * iy * iy;
            lb[n] += a * py2 + b * iy;
          }
        } else if (MODE == kBackWH) {
          for (int n = 0; n < N; ++n) {
            const double gg = sg[n * M + m];
            ybar += gg * (cb[n] * (-2.0 * py2 * iy) - db[n] * iy * iy);
            pbar += cb[n] * gg * iy * iy;
          }
        } else if (MODE == kBackY) {
          ybar = c1[ft * M + m];
        }
        const double ubar = live ? ybar : 0.0;
        if (MODE != kFwdG) {
          for (int n = 0; n < N; ++n) lb[n] += ubar * sg[n * M + m];
          if (MODE == kCost)
            Pbar[ft * M + m] = pbar;
          else if (MODE != kBackY)
            Pbar[ft * M + m] += pbar;
        }
        su[tid * M + m] = ubar;
        sy[tid * M + m] = iy;
        sp[tid * M + m] = py2;
      }
      for (int n = 0; n < N; ++n) {
        sl[tid * N + n] = lam[n];
        if (MODE == kBackWH) {
          sc[tid * N + n] = cb[n];
          sd[tid * N + n] = db[n];
        }
        if (MODE != kFwdG) lbar[ft * N + n] = lb[n];
      }
    }
    __syncthreads();
    // Phase 2: the slice's sum over frames of each (n, m) entry.  With N M <= kB the entries are
    // dealt to G = kB / (N M) thread groups, group q taking frames q, q + G, ..., and the groups'
    // partials are added in group order; otherwise one thread per entry (N M <= 4 kB).
    auto frame_sum = [&](int i, int j0, int js, double& s1, double& s2) {
      const int n = i / M, m = i - n * M;
#pragma unroll 2
      for (int j = j0; j < nt; j += js) {
        const double lam = sl[j * N + n];
        if (MODE == kFwdG) {
          s1 += lam * sp[j * M + m];
          s2 += lam * sy[j * M + m];
        } else if (MODE == kBackWH) {
          s1 += sc[j * N + n] * sp[j * M + m] + sd[j * N + n] * sy[j * M + m] + su[j * M + m] * lam;
        } else {
          s1 += su[j * M + m] * lam;
        }
      }
    };
    const int E = N * M;
    if (E <= kB) {
      const int G = kB / E, i = tid % E, q = tid / E;
      double s1 = 0.0, s2 = 0.0;
      if (q < G) frame_sum(i, q, G, s1, s2);
      gpart2[tid] = s1;
      gpart2[kB + tid] = s2;
      __syncthreads();
      if (q == 0) {
        for (int r = 1; r < G; ++r) {
          s1 += gpart2[r * E + i];
          s2 += gpart2[kB + r * E + i];
        }
        acc1[0] = s1;
        acc2[0] = s2;
      }
    } else {
      for (int e = 0; e < 4; ++e) {  // entries tid, tid + kB, ...
        const int i = tid + e * kB;
        if (i >= E) break;
        double s1 = 0.0, s2 = 0.0;
        frame_sum(i, 0, 1, s1, s2);
        acc1[e] = s1;
        acc2[e] = s2;
      }
    }
  }
  double* pf = part + ((size_t)f * gridDim.y + blockIdx.y) * 2 * N * M;
  for (int e = 0; e < 4; ++e) {
    const int i = tid + e * kB;
    if (i >= N * M) break;
    pf[i] = acc1[e];
    if (MODE == kFwdG) pf[N * M + i] = acc2[e];
  }
}

// The slices' partial sums of kb_frame, added in slice order: gout (and gout2 for kFwdG) written
// (kCost, kFwdG) or added to.
template <int MODE>
__global__ __launch_bounds__(kB) void kb_gsum(Dims d, int S, const double* __restrict__ part,
                                              double* __restrict__ gout, double* __restrict__ gout2) {
  const int i = blockIdx.x * kB + threadIdx.x, NM = d.N * d.M;
  if (i >= d.F * NM) return;
  const int f = i / NM, e = i - f * NM;
  const double* pf = part + (size_t)f * S * 2 * NM + e;
  double s1 = 0.0, s2 = 0.0;
  for (int s = 0; s < S; ++s) {
    s1 += pf[(size_t)s * 2 * NM];
    if (MODE == kFwdG) s2 += pf[(size_t)s * 2 * NM + NM];
  }
  if (MODE == kFwdG) {
    gout[i] = s1;
    gout2[i] = s2;
  } else if (MODE == kCost) {
    gout[i] = s1;
  } else {
    gout[i] += s1;
  }
}

// dL/dRe Q + i dL/dIm Q per (f, l) block: 2 sum_t Pbar z conj(x) - 2T Q^-H; Qinv from k_qinv, or
// null for the first term alone; written, or added to dQ (`accumulate`).  Grid (F, L): where the
// block's M_l^2 entries leave threads over, the frames are split into kB / M_l^2 interleaved
// slices whose partials are added in slice order.
template <typename R, typename RQ, typename RO>
__global__ __launch_bounds__(kB) void kb_qgrad(Dims d, const cx<R>* __restrict__ X, const cx<RQ>* __restrict__ Q,
                                               const cd* __restrict__ Qinv, const double* __restrict__ Pbar,
                                               cx<RO>* __restrict__ dQ, int accumulate) {
  __shared__ double part[2 * kB];
  const int f = blockIdx.x, l = blockIdx.y, tid = threadIdx.x;
  const int ml = d.mics[l], o = d.moff[l], q0 = d.qoff[l], E = ml * ml;
  const int S = E <= kB ? kB / E : 1;  // frame slices
  const cx<RQ>* qf = Q + (size_t)f * d.QF + q0;
  for (int i0 = 0; i0 < E; i0 += kB) {  // one pass unless M_l^2 > kB
    const int e = S > 1 ? tid % E : i0 + tid, sl = S > 1 ? tid / E : 0;
    double ar = 0.0, ai = 0.0;
    if (e < E && sl < S) {
      const int mu = e / ml, c = e - mu * ml;
      for (int t = sl; t < d.T; t += S) {
        const cx<R>* x = X + ((size_t)f * d.T + t) * d.M + o;
        double zr = 0.0, zi = 0.0;
        for (int b = 0; b < ml; ++b) {
          const double qr = qf[mu * ml + b].re, qi = qf[mu * ml + b].im, xr = x[b].re, xi = x[b].im;
          zr += qr * xr - qi * xi;
          zi += qr * xi + qi * xr;
        }
        const double pb = Pbar[((size_t)f * d.T + t) * d.M + o + mu], xr = x[c].re, xi = x[c].im;
        ar += pb * (zr * xr + zi * xi);  // Re(z conj(x_c))
        ai += pb * (zi * xr - zr * xi);  // Im(z conj(x_c))
      }
    }
    part[tid] = ar;
    part[kB + tid] = ai;
    __syncthreads();
    if (sl == 0 && e < E) {
      for (int j = 1; j < S; ++j) {
        ar += part[tid + j * E];
        ai += part[kB + tid + j * E];
      }
      const int mu = e / ml, c = e - mu * ml;
      double gr = 2.0 * ar, gi = 2.0 * ai;
      if (Qinv) {
        const cd qi = Qinv[(size_t)f * d.QF + q0 + c * ml + mu];  // (Q^-1)_{c mu}; (Q^-H)_{mu c} = conj
        gr -= 2.0 * d.T * qi.re;
        gi += 2.0 * d.T * qi.im;
      }
      cx<RO>& out = dQ[(size_t)f * d.QF + q0 + e];
      if (accumulate) {
        gr += (double)out.re;
        gi += (double)out.im;
      }
      out = {(RO)gr, (RO)gi};
    }
    __syncthreads();
  }
}

// ---- Full iterations.

// u[f][t][m] = sum_n lambda g (unfloored) for the state (W, H, g); grid (F, T / kB).
template <typename RW, typename RH, typename RG>
__global__ __launch_bounds__(kB) void kb_y(Dims d, const RW* __restrict__ W, const RH* __restrict__ H,
                                           const RG* __restrict__ g, double* __restrict__ U) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* sW = reinterpret_cast<double*>(smem);
  double* sg = sW + d.N * d.K;
  const int f = blockIdx.x, t = blockIdx.y * kB + threadIdx.x;
  stage_bin(d, W, g, f, sW, sg);
  __syncthreads();
  if (t >= d.T) return;
  double lam[kMaxN];
  for (int n = 0; n < d.N; ++n) lam[n] = lam_at(d, sW, H, n, t);
  for (int m = 0; m < d.M; ++m) {
    double u = 0.0;
    for (int n = 0; n < d.N; ++n) u += lam[n] * sg[n * d.M + m];
    U[((size_t)f * d.T + t) * d.M + m] = u;
  }
}

// Eq. (14) in full complex form: V[f][voff_l + (mu M_l + a) M_l + b] =
// (1/T) sum_t x_a conj(x_b) / max(u_mu, eps) over subarray l's mics; one workgroup of kCovB threads
// per bin.  Where the bin's entries leave threads over, the frames are split into kCovB / VC
// interleaved slices whose partials are added in slice order.
constexpr int kCovB = 1024;
template <typename R>
__global__ __launch_bounds__(kCovB) void kb_cov(Dims d, const cx<R>* __restrict__ X, const double* __restrict__ U,
                                                cd* __restrict__ V) {
  __shared__ cd part[kCovB];
  const int f = blockIdx.x, tid = threadIdx.x, E = d.VC;
  const int S = E <= kCovB ? kCovB / E : 1;
  for (int i0 = 0; i0 < E; i0 += kCovB) {  // one pass unless VC > kCovB
    const int i = S > 1 ? tid % E : i0 + tid, sl = S > 1 ? tid / E : 0;
    double sr = 0.0, si = 0.0;
    if (i < E && sl < S) {
      const int l = subarray_of_vidx(d, i), ml = d.mics[l], o = d.moff[l], r = i - d.voff[l];
      const int mu = r / (ml * ml), ab = r - mu * ml * ml, a = ab / ml, b = ab - a * ml;
      for (int t = sl; t < d.T; t += S) {
        const size_t ft = (size_t)f * d.T + t;
        const cx<R> xa = X[ft * d.M + o + a], xb = X[ft * d.M + o + b];
        const double u = U[ft * d.M + o + mu], w = 1.0 / (u > d.eps ? u : d.eps);
        const double ar = xa.re, ai = xa.im, br = xb.re, bi = xb.im;
        sr += w * (ar * br + ai * bi);
        si += w * (ai * br - ar * bi);
      }
    }
    part[tid] = {sr, si};
    __syncthreads();
    if (sl == 0 && i < E) {
      for (int j = 1; j < S; ++j) {
        sr += part[tid + j * E].re;
        si += part[tid + j * E].im;
      }
      V[(size_t)f * d.VC + i] = {sr / d.T, si / d.T};
    }
    __syncthreads();
  }
}

// LU factorisation with partial pivoting of an m x m complex A (row-major in A[MX][MX], in place):
// at step k rows k and piv[k] are swapped, so that P A = L U with L unit lower triangular.
template <int MX>
__device__ void lu_factor(int m, cd (&A)[MX][MX], int (&piv)[MX]) {
  for (int k = 0; k < m; ++k) {
    int p = k;
    double best = cabs2(A[k][k]);
    for (int r = k + 1; r < m; ++r)
      if (cabs2(A[r][k]) > best) {
        best = cabs2(A[r][k]);
        p = r;
      }
    piv[k] = p;
    if (p != k)
      for (int c = 0; c < m; ++c) {
        const cd tmp = A[k][c];
        A[k][c] = A[p][c];
        A[p][c] = tmp;
      }
    const cd inv = cinv(A[k][k]);  // a zero pivot gives non-finite results
    for (int r = k + 1; r < m; ++r) {
      const cd fac = cmul(A[r][k], inv);
      A[r][k] = fac;
      for (int c = k + 1; c < m; ++c) A[r][c] = cfms(A[r][c], fac, A[k][c]);
    }
  }
}

// x <- A^-1 x from lu_factor's output.
template <int MX>
__device__ void lu_solve(int m, const cd (&A)[MX][MX], const int (&piv)[MX], cd (&x)[MX]) {
  for (int k = 0; k < m; ++k)
    if (piv[k] != k) {
      const cd tmp = x[k];
      x[k] = x[piv[k]];
      x[piv[k]] = tmp;
    }
  for (int r = 1; r < m; ++r)
    for (int c = 0; c < r; ++c) x[r] = cfms(x[r], A[r][c], x[c]);
  for (int r = m - 1; r >= 0; --r) {
    cd acc = x[r];
    for (int c = r + 1; c < m; ++c) acc = cfms(acc, A[r][c], x[c]);
    x[r] = cmul(acc, cinv(A[r][r]));
  }
}

// x <- A^-H x from lu_factor's output: A^H = U^H L^H P, so U^H w = x, L^H v = w, x = P^T v.
template <int MX>
__device__ void lu_solve_h(int m, const cd (&A)[MX][MX], const int (&piv)[MX], cd (&x)[MX]) {
  for (int r = 0; r < m; ++r) {
    cd acc = x[r];
    for (int c = 0; c < r; ++c) acc = cfms(acc, cconj(A[c][r]), x[c]);
    x[r] = cmul(acc, cinv(cconj(A[r][r])));
  }
  for (int r = m - 2; r >= 0; --r)
    for (int c = r + 1; c < m; ++c) x[r] = cfms(x[r], cconj(A[c][r]), x[c]);
  for (int k = m - 1; k >= 0; --k)
    if (piv[k] != k) {
      const cd tmp = x[k];
      x[k] = x[piv[k]];
      x[piv[k]] = tmp;
    }
}

// One row of the sweep of a block: A = Q V_mu (Q row r from Qlo for r < mu, else from Qhi; both
// row-major m x m in global memory), factorised into LU; b = A^-1 e_mu, Vb = V_mu b,
// s = Re(b^H V_mu b).
template <typename RQ, int MX>
__device__ void ip_row(int m, int mu, const cd* Qlo, const cx<RQ>* __restrict__ Qhi,
                       const cd* __restrict__ Vm, cd (&LU)[MX][MX], int (&piv)[MX], cd (&b)[MX], cd (&Vb)[MX],
                       double& s) {
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < m; ++c) {
      cd acc = {0.0, 0.0};
      for (int k = 0; k < m; ++k) {
        const cd q = r < mu ? Qlo[r * m + k] : cd{(double)Qhi[r * m + k].re, (double)Qhi[r * m + k].im};
        acc = cfma(acc, q, Vm[k * m + c]);
      }
      LU[r][c] = acc;
    }
  lu_factor<MX>(m, LU, piv);
  for (int r = 0; r < m; ++r) b[r] = {r == mu ? 1.0 : 0.0, 0.0};
  lu_solve<MX>(m, LU, piv, b);
  s = 0.0;
  for (int r = 0; r < m; ++r) {
    cd acc = {0.0, 0.0};
    for (int c = 0; c < m; ++c) acc = cfma(acc, Vm[r * m + c], b[c]);
    Vb[r] = acc;
    s += b[r].re * acc.re + b[r].im * acc.im;  // Re(conj(b_r) (V b)_r)
  }
}

// The IP sweep (eqs. (15)-(16)) of block (f, l) from Q (plan precision) and V: Q1 (FP64), the
// updated rows written as they come; one thread per block.
template <typename RQ, int MX>
__global__ __launch_bounds__(64) void kb_ipfwd(Dims d, const cx<RQ>* __restrict__ Q, const cd* __restrict__ V,
                                               cd* __restrict__ Q1) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= d.F * d.L) return;
  const int f = i / d.L, l = i - f * d.L, m = d.mics[l];
  const size_t q0 = (size_t)f * d.QF + d.qoff[l];
  cd LU[MX][MX], b[MX], Vb[MX];
  int piv[MX];
  for (int mu = 0; mu < m; ++mu) {
    double s;
    ip_row<RQ, MX>(m, mu, Q1 + q0, Q + q0, V + (size_t)f * d.VC + d.voff[l] + (size_t)mu * m * m, LU, piv, b, Vb,
                   s);
    const double c = 1.0 / sqrt(s > d.eps ? s : d.eps);
    for (int j = 0; j < m; ++j) Q1[q0 + mu * m + j] = {c * b[j].re, -c * b[j].im};
  }
}

// Adjoint of the sweep of block (f, l): Qbar (in: of the sweep's output Q1; out: of its input Q0,
// updated in place) and Vbar [f][voff_l + (mu M_l + a) M_l + b]; rows in reverse order, each
// recomputed from Q1's rows ..mu-1 and Q0's rows mu...  One thread per block.
template <typename RQ, int MX>
__global__ __launch_bounds__(64) void kb_ipbwd(Dims d, const cx<RQ>* __restrict__ Q0, const cd* __restrict__ Q1,
                                               const cd* __restrict__ V, cd* __restrict__ Qbar,
                                               cd* __restrict__ Vbar) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= d.F * d.L) return;
  const int f = i / d.L, l = i - f * d.L, m = d.mics[l];
  const size_t q0 = (size_t)f * d.QF + d.qoff[l];
  cd* Qb = Qbar + q0;
  cd LU[MX][MX], b[MX], Vb[MX], bb[MX];
  int piv[MX];
  for (int mu = m - 1; mu >= 0; --mu) {
    const size_t v0 = (size_t)f * d.VC + d.voff[l] + (size_t)mu * m * m;
    double s;
    ip_row<RQ, MX>(m, mu, Q1 + q0, Q0 + q0, V + v0, LU, piv, b, Vb, s);
    const bool live = s > d.eps;
    const double c = 1.0 / sqrt(live ? s : d.eps);
    double cbar = 0.0;  // Re(bhbar^H b), bhbar = conj(row mu of Qbar)
    for (int j = 0; j < m; ++j) cbar += Qb[mu * m + j].re * b[j].re - Qb[mu * m + j].im * b[j].im;
    const double sbar = live ? -0.5 * cbar * c * c * c : 0.0;
    for (int j = 0; j < m; ++j)
      bb[j] = {c * Qb[mu * m + j].re + 2.0 * sbar * Vb[j].re, -c * Qb[mu * m + j].im + 2.0 * sbar * Vb[j].im};
    lu_solve_h<MX>(m, LU, piv, bb);  // gamma
    for (int j = 0; j < m; ++j) Qb[mu * m + j] = {0.0, 0.0};
    for (int r = 0; r < m; ++r)
      for (int j = 0; j < m; ++j) Qb[r * m + j] = cfms(Qb[r * m + j], bb[r], cconj(Vb[j]));
    for (int a = 0; a < m; ++a) {
      cd qg = {0.0, 0.0};  // (Q^H gamma)_a with the Q that row mu's step saw
      for (int r = 0; r < m; ++r) {
        const cd q = r < mu ? Q1[q0 + r * m + a] : cd{(double)Q0[q0 + r * m + a].re, (double)Q0[q0 + r * m + a].im};
        qg = cfmac(qg, q, bb[r]);
      }
      const cd coef = {sbar * b[a].re - qg.re, sbar * b[a].im - qg.im};
      for (int j = 0; j < m; ++j) Vbar[v0 + a * m + j] = cmul(coef, cconj(b[j]));
    }
  }
}

// ---- The sweep and its adjoint for subarrays of at most 4 mics, in registers: every block is
// padded to 4 x 4 with the identity (Q and V_mu block-diagonal with I in the unused rows and
// columns), which leaves the used part of A = Q V_mu, b, s, the rows and every adjoint unchanged
// (the padded entries of b, V b, bbar and gamma stay zero), so that all loop bounds and indices
// are compile-time constants.  Row exchanges are selects, not indexed moves.
constexpr int kPad = 4;

struct Pad4 {
  cd a[kPad][kPad];
};

__device__ __forceinline__ void pad_lu(Pad4& A, int (&piv)[kPad]) {
#pragma unroll
  for (int k = 0; k < kPad; ++k) {
    int p = k;
    double best = cabs2(A.a[k][k]);
#pragma unroll
    for (int r = k + 1; r < kPad; ++r) {
      const double v = cabs2(A.a[r][k]);
      if (v > best) {
        best = v;
        p = r;
      }
    }
    piv[k] = p;
#pragma unroll
    for (int r = k + 1; r < kPad; ++r) {
      const bool sw = p == r;
#pragma unroll
      for (int c = 0; c < kPad; ++c) {
        const cd tk = A.a[k][c], tr = A.a[r][c];
        A.a[k][c] = sw ? tr : tk;
        A.a[r][c] = sw ? tk : tr;
      }
    }
    const cd inv = cinv(A.a[k][k]);
#pragma unroll
    for (int r = k + 1; r < kPad; ++r) {
      const cd fac = cmul(A.a[r][k], inv);
      A.a[r][k] = fac;
#pragma unroll
      for (int c = k + 1; c < kPad; ++c) A.a[r][c] = cfms(A.a[r][c], fac, A.a[k][c]);
    }
  }
}

__device__ __forceinline__ void pad_swap(const int (&piv)[kPad], cd (&x)[kPad], bool reverse) {
#pragma unroll
  for (int i = 0; i < kPad; ++i) {
    const int k = reverse ? kPad - 1 - i : i;
#pragma unroll
    for (int r = k + 1; r < kPad; ++r) {
      const bool sw = piv[k] == r;
      const cd tk = x[k], tr = x[r];
      x[k] = sw ? tr : tk;
      x[r] = sw ? tk : tr;
    }
  }
}

__device__ __forceinline__ void pad_solve(const Pad4& A, const int (&piv)[kPad], cd (&x)[kPad]) {
  pad_swap(piv, x, false);
#pragma unroll
  for (int r = 1; r < kPad; ++r)
#pragma unroll
    for (int c = 0; c < r; ++c) x[r] = cfms(x[r], A.a[r][c], x[c]);
#pragma unroll
  for (int r = kPad - 1; r >= 0; --r) {
    cd acc = x[r];
#pragma unroll
    for (int c = r + 1; c < kPad; ++c) acc = cfms(acc, A.a[r][c], x[c]);
    x[r] = cmul(acc, cinv(A.a[r][r]));
  }
}

__device__ __forceinline__ void pad_solve_h(const Pad4& A, const int (&piv)[kPad], cd (&x)[kPad]) {
#pragma unroll
  for (int r = 0; r < kPad; ++r) {
    cd acc = x[r];
#pragma unroll
    for (int c = 0; c < r; ++c) acc = cfms(acc, cconj(A.a[c][r]), x[c]);
    x[r] = cmul(acc, cinv(cconj(A.a[r][r])));
  }
#pragma unroll
  for (int r = kPad - 2; r >= 0; --r)
#pragma unroll
    for (int c = r + 1; c < kPad; ++c) x[r] = cfms(x[r], cconj(A.a[c][r]), x[c]);
  pad_swap(piv, x, true);
}

// Padded block (r, c) of an m x m row-major block in global memory.
__device__ __forceinline__ cd pad_at(const cd* p, int m, int r, int c) {
  return r < m && c < m ? p[r * m + c] : cd{r == c ? 1.0 : 0.0, 0.0};
}
template <typename RQ>
__device__ __forceinline__ cd pad_at(const cx<RQ>* p, int m, int r, int c) {
  return r < m && c < m ? cd{(double)p[r * m + c].re, (double)p[r * m + c].im} : cd{r == c ? 1.0 : 0.0, 0.0};
}

// One row of the sweep, padded: Q (rows from Qlo before mu, else from Qhi), V_mu from Vm.
template <typename RQ>
__device__ __forceinline__ void pad_row(int m, int mu, const cd* Qlo, const cx<RQ>* Qhi, const cd* Vm, Pad4& LU,
                                        int (&piv)[kPad], cd (&b)[kPad], cd (&Vb)[kPad], double& s) {
  cd V[kPad][kPad];
#pragma unroll
  for (int k = 0; k < kPad; ++k)
#pragma unroll
    for (int c = 0; c < kPad; ++c) V[k][c] = pad_at(Vm, m, k, c);
#pragma unroll
  for (int r = 0; r < kPad; ++r) {
    cd q[kPad];
#pragma unroll
    for (int k = 0; k < kPad; ++k) q[k] = r < mu ? pad_at(Qlo, m, r, k) : pad_at(Qhi, m, r, k);
#pragma unroll
    for (int c = 0; c < kPad; ++c) {
      cd acc = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < kPad; ++k) acc = cfma(acc, q[k], V[k][c]);
      LU.a[r][c] = acc;
    }
  }
  pad_lu(LU, piv);
#pragma unroll
  for (int r = 0; r < kPad; ++r) b[r] = {r == mu ? 1.0 : 0.0, 0.0};
  pad_solve(LU, piv, b);
  s = 0.0;
#pragma unroll
  for (int r = 0; r < kPad; ++r) {
    cd acc = {0.0, 0.0};
#pragma unroll
    for (int c = 0; c < kPad; ++c) acc = cfma(acc, V[r][c], b[c]);
    Vb[r] = acc;
    s += b[r].re * acc.re + b[r].im * acc.im;
  }
}

template <typename RQ>
__global__ __launch_bounds__(64) void kb_ipfwd4(Dims d, const cx<RQ>* __restrict__ Q, const cd* __restrict__ V,
                                                cd* __restrict__ Q1) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= d.F * d.L) return;
  const int f = i / d.L, l = i - f * d.L, m = d.mics[l];
  const size_t q0 = (size_t)f * d.QF + d.qoff[l];
  Pad4 LU;
  cd b[kPad], Vb[kPad];
  int piv[kPad];
#pragma unroll
  for (int mu = 0; mu < kPad; ++mu) {
    if (mu >= m) break;
    double s;
    pad_row<RQ>(m, mu, Q1 + q0, Q + q0, V + (size_t)f * d.VC + d.voff[l] + (size_t)mu * m * m, LU, piv, b, Vb, s);
    const double c = 1.0 / sqrt(s > d.eps ? s : d.eps);
#pragma unroll
    for (int j = 0; j < kPad; ++j)
      if (j < m) Q1[q0 + mu * m + j] = {c * b[j].re, -c * b[j].im};
  }
}

template <typename RQ>
__global__ __launch_bounds__(64) void kb_ipbwd4(Dims d, const cx<RQ>* __restrict__ Q0, const cd* __restrict__ Q1,
                                                const cd* __restrict__ V, cd* __restrict__ Qbar,
                                                cd* __restrict__ Vbar) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= d.F * d.L) return;
  const int f = i / d.L, l = i - f * d.L, m = d.mics[l];
  const size_t q0 = (size_t)f * d.QF + d.qoff[l];
  cd Qb[kPad][kPad];  // zero outside the block
#pragma unroll
  for (int r = 0; r < kPad; ++r)
#pragma unroll
    for (int c = 0; c < kPad; ++c) Qb[r][c] = r < m && c < m ? Qbar[q0 + r * m + c] : cd{0.0, 0.0};
  Pad4 LU;
  cd b[kPad], Vb[kPad], bb[kPad];
  int piv[kPad];
#pragma unroll
  for (int mu = kPad - 1; mu >= 0; --mu) {
    if (mu >= m) continue;
    const size_t v0 = (size_t)f * d.VC + d.voff[l] + (size_t)mu * m * m;
    double s;
    pad_row<RQ>(m, mu, Q1 + q0, Q0 + q0, V + v0, LU, piv, b, Vb, s);
    const bool live = s > d.eps;
    const double c = 1.0 / sqrt(live ? s : d.eps);
    double cbar = 0.0;
#pragma unroll
    for (int j = 0; j < kPad; ++j) cbar += Qb[mu][j].re * b[j].re - Qb[mu][j].im * b[j].im;
    const double sbar = live ? -0.5 * cbar * c * c * c : 0.0;
#pragma unroll
    for (int j = 0; j < kPad; ++j)
      bb[j] = {c * Qb[mu][j].re + 2.0 * sbar * Vb[j].re, -c * Qb[mu][j].im + 2.0 * sbar * Vb[j].im};
    pad_solve_h(LU, piv, bb);  // gamma
#pragma unroll
    for (int j = 0; j < kPad; ++j) Qb[mu][j] = {0.0, 0.0};
#pragma unroll
    for (int r = 0; r < kPad; ++r)
#pragma unroll
      for (int j = 0; j < kPad; ++j) Qb[r][j] = cfms(Qb[r][j], bb[r], cconj(Vb[j]));
#pragma unroll
    for (int a = 0; a < kPad; ++a) {
      if (a >= m) break;
      cd qg = {0.0, 0.0};
#pragma unroll
      for (int r = 0; r < kPad; ++r) qg = cfmac(qg, r < mu ? pad_at(Q1 + q0, m, r, a) : pad_at(Q0 + q0, m, r, a), bb[r]);
      const cd coef = {sbar * b[a].re - qg.re, sbar * b[a].im - qg.im};
#pragma unroll
      for (int j = 0; j < kPad; ++j)
        if (j < m) Vbar[v0 + a * m + j] = cmul(coef, cconj(b[j]));
    }
  }
#pragma unroll
  for (int r = 0; r < kPad; ++r)
#pragma unroll
    for (int c = 0; c < kPad; ++c)
      if (r < m && c < m) Qbar[q0 + r * m + c] = Qb[r][c];
}

// ybar[f][t][o_l + mu] = -Re(x^H Vbar_mu x) / (T y^2), zero where y is floored; one thread per
// (t, m) of bin f (grid (F, T M / kB)).  With LDS the bin's Vbar is staged there first, each
// (l, mu) block followed by one pad entry: the block of mic m then starts at voff_l + m + mu M_l^2,
// so the lanes of one frame, which read the same entry of their blocks, fall in distinct banks.
template <typename R, bool LDS>
__global__ __launch_bounds__(kB) void kb_vbar(Dims d, const cx<R>* __restrict__ X, const double* __restrict__ U,
                                              const cd* __restrict__ Vbar, double* __restrict__ Ybar) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int f = blockIdx.x, i = blockIdx.y * kB + threadIdx.x;
  const cd* vf = Vbar + (size_t)f * d.VC;
  cd* sv = reinterpret_cast<cd*>(smem);
  if (LDS) {
    for (int j = threadIdx.x; j < d.VC; j += kB) {
      const int l = subarray_of_vidx(d, j), ml2 = d.mics[l] * d.mics[l], r = j - d.voff[l], mu = r / ml2;
      sv[j + d.moff[l] + mu] = vf[j];
    }
    __syncthreads();
  }
  if (i >= d.T * d.M) return;
  const int t = i / d.M, m = i - t * d.M, l = d.msub[m], ml = d.mics[l], o = d.moff[l], mu = m - o;
  const size_t ft = (size_t)f * d.T + t;
  const cx<R>* x = X + ft * d.M + o;
  const cd* vb = LDS ? sv + d.voff[l] + m + (size_t)mu * ml * ml : vf + d.voff[l] + (size_t)mu * ml * ml;
  double q = 0.0;  // Re(x^H Vbar x)
  for (int a = 0; a < ml; ++a) {
    cd row = {0.0, 0.0};
    for (int b = 0; b < ml; ++b) row = cfma(row, vb[a * ml + b], cd{(double)x[b].re, (double)x[b].im});
    q += (double)x[a].re * row.re + (double)x[a].im * row.im;
  }
  const double u = U[ft * d.M + m];
  Ybar[ft * d.M + m] = u > d.eps ? -q / ((double)d.T * u * u) : 0.0;
}

__global__ __launch_bounds__(kB) void kb_zero(size_t n, double* __restrict__ p) {
  const size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

template <typename R>
__global__ __launch_bounds__(kB) void kb_store(int n, const double* __restrict__ src, R* __restrict__ dst) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i < n) dst[i] = (R)src[i];
}

}  // namespace grad

// ---- Tape layout: checkpoints (plan precision), then FP64 work arrays.
struct GradTape {
  void* ckg;  // [n_iter][F N M]
  void* ckW;  // [n_iter][N F K]
  void* ckH;  // [n_iter][N K T]
  void* ckQ;  // full iterations: [n_iter][F QF] complex
  cd *Q1, *Qbar;                                                  // full: [F][QF]
  cd *V, *Vbar;                                                   // full: [F][VC]
  double *U, *Ybar;                                               // full: [F][T][M]
  double *P, *Pbar, *lbar, *c0, *d0, *c1, *d1, *cb, *db;           // [F][T][M] / [F][T][N]
  double *aW, *bW, *aWb, *bWb, *W1, *Wacc;                        // [N][F][K]
  double *aH, *bH, *aHb, *bHb, *H1, *Hacc;                        // [N][K][T]
  double *ag, *bg, *agb, *bgb, *gacc;                             // [F][N][M]
  double* fpart;                                                  // [F][ceil(T / CH)][2][N][M] (kb_frame)
};

static size_t alg(size_t x) { return (x + 255) / 256 * 256; }

// Frames per kb_frame workgroup: as many as fit 48 KB of LDS next to the bin's W, g, abar, bbar,
// at most 128.
static int frame_chunk(const Dims& d) {
  const size_t fixed = 8 * ((size_t)d.N * d.K + 3 * (size_t)d.N * d.M);
  const size_t per = 8 * (3 * (size_t)d.N + 3 * (size_t)d.M);
  size_t ch = fixed < 48 * 1024 ? (48 * 1024 - fixed) / per : 1;
  if (ch > 128) ch = 128;
  return ch < 1 ? 1 : (int)ch;
}
static int frame_slices(const Dims& d) { return (d.T + frame_chunk(d) - 1) / frame_chunk(d); }
static size_t frame_smem(const Dims& d, int ch) {
  return 8 * ((size_t)d.N * d.K + 3 * (size_t)d.N * d.M + (size_t)ch * (3 * d.N + 3 * d.M));
}

static size_t carve_tape(const Dims& d, int dtype, int n_iter, bool full, char* base, GradTape* t) {
  const size_t r = dtype == DFM_C64 ? 4 : 8;
  const size_t FQ = (size_t)d.F * d.QF, FV = (size_t)d.F * d.VC;
  const size_t NG = (size_t)d.F * d.N * d.M, NW = (size_t)d.N * d.F * d.K, NH = (size_t)d.N * d.K * d.T;
  const size_t FTM = (size_t)d.F * d.T * d.M, FTN = (size_t)d.F * d.T * d.N;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += alg(bytes);
    return p;
  };
  GradTape tt;
  tt.ckg = take(r * NG * n_iter);
  tt.ckW = take(r * NW * n_iter);
  tt.ckH = take(r * NH * n_iter);
  tt.ckQ = take(full ? 2 * r * FQ * n_iter : 0);
  tt.Q1 = reinterpret_cast<cd*>(take(full ? 16 * FQ : 0));
  tt.Qbar = reinterpret_cast<cd*>(take(full ? 16 * FQ : 0));
  tt.V = reinterpret_cast<cd*>(take(full ? 16 * FV : 0));
  tt.Vbar = reinterpret_cast<cd*>(take(full ? 16 * FV : 0));
  tt.U = reinterpret_cast<double*>(take(full ? 8 * FTM : 0));
  tt.Ybar = reinterpret_cast<double*>(take(full ? 8 * FTM : 0));
  double** ftm[] = {&tt.P, &tt.Pbar};
  for (double** p : ftm) *p = reinterpret_cast<double*>(take(8 * FTM));
  double** ftn[] = {&tt.lbar, &tt.c0, &tt.d0, &tt.c1, &tt.d1, &tt.cb, &tt.db};
  for (double** p : ftn) *p = reinterpret_cast<double*>(take(8 * FTN));
  double** nw[] = {&tt.aW, &tt.bW, &tt.aWb, &tt.bWb, &tt.W1, &tt.Wacc};
  for (double** p : nw) *p = reinterpret_cast<double*>(take(8 * NW));
  double** nh[] = {&tt.aH, &tt.bH, &tt.aHb, &tt.bHb, &tt.H1, &tt.Hacc};
  for (double** p : nh) *p = reinterpret_cast<double*>(take(8 * NH));
  double** ng[] = {&tt.ag, &tt.bg, &tt.agb, &tt.bgb, &tt.gacc};
  for (double** p : ng) *p = reinterpret_cast<double*>(take(8 * NG));
  tt.fpart = reinterpret_cast<double*>(take(8 * 2 * NG * (size_t)frame_slices(d)));
  if (t) *t = tt;
  return off;
}

size_t grad_tape_bytes(const Dims& d, int dtype, int n_iter, bool full) {
  return carve_tape(d, dtype, n_iter, full, nullptr, nullptr);
}

void grad_checkpoints(const Dims& d, int dtype, int n_iter, bool full, void* tape, int it, void** Q, void** g,
                      void** W, void** H) {
  GradTape t;
  carve_tape(d, dtype, n_iter, full, static_cast<char*>(tape), &t);
  const size_t r = dtype == DFM_C64 ? 4 : 8;
  *g = static_cast<char*>(t.ckg) + r * (size_t)d.F * d.N * d.M * it;
  *W = static_cast<char*>(t.ckW) + r * (size_t)d.N * d.F * d.K * it;
  *H = static_cast<char*>(t.ckH) + r * (size_t)d.N * d.K * d.T * it;
  if (Q) *Q = full ? static_cast<char*>(t.ckQ) + 2 * r * (size_t)d.F * d.QF * it : nullptr;
}

static unsigned nblk(size_t n) { return (unsigned)((n + grad::kB - 1) / grad::kB); }


// kb_frame (per-thread arrays sized for N: 8 or 16 sources) over (bin, slice), then kb_gsum.
template <typename RW, typename RH, typename RG, int MODE>
static void frame(const Dims& d, const GradTape& t, hipStream_t s, const RW* W, const RH* H, const RG* g,
                  const double* P, const double* c1, const double* c2, double* Pbar, double* lbar, double* gout,
                  double* gout2) {
  const int CH = frame_chunk(d), S = frame_slices(d);
  const size_t fsm = frame_smem(d, CH);
  const dim3 grid(d.F, S), blk(grad::kB);
  if (d.N <= 8)
    hipLaunchKernelGGL((grad::kb_frame<RW, RH, RG, MODE, 8>), grid, blk, fsm, s, d, W, H, g, P, c1, c2, Pbar, lbar,
                       t.fpart, CH);
  else
    hipLaunchKernelGGL((grad::kb_frame<RW, RH, RG, MODE, kMaxN>), grid, blk, fsm, s, d, W, H, g, P, c1, c2, Pbar,
                       lbar, t.fpart, CH);
  hipLaunchKernelGGL(grad::kb_gsum<MODE>, dim3(nblk((size_t)d.F * d.N * d.M)), blk, 0, s, d, S,
                     (const double*)t.fpart, gout, gout2);
}

// Back through the MM updates of one iteration from its checkpoint (g0, W0, H0) against t.P: on
// entry (gacc, Wacc, Hacc) hold the adjoints of the iteration's output, on exit those of its input
// through the updates; Pbar gathers the adjoint of P.
template <typename R>
static void mm_back_iteration(const Dims& d, const GradTape& t, const R* g0, const R* W0, const R* H0,
                              hipStream_t s) {
  using namespace grad;
  const int NG = d.F * d.N * d.M, NW = d.N * d.F * d.K, NH = d.N * d.K * d.T, FTN = d.F * d.T * d.N;
  const size_t csm = 8 * ((size_t)d.N * d.K + (size_t)d.N * d.M);
  const dim3 ft(d.F, (d.T + kB - 1) / kB), blk(kB);
  const dim3 gW(nblk(NW)), gH(nblk(NH)), gG(nblk(NG)), gFTN(nblk(FTN));
  const dim3 gSt(d.N * d.F), gSf(d.N * d.K, (d.T + 63) / 64);
  const double* nul = nullptr;
  // This iteration's forward from its checkpoint, in FP64: W1 (eq. (8)), H1 (eq. (9)), the sums
  // of eq. (10).
  hipLaunchKernelGGL((kb_coef<R, R, R>), ft, blk, csm, s, d, W0, H0, g0, t.P, t.c0, t.d0);
  hipLaunchKernelGGL(kb_sum_t<R>, gSt, blk, 0, s, d, H0, t.c0, (const R*)nullptr, nul, t.aW, 0);
  hipLaunchKernelGGL(kb_sum_t<R>, gSt, blk, 0, s, d, H0, t.d0, (const R*)nullptr, nul, t.bW, 0);
  hipLaunchKernelGGL(kb_apply<R>, gW, blk, 0, s, NW, W0, t.aW, t.bW, d.eps, t.W1);
  hipLaunchKernelGGL((kb_coef<double, R, R>), ft, blk, csm, s, d, (const double*)t.W1, H0, g0, t.P, t.c1, t.d1);
  hipLaunchKernelGGL(kb_sum_f<double>, gSf, blk, 0, s, d, (const double*)t.W1, t.c1, (const double*)nullptr, nul,
                     t.aH, 0);
  hipLaunchKernelGGL(kb_sum_f<double>, gSf, blk, 0, s, d, (const double*)t.W1, t.d1, (const double*)nullptr, nul,
                     t.bH, 0);
  hipLaunchKernelGGL(kb_apply<R>, gH, blk, 0, s, NH, H0, t.aH, t.bH, d.eps, t.H1);
  frame<double, double, R, kFwdG>(d, t, s, (const double*)t.W1,
                     (const double*)t.H1, g0, t.P, nul, nul, (double*)nullptr, (double*)nullptr, t.ag, t.bg);
  // Back through eq. (10): g1 = g0 sqrt(ag / max(bg, eps)) with lambda2 = W1 H1.
  hipLaunchKernelGGL(kb_mmback<R>, gG, blk, 0, s, NG, g0, t.ag, t.bg, d.eps, t.gacc, t.agb, t.bgb);
  frame<double, double, R, kBackG>(d, t, s, (const double*)t.W1,
                     (const double*)t.H1, g0, t.P, (const double*)t.agb, (const double*)t.bgb, t.Pbar, t.lbar,
                     t.gacc, (double*)nullptr);
  hipLaunchKernelGGL(kb_sum_t<double>, gSt, blk, 0, s, d, (const double*)t.H1, t.lbar, (const double*)nullptr, nul,
                     t.Wacc, 1);
  hipLaunchKernelGGL(kb_sum_f<double>, gSf, blk, 0, s, d, (const double*)t.W1, t.lbar, (const double*)nullptr, nul,
                     t.Hacc, 1);
  // Back through eq. (9): H1 = H0 sqrt(aH / max(bH, eps)), aH = sum_f W1 c1, bH = sum_f W1 d1.
  hipLaunchKernelGGL(kb_mmback<R>, gH, blk, 0, s, NH, H0, t.aH, t.bH, d.eps, t.Hacc, t.aHb, t.bHb);
  hipLaunchKernelGGL(kb_sum_t<double>, gSt, blk, 0, s, d, (const double*)t.aHb, t.c1, (const double*)t.bHb, t.d1,
                     t.Wacc, 1);
  hipLaunchKernelGGL((kb_cbar<double, double>), gFTN, blk, 0, s, d, (const double*)t.W1, (const double*)t.aHb,
                     (const double*)t.W1, (const double*)t.bHb, t.cb, t.db);
  frame<double, R, R, kBackWH>(d, t, s, (const double*)t.W1, H0, g0, t.P,
                     (const double*)t.cb, (const double*)t.db, t.Pbar, t.lbar, t.gacc, (double*)nullptr);
  hipLaunchKernelGGL(kb_sum_t<R>, gSt, blk, 0, s, d, H0, t.lbar, (const R*)nullptr, nul, t.Wacc, 1);
  hipLaunchKernelGGL(kb_sum_f<double>, gSf, blk, 0, s, d, (const double*)t.W1, t.lbar, (const double*)nullptr, nul,
                     t.Hacc, 1);
  // Back through eq. (8): W1 = W0 sqrt(aW / max(bW, eps)), aW = sum_t H0 c0, bW = sum_t H0 d0.
  hipLaunchKernelGGL(kb_mmback<R>, gW, blk, 0, s, NW, W0, t.aW, t.bW, d.eps, t.Wacc, t.aWb, t.bWb);
  hipLaunchKernelGGL(kb_sum_f<double>, gSf, blk, 0, s, d, (const double*)t.aWb, t.c0, (const double*)t.bWb, t.d0,
                     t.Hacc, 1);
  hipLaunchKernelGGL((kb_cbar<double, R>), gFTN, blk, 0, s, d, (const double*)t.aWb, H0, (const double*)t.bWb, H0,
                     t.cb, t.db);
  frame<R, R, R, kBackWH>(d, t, s, W0, H0, g0, t.P, (const double*)t.cb,
                     (const double*)t.db, t.Pbar, t.lbar, t.gacc, (double*)nullptr);
  hipLaunchKernelGGL(kb_sum_t<R>, gSt, blk, 0, s, d, H0, t.lbar, (const R*)nullptr, nul, t.Wacc, 1);
  hipLaunchKernelGGL(kb_sum_f<R>, gSf, blk, 0, s, d, W0, t.lbar, (const R*)nullptr, nul, t.Hacc, 1);
}

template <typename RQ, int MX>
static void ip_launch(const Dims& d, const GradTape& t, const cx<RQ>* Q0, bool backward, hipStream_t s) {
  const dim3 grid((d.F * d.L + 63) / 64), blk(64);
  if (backward)
    hipLaunchKernelGGL((grad::kb_ipbwd<RQ, MX>), grid, blk, 0, s, d, Q0, (const cd*)t.Q1, (const cd*)t.V, t.Qbar,
                       t.Vbar);
  else
    hipLaunchKernelGGL((grad::kb_ipfwd<RQ, MX>), grid, blk, 0, s, d, Q0, (const cd*)t.V, t.Q1);
}

template <typename RQ>
static void ip_dispatch(const Dims& d, const GradTape& t, const cx<RQ>* Q0, bool backward, hipStream_t s) {
  const dim3 grid((d.F * d.L + 63) / 64), blk(64);
  if (d.MLX <= grad::kPad) {  // registers
    if (backward)
      hipLaunchKernelGGL(grad::kb_ipbwd4<RQ>, grid, blk, 0, s, d, Q0, (const cd*)t.Q1, (const cd*)t.V, t.Qbar, t.Vbar);
    else
      hipLaunchKernelGGL(grad::kb_ipfwd4<RQ>, grid, blk, 0, s, d, Q0, (const cd*)t.V, t.Q1);
  } else if (d.MLX <= 8)
    ip_launch<RQ, 8>(d, t, Q0, backward, s);
  else
    ip_launch<RQ, 16>(d, t, Q0, backward, s);
}

template <typename R>
static hipError_t backward_impl(const Dims& d, const Buffers& b, int n_iter, bool full, void* tape, void* dQ,
                                void* dg, void* dW, void* dH, hipStream_t s) {
  using namespace grad;
  const int dtype = sizeof(R) == 4 ? DFM_C64 : DFM_C128;
  GradTape t;
  carve_tape(d, dtype, n_iter, full, static_cast<char*>(tape), &t);
  const cx<R>* X = static_cast<const cx<R>*>(b.X);
  const cx<R>* Q = static_cast<const cx<R>*>(b.Q);
  const int NG = d.F * d.N * d.M, NW = d.N * d.F * d.K, NH = d.N * d.K * d.T;
  const size_t FTM = (size_t)d.F * d.T * d.M;
  const size_t csm = 8 * ((size_t)d.N * d.K + (size_t)d.N * d.M);
  const dim3 ft(d.F, (d.T + kB - 1) / kB), blk(kB), ftm(d.F, (d.T * d.M + kB - 1) / kB);
  const dim3 gW(nblk(NW)), gH(nblk(NH)), gG(nblk(NG));
  const dim3 gSt(d.N * d.F), gSf(d.N * d.K, (d.T + 63) / 64);
  const double* nul = nullptr;
  hipLaunchKernelGGL((kb_powers<R, R>), ftm, blk, 0, s, d, X, Q, t.P);
  // The cost's own gradient at the final state (the plan's current Q, g, W, H).
  const R* gK = static_cast<const R*>(b.g);
  const R* WK = static_cast<const R*>(b.W);
  const R* HK = static_cast<const R*>(b.H);
  frame<R, R, R, kCost>(d, t, s, WK, HK, gK, t.P, nul, nul, t.Pbar,
                     t.lbar, t.gacc, (double*)nullptr);
  hipLaunchKernelGGL(kb_sum_t<R>, gSt, blk, 0, s, d, HK, t.lbar, (const R*)nullptr, nul, t.Wacc, 0);
  hipLaunchKernelGGL(kb_sum_f<R>, gSf, blk, 0, s, d, WK, t.lbar, (const R*)nullptr, nul, t.Hacc, 0);
  // Q^-1 of the final Q by the generic elimination kernel, for the log-determinant's term.
  hipError_t e = launch_qinv(d, b, dtype, s);
  if (e != hipSuccess) return e;
  const cd* Qinv = static_cast<const cd*>(b.Qinv);
  if (full)  // Qbar of the final Q now; P's adjoint is then gathered per iteration
    hipLaunchKernelGGL((kb_qgrad<R, R, double>), dim3(d.F, d.L), blk, 0, s, d, X, Q, Qinv, t.Pbar,
                       reinterpret_cast<cx<double>*>(t.Qbar), 0);
  for (int it = n_iter - 1; it >= 0; --it) {
    void *pQ, *pg, *pW, *pH;
    grad_checkpoints(d, dtype, n_iter, full, tape, it, &pQ, &pg, &pW, &pH);
    const R* g0 = static_cast<const R*>(pg);
    const R* W0 = static_cast<const R*>(pW);
    const R* H0 = static_cast<const R*>(pH);
    const cx<R>* Q0 = static_cast<const cx<R>*>(pQ);
    if (full) {
      // The sweep from the checkpoint: u, V (eq. (14)), Q_{i+1} (eqs. (15)-(16)), P_{i+1}.
      hipLaunchKernelGGL((kb_y<R, R, R>), ft, blk, csm, s, d, W0, H0, g0, t.U);
      hipLaunchKernelGGL(kb_cov<R>, dim3(d.F), dim3(kCovB), 0, s, d, X, (const double*)t.U, t.V);
      ip_dispatch<R>(d, t, Q0, false, s);
      hipLaunchKernelGGL((kb_powers<R, double>), ftm, blk, 0, s, d, X, reinterpret_cast<const cx<double>*>(t.Q1),
                         t.P);
      hipLaunchKernelGGL(kb_zero, dim3(nblk(FTM)), blk, 0, s, FTM, t.Pbar);
    }
    mm_back_iteration<R>(d, t, g0, W0, H0, s);
    if (full) {
      // Qbar_{i+1} += 2 sum_t Pbar z conj(x) (z = Q_{i+1} x), then back through the sweep and the
      // covariances to (g_i, W_i, H_i).
      hipLaunchKernelGGL((kb_qgrad<R, double, double>), dim3(d.F, d.L), blk, 0, s, d, X,
                         reinterpret_cast<const cx<double>*>(t.Q1), (const cd*)nullptr, t.Pbar,
                         reinterpret_cast<cx<double>*>(t.Qbar), 1);
      ip_dispatch<R>(d, t, Q0, true, s);
      if ((size_t)(d.VC + d.M) * sizeof(cd) <= 64 * 1024)
        hipLaunchKernelGGL((kb_vbar<R, true>), ftm, blk, (size_t)(d.VC + d.M) * sizeof(cd), s, d, X,
                           (const double*)t.U, (const cd*)t.Vbar, t.Ybar);
      else
        hipLaunchKernelGGL((kb_vbar<R, false>), ftm, blk, 0, s, d, X, (const double*)t.U, (const cd*)t.Vbar, t.Ybar);
      frame<R, R, R, kBackY>(d, t, s, W0, H0, g0, t.P,
                         (const double*)t.Ybar, nul, t.Pbar, t.lbar, t.gacc, (double*)nullptr);
      hipLaunchKernelGGL(kb_sum_t<R>, gSt, blk, 0, s, d, H0, t.lbar, (const R*)nullptr, nul, t.Wacc, 1);
      hipLaunchKernelGGL(kb_sum_f<R>, gSf, blk, 0, s, d, W0, t.lbar, (const R*)nullptr, nul, t.Hacc, 1);
    }
  }
  if (full)
    hipLaunchKernelGGL(kb_store<R>, dim3(nblk(2 * (size_t)d.F * d.QF)), blk, 0, s, 2 * d.F * d.QF,
                       (const double*)t.Qbar, static_cast<R*>(dQ));
  else  // Q fixed: P's adjoint from every iteration and the cost gives the gradient with respect to Q
    hipLaunchKernelGGL((kb_qgrad<R, R, R>), dim3(d.F, d.L), blk, 0, s, d, X, Q, Qinv, t.Pbar,
                       static_cast<cx<R>*>(dQ), 0);
  hipLaunchKernelGGL(kb_store<R>, gG, blk, 0, s, NG, (const double*)t.gacc, static_cast<R*>(dg));
  hipLaunchKernelGGL(kb_store<R>, gW, blk, 0, s, NW, (const double*)t.Wacc, static_cast<R*>(dW));
  hipLaunchKernelGGL(kb_store<R>, gH, blk, 0, s, NH, (const double*)t.Hacc, static_cast<R*>(dH));
  return hipGetLastError();
}

hipError_t launch_grad_backward(const Dims& d, const Buffers& b, int dtype, int n_iter, bool full, void* tape,
                                void* dQ, void* dg, void* dW, void* dH, hipStream_t s) {
  return dtype == DFM_C64 ? backward_impl<float>(d, b, n_iter, full, tape, dQ, dg, dW, dH, s)
                          : backward_impl<double>(d, b, n_iter, full, tape, dQ, dg, dW, dH, s);
}

}  // namespace dfm
