// HIP kernels of distributed FastMNMF for gfx950.
//
// Data layout in HBM (all row-major, caller-owned unless noted):
//   X [F][T][M] complex, Q [F][sum M_l^2] complex, g [F][N][M], W [N][F][K], H [N][K][T]
//   P [F][T][M] real (workspace): powers |(Q_fl x_ft^(l))_mu|^2 of the latest W sub-step.
//
// Streaming kernels work on tiles (f, time slice) of d.SL frames with 256 threads:
// phase 1 puts one frame (in k_pw, one (frame, source) or (frame, mic) pair) per thread
// and writes per-frame quantities to LDS; phase 2
// puts one output per thread and contracts over the slice's frames from LDS, so no
// cross-lane reductions are needed.  Per-frequency sums over slices (and the
// activation update's sum over frequency tiles) are finished by small "apply"
// kernels in a fixed order, so every result is deterministic run to run.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dfm_device.h"

namespace dfm {

// ---------------------------------------------------------------------------------------
// Weighted covariances, eq. (14): per tile (f, slice) the packed sums
//   sum_t x_ta conj(x_tb) / y_{t, o_l + mu}   for every (l, mu, a <= b).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_gram(Dims d, const cx<R>* __restrict__ X, const R* __restrict__ W,
                                                 const R* __restrict__ H, const R* __restrict__ g,
                                                 double* __restrict__ Vpart) {
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, d.T - t0);
  extern __shared__ __align__(16) unsigned char smem[];
  R* sW = reinterpret_cast<R*>(smem);
  R* sg = sW + d.N * d.K;
  R* sinv = sg + d.N * d.M;
  cx<R>* sx = reinterpret_cast<cx<R>*>(smem + align_up(sizeof(R) * (d.N * d.K + d.N * d.M + d.SL * d.M), 16));

  for (int i = tid; i < d.N * d.K; i += kBlock) {
    const int n = i / d.K, k = i - n * d.K;
    sW[i] = W[((size_t)n * d.F + f) * d.K + k];
  }
  for (int i = tid; i < d.N * d.M; i += kBlock) sg[i] = g[(size_t)f * d.N * d.M + i];
  const cx<R>* xf = X + ((size_t)f * d.T + t0) * d.M;
  for (int i = tid; i < nt * d.M; i += kBlock) sx[i] = xf[i];
  __syncthreads();

  for (int tl = tid; tl < nt; tl += kBlock) {
    R lam[kMaxN];
    source_psd(d, sW, d.K, H, t0 + tl, lam);
    for (int m = 0; m < d.M; ++m) sinv[tl * d.M + m] = (R)1 / model_var(d, lam, sg, m);
  }
  __syncthreads();

  // Sums in FP64 of exact products (the solve of eq. (15) amplifies summation error by
  // cond(V), which is large for nearly rank-deficient mixing).
  // One work item per (subarray, pair of rows mu, mic pair a <= b): per frame it forms both
  // parts of x_a conj(x_b) once and adds them into both rows' sums.
  double* out = Vpart + ((size_t)f * d.S + s) * d.VF;
  int items = 0;
  for (int l = 0; l < d.L; ++l) items += (d.mics[l] + 1) / 2 * (d.mics[l] * (d.mics[l] + 1) / 2);
  for (int it = tid; it < items; it += kBlock) {
    int l = 0, i = it;
    for (;; ++l) {
      const int n = (d.mics[l] + 1) / 2 * (d.mics[l] * (d.mics[l] + 1) / 2);
      if (i < n) break;
      i -= n;
    }
    const int Ml = d.mics[l], npair = Ml * (Ml + 1) / 2, q = i / npair, pi = i - q * npair;
    const int mu0 = 2 * q, mu1 = mu0 + 1 < Ml ? mu0 + 1 : -1;
    const int jre = pi < Ml ? pi : Ml + 2 * (pi - Ml);  // packed index of (a, b) (real part)
    int a, b, part;
    packed_pair(Ml, jre, a, b, part);
    const bool diag = a == b;
    const int o = d.moff[l];
    double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
    for (int tl = 0; tl < nt; ++tl) {
      const cx<R> xa = sx[tl * d.M + o + a];
      const cx<R> xb = sx[tl * d.M + o + b];
      const double ar = xa.re, ai = xa.im, br = xb.re, bi = xb.im;
      const double vr = ar * br + ai * bi, vi = ai * br - ar * bi;
      const double w0 = sinv[tl * d.M + o + mu0];
      re0 += w0 * vr;
      im0 += w0 * vi;
      if (mu1 >= 0) {
        const double w1 = sinv[tl * d.M + o + mu1];
        re1 += w1 * vr;
        im1 += w1 * vi;
      }
    }
    double* o0 = out + d.voff[l] + (size_t)mu0 * Ml * Ml + jre;
    o0[0] = re0;
    if (!diag) o0[1] = im0;
    if (mu1 >= 0) {
      double* o1 = out + d.voff[l] + (size_t)mu1 * Ml * Ml + jre;
      o1[0] = re1;
      if (!diag) o1[1] = im1;
    }
  }
}

// IP sweep over the rows of one subarray block Q_fl, eqs. (15)-(16), in FP64; block (f, l).
// (Q V_mu) b = e_mu is solved as V_mu b = c with c = Q^{-1} e_mu (the same system, Q being
// nonsingular).  Q^{-1} comes from Q once per sweep (Gauss-Jordan elimination with partial
// pivoting); then for mu = 0..M_l-1: V_mu from the slot sums, V_mu b = c by Gauss-Jordan
// elimination without pivoting (V_mu is Hermitian positive definite), b <- b / sqrt(max(b^H c,
// eps)) (b^H c = b^H V_mu b, eq. (16)), row mu of Q <- b^H, and with u^H = b^H Q^{-1} the
// rank-1 update Q^{-1} <- Q^{-1} - c (u^H - e_mu^T) / (b^H c) of the inverse for the new row;
// ln|det Q_fl| (for the cost (13)) from the pivots of Q and ln|b^H c| of each row.  Every
// elimination step updates all rows at once, one element per thread.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_ip(Dims d, const double* __restrict__ Vpart, cx<R>* __restrict__ Q,
                                               double* __restrict__ logdet, int* __restrict__ status) {
  const int f = blockIdx.x, l = blockIdx.y, tid = threadIdx.x, bd = blockDim.x;
  const int Ml = d.mics[l], l2 = 2 * Ml, lv = Ml + 1;
  // LDS sized for the partition's largest subarray (ip_smem), so that small blocks keep many
  // workgroups per CU.
  extern __shared__ __align__(16) unsigned char smem[];
  const int mx = d.MLX;
  cd* sQ = reinterpret_cast<cd*>(smem);  // Q, rows replaced as the sweep goes [mx * mx]
  cd* sI = sQ + mx * mx;                  // [Q | I] -> columns Ml .. 2 Ml - 1: Q^{-1} [mx * 2 mx]
  cd* sV = sI + 2 * mx * mx;              // [V_mu | c] [mx * (mx + 1)]
  cd* sc = sV + mx * (mx + 1);            // [mx] each
  cd* sb = sc + mx;
  cd* su = sb + mx;
  __shared__ double s_logabs, s_w2;
  __shared__ int s_sing, s_ok;

  cx<R>* qb = Q + (size_t)f * d.QF + d.qoff[l];
  for (int i = tid; i < Ml * l2; i += bd) {
    const int r = i / l2, c = i - r * l2;
    const cd q = c < Ml ? cd{(double)qb[r * Ml + c].re, (double)qb[r * Ml + c].im} : cd{c - Ml == r ? 1.0 : 0.0, 0.0};
    sI[i] = q;
    if (c < Ml) sQ[r * Ml + c] = q;
  }
  __syncthreads();
  eliminate(sI, l2, Ml, l2, &s_logabs, &s_sing);
  if (s_sing) {  // Q itself singular: keep it, report it (uniform: read after the last barrier)
    if (tid == 0) {
      atomicOr(status, kStSingular);
      logdet[(size_t)f * d.L + l] = -INFINITY;
    }
    return;
  }
  // Back substitution, one thread per column of the inverse.
  for (int c = tid; c < Ml; c += bd)
    for (int r = Ml - 1; r >= 0; --r) {
      cd acc = sI[r * l2 + Ml + c];
      for (int j = r + 1; j < Ml; ++j) acc = csub(acc, cmul(sI[r * l2 + j], sI[j * l2 + Ml + c]));
      sI[r * l2 + Ml + c] = cabs2(sI[r * l2 + r]) == 0.0 ? cd{0.0, 0.0} : cmul(acc, cinv(sI[r * l2 + r]));
    }
  auto qinv = [&](int r, int c) -> cd& { return sI[r * l2 + Ml + c]; };
  const double invT = 1.0 / d.T;

  for (int mu = 0; mu < Ml; ++mu) {
    __syncthreads();  // Q^{-1} (and the previous row's update) complete
    const double* vp = Vpart + (size_t)f * d.SG * d.VF + d.voff[l] + mu * Ml * Ml;
    const int ns = cov_slots(d, f);
    for (int j = tid; j < Ml * Ml; j += bd) {
      double acc = 0.0;
      for (int s = 0; s < ns; ++s) acc += vp[(size_t)s * d.VF + j];
      acc *= invT;
      int a, b, part;
      packed_pair(Ml, j, a, b, part);
      if (a == b) {
        sV[a * lv + a] = {acc, 0.0};
      } else if (part == 0) {
        sV[a * lv + b].re = acc;
        sV[b * lv + a].re = acc;
      } else {
        sV[a * lv + b].im = acc;
        sV[b * lv + a].im = -acc;
      }
    }
    for (int r = tid; r < Ml; r += bd) {
      sc[r] = qinv(r, mu);
      sV[r * lv + Ml] = qinv(r, mu);
    }
    if (tid == 0) s_ok = 1;
    __syncthreads();
    // Gauss-Jordan on [V_mu | c]: step p clears column p above and below the pivot.  A step
    // reads row p and column p only, which it does not write.
    for (int p = 0; p < Ml; ++p) {
      const cd pv = sV[p * lv + p];
      if (cabs2(pv) == 0.0) {  // same value in every thread: uniform exit
        if (tid == 0) s_ok = 0;
        break;
      }
      const cd inv = cinv(pv);
      const int w = Ml - p;  // columns p + 1 .. Ml
      for (int i = tid; i < (Ml - 1) * w; i += bd) {
        const int rr = i / w, r = rr < p ? rr : rr + 1, c = p + 1 + (i - rr * w);
        sV[r * lv + c] = csub(sV[r * lv + c], cmul(cmul(sV[r * lv + p], inv), sV[p * lv + c]));
      }
      __syncthreads();
    }
    __syncthreads();
    if (s_ok)
      for (int r = tid; r < Ml; r += bd) sb[r] = cmul(sV[r * lv + Ml], cinv(sV[r * lv + r]));
    __syncthreads();
    if (tid == 0) {
      bool ok = s_ok != 0;
      if (ok) {
        cd bc = {0.0, 0.0};
        for (int r = 0; r < Ml; ++r) bc = cadd(bc, cmul(cconj(sb[r]), sc[r]));
        const double scl = 1.0 / sqrt(bc.re > d.eps ? bc.re : d.eps);
        for (int r = 0; r < Ml; ++r) sb[r] = {sb[r].re * scl, sb[r].im * scl};
        s_w2 = cabs2(bc) * scl * scl;  // |b^H c|^2 after the scaling
        ok = s_w2 > 0.0;
      }
      s_ok = ok;
      if (!ok) atomicOr(status, kStSingular);  // row kept; reported as DFM_E_SINGULAR
    }
    __syncthreads();
    if (!s_ok) continue;
    for (int c = tid; c < Ml; c += bd) {
      sQ[mu * Ml + c] = cconj(sb[c]);
      cd acc = {0.0, 0.0};  // u_c = (b^H Q^{-1})_c
      for (int k = 0; k < Ml; ++k) acc = cadd(acc, cmul(cconj(sb[k]), qinv(k, c)));
      su[c] = acc;
    }
    __syncthreads();
    const cd winv = cinv(su[mu]);  // 1 / (b^H c)
    for (int i = tid; i < Ml * Ml; i += bd) {
      const int r = i / Ml, c = i - r * Ml;
      const cd uc = c == mu ? csub(su[c], cd{1.0, 0.0}) : su[c];
      qinv(r, c) = csub(qinv(r, c), cmul(sc[r], cmul(uc, winv)));
    }
    if (tid == 0) s_logabs += 0.5 * log(s_w2);
  }
  __syncthreads();
  for (int i = tid; i < Ml * Ml; i += bd) {
    qb[i].re = (R)sQ[i].re;
    qb[i].im = (R)sQ[i].im;
  }
  if (tid == 0) logdet[(size_t)f * d.L + l] = s_logabs;
}

// ---------------------------------------------------------------------------------------
// The same sweep for subarrays of at most kIpvMax mics, with the V_mu inverted up front: the
// M_l covariances of the block do not depend on the sweep, so all of them are inverted together
// in LDS (Gauss-Jordan in place, without pivoting: V_mu is Hermitian positive definite), one
// elimination step for all of them at once.  Row mu then takes b = V_mu^{-1} c (c = Q^{-1} e_mu),
// the scaling of eq. (16), the new row and the rank-1 update of Q^{-1}, as in k_ip: four barriers
// per row instead of one per elimination step.
constexpr int kIpvMax = 12;

template <typename R>
__global__ __launch_bounds__(kBlock) void k_ipv(Dims d, const double* __restrict__ Vpart, cx<R>* __restrict__ Q,
                                                double* __restrict__ logdet, int* __restrict__ status) {
  const int f = blockIdx.x, l = blockIdx.y, tid = threadIdx.x, bd = blockDim.x;
  const int Ml = d.mics[l], l2 = 2 * Ml, M2 = Ml * Ml, M3 = M2 * Ml;
  extern __shared__ __align__(16) unsigned char smem[];
  const int mx = d.MLX;
  cd* sQ = reinterpret_cast<cd*>(smem);  // Q, rows replaced as the sweep goes [mx * mx]
  cd* sI = sQ + mx * mx;                  // [Q | I] -> columns Ml .. 2 Ml - 1: Q^{-1} [mx * 2 mx]
  cd* sV = sI + 2 * mx * mx;              // V_mu -> V_mu^{-1}, [mu][r][c] [mx^3]
  cd* sp = sV + mx * mx * mx;             // pivot inverses of the current step [mx]
  cd* sc = sp + mx;                       // [mx] each
  cd* sb = sc + mx;
  cd* su = sb + mx;
  __shared__ double s_logabs, s_w2;
  __shared__ int s_sing, s_ok, s_vok;

  cx<R>* qb = Q + (size_t)f * d.QF + d.qoff[l];
  for (int i = tid; i < Ml * l2; i += bd) {
    const int r = i / l2, c = i - r * l2;
    const cd q = c < Ml ? cd{(double)qb[r * Ml + c].re, (double)qb[r * Ml + c].im} : cd{c - Ml == r ? 1.0 : 0.0, 0.0};
    sI[i] = q;
    if (c < Ml) sQ[r * Ml + c] = q;
  }
  {
    const double* vp = Vpart + (size_t)f * d.SG * d.VF + d.voff[l];
    const int ns = cov_slots(d, f);
    const double invT = 1.0 / d.T;
    for (int i = tid; i < M3; i += bd) {
      const int mu = i / M2, rc = i - mu * M2, r = rc / Ml, c = rc - r * Ml;
      const int a = r < c ? r : c, b = r < c ? c : r;  // packed entry of (a, b), a <= b
      const int pj = a == b ? a : Ml + 2 * (a * Ml - a * (a + 1) / 2 + (b - a - 1));
      double re = 0.0, im = 0.0;
      for (int s = 0; s < ns; ++s) {
        re += vp[(size_t)s * d.VF + mu * M2 + pj];
        if (a != b) im += vp[(size_t)s * d.VF + mu * M2 + pj + 1];
      }
      sV[i] = {re * invT, (r < c ? im : -im) * invT};
    }
  }
  if (tid == 0) s_vok = 0;  // bit mu: V_mu had a zero pivot
  __syncthreads();
  eliminate(sI, l2, Ml, l2, &s_logabs, &s_sing);
  if (s_sing) {  // Q itself singular: keep it, report it (uniform: read after the last barrier)
    if (tid == 0) {
      atomicOr(status, kStSingular);
      logdet[(size_t)f * d.L + l] = -INFINITY;
    }
    return;
  }
  for (int c = tid; c < Ml; c += bd)
    for (int r = Ml - 1; r >= 0; --r) {
      cd acc = sI[r * l2 + Ml + c];
      for (int j = r + 1; j < Ml; ++j) acc = csub(acc, cmul(sI[r * l2 + j], sI[j * l2 + Ml + c]));
      sI[r * l2 + Ml + c] = cabs2(sI[r * l2 + r]) == 0.0 ? cd{0.0, 0.0} : cmul(acc, cinv(sI[r * l2 + r]));
    }
  // All V_mu^{-1} in place.  Step p: the pivots' inverses; every entry outside row and column p,
  // A_rc -= A_rp A_pc / A_pp; then row p (A_pc / A_pp), column p (-A_rp / A_pp) and A_pp <- 1 / A_pp.
  for (int p = 0; p < Ml; ++p) {
    for (int mu = tid; mu < Ml; mu += bd) {
      const cd pv = sV[mu * M2 + p * Ml + p];
      const bool zero = cabs2(pv) == 0.0;
      if (zero) atomicOr(&s_vok, 1 << mu);
      sp[mu] = zero ? cd{0.0, 0.0} : cinv(pv);
    }
    __syncthreads();
    for (int i = tid; i < M3; i += bd) {
      const int mu = i / M2, rc = i - mu * M2, r = rc / Ml, c = rc - r * Ml;
      if (r == p || c == p) continue;
      const cd* A = sV + mu * M2;
      sV[i] = csub(sV[i], cmul(cmul(A[r * Ml + p], sp[mu]), A[p * Ml + c]));
    }
    __syncthreads();
    for (int i = tid; i < Ml * (2 * Ml - 1); i += bd) {
      const int mu = i / (2 * Ml - 1), k = i - mu * (2 * Ml - 1);
      cd* A = sV + mu * M2;
      if (k < Ml) {  // row p, column k
        A[p * Ml + k] = k == p ? sp[mu] : cmul(A[p * Ml + k], sp[mu]);
      } else {  // column p, row k - Ml (skipping p)
        const int r = k - Ml < p ? k - Ml : k - Ml + 1;
        A[r * Ml + p] = cmul(cd{-A[r * Ml + p].re, -A[r * Ml + p].im}, sp[mu]);
      }
    }
    __syncthreads();
  }
  auto qinv = [&](int r, int c) -> cd& { return sI[r * l2 + Ml + c]; };

  for (int mu = 0; mu < Ml; ++mu) {
    // b = V_mu^{-1} c with c = Q^{-1} e_mu.
    for (int r = tid; r < Ml; r += bd) {
      const cd* A = sV + mu * M2 + r * Ml;
      cd acc = {0.0, 0.0};
      for (int k = 0; k < Ml; ++k) acc = cfma(acc, A[k], qinv(k, mu));
      sb[r] = acc;
      sc[r] = qinv(r, mu);
    }
    __syncthreads();
    if (tid == 0) {
      bool ok = !((s_vok >> mu) & 1);
      if (ok) {
        cd bc = {0.0, 0.0};
        for (int r = 0; r < Ml; ++r) bc = cadd(bc, cmul(cconj(sb[r]), sc[r]));
        const double scl = 1.0 / sqrt(bc.re > d.eps ? bc.re : d.eps);
        for (int r = 0; r < Ml; ++r) sb[r] = {sb[r].re * scl, sb[r].im * scl};
        s_w2 = cabs2(bc) * scl * scl;  // |b^H c|^2 after the scaling
        ok = s_w2 > 0.0;
      }
      s_ok = ok;
      if (!ok) atomicOr(status, kStSingular);  // row kept; reported as DFM_E_SINGULAR
    }
    __syncthreads();
    if (!s_ok) continue;
    for (int c = tid; c < Ml; c += bd) {
      sQ[mu * Ml + c] = cconj(sb[c]);
      cd acc = {0.0, 0.0};  // u_c = (b^H Q^{-1})_c
      for (int k = 0; k < Ml; ++k) acc = cadd(acc, cmul(cconj(sb[k]), qinv(k, c)));
      su[c] = acc;
    }
    __syncthreads();
    const cd winv = cinv(su[mu]);  // 1 / (b^H c)
    for (int i = tid; i < M2; i += bd) {
      const int r = i / Ml, c = i - r * Ml;
      const cd uc = c == mu ? csub(su[c], cd{1.0, 0.0}) : su[c];
      qinv(r, c) = csub(qinv(r, c), cmul(sc[r], cmul(uc, winv)));
    }
    if (tid == 0) s_logabs += 0.5 * log(s_w2);
    __syncthreads();
  }
  for (int i = tid; i < M2; i += bd) {
    qb[i].re = (R)sQ[i].re;
    qb[i].im = (R)sQ[i].im;
  }
  if (tid == 0) logdet[(size_t)f * d.L + l] = s_logabs;
}

// ---------------------------------------------------------------------------------------
// Powers P = |Q x|^2 and the slice sums of eq. (8):
//   num_W[n][k] = sum_t H[n][k][t] sum_m g P / y^2,  den_W[n][k] = sum_t H sum_m g / y.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_pw(Dims d, const cx<R>* __restrict__ X, const cx<R>* __restrict__ Q,
                                               const R* __restrict__ W, const R* __restrict__ H,
                                               const R* __restrict__ g, R* __restrict__ P, R* __restrict__ Wpart) {
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, d.T - t0);
  const int N = d.N, M = d.M;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<R>* sQ = reinterpret_cast<cx<R>*>(smem);
  R* sW = reinterpret_cast<R*>(smem + align_up(sizeof(cx<R>) * d.QF, 16));
  R* sg = sW + N * d.K;
  R* sab = sg + N * M;       // [SL][N][2]
  R* slam = sab + d.SL * N * 2;  // [SL][N]: lambda
  R* sp = slam + d.SL * N;   // [SL][M]: P / y^2
  R* sy = sp + d.SL * M;     // [SL][M]: 1 / y

  for (int i = tid; i < d.QF; i += kBlock) sQ[i] = Q[(size_t)f * d.QF + i];
  for (int i = tid; i < N * d.K; i += kBlock) {
    const int n = i / d.K, k = i - n * d.K;
    sW[i] = W[((size_t)n * d.F + f) * d.K + k];
  }
  for (int i = tid; i < N * M; i += kBlock) sg[i] = g[(size_t)f * N * M + i];
  __syncthreads();

  // lambda per (frame, source).
  for (int i = tid; i < nt * N; i += kBlock) {
    const int tl = i / N, n = i - tl * N;
    const R* hn = H + (size_t)n * d.K * d.T + t0 + tl;
    R acc = 0;
    for (int k = 0; k < d.K; ++k) acc += sW[n * d.K + k] * hn[(size_t)k * d.T];
    slam[i] = acc;
  }
  __syncthreads();
  // P = |Q x|^2, 1 / y and P / y^2 per (frame, mic): the threads of one frame share its x and
  // write its row of P together.
  for (int i = tid; i < nt * M; i += kBlock) {
    const int tl = i / M, m = i - tl * M, l = d.msub[m], Ml = d.mics[l], o = d.moff[l], mu = m - o;
    const size_t ft = (size_t)f * d.T + t0 + tl;
    const cx<R>* xr = X + ft * M + o;
    const cx<R>* qr = sQ + d.qoff[l] + mu * Ml;
    R zr = 0, zi = 0;
    for (int c = 0; c < Ml; ++c) {
      const cx<R> q = qr[c], x = xr[c];
      zr += q.re * x.re - q.im * x.im;
      zi += q.re * x.im + q.im * x.re;
    }
    const R p = zr * zr + zi * zi;
    P[ft * M + m] = p;
    R y = 0;
    for (int n = 0; n < N; ++n) y += slam[tl * N + n] * sg[n * M + m];
    const R iy = (R)1 / rmax(y, (R)d.eps);
    sp[i] = p * iy * iy;
    sy[i] = iy;
  }
  __syncthreads();
  // The per-frame coefficients of eq. (8): a_n = sum_m g P / y^2, b_n = sum_m g / y.
  for (int i = tid; i < nt * N; i += kBlock) {
    const int tl = i / N, n = i - tl * N;
    R a = 0, b = 0;
    for (int m = 0; m < M; ++m) {
      a += sg[n * M + m] * sp[tl * M + m];
      b += sg[n * M + m] * sy[tl * M + m];
    }
    sab[i * 2 + 0] = a;
    sab[i * 2 + 1] = b;
  }
  __syncthreads();

  R* out = Wpart + ((size_t)f * d.S + s) * d.N * d.K * 2;
  for (int idx = tid; idx < d.N * d.K * 2; idx += kBlock) {
    const int which = idx & 1, nk = idx >> 1;
    const int n = nk / d.K;
    const R* hr = H + (size_t)nk * d.T + t0;
    R acc = 0;
    for (int tl = 0; tl < nt; ++tl) acc += hr[tl] * sab[(tl * d.N + n) * 2 + which];
    out[idx] = acc;
  }
}

// W[n][f][k] <- W sqrt(num / max(den, eps)), sums over slices in order (eq. (8)).
template <typename R>
__global__ void k_wapply(Dims d, R* __restrict__ W, const R* __restrict__ Wpart, int* __restrict__ status) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.N * d.F * d.K) return;
  const int k = idx % d.K, nf = idx / d.K, f = nf % d.F, n = nf / d.F;
  R num = 0, den = 0;
  for (int s = 0; s < d.S; ++s) {
    const R* pp = Wpart + (((size_t)f * d.S + s) * d.N * d.K + n * d.K + k) * 2;
    num += pp[0];
    den += pp[1];
  }
  const R v = W[idx] * sqrt(num / rmax(den, (R)d.eps));
  if (d.check && !isfinite(v)) atomicOr(status, kStNonFinite);
  W[idx] = v;
}

// ---------------------------------------------------------------------------------------
// Activation update sums over a tile of FB frequencies x TB frames (eq. (9)):
//   num_H[n][k][t] = sum_f W[n][f][k] sum_m g P / y^2,  den_H = sum_f W sum_m g / y.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_h(Dims d, const R* __restrict__ W, const R* __restrict__ H,
                                              const R* __restrict__ g, const R* __restrict__ P,
                                              R* __restrict__ Hpart) {
  const int fs = blockIdx.x, tb = blockIdx.y, tid = threadIdx.x;
  const int f0 = fs * d.FB, nf = min(d.FB, d.F - f0);
  const int t0 = tb * d.TB, ntb = min(d.TB, d.T - t0);
  extern __shared__ __align__(16) unsigned char smem[];
  R* sab = reinterpret_cast<R*>(smem);  // [FB][TB][N][2]

  for (int i = tid; i < nf * ntb; i += kBlock) {
    const int fl = i / ntb, tl = i - fl * ntb;
    const int f = f0 + fl, t = t0 + tl;
    R lam[kMaxN], a[kMaxN], b[kMaxN];
    source_psd(d, W + (size_t)f * d.K, d.F * d.K, H, t, lam);
#pragma unroll
    for (int n = 0; n < kMaxN; ++n) {
      a[n] = 0;
      b[n] = 0;
    }
    const R* gf = g + (size_t)f * d.N * d.M;
    const R* pr = P + ((size_t)f * d.T + t) * d.M;
    for (int m = 0; m < d.M; ++m) {
      const R iy = (R)1 / model_var(d, lam, gf, m);
      const R piy2 = pr[m] * iy * iy;
#pragma unroll
      for (int n = 0; n < kMaxN; ++n)
        if (n < d.N) {
          a[n] += gf[n * d.M + m] * piy2;
          b[n] += gf[n * d.M + m] * iy;
        }
    }
#pragma unroll
    for (int n = 0; n < kMaxN; ++n)
      if (n < d.N) {
        sab[((fl * d.TB + tl) * d.N + n) * 2 + 0] = a[n];
        sab[((fl * d.TB + tl) * d.N + n) * 2 + 1] = b[n];
      }
  }
  __syncthreads();

  for (int idx = tid; idx < d.N * d.K * ntb * 2; idx += kBlock) {
    const int which = idx & 1;
    const int rest = idx >> 1;
    const int tl = rest % ntb, nk = rest / ntb;
    const int n = nk / d.K, k = nk - n * d.K;
    R acc = 0;
    for (int fl = 0; fl < nf; ++fl)
      acc += W[((size_t)n * d.F + f0 + fl) * d.K + k] * sab[((fl * d.TB + tl) * d.N + n) * 2 + which];
    Hpart[((((size_t)fs * d.N + n) * d.K + k) * d.T + t0 + tl) * 2 + which] = acc;
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_happly(Dims d, R* __restrict__ H, const R* __restrict__ Hpart,
                                                   int* __restrict__ status) {
  // kHaG thread groups per block of kBlock / kHaG entries: group q adds the frequency tiles
  // q, q + kHaG, ... of its entry, and the groups' partials are added in group order.
  constexpr int kHaG = 8, kHaE = kBlock / kHaG;
  __shared__ R part[2][kHaG][kHaE];
  const int e = threadIdx.x % kHaE, q = threadIdx.x / kHaE;
  const int idx = blockIdx.x * kHaE + e;
  const int total = d.N * d.K * d.T;
  R num = 0, den = 0;
  if (idx < total)
    for (int fs = q; fs < d.FS; fs += kHaG) {
      const R* pp = Hpart + ((size_t)fs * total + idx) * 2;
      num += pp[0];
      den += pp[1];
    }
  part[0][q][e] = num;
  part[1][q][e] = den;
  __syncthreads();
  if (q != 0 || idx >= total) return;
  for (int j = 1; j < kHaG; ++j) {
    num += part[0][j][e];
    den += part[1][j][e];
  }
  const R v = H[idx] * sqrt(num / rmax(den, (R)d.eps));
  if (d.check && !isfinite(v)) atomicOr(status, kStNonFinite);
  H[idx] = v;
}

// ---------------------------------------------------------------------------------------
// Diagonal SCM update slice sums (eq. (10)):
//   num_g[n][m] = sum_t lambda_tn P_tm / y_tm^2,  den_g[n][m] = sum_t lambda_tn / y_tm.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_g(Dims d, const R* __restrict__ W, const R* __restrict__ H,
                                              const R* __restrict__ g, const R* __restrict__ P,
                                              R* __restrict__ gpart) {
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, d.T - t0);
  extern __shared__ __align__(16) unsigned char smem[];
  R* sW = reinterpret_cast<R*>(smem);
  R* sg = sW + d.N * d.K;
  R* slam = sg + d.N * d.M;       // [SL][N]
  R* sr = slam + d.SL * d.N;      // [SL][M][2]

  for (int i = tid; i < d.N * d.K; i += kBlock) {
    const int n = i / d.K, k = i - n * d.K;
    sW[i] = W[((size_t)n * d.F + f) * d.K + k];
  }
  for (int i = tid; i < d.N * d.M; i += kBlock) sg[i] = g[(size_t)f * d.N * d.M + i];
  __syncthreads();

  for (int tl = tid; tl < nt; tl += kBlock) {
    const int t = t0 + tl;
    R lam[kMaxN];
    source_psd(d, sW, d.K, H, t, lam);
#pragma unroll
    for (int n = 0; n < kMaxN; ++n)
      if (n < d.N) slam[tl * d.N + n] = lam[n];
    const R* pr = P + ((size_t)f * d.T + t) * d.M;
    for (int m = 0; m < d.M; ++m) {
      const R iy = (R)1 / model_var(d, lam, sg, m);
      sr[(tl * d.M + m) * 2 + 0] = pr[m] * iy * iy;
      sr[(tl * d.M + m) * 2 + 1] = iy;
    }
  }
  __syncthreads();

  R* out = gpart + ((size_t)f * d.S + s) * d.N * d.M * 2;
  for (int idx = tid; idx < d.N * d.M * 2; idx += kBlock) {
    const int which = idx & 1, nm = idx >> 1;
    const int n = nm / d.M, m = nm - n * d.M;
    R acc = 0;
    for (int tl = 0; tl < nt; ++tl) acc += slam[tl * d.N + n] * sr[(tl * d.M + m) * 2 + which];
    out[idx] = acc;
  }
}

template <typename R>
__global__ void k_gapply(Dims d, R* __restrict__ g, const R* __restrict__ gpart, int* __restrict__ status) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int per_f = d.N * d.M;
  if (idx >= d.F * per_f) return;
  const int f = idx / per_f, nm = idx - f * per_f;
  R num = 0, den = 0;
  for (int s = 0; s < d.S; ++s) {
    const R* pp = gpart + (((size_t)f * d.S + s) * per_f + nm) * 2;
    num += pp[0];
    den += pp[1];
  }
  const R v = g[idx] * sqrt(num / rmax(den, (R)d.eps));
  if (d.check && !isfinite(v)) atomicOr(status, kStNonFinite);
  g[idx] = v;
}

// ---------------------------------------------------------------------------------------
// Cost (13), data part: per tile the FP64 sum of |Q x|^2 / y + ln y.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_nll(Dims d, const cx<R>* __restrict__ X, const cx<R>* __restrict__ Q,
                                                const R* __restrict__ W, const R* __restrict__ H,
                                                const R* __restrict__ g, double* __restrict__ nllpart) {
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, d.T - t0);
  __shared__ double red[kBlock];
  const cx<R>* qf = Q + (size_t)f * d.QF;
  const R* gf = g + (size_t)f * d.N * d.M;
  double acc = 0.0;
  for (int tl = tid; tl < nt; tl += kBlock) {
    const int t = t0 + tl;
    R lam[kMaxN];
    source_psd(d, W + (size_t)f * d.K, d.F * d.K, H, t, lam);
    const cx<R>* xr = X + ((size_t)f * d.T + t) * d.M;
    for (int l = 0; l < d.L; ++l) {
      const int Ml = d.mics[l], o = d.moff[l];
      for (int mu = 0; mu < Ml; ++mu) {
        R zr = 0, zi = 0;
        for (int c = 0; c < Ml; ++c) {
          const cx<R> q = qf[d.qoff[l] + mu * Ml + c];
          const cx<R> x = xr[o + c];
          zr += q.re * x.re - q.im * x.im;
          zi += q.re * x.im + q.im * x.re;
        }
        const R y = model_var(d, lam, gf, o + mu);
        acc += (double)((zr * zr + zi * zi) / y) + log((double)y);
      }
    }
  }
  red[tid] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) nllpart[(size_t)f * d.S + s] = red[0];
}

// ln|det Q_fl| by elimination in FP64.  Block (f, l).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_logdet(Dims d, const cx<R>* __restrict__ Q, double* __restrict__ logdet) {
  const int f = blockIdx.x, l = blockIdx.y, tid = threadIdx.x;
  const int Ml = d.mics[l];
  extern __shared__ __align__(16) unsigned char smem[];
  cd* sA = reinterpret_cast<cd*>(smem);  // [MLX * MLX]
  __shared__ double s_logabs;
  __shared__ int s_sing;
  const cx<R>* qb = Q + (size_t)f * d.QF + d.qoff[l];
  for (int i = tid; i < Ml * Ml; i += blockDim.x) sA[i] = {(double)qb[i].re, (double)qb[i].im};
  __syncthreads();
  eliminate(sA, Ml, Ml, Ml, &s_logabs, &s_sing);
  if (tid == 0) logdet[(size_t)f * d.L + l] = s_logabs;
}

// Q_fl^{-1} in FP64 by Gauss-Jordan on [Q | I].  Block (f, l).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_qinv(Dims d, const cx<R>* __restrict__ Q, cd* __restrict__ Qinv,
                                                 int* __restrict__ status) {
  const int f = blockIdx.x, l = blockIdx.y, tid = threadIdx.x, bd = blockDim.x;
  const int Ml = d.mics[l], ld = 2 * Ml;
  extern __shared__ __align__(16) unsigned char smem[];
  cd* sA = reinterpret_cast<cd*>(smem);  // [MLX * 2 MLX]
  __shared__ double s_logabs;
  __shared__ int s_sing;
  const cx<R>* qb = Q + (size_t)f * d.QF + d.qoff[l];
  for (int i = tid; i < Ml * ld; i += bd) {
    const int r = i / ld, c = i - r * ld;
    sA[i] = c < Ml ? cd{(double)qb[r * Ml + c].re, (double)qb[r * Ml + c].im} : cd{c - Ml == r ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  eliminate(sA, ld, Ml, ld, &s_logabs, &s_sing);
  if (tid == 0 && s_sing) atomicOr(status, kStSingular);
  // back substitution for all right-hand sides (one thread per column of the inverse)
  cd* out = Qinv + (size_t)f * d.QF + d.qoff[l];
  for (int c = tid; c < Ml; c += bd) {
    for (int r = Ml - 1; r >= 0; --r) {
      cd acc = sA[r * ld + Ml + c];
      for (int j = r + 1; j < Ml; ++j) acc = csub(acc, cmul(sA[r * ld + j], out[j * Ml + c]));
      out[r * Ml + c] = cmul(acc, cinv(sA[r * ld + r]));
    }
  }
}

// Multichannel Wiener filter per subarray; tile (f, slice), one frame per thread.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_sep(Dims d, const cx<R>* __restrict__ X, const cx<R>* __restrict__ Q,
                                                const cd* __restrict__ Qinv, const R* __restrict__ W,
                                                const R* __restrict__ H, const R* __restrict__ g,
                                                cx<R>* __restrict__ S) {
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, d.T - t0);
  const cx<R>* qf = Q + (size_t)f * d.QF;
  const cd* qi = Qinv + (size_t)f * d.QF;
  const R* gf = g + (size_t)f * d.N * d.M;
  for (int tl = tid; tl < nt; tl += kBlock) {
    const int t = t0 + tl;
    R lam[kMaxN];
    source_psd(d, W + (size_t)f * d.K, d.F * d.K, H, t, lam);
    const cx<R>* xr = X + ((size_t)f * d.T + t) * d.M;
    for (int l = 0; l < d.L; ++l) {
      const int Ml = d.mics[l], o = d.moff[l];
      R zr[kMaxMl], zi[kMaxMl], iy[kMaxMl];
      for (int mu = 0; mu < Ml; ++mu) {
        R ar = 0, ai = 0;
        for (int c = 0; c < Ml; ++c) {
          const cx<R> q = qf[d.qoff[l] + mu * Ml + c];
          const cx<R> x = xr[o + c];
          ar += q.re * x.re - q.im * x.im;
          ai += q.re * x.im + q.im * x.re;
        }
        zr[mu] = ar;
        zi[mu] = ai;
        iy[mu] = (R)1 / model_var(d, lam, gf, o + mu);
      }
      for (int n = 0; n < d.N; ++n) {
        cx<R>* sr = S + (((size_t)n * d.F + f) * d.T + t) * d.M + o;
        for (int a = 0; a < Ml; ++a) {
          R vr = 0, vi = 0;
          for (int mu = 0; mu < Ml; ++mu) {
            const R gain = lam[n] * gf[n * d.M + o + mu] * iy[mu];
            const cd q = qi[d.qoff[l] + a * Ml + mu];
            const R ur = gain * zr[mu], ui = gain * zi[mu];
            vr += (R)q.re * ur - (R)q.im * ui;
            vi += (R)q.re * ui + (R)q.im * ur;
          }
          sr[a].re = vr;
          sr[a].im = vi;
        }
      }
    }
  }
}

// Full Hermitian covariances from the slice sums (diagnostic export of eq. (14)).
template <typename R, typename VT>
__global__ void k_expand(Dims d, const VT* __restrict__ Vpart, cx<R>* __restrict__ V) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.F * d.VF) return;
  const int f = idx / d.VF, r = idx - f * d.VF;
  const int l = subarray_of_vidx(d, r);
  const int Ml = d.mics[l];
  const int rl = r - d.voff[l];
  const int mu = rl / (Ml * Ml);
  int a, b, part;
  packed_pair(Ml, rl - mu * Ml * Ml, a, b, part);
  double acc = 0.0;
  for (int s = 0; s < cov_slots(d, f); ++s) acc += (double)Vpart[((size_t)f * d.SG + s) * d.VF + r];
  const R v = (R)(acc / d.T);
  cx<R>* vb = V + (size_t)f * d.VC + d.voff[l] + mu * Ml * Ml;
  if (a == b) {
    vb[a * Ml + a] = {v, (R)0};
  } else if (part == 0) {
    vb[a * Ml + b].re = v;
    vb[b * Ml + a].re = v;
  } else {
    vb[a * Ml + b].im = v;
    vb[b * Ml + a].im = -v;
  }
}

__global__ void k_zero_int(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Cost (13) = sum of the data-term partials [F][S] - 2T sum of ln|det Q_fl| [F][L], in FP64 by
// one workgroup in a fixed order (strided lane sums, then a tree over the lanes), so the total
// is reproducible run to run.  With `trace`, the total is also stored at trace[c], c = *counter
// (if c is below the trace capacity), and the counter advanced: one launch per recorded
// iteration, so the index needs no host round trip and the launch can sit in a HIP graph.
constexpr int kTotThreads = 256;
__global__ __launch_bounds__(kTotThreads) void k_nll_total(Dims d, const double* __restrict__ nllpart,
                                                           const double* __restrict__ logdet,
                                                           double* __restrict__ out, double* __restrict__ trace,
                                                           int* __restrict__ counter) {
  __shared__ double sd[kTotThreads], sl[kTotThreads];
  const int tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = tid; i < d.F * d.S; i += kTotThreads) a += nllpart[i];
  for (int i = tid; i < d.F * d.L; i += kTotThreads) b += logdet[i];
  sd[tid] = a;
  sl[tid] = b;
  __syncthreads();
  for (int w = kTotThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      sd[tid] += sd[tid + w];
      sl[tid] += sl[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double tot = sd[0] - 2.0 * d.T * sl[0];
    *out = tot;
    if (trace) {
      const int c = *counter;
      if (c < DFM_TRACE_CAPACITY) trace[c] = tot;
      *counter = c + 1;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Host-side launchers.
template <typename R>
static size_t smem_gram(const Dims& d) {
  return align_up(sizeof(R) * (d.N * d.K + d.N * d.M + d.SL * d.M), 16) + sizeof(cx<R>) * d.SL * d.M;
}
template <typename R>
static size_t smem_pw(const Dims& d) {
  return align_up(sizeof(cx<R>) * d.QF, 16) + sizeof(R) * (d.N * d.K + d.N * d.M + d.SL * (3 * d.N + 2 * d.M));
}
template <typename R>
static size_t smem_g(const Dims& d) {
  return sizeof(R) * (d.N * d.K + d.N * d.M + d.SL * d.N + d.SL * d.M * 2);
}
template <typename R>
static size_t smem_h(const Dims& d) {
  return sizeof(R) * d.FB * d.TB * d.N * 2;
}

// Dynamic LDS of the generic IP sweep, ln|det Q| and Q^{-1} kernels: sized for the largest subarray.
static size_t ip_smem(const Dims& d) {
  const size_t m = d.MLX;
  return sizeof(cd) * (m * m + 2 * m * m + m * (m + 1) + 3 * m);
}
static size_t ipv_smem(const Dims& d) {
  const size_t m = d.MLX;
  return sizeof(cd) * (3 * m * m + m * m * m + 4 * m);
}
static size_t logdet_smem(const Dims& d) { return sizeof(cd) * d.MLX * d.MLX; }
static size_t qinv_smem(const Dims& d) { return sizeof(cd) * 2 * d.MLX * d.MLX; }

static int ip_threads(const Dims& d) {
  int mx = 1;
  for (int l = 0; l < d.L; ++l) mx = d.mics[l] > mx ? d.mics[l] : mx;
  return mx * mx <= 64 ? 64 : kBlock;
}

static inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

template <typename R>
static hipError_t kernel_impl(const Dims& d, const Buffers& b, int kid, hipStream_t s) {
  const cx<R>* X = static_cast<const cx<R>*>(b.X);
  cx<R>* Q = static_cast<cx<R>*>(b.Q);
  R* g = static_cast<R*>(b.g);
  R* W = static_cast<R*>(b.W);
  R* H = static_cast<R*>(b.H);
  R* P = static_cast<R*>(b.P);
  const dim3 tiles(d.F, d.S);
  switch (kid) {
    case kKGram:
      hipLaunchKernelGGL(k_gram<R>, tiles, dim3(kBlock), smem_gram<R>(d), s, d, X, W, H, g,
                         static_cast<double*>(b.Vpart));
      break;
    case kKIp:
      if (d.MLX > 4 && d.MLX <= kIpvMax)
        hipLaunchKernelGGL(k_ipv<R>, dim3(d.F, d.L), dim3(kBlock), ipv_smem(d), s, d,
                           static_cast<const double*>(b.Vpart), Q, b.logdet, b.status);
      else
        hipLaunchKernelGGL(k_ip<R>, dim3(d.F, d.L), dim3(ip_threads(d)), ip_smem(d), s, d,
                           static_cast<const double*>(b.Vpart), Q, b.logdet, b.status);
      break;
    case kKPw:
      hipLaunchKernelGGL(k_pw<R>, tiles, dim3(kBlock), smem_pw<R>(d), s, d, X, Q, W, H, g, P,
                         static_cast<R*>(b.Wpart));
      break;
    case kKWApply:
      hipLaunchKernelGGL(k_wapply<R>, dim3(cdiv((size_t)d.N * d.F * d.K, kBlock)), dim3(kBlock), 0, s, d, W,
                         static_cast<const R*>(b.Wpart), b.status);
      break;
    case kKH:
      hipLaunchKernelGGL(k_h<R>, dim3(d.FS, d.TBN), dim3(kBlock), smem_h<R>(d), s, d, W, H, g, P,
                         static_cast<R*>(b.Hpart));
      break;
    case kKHApply:
      hipLaunchKernelGGL(k_happly<R>, dim3(cdiv((size_t)d.N * d.K * d.T, kBlock / 8)), dim3(kBlock), 0, s, d, H,
                         static_cast<const R*>(b.Hpart), b.status);
      break;
    case kKG:
      hipLaunchKernelGGL(k_g<R>, tiles, dim3(kBlock), smem_g<R>(d), s, d, W, H, g, P, static_cast<R*>(b.gpart));
      break;
    case kKGApply:
      hipLaunchKernelGGL(k_gapply<R>, dim3(cdiv((size_t)d.F * d.N * d.M, kBlock)), dim3(kBlock), 0, s, d, g,
                         static_cast<const R*>(b.gpart), b.status);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename R>
static hipError_t nll_impl(const Dims& d, const Buffers& b, hipStream_t s) {
  const cx<R>* X = static_cast<const cx<R>*>(b.X);
  const cx<R>* Q = static_cast<const cx<R>*>(b.Q);
  hipLaunchKernelGGL(k_nll<R>, dim3(d.F, d.S), dim3(kBlock), 0, s, d, X, Q, static_cast<const R*>(b.W),
                     static_cast<const R*>(b.H), static_cast<const R*>(b.g), b.nllpart);
  hipLaunchKernelGGL(k_logdet<R>, dim3(d.F, d.L), dim3(ip_threads(d)), logdet_smem(d), s, d, Q, b.logdet);
  return hipGetLastError();
}

template <typename R>
static hipError_t sep_impl(const Dims& d, const Buffers& b, void* S, hipStream_t s) {
  const cx<R>* X = static_cast<const cx<R>*>(b.X);
  const cx<R>* Q = static_cast<const cx<R>*>(b.Q);
  hipLaunchKernelGGL(k_qinv<R>, dim3(d.F, d.L), dim3(ip_threads(d)), qinv_smem(d), s, d, Q, static_cast<cd*>(b.Qinv),
                     b.status);
  hipLaunchKernelGGL(k_sep<R>, dim3(d.F, d.S), dim3(kBlock), 0, s, d, X, Q, static_cast<const cd*>(b.Qinv),
                     static_cast<const R*>(b.W), static_cast<const R*>(b.H), static_cast<const R*>(b.g),
                     static_cast<cx<R>*>(S));
  return hipGetLastError();
}

template <typename R>
static hipError_t cov_impl(const Dims& d, const Buffers& b, void* V, hipStream_t s) {
  // The plan's own covariance kernel (both write the same packed slice-sum layout).
  if (d.fast >= 0) {
    const int dt = sizeof(R) == 4 ? DFM_C64 : DFM_C128;
    hipError_t e = fast_launch(d, b, dt, kFLam, s);
    if (e == hipSuccess) e = fast_launch(d, b, dt, kFGram, s);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_gram<R>, dim3(d.F, d.S), dim3(kBlock), smem_gram<R>(d), s, d,
                       static_cast<const cx<R>*>(b.X), static_cast<const R*>(b.W), static_cast<const R*>(b.H),
                       static_cast<const R*>(b.g), static_cast<double*>(b.Vpart));
  }
  hipLaunchKernelGGL((k_expand<R, double>), dim3(cdiv((size_t)d.F * d.VF, kBlock)), dim3(kBlock), 0, s, d,
                     static_cast<const double*>(b.Vpart), static_cast<cx<R>*>(V));
  return hipGetLastError();
}

hipError_t launch_init(const Dims& d, const Buffers& b, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, b.status, 16);
  return hipGetLastError();
}

__global__ void k_copy_int(const int* src, int* dst) {
  if (threadIdx.x == 0) *dst = *src;
}

hipError_t launch_copy_status(const Buffers& b, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_int, dim3(1), dim3(64), 0, s, b.status, out);
  return hipGetLastError();
}

hipError_t launch_qinv(const Dims& d, const Buffers& b, int dtype, hipStream_t s) {
  if (dtype == DFM_C64)
    hipLaunchKernelGGL(k_qinv<float>, dim3(d.F, d.L), dim3(ip_threads(d)), qinv_smem(d), s, d,
                       static_cast<const cx<float>*>(b.Q), static_cast<cd*>(b.Qinv), b.status);
  else
    hipLaunchKernelGGL(k_qinv<double>, dim3(d.F, d.L), dim3(ip_threads(d)), qinv_smem(d), s, d,
                       static_cast<const cx<double>*>(b.Q), static_cast<cd*>(b.Qinv), b.status);
  return hipGetLastError();
}

hipError_t launch_clear_status(const Buffers& b, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, b.status, 1);
  return hipGetLastError();
}

hipError_t launch_nll_total(const Dims& d, const Buffers& b, double* out, bool trace, hipStream_t s) {
  hipLaunchKernelGGL(k_nll_total, dim3(1), dim3(kTotThreads), 0, s, d, b.nllpart, b.logdet, out,
                     trace ? b.trace : nullptr, b.status + kTraceSlot);
  return hipGetLastError();
}

hipError_t launch_kernel(const Dims& d, const Buffers& b, int dtype, int kid, hipStream_t s) {
  if (kid >= kFGram) return fast_launch(d, b, dtype, kid, s);
  return dtype == DFM_C64 ? kernel_impl<float>(d, b, kid, s) : kernel_impl<double>(d, b, kid, s);
}

const char* kernel_name(int kid) {
  static const char* names[kNumKernels] = {"k_gram",   "k_ip",    "k_pw",    "k_wapply",  "k_h",
                                           "k_happly", "k_g",     "k_gapply", "k_gram_f", "k_ip_f",
                                           "k_pw_f",   "k_wgemm_f", "k_h_f",  "k_hgemm_f", "k_g_f",
                                           "k_lam_f",  "k_gfin_f", "k_hlam_f"};
  return kid >= 0 && kid < kNumKernels ? names[kid] : nullptr;
}

// Kernels of each sub-step, in launch order.
int stage_kernels(const Dims& d, int stage, int* kids) {
  if (d.fast >= 0) {
    switch (stage) {
      case DFM_STAGE_IP: kids[0] = kFGram; kids[1] = kFIp; return 2;
      case DFM_STAGE_W: kids[0] = kFPw; kids[1] = kFWGemm; return 2;
      case DFM_STAGE_H:
        kids[0] = kFH;
        kids[1] = kFHGemm;
        if (d.HC <= 1) return 2;
        kids[2] = kFHLam;
        return 3;
      case DFM_STAGE_G:
        kids[0] = kFG;
        if (g_update_deferred(d)) return 1;
        kids[1] = kFGFin;
        return 2;
    }
    return 0;
  }
  switch (stage) {
    case DFM_STAGE_IP: kids[0] = kKGram; kids[1] = kKIp; return 2;
    case DFM_STAGE_W: kids[0] = kKPw; kids[1] = kKWApply; return 2;
    case DFM_STAGE_H: kids[0] = kKH; kids[1] = kKHApply; return 2;
    case DFM_STAGE_G: kids[0] = kKG; kids[1] = kKGApply; return 2;
  }
  return 0;
}

int iteration_kernels(const Dims& d, int* kids) {
  int n = 0;
  for (int stage = DFM_STAGE_IP; stage <= DFM_STAGE_G; ++stage) n += stage_kernels(d, stage, kids + n);
  return n;
}

hipError_t launch_nll(const Dims& d, const Buffers& b, int dtype, hipStream_t s) {
  if (d.fast >= 0 && d.ML <= 4) return fast_finish(d, b, dtype, false, nullptr, s);
  return dtype == DFM_C64 ? nll_impl<float>(d, b, s) : nll_impl<double>(d, b, s);
}

hipError_t launch_separate(const Dims& d, const Buffers& b, int dtype, void* S, hipStream_t s) {
  if (d.fast >= 0 && d.ML <= 4) return fast_finish(d, b, dtype, true, S, s);
  return dtype == DFM_C64 ? sep_impl<float>(d, b, S, s) : sep_impl<double>(d, b, S, s);
}

hipError_t launch_covariances(const Dims& d, const Buffers& b, int dtype, void* V, hipStream_t s) {
  return dtype == DFM_C64 ? cov_impl<float>(d, b, V, s) : cov_impl<double>(d, b, V, s);
}

}  // namespace dfm
