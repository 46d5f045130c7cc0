// Shape-specialised kernels of distributed FastMNMF for gfx950.
//
// Used when every subarray has the same size ML and (N, K, ML, L) is one of the compiled
// sets (DFM_FAST_SETS below).  All four are compile-time constants, so every per-frame
// array (lambda_n, y_m, |Qx|^2, x) lives in registers with a compile-time size and every
// loop over sources, bases and mics is unrolled.  Global loads that feed a computation
// are issued as one batch behind a scheduling barrier (left alone, the scheduler trades
// them for occupancy and waits on each load in turn).
//
// One iteration is eight kernels: the five below, k_happly_f, and the generic W and g
// apply kernels, which sum the per-tile partials in a fixed order (so every result is
// deterministic run to run) and update W and g.  Finishing the reductions inside the
// streaming kernels with a last-arriving workgroup was measured slower on gfx950: the
// device-scope release/acquire it needs writes back and invalidates L2 in every
// workgroup.
//
//   k_ht_f    frame-major copy of H (once per call; afterwards the H update keeps it).
//   k_lam_f   lambda = W H at every frame (once per call; afterwards k_g_f refreshes it).
//   k_gram_f  tile (f, time slice), 128 threads.  1/y per frame on the vector units,
//             then the weighted covariances of eq. (14) as a real contraction over
//             frames on the matrix cores (v_mfma 16x16x4: rows = mu, columns = packed
//             Hermitian entries of x x^H, K = 4 frames).
//   k_ip_f    one lane per (f, subarray): FP64 IP sweep of eqs. (15)-(16) (M_l <= 4;
//             larger blocks use the cooperative generic kernel).
//   k_pw_f    tile (f, time slice), 128 threads.  P = |Q x|^2 and the per-frame sums of
//             eq. (8); the contraction with H over frames reads H staged in LDS.
//   k_h_f     2 x 16 bins x 16 frames per 4-wave workgroup.  lambda = W H and the sum
//             over frequencies of eq. (9) are both 16x16x4 matrix-core contractions.
//   k_happly_f  H update of eq. (9) from the frequency-group partials (H and its copy).
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

// num = sum_t c[t] a[t], den = sum_t c[t] b[t] over ntp (a multiple of 4) frames of three
// LDS rows, read four frames per access (rows are 4-element aligned).
template <typename R>
__device__ __forceinline__ void dot2_frames(const R* c, const R* a, const R* b, int ntp, R& num, R& den) {
  typedef R v4r __attribute__((ext_vector_type(4)));
  R n0 = 0, n1 = 0, d0 = 0, d1 = 0;
  const int nb = ntp >> 2;
  for (int q0 = 0; q0 < nb; q0 += 4) {
    v4r cv[4], av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = min(q0 + u, nb - 1) * 4;  // clamped in bounds; extra blocks are zeroed below
      cv[u] = *reinterpret_cast<const v4r*>(c + q);
      av[u] = *reinterpret_cast<const v4r*>(a + q);
      bv[u] = *reinterpret_cast<const v4r*>(b + q);
      if (q0 + u >= nb) cv[u] = v4r{0, 0, 0, 0};
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      n0 += cv[u].x * av[u].x + cv[u].z * av[u].z;
      n1 += cv[u].y * av[u].y + cv[u].w * av[u].w;
      d0 += cv[u].x * bv[u].x + cv[u].z * bv[u].z;
      d1 += cv[u].y * bv[u].y + cv[u].w * bv[u].w;
    }
  }
  num = n0 + n1;
  den = d0 + d1;
}

// H[n][k][t] for every (n, k) at one frame, from the frame-major copy Ht[t][n*K + k]
// (one batch of 16-byte loads).
template <typename R, int NK>
__device__ __forceinline__ void load_h_column(R (&hv)[NK], const R* __restrict__ Ht, int t) {
  load16<R, NK>(hv, Ht + (size_t)t * NK);
}

// ------------------------------------------------------------------------------------
// FP64 IP sweep of one subarray block (M_l <= 4), eqs. (15)-(16), by one lane.  The lane's
// Q_fl and the covariance of the current row live in LDS slots laid out element-major,
// lane-minor (element e of lane i at e * 64 + i, so a wave's accesses are conflict-free);
// the system A = Q V_mu is eliminated in registers.
// vp: packed slice sums of the block, [slice (stride vstride)][mu][M_l^2]; V = sum / T.
template <typename R, int ML>
__device__ void ip_sweep_lane(const R* vp, size_t vstride, int S, double invT, cd* q, cd* v, double eps,
                              int* status) {
  constexpr int ML2 = ML * ML;
#define QS(r, c) q[((r) * ML + (c)) * 64]
#define VS(r, c) v[((r) * ML + (c)) * 64]
#pragma unroll
  for (int mu = 0; mu < ML; ++mu) {
    double vs[ML2];
#pragma unroll
    for (int j = 0; j < ML2; ++j) vs[j] = 0.0;
    for (int s = 0; s < S; ++s) {
      R part[ML2];
#pragma unroll
      for (int j = 0; j < ML2; ++j) part[j] = vp[s * vstride + mu * ML2 + j];
#pragma unroll
      for (int j = 0; j < ML2; ++j) vs[j] += (double)part[j];
    }
#pragma unroll
    for (int j = 0; j < ML2; ++j) {
      int a, b, part;
      packed_pair(ML, j, a, b, part);
      const double val = vs[j] * invT;
      if (a == b) {
        VS(a, a) = {val, 0.0};
      } else if (part == 0) {
        VS(a, b).re = val;
        VS(b, a).re = val;
      } else {
        VS(a, b).im = val;
        VS(b, a).im = -val;
      }
    }
    cd A[ML][ML + 1];
#pragma unroll
    for (int r = 0; r < ML; ++r) {
#pragma unroll
      for (int c = 0; c < ML; ++c) {
        cd acc = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < ML; ++j) acc = cadd(acc, cmul(QS(r, j), VS(j, c)));
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
        const double val = cabs2(A[r][p]);
        if (val > best) {
          best = val;
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
      for (int b = 0; b < ML; ++b) vb = cadd(vb, cmul(VS(a, b), bsol[b]));
      sv += bsol[a].re * vb.re + bsol[a].im * vb.im;
    }
    const double sc = 1.0 / sqrt(sv > eps ? sv : eps);
#pragma unroll
    for (int c = 0; c < ML; ++c) QS(mu, c) = {bsol[c].re * sc, -bsol[c].im * sc};
  }
#undef QS
#undef VS
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
//
// Per-frame operand rows live in LDS, frame-major, with row strides padded so that the
// 16-byte row writes of one frame per thread are free of bank conflicts:
//   sInv[t][m] = 1 / y_ftm, and per subarray either the packed entries of x^(l) x^(l)H
//   (M_l <= 4, formed once per frame) or the x tile itself (larger blocks, whose
//   M_l^2 packed reals per frame would not fit).
// FP32 with M_l <= 4: one v_mfma_f32_4x4x1 (16 independent 4x4 blocks) per frame, block
// b = (subarray, group of 4 packed entries), rows = mu; the frames of a slice are split
// over the two waves and their sums combined through LDS.
// Otherwise: v_mfma 16x16x4 per subarray and 16 packed entries, K = 4 frames.

// Row stride (elements) >= n whose 16-byte row segments start in distinct bank groups.
template <typename R>
constexpr int padded(int n) {
  return sizeof(R) == 4 ? n + ((4 - n % 8) + 8) % 8 : n + ((2 - n % 4) + 4) % 4;
}

template <typename R, int N, int K, int ML, int L>
struct GramShape {
  static constexpr int M = ML * L, ML2 = ML * ML, OF = L * ML2;
  static constexpr bool kPre = ML <= 4;
  static constexpr bool kBlocks = kPre && sizeof(R) == 4;  // 4x4x1 matrix-core path
  static constexpr int MP = padded<R>(M);
  static constexpr int OP = kPre ? padded<R>(OF) : padded<R>(2 * M);
  static constexpr int JG4 = (ML2 + 3) / 4;           // groups of 4 packed entries per subarray
  static constexpr int NG = (L * JG4 + 15) / 16;      // 4x4x1 ops per frame
};

template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(kT) void k_gram_f(Dims d, const cx<R>* __restrict__ X,
                                               const R* __restrict__ lamin, const R* __restrict__ g,
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
    load16<R, 2 * M>(xv, reinterpret_cast<const R*>(X + ((size_t)f * T + t0 + tid) * M));
#pragma unroll
    for (int n = 0; n < N; ++n) lam[n] = lamin[((size_t)f * N + n) * T + t0 + tid];
  } else {  // padding frames contribute zero products
#pragma unroll
    for (int i = 0; i < 2 * M; ++i) xv[i] = 0;
#pragma unroll
    for (int n = 0; n < N; ++n) lam[n] = 0;
  }
  if (tid < N * M) gv = g[(size_t)f * N * M + tid];
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
          for (int j = 0; j < ML2; ++j) {
            int a, b, part;
            packed_pair(ML, j, a, b, part);
            const R ar = xv[2 * (l * ML + a)], ai = xv[2 * (l * ML + a) + 1];
            const R br = xv[2 * (l * ML + b)], bi = xv[2 * (l * ML + b) + 1];
            op[l * ML2 + j] = part == 0 ? ar * br + ai * bi : ai * br - ar * bi;
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

  if constexpr (G::kBlocks) {
    // Lane i, op group q: block b = 16 q + i / 4 = (subarray l, entry group jg); A row
    // (mu) and B column (entry) = i % 4.  Frames of the slice alternate between waves.
    constexpr int JG4 = G::JG4, NG = G::NG;
    const int sub = lane & 3;
    v4 acc[NG];
    int aoff[NG], boff[NG];
    bool av_ok[NG], bv_ok[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      acc[q] = v4{0, 0, 0, 0};
      const int b = 16 * q + (lane >> 2), l = b / JG4, jg = b - l * JG4, j = 4 * jg + sub;
      av_ok[q] = l < L && sub < ML;
      bv_ok[q] = l < L && j < ML2;
      aoff[q] = av_ok[q] ? l * ML + sub : 0;
      boff[q] = bv_ok[q] ? l * ML2 + j : 0;
    }
    const int half = ((ntp >> 1) + 3) & ~3;  // frames of wave 0; wave 1 takes the rest
    const int fb = wave == 0 ? 0 : half, fe = wave == 0 ? min(half, ntp) : ntp;
    for (int t4 = fb; t4 < fe; t4 += 4) {
      R av[4][NG], bv[4][NG];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < NG; ++q) {
          const R a = sInv[(t4 + u) * MP + aoff[q]], b = sOp[(t4 + u) * OP + boff[q]];
          av[u][q] = av_ok[q] ? a : (R)0;
          bv[u][q] = bv_ok[q] ? b : (R)0;
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < NG; ++q) acc[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[u][q], bv[u][q], acc[q], 0, 0, 0);
    }
    // Combine the two waves (LDS area of sInv is free now) and store the slice sums.
    __syncthreads();
    R* sRed = sInv;  // [NG][64][4]
    if (wave == 1)
#pragma unroll
      for (int q = 0; q < NG; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) sRed[(q * 64 + lane) * 4 + r] = acc[q][r];
    __syncthreads();
    if (wave == 0) {
      R* out = Vpart + ((size_t)f * d.S + s) * d.VF;
#pragma unroll
      for (int q = 0; q < NG; ++q) {
        const int b = 16 * q + (lane >> 2), l = b / JG4, jg = b - l * JG4, j = 4 * jg + sub;
        if (l < L && j < ML2)
#pragma unroll
          for (int r = 0; r < ML; ++r)
            out[(size_t)l * ML * ML2 + r * ML2 + j] = acc[q][r] + sRed[(q * 64 + lane) * 4 + r];
      }
    }
  } else {
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
}

// Frame-major copy of the activations: Ht[t][n*K + k] = H[n][k][t].
template <typename R, int NK>
__global__ __launch_bounds__(kT) void k_ht_f(Dims d, const R* __restrict__ H, R* __restrict__ Ht) {
  const int t = blockIdx.x * kT + threadIdx.x;
  if (t >= d.T) return;
  R hv[NK];
#pragma unroll
  for (int i = 0; i < NK; ++i) hv[i] = H[(size_t)i * d.T + t];
  sched_fence();
  constexpr int E = V16<R>::E;
#pragma unroll
  for (int i = 0; i < NK / E; ++i) {
    typename V16<R>::type v;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = hv[i * E + e];
    reinterpret_cast<typename V16<R>::type*>(Ht + (size_t)t * NK)[i] = v;
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

// Activation update, eq. (9): H <- H sqrt(num / max(den, eps)) with num, den summed over
// the frequency-group partials in order; writes H and its frame-major copy.  W is final
// for the iteration at this point, so lambda = W H (eq. (2)) for the new H is formed here
// too (it serves the eq. (10) sums and the next iteration's covariances and powers).
// Workgroup: one source n, 16 frames.
template <typename R, int N, int K>
__global__ __launch_bounds__(64 * kLamWaves) void k_happly_f(Dims d, const R* __restrict__ W, R* __restrict__ H,
                                                             R* __restrict__ Ht, const R* __restrict__ Hpart,
                                                             R* __restrict__ lam, int* __restrict__ status) {
  constexpr int NK = N * K, KS = (K + 3) / 4;
  __shared__ R sHn[4 * KS * 16];
  const int n = blockIdx.x, t0 = blockIdx.y * 16, tid = threadIdx.x;
  const int tl = tid & 15, t = t0 + tl;
  for (int k = tid >> 4; k < 4 * KS; k += 4 * kLamWaves) {
    R v = 0;
    if (k < K && t < d.T) {
      const size_t idx = ((size_t)n * K + k) * d.T + t;
      R num = 0, den = 0;
      for (int q = 0; q < d.FG; ++q) {
        const R* pp = Hpart + (((size_t)q * NK + n * K + k) * d.T + t) * 2;
        num += pp[0];
        den += pp[1];
      }
      v = H[idx] * sqrt(num / rmax(den, (R)d.eps));
      if (!isfinite(v)) atomicOr(status, kStNonFinite);
      H[idx] = v;
      Ht[(size_t)t * NK + n * K + k] = v;
    }
    sHn[k * 16 + tl] = v;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  for (int f0 = wave * 16; f0 < d.F; f0 += 16 * kLamWaves) lambda_tile<R, N, K>(d, W, sHn, n, f0, t0, lane, lam);
}

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

// IP sweep, eqs. (15)-(16), one lane per (f, subarray) block of size M_l <= 4, in FP64;
// then ln|det Q_fl| for the cost (13).
template <typename R, int ML>
__global__ __launch_bounds__(64) void k_ip_f(Dims d, const R* __restrict__ Vpart, cx<R>* __restrict__ Q,
                                             double* __restrict__ logdet, int* __restrict__ status) {
  constexpr int ML2 = ML * ML;
  __shared__ cd sQ[ML2 * 64];
  __shared__ cd sV[ML2 * 64];
  const int idx = blockIdx.x * 64 + threadIdx.x;
  if (idx >= d.F * d.L) return;
  const int f = idx / d.L, l = idx - f * d.L;
  cd* q = sQ + threadIdx.x;
  cx<R>* qb = Q + (size_t)f * d.QF + l * ML2;
  {
    cx<R> qv[ML2];
#pragma unroll
    for (int e = 0; e < ML2; ++e) qv[e] = qb[e];
#pragma unroll
    for (int e = 0; e < ML2; ++e) q[e * 64] = {(double)qv[e].re, (double)qv[e].im};
  }
  ip_sweep_lane<R, ML>(Vpart + (size_t)f * d.S * d.VF + (size_t)l * ML * ML2, d.VF, d.S, 1.0 / d.T, q,
                       sV + threadIdx.x, d.eps, status);
  cd A[ML][ML];
#pragma unroll
  for (int r = 0; r < ML; ++r)
#pragma unroll
    for (int c = 0; c < ML; ++c) {
      const cd qq = q[(r * ML + c) * 64];
      const cx<R> o = {(R)qq.re, (R)qq.im};
      qb[r * ML + c] = o;
      A[r][c] = {(double)o.re, (double)o.im};
    }
  logdet[idx] = logabsdet_lane<ML>(A);
}

// ------------------------------------------------------------------------------------
// P = |Q x|^2 and the eq. (8) sums per (f, slice).  Per frame: the powers, 1/y, and
// a_n = sum_m g_nm P_m / y_m^2, b_n = sum_m g_nm / y_m, stored frame-major in LDS.  Then
// num/den[n][k] = sum_t H[n][k][t] (a_n, b_n)[t]: in FP32 on the 4x4x1 matrix-core blocks
// (block = (n, group of 4 bases), rows = bases, columns = (a_n, b_n, -, -)), one op per
// frame and 16 blocks, with H read from its frame-major copy; frames alternate between
// the two waves.
template <typename R, int N, int K, int ML, int L>
struct PwShape {
  static constexpr int M = ML * L, NK = N * K, ML2 = ML * ML, QF = L * ML2;
  static constexpr int NP = (N + 3) & ~3;
  static constexpr int CP = padded<R>(2 * NP);  // LDS row: a_0 .. a_{NP-1}, b_0 .. b_{NP-1}
  static constexpr int KG = K / 4;
  static constexpr int NI = (N * KG + 15) / 16;  // 4x4x1 ops per frame
};

template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(kT) void k_pw_f(Dims d, const cx<R>* __restrict__ X, const cx<R>* __restrict__ Q,
                                             const R* __restrict__ lamin, const R* __restrict__ Ht,
                                             const R* __restrict__ g, R* __restrict__ P, R* __restrict__ Wpart) {
  typedef PwShape<R, N, K, ML, L> S_;
  constexpr int M = S_::M, NK = S_::NK, ML2 = S_::ML2, QF = S_::QF, NP = S_::NP, CP = S_::CP;
  constexpr int E = V16<R>::E;
  static_assert(K % 4 == 0 && (2 * M) % E == 0 && M % E == 0 && (2 * NP) % E == 0, "shape");
  typedef typename V16<R>::type vt;
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int T = d.T;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, T - t0);
  const int ntp = (nt + 3) & ~3;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<R>* sQ = reinterpret_cast<cx<R>*>(smem);
  R* sg = reinterpret_cast<R*>(smem + align_up(sizeof(cx<R>) * QF, 16));
  R* sC = reinterpret_cast<R*>(smem + align_up(sizeof(cx<R>) * QF, 16) + align_up(sizeof(R) * N * M, 16));
  R* sRed = sC + (size_t)d.SLP * CP;  // FP32: [NI][64][4]

  // One batch of loads: x and lambda at this thread's frame.
  R xv[2 * M], lam[N];
  if (tid < nt) {
    load16<R, 2 * M>(xv, reinterpret_cast<const R*>(X + ((size_t)f * T + t0 + tid) * M));
#pragma unroll
    for (int n = 0; n < N; ++n) lam[n] = lamin[((size_t)f * N + n) * T + t0 + tid];
  } else {
#pragma unroll
    for (int i = 0; i < 2 * M; ++i) xv[i] = 0;
#pragma unroll
    for (int n = 0; n < N; ++n) lam[n] = 0;
  }
  for (int i = tid; i < QF; i += kT) sQ[i] = Q[(size_t)f * QF + i];
  for (int i = tid; i < N * M; i += kT) sg[i] = g[(size_t)f * N * M + i];
  sched_fence();
  __syncthreads();

  if (tid < ntp) {
    R a[NP], b[NP], pv[M];
#pragma unroll
    for (int n = 0; n < NP; ++n) {
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
        const R iy = tid < nt ? rcp(rmax(y, (R)d.eps)) : (R)0;
        const R piy2 = p * iy * iy;
#pragma unroll
        for (int n = 0; n < N; ++n) {
          a[n] += sg[n * M + m] * piy2;
          b[n] += sg[n * M + m] * iy;
        }
      }
    }
    if (tid < nt) store16_nt<R, M>(P + ((size_t)f * T + t0 + tid) * M, pv);
#pragma unroll
    for (int i = 0; i < NP / E; ++i) {
      vt va, vb;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        va[e] = a[i * E + e];
        vb[e] = b[i * E + e];
      }
      reinterpret_cast<vt*>(sC + (size_t)tid * CP)[i] = va;
      reinterpret_cast<vt*>(sC + (size_t)tid * CP + NP)[i] = vb;
    }
  }
  __syncthreads();

  R* out = Wpart + ((size_t)f * d.S + s) * NK * 2;
  if constexpr (sizeof(R) == 4) {
    constexpr int NI = S_::NI, KG = S_::KG;
    typedef float v4f __attribute__((ext_vector_type(4)));
    const int sub = lane & 3;
    v4f acc[NI];
    int hcol[NI], coff[NI];
    bool aok[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      acc[q] = v4f{0, 0, 0, 0};
      const int blk = 16 * q + (lane >> 2), n = blk / KG;
      aok[q] = blk < N * KG;
      hcol[q] = aok[q] ? 64 * q + lane : 0;  // = n * K + 4 * (blk % KG) + sub
      coff[q] = (aok[q] && sub < 2) ? sub * NP + n : -1;
    }
    const int half = ((ntp >> 1) + 3) & ~3;
    const int fb = wave == 0 ? 0 : half, fe = wave == 0 ? min(half, ntp) : ntp;
    const R* hbase = Ht + (size_t)t0 * NK;
    for (int t4 = fb; t4 < fe; t4 += 4) {
      R av[4][NI], bv[4][NI];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int tt = min(t4 + u, nt - 1);  // padding frames: any in-bounds row (their b is zero)
#pragma unroll
        for (int q = 0; q < NI; ++q) av[u][q] = hbase[(size_t)tt * NK + hcol[q]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < NI; ++q) {
          const R c = sC[(size_t)(t4 + u) * CP + (coff[q] < 0 ? 0 : coff[q])];
          bv[u][q] = coff[q] < 0 ? (R)0 : c;
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < NI; ++q) acc[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[u][q], bv[u][q], acc[q], 0, 0, 0);
    }
    if (wave == 1)
#pragma unroll
      for (int q = 0; q < NI; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) sRed[(q * 64 + lane) * 4 + r] = acc[q][r];
    __syncthreads();
    if (wave == 0)
#pragma unroll
      for (int q = 0; q < NI; ++q) {
        if (coff[q] < 0) continue;
        const int blk = 16 * q + (lane >> 2), n = blk / KG, kg = blk - n * KG;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          out[(n * K + 4 * kg + r) * 2 + sub] = acc[q][r] + sRed[(q * 64 + lane) * 4 + r];
      }
  } else {
    for (int o = tid; o < NK; o += kT) {
      const int n = o / K;
      R num = 0, den = 0;
      for (int tt = 0; tt < nt; ++tt) {
        const R h = Ht[(size_t)(t0 + tt) * NK + o];
        num += h * sC[(size_t)tt * CP + n];
        den += h * sC[(size_t)tt * CP + NP + n];
      }
      out[o * 2 + 0] = num;
      out[o * 2 + 1] = den;
    }
  }
}

// ------------------------------------------------------------------------------------
// Activation update sums, eq. (9).  A workgroup of 4 waves covers kHCPW chunks of 16 bins
// for one block of 16 frames.  Per chunk: lambda = W H by the matrix cores (each wave
// holds the 16 x 16 tile in the accumulator layout); wave w then computes a' and b' of
// eq. (9) for the (f, t) pair in accumulator row w of every lane (one pair per lane);
// finally the sums over the chunk's bins, num/den[n][k][t] = sum_f W[n][f][k] (a', b'),
// run on the matrix cores with the sources split across the waves.
constexpr int kHCPW = 2;  // 16-bin chunks per activation workgroup

template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(256) void k_h_f(Dims d, const R* __restrict__ W, const R* __restrict__ H,
                                             const R* __restrict__ g, const R* __restrict__ P,
                                             R* __restrict__ Hpart) {
  constexpr int M = ML * L, NK = N * K;
  constexpr int KS = (K + 3) / 4;    // 4-deep steps over bases for lambda = W H
  constexpr int KT = (K + 15) / 16;  // 16-row tiles of bases for the sum over bins
  constexpr int NW = (N + 3) / 4;    // sources per wave in the sum over bins
  typedef typename Mma<R>::v4 v4;
  const int fg = blockIdx.x, tb = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int T = d.T, F = d.F;
  const int t0 = tb * kHTB;
  const int ntb = min(kHTB, T - t0);
  const int cl = lane & 15, ck = lane >> 4;
  extern __shared__ __align__(16) unsigned char smem[];
  R* sHt = reinterpret_cast<R*>(smem);  // [NK][16]
  R* sgc = sHt + NK * kHTB;             // [16 f][N*M]
  R* sAB = sgc + 16 * N * M;            // [N][2][16 f][16 t]

  for (int i = tid; i < NK * kHTB; i += 256) {
    const int nk = i / kHTB, tl = i % kHTB;
    sHt[i] = tl < ntb ? H[(size_t)nk * T + t0 + tl] : (R)0;
  }
  v4 accN[NW][KT], accD[NW][KT];
#pragma unroll
  for (int i = 0; i < NW; ++i)
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      accN[i][kt] = v4{0, 0, 0, 0};
      accD[i][kt] = v4{0, 0, 0, 0};
    }

  for (int c = 0; c < kHCPW; ++c) {
    const int f0 = (fg * kHCPW + c) * 16;
    const int nf = min(16, F - f0);
    if (nf <= 0) break;  // uniform over the workgroup
    // One batch: W operands of both contractions, g of the chunk, P of this lane's pair.
    R wl[N][KS], wh[NW][KT][4], pv[M];
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
      for (int st = 0; st < KS; ++st) {
        const int k = 4 * st + ck;
        wl[n][st] = (k < K && cl < nf) ? W[((size_t)n * F + f0 + cl) * K + k] : (R)0;
      }
#pragma unroll
    for (int i = 0; i < NW; ++i)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int n = wave + 4 * i, fl = 4 * st + ck, k = kt * 16 + cl;
          wh[i][kt][st] = (n < N && k < K && fl < nf) ? W[((size_t)n * F + f0 + fl) * K + k] : (R)0;
        }
    const int fl = Mma<R>::row(lane, wave);
    const bool pair_ok = fl < nf && cl < ntb;
    if (pair_ok) {
      load16<R, M>(pv, P + ((size_t)(f0 + fl) * T + t0 + cl) * M);
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) pv[m] = 0;
    }
    for (int i = tid; i < 16 * N * M; i += 256) {
      const int fi = i / (N * M);
      sgc[i] = fi < nf ? g[(size_t)(f0 + fi) * N * M + i % (N * M)] : (R)0;
    }
    sched_fence();
    __syncthreads();  // sHt (first chunk), sgc
    // lambda for the lane's pair (accumulator row `wave`).
    R lam[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      v4 acc = {0, 0, 0, 0};
#pragma unroll
      for (int st = 0; st < KS; ++st) {
        const int k = 4 * st + ck;
        const R bv = k < K ? sHt[(n * K + k) * kHTB + cl] : (R)0;
        acc = Mma<R>::run(wl[n][st], bv, acc);
      }
      lam[n] = acc[0];
#pragma unroll
      for (int r = 1; r < 4; ++r)
        if (wave == r) lam[n] = acc[r];
    }
    R a[N], b[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      a[n] = 0;
      b[n] = 0;
    }
    if (pair_ok) {
      const R* gf = sgc + fl * N * M;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        R y = 0;
#pragma unroll
        for (int n = 0; n < N; ++n) y += lam[n] * gf[n * M + m];
        const R iy = rcp(rmax(y, (R)d.eps));
        const R piy2 = pv[m] * iy * iy;
#pragma unroll
        for (int n = 0; n < N; ++n) {
          a[n] += gf[n * M + m] * piy2;
          b[n] += gf[n * M + m] * iy;
        }
      }
    }
#pragma unroll
    for (int n = 0; n < N; ++n) {
      sAB[((n * 2 + 0) * 16 + fl) * 16 + cl] = a[n];
      sAB[((n * 2 + 1) * 16 + fl) * 16 + cl] = b[n];
    }
    __syncthreads();
    // num/den for this wave's sources: A = W^T (rows k), B = a'/b' (columns t).
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int n = wave + 4 * i;
      if (n < N) {
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            const int fb = 4 * st + ck;
            accN[i][kt] = Mma<R>::run(wh[i][kt][st], sAB[((n * 2 + 0) * 16 + fb) * 16 + cl], accN[i][kt]);
            accD[i][kt] = Mma<R>::run(wh[i][kt][st], sAB[((n * 2 + 1) * 16 + fb) * 16 + cl], accD[i][kt]);
          }
      }
    }
    __syncthreads();  // before the next chunk overwrites sgc / sAB
  }
  // This workgroup's partial for its frequency group: lane holds rows k = row(lane, r).
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const int n = wave + 4 * i;
    if (n >= N || cl >= ntb) continue;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = kt * 16 + Mma<R>::row(lane, r);
        if (k < K) {
          R* dst = Hpart + (((size_t)fg * NK + n * K + k) * T + t0 + cl) * 2;
          dst[0] = accN[i][kt][r];
          dst[1] = accD[i][kt][r];
        }
      }
  }
}

// ------------------------------------------------------------------------------------
// Eq. (10) sums per (f, slice).  Per frame: 1/y and P/y^2 from lambda (read), stored
// frame-major in LDS with lambda.  Then num/den[n][m] = sum_t lambda_n (P_m/y_m^2, 1/y_m):
// in FP32 on the 4x4x1 matrix-core blocks (block = (group of 4 sources, group of 4 mics,
// numerator or denominator)), one op per frame and 16 blocks; frames alternate between
// the two waves.
template <typename R, int N, int K, int ML, int L>
struct GShape {
  static constexpr int M = ML * L;
  static constexpr int NP = (N + 3) & ~3;
  static constexpr int AP = padded<R>(NP);     // LDS row of lambda
  static constexpr int BP = padded<R>(2 * M);  // LDS row of P/y^2 then 1/y
  static constexpr int NGR = NP / 4, MG = M / 4;
  static constexpr int NI = (2 * NGR * MG + 15) / 16;
};

template <typename R, int N, int K, int ML, int L>
__global__ __launch_bounds__(kT) void k_g_f(Dims d, const R* __restrict__ lamin, const R* __restrict__ g,
                                            const R* __restrict__ P, R* __restrict__ gpart) {
  typedef GShape<R, N, K, ML, L> G;
  constexpr int M = G::M, NP = G::NP, AP = G::AP, BP = G::BP;
  constexpr int E = V16<R>::E;
  static_assert(M % 4 == 0 && M % E == 0 && NP % E == 0 && N * M <= kT, "shape");
  typedef typename V16<R>::type vt;
  const int f = blockIdx.x, s = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int T = d.T;
  const int t0 = s * d.SL;
  const int nt = min(d.SL, T - t0);
  const int ntp = (nt + 3) & ~3;
  extern __shared__ __align__(16) unsigned char smem[];
  R* sg = reinterpret_cast<R*>(smem);
  R* sA = reinterpret_cast<R*>(smem + align_up(sizeof(R) * N * M, 16));  // [SLP][AP]
  R* sB = sA + (size_t)d.SLP * AP;                                         // [SLP][BP]
  R* sRed = sB + (size_t)d.SLP * BP;                                       // FP32: [NI][64][4]

  R pv[M], lam[NP], gv = 0;
#pragma unroll
  for (int n = N; n < NP; ++n) lam[n] = 0;
  if (tid < nt) {
    load16<R, M>(pv, P + ((size_t)f * T + t0 + tid) * M);
#pragma unroll
    for (int n = 0; n < N; ++n) lam[n] = lamin[((size_t)f * N + n) * T + t0 + tid];
  } else {
#pragma unroll
    for (int m = 0; m < M; ++m) pv[m] = 0;
#pragma unroll
    for (int n = 0; n < N; ++n) lam[n] = 0;
  }
  if (tid < N * M) gv = g[(size_t)f * N * M + tid];
  sched_fence();
  if (tid < N * M) sg[tid] = gv;
  __syncthreads();
  if (tid < ntp) {
    R u[2 * M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      R y = 0;
#pragma unroll
      for (int n = 0; n < N; ++n) y += lam[n] * sg[n * M + m];
      const R iy = tid < nt ? rcp(rmax(y, (R)d.eps)) : (R)0;
      u[m] = pv[m] * iy * iy;
      u[M + m] = iy;
    }
#pragma unroll
    for (int i = 0; i < NP / E; ++i) {
      vt v;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = lam[i * E + e];
      reinterpret_cast<vt*>(sA + (size_t)tid * AP)[i] = v;
    }
#pragma unroll
    for (int i = 0; i < 2 * M / E; ++i) {
      vt v;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = u[i * E + e];
      reinterpret_cast<vt*>(sB + (size_t)tid * BP)[i] = v;
    }
  }
  __syncthreads();

  R* out = gpart + ((size_t)f * d.S + s) * N * M * 2;
  if constexpr (sizeof(R) == 4) {
    constexpr int NI = G::NI, NGR = G::NGR, MG = G::MG;
    typedef float v4f __attribute__((ext_vector_type(4)));
    const int sub = lane & 3;
    v4f acc[NI];
    int aoff[NI], boff[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      acc[q] = v4f{0, 0, 0, 0};
      const int blk = 16 * q + (lane >> 2);
      const bool ok = blk < 2 * NGR * MG;
      const int ng = blk % NGR, rest = blk / NGR, mg = rest % MG, uz = rest / MG;
      aoff[q] = ok ? 4 * ng + sub : 0;
      boff[q] = ok ? uz * M + 4 * mg + sub : 0;
    }
    const int half = ((ntp >> 1) + 3) & ~3;
    const int fb = wave == 0 ? 0 : half, fe = wave == 0 ? min(half, ntp) : ntp;
    for (int t4 = fb; t4 < fe; t4 += 4) {
      R av[4][NI], bv[4][NI];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < NI; ++q) {
          av[u][q] = sA[(size_t)(t4 + u) * AP + aoff[q]];
          bv[u][q] = sB[(size_t)(t4 + u) * BP + boff[q]];
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < NI; ++q) acc[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[u][q], bv[u][q], acc[q], 0, 0, 0);
    }
    if (wave == 1)
#pragma unroll
      for (int q = 0; q < NI; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) sRed[(q * 64 + lane) * 4 + r] = acc[q][r];
    __syncthreads();
    if (wave == 0)
#pragma unroll
      for (int q = 0; q < NI; ++q) {
        const int blk = 16 * q + (lane >> 2);
        if (blk >= 2 * NGR * MG) continue;
        const int ng = blk % NGR, rest = blk / NGR, mg = rest % MG, uz = rest / MG;
        const int m = 4 * mg + sub;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int n = 4 * ng + r;
          if (n < N) out[(n * M + m) * 2 + uz] = acc[q][r] + sRed[(q * 64 + lane) * 4 + r];
        }
      }
  } else {
    for (int o = tid; o < N * M; o += kT) {
      const int n = o / M, m = o - n * M;
      R num = 0, den = 0;
      for (int tt = 0; tt < ntp; ++tt) {
        const R lv = sA[(size_t)tt * AP + n];
        num += lv * sB[(size_t)tt * BP + m];
        den += lv * sB[(size_t)tt * BP + M + m];
      }
      out[o * 2 + 0] = num;
      out[o * 2 + 1] = den;
    }
  }
}

// ------------------------------------------------------------------------------------
// LDS budgets (bytes) and launches of one compiled set.
template <typename R, int N, int K, int ML, int L>
struct Set {
  static constexpr int M = ML * L;
  static size_t smem_gram(const Dims& d) {
    typedef GramShape<R, N, K, ML, L> G;
    const size_t rows = (size_t)d.SLP * (G::MP + G::OP);
    const size_t red = G::kBlocks ? (size_t)G::NG * 64 * 4 : 0;  // cross-wave sums reuse the rows
    return align_up(sizeof(R) * N * M, 16) + sizeof(R) * (rows > red ? rows : red);
  }
  static size_t smem_pw(const Dims& d) {
    typedef PwShape<R, N, K, ML, L> S_;
    return align_up(sizeof(cx<R>) * S_::QF, 16) + align_up(sizeof(R) * N * M, 16) +
           sizeof(R) * ((size_t)d.SLP * S_::CP + S_::NI * 256);
  }
  static size_t smem_h(const Dims&) { return sizeof(R) * (N * K * kHTB + 16 * N * M + N * 2 * 256); }
  static size_t smem_g(const Dims& d) {
    typedef GShape<R, N, K, ML, L> G;
    return align_up(sizeof(R) * N * M, 16) + sizeof(R) * ((size_t)d.SLP * (G::AP + G::BP) + G::NI * 256);
  }
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
      case kFHt:
        hipLaunchKernelGGL((k_ht_f<R, N * K>), dim3((d.T + kT - 1) / kT), dim3(kT), 0, s, d, H,
                           static_cast<R*>(b.Ht));
        break;
      case kFHApply:
        hipLaunchKernelGGL((k_happly_f<R, N, K>), dim3(N, (d.T + 15) / 16), dim3(64 * kLamWaves), 0, s, d, W, H,
                           static_cast<R*>(b.Ht), static_cast<const R*>(b.Hpart), static_cast<R*>(b.lam),
                           b.status);
        break;
      case kFLam:
        hipLaunchKernelGGL((k_lam_f<R, N, K>), dim3(N, (d.T + 15) / 16), dim3(64 * kLamWaves), 0, s, d, W, H,
                           static_cast<R*>(b.lam));
        break;
      case kFGram:
        hipLaunchKernelGGL((k_gram_f<R, N, K, ML, L>), dim3(d.F * d.S), dim3(kT), smem_gram(d), s, d, X,
                           static_cast<const R*>(b.lam), g, static_cast<R*>(b.Vpart));
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
        hipLaunchKernelGGL((k_pw_f<R, N, K, ML, L>), dim3(d.F, d.S), dim3(kT), smem_pw(d), s, d, X, Q,
                           static_cast<const R*>(b.lam), static_cast<const R*>(b.Ht), g, P,
                           static_cast<R*>(b.Wpart));
        break;
      case kFH:
        hipLaunchKernelGGL((k_h_f<R, N, K, ML, L>), dim3(d.FG, d.TBN), dim3(256), smem_h(d), s, d, W, H, g, P,
                           static_cast<R*>(b.Hpart));
        break;
      case kFG:
        hipLaunchKernelGGL((k_g_f<R, N, K, ML, L>), dim3(d.F, d.S), dim3(kT), smem_g(d), s, d,
                           static_cast<const R*>(b.lam), g, P, static_cast<R*>(b.gpart));
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

int fast_h_chunks() { return fast::kHCPW; }

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
