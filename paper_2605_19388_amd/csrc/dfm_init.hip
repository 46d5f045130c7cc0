// Initial parameters from estimates of the source images (Sec. IV-A, steps 3, 5 and 6), FP64
// throughout (the images may be complex64 or complex128):
//
//   k_icov   R_fn = (1/T) sum_t c_ftn c_ftn^H, full M x M, one workgroup per (f, n);
//   k_ih     h_ftn = c_ftn^H R_fn^{-1} c_ftn / M: R_fn inverted in LDS by Gauss-Jordan steps
//            without pivoting (R_fn is Hermitian positive definite), then one frame per thread;
//   k_igevd  per (f, l): the joint diagonaliser of the l-th diagonal blocks A = R_f,N-1^(l) and
//            B = R_f,N^(l) (the last two sources): B = L L^H (Cholesky), the Hermitian matrix
//            L^-1 A L^-H diagonalised by cyclic complex Jacobi rotations (V), W = L^-H V, so
//            W^H B W = I and W^H A W = diag(lambda); columns in ascending lambda, each with its
//            largest entry (the first on a tie) made real and positive; Q_fl = W^H; then
//            g[f][n][o_l + mu] = w_mu^H R_fn^(l) w_mu for every source (step 6).
//
// A zero or negative pivot (an image estimate whose covariance is singular) sets the sticky
// singular bit; the outputs of that block are then not meaningful.
#include <hip/hip_runtime.h>

#include "dfm_device.h"

namespace dfm {
namespace init {

__global__ void k_zero_status(int* p) {
  if (threadIdx.x == 0) *p = 0;
}

constexpr int kIB = 256;  // threads of k_icov / k_ih
constexpr int kGB = 64;   // threads of k_igevd

// ------------------------------------------------------------------------------------ step 3
// R[(f N + n) M^2 + a M + b] = (1/T) sum_t c_a conj(c_b); frames staged in LDS tiles of TT.
template <typename R>
__global__ __launch_bounds__(kIB) void k_icov(Dims d, const cx<R>* __restrict__ C, cd* __restrict__ Rm, int TT) {
  const int f = blockIdx.x, n = blockIdx.y, tid = threadIdx.x;
  const int M = d.M, T = d.T;
  extern __shared__ __align__(16) unsigned char smem[];
  cd* sx = reinterpret_cast<cd*>(smem);  // [TT][M]
  const cx<R>* cf = C + ((size_t)n * d.F + f) * T * M;
  const int NE = M * (M + 1) / 2;        // upper triangle, row-major
  constexpr int EPT = 64 * 65 / 2 / kIB + 1;
  double ar[EPT], ai[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) ar[e] = ai[e] = 0.0;
  for (int t0 = 0; t0 < T; t0 += TT) {
    const int nt = min(TT, T - t0);
    __syncthreads();
    for (int i = tid; i < nt * M; i += kIB) {
      const cx<R> v = cf[(size_t)t0 * M + i];
      sx[i] = {(double)v.re, (double)v.im};
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int idx = tid + e * kIB;
      if (idx < NE) {
        int a = 0, rem = idx;
        while (rem >= M - a) {
          rem -= M - a;
          ++a;
        }
        const int b = a + rem;
        double sr = 0.0, si = 0.0;
        for (int t = 0; t < nt; ++t) {
          const cd xa = sx[t * M + a], xb = sx[t * M + b];
          sr += xa.re * xb.re + xa.im * xb.im;
          si += xa.im * xb.re - xa.re * xb.im;
        }
        ar[e] += sr;
        ai[e] += si;
      }
    }
  }
  cd* out = Rm + ((size_t)f * d.N + n) * M * M;
  const double invT = 1.0 / T;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int idx = tid + e * kIB;
    if (idx < NE) {
      int a = 0, rem = idx;
      while (rem >= M - a) {
        rem -= M - a;
        ++a;
      }
      const int b = a + rem;
      out[a * M + b] = {ar[e] * invT, a == b ? 0.0 : ai[e] * invT};
      if (a != b) out[b * M + a] = {ar[e] * invT, -ai[e] * invT};
    }
  }
}

// In-place inverse of the n x n Hermitian positive definite matrix A (LDS, row stride n) by
// Gauss-Jordan steps without pivoting, all threads cooperating.  Returns false (in every
// thread) on a non-positive pivot.
__device__ bool hpd_invert(cd* A, int n, int* s_bad) {
  const int tid = threadIdx.x, bd = blockDim.x;
  if (tid == 0) *s_bad = 0;
  __syncthreads();
  for (int p = 0; p < n; ++p) {
    const double piv = A[p * n + p].re;
    if (!(piv > 0.0)) {  // the same value in every thread: uniform exit
      if (tid == 0) *s_bad = 1;
      break;
    }
    const double inv = 1.0 / piv;
    __syncthreads();
    for (int j = tid; j < n; j += bd)  // row p scaled
      if (j != p) A[p * n + j] = {A[p * n + j].re * inv, A[p * n + j].im * inv};
    __syncthreads();
    for (int i = tid; i < n * n; i += bd) {  // every other entry
      const int r = i / n, c = i - r * n;
      if (r != p && c != p) A[i] = csub(A[i], cmul(A[r * n + p], A[p * n + c]));
    }
    __syncthreads();
    for (int r = tid; r < n; r += bd)  // column p
      if (r != p) A[r * n + p] = {-A[r * n + p].re * inv, -A[r * n + p].im * inv};
    if (tid == 0) A[p * n + p] = {inv, 0.0};
    __syncthreads();
  }
  __syncthreads();
  return *s_bad == 0;
}

// h[(n F + f) T + t] = Re(c^H R^-1 c) / M.
template <typename R>
__global__ __launch_bounds__(kIB) void k_ih(Dims d, const cx<R>* __restrict__ C, const cd* __restrict__ Rm,
                                            R* __restrict__ h, int* __restrict__ status) {
  const int f = blockIdx.x, n = blockIdx.y, tid = threadIdx.x;
  const int M = d.M, T = d.T;
  extern __shared__ __align__(16) unsigned char smem[];
  cd* sA = reinterpret_cast<cd*>(smem);  // [M][M]
  __shared__ int s_bad;
  const cd* rf = Rm + ((size_t)f * d.N + n) * M * M;
  for (int i = tid; i < M * M; i += kIB) sA[i] = rf[i];
  __syncthreads();
  const bool ok = hpd_invert(sA, M, &s_bad);
  if (!ok && tid == 0) atomicOr(status, kStSingular);
  const cx<R>* cf = C + ((size_t)n * d.F + f) * T * M;
  R* hf = h + ((size_t)n * d.F + f) * T;
  const double invM = 1.0 / M;
  for (int t = tid; t < T; t += kIB) {
    const cx<R>* c = cf + (size_t)t * M;
    double acc = 0.0;
    for (int a = 0; a < M; ++a) {
      cd u = {0.0, 0.0};  // (R^-1 c)_a
      for (int b = 0; b < M; ++b) u = cfma(u, sA[a * M + b], cd{(double)c[b].re, (double)c[b].im});
      acc += (double)c[a].re * u.re + (double)c[a].im * u.im;  // Re(conj(c_a) u_a)
    }
    hf[t] = ok ? (R)(acc * invM) : (R)0;
  }
}

// ------------------------------------------------------------------------------------ steps 5, 6
// LDS of one (f, l) block of k_igevd, n = M_l <= MX: A, B -> L, C -> Jacobi, V, W.
__host__ __device__ inline size_t gevd_smem(int mx) { return sizeof(cd) * 4 * (size_t)mx * mx + 16 * mx; }

template <typename R>
__global__ __launch_bounds__(kGB) void k_igevd(Dims d, const cd* __restrict__ Rm, cx<R>* __restrict__ Q,
                                               R* __restrict__ g, int* __restrict__ status) {
  const int f = blockIdx.x, l = blockIdx.y, tid = threadIdx.x;
  const int n = d.mics[l], o = d.moff[l], M = d.M, mx = d.MLX;
  extern __shared__ __align__(16) unsigned char smem[];
  cd* sA = reinterpret_cast<cd*>(smem);   // A, then Y = L^-1 A
  cd* sL = sA + mx * mx;                  // B -> its Cholesky factor L (lower)
  cd* sC = sL + mx * mx;                  // L^-1 A L^-H, rotated to diagonal
  cd* sV = sC + mx * mx;                  // eigenvectors of C, then W
  int* sperm = reinterpret_cast<int*>(sV + mx * mx);  // ascending order of the eigenvalues
  __shared__ int s_bad, s_rot, s_skip;
  __shared__ double s_cs, s_sn;
  __shared__ cd s_ph;  // e^{-i phi}
  const cd* RA = Rm + ((size_t)f * d.N + (d.N - 2)) * M * M;
  const cd* RB = Rm + ((size_t)f * d.N + (d.N - 1)) * M * M;
  for (int i = tid; i < n * n; i += kGB) {
    const int r = i / n, c = i - r * n;
    sA[i] = RA[(o + r) * M + o + c];
    sL[i] = RB[(o + r) * M + o + c];
    sV[i] = {r == c ? 1.0 : 0.0, 0.0};
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  // Cholesky B = L L^H, column by column (lower triangle of sL).
  for (int p = 0; p < n; ++p) {
    if (tid == 0) {
      const double dpp = sL[p * n + p].re;
      if (!(dpp > 0.0)) s_bad = 1;
      sL[p * n + p] = {dpp > 0.0 ? sqrt(dpp) : 1.0, 0.0};
    }
    __syncthreads();
    const double linv = 1.0 / sL[p * n + p].re;
    for (int r = p + 1 + tid; r < n; r += kGB) sL[r * n + p] = {sL[r * n + p].re * linv, sL[r * n + p].im * linv};
    __syncthreads();
    for (int i = tid; i < n * n; i += kGB) {  // trailing update, lower triangle: B_rc -= L_rp conj(L_cp)
      const int r = i / n, c = i - r * n;
      if (c > p && r >= c) sL[i] = cfms(sL[i], sL[r * n + p], cconj(sL[c * n + p]));
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) atomicOr(status, kStSingular);
    return;
  }
  // Y = L^-1 A (column j of A by forward substitution), then C = L^-1 Y^H (= L^-1 A L^-H,
  // Hermitian since A is): column j of C from column j of Y^H, i.e. the conjugated row j of Y.
  for (int j = tid; j < n; j += kGB)
    for (int r = 0; r < n; ++r) {
      cd acc = sA[r * n + j];
      for (int k = 0; k < r; ++k) acc = cfms(acc, sL[r * n + k], sA[k * n + j]);
      sA[r * n + j] = {acc.re / sL[r * n + r].re, acc.im / sL[r * n + r].re};
    }
  __syncthreads();
  for (int j = tid; j < n; j += kGB)
    for (int r = 0; r < n; ++r) {
      cd acc = cconj(sA[j * n + r]);
      for (int k = 0; k < r; ++k) acc = cfms(acc, sL[r * n + k], sC[k * n + j]);
      sC[r * n + j] = {acc.re / sL[r * n + r].re, acc.im / sL[r * n + r].re};
    }
  __syncthreads();
  for (int i = tid; i < n * n; i += kGB) {  // exact Hermitian symmetry: the upper triangle mirrored
    const int r = i / n, c = i - r * n;
    if (r > c) sC[i] = cconj(sC[c * n + r]);
    if (r == c) sC[i].im = 0.0;
  }
  __syncthreads();
  // Cyclic Jacobi: rotate (p, q) while |C_pq| > 1e-16 sqrt(C_pp C_qq); stop after a sweep with
  // no rotation (at most 60 sweeps).
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        if (tid == 0) {
          const cd c = sC[p * n + q];
          const double a = sC[p * n + p].re, b = sC[q * n + q].re, ac = sqrt(cabs2(c));
          const bool skip = !(ac > 1e-16 * sqrt(fabs(a * b))) || ac == 0.0;
          s_skip = skip;
          if (!skip) {
            const double tau = (b - a) / (2.0 * ac);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            s_cs = 1.0 / sqrt(1.0 + t * t);
            s_sn = t * s_cs;
            s_ph = {c.re / ac, -c.im / ac};  // e^{-i phi}, c = |c| e^{i phi}
            s_rot = 1;
          }
        }
        __syncthreads();
        if (!s_skip) {
          const double cs = s_cs, sn = s_sn;
          const cd ph = s_ph, phc = cconj(ph);
          // columns p, q of C and V: (X G)_kp = X_kp cs - X_kq sn e^{-i phi}, (X G)_kq = X_kp sn + X_kq cs e^{-i phi}
          for (int k = tid; k < 2 * n; k += kGB) {
            cd* X = k < n ? sC : sV;
            const int r = k < n ? k : k - n;
            const cd xp = X[r * n + p], xq = cmul(X[r * n + q], ph);
            X[r * n + p] = {xp.re * cs - xq.re * sn, xp.im * cs - xq.im * sn};
            X[r * n + q] = {xp.re * sn + xq.re * cs, xp.im * sn + xq.im * cs};
          }
          __syncthreads();
          // rows p, q of C: (G^H Y)_pj = cs Y_pj - sn e^{i phi} Y_qj, (G^H Y)_qj = sn Y_pj + cs e^{i phi} Y_qj
          for (int j = tid; j < n; j += kGB) {
            const cd yp = sC[p * n + j], yq = cmul(sC[q * n + j], phc);
            sC[p * n + j] = {yp.re * cs - yq.re * sn, yp.im * cs - yq.im * sn};
            sC[q * n + j] = {yp.re * sn + yq.re * cs, yp.im * sn + yq.im * cs};
          }
          __syncthreads();
          if (tid == 0) sC[p * n + q] = sC[q * n + p] = {0.0, 0.0};
        }
        __syncthreads();  // s_skip, s_cs, s_sn, s_ph are rewritten for the next pair
      }
    __syncthreads();
    if (!s_rot) break;  // uniform: written by thread 0 before the last barrier
  }
  // W = L^-H V (back substitution per column, in place in sV), ascending order of the eigenvalues.
  for (int j = tid; j < n; j += kGB)
    for (int r = n - 1; r >= 0; --r) {
      cd acc = sV[r * n + j];
      for (int k = r + 1; k < n; ++k) acc = cfms(acc, cconj(sL[k * n + r]), sV[k * n + j]);
      sV[r * n + j] = {acc.re / sL[r * n + r].re, acc.im / sL[r * n + r].re};
    }
  if (tid == 0) {
    for (int i = 0; i < n; ++i) sperm[i] = i;
    for (int i = 1; i < n; ++i) {  // insertion sort, stable
      const int v = sperm[i];
      int k = i - 1;
      while (k >= 0 && sC[sperm[k] * n + sperm[k]].re > sC[v * n + v].re) {
        sperm[k + 1] = sperm[k];
        --k;
      }
      sperm[k + 1] = v;
    }
  }
  __syncthreads();
  // Phase of each column: its largest entry (the first on a tie) real and positive.
  for (int j = tid; j < n; j += kGB) {
    int im = 0;
    double best = -1.0;
    for (int r = 0; r < n; ++r) {
      const double v = cabs2(sV[r * n + j]);
      if (v > best) {
        best = v;
        im = r;
      }
    }
    const double a = sqrt(best);
    const cd ph = {sV[im * n + j].re / a, -sV[im * n + j].im / a};  // conj(w_i) / |w_i|
    for (int r = 0; r < n; ++r) sV[r * n + j] = cmul(sV[r * n + j], ph);
  }
  __syncthreads();
  // Q_fl row mu = w_perm(mu)^H.
  cx<R>* qb = Q + (size_t)f * d.QF + d.qoff[l];
  for (int i = tid; i < n * n; i += kGB) {
    const int mu = i / n, c = i - mu * n;
    const cd w = sV[c * n + sperm[mu]];
    qb[i] = {(R)w.re, (R)(-w.im)};
  }
  // Step 6: g[f][s][o + mu] = w^H R_fs^(l) w for every source s.
  for (int i = tid; i < d.N * n; i += kGB) {
    const int s = i / n, mu = i - s * n, j = sperm[mu];
    const cd* rs = Rm + ((size_t)f * d.N + s) * M * M;
    double acc = 0.0;
    for (int a = 0; a < n; ++a) {
      cd u = {0.0, 0.0};  // (R w)_a
      for (int b = 0; b < n; ++b) u = cfma(u, rs[(o + a) * M + o + b], sV[b * n + j]);
      acc += sV[a * n + j].re * u.re + sV[a * n + j].im * u.im;
    }
    g[((size_t)f * d.N + s) * M + o + mu] = (R)acc;
  }
}

}  // namespace init

// Frames per LDS tile of k_icov: as many as fit 32 KB.
static int icov_tile(const Dims& d) { return d.M > 0 ? (2048 / d.M > 1 ? 2048 / d.M : 1) : 1; }

size_t initialise_workspace_bytes(const Dims& d) {
  return align_up(sizeof(cd) * (size_t)d.F * d.N * d.M * d.M, 256) + 256;
}

template <typename R>
static hipError_t initialise_impl(const Dims& d, const void* C, void* Q, void* g, void* h, char* ws, int* status,
                                  hipStream_t s) {
  cd* Rm = reinterpret_cast<cd*>(ws);
  const cx<R>* Cc = static_cast<const cx<R>*>(C);
  const int TT = icov_tile(d);
  hipLaunchKernelGGL(init::k_icov<R>, dim3(d.F, d.N), dim3(init::kIB), sizeof(cd) * TT * d.M, s, d, Cc, Rm, TT);
  if (h)
    hipLaunchKernelGGL(init::k_ih<R>, dim3(d.F, d.N), dim3(init::kIB), sizeof(cd) * d.M * d.M, s, d, Cc,
                       static_cast<const cd*>(Rm), static_cast<R*>(h), status);
  hipLaunchKernelGGL(init::k_igevd<R>, dim3(d.F, d.L), dim3(init::kGB), init::gevd_smem(d.MLX), s, d,
                     static_cast<const cd*>(Rm), static_cast<cx<R>*>(Q), static_cast<R*>(g), status);
  return hipGetLastError();
}

hipError_t launch_initialise(const Dims& d, int dtype, const void* C, void* Q, void* g, void* h, void* ws,
                             hipStream_t s) {
  char* w = static_cast<char*>(ws);
  int* status = reinterpret_cast<int*>(w + align_up(sizeof(cd) * (size_t)d.F * d.N * d.M * d.M, 256));
  hipLaunchKernelGGL(init::k_zero_status, dim3(1), dim3(64), 0, s, status);
  return dtype == DFM_C64 ? initialise_impl<float>(d, C, Q, g, h, w, status, s)
                          : initialise_impl<double>(d, C, Q, g, h, w, status, s);
}

int* initialise_status(const Dims& d, void* ws) {
  return reinterpret_cast<int*>(static_cast<char*>(ws) + align_up(sizeof(cd) * (size_t)d.F * d.N * d.M * d.M, 256));
}

}  // namespace dfm
