// Device-side helpers shared by the generic and the shape-specialised kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "dfm_internal.h"

namespace dfm {

template <typename R>
struct cx {
  R re, im;
};

struct cd {
  double re, im;
};

__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd cconj(cd a) { return {a.re, -a.im}; }
// c + a b and c - a b with two fused multiply-adds per part (the unfused forms round the
// product before the sum and take a third instruction).
__device__ __forceinline__ cd cfma(cd c, cd a, cd b) {
  return {fma(-a.im, b.im, fma(a.re, b.re, c.re)), fma(a.im, b.re, fma(a.re, b.im, c.im))};
}
__device__ __forceinline__ cd cfms(cd c, cd a, cd b) {
  return {fma(a.im, b.im, fma(-a.re, b.re, c.re)), fma(-a.im, b.re, fma(-a.re, b.im, c.im))};
}
// c + conj(a) b.
__device__ __forceinline__ cd cfmac(cd c, cd a, cd b) {
  return {fma(a.im, b.im, fma(a.re, b.re, c.re)), fma(-a.im, b.re, fma(a.re, b.im, c.im))};
}
__device__ __forceinline__ double cabs2(cd a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ cd cinv(cd a) {
  const double s = 1.0 / cabs2(a);
  return {a.re * s, -a.im * s};
}

// The floor max(a, b) of Sec. IV-A (b = eps > 0), one max instruction; like the comparison
// a > b ? a : b it gives b for a NaN a.
template <typename R>
__device__ __forceinline__ R rmax(R a, R b) { return fmax(a, b); }

// ---------------------------------------------------------------------------------------
// Packed Hermitian index j in [0, M_l^2): j < M_l is the diagonal entry (j, j) (real);
// otherwise pair p = (j - M_l) / 2 of the strict upper triangle in row-major order,
// part (j - M_l) % 2 = 0 for the real and 1 for the imaginary part of V[a][b], a < b.
__device__ __forceinline__ void packed_pair(int Ml, int j, int& a, int& b, int& part) {
  if (j < Ml) {
    a = j;
    b = j;
    part = 0;
    return;
  }
  int p = (j - Ml) >> 1;
  part = (j - Ml) & 1;
  int row = 0, cnt = Ml - 1;
  while (p >= cnt) {
    p -= cnt;
    ++row;
    --cnt;
  }
  a = row;
  b = row + 1 + p;
}

// Partial-sum slots of bin f's covariances: the S frame slices, or, for the balanced
// covariance kernel (ranges of GR flattened frames), one per workgroup that touched f.
__device__ __forceinline__ int cov_slots(const Dims& d, int f) {
  if (d.GR <= 0) return d.SG;
  if (d.GSB > 0) return d.GSB;
  return (int)((((long long)f + 1) * d.T - 1) / d.GR - ((long long)f * d.T) / d.GR) + 1;
}

__device__ __forceinline__ int subarray_of_vidx(const Dims& d, int idx) {
  int l = 0;
  while (l + 1 < d.L && idx >= d.voff[l + 1]) ++l;
  return l;
}

// lambda_n = sum_k W[n][f][k] H[n][k][t] for every source (eq. (2)).
// w points at W[0][f][0] and wsn is the stride between sources.
template <typename R>
__device__ __forceinline__ void source_psd(const Dims& d, const R* w, int wsn, const R* __restrict__ H, int t,
                                           R (&lam)[kMaxN]) {
#pragma unroll
  for (int n = 0; n < kMaxN; ++n) {
    R acc = 0;
    if (n < d.N) {
      const R* hn = H + (size_t)n * d.K * d.T + t;
      const R* wn = w + (size_t)n * wsn;
      for (int k = 0; k < d.K; ++k) acc += wn[k] * hn[(size_t)k * d.T];
    }
    lam[n] = acc;
  }
}

// y_m = max(sum_n lambda_n g[n][m], eps) with gf = g[f][0][0].
template <typename R>
__device__ __forceinline__ R model_var(const Dims& d, const R (&lam)[kMaxN], const R* gf, int m) {
  R acc = 0;
#pragma unroll
  for (int n = 0; n < kMaxN; ++n)
    if (n < d.N) acc += lam[n] * gf[n * d.M + m];
  return rmax(acc, (R)d.eps);
}

__host__ __device__ __forceinline__ size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }


// ---------------------------------------------------------------------------------------
// In-LDS Gaussian elimination with partial pivoting of the n x ncols row-major
// matrix A (leading dimension ld), all threads cooperating.  Thread 0 searches the
// pivot and swaps rows; the others update the trailing rows.  Returns, in thread 0,
// sum_p ln|A_pp| of the eliminated matrix and whether a zero pivot appeared.
__device__ inline void eliminate(cd* A, int ld, int n, int ncols, double* s_logabs, int* s_sing) {
  const int tid = threadIdx.x, bd = blockDim.x;
  if (tid == 0) {
    *s_logabs = 0.0;
    *s_sing = 0;
  }
  for (int p = 0; p < n; ++p) {
    if (tid == 0) {
      int piv = p;
      double best = cabs2(A[p * ld + p]);
      for (int r = p + 1; r < n; ++r) {
        const double v = cabs2(A[r * ld + p]);
        if (v > best) {
          best = v;
          piv = r;
        }
      }
      if (piv != p)
        for (int c = p; c < ncols; ++c) {
          const cd tmp = A[p * ld + c];
          A[p * ld + c] = A[piv * ld + c];
          A[piv * ld + c] = tmp;
        }
      if (best == 0.0)
        *s_sing = 1;
      else
        *s_logabs += 0.5 * log(best);
    }
    __syncthreads();
    const cd pv = A[p * ld + p];
    if (cabs2(pv) != 0.0) {
      const cd inv = cinv(pv);
      const int w = ncols - p - 1;
      for (int i = tid; i < (n - p - 1) * w; i += bd) {
        const int r = p + 1 + i / w, c = p + 1 + i % w;
        const cd fac = cmul(A[r * ld + p], inv);
        A[r * ld + c] = csub(A[r * ld + c], cmul(fac, A[p * ld + c]));
      }
    }
    __syncthreads();
  }
}

// Matrix-core helper: D += A * B on one wave with the 16x16x4 shape (A 16x4, B 4x16).
// Operand layouts (both precisions): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].
// Result: column l % 16; the row held in accumulator element r differs by precision.
template <typename R>
struct Mma;

template <>
struct Mma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <>
struct Mma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

}  // namespace dfm
