// exp(H) of a small dense matrix on one workgroup (Sec. 4.3 of the paper: Taylor series
// when ||H|| <= 1, scaling and squaring otherwise, no eigendecomposition).  The squaring
// branch uses the degree-13 diagonal Pade approximant and the scaling rule of Higham,
// "The scaling and squaring method for the matrix exponential revisited", SIAM J. Matrix
// Anal. Appl. 26 (2005): s = max(0, ceil(log2(||H||_1 / theta_13))).
// Matrices are row major with leading dimension m and live in device memory private to
// the calling workgroup (L2 resident); every thread of the workgroup must call.
#pragma once

#include "ep_common.hpp"

namespace ep {

constexpr double kTheta13 = 5.371920351148152;

// numerator coefficient c_j of the [13/13] Pade approximant: (26-j)! 13! / (26! j! (13-j)!)
__device__ __forceinline__ double pade13(int j) {
  double c = 1.0;
  for (int i = 1; i <= j; ++i) c *= double(13 - i + 1) / double(i * (26 - i + 1));
  return c;
}

__device__ __forceinline__ void wg_sync() { __syncthreads(); }

// C = A * B
__device__ inline void wg_gemm(const double* A, const double* B, double* C, int m) {
  const int n = m * m;
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int i = idx / m, j = idx - (idx / m) * m;
    const double* a = A + (size_t)i * m;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += a[k] * B[(size_t)k * m + j];
    C[idx] = s;
  }
  wg_sync();
}

// 1-norm (max column sum), same value in every thread
__device__ inline double wg_norm1(const double* A, int m, double* red) {
  double mx = 0.0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += fabs(A[(size_t)i * m + j]);
    mx = fmax(mx, s);
  }
  // max-reduce
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

// Solve A X = B in place (A destroyed, B <- X) by Gaussian elimination with partial
// pivoting (ties: smallest row index).  piv_red: LDS scratch of >= 32 doubles + 16 ints.
__device__ inline void wg_solve(double* A, double* B, int m, double* red, int* ired) {
  for (int k = 0; k < m; ++k) {
    // pivot search over rows k..m-1
    double best = -1.0;
    int bi = m;
    for (int i = k + threadIdx.x; i < m; i += blockDim.x) {
      const double v = fabs(A[(size_t)i * m + k]);
      if (v > best) { best = v; bi = i; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6] = best; ired[threadIdx.x >> 6] = bi; }
    __syncthreads();
    double gb = -1.0;
    int p = m;
    for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) {
      if (red[w] > gb || (red[w] == gb && ired[w] < p)) { gb = red[w]; p = ired[w]; }
    }
    __syncthreads();
    if (p != k && p < m) {
      for (int j = threadIdx.x; j < m; j += blockDim.x) {
        double t = A[(size_t)k * m + j]; A[(size_t)k * m + j] = A[(size_t)p * m + j]; A[(size_t)p * m + j] = t;
        t = B[(size_t)k * m + j]; B[(size_t)k * m + j] = B[(size_t)p * m + j]; B[(size_t)p * m + j] = t;
      }
      wg_sync();
    }
    const double piv = A[(size_t)k * m + k];
    // multipliers stored below the diagonal
    for (int i = k + 1 + threadIdx.x; i < m; i += blockDim.x) A[(size_t)i * m + k] /= piv;
    wg_sync();
    const int rows = m - k - 1;
    const int cols = m - k - 1;     // A columns k+1..m-1
    const int tot = rows * (cols + m);
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      const int r = idx / (cols + m);
      const int cc = idx - r * (cols + m);
      const int i = k + 1 + r;
      const double l = A[(size_t)i * m + k];
      if (cc < cols) {
        const int j = k + 1 + cc;
        A[(size_t)i * m + j] -= l * A[(size_t)k * m + j];
      } else {
        const int j = cc - cols;
        B[(size_t)i * m + j] -= l * B[(size_t)k * m + j];
      }
    }
    wg_sync();
  }
  // back substitution, one column of B per thread
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    for (int k = m - 1; k >= 0; --k) {
      double s = B[(size_t)k * m + j];
      for (int c = k + 1; c < m; ++c) s -= A[(size_t)k * m + c] * B[(size_t)c * m + j];
      B[(size_t)k * m + j] = s / A[(size_t)k * m + k];
    }
  }
  wg_sync();
}

// E = exp(Hin).  Hin is m x m with leading dimension ldh; E gets leading dimension m.
// scr: 8 m^2 doubles of workgroup-private device memory.  Returns E.
__device__ inline double* wg_expm(const double* Hin, int ldh, int m, double* scr, double* red, int* ired) {
  const size_t mm = (size_t)m * m;
  double* A = scr;
  double* A2 = scr + mm;
  double* A4 = scr + 2 * mm;
  double* A6 = scr + 3 * mm;
  double* U = scr + 4 * mm;
  double* V = scr + 5 * mm;
  double* T1 = scr + 6 * mm;
  double* T2 = scr + 7 * mm;
  for (int idx = threadIdx.x; idx < (int)mm; idx += blockDim.x) {
    const int i = idx / m, j = idx - i * m;
    A[idx] = Hin[(size_t)i * ldh + j];
  }
  wg_sync();
  const double nrm = wg_norm1(A, m, red);
  if (nrm <= 1.0) {
    // Taylor: E = sum_k A^k / k!, stopped when the term's norm drops below 2^-53 ||E||
    double* E = U;
    double* Tm = V;
    for (int idx = threadIdx.x; idx < (int)mm; idx += blockDim.x) {
      const int i = idx / m, j = idx - i * m;
      E[idx] = (i == j) ? 1.0 : 0.0;
      Tm[idx] = (i == j) ? 1.0 : 0.0;
    }
    wg_sync();
    for (int k = 1; k <= 60; ++k) {
      wg_gemm(Tm, A, T1, m);
      const double inv = 1.0 / double(k);
      for (int idx = threadIdx.x; idx < (int)mm; idx += blockDim.x) {
        const double t = T1[idx] * inv;
        Tm[idx] = t;
        E[idx] += t;
      }
      wg_sync();
      const double tn = wg_norm1(Tm, m, red);
      const double en = wg_norm1(E, m, red);
      if (tn <= 0x1p-53 * en) break;
    }
    return E;
  }
  int s = 0;
  {
    const double r = nrm / kTheta13;
    if (r > 1.0) s = (int)ceil(log2(r));
  }
  const double sc = ldexp(1.0, -s);
  for (int idx = threadIdx.x; idx < (int)mm; idx += blockDim.x) A[idx] *= sc;
  wg_sync();
  wg_gemm(A, A, A2, m);
  wg_gemm(A2, A2, A4, m);
  wg_gemm(A4, A2, A6, m);
  double c[14];
  for (int j = 0; j < 14; ++j) c[j] = pade13(j);
  // T1 = c13 A6 + c11 A4 + c9 A2 ; T2 = c12 A6 + c10 A4 + c8 A2
  for (int idx = threadIdx.x; idx < (int)mm; idx += blockDim.x) {
    T1[idx] = c[13] * A6[idx] + c[11] * A4[idx] + c[9] * A2[idx];
    T2[idx] = c[12] * A6[idx] + c[10] * A4[idx] + c[8] * A2[idx];
  }
  wg_sync();
  wg_gemm(A6, T1, U, m);     // U <- A6 T1
  wg_gemm(A6, T2, V, m);     // V <- A6 T2
  for (int idx = threadIdx.x; idx < (int)mm; idx += blockDim.x) {
    const int i = idx / m, j = idx - i * m;
    const double id = (i == j) ? 1.0 : 0.0;
    T1[idx] = U[idx] + c[7] * A6[idx] + c[5] * A4[idx] + c[3] * A2[idx] + c[1] * id;
    V[idx] = V[idx] + c[6] * A6[idx] + c[4] * A4[idx] + c[2] * A2[idx] + c[0] * id;
  }
  wg_sync();
  wg_gemm(A, T1, U, m);      // U = A (A6 (...) + ...)
  // solve (V - U) R = (V + U)
  for (int idx = threadIdx.x; idx < (int)mm; idx += blockDim.x) {
    const double u = U[idx], v = V[idx];
    T1[idx] = v - u;
    T2[idx] = v + u;
  }
  wg_sync();
  wg_solve(T1, T2, m, red, ired);
  double* R = T2;
  double* Rn = A;
  for (int q = 0; q < s; ++q) {
    wg_gemm(R, R, Rn, m);
    double* t = R; R = Rn; Rn = t;
  }
  return R;
}

}  // namespace ep
