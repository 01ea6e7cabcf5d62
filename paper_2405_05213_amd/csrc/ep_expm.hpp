// exp(H) of a small dense matrix on one workgroup (Sec. 4.3 of the paper: Taylor series
// when ||H|| <= 1, scaling and squaring otherwise, no eigendecomposition).  The squaring
// branch uses the degree-13 diagonal Pade approximant and the scaling rule of Higham,
// "The scaling and squaring method for the matrix exponential revisited", SIAM J. Matrix
// Anal. Appl. 26 (2005): s = max(0, ceil(log2(||H||_1 / theta_13))).
// Matrices are row major with leading dimension m and live in LDS when they fit, else in
// device memory private to the calling workgroup; every thread of the workgroup must call.
#pragma once

#include "ep_common.hpp"

namespace ep {

constexpr double kTheta13 = 5.371920351148152;

// numerator coefficient c_j of the [13/13] Pade approximant: (26-j)! 13! / (26! j! (13-j)!),
// built by the ratio c_j / c_{j-1} = (13 - j + 1) / (j (26 - j + 1)); evaluated at compile time
struct Pade13 {
  double c[14];
  constexpr Pade13() : c{} {
    double v = 1.0;
    c[0] = 1.0;
    for (int j = 1; j <= 13; ++j) {
      v *= double(13 - j + 1) / double(j * (26 - j + 1));
      c[j] = v;
    }
  }
};
__device__ constexpr Pade13 kPade13{};

__device__ __forceinline__ void wg_sync() { __syncthreads(); }

// Leading dimension of the work matrices: odd for even m >= 8, so that the 16 rows of a
// matrix-core fragment fall in distinct LDS banks.
__host__ __device__ __forceinline__ int expm_ld(int m) { return (m >= 8 && (m & 1) == 0) ? m + 1 : m; }
// doubles of scratch wg_expm needs: six m x ld matrices and two m-vectors
__host__ __device__ __forceinline__ int expm_scratch(int m) { return 6 * m * expm_ld(m) + 2 * m; }

// C = A * B on the FP64 matrix cores: each wave computes 16 x 16 tiles of C with
// v_mfma_f64_16x16x4 (A fragment 16 x 4: lane l holds A[l % 16][l / 16]; B fragment
// 4 x 16: lane l holds B[l / 16][l % 16]; accumulator: lane l, item v holds
// C[l / 16 + 4 v][l % 16]); out-of-range entries load as zero and are not stored.
typedef double ep_f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wg_gemm(const double* A, const double* B, double* C, int m, int ld) {
  const int nt = (m + 15) >> 4;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int r16 = lane & 15, q = lane >> 4;
  for (int t = w; t < nt * nt; t += nw) {
    const int ti = t / nt, tj = t - (t / nt) * nt;
    const int i0 = 16 * ti, j0 = 16 * tj;
    ep_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    const int ia = i0 + r16, jb = j0 + r16;
    for (int k0 = 0; k0 < m; k0 += 4) {
      const int k = k0 + q;
      const double a = (ia < m && k < m) ? A[(size_t)ia * ld + k] : 0.0;
      const double b = (k < m && jb < m) ? B[(size_t)k * ld + jb] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + q + 4 * v;
      if (i < m && jb < m) C[(size_t)i * ld + jb] = acc[v];
    }
  }
  wg_sync();
}

// 1-norm (max column sum), same value in every thread; eight lanes per column
__device__ __forceinline__ double wg_norm1(const double* A, int m, int ld, double* red) {
  double mx = 0.0;
  const int sub = threadIdx.x & 7;
  for (int j = threadIdx.x >> 3; j < m; j += blockDim.x >> 3) {
    double s = 0.0;
    for (int i = sub; i < m; i += 8) s += fabs(A[(size_t)i * ld + j]);
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 4, 64);
    mx = fmax(mx, s);
  }
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

// Solve A X = B (A destroyed, B <- X) by Gaussian elimination with partial pivoting
// (ties: smallest row index).  Per column k: wave 0 finds the pivot row; rows k and p are
// exchanged in the columns still needed (A columns > k, all of B) while the multipliers
// l_r = A[r][k] / A[p][k] (after the exchange) go to mult[] and the pivot to diag[k]; then
// the trailing update, a thread per column and every ng-th row.  The back substitution
// gives every column of B eight lanes of one wave.  diag, mult: m doubles; ired: >= 1 int.
__device__ __forceinline__ void wg_solve(double* A, double* B, int m, int ld, double* diag, double* mult, int* ired) {
  for (int k = 0; k < m; ++k) {
    if (threadIdx.x < 64) {
      double best = -1.0;
      int bi = m;
      for (int r = k + (int)threadIdx.x; r < m; r += 64) {
        const double v = fabs(A[(size_t)r * ld + k]);
        if (v > best) { best = v; bi = r; }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (threadIdx.x == 0) ired[0] = bi < m ? bi : k;
    }
    __syncthreads();
    const int p = ired[0];
    const double piv = A[(size_t)p * ld + k];
    const int ca = m - k - 1;                 // A columns k+1..m-1, then the m columns of B
    const int cols = ca + m;
    for (int c = threadIdx.x; c < cols; c += blockDim.x) {
      if (p == k) break;
      double* X = c < ca ? A : B;
      const int j = c < ca ? k + 1 + c : c - ca;
      const double t = X[(size_t)k * ld + j];
      X[(size_t)k * ld + j] = X[(size_t)p * ld + j];
      X[(size_t)p * ld + j] = t;
    }
    for (int r = k + 1 + (int)threadIdx.x; r < m; r += blockDim.x)
      mult[r] = (r == p ? A[(size_t)k * ld + k] : A[(size_t)r * ld + k]) / piv;
    if (threadIdx.x == 0) diag[k] = piv;
    __syncthreads();
    const int ng = cols <= (int)blockDim.x ? (int)blockDim.x / cols : 1;
    for (int idx = threadIdx.x; idx < ng * cols; idx += blockDim.x) {
      const int c = idx % cols, g = idx / cols;
      double* X = c < ca ? A : B;
      const int j = c < ca ? k + 1 + c : c - ca;
      const double xk = X[(size_t)k * ld + j];
      for (int r = k + 1 + g; r < m; r += ng) X[(size_t)r * ld + j] -= mult[r] * xk;
    }
    __syncthreads();
  }
  // back substitution: lanes 8g..8g+7 take column j, splitting each row sum by c mod 8
  const int r8 = threadIdx.x & 7;
  for (int j = threadIdx.x >> 3; j < m; j += blockDim.x >> 3) {
    for (int k = m - 1; k >= 0; --k) {
      double s = 0.0;
      for (int c = k + 1 + r8; c < m; c += 8) s += A[(size_t)k * ld + c] * B[(size_t)c * ld + j];
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      const double x = (B[(size_t)k * ld + j] - s) / diag[k];
      if (r8 == (k & 7)) B[(size_t)k * ld + j] = x;   // later read only by this lane
    }
  }
  __syncthreads();
}

// E = exp(Hin).  Hin is m x m with leading dimension ldh; E is returned inside scr with
// leading dimension expm_ld(m).  scr: expm_scratch(m) doubles private to the workgroup
// (LDS or device memory).
__device__ __forceinline__ double* wg_expm(const double* Hin, int ldh, int m, double* scr, double* red, int* ired) {
  const int ld = expm_ld(m);
  const size_t mm = (size_t)m * ld;
  double* B0 = scr;
  double* B1 = scr + mm;
  double* B2 = scr + 2 * mm;
  double* B3 = scr + 3 * mm;
  double* B4 = scr + 4 * mm;
  double* B5 = scr + 5 * mm;
  double* diag = scr + 6 * mm;
  double* mult = diag + m;
  const int n = m * ld;
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int i = idx / ld, j = idx - i * ld;
    if (j < m) B0[idx] = Hin[(size_t)i * ldh + j];
  }
  wg_sync();
  const double nrm = wg_norm1(B0, m, ld, red);
  if (nrm <= 1.0) {
    // Taylor: E = sum_k A^k / k!, stopped when the term's norm drops below 2^-53 ||E||
    double* E = B1;
    double* Tm = B2;
    double* T1 = B3;
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
      const int i = idx / ld, j = idx - i * ld;
      E[idx] = (i == j) ? 1.0 : 0.0;
      Tm[idx] = (i == j) ? 1.0 : 0.0;
    }
    wg_sync();
    for (int k = 1; k <= 60; ++k) {
      wg_gemm(Tm, B0, T1, m, ld);
      const double inv = 1.0 / double(k);
      for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
        const double t = T1[idx] * inv;
        Tm[idx] = t;
        E[idx] += t;
      }
      wg_sync();
      const double tn = wg_norm1(Tm, m, ld, red);
      const double en = wg_norm1(E, m, ld, red);
      if (tn <= 0x1p-53 * en) break;
    }
    return E;
  }
  // s = max(0, ceil(log2(||A||_1 / theta_13))): halvings are exact, so this is the least s
  // with ||A||_1 / theta_13 / 2^s <= 1
  int s = 0;
  double sc = 1.0;
  for (double r = nrm / kTheta13; r > 1.0 && s < 1024; r *= 0.5) {
    ++s;
    sc *= 0.5;
  }
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) B0[idx] *= sc;   // A
  wg_sync();
  const double* c = kPade13.c;
  wg_gemm(B0, B0, B1, m, ld);      // A2
  wg_gemm(B1, B1, B2, m, ld);      // A4
  wg_gemm(B2, B1, B3, m, ld);      // A6
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x)
    B4[idx] = c[13] * B3[idx] + c[11] * B2[idx] + c[9] * B1[idx];
  wg_sync();
  wg_gemm(B3, B4, B5, m, ld);      // A6 (c13 A6 + c11 A4 + c9 A2)
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int i = idx / ld, j = idx - i * ld;
    B5[idx] += c[7] * B3[idx] + c[5] * B2[idx] + c[3] * B1[idx] + ((i == j) ? c[1] : 0.0);
  }
  wg_sync();
  wg_gemm(B0, B5, B4, m, ld);      // U = A (A6 (...) + c7 A6 + c5 A4 + c3 A2 + c1 I)
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x)
    B5[idx] = c[12] * B3[idx] + c[10] * B2[idx] + c[8] * B1[idx];
  wg_sync();
  wg_gemm(B3, B5, B0, m, ld);      // A6 (c12 A6 + c10 A4 + c8 A2); A is no longer needed
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int i = idx / ld, j = idx - i * ld;
    const double v = B0[idx] + c[6] * B3[idx] + c[4] * B2[idx] + c[2] * B1[idx] + ((i == j) ? c[0] : 0.0);
    const double u = B4[idx];
    B0[idx] = v - u;               // Q = V - U
    B4[idx] = v + u;               // P = V + U
  }
  wg_sync();
  wg_solve(B0, B4, m, ld, diag, mult, ired);    // R = Q^{-1} P
  double* R = B4;
  double* Rn = B1;
  for (int qq = 0; qq < s; ++qq) {
    wg_gemm(R, R, Rn, m, ld);
    double* t = R; R = Rn; Rn = t;
  }
  return R;
}

// Out-of-line variant (scratch in LDS or device memory, reached through generic addresses):
// the Krylov kernels call it at check points only, and keeping its matrix-core and solve
// code out of their Arnoldi loop lowers that loop's register spills (c2: 7.15 -> 6.83 ms per
// step) by more than the generic LDS addressing costs the exponential.
__device__ __noinline__ double* wg_expm_call(const double* Hin, int ldh, int m, double* scr, double* red,
                                             int* ired) {
  return wg_expm(Hin, ldh, m, scr, red, ired);
}

}  // namespace ep
