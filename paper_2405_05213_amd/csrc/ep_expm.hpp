// exp(H) of a small dense matrix on one workgroup (Sec. 4.3 of the paper: Taylor series
// when ||H|| <= 1, scaling and squaring otherwise, no eigendecomposition).  The Taylor
// polynomial has the fixed degree 18 and is evaluated in the Paterson-Stockmeyer form
// (Paterson & Stockmeyer, SIAM J. Comput. 2 (1973)): 7 matrix products; when ||H||_1 > 1 it
// is applied to H / 2^s, s = ceil(log2 ||H||_1), and squared s times.  Only matrix products
// (on the FP64 matrix cores) and elementwise passes: no linear solve, whose column-by-column
// latency on one workgroup would exceed all the products together.
// Matrices are row major with leading dimension m and live in LDS when they fit, else in
// device memory private to the calling workgroup; every thread of the workgroup must call.
#pragma once

#include "ep_common.hpp"

namespace ep {

// Degree and scaling threshold: for ||A||_1 <= 1 the omitted terms sum to at most
// sum_{k > 18} 1/k! = 8.7e-18 in norm, and ||e^A|| >= e^{-||A||} >= e^{-1}, so the relative
// truncation error stays below 2.4e-17, under the unit roundoff 2^-53.
constexpr int kTaylorDeg = 18;
constexpr double kTaylorTheta = 1.0;

// 1/k!, k = 0..18, evaluated at compile time
struct Taylor18 {
  double c[kTaylorDeg + 1];
  constexpr Taylor18() : c{} {
    double v = 1.0;
    for (int k = 0; k <= kTaylorDeg; ++k) {
      if (k > 0) v /= double(k);
      c[k] = v;
    }
  }
};
__device__ constexpr Taylor18 kTaylor18{};

__device__ __forceinline__ void wg_sync() { __syncthreads(); }

// Leading dimension of the work matrices: odd for even m >= 8, so that the 16 rows of a
// matrix-core fragment fall in distinct LDS banks.
__host__ __device__ __forceinline__ int expm_ld(int m) { return (m >= 8 && (m & 1) == 0) ? m + 1 : m; }
// doubles of scratch wg_expm needs: six m x ld matrices
__host__ __device__ __forceinline__ int expm_scratch(int m) { return 6 * m * expm_ld(m); }

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

// E = exp(Hin).  Hin is m x m with leading dimension ldh; E is returned inside scr with
// leading dimension expm_ld(m).  scr: expm_scratch(m) doubles private to the workgroup
// (LDS or device memory); red: one double per wave.
__device__ __forceinline__ double* wg_expm(const double* Hin, int ldh, int m, double* scr, double* red) {
  const int ld = expm_ld(m);
  const size_t mm = (size_t)m * ld;
  double* A = scr;
  double* A2 = scr + mm;
  double* A3 = scr + 2 * mm;
  double* A4 = scr + 3 * mm;
  double* X = scr + 4 * mm;
  double* Y = scr + 5 * mm;
  const int n = m * ld;
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int i = idx / ld, j = idx - i * ld;
    if (j < m) A[idx] = Hin[(size_t)i * ldh + j];
  }
  wg_sync();
  // s = max(0, ceil(log2(||H||_1 / theta))): halvings are exact, so this is the least s with
  // ||H||_1 / theta / 2^s <= 1
  const double nrm = wg_norm1(A, m, ld, red);
  int s = 0;
  double sc = 1.0;
  for (double r = nrm / kTaylorTheta; r > 1.0 && s < 1024; r *= 0.5) {
    ++s;
    sc *= 0.5;
  }
  if (s > 0) {
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) A[idx] *= sc;
    wg_sync();
  }
  const double* c = kTaylor18.c;
  wg_gemm(A, A, A2, m, ld);
  wg_gemm(A2, A, A3, m, ld);
  wg_gemm(A2, A2, A4, m, ld);
  // T(A) = B_0 + A^4 (B_1 + A^4 (B_2 + A^4 (B_3 + A^4 B_4))), B_j = sum_{i<4} c_{4j+i} A^i
  // (B_4 = c_16 I + c_17 A + c_18 A^2): Horner's rule in A^4
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int i = idx / ld, j = idx - i * ld;
    X[idx] = c[17] * A[idx] + c[18] * A2[idx] + ((i == j) ? c[16] : 0.0);
  }
  wg_sync();
  for (int b = 3; b >= 0; --b) {
    wg_gemm(A4, X, Y, m, ld);
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
      const int i = idx / ld, j = idx - i * ld;
      X[idx] = Y[idx] + c[4 * b + 1] * A[idx] + c[4 * b + 2] * A2[idx] + c[4 * b + 3] * A3[idx] +
               ((i == j) ? c[4 * b] : 0.0);
    }
    wg_sync();
  }
  double* R = X;
  double* Rn = Y;
  for (int q = 0; q < s; ++q) {
    wg_gemm(R, R, Rn, m, ld);
    double* t = R; R = Rn; Rn = t;
  }
  return R;
}

// Out-of-line variant (scratch in LDS or device memory, reached through generic addresses):
// the Krylov kernels call it at check points only, and keeping its matrix-core code out of
// their Arnoldi loop lowers that loop's register spills (c2 with the earlier Pade form of the
// exponential: 7.15 -> 6.83 ms per step) by more than the generic LDS addressing costs it.
__device__ __noinline__ double* wg_expm_call(const double* Hin, int ldh, int m, double* scr, double* red) {
  return wg_expm(Hin, ldh, m, scr, red);
}

}  // namespace ep
