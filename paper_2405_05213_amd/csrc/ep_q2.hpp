// Quadratic 27-node hexahedra (Q2): the paper's element (Sec. 2.2: quadratic Lagrange
// interpolation; Gauss quadrature for the internal force and the loads, Gauss-Lobatto for a
// diagonal mass).  Local node a = i + 3 j + 9 k sits at (i-1, j-1, k-1); Gauss point
// q = qi + 3 qj + 9 qk at (g_qi, g_qj, g_qk), g = (-sqrt(3/5), 0, sqrt(3/5)), weights
// (5/9, 8/9, 5/9) per direction.  Shape functions N_a = l_i(xi) l_j(eta) l_k(zeta) with the
// quadratic Lagrange polynomials l_0 = x(x-1)/2, l_1 = 1 - x^2, l_2 = x(x+1)/2.
//
// Element forces run on 32 lanes per element (lanes 0..26 active): lane q forms the
// gradients and the stress at Gauss point q from the element's nodal values, then lane a
// sums node a's force over the 27 points.  Both use sum factorisation over the
// tensor-product basis (three one-dimensional contractions, the values of the lane's line
// taken by shuffles).  No LDS: the persistent Krylov kernel keeps its LDS
// for the basis slices.
#pragma once

#include "ep_device.hpp"

namespace ep {

constexpr int kQ2Nodes = 27;
constexpr int kQ2Lanes = 32;
constexpr double kG3 = 0.77459666924148337704;   // sqrt(3/5)

__host__ __device__ constexpr double q2_gpt(int i) { return i == 0 ? -kG3 : (i == 1 ? 0.0 : kG3); }
__host__ __device__ constexpr double q2_gw(int i) { return i == 1 ? 8.0 / 9.0 : 5.0 / 9.0; }
// Lagrange polynomial l_i and its derivative at x
__host__ __device__ constexpr double lag3(int i, double x) {
  return i == 0 ? 0.5 * x * (x - 1.0) : (i == 1 ? 1.0 - x * x : 0.5 * x * (x + 1.0));
}
__host__ __device__ constexpr double dlag3(int i, double x) { return i == 0 ? x - 0.5 : (i == 1 ? -2.0 * x : x + 0.5); }

// dN_a/dxi_d at Gauss point q (reference element)
template <typename T>
__device__ __forceinline__ void q2_dN(int a, int q, T (&d)[3]) {
  const int i = a % 3, j = (a / 3) % 3, k = a / 9;
  const double x = q2_gpt(q % 3), y = q2_gpt((q / 3) % 3), z = q2_gpt(q / 9);
  const double li = lag3(i, x), lj = lag3(j, y), lk = lag3(k, z);
  d[0] = T(dlag3(i, x) * lj * lk);
  d[1] = T(li * dlag3(j, y) * lk);
  d[2] = T(li * lj * dlag3(k, z));
}

template <typename T>
__device__ __forceinline__ T shfl_q2(T v, int src_lane) {
  return __shfl(v, src_lane, 64);
}

// Select among three per-coordinate constants by the lane's coordinate c (0, 1, 2).
template <typename T>
__device__ __forceinline__ T sel3(int c, double v0, double v1, double v2) {
  return c == 0 ? T(v0) : (c == 1 ? T(v1) : T(v2));
}
// l_n(g_c) and l_n'(g_c): polynomial n (a compile-time index) at the lane's Gauss coordinate c
template <typename T>
__device__ __forceinline__ T lq(int n, int c) {
  return sel3<T>(c, lag3(n, q2_gpt(0)), lag3(n, q2_gpt(1)), lag3(n, q2_gpt(2)));
}
template <typename T>
__device__ __forceinline__ T dlq(int n, int c) {
  return sel3<T>(c, dlag3(n, q2_gpt(0)), dlag3(n, q2_gpt(1)), dlag3(n, q2_gpt(2)));
}
// l_c(g_n) and l_c'(g_n): the lane's polynomial c at Gauss point n (a compile-time index)
template <typename T>
__device__ __forceinline__ T lp(int c, int n) {
  return sel3<T>(c, lag3(0, q2_gpt(n)), lag3(1, q2_gpt(n)), lag3(2, q2_gpt(n)));
}
template <typename T>
__device__ __forceinline__ T dlp(int c, int n) {
  return sel3<T>(c, dlag3(0, q2_gpt(n)), dlag3(1, q2_gpt(n)), dlag3(2, q2_gpt(n)));
}

// Gradient at the lane's Gauss point (x, y, z) of the field whose nodal values lane
// a = i + 3 j + 9 k of the group holds in va[3], by sum factorisation over the tensor-product
// basis: contract along xi (value and derivative), then eta, then zeta, each step taking the
// three values of the lane's line by shuffles (18 per component instead of 27 sums of 27).
// G[i][k] = sum_a va_i dN_a/dX_k with dN/dX = dN/dxi J^{-1}.
template <typename T>
__device__ __forceinline__ void q2_grad(const T (&va)[3], int x, int y, int z, int base, const T* Jinv,
                                        T (&G)[3][3]) {
  T Dxi[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T a0 = T(0), a1 = T(0);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const T v = shfl_q2(va[i], base + n + 3 * y + 9 * z);
      a0 += v * lq<T>(n, x);
      a1 += v * dlq<T>(n, x);
    }
    T bx = T(0), by = T(0), bz = T(0);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int src = base + x + 3 * n + 9 * z;
      const T p0 = shfl_q2(a0, src), p1 = shfl_q2(a1, src);
      bx += p1 * lq<T>(n, y);
      by += p0 * dlq<T>(n, y);
      bz += p0 * lq<T>(n, y);
    }
    T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int src = base + x + 3 * y + 9 * n;
      gx += shfl_q2(bx, src) * lq<T>(n, z);
      gy += shfl_q2(by, src) * lq<T>(n, z);
      gz += shfl_q2(bz, src) * dlq<T>(n, z);
    }
    Dxi[i][0] = gx;
    Dxi[i][1] = gy;
    Dxi[i][2] = gz;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      G[i][k] = Dxi[i][0] * Jinv[0 * 3 + k] + Dxi[i][1] * Jinv[1 * 3 + k] + Dxi[i][2] * Jinv[2 * 3 + k];
}

// Element forces of Q2 element e into its 27 slots (slot a n_e + e).  Every lane of the
// 32-lane group must call with the same e.  x_a = src[dof] * srcscale (* mih[dof]); FP32: the
// element's inputs relative to node 0 (taken in FP64).  Returns false if a secant set has
// J <= 0 at one of this lane's points.
template <typename T, int MODEL>
__device__ __forceinline__ bool elem_force_q2(const Mesh& M, const OpArgs& op, int e, const double* src,
                                              double srcscale, bool scale_mih, T* F) {
  const int l = threadIdx.x & (kQ2Lanes - 1), base = (threadIdx.x & 63) & ~(kQ2Lanes - 1);
  const bool act = l < kQ2Nodes;
  const int a = act ? l : 0;
  const int cx = a % 3, cy = (a / 3) % 3, cz = a / 9;
  const int nd = M.conn[(size_t)e * kQ2Nodes + a];
  constexpr bool shift = sizeof(T) == 4;
  // nodal values of this lane's node: the input and the secant sets' displacements
  T xa[3], ua[2][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const size_t d = (size_t)nd * 3 + i;
    double v = src[d] * srcscale;
    if (scale_mih) v *= M.mih[d];
    const double v0 = shift ? __shfl(v, base, 64) : 0.0;
    xa[i] = T(v - v0);
  }
  const int nsets = (MODEL == kLinear) ? 0 : op.nsets;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double v = 0.0;
      if (s < nsets) v = op.ulin[s][(size_t)nd * 3 + i];
      const double v0 = shift ? __shfl(v, base, 64) : 0.0;
      ua[s][i] = T(v - v0);
    }
  // ---- lane = Gauss point q: gradients, stress, St = w det J S J^{-T}
  const int q = a;
  T Jinv[9], wdet;
  const size_t gi = (M.congruent ? (size_t)q : (size_t)e * kQ2Nodes + q) * 10;
  if (sizeof(T) == 8) {
#pragma unroll
    for (int k = 0; k < 9; ++k) Jinv[k] = T(M.geo[gi + k]);
    wdet = T(M.geo[gi + 9]);
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) Jinv[k] = T(M.geo32[gi + k]);
    wdet = T(M.geo32[gi + 9]);
  }
  if (!act) wdet = T(0);
  T X[3][3];
  q2_grad(xa, cx, cy, cz, base, Jinv, X);
  T S[3][3];
  bool ok = true;
  if (nsets == 0) {
    double lam_d, mu_d;
    rest_lame(M.model, M.mp, lam_d, mu_d);
    const T lam = T(lam_d), mu = T(mu_d);
    const T tr = X[0][0] + X[1][1] + X[2][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) S[i][k] = mu * (X[i][k] + X[k][i]) + (i == k ? lam * tr : T(0));
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) S[i][k] = T(0);
    for (int s = 0; s < nsets; ++s) {
      T Du[3][3];
      q2_grad(ua[s], cx, cy, cz, base, Jinv, Du);
      if constexpr (MODEL == kSVK) {
        double lam_d, mu_d;
        rest_lame(kSVK, M.mp, lam_d, mu_d);
        SecantSVK<T> sv;
        svk_coeffs(Du, T(lam_d), T(mu_d), sv);
        svk_apply(sv, T(lam_d), T(mu_d), T(op.wts[s]), X, S);
      } else if constexpr (MODEL != kLinear) {
        ok &= secant_stress_add<T, MODEL>(Du, X, M.mp, T(op.wts[s]), S) || !act;
      }
    }
  }
  T St[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      St[3 * i + j] = wdet * (S[i][0] * Jinv[j * 3 + 0] + S[i][1] * Jinv[j * 3 + 1] + S[i][2] * Jinv[j * 3 + 2]);
  // ---- lane = node a: f_a,i = sum_q sum_d St_q[i][d] dN_a/dxi_d(q), the transposed sum
  // factorisation: contract the Gauss points along zeta, then eta, then xi
  T f[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T t0 = T(0), t1 = T(0), t2 = T(0);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int src = base + cx + 3 * cy + 9 * n;
      t0 += shfl_q2(St[3 * i], src) * lp<T>(cz, n);
      t1 += shfl_q2(St[3 * i + 1], src) * lp<T>(cz, n);
      t2 += shfl_q2(St[3 * i + 2], src) * dlp<T>(cz, n);
    }
    T u0 = T(0), v = T(0);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int src = base + cx + 3 * n + 9 * cz;
      u0 += shfl_q2(t0, src) * lp<T>(cy, n);
      v += shfl_q2(t1, src) * dlp<T>(cy, n) + shfl_q2(t2, src) * lp<T>(cy, n);
    }
    T fi = T(0);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int src = base + n + 3 * cy + 9 * cz;
      fi += shfl_q2(u0, src) * dlp<T>(cx, n) + shfl_q2(v, src) * lp<T>(cx, n);
    }
    f[i] = fi;
  }
  if (act) {
#pragma unroll
    for (int i = 0; i < 3; ++i) F[((size_t)a * M.n_elems + e) * 3 + i] = f[i];
  }
  return ok;
}

}  // namespace ep
