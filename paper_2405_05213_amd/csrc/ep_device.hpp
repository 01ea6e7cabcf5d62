// Device building blocks: hex8 element kernels, constitutive coefficients, reductions and
// the workgroup-team synchronisation used by the persistent Krylov kernels.
#pragma once

#include "ep_common.hpp"

namespace ep {

// ---------------------------------------------------------------------------------------
// hex8 reference element (VTK order) and the 2x2x2 Gauss rule (Sec. 2.2).
// Node a sits at (sx, sy, sz) in {-1,1}^3; Gauss point q at g * (signs of node q).
// ---------------------------------------------------------------------------------------
__host__ __device__ constexpr int node_sx(int a) { return (a == 1 || a == 2 || a == 5 || a == 6) ? 1 : -1; }
__host__ __device__ constexpr int node_sy(int a) { return (a == 2 || a == 3 || a == 6 || a == 7) ? 1 : -1; }
__host__ __device__ constexpr int node_sz(int a) { return a >= 4 ? 1 : -1; }
constexpr double kGauss = 0.57735026918962576451;   // 1/sqrt(3)

// Factors (1 + s g_d) of the Gauss point q for node signs s = +1 (p) and -1 (m).
template <typename T>
struct QFactors {
  T p[3], m[3];
  __device__ __forceinline__ explicit QFactors(int q) {
    const int s[3] = {node_sx(q), node_sy(q), node_sz(q)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      p[d] = T(1) + T(kGauss) * T(s[d]);
      m[d] = T(1) - T(kGauss) * T(s[d]);
    }
  }
  // dN_a / dxi_j at this point (a compile-time after unrolling)
  __device__ __forceinline__ T dN(int a, int j) const {
    const int s[3] = {node_sx(a), node_sy(a), node_sz(a)};
    T f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) f[d] = s[d] > 0 ? p[d] : m[d];
    const T eighth = T(0.125);
    if (j == 0) return eighth * T(s[0]) * f[1] * f[2];
    if (j == 1) return eighth * T(s[1]) * f[0] * f[2];
    return eighth * T(s[2]) * f[0] * f[1];
  }
};

// Gradient at a Gauss point: G[i][k] = sum_a x[a][i] dN_a/dX_k with dN/dX = dN/dxi Jinv.
template <typename T>
__device__ __forceinline__ void grad_at(const QFactors<T>& Q, const T (&x)[8][3], const T* Jinv, T (&G)[3][3]) {
  T Dxi[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Dxi[i][j] = T(0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const T d0 = Q.dN(a, 0), d1 = Q.dN(a, 1), d2 = Q.dN(a, 2);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Dxi[i][0] += x[a][i] * d0;
      Dxi[i][1] += x[a][i] * d1;
      Dxi[i][2] += x[a][i] * d2;
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      G[i][k] = Dxi[i][0] * Jinv[0 * 3 + k] + Dxi[i][1] * Jinv[1 * 3 + k] + Dxi[i][2] * Jinv[2 * 3 + k];
}

// f[a][i] += wdet * sum_k S[i][k] dN_a/dX_k
template <typename T>
__device__ __forceinline__ void scatter_at(const QFactors<T>& Q, const T (&S)[3][3], const T* Jinv, T wdet,
                                           T (&f)[8][3]) {
  T St[3][3];   // wdet * S Jinv^T
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      St[i][j] = wdet * (S[i][0] * Jinv[j * 3 + 0] + S[i][1] * Jinv[j * 3 + 1] + S[i][2] * Jinv[j * 3 + 2]);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const T d0 = Q.dN(a, 0), d1 = Q.dN(a, 1), d2 = Q.dN(a, 2);
#pragma unroll
    for (int i = 0; i < 3; ++i) f[a][i] += St[i][0] * d0 + St[i][1] * d1 + St[i][2] * d2;
  }
}

// ---------------------------------------------------------------------------------------
// The H-matrix of App. A as an operator on X = grad x at one Gauss point.  App. A builds
// H(u) from the internal virtual work int grad w : (F S) dV; its blocks H_AB act on x as
//   Phi(D, X) = S_lin(D, X) + X S(D),     S_lin(D, D) = S(D)  (second Piola-Kirchhoff),
// so that Phi(D, D) = F S and H(u) u = R(u).  For the Yeoh solid (App. A, last equation,
// with the 1/2 of the internal virtual work) and the compressible Neo-Hookean solid built
// the same way, the printed terms sum to
//   Phi = a sym(X N) + (W : X) Ci + X S,   sym(Z) = (Z + Z^T) / 2,
// with Ci = C^{-1} = F^{-1} F^{-T}, N = F^{-1} + Ci, S = Ci Sigma and
//   Yeoh: a = alpha_e, W = -(a/3)(2I + D) + beta_e P_e, Sigma = a dev(E2) + beta_e (J-1) I
//   NH:   a = mu,      W = lambda l(J) P_e,             Sigma = mu E2 + lambda ln J I
// (E2 = C - I = D + D^T + D^T D, dev(E2) = E2 - tr(E2)/3 I, l(J) = ln J / (J - 1),
// beta_e = 2 J / D1, P_e the matrix of App. A with J - 1 = P_e : D).  The first terms
// are the printed F^{-1}, F^{-T}, C^{-1} D^T and D C^{-1} blocks (F^{-1} - C^{-1} D^T / 2
// = N / 2), the (W : X) Ci term the (2I + D^T) and P_e^T blocks, X S the two blocks with
// grad N_B . [..] . grad N_A.  S = Ci Sigma equals alpha (I - Ci tr C / 3) + beta (J-1) Ci
// without the cancellation of I - Ci near D = 0.
// ---------------------------------------------------------------------------------------
template <typename T>
struct Secant {
  T a;
  T N[3][3];
  T W[3][3];
  T S[3][3];
  T Ci[6];      // symmetric: 00 11 22 01 12 02
};

__device__ __forceinline__ double ep_log1p(double x) { return log1p(x); }
__device__ __forceinline__ float ep_log1p(float x) { return log1pf(x); }
__device__ __forceinline__ double ep_exp(double x) { return exp(x); }
__device__ __forceinline__ float ep_exp(float x) { return expf(x); }

// 1/x: correctly rounded in FP64; in FP32 the hardware reciprocal (1 ulp), whose error is
// far below the FP32 operator's own rounding (the IEEE division costs about ten instructions
// in the secant stress's Gauss-point loop, which is bound by its instruction count)
__device__ __forceinline__ double ep_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float ep_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ln(1+x)/x, continuous through x = 0
template <typename T>
__device__ __forceinline__ T log_ratio(T x) {
  const T ax = x < T(0) ? -x : x;
  if (ax < T(sizeof(T) == 8 ? 1e-8 : 1e-4)) return T(1) - T(0.5) * x + x * x * T(1.0 / 3.0);
  return ep_log1p(x) * ep_rcp(x);
}

// J^{-2/3} for J = 1 + x > 0: an FP32 estimate of y = J^{-1/3} refined by Newton steps on
// y^{-3} = J, y <- y (4 - J y^3) / 3, whose relative error squares at each step, instead of
// two library transcendentals.  FP64: two steps (2e-6 -> 1e-11 -> rounding; 8e-16 relative
// over 0.05 <= J <= 20); FP32: the hardware log2 / exp2 estimate and one step.  Outside
// 1e-30 < J < 1e30, beyond the estimate's range, the logarithmic form exp(-2/3 ln(1 + x)).
template <typename T>
__device__ __forceinline__ T j_pow_m23(T J, T x) {
  if constexpr (sizeof(T) == 8) {
    if (J > 1e-30 && J < 1e30) {
      double y = (double)exp2f(-log2f((float)J) * (1.0f / 3.0f));
      y = y * (4.0 - J * y * y * y) * (1.0 / 3.0);
      y = y * (4.0 - J * y * y * y) * (1.0 / 3.0);
      return y * y;
    }
  } else {
    if (J > 1e-30f && J < 1e30f) {
      float y = __builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(J) * (1.0f / 3.0f));
      y = y * (4.0f - J * y * y * y) * (1.0f / 3.0f);
      return y * y;
    }
  }
  return ep_exp(T(-2.0 / 3.0) * ep_log1p(x));
}

__host__ __device__ constexpr int sym_idx(int i, int k) {
  return i == k ? i : ((i + k == 1) ? 3 : ((i + k == 3) ? 4 : 5));
}

// Coefficients of Phi at D (Neo-Hookean or Yeoh).  Returns false if J <= 0 (or not finite).
template <typename T, int MODEL>
__device__ __forceinline__ bool secant_coeffs(const T (&D)[3][3], const double* mp, Secant<T>& s) {
  // polynomial cofactor of D
  T c[3][3];
  c[0][0] = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  c[0][1] = D[1][2] * D[2][0] - D[1][0] * D[2][2];
  c[0][2] = D[1][0] * D[2][1] - D[1][1] * D[2][0];
  c[1][0] = D[0][2] * D[2][1] - D[0][1] * D[2][2];
  c[1][1] = D[0][0] * D[2][2] - D[0][2] * D[2][0];
  c[1][2] = D[0][1] * D[2][0] - D[0][0] * D[2][1];
  c[2][0] = D[0][1] * D[1][2] - D[0][2] * D[1][1];
  c[2][1] = D[0][2] * D[1][0] - D[0][0] * D[1][2];
  c[2][2] = D[0][0] * D[1][1] - D[0][1] * D[1][0];
  const T trD = D[0][0] + D[1][1] + D[2][2];
  // P_e = I + (trD I - D^T)/2 + cof(D)/3 (App. A), J - 1 = P_e : D; kept in W for now
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      s.W[i][k] = (i == k ? T(1) + T(0.5) * trD : T(0)) - T(0.5) * D[k][i] + c[i][k] * T(1.0 / 3.0);
  T x = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) x += s.W[i][k] * D[i][k];
  const T J = T(1) + x;
  if (!(J > T(0))) return false;
  // F^{-1} = cof(F)^T / J with cof(I + D) = cof(D) + (trD I - D^T) + I; N = F^{-1} for now
  const T Jinv = T(1) / J;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      s.N[i][k] = (c[k][i] + (i == k ? T(1) + trD : T(0)) - D[i][k]) * Jinv;
  // Ci = F^{-1} F^{-T}
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = i; k < 3; ++k)
      s.Ci[sym_idx(i, k)] = s.N[i][0] * s.N[k][0] + s.N[i][1] * s.N[k][1] + s.N[i][2] * s.N[k][2];
  // E2 = D + D^T + D^T D (symmetric)
  T E2[6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = i; k < 3; ++k)
      E2[sym_idx(i, k)] = D[i][k] + D[k][i] + D[0][i] * D[0][k] + D[1][i] * D[1][k] + D[2][i] * D[2][k];
  T Sg[6];   // Sigma
  T a;
  if (MODEL == kNH) {
    const T mu = T(mp[0]), lam = T(mp[1]);
    a = mu;
    const T l = log_ratio(x);
    const T vol = lam * l * x;      // lambda ln J
#pragma unroll
    for (int t = 0; t < 6; ++t) Sg[t] = mu * E2[t] + (t < 3 ? vol : T(0));
    const T f = lam * l;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) s.W[i][k] *= f;
  } else {   // Yeoh
    const T C10 = T(mp[0]), C20 = T(mp[1]), C30 = T(mp[2]), D1 = T(mp[3]);
    const T Jm23 = j_pow_m23(J, x);
    const T trE2 = E2[0] + E2[1] + E2[2];
    const T z = (T(3) + trE2) * Jm23 - T(3);     // I1bar - 3, tr C = 3 + tr E2
    a = T(2) * Jm23 * (C10 + T(2) * C20 * z + T(3) * C30 * z * z);
    const T beta = T(2) / D1 * J;
    const T bj = beta * x;
#pragma unroll
    for (int t = 0; t < 6; ++t) Sg[t] = a * E2[t] + (t < 3 ? bj - a * trE2 * T(1.0 / 3.0) : T(0));
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        s.W[i][k] = -(a * T(1.0 / 3.0)) * ((i == k ? T(2) : T(0)) + D[i][k]) + beta * s.W[i][k];
  }
  s.a = a;
  // S = Ci Sigma
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      s.S[i][k] = s.Ci[sym_idx(i, 0)] * Sg[sym_idx(0, k)] + s.Ci[sym_idx(i, 1)] * Sg[sym_idx(1, k)] +
                  s.Ci[sym_idx(i, 2)] * Sg[sym_idx(2, k)];
  // N = F^{-1} + Ci
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) s.N[i][k] += s.Ci[sym_idx(i, k)];
  return true;
}

// P += w * Phi(D, X) for the Neo-Hookean or Yeoh solid in one pass, the coefficients used
// as soon as they are formed (fewer values live at once than secant_coeffs + secant_apply):
//   W : X = -(a/3)(2 tr X + D : X) + b (P_e : X)     (Yeoh; NH: lambda l(J) (P_e : X))
//   Fi = F^{-1}, Ci = Fi Fi^T, Y = X Ci, Z = X Fi + Y = X N, X S = X Ci Sigma = Y Sigma
//   P += w [a (Z + Z^T) / 2 + (W : X) Ci + Y Sigma].
// Returns false if J <= 0 (or not finite).
template <typename T, int MODEL>
__device__ __forceinline__ bool secant_stress_add(const T (&D)[3][3], const T (&X)[3][3], const double* mp, T w,
                                                  T (&P)[3][3]) {
  T c[3][3];
  c[0][0] = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  c[0][1] = D[1][2] * D[2][0] - D[1][0] * D[2][2];
  c[0][2] = D[1][0] * D[2][1] - D[1][1] * D[2][0];
  c[1][0] = D[0][2] * D[2][1] - D[0][1] * D[2][2];
  c[1][1] = D[0][0] * D[2][2] - D[0][2] * D[2][0];
  c[1][2] = D[0][1] * D[2][0] - D[0][0] * D[2][1];
  c[2][0] = D[0][1] * D[1][2] - D[0][2] * D[1][1];
  c[2][1] = D[0][2] * D[1][0] - D[0][0] * D[1][2];
  c[2][2] = D[0][0] * D[1][1] - D[0][1] * D[1][0];
  const T trD = D[0][0] + D[1][1] + D[2][2];
  T x = T(0), pex = T(0), dx = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T pe = (i == k ? T(1) + T(0.5) * trD : T(0)) - T(0.5) * D[k][i] + c[i][k] * T(1.0 / 3.0);
      x += pe * D[i][k];
      pex += pe * X[i][k];
      dx += D[i][k] * X[i][k];
    }
  const T J = T(1) + x;
  if (!(J > T(0))) return false;
  const T trX = X[0][0] + X[1][1] + X[2][2];
  const T Jinv = ep_rcp(J);
  T Fi[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) Fi[i][k] = (c[k][i] + (i == k ? T(1) + trD : T(0)) - D[i][k]) * Jinv;
  T Ci[6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = i; k < 3; ++k)
      Ci[sym_idx(i, k)] = Fi[i][0] * Fi[k][0] + Fi[i][1] * Fi[k][1] + Fi[i][2] * Fi[k][2];
  T Y[3][3], Z[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Y[i][k] = X[i][0] * Ci[sym_idx(0, k)] + X[i][1] * Ci[sym_idx(1, k)] + X[i][2] * Ci[sym_idx(2, k)];
      Z[i][k] = Y[i][k] + X[i][0] * Fi[0][k] + X[i][1] * Fi[1][k] + X[i][2] * Fi[2][k];
    }
  T E2[6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = i; k < 3; ++k)
      E2[sym_idx(i, k)] = D[i][k] + D[k][i] + D[0][i] * D[0][k] + D[1][i] * D[1][k] + D[2][i] * D[2][k];
  T a, wx, sd, sg;         // Sigma = sg E2 + sd I
  if (MODEL == kNH) {
    const T mu = T(mp[0]), lam = T(mp[1]);
    const T l = log_ratio(x);
    a = mu;
    wx = lam * l * pex;
    sg = mu;
    sd = lam * l * x;
  } else {
    const T C10 = T(mp[0]), C20 = T(mp[1]), C30 = T(mp[2]), D1 = T(mp[3]);
    const T Jm23 = j_pow_m23(J, x);
    const T trE2 = E2[0] + E2[1] + E2[2];
    const T z = (T(3) + trE2) * Jm23 - T(3);
    a = T(2) * Jm23 * (C10 + T(2) * C20 * z + T(3) * C30 * z * z);
    const T beta = T(2) / D1 * J;
    wx = -(a * T(1.0 / 3.0)) * (T(2) * trX + dx) + beta * pex;
    sg = a;
    sd = beta * x - a * trE2 * T(1.0 / 3.0);
  }
  const T ah = T(0.5) * w * a, bw = w * wx, ws = w * sg, wd = w * sd;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T ys = Y[i][0] * E2[sym_idx(0, k)] + Y[i][1] * E2[sym_idx(1, k)] + Y[i][2] * E2[sym_idx(2, k)];
      P[i][k] += ah * (Z[i][k] + Z[k][i]) + bw * Ci[sym_idx(i, k)] + ws * ys + wd * Y[i][k];
    }
  return true;
}

// P += w * [a sym(X N) + (W : X) Ci + X S]
template <typename T>
__device__ __forceinline__ void secant_apply(const Secant<T>& s, T w, const T (&X)[3][3], T (&P)[3][3]) {
  T wx = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) wx += s.W[i][k] * X[i][k];
  T Z[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) Z[i][k] = X[i][0] * s.N[0][k] + X[i][1] * s.N[1][k] + X[i][2] * s.N[2][k];
  const T ah = T(0.5) * w * s.a, bw = w * wx;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T xs = X[i][0] * s.S[0][k] + X[i][1] * s.S[1][k] + X[i][2] * s.S[2][k];
      P[i][k] += ah * (Z[i][k] + Z[k][i]) + bw * s.Ci[sym_idx(i, k)] + w * xs;
    }
}

// St. Venant-Kirchhoff (App. A, its H-matrix with the leading 1/2): the printed blocks act
// on X = grad x as
//   lambda ((I + D/2) : X) I + mu (X + X^T + (X^T D + D^T X) / 2) + X S,
// S = lambda tr(E) I + 2 mu E = (lambda tr(E2) / 2) I + mu E2 (the nodal sum S_SVK,e).
// Written as lambda (Hh : X) I + mu sym(B X) + X S with Hh = I + D/2, B = 2I + D^T.
template <typename T>
struct SecantSVK {
  T Hh[3][3];
  T S[6];       // symmetric: 00 11 22 01 12 02
};

template <typename T>
__device__ __forceinline__ void svk_coeffs(const T (&D)[3][3], T lam, T mu, SecantSVK<T>& s) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) s.Hh[i][k] = T(0.5) * D[i][k] + (i == k ? T(1) : T(0));
  T E2[6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = i; k < 3; ++k)
      E2[sym_idx(i, k)] = D[i][k] + D[k][i] + D[0][i] * D[0][k] + D[1][i] * D[1][k] + D[2][i] * D[2][k];
  const T lt = T(0.5) * lam * (E2[0] + E2[1] + E2[2]);
#pragma unroll
  for (int t = 0; t < 6; ++t) s.S[t] = mu * E2[t] + (t < 3 ? lt : T(0));
}

// P += w * [lambda (Hh : X) I + mu sym(B X) + X S], B = 2 Hh^T (= 2I + D^T)
template <typename T>
__device__ __forceinline__ void svk_apply(const SecantSVK<T>& s, T lam, T mu, T w, const T (&X)[3][3],
                                          T (&P)[3][3]) {
  T c = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) c += s.Hh[i][k] * X[i][k];
  T Y[3][3];   // Hh^T X = B X / 2
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) Y[i][k] = s.Hh[0][i] * X[0][k] + s.Hh[1][i] * X[1][k] + s.Hh[2][i] * X[2][k];
  const T lc = w * lam * c, wm = w * mu;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T xs = X[i][0] * s.S[sym_idx(0, k)] + X[i][1] * s.S[sym_idx(1, k)] + X[i][2] * s.S[sym_idx(2, k)];
      P[i][k] += (i == k ? lc : T(0)) + wm * (Y[i][k] + Y[k][i]) + w * xs;
    }
}

// Lame constants of the linear material (E, nu) or of the rest-state tangent.
__device__ __forceinline__ void rest_lame(int model, const double* mp, double& lam, double& mu) {
  if (model == kLinear) {
    const double E = mp[0], nu = mp[1];
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    mu = E / (2.0 * (1.0 + nu));
  } else if (model == kNH) {
    mu = mp[0];
    lam = mp[1];
  } else if (model == kSVK) {
    lam = mp[0];
    mu = mp[1];
  } else {
    mu = 2.0 * mp[0];
    lam = 2.0 / mp[3] - 2.0 * mu / 3.0;
  }
}

// ---------------------------------------------------------------------------------------
// Element force of one element in nodal form (8-node sums at each Gauss point):
// f_e = sum_q w detJ S(grad x) . grad N.  The linear material keeps this form: in the
// kernels of the linear operator the modal form's extra live values cost register spills
// (the single-instance FP64 kernel: 97 -> 269 spilled registers) for little VALU work saved.
//   x_a = src[dof] * srcscale (* mih[dof] when scale_mih)
// ---------------------------------------------------------------------------------------
template <typename T, int MODEL>
__device__ __forceinline__ bool elem_force_nodal(const Mesh& M, const OpArgs& op, int e, const double* src,
                                           double srcscale, bool scale_mih, T (&f)[8][3]) {
  int nd[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) nd[a] = M.conn[(size_t)e * 8 + a];
  // In FP32 the element's inputs are taken relative to node 0 (in FP64 before rounding):
  // the forces depend on gradients only, and a large common translation would otherwise
  // cost the deformation its significant bits.
  constexpr bool shift = sizeof(T) == 4;
  T x[8][3];
  double x0[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t d = (size_t)nd[a] * 3 + i;
      double v = src[d] * srcscale;
      if (scale_mih) v *= M.mih[d];
      if (shift && a == 0) x0[i] = v;
      x[a][i] = T(v - x0[i]);
      f[a][i] = T(0);
    }
  const int nsets = (MODEL == kLinear) ? 0 : op.nsets;
  T u0[8][3], u1[8][3];
  if (nsets >= 1) {
    const double* ul = op.ulin[0];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        u0[a][i] = T(ul[(size_t)nd[a] * 3 + i] - (shift ? ul[(size_t)nd[0] * 3 + i] : 0.0));
  }
  if (nsets >= 2) {
    const double* ul = op.ulin[1];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        u1[a][i] = T(ul[(size_t)nd[a] * 3 + i] - (shift ? ul[(size_t)nd[0] * 3 + i] : 0.0));
  }
  double lam_d, mu_d;
  rest_lame(M.model, M.mp, lam_d, mu_d);
  const T lam = T(lam_d), mu = T(mu_d);
  bool ok = true;
  for (int q = 0; q < 8; ++q) {
    const QFactors<T> Q(q);
    T Jinv[9], wdet;
    const size_t gi = (M.congruent ? (size_t)q : (size_t)e * 8 + q) * 10;
    if (sizeof(T) == 8) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Jinv[k] = T(M.geo[gi + k]);
      wdet = T(M.geo[gi + 9]);
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) Jinv[k] = T(M.geo32[gi + k]);
      wdet = T(M.geo32[gi + 9]);
    }
    T X[3][3];
    grad_at(Q, x, Jinv, X);
    T S[3][3];
    if (nsets == 0) {
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
      if constexpr (MODEL == kSVK) {
        T Du[3][3];
        SecantSVK<T> sv;
        grad_at(Q, u0, Jinv, Du);
        svk_coeffs(Du, lam, mu, sv);
        svk_apply(sv, lam, mu, T(op.wts[0]), X, S);
        if (nsets >= 2) {
          grad_at(Q, u1, Jinv, Du);
          svk_coeffs(Du, lam, mu, sv);
          svk_apply(sv, lam, mu, T(op.wts[1]), X, S);
        }
      } else if (MODEL != kLinear) {
        T Du[3][3];
        grad_at(Q, u0, Jinv, Du);
        ok &= secant_stress_add<T, MODEL>(Du, X, M.mp, T(op.wts[0]), S);
        if (nsets >= 2) {
          grad_at(Q, u1, Jinv, Du);
          ok &= secant_stress_add<T, MODEL>(Du, X, M.mp, T(op.wts[1]), S);
        }
      }
    }
    scatter_at(Q, S, Jinv, wdet, f);
  }
  return ok;
}

// ---------------------------------------------------------------------------------------
// Modal form of a trilinear field on the hex8 reference element.  With the signs (sx, sy, sz)
// of node a, N_a = (1 + sx xi)(1 + sy eta)(1 + sz zeta) / 8, so a field sum_a x_a N_a is
//   m0 + m1 xi + m2 eta + m3 zeta + m4 xi eta + m5 eta zeta + m6 xi zeta + m7 xi eta zeta,
// m_c = (1/8) sum_a h_c(a) x_a, h_c(a) the product of node a's signs in the directions of
// mode c.  Modes 1..7 carry the gradient: a reference derivative at a point costs 3 FMAs
// instead of an 8-node sum, and the force scatter becomes an update of 7 modal sums per
// component at each point plus one transform back to the nodes per element.
// Stored mode order: xi, eta, zeta, xi eta, eta zeta, xi zeta, xi eta zeta.
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void to_modes(const T (&x)[8][3], T (&m)[3][7]) {
  constexpr int nd[2][2][2] = {{{0, 4}, {3, 7}}, {{1, 5}, {2, 6}}};   // VTK node at [bx][by][bz]
  const T h = T(0.125);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T s[2][2], d[2][2];   // sum and difference over xi, [by][bz]
#pragma unroll
    for (int by = 0; by < 2; ++by)
#pragma unroll
      for (int bz = 0; bz < 2; ++bz) {
        s[by][bz] = x[nd[1][by][bz]][i] + x[nd[0][by][bz]][i];
        d[by][bz] = x[nd[1][by][bz]][i] - x[nd[0][by][bz]][i];
      }
    T ss[2], sd[2], ds[2], dd[2];   // then over eta, [bz]
#pragma unroll
    for (int bz = 0; bz < 2; ++bz) {
      ss[bz] = s[1][bz] + s[0][bz];
      sd[bz] = s[1][bz] - s[0][bz];
      ds[bz] = d[1][bz] + d[0][bz];
      dd[bz] = d[1][bz] - d[0][bz];
    }
    m[i][0] = h * (ds[1] + ds[0]);
    m[i][1] = h * (sd[1] + sd[0]);
    m[i][2] = h * (ss[1] - ss[0]);
    m[i][3] = h * (dd[1] + dd[0]);
    m[i][4] = h * (sd[1] - sd[0]);
    m[i][5] = h * (ds[1] - ds[0]);
    m[i][6] = h * (dd[1] - dd[0]);
  }
}

// Reference point of Gauss point q (signs of node q times 1/sqrt(3)) and its pair products.
template <typename T>
struct GaussPt {
  T xi, eta, zeta, ez, xz, xe;
  __device__ __forceinline__ explicit GaussPt(int q) {
    xi = T(kGauss) * T(node_sx(q));
    eta = T(kGauss) * T(node_sy(q));
    zeta = T(kGauss) * T(node_sz(q));
    ez = eta * zeta;
    xz = xi * zeta;
    xe = xi * eta;
  }
};

// G[i][k] = d x_i / d X_k at the point: reference derivatives from the modes, then Jinv
// (only its diagonal when jd: axis-aligned boxes)
template <typename T>
__device__ __forceinline__ void modal_grad(const T (&m)[3][7], const GaussPt<T>& P, const T* Jinv, bool jd,
                                           T (&G)[3][3]) {
  T d[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T d0 = m[i][0], d1 = m[i][1], d2 = m[i][2];
    d0 += m[i][3] * P.eta;
    d0 += m[i][5] * P.zeta;
    d0 += m[i][6] * P.ez;
    d1 += m[i][3] * P.xi;
    d1 += m[i][4] * P.zeta;
    d1 += m[i][6] * P.xz;
    d2 += m[i][5] * P.xi;
    d2 += m[i][4] * P.eta;
    d2 += m[i][6] * P.xe;
    d[i][0] = d0;
    d[i][1] = d1;
    d[i][2] = d2;
  }
  if (jd) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) G[i][k] = d[i][k] * Jinv[4 * k];
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        G[i][k] = d[i][0] * Jinv[0 * 3 + k] + d[i][1] * Jinv[1 * 3 + k] + d[i][2] * Jinv[2 * 3 + k];
  }
}

// Modal force sums g += the point's contribution: st = wdet S Jinv^T weighs the three
// reference derivatives, each mode takes its own derivative at the point
template <typename T>
__device__ __forceinline__ void modal_scatter(const T (&S)[3][3], const T* Jinv, bool jd, T wdet, const GaussPt<T>& P,
                                              T (&g)[3][7]) {
  T sw[3][3];
  if (jd) {
    const T w0 = wdet * Jinv[0], w1 = wdet * Jinv[4], w2 = wdet * Jinv[8];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      sw[i][0] = S[i][0] * w0;
      sw[i][1] = S[i][1] * w1;
      sw[i][2] = S[i][2] * w2;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        sw[i][j] = wdet * (S[i][0] * Jinv[j * 3 + 0] + S[i][1] * Jinv[j * 3 + 1] + S[i][2] * Jinv[j * 3 + 2]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T st[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) st[j] = sw[i][j];
    g[i][0] += st[0];
    g[i][1] += st[1];
    g[i][2] += st[2];
    g[i][3] += st[0] * P.eta;
    g[i][3] += st[1] * P.xi;
    g[i][4] += st[1] * P.zeta;
    g[i][4] += st[2] * P.eta;
    g[i][5] += st[0] * P.zeta;
    g[i][5] += st[2] * P.xi;
    g[i][6] += st[0] * P.ez;
    g[i][6] += st[1] * P.xz;
    g[i][6] += st[2] * P.xe;
  }
}

// Nodal forces from the modal sums: f[a][i] = (1/8) sum_c h_c(a) g_c,i, i.e. per node
//   (1/8) [sx (c + sy d) + sy a + b],  a = g_eta + sz g_eta.zeta, b = sz g_zeta,
//   c = g_xi + sz g_xi.zeta, d = g_xi.eta + sz g_xi.eta.zeta
template <typename T>
__device__ __forceinline__ void from_modes(const T (&g)[3][7], T (&f)[8][3]) {
  constexpr int nd[2][2][2] = {{{0, 4}, {3, 7}}, {{1, 5}, {2, 6}}};
  const T h = T(0.125);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int bz = 0; bz < 2; ++bz) {
      const T a = bz ? g[i][1] + g[i][4] : g[i][1] - g[i][4];
      const T b = bz ? g[i][2] : -g[i][2];
      const T c = bz ? g[i][0] + g[i][5] : g[i][0] - g[i][5];
      const T d = bz ? g[i][3] + g[i][6] : g[i][3] - g[i][6];
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        const T p = by ? b + a : b - a;
        const T r = by ? c + d : c - d;
        f[nd[1][by][bz]][i] = h * (p + r);
        f[nd[0][by][bz]][i] = h * (p - r);
      }
    }
}

// ---------------------------------------------------------------------------------------
// Element force of one element: f_e = sum_q w detJ S(grad x) . grad N, S the (secant)
// stress of the material at the operator's linearisation points (one lane per element;
// the secant materials take the fields in modal form, the linear one the nodal form).
//   x_a = src[dof] * srcscale (* mih[dof] when scale_mih)
// ---------------------------------------------------------------------------------------
template <typename T, int MODEL>
__device__ __forceinline__ bool elem_force(const Mesh& M, const OpArgs& op, int e, const double* src,
                                           double srcscale, bool scale_mih, T (&f)[8][3]) {
  if constexpr (MODEL == kLinear) return elem_force_nodal<T, MODEL>(M, op, e, src, srcscale, scale_mih, f);
  int nd[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) nd[a] = M.conn[(size_t)e * 8 + a];
  // In FP32 the element's inputs are taken relative to node 0 (in FP64 before rounding):
  // the forces depend on gradients only, and a large common translation would otherwise
  // cost the deformation its significant bits.
  constexpr bool shift = sizeof(T) == 4;
  T xm[3][7];
  {
    T x[8][3];
    double x0[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const size_t d = (size_t)nd[a] * 3 + i;
        double v = src[d] * srcscale;
        if (scale_mih) v *= M.mih[d];
        if (shift && a == 0) x0[i] = v;
        x[a][i] = T(v - x0[i]);
      }
    to_modes(x, xm);
  }
  const int nsets = (MODEL == kLinear) ? 0 : op.nsets;
  T um0[3][7], um1[3][7];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (nsets > k) {
      const double* ul = op.ulin[k];
      T u[8][3];
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i)
          u[a][i] = T(ul[(size_t)nd[a] * 3 + i] - (shift ? ul[(size_t)nd[0] * 3 + i] : 0.0));
      to_modes(u, k == 0 ? um0 : um1);
    }
  }
  T g[3][7];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 7; ++c) g[i][c] = T(0);
  double lam_d, mu_d;
  rest_lame(M.model, M.mp, lam_d, mu_d);
  const T lam = T(lam_d), mu = T(mu_d);
  // FP32 only: in the FP64 kernels the unswitched second copy of the Gauss-point loop costs
  // more (register pressure) than its multiplies save (batch FP64 5.05 -> 5.28 ms per step)
  const bool jd = sizeof(T) == 4 && M.jdiag != 0;
  bool ok = true;
  for (int q = 0; q < 8; ++q) {
    const GaussPt<T> P(q);
    T Jinv[9], wdet;
    const size_t gi = (M.congruent ? (size_t)q : (size_t)e * 8 + q) * 10;
    if (sizeof(T) == 8) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Jinv[k] = T(M.geo[gi + k]);
      wdet = T(M.geo[gi + 9]);
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) Jinv[k] = T(M.geo32[gi + k]);
      wdet = T(M.geo32[gi + 9]);
    }
    T X[3][3];
    modal_grad(xm, P, Jinv, jd, X);
    T S[3][3];
    if (nsets == 0) {
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
      if constexpr (MODEL == kSVK) {
        T Du[3][3];
        SecantSVK<T> sv;
        modal_grad(um0, P, Jinv, jd, Du);
        svk_coeffs(Du, lam, mu, sv);
        svk_apply(sv, lam, mu, T(op.wts[0]), X, S);
        if (nsets >= 2) {
          modal_grad(um1, P, Jinv, jd, Du);
          svk_coeffs(Du, lam, mu, sv);
          svk_apply(sv, lam, mu, T(op.wts[1]), X, S);
        }
      } else if (MODEL != kLinear) {
        T Du[3][3];
        modal_grad(um0, P, Jinv, jd, Du);
        ok &= secant_stress_add<T, MODEL>(Du, X, M.mp, T(op.wts[0]), S);
        if (nsets >= 2) {
          modal_grad(um1, P, Jinv, jd, Du);
          ok &= secant_stress_add<T, MODEL>(Du, X, M.mp, T(op.wts[1]), S);
        }
      }
    }
    modal_scatter(S, Jinv, jd, wdet, P, g);
  }
  from_modes(g, f);
  return ok;
}

// ---------------------------------------------------------------------------------------
// Element force with one lane per Gauss point: 8 consecutive lanes share element e (all 8
// must call with the same e).  Each lane builds grad x (and grad u of the secant sets) at
// its point from the gathered nodal values, forms its stress and its contribution to the 24
// nodal forces; a 3-round reduce-scatter over the 8 lanes (12 + 6 + 3 exchanges) leaves
// lane q with the summed force of node q, which it stores to its element slot.
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T shfl_x(T v, int o) { return __shfl_xor(v, o, 64); }

// Lanes per element of the operator's element kernel: the FP64 secant materials keep too
// many values live for one lane per element (register spills), so they spread an element
// over 8 lanes; the linear and FP32 kernels fit one lane per element and avoid the 8-fold
// gathers.  (The batch kernel overrides this with one lane per element in FP64 as well:
// rubber batch 10.8 -> 10.0 ms per FP64 step, where single instances lose: c3 1.9 -> 2.9 ms.)
template <typename T, int MODEL>
__host__ __device__ constexpr int elem_lanes() { return (sizeof(T) == 8 && MODEL != kLinear) ? 8 : 1; }

template <typename T>
__device__ __forceinline__ void grad_gather(const QFactors<T>& Q, const int (&nd)[8], const double* v, double sc,
                                            const double* mih, const T* Jinv, T (&G)[3][3]) {
  T Dxi[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Dxi[i][j] = T(0);
  double x0[3] = {0.0, 0.0, 0.0};     // FP32: inputs relative to node 0 (see elem_force)
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const T d0 = Q.dN(a, 0), d1 = Q.dN(a, 1), d2 = Q.dN(a, 2);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const size_t d = (size_t)nd[a] * 3 + i;
      double xv = v[d] * sc;
      if (mih) xv *= mih[d];
      if (sizeof(T) == 4 && a == 0) x0[i] = xv;
      const T x = T(xv - x0[i]);
      Dxi[i][0] += x * d0;
      Dxi[i][1] += x * d1;
      Dxi[i][2] += x * d2;
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      G[i][k] = Dxi[i][0] * Jinv[0 * 3 + k] + Dxi[i][1] * Jinv[1 * 3 + k] + Dxi[i][2] * Jinv[2 * 3 + k];
}

template <typename T, int MODEL>
__device__ __forceinline__ bool elem_force_qp(const Mesh& M, const OpArgs& op, int e, const double* src,
                                              double srcscale, bool scale_mih, T* F) {
  const int q = threadIdx.x & 7;
  const QFactors<T> Q(q);
  int nd[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) nd[a] = M.conn[(size_t)e * 8 + a];
  T Jinv[9], wdet;
  const size_t gi = (M.congruent ? (size_t)q : (size_t)e * 8 + q) * 10;
  if (sizeof(T) == 8) {
#pragma unroll
    for (int k = 0; k < 9; ++k) Jinv[k] = T(M.geo[gi + k]);
    wdet = T(M.geo[gi + 9]);
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) Jinv[k] = T(M.geo32[gi + k]);
    wdet = T(M.geo32[gi + 9]);
  }
  T X[3][3];
  grad_gather(Q, nd, src, srcscale, scale_mih ? M.mih : nullptr, Jinv, X);
  T S[3][3];
  bool ok = true;
  const int nsets = (MODEL == kLinear) ? 0 : op.nsets;
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
    if constexpr (MODEL == kSVK) {
      double lam_d, mu_d;
      rest_lame(kSVK, M.mp, lam_d, mu_d);
      for (int s = 0; s < nsets; ++s) {
        T Du[3][3];
        SecantSVK<T> sv;
        grad_gather(Q, nd, op.ulin[s], 1.0, nullptr, Jinv, Du);
        svk_coeffs(Du, T(lam_d), T(mu_d), sv);
        svk_apply(sv, T(lam_d), T(mu_d), T(op.wts[s]), X, S);
      }
    } else if (MODEL != kLinear) {
      for (int s = 0; s < nsets; ++s) {
        T Du[3][3];
        grad_gather(Q, nd, op.ulin[s], 1.0, nullptr, Jinv, Du);
        ok &= secant_stress_add<T, MODEL>(Du, X, M.mp, T(op.wts[s]), S);
      }
    }
  }
  // contribution of this point: f_a,i = sum_j St[i][j] dN_a/dxi_j, St = wdet S Jinv^T
  T St[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      St[i][j] = wdet * (S[i][0] * Jinv[j * 3 + 0] + S[i][1] * Jinv[j * 3 + 1] + S[i][2] * Jinv[j * 3 + 2]);
  T f[8][3];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const T d0 = Q.dN(a, 0), d1 = Q.dN(a, 1), d2 = Q.dN(a, 2);
#pragma unroll
    for (int i = 0; i < 3; ++i) f[a][i] = St[i][0] * d0 + St[i][1] * d1 + St[i][2] * d2;
  }
  // reduce-scatter over the 8 lanes: keep the half of the nodes that matches the lane bit
  const bool b4 = (q >> 2) & 1, b2 = (q >> 1) & 1, b1 = q & 1;
  T k4[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T send = b4 ? f[a][i] : f[a + 4][i];
      const T keep = b4 ? f[a + 4][i] : f[a][i];
      k4[a][i] = keep + shfl_x(send, 4);
    }
  T k2[2][3];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T send = b2 ? k4[a][i] : k4[a + 2][i];
      const T keep = b2 ? k4[a + 2][i] : k4[a][i];
      k2[a][i] = keep + shfl_x(send, 2);
    }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T send = b1 ? k2[0][i] : k2[1][i];
    const T keep = b1 ? k2[1][i] : k2[0][i];
    F[((size_t)q * M.n_elems + e) * 3 + i] = keep + shfl_x(send, 1);
  }
  return ok;
}

// Contribution of one Gauss point's stress S to its element's 24 nodal forces, summed over
// the element's 8 lanes by a reduce-scatter: lane q stores node q's force to its slot.
template <typename T>
__device__ __forceinline__ void qp_scatter_store(const Mesh& M, const QFactors<T>& Q, const T (&S)[3][3],
                                                 const T* Jinv, T wdet, int q, int e, T* F) {
  T St[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      St[i][j] = wdet * (S[i][0] * Jinv[j * 3 + 0] + S[i][1] * Jinv[j * 3 + 1] + S[i][2] * Jinv[j * 3 + 2]);
  T f[8][3];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const T d0 = Q.dN(a, 0), d1 = Q.dN(a, 1), d2 = Q.dN(a, 2);
#pragma unroll
    for (int i = 0; i < 3; ++i) f[a][i] = St[i][0] * d0 + St[i][1] * d1 + St[i][2] * d2;
  }
  const bool b4 = (q >> 2) & 1, b2 = (q >> 1) & 1, b1 = q & 1;
  T k4[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T send = b4 ? f[a][i] : f[a + 4][i];
      const T keep = b4 ? f[a + 4][i] : f[a][i];
      k4[a][i] = keep + shfl_x(send, 4);
    }
  T k2[2][3];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T send = b2 ? k4[a][i] : k4[a + 2][i];
      const T keep = b2 ? k4[a + 2][i] : k4[a][i];
      k2[a][i] = keep + shfl_x(send, 2);
    }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T send = b1 ? k2[0][i] : k2[1][i];
    const T keep = b1 ? k2[1][i] : k2[0][i];
    F[((size_t)q * M.n_elems + e) * 3 + i] = keep + shfl_x(send, 1);
  }
}

// Element forces of the fourth-order scheme's operator (one lane per Gauss point, 8 lanes
// per element).  With X_u, X_v the gradients of M^{-1/2} x_u and M^{-1/2} x_v (times hinv),
// h = dt/2 and c = sqrt(3) dt^2 / 12, and Phi_i the per-point H-matrix operator of set i:
//   Fv <- Phi_1(h X_u - c X_v) + Phi_2(h X_u + c X_v)     (v-part of Omega x: -M^{-1/2} Fv)
//   Fu <- Phi_1(c X_u) - Phi_2(c X_u)                      (u-part: -M^{-1/2} Fu)
// since dt/2 (Hbar_1 + Hbar_2) x_u + c (Hbar_2 - Hbar_1) x_v and c (Hbar_1 - Hbar_2) x_u are
// the H parts of Omega x.  Returns false if a set has J <= 0.
template <typename T, int MODEL>
__device__ __forceinline__ bool elem_force_qp_m4(const Mesh& M, const OpArgs& op, int e, const double* src,
                                                 double hinv, T* Fv, T* Fu) {
  const int q = threadIdx.x & 7;
  const QFactors<T> Q(q);
  int nd[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) nd[a] = M.conn[(size_t)e * 8 + a];
  T Jinv[9], wdet;
  const size_t gi = (M.congruent ? (size_t)q : (size_t)e * 8 + q) * 10;
  if (sizeof(T) == 8) {
#pragma unroll
    for (int k = 0; k < 9; ++k) Jinv[k] = T(M.geo[gi + k]);
    wdet = T(M.geo[gi + 9]);
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) Jinv[k] = T(M.geo32[gi + k]);
    wdet = T(M.geo32[gi + 9]);
  }
  T Xu[3][3], Xv[3][3];
  grad_gather(Q, nd, src, hinv, M.mih, Jinv, Xu);
  grad_gather(Q, nd, src + M.n3, hinv, M.mih, Jinv, Xv);
  const T h = T(0.5 * op.dt4), c = T(op.c4);
  T Sv[3][3], Su[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) Sv[i][k] = Su[i][k] = T(0);
  bool ok = true;
  double lam_d = 0.0, mu_d = 0.0;
  if (MODEL == kSVK) rest_lame(kSVK, M.mp, lam_d, mu_d);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const T sg = s == 0 ? T(-1) : T(1);    // -c X_v for set 1, +c X_v for set 2
    T Ai[3][3], B[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        Ai[i][k] = h * Xu[i][k] + sg * c * Xv[i][k];
        B[i][k] = c * Xu[i][k];
      }
    T Du[3][3];
    grad_gather(Q, nd, op.ulin[s], 1.0, nullptr, Jinv, Du);
    if constexpr (MODEL == kSVK) {
      SecantSVK<T> sv;
      svk_coeffs(Du, T(lam_d), T(mu_d), sv);
      svk_apply(sv, T(lam_d), T(mu_d), T(1), Ai, Sv);
      svk_apply(sv, T(lam_d), T(mu_d), -sg, B, Su);
    } else {
      Secant<T> sc;
      ok &= secant_coeffs<T, MODEL>(Du, M.mp, sc);
      secant_apply(sc, T(1), Ai, Sv);
      secant_apply(sc, -sg, B, Su);
    }
  }
  qp_scatter_store(M, Q, Sv, Jinv, wdet, q, e, Fv);
  qp_scatter_store(M, Q, Su, Jinv, wdet, q, e, Fu);
  return ok;
}

template <typename T>
__device__ __forceinline__ void store_force(const Mesh& M, int e, const T (&f)[8][3], T* F) {
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) F[((size_t)a * M.n_elems + e) * 3 + i] = f[a][i];
}

// Stiffness of the reference element of a congruent mesh at the rest state (the linear
// branch of elem_force applied to unit vectors): column c = 3b + j of K_e is the element
// force of the unit displacement of node b in direction j.  Ke row stride kKeLd (odd, so
// that the 8 lanes of an element read distinct LDS banks).

__device__ __forceinline__ void ke_column(const Mesh& M, int c, double* Ke) {
  double x[8][3], f[8][3];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      x[a][i] = (3 * a + i == c) ? 1.0 : 0.0;
      f[a][i] = 0.0;
    }
  double lam, mu;
  rest_lame(M.model, M.mp, lam, mu);
  for (int q = 0; q < 8; ++q) {
    const QFactors<double> Q(q);
    double Jinv[9];
    for (int k = 0; k < 9; ++k) Jinv[k] = M.geo[(size_t)q * 10 + k];
    const double wdet = M.geo[(size_t)q * 10 + 9];
    double X[3][3], S[3][3];
    grad_at(Q, x, Jinv, X);
    const double tr = X[0][0] + X[1][1] + X[2][2];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) S[i][k] = mu * (X[i][k] + X[k][i]) + (i == k ? lam * tr : 0.0);
    scatter_at(Q, S, Jinv, wdet, f);
  }
  for (int a = 0; a < 8; ++a)
    for (int i = 0; i < 3; ++i) Ke[(3 * a + i) * kKeLd + c] = f[a][i];
}

// Element forces F = K_e x_e of a congruent mesh with K_e in LDS (FP64): eight lanes per
// element, lane a owns node a, loads its three inputs and obtains the other 21 by
// shuffles.  Every lane of the 8-lane group must call with the same e.
__device__ __forceinline__ void elem_force_ke(const Mesh& M, int e, const double* src, double srcscale,
                                              const double* Ke, double* F) {
  const int lane = threadIdx.x & 63;
  const int a = lane & 7, base = lane & ~7;
  const int nd = M.conn[(size_t)e * 8 + a];
  double xa[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const size_t d = (size_t)nd * 3 + i;
    xa[i] = src[d] * srcscale * M.mih[d];
  }
  double xe[24];
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int i = 0; i < 3; ++i) xe[3 * b + i] = __shfl(xa[i], base + b, 64);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double* row = Ke + (3 * a + i) * kKeLd;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 24; ++c) s += row[c] * xe[c];
    F[((size_t)a * M.n_elems + e) * 3 + i] = s;
  }
}

// VTK corner c of a hex as offsets (di, dj, dk) in {0, 1}^3
__host__ __device__ __forceinline__ int vtk_di(int c) { return (c == 1 || c == 2 || c == 5 || c == 6) ? 1 : 0; }
__host__ __device__ __forceinline__ int vtk_dj(int c) { return (c == 2 || c == 3 || c == 6 || c == 7) ? 1 : 0; }
__host__ __device__ __forceinline__ int vtk_dk(int c) { return c >= 4 ? 1 : 0; }

// Force rows of node A, (K x)_{3A+c} = sum over the elements e around A of
// sum_{b,d} K_e[3a+c][3b+d] x_{3 n_b + d} (a = A's local index in e), for a congruent mesh
// with K_e in LDS: the 8 lanes of a group take the element slots p, p+8, ... of A and the
// group sums with a butterfly; every lane returns the three sums.  x = src * scale (times
// M^{-1/2} when scale_mih).  Every lane of the group must call with the same A.
__device__ __forceinline__ void node_force_ke(const Mesh& M, int A, const double* src, double scale, bool scale_mih,
                                              const double* Ke, double (&f)[3]) {
  const int p = threadIdx.x & 7;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  const int q1 = M.inc_ptr[A + 1];
  for (int q = M.inc_ptr[A] + p; q < q1; q += 8) {
    const int slot = M.inc[q];
    const int a = slot / M.n_elems, e = slot - a * M.n_elems;
    int nd[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) nd[b] = M.conn[(size_t)e * 8 + b];
    const double* r0 = Ke + (3 * a) * kKeLd;
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const size_t g = (size_t)nd[b] * 3 + d;
        double x = src[g] * scale;
        if (scale_mih) x *= M.mih[g];
        s0 += r0[3 * b + d] * x;
        s1 += r0[kKeLd + 3 * b + d] * x;
        s2 += r0[2 * kKeLd + 3 * b + d] * x;
      }
  }
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) {
    s0 += __shfl_xor(s0, o, 64);
    s1 += __shfl_xor(s1, o, 64);
    s2 += __shfl_xor(s2, o, 64);
  }
  f[0] = s0;
  f[1] = s1;
  f[2] = s2;
}

// Node -> element-slot map of an operator pass, set up once per pass.  Lattice meshes
// (elements i-fastest, VTK corners, slot indices below 2^31) find the slots by index
// arithmetic: corner a of the element whose origin is node - offset(a), in increasing a,
// which is the order of the node's incidence list, so both forms add the same terms in the
// same order.  Otherwise the node's incidence list is read.
struct SlotMap {
  const int* inc_ptr;
  const int* inc;
  bool lat;
  int nx, ny, nz, NX, NXY;
  double rNX, rNXY;           // 1/NX, 1/NXY: (A + 1/2) / N rounds to the exact quotient for A < 2^51
  int base[8];                // slot of corner a of the element at the node, minus that element
};

__device__ __forceinline__ SlotMap slot_map(const Mesh& M) {
  SlotMap S;
  S.inc_ptr = M.inc_ptr;
  S.inc = M.inc;
  S.lat = M.lat[0] > 0 && (long long)M.n_elems * 24 < (1LL << 31);
  S.nx = M.lat[0];
  S.ny = M.lat[1];
  S.nz = M.lat[2];
  S.NX = S.nx + 1;
  S.NXY = S.NX * (S.ny + 1);
  S.rNX = 1.0 / (double)max(S.NX, 1);
  S.rNXY = 1.0 / (double)max(S.NXY, 1);
#pragma unroll
  for (int a = 0; a < 8; ++a)
    S.base[a] = a * M.n_elems - ((((a + 1) >> 1) & 1) + S.nx * (((a >> 1) & 1) + S.ny * (a >> 2)));
  return S;
}

// sum of element-slot forces of DOF 3*A + c over the elements around node A
template <typename T>
__device__ __forceinline__ double gather_slots(const SlotMap& S, const T* F, int A, int c) {
  if (S.lat) {
    const int k = (int)(((double)A + 0.5) * S.rNXY);
    const int r = A - k * S.NXY;
    const int j = (int)(((double)r + 0.5) * S.rNX);
    const int i = r - j * S.NX;
    const int e0 = i + S.nx * (j + S.ny * k);       // the element with its origin at the node
    const bool x0 = i < S.nx, x1 = i > 0, y0 = j < S.ny, y1 = j > 0, z0 = k < S.nz, z1 = k > 0;
    T f[8];
    bool in[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const bool di = ((a + 1) >> 1) & 1, dj = (a >> 1) & 1, dk = a >> 2;
      in[a] = (di ? x1 : x0) && (dj ? y1 : y0) && (dk ? z1 : z0);
      f[a] = in[a] ? F[(e0 + S.base[a]) * 3 + c] : T(0);
    }
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a)
      if (in[a]) s += double(f[a]);
    return s;
  }
  // slot indices, then forces, loaded 8 at a time so that the loads overlap
  double s = 0.0;
  const int p0 = S.inc_ptr[A], p1 = S.inc_ptr[A + 1];
  for (int p = p0; p < p1; p += 8) {
    int sl[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) sl[u] = p + u < p1 ? S.inc[p + u] : -1;
    T f[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) f[u] = sl[u] >= 0 ? F[(size_t)sl[u] * 3 + c] : T(0);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (sl[u] >= 0) s += double(f[u]);
  }
  return s;
}

// The three summed forces of node A's DOFs in one pass: the node's position in the lattice
// (or its slot list) once, and each slot's three components together; every component is
// summed over the corners in the order of gather_slots, so the sums are the same numbers.
template <typename T>
__device__ __forceinline__ void gather_node(const SlotMap& S, const T* F, int A, double (&s)[3]) {
  s[0] = s[1] = s[2] = 0.0;
  if (S.lat) {
    const int k = (int)(((double)A + 0.5) * S.rNXY);
    const int r = A - k * S.NXY;
    const int j = (int)(((double)r + 0.5) * S.rNX);
    const int i = r - j * S.NX;
    const int e0 = i + S.nx * (j + S.ny * k);
    const bool x0 = i < S.nx, x1 = i > 0, y0 = j < S.ny, y1 = j > 0, z0 = k < S.nz, z1 = k > 0;
    T f[8][3];
    bool in[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const bool di = ((a + 1) >> 1) & 1, dj = (a >> 1) & 1, dk = a >> 2;
      in[a] = (di ? x1 : x0) && (dj ? y1 : y0) && (dk ? z1 : z0);
      const T* q = F + (e0 + S.base[a]) * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) f[a][c] = in[a] ? q[c] : T(0);
    }
#pragma unroll
    for (int a = 0; a < 8; ++a)
      if (in[a]) {
        s[0] += double(f[a][0]);
        s[1] += double(f[a][1]);
        s[2] += double(f[a][2]);
      }
    return;
  }
  const int p0 = S.inc_ptr[A], p1 = S.inc_ptr[A + 1];
  for (int p = p0; p < p1; p += 8) {
    int sl[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) sl[u] = p + u < p1 ? S.inc[p + u] : -1;
    T f[8][3];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int c = 0; c < 3; ++c) f[u][c] = sl[u] >= 0 ? F[(size_t)sl[u] * 3 + c] : T(0);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (sl[u] >= 0) {
        s[0] += double(f[u][0]);
        s[1] += double(f[u][1]);
        s[2] += double(f[u][2]);
      }
  }
}

template <typename T>
__device__ __forceinline__ double gather_force(const Mesh& M, const T* F, int A, int c) {
  return gather_slots(slot_map(M), F, A, c);
}

// load scale(t): piecewise linear through the knots, constant outside
__device__ __forceinline__ double load_scale(const Mesh& M, double t) {
  const int n = M.n_knots;
  if (n <= 0) return 0.0;
  const double* kt = M.knots;
  const double* ks = M.knots + n;
  if (t <= kt[0]) return ks[0];
  if (t >= kt[n - 1]) return ks[n - 1];
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (kt[mid] <= t) lo = mid; else hi = mid;
  }
  const double th = (t - kt[lo]) / (kt[hi] - kt[lo]);
  return ks[lo] + th * (ks[hi] - ks[lo]);
}

// ---------------------------------------------------------------------------------------
// Reductions (wave64 butterflies give every lane the same bits) and team synchronisation.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup, same value in every thread; red: >= 16 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// A team of G co-resident workgroups (cooperative launch) synchronised through device
// memory; G == 1 degenerates to the workgroup barrier.
//  * sync(): every workgroup publishes its barrier generation in its own flag (after a
//    release fence) and polls all G flags, then acquires.  Used where bulk data written by
//    other workgroups is read next.
//  * post() / wait(): an all-reduce split in two so that independent loads can be issued
//    while it is in flight.  The workgroup partial itself is the signal: post() stores it
//    with an agent-coherent atomic into this round's slot of a ring (empty slots hold a
//    sentinel NaN pattern); wait() has every wave poll the G slots and sum them in rank
//    order, so every wave of every workgroup obtains the same bits without a broadcast.
//    At the start of round r a workgroup empties its slot of round r-2 (every workgroup has
//    finished reading it: they all published round r-1); the store is performed before the
//    workgroup's next publication (wait count at the start of round r+1).  No cache flush.
// Waits are bounded.  A wave that times out records the sticky error and clears the
// workgroup's LDS alive flag; the workgroup agrees on it after its next barrier and every
// wave then leaves the kernel together.
constexpr unsigned long long kEmpty = 0x7ff4deadbeef1234ull;
constexpr unsigned long long kSpinLimit = 1ull << 26;
constexpr int kAllWavePoll = 64;

__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup sum with one barrier: red holds two 16-entry halves used alternately (a half
// is rewritten only after the barrier of the other half has been passed by every wave).
__device__ __forceinline__ double block_sum2(double v, double* red, unsigned& sel) {
  double* rb = red + (sel & 1u) * 16;
  sel ^= 1u;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) rb[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < nw; ++i) s += rb[i];
  return s;
}

struct GridTeam {
  static constexpr bool kVecReduce = true;
  int G, rank;
  unsigned long long* flags;   // [G] barrier generations
  unsigned long long* ring;    // [kRing * G] all-reduce slots
  int* err;
  unsigned long long gen;
  unsigned rnd;
  bool dead;
  unsigned sel;                // alternating half of the reduction scratch
  unsigned long long* vring;   // [kRing * G * vw] vector all-reduce slots
  int vw;
  unsigned vrnd;

  __device__ void timeout(int* lds_flag) {
    *lds_flag = 0;
    atomicCAS(err, 0, kErrDevice);
  }

  __device__ bool sync(int* lds_flag) {
    __syncthreads();
    if (*lds_flag == 0) { dead = true; return false; }
    if (G == 1) return true;
    gen += 1;
    if (threadIdx.x == 0) {
      __threadfence();
      st_agent(&flags[rank], gen);
    }
    for (int i = threadIdx.x; i < G; i += blockDim.x) {
      unsigned long long spins = 0;
      while (ld_agent(&flags[i]) < gen) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) { timeout(lds_flag); break; }
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) __threadfence();
    __syncthreads();
    if (*lds_flag == 0) { dead = true; return false; }
    return true;
  }

  // Publish this workgroup's partial of the current round; returns the workgroup sum.
  // fenced = true also releases this workgroup's earlier global stores (see wait()).
  __device__ double post(double partial, double* red, int* lds_flag, bool fenced) {
    const double p = block_sum2(partial, red, sel);
    if (*lds_flag == 0) { dead = true; return 0.0; }
    if (G == 1) return p;
    if (threadIdx.x == 0) {
      if (fenced) __threadfence();
      __builtin_amdgcn_s_waitcnt(0);
      if (rnd >= 2) st_agent(&ring[(size_t)((rnd - 2) % kRing) * G + rank], kEmpty);
      st_agent(&ring[(size_t)(rnd % kRing) * G + rank],
               p == p ? (unsigned long long)__double_as_longlong(p) : 0x7ff8000000000000ull);
    }
    return p;
  }

  // Sum of the round's G partials, identical bits in every wave.  fenced = true acquires
  // after every slot has been observed, so that bulk data released by the other
  // workgroups before their post() is visible afterwards.
  __device__ double wait(double p, int* lds_flag, bool fenced, double* red = nullptr) {
    if (G == 1 || dead) return p;
    const unsigned long long* slot = ring + (size_t)(rnd % kRing) * G;
    double tot;
    // small teams: every wave polls all slots (no broadcast barrier); large teams: wave 0
    // polls and broadcasts through LDS, keeping the polling traffic on the ring lines low
    const bool all_waves = G <= kAllWavePoll || red == nullptr;
    if (all_waves) {
      double s = 0.0;
      for (int i = (threadIdx.x & 63); i < G; i += 64) {
        unsigned long long x, spins = 0;
        while ((x = ld_agent(&slot[i])) == kEmpty) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kSpinLimit) { timeout(lds_flag); break; }
        }
        s += __longlong_as_double((long long)x);
      }
      tot = wave_sum(s);
    } else {
      // one slot per thread over the first ceil(G/64) waves, then a fixed-order wave sum
      double s = 0.0;
      for (int i = threadIdx.x; i < G; i += blockDim.x) {
        unsigned long long x, spins = 0;
        while ((x = ld_agent(&slot[i])) == kEmpty) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kSpinLimit) { timeout(lds_flag); break; }
        }
        s += __longlong_as_double((long long)x);
      }
      s = wave_sum(s);
      double* rb = red + (sel & 1u) * 16;
      sel ^= 1u;
      if ((threadIdx.x & 63) == 0) rb[threadIdx.x >> 6] = s;
      __syncthreads();
      tot = 0.0;
      const int nw = (blockDim.x + 63) >> 6;
      for (int w = 0; w < nw; ++w) tot += rb[w];
    }
    if (fenced) {
      __syncthreads();
      if (threadIdx.x == 0) __threadfence();
      __syncthreads();
      if (*lds_flag == 0) dead = true;
    }
    rnd += 1;
    return tot;
  }

  __device__ double allreduce(double partial, double* red, int* lds_flag, bool fenced = false) {
    const double p = post(partial, red, lds_flag, fenced);
    return wait(p, lds_flag, fenced, red);
  }

  // All-reduce of K <= min(vw, blockDim.x) values.  On entry vals[0..K) holds this
  // workgroup's partials behind a barrier; on return it holds the team sums, the same bits
  // in every workgroup (rank-ordered sums).  Same slot protocol as post()/wait(), one slot
  // entry per value; a thread polls up to 8 entries at once.  gp: blockDim.x doubles of LDS.
  __device__ bool allreduce_vec(double* vals, int K, double* gp, int* lds_flag) {
    if (*lds_flag == 0) { dead = true; return false; }
    if (G == 1) return true;
    const size_t slot = (size_t)G * vw;
    unsigned long long* cur = vring + (size_t)(vrnd % kRing) * slot;
    const size_t row = (size_t)rank * vw;
    if (vrnd >= 2) {
      unsigned long long* old = vring + (size_t)((vrnd - 2) % kRing) * slot + row;
      for (int t = threadIdx.x; t < vw; t += blockDim.x) st_agent(old + t, kEmpty);
    }
    for (int t = threadIdx.x; t < K; t += blockDim.x) {
      const double p = vals[t];
      st_agent(cur + row + t, p == p ? (unsigned long long)__double_as_longlong(p) : 0x7ff8000000000000ull);
    }
    const int Q = (int)blockDim.x / K;          // rank groups per value
    const int t = threadIdx.x;
    if (t < Q * K) {
      const int k = t % K, g = t / K;
      constexpr int U = 8;
      double s = 0.0;
      for (int i0 = g; i0 < G; i0 += U * Q) {
        unsigned long long x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * Q;
          x[u] = i < G ? ld_agent(cur + (size_t)i * vw + k) : 0ull;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + u * Q;
          unsigned long long spins = 0;
          while (x[u] == kEmpty) {
            __builtin_amdgcn_s_sleep(1);
            x[u] = ld_agent(cur + (size_t)i * vw + k);
            if (++spins > kSpinLimit) { timeout(lds_flag); break; }
          }
          s += __longlong_as_double((long long)x[u]);
        }
      }
      gp[g * K + k] = s;
    }
    __syncthreads();
    if (t < K) {
      double tot = 0.0;
      for (int g = 0; g < Q; ++g) tot += gp[g * K + t];
      vals[t] = tot;
    }
    __syncthreads();
    vrnd += 1;
    if (*lds_flag == 0) { dead = true; return false; }
    return true;
  }
};

}  // namespace ep
