// Stored element tangents in BF16 (precision mode EP_PREC_MIXED_BF16).
//
// The operator's element matrix (Sec. 2.3 with the H-matrix of App. A) is
//   K_e[(A,i),(B,k)] = sum_q sum_{j,l} dN_A/dX_j(q) dN_B/dX_l(q) C_q[(i,j),(k,l)],
//   C_q[(i,j),(k,l)] = w_q det J_q sum_s w_s dPhi_s,ij / dX_kl,
// the derivative of the per-point operator Phi (linear in X = grad x; for the Neo-Hookean
// and Yeoh solids a sym(X N) + (W : X) Ci + X S, for St. Venant-Kirchhoff
// lambda (Hh : X) I + mu (Hh^T X + X^T Hh) + X S; ep_device.hpp),
// summed over the operator's coefficient sets s (predictor: 1.75 and -0.75; corrector: 1;
// rest state: C = mu (d_ik d_jl + d_il d_jk) + lambda d_ij d_kl).  On a congruent mesh the
// gradients dN/dX are the same for every element, so all element matrices come from one
// product with a shared left factor:
//   K[(A,B), (i,k,e)] = Psi[(A,B), (q,j,l)] . Cbar[(q,j,l), (i,k,e)],
//   Psi = dN_A/dX_j(q) dN_B/dX_l(q)   (64 x 80: column 10 q + 3 j + l, 10 q + 9 zero),
// formed by k_form_tangent with BF16 matrix-core products and FP32 accumulation, and stored
// rounded to BF16.  Every operator apply then reads K_e and computes K_e x_e in FP32.
//
// Storage: elements in groups of 8 (the 8 elements one wave applies); group g holds
// 9 chunks x 64 lanes x 8 BF16 values; lane L = 8 (e mod 8) + A of chunk c = 3 i + k holds
// K_e[(A, i), (B, k)] for B = 0..7, so that each of the nine 16-byte loads of a wave reads
// 1 KiB of contiguous memory.
#pragma once

#include "ep_device.hpp"

namespace ep {

constexpr int kTanElems = 32;                      // elements per formation workgroup
constexpr int kTanThreads = 256;                   // 8 lanes (Gauss points) per element
constexpr int kTanLd = 88;                         // LDS row stride (BF16) of Cbar^T

// FP32 -> BF16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// Element forces F = K_e x_e from the stored tangents: eight lanes per element (lane a owns
// node a; every lane of the group calls with the same e).  The inputs are taken relative to
// node 0 in FP64 before rounding to FP32 (a translation is in the null space of K_e; rounded
// K_e no longer maps it to zero exactly).  F: FP32 element-force slots (a n_e + e).
__device__ __forceinline__ void elem_force_kst(const Mesh& M, int e, const double* src, double srcscale,
                                               bool scale_mih, float* F) {
  const int lane = threadIdx.x & 63;
  const int a = lane & 7, base = lane & ~7;
  const uint4* kp = reinterpret_cast<const uint4*>(M.kst) + (size_t)(e >> 3) * (9 * 64) + ((e & 7) * 8 + a);
  uint4 kv[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) kv[c] = kp[c * 64];
  const int nd = M.conn[(size_t)e * 8 + a];
  double xa[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const size_t d = (size_t)nd * 3 + i;
    xa[i] = src[d] * srcscale;
    if (scale_mih) xa[i] *= M.mih[d];
  }
  float xr[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) xr[i] = float(xa[i] - __shfl(xa[i], base, 64));
  float xe[24];
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int i = 0; i < 3; ++i) xe[3 * b + i] = __shfl(xr[i], base + b, 64);
  float s[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const uint32_t w4[4] = {kv[c].x, kv[c].y, kv[c].z, kv[c].w};
    const int i = c / 3, k = c % 3;
#pragma unroll
    for (int B = 0; B < 8; ++B) {
      const uint32_t bits = (B & 1) ? (w4[B >> 1] >> 16) : (w4[B >> 1] & 0xffffu);
      s[i] += bf16_to_f32(bits) * xe[3 * B + k];
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) F[((size_t)a * M.n_elems + e) * 3 + i] = s[i];
}

}  // namespace ep
