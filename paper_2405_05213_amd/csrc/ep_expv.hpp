// The persistent projection kernel (one cooperative launch per exp(tau A) w), shared by
// the translation unit that keeps the Krylov-vector slices in LDS (ep_kernels.hip) and the
// one that keeps them in device memory for meshes too large for LDS (ep_expv_global.hip).
#pragma once

#include "ep_kernels.hpp"
#include "ep_krylov.hpp"

namespace ep {

// LDS: red[32] | yb[kMaxM] | ke[24 kKeLd] | (compact WY: T[m_max^2] | vals[2 m_max] | gp[kThreads]) |
//      ints: flag[16], 16 unused | region U: the slice buffers lw, lv (2 chunk, SG = 0 only)
//      overlaid with the check point's expm scratch (ex_cap doubles)
__host__ __device__ inline size_t expv_head_doubles(int ortho, int m_max) {
  size_t d = 32 + kMaxM + 24 * kKeLd + 16;
  if (ortho == 1) d += (size_t)m_max * m_max + 2 * (size_t)m_max + kExpvThreads;
  return d;
}

// SG = 1: the workgroup's slices of w and of the newest basis vector live in device memory
// (W.wscr, [w | v] rows of Lp doubles) and U holds only the expm scratch.
// SCH = 4: the operator of the fourth-order scheme (Omega of the two-term Magnus series).
// NPE = 27: quadratic (27-node) elements.
template <typename T, int MODEL, int ORTHO, int SG, int SCH = 2, int NPE = 8>
__global__ __launch_bounds__(kExpvThreads) void k_expv(ExpvArgs A) {
  extern __shared__ double lds[];
  const int C = A.W.chunk;
  const int mm = A.cfg.m_max;
  double* red = lds;
  double* yb = red + 32;
  double* ke = yb + kMaxM;
  double* p = ke + 24 * kKeLd;
  KLds X{nullptr, nullptr, nullptr, nullptr, nullptr, 0, SG == 0};
  if (MODEL == kLinear && sizeof(T) == 8 && A.M.ke != nullptr) {
    for (int i = threadIdx.x; i < 24 * kKeLd; i += blockDim.x) ke[i] = A.M.ke[i];
    X.ke = ke;
  }
  if (ORTHO == 1) {
    X.T = p;
    X.vals = X.T + mm * mm;
    X.gp = X.vals + 2 * mm;
    p = X.gp + kExpvThreads;
  }
  int* ints = (int*)p;
  int* flag = ints;
  double* U = p + 16;
  double* lw;
  double* lv;
  if constexpr (SG == 0) {
    lw = U;
    lv = U + C;
  } else {
    const size_t c0 = (size_t)blockIdx.x * C;
    lw = A.W.wscr + c0;
    lv = A.W.wscr + A.M.Lp + c0;
  }
  X.ex = U;
  X.ex_cap = A.W.ex_cap;
  if (threadIdx.x == 0) *flag = 1;   // workgroup alive flag (cleared on a synchronisation timeout)
  __syncthreads();
  GridTeam tm{(int)gridDim.x, (int)blockIdx.x, A.W.flags, A.W.ring, &A.W.ctrl->err, 0ull, 0u, false, 0u,
              A.W.vring, A.W.vw, 0u};
  expv_body<T, MODEL, GridTeam, ORTHO, SCH, NPE>(tm, A, lw, lv, red, yb, flag, X);
}

template <typename T, int MODEL, int SG>
inline const void* expv_fn(int ortho) {
  return ortho == 1 ? reinterpret_cast<const void*>(&k_expv<T, MODEL, 1, SG>)
                    : reinterpret_cast<const void*>(&k_expv<T, MODEL, 0, SG>);
}

template <typename T, int MODEL>
inline const void* expv_fn_m4(int ortho) {
  return ortho == 1 ? reinterpret_cast<const void*>(&k_expv<T, MODEL, 1, 0, 4>)
                    : reinterpret_cast<const void*>(&k_expv<T, MODEL, 0, 0, 4>);
}

template <typename T, int MODEL, int SG>
inline const void* expv_fn_q2(int ortho) {
  return ortho == 1 ? reinterpret_cast<const void*>(&k_expv<T, MODEL, 1, SG, 2, 27>)
                    : reinterpret_cast<const void*>(&k_expv<T, MODEL, 0, SG, 2, 27>);
}

template <int SG>
inline const void* expv_kernel_sg(int prec, int model, int ortho) {
  if (prec == 0) {
    if (model == kLinear) return expv_fn<double, kLinear, SG>(ortho);
    if (model == kNH) return expv_fn<double, kNH, SG>(ortho);
    if (model == kSVK) return expv_fn<double, kSVK, SG>(ortho);
    return expv_fn<double, kYeoh, SG>(ortho);
  }
  if (prec == 2) return expv_fn<float, kStored, SG>(ortho);
  if (model == kLinear) return expv_fn<float, kLinear, SG>(ortho);
  if (model == kNH) return expv_fn<float, kNH, SG>(ortho);
  if (model == kSVK) return expv_fn<float, kSVK, SG>(ortho);
  return expv_fn<float, kYeoh, SG>(ortho);
}

}  // namespace ep
