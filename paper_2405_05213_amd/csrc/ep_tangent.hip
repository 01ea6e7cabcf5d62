// Formation of the stored BF16 element tangents (see ep_tangent.hpp) and the stand-alone
// operator apply that uses them.
#include <type_traits>

#include "ep_kernels.hpp"
#include "ep_tangent.hpp"

namespace ep {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Psi[(A,B), (q,j,l)] = dN_A/dX_j(q) dN_B/dX_l(q) of the congruent mesh (FP64, rounded to
// BF16) at column 10 q + 3 j + l (column 10 q + 9 is zero padding), stored as the A operands of
// v_mfma_f32_16x16x16_bf16: row tile w (rows 16 w .. 16 w + 15), K-step s, lane l holds
// Psi[16 w + l % 16][16 s + 4 (l / 16) + v], v = 0..3.  One thread per value.
__global__ void k_psi(Mesh M, uint16_t* __restrict__ psi) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kPsiValues) return;
  const int v = t & 3, l = (t >> 2) & 63, ws = t >> 8;
  const int s = ws % kPsiSteps, w = ws / kPsiSteps;
  const int r = 16 * w + (l & 15), kk = 16 * s + 4 * (l >> 4) + v;
  double val = 0.0;
  if (kk % 10 != 9) {
    const int A = r >> 3, B = r & 7;
    const int q = kk / 10, j = (kk % 10) / 3, jl = (kk % 10) % 3;
    const QFactors<double> Q(q);
    const double* Ji = M.geo + (size_t)q * 10;
    double gA = 0.0, gB = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      gA += Q.dN(A, m) * Ji[m * 3 + j];
      gB += Q.dN(B, m) * Ji[m * 3 + jl];
    }
    val = gA * gB;
  }
  psi[t] = f32_to_bf16((float)val);
}

// One workgroup forms the tangents of kTanElems elements:
//  1. lane (element el, Gauss point q) loads node q of the element, obtains the others by
//     shuffles, evaluates the secant coefficients of the operator's sets at q (FP32, inputs
//     relative to node 0) and writes its 81 entries of C_q, times w det J, as BF16 into
//     Cbar^T (LDS, row n = 9 el + 3 i + k, columns 10 q .. 10 q + 9: 3 j + l, then a zero),
//     five 4-byte stores per row;
//  2. wave w multiplies its row tile of Psi (A in {2w, 2w+1}) by all 18 column tiles of
//     Cbar on the matrix cores (5 K-steps each, FP32 accumulation);
//  3. the results, rounded to BF16, are staged in LDS in the stored layout (each lane's four
//     accumulator rows are four consecutive B of one (A, i, k): one 8-byte store) and written
//     out with 16-byte stores.
template <int MODEL>
__global__ __launch_bounds__(kTanThreads) void k_form_tangent(Mesh M, OpArgs op, const uint16_t* __restrict__ psi,
                                                             uint16_t* __restrict__ kst, int* err) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[9 * kTanElems * kTanLd];
  const int el = threadIdx.x >> 3, q = threadIdx.x & 7;
  const int e = blockIdx.x * kTanElems + el;
  // ---- 1. C_q of this (element, point): coefficients of every set first, then the 81
  //         entries row by row (few values live at once)
  bool ok = true;
  const int nsets = (MODEL == kLinear || e >= M.n_elems) ? 0 : op.nsets;
  const float wdet = e < M.n_elems ? M.geo32[(size_t)q * 10 + 9] : 0.f;
  // coefficient sets of the operator (zero for an absent set, whose weight is 0)
  using SetT = typename std::conditional<MODEL == kSVK, SecantSVK<float>, Secant<float>>::type;
  SetT sc[2] = {};
  float wsv[2] = {0.f, 0.f};
  float lam_u = 0.f, mu_u = 0.f;   // rest-state (linear) / St. Venant-Kirchhoff moduli
  if (e < M.n_elems) {
    double lam_d, mu_d;
    rest_lame(M.model, M.mp, lam_d, mu_d);
    lam_u = float(lam_d);
    mu_u = float(mu_d);
  }
  if (nsets > 0) {                 // uniform over the element's 8 lanes
    const QFactors<float> Q(q);
    float Jinv[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Jinv[k] = M.geo32[(size_t)q * 10 + k];
    const int base = threadIdx.x & 63 & ~7;
    const size_t dq = (size_t)M.conn[(size_t)e * 8 + q] * 3;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s < nsets) {
        const double* ul = op.ulin[s];
        float ue[8][3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const double v = ul[dq + i];
          const float r = float(v - __shfl(v, base, 64));
#pragma unroll
          for (int a = 0; a < 8; ++a) ue[a][i] = __shfl(r, base + a, 64);
        }
        float Du[3][3];
        grad_at(Q, ue, Jinv, Du);
        if constexpr (MODEL == kSVK) svk_coeffs(Du, lam_u, mu_u, sc[s]);
        else ok &= secant_coeffs<float, MODEL>(Du, M.mp, sc[s]);
        wsv[s] = float(op.wts[s]) * wdet;
      }
    }
  }
  if (!ok) atomicCAS(err, 0, kErrInverted);
  const float lam = lam_u * wdet, mu = mu_u * wdet;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint16_t cv[10];
      cv[9] = 0;
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          float c;
          if (nsets == 0) {
            c = ((i == k && j == l) ? mu : 0.f) + ((i == l && j == k) ? mu : 0.f) + ((i == j && k == l) ? lam : 0.f);
          } else {
            c = 0.f;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
              // c = d Phi_ij / d X_kl of the operator at this point, unscaled by w det J
              float t;
              if constexpr (MODEL == kSVK) {
                // lambda (Hh : X) I + mu (Hh^T X + X^T Hh) + X S
                t = (i == j ? lam_u * sc[s].Hh[k][l] : 0.f) +
                    mu_u * ((j == l ? sc[s].Hh[k][i] : 0.f) + (i == l ? sc[s].Hh[k][j] : 0.f)) +
                    (i == k ? sc[s].S[sym_idx(l, j)] : 0.f);
              } else {
                // a sym(X N) + (W : X) Ci + X S
                t = sc[s].W[k][l] * sc[s].Ci[sym_idx(i, j)];
                if (i == k) t += 0.5f * sc[s].a * sc[s].N[l][j] + sc[s].S[l][j];
                if (j == k) t += 0.5f * sc[s].a * sc[s].N[l][i];
              }
              c += wsv[s] * t;          // wsv = 0 for an absent set
            }
          }
          cv[3 * j + l] = f32_to_bf16(c);
        }
      uint32_t* row = reinterpret_cast<uint32_t*>(lds + (size_t)(9 * el + 3 * i + k) * kTanLd + 10 * q);
#pragma unroll
      for (int h = 0; h < 5; ++h) row[h] = (uint32_t)cv[2 * h] | ((uint32_t)cv[2 * h + 1] << 16);
    }
  __syncthreads();
  // ---- 2. matrix-core products
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  bf16x4 af[kPsiSteps];
  {
    const uint2* pp = reinterpret_cast<const uint2*>(psi);
#pragma unroll
    for (int s = 0; s < kPsiSteps; ++s) {
      const uint2 u = pp[(w * kPsiSteps + s) * 64 + lane];
      af[s][0] = (short)(u.x & 0xffffu);
      af[s][1] = (short)(u.x >> 16);
      af[s][2] = (short)(u.y & 0xffffu);
      af[s][3] = (short)(u.y >> 16);
    }
  }
  constexpr int kCT = 9 * kTanElems / 16;          // 18 column tiles
  f32x4 acc[kCT];
#pragma unroll
  for (int ct = 0; ct < kCT; ++ct) {
    acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t* bro = lds + (size_t)(16 * ct + (lane & 15)) * kTanLd + 4 * (lane >> 4);
#pragma unroll
    for (int s = 0; s < kPsiSteps; ++s) {
      const uint2 u = *reinterpret_cast<const uint2*>(bro + 16 * s);
      bf16x4 bf;
      bf[0] = (short)(u.x & 0xffffu);
      bf[1] = (short)(u.x >> 16);
      bf[2] = (short)(u.y & 0xffffu);
      bf[3] = (short)(u.y >> 16);
      acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[s], bf, acc[ct], 0, 0, 0);
    }
  }
  __syncthreads();
  // ---- 3. stage in the stored layout (lane l, item v: row 16 w + 4 (l / 16) + v, column
  //         16 ct + l % 16), then write the workgroup's groups of 8 elements
  {
    const int A = 2 * w + ((lane >> 4) >> 1), B0 = 4 * ((lane >> 4) & 1);   // rows 8 A + B0 + v
#pragma unroll
    for (int ct = 0; ct < kCT; ++ct) {
      const int n = 16 * ct + (lane & 15);
      const int eo = n / 9, ik = n % 9;
      const int L = (eo & 7) * 8 + A;
      uint2 pk;
      pk.x = (uint32_t)f32_to_bf16(acc[ct][0]) | ((uint32_t)f32_to_bf16(acc[ct][1]) << 16);
      pk.y = (uint32_t)f32_to_bf16(acc[ct][2]) | ((uint32_t)f32_to_bf16(acc[ct][3]) << 16);
      *reinterpret_cast<uint2*>(lds + (size_t)(eo >> 3) * kKstGroup + (ik * 64 + L) * 8 + B0) = pk;
    }
  }
  __syncthreads();
  const long long groups = (M.n_elems + 7) / 8;
  const long long g0 = (long long)blockIdx.x * (kTanElems / 8);
  const int ng = (int)min<long long>(kTanElems / 8, groups - g0);
  const uint4* src = reinterpret_cast<const uint4*>(lds);
  uint4* dst = reinterpret_cast<uint4*>(kst) + (size_t)g0 * (kKstGroup / 8);
  for (int t = threadIdx.x; t < ng * (kKstGroup / 8); t += blockDim.x) dst[t] = src[t];
}

// F = K_e x_e over all elements (stand-alone apply), 8 lanes per element
__global__ __launch_bounds__(256) void k_elem_forces_kst(Mesh M, const double* __restrict__ src, double sc,
                                                         int scale_mih, float* __restrict__ F) {
  const int e = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 3);
  if (e < M.n_elems) elem_force_kst(M, e, src, sc, scale_mih != 0, F);
}

void launch_psi(const Mesh& M, uint16_t* psi, hipStream_t st) {
  k_psi<<<(kPsiValues + 255) / 256, 256, 0, st>>>(M, psi);
}

void launch_form_tangent(const Mesh& M, const OpArgs& op, const uint16_t* psi, uint16_t* kst, int* err,
                         hipStream_t st) {
  if (M.n_elems <= 0) return;
  const int nb = (M.n_elems + kTanElems - 1) / kTanElems;
  if (M.model == kLinear) k_form_tangent<kLinear><<<nb, kTanThreads, 0, st>>>(M, op, psi, kst, err);
  else if (M.model == kNH) k_form_tangent<kNH><<<nb, kTanThreads, 0, st>>>(M, op, psi, kst, err);
  else if (M.model == kSVK) k_form_tangent<kSVK><<<nb, kTanThreads, 0, st>>>(M, op, psi, kst, err);
  else k_form_tangent<kYeoh><<<nb, kTanThreads, 0, st>>>(M, op, psi, kst, err);
}

void launch_elem_forces_kst(const Mesh& M, const double* src, double sc, int scale_mih, float* F, hipStream_t st) {
  if (M.n_elems <= 0) return;
  const long long threads = (long long)M.n_elems * 8;
  k_elem_forces_kst<<<(int)((threads + 255) / 256), 256, 0, st>>>(M, src, sc, scale_mih, F);
}

}  // namespace ep
