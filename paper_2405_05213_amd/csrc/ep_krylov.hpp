// Krylov projection of exp(tau A) w for the augmented first-order elastodynamics system
// (Sec. 4.3 of the paper), executed by a team of workgroups inside one launch:
//   * operator apply (Sec. 2.3): element forces of the u-part (matrix-free hex8, fused
//     M^{-1/2} scaling), then a per-DOF gather over the node's element slots;
//   * Arnoldi with modified Gram-Schmidt, in one of two forms:
//     - sequential: each projection h_ij = <w, v_i> is taken on the vector already reduced
//       by the previous ones; the team's slice of w stays in LDS and every projection costs
//       one team all-reduce (j + 1 reductions in step j);
//     - compact WY: the same recurrence written as (I + L_j) h = V_j^T w, with L_j the
//       strictly lower triangle of V_j^T V_j; V_j^T w and the new row of L_j form one
//       vector all-reduce, T_j = (I + L_j)^{-1} grows by one row per step and h = T_j V_j^T w
//       (2 reductions per step, norm included);
//   * at check points workgroup 0 exponentiates H_j and evaluates the error estimate
//     eps_j = h_{j+1,j} ||w|| |[exp(H_j)]_{j,1}|; the decision is broadcast;
//   * the result ||w|| V_m exp(H_m) e_1 is combined in place;
//   * unconverged projections are redone with 2, 4, ... substeps of the frozen operator.
#pragma once

#include "ep_device.hpp"
#include "ep_expm.hpp"
#include "ep_q2.hpp"
#include "ep_tangent.hpp"

namespace ep {

constexpr double kBreakdown = 1e-14;

// One workgroup acting alone (batched instances): team barrier = workgroup barrier; sums
// with one barrier each, alternating between the two halves of the reduction scratch.
struct BlockTeam {
  static constexpr bool kVecReduce = false;
  int G = 1, rank = 0;
  bool dead = false;
  unsigned sel = 0;
  __device__ bool sync(int*) {
    __syncthreads();
    return true;
  }
  __device__ double allreduce(double p, double* red, int*, bool = false) { return block_sum2(p, red, sel); }
  __device__ double post(double p, double* red, int*, bool) { return block_sum2(p, red, sel); }
  __device__ double wait(double p, int*, bool, double* = nullptr) { return p; }
};

// LDS scratch of a projection: T (m_max x m_max, row major), the step's inner products
// (2 m_max) and reduction partials (blockDim.x) of the compact-WY form; the region ex of
// ex_cap doubles that the check point may use for exp(H_j) (it overlays the slice buffers,
// which the check does not need).
struct KLds {
  double* ke;                 // rest-state element stiffness (T-typed, 24 x kKeLd) or null
  double* T;
  double* vals;
  double* gp;
  double* ex;
  int ex_cap;
  bool ex_aliases;            // ex overlays the slice buffers (reload v_j after a check)
};

// Entries of the next basis vector's slice that a thread can hold in registers while a
// reduction is in flight (a slice of up to kPF * blockDim entries); larger windows push
// the kernel's register allocation into spills.
constexpr int kPF = 4;

// Entries per thread whose loads a slice loop issues before their stores (template parameter
// LB of the projections).  The slices may sit in LDS or in device memory behind one generic
// pointer, so a store can alias any later load and would otherwise hold back the next entry's
// loads for a full memory round trip.  Worth it where a thread owns many entries (a batch
// instance on one workgroup: 8.63 -> 7.31 ms per rubber-batch step with 4); a cost where it
// owns about one (the single-instance team: c2 6.43 -> 6.54 ms), so the team kernel uses 1.
// The batch kernel uses 2: with its registers already scarce, 2 / 4 / 8 give 4.07 / 4.16 /
// 4.36 ms per planned rubber-batch step.
constexpr int kLBBatch = 2;

__device__ __forceinline__ void prefetch_row(double (&pf)[kPF], const double* row, int nloc) {
#pragma unroll
  for (int r = 0; r < kPF; ++r) {
    const int t = threadIdx.x + r * blockDim.x;
    if (t < nloc) pf[r] = row[t];
  }
}

struct ProjResult {
  int m;
  double eps;
  bool converged;
  bool breakdown;
  int status;
  double beta_next;
  int nmv;
};

__device__ __forceinline__ int read_err(const int* err) {
  return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Element forces of this team member's elements (operator apply, part 1).  With the
// element stiffness of a congruent mesh in LDS (ke) the FP64 linear-elastic operator is
// K_e x_e.  The FP32 kernels keep the quadrature form: K_e rounded to FP32 no longer maps
// rigid motions to zero force, and its rounding costs about four orders of magnitude of
// energy accuracy on a bending cantilever.
template <typename T, int MODEL, int NPE = 8, int EL = 0>
__device__ __forceinline__ bool phase_elements(const Mesh& M, const OpArgs& op, const double* src,
                                                         double hinv, T* F, int rank, int G, const T* ke) {
  bool okA = true;
  if constexpr (NPE == kQ2Nodes) {
    // quadratic elements (kernels of their own, so that the hex8 kernels carry no Q2 code):
    // 32 lanes per element, the loop bound uniform in each lane group
    for (int e = (rank * blockDim.x + threadIdx.x) >> 5; e < M.n_elems; e += (G * blockDim.x) >> 5)
      okA &= elem_force_q2<T, MODEL>(M, op, e, src, hinv, true, F);
    return okA;
  } else if constexpr (MODEL == kStored) {
    // stored BF16 element tangents, 8 lanes per element (formed before the launch)
    for (int e = (rank * blockDim.x + threadIdx.x) >> 3; e < M.n_elems; e += (G * blockDim.x) >> 3)
      elem_force_kst(M, e, src, hinv, true, (float*)F);
  } else {
    if constexpr (MODEL == kLinear && sizeof(T) == 8) {
      if (ke != nullptr) {
        for (int e = (rank * blockDim.x + threadIdx.x) >> 3; e < M.n_elems; e += (G * blockDim.x) >> 3)
          elem_force_ke(M, e, src, hinv, (const double*)ke, (double*)F);
        return true;
      }
    }
    // EL: lanes per element chosen by the kernel (0: elem_lanes) - the batch kernel takes one
    // lane per element in FP64 too (its workgroups are latency-bound on a mesh each)
    constexpr int lanes = EL ? EL : elem_lanes<T, MODEL>();
    if (lanes == 8) {
      // 8 lanes per element (one per Gauss point); the loop bound is uniform in each lane group
      for (int e = (rank * blockDim.x + threadIdx.x) >> 3; e < M.n_elems; e += (G * blockDim.x) >> 3)
        okA &= elem_force_qp<T, MODEL>(M, op, e, src, hinv, true, F);
    } else {
      for (int e = rank * blockDim.x + threadIdx.x; e < M.n_elems; e += G * blockDim.x) {
        T fe[8][3];
        okA &= elem_force<T, MODEL>(M, op, e, src, hinv, true, fe);
        store_force(M, e, fe, F);
      }
    }
  }
  return okA;
}

// Element forces of the fourth-order scheme's operator Omega (see elem_force_qp_m4): F gets
// the v-part forces, F2 the u-part forces.  Linear elasticity: both sets are K, the u-part
// vanishes and F = K M^{-1/2} x_u as in the second-order operator.
template <typename T, int MODEL>
__device__ __forceinline__ bool phase_elements_m4(const Mesh& M, const OpArgs& op, const double* src,
                                                  double hinv, T* F, T* F2, int rank, int G, const T* ke) {
  if constexpr (MODEL == kLinear) {
    return phase_elements<T, MODEL>(M, op, src, hinv, F, rank, G, ke);
  } else {
    bool ok = true;
    for (int e = (rank * blockDim.x + threadIdx.x) >> 3; e < M.n_elems; e += (G * blockDim.x) >> 3)
      ok &= elem_force_qp_m4<T, MODEL>(M, op, e, src, hinv, F, F2);
    return ok;
  }
}

// Entry g of f Omega v for the fourth-order scheme (src = v / hinv, xs = its augmented entry
// / s0, ps1 / ps2 the load scales at the two Gauss nodes):
//   u-part  dt x_v - M^{-1/2} Fu - c xs (p_2 - p_1)
//   v-part  -M^{-1/2} Fv + dt/2 xs (p_1 + p_2)        (linear: -dt M^{-1/2} K M^{-1/2} x_u)
template <typename T, int MODEL>
__device__ __forceinline__ double m4_entry(const Mesh& M, const SlotMap& sm, const OpArgs& op, const T* F,
                                           const T* F2, const double* src, double hinv, double xs, double ps1,
                                           double ps2, double f, int g) {
  const int n3 = M.n3;
  if (g < n3) {
    double w = op.dt4 * (src[n3 + g] * hinv) - op.c4 * xs * (ps2 - ps1) * M.p0bar[g];
    if constexpr (MODEL != kLinear) w -= M.mih[g] * gather_slots(sm, F2, g / 3, g - (g / 3) * 3);
    return f * w;
  }
  if (g < 2 * n3) {
    const int d = g - n3;
    const double s = gather_slots(sm, F, d / 3, d - (d / 3) * 3);
    const double sc = MODEL == kLinear ? op.dt4 : 1.0;
    return f * (-M.mih[d] * sc * s + 0.5 * op.dt4 * xs * (ps1 + ps2) * M.p0bar[d]);
  }
  return 0.0;
}

// Check point of step j (shared by both orthogonalisation forms): workgroup 0 exponentiates
// H_j and decides; on convergence X <- V_j y with y = beta exp(H_j) e_1.  Returns 0 to go
// on, 1 when the projection ends (R filled), -1 when the team died.
template <class Team>
__device__ __forceinline__ int check_point(Team& tm, const ExpvArgs& A, int j, double hn, double beta,
                                           bool breakdown, double* red, double* yb, const KLds& X, int* flag,
                                           int nloc, int c0, ProjResult& R) {
  const KWork& W = A.W;
  const KrylovCfg& cfg = A.cfg;
  const int ldH = cfg.m_max;
  const size_t Lp = (size_t)A.M.Lp;
  if (tm.rank == 0) {
    __syncthreads();
    // out of line (see wg_expm_call); scratch in LDS when it fits, else in device memory
    double* scr = (X.ex != nullptr && expm_scratch(j) <= X.ex_cap) ? X.ex : W.Escr;
    const double* E = wg_expm_call(W.H, ldH, j, scr, red);
    const int le = expm_ld(j);
    const double eps = hn * beta * fabs(E[(size_t)(j - 1) * le]);
    int dec = 0;
    if (breakdown || cfg.m_fixed > 0 || eps <= cfg.tol * beta) dec = 1;
    else if (j == cfg.m_max) dec = 2;
    for (int t = threadIdx.x; t < j; t += blockDim.x) W.y[t] = beta * E[(size_t)t * le];
    if (threadIdx.x == 0) {
      W.ctrl->decision = dec;
      W.ctrl->bcast[0] = eps;
    }
  }
  if (!tm.sync(flag)) return -1;
  const int dec = __hip_atomic_load(&W.ctrl->decision, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double eps = W.ctrl->bcast[0];
  R.m = j;
  R.eps = eps;
  R.breakdown = breakdown;
  if (dec == 2) { R.converged = false; return 1; }
  if (dec == 1) {
    for (int t = threadIdx.x; t < j; t += blockDim.x) yb[t] = W.y[t];
    __syncthreads();
    double part = 0.0;
    for (int i = threadIdx.x; i < nloc; i += blockDim.x) {
      const double* Vi = W.V + c0 + i;
      double s = 0.0;
      int t = 0;
      for (; t + 8 <= j; t += 8) {
        double q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = Vi[(size_t)(t + u) * Lp];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += yb[t + u] * q[u];
      }
      for (; t < j; ++t) s += yb[t] * Vi[(size_t)t * Lp];
      W.X[c0 + i] = s;
      part += s * s;
    }
    R.beta_next = sqrt(tm.allreduce(part, red, flag, true));
    R.converged = true;
    return 1;
  }
  // not converged yet: workgroup 0 can only rewrite the broadcast after the next operator
  // barrier, which every workgroup reaches after reading it
  return 0;
}

// X <- exp(f A) X on entry ||X|| = beta (SCH = 4: exp(f Omega) X).  Every workgroup returns
// the same result.
template <typename T, int MODEL, class Team, int SCH = 2, int NPE = 8, int LB = 1, int EL = 0>
__device__ ProjResult project(Team& tm, const ExpvArgs& A, double f, double beta, int hint, double pscale,
                              double* lw, double* lv, double* red, double* yb, int* flag, const KLds& X) {
  const Mesh& M = A.M;
  const KWork& W = A.W;
  const KrylovCfg& cfg = A.cfg;
  ProjResult R{0, 0.0, true, true, 0, 0.0, 0};
  if (beta == 0.0) return R;                 // exp(fA) 0 = 0
  if (!(beta < INFINITY)) { R.status = kErrNonfinite; return R; }
  const int C = W.chunk;
  const int c0 = tm.rank * C;
  const int nloc = max(0, min(c0 + C, M.Lp) - c0);
  const int n3 = M.n3;
  const size_t Lp = (size_t)M.Lp;
  const int ldH = cfg.m_max;
  const int mcap = cfg.m_fixed > 0 ? cfg.m_fixed : cfg.m_max;
  const bool lead = tm.rank == 0;
  T* F = (sizeof(T) == 8) ? (T*)W.F : (T*)W.F32;
  T* F2 = (sizeof(T) == 8) ? (T*)W.F2 : (T*)W.F2_32;
  const double pscale2 = SCH == 4 ? load_scale(M, A.op.t_eval2) : 0.0;

  double hinv = 1.0 / beta;
  const double* src = W.X;
  // lv == nullptr: only w's slice is held (LDS too small for two); the newest basis vector
  // is read back from its row of V where the held copy would be used
  const bool lvV = lv == nullptr;
  for (int i0 = threadIdx.x; i0 < nloc; i0 += LB * blockDim.x) {
    double x[LB];
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int i = i0 + u * blockDim.x;
      x[u] = i < nloc ? W.X[c0 + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int i = i0 + u * blockDim.x;
      if (i < nloc) W.V[c0 + i] = x[u] * hinv;
    }
  }
  double hmax = 0.0;

  for (int j = 1; j <= mcap; ++j) {
    // ---- operator apply, part 1: element forces of the u-part of v_{j-1}
    bool okA;
    if constexpr (SCH == 4) okA = phase_elements_m4<T, MODEL>(M, A.op, src, hinv, F, F2, tm.rank, tm.G, (const T*)X.ke);
    else okA = phase_elements<T, MODEL, NPE, EL>(M, A.op, src, hinv, F, tm.rank, tm.G, (const T*)X.ke);
    if (!okA) atomicCAS(&W.ctrl->err, 0, kErrInverted);
    if (!tm.sync(flag)) return R;
    {
      const int er = read_err(&W.ctrl->err);
      if (er != 0) { R.status = er; return R; }
    }
    R.nmv += 1;
    // ---- part 2 (own slice): w = f A v_{j-1}; fused with the first projection
    const double xs = src[2 * n3] * hinv * M.s_inv;      // s-entry of v_{j-1} / s0
    const SlotMap sm = slot_map(M);                       // not held across the element pass
    double part = 0.0;
    if constexpr (SCH == 4) {
      for (int i0 = threadIdx.x; i0 < nloc; i0 += LB * blockDim.x) {
        double w[LB], v0[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int i = i0 + u * blockDim.x;
          w[u] = 0.0;
          v0[u] = 0.0;
          if (i < nloc) {
            w[u] = m4_entry<T, MODEL>(M, sm, A.op, F, F2, src, hinv, xs, pscale, pscale2, f, c0 + i);
            v0[u] = W.V[c0 + i];
          }
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int i = i0 + u * blockDim.x;
          if (i < nloc) {
            lw[i] = w[u];
            if (!lvV) lv[i] = v0[u];
            part += w[u] * v0[u];
          }
        }
      }
    } else {
      // own entries [0, uhi): u-part, w = f v-part of v_{j-1}; [uhi, vhi): v-part, from the
      // element forces, node by node; [vhi, nloc): the s-row and padding, w = 0
      const int uhi = min(nloc, max(0, n3 - c0));
      const int vhi = min(nloc, max(uhi, 2 * n3 - c0));
      for (int r = 0; r < 2; ++r) {
        const int lo = r == 0 ? 0 : vhi, hi = r == 0 ? uhi : nloc;
        for (int i0 = lo + threadIdx.x; i0 < hi; i0 += LB * blockDim.x) {
          double w[LB], v0[LB];
#pragma unroll
          for (int u = 0; u < LB; ++u) {
            const int i = i0 + u * blockDim.x;
            w[u] = 0.0;
            v0[u] = 0.0;
            if (i < hi) {
              if (r == 0) w[u] = f * (src[n3 + c0 + i] * hinv);
              v0[u] = W.V[c0 + i];
            }
          }
#pragma unroll
          for (int u = 0; u < LB; ++u) {
            const int i = i0 + u * blockDim.x;
            if (i < hi) {
              lw[i] = w[u];
              if (!lvV) lv[i] = v0[u];
              part += w[u] * v0[u];
            }
          }
        }
      }
      if (uhi < vhi) {
        const int a0 = (c0 + uhi - n3) / 3, a1 = (c0 + vhi - 1 - n3) / 3;   // first and last node
        const double ps = xs * pscale;
        for (int An = a0 + threadIdx.x; An <= a1; An += blockDim.x) {
          double s[3];
          gather_node(sm, F, An, s);
          double w[3], v0[3];
          bool own[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const int d = 3 * An + c;
            const int i = n3 + d - c0;
            own[c] = i >= uhi && i < vhi;
            w[c] = own[c] ? f * (-M.mih[d] * s[c] + ps * M.p0bar[d]) : 0.0;
            v0[c] = own[c] ? W.V[c0 + i] : 0.0;
          }
#pragma unroll
          for (int c = 0; c < 3; ++c)
            if (own[c]) {
              const int i = n3 + 3 * An + c - c0;
              lw[i] = w[c];
              if (!lvV) lv[i] = v0[c];
              part += w[c] * v0[c];
            }
        }
      }
    }
    // the next basis slice is loaded while each reduction is in flight
    // prefetch only in the linear kernels (reduction-latency bound); the secant-material
    // kernels need those registers for their element code
    const bool pf_ok = (MODEL == kLinear || MODEL == kStored) && nloc <= kPF * (int)blockDim.x && !lvV;
    double pf[kPF];
    double hp = tm.post(part, red, flag, false);
    if (pf_ok && 1 < j) prefetch_row(pf, W.V + Lp + c0, nloc);
    double h = tm.wait(hp, flag, false, red);
    if (tm.dead) return R;
    if (lead && threadIdx.x == 0) W.H[0 * ldH + (j - 1)] = h;
    hmax = fmax(hmax, fabs(h));
    bool finite = fabs(h) < INFINITY;
    double hprev = h, hn = 0.0;
    // ---- modified Gram-Schmidt against v_1 .. v_{j-1}, then the norm
    for (int i = 1; i <= j; ++i) {
      part = 0.0;
      if (i < j) {
        if (pf_ok) {
#pragma unroll
          for (int r = 0; r < kPF; ++r) {
            const int t = threadIdx.x + r * blockDim.x;
            if (t < nloc) {
              const double w = lw[t] - hprev * lv[t];
              lw[t] = w;
              lv[t] = pf[r];
              part += w * pf[r];
            }
          }
        } else {
          const double* Vi = W.V + (size_t)i * Lp + c0;
          const double* Vp = lvV ? Vi - Lp : lv;         // v_{i-1}
          for (int t0 = threadIdx.x; t0 < nloc; t0 += LB * blockDim.x) {
            double a[LB], b[LB], q[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
              const int t = t0 + u * blockDim.x;
              if (t < nloc) {
                a[u] = lw[t];
                b[u] = Vp[t];
                q[u] = Vi[t];
              }
            }
#pragma unroll
            for (int u = 0; u < LB; ++u) {
              const int t = t0 + u * blockDim.x;
              if (t < nloc) {
                const double w = a[u] - hprev * b[u];
                lw[t] = w;
                if (!lvV) lv[t] = q[u];
                part += w * q[u];
              }
            }
          }
        }
        hp = tm.post(part, red, flag, false);
        if (pf_ok && i + 1 < j) prefetch_row(pf, W.V + (size_t)(i + 1) * Lp + c0, nloc);
        h = tm.wait(hp, flag, false, red);
        if (tm.dead) return R;
        if (lead && threadIdx.x == 0) W.H[(size_t)i * ldH + (j - 1)] = h;
        hmax = fmax(hmax, fabs(h));
        finite &= fabs(h) < INFINITY;
        hprev = h;
      } else {
        const double* Vp = lvV ? W.V + (size_t)(j - 1) * Lp + c0 : lv;   // v_{j-1}
        for (int t0 = threadIdx.x; t0 < nloc; t0 += LB * blockDim.x) {
          double a[LB], b[LB];
#pragma unroll
          for (int u = 0; u < LB; ++u) {
            const int t = t0 + u * blockDim.x;
            if (t < nloc) {
              a[u] = lw[t];
              b[u] = Vp[t];
            }
          }
#pragma unroll
          for (int u = 0; u < LB; ++u) {
            const int t = t0 + u * blockDim.x;
            if (t < nloc) {
              const double w = a[u] - hprev * b[u];
              lw[t] = w;
              W.Wun[c0 + t] = w;
              part += w * w;
            }
          }
        }
        hn = sqrt(tm.allreduce(part, red, flag, true));
        if (tm.dead) return R;
        if (lead && threadIdx.x == 0) W.H[(size_t)j * ldH + (j - 1)] = hn;
        hmax = fmax(hmax, hn);
        finite &= hn < INFINITY;
      }
    }
    if (!finite) { R.status = kErrNonfinite; return R; }
    const bool breakdown = hn <= kBreakdown * hmax;
    // v_j = w / h_{j+1,j} (also kept when the projection stops here: A V_m = V_{m+1} Htilde)
    if (!breakdown) {
      hinv = 1.0 / hn;
      double* Vj = W.V + (size_t)j * Lp + c0;
      for (int t0 = threadIdx.x; t0 < nloc; t0 += LB * blockDim.x) {
        double a[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int t = t0 + u * blockDim.x;
          a[u] = t < nloc ? lw[t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int t = t0 + u * blockDim.x;
          if (t < nloc) Vj[t] = a[u] * hinv;
        }
      }
    }
    bool check;
    if (cfg.m_fixed > 0) check = breakdown || j == cfg.m_fixed;
    else check = breakdown || j == cfg.m_max || (j % cfg.check_every == 0 && j >= hint - cfg.check_every);
    if (check) {
      const int c = check_point(tm, A, j, hn, beta, breakdown, red, yb, X, flag, nloc, c0, R);
      if (c != 0) return R;
    }
    src = W.Wun;
  }
  R.converged = false;
  return R;
}

// Compact-WY form of the projection (see the file header).  Per step: the operator barrier,
// one vector all-reduce of the 2j - 1 inner products, the fenced norm all-reduce.
template <typename T, int MODEL, class Team, int SCH = 2, int NPE = 8, int LB = 1, int EL = 0>
__device__ ProjResult project_cwy(Team& tm, const ExpvArgs& A, double f, double beta, int hint, double pscale,
                                  double* lw, double* lv, double* red, double* yb, int* flag, const KLds& X) {
  const Mesh& M = A.M;
  const KWork& W = A.W;
  const KrylovCfg& cfg = A.cfg;
  ProjResult R{0, 0.0, true, true, 0, 0.0, 0};
  if (beta == 0.0) return R;
  if (!(beta < INFINITY)) { R.status = kErrNonfinite; return R; }
  const int C = W.chunk;
  const int c0 = tm.rank * C;
  const int nloc = max(0, min(c0 + C, M.Lp) - c0);
  const int n3 = M.n3;
  const size_t Lp = (size_t)M.Lp;
  const int ldH = cfg.m_max, ldT = cfg.m_max;
  const int mcap = cfg.m_fixed > 0 ? cfg.m_fixed : cfg.m_max;
  const bool lead = tm.rank == 0;
  const int nw = (int)(blockDim.x >> 6), lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  T* F = (sizeof(T) == 8) ? (T*)W.F : (T*)W.F32;
  T* F2 = (sizeof(T) == 8) ? (T*)W.F2 : (T*)W.F2_32;
  const double pscale2 = SCH == 4 ? load_scale(M, A.op.t_eval2) : 0.0;

  double hinv = 1.0 / beta;
  const double* src = W.X;
  for (int i = threadIdx.x; i < nloc; i += blockDim.x) {
    const double v = W.X[c0 + i] * hinv;
    W.V[c0 + i] = v;
    lv[i] = v;                                   // lv: slice of the newest basis vector
  }
  double hmax = 0.0;

  for (int j = 1; j <= mcap; ++j) {
    bool okA;
    if constexpr (SCH == 4) okA = phase_elements_m4<T, MODEL>(M, A.op, src, hinv, F, F2, tm.rank, tm.G, (const T*)X.ke);
    else okA = phase_elements<T, MODEL, NPE, EL>(M, A.op, src, hinv, F, tm.rank, tm.G, (const T*)X.ke);
    if (!okA) atomicCAS(&W.ctrl->err, 0, kErrInverted);
    if (!tm.sync(flag)) return R;
    {
      const int er = read_err(&W.ctrl->err);
      if (er != 0) { R.status = er; return R; }
    }
    R.nmv += 1;
    // w = f A v_{j-1} on the own slice
    const double xs = src[2 * n3] * hinv * M.s_inv;
    const SlotMap sm = slot_map(M);
    if constexpr (SCH == 4) {
      for (int i0 = threadIdx.x; i0 < nloc; i0 += LB * blockDim.x) {
        double w[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int i = i0 + u * blockDim.x;
          w[u] = i < nloc ? m4_entry<T, MODEL>(M, sm, A.op, F, F2, src, hinv, xs, pscale, pscale2, f, c0 + i) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int i = i0 + u * blockDim.x;
          if (i < nloc) lw[i] = w[u];
        }
      }
    } else {
      // as in the sequential form: u-part entries one by one, the v-part node by node
      const int uhi = min(nloc, max(0, n3 - c0));
      const int vhi = min(nloc, max(uhi, 2 * n3 - c0));
      for (int r = 0; r < 2; ++r) {
        const int lo = r == 0 ? 0 : vhi, hi = r == 0 ? uhi : nloc;
        for (int i0 = lo + threadIdx.x; i0 < hi; i0 += LB * blockDim.x) {
          double w[LB];
#pragma unroll
          for (int u = 0; u < LB; ++u) {
            const int i = i0 + u * blockDim.x;
            w[u] = (i < hi && r == 0) ? f * (src[n3 + c0 + i] * hinv) : 0.0;
          }
#pragma unroll
          for (int u = 0; u < LB; ++u) {
            const int i = i0 + u * blockDim.x;
            if (i < hi) lw[i] = w[u];
          }
        }
      }
      if (uhi < vhi) {
        const int a0 = (c0 + uhi - n3) / 3, a1 = (c0 + vhi - 1 - n3) / 3;
        const double ps = xs * pscale;
        for (int An = a0 + threadIdx.x; An <= a1; An += blockDim.x) {
          double s[3];
          gather_node(sm, F, An, s);
          double w[3];
          bool own[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const int d = 3 * An + c;
            const int i = n3 + d - c0;
            own[c] = i >= uhi && i < vhi;
            w[c] = own[c] ? f * (-M.mih[d] * s[c] + ps * M.p0bar[d]) : 0.0;
          }
#pragma unroll
          for (int c = 0; c < 3; ++c)
            if (own[c]) lw[n3 + 3 * An + c - c0] = w[c];
        }
      }
    }
    __syncthreads();
    // partial inner products b_k = <v_k, w> (k < j) and l_k = <v_k, v_{j-1}> (k < j - 1):
    // each wave takes one (value, segment) unit at a time, lanes stride the segment
    const int S = max(1, nw / j);
    const int seg = (nloc + S - 1) / S;
    const int K2 = 2 * j;
    for (int u = wv; u < j * S; u += nw) {
      const int k = u % j, sg = u / j;
      const int t0 = sg * seg, t1 = min(nloc, t0 + seg);
      double b = 0.0, l = 0.0;
      if (k == j - 1) {
        for (int t = t0 + lane; t < t1; t += 64) b += lv[t] * lw[t];
      } else {
        // 8 loads in flight per lane
        const double* Vk = W.V + (size_t)k * Lp + c0;
        for (int tb = t0 + lane; tb < t1; tb += 64 * 8) {
          double q[8];
#pragma unroll
          for (int r = 0; r < 8; ++r) q[r] = tb + 64 * r < t1 ? Vk[tb + 64 * r] : 0.0;
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const int t = tb + 64 * r;
            if (t < t1) {
              b += q[r] * lw[t];
              l += q[r] * lv[t];
            }
          }
        }
      }
      b = wave_sum(b);
      l = wave_sum(l);
      if (lane == 0) {
        X.gp[sg * K2 + k] = b;
        X.gp[sg * K2 + j + k] = l;
      }
    }
    __syncthreads();
    const int K = 2 * j - 1;
    for (int t = threadIdx.x; t < K; t += blockDim.x) {
      double s = 0.0;
      for (int sg = 0; sg < S; ++sg) s += X.gp[sg * K2 + t];
      X.vals[t] = s;
    }
    __syncthreads();
    if (!tm.allreduce_vec(X.vals, K, X.gp, flag)) return R;
    // new row of T = (I + L)^{-1}: T[j-1][i] = -sum_{k=i}^{j-2} l_k T[k][i]; then h = T b.
    // Eight lanes per row, each summing every eighth term, then a 3-step butterfly.
    const double* bv = X.vals;
    const double* lv2 = X.vals + j;
    double* Tr = X.T + (size_t)(j - 1) * ldT;
    const int sub = threadIdx.x & 7;
    for (int i = threadIdx.x >> 3; i < j - 1; i += blockDim.x >> 3) {
      double s = 0.0;
      for (int k = i + sub; k < j - 1; k += 8) s += lv2[k] * X.T[(size_t)k * ldT + i];
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      if (sub == 0) Tr[i] = -s;
    }
    if (threadIdx.x == 0) Tr[j - 1] = 1.0;
    __syncthreads();
    for (int i = threadIdx.x >> 3; i < j; i += blockDim.x >> 3) {
      const double* Ti = X.T + (size_t)i * ldT;
      double s = 0.0;
      for (int k = sub; k <= i; k += 8) s += Ti[k] * bv[k];
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      if (sub == 0) {
        yb[i] = s;
        if (lead) W.H[(size_t)i * ldH + (j - 1)] = s;
      }
    }
    __syncthreads();
    bool finite = true;
    for (int i = 0; i < j; ++i) {
      const double h = yb[i];
      hmax = fmax(hmax, fabs(h));
      finite &= fabs(h) < INFINITY;
    }
    // w <- w - V_j h, its norm, and the unnormalised vector for the next operator apply
    double part = 0.0;
    for (int t = threadIdx.x; t < nloc; t += blockDim.x) {
      double w = lw[t];
      const double* Vt = W.V + c0 + t;
      int k = 0;
      for (; k + 16 <= j - 1; k += 16) {
        double q[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) q[u] = Vt[(size_t)(k + u) * Lp];
#pragma unroll
        for (int u = 0; u < 16; ++u) w -= yb[k + u] * q[u];
      }
      for (; k + 4 <= j - 1; k += 4) {
        double q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = Vt[(size_t)(k + u) * Lp];
#pragma unroll
        for (int u = 0; u < 4; ++u) w -= yb[k + u] * q[u];
      }
      for (; k < j - 1; ++k) w -= yb[k] * Vt[(size_t)k * Lp];
      w -= yb[j - 1] * lv[t];
      lw[t] = w;
      W.Wun[c0 + t] = w;
      part += w * w;
    }
    const double hn = sqrt(tm.allreduce(part, red, flag, true));
    if (tm.dead) return R;
    if (lead && threadIdx.x == 0) W.H[(size_t)j * ldH + (j - 1)] = hn;
    hmax = fmax(hmax, hn);
    finite &= hn < INFINITY;
    if (!finite) { R.status = kErrNonfinite; return R; }
    const bool breakdown = hn <= kBreakdown * hmax;
    if (!breakdown) {
      hinv = 1.0 / hn;
      double* Vj = W.V + (size_t)j * Lp + c0;
      for (int t0 = threadIdx.x; t0 < nloc; t0 += LB * blockDim.x) {
        double a[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int t = t0 + u * blockDim.x;
          a[u] = t < nloc ? lw[t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
          const int t = t0 + u * blockDim.x;
          if (t < nloc) {
            const double v = a[u] * hinv;
            Vj[t] = v;
            lv[t] = v;
          }
        }
      }
    }
    bool check;
    if (cfg.m_fixed > 0) check = breakdown || j == cfg.m_fixed;
    else check = breakdown || j == cfg.m_max || (j % cfg.check_every == 0 && j >= hint - cfg.check_every);
    if (check) {
      const int c = check_point(tm, A, j, hn, beta, breakdown, red, yb, X, flag, nloc, c0, R);
      if (c != 0) return R;
      if (lead && X.ex_aliases && X.ex != nullptr && expm_scratch(j) <= X.ex_cap) {
        // exp(H_j) overwrote the slice buffers of workgroup 0: reload v_j (w is rebuilt)
        const double* Vj = W.V + (size_t)j * Lp + c0;
        for (int t = threadIdx.x; t < nloc; t += blockDim.x) lv[t] = Vj[t];
      }
    }
    src = W.Wun;
  }
  R.converged = false;
  return R;
}

// wbar_out = exp(tau A) wbar_in with the sticky substep count and subspace-size hint of
// this projection kind; writes statistics and sticky errors.
template <typename T, int MODEL, class Team, int ORTHO = 0, int SCH = 2, int NPE = 8, int LB = 1, int EL = 0>
__device__ void expv_body(Team& tm, const ExpvArgs& A, double* lw, double* lv, double* red, double* yb,
                          int* flag, const KLds& cx) {
  const Mesh& M = A.M;
  const KWork& W = A.W;
  const KrylovCfg& cfg = A.cfg;
  const int C = W.chunk;
  const int c0 = tm.rank * C;
  const int nloc = max(0, min(c0 + C, M.Lp) - c0);
  const int n3 = M.n3;
  const double pscale = load_scale(M, A.op.t_eval);
  KState ks = W.ctrl->ks[A.kind];
  int k = cfg.k_fixed > 0 ? cfg.k_fixed : max(1, ks.k);
  int hint = ks.m_hint;
  int status = 0, last_m = 0, first_m = 0, nmv = 0;
  double last_eps = 0.0;
  for (;;) {
    double part = 0.0;
    for (int i0 = threadIdx.x; i0 < nloc; i0 += LB * blockDim.x) {
      double x[LB];
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int i = i0 + u * blockDim.x;
        x[u] = i < nloc ? A.x_in[c0 + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < LB; ++u) {
        const int i = i0 + u * blockDim.x;
        if (i < nloc) {
          W.X[c0 + i] = x[u];
          part += x[u] * x[u];
        }
      }
    }
    double beta = sqrt(tm.allreduce(part, red, flag, true));
    if (tm.dead) return;
    bool ok = true;
    int hint_run = hint;
    for (int sub = 0; sub < k; ++sub) {
      ProjResult r;
      if constexpr (Team::kVecReduce && ORTHO == 1)
        r = project_cwy<T, MODEL, Team, SCH, NPE, LB, EL>(tm, A, A.op.tau / k, beta, hint_run, pscale, lw, lv, red, yb, flag, cx);
      else
        r = project<T, MODEL, Team, SCH, NPE, LB, EL>(tm, A, A.op.tau / k, beta, hint_run, pscale, lw, lv, red, yb, flag, cx);
      if (tm.dead) return;
      nmv += r.nmv;
      if (r.status != 0) { status = r.status; ok = false; break; }
      if (!r.converged) { ok = false; break; }
      last_m = r.m;
      last_eps = r.eps;
      if (sub == 0) first_m = r.m;
      if (!r.breakdown) hint_run = r.m;
      beta = r.beta_next;
    }
    if (status != 0) break;
    if (ok) { hint = hint_run; break; }
    if (cfg.k_fixed > 0 || 2 * k > cfg.max_substeps) { status = kErrKrylov; break; }
    k *= 2;
    hint = 0;
  }
  if (status == 0) {
    if (A.out_mode == 0) {
      for (int i = threadIdx.x; i < nloc; i += blockDim.x) {
        const int g = c0 + i;
        double v = W.X[g];
        if (g == 2 * n3) {
          W.ctrl->drift = fabs(v - M.s0);
          v = M.s0;
        }
        A.x_out[g] = v;
      }
    } else if (A.out_mode == 1) {
      for (int i = threadIdx.x; i < nloc; i += blockDim.x) {
        const int g = c0 + i;
        if (g < n3) A.x_out[g] = M.mih[g] * W.X[g];
      }
    } else {
      for (int i = threadIdx.x; i < nloc; i += blockDim.x) A.x_out[c0 + i] = W.X[c0 + i];
    }
  }
  if (tm.rank == 0 && threadIdx.x == 0) {
    KState& o = W.ctrl->ks[A.kind];
    o.matvecs = ks.matvecs + nmv;
    if (status == 0) {
      o.k = k;
      o.m_hint = hint;
      o.last_m = last_m;
      o.last_k = k;
      o.last_eps = last_eps;
    } else {
      atomicCAS(&W.ctrl->err, 0, status);
    }
    if (A.log_idx >= 0 && W.log != nullptr && A.kind < 2) {
      const int s = A.log_idx % kLogSteps;
      if (A.kind == 0) {
        W.log->m_corr[s] = first_m;
        W.log->k_corr[s] = k;
        W.log->eps_corr[s] = last_eps;
      } else {
        W.log->m_pred[s] = first_m;
      }
    }
  }
  // outputs and the adaptive state are visible to the whole team before anything reads them
  tm.sync(flag);
}

}  // namespace ep
