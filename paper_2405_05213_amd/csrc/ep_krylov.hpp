// Krylov projection of exp(tau A) w for the augmented first-order elastodynamics system
// (Sec. 4.3 of the paper), executed by a team of workgroups inside one launch:
//   * operator apply (Sec. 2.3): element forces of the u-part (matrix-free hex8, fused
//     M^{-1/2} scaling), then a per-DOF gather over the node's element slots;
//   * Arnoldi with modified Gram-Schmidt: each projection h_ij = <w, v_i> is taken on the
//     vector already reduced by the previous ones; the team's slice of w stays in LDS and
//     every projection costs one team all-reduce;
//   * at check points workgroup 0 exponentiates H_j and evaluates the error estimate
//     eps_j = h_{j+1,j} ||w|| |[exp(H_j)]_{j,1}|; the decision is broadcast;
//   * the result ||w|| V_m exp(H_m) e_1 is combined in place;
//   * unconverged projections are redone with 2, 4, ... substeps of the frozen operator.
#pragma once

#include "ep_device.hpp"
#include "ep_expm.hpp"

namespace ep {

constexpr double kBreakdown = 1e-14;

// One workgroup acting alone (batched instances): team barrier = workgroup barrier.
struct BlockTeam {
  int G = 1, rank = 0;
  bool dead = false;
  __device__ bool sync(int*) {
    __syncthreads();
    return true;
  }
  __device__ double allreduce(double p, double* red, int*, bool = false) { return block_sum(p, red); }
  __device__ double post(double p, double* red, int*, bool) { return block_sum(p, red); }
  __device__ double wait(double p, int*, bool, double* = nullptr) { return p; }
};

// Entries of the next basis vector's slice that a thread can hold in registers while a
// reduction is in flight (a slice of up to kPF * blockDim entries); larger windows push
// the kernel's register allocation into spills.
constexpr int kPF = 4;

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

// Element forces of this team member's elements (operator apply, part 1).
template <typename T, int MODEL>
__device__ __forceinline__ bool phase_elements(const Mesh& M, const OpArgs& op, const double* src,
                                                         double hinv, T* F, int rank, int G) {
  bool okA = true;
  if (elem_lanes<T, MODEL>() == 8) {
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
  return okA;
}

// X <- exp(f A) X on entry ||X|| = beta.  Every workgroup returns the same result.
template <typename T, int MODEL, class Team>
__device__ ProjResult project(Team& tm, const ExpvArgs& A, double f, double beta, int hint, double pscale,
                              double* lw, double* lv, double* red, double* yb, int* flag) {
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

  double hinv = 1.0 / beta;
  const double* src = W.X;
  for (int i = threadIdx.x; i < nloc; i += blockDim.x) W.V[c0 + i] = W.X[c0 + i] * hinv;
  double hmax = 0.0;

  for (int j = 1; j <= mcap; ++j) {
    // ---- operator apply, part 1: element forces of the u-part of v_{j-1}
    const bool okA = phase_elements<T, MODEL>(M, A.op, src, hinv, F, tm.rank, tm.G);
    if (!okA) atomicCAS(&W.ctrl->err, 0, kErrInverted);
    if (!tm.sync(flag)) return R;
    {
      const int er = read_err(&W.ctrl->err);
      if (er != 0) { R.status = er; return R; }
    }
    R.nmv += 1;
    // ---- part 2 (own slice): w = f A v_{j-1}; fused with the first projection
    const double xs = src[2 * n3] * hinv * M.s_inv;      // s-entry of v_{j-1} / s0
    double part = 0.0;
    for (int i = threadIdx.x; i < nloc; i += blockDim.x) {
      const int g = c0 + i;
      double w;
      if (g < n3) {
        w = f * (src[n3 + g] * hinv);
      } else if (g < 2 * n3) {
        const int d = g - n3;
        const double s = gather_force(M, F, d / 3, d - (d / 3) * 3);
        w = f * (-M.mih[d] * s + xs * pscale * M.p0bar[d]);
      } else {
        w = 0.0;
      }
      lw[i] = w;
      const double v0 = W.V[c0 + i];
      lv[i] = v0;
      part += w * v0;
    }
    // the next basis slice is loaded while each reduction is in flight
    // prefetch only in the linear kernels (reduction-latency bound); the secant-material
    // kernels need those registers for their element code
    const bool pf_ok = (MODEL == kLinear) && nloc <= kPF * (int)blockDim.x;
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
          for (int t = threadIdx.x; t < nloc; t += blockDim.x) {
            const double w = lw[t] - hprev * lv[t];
            lw[t] = w;
            const double vi = Vi[t];
            lv[t] = vi;
            part += w * vi;
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
        for (int t = threadIdx.x; t < nloc; t += blockDim.x) {
          const double w = lw[t] - hprev * lv[t];
          lw[t] = w;
          W.Wun[c0 + t] = w;
          part += w * w;
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
      for (int t = threadIdx.x; t < nloc; t += blockDim.x) Vj[t] = lw[t] * hinv;
    }
    bool check;
    if (cfg.m_fixed > 0) check = breakdown || j == cfg.m_fixed;
    else check = breakdown || j == cfg.m_max || (j % cfg.check_every == 0 && j >= hint - cfg.check_every);
    if (check) {
      if (lead) {
        __syncthreads();
        const double* E = wg_expm(W.H, ldH, j, W.Escr, red, flag);
        const double eps = hn * beta * fabs(E[(size_t)(j - 1) * j]);
        int dec = 0;
        if (breakdown || cfg.m_fixed > 0 || eps <= cfg.tol * beta) dec = 1;
        else if (j == cfg.m_max) dec = 2;
        for (int t = threadIdx.x; t < j; t += blockDim.x) W.y[t] = beta * E[(size_t)t * j];
        if (threadIdx.x == 0) {
          W.ctrl->decision = dec;
          W.ctrl->bcast[0] = eps;
        }
      }
      if (!tm.sync(flag)) return R;
      const int dec = __hip_atomic_load(&W.ctrl->decision, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const double eps = W.ctrl->bcast[0];
      R.m = j;
      R.eps = eps;
      R.breakdown = breakdown;
      if (dec == 2) { R.converged = false; return R; }
      if (dec == 1) {
        for (int t = threadIdx.x; t < j; t += blockDim.x) yb[t] = W.y[t];
        __syncthreads();
        part = 0.0;
        for (int i = threadIdx.x; i < nloc; i += blockDim.x) {
          double s = 0.0;
          for (int t = 0; t < j; ++t) s += yb[t] * W.V[(size_t)t * Lp + c0 + i];
          W.X[c0 + i] = s;
          part += s * s;
        }
        R.beta_next = sqrt(tm.allreduce(part, red, flag, true));
        R.converged = true;
        return R;
      }
      // not converged yet: workgroup 0 can only rewrite the broadcast after the next
      // operator barrier, which every workgroup reaches after reading it
    }
    src = W.Wun;
  }
  R.converged = false;
  return R;
}

// wbar_out = exp(tau A) wbar_in with the sticky substep count and subspace-size hint of
// this projection kind; writes statistics and sticky errors.
template <typename T, int MODEL, class Team>
__device__ void expv_body(Team& tm, const ExpvArgs& A, double* lw, double* lv, double* red, double* yb,
                          int* flag) {
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
    for (int i = threadIdx.x; i < nloc; i += blockDim.x) {
      const double v = A.x_in[c0 + i];
      W.X[c0 + i] = v;
      part += v * v;
    }
    double beta = sqrt(tm.allreduce(part, red, flag, true));
    if (tm.dead) return;
    bool ok = true;
    int hint_run = hint;
    for (int sub = 0; sub < k; ++sub) {
      ProjResult r = project<T, MODEL>(tm, A, A.op.tau / k, beta, hint_run, pscale, lw, lv, red, yb, flag);
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
