// Batched instances (many independent meshes / materials / loads): one workgroup per
// instance runs the whole predictor-corrector step of its instance, so the Krylov
// reductions never leave the workgroup.  The stepping state lives in device records and
// one launch advances every instance by one step, which makes the launch replayable from a
// captured graph.
#include "ep_kernels.hpp"
#include "ep_krylov.hpp"

namespace ep {

// u = M^{-1/2} ubar over the team's slice, then a team barrier
template <class Team>
__device__ void team_get_u(Team& tm, const Mesh& M, const double* S, double* u, int* flag) {
  for (int d = threadIdx.x; d < M.n3; d += blockDim.x) u[d] = M.mih[d] * S[d];
  tm.sync(flag);
}

static __device__ __forceinline__ int free_slot(int a, int b) {
  for (int s = 0; s < 3; ++s)
    if (s != a && s != b) return s;
  return 0;
}

// One step of one instance (Sec. 4.1-4.2); returns false after a sticky error.
template <typename T, int MODEL, class Team>
__device__ bool device_step(Team& tm, BatchInst& B, const KrylovCfg& cfg, double dt, double* lw, double* lv,
                            double* red, double* yb, int* flag, const KLds& X) {
  ExpvArgs a;
  a.M = B.M;
  a.W = B.W;
  a.cfg = cfg;
  a.log_idx = (int)(B.step_idx % kLogSteps);
  const double t = B.t;
  const int n3 = B.M.n3;
  if (MODEL == kLinear) {
    a.op.tau = dt;
    a.op.t_eval = t + 0.5 * dt;
    a.op.nsets = 0;
    a.kind = 0;
    a.x_in = B.S;
    a.x_out = B.S;
    a.out_mode = 0;
    expv_body<T, MODEL>(tm, a, lw, lv, red, yb, flag, X);
  } else {
    OpArgs pred{};
    pred.tau = 0.5 * dt;
    pred.t_eval = t + 0.25 * dt;
    int reserve = -1;
    if (B.nhist == 0) {
      const int s0 = free_slot(B.hist_new, B.hist_old);
      team_get_u(tm, B.M, B.S, B.hist + (size_t)s0 * n3, flag);
      pred.nsets = 1;
      pred.ulin[0] = B.hist + (size_t)s0 * n3;
      pred.wts[0] = 1.0;
      reserve = s0;
    } else if (B.nhist == 1) {
      pred.nsets = 1;
      pred.ulin[0] = B.hist + (size_t)B.hist_new * n3;
      pred.wts[0] = 1.0;
    } else {
      pred.nsets = 2;
      pred.ulin[0] = B.hist + (size_t)B.hist_new * n3;
      pred.wts[0] = 1.75;
      pred.ulin[1] = B.hist + (size_t)B.hist_old * n3;
      pred.wts[1] = -0.75;
    }
    const int snew = free_slot(B.hist_new, reserve >= 0 ? reserve : B.hist_old);
    a.op = pred;
    a.kind = 1;
    a.x_in = B.S;
    a.x_out = B.hist + (size_t)snew * n3;
    a.out_mode = 1;
    expv_body<T, MODEL>(tm, a, lw, lv, red, yb, flag, X);
    if (tm.dead || read_err(&B.W.ctrl->err) != 0) return false;
    OpArgs corr{};
    corr.tau = dt;
    corr.t_eval = t + 0.5 * dt;
    corr.nsets = 1;
    corr.ulin[0] = B.hist + (size_t)snew * n3;
    corr.wts[0] = 1.0;
    a.op = corr;
    a.kind = 0;
    a.x_in = B.S;
    a.x_out = B.S;
    a.out_mode = 0;
    expv_body<T, MODEL>(tm, a, lw, lv, red, yb, flag, X);
    if (B.nhist == 0) {
      B.hist_old = -1;
      B.hist_new = snew;
      B.nhist = 1;
    } else {
      B.hist_old = B.hist_new;
      B.hist_new = snew;
      B.nhist = 2;
    }
  }
  if (tm.dead || read_err(&B.W.ctrl->err) != 0) return false;
  B.t = t + dt;
  B.step_idx += 1;
  return true;
}

// doubles of LDS before the slice buffers: red[32] | yb[kMaxM] | ints flag[16], 16 unused
constexpr int kBatchHead = 32 + kMaxM + 16;

template <typename T, int MODEL>
__global__ __launch_bounds__(kThreads) void k_batch(BatchInst* tab, const int* ids, KrylovCfg cfg, double dt,
                                                    int n_steps, int lds_slices) {
  extern __shared__ double lds[];
  double* red = lds;
  double* yb = lds + 32;
  int* flag = (int*)(lds + 32 + kMaxM);
  // the slice region (lds_slices doubles) doubles as expm scratch: the sequential form
  // reloads both slice buffers after a check point
  const KLds X{nullptr, nullptr, nullptr, nullptr, lds + kBatchHead, lds_slices, true};
  if (threadIdx.x == 0) *flag = 1;
  __syncthreads();
  const int id = ids[blockIdx.x];
  BatchInst B = tab[id];
  double* lw;
  double* lv;
  if (B.use_lds) {
    lw = lds + kBatchHead;
    lv = lw + B.W.chunk;
  } else {
    lw = B.W.wscr;
    lv = B.W.wscr + B.M.Lp;
  }
  BlockTeam tm;
  for (int s = 0; s < n_steps; ++s)
    if (!device_step<T, MODEL>(tm, B, cfg, dt, lw, lv, red, yb, flag, X)) break;
  if (threadIdx.x == 0) {
    tab[id].t = B.t;
    tab[id].step_idx = B.step_idx;
    tab[id].nhist = B.nhist;
    tab[id].hist_new = B.hist_new;
    tab[id].hist_old = B.hist_old;
  }
}

size_t batch_lds_bytes(int max_lds_chunk) { return (size_t)(kBatchHead + 2 * max_lds_chunk) * sizeof(double); }

static const void* batch_kernel(int prec, int model) {
  if (prec == 0) {
    if (model == kLinear) return reinterpret_cast<const void*>(&k_batch<double, kLinear>);
    if (model == kNH) return reinterpret_cast<const void*>(&k_batch<double, kNH>);
    if (model == kSVK) return reinterpret_cast<const void*>(&k_batch<double, kSVK>);
    return reinterpret_cast<const void*>(&k_batch<double, kYeoh>);
  }
  if (model == kLinear) return reinterpret_cast<const void*>(&k_batch<float, kLinear>);
  if (model == kNH) return reinterpret_cast<const void*>(&k_batch<float, kNH>);
  if (model == kSVK) return reinterpret_cast<const void*>(&k_batch<float, kSVK>);
  return reinterpret_cast<const void*>(&k_batch<float, kYeoh>);
}

hipError_t launch_batch(BatchInst* tab, const int* ids, int count, int model, const KrylovCfg& cfg, double dt,
                        int n_steps, int max_lds_chunk, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const void* fn = batch_kernel(cfg.prec, model);
  const size_t lds = batch_lds_bytes(max_lds_chunk);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  KrylovCfg c = cfg;
  double d = dt;
  int n = n_steps;
  int ls = 2 * max_lds_chunk;
  void* args[] = {&tab, &ids, &c, &d, &n, &ls};
  return hipLaunchKernel(fn, dim3(count), dim3(kThreads), args, lds, st);
}

}  // namespace ep
