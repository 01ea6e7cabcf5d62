// Batched instances (many independent meshes / materials / loads).  A workgroup either
// steps a list of instances one after the other (their Krylov reductions never leave the
// workgroup), or is one member of a team of workgroups that steps one large instance
// together (the data-as-flag team of the single-instance kernel, with its bounded waits).
// The host plans the assignment so that the launch's longest workgroup is as short as the
// compute units allow.  The stepping state lives in device records and one launch advances
// every instance by one step, which makes the launch replayable from a captured graph.
#include "ep_kernels.hpp"
#include "ep_krylov.hpp"

namespace ep {

// u = M^{-1/2} ubar, each team member its share, then a team barrier
template <class Team>
__device__ void team_get_u(Team& tm, const Mesh& M, const double* S, double* u, int* flag) {
  for (int d = tm.rank * blockDim.x + threadIdx.x; d < M.n3; d += tm.G * blockDim.x) u[d] = M.mih[d] * S[d];
  tm.sync(flag);
}

static __device__ __forceinline__ int free_slot(int a, int b) {
  for (int s = 0; s < 3; ++s)
    if (s != a && s != b) return s;
  return 0;
}

// One step of one instance (Sec. 4.1-4.2); returns false after a sticky error.  B (the
// instance record) and a (the projection arguments) live in LDS: thread 0 writes them, a
// workgroup barrier publishes them, every lane reads them (per-lane copies of these records
// would live in scratch memory).
template <typename T, int MODEL, class Team>
__device__ bool device_step(Team& tm, BatchInst& B, ExpvArgs& a, const KrylovCfg& cfg, double dt, double* lw,
                            double* lv, double* red, double* yb, int* flag, const KLds& X) {
  const bool w0 = threadIdx.x == 0;
  const double t = B.t;
  const int n3 = B.M.n3;
  if (w0) {
    a.M = B.M;
    a.W = B.W;
    a.cfg = cfg;
    a.log_idx = (int)(B.step_idx % kLogSteps);
  }
  if (MODEL == kLinear) {
    if (w0) {
      a.op = OpArgs{};
      a.op.tau = dt;
      a.op.t_eval = t + 0.5 * dt;
      a.op.nsets = 0;
      a.kind = 0;
      a.x_in = B.S;
      a.x_out = B.S;
      a.out_mode = 0;
    }
    __syncthreads();
    expv_body<T, MODEL, Team, 0, 2, 8, kLBBatch, 1>(tm, a, lw, lv, red, yb, flag, X);
  } else {
    const int nhist = B.nhist, hnew = B.hist_new, hold = B.hist_old;
    int reserve = -1;
    if (nhist == 0) {
      reserve = free_slot(hnew, hold);
      team_get_u(tm, B.M, B.S, B.hist + (size_t)reserve * n3, flag);
    }
    const int snew = free_slot(hnew, reserve >= 0 ? reserve : hold);
    if (w0) {
      OpArgs pred{};
      pred.tau = 0.5 * dt;
      pred.t_eval = t + 0.25 * dt;
      if (nhist == 0) {
        pred.nsets = 1;
        pred.ulin[0] = B.hist + (size_t)reserve * n3;
        pred.wts[0] = 1.0;
      } else if (nhist == 1) {
        pred.nsets = 1;
        pred.ulin[0] = B.hist + (size_t)hnew * n3;
        pred.wts[0] = 1.0;
      } else {
        pred.nsets = 2;
        pred.ulin[0] = B.hist + (size_t)hnew * n3;
        pred.wts[0] = 1.75;
        pred.ulin[1] = B.hist + (size_t)hold * n3;
        pred.wts[1] = -0.75;
      }
      a.op = pred;
      a.kind = 1;
      a.x_in = B.S;
      a.x_out = B.hist + (size_t)snew * n3;
      a.out_mode = 1;
    }
    __syncthreads();
    expv_body<T, MODEL, Team, 0, 2, 8, kLBBatch, 1>(tm, a, lw, lv, red, yb, flag, X);
    if (tm.dead || read_err(&B.W.ctrl->err) != 0) return false;
    __syncthreads();                             // every lane is done reading a
    if (w0) {
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
    }
    __syncthreads();
    expv_body<T, MODEL, Team, 0, 2, 8, kLBBatch, 1>(tm, a, lw, lv, red, yb, flag, X);
    __syncthreads();                             // every lane is done reading B and a
    if (w0) {
      if (nhist == 0) {
        B.hist_old = -1;
        B.hist_new = snew;
        B.nhist = 1;
      } else {
        B.hist_old = hnew;
        B.hist_new = snew;
        B.nhist = 2;
      }
    }
  }
  const bool failed = tm.dead || read_err(&B.W.ctrl->err) != 0;
  __syncthreads();
  if (failed) return false;
  if (w0) {
    B.t = t + dt;
    B.step_idx += 1;
  }
  __syncthreads();
  return true;
}

// doubles of LDS before the slice buffers: red[32] | yb[kMaxM] | ints flag[16], 16 unused
constexpr int kBatchHead = 32 + kMaxM + 16;

// Steps of instance id by this workgroup (team tm), with B and a the workgroup's LDS copies
// of its record and projection arguments.  Rank 0's lane 0 writes the stepping state back
// and adds the steps' wall-clock ticks to the instance's control block.
template <typename T, int MODEL, class Team>
__device__ void run_instance(Team& tm, BatchInst* tab, int id, BatchInst& B, ExpvArgs& a, const KrylovCfg& cfg,
                             double dt, int n_steps, double* lds, int lds_slices, int* flag) {
  double* red = lds;
  double* yb = lds + 32;
  // the slice region (lds_slices doubles) doubles as expm scratch: the sequential form
  // reloads both slice buffers after a check point
  const KLds X{nullptr, nullptr, nullptr, nullptr, lds + kBatchHead, lds_slices, true};
  if (threadIdx.x == 0) {
    *flag = 1;
    B = tab[id];
  }
  __syncthreads();
  // slices: both in LDS (use_lds 1), w's in LDS and the newest basis vector read back from V
  // (2), or w's in device memory and the basis vector from V (0)
  double* lw;
  double* lv = nullptr;
  if (B.use_lds == 1) {
    lw = lds + kBatchHead;
    lv = lw + B.W.chunk;
  } else if (B.use_lds == 2) {
    lw = lds + kBatchHead;
  } else {
    lw = B.W.wscr + (size_t)tm.rank * B.W.chunk;
  }
  const unsigned long long t0 = wall_clock64();
  int s = 0;
  for (; s < n_steps; ++s)
    if (!device_step<T, MODEL>(tm, B, a, cfg, dt, lw, lv, red, yb, flag, X)) break;
  if (tm.rank == 0 && threadIdx.x == 0) {
    tab[id].t = B.t;
    tab[id].step_idx = B.step_idx;
    tab[id].nhist = B.nhist;
    tab[id].hist_new = B.hist_new;
    tab[id].hist_old = B.hist_old;
    B.W.ctrl->ticks += wall_clock64() - t0;
    B.W.ctrl->ticked_steps += s;
  }
  __syncthreads();                               // B is rewritten for the next instance
}

template <typename T, int MODEL>
__global__ __launch_bounds__(kThreads) void k_batch(BatchInst* tab, const BatchWork* work, const int* ids,
                                                    KrylovCfg cfg, double dt, int n_steps, int lds_slices) {
  extern __shared__ double lds[];
  int* flag = (int*)(lds + 32 + kMaxM);
  // the instance record and the projection arguments: one copy per workgroup in LDS
  __shared__ BatchInst B;
  __shared__ ExpvArgs a;
  const BatchWork wk = work[blockIdx.x];
  if (wk.G > 1) {
    // one member of a team (flags and ring emptied by k_prep_batch_teams before the launch)
    const KWork& W = tab[wk.inst].W;
    GridTeam tm{wk.G, wk.rank, W.flags, W.ring, &W.ctrl->err, 0ull, 0u, false, 0u, nullptr, 0, 0u};
    run_instance<T, MODEL>(tm, tab, wk.inst, B, a, cfg, dt, n_steps, lds, lds_slices, flag);
  } else {
    for (int q = 0; q < wk.count; ++q) {
      BlockTeam tm;
      run_instance<T, MODEL>(tm, tab, ids[wk.first + q], B, a, cfg, dt, n_steps, lds, lds_slices, flag);
    }
  }
}

// Barrier flags to zero and all-reduce rings to empty for every team of the launch (one
// workgroup per work item; only rank 0's item does the team's).
__global__ void k_prep_batch_teams(BatchInst* tab, const BatchWork* work) {
  const BatchWork wk = work[blockIdx.x];
  if (wk.G <= 1 || wk.rank != 0) return;
  const KWork& W = tab[wk.inst].W;
  for (int i = threadIdx.x; i < kRing * wk.G; i += blockDim.x) {
    if (i < wk.G) W.flags[i] = 0ull;
    W.ring[i] = kEmpty;
  }
}

// dynamic LDS of the batch kernel (its static LDS, the record and arguments, comes on top:
// sizeof(BatchInst) + sizeof(ExpvArgs) = 864 bytes, within the 160 KB beside the largest
// dynamic part, 2 * 9984 + 304 doubles)
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

hipError_t launch_batch(BatchInst* tab, const BatchWork* work, const int* ids, int n_work, bool teams, int model,
                        const KrylovCfg& cfg, double dt, int n_steps, int max_lds_chunk, hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  if (teams) k_prep_batch_teams<<<n_work, 64, 0, st>>>(tab, work);
  const void* fn = batch_kernel(cfg.prec, model);
  const size_t lds = batch_lds_bytes(max_lds_chunk);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  KrylovCfg c = cfg;
  double d = dt;
  int n = n_steps;
  int ls = 2 * max_lds_chunk;
  void* args[] = {&tab, &work, &ids, &c, &d, &n, &ls};
  return hipLaunchKernel(fn, dim3(n_work), dim3(kThreads), args, lds, st);
}

hipError_t batch_max_blocks(int prec, int model, int max_lds_chunk, int* blocks_per_cu) {
  const void* fn = batch_kernel(prec, model);
  const size_t lds = batch_lds_bytes(max_lds_chunk);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, kThreads, lds);
}

}  // namespace ep
