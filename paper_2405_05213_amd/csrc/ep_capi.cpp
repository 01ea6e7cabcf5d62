// Host runtime and C ABI of the exponential propagator (see include/ep.h).
// Owns argument validation, the workspace layout in the caller's device buffer, integer
// bookkeeping of the mesh (node -> element-slot and node -> face-slot incidence), launch
// sizing of the persistent kernels and the step sequencing of the predictor-corrector.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ep.h"
#include "ep_common.hpp"
#include "ep_kernels.hpp"

using namespace ep;

namespace {

constexpr size_t kAlign = 256;
constexpr long long kMaxChunk = 9984;     // (2 * 9984 + 304) doubles of LDS fit in 160 KB
constexpr long long kLdsBytes = 160 * 1024;

struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    const size_t o = off;
    off += bytes;
    return o;
  }
};

// host description + device view of one instance
struct Inst {
  // inputs
  int64_t n_nodes = 0, n_elems = 0;
  int npe = 8;                  // nodes per element: 8 (hex8) or 27 (quadratic hexahedron)
  int nfn = 4;                  // nodes per loaded face: 4 or 9
  std::vector<double> xyz;
  std::vector<int32_t> conn;
  int model = -1;
  double mp[4] = {0, 0, 0, 0};
  double rho = 0.0;
  std::vector<int32_t> clamped;
  std::vector<int32_t> faces;
  double t0[3] = {0, 0, 0};
  std::vector<double> knots;   // times then scales
  int n_knots = 0;
  // derived
  std::vector<int32_t> inc_ptr, inc, finc_ptr, finc;
  std::vector<unsigned char> clamp_mask;
  int n3 = 0, L = 0, Lp = 0;
  // workspace offsets
  size_t o_xyz, o_conn, o_incp, o_inc, o_geo, o_geo32, o_vdet, o_mih, o_mh, o_p0, o_p0bar, o_faces, o_fincp,
      o_finc, o_ff, o_knots, o_clamp, o_S, o_X, o_Wun, o_V, o_F, o_F32, o_hist, o_stage, o_slots, o_H, o_Escr, o_y, o_ke,
      o_stencil,
      o_ctrl, o_log, o_pe, o_pv, o_eout, o_flags, o_wscr, o_psi, o_kst, o_F2, o_F2_32, o_Sprev;
  Mesh M{};
  bool kst_rest = false;       // the stored tangents are those of the rest-state operator
  KWork W{};
  // stepping state (host mirror)
  double t = 0.0;
  int64_t step_idx = 0;
  int hist_new = -1, hist_old = -1;
  int nhist = 0;
  bool state_set = false;
  bool s0_pending = false;      // scaled s0: resolved at the next step (needs dt)
  bool m4_prev = false;         // fourth-order scheme: the previous step's start state is in o_Sprev
  double t_prev = 0.0;
};

}  // namespace

struct ep_ctx {
  int device = -1;
  hipStream_t stream = nullptr;
  std::string err;
  bool bound = false;
  bool batch = false;
  bool mesh_set = false, material_set = false;
  Inst one;
  std::vector<Inst> insts;
  KrylovCfg cfg{1e-10, 64, 4, 0, 0, 64, 0, 0};
  int ortho_user = -1;                  // -1: automatic
  double s0_user = -1.0;
  int G_user = 0;
  int cus = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t o_batch_tab = 0;
  // batch
  std::vector<BatchInst> btab;          // host mirror of the device records
  std::vector<int> bids[kModels];       // instance ids per material model (packed lists of the plan)
  size_t o_bids[kModels] = {};
  std::vector<BatchWork> bwork[kModels];  // the launch plan: one record per workgroup
  size_t o_bwork[kModels] = {};
  size_t bwork_cap = 0;
  int bteam_max = 1;                    // largest team of the current plan
  int max_lds_chunk = 0;
  hipGraphExec_t bgraph = nullptr;
  hipGraph_t bgraph_src = nullptr;
  double bgraph_dt = 0.0;
  ~ep_ctx() {
    if (bgraph) (void)hipGraphExecDestroy(bgraph);
    if (bgraph_src) (void)hipGraphDestroy(bgraph_src);
  }
};

static ep_status fail(ep_ctx* c, ep_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define EP_HIP(c, call)                                                                      \
  do {                                                                                       \
    hipError_t _e = (call);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return fail((c), EP_ERR_HIP, std::string(#call " failed: ") + hipGetErrorString(_e));  \
  } while (0)

static bool is_gpu(const ep_ctx* c) { return c->device >= 0; }

// ------------------------------------------------------------------------------ validation
static ep_status check_mesh(ep_ctx* c, int64_t n_nodes, const double* xyz, int64_t n_elems, const int32_t* conn,
                            int npe = 8) {
  if (n_nodes <= 0 || n_elems <= 0) return fail(c, EP_ERR_ARG, "mesh needs n_nodes > 0 and n_elems > 0");
  if (!xyz || !conn) return fail(c, EP_ERR_ARG, "null mesh array");
  if (n_nodes > (1LL << 28) || n_elems > (1LL << 27)) return fail(c, EP_ERR_ARG, "mesh too large for 32-bit indexing");
  for (int64_t i = 0; i < 3 * n_nodes; ++i)
    if (!std::isfinite(xyz[i])) return fail(c, EP_ERR_ARG, "non-finite node coordinate");
  for (int64_t i = 0; i < npe * n_elems; ++i)
    if (conn[i] < 0 || conn[i] >= n_nodes) return fail(c, EP_ERR_ARG, "connectivity entry out of range");
  return EP_OK;
}

static ep_status check_material(ep_ctx* c, int model, const double* p, int n, double rho) {
  if (!p) return fail(c, EP_ERR_ARG, "null material parameters");
  if (!(rho > 0.0) || !std::isfinite(rho)) return fail(c, EP_ERR_ARG, "density must be positive");
  if (model == EP_LINEAR) {
    if (n != 2) return fail(c, EP_ERR_ARG, "EP_LINEAR takes {E, nu}");
    if (!(p[0] > 0.0) || !(p[1] > -1.0 && p[1] < 0.5)) return fail(c, EP_ERR_ARG, "need E > 0 and -1 < nu < 0.5");
  } else if (model == EP_NH) {
    if (n != 2) return fail(c, EP_ERR_ARG, "EP_NH takes {mu, lambda}");
    if (!(p[0] > 0.0) || !(p[1] >= 0.0)) return fail(c, EP_ERR_ARG, "need mu > 0 and lambda >= 0");
  } else if (model == EP_YEOH) {
    if (n != 4) return fail(c, EP_ERR_ARG, "EP_YEOH takes {C10, C20, C30, D1}");
    if (!(p[0] > 0.0) || !(p[3] > 0.0)) return fail(c, EP_ERR_ARG, "need C10 > 0 and D1 > 0");
  } else if (model == EP_SVK) {
    if (n != 2) return fail(c, EP_ERR_ARG, "EP_SVK takes {lambda, mu}");
    if (!(p[1] > 0.0) || !(p[0] >= 0.0)) return fail(c, EP_ERR_ARG, "need mu > 0 and lambda >= 0");
  } else {
    return fail(c, EP_ERR_ARG, "unknown material model");
  }
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return fail(c, EP_ERR_ARG, "non-finite material parameter");
  return EP_OK;
}

static ep_status check_traction(ep_ctx* c, int64_t n_nodes, int64_t n_faces, const int32_t* fn, const double* t0,
                                int64_t n_knots, const double* kt, const double* ks, int nfn = 4) {
  if (n_faces < 0 || n_knots < 0) return fail(c, EP_ERR_ARG, "negative count");
  if (n_faces > 0 && (!fn || !t0)) return fail(c, EP_ERR_ARG, "null face array or traction");
  for (int64_t i = 0; i < nfn * n_faces; ++i)
    if (fn[i] < 0 || fn[i] >= n_nodes) return fail(c, EP_ERR_ARG, "face node out of range");
  if (n_faces > 0)
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(t0[i])) return fail(c, EP_ERR_ARG, "non-finite traction");
  if (n_knots > kMaxKnots) return fail(c, EP_ERR_ARG, "too many load knots");
  if (n_knots > 0 && (!kt || !ks)) return fail(c, EP_ERR_ARG, "null load table");
  for (int64_t i = 0; i < n_knots; ++i) {
    if (!std::isfinite(kt[i]) || !std::isfinite(ks[i])) return fail(c, EP_ERR_ARG, "non-finite load table");
    if (i > 0 && !(kt[i] > kt[i - 1])) return fail(c, EP_ERR_ARG, "load knot times must be ascending");
  }
  return EP_OK;
}

static void fill_mesh(Inst& I, int64_t n_nodes, const double* xyz, int64_t n_elems, const int32_t* conn,
                      int npe = 8) {
  I.n_nodes = n_nodes;
  I.n_elems = n_elems;
  I.npe = npe;
  I.nfn = npe == 27 ? 9 : 4;
  I.xyz.assign(xyz, xyz + 3 * n_nodes);
  I.conn.assign(conn, conn + (size_t)npe * n_elems);
  I.n3 = (int)(3 * n_nodes);
  I.L = 2 * I.n3 + 1;
  I.Lp = (I.L + 63) / 64 * 64;
}

static void fill_traction(Inst& I, int64_t n_faces, const int32_t* fn, const double* t0, int64_t n_knots,
                          const double* kt, const double* ks) {
  I.faces.assign(fn ? fn : (const int32_t*)nullptr, fn ? fn + (size_t)I.nfn * n_faces : (const int32_t*)nullptr);
  for (int i = 0; i < 3; ++i) I.t0[i] = (n_faces > 0 && t0) ? t0[i] : 0.0;
  I.n_knots = (int)n_knots;
  I.knots.assign(2 * n_knots, 0.0);
  for (int64_t i = 0; i < n_knots; ++i) {
    I.knots[i] = kt[i];
    I.knots[n_knots + i] = ks[i];
  }
}

// ------------------------------------------------------------------------------ layout
// Orthogonalisation form of the single-instance kernel: compact WY (one vector reduction
// per Arnoldi step) unless asked otherwise or the subspace exceeds its LDS triangle.
static int eff_ortho(const ep_ctx* c) {
  if (c->batch) return 0;
  if (c->ortho_user >= 0) return c->ortho_user;
  return c->cfg.m_max <= kMaxCwyM ? 1 : 0;
}

// Largest Krylov-vector slice per workgroup: two slices of it share the LDS with the
// reduction scratch (and T of the compact-WY form).
static long long max_chunk(const ep_ctx* c) {
  const long long fixed = (long long)expv_lds_head_bytes(c->cfg.ortho, c->cfg.m_max);
  return std::max(0LL, (kLdsBytes - fixed) / 16 / 64 * 64);
}

// Slice size for a team of G, and whether the slices fit in LDS (sg = 0) or must live in
// device memory (sg = 1: meshes beyond max_chunk entries per workgroup on every CU).
static int chunk_of(const ep_ctx* c, const Inst& I, int G, int* sg) {
  int C = (I.Lp + G - 1) / G;
  C = (C + 63) / 64 * 64;
  *sg = C > std::max(64LL, max_chunk(c)) ? 1 : 0;
  return C;
}

static int pick_G(const ep_ctx* c, const Inst& I, int* chunk, int* sg) {
  const int maxG = std::max(1, c->cus);
  // the workgroup's slice of the Arnoldi vector (and of the newest basis vector) lives in
  // LDS when it has at most max_chunk entries; teams grow up to one workgroup per CU for that
  const long long mc = std::max(64LL, max_chunk(c));
  const int Gmin = (int)std::min<long long>(maxG, (I.Lp + mc - 1) / mc);
  int G = c->G_user > 0 ? c->G_user : (int)std::min<long long>(maxG, std::max<long long>(1, (I.Lp + 2047) / 2048));
  if (c->G_user <= 0) G = std::max(G, Gmin);
  G = std::max(1, std::min(G, std::min(I.Lp / 64 > 0 ? I.Lp / 64 : 1, 1024)));
  *chunk = chunk_of(c, I, G, sg);
  return G;
}

static void plan_inst(const ep_ctx* c, Inst& I, Layout& L, int Gmax) {
  const size_t n3 = I.n3, ne = I.n_elems, nn = I.n_nodes, nf = I.faces.size() / I.nfn;
  const size_t npe = I.npe, nfn = I.nfn;
  const size_t Lp = I.Lp, mm = c->cfg.m_max;
  I.o_xyz = L.take(8 * 3 * nn);
  I.o_conn = L.take(4 * npe * ne);
  I.o_incp = L.take(4 * (nn + 1));
  I.o_inc = L.take(4 * npe * ne);
  I.o_geo = L.take(8 * 10 * npe * ne);      // J^{-1}, w det J at the npe Gauss points
  I.o_geo32 = L.take(4 * 10 * npe * ne);
  I.o_vdet = L.take(8 * npe * ne);
  I.o_mih = L.take(8 * n3);
  I.o_mh = L.take(8 * n3);
  I.o_p0 = L.take(8 * n3);
  I.o_p0bar = L.take(8 * n3);
  I.o_faces = L.take(4 * nfn * std::max<size_t>(nf, 1));
  I.o_fincp = L.take(4 * (nn + 1));
  I.o_finc = L.take(4 * nfn * std::max<size_t>(nf, 1));
  I.o_ff = L.take(8 * 3 * nfn * std::max<size_t>(nf, 1));
  I.o_knots = L.take(8 * std::max<size_t>(I.knots.size(), 2));
  I.o_clamp = L.take(n3);
  I.o_S = L.take(8 * Lp);
  I.o_X = L.take(8 * Lp);
  I.o_Wun = L.take(8 * Lp);
  I.o_V = L.take(8 * Lp * (mm + 1));
  I.o_F = L.take(8 * 3 * npe * ne);
  I.o_F32 = L.take(4 * 3 * npe * ne);
  I.o_hist = L.take(8 * 3 * n3);
  I.o_stage = L.take(8 * 2 * n3);
  // G barrier flags + 8 G ring slots (+ 8 G vector slots of 2 m_max values)
  const size_t vw = c->cfg.ortho == 1 ? 2 * mm : 0;
  I.o_slots = L.take(8 * (1 + kRing + kRing * vw) * (size_t)std::max(Gmax, 1));
  I.o_H = L.take(8 * (mm + 1) * mm);
  I.o_Escr = L.take(8 * 9 * mm * mm);     // 8 m^2 expm work + m^2 output staging
  I.o_y = L.take(8 * (mm + 1));
  I.o_ctrl = L.take(sizeof(Ctrl));
  I.o_log = L.take(sizeof(StepLog));
  I.o_pe = L.take(8 * ((ne + 255) / 256 + 1));
  I.o_pv = L.take(8 * 2 * ((n3 + 255) / 256 + 1));
  I.o_eout = L.take(8 * 4);
  I.o_flags = L.take(4 * 4);
  I.o_wscr = L.take(8 * 2 * Lp);
  I.o_ke = L.take(8 * 24 * kKeLd);
  I.o_stencil = L.take(8 * 27 * 9);
  I.o_psi = L.take(2 * (size_t)kPsiValues);
  I.o_kst = L.take(c->cfg.prec == 2 ? 2 * kst_values((long long)ne) : 0);
  const bool m4 = c->cfg.scheme == 4;
  I.o_F2 = L.take(m4 ? 8 * 24 * ne : 0);
  I.o_F2_32 = L.take(m4 ? 4 * 24 * ne : 0);
  I.o_Sprev = L.take(m4 ? 8 * 2 * n3 : 0);
}

static int Gmax_of(const ep_ctx* c) { return std::max(1, std::max(c->cus, c->G_user)); }

static size_t plan_all(ep_ctx* c) {
  Layout L;
  const int Gmax = Gmax_of(c);
  if (!c->batch) {
    plan_inst(c, c->one, L, Gmax);
  } else {
    for (auto& I : c->insts) plan_inst(c, I, L, kBatchGmax);
    c->o_batch_tab = L.take(sizeof(BatchInst) * std::max<size_t>(c->insts.size(), 1));
    for (int k = 0; k < kModels; ++k) c->o_bids[k] = L.take(4 * std::max<size_t>(c->insts.size(), 1));
    c->bwork_cap = std::max<size_t>(c->insts.size(), 4 * (size_t)std::max(c->cus, 1)) + 1;
    for (int k = 0; k < kModels; ++k) c->o_bwork[k] = L.take(sizeof(BatchWork) * c->bwork_cap);
  }
  return L.off + kAlign;
}

// incidence lists (integer bookkeeping)
static void build_incidence(Inst& I) {
  const int64_t nn = I.n_nodes, ne = I.n_elems;
  const int npe = I.npe;
  I.inc_ptr.assign(nn + 1, 0);
  for (int64_t e = 0; e < ne; ++e)
    for (int a = 0; a < npe; ++a) I.inc_ptr[I.conn[e * npe + a] + 1]++;
  for (int64_t n = 0; n < nn; ++n) I.inc_ptr[n + 1] += I.inc_ptr[n];
  I.inc.assign(npe * ne, 0);
  std::vector<int32_t> pos(I.inc_ptr.begin(), I.inc_ptr.end() - 1);
  for (int a = 0; a < npe; ++a)        // slot-major order: a outer, e inner
    for (int64_t e = 0; e < ne; ++e) I.inc[pos[I.conn[e * npe + a]]++] = (int32_t)(a * ne + e);
  const int nfn = I.nfn;
  const int64_t nf = I.faces.size() / nfn;
  I.finc_ptr.assign(nn + 1, 0);
  for (int64_t f = 0; f < nf; ++f)
    for (int b = 0; b < nfn; ++b) I.finc_ptr[I.faces[f * nfn + b] + 1]++;
  for (int64_t n = 0; n < nn; ++n) I.finc_ptr[n + 1] += I.finc_ptr[n];
  I.finc.assign(std::max<int64_t>(nfn * nf, 1), 0);
  std::vector<int32_t> fp(I.finc_ptr.begin(), I.finc_ptr.end() - 1);
  for (int64_t f = 0; f < nf; ++f)
    for (int b = 0; b < nfn; ++b) I.finc[fp[I.faces[f * nfn + b]]++] = (int32_t)(f * nfn + b);
  I.clamp_mask.assign(I.n3, 0);
  for (int32_t d : I.clamped) I.clamp_mask[d] = 1;
}

template <typename P>
static P* dptr(ep_ctx* c, size_t off) {
  return reinterpret_cast<P*>(c->ws + off);
}

static double auto_s0(const ep_ctx* c, const Inst& I) {
  if (c->s0_user >= 0.0) return c->s0_user;
  bool load = !I.faces.empty() && (I.t0[0] != 0.0 || I.t0[1] != 0.0 || I.t0[2] != 0.0);
  bool nonzero_scale = false;
  for (int i = 0; i < I.n_knots; ++i) nonzero_scale |= I.knots[I.n_knots + i] != 0.0;
  return (load && nonzero_scale) ? 1.0 : 0.0;
}

// Scaled augmented entry (ep_set_krylov with s0 = EP_S0_SCALED): the augmented entry of wbar is
// taken at the problem's own scale, s0 = max(||[ubar; vbar]||_2, dt ||Pbar_0||_2 max_k |scale_k|),
// fixed at the first step after a state is set (when dt is known).  The exact propagation does
// not depend on s0; the stopping rule eps <= tol ||wbar|| does, and with s0 = 1 it is loose
// for states far smaller than one in SI units.  Stays 0 without a load.
static bool scaled_s0_mode(const ep_ctx* c) { return c->s0_user == EP_S0_SCALED; }

static ep_status resolve_s0(ep_ctx* c, Inst& I, double dt) {
  if (!I.s0_pending) return EP_OK;
  I.s0_pending = false;
  if (I.M.s0 == 0.0) return EP_OK;              // unloaded: the 2N form
  std::vector<double> w(2 * (size_t)I.n3), pb((size_t)I.n3);
  EP_HIP(c, hipStreamSynchronize(c->stream));
  EP_HIP(c, hipMemcpy(w.data(), dptr<double>(c, I.o_S), 8 * w.size(), hipMemcpyDeviceToHost));
  EP_HIP(c, hipMemcpy(pb.data(), I.M.p0bar, 8 * pb.size(), hipMemcpyDeviceToHost));
  double nw = 0.0, np = 0.0, smax = 0.0;
  for (double x : w) nw += x * x;
  for (double x : pb) np += x * x;
  for (int i = 0; i < I.n_knots; ++i) smax = std::max(smax, std::fabs(I.knots[I.n_knots + i]));
  const double s0 = std::max(std::sqrt(nw), dt * std::sqrt(np) * smax);
  if (!(s0 > 0.0) || !std::isfinite(s0)) return EP_OK;
  I.M.s0 = s0;
  I.M.s_inv = 1.0 / s0;
  EP_HIP(c, hipMemcpy(dptr<double>(c, I.o_S) + 2 * (size_t)I.n3, &s0, 8, hipMemcpyHostToDevice));
  return EP_OK;
}

// A structured box: node (i, j, k) = i + (nx+1)(j + (ny+1)k), elements in i-fastest order
// with VTK corner order.  Read off element 0 and verified on every element.
static bool lattice_dims(const Inst& I, int lat[3]) {
  if (I.n_elems < 1 || I.npe != 8) return false;
  const int32_t* c0 = I.conn.data();
  const int64_t sx = c0[3] - c0[0], sxy = c0[4] - c0[0];
  if (c0[0] != 0 || c0[1] != 1 || sx < 2 || sxy % sx != 0) return false;
  const int64_t nx = sx - 1, ny = sxy / sx - 1;
  if (ny < 1 || I.n_elems % (nx * ny) != 0) return false;
  const int64_t nz = I.n_elems / (nx * ny);
  if ((nx + 1) * (ny + 1) * (nz + 1) != I.n_nodes) return false;
  static const int di[8] = {0, 1, 1, 0, 0, 1, 1, 0}, dj[8] = {0, 0, 1, 1, 0, 0, 1, 1}, dk[8] = {0, 0, 0, 0, 1, 1, 1, 1};
  for (int64_t e = 0; e < I.n_elems; ++e) {
    const int64_t i = e % nx, j = (e / nx) % ny, k = e / (nx * ny);
    for (int a = 0; a < 8; ++a) {
      const int64_t n = (i + di[a]) + (nx + 1) * ((j + dj[a]) + (ny + 1) * (k + dk[a]));
      if (I.conn[(size_t)e * 8 + a] != n) return false;
    }
  }
  lat[0] = (int)nx;
  lat[1] = (int)ny;
  lat[2] = (int)nz;
  return true;
}

// Tolerance of the congruence test: 1e-13, or 32 eps R / h when larger, R the largest node
// coordinate magnitude and h the mean element size (cube root of the bounding-box volume per
// element): the rounding of the coordinates themselves leaves relative differences of about
// eps R / h between the edges of otherwise identical elements.
static double congruence_tol(const Inst& I) {
  if (I.n_nodes < 1 || I.n_elems < 1) return 1e-13;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, R = 0.0;
  for (int64_t n = 0; n < I.n_nodes; ++n)
    for (int d = 0; d < 3; ++d) {
      const double x = I.xyz[(size_t)n * 3 + d];
      lo[d] = std::min(lo[d], x);
      hi[d] = std::max(hi[d], x);
      R = std::max(R, std::fabs(x));
    }
  const double vol = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
  if (!(vol > 0.0)) return 1e-13;
  const double h = std::cbrt(vol / (double)I.n_elems);
  return std::max(1e-13, 32.0 * 2.220446049250313e-16 * R / h);
}

static ep_status setup_inst(ep_ctx* c, Inst& I, int G, int chunk, int Gslots) {
  hipStream_t st = c->stream;
  build_incidence(I);
  const size_t nf = I.faces.size() / I.nfn;
  EP_HIP(c, hipMemcpyAsync(dptr<char>(c, I.o_xyz), I.xyz.data(), 8 * I.xyz.size(), hipMemcpyHostToDevice, st));
  EP_HIP(c, hipMemcpyAsync(dptr<char>(c, I.o_conn), I.conn.data(), 4 * I.conn.size(), hipMemcpyHostToDevice, st));
  EP_HIP(c, hipMemcpyAsync(dptr<char>(c, I.o_incp), I.inc_ptr.data(), 4 * I.inc_ptr.size(), hipMemcpyHostToDevice, st));
  EP_HIP(c, hipMemcpyAsync(dptr<char>(c, I.o_inc), I.inc.data(), 4 * I.inc.size(), hipMemcpyHostToDevice, st));
  EP_HIP(c, hipMemcpyAsync(dptr<char>(c, I.o_fincp), I.finc_ptr.data(), 4 * I.finc_ptr.size(), hipMemcpyHostToDevice, st));
  EP_HIP(c, hipMemcpyAsync(dptr<char>(c, I.o_finc), I.finc.data(), 4 * I.finc.size(), hipMemcpyHostToDevice, st));
  if (nf > 0)
    EP_HIP(c, hipMemcpyAsync(dptr<char>(c, I.o_faces), I.faces.data(), 4 * I.faces.size(), hipMemcpyHostToDevice, st));
  if (!I.knots.empty())
    EP_HIP(c, hipMemcpyAsync(dptr<char>(c, I.o_knots), I.knots.data(), 8 * I.knots.size(), hipMemcpyHostToDevice, st));
  EP_HIP(c, hipMemcpyAsync(dptr<char>(c, I.o_clamp), I.clamp_mask.data(), I.clamp_mask.size(), hipMemcpyHostToDevice, st));
  EP_HIP(c, hipMemsetAsync(dptr<char>(c, I.o_flags), 0, 16, st));
  EP_HIP(c, hipMemsetAsync(dptr<char>(c, I.o_S), 0, 8 * (size_t)I.Lp, st));
  EP_HIP(c, hipMemsetAsync(dptr<char>(c, I.o_X), 0, 8 * (size_t)I.Lp, st));
  EP_HIP(c, hipMemsetAsync(dptr<char>(c, I.o_Wun), 0, 8 * (size_t)I.Lp, st));
  EP_HIP(c, hipMemsetAsync(dptr<char>(c, I.o_hist), 0, 8 * 3 * (size_t)I.n3, st));
  EP_HIP(c, hipMemsetAsync(dptr<char>(c, I.o_log), 0, sizeof(StepLog), st));
  EP_HIP(c, hipMemsetAsync(dptr<char>(c, I.o_H), 0, 8 * (size_t)(c->cfg.m_max + 1) * c->cfg.m_max, st));
  int* flags = dptr<int>(c, I.o_flags);
  launch_geometry(dptr<double>(c, I.o_xyz), dptr<int>(c, I.o_conn), (int)I.n_elems, I.npe, dptr<double>(c, I.o_geo),
                  dptr<float>(c, I.o_geo32), dptr<double>(c, I.o_vdet), flags + 0, st);
  launch_congruence(dptr<double>(c, I.o_geo), (int)I.n_elems, I.npe, congruence_tol(I), flags + 1, st);
  EP_HIP(c, hipGetLastError());
  launch_mass((int)I.n_nodes, (int)I.n_elems, I.npe, dptr<int>(c, I.o_incp), dptr<int>(c, I.o_inc),
              dptr<double>(c, I.o_vdet), I.rho, dptr<unsigned char>(c, I.o_clamp), dptr<double>(c, I.o_mih),
              dptr<double>(c, I.o_mh), st);
  launch_faces(dptr<double>(c, I.o_xyz), dptr<int>(c, I.o_faces), (int)nf, I.nfn, I.t0, dptr<double>(c, I.o_ff),
               (int)I.n_nodes, dptr<int>(c, I.o_fincp), dptr<int>(c, I.o_finc), dptr<double>(c, I.o_mih),
               dptr<double>(c, I.o_p0), dptr<double>(c, I.o_p0bar), st);
  EP_HIP(c, hipGetLastError());
  int hflags[2] = {0, 0};
  EP_HIP(c, hipMemcpyAsync(hflags, flags, 8, hipMemcpyDeviceToHost, st));
  EP_HIP(c, hipStreamSynchronize(st));
  if (hflags[0]) return fail(c, EP_ERR_INVERTED, "inverted or degenerate reference element (det J <= 0)");
  Mesh& M = I.M;
  M.n_nodes = (int)I.n_nodes;
  M.n_elems = (int)I.n_elems;
  M.npe = I.npe;
  M.n3 = I.n3;
  M.L = I.L;
  M.Lp = I.Lp;
  M.conn = dptr<int>(c, I.o_conn);
  M.inc_ptr = dptr<int>(c, I.o_incp);
  M.inc = dptr<int>(c, I.o_inc);
  M.geo = dptr<double>(c, I.o_geo);
  M.geo32 = dptr<float>(c, I.o_geo32);
  M.congruent = hflags[1] ? 0 : 1;
  // an axis-aligned box element has a diagonal Jacobian; the 8-node sums leave rounding
  // residue of the order of 1e-17 relative off the diagonal, which the diagonal form drops
  M.jdiag = 0;
  if (M.congruent && I.npe == 8 && I.n_elems > 0) {
    double g[8 * 10];
    EP_HIP(c, hipMemcpy(g, M.geo, sizeof(g), hipMemcpyDeviceToHost));
    bool diag = true;
    for (int q = 0; q < 8; ++q) {
      const double dmax = std::max(std::fabs(g[q * 10]), std::max(std::fabs(g[q * 10 + 4]), std::fabs(g[q * 10 + 8])));
      for (int k = 0; k < 9; ++k)
        if (k % 4 != 0 && !(std::fabs(g[q * 10 + k]) <= 1e-12 * dmax)) diag = false;
    }
    M.jdiag = diag ? 1 : 0;
  }
  M.mih = dptr<double>(c, I.o_mih);
  M.mh = dptr<double>(c, I.o_mh);
  M.p0bar = dptr<double>(c, I.o_p0bar);
  M.p0 = dptr<double>(c, I.o_p0);
  M.knots = dptr<double>(c, I.o_knots);
  M.n_knots = I.n_knots;
  M.model = I.model;
  for (int i = 0; i < 4; ++i) M.mp[i] = I.mp[i];
  M.s0 = auto_s0(c, I);
  M.s_inv = M.s0 != 0.0 ? 1.0 / M.s0 : 0.0;
  M.ke = nullptr;
  M.lat[0] = M.lat[1] = M.lat[2] = 0;
  M.stencil = nullptr;
  if (M.congruent && I.n_elems > 0 && I.npe == 8) {
    launch_stiffness(M, dptr<double>(c, I.o_ke), st);
    EP_HIP(c, hipGetLastError());
    M.ke = dptr<double>(c, I.o_ke);
    int lat[3];
    if (lattice_dims(I, lat)) {
      launch_stencil_blocks(M.ke, dptr<double>(c, I.o_stencil), st);
      EP_HIP(c, hipGetLastError());
      for (int d = 0; d < 3; ++d) M.lat[d] = lat[d];
      M.stencil = dptr<double>(c, I.o_stencil);
    }
  }
  M.kst = nullptr;
  I.kst_rest = false;
  if (c->cfg.prec == 2) {
    if (!M.congruent)
      return fail(c, EP_ERR_ARG, "BF16 element tangents need a congruent mesh (every element a translate of element 0)");
    launch_psi(M, dptr<uint16_t>(c, I.o_psi), st);
    EP_HIP(c, hipGetLastError());
    M.kst = dptr<uint16_t>(c, I.o_kst);
  }
  KWork& W = I.W;
  W.V = dptr<double>(c, I.o_V);
  W.Wun = dptr<double>(c, I.o_Wun);
  W.X = dptr<double>(c, I.o_X);
  W.F = dptr<double>(c, I.o_F);
  W.F32 = dptr<float>(c, I.o_F32);
  W.F2 = c->cfg.scheme == 4 ? dptr<double>(c, I.o_F2) : nullptr;
  W.F2_32 = c->cfg.scheme == 4 ? dptr<float>(c, I.o_F2_32) : nullptr;
  W.flags = dptr<unsigned long long>(c, I.o_slots);
  W.ring = W.flags + std::max(Gslots, 1);
  W.vw = c->cfg.ortho == 1 ? 2 * c->cfg.m_max : 0;
  W.vring = W.vw > 0 ? W.ring + (size_t)kRing * std::max(Gslots, 1) : nullptr;
  W.H = dptr<double>(c, I.o_H);
  W.Escr = dptr<double>(c, I.o_Escr);
  W.y = dptr<double>(c, I.o_y);
  W.ctrl = dptr<Ctrl>(c, I.o_ctrl);
  W.log = dptr<StepLog>(c, I.o_log);
  W.G = G;
  W.chunk = chunk;
  W.wscr = dptr<double>(c, I.o_wscr);
  launch_reset_ctrl(W.ctrl, st);
  EP_HIP(c, hipGetLastError());
  EP_HIP(c, hipStreamSynchronize(st));
  return EP_OK;
}

static ep_status read_err(ep_ctx* c, Inst& I) {
  int e = 0;
  EP_HIP(c, hipMemcpyAsync(&e, &I.W.ctrl->err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  EP_HIP(c, hipStreamSynchronize(c->stream));
  if (e == 0) return EP_OK;
  const char* what = e == kErrKrylov ? "Krylov error estimate above tol at m_max after the allowed substeps"
                     : e == kErrInverted ? "det F <= 0 at a Gauss point (inverted deformation)"
                     : e == kErrNonfinite ? "non-finite value in the Krylov recurrence"
                     : e == kErrDevice ? "device synchronisation timed out"
                                       : "device error";
  return fail(c, (ep_status)e, what);
}

// ------------------------------------------------------------------------------ stepping
static OpArgs op_linear(double tau, double t_eval) {
  OpArgs op{};
  op.tau = tau;
  op.t_eval = t_eval;
  op.nsets = 0;
  return op;
}

static OpArgs op_from(const double* ulin, double tau, double t_eval) {
  OpArgs op{};
  op.tau = tau;
  op.t_eval = t_eval;
  op.nsets = ulin ? 1 : 0;
  op.ulin[0] = ulin;
  op.wts[0] = 1.0;
  return op;
}

// EP_PREC_MIXED_BF16: the element tangents of the operator about to be applied, formed
// before its projection (those of the rest-state operator are kept while they stay valid).
static ep_status form_tangents(ep_ctx* c, Inst& I, const OpArgs& op) {
  if (c->cfg.prec != 2) return EP_OK;
  const bool rest = I.model == EP_LINEAR || op.nsets == 0;
  if (rest && I.kst_rest) return EP_OK;
  launch_form_tangent(I.M, op, dptr<uint16_t>(c, I.o_psi), dptr<uint16_t>(c, I.o_kst), &I.W.ctrl->err, c->stream);
  EP_HIP(c, hipGetLastError());
  I.kst_rest = rest;
  return EP_OK;
}

static ep_status run_expv(ep_ctx* c, Inst& I, const OpArgs& op, int kind, const double* xin, double* xout, int mode,
                          int log_idx) {
  ep_status s = form_tangents(c, I, op);
  if (s != EP_OK) return s;
  ExpvArgs a{};
  a.M = I.M;
  a.W = I.W;
  a.cfg = c->cfg;
  a.op = op;
  a.kind = kind;
  a.x_in = xin;
  a.x_out = xout;
  a.out_mode = mode;
  a.log_idx = log_idx;
  EP_HIP(c, launch_expv(a, c->cfg.prec, c->stream));
  return EP_OK;
}

// load scale(t) on the host: piecewise linear through the knots, constant outside
static double load_scale_host(const Inst& I, double t) {
  const int n = I.n_knots;
  if (n <= 0) return 0.0;
  const double* kt = I.knots.data();
  const double* ks = kt + n;
  if (t <= kt[0]) return ks[0];
  if (t >= kt[n - 1]) return ks[n - 1];
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (kt[mid] <= t) lo = mid; else hi = mid;
  }
  return ks[lo] + (t - kt[lo]) / (kt[hi] - kt[lo]) * (ks[hi] - ks[lo]);
}

static double* hist_slot(ep_ctx* c, Inst& I, int s) { return dptr<double>(c, I.o_hist) + (size_t)s * I.n3; }

static int free_slot(const Inst& I) {
  for (int s = 0; s < 3; ++s)
    if (s != I.hist_new && s != I.hist_old) return s;
  return 0;
}

// One step of the fourth-order scheme: exp(Omega) wbar with Omega the two-term Magnus
// exponent at the Gauss-Legendre nodes tau_{1,2} = t + (1/2 -+ sqrt(3)/6) dt (Sec. 3.3's
// two-term truncation), the H-matrices at the displacements predicted for tau_1, tau_2:
// cubic Hermite through the (u, v) of this and the previous step's start, or on the first
// step (after a state is set) u + s v + s^2/2 M^{-1}(P(t) - R(u)), R(u) = H(u) u.
static ep_status step_m4(ep_ctx* c, Inst& I, double dt) {
  double* S = dptr<double>(c, I.o_S);
  const double t = I.t;
  const int log_idx = (int)(I.step_idx % kLogSteps);
  const double g = std::sqrt(3.0) / 6.0;
  OpArgs op{};
  op.tau = 1.0;
  op.t_eval = t + (0.5 - g) * dt;
  op.t_eval2 = t + (0.5 + g) * dt;
  op.dt4 = dt;
  op.c4 = std::sqrt(3.0) * dt * dt / 12.0;
  op.nsets = 0;
  if (I.model != EP_LINEAR) {
    double* u1 = hist_slot(c, I, 0);
    double* u2 = hist_slot(c, I, 1);
    double* R = hist_slot(c, I, 2);
    double* st = dptr<double>(c, I.o_stage);
    if (!I.m4_prev) {
      launch_get_state(I.n3, I.M.mih, S, st, st + I.n3, c->stream);
      launch_apply_H(I.M, op_from(st, 1.0, 0.0), 0, st, R, I.W.F, I.W.F32, &I.W.ctrl->err, c->stream);
      EP_HIP(c, hipGetLastError());
    }
    launch_m4_predict(I.M, S, dptr<double>(c, I.o_Sprev), R, load_scale_host(I, t), t, I.t_prev, op.t_eval,
                      op.t_eval2, I.m4_prev ? 0 : 1, u1, u2, c->stream);
    EP_HIP(c, hipGetLastError());
    op.nsets = 2;
    op.ulin[0] = u1;
    op.ulin[1] = u2;
    op.wts[0] = op.wts[1] = 1.0;
  }
  // this step's start state feeds the next step's extrapolation
  EP_HIP(c, hipMemcpyAsync(dptr<double>(c, I.o_Sprev), S, 8 * 2 * (size_t)I.n3, hipMemcpyDeviceToDevice,
                           c->stream));
  ep_status s = run_expv(c, I, op, 0, S, S, 0, log_idx);
  if (s != EP_OK) return s;
  I.m4_prev = true;
  I.t_prev = t;
  I.t = t + dt;
  I.step_idx += 1;
  return EP_OK;
}

static ep_status step_one(ep_ctx* c, Inst& I, double dt) {
  if (c->cfg.scheme == 4) return step_m4(c, I, dt);
  double* S = dptr<double>(c, I.o_S);
  const double t = I.t;
  const int log_idx = (int)(I.step_idx % kLogSteps);
  if (I.model == EP_LINEAR) {
    ep_status s = run_expv(c, I, op_linear(dt, t + 0.5 * dt), 0, S, S, 0, log_idx);
    if (s != EP_OK) return s;
  } else {
    OpArgs pred{};
    pred.tau = 0.5 * dt;
    pred.t_eval = t + 0.25 * dt;
    if (I.nhist == 0) {
      // first step: H(u_0) at the current displacement
      const int s0 = free_slot(I);
      launch_get_state(I.n3, I.M.mih, S, hist_slot(c, I, s0), nullptr, c->stream);
      EP_HIP(c, hipGetLastError());
      pred.nsets = 1;
      pred.ulin[0] = hist_slot(c, I, s0);
      pred.wts[0] = 1.0;
      I.hist_old = s0;   // reserve while the predictor reads it
    } else if (I.nhist == 1) {
      pred.nsets = 1;
      pred.ulin[0] = hist_slot(c, I, I.hist_new);
      pred.wts[0] = 1.0;
    } else {
      pred.nsets = 2;
      pred.ulin[0] = hist_slot(c, I, I.hist_new);
      pred.wts[0] = 1.75;
      pred.ulin[1] = hist_slot(c, I, I.hist_old);
      pred.wts[1] = -0.75;
    }
    const int snew = free_slot(I);
    ep_status s = run_expv(c, I, pred, 1, S, hist_slot(c, I, snew), 1, log_idx);
    if (s != EP_OK) return s;
    OpArgs corr{};
    corr.tau = dt;
    corr.t_eval = t + 0.5 * dt;
    corr.nsets = 1;
    corr.ulin[0] = hist_slot(c, I, snew);
    corr.wts[0] = 1.0;
    s = run_expv(c, I, corr, 0, S, S, 0, log_idx);
    if (s != EP_OK) return s;
    if (I.nhist == 0) {
      I.hist_old = -1;
      I.hist_new = snew;
      I.nhist = 1;
    } else {
      I.hist_old = I.hist_new;
      I.hist_new = snew;
      I.nhist = 2;
    }
  }
  I.t = t + dt;
  I.step_idx += 1;
  return EP_OK;
}

// ============================================================================== C ABI
extern "C" {

const char* ep_version(void) { return "ep-mi355x 0.1 (gfx950)"; }

ep_status ep_create(ep_ctx** out, int hip_device) {
  if (!out) return EP_ERR_ARG;
  *out = nullptr;
  if (hip_device < -1) return EP_ERR_ARG;
  ep_ctx* c = new (std::nothrow) ep_ctx();
  if (!c) return EP_ERR_ARG;
  c->device = hip_device;
  if (hip_device >= 0) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device >= n) {
      delete c;
      return EP_ERR_HIP;
    }
    if (hipSetDevice(hip_device) != hipSuccess) {
      delete c;
      return EP_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
      delete c;
      return EP_ERR_HIP;
    }
    c->cus = prop.multiProcessorCount;
  } else {
    c->cus = 256;
  }
  *out = c;
  return EP_OK;
}

ep_status ep_destroy(ep_ctx* c) {
  if (!c) return EP_ERR_ARG;
  delete c;
  return EP_OK;
}

const char* ep_last_error(const ep_ctx* c) { return c ? c->err.c_str() : "null context"; }

ep_status ep_set_stream(ep_ctx* c, void* s) {
  if (!c) return EP_ERR_ARG;
  c->stream = reinterpret_cast<hipStream_t>(s);
  return EP_OK;
}

ep_status ep_set_mesh_hex8(ep_ctx* c, int64_t n_nodes, const double* xyz, int64_t n_elems, const int32_t* conn) {
  if (!c) return EP_ERR_ARG;
  if (c->bound) return fail(c, EP_ERR_ORDER, "setup after ep_bind_workspace");
  if (c->batch) return fail(c, EP_ERR_ORDER, "batch context: use ep_batch_add_instance");
  ep_status s = check_mesh(c, n_nodes, xyz, n_elems, conn);
  if (s != EP_OK) return s;
  fill_mesh(c->one, n_nodes, xyz, n_elems, conn);
  c->one.clamped.clear();
  c->one.faces.clear();
  c->one.n_knots = 0;
  c->one.knots.clear();
  c->mesh_set = true;
  return EP_OK;
}

ep_status ep_set_mesh_hex27(ep_ctx* c, int64_t n_nodes, const double* xyz, int64_t n_elems, const int32_t* conn) {
  if (!c) return EP_ERR_ARG;
  if (c->bound) return fail(c, EP_ERR_ORDER, "setup after ep_bind_workspace");
  if (c->batch) return fail(c, EP_ERR_ARG, "batches take hex8 meshes");
  ep_status s = check_mesh(c, n_nodes, xyz, n_elems, conn, 27);
  if (s != EP_OK) return s;
  fill_mesh(c->one, n_nodes, xyz, n_elems, conn, 27);
  c->one.clamped.clear();
  c->one.faces.clear();
  c->one.n_knots = 0;
  c->one.knots.clear();
  c->mesh_set = true;
  return EP_OK;
}

ep_status ep_set_material(ep_ctx* c, ep_model model, const double* p, int n, double rho) {
  if (!c) return EP_ERR_ARG;
  if (c->bound) return fail(c, EP_ERR_ORDER, "setup after ep_bind_workspace");
  ep_status s = check_material(c, (int)model, p, n, rho);
  if (s != EP_OK) return s;
  c->one.model = (int)model;
  for (int i = 0; i < 4; ++i) c->one.mp[i] = i < n ? p[i] : 0.0;
  c->one.rho = rho;
  c->material_set = true;
  return EP_OK;
}

ep_status ep_set_dirichlet(ep_ctx* c, int64_t n, const int32_t* ids) {
  if (!c) return EP_ERR_ARG;
  if (c->bound) return fail(c, EP_ERR_ORDER, "setup after ep_bind_workspace");
  if (!c->mesh_set) return fail(c, EP_ERR_ORDER, "ep_set_dirichlet before ep_set_mesh_hex8");
  if (n < 0 || (n > 0 && !ids)) return fail(c, EP_ERR_ARG, "bad Dirichlet list");
  for (int64_t i = 0; i < n; ++i)
    if (ids[i] < 0 || ids[i] >= c->one.n3) return fail(c, EP_ERR_ARG, "Dirichlet DOF out of range");
  c->one.clamped.assign(ids, ids + n);
  return EP_OK;
}

ep_status ep_set_traction(ep_ctx* c, int64_t n_faces, const int32_t* fn, const double t0[3], int64_t n_knots,
                          const double* kt, const double* ks) {
  if (!c) return EP_ERR_ARG;
  if (c->bound) return fail(c, EP_ERR_ORDER, "setup after ep_bind_workspace");
  if (!c->mesh_set) return fail(c, EP_ERR_ORDER, "ep_set_traction before ep_set_mesh_hex8");
  ep_status s = check_traction(c, c->one.n_nodes, n_faces, fn, t0, n_knots, kt, ks, c->one.nfn);
  if (s != EP_OK) return s;
  fill_traction(c->one, n_faces, fn, t0, n_knots, kt, ks);
  return EP_OK;
}

ep_status ep_set_krylov(ep_ctx* c, double tol, int m_max, int check_every, int m_fixed, int k_fixed,
                        int max_substeps, double s0) {
  if (!c) return EP_ERR_ARG;
  if (c->bound) return fail(c, EP_ERR_ORDER, "ep_set_krylov after ep_bind_workspace");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(c, EP_ERR_ARG, "tol must be positive");
  if (m_max < 1 || m_max > kMaxM) return fail(c, EP_ERR_ARG, "m_max must be in [1, 256]");
  if (check_every < 1) return fail(c, EP_ERR_ARG, "check_every must be >= 1");
  if (m_fixed < 0 || m_fixed > m_max) return fail(c, EP_ERR_ARG, "m_fixed must be in [0, m_max]");
  if (k_fixed < 0 || max_substeps < 1 || k_fixed > (1 << 20)) return fail(c, EP_ERR_ARG, "bad substep settings");
  if (!std::isfinite(s0)) return fail(c, EP_ERR_ARG, "s0 must be finite");
  c->cfg.tol = tol;
  c->cfg.m_max = m_max;
  c->cfg.check_every = check_every;
  c->cfg.m_fixed = m_fixed;
  c->cfg.k_fixed = k_fixed;
  c->cfg.max_substeps = max_substeps;
  c->s0_user = s0;
  return EP_OK;
}

ep_status ep_set_orthogonalization(ep_ctx* c, int mode) {
  if (!c) return EP_ERR_ARG;
  if (c->bound) return fail(c, EP_ERR_ORDER, "ep_set_orthogonalization after ep_bind_workspace");
  if (mode < -1 || mode > 1) return fail(c, EP_ERR_ARG, "orthogonalisation mode must be -1, 0 or 1");
  c->ortho_user = mode;
  return EP_OK;
}

ep_status ep_get_orthogonalization(ep_ctx* c, int* mode) {
  if (!c || !mode) return EP_ERR_ARG;
  *mode = c->bound ? c->cfg.ortho : eff_ortho(c);
  return EP_OK;
}

ep_status ep_set_scheme(ep_ctx* c, int order) {
  if (!c) return EP_ERR_ARG;
  if (c->bound) return fail(c, EP_ERR_ORDER, "ep_set_scheme after ep_bind_workspace");
  if (order != 2 && order != 4) return fail(c, EP_ERR_ARG, "the time integrator order must be 2 or 4");
  c->cfg.scheme = order;
  return EP_OK;
}

ep_status ep_set_precision(ep_ctx* c, ep_precision p) {
  if (!c) return EP_ERR_ARG;
  if (p != EP_PREC_F64 && p != EP_PREC_MIXED_F32 && p != EP_PREC_MIXED_BF16)
    return fail(c, EP_ERR_ARG, "unknown precision");
  if (p == EP_PREC_MIXED_BF16 && c->batch)
    return fail(c, EP_ERR_ARG, "batches take EP_PREC_F64 or EP_PREC_MIXED_F32");
  if (p == EP_PREC_MIXED_BF16 && c->bound && c->one.M.kst == nullptr)
    return fail(c, EP_ERR_ORDER, "EP_PREC_MIXED_BF16 must be set before ep_bind_workspace");
  c->cfg.prec = (int)p;
  c->one.kst_rest = false;
  return EP_OK;
}

ep_status ep_set_launch(ep_ctx* c, int G) {
  if (!c) return EP_ERR_ARG;
  if (c->bound) return fail(c, EP_ERR_ORDER, "ep_set_launch after ep_bind_workspace");
  if (G < 0 || G > 1024) return fail(c, EP_ERR_ARG, "workgroups must be in [0, 1024]");
  c->G_user = G;
  return EP_OK;
}

ep_status ep_workspace_size(ep_ctx* c, size_t* bytes) {
  if (!c || !bytes) return EP_ERR_ARG;
  if (!c->batch && (!c->mesh_set || !c->material_set))
    return fail(c, EP_ERR_ORDER, "workspace size needs the mesh and the material");
  if (c->batch && c->insts.empty()) return fail(c, EP_ERR_ORDER, "batch has no instances");
  if (c->batch && c->cfg.prec == 2) return fail(c, EP_ERR_ARG, "batches take EP_PREC_F64 or EP_PREC_MIXED_F32");
  if (!c->bound) {
    if (!c->batch && c->ortho_user == 1 && c->cfg.m_max > kMaxCwyM)
      return fail(c, EP_ERR_ARG, "compact-WY orthogonalisation needs m_max <= 64");
    c->cfg.ortho = eff_ortho(c);
  }
  *bytes = plan_all(c);
  return EP_OK;
}

ep_status ep_batch_bind(ep_ctx* c);   // ep_batch.cpp

ep_status ep_bind_workspace(ep_ctx* c, void* p, size_t bytes) {
  if (!c) return EP_ERR_ARG;
  if (c->bound) return fail(c, EP_ERR_ORDER, "workspace already bound");
  size_t need = 0;
  ep_status s = ep_workspace_size(c, &need);
  if (s != EP_OK) return s;
  if (!p) return fail(c, EP_ERR_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(p) % kAlign != 0) return fail(c, EP_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (bytes < need) return fail(c, EP_ERR_WORKSPACE, "workspace too small");
  if (!is_gpu(c)) return fail(c, EP_ERR_HIP, "host-only context cannot bind device memory");
  EP_HIP(c, hipSetDevice(c->device));
  if (c->cfg.scheme == 4 && c->batch) return fail(c, EP_ERR_ARG, "the fourth-order scheme runs single instances");
  if (!c->batch && c->one.npe == 27 && (c->cfg.prec == 2 || c->cfg.scheme == 4))
    return fail(c, EP_ERR_ARG, "quadratic elements take EP_PREC_F64 / EP_PREC_MIXED_F32 and the second-order scheme");
  if (c->cfg.scheme == 4 && c->cfg.prec == 2)
    return fail(c, EP_ERR_ARG, "the fourth-order scheme takes EP_PREC_F64 or EP_PREC_MIXED_F32");
  c->ws = reinterpret_cast<char*>(p);
  c->ws_bytes = bytes;
  if (c->batch) {
    s = ep_batch_bind(c);
    if (s != EP_OK) return s;
  } else {
    int chunk = 0, sg = 0;
    int G = pick_G(c, c->one, &chunk, &sg);
    // cooperative residency: shrink G until it fits
    int bpc = 0;
    for (;;) {
      if (c->cfg.scheme == 4 && sg)
        return fail(c, EP_ERR_ARG, "the fourth-order scheme needs the Krylov slices in LDS (team too small)");
      EP_HIP(c, expv_max_blocks(c->cfg, c->one.model, c->one.npe, chunk, sg, &bpc));
      if ((long long)bpc * c->cus >= G || G == 1) break;
      G = std::max(1, (int)((long long)bpc * c->cus));
      chunk = chunk_of(c, c->one, G, &sg);
    }
    if (bpc < 1) return fail(c, EP_ERR_WORKSPACE, "persistent kernel does not fit on a compute unit");
    s = setup_inst(c, c->one, G, chunk, Gmax_of(c));
    c->one.W.slices_global = sg;
    if (s != EP_OK) return s;
  }
  c->bound = true;
  return EP_OK;
}

static ep_status need_bound(ep_ctx* c) {
  if (!c) return EP_ERR_ARG;
  if (!c->bound) return fail(c, EP_ERR_ORDER, "call ep_bind_workspace first");
  if (c->batch) return fail(c, EP_ERR_ORDER, "batch context: use the ep_batch_* calls");
  return EP_OK;
}

ep_status ep_set_state(ep_ctx* c, double t, const double* u, const double* v) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  if (!u || !v || !std::isfinite(t)) return fail(c, EP_ERR_ARG, "bad state arguments");
  Inst& I = c->one;
  for (int i = 0; i < I.n3; ++i)
    if (!std::isfinite(u[i]) || !std::isfinite(v[i])) return fail(c, EP_ERR_ARG, "non-finite state");
  double* st = dptr<double>(c, I.o_stage);
  EP_HIP(c, hipMemcpyAsync(st, u, 8 * (size_t)I.n3, hipMemcpyHostToDevice, c->stream));
  EP_HIP(c, hipMemcpyAsync(st + I.n3, v, 8 * (size_t)I.n3, hipMemcpyHostToDevice, c->stream));
  launch_set_state(I.n3, I.Lp, I.M.mh, st, st + I.n3, I.M.s0, dptr<double>(c, I.o_S), c->stream);
  launch_reset_ctrl(I.W.ctrl, c->stream);
  EP_HIP(c, hipGetLastError());
  EP_HIP(c, hipStreamSynchronize(c->stream));
  I.t = t;
  I.step_idx = 0;
  I.nhist = 0;
  I.hist_new = I.hist_old = -1;
  I.state_set = true;
  I.s0_pending = scaled_s0_mode(c);
  I.m4_prev = false;
  return EP_OK;
}

ep_status ep_step(ep_ctx* c, double dt, int64_t n) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  if (!c->one.state_set) return fail(c, EP_ERR_ORDER, "call ep_set_state first");
  if (!(dt > 0.0) || !std::isfinite(dt) || n < 0) return fail(c, EP_ERR_ARG, "need dt > 0 and n_steps >= 0");
  if (n > 0) {
    s = resolve_s0(c, c->one, dt);
    if (s != EP_OK) return s;
  }
  for (int64_t i = 0; i < n; ++i) {
    s = step_one(c, c->one, dt);
    if (s != EP_OK) return s;
  }
  return EP_OK;
}

ep_status ep_sync(ep_ctx* c) {
  if (!c) return EP_ERR_ARG;
  if (!c->bound) return fail(c, EP_ERR_ORDER, "call ep_bind_workspace first");
  EP_HIP(c, hipStreamSynchronize(c->stream));
  if (c->batch) {
    for (auto& I : c->insts) {
      ep_status s = read_err(c, I);
      if (s != EP_OK) return s;
    }
    return EP_OK;
  }
  return read_err(c, c->one);
}

ep_status ep_get_state(ep_ctx* c, double* t, double* u, double* v) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  if (!t || !u || !v) return fail(c, EP_ERR_ARG, "null output");
  s = ep_sync(c);
  if (s != EP_OK) return s;
  Inst& I = c->one;
  double* st = dptr<double>(c, I.o_stage);
  launch_get_state(I.n3, I.M.mih, dptr<double>(c, I.o_S), st, st + I.n3, c->stream);
  EP_HIP(c, hipGetLastError());
  EP_HIP(c, hipMemcpyAsync(u, st, 8 * (size_t)I.n3, hipMemcpyDeviceToHost, c->stream));
  EP_HIP(c, hipMemcpyAsync(v, st + I.n3, 8 * (size_t)I.n3, hipMemcpyDeviceToHost, c->stream));
  EP_HIP(c, hipStreamSynchronize(c->stream));
  *t = I.t;
  return EP_OK;
}

ep_status ep_get_energy(ep_ctx* c, double* ke, double* se, double* we) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  if (!ke || !se || !we) return fail(c, EP_ERR_ARG, "null output");
  s = ep_sync(c);
  if (s != EP_OK) return s;
  Inst& I = c->one;
  double* out = dptr<double>(c, I.o_eout);
  launch_energy(I.M, dptr<double>(c, I.o_S), I.t, dptr<double>(c, I.o_pe), dptr<double>(c, I.o_pv), out, c->stream);
  EP_HIP(c, hipGetLastError());
  double h[3];
  EP_HIP(c, hipMemcpyAsync(h, out, 24, hipMemcpyDeviceToHost, c->stream));
  EP_HIP(c, hipStreamSynchronize(c->stream));
  *ke = h[0];
  *se = h[1];
  *we = h[2];
  return EP_OK;
}

ep_status ep_get_stats(ep_ctx* c, int64_t* matvecs, int* last_m, double* last_eps, int* last_k, double* drift) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  EP_HIP(c, hipStreamSynchronize(c->stream));
  Ctrl h;
  EP_HIP(c, hipMemcpy(&h, c->one.W.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
  if (matvecs) *matvecs = h.ks[0].matvecs + h.ks[1].matvecs;
  if (last_m) *last_m = h.ks[0].last_m;
  if (last_eps) *last_eps = h.ks[0].last_eps;
  if (last_k) *last_k = h.ks[0].last_k;
  if (drift) *drift = h.drift;
  return EP_OK;
}

ep_status ep_get_launch(ep_ctx* c, int* workgroups, int* chunk, int* slices_global, int* congruent) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  if (workgroups) *workgroups = c->one.W.G;
  if (chunk) *chunk = c->one.W.chunk;
  if (slices_global) *slices_global = c->one.W.slices_global;
  if (congruent) *congruent = c->one.M.congruent ? (c->one.M.lat[0] > 0 ? 2 : 1) : 0;
  return EP_OK;
}

ep_status ep_get_step_log(ep_ctx* c, int n, int32_t* m_corr, int32_t* m_pred, int32_t* k_corr, double* eps_corr) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  if (n < 0 || n > kLogSteps) return fail(c, EP_ERR_ARG, "n must be in [0, 4096]");
  EP_HIP(c, hipStreamSynchronize(c->stream));
  std::vector<StepLog> h(1);
  EP_HIP(c, hipMemcpy(h.data(), c->one.W.log, sizeof(StepLog), hipMemcpyDeviceToHost));
  const int64_t end = c->one.step_idx;
  for (int i = 0; i < n; ++i) {
    const int64_t idx = end - n + i;
    const int sl = (int)(((idx % kLogSteps) + kLogSteps) % kLogSteps);
    const bool ok = idx >= 0;
    if (m_corr) m_corr[i] = ok ? h[0].m_corr[sl] : 0;
    if (m_pred) m_pred[i] = ok ? h[0].m_pred[sl] : 0;
    if (k_corr) k_corr[i] = ok ? h[0].k_corr[sl] : 0;
    if (eps_corr) eps_corr[i] = ok ? h[0].eps_corr[sl] : 0.0;
  }
  return EP_OK;
}

// --------------------------------------------------------------------------- stage calls

ep_status ep_apply_H(ep_ctx* c, const double* u_lin, const double* x, double* y) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  if (!x || !y) return fail(c, EP_ERR_ARG, "null vector");
  Inst& I = c->one;
  s = form_tangents(c, I, op_from(u_lin, 1.0, 0.0));
  if (s != EP_OK) return s;
  launch_apply_H(I.M, op_from(u_lin, 1.0, 0.0), c->cfg.prec, x, y, I.W.F, I.W.F32, &I.W.ctrl->err, c->stream);
  EP_HIP(c, hipGetLastError());
  return EP_OK;   // enqueued; a sticky device error is reported by the next ep_sync
}

ep_status ep_form_tangents(ep_ctx* c, const double* u_lin) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  if (c->cfg.prec != 2) return fail(c, EP_ERR_ORDER, "ep_form_tangents needs EP_PREC_MIXED_BF16");
  Inst& I = c->one;
  I.kst_rest = false;          // always form
  return form_tangents(c, I, op_from(u_lin, 1.0, 0.0));
}

ep_status ep_vector_length(ep_ctx* c, int64_t* len, int64_t* padded) {
  if (!c || !len || !padded) return EP_ERR_ARG;
  if (c->batch || !c->mesh_set) return fail(c, EP_ERR_ORDER, "needs a single-instance mesh");
  *len = c->one.L;
  *padded = c->one.Lp;
  return EP_OK;
}

ep_status ep_apply_A(ep_ctx* c, const double* u_lin, double tau, double pscale, const double* x, double* y) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  if (!x || !y || !std::isfinite(tau) || !std::isfinite(pscale)) return fail(c, EP_ERR_ARG, "bad arguments");
  Inst& I = c->one;
  // the load scale is passed through a one-knot table evaluated at t = 0
  Mesh M = I.M;
  double* kn = dptr<double>(c, I.o_stage);
  double h2[2] = {0.0, pscale};
  EP_HIP(c, hipMemcpyAsync(kn, h2, 16, hipMemcpyHostToDevice, c->stream));
  M.knots = kn;
  M.n_knots = 1;
  s = form_tangents(c, I, op_from(u_lin, tau, 0.0));
  if (s != EP_OK) return s;
  launch_apply_A(M, op_from(u_lin, tau, 0.0), c->cfg.prec, x, y, I.W.F, I.W.F32, &I.W.ctrl->err, c->stream);
  EP_HIP(c, hipGetLastError());
  return ep_sync(c);
}

ep_status ep_expm(ep_ctx* c, int m, const double* H, double* E) {
  if (!c) return EP_ERR_ARG;
  if (m < 1 || m > kMaxM || !H || !E) return fail(c, EP_ERR_ARG, "need 1 <= m <= 256 and host arrays");
  for (int i = 0; i < m * m; ++i)
    if (!std::isfinite(H[i])) return fail(c, EP_ERR_ARG, "non-finite matrix entry");
  if (!c->bound || c->batch) return fail(c, EP_ERR_ORDER, "call ep_bind_workspace first");
  Inst& I = c->one;
  if (m > c->cfg.m_max) return fail(c, EP_ERR_ARG, "m exceeds the m_max the workspace was sized for");
  double* dH = I.W.H;
  double* dE = I.W.Escr + (size_t)8 * c->cfg.m_max * c->cfg.m_max;
  EP_HIP(c, hipMemcpyAsync(dH, H, 8 * (size_t)m * m, hipMemcpyHostToDevice, c->stream));
  launch_expm(m, dH, dE, I.W.Escr, c->stream);
  EP_HIP(c, hipGetLastError());
  EP_HIP(c, hipMemcpyAsync(E, dE, 8 * (size_t)m * m, hipMemcpyDeviceToHost, c->stream));
  EP_HIP(c, hipStreamSynchronize(c->stream));
  return EP_OK;
}

ep_status ep_arnoldi(ep_ctx* c, const double* u_lin, double tau, double pscale, const double* w, int m, double* V,
                     double* H, int* steps) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  Inst& I = c->one;
  if (!w || !H || !steps || m < 1 || m > c->cfg.m_max) return fail(c, EP_ERR_ARG, "bad arguments");
  double* kn = dptr<double>(c, I.o_stage);
  double h2[2] = {0.0, pscale};
  EP_HIP(c, hipMemcpyAsync(kn, h2, 16, hipMemcpyHostToDevice, c->stream));
  ExpvArgs a{};
  a.M = I.M;
  a.M.knots = kn;
  a.M.n_knots = 1;
  a.W = I.W;
  a.cfg = c->cfg;
  a.cfg.m_fixed = m;
  a.cfg.k_fixed = 1;
  a.op = op_from(u_lin, tau, 0.0);
  a.kind = 2;
  a.x_in = w;
  a.x_out = I.W.X;   // result discarded
  a.out_mode = 2;
  a.log_idx = -1;
  EP_HIP(c, hipMemsetAsync(I.W.H, 0, 8 * (size_t)(c->cfg.m_max + 1) * c->cfg.m_max, c->stream));
  s = form_tangents(c, I, a.op);
  if (s != EP_OK) return s;
  EP_HIP(c, launch_expv(a, c->cfg.prec, c->stream));
  s = ep_sync(c);
  if (s != EP_OK) return s;
  Ctrl h;
  EP_HIP(c, hipMemcpy(&h, I.W.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
  *steps = h.ks[2].last_m;
  const int ld = c->cfg.m_max;
  std::vector<double> Hs((size_t)(ld + 1) * ld);
  EP_HIP(c, hipMemcpy(Hs.data(), I.W.H, 8 * Hs.size(), hipMemcpyDeviceToHost));
  for (int i = 0; i <= m; ++i)
    for (int j = 0; j < m; ++j) H[(size_t)i * m + j] = Hs[(size_t)i * ld + j];
  if (V) EP_HIP(c, hipMemcpy(V, I.W.V, 8 * (size_t)I.Lp * (m + 1), hipMemcpyDeviceToDevice));
  return EP_OK;
}

ep_status ep_expv(ep_ctx* c, const double* u_lin, double tau, double pscale, const double* w, double* y, int* m_used,
                  int* k_used, double* eps) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  Inst& I = c->one;
  if (!w || !y || !std::isfinite(tau)) return fail(c, EP_ERR_ARG, "bad arguments");
  double* kn = dptr<double>(c, I.o_stage);
  double h2[2] = {0.0, pscale};
  EP_HIP(c, hipMemcpyAsync(kn, h2, 16, hipMemcpyHostToDevice, c->stream));
  ExpvArgs a{};
  a.M = I.M;
  a.M.knots = kn;
  a.M.n_knots = 1;
  a.W = I.W;
  a.cfg = c->cfg;
  a.op = op_from(u_lin, tau, 0.0);
  a.kind = 2;
  a.x_in = w;
  a.x_out = y;
  a.out_mode = 2;
  a.log_idx = -1;
  s = form_tangents(c, I, a.op);
  if (s != EP_OK) return s;
  EP_HIP(c, launch_expv(a, c->cfg.prec, c->stream));
  s = ep_sync(c);
  if (s != EP_OK) return s;
  Ctrl h;
  EP_HIP(c, hipMemcpy(&h, I.W.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
  if (m_used) *m_used = h.ks[2].last_m;
  if (k_used) *k_used = h.ks[2].last_k;
  if (eps) *eps = h.ks[2].last_eps;
  return EP_OK;
}

}  // extern "C"

// ============================================================================== autotuner
extern "C" {

ep_status ep_autotune(ep_ctx* c, double dt, int m_trial, int trials, int* best_G, double* best_ms) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  Inst& I = c->one;
  if (!I.state_set) return fail(c, EP_ERR_ORDER, "call ep_set_state first");
  if (!(dt > 0.0) || !std::isfinite(dt) || m_trial < 1 || trials < 1 || trials > 1000)
    return fail(c, EP_ERR_ARG, "need dt > 0, m_trial >= 1, 1 <= trials <= 1000");
  const int m = std::min(m_trial, c->cfg.m_max);
  // linearisation point of the nonlinear operator: the current displacement (staging area)
  double* ucur = dptr<double>(c, I.o_stage);
  launch_get_state(I.n3, I.M.mih, dptr<double>(c, I.o_S), ucur, nullptr, c->stream);
  EP_HIP(c, hipGetLastError());
  ExpvArgs a{};
  a.M = I.M;
  a.W = I.W;
  a.cfg = c->cfg;
  a.cfg.m_fixed = m;
  a.cfg.k_fixed = 1;
  a.op.tau = dt;
  a.op.t_eval = I.t + 0.5 * dt;
  a.op.nsets = I.model == EP_LINEAR ? 0 : 1;
  a.op.ulin[0] = ucur;
  a.op.wts[0] = 1.0;
  a.kind = 2;
  a.x_in = dptr<double>(c, I.o_S);
  a.x_out = I.W.X;
  a.out_mode = 2;
  a.log_idx = -1;
  s = form_tangents(c, I, a.op);
  if (s != EP_OK) return s;
  static const int cand[] = {1, 2, 4, 8, 12, 16, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192, 256, 320, 384, 512};
  hipEvent_t e0, e1;
  EP_HIP(c, hipEventCreate(&e0));
  EP_HIP(c, hipEventCreate(&e1));
  int bestG = I.W.G, bestC = I.W.chunk, bestS = I.W.slices_global;
  float best = 1e30f;
  const int Gslots = Gmax_of(c);
  for (int G : cand) {
    if (G > Gslots || G > std::max(1, I.Lp / 64)) continue;
    int sg = 0;
    const int chunk = chunk_of(c, I, G, &sg);
    int bpc = 0;
    if (expv_max_blocks(c->cfg, I.model, I.npe, chunk, sg, &bpc) != hipSuccess || (long long)bpc * c->cus < G) continue;
    a.W.G = G;
    a.W.chunk = chunk;
    a.W.slices_global = sg;
    if (launch_expv(a, c->cfg.prec, c->stream) != hipSuccess) continue;   // warm-up
    (void)hipEventRecord(e0, c->stream);
    bool ok = true;
    for (int r = 0; r < trials && ok; ++r) ok = launch_expv(a, c->cfg.prec, c->stream) == hipSuccess;
    (void)hipEventRecord(e1, c->stream);
    if (hipEventSynchronize(e1) != hipSuccess || !ok) continue;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= trials;
    if (ms < best) {
      best = ms;
      bestG = G;
      bestC = chunk;
      bestS = sg;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s = read_err(c, I);
  if (s != EP_OK) return s;
  I.W.G = bestG;
  I.W.chunk = bestC;
  I.W.slices_global = bestS;
  if (best_G) *best_G = bestG;
  if (best_ms) *best_ms = best < 1e29f ? best : -1.0;
  return EP_OK;
}

}  // extern "C"

// ============================================================================== batches
extern "C" {

ep_status ep_batch_add_instance(ep_ctx* c, int64_t n_nodes, const double* xyz, int64_t n_elems, const int32_t* conn,
                                ep_model model, const double* params, int n_params, double rho, int64_t n_dirichlet,
                                const int32_t* dofs, int64_t n_faces, const int32_t* faces, const double t0[3],
                                int64_t n_knots, const double* kt, const double* ks, int32_t* id) {
  if (!c || !id) return EP_ERR_ARG;
  if (c->bound) return fail(c, EP_ERR_ORDER, "ep_batch_add_instance after ep_bind_workspace");
  if (c->mesh_set) return fail(c, EP_ERR_ORDER, "single-instance context: cannot add batch instances");
  ep_status s = check_mesh(c, n_nodes, xyz, n_elems, conn);
  if (s != EP_OK) return s;
  s = check_material(c, (int)model, params, n_params, rho);
  if (s != EP_OK) return s;
  if (n_dirichlet < 0 || (n_dirichlet > 0 && !dofs)) return fail(c, EP_ERR_ARG, "bad Dirichlet list");
  for (int64_t i = 0; i < n_dirichlet; ++i)
    if (dofs[i] < 0 || dofs[i] >= 3 * n_nodes) return fail(c, EP_ERR_ARG, "Dirichlet DOF out of range");
  s = check_traction(c, n_nodes, n_faces, faces, t0, n_knots, kt, ks);
  if (s != EP_OK) return s;
  Inst I;
  fill_mesh(I, n_nodes, xyz, n_elems, conn);
  I.model = (int)model;
  for (int i = 0; i < 4; ++i) I.mp[i] = i < n_params ? params[i] : 0.0;
  I.rho = rho;
  I.clamped.assign(dofs, dofs + n_dirichlet);
  fill_traction(I, n_faces, faces, t0, n_knots, kt, ks);
  c->batch = true;
  c->insts.push_back(std::move(I));
  *id = (int32_t)(c->insts.size() - 1);
  return EP_OK;
}

// ------------------------------------------------------------------------- batch plans
// A plan gives instance i a team of G[i] workgroups (G[i] > 1) or a place in one of the
// bins (lists of instances that one workgroup steps one after the other).  Applying it sets
// each instance's slice size and placement, uploads the work records and the bins, and
// drops the captured step graph.
static ep_status apply_batch_plan(ep_ctx* c, const std::vector<int>& G, const std::vector<std::vector<int>>& bins) {
  const int n = (int)c->insts.size();
  EP_HIP(c, hipStreamSynchronize(c->stream));
  EP_HIP(c, hipMemcpy(c->btab.data(), dptr<BatchInst>(c, c->o_batch_tab), sizeof(BatchInst) * n,
                      hipMemcpyDeviceToHost));
  c->max_lds_chunk = 0;
  c->bteam_max = 1;
  for (int i = 0; i < n; ++i) {
    Inst& I = c->insts[i];
    const int g = std::max(1, std::min(G[i], kBatchGmax));
    int chunk = (I.Lp + g - 1) / g;
    chunk = (chunk + 63) / 64 * 64;
    I.W.G = g;
    I.W.chunk = chunk;
    BatchInst& B = c->btab[i];
    B.W.G = g;
    B.W.chunk = chunk;
    B.use_lds = chunk <= kMaxChunk ? 1 : (chunk <= 2 * kMaxChunk ? 2 : 0);
    if (B.use_lds == 1) c->max_lds_chunk = std::max(c->max_lds_chunk, chunk);
    if (B.use_lds == 2) c->max_lds_chunk = std::max(c->max_lds_chunk, (chunk + 1) / 2);
    c->bteam_max = std::max(c->bteam_max, g);
  }
  for (int k = 0; k < kModels; ++k) {
    c->bwork[k].clear();
    c->bids[k].clear();
  }
  for (int i = 0; i < n; ++i)
    if (c->insts[i].W.G > 1) {
      const int k = c->insts[i].model;
      for (int r = 0; r < c->insts[i].W.G; ++r) c->bwork[k].push_back(BatchWork{i, r, c->insts[i].W.G, 0, 0});
    }
  for (const auto& bin : bins) {
    // a bin holds instances of one material model (one launch per model)
    std::vector<int> members[kModels];
    for (int i : bin)
      if (c->insts[i].W.G == 1) members[c->insts[i].model].push_back(i);
    for (int k = 0; k < kModels; ++k) {
      if (members[k].empty()) continue;
      c->bwork[k].push_back(BatchWork{-1, 0, 1, (int)c->bids[k].size(), (int)members[k].size()});
      for (int i : members[k]) c->bids[k].push_back(i);
    }
  }
  for (int k = 0; k < kModels; ++k) {
    if (c->bwork[k].size() > c->bwork_cap) return fail(c, EP_ERR_ARG, "batch plan has too many workgroups");
    if (c->bwork[k].empty()) continue;
    EP_HIP(c, hipMemcpy(dptr<char>(c, c->o_bwork[k]), c->bwork[k].data(), sizeof(BatchWork) * c->bwork[k].size(),
                        hipMemcpyHostToDevice));
    EP_HIP(c, hipMemcpy(dptr<char>(c, c->o_bids[k]), c->bids[k].data(), 4 * c->bids[k].size(),
                        hipMemcpyHostToDevice));
  }
  EP_HIP(c, hipMemcpy(dptr<char>(c, c->o_batch_tab), c->btab.data(), sizeof(BatchInst) * n, hipMemcpyHostToDevice));
  if (c->bgraph) { (void)hipGraphExecDestroy(c->bgraph); c->bgraph = nullptr; }
  if (c->bgraph_src) { (void)hipGraphDestroy(c->bgraph_src); c->bgraph_src = nullptr; }
  return EP_OK;
}

// Workgroups of one batch launch that can be resident together (teams wait on each other,
// so a plan with teams must not exceed it).
static ep_status batch_capacity(ep_ctx* c, int* cap) {
  int bpc = 0;
  int best = 1 << 30;
  for (int k = 0; k < kModels; ++k) {
    if (c->bids[k].empty() && c->bwork[k].empty()) continue;
    // the largest slice the plan may choose keeps the LDS of one workgroup per CU
    EP_HIP(c, batch_max_blocks(c->cfg.prec, k, kMaxChunk, &bpc));
    best = std::min(best, std::max(1, bpc) * std::max(1, c->cus));
  }
  *cap = best == (1 << 30) ? std::max(1, c->cus) : best;
  return EP_OK;
}

// Cost of one step of each instance on one workgroup: the measured wall-clock ticks per step
// when every instance has them, else elements + Lp / 10 (the element pass dominates).
static std::vector<double> batch_costs(ep_ctx* c) {
  const int n = (int)c->insts.size();
  std::vector<double> cost(n, 0.0);
  bool measured = true;
  for (int i = 0; i < n; ++i) {
    Ctrl h;
    if (hipMemcpy(&h, c->insts[i].W.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost) != hipSuccess || h.ticked_steps <= 0) {
      measured = false;
      break;
    }
    cost[i] = (double)h.ticks / (double)h.ticked_steps;
  }
  if (!measured)
    for (int i = 0; i < n; ++i) cost[i] = (double)c->insts[i].n_elems + 0.1 * (double)c->insts[i].Lp;
  return cost;
}

// Smallest makespan plan within `cap` workgroups per launch.  A team of G workgroups is
// modelled to step an instance of cost c in c (a + (1 - a) / G), a the part of a step that a
// team does not divide (its synchronisations, the check points, latency-bound phases);
// instances costlier than the target T get the smallest team that meets it, the others are
// packed first-fit-decreasing into lists of cost <= T; T is found by bisection.
static void make_batch_plan(ep_ctx* c, const std::vector<double>& cost, int cap, double serial,
                            std::vector<int>& G, std::vector<std::vector<int>>& bins) {
  const int n = (int)cost.size();
  double cmax = 0.0, csum = 0.0;
  for (double x : cost) { cmax = std::max(cmax, x); csum += x; }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  auto build = [&](double T, std::vector<int>& g, std::vector<std::vector<int>>& b) -> long long {
    g.assign(n, 1);
    b.clear();
    std::vector<double> load;
    long long used = 0;
    for (int i : order) {
      if (cost[i] > T) {
        int need = 0;
        for (int q = 2; q <= kBatchGmax && !need; ++q)
          if (cost[i] * (serial + (1.0 - serial) / q) <= T) need = q;
        if (!need) return -1;
        g[i] = need;
        used += need;
        continue;
      }
      size_t k = 0;
      while (k < load.size() && load[k] + cost[i] > T) ++k;
      if (k == load.size()) { load.push_back(0.0); b.emplace_back(); }
      load[k] += cost[i];
      b[k].push_back(i);
    }
    return used + (long long)b.size();
  };
  double lo = std::max(csum / std::max(cap, 1), cmax * (serial + (1.0 - serial) / kBatchGmax)),
         hi = std::max(cmax, csum);
  std::vector<int> g;
  std::vector<std::vector<int>> b;
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    const long long w = build(mid, g, b);
    if (w >= 0 && w <= cap) hi = mid; else lo = mid;
  }
  build(hi, G, bins);
}

ep_status ep_batch_plan(ep_ctx* c, int max_workgroups, double serial) {
  if (!c) return EP_ERR_ARG;
  if (!c->bound || !c->batch) return fail(c, EP_ERR_ORDER, "needs a bound batch context");
  if (!(serial >= 0.0) || !(serial < 1.0)) return fail(c, EP_ERR_ARG, "serial fraction must be in [0, 1)");
  int cap = 0;
  ep_status s = batch_capacity(c, &cap);
  if (s != EP_OK) return s;
  if (max_workgroups > 0) cap = std::min(cap, max_workgroups);
  std::vector<int> G;
  std::vector<std::vector<int>> bins;
  make_batch_plan(c, batch_costs(c), cap, serial, G, bins);
  return apply_batch_plan(c, G, bins);
}

ep_status ep_batch_get_plan(ep_ctx* c, int32_t id, int* team, int* workgroups) {
  if (!c) return EP_ERR_ARG;
  if (!c->bound || !c->batch) return fail(c, EP_ERR_ORDER, "needs a bound batch context");
  if (id >= (int32_t)c->insts.size()) return fail(c, EP_ERR_ARG, "instance id out of range");
  if (team && id >= 0) *team = c->insts[id].W.G;
  if (workgroups) {
    size_t w = 0;
    for (int k = 0; k < kModels; ++k) w += c->bwork[k].size();
    *workgroups = (int)w;
  }
  return EP_OK;
}

ep_status ep_batch_bind(ep_ctx* c) {
  const int n = (int)c->insts.size();
  c->btab.assign(n, BatchInst{});
  c->max_lds_chunk = 0;
  for (int k = 0; k < kModels; ++k) c->bids[k].clear();
  for (int i = 0; i < n; ++i) {
    Inst& I = c->insts[i];
    ep_status s = setup_inst(c, I, 1, I.Lp, kBatchGmax);
    if (s != EP_OK) return fail(c, s, "batch instance " + std::to_string(i) + ": " + c->err);
    BatchInst& B = c->btab[i];
    B.M = I.M;
    B.W = I.W;
    B.S = dptr<double>(c, I.o_S);
    B.hist = dptr<double>(c, I.o_hist);
    B.t = 0.0;
    B.step_idx = 0;
    B.nhist = 0;
    B.hist_new = B.hist_old = -1;
    B.use_lds = 0;                               // set by the plan
    c->bids[I.model].push_back(i);
  }
  EP_HIP(c, hipMemcpy(dptr<char>(c, c->o_batch_tab), c->btab.data(), sizeof(BatchInst) * n, hipMemcpyHostToDevice));
  // default plan: one workgroup per instance
  std::vector<int> G(n, 1);
  std::vector<std::vector<int>> bins;
  for (int i = 0; i < n; ++i) bins.push_back({i});
  return apply_batch_plan(c, G, bins);
}

static ep_status need_batch(ep_ctx* c, int32_t id) {
  if (!c) return EP_ERR_ARG;
  if (!c->bound || !c->batch) return fail(c, EP_ERR_ORDER, "needs a bound batch context");
  if (id < 0 || id >= (int32_t)c->insts.size()) return fail(c, EP_ERR_ARG, "instance id out of range");
  return EP_OK;
}

static ep_status pull_record(ep_ctx* c, int32_t id) {
  EP_HIP(c, hipStreamSynchronize(c->stream));
  EP_HIP(c, hipMemcpy(&c->btab[id], dptr<BatchInst>(c, c->o_batch_tab) + id, sizeof(BatchInst),
                      hipMemcpyDeviceToHost));
  return EP_OK;
}

ep_status ep_batch_set_state(ep_ctx* c, int32_t id, double t, const double* u, const double* v) {
  ep_status s = need_batch(c, id);
  if (s != EP_OK) return s;
  if (!u || !v || !std::isfinite(t)) return fail(c, EP_ERR_ARG, "bad state arguments");
  Inst& I = c->insts[id];
  for (int i = 0; i < I.n3; ++i)
    if (!std::isfinite(u[i]) || !std::isfinite(v[i])) return fail(c, EP_ERR_ARG, "non-finite state");
  s = pull_record(c, id);
  if (s != EP_OK) return s;
  double* st = dptr<double>(c, I.o_stage);
  EP_HIP(c, hipMemcpyAsync(st, u, 8 * (size_t)I.n3, hipMemcpyHostToDevice, c->stream));
  EP_HIP(c, hipMemcpyAsync(st + I.n3, v, 8 * (size_t)I.n3, hipMemcpyHostToDevice, c->stream));
  launch_set_state(I.n3, I.Lp, I.M.mh, st, st + I.n3, I.M.s0, dptr<double>(c, I.o_S), c->stream);
  launch_reset_ctrl(I.W.ctrl, c->stream);
  EP_HIP(c, hipGetLastError());
  BatchInst& B = c->btab[id];
  B.t = t;
  B.step_idx = 0;
  B.nhist = 0;
  B.hist_new = B.hist_old = -1;
  EP_HIP(c, hipMemcpyAsync(dptr<BatchInst>(c, c->o_batch_tab) + id, &B, sizeof(BatchInst), hipMemcpyHostToDevice,
                           c->stream));
  EP_HIP(c, hipStreamSynchronize(c->stream));
  I.state_set = true;
  I.s0_pending = scaled_s0_mode(c);
  I.m4_prev = false;
  return EP_OK;
}

static ep_status batch_launch_all(ep_ctx* c, double dt, int n_steps, hipStream_t st) {
  for (int k = 0; k < kModels; ++k) {
    if (c->bwork[k].empty()) continue;
    bool teams = false;
    for (const auto& w : c->bwork[k]) teams |= w.G > 1;
    EP_HIP(c, launch_batch(dptr<BatchInst>(c, c->o_batch_tab), dptr<BatchWork>(c, c->o_bwork[k]),
                           dptr<int>(c, c->o_bids[k]), (int)c->bwork[k].size(), teams, k, c->cfg, dt, n_steps,
                           c->max_lds_chunk, st));
  }
  return EP_OK;
}

ep_status ep_batch_step(ep_ctx* c, double dt, int64_t n) {
  if (!c) return EP_ERR_ARG;
  if (!c->bound || !c->batch) return fail(c, EP_ERR_ORDER, "needs a bound batch context");
  if (!(dt > 0.0) || !std::isfinite(dt) || n < 0) return fail(c, EP_ERR_ARG, "need dt > 0 and n_steps >= 0");
  for (auto& I : c->insts)
    if (!I.state_set) return fail(c, EP_ERR_ORDER, "every instance needs ep_batch_set_state");
  if (n == 0) return EP_OK;
  for (int32_t id = 0; id < (int32_t)c->insts.size(); ++id) {
    Inst& I = c->insts[id];
    if (!I.s0_pending) continue;
    ep_status s = resolve_s0(c, I, dt);
    if (s != EP_OK) return s;
    s = pull_record(c, id);
    if (s != EP_OK) return s;
    c->btab[id].M.s0 = I.M.s0;
    c->btab[id].M.s_inv = I.M.s_inv;
    EP_HIP(c, hipMemcpy(dptr<BatchInst>(c, c->o_batch_tab) + id, &c->btab[id], sizeof(BatchInst),
                        hipMemcpyHostToDevice));
  }
  // one step = one launch per material model present, captured once into a graph and replayed
  if (c->bgraph == nullptr || c->bgraph_dt != dt) {
    if (c->bgraph) { (void)hipGraphExecDestroy(c->bgraph); c->bgraph = nullptr; }
    if (c->bgraph_src) { (void)hipGraphDestroy(c->bgraph_src); c->bgraph_src = nullptr; }
    hipStream_t cs;
    EP_HIP(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    ep_status s = EP_OK;
    if (e == hipSuccess) s = batch_launch_all(c, dt, 1, cs);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess || e2 != hipSuccess || s != EP_OK) {
      if (g) (void)hipGraphDestroy(g);
      if (s != EP_OK) return s;
      return fail(c, EP_ERR_HIP, "graph capture of the batch step failed");
    }
    c->bgraph_src = g;
    EP_HIP(c, hipGraphInstantiate(&c->bgraph, g, nullptr, nullptr, 0));
    c->bgraph_dt = dt;
  }
  for (int64_t i = 0; i < n; ++i) EP_HIP(c, hipGraphLaunch(c->bgraph, c->stream));
  return EP_OK;
}

ep_status ep_batch_get_state(ep_ctx* c, int32_t id, double* t, double* u, double* v) {
  ep_status s = need_batch(c, id);
  if (s != EP_OK) return s;
  if (!t || !u || !v) return fail(c, EP_ERR_ARG, "null output");
  EP_HIP(c, hipStreamSynchronize(c->stream));
  s = read_err(c, c->insts[id]);                 // this instance's failure only
  if (s != EP_OK) return s;
  s = pull_record(c, id);
  if (s != EP_OK) return s;
  Inst& I = c->insts[id];
  double* st = dptr<double>(c, I.o_stage);
  launch_get_state(I.n3, I.M.mih, dptr<double>(c, I.o_S), st, st + I.n3, c->stream);
  EP_HIP(c, hipGetLastError());
  EP_HIP(c, hipMemcpyAsync(u, st, 8 * (size_t)I.n3, hipMemcpyDeviceToHost, c->stream));
  EP_HIP(c, hipMemcpyAsync(v, st + I.n3, 8 * (size_t)I.n3, hipMemcpyDeviceToHost, c->stream));
  EP_HIP(c, hipStreamSynchronize(c->stream));
  *t = c->btab[id].t;
  return EP_OK;
}

// ------------------------------------------------------------------------- checkpoints
// Opaque image of an instance's stepping state: a fixed header, then the device state vector
// (Lp doubles: ubar | vbar | s | padding, as held), the predictor's three midpoint
// displacement fields (3 n3 doubles), the fourth-order scheme's previous start state (2 n3
// doubles, scheme 4 only) and the control block (adaptive Krylov state per projection kind).
namespace {
struct CkptHead {
  char magic[8];
  int32_t version, n3, Lp, npe, model, prec, scheme, batch;
  int32_t nhist, hist_new, hist_old, s0_pending, m4_prev, G;
  int64_t step_idx;
  double t, t_prev, s0;
};
constexpr char kCkptMagic[8] = {'E', 'P', 'C', 'K', 'P', 'T', '0', '1'};
}  // namespace

static size_t ckpt_sprev(const ep_ctx* c, const Inst& I) { return c->cfg.scheme == 4 ? 2 * (size_t)I.n3 : 0; }

static size_t ckpt_bytes(const ep_ctx* c, const Inst& I) {
  return sizeof(CkptHead) + 8 * ((size_t)I.Lp + 3 * (size_t)I.n3 + ckpt_sprev(c, I)) + sizeof(Ctrl);
}

static ep_status ckpt_save(ep_ctx* c, Inst& I, CkptHead h, void* buf, size_t bytes) {
  if (!buf) return fail(c, EP_ERR_ARG, "null checkpoint buffer");
  if (bytes < ckpt_bytes(c, I)) return fail(c, EP_ERR_ARG, "checkpoint buffer too small");
  if (!I.state_set) return fail(c, EP_ERR_ORDER, "no state to save: set a state first");
  std::memcpy(h.magic, kCkptMagic, 8);
  h.version = 1;
  h.n3 = I.n3;
  h.Lp = I.Lp;
  h.npe = I.npe;
  h.model = I.model;
  h.prec = c->cfg.prec;
  h.scheme = c->cfg.scheme == 4 ? 4 : 2;
  h.G = I.W.G;
  h.s0 = I.M.s0;
  h.s0_pending = I.s0_pending ? 1 : 0;
  char* p = static_cast<char*>(buf);
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  EP_HIP(c, hipMemcpy(p, dptr<double>(c, I.o_S), 8 * (size_t)I.Lp, hipMemcpyDeviceToHost));
  p += 8 * (size_t)I.Lp;
  EP_HIP(c, hipMemcpy(p, dptr<double>(c, I.o_hist), 8 * 3 * (size_t)I.n3, hipMemcpyDeviceToHost));
  p += 8 * 3 * (size_t)I.n3;
  if (ckpt_sprev(c, I)) {
    EP_HIP(c, hipMemcpy(p, dptr<double>(c, I.o_Sprev), 8 * ckpt_sprev(c, I), hipMemcpyDeviceToHost));
    p += 8 * ckpt_sprev(c, I);
  }
  EP_HIP(c, hipMemcpy(p, I.W.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
  return EP_OK;
}

// Checks the header against the instance and copies the device parts; returns the header.
static ep_status ckpt_load(ep_ctx* c, Inst& I, const void* buf, size_t bytes, bool batch, CkptHead* out) {
  if (!buf) return fail(c, EP_ERR_ARG, "null checkpoint buffer");
  if (bytes < sizeof(CkptHead)) return fail(c, EP_ERR_ARG, "not a checkpoint");
  CkptHead h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != 1) return fail(c, EP_ERR_ARG, "not a checkpoint");
  if (bytes != ckpt_bytes(c, I)) return fail(c, EP_ERR_ARG, "checkpoint size does not match this instance");
  if (h.n3 != I.n3 || h.Lp != I.Lp || h.npe != I.npe || h.model != I.model || h.prec != c->cfg.prec ||
      h.scheme != (c->cfg.scheme == 4 ? 4 : 2) || h.batch != (batch ? 1 : 0))
    return fail(c, EP_ERR_ARG, "checkpoint of a different mesh size, element, material, precision, scheme or "
                               "context kind");
  if (!(std::isfinite(h.t) && std::isfinite(h.s0) && h.s0 >= 0.0) || h.nhist < 0 || h.nhist > 2 ||
      h.hist_new < -1 || h.hist_new > 2 || h.hist_old < -1 || h.hist_old > 2 || h.step_idx < 0)
    return fail(c, EP_ERR_ARG, "corrupt checkpoint header");
  const char* p = static_cast<const char*>(buf) + sizeof(h);
  EP_HIP(c, hipStreamSynchronize(c->stream));
  EP_HIP(c, hipMemcpy(dptr<double>(c, I.o_S), p, 8 * (size_t)I.Lp, hipMemcpyHostToDevice));
  p += 8 * (size_t)I.Lp;
  EP_HIP(c, hipMemcpy(dptr<double>(c, I.o_hist), p, 8 * 3 * (size_t)I.n3, hipMemcpyHostToDevice));
  p += 8 * 3 * (size_t)I.n3;
  if (ckpt_sprev(c, I)) {
    EP_HIP(c, hipMemcpy(dptr<double>(c, I.o_Sprev), p, 8 * ckpt_sprev(c, I), hipMemcpyHostToDevice));
    p += 8 * ckpt_sprev(c, I);
  }
  Ctrl ctl;
  std::memcpy(&ctl, p, sizeof(Ctrl));
  ctl.err = 0;
  ctl.bar = 0;
  EP_HIP(c, hipMemcpy(I.W.ctrl, &ctl, sizeof(Ctrl), hipMemcpyHostToDevice));
  I.M.s0 = h.s0;
  I.M.s_inv = h.s0 != 0.0 ? 1.0 / h.s0 : 0.0;
  I.s0_pending = h.s0_pending != 0;
  I.m4_prev = h.m4_prev != 0;
  I.t_prev = h.t_prev;
  I.state_set = true;
  *out = h;
  return EP_OK;
}

ep_status ep_checkpoint_size(ep_ctx* c, size_t* bytes) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  if (!bytes) return fail(c, EP_ERR_ARG, "null output");
  *bytes = ckpt_bytes(c, c->one);
  return EP_OK;
}

ep_status ep_save_checkpoint(ep_ctx* c, void* buf, size_t bytes) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  s = ep_sync(c);
  if (s != EP_OK) return s;
  Inst& I = c->one;
  CkptHead h{};
  h.batch = 0;
  h.nhist = I.nhist;
  h.hist_new = I.hist_new;
  h.hist_old = I.hist_old;
  h.m4_prev = I.m4_prev ? 1 : 0;
  h.step_idx = I.step_idx;
  h.t = I.t;
  h.t_prev = I.t_prev;
  return ckpt_save(c, I, h, buf, bytes);
}

ep_status ep_load_checkpoint(ep_ctx* c, const void* buf, size_t bytes) {
  ep_status s = need_bound(c);
  if (s != EP_OK) return s;
  Inst& I = c->one;
  CkptHead h;
  s = ckpt_load(c, I, buf, bytes, false, &h);
  if (s != EP_OK) return s;
  I.t = h.t;
  I.step_idx = h.step_idx;
  I.nhist = h.nhist;
  I.hist_new = h.hist_new;
  I.hist_old = h.hist_old;
  return EP_OK;
}

ep_status ep_batch_checkpoint_size(ep_ctx* c, int32_t id, size_t* bytes) {
  ep_status s = need_batch(c, id);
  if (s != EP_OK) return s;
  if (!bytes) return fail(c, EP_ERR_ARG, "null output");
  *bytes = ckpt_bytes(c, c->insts[id]);
  return EP_OK;
}

ep_status ep_batch_save_checkpoint(ep_ctx* c, int32_t id, void* buf, size_t bytes) {
  ep_status s = need_batch(c, id);
  if (s != EP_OK) return s;
  EP_HIP(c, hipStreamSynchronize(c->stream));
  s = read_err(c, c->insts[id]);
  if (s != EP_OK) return s;
  s = pull_record(c, id);
  if (s != EP_OK) return s;
  const BatchInst& B = c->btab[id];
  CkptHead h{};
  h.batch = 1;
  h.nhist = B.nhist;
  h.hist_new = B.hist_new;
  h.hist_old = B.hist_old;
  h.step_idx = B.step_idx;
  h.t = B.t;
  return ckpt_save(c, c->insts[id], h, buf, bytes);
}

ep_status ep_batch_load_checkpoint(ep_ctx* c, int32_t id, const void* buf, size_t bytes) {
  ep_status s = need_batch(c, id);
  if (s != EP_OK) return s;
  Inst& I = c->insts[id];
  CkptHead h;
  s = ckpt_load(c, I, buf, bytes, true, &h);
  if (s != EP_OK) return s;
  s = pull_record(c, id);
  if (s != EP_OK) return s;
  BatchInst& B = c->btab[id];
  B.t = h.t;
  B.step_idx = h.step_idx;
  B.nhist = h.nhist;
  B.hist_new = h.hist_new;
  B.hist_old = h.hist_old;
  B.M.s0 = I.M.s0;
  B.M.s_inv = I.M.s_inv;
  EP_HIP(c, hipMemcpy(dptr<BatchInst>(c, c->o_batch_tab) + id, &B, sizeof(BatchInst), hipMemcpyHostToDevice));
  return EP_OK;
}

// Autotuner of the batch plan: times `steps` steps of the plain plan (one workgroup per
// instance), which also measures each instance's cost per step, then of the plans
// make_batch_plan builds from those costs for a few serial fractions; keeps the fastest.
// Every timing run starts from the same states (checkpoints) and the states are restored
// afterwards, so the call leaves the trajectory where it was.
ep_status ep_batch_autotune(ep_ctx* c, double dt, int steps, int* workgroups, double* ms_per_step) {
  if (!c) return EP_ERR_ARG;
  if (!c->bound || !c->batch) return fail(c, EP_ERR_ORDER, "needs a bound batch context");
  if (!(dt > 0.0) || !std::isfinite(dt) || steps < 1) return fail(c, EP_ERR_ARG, "need dt > 0 and steps >= 1");
  const int n = (int)c->insts.size();
  for (auto& I : c->insts)
    if (!I.state_set) return fail(c, EP_ERR_ORDER, "every instance needs a state");
  std::vector<std::vector<char>> img(n);
  for (int i = 0; i < n; ++i) {
    img[i].resize(ckpt_bytes(c, c->insts[i]));
    ep_status s = ep_batch_save_checkpoint(c, i, img[i].data(), img[i].size());
    if (s != EP_OK) return s;
  }
  auto restore = [&]() -> ep_status {
    for (int i = 0; i < n; ++i) {
      ep_status s = ep_batch_load_checkpoint(c, i, img[i].data(), img[i].size());
      if (s != EP_OK) return s;
    }
    return EP_OK;
  };
  hipEvent_t e0, e1;
  EP_HIP(c, hipEventCreate(&e0));
  EP_HIP(c, hipEventCreate(&e1));
  auto timed = [&](double* ms) -> ep_status {
    ep_status s = restore();
    if (s == EP_OK) s = ep_batch_step(c, dt, 1);                 // captures the plan's graph
    if (s == EP_OK) s = ep_sync(c);
    if (s != EP_OK) return s;
    EP_HIP(c, hipEventRecord(e0, c->stream));
    s = ep_batch_step(c, dt, steps);
    if (s != EP_OK) return s;
    EP_HIP(c, hipEventRecord(e1, c->stream));
    EP_HIP(c, hipEventSynchronize(e1));
    s = ep_sync(c);
    if (s != EP_OK) return s;
    float t = 0.0f;
    EP_HIP(c, hipEventElapsedTime(&t, e0, e1));
    *ms = (double)t / steps;
    return EP_OK;
  };
  ep_status s = EP_OK;
  std::vector<int> bestG(n, 1), G;
  std::vector<std::vector<int>> bestBins, bins;
  for (int i = 0; i < n; ++i) bestBins.push_back({i});
  double best = 0.0;
  std::vector<double> cost(n, 0.0);
  int cap = 0;
  do {
    s = apply_batch_plan(c, bestG, bestBins);
    if (s != EP_OK) break;
    // costs: ticks of the timed steps of the plain plan
    std::vector<Ctrl> h0(n), h1(n);
    s = restore();
    if (s != EP_OK) break;
    s = ep_batch_step(c, dt, 1);
    if (s == EP_OK) s = ep_sync(c);
    if (s != EP_OK) break;
    for (int i = 0; i < n; ++i) EP_HIP(c, hipMemcpy(&h0[i], c->insts[i].W.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    EP_HIP(c, hipEventRecord(e0, c->stream));
    s = ep_batch_step(c, dt, steps);
    if (s != EP_OK) break;
    EP_HIP(c, hipEventRecord(e1, c->stream));
    EP_HIP(c, hipEventSynchronize(e1));
    s = ep_sync(c);
    if (s != EP_OK) break;
    float t = 0.0f;
    EP_HIP(c, hipEventElapsedTime(&t, e0, e1));
    best = (double)t / steps;
    for (int i = 0; i < n; ++i) {
      EP_HIP(c, hipMemcpy(&h1[i], c->insts[i].W.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
      const long long ds = h1[i].ticked_steps - h0[i].ticked_steps;
      cost[i] = ds > 0 ? (double)(h1[i].ticks - h0[i].ticks) / (double)ds : 1.0;
    }
    s = batch_capacity(c, &cap);
    if (s != EP_OK) break;
    // three rounds: the plans of the plain plan's costs, then twice those of the costs
    // measured under the best plan so far (a fuller machine slows every instance down; a
    // team's time is converted back to one workgroup's through the same model)
    double best_sf = -1.0;
    for (int round = 0; round < 3 && s == EP_OK; ++round) {
      if (round >= 1) {
        if (best_sf < 0.0) break;
        s = apply_batch_plan(c, bestG, bestBins);
        if (s != EP_OK) break;
        s = restore();
        if (s == EP_OK) s = ep_batch_step(c, dt, 1);
        if (s == EP_OK) s = ep_sync(c);
        if (s != EP_OK) break;
        for (int i = 0; i < n; ++i) EP_HIP(c, hipMemcpy(&h0[i], c->insts[i].W.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        s = ep_batch_step(c, dt, steps);
        if (s == EP_OK) s = ep_sync(c);
        if (s != EP_OK) break;
        for (int i = 0; i < n; ++i) {
          EP_HIP(c, hipMemcpy(&h1[i], c->insts[i].W.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
          const long long ds = h1[i].ticked_steps - h0[i].ticked_steps;
          const double t = ds > 0 ? (double)(h1[i].ticks - h0[i].ticks) / (double)ds : cost[i];
          const int g = c->insts[i].W.G;
          cost[i] = t / (best_sf + (1.0 - best_sf) / g);
        }
      }
      for (double sf : {0.1, 0.2, 0.3, 0.4, 0.5, 0.65}) {
        make_batch_plan(c, cost, cap, sf, G, bins);
        s = apply_batch_plan(c, G, bins);
        if (s != EP_OK) break;
        double ms = 0.0;
        s = timed(&ms);
        if (s != EP_OK) break;
        if (ms < best) {
          best = ms;
          bestG = G;
          bestBins = bins;
          best_sf = sf;
        }
      }
    }
  } while (false);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != EP_OK) {
    // leave the batch as it was found: one workgroup per instance, the saved states (the
    // error stays the call's result)
    const std::string why = c->err;
    std::vector<int> g1(n, 1);
    std::vector<std::vector<int>> b1;
    for (int i = 0; i < n; ++i) b1.push_back({i});
    if (apply_batch_plan(c, g1, b1) == EP_OK) (void)restore();
    c->err = why;
    return s;
  }
  s = apply_batch_plan(c, bestG, bestBins);
  if (s == EP_OK) s = restore();
  if (s != EP_OK) return s;
  if (workgroups) {
    size_t w = 0;
    for (int k = 0; k < kModels; ++k) w += c->bwork[k].size();
    *workgroups = (int)w;
  }
  if (ms_per_step) *ms_per_step = best;
  return EP_OK;
}

ep_status ep_batch_get_time(ep_ctx* c, int32_t id, double* us_per_step, int64_t* steps) {
  ep_status s = need_batch(c, id);
  if (s != EP_OK) return s;
  EP_HIP(c, hipStreamSynchronize(c->stream));
  Ctrl h;
  EP_HIP(c, hipMemcpy(&h, c->insts[id].W.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
  int khz = 0;
  EP_HIP(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device));
  if (us_per_step) *us_per_step = (h.ticked_steps > 0 && khz > 0) ? 1e3 * (double)h.ticks / khz / h.ticked_steps : 0.0;
  if (steps) *steps = h.ticked_steps;
  return EP_OK;
}

ep_status ep_batch_get_stats(ep_ctx* c, int32_t id, int64_t* matvecs, int* last_m, int* last_k, double* last_eps,
                             int64_t* matvecs_pred, int* last_m_pred, int* last_k_pred) {
  ep_status s = need_batch(c, id);
  if (s != EP_OK) return s;
  EP_HIP(c, hipStreamSynchronize(c->stream));
  Ctrl h;
  EP_HIP(c, hipMemcpy(&h, c->insts[id].W.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
  if (matvecs) *matvecs = h.ks[0].matvecs + h.ks[1].matvecs;
  if (last_m) *last_m = h.ks[0].last_m;
  if (last_k) *last_k = h.ks[0].last_k;
  if (last_eps) *last_eps = h.ks[0].last_eps;
  if (matvecs_pred) *matvecs_pred = h.ks[1].matvecs;
  if (last_m_pred) *last_m_pred = h.ks[1].last_m;
  if (last_k_pred) *last_k_pred = h.ks[1].last_k;
  return EP_OK;
}

ep_status ep_batch_get_energy(ep_ctx* c, int32_t id, double* ke, double* se, double* we) {
  ep_status s = need_batch(c, id);
  if (s != EP_OK) return s;
  if (!ke || !se || !we) return fail(c, EP_ERR_ARG, "null output");
  EP_HIP(c, hipStreamSynchronize(c->stream));
  s = read_err(c, c->insts[id]);                 // this instance's failure only
  if (s != EP_OK) return s;
  s = pull_record(c, id);
  if (s != EP_OK) return s;
  Inst& I = c->insts[id];
  double* out = dptr<double>(c, I.o_eout);
  launch_energy(I.M, dptr<double>(c, I.o_S), c->btab[id].t, dptr<double>(c, I.o_pe), dptr<double>(c, I.o_pv), out,
                c->stream);
  EP_HIP(c, hipGetLastError());
  double h[3];
  EP_HIP(c, hipMemcpyAsync(h, out, 24, hipMemcpyDeviceToHost, c->stream));
  EP_HIP(c, hipStreamSynchronize(c->stream));
  *ke = h[0];
  *se = h[1];
  *we = h[2];
  return EP_OK;
}

}  // extern "C"
