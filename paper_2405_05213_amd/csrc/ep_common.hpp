// Shared host/device definitions of the MI355X exponential-propagator library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ep {

constexpr int kThreads = 512;        // workgroup size of the batch, expm and element kernels
constexpr int kExpvThreads = 512;    // workgroup size of the persistent projection kernel (256
                                     // removes its scratch spills, one wave per SIMD, but is
                                     // slower on every single-instance workload)
constexpr int kMaxM = 256;           // largest Krylov subspace
constexpr int kLogSteps = 4096;      // per-step statistics ring
constexpr int kMaxKnots = 4096;
constexpr int kMaxCwyM = 64;         // largest subspace of the compact-WY orthogonalisation
constexpr int kRing = 8;
constexpr int kKeLd = 25;            // row stride of the stored element stiffness             // rounds of all-reduce slots of a workgroup team

// stored BF16 element tangents (ep_tangent.hpp): Psi has 72 (q, j, l) columns padded to
// 5 K-steps of 16; tangents are stored in groups of 8 elements of 9 x 64 x 8 values
constexpr int kPsiK = 80;
constexpr int kPsiSteps = kPsiK / 16;
constexpr int kPsiValues = 4 * kPsiSteps * 64 * 4;
constexpr int kKstGroup = 9 * 64 * 8;
__host__ __device__ inline size_t kst_values(long long n_e) { return (size_t)((n_e + 7) / 8) * kKstGroup; }

// material ids (ep_model); kStored selects the operator kernels that apply stored element
// tangents (any material, formed beforehand)
constexpr int kLinear = 0, kNH = 1, kYeoh = 2, kSVK = 3, kStored = 4;
constexpr int kModels = 4;

// sticky device error codes (match ep_status)
constexpr int kErrKrylov = -4, kErrInverted = -5, kErrNonfinite = -6, kErrDevice = -8;

// Device view of one mesh instance.  All vectors are node-major doubles; the Krylov
// vector layout is [ubar (n3) | vbar (n3) | s | zero padding up to Lp].
struct Mesh {
  int n_nodes, n_elems, n3;
  int npe;                    // nodes (and Gauss points) per element: 8 (hex8) or 27 (Q2)
  int L, Lp;                  // L = 2*n3 + 1, Lp = padded row stride of V
  const int* conn;            // [n_elems*8]
  const int* inc_ptr;         // [n_nodes+1] node -> element-slot CSR
  const int* inc;             // slot ids a*n_elems + e
  const double* geo;          // per quadrature point: Jinv (3x3 row major) + w*detJ
  const float* geo32;
  int congruent;              // 1: one geometry set shared by all elements
  int jdiag;                  // 1: congruent hex8 mesh whose Gauss-point J^{-1} are diagonal
                              // (axis-aligned boxes; off-diagonals are rounding residue)
  const double* ke;           // congruent meshes: rest-state element stiffness (24 x kKeLd),
                              // null otherwise
  int lat[3];                 // congruent lattice (node i + (nx+1)(j + (ny+1)k), VTK order):
                              // nx, ny, nz; zeros otherwise
  const double* stencil;      // lattice: the 27 3x3 blocks of an interior node's rows of K
  const uint16_t* kst;        // BF16 element tangents of the current operator (groups of 8
                              // elements, see ep_tangent.hpp), null unless that mode is bound
  const double* mih;          // M^{-1/2} per DOF (0 on clamped DOFs)
  const double* mh;           // M^{1/2}  per DOF (0 on clamped DOFs)
  const double* p0bar;        // M^{-1/2} P0 per DOF (0 on clamped DOFs)
  const double* p0;           // P0 per DOF
  const double* knots;        // [2*n_knots]: times then scales
  int n_knots;
  int model;
  double mp[4];               // linear (E, nu) | nh (mu, lambda) | yeoh (C10, C20, C30, D1) |
                              // svk (lambda, mu)
  double s0, s_inv;           // augmented entry value and 1/s0 (0 when s0 == 0)
};

// Operator tau * A[H(u_lin), pbar(t)] of the augmented first-order system.
struct OpArgs {
  double tau;                 // time-step factor (dt / substeps)
  double t_eval;              // time at which the load scale is evaluated
  int nsets;                  // 0: H(0) (linear-elastic or rest state); 1 or 2 secant sets
  const double* ulin[2];      // physical nodal displacements of the secant sets
  double wts[2];              // weights of the sets (predictor: 1.75, -0.75)
  // fourth-order scheme (kernels instantiated with SCH = 4): the operator is
  // Omega = dt/2 (A_1 + A_2) - c4 [A_1, A_2], A_i with the set i and the load at t_eval
  // (i = 1) or t_eval2 (i = 2); tau = 1
  double dt4, c4, t_eval2;
};

struct KrylovCfg {
  double tol;
  int m_max, check_every, m_fixed, k_fixed, max_substeps;
  int prec;                   // 0 FP64, 1 FP32 element kernels, 2 stored BF16 element tangents
  int ortho;                  // 0: one team reduction per projection (sequential MGS);
                              // 1: MGS in compact-WY form, one vector reduction per step
  int scheme;                 // time integrator: 2 (0 = 2) the paper's midpoint Magnus step with
                              // predictor-corrector, 4 the two-term (fourth-order) Magnus step
};

// Per-projection-kind adaptive state (kept on device between launches).
struct KState {
  int k;                      // sticky substep count
  int m_hint;                 // last converged subspace size
  int last_m, last_k;
  double last_eps;
  long long matvecs;
};

// Device control block of one instance.
struct Ctrl {
  unsigned long long bar;     // grid barrier arrivals (zeroed before every launch)
  int err;                    // sticky error
  int pad0;
  int decision;               // broadcast from workgroup 0
  int pad1;
  double bcast[4];
  KState ks[3];               // 0 = corrector / linear, 1 = predictor, 2 = stage calls
  int log_pos;
  int pad2;
  double drift;
  unsigned long long ticks;   // batch: wall-clock ticks of this instance's steps (its team's rank 0)
  long long ticked_steps;     // steps those ticks cover
};

struct StepLog {
  int m_corr[kLogSteps];
  int m_pred[kLogSteps];
  int k_corr[kLogSteps];
  double eps_corr[kLogSteps];
};

// Scratch of the persistent Krylov kernel for one instance.
struct KWork {
  double* V;                  // (m_max+1) x Lp
  double* Wun;                // Lp: unnormalised Arnoldi vector
  double* X;                  // Lp: propagated vector
  double* F;                  // 24*n_elems element forces (slot-major)
  float* F32;
  double* F2;                 // second slot array of the fourth-order scheme (u-part forces)
  float* F2_32;
  unsigned long long* flags;  // G barrier generations
  unsigned long long* ring;   // 8 * G all-reduce slots
  unsigned long long* vring;  // 8 * G * vw vector all-reduce slots (compact-WY MGS)
  int vw;                     // row width of a vector slot (2 * m_max)
  double* H;                  // (m_max+1) x m_max Hessenberg (row major, stride m_max)
  double* Escr;               // expm scratch 8 * m_max^2 (+ m_max^2 output staging)
  double* y;                  // m_max coefficients
  Ctrl* ctrl;
  StepLog* log;
  int G;                      // workgroups of the team
  int chunk;                  // Krylov-vector entries owned by each workgroup
  double* wscr;               // 2 * Lp: slice buffers in device memory when they exceed LDS
  int ex_cap;                 // doubles of LDS the check point may use for exp(H) (set per launch)
  int slices_global;          // 1: the slice buffers live in wscr instead of LDS
};

// Device-side record of one instance of a batch: the stepping state lives on the device so
// that one step is a fixed launch (replayable from a captured graph).
struct BatchInst {
  Mesh M;
  KWork W;
  double* S;                  // wbar (Lp)
  double* hist;               // 3 * n3 midpoint displacements
  double t;
  long long step_idx;
  int nhist, hist_new, hist_old;
  int use_lds;                // slices of w and the newest basis vector in LDS (1), w's only (2:
                              // the basis vector is read from V), or w's in W.wscr (0)
};

// Work of one workgroup of a batch launch: member `rank` of a team of G > 1 workgroups that
// steps instance `inst` together, or (G == 1) the `count` instances ids[first ..] stepped one
// after the other.
struct BatchWork {
  int inst, rank, G, first, count;
};

// Largest team of a batch instance (its barrier flags and all-reduce ring are sized for it).
constexpr int kBatchGmax = 8;

// One launch of the persistent projection kernel: wbar_out = exp(tau A) wbar_in.
struct ExpvArgs {
  Mesh M;
  KWork W;
  KrylovCfg cfg;
  OpArgs op;
  int kind;                   // 0: corrector (or linear step), 1: predictor, 2: stage call
  const double* x_in;         // Lp doubles
  double* x_out;              // out_mode 0: Lp doubles, augmented entry reset to s0 (drift
                              // recorded); 1: n3 doubles of M^{-1/2} ubar; 2: Lp doubles as is
  int out_mode;
  int log_idx;                // step-log slot (-1: none)
};

}  // namespace ep
