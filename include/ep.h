/*
 * ep.h -- C ABI of the MI355X (gfx950) exponential time propagator for elastodynamics.
 *
 * Method: Pari, Kanungo & Gavini, "Exponential time propagators for elastodynamics".
 *   The finite-element semi-discrete system M u'' + H(u) u = P(t) (Sec. 2.2-2.3) is
 *   rewritten with ubar = M^{1/2} u as d/dt wbar = A wbar, wbar = [ubar; vbar; s],
 *   A = [[0, I, 0], [-M^{-1/2} H M^{-1/2}, 0, M^{-1/2} P / s0], [0, 0, 0]] (Sec. 2.3),
 *   advanced by wbar_n = exp(dt A(t_{n-1} + dt/2)) wbar_{n-1} (first Magnus term and the
 *   midpoint rule, Sec. 3.3 and 4.1) with a predictor-corrector for the nonlinear
 *   H at the midpoint (Sec. 4.2).  exp(dt A) wbar is evaluated by Arnoldi (modified
 *   Gram-Schmidt) with the subspace error estimate choosing the subspace size and
 *   exp(H_m) by Taylor with scaling and squaring (Sec. 4.3).
 *
 * Discretisation: 8-node hexahedra (VTK node order), 2x2x2 Gauss quadrature for the
 *   internal force, vertex (2-point Gauss-Lobatto) rule for a diagonal mass, 2x2 Gauss
 *   on loaded quad faces.  Nodal vectors are node-major doubles, DOF = 3*node + comp.
 *
 * Conventions for every function:
 *   - returns ep_status: EP_OK (0) or a negative code; never throws or aborts;
 *   - ep_last_error(ctx) describes the last failure (string owned by ctx, valid until
 *     the next call on ctx);
 *   - pointer arguments named *_host are host memory, copied during the call; the
 *     caller keeps ownership; *_dev arguments are device memory on the context's GPU;
 *   - a context is not thread-safe; calls on one context must be serialised;
 *   - device work is enqueued on the context's stream (ep_set_stream) and the calls
 *     that return data to the host synchronise that stream.
 */
#ifndef EP_H
#define EP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ep_ctx ep_ctx;

typedef enum {
  EP_OK = 0,
  EP_ERR_ARG = -1,        /* invalid argument (null pointer, size, range, value)          */
  EP_ERR_ORDER = -2,      /* call out of order (e.g. step before bind_workspace)          */
  EP_ERR_HIP = -3,        /* HIP runtime failure (launch, copy, no device)                */
  EP_ERR_KRYLOV = -4,     /* error estimate above tol at m_max after max_substeps splits  */
  EP_ERR_INVERTED = -5,   /* det J <= 0: inverted reference element or deformed state     */
  EP_ERR_NONFINITE = -6,  /* NaN / Inf reached the Krylov recurrence                      */
  EP_ERR_WORKSPACE = -7,  /* bound workspace too small or misaligned                      */
  EP_ERR_DEVICE = -8      /* device-side synchronisation timed out (kernel aborted)       */
} ep_status;

/* Material models and their parameter arrays (App. A of the paper; SI units):
 *   EP_LINEAR : {E, nu}                      linear elasticity, H = K constant
 *   EP_NH     : {mu, lambda}                 compressible Neo-Hookean,
 *               psi = mu/2 (I1 - 3) - mu ln J + lambda/2 (ln J)^2
 *   EP_YEOH   : {C10, C20, C30, D1}          Yeoh, psi = sum_k Ck0 (I1bar - 3)^k + (J-1)^2 / D1;
 *               C20 = C30 = 0 is the decoupled Neo-Hookean solid (mu = 2 C10, kappa = 2/D1)
 *   EP_SVK    : {lambda, mu}                 St. Venant-Kirchhoff, S = lambda tr(E) I + 2 mu E,
 *               E = (F^T F - I) / 2, psi = lambda/2 (tr E)^2 + mu E : E
 * H(u) is the H-matrix of App. A (R(u) = H(u) u exactly), applied matrix-free as
 *   (H(u) x)_A = sum_e sum_q w detJ Phi(grad u, X) . grad N_A,   X = grad x,
 * where Phi is the sum of App. A's printed blocks acting on X:
 *   EP_SVK  (App. A, St. Venant-Kirchhoff H-matrix):
 *     Phi = lambda ((I + D/2) : X) I + mu (X + X^T + (X^T D + D^T X)/2) + X S,  D = grad u;
 *   EP_YEOH (App. A, Yeoh H-matrix, each printed term with the 1/2 of the internal virtual
 *     work): Phi = alpha_e sym(X (F^{-1} + C^{-1})) + (W : X) C^{-1} + X S with
 *     W = -(alpha_e/3)(2I + D) + beta_e P_e, P_e the matrix with det F - 1 = P_e : D;
 *   EP_NH   (the same construction, App. A "trivially extended"): alpha_e -> mu,
 *     W = lambda (ln J / (J - 1)) P_e;
 * S is the model's second Piola-Kirchhoff stress at D and sym(Z) = (Z + Z^T)/2. */
typedef enum { EP_LINEAR = 0, EP_NH = 1, EP_YEOH = 2, EP_SVK = 3 } ep_model;

/* Arithmetic of the operator apply (stiffness matvec).  The Krylov recurrence, error
 * estimate, Hessenberg exponential and state are FP64 in every mode.
 *   EP_PREC_F64        : matvec in FP64
 *   EP_PREC_MIXED_F32  : element kernels in FP32 with FP32 accumulation; converted at the
 *                        FP64 Krylov vector boundary.
 *   EP_PREC_MIXED_BF16 : element tangents (the element matrices of the operator's H, Sec. 2.3
 *                        with the H-matrix of App. A) formed once per projection with
 *                        BF16 matrix-core products and FP32 accumulation, stored in BF16
 *                        (1152 bytes per element); every apply computes K_e x_e in FP32 with
 *                        FP32 accumulation.  Needs a congruent mesh (every element a
 *                        translate of element 0; EP_ERR_ARG at ep_bind_workspace otherwise),
 *                        must be set before ep_bind_workspace, not available for batches.
 *                        BF16 keeps 8 significant bits: operator and trajectory errors are of
 *                        order 1e-3 relative (measured values are stated with the tests). */
typedef enum { EP_PREC_F64 = 0, EP_PREC_MIXED_F32 = 1, EP_PREC_MIXED_BF16 = 2 } ep_precision;

/* ------------------------------------------------------------------ lifetime */

/* Create a context on HIP device `hip_device` (>= 0).  hip_device = -1 creates a
 * host-only context that validates arguments and sizes but can never launch work. */
ep_status ep_create(ep_ctx** out, int hip_device);
ep_status ep_destroy(ep_ctx* ctx);
const char* ep_last_error(const ep_ctx* ctx);
/* Library version string (static storage). */
const char* ep_version(void);

/* Stream for all device work (a hipStream_t; NULL = the default stream). */
ep_status ep_set_stream(ep_ctx* ctx, void* hip_stream);

/* ------------------------------------------------------------------ problem setup
 * Setup calls must precede ep_bind_workspace; calling one after it returns EP_ERR_ORDER. */

/* Mesh: n_nodes reference coordinates xyz_host[3*n_nodes] (m) and n_elems hex8 cells
 * conn_host[8*n_elems] (0-based node ids, VTK order).  Sec. 2.2 (finite elements). */
ep_status ep_set_mesh_hex8(ep_ctx* ctx, int64_t n_nodes, const double* xyz_host,
                           int64_t n_elems, const int32_t* conn_host);

/* Mesh of quadratic 27-node hexahedra, the paper's element (Sec. 2.2: quadratic Lagrange
 * interpolation; 3x3x3 Gauss for the internal force, the 3-point Gauss-Lobatto rule at the
 * nodes for a diagonal mass).  conn_host[27*n_elems]: local node a = i + 3 j + 9 k at the
 * local point (i-1, j-1, k-1).  Loaded faces (ep_set_traction) then list 9 nodes each,
 * p + 3 q at (p-1, q-1) with the outward normal along d/dp x d/dq; 3x3 Gauss.  Single-instance
 * contexts, EP_PREC_F64 or EP_PREC_MIXED_F32, second-order scheme (EP_ERR_ARG otherwise, at
 * ep_bind_workspace). */
ep_status ep_set_mesh_hex27(ep_ctx* ctx, int64_t n_nodes, const double* xyz_host,
                            int64_t n_elems, const int32_t* conn_host);

/* Material (see ep_model) and reference density rho (kg/m^3). */
ep_status ep_set_material(ep_ctx* ctx, ep_model model, const double* params_host,
                          int n_params, double rho);

/* Homogeneous Dirichlet DOFs (u = v = 0 for all t): dof ids 3*node + comp.  Duplicates
 * are allowed.  The clamped DOFs are eliminated from the system (held at zero). */
ep_status ep_set_dirichlet(ep_ctx* ctx, int64_t n_dofs, const int32_t* dof_ids_host);

/* Dead traction t(t) = scale(t) * t0 on quad faces face_nodes_host[4*n_faces] (9 per face
 * on a mesh of quadratic hexahedra)
 * (weak-form term 3, Sec. 2.2).  scale(t) is piecewise linear through the n_knots
 * pairs (t_knots, scale), held constant before the first and after the last knot;
 * t_knots must be ascending.  n_faces = 0 means no load. */
ep_status ep_set_traction(ep_ctx* ctx, int64_t n_faces, const int32_t* face_nodes_host,
                          const double t0_host[3], int64_t n_knots, const double* t_knots_host,
                          const double* scale_host);

/* Krylov controls (Sec. 4.3).  tol: stop when eps_m <= tol * ||wbar||; m_max: largest
 * subspace (<= 256); check_every: evaluate eps every this many Arnoldi steps (not
 * before the size that sufficed on the previous call minus check_every); m_fixed > 0:
 * exactly m_fixed steps (the paper's fixed-m production mode, Sec. 6.2); k_fixed > 0:
 * exactly k_fixed substeps; max_substeps: unconverged projections are redone with
 * 2, 4, ... substeps of the same frozen operator up to this count, then EP_ERR_KRYLOV.
 * s0: value of the augmented entry of wbar.  EP_S0_AUTO (or any other negative value except
 * EP_S0_SCALED): 1 with a load, 0 without, which is the paper's 2N form for P = 0.
 * EP_S0_SCALED: the entry at the problem's own scale, s0 = max(||[ubar; vbar]||_2,
 * dt ||Pbar_0||_2 max_k |scale_k|), fixed per instance at the first ep_step / ep_batch_step
 * after its state is set (0 without a load).  The exact propagation does not depend on s0
 * (A's last column is Pbar / s0); the stopping rule does, since ||wbar|| includes s0: with
 * s0 = 1 and a state far below 1 in SI units the Krylov error is not small relative to the
 * state.  s0 >= 0: that value. */
#define EP_S0_AUTO (-1.0)
#define EP_S0_SCALED (-2.0)
ep_status ep_set_krylov(ep_ctx* ctx, double tol, int m_max, int check_every, int m_fixed,
                        int k_fixed, int max_substeps, double s0);

ep_status ep_set_precision(ep_ctx* ctx, ep_precision prec);

/* Time integrator (before ep_bind_workspace; single-instance contexts):
 *   2 (default): the paper's second-order step, the Magnus series truncated after its first
 *     term at the step midpoint, with the predictor-corrector of Sec. 4.2 for nonlinear H;
 *   4: the series truncated after two terms (Sec. 3.3 remark), the two-point Gauss-Legendre
 *     rule at t + (1/2 -+ sqrt(3)/6) dt: Omega = dt/2 (A_1 + A_2) - sqrt(3) dt^2/12 [A_1, A_2],
 *     one Krylov projection of exp(Omega) wbar per step, each Arnoldi step applying both
 *     H-matrices to the u- and v-parts of the vector; H at the displacements predicted for the
 *     nodes by cubic Hermite extrapolation of this and the previous step's start state (first
 *     step after ep_set_state: u + s v + s^2/2 M^{-1}(P - R(u))).  Fourth order in dt.
 * EP_ERR_ARG for another order, and at ep_bind_workspace for a batch, EP_PREC_MIXED_BF16, or a
 * team whose Krylov slices do not fit in LDS. */
ep_status ep_set_scheme(ep_ctx* ctx, int order);

/* Form of the Arnoldi modified Gram-Schmidt loop (Sec. 4.3) in the single-instance kernel,
 * set before ep_bind_workspace.  mode 0: sequential, one team reduction per inner
 * product (j + 1 in step j).  mode 1: compact WY, the same recurrence written as the
 * triangular solve (I + L_j) h = V_j^T w with L_j the strictly lower triangle of V_j^T V_j;
 * one vector reduction of the 2j - 1 inner products plus the norm per step; needs
 * m_max <= 64 (else EP_ERR_ARG at ep_workspace_size / ep_bind_workspace).  mode -1
 * (default): 1 when m_max <= 64, else 0.  Batches always use mode 0.  Both forms give the same H and V up to rounding. */
ep_status ep_set_orthogonalization(ep_ctx* ctx, int mode);
/* The form in effect (after binding) or that binding would choose. */
ep_status ep_get_orthogonalization(ep_ctx* ctx, int* mode);

/* Number of workgroups of the persistent Krylov kernel (0 = automatic). */
ep_status ep_set_launch(ep_ctx* ctx, int workgroups);

/* Autotuner of the persistent Krylov kernel's launch: after ep_set_state, times `trials`
 * fixed-size projections (m_trial Arnoldi steps of dt * A at the current state) for every
 * feasible workgroup count (LDS slice and co-residency limits) and keeps the fastest for
 * this context.  Reports the choice and its time per projection (ms).  Uses only scratch
 * memory; the state is unchanged. */
ep_status ep_autotune(ep_ctx* ctx, double dt, int m_trial, int trials, int* best_workgroups,
                      double* best_ms);

/* ------------------------------------------------------------------ workspace
 * All device memory is caller-owned: query the size, allocate (e.g. a torch uint8
 * tensor), bind.  The library never allocates or frees device memory itself.
 * Binding uploads the setup data and runs the setup kernels (geometry, lumped mass,
 * loads; Sec. 2.2).  The pointer must be 256-byte aligned and stay valid until
 * ep_destroy.  An inverted reference element gives EP_ERR_INVERTED. */
ep_status ep_workspace_size(ep_ctx* ctx, size_t* bytes);
ep_status ep_bind_workspace(ep_ctx* ctx, void* dev_ptr, size_t bytes);

/* ------------------------------------------------------------------ state and stepping */

/* Set time t and nodal displacement / velocity (u_host, v_host: 3*n_nodes doubles;
 * clamped entries are ignored).  Clears the predictor history and the sticky error. */
ep_status ep_set_state(ep_ctx* ctx, double t, const double* u_host, const double* v_host);

/* Advance n_steps steps of size dt (asynchronous on the stream).  Linear: one
 * propagation per step; nonlinear: predictor (dt/2) and corrector (dt).  Device-side
 * failures are sticky and reported by the next synchronising call. */
ep_status ep_step(ep_ctx* ctx, double dt, int64_t n_steps);

/* Wait for the stream; returns the sticky device error, if any. */
ep_status ep_sync(ep_ctx* ctx);

/* Synchronising reads.  u_host / v_host: 3*n_nodes doubles (clamped entries 0). */
ep_status ep_get_state(ep_ctx* ctx, double* t, double* u_host, double* v_host);

/* Checkpoint and resume.  A checkpoint is an opaque host image of the whole stepping state
 * (Sec. 4.1-4.2: what the next step reads): t and the step count, the augmented state
 * vector as held on the device (ubar = M^{1/2} u, vbar, s; not re-derived from u and v, so
 * nothing is rounded), the predictor's midpoint displacements and which of them the next
 * predictor extrapolates from, the adaptive Krylov state (sticky substep counts, subspace
 * hints), the resolved augmented entry s0 and, for the fourth-order scheme, the previous
 * step's start state.  ep_checkpoint_size gives the byte count (fixed for a bound
 * context); ep_save_checkpoint fills a caller-owned host buffer of exactly that size
 * (synchronising; fails with the sticky device error if one is pending, EP_ERR_ORDER
 * before a state is set); ep_load_checkpoint restores it into this or another context bound
 * for the same mesh size, element family, material model, precision and scheme (EP_ERR_ARG
 * otherwise, and on a corrupt header) and clears the sticky error.  Steps after a load
 * reproduce, bit for bit, the steps the saving context takes from the same point when both
 * contexts run with the same team size (ep_get_launch); another team size sums the
 * reductions in another order (results equal to rounding). */
ep_status ep_checkpoint_size(ep_ctx* ctx, size_t* bytes);
ep_status ep_save_checkpoint(ep_ctx* ctx, void* buf_host, size_t bytes);
ep_status ep_load_checkpoint(ep_ctx* ctx, const void* buf_host, size_t bytes);

/* Energies at the current state (Sec. 5.2 generalised): kinetic 1/2 v^T M v, strain
 * sum_e sum_q w detJ psi(F), and the work of the current load P(t)^T u. */
ep_status ep_get_energy(ep_ctx* ctx, double* kinetic, double* strain, double* ext_work);

/* Statistics: total operator applications since ep_set_state, and for the last step
 * the subspace size and estimate of its last corrector projection, its substep count,
 * and |s - s0| before the reset of the augmented entry. */
ep_status ep_get_stats(ep_ctx* ctx, int64_t* matvecs, int* last_m, double* last_eps,
                       int* last_k, double* aug_drift);

/* Launch layout of the persistent Krylov kernel after binding (or autotuning): the
 * number of workgroups, the Krylov-vector entries each owns, whether those slices live in
 * device memory (1; meshes too large for them to fit in LDS with one workgroup per
 * compute unit, or a forced small team) or in LDS (0), and whether the mesh was found
 * congruent (every element a translate of element 0: J^{-1} and det J agree to 1e-13 at
 * every quadrature point), which selects the stored-element-stiffness path of the
 * linear-elastic operator.  Null outputs are skipped. */
ep_status ep_get_launch(ep_ctx* ctx, int* workgroups, int* chunk, int* slices_global, int* congruent);
/* (congruent: 0 general mesh, 1 congruent, 2 congruent lattice -- node (i, j, k) numbered
 * i + (nx+1)(j + (ny+1)k), elements i-fastest, VTK corner order -- whose FP64 linear
 * operator apply (ep_apply_H) runs as a 27-block stencil over LDS tiles) */

/* Per-step log of the last n steps (n <= 4096): m of the corrector and predictor
 * projections (first substep), substep counts and eps.  Arrays of length n. */
ep_status ep_get_step_log(ep_ctx* ctx, int n, int32_t* m_corr, int32_t* m_pred,
                          int32_t* k_corr, double* eps_corr);

/* ------------------------------------------------------------------ stage entry points
 * Single stages of the path on device memory of this context's GPU, for checking and
 * timing.  They use the bound workspace; they do not change the stepping state except
 * where stated. */

/* y = H(u_lin) x on all 3*n_nodes DOFs (rows and columns of clamped DOFs included;
 * u_lin = NULL means u = 0, i.e. the linear-elastic stiffness).  x_dev, y_dev, u_lin_dev:
 * 3*n_nodes doubles.  Weak-form term 2 (Sec. 2.2) with the H-matrix of App. A.
 * Enqueued on the context's stream without waiting; an inverted element (secant
 * materials) is reported by the next ep_sync.  FP64 linear elasticity on a congruent mesh
 * runs as one node-by-node pass with the stored element stiffness. */
ep_status ep_apply_H(ep_ctx* ctx, const double* u_lin_dev, const double* x_dev, double* y_dev);

/* EP_PREC_MIXED_BF16 contexts: form the stored BF16 element tangents of H(u_lin) (u_lin_dev:
 * 3*n_nodes doubles on the device, NULL = rest state), the H formation of the predictor and
 * corrector operators (Sec. 4.2, App. A) as one stage, for checking and timing.  ep_apply_H
 * and the stepping calls form the tangents they need themselves.  Enqueued without waiting;
 * det F <= 0 is reported by the next ep_sync.  EP_ERR_ORDER in the other modes. */
ep_status ep_form_tangents(ep_ctx* ctx, const double* u_lin_dev);

/* y = tau * A x with A the augmented first-order matrix (Sec. 2.3) at load scale
 * `pscale`, u_lin as in ep_apply_H.  x_dev, y_dev: vectors of ep_vector_length() doubles
 * in the library's layout [ubar (3 n_nodes) | vbar (3 n_nodes) | s | padding]. */
ep_status ep_apply_A(ep_ctx* ctx, const double* u_lin_dev, double tau, double pscale,
                     const double* x_dev, double* y_dev);
ep_status ep_vector_length(ep_ctx* ctx, int64_t* length, int64_t* padded_length);

/* E = exp(H) for a dense m x m row-major matrix (m <= 256) on one workgroup:
 * degree-18 Taylor polynomial, applied to H / 2^s and squared s times when ||H||_1 > 1
 * (Sec. 4.3).  Host arrays. */
ep_status ep_expm(ep_ctx* ctx, int m, const double* H_host, double* E_host);

/* Allocation-free variant of ep_expm, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): E = exp(H)
 * for a dense m x m row-major FP64 matrix in device memory of the current HIP device, the
 * same kernel and result as ep_expm.  No context is needed.
 *   m:          1 <= m <= 256, else EP_ERR_ARG (the scratch is sized for m = 256);
 *   H_dev:      m*m doubles, read only; E_dev: m*m doubles, written (must not overlap H_dev);
 *   hip_stream: stream of the current device (NULL: the null stream); enqueued without
 *               waiting.
 * Scratch: up to 6 m (m+1) doubles (3,158,016 bytes at m = 256) in a library-owned device
 * array, one per GPU, held until the process ends; no hipMalloc/hipFree or allocating
 * library call is made.  Every call on a GPU shares that GPU's array, so calls that overlap
 * on one GPU (different streams, or host threads) race: order them on one stream.
 * EP_ERR_HIP if the scratch address cannot be resolved or the launch fails. */
ep_status ep_expm_noalloc(int m, const double* H_dev, double* E_dev, void* hip_stream);

/* m Arnoldi steps with modified Gram-Schmidt (Sec. 4.3) on tau * A (as ep_apply_A) from
 * w_dev.  Writes V (m+1 rows of padded_length doubles, device) and the Hessenberg
 * Htilde ((m+1) x m row-major, host).  Returns the number of completed steps in
 * *steps (< m on breakdown). */
ep_status ep_arnoldi(ep_ctx* ctx, const double* u_lin_dev, double tau, double pscale,
                     const double* w_dev, int m, double* V_dev, double* H_host, int* steps);

/* y = exp(tau A) w (one adaptive projection with substeps, Sec. 4.3) on device vectors
 * of the library layout; reports the subspace size, substeps and estimate. */
ep_status ep_expv(ep_ctx* ctx, const double* u_lin_dev, double tau, double pscale,
                  const double* w_dev, double* y_dev, int* m_used, int* k_used, double* eps);

/* ------------------------------------------------------------------ batches
 * A batch context advances many independent instances (own mesh, material, loads and
 * state) together: every instance's projections run inside one persistent launch per
 * step (per material model), each instance with its own subspace size, on a workgroup of
 * its own (at binding), in a list of instances one workgroup steps one after the other, or
 * on a team of workgroups (see ep_batch_plan).  Instances are
 * added after ep_create and before ep_bind_workspace; the single-instance setup calls
 * are then not used.  The Krylov / precision settings apply to all instances.
 * Device-side failures are per instance: a failed instance stops advancing while the
 * others go on; its ep_batch_get_state / ep_batch_get_energy return the error (sticky),
 * ep_sync returns the first failed instance's, and ep_batch_set_state clears it. */
/* Add one instance (Sec. 2.2 setup): the arguments are those of ep_set_mesh_hex8,
 * ep_set_material, ep_set_dirichlet and ep_set_traction in that order (host arrays, copied
 * at the call).  *instance_id receives its index; ids are consecutive from 0. */
ep_status ep_batch_add_instance(ep_ctx* ctx, int64_t n_nodes, const double* xyz_host,
                                int64_t n_elems, const int32_t* conn_host, ep_model model,
                                const double* params_host, int n_params, double rho,
                                int64_t n_dirichlet, const int32_t* dof_ids_host,
                                int64_t n_faces, const int32_t* face_nodes_host,
                                const double t0_host[3], int64_t n_knots,
                                const double* t_knots_host, const double* scale_host,
                                int32_t* instance_id);
/* As ep_set_state, for one instance: also clears its predictor history and its failure. */
ep_status ep_batch_set_state(ep_ctx* ctx, int32_t instance_id, double t, const double* u_host,
                             const double* v_host);
/* Advance every instance n_steps steps of size dt (linear instances: one propagation per
 * step; nonlinear: predictor and corrector, Sec. 4.2).  One step is one persistent launch
 * per material model present, captured into a graph on the first call with this dt and
 * replayed n_steps times on the context's stream (asynchronous); every instance needs a
 * state first (EP_ERR_ORDER). */
ep_status ep_batch_step(ep_ctx* ctx, double dt, int64_t n_steps);
/* As ep_get_state, for one instance (synchronising; returns that instance's failure only). */
ep_status ep_batch_get_state(ep_ctx* ctx, int32_t instance_id, double* t, double* u_host,
                             double* v_host);
/* Per-instance statistics (synchronising): operator applies so far (both kinds), the last
 * corrector (or linear) projection's m, substeps and error estimate, and - for the
 * predictor projections of a nonlinear instance - their applies so far, last m and
 * substeps (0 for a linear instance).  Any output may be NULL. */
ep_status ep_batch_get_stats(ep_ctx* ctx, int32_t instance_id, int64_t* matvecs, int* last_m,
                             int* last_k, double* last_eps, int64_t* matvecs_pred, int* last_m_pred,
                             int* last_k_pred);
/* Launch plan of a batch (the batched form of the workload definition, with its
 * autotuned tiles).  One step is one launch per material model; each of its workgroups
 * either steps a list of instances one after the other or is one member of a team of up
 * to 8 workgroups that steps one instance together (Krylov slices split over the team,
 * its reductions through device memory with bounded waits: a team whose members are not
 * all resident records EP_ERR_DEVICE instead of hanging).  The step lasts as long as its
 * longest workgroup.
 * At binding every instance has a workgroup of its own.  ep_batch_plan re-plans, modelling a
 * team of G workgroups to step an instance of cost c in c (serial + (1 - serial) / G) (serial
 * in [0, 1): the part of a step a team does not divide - synchronisation, check points):
 * instances whose cost exceeds a target T get the smallest team that meets it, the others
 * are packed first-fit-decreasing into lists of cost <= T, and T is the smallest target whose
 * plan needs at most max_workgroups workgroups (<= 0: as many as can be resident together on
 * this GPU) per launch.  The cost of an instance is its measured wall-clock time per step
 * when every instance has stepped since its state was set, else its element count plus a
 * tenth of its Krylov-vector length.  Results of an instance depend on its team size at
 * rounding level (reductions in another order).
 * ep_batch_autotune times `steps` steps of dt (after one untimed step) for the one-
 * workgroup-per-instance plan, which measures the costs, and for the plans of serial
 * fractions 0.1, 0.2, 0.3, 0.4, 0.5 and 0.65; then, twice, re-measures the costs under the
 * fastest plan so far (team times converted back through the model) and times the six plans
 * of those costs; each run starts from the same states.  Keeps the fastest plan and restores the states
 * (checkpoints), so the trajectory is where it was; outputs the workgroups per launch and
 * the time per step of the kept plan (either may be NULL).  On a failure (a device error in
 * a timing run) it returns that error after putting back one workgroup per instance and
 * the saved states.
 * ep_batch_get_plan: the team size of instance instance_id (1: a list member) and the total
 * workgroups of the current plan (either may be NULL; instance_id < 0 skips the first). */
ep_status ep_batch_plan(ep_ctx* ctx, int max_workgroups, double serial);
ep_status ep_batch_autotune(ep_ctx* ctx, double dt, int steps, int* workgroups, double* ms_per_step);
ep_status ep_batch_get_plan(ep_ctx* ctx, int32_t instance_id, int* team, int* workgroups);
/* Device wall-clock time per step of one instance (its workgroup's, or its team's first
 * member's, time from the start of its first step in a launch to the end of its last),
 * averaged over the steps since its state was set (synchronising; either output may be
 * NULL).  The plan's costs; a list's members run one after the other. */
ep_status ep_batch_get_time(ep_ctx* ctx, int32_t instance_id, double* us_per_step, int64_t* steps);
/* Checkpoints of one instance, as ep_checkpoint_size / ep_save_checkpoint /
 * ep_load_checkpoint (the save synchronises and returns that instance's failure only; a
 * load needs a batch instance of the same sizes, material, precision). */
ep_status ep_batch_checkpoint_size(ep_ctx* ctx, int32_t instance_id, size_t* bytes);
ep_status ep_batch_save_checkpoint(ep_ctx* ctx, int32_t instance_id, void* buf_host, size_t bytes);
ep_status ep_batch_load_checkpoint(ep_ctx* ctx, int32_t instance_id, const void* buf_host,
                                   size_t bytes);
/* Per-instance energies, as ep_get_energy. */
ep_status ep_batch_get_energy(ep_ctx* ctx, int32_t instance_id, double* kinetic, double* strain,
                              double* ext_work);

#ifdef __cplusplus
}
#endif

#endif /* EP_H */
