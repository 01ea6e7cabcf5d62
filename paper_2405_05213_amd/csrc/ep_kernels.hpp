// Host-side launch wrappers of the kernels in ep_kernels.hip / ep_batch.hip.
#pragma once

#include "ep_common.hpp"

namespace ep {

size_t expv_lds_bytes(int chunk, int ortho, int m_max, int sg);
size_t expv_lds_head_bytes(int ortho, int m_max);
void launch_stiffness(const Mesh& M, double* Ke, hipStream_t st);
void launch_stencil_blocks(const double* Ke, double* B, hipStream_t st);
hipError_t expv_max_blocks(const KrylovCfg& cfg, int model, int npe, int chunk, int sg, int* blocks_per_cu);
const void* expv_kernel_global(int prec, int model, int ortho);
const void* expv_kernel_m4(int prec, int model, int ortho);
hipError_t launch_expv(const ExpvArgs& a, int prec, hipStream_t st);

void launch_geometry(const double* xyz, const int* conn, int n_e, int npe, double* geo, float* geo32, double* vdet,
                     int* bad,
                     hipStream_t st);
void launch_congruence(const double* geo, int n_e, int npe, double tol, int* mismatch, hipStream_t st);
void launch_mass(int n_nodes, int n_e, int npe, const int* inc_ptr, const int* inc, const double* vdet, double rho,
                 const unsigned char* clamp, double* mih, double* mh, hipStream_t st);
void launch_faces(const double* xyz, const int* faces, int n_f, int nfn, const double* t0, double* ff, int n_nodes,
                  const int* finc_ptr, const int* finc, const double* mih, double* p0, double* p0bar, hipStream_t st);
void launch_set_state(int n3, int Lp, const double* mh, const double* u, const double* v, double s0, double* S,
                      hipStream_t st);
void launch_get_state(int n3, const double* mih, const double* S, double* u, double* v, hipStream_t st);
void launch_reset_ctrl(Ctrl* c, hipStream_t st);
void launch_apply_H(const Mesh& M, const OpArgs& op, int prec, const double* x, double* y, double* F, float* F32,
                    int* err, hipStream_t st);
void launch_apply_A(const Mesh& M, const OpArgs& op, int prec, const double* x, double* y, double* F, float* F32,
                    int* err, hipStream_t st);
void launch_expm(int m, const double* H, double* E, double* scr, hipStream_t st);
void launch_m4_predict(const Mesh& M, const double* S, const double* Sprev, const double* R, double pscale_t,
                       double t, double t_prev, double tau1, double tau2, int first, double* u1, double* u2,
                       hipStream_t st);
// stored BF16 element tangents (ep_tangent.hip)
void launch_psi(const Mesh& M, uint16_t* psi, hipStream_t st);
void launch_form_tangent(const Mesh& M, const OpArgs& op, const uint16_t* psi, uint16_t* kst, int* err,
                         hipStream_t st);
void launch_elem_forces_kst(const Mesh& M, const double* src, double sc, int scale_mih, float* F, hipStream_t st);
int energy_blocks(const Mesh& M);
int energy_vec_blocks(const Mesh& M);
void launch_energy(const Mesh& M, const double* S, double t, double* pe, double* pv, double* out, hipStream_t st);

size_t batch_lds_bytes(int max_lds_chunk);
hipError_t launch_batch(BatchInst* tab, const BatchWork* work, const int* ids, int n_work, bool teams, int model,
                        const KrylovCfg& cfg, double dt, int n_steps, int max_lds_chunk, hipStream_t st);
hipError_t batch_max_blocks(int prec, int model, int max_lds_chunk, int* blocks_per_cu);

}  // namespace ep
