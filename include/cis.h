/*
 * cis.h -- C ABI of the MI355X library for the conservative implicit scheme for
 * steady diatomic (Rykov) flow on unstructured physical and velocity meshes
 * (arXiv 2303.10846).
 *
 * One call of cis_iterate performs Steps 2-6 of the scheme (Sec. 3.5) on the
 * GPU: reconstruction of the reduced distributions G, R at every face (Eq. 46),
 * the collision-coupled face distribution (Eqs. 45, 47-52), the micro flux
 * (Eq. 31) and macro flux (Eq. 37), the implicit macroscopic prediction
 * (Eqs. 38-43), the implicit microscopic sweeps (Eqs. 30-33) and the
 * conservative update with integral error compensation (Eqs. 62-67).
 *
 * Conventions
 *  - Every function returns a cis_status; 0 is success.  No C++ exception
 *    crosses the ABI.  On error cis_last_error() returns a message (valid until
 *    the next cis_* call on the same thread) and the state is unchanged, except
 *    after CIS_E_NONFINITE, which leaves the state at the failing iteration.
 *  - Arguments are validated before any device work is enqueued.
 *  - Host pointers are borrowed for the duration of the call only.
 *  - Device pointers (cis_device_buffers and the explicit "device" outputs) are
 *    owned by the caller, must stay valid for the life of the state and are
 *    never freed by the library.  The library allocates only small
 *    per-cell/per-face scratch (geometry, macro arrays), freed by
 *    cis_state_destroy.
 *  - All device work is enqueued on the stream given to cis_state_create.
 *    Functions returning host data synchronise that stream.
 *  - Distribution arrays are row-major [n_cells][n_vel] (velocity contiguous),
 *    FP64 in CIS_FP64 mode and FP32 in CIS_MIXED mode.  W and q are FP64
 *    [n_cells][6]: W = (rho, rho U, rho E, rho E_rot) (Eq. 24),
 *    q = (q_tr, q_rot) (Eqs. 26-27).  Offsets are 64-bit.
 *  - Quantities are dimensionless as in Sec. 4 (R = 1/2 for U_ref = sqrt(2 R T_ref)).
 */
#ifndef CIS_H
#define CIS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cis_status;
enum {
  CIS_OK = 0,
  CIS_E_INVALID_ARG = -1, /* null pointer, bad size, bad layout or unknown enum value */
  CIS_E_MESH = -2,        /* V <= 0, open cell (|sum A n| > tol), non-manifold face, untagged open face,
                             or a colouring that puts two face neighbours in one colour */
  CIS_E_DVS = -3,         /* weight <= 0 or non-finite velocity */
  CIS_E_DEVICE = -4,      /* a HIP runtime call failed */
  CIS_E_NONFINITE = -5,   /* NaN/Inf, or rho <= 0 / T <= 0 in a predicted or updated cell state */
  CIS_E_UNSUPPORTED = -6  /* request outside what this build supports (more than 16384 velocities) */
};

enum { CIS_FP64 = 0, CIS_MIXED = 1 };
enum { CIS_BC_WALL = 1, CIS_BC_FARFIELD = 2 };

typedef struct cis_mesh cis_mesh;
typedef struct cis_dvs cis_dvs;
typedef struct cis_state cis_state;

/* Gas constants.  Rykov model, Sec. 2: Z_rot, delta, omega0, omega1 (Eqs. 11-12, 19-22);
   VHS viscosity mu = mu_ref (T_tr/T_ref)^omega_vhs (Eq. 13); relaxation time tau = mu/p_tr. */
typedef struct {
  double R, gamma, Z, delta, omega0, omega1, mu_ref, omega_vhs, T_ref;
} cis_gas;

/* Numerics.
   cfl      : local physical step of the face flux, dt_i = cfl h_i / max_k |u_k|, h_i = 6 V_i / sum_f A_f,
              s_ij = min(dt_i, dt_j) (Eq. 45).
   inv_dt, cfl_imp : implicit time step of Eqs. 29 and 34, one per cell,
              1/dt_i = inv_dt + max_k|u_k| / (cfl_imp h_i) (second term dropped when cfl_imp = 0).
   lim_K    : Venkatakrishnan constant, eps^2 = (K h)^3 max_stencil|phi|^2; limiter = 0 turns it off.
   snap     : |u.n| <= snap |u| counts as u.n = 0 (upwind side x_j, Eq. 46).
   n_macro, n_micro : forward+backward sweep pairs of the macro (Eq. 43) and micro (Eq. 33) PR-SGS. */
typedef struct {
  double cfl, inv_dt, cfl_imp, lim_K, snap;
  int32_t limiter, n_macro, n_micro, reserved;
} cis_numerics;

/* Boundary condition of the faces carrying `tag`.
   CIS_BC_WALL     : diffuse reflection, full accommodation, at (U, T); rho is ignored.
   CIS_BC_FARFIELD : free-stream Maxwellian (rho, U, T) for incoming velocities. */
typedef struct {
  int32_t tag, kind;
  double rho, U[3], T;
} cis_bc;

typedef struct {
  int64_t n_cells, n_faces, n_interior, n_boundary, n_colors;
} cis_mesh_info_t;

typedef struct {
  int64_t phi_bytes;   /* one [n_cells][n_vel] distribution array */
  int64_t face_bytes;  /* one [n_faces][n_vel] face array */
  int64_t cell6_bytes; /* one [n_cells][6] FP64 array (W or q) */
  int64_t total_bytes; /* sum over all cis_device_buffers members */
} cis_buffer_sizes;

/* Caller-owned device memory of a state (sizes from cis_state_required_bytes). */
typedef struct {
  void* G;      /* phi^n, [n_cells][n_vel] */
  void* R;
  void* dG;     /* increments of the micro sweeps (Eq. 33) */
  void* dR;
  void* resG;   /* right-hand side Res of Eq. 33 */
  void* resR;
  void* faceG;  /* [n_faces][n_vel]: reconstructed phi_bar, then A (u.n) phi_f */
  void* faceR;
  double* W;    /* [n_cells][6] */
  double* q;    /* [n_cells][6] */
} cis_device_buffers;

/* Last error message of this thread. */
const char* cis_last_error(void);

/* Mesh of tetrahedra.  xyz [n_nodes][3]; tet [n_cells][4] node ids; btri [n_b][3] boundary triangles with
   tags btag [n_b] (every open face must be tagged).  color_offsets [n_colors+1]: cells
   color_offsets[c] .. color_offsets[c+1]-1 form colour c; no two cells of one colour may share a face
   (checked; the sweeps run colour by colour).  NULL means one cell per colour is not allowed: colours are
   required.  Interior faces are oriented so that the first normal component beyond 1e-9 is positive;
   i is the cell the normal points out of. */
cis_status cis_mesh_create(const double* xyz, int64_t n_nodes, const int32_t* tet, int64_t n_cells,
                           const int32_t* btri, const int32_t* btag, int64_t n_b,
                           const int64_t* color_offsets, int64_t n_colors, cis_mesh** out);
cis_status cis_mesh_info(const cis_mesh* mesh, cis_mesh_info_t* out);
void cis_mesh_destroy(cis_mesh* mesh);

/* Discrete velocity set: u [n][3] (cell centroids of the velocity mesh), w [n] (cell volumes), Sec. 3.2. */
cis_status cis_dvs_create(const double* u, const double* w, int64_t n, cis_dvs** out);
void cis_dvs_destroy(cis_dvs* dvs);

cis_status cis_state_required_bytes(const cis_mesh* mesh, const cis_dvs* dvs, int32_t precision,
                                    cis_buffer_sizes* out);

/* Create a state on the current HIP device.  `stream` is a hipStream_t (NULL = default stream).
   The state borrows mesh and dvs, which must outlive it. */
cis_status cis_state_create(const cis_mesh* mesh, const cis_dvs* dvs, const cis_gas* gas, const cis_numerics* num,
                            const cis_bc* bc, int32_t n_bc, int32_t precision, const cis_device_buffers* buf,
                            void* stream, cis_state** out);
cis_status cis_state_set_numerics(cis_state* s, const cis_numerics* num);
void cis_state_destroy(cis_state* s);

/* Step 1: phi = phi*(W0, q = 0) in every cell (Eqs. 17-23).  W0 is host [6] (per_cell = 0) or
   [n_cells][6] (per_cell = 1). */
cis_status cis_state_init_equilibrium(cis_state* s, const double* W0, int32_t per_cell);

/* Host <-> device copies of the state (phi in the state's precision; W, q FP64).  get synchronises. */
cis_status cis_state_set(cis_state* s, const void* G, const void* R, const double* W, const double* q);
cis_status cis_state_get(cis_state* s, void* G, void* R, double* W, double* q);

/* n_iter implicit iterations (Steps 2-6).  res_hist (host, [n_iter][6] or NULL) receives the residual
   (1/N_c) sum_i |W_i^{n+1} - W_i^n| per component after each iteration (Step 7). */
cis_status cis_iterate(cis_state* s, int32_t n_iter, double* res_hist);

/* Explicit operator on the current state (Steps 2-3): micro flux F [n_cells][n_vel] (Eq. 31) into the
   device arrays FG, FR (state precision) and macro flux F [n_cells][6] (Eq. 37) into host Fmac (or NULL). */
cis_status cis_residual(cis_state* s, void* FG_dev, void* FR_dev, double* Fmac_host);

/* Cell moments of the current state: W, q (host [n_cells][6] each; either may be NULL). */
cis_status cis_moments(cis_state* s, double* W, double* q);

/* Wall heat flux of the current state: sum over the faces of `tag` of A_f sum_k w_k (u_k.n)(|u_k|^2/2 G_f + R_f),
   n pointing from the fluid into the wall (Eq. 72 numerator). */
cis_status cis_wall_heat_flux(cis_state* s, int32_t tag, double* Q);

/* Small internal arrays of the last iteration, copied to host (for stage-by-stage checks):
   which = 0: dW~ [n_cells][6] (Eq. 43 solution), 1: W~ [n_cells][6], 2: macro flux F [n_cells][6] (Eq. 37),
   3: tau~ [n_cells]. */
cis_status cis_debug_stage(cis_state* s, int32_t which, double* out_host);

/* Per-stage device time of cis_iterate, measured with hipEvents recorded on the state's stream between the
   stages of every iteration, accumulated while enabled (enable = 1 also resets the accumulators).
   Stages: 0 reconstruction (Eq. 46), 1 face pass (Eqs. 45, 47-52; Eq. 31 and 37 summands),
   2 macro prediction (Eqs. 38-43), 3 micro residual (Eq. 31 per cell, Eq. 33 right-hand side),
   4 micro sweeps (Eq. 33), 5 update and compensation (Eqs. 62-67) with the residual of Step 7.
   ms [6] receives milliseconds, launches [6] the number of kernel launches per stage (either may be NULL). */
cis_status cis_profile_enable(cis_state* s, int32_t enable);
cis_status cis_profile_read(cis_state* s, double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* CIS_H */
