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
  CIS_E_UNSUPPORTED = -6  /* request outside what the library supports (more than 16384 velocities) */
};

enum { CIS_FP64 = 0, CIS_MIXED = 1 };
enum { CIS_BC_WALL = 1, CIS_BC_FARFIELD = 2 };

typedef struct cis_mesh cis_mesh;
typedef struct cis_dvs cis_dvs;
typedef struct cis_state cis_state;

/* Gas constants.  Rykov model, Sec. 2: Z_rot, delta, omega0, omega1 (Eqs. 11-12, 19-22); relaxation time
   tau = mu/p_tr.  Viscosity: C_s = 0 selects the VHS law mu = mu_ref (T_tr/T_ref)^omega_vhs (Eq. 13); C_s > 0
   selects Sutherland's law mu = mu_ref (T_tr/T_ref)^(3/2) (T_ref + C_s)/(T_tr + C_s) (Eq. 14), and omega_vhs
   is then unused.  C_s < 0 is rejected. */
typedef struct {
  double R, gamma, Z, delta, omega0, omega1, mu_ref, omega_vhs, T_ref, C_s;
} cis_gas;

/* Numerics.
   cfl      : local physical step of the face flux, dt_i = cfl h_i / max_k |u_k|, h_i = 6 V_i / sum_f A_f,
              s_ij = min(dt_i, dt_j) (Eq. 45).
   inv_dt, cfl_imp : implicit time step of Eqs. 29 and 34, one per cell,
              1/dt_i = inv_dt + max_k|u_k| / (cfl_imp h_i) (second term dropped when cfl_imp = 0).
   lim_K    : Venkatakrishnan constant, eps^2 = (K h)^3 max_stencil|phi|^2.
   limiter  : 0 off; 1 Venkatakrishnan, differentiated by cis_residual_vjp on the branch the state takes;
              2 the same limiter in the iteration, held fixed (frozen) by cis_residual_vjp, whose product is
              then the derivative of the scheme with the limiter values of the current state;
              3 stored values: the values attached by cis_limiter_freeze are used in place of the limiter in
              every reconstruction (and are constants of cis_residual_vjp);
              4 monotone freezing: every reconstruction takes the smaller of limiter 1's value and the stored
              one, and stores it back, so the stored values only decrease (the steady residual, VJP and adjoint
              refuse it: switch to 3 once the values have settled).
              3 and 4 are refused until cis_limiter_freeze has attached values.
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
  int64_t max_faces; /* face slots per cell: 4 when every cell is a tetrahedron, else 6 */
} cis_mesh_info_t;

typedef struct {
  int64_t phi_bytes;   /* one [n_cells][n_vel] distribution array */
  int64_t face_bytes;  /* one [n_faces][n_vel] face array */
  int64_t cell6_bytes; /* one [n_cells][6] FP64 array (W or q) */
  int64_t code_bytes;  /* the [n_cells][n_vel] upwind-code array: uint8 (4 face slots) or uint16 (6) */
  int64_t total_bytes; /* sum over all cis_device_buffers members */
} cis_buffer_sizes;

/* Caller-owned device memory of a state (sizes from cis_state_required_bytes).  Alignment: element alignment is
   required.  Faster paths with the same results need more (torch and hipMalloc give 256): faceG and faceR aligned
   to 16 bytes and upwind to 4 bytes let the face pass copy each face row into LDS with LDS-DMA loads when n_vel
   is a multiple of 4; G, R, dG, dR, resG, resR, faceG and faceR aligned to 16 bytes let the micro residual and
   sweep move 16-byte vectors of velocities when n_vel is a multiple of 4 (mixed) or 2 (FP64). */
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
  uint8_t* upwind; /* [n_cells][n_vel] uint8 (mesh with 4 face slots) or uint16 (6 slots) codes, written by
                      cis_state_create: for face slot a of cell i (its a-th face), bits 2a..2a+1 of entry (i, k) are
                      1 if u_k.n > 0 (out of the cell), 2 if u_k.n < 0, 0 if |u_k.n| is within the tie tolerance of
                      zero or the slot is unused (Eq. 46 upwinding, Eq. 33 diagonal) */
} cis_device_buffers;

/* Last error message of this thread. */
const char* cis_last_error(void);

/* Mesh of tetrahedra: the unstructured physical mesh of Sec. 3.1 (cells V_i, interfaces A_ij with unit normals
   n_ij from cell i to cell j, interface midpoints x_ij of Eq. 46).  xyz [n_nodes][3]; tet [n_cells][4] node ids; btri [n_b][3] boundary triangles with
   tags btag [n_b] (every open face must be tagged).  color_offsets [n_colors+1]: cells
   color_offsets[c] .. color_offsets[c+1]-1 form colour c; no two cells of one colour may share a face
   (checked; the sweeps run colour by colour).  NULL means one cell per colour is not allowed: colours are
   required.  Interior faces are oriented so that the first normal component beyond 1e-9 is positive;
   i is the cell the normal points out of. */
cis_status cis_mesh_create(const double* xyz, int64_t n_nodes, const int32_t* tet, int64_t n_cells,
                           const int32_t* btri, const int32_t* btag, int64_t n_b,
                           const int64_t* color_offsets, int64_t n_colors, cis_mesh** out);
/* Mesh of mixed cells (the paper's meshes are hexahedral, Sec. 4): cells [n_cells][8] node ids (unused places
   ignored) of the kinds kinds [n_cells] = node count: 4 tetrahedron, 5 pyramid (base quad 0-3 in cyclic order,
   apex 4), 6 prism (triangles 0-2 and 3-5, with 0-3, 1-4, 2-5 edges), 8 hexahedron (quads 0-3 and 4-7 in
   cyclic order, with 0-4, 1-5, 2-6, 3-7 edges).  bface [n_b][4] boundary faces (-1 in the last place of a
   triangle) with tags btag.  A quad face need not be planar: its area vector is half the cross product of its
   diagonals and its centroid the area-weighted centroid of the four triangles it makes with its node average;
   a cell other than a tetrahedron has the volume and centroid of the tetrahedra from its node average to those
   triangles.  Face slot a of a cell is its a-th local face: for a tetrahedron the face opposite local vertex a;
   a pyramid: base, then (0,1,4), (1,2,4), (2,3,4), (3,0,4); a prism: (0,1,2), (3,4,5), (0,1,4,3), (1,2,5,4),
   (2,0,3,5); a hexahedron: (0,1,2,3), (4,5,6,7), (0,1,5,4), (1,2,6,5), (2,3,7,6), (3,0,4,7).  Colours and errors as
   for cis_mesh_create (plus CIS_E_INVALID_ARG for an unknown kind, CIS_E_MESH for a folded cell). */
cis_status cis_mesh_create_cells(const double* xyz, int64_t n_nodes, const int32_t* cells, const int32_t* kinds,
                                 int64_t n_cells, const int32_t* bface, const int32_t* btag, int64_t n_b,
                                 const int64_t* color_offsets, int64_t n_colors, cis_mesh** out);
cis_status cis_mesh_info(const cis_mesh* mesh, cis_mesh_info_t* out);
void cis_mesh_destroy(cis_mesh* mesh);

/* Discrete velocity set: u [n][3] (cell centroids of the velocity mesh), w [n] (cell volumes), Sec. 3.2. */
cis_status cis_dvs_create(const double* u, const double* w, int64_t n, cis_dvs** out);
void cis_dvs_destroy(cis_dvs* dvs);

cis_status cis_state_required_bytes(const cis_mesh* mesh, const cis_dvs* dvs, int32_t precision,
                                    cis_buffer_sizes* out);

/* Create a state on the current HIP device: the distributions G, R and the macroscopic W, q of every cell for
   Steps 2-6 of Sec. 3.5, with the geometry of Step 1 (local steps dt_i by the CFL condition, s_ij = min(dt_i,
   dt_j) of Eq. 45, least-squares weights of Eq. 46) prepared on the host.  `stream` is a hipStream_t (NULL =
   default stream).  The state borrows mesh and dvs, which must outlive it.  The initial field is set by
   cis_state_init_equilibrium (Step 1) or cis_state_set.  Errors: CIS_E_INVALID_ARG (NULL buffers, numerics or
   gas constants out of range, a boundary tag without a condition), CIS_E_UNSUPPORTED (too many velocities),
   CIS_E_MESH (singular least-squares matrix), CIS_E_DEVICE. */
cis_status cis_state_create(const cis_mesh* mesh, const cis_dvs* dvs, const cis_gas* gas, const cis_numerics* num,
                            const cis_bc* bc, int32_t n_bc, int32_t precision, const cis_device_buffers* buf,
                            void* stream, cis_state** out);
cis_status cis_state_set_numerics(cis_state* s, const cis_numerics* num);
void cis_state_destroy(cis_state* s);

/* Limiter freezing.  L: caller-owned device memory of 2 * n_cells * n_vel values in the state's precision
   ([G | R], each [n_cells][n_vel]).  compute != 0: Venkatakrishnan's limiter values of the current state (Eq. 46,
   as limiter 1, with the state's lim_K) are written to L for every (cell, velocity) of G and of R (the face
   buffers are overwritten); compute = 0: L's contents are taken as they are (values in [0, 1], e.g. those of
   another state).  L is then attached to the state: with numerics.limiter = 3 the reconstruction uses these
   values instead of recomputing them, so near a steady state the scheme is a smooth function of phi (the min
   over faces and the stencil extrema no longer switch); with limiter 4 it also lowers them where the computed
   limiter is smaller.  L must stay valid while attached.  L = NULL detaches (refused while limiter 3 or 4 is in
   use).  Errors: CIS_E_INVALID_ARG, CIS_E_DEVICE. */
cis_status cis_limiter_freeze(cis_state* s, void* L, int32_t compute);

/* Step 1: phi = phi*(W0, q = 0) in every cell (Eqs. 17-23).  W0 is host [6] (per_cell = 0) or
   [n_cells][6] (per_cell = 1). */
cis_status cis_state_init_equilibrium(cis_state* s, const double* W0, int32_t per_cell);

/* Host <-> device copies of the state (phi in the state's precision; W, q FP64).  get synchronises. */
cis_status cis_state_set(cis_state* s, const void* G, const void* R, const double* W, const double* q);
cis_status cis_state_get(cis_state* s, void* G, void* R, double* W, double* q);

/* n_iter implicit iterations (Steps 2-6).  res_hist (host, [n_iter][6] or NULL) receives the residual
   (1/N_c) sum_i |W_i^{n+1} - W_i^n| per component after each iteration (Step 7). */
cis_status cis_iterate(cis_state* s, int32_t n_iter, double* res_hist);

/* cis_iterate for callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc): the same kernels and results, bitwise, but no hipMalloc, hipFree, event or
   other allocation.  The residual partial sums, the residual history and the positivity flags live in a fixed
   device array of the library (about 205 KB per GPU, held until the process ends) instead of the state's
   own, so n_iter is limited to 0..4096 per call (CIS_E_INVALID_ARG beyond, before any device work).  Every
   call on one GPU shares that array: calls that overlap on one GPU (two host threads, or states on different
   streams) race and must be serialised by the caller.  Per-stage profiling (cis_profile_enable) does not
   apply.  res_hist (host, [n_iter][6], or NULL) as for cis_iterate; synchronises the state's stream. */
cis_status cis_iterate_noalloc(cis_state* s, int32_t n_iter, double* res_hist);

/* Explicit operator on the current state (Steps 2-3): micro flux F [n_cells][n_vel] (Eq. 31) into the
   device arrays FG, FR (state precision) and macro flux F [n_cells][6] (Eq. 37) into host Fmac (or NULL). */
cis_status cis_residual(cis_state* s, void* FG_dev, void* FR_dev, double* Fmac_host);

/* Cell moments of the current state: W, q (host [n_cells][6] each; either may be NULL). */
cis_status cis_moments(cis_state* s, double* W, double* q);

/* Wall heat flux of the current state: sum over the faces of `tag` of A_f sum_k w_k (u_k.n)(|u_k|^2/2 G_f + R_f),
   n pointing from the fluid into the wall (Eq. 72 numerator). */
cis_status cis_wall_heat_flux(cis_state* s, int32_t tag, double* Q);

/* Loads on the faces of one wall, from the face distributions of the current state (Sec. 4, Eqs. 70-72).
   n points from the gas into the wall.  Per face:
     p   = sum_k w (u.n)^2 G_w                    the Eq. 70 numerator before p_inf is subtracted;
     tau = sum_k w (u.n) u G_w - n p               the Eq. 71 numerator, as a vector (|tau| is the shear);
     q   = sum_k w (u.n)(|u|^2/2 G_w + R_w)        the Eq. 72 numerator.
   The force on the wall is sum_f A_f (p n + tau) and its heat load sum_f A_f q.  Divide by the free-stream
   references to get C_p, C_tau, C_h and force coefficients. */
typedef struct {
  double x[3];   /* face centroid */
  double area;
  double n[3];   /* unit normal, gas -> wall */
  double p;
  double tau[3];
  double q;
} cis_wall_face;

/* faces (host, [*n_faces], or NULL) receives the faces of `tag` in face order; *n_faces (or NULL) their count.
   force (host [3], or NULL) and heat (host, or NULL) receive the integrated loads. */
cis_status cis_wall_loads(cis_state* s, int32_t tag, int64_t* n_faces, cis_wall_face* faces, double* force,
                          double* heat);

/* Free-stream references of the wall coefficients (Sec. 4, Eqs. 70-72): dynamic pressure
   q_inf = rho_inf |U_inf|^2 / 2 and pressure p_inf = rho_inf R T_inf.  A_ref > 0 also asks for the force,
   moment and heat-load coefficients, with the moment about x_ref scaled by L_ref.  Drag is along U_inf; lift
   is along the part of lift_dir normal to U_inf (all zero: e_z, or e_y when U_inf is along z). */
typedef struct {
  double rho_inf, U_inf[3], T_inf;
  double A_ref, L_ref, x_ref[3], lift_dir[3];
} cis_wall_ref;

/* Per wall face: C_p = (p - p_inf)/q_inf (Eq. 70), C_tau = |tau|/q_inf (Eq. 71), C_h = q/(q_inf |U_inf|)
   (Eq. 72), from the face loads of cis_wall_loads. */
typedef struct {
  double Cp, Ctau, Ch;
} cis_wall_coef;

/* Integrated loads of one wall: force F = sum_f A_f (p n + tau), moment M = sum_f (x_f - x_ref) x A_f (p n + tau),
   heat load sum_f A_f q; with A_ref > 0 also CF = F/(q_inf A_ref), C_d = CF.e_drag, C_l = CF.e_lift,
   CM = M/(q_inf A_ref L_ref), the pitching moment C_m = CM.(e_lift x e_drag) and CQ = heat/(q_inf |U_inf| A_ref)
   (zero when A_ref = 0). */
typedef struct {
  double force[3], moment[3], heat;
  double e_drag[3], e_lift[3];
  double CF[3], Cd, Cl, CM[3], Cm, CQ;
} cis_wall_totals;

/* Wall coefficients of Eqs. 70-72 and the force and moment coefficients from per-face loads (host arithmetic
   only; R is the gas constant of p_inf).  coef (host, [n_faces], or NULL) receives the per-face coefficients
   in the order of faces; totals (host, or NULL) the integrated values.  CIS_E_INVALID_ARG for NULL
   faces with n_faces > 0, non-positive rho_inf, |U_inf|, T_inf or R, A_ref < 0, L_ref <= 0 with A_ref > 0,
   or a lift direction parallel to U_inf. */
cis_status cis_wall_coefficients_of_loads(const cis_wall_face* faces, int64_t n_faces, double R,
                                          const cis_wall_ref* ref, cis_wall_coef* coef, cis_wall_totals* totals);

/* The same for the faces of wall `tag` of the current state: runs the face pass (as cis_wall_loads), then
   cis_wall_coefficients_of_loads with the state's gas constant.  *n_faces (or NULL) receives the face count;
   coef, if set, must hold that many records (call once with coef = NULL to size it). */
cis_status cis_wall_coefficients(cis_state* s, int32_t tag, const cis_wall_ref* ref, int64_t* n_faces,
                                 cis_wall_coef* coef, cis_wall_totals* totals);

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

/* Replace the boundary-condition values of a state (same count, order, tags and kinds as at creation).
   Used to move the parameters p of the adjoint (wall temperature, free-stream density and speed). */
cis_status cis_state_set_bc(cis_state* s, const cis_bc* bc, int32_t n_bc);

/* ---- Steady residual, its vector-Jacobian product and the discrete adjoint (FP64 states only;
   CIS_E_UNSUPPORTED in CIS_MIXED).  Not in the paper: this is the derivative of its steady scheme.

   The state x = (G, R, W, q) is steady when one implicit iteration (Sec. 3.5, Steps 2-6) with the
   predicted state equal to the current one leaves it unchanged, i.e. R(x; p) = 0 with
     R_phi = (phi*(W, q) - phi)/tau(W) - F(phi; p)              (right-hand side of Eq. 33, Eq. 31)
     R_W   = W - [sum_k w_k Phi_k (phi_k - phi*_k) + M(W)]      (Eqs. 62-65, M = analytic moments of phi*)
     R_q   = q - [heat-flux sums of phi - phi* + a q]            (Eqs. 66-67)
   The parameters are p = (T_w of the wall with tag wall_tag, rho_inf and |U_inf| of the far field with
   tag ff_tag; |U_inf| moves along the fixed direction of U_inf).  The objective is the heat flux into the
   wall of wall_tag, J = sum_f A_f sum_k w_k (u_k.n_f)(|u_k|^2/2 G_f,k + R_f,k) (Eq. 72 numerator).
   The DVS and the mesh are held fixed.

   These calls overwrite the state's face buffers (faceG, faceR) and internal macro arrays; G, R, W, q are
   not modified.  All array arguments below are device pointers with the layouts of the state
   ([n_cells][n_vel] FP64 for G-like arrays, [n_cells][6] FP64 for W-like arrays) unless marked host. */

/* R(x; p) at the current state into rG, rR, rW, rq; J (host, or NULL) = heat flux into wall_tag. */
cis_status cis_steady_residual(cis_state* s, int32_t wall_tag, double* rG, double* rR, double* rW, double* rq,
                               double* J);

/* g = v^T dR/dx + cJ dJ/dx into gG, gR, gW, gq and gp (host [3], or NULL) = v^T dR/dp + cJ dJ/dp.
   vG, vR, vW, vq are all set or all NULL (v = 0, e.g. for dJ/dx alone with cJ = 1).  Outputs must not
   overlap the inputs.  Faces whose tag is not wall_tag / ff_tag contribute nothing to gp; a tag of -1
   means none (wall_tag must exist when cJ != 0).  The limiter (Eq. 46) is differentiated on the branch
   that the current state takes (numerics.limiter = 1) or held fixed (numerics.limiter = 2). */
cis_status cis_residual_vjp(cis_state* s, const double* vG, const double* vR, const double* vW, const double* vq,
                            double cJ, int32_t wall_tag, int32_t ff_tag, double* gG, double* gR, double* gW,
                            double* gq, double* gp);

typedef struct {
  int32_t iterations; /* Krylov iterations (VJP applications) */
  int32_t converged;  /* 1 when |(dR/dx)^T lam - dJ/dx| <= rtol |dJ/dx| */
  double rel_residual;
} cis_adjoint_info;

/* Device workspace of cis_adjoint_solve for GMRES(restart), in bytes: (restart + 4) vectors of
   2 n_cells n_vel + 12 n_cells doubles, plus reduction scratch and 24 doubles per cell. */
cis_status cis_adjoint_required_bytes(const cis_state* s, int32_t restart, int64_t* bytes);

/* Discrete adjoint at the current (steady) state: solves (dR/dx)^T lam = (dJ/dx)^T by restarted GMRES
   with a right preconditioner, then dJdp (host [3]) = dJ/dp - lam^T dR/dp for
   p = (T_w, rho_inf, |U_inf|).  lam: device [2 n_cells n_vel + 12 n_cells] FP64, laid out as
   [lam_G | lam_R | lam_W | lam_q].  work: caller-owned device memory of at least
   cis_adjoint_required_bytes(restart).  J (host, or NULL) receives the objective.  Stops after max_iter
   Krylov iterations or when the true residual is below rtol relative to |dJ/dx|; info (or NULL) reports
   which.  dJdp is only the steady-state derivative when R(x; p) is near zero.
   The preconditioner approximates the phi block of (dR/dx)^T by -(D + N^T), where -(D + N) is dR_phi/dphi
   with first-order upwind faces (Eq. 32) and the collision term frozen, D_i = 1/tau_i + sum_f (A_f/V_i)
   max(u.n, 0).  precond_pairs = 0 applies -D^-1; n > 0 applies n forward + backward Gauss-Seidel pairs over
   the colours, from zero (0..64).
   macro_pairs = 0: the W and q rows are left as they are.  macro_pairs > 0 (up to 200) selects the block
   preconditioner over (phi, W, q): the W and q rows are eliminated exactly (their diagonal block taken as the
   identity), and the phi Schur complement is approximated by the transpose of the linearised implicit step
   of Steps 4-5: the transport solve above, then the steady macroscopic system of Eq. 43 (no 1/dt term),
   transposed, with macro_pairs forward + backward PR-SGS pairs, whose correction is spread back over the
   velocities through the conserved moments.  Errors: CIS_E_INVALID_ARG for NULL pointers, a short work
   buffer or counts out of range; CIS_E_UNSUPPORTED in the mixed mode; CIS_E_DEVICE on a HIP error. */
cis_status cis_adjoint_solve(cis_state* s, int32_t wall_tag, int32_t ff_tag, int32_t restart, int32_t max_iter,
                             double rtol, int32_t precond_pairs, int32_t macro_pairs, void* work,
                             int64_t work_bytes, double* lam, double* dJdp, double* J, cis_adjoint_info* info);

#ifdef __cplusplus
}
#endif

#endif /* CIS_H */
