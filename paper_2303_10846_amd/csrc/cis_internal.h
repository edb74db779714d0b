// Internal device layouts and kernel launchers of the cis library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <vector>

namespace cis {

// Face slots per cell: NF = 4 when every cell is a tetrahedron (slot a = the face opposite local vertex a),
// else kMaxFaces = 6 (slot a = the a-th local face of the cell's kind; a cell with fewer faces leaves the last
// slots unused: neighbour kNoFace, face -1, geometry zero).
constexpr int kMaxFaces = 6;
constexpr int32_t kNoFace = -2;

// Per-cell geometry record, FP64, CG doubles per cell:
//   [0] V  [1] 1/V  [2] h = 6V/sum A  [3] unused  [4..6] centroid  [7] unused
//   face slot a at 8 + 12a:
//   [0] sign (+1: the face normal points out of this cell, -1: into it)  [1] A/V
//   [2..4] outward unit normal  [5..7] x_f - x_i  [8] s_f (Eq. 45)  [9..11] least-squares weight M^-1 d
// FP32 reconstruction geometry per cell: for face slot a, [7a, 7a + 3) = x_f - x_i, [7a + 3] = s_f,
// [7a + 4, 7a + 7) = the least-squares weights of the neighbour difference
// Upwind codes: 2 bits per slot, one byte per (cell, velocity) for NF = 4, two for NF = 6.
template <int NF> struct Lay {
  static constexpr int CG = 8 + 12 * NF;
  static constexpr int CGF = NF == 4 ? 32 : 48;
  using Code = typename std::conditional<NF == 4, uint8_t, uint16_t>::type;
};
// the tetrahedral layout (the adjoint kernels run on tetrahedral meshes only)
constexpr int CG = Lay<4>::CG;
constexpr int CG_FACE = 8;
constexpr int CG_SLOT = 12;
constexpr int CGF = Lay<4>::CGF;

// Per-face record, FP64, FGW doubles: [0] A  [1..3] unit normal (out of face_cell[2f])  [4] s  [5] dl
constexpr int FGW = 8;

// DVS, structure of arrays: dvs = 6 FP64 arrays of nv values (u_x, u_y, u_z, w, |u|, |u|^2/2),
// dvs_f = 3 FP32 arrays (u_x, u_y, u_z) for the FP32 equilibrium evaluation of the mixed mode.
constexpr int DVS_ARRAYS = 6;
constexpr int DVS_F_ARRAYS = 3;

// Boundary-condition record: [0] kind  [1] rho  [2..4] U  [5] T  [6..7] unused
constexpr int BCW = 8;

// Cell equilibrium record (predicted state of Step 4), ER doubles:
//   [0] rho [1..3] U [4] T [5] T_tr [6] T_rot [7] tau [8..10] q_tr [11..13] q_rot
//   [14] a_tr [15] b_tr [16] a_T [17] b_T [18] k_tr [19] k_T [20] k_tr_r [21] k_T_r
//   [22] 1/(R T_tr) [23] 1/(R T) [24] R T_rot [25] R T [26] 1-1/Z [27] 1/Z
constexpr int ER = 32;

struct GasC {
  double R, gamma, Z, delta, omega0, omega1, mu_ref, omega_v, T_ref, C_s;  // C_s > 0: Sutherland (Eq. 14)
};

struct Dev {
  int64_t nc, nf, nv;
  int mf;                    // face slots per cell, 4 or kMaxFaces
  const int32_t* cell_nb;    // [nc][mf] neighbour cell, -1 (boundary face) or kNoFace (unused slot)
  const int32_t* spatial;    // [nc] cells in Morton order of their centroids
  const int32_t* cell_face;  // [nc][mf] (-1: unused slot)
  const double* cell_geo;    // [nc][Lay<mf>::CG]
  const float* cell_geo_f;   // [nc][Lay<mf>::CGF] FP32 copy of the reconstruction geometry
  uint8_t* upw;              // [nc][nv] upwind codes (Lay<mf>::Code): bits 2a..2a+1 = 1 (u.n > 0), 2 (u.n < 0),
                             // 0 (tie or unused slot) of slot a
  const int32_t* face_cell;  // [nf][2] (cell the normal points out of, other cell or -1)
  const int32_t* face_bc;    // [nf] slot in bc table, -1 interior
  const double* face_geo;    // [nf][FGW]
  const double* dvs;         // [DVS_ARRAYS][nv]
  const float* dvs_f;        // [DVS_F_ARRAYS][nv]
  const double* bc;          // [nbc][BCW]
  GasC gas;
  double snap, lim_K, inv_dt, cfl_imp, umax;
  int limiter;               // 0 off, 1 Venkatakrishnan, 2 the same (held fixed by the VJP), 3 stored values,
                             // 4 the smaller of the computed and the stored value, stored back
  const void* lim_frozen;    // limiter 3, 4: [2][nc][nv] stored limiter values of G then R (state precision)
};

// Step 7's residual is reduced in two stages over a fixed partition of the cells: kResidualParts partial sums of
// 6 doubles each (Work::respart), then one workgroup adds them in order.
constexpr int kResidualParts = 256;

struct Work {
  double* face_mac;  // [nf][6]
  double* cell_prim; // [nc][8]: rho U T T_tr tau 0
  double* rcf;       // [nc][mf] spectral radius r_ij of each face slot (Eq. 41)
  double* G0;        // [nc][mf][6] Euler flux of the neighbour's W^n along the outward normal
  double* mres;      // [nc][6]
  double* mD;        // [nc][2]
  double* Fmac;      // [nc][6]
  double* dW;        // [nc][6]
  double* mbase;     // [nc] 1/dt_i + 1/tau~_i, the velocity-independent part of the diagonal of Eq. 33
  double* Wt;        // [nc][6]
  double* eq;        // [nc][ER]
  double* cellres;   // [nc][6]
  double* res;       // [hist][6]
  double* respart;   // [kResidualParts][6] partial sums of the residual
  int32_t* flag;     // [4]
  double* gpf;       // [nf][3] per-face parameter adjoints of the VJP
};

struct Bufs {
  void *G, *R, *dG, *dR, *resG, *resR, *faceG, *faceR;
  double *W, *q;
};

// Launchers (all enqueue on `st`); T = double or float selects the precision mode.
template <class T> void launch_init_eq(const Dev& d, const Bufs& b, const double* W0, int per_cell, double* eqtmp,
                                       hipStream_t st);
// cap != nullptr: also store the limiter values (limiter 1's, whatever d.limiter is) into cap, [2][nc][nv]
template <class T> void launch_recon(const Dev& d, const Bufs& b, hipStream_t st, void* cap = nullptr);
template <class T> void launch_face(const Dev& d, const Bufs& b, const Work& w, hipStream_t st);
void launch_macro(const Dev& d, const Bufs& b, const Work& w, const int64_t* color_off, int64_t n_colors,
                  int n_macro, hipStream_t st);
template <class T> void launch_residual(const Dev& d, const Bufs& b, const Work& w, void* outG, void* outR,
                                        int flux_only, hipStream_t st);
template <class T> void launch_micro(const Dev& d, const Bufs& b, const Work& w, const int64_t* color_off,
                                     int64_t n_colors, int n_micro, hipStream_t st);
template <class T> void launch_update(const Dev& d, const Bufs& b, const Work& w, int64_t it, hipStream_t st);
void launch_macro_flux_cells(const Dev& d, const Work& w, hipStream_t st);
void launch_upwind_codes(const Dev& d, hipStream_t st);
int max_velocities();
std::vector<int64_t> sweep_sequence(const int64_t* color_off, int64_t n_colors, int n_pairs);

// Steady residual and its vector-Jacobian product (FP64 only).
struct AdjArgs {
  const double *vG, *vR, *vW, *vq;  // seed v (all NULL: zero)
  double cJ;                        // seed of the objective
  int32_t jslot, wslot, fslot;      // bc slots: objective faces, wall temperature, far-field state (-1: none)
  double *gG, *gR, *gW, *gq;        // v^T dR/dx + cJ dJ/dx
  double* gpf;                      // [nf][3] per-face parts of v^T dR/dp + cJ dJ/dp
};
void launch_cell_steady(const Dev& d, const Bufs& b, double* rG, double* rR, double* rW, double* rq, hipStream_t st);
void launch_vjp(const Dev& d, const Bufs& b, const AdjArgs& a, hipStream_t st);
void launch_precond(const Dev& d, const Bufs& b, const double* in, double* out, hipStream_t st);
void launch_adj_sweeps(const Dev& d, const Bufs& b, const double* in, double* out, const int64_t* color_off,
                       int64_t n_colors, int n_pairs, hipStream_t st);
void launch_dots(const double* V, int64_t n, int nvec, const double* w, double* part, double* out, hipStream_t st);
void launch_gemv_sub(const double* V, int64_t n, int nvec, const double* h, double* w, hipStream_t st);
void launch_axpby(int64_t n, double a, const double* x, double c, double* y, hipStream_t st);
int dot_partials();

}  // namespace cis
