// gfx950 kernels of one implicit iteration of the conservative implicit scheme
// (arXiv 2303.10846, Sec. 3.5, Steps 2-6).
//
// Layout: distributions are [cell][velocity] rows (velocity contiguous); the
// discrete velocity set is stored as separate coalesced arrays; the sign of u.n
// through each face of each cell is precomputed once per state (upwind codes,
// read by the reconstruction and the micro sweeps).  Kernels that
// read neighbour rows (reconstruction, micro residual, micro sweeps) run one
// workgroup per (cell, velocity chunk) in chunk-major order, so one velocity
// chunk of every row is touched within a short window; each thread issues all
// its loads before its first store.  Kernels that reduce over the whole
// velocity set of one face or cell (face pass, update) run one workgroup per
// face or cell.  DVS moment sums are FP64: per-thread running sums, a pairwise
// shuffle tree per wavefront, and a merge of the wavefronts; in the mixed mode
// the sums of the conservative update are compensated (TwoSum error terms).  The coloured
// Gauss-Seidel sweeps update one colour at a time: cells of one colour share no
// face.  Nothing here is a dense contraction; the kernels are bound by HBM
// bandwidth, latency and vector ALU, not MFMA.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "cis_device.h"
#include "cis_internal.h"

namespace cis {

// Velocities per thread in the (cell, chunk) kernels, chunk = kBlock * Vpt<T>: 2 in FP32, 1 in FP64 (measured
// on the sphere workload: more velocities per thread raise the loads in flight but cost occupancy).  The
// reconstruction takes VptRecon<T>: 3 strided velocities per thread in FP32, 1 in FP64 (measured: FP32 2.42 ms
// with one, 2.31 with two, 2.25 with three, 2.34 with four; FP64 3.9 ms with one, 5.5 with two).  The scalar
// micro sweep takes one in both precisions (kVptOne: measured faster in FP32).
// The micro sweep and the micro residual have vector forms (k_micro_sweep_vec, k_residual_vec) that move
// 16 bytes per row access (four FP32 or two FP64 velocities) when nv is a multiple of that and the rows are
// 16-byte aligned, and a two-velocity FP32 form for an even nv.
template <class T> struct Vpt;
template <> struct Vpt<double> { static constexpr int v = 1; };
template <> struct Vpt<float> { static constexpr int v = 2; };
constexpr int kVptOne = 1;
template <class T> struct VptRecon { static constexpr int v = sizeof(T) == 4 ? 3 : 1; };

template <int U> static inline unsigned n_chunks_u(int64_t nv) {
  constexpr int c = kBlock * U;
  return (unsigned)((nv + c - 1) / c);
}
template <class T> static inline unsigned n_chunks(int64_t nv) { return n_chunks_u<Vpt<T>::v>(nv); }

// (cell, chunk) workgroups run on a 1-D grid in chunk-major order: all cells of chunk 0, then of chunk 1, ...,
// so that at any time the whole GPU works on one velocity chunk of every row (a slice that stays in the
// last-level cache).  Within a chunk the cells are padded to a multiple of the XCD count and dealt out so
// that every XCD gets one contiguous range of the (Morton-ordered) cells.
struct CellChunk {
  int64_t cell, chunk;
};
__host__ __device__ inline int64_t padded_cells(int64_t ncells) { return (ncells + kXcd - 1) / kXcd * kXcd; }
__device__ inline CellChunk cell_chunk(int64_t ncells) {
  const int64_t np = padded_cells(ncells);
  const int64_t r = (int64_t)blockIdx.x % np;
  return CellChunk{xcd_block(r, np), (int64_t)blockIdx.x / np};
}

// Velocity loop of a (cell, chunk) workgroup: Vpt<T> coalesced velocities per thread.
template <class T, class F> __device__ inline void chunk_loop(int64_t nv, int64_t chunk, F&& body) {
  constexpr int U = Vpt<T>::v;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t k = chunk * (kBlock * U) + (int64_t)u * kBlock + threadIdx.x;
    if (k < nv) body(k);
  }
}

template <int U> static inline dim3 cell_chunk_grid_u(int64_t ncells, int64_t nv) {
  return dim3((unsigned)(padded_cells(ncells) * (int64_t)n_chunks_u<U>(nv)));
}
template <class T> static inline dim3 cell_chunk_grid(int64_t ncells, int64_t nv) {
  return cell_chunk_grid_u<Vpt<T>::v>(ncells, nv);
}



// ---------------------------------------------------------------------------
// Step 1: equilibrium initial state
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_eq_from_W(const double* W0, int per_cell, GasC g, int64_t nc, double* eq) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const double* w = per_cell ? W0 + 6 * i : W0;
  Prim p = prim_of(w, g.R);
  double q0[6] = {0, 0, 0, 0, 0, 0};
  eq_coeffs(p, q0, g, eq + ER * i);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_fill_eq(Dev d, const double* eq, T* G, T* R, double* W, double* q,
                                                    const double* W0, int per_cell) {
  const CellChunk cc = cell_chunk(d.nc);
  if (cc.cell >= d.nc) return;
  const int64_t i = cc.cell;
  const int64_t nv = d.nv;
  if (cc.chunk == 0 && threadIdx.x < 6) {
    W[6 * i + threadIdx.x] = per_cell ? W0[6 * i + threadIdx.x] : W0[threadIdx.x];
    q[6 * i + threadIdx.x] = 0.0;
  }
  Eq<T> e;
  e.load(eq + ER * i);
  chunk_loop<T>(nv, cc.chunk, [&](int64_t k) {
    T ux, uy, uz, gs, rs;
    vel_t<T>(d, k, ux, uy, uz);
    e.eval(ux, uy, uz, gs, rs);
    G[i * nv + k] = gs;
    R[i * nv + k] = rs;
  });
}

template <class T>
void launch_init_eq(const Dev& d, const Bufs& b, const double* W0, int per_cell, double* eqtmp, hipStream_t st) {
  int nb = (int)((d.nc + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_eq_from_W, dim3(nb), dim3(kBlock), 0, st, W0, per_cell, d.gas, d.nc, eqtmp);
  hipLaunchKernelGGL(k_fill_eq<T>, cell_chunk_grid<T>(d.nc, d.nv), dim3(kBlock), 0, st, d, (const double*)eqtmp,
                     (T*)b.G, (T*)b.R, b.W, b.q, W0, per_cell);
}

// ---------------------------------------------------------------------------
// Step 2(a): least-squares gradient, Venkatakrishnan limiter and upwind reconstruction (Eq. 46).
// Workgroup (cell, velocity chunk); each (face, velocity) value phi_bar is written once, by its upwind cell.
// ---------------------------------------------------------------------------

// Stores of write-once streams (phi_bar of the reconstruction, Res, phi^{n+1}) are non-temporal, so that they
// do not push the row slices the same kernel re-reads out of the caches (measured: reconstruction and micro
// residual faster; the face kernel's flux rows are better stored normally).
template <class T> __device__ inline void st_stream(T* p, T v) { __builtin_nontemporal_store(v, p); }

// Division in the limiter function: exact in FP64; in FP32 the fast reciprocal form (a few ulp on a value that
// only scales a slope).
__device__ inline double lim_div(double a, double b) { return a / b; }
__device__ inline float lim_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// One distribution at one velocity: limited least-squares gradient of the cell and the upwind face values
// (written at dst[a] + k).  limiter 3 takes L from the frozen row Lin; Lcap (if set) receives L.
// With d2_a = grad . (x_f - x_i) (the unlimited gradient's increment to face a, which the limiter needs anyway)
// and ug = u . grad, the face value of Eq. 46 is phi + L (d2_a - s_f ug): two operations per face.
template <class T, int NF>
__device__ inline void recon_write(T phi, const T* pn, const int32_t* nb, const T* wx, const T* wy, const T* wz,
                                   const T* fx, const T* fy, const T* fz, const T* sf, T kh3, int limiter,
                                   const bool* up, T ux, T uy, T uz, T* const* dst, uint32_t k, const T* Lin,
                                   T* Lcap) {
  // dmax, dmin: the largest and smallest neighbour difference, or 0 (max_a phi_a - phi and min_a phi_a - phi
  // over the cell and its neighbours; taken over the differences, which need no NaN canonicalisation as the
  // loaded values would)
  T gx = 0, gy = 0, gz = 0, dmax = 0, dmin = 0;
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    if (nb[a] < 0) continue;
    const T dphi = pn[a] - phi;
    gx += wx[a] * dphi;
    gy += wy[a] * dphi;
    gz += wz[a] * dphi;
    dmax = vmax(dmax, dphi);
    dmin = vmin(dmin, dphi);
  }
  T d2[NF];
#pragma unroll
  for (int a = 0; a < NF; ++a) d2[a] = gx * fx[a] + gy * fy[a] + gz * fz[a];
  T L = 1;
  if (limiter == 3) {
    L = ld_row(Lin, k);
  } else if (limiter) {  // 1, 2, and 4 (the smaller of this value and the stored one, stored back)
    const T scale = vmax(fabs(phi + dmax), fabs(phi + dmin));  // max(|phi_max|, |phi_min|)
    const T eps2 = kh3 * scale * scale;
    // Venkatakrishnan's function of face a with the common factor d2_a divided out of both parts:
    // psi_a = (d1^2 + eps^2 + 2 d1 d2_a) / (d1^2 + 2 d2_a^2 + d1 d2_a + eps^2), d1 = dmax where d2_a > 0 and
    // dmin where d2_a < 0, and psi_a = 1 where d2_a = 0 (an unused slot has zero geometry, so d2 = 0).
    // L = min(1, min_a psi_a) needs only the two extreme faces: for d1 >= 0 fixed, min(1, psi) does not grow
    // with d2 > 0, since psi < 1 exactly where d2 > d1/2 and there dpsi/dd2 has the sign of
    // (d1^2 + eps^2)(d1 - 4 d2) - 4 d1 d2^2 < 0; the same holds with every sign reversed (d1 = dmin <= 0,
    // d2 < 0).  So the smallest value over the faces is at the largest positive d2 or at the most negative.
    T hi = d2[0], lo = d2[0];
#pragma unroll
    for (int a = 1; a < NF; ++a) {
      hi = vmax(hi, d2[a]);
      lo = vmin(lo, d2[a]);
    }
    if (hi > T(0)) {  // skipped by a whole wavefront where the field is locally uniform
      const T dd = hi + hi;
      L = vmin(L, lim_div(dmax * (dmax + dd) + eps2, dmax * (dmax + hi) + (dd * hi + eps2)));
    }
    if (lo < T(0)) {
      const T dd = lo + lo;
      L = vmin(L, lim_div(dmin * (dmin + dd) + eps2, dmin * (dmin + lo) + (dd * lo + eps2)));
    }
    if (limiter == 4) L = vmin(L, ld_row(Lin, k));
  }
  if (Lcap) *at_row(Lcap, k) = L;
  const T ug = ux * gx + uy * gy + uz * gz;
  // all face values and addresses first, then the stores, with every store's registers kept live to the last
  // (measured: the kernel is 13% slower when the stores wait for one another)
  T val[NF];
  T* adr[NF];
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    val[a] = phi + L * (d2[a] - sf[a] * ug);
    adr[a] = at_row(dst[a], k);
  }
#pragma unroll
  for (int a = 0; a < NF; ++a)
    if (up[a]) st_stream(adr[a], val[a]);
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    keep_live(val[a]);
    keep_live(adr[a]);
  }
}

// Every load of a thread's velocities is issued before its first store (the stores could alias later loads
// as far as the compiler knows); per-cell geometry is converted once into registers.  Rows are addressed
// from uniform base pointers with 32-bit element offsets.
template <class T, int NF> __global__ __launch_bounds__(kBlock) void k_recon(Dev d, Bufs b, T* cap) {
  using L = Lay<NF>;
  constexpr int U = VptRecon<T>::v;
  const CellChunk cc = cell_chunk(d.nc);
  if (cc.cell >= d.nc) return;
  const int64_t i = d.spatial[cc.cell];
  const int64_t nv = d.nv;
  const double* geo = d.cell_geo + L::CG * i;
  const T* G = (const T*)b.G;
  const T* R = (const T*)b.R;
  int32_t nb[NF];
  const T *rowG[NF], *rowR[NF];  // neighbour rows (the cell's own row at a boundary face)
  T *dstG[NF], *dstR[NF];        // face rows
  bool own[NF];
  T wx[NF], wy[NF], wz[NF], fx[NF], fy[NF], fz[NF], sf[NF];
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    nb[a] = d.cell_nb[NF * i + a];
    const int64_t srow = (int64_t)(nb[a] >= 0 ? nb[a] : i) * nv;
    rowG[a] = G + srow;
    rowR[a] = R + srow;
    const int64_t frow = (int64_t)d.cell_face[NF * i + a] * nv;  // unused slot: never written (its code is 0)
    dstG[a] = (T*)b.faceG + frow;
    dstR[a] = (T*)b.faceR + frow;
    const double* s = geo + CG_FACE + CG_SLOT * a;
    own[a] = s[0] > 0.0;
    if constexpr (std::is_same<T, float>::value) {
      // the FP32 copy: used straight from scalar registers, no conversions
      const float* sg = d.cell_geo_f + L::CGF * i + 7 * a;
      fx[a] = sg[0];
      fy[a] = sg[1];
      fz[a] = sg[2];
      sf[a] = sg[3];
      wx[a] = sg[4];
      wy[a] = sg[5];
      wz[a] = sg[6];
    } else {
      fx[a] = s[5];
      fy[a] = s[6];
      fz[a] = s[7];
      sf[a] = s[8];
      wx[a] = s[9];
      wy[a] = s[10];
      wz[a] = s[11];
    }
  }
  double kh3d = d.lim_K * geo[2];
  kh3d = kh3d * kh3d * kh3d;
  const T kh3 = (T)kh3d;
  const int limiter = cap ? 1 : d.limiter;
  const int64_t self = i * nv;
  const int64_t P = d.nc * nv;
  const bool stored = limiter == 3 || limiter == 4;
  const T* LinG = stored ? (const T*)d.lim_frozen + self : nullptr;
  const T* LinR = stored ? LinG + P : nullptr;
  // limiter 4 writes the smaller value back in place (each (cell, velocity) entry has one thread)
  T* capG = cap ? cap + self : limiter == 4 ? (T*)d.lim_frozen + self : nullptr;
  T* capR = cap ? cap + P + self : limiter == 4 ? (T*)d.lim_frozen + P + self : nullptr;
  const T* selfG = G + self;
  const T* selfR = R + self;
  const T* ux_row = std::is_same<T, float>::value ? (const T*)d.dvs_f : (const T*)d.dvs;
  const T* uy_row = ux_row + nv;
  const T* uz_row = ux_row + 2 * nv;
  const typename L::Code* upw = reinterpret_cast<const typename L::Code*>(d.upw) + self;
  const uint32_t nvi = (uint32_t)nv;
  const uint32_t k0 = (uint32_t)cc.chunk * (kBlock * U) + threadIdx.x;
  T pG[U], pR[U], nG[U][NF], nR[U][NF], tx[U], ty[U], tz[U];
  unsigned code[U];
  bool up[U][NF];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t k = k0 + u * kBlock;
    if (k >= nvi) continue;
    code[u] = ld_row(upw, k);
    tx[u] = ld_row(ux_row, k);
    ty[u] = ld_row(uy_row, k);
    tz[u] = ld_row(uz_row, k);
    pG[u] = ld_row(selfG, k);
    pR[u] = ld_row(selfR, k);
#pragma unroll
    for (int a = 0; a < NF; ++a) {
      nG[u][a] = ld_row(rowG[a], k);
      nR[u][a] = ld_row(rowR[a], k);
    }
  }
  // upwind cell of the face for this velocity: the owner when u.n_face > 0, else the neighbour (a tie goes to
  // the neighbour); the code of slot a holds the sign of u.n out of this cell
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (k0 + u * kBlock >= nvi) continue;
#pragma unroll
    for (int a = 0; a < NF; ++a) {
      const unsigned c = (code[u] >> (2 * a)) & 3u;
      up[u][a] = nb[a] >= 0 ? (own[a] ? c == 1u : c != 2u) : c == 1u;
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t k = k0 + u * kBlock;
    if (k >= nvi) continue;
    recon_write<T, NF>(pG[u], nG[u], nb, wx, wy, wz, fx, fy, fz, sf, kh3, limiter, up[u], tx[u], ty[u], tz[u],
                       dstG, k, LinG, capG);
    recon_write<T, NF>(pR[u], nR[u], nb, wx, wy, wz, fx, fy, fz, sf, kh3, limiter, up[u], tx[u], ty[u], tz[u],
                       dstR, k, LinR, capR);
  }
}

template <class T> void launch_recon(const Dev& d, const Bufs& b, hipStream_t st, void* cap) {
  if (d.mf == 4)
    hipLaunchKernelGGL((k_recon<T, 4>), cell_chunk_grid_u<VptRecon<T>::v>(d.nc, d.nv), dim3(kBlock), 0, st, d, b, (T*)cap);
  else
    hipLaunchKernelGGL((k_recon<T, kMaxFaces>), cell_chunk_grid_u<VptRecon<T>::v>(d.nc, d.nv), dim3(kBlock), 0, st, d, b,
                       (T*)cap);
}

// ---------------------------------------------------------------------------
// Steps 2(b)-(e) and 3 on one face per workgroup: face moments (Eqs. 47-52), face equilibrium,
// collision-coupled face distribution (Eq. 45), micro flux A (u.n) phi_f (written in place over phi_bar)
// and the face's macro flux A sum_k w (u.n) Phi phi_f (Eq. 37).  Boundary faces: diffuse wall with rho_w
// from zero net mass flux, or far-field Maxwellian, for incoming velocities.  phi_bar is staged in LDS
// (Stage = 3: G, R and the upwind codes by LDS-DMA, 2: G and R, 0: the first velocities of G and R) or re-read
// from global memory in pass 2; the interior passes issue the loads of Prefetch<T> velocities per thread before
// their arithmetic, the other velocity loops kUnroll per trip.  The face sums are plain FP64 (each face flux is computed once and applied with opposite signs to its two
// cells, so conservation does not depend on their rounding; compensating them was measured at +40% face time).
// ---------------------------------------------------------------------------

#ifndef CIS_UNROLL
#define CIS_UNROLL 2
#endif
constexpr int kUnroll = CIS_UNROLL;

// Velocity loop of a per-face / per-cell workgroup of NT threads over all nv velocities, kUnroll independent
// velocities per trip.
template <int NT = kBlock, class F> __device__ inline void k_loop(int64_t nv, F&& body) {
  const int n = (int)nv;
  for (int k0 = threadIdx.x; k0 < n; k0 += kUnroll * NT) {
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const int k = k0 + q * NT;
      if (k < n) body(k);
    }
  }
}

// The same loop with the loads of P velocities per thread issued before any of their arithmetic:
// load(k, q) fills the registers of slot q (loads only), body(k, q) consumes them.  A face workgroup that
// loops over a whole row is otherwise bound by one memory round trip per trip (measured: face kernel -12%;
// the update kernel loses occupancy with it and is not faster).  P = 3 in FP32 (on the sphere, with the rows
// staged by LDS-DMA: face 2.79 ms against 2.86 with P = 4; before the staging 2 and 8 were slower than 4) and
// 1 in FP64 (512-thread workgroups over staged rows: 4.08 ms against 4.09 with P = 2).
template <class T> struct Prefetch { static constexpr int v = sizeof(T) == 4 ? 3 : 1; };
// The same over the velocities [begin, end), begin a multiple of NT.
template <int P, int NT = kBlock, class L, class B>
__device__ inline void k_loop_pf_range(int64_t begin, int64_t end, L&& load, B&& body) {
  const int n = (int)end;
  for (int k0 = (int)begin + threadIdx.x; k0 < n; k0 += P * NT) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int k = k0 + q * NT;
      if (k < n) load(k, q);
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int k = k0 + q * NT;
      if (k < n) body(k, q);
    }
  }
}
template <int P, int NT = kBlock, class L, class B> __device__ inline void k_loop_pf(int64_t nv, L&& load, B&& body) {
  k_loop_pf_range<P, NT>(0, nv, load, body);
}

// The DVS arrays as uniform row pointers (32-bit velocity offsets)
struct DvsRows {
  const double *ux, *uy, *uz, *w, *um, *h2;
};
__device__ inline DvsRows dvs_rows(const Dev& d) {
  const double* v = d.dvs;
  const int64_t n = d.nv;
  return DvsRows{v, v + n, v + 2 * n, v + 3 * n, v + 4 * n, v + 5 * n};
}
__device__ inline Vel vel(const DvsRows& V, int k) { return Vel{V.ux[k], V.uy[k], V.uz[k], V.w[k], V.um[k], V.h2[k]}; }


// Face state after the collision coupling (Eqs. 47-52) from the 17 moment sums of pass 1 about U0, and the
// coefficients of its equilibrium: ec[0..27] as eq_coeffs, ec[28] = tau/(tau+s), ec[29] = s/(tau+s).
// (Its FP64 temporaries set the face kernel's register peak; an out-of-line call was measured slower.)
__device__ inline void face_state_coeffs(const double* m, const double* U0, double s, const GasC& g, double* ec) {
  const double rho = m[0];
  const double dl[3] = {m[1] / rho, m[2] / rho, m[3] / rho};
  const double U[3] = {U0[0] + dl[0], U0[1] + dl[1], U0[2] + dl[2]};
  const double trM = m[4] + m[5] + m[6];
  const double mdl = m[1] * dl[0] + m[2] * dl[1] + m[3] * dl[2];
  const double eint = 0.5 * (trM - mdl) + m[13];  // rho E - rho |U|^2 / 2
  const double Er = m[13];
  const double rR = rho * g.R;
  Prim p;
  p.rho = rho;
  p.U[0] = U[0];
  p.U[1] = U[1];
  p.U[2] = U[2];
  p.T = 0.4 * eint / rR;
  const double Ttr_bar = (2.0 / 3.0) * (eint - Er) / rR;
  const double tau = visc(Ttr_bar, g) / (rR * Ttr_bar);
  const double Erot = (g.Z * tau * Er + s * rR * p.T) / (g.Z * tau + s);  // Eq. 50
  p.Trot = Erot / rR;
  p.Ttr = (2.0 / 3.0) * (eint - Erot) / rR;
  // heat fluxes, Eqs. 51-52
  const double Mx[3] = {m[4] * dl[0] + m[7] * dl[1] + m[8] * dl[2], m[7] * dl[0] + m[5] * dl[1] + m[9] * dl[2],
                        m[8] * dl[0] + m[9] * dl[1] + m[6] * dl[2]};
  const double d2 = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
  const double den_tr = tau + s - (s / 3.0) * (1.0 - 1.0 / g.Z + g.omega0 / g.Z);
  const double den_rot = tau + s - s * (1.0 - g.delta) * (1.0 - 1.0 / g.Z + g.omega1 / g.Z);
  double q[6];
  for (int e2 = 0; e2 < 3; ++e2) {
    const double sq3 = m[10 + e2] - 2.0 * Mx[e2] - dl[e2] * trM + 2.0 * rho * d2 * dl[e2];
    const double sr = m[14 + e2] - dl[e2] * m[13];
    q[e2] = tau * 0.5 * sq3 / den_tr;
    q[3 + e2] = tau * sr / den_rot;
  }
  eq_coeffs(p, q, g, ec);
  ec[28] = tau / (tau + s);
  ec[29] = s / (tau + s);
}

// LDS staging of one face row: at most 38 KB per 256-thread workgroup (with the kernel's 1.2 KB of static LDS,
// four face workgroups still share a CU's 160 KB), or 77 KB per 512-thread workgroup (two per CU: the same 16
// wavefronts).  Stage 0 stages the first kStagePrefix<T> velocities of G and R (a multiple of the workgroup
// size) when not even the wide budget holds both rows.
constexpr int64_t kLdsStageMax = 38 * 1024;
constexpr int64_t kLdsStageWide = 77 * 1024;
constexpr int kFaceWide = 2 * kBlock;
template <class T> constexpr int64_t kStagePrefix = kLdsStageMax / (2 * (int64_t)sizeof(T)) / kBlock * kBlock;

// Stage 3: G, R and the owner's upwind codes are copied into LDS by LDS-DMA loads (global_load_lds), all
// issued before any arithmetic, so the row costs one memory round trip instead of one per loop trip.
typedef __attribute__((address_space(1))) const void* GlobalPtr;
typedef __attribute__((address_space(3))) void* LdsPtr;

// Copy n bytes (n a multiple of 4 * Dw, src and dst aligned to 4 * Dw bytes) from global memory into LDS with
// LDS-DMA loads of Dw dwords per lane: wavefront w of the NT-thread block copies 64-lane blocks w, w + NT/64,
// ...; a lane past the end is inactive and writes nothing.
template <int Dw, int NT> __device__ inline void lds_dma_copy(const void* src, void* dst, int64_t n) {
  static_assert(Dw == 1 || Dw == 4, "LDS-DMA loads of 4 or 16 bytes per lane");
  constexpr int kLane = 4 * Dw, kWave = 64 * kLane;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t nblk = (n + kWave - 1) / kWave;
  for (int64_t blk = wid; blk < nblk; blk += NT / 64) {
    const int64_t off = blk * kWave + (int64_t)lane * kLane;
    if (off < n) {
      const GlobalPtr g = (GlobalPtr)((const char*)src + off);
      const LdsPtr l = (LdsPtr)((char*)dst + blk * kWave);
      if constexpr (Dw == 4)
        __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
      else
        __builtin_amdgcn_global_load_lds(g, l, 4, 0, 0);
    }
  }
}

template <class T, int Stage, int NF, int NT>
__global__ __launch_bounds__(NT) void k_face(Dev d, Bufs b, Work w) {
  static_assert(Stage == 0 || Stage == 2 || Stage == 3, "staging paths 0, 2, 3");
  static_assert(Stage != 0 || NT == kBlock, "prefix staging runs 256-thread workgroups");
  using Code = typename Lay<NF>::Code;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sG = reinterpret_cast<T*>(smem_raw);
  T* sR = sG + d.nv;                                // Stage >= 2
  Code* sC = reinterpret_cast<Code*>(sR + d.nv);  // Stage 3
  // Stage 0: velocities [0, M) of G and R staged at sG and sG + M
  const int64_t M = Stage == 0 ? (d.nv < kStagePrefix<T> ? d.nv : kStagePrefix<T>) : 0;
  T* sR0 = sG + M;
  __shared__ double red[(NT / 64) * 6];
  __shared__ double red17[(NT / 64) * 17];
  const int64_t f = blockIdx.x;
  const int64_t nv = d.nv;
  const double* fg = d.face_geo + FGW * f;
  const double A = fg[0], nx = fg[1], ny = fg[2], nz = fg[3], s = fg[4];
  T* rowG = (T*)b.faceG + f * nv;
  T* rowR = (T*)b.faceR + f * nv;
  const int32_t bcs = d.face_bc[f];
  const GasC& g = d.gas;
  const DvsRows V = dvs_rows(d);
  Acc<6, false, NT> acc;
  __shared__ double tot[6];

  if (bcs < 0) {
    // pass 1: the moments of Eqs. 47-49 and 51-52 in one sweep, taken about a reference velocity U0 (the mean
    // of the two cells' velocities), v = u - U0: m0 = sum w G, m = sum w v G, M = sum w v v G,
    // T3 = sum w v|v|^2 G, r0 = sum w R, r = sum w v R.  With delta = U_f - U0 = m/m0 the sums about the face
    // velocity follow exactly:  sum w c|c|^2 G = T3 - 2 M delta - delta tr(M) + 2 m0 |delta|^2 delta,
    // sum w c R = r - delta r0,  and the internal energy rho E - rho|U|^2/2 = tr(M)/2 - m.delta/2 + r0.
    const double* Wo = b.W + 6 * (int64_t)d.face_cell[2 * f];
    const double* Wn = b.W + 6 * (int64_t)d.face_cell[2 * f + 1];
    const double U0[3] = {0.5 * (Wo[1] / Wo[0] + Wn[1] / Wn[0]), 0.5 * (Wo[2] / Wo[0] + Wn[2] / Wn[0]),
                          0.5 * (Wo[3] / Wo[0] + Wn[3] / Wn[0])};
    const int64_t own = d.face_cell[2 * f];
    const Code* code = reinterpret_cast<const Code*>(d.upw) + own * nv;
    if constexpr (Stage == 3) {
      lds_dma_copy<4, NT>(rowG, sG, nv * (int64_t)sizeof(T));
      lds_dma_copy<4, NT>(rowR, sR, nv * (int64_t)sizeof(T));
      lds_dma_copy<1, NT>(code, sC, nv * (int64_t)sizeof(Code));
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    Acc<17, false, NT> a17;
    a17.zero();
    constexpr int P = Prefetch<T>::v;
    T pg[P], pr[P];
    double px[P], py[P], pz[P], pw[P];
    auto load1 = [&](int k, int q) {
      pg[q] = Stage == 3 ? sG[k] : rowG[k];
      pr[q] = Stage == 3 ? sR[k] : rowR[k];
      px[q] = V.ux[k];
      py[q] = V.uy[k];
      pz[q] = V.uz[k];
      pw[q] = V.w[k];
    };
    auto body1 = [&](auto prefix, int k, int q) {
      const T gb = pg[q], rb = pr[q];
      if (Stage == 2) {
        sG[k] = gb;
        sR[k] = rb;
      }
      if constexpr (decltype(prefix)::value) {
        sG[k] = gb;
        sR0[k] = rb;
      }
      const double vx = px[q] - U0[0], vy = py[q] - U0[1], vz = pz[q] - U0[2], w = pw[q];
      const double wg = w * (double)gb, wr = w * (double)rb;
      const double gx = wg * vx, gy = wg * vy, gz = wg * vz, v2 = vx * vx + vy * vy + vz * vz;
      a17.add(0, wg);
      a17.add(1, gx);
      a17.add(2, gy);
      a17.add(3, gz);
      a17.add(4, gx * vx);
      a17.add(5, gy * vy);
      a17.add(6, gz * vz);
      a17.add(7, gx * vy);
      a17.add(8, gx * vz);
      a17.add(9, gy * vz);
      a17.add(10, gx * v2);
      a17.add(11, gy * v2);
      a17.add(12, gz * v2);
      a17.add(13, wr);
      a17.add(14, wr * vx);
      a17.add(15, wr * vy);
      a17.add(16, wr * vz);
    };
    if constexpr (Stage == 0) {
      k_loop_pf_range<P>(0, M, load1, [&](int k, int q) { body1(std::true_type{}, k, q); });
      k_loop_pf_range<P>(M, nv, load1, [&](int k, int q) { body1(std::false_type{}, k, q); });
    } else {
      k_loop_pf<P, NT>(nv, load1, [&](int k, int q) { body1(std::false_type{}, k, q); });
    }
    __shared__ double sh_m[17];
    a17.reduce_to_lds(sh_m, red17);
    // the face state (Eqs. 47-52) and its equilibrium coefficients, computed by one thread, shared through LDS
    __shared__ double sh_ec[ER];
    if (threadIdx.x == 0) face_state_coeffs(sh_m, U0, s, g, sh_ec);
    __syncthreads();
    Eq<T> e;  // s/(tau+s) times the face equilibrium
    e.load(sh_ec, sh_ec[29]);
    const T ct = (T)sh_ec[28];
    // pass 2: phi_f (Eq. 45), micro flux and macro flux.  The upwind side (with its tie rule) is the owner's
    // upwind code, as in the reconstruction, and A u.n is the plain FP64 product with the area-scaled normal;
    // |u|^2 is formed in registers (fewer cached DVS loads per velocity).  The energy sum runs as
    // sum w (A u.n) G_f |u|^2 alone; the half and the rotational part sum w (A u.n) R_f are added once after
    // the reduction.
    const double an_x = A * nx, an_y = A * ny, an_z = A * nz;
    int slot = 0;
    for (int a = 1; a < NF; ++a)
      if (d.cell_face[NF * own + a] == (int32_t)f) slot = a;
    acc.zero();
    unsigned pc[P];
    auto load2 = [&](auto prefix, int k, int q) {
      if constexpr (decltype(prefix)::value) {
        pg[q] = sG[k];
        pr[q] = sR0[k];
      } else {
        pg[q] = Stage >= 2 ? sG[k] : rowG[k];
        pr[q] = Stage >= 2 ? sR[k] : rowR[k];
      }
      px[q] = V.ux[k];
      py[q] = V.uy[k];
      pz[q] = V.uz[k];
      pw[q] = V.w[k];
      pc[q] = Stage == 3 ? sC[k] : code[k];
    };
    auto body2 = [&](int k, int q) {
      const T gb = pg[q], rb = pr[q];
      const double ux = px[q], uy = py[q], uz = pz[q], vw = pw[q];
      T gs, rs;
      e.eval((T)ux, (T)uy, (T)uz, gs, rs);
      const T gf = ct * gb + gs;
      const T rf = ct * rb + rs;
      const double aun = ((pc[q] >> (2 * slot)) & 3u) == 0u ? 0.0 : ux * an_x + uy * an_y + uz * an_z;
      *at_row(rowG, (uint32_t)k) = (T)aun * gf;
      *at_row(rowR, (uint32_t)k) = (T)aun * rf;
      double wg = vw * aun * (double)gf, wr = vw * aun * (double)rf;
      acc.add(0, wg);
      acc.add(1, ux * wg);
      acc.add(2, uy * wg);
      acc.add(3, uz * wg);
      acc.add(4, (ux * ux + uy * uy + uz * uz) * wg);
      acc.add(5, wr);
    };
    if constexpr (Stage == 0) {
      k_loop_pf_range<P>(0, M, [&](int k, int q) { load2(std::true_type{}, k, q); }, body2);
      k_loop_pf_range<P>(M, nv, [&](int k, int q) { load2(std::false_type{}, k, q); }, body2);
    } else {
      k_loop_pf<P, NT>(nv, [&](int k, int q) { load2(std::false_type{}, k, q); }, body2);
    }
    acc.reduce_to_lds(tot, red);
    if (threadIdx.x < 6)
      w.face_mac[6 * f + threadIdx.x] = threadIdx.x == 4 ? 0.5 * tot[4] + tot[5] : tot[threadIdx.x];
  } else {
    const double* bc = d.bc + BCW * bcs;
    const bool wall = bc[0] == 1.0;
    const double Ub[3] = {bc[2], bc[3], bc[4]}, Tb = bc[5];
    const double RTb = g.R * Tb;
    double rho_g = bc[1];
    if (wall) {
      // rho_w from zero net mass flux through the wall
      Acc<2, false, NT> a2;
      a2.zero();
      const double anorm = maxwell_norm(RTb);
      k_loop<NT>(nv, [&](int k) {
        const Vel v = vel(V, k);
        const double un = udotn(v, nx, ny, nz, d.snap);
        if (un > 0.0) {
          a2.add(0, v.w * un * (double)rowG[k]);
        } else {
          double cx = v.ux - Ub[0], cy = v.uy - Ub[1], cz = v.uz - Ub[2];
          a2.add(1, v.w * (-un) * anorm * exp(-(cx * cx + cy * cy + cz * cz) / (2.0 * RTb)));
        }
      });
      double t2[2];
      a2.reduce(t2, red);
      rho_g = t2[0] / t2[1];
    }
    const T amax = (T)(rho_g * maxwell_norm(RTb));
    const T bmax = (T)(1.0 / (2.0 * RTb));
    acc.zero();
    k_loop<NT>(nv, [&](int k) {
      const Vel v = vel(V, k);
      const double un = udotn(v, nx, ny, nz, d.snap);
      T gf, rf;
      if (un > 0.0) {
        gf = rowG[k];
        rf = rowR[k];
      } else {
        T cx = (T)(v.ux - Ub[0]), cy = (T)(v.uy - Ub[1]), cz = (T)(v.uz - Ub[2]);
        gf = amax * eq_exp(-(cx * cx + cy * cy + cz * cz) * bmax);
        rf = (T)RTb * gf;
      }
      rowG[k] = (T)(A * un) * gf;
      rowR[k] = (T)(A * un) * rf;
      double wg = v.w * un * (double)gf, wr = v.w * un * (double)rf;
      acc.add(0, wg);
      acc.add(1, v.ux * wg);
      acc.add(2, v.uy * wg);
      acc.add(3, v.uz * wg);
      acc.add(4, v.h2 * wg + wr);
      acc.add(5, wr);
    });
    acc.reduce_to_lds(tot, red);
    if (threadIdx.x < 6) w.face_mac[6 * f + threadIdx.x] = A * tot[threadIdx.x];
  }
}

// phi_bar of one face is staged in LDS whole where it fits: in 38 KB with 256 threads per face (four face
// workgroups per CU), else in 77 KB with 512 threads per face (two per CU, the same 16 wavefronts), G, R and
// the owner's codes by LDS-DMA where the rows allow it, else G and R by ordinary stores; rows too long for both
// stage the first kStagePrefix<T> velocities of G and R (the capsule's FP32 rows, 42 KB each).  Measured on the
// sphere (4 140 velocities): FP32 rows (37 KB with the codes) run fastest at 256 threads; FP64 rows (69 KB with
// the codes) at 512 threads, where staging G alone at 256 threads re-read R from global memory and staging
// both at 256 threads halved the wavefronts per CU.
struct FacePlan {
  int stage, nt;
  size_t lds;
};
template <class T, int NF> static FacePlan face_plan(const Dev& d, const Bufs& b) {
  const int64_t nv = d.nv;
  const int64_t row = nv * (int64_t)sizeof(T);
  // LDS-DMA staging needs 16-byte aligned rows (aligned arrays, nv a multiple of 4), 4-byte aligned code rows
  // and room for the code row
  const int64_t code_row = nv * (int64_t)sizeof(typename Lay<NF>::Code);
  const bool dma = (uintptr_t)b.faceG % 16 == 0 && (uintptr_t)b.faceR % 16 == 0 && (uintptr_t)d.upw % 4 == 0 &&
                   nv % 4 == 0;
  const int64_t budget[2] = {kLdsStageMax, kLdsStageWide};
  const int nt[2] = {kBlock, kFaceWide};
  for (int i = 0; i < 2; ++i) {
    if (dma && 2 * row + code_row <= budget[i]) return FacePlan{3, nt[i], (size_t)(2 * row + code_row)};
    if (2 * row <= budget[i]) return FacePlan{2, nt[i], (size_t)(2 * row)};
  }
  return FacePlan{0, kBlock, (size_t)std::min<int64_t>(nv, kStagePrefix<T>) * 2 * sizeof(T)};
}

template <class T, int NF> void launch_face_nf(const Dev& d, const Bufs& b, const Work& w, hipStream_t st) {
  const FacePlan p = face_plan<T, NF>(d, b);
  const dim3 grid((unsigned)d.nf);
  if (p.stage == 3 && p.nt == kBlock)
    hipLaunchKernelGGL((k_face<T, 3, NF, kBlock>), grid, dim3(kBlock), p.lds, st, d, b, w);
  else if (p.stage == 3)
    hipLaunchKernelGGL((k_face<T, 3, NF, kFaceWide>), grid, dim3(kFaceWide), p.lds, st, d, b, w);
  else if (p.stage == 2 && p.nt == kBlock)
    hipLaunchKernelGGL((k_face<T, 2, NF, kBlock>), grid, dim3(kBlock), p.lds, st, d, b, w);
  else if (p.stage == 2)
    hipLaunchKernelGGL((k_face<T, 2, NF, kFaceWide>), grid, dim3(kFaceWide), p.lds, st, d, b, w);
  else
    hipLaunchKernelGGL((k_face<T, 0, NF, kBlock>), grid, dim3(kBlock), p.lds, st, d, b, w);
}

template <class T> void launch_face(const Dev& d, const Bufs& b, const Work& w, hipStream_t st) {
  if (d.mf == 4)
    launch_face_nf<T, 4>(d, b, w, st);
  else
    launch_face_nf<T, kMaxFaces>(d, b, w, st);
}

// ---------------------------------------------------------------------------
// Step 4: implicit macroscopic prediction (Eqs. 38-43), one thread per cell.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_cell_prim(Dev d, const double* W, Work w) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.nc) return;
  Prim p = prim_of(W + 6 * i, d.gas.R);
  double* o = w.cell_prim + 8 * i;
  o[0] = p.rho;
  o[1] = p.U[0];
  o[2] = p.U[1];
  o[3] = p.U[2];
  o[4] = p.T;
  o[5] = p.Ttr;
  o[6] = visc(p.Ttr, d.gas) / (p.rho * d.gas.R * p.Ttr);
  o[7] = 0.0;
}

// Macro flux per cell (Eq. 37), diagonal D_i and right-hand side Res_i of Eq. 43, spectral radii r_ij (Eq. 41)
template <int NF> __global__ __launch_bounds__(kBlock) void k_macro_prep(Dev d, const double* W, Work w) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.nc) return;
  const double* geo = d.cell_geo + Lay<NF>::CG * i;
  const double* pa = w.cell_prim + 8 * i;
  const GasC& g = d.gas;
  double F[6] = {0, 0, 0, 0, 0, 0};
  double acc = 0.0;
  for (int a = 0; a < NF; ++a) {
    const double* s = geo + CG_FACE + CG_SLOT * a;
    int32_t nb = d.cell_nb[NF * i + a];
    int32_t f = d.cell_face[NF * i + a];
    if (f < 0) {  // unused slot
      w.rcf[NF * i + a] = 0.0;
      continue;
    }
    const double* pb = nb >= 0 ? w.cell_prim + 8 * (int64_t)nb : pa;
    // face state: arithmetic mean of the two cells
    double rho = 0.5 * (pa[0] + pb[0]);
    double T = 0.5 * (pa[4] + pb[4]);
    double Ttr = 0.5 * (pa[5] + pb[5]);
    double Un = 0.5 * (pa[1] + pb[1]) * s[2] + 0.5 * (pa[2] + pb[2]) * s[3] + 0.5 * (pa[3] + pb[3]) * s[4];
    double r = fabs(Un) + sqrt(g.gamma * g.R * T) + 2.0 * visc(Ttr, g) / (rho * d.face_geo[FGW * (int64_t)f + 5]);
    w.rcf[NF * i + a] = r;
    acc += 0.5 * s[1] * r;
    // G_n(W_j^n) along the outward normal, constant during the sweeps
    if (nb >= 0) euler_flux(W + 6 * (int64_t)nb, s[2], s[3], s[4], w.G0 + 6 * NF * i + 6 * a);
    const double* fm = w.face_mac + 6 * (int64_t)f;
    for (int m = 0; m < 6; ++m) F[m] += s[0] * fm[m] * geo[1];
  }
  const double tau = pa[6];
  const double D = inv_dt_cell(d, geo[2]) + acc;
  w.mD[2 * i] = D;
  w.mD[2 * i + 1] = D + 1.0 / (g.Z * tau);
  for (int m = 0; m < 6; ++m) {
    w.Fmac[6 * i + m] = F[m];
    w.mres[6 * i + m] = -F[m];
    w.dW[6 * i + m] = 0.0;
  }
  w.mres[6 * i + 5] += (pa[0] * g.R * pa[4] - W[6 * i + 5]) / (g.Z * tau);
}

// One point relaxation of Eq. 43 per cell of one colour (matrix-free increment G(W_j + dW_j) - G(W_j)).  The
// sweep is latency bound: the four faces of a cell run on four consecutive lanes (each loads one neighbour
// and evaluates one flux increment), and the cell's first lane subtracts the four terms in face order.  A
// colour is ~N_c/5 cells, so small workgroups spread each launch over more CUs.
constexpr int kMacroBlock = 64;

// Lanes per cell: NF rounded up to a power of two (4 or 8); lanes past NF carry zero terms.
template <int NF> struct MacroLanes { static constexpr int n = NF <= 4 ? 4 : 8, shift = NF <= 4 ? 2 : 3; };

template <int NF>
__global__ __launch_bounds__(kMacroBlock) void k_macro_sweep(Dev d, const double* W, Work w, int64_t c0, int64_t c1) {
  constexpr int NL = MacroLanes<NF>::n;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = c0 + (t >> MacroLanes<NF>::shift);
  const int a = (int)(t & (NL - 1));
  const bool valid = i < c1;
  double term[6] = {0, 0, 0, 0, 0, 0};
  double acc[6], D = 1.0, D5 = 1.0;
  if (valid) {
    // the cell's right-hand side and diagonal are loaded up front, with the neighbour's state
    for (int m = 0; m < 6; ++m) acc[m] = w.mres[6 * i + m];
    D = w.mD[2 * i];
    D5 = w.mD[2 * i + 1];
    const int32_t nb = a < NF ? d.cell_nb[NF * i + a] : kNoFace;
    if (nb >= 0) {
      const double* s = d.cell_geo + Lay<NF>::CG * i + CG_FACE + CG_SLOT * a;
      double Wp[6], dWj[6], G1[6];
      for (int m = 0; m < 6; ++m) {
        dWj[m] = w.dW[6 * (int64_t)nb + m];
        Wp[m] = W[6 * (int64_t)nb + m] + dWj[m];
      }
      euler_flux(Wp, s[2], s[3], s[4], G1);
      const double* G0 = w.G0 + 6 * NF * i + 6 * a;
      const double r = w.rcf[NF * i + a];
      for (int m = 0; m < 6; ++m) term[m] = 0.5 * s[1] * ((G1[m] - G0[m]) - r * dWj[m]);
    }
  }
  double tn[NL][6];
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 1; q < NL; ++q)
    for (int m = 0; m < 6; ++m) tn[q][m] = __shfl(term[m], lane + q, 64);
  if (!valid || a != 0) return;
  for (int m = 0; m < 6; ++m) {
    acc[m] -= term[m];
#pragma unroll
    for (int q = 1; q < NF; ++q) acc[m] -= tn[q][m];
  }
  const double iD = 1.0 / D;  // one division on the cell's lane instead of five (measured: macro stage -2.6%)
  for (int m = 0; m < 5; ++m) w.dW[6 * i + m] = acc[m] * iD;
  w.dW[6 * i + 5] = acc[5] / D5;
}

// W~ = W^n + dW~; predicted equilibrium coefficients with q~ = q^n
template <int NF> __global__ __launch_bounds__(kBlock) void k_cell_eq(Dev d, const double* W, const double* q, Work w) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.nc) return;
  double Wt[6];
  for (int m = 0; m < 6; ++m) {
    Wt[m] = W[6 * i + m] + w.dW[6 * i + m];
    w.Wt[6 * i + m] = Wt[m];
  }
  Prim p = prim_of(Wt, d.gas.R);
  if (!(p.rho > 0.0) || !(p.T > 0.0) || !(p.Ttr > 0.0) || !(p.Trot > 0.0)) atomicOr(&w.flag[0], 1);
  double* e = w.eq + ER * i;
  eq_coeffs(p, q + 6 * i, d.gas, e);
  e[7] = visc(p.Ttr, d.gas) / (p.rho * d.gas.R * p.Ttr);
  w.mbase[i] = inv_dt_cell(d, d.cell_geo[Lay<NF>::CG * i + 2]) + 1.0 / e[7];
}

template <int NF> __global__ __launch_bounds__(kBlock) void k_macro_flux_cells(Dev d, Work w) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.nc) return;
  const double* geo = d.cell_geo + Lay<NF>::CG * i;
  double F[6] = {0, 0, 0, 0, 0, 0};
  for (int a = 0; a < NF; ++a) {
    const double* s = geo + CG_FACE + CG_SLOT * a;
    const int32_t f = d.cell_face[NF * i + a];
    if (f < 0) continue;
    const double* fm = w.face_mac + 6 * (int64_t)f;
    for (int m = 0; m < 6; ++m) F[m] += s[0] * fm[m] * geo[1];
  }
  for (int m = 0; m < 6; ++m) w.Fmac[6 * i + m] = F[m];
}

void launch_macro_flux_cells(const Dev& d, const Work& w, hipStream_t st) {
  int nb = (int)((d.nc + kBlock - 1) / kBlock);
  if (d.mf == 4)
    hipLaunchKernelGGL(k_macro_flux_cells<4>, dim3(nb), dim3(kBlock), 0, st, d, w);
  else
    hipLaunchKernelGGL(k_macro_flux_cells<kMaxFaces>, dim3(nb), dim3(kBlock), 0, st, d, w);
}

// Colour order of n_pairs forward + backward Gauss-Seidel passes over the non-empty colours.  A colour that
// follows itself (at each turn of direction) is relaxed only once: its neighbours, all of other colours, have
// not changed in between, so a second relaxation would reproduce the first bit for bit.
std::vector<int64_t> sweep_sequence(const int64_t* color_off, int64_t n_colors, int n_pairs) {
  std::vector<int64_t> seq;
  auto push = [&](int64_t c) {
    if (color_off[c + 1] <= color_off[c]) return;
    if (!seq.empty() && seq.back() == c) return;
    seq.push_back(c);
  };
  for (int it = 0; it < n_pairs; ++it) {
    for (int64_t c = 0; c < n_colors; ++c) push(c);
    for (int64_t c = n_colors - 1; c >= 0; --c) push(c);
  }
  return seq;
}

template <int NF>
void launch_macro_nf(const Dev& d, const Bufs& b, const Work& w, const int64_t* color_off, int64_t n_colors,
                     int n_macro, hipStream_t st) {
  int nb = (int)((d.nc + kBlock - 1) / kBlock);
  constexpr int NL = MacroLanes<NF>::n;
  hipLaunchKernelGGL(k_cell_prim, dim3(nb), dim3(kBlock), 0, st, d, (const double*)b.W, w);
  hipLaunchKernelGGL(k_macro_prep<NF>, dim3(nb), dim3(kBlock), 0, st, d, (const double*)b.W, w);
  for (const int64_t c : sweep_sequence(color_off, n_colors, n_macro)) {
    const int64_t n = color_off[c + 1] - color_off[c];
    hipLaunchKernelGGL(k_macro_sweep<NF>, dim3((unsigned)((NL * n + kMacroBlock - 1) / kMacroBlock)),
                       dim3(kMacroBlock), 0, st, d, (const double*)b.W, w, color_off[c], color_off[c + 1]);
  }
  hipLaunchKernelGGL(k_cell_eq<NF>, dim3(nb), dim3(kBlock), 0, st, d, (const double*)b.W, (const double*)b.q, w);
}

void launch_macro(const Dev& d, const Bufs& b, const Work& w, const int64_t* color_off, int64_t n_colors, int n_macro,
                  hipStream_t st) {
  if (d.mf == 4)
    launch_macro_nf<4>(d, b, w, color_off, n_colors, n_macro, st);
  else
    launch_macro_nf<kMaxFaces>(d, b, w, color_off, n_colors, n_macro, st);
}

// ---------------------------------------------------------------------------
// Step 4-5: micro flux per cell (Eq. 31) and right-hand side of Eq. 33, Res = (phi~* - phi)/tau~ - F.
// flux_only = 1 writes F instead (explicit operator).  Workgroup (cell, velocity chunk).
// ---------------------------------------------------------------------------

// Eq. 31 of one cell and velocity: the signed sum of the face fluxes, in slot order (left to right).
template <class T, int NF> __device__ inline T face_sum(const T* sg, const T* x) {
  T acc = sg[0] * x[0];
#pragma unroll
  for (int a = 1; a < NF; ++a) acc += sg[a] * x[a];
  return acc;
}

template <class T, int NF>
__global__ __launch_bounds__(kBlock) void k_residual(Dev d, Bufs b, Work w, T* outG, T* outR, int flux_only) {
  constexpr int U = Vpt<T>::v;
  const CellChunk cc = cell_chunk(d.nc);
  if (cc.cell >= d.nc) return;
  const int64_t i = d.spatial[cc.cell];
  const int64_t nv = d.nv;
  const double* geo = d.cell_geo + Lay<NF>::CG * i;
  const T *fG[NF], *fR[NF];
  T sg[NF];
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    // an unused slot reads the first face's row with a zero sign (its geometry is zero)
    const int32_t fa = d.cell_face[NF * i + a];
    const int64_t f = fa >= 0 ? fa : d.cell_face[NF * i];
    fG[a] = (const T*)b.faceG + f * nv;
    fR[a] = (const T*)b.faceR + f * nv;
    sg[a] = (T)(geo[CG_FACE + CG_SLOT * a] * geo[1]);
  }
  const int nvi = (int)nv;
  const int k0 = (int)cc.chunk * (kBlock * U) + (int)threadIdx.x;
  T* oG = outG + i * nv;
  T* oR = outR + i * nv;
  T xG[U][NF], xR[U][NF];
  if (flux_only) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * kBlock;
      if (k >= nvi) continue;
#pragma unroll
      for (int a = 0; a < NF; ++a) {
        xG[u][a] = fG[a][k];
        xR[u][a] = fR[a][k];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * kBlock;
      if (k >= nvi) continue;
      oG[k] = face_sum<T, NF>(sg, xG[u]);
      oR[k] = face_sum<T, NF>(sg, xR[u]);
    }
    return;
  }
  const double* ec = w.eq + ER * i;
  Eq<T> e;
  e.load(ec);
  const T itau = (T)(1.0 / ec[7]);
  const T* G = (const T*)b.G + i * nv;
  const T* R = (const T*)b.R + i * nv;
  T pG[U], pR[U], ux[U], uy[U], uz[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = k0 + u * kBlock;
    if (k >= nvi) continue;
#pragma unroll
    for (int a = 0; a < NF; ++a) {
      xG[u][a] = fG[a][k];
      xR[u][a] = fR[a][k];
    }
    pG[u] = G[k];
    pR[u] = R[k];
    vel_t<T>(d, k, ux[u], uy[u], uz[u]);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = k0 + u * kBlock;
    if (k >= nvi) continue;
    const T FG = face_sum<T, NF>(sg, xG[u]);
    const T FR = face_sum<T, NF>(sg, xR[u]);
    T gs, rs;
    e.eval(ux[u], uy[u], uz[u], gs, rs);
    st_stream(oG + k, (gs - pG[u]) * itau - FG);
    st_stream(oR + k, (rs - pR[u]) * itau - FR);
  }
}

template <class T, int V> struct alignas(sizeof(T) * V) VecR { T v[V]; };

// The micro residual with V adjacent velocities per thread moved as 16-byte vectors (four FP32 or two FP64
// values; nv a multiple of V and 16-byte aligned rows, so every row offset keeps them aligned), Res stored
// non-temporally; the arithmetic of k_residual<T>, velocity by velocity.  Measured on the sphere (4140
// velocities): mixed 1.68 -> 1.50 ms with V = 4; FP64 4.10 -> 2.89 ms with V = 2.
template <class T, int V, int NF>
__global__ __launch_bounds__(kBlock) void k_residual_vec(Dev d, Bufs b, Work w, T* outG, T* outR) {
  const CellChunk cc = cell_chunk(d.nc);
  if (cc.cell >= d.nc) return;
  const int64_t i = d.spatial[cc.cell];
  const int64_t nv = d.nv;
  const int k = (int)cc.chunk * (V * kBlock) + V * (int)threadIdx.x;
  if (k >= (int)nv) return;
  using VF = VecR<T, V>;
  const double* geo = d.cell_geo + Lay<NF>::CG * i;
  VF xG[NF], xR[NF];
  T sg[NF];
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    const int32_t fa = d.cell_face[NF * i + a];
    const int64_t f = fa >= 0 ? fa : d.cell_face[NF * i];
    xG[a] = *reinterpret_cast<const VF*>((const T*)b.faceG + f * nv + k);
    xR[a] = *reinterpret_cast<const VF*>((const T*)b.faceR + f * nv + k);
    sg[a] = (T)(geo[CG_FACE + CG_SLOT * a] * geo[1]);
  }
  const VF pG = *reinterpret_cast<const VF*>((const T*)b.G + i * nv + k);
  const VF pR = *reinterpret_cast<const VF*>((const T*)b.R + i * nv + k);
  const T* dvs = std::is_same<T, float>::value ? (const T*)d.dvs_f : (const T*)d.dvs;
  const VF ux = *reinterpret_cast<const VF*>(dvs + k);
  const VF uy = *reinterpret_cast<const VF*>(dvs + nv + k);
  const VF uz = *reinterpret_cast<const VF*>(dvs + 2 * nv + k);
  const double* ec = w.eq + ER * i;
  Eq<T> e;
  e.load(ec);
  const T itau = (T)(1.0 / ec[7]);
  VF oG, oR;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    T FG = sg[0] * xG[0].v[q], FR = sg[0] * xR[0].v[q];
#pragma unroll
    for (int a = 1; a < NF; ++a) {
      FG += sg[a] * xG[a].v[q];
      FR += sg[a] * xR[a].v[q];
    }
    T gs, rs;
    e.eval(ux.v[q], uy.v[q], uz.v[q], gs, rs);
    oG.v[q] = (gs - pG.v[q]) * itau - FG;
    oR.v[q] = (rs - pR.v[q]) * itau - FR;
  }
  typedef T ev __attribute__((ext_vector_type(V)));
  ev sG, sR;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    sG[q] = oG.v[q];
    sR[q] = oR.v[q];
  }
  __builtin_nontemporal_store(sG, reinterpret_cast<ev*>(outG + i * nv + k));
  __builtin_nontemporal_store(sR, reinterpret_cast<ev*>(outR + i * nv + k));
}

// Whether every row of the distribution, right-hand side and face arrays keeps V-element vectors of T aligned
// to their size (nv a multiple of V, arrays aligned to V sizeof(T) bytes): the condition of the vector kernels
// of the micro residual and sweep; otherwise the scalar kernels run.
template <class T> static bool rows_aligned(const Dev& d, const Bufs& b, int V) {
  const void* p[8] = {b.G, b.R, b.dG, b.dR, b.resG, b.resR, b.faceG, b.faceR};
  const uintptr_t bytes = sizeof(T) * (uintptr_t)V;
  bool ok = d.nv % V == 0;
  for (const void* x : p) ok = ok && (uintptr_t)x % bytes == 0;
  return ok;
}

template <class T, int NF>
void launch_residual_nf(const Dev& d, const Bufs& b, const Work& w, void* outG, void* outR, int flux_only,
                        hipStream_t st) {
  constexpr int V = 16 / sizeof(T);
  if (!flux_only && rows_aligned<T>(d, b, V) && (uintptr_t)outG % 16 == 0 && (uintptr_t)outR % 16 == 0) {
    hipLaunchKernelGGL((k_residual_vec<T, V, NF>), cell_chunk_grid_u<V>(d.nc, d.nv), dim3(kBlock), 0, st, d, b, w,
                       (T*)outG, (T*)outR);
    return;
  }
  if (std::is_same<T, float>::value && !flux_only && rows_aligned<T>(d, b, 2) && (uintptr_t)outG % 8 == 0 &&
      (uintptr_t)outR % 8 == 0) {
    hipLaunchKernelGGL((k_residual_vec<float, 2, NF>), cell_chunk_grid_u<2>(d.nc, d.nv), dim3(kBlock), 0, st, d, b,
                       w, (float*)outG, (float*)outR);
    return;
  }
  hipLaunchKernelGGL((k_residual<T, NF>), cell_chunk_grid<T>(d.nc, d.nv), dim3(kBlock), 0, st, d, b, w, (T*)outG,
                     (T*)outR, flux_only);
}

template <class T>
void launch_residual(const Dev& d, const Bufs& b, const Work& w, void* outG, void* outR, int flux_only, hipStream_t st) {
  if (d.mf == 4)
    launch_residual_nf<T, 4>(d, b, w, outG, outR, flux_only, st);
  else
    launch_residual_nf<T, kMaxFaces>(d, b, w, outG, outR, flux_only, st);
}

// ---------------------------------------------------------------------------
// Step 5: PR-SGS sweep of Eq. 33 over one colour, first-order upwind increments (Eq. 32).
// D_ik = 1/dt_i + 1/tau~_i + sum_f (A/V) max(u.n, 0) in FP64.  In the first forward sweep the
// increments of later colours are still zero and are not read.  Workgroup (cell, velocity chunk).
// ---------------------------------------------------------------------------

// Per-cell operands of one relaxation.  The signs of u.n come from the upwind codes (the same decisions as in
// every other kernel); the magnitudes u.n are computed in the precision of the distributions (FP32 in the
// mixed mode; the increments of the sweep only steer the iteration, its fixed point is set by Res).  The
// diagonal D = 1/dt + 1/tau~ + sum_f (A/V) max(u.n, 0) is summed and inverted in FP64 in both modes.
template <class T, int NF> struct MicroCell {
  const T *nG[NF], *nR[NF], *rG, *rR;
  T *oG, *oR;
  T nx[NF], ny[NF], nz[NF], av[NF];
  double dbase;  // 1/dt + 1/tau~
  bool use[NF];
};

template <class T, int NF>
__device__ inline void micro_setup(const Dev& d, const Bufs& b, const Work& w, int64_t i, int64_t cnext, int first,
                                   MicroCell<T, NF>& c) {
  const int64_t nv = d.nv;
  const double* geo = d.cell_geo + Lay<NF>::CG * i;
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    const int32_t nb = d.cell_nb[NF * i + a];
    c.use[a] = nb >= 0 && !(first && nb >= cnext);
    const int64_t row = (nb >= 0 ? nb : i) * nv;
    c.nG[a] = (const T*)b.dG + row;
    c.nR[a] = (const T*)b.dR + row;
    const double* s = geo + CG_FACE + CG_SLOT * a;
    c.nx[a] = (T)s[2];
    c.ny[a] = (T)s[3];
    c.nz[a] = (T)s[4];
    c.av[a] = (T)s[1];
  }
  c.dbase = w.mbase[i];
  c.rG = (const T*)b.resG + i * nv;
  c.rR = (const T*)b.resR + i * nv;
  c.oG = (T*)b.dG + i * nv;
  c.oR = (T*)b.dR + i * nv;
}

// Values a relaxation reads: the outflow part max(u.n, 0) and inflow part min(u.n, 0) per face, the right-hand
// sides and the upstream neighbours' increments
template <class T, int U, int NF> struct MicroIn {
  T pos[U][NF], neg[U][NF];
  T xG[U], xR[U], yG[U][NF], yR[U][NF];
};

template <class T, int U, int NF>
__device__ inline void micro_load(const MicroCell<T, NF>& c, const T (*uv)[3], const unsigned* code, const int* k,
                                  int nvi, MicroIn<T, U, NF>& in) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (k[u] >= nvi) continue;
    in.xG[u] = __builtin_nontemporal_load(c.rG + k[u]);
    in.xR[u] = __builtin_nontemporal_load(c.rR + k[u]);
#pragma unroll
    for (int a = 0; a < NF; ++a) {
      const unsigned cd = (code[u] >> (2 * a)) & 3u;
      const T t = uv[u][0] * c.nx[a] + uv[u][1] * c.ny[a] + uv[u][2] * c.nz[a];
      in.pos[u][a] = cd == 1u ? fmax(t, T(0)) : T(0);
      in.neg[u][a] = cd == 2u ? fmin(t, T(0)) : T(0);
      if (c.use[a] && cd == 2u) {
        in.yG[u][a] = c.nG[a][k[u]];
        in.yR[u][a] = c.nR[a][k[u]];
      }
    }
  }
}

template <class T, int U, int NF>
__device__ inline void micro_store(const MicroCell<T, NF>& c, const MicroIn<T, U, NF>& in, const unsigned* code,
                                   const int* k, int nvi) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (k[u] >= nvi) continue;
    double D = c.dbase;
    T aG = in.xG[u], aR = in.xR[u];
#pragma unroll
    for (int a = 0; a < NF; ++a) {
      D += (double)(c.av[a] * in.pos[u][a]);
      if (c.use[a] && ((code[u] >> (2 * a)) & 3u) == 2u) {
        aG -= c.av[a] * in.neg[u][a] * in.yG[u][a];
        aR -= c.av[a] * in.neg[u][a] * in.yR[u][a];
      }
    }
    const double iD = 1.0 / D;
    st_stream(c.oG + k[u], (T)((double)aG * iD));
    st_stream(c.oR + k[u], (T)((double)aR * iD));
  }
}

// Workgroup (cell, velocity chunk): velocities first, then every load of the relaxation, then the stores.
// (Relaxing several cells per workgroup with the next cell's loads issued ahead was measured slower.)
template <class T, int NF>
__global__ __launch_bounds__(kBlock) void k_micro_sweep(Dev d, Bufs b, Work w, int64_t c0, int64_t cnext, int first) {
  constexpr int U = kVptOne;
  const CellChunk cc = cell_chunk(cnext - c0);
  if (cc.cell >= cnext - c0) return;
  const int64_t nv = d.nv;
  const int nvi = (int)nv;
  const int64_t i = c0 + cc.cell;
  int k[U];
  unsigned code[U];
  T uv[U][3];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    k[u] = (int)cc.chunk * (kBlock * U) + u * kBlock + (int)threadIdx.x;
    if (k[u] >= nvi) continue;
    code[u] = reinterpret_cast<const typename Lay<NF>::Code*>(d.upw)[i * nv + k[u]];
    if constexpr (std::is_same<T, float>::value) {
      uv[u][0] = d.dvs_f[k[u]];
      uv[u][1] = d.dvs_f[nv + k[u]];
      uv[u][2] = d.dvs_f[2 * nv + k[u]];
    } else {
      uv[u][0] = d.dvs[k[u]];
      uv[u][1] = d.dvs[nv + k[u]];
      uv[u][2] = d.dvs[2 * nv + k[u]];
    }
  }
  MicroCell<T, NF> c;
  MicroIn<T, U, NF> in;
  micro_setup<T, NF>(d, b, w, i, cnext, first, c);
  micro_load<T, U, NF>(c, uv, code, k, nvi, in);
  micro_store<T, U, NF>(c, in, code, k, nvi);
}

// The vector sweep moves V adjacent velocities per thread as one vector per row (one load or store of
// V sizeof(T) bytes instead of V), when nv is a multiple of V so that every row offset keeps the vectors aligned.
// The arithmetic is that of k_micro_sweep<T>, velocity by velocity; a neighbour's vector is loaded when any of
// the V velocities takes it as its upstream value.  The right-hand sides are read and the increments written
// non-temporally (in every precision): the increments are next read by other colours' launches and the update,
// after the caches have turned over.  Measured on the sphere (4140 velocities): micro sweep 3.79 -> 3.45 ms
// with V = 4 (90 VGPRs, 5 waves per SIMD), 3.52 ms with V = 2; non-temporal 3.44 -> 3.14 ms (FP64 6.89 ->
// 6.58 ms); FP64 with V = 2: 6.35 -> 6.13 ms.
template <class T, int V> struct alignas(sizeof(T) * V) VecF { T v[V]; };
template <class T, int V> struct ExtV { typedef T type __attribute__((ext_vector_type(V))); };
template <class T, int V> __device__ inline VecF<T, V> ld_nt(const T* p) {
  using E = typename ExtV<T, V>::type;
  const E x = __builtin_nontemporal_load(reinterpret_cast<const E*>(p));
  VecF<T, V> r;
#pragma unroll
  for (int q = 0; q < V; ++q) r.v[q] = x[q];
  return r;
}
template <class T, int V> __device__ inline void st_nt(T* p, const VecF<T, V>& v) {
  using E = typename ExtV<T, V>::type;
  E x;
#pragma unroll
  for (int q = 0; q < V; ++q) x[q] = v.v[q];
  __builtin_nontemporal_store(x, reinterpret_cast<E*>(p));
}
// The codes of V adjacent velocities as one word: V bytes (4 face slots) or V 16-bit codes (6 slots)
template <int V, int NF> struct CodeT;
template <> struct CodeT<2, 4> { using type = uint16_t; };
template <> struct CodeT<4, 4> { using type = uint32_t; };
template <> struct CodeT<2, kMaxFaces> { using type = uint32_t; };
template <> struct CodeT<4, kMaxFaces> { using type = uint64_t; };

template <class T, int V, int NF>
__global__ __launch_bounds__(kBlock) void k_micro_sweep_vec(Dev d, Bufs b, Work w, int64_t c0, int64_t cnext,
                                                            int first) {
  using Code = typename Lay<NF>::Code;
  constexpr int bits = 8 * (int)sizeof(Code);
  const CellChunk cc = cell_chunk(cnext - c0);
  if (cc.cell >= cnext - c0) return;
  const int64_t nv = d.nv;
  const int64_t i = c0 + cc.cell;
  const int k = (int)cc.chunk * (V * kBlock) + V * (int)threadIdx.x;
  if (k >= (int)nv) return;
  using VF = VecF<T, V>;
  const uint64_t cw = *reinterpret_cast<const typename CodeT<V, NF>::type*>(reinterpret_cast<const Code*>(d.upw) +
                                                                             i * nv + k);
  const T* dvs = std::is_same<T, float>::value ? (const T*)d.dvs_f : (const T*)d.dvs;
  const VF vx = *reinterpret_cast<const VF*>(dvs + k);
  const VF vy = *reinterpret_cast<const VF*>(dvs + nv + k);
  const VF vz = *reinterpret_cast<const VF*>(dvs + 2 * nv + k);
  MicroCell<T, NF> c;
  micro_setup<T, NF>(d, b, w, i, cnext, first, c);
  const VF xG = ld_nt<T, V>(c.rG + k);
  const VF xR = ld_nt<T, V>(c.rR + k);
  unsigned code[V];
#pragma unroll
  for (int q = 0; q < V; ++q) code[q] = (unsigned)((cw >> (bits * q)) & ((1ull << bits) - 1));
  T pos[V][NF], neg[V][NF];
  VF yG[NF], yR[NF];
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    bool need = false;
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const unsigned cd = (code[q] >> (2 * a)) & 3u;
      const T t = vx.v[q] * c.nx[a] + vy.v[q] * c.ny[a] + vz.v[q] * c.nz[a];
      pos[q][a] = cd == 1u ? vmax(t, T(0)) : T(0);
      neg[q][a] = cd == 2u ? vmin(t, T(0)) : T(0);
      need = need || cd == 2u;
    }
#pragma unroll
    for (int q = 0; q < V; ++q) yG[a].v[q] = yR[a].v[q] = T(0);
    if (c.use[a] && need) {
      yG[a] = *reinterpret_cast<const VF*>(c.nG[a] + k);
      yR[a] = *reinterpret_cast<const VF*>(c.nR[a] + k);
    }
  }
  VF oG, oR;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    double D = c.dbase;
    T aG = xG.v[q], aR = xR.v[q];
#pragma unroll
    for (int a = 0; a < NF; ++a) {
      D += (double)(c.av[a] * pos[q][a]);
      if (c.use[a] && ((code[q] >> (2 * a)) & 3u) == 2u) {
        aG -= c.av[a] * neg[q][a] * yG[a].v[q];
        aR -= c.av[a] * neg[q][a] * yR[a].v[q];
      }
    }
    const double iD = 1.0 / D;
    oG.v[q] = (T)((double)aG * iD);
    oR.v[q] = (T)((double)aR * iD);
  }
  st_nt<T, V>(c.oG + k, oG);
  st_nt<T, V>(c.oR + k, oR);
}

// Preconditioner of the discrete adjoint (FP64): point relaxation over one colour of
// (D + N^T) x = -in for both distributions, where -(D + N) is dR_phi/dphi with first-order upwind faces and
// the collision term frozen: D_i = 1/tau_i + sum_f (A_f/V_i) max(u.n_i, 0) and N_ij = (A_f/V_i) min(u.n_i, 0).
// Transposed, cell i couples to the neighbours it feeds (u.n_i > 0) with (N^T)_ij = -(A_f/V_j) u.n_i.  The W and
// q rows are copied.  With a zero start the first forward pass reads no later colour.
template <int NF>
__global__ __launch_bounds__(kBlock) void k_adj_sweep(Dev d, Bufs b, const double* in, double* x, int64_t c0,
                                                      int64_t cnext, int first) {
  const CellChunk cc = cell_chunk(cnext - c0);
  if (cc.cell >= cnext - c0) return;
  const int64_t i = c0 + cc.cell, nv = d.nv, P = d.nc * nv;
  const int64_t k = cc.chunk * kBlock + threadIdx.x;
  const double* geo = d.cell_geo + Lay<NF>::CG * i;
  const Prim p = prim_of(b.W + 6 * i, d.gas.R);
  const double itau = (p.rho * d.gas.R * p.Ttr) / visc(p.Ttr, d.gas);
  int64_t nrow[NF];
  double cT[NF];
  bool use[NF];
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    const int32_t nb = d.cell_nb[NF * i + a];
    use[a] = nb >= 0 && !(first && nb >= cnext);
    nrow[a] = (nb >= 0 ? nb : i) * nv;
    // A_f / V_j = (A_f / V_i) V_i (1 / V_j)
    cT[a] = nb >= 0 ? geo[CG_FACE + CG_SLOT * a + 1] * geo[0] * d.cell_geo[Lay<NF>::CG * (int64_t)nb + 1] : 0.0;
  }
  if (k >= nv) return;
  const unsigned code = reinterpret_cast<const typename Lay<NF>::Code*>(d.upw)[i * nv + k];
  const double ux = d.dvs[k], uy = d.dvs[nv + k], uz = d.dvs[2 * nv + k];
  double un[NF], yG[NF], yR[NF];
  double D = itau;
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    const double* s = geo + CG_FACE + CG_SLOT * a;
    un[a] = ux * s[2] + uy * s[3] + uz * s[4];
    const bool out = ((code >> (2 * a)) & 3u) == 1u;
    if (out) D += s[1] * un[a];
    yG[a] = yR[a] = 0.0;
    if (use[a] && out) {
      yG[a] = x[nrow[a] + k];
      yR[a] = x[P + nrow[a] + k];
    }
  }
  const double rG = in[i * nv + k], rR = in[P + i * nv + k];
  double aG = -rG, aR = -rR;
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    aG += cT[a] * un[a] * yG[a];
    aR += cT[a] * un[a] * yR[a];
  }
  x[i * nv + k] = aG / D;
  x[P + i * nv + k] = aR / D;
}

__global__ __launch_bounds__(kBlock) void k_copy_tail(const double* in, double* out, int64_t off, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n; t += (int64_t)gridDim.x * kBlock)
    out[off + t] = in[off + t];
}

void launch_adj_sweeps(const Dev& d, const Bufs& b, const double* in, double* out, const int64_t* color_off,
                       int64_t n_colors, int n_pairs, hipStream_t st) {
  const std::vector<int64_t> seq = sweep_sequence(color_off, n_colors, n_pairs);
  int64_t nonempty = 0;
  for (int64_t c = 0; c < n_colors; ++c) nonempty += color_off[c + 1] > color_off[c];
  for (size_t q = 0; q < seq.size(); ++q) {
    const int64_t c = seq[q];
    const int64_t n = color_off[c + 1] - color_off[c];
    if (d.mf == 4)
      hipLaunchKernelGGL(k_adj_sweep<4>, cell_chunk_grid<double>(n, d.nv), dim3(kBlock), 0, st, d, b, in, out,
                         color_off[c], color_off[c + 1], (int64_t)q < nonempty ? 1 : 0);
    else
      hipLaunchKernelGGL(k_adj_sweep<kMaxFaces>, cell_chunk_grid<double>(n, d.nv), dim3(kBlock), 0, st, d, b, in,
                         out, color_off[c], color_off[c + 1], (int64_t)q < nonempty ? 1 : 0);
  }
  const int64_t tail = 12 * d.nc;
  hipLaunchKernelGGL(k_copy_tail, dim3((unsigned)std::min<int64_t>((tail + kBlock - 1) / kBlock, 4096)), dim3(kBlock),
                     0, st, in, out, 2 * d.nc * d.nv, tail);
}

// Upwind codes of every (cell, velocity): the sign of u.n out of the cell through each of its four faces, with
// the tie rule |u.n| <= snap |u| -> 0 (Eq. 46), in FP64.  Computed once per state (and when snap changes).
template <int NF> __global__ __launch_bounds__(kBlock) void k_upwind_codes(Dev d) {
  const int64_t nv = d.nv;
  const int64_t n = d.nc * nv;
  for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < n; x += (int64_t)gridDim.x * kBlock) {
    const int64_t i = x / nv, k = x - i * nv;
    const double ux = d.dvs[k], uy = d.dvs[nv + k], uz = d.dvs[2 * nv + k], um = d.dvs[4 * nv + k];
    const double* geo = d.cell_geo + Lay<NF>::CG * i;
    unsigned code = 0;
    for (int a = 0; a < NF; ++a) {
      const double* s = geo + CG_FACE + CG_SLOT * a;  // an unused slot has a zero normal: code 0
      double un = ux * s[2] + uy * s[3] + uz * s[4];
      un = fabs(un) <= d.snap * um ? 0.0 : un;
      code |= (un > 0.0 ? 1u : (un < 0.0 ? 2u : 0u)) << (2 * a);
    }
    reinterpret_cast<typename Lay<NF>::Code*>(d.upw)[x] = (typename Lay<NF>::Code)code;
  }
}

void launch_upwind_codes(const Dev& d, hipStream_t st) {
  const int64_t n = d.nc * d.nv;
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 65536));
  if (d.mf == 4)
    hipLaunchKernelGGL(k_upwind_codes<4>, dim3(nb), dim3(kBlock), 0, st, d);
  else
    hipLaunchKernelGGL(k_upwind_codes<kMaxFaces>, dim3(nb), dim3(kBlock), 0, st, d);
}

template <class T> __global__ __launch_bounds__(kBlock) void k_zero(T* a, T* b, int64_t n) {
  for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < n; x += (int64_t)gridDim.x * kBlock) {
    a[x] = T(0);
    b[x] = T(0);
  }
}

template <class T, int NF>
void launch_micro_nf(const Dev& d, const Bufs& b, const Work& w, const int64_t* color_off, int64_t n_colors,
                     int n_micro, hipStream_t st) {
  const std::vector<int64_t> seq = sweep_sequence(color_off, n_colors, n_micro);
  if (seq.empty()) {
    // no sweep: the increments of Eq. 33 stay zero
    const int64_t n = d.nc * d.nv;
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 65536));
    hipLaunchKernelGGL(k_zero<T>, dim3(nb), dim3(kBlock), 0, st, (T*)b.dG, (T*)b.dR, n);
    return;
  }
  int64_t nonempty = 0;
  for (int64_t c = 0; c < n_colors; ++c) nonempty += color_off[c + 1] > color_off[c];
  constexpr int V = 16 / sizeof(T);  // 16-byte vectors: four FP32 or two FP64 velocities
  const bool vec = rows_aligned<T>(d, b, V);
  const bool vec2 = std::is_same<T, float>::value && rows_aligned<T>(d, b, 2);
  for (size_t p = 0; p < seq.size(); ++p) {
    const int64_t c = seq[p];
    const int64_t n = color_off[c + 1] - color_off[c];
    if (vec)
      hipLaunchKernelGGL((k_micro_sweep_vec<T, V, NF>), cell_chunk_grid_u<V>(n, d.nv), dim3(kBlock), 0, st, d, b, w,
                         color_off[c], color_off[c + 1], (int64_t)p < nonempty ? 1 : 0);
    else if (vec2)
      hipLaunchKernelGGL((k_micro_sweep_vec<float, 2, NF>), cell_chunk_grid_u<2>(n, d.nv), dim3(kBlock), 0, st, d,
                         b, w, color_off[c], color_off[c + 1], (int64_t)p < nonempty ? 1 : 0);
    else
      hipLaunchKernelGGL((k_micro_sweep<T, NF>), cell_chunk_grid_u<kVptOne>(n, d.nv), dim3(kBlock), 0, st, d, b, w,
                         color_off[c], color_off[c + 1], (int64_t)p < nonempty ? 1 : 0);
  }
}

template <class T>
void launch_micro(const Dev& d, const Bufs& b, const Work& w, const int64_t* color_off, int64_t n_colors, int n_micro,
                  hipStream_t st) {
  if (d.mf == 4)
    launch_micro_nf<T, 4>(d, b, w, color_off, n_colors, n_micro, st);
  else
    launch_micro_nf<T, kMaxFaces>(d, b, w, color_off, n_colors, n_micro, st);
}

// ---------------------------------------------------------------------------
// Step 6: phi^{n+1} = phi^n + dphi and the integral error compensation (Eqs. 62-67), c = u - U~;
// Step 7: per-cell |W^{n+1} - W^n|, reduced by k_reduce_res.  One workgroup per cell.
// ---------------------------------------------------------------------------

// The 12 moment sums of Eqs. 62-67 of one velocity: phi^{n+1} - phi~* weighted by Phi (conserved moments) and
// by c |c|^2 / 2, c (heat fluxes), c = u - U~.  Sums 4 and 6-8 leave out the factor 1/2 (and sum 4 the R part,
// which is sum 5): update_cell applies them to the totals.
template <class T, class A>
__device__ inline void update_moments(A& acc, T g, T r, T gs, T rs, double vx, double vy, double vz, double vw,
                                      double Ux, double Uy, double Uz) {
  double gd = (double)g - (double)gs, rd = (double)r - (double)rs;
  double cx = vx - Ux, cy = vy - Uy, cz = vz - Uz;
  double c2 = cx * cx + cy * cy + cz * cz;
  double wg = vw * gd, wr = vw * rd;
  acc.add(0, wg);
  acc.add(1, vx * wg);
  acc.add(2, vy * wg);
  acc.add(3, vz * wg);
  acc.add(4, (vx * vx + vy * vy + vz * vz) * wg);
  acc.add(5, wr);
  double hc = c2 * wg;
  acc.add(6, cx * hc);
  acc.add(7, cy * hc);
  acc.add(8, cz * hc);
  acc.add(9, cx * wr);
  acc.add(10, cy * wr);
  acc.add(11, cz * wr);
}

// W^{n+1} and q^{n+1} of cell i from its 12 sums (Eqs. 62-67), and |W^{n+1} - W^n| for the residual.
__device__ inline void update_cell(const Dev& d, const Bufs& b, const Work& w, int64_t i, const double* s) {
  const GasC& gg = d.gas;
  const double* ec = w.eq + ER * i;
  const double* Wt = w.Wt + 6 * i;
  double* W = b.W + 6 * i;
  double* q = b.q + 6 * i;
  double Wn[6], qn[6];
  Wn[0] = s[0] + Wt[0];                                                      // Eq. 62
  Wn[1] = s[1] + Wt[1];                                                      // Eq. 63
  Wn[2] = s[2] + Wt[2];
  Wn[3] = s[3] + Wt[3];
  Wn[4] = (0.5 * s[4] + s[5]) + Wt[4];                                      // Eq. 64
  Wn[5] = s[5] + ec[0] * gg.R * ((1.0 - 1.0 / gg.Z) * ec[6] + ec[4] / gg.Z);  // Eq. 65
  const double ctr = (1.0 / 3.0) * (1.0 - (1.0 - gg.omega0) / gg.Z);
  const double crot = (1.0 - gg.delta) * (1.0 - (1.0 - gg.omega1) / gg.Z);
  for (int m = 0; m < 3; ++m) {
    qn[m] = 0.5 * s[6 + m] + q[m] * ctr;    // Eq. 66
    qn[3 + m] = s[9 + m] + q[3 + m] * crot;  // Eq. 67
  }
  for (int m = 0; m < 6; ++m) {
    w.cellres[6 * i + m] = fabs(Wn[m] - W[m]);
    W[m] = Wn[m];
    q[m] = qn[m];
  }
}

template <class T, bool Comp> __global__ __launch_bounds__(kBlock) void k_update(Dev d, Bufs b, Work w) {
  __shared__ double red[(kBlock / 64) * 2 * 12];
  const int64_t i = blockIdx.x;
  const int64_t nv = d.nv;
  const double* ec = w.eq + ER * i;
  Eq<T> e;
  e.load(ec);
  const double Ux = ec[1], Uy = ec[2], Uz = ec[3];
  T* G = (T*)b.G + i * nv;
  T* R = (T*)b.R + i * nv;
  const T* dG = (const T*)b.dG + i * nv;
  const T* dR = (const T*)b.dR + i * nv;
  const DvsRows V = dvs_rows(d);
  Acc<12, Comp, kBlock> acc;
  acc.zero();
  k_loop(nv, [&](int k) {
    const T g = G[k] + dG[k];
    const T r = R[k] + dR[k];
    st_stream(G + k, g);
    st_stream(R + k, r);
    const double vx = V.ux[k], vy = V.uy[k], vz = V.uz[k], vw = V.w[k];
    T gs, rs;
    e.eval((T)vx, (T)vy, (T)vz, gs, rs);
    update_moments(acc, g, r, gs, rs, vx, vy, vz, vw, Ux, Uy, Uz);
  });
  __shared__ double s[12];
  acc.reduce_to_lds(s, red);
  if (threadIdx.x == 0) update_cell(d, b, w, i, s);
}

constexpr int kResParts = kResidualParts;

// Step 7, stage 1: partial sums of |W^{n+1} - W^n| over a fixed cell partition (deterministic), positivity check
__global__ __launch_bounds__(kBlock) void k_reduce_res_part(int64_t nc, const double* cellres, double* part,
                                                            int32_t* flag, const double* W) {
  __shared__ double red[(kBlock / 64) * 2 * 6];
  Acc<6, false, kBlock> acc;
  acc.zero();
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nc; i += (int64_t)kResParts * kBlock) {
    for (int m = 0; m < 6; ++m) acc.add(m, cellres[6 * i + m]);
    const double* Wi = W + 6 * i;
    double ke = 0.5 * (Wi[1] * Wi[1] + Wi[2] * Wi[2] + Wi[3] * Wi[3]) / Wi[0];
    if (!(Wi[0] > 0.0) || !(Wi[4] - ke > 0.0) || !(Wi[5] > 0.0)) bad = 1;
  }
  double tot[6];
  acc.reduce(tot, red);
  if (bad) atomicOr(&flag[0], 2);
  if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = tot[threadIdx.x];
}

// stage 2: one workgroup adds the kResParts partials in a fixed order
__global__ __launch_bounds__(kBlock) void k_reduce_res(int64_t nc, const double* part, double* res, int32_t* flag) {
  __shared__ double red[(kBlock / 64) * 2 * 6];
  Acc<6, false, kBlock> acc;
  acc.zero();
  for (int p = threadIdx.x; p < kResParts; p += kBlock)
    for (int m = 0; m < 6; ++m) acc.add(m, part[6 * p + m]);
  double tot[6];
  acc.reduce(tot, red);
  if (threadIdx.x < 6) {
    double v = tot[threadIdx.x] / (double)nc;
    res[threadIdx.x] = v;
    if (!isfinite(v)) atomicOr(&flag[0], 4);
  }
}

template <class T> void launch_update(const Dev& d, const Bufs& b, const Work& w, int64_t it, hipStream_t st) {
  constexpr bool Comp = sizeof(T) == 4;
  hipLaunchKernelGGL((k_update<T, Comp>), dim3((unsigned)d.nc), dim3(kBlock), 0, st, d, b, w);
  hipLaunchKernelGGL(k_reduce_res_part, dim3(kResParts), dim3(kBlock), 0, st, d.nc, (const double*)w.cellres,
                     w.respart, w.flag, (const double*)b.W);
  hipLaunchKernelGGL(k_reduce_res, dim3(1), dim3(kBlock), 0, st, d.nc, (const double*)w.respart, w.res + 6 * it,
                     w.flag);
}

int max_velocities() { return 16384; }

// explicit instantiations
template void launch_init_eq<double>(const Dev&, const Bufs&, const double*, int, double*, hipStream_t);
template void launch_init_eq<float>(const Dev&, const Bufs&, const double*, int, double*, hipStream_t);
template void launch_recon<double>(const Dev&, const Bufs&, hipStream_t, void*);
template void launch_recon<float>(const Dev&, const Bufs&, hipStream_t, void*);
template void launch_face<double>(const Dev&, const Bufs&, const Work&, hipStream_t);
template void launch_face<float>(const Dev&, const Bufs&, const Work&, hipStream_t);
template void launch_residual<double>(const Dev&, const Bufs&, const Work&, void*, void*, int, hipStream_t);
template void launch_residual<float>(const Dev&, const Bufs&, const Work&, void*, void*, int, hipStream_t);
template void launch_micro<double>(const Dev&, const Bufs&, const Work&, const int64_t*, int64_t, int, hipStream_t);
template void launch_micro<float>(const Dev&, const Bufs&, const Work&, const int64_t*, int64_t, int, hipStream_t);
template void launch_update<double>(const Dev&, const Bufs&, const Work&, int64_t, hipStream_t);
template void launch_update<float>(const Dev&, const Bufs&, const Work&, int64_t, hipStream_t);

}  // namespace cis
