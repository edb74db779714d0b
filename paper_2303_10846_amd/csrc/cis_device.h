// Device helpers shared by the kernels of one iteration and the adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "cis_internal.h"

namespace cis {

constexpr int kBlock = 256;  // threads per workgroup
constexpr int kXcd = 8;      // accelerator complex dies, each with its own L2

// Logical index of workgroup w among n.  The dispatcher deals workgroups to the XCDs round-robin
// (w -> XCD w % 8); this bijection on [0, n) gives every XCD one contiguous range of logical blocks, so
// that workgroups of neighbouring cells share that XCD's L2.
__device__ inline int64_t xcd_block(int64_t w, int64_t n) {
  const int64_t q = n / kXcd, r = n % kXcd;
  const int64_t x = w % kXcd, j = w / kXcd;
  return x * q + (x < r ? x : r) + j;
}

// Element k of a row whose base pointer is uniform over the workgroup, with the byte offset formed in 32 bits
// (the scalar-base addressing form where the compiler can match it).  Callers keep k * sizeof(T) below 2^32
// (the velocity count is bounded).
template <class T> __device__ inline T ld_row(const T* row, uint32_t k) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(row) + (uint64_t)(k * (uint32_t)sizeof(T)));
}
template <class T> __device__ inline T* at_row(T* row, uint32_t k) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(row) + (uint64_t)(k * (uint32_t)sizeof(T)));
}
// An empty asm statement (no instruction) that uses x in a VGPR: placed after a group of stores it keeps their
// data and address registers live until the last store has issued.  A register that a pending store still
// reads is otherwise reused for the next store, and the compiler then waits for every outstanding memory
// operation before each store (vmcnt(0)).
template <class T> __device__ inline void keep_live(const T& x) { asm volatile("" : : "v"(x)); }

__device__ inline float vmin(float a, float b) { return fminf(a, b); }
__device__ inline double vmin(double a, double b) { return fmin(a, b); }
__device__ inline float vmax(float a, float b) { return fmaxf(a, b); }
__device__ inline double vmax(double a, double b) { return fmax(a, b); }

// ---------------------------------------------------------------------------
// Reductions over a workgroup of NT threads (NT/64 wave64 wavefronts)
// ---------------------------------------------------------------------------

// s + x with its exact rounding error added to c (Knuth's branch-free TwoSum)
__device__ inline void two_sum_add(double& s, double& c, double x) {
  const double t = s + x;
  const double z = t - s;
  c += (s - (t - z)) + (x - z);
  s = t;
}

// One 64-bit value moved across lanes by a DPP control (two 32-bit data-parallel-primitive moves, all rows
// enabled; a lane without a source receives 0).
template <int Ctrl> __device__ inline double dpp_move(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, Ctrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), Ctrl, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// The wavefront sums of N values per lane, written to dst[0..N) (LDS) by one lane each.  Recursive halving:
// the gfx950 lane swaps exchange half of two registers at a time (permlane32_swap: lanes 32-63 of the first
// with lanes 0-31 of the second; permlane16_swap: the odd 16-lane rows of the first with the even rows of the
// second), so one swap and one add fold two values over 32 lanes, then pairs of those over 16 lanes; DPP
// rotations and quad permutations finish each 16-lane row.  For N = 17 that is 102 VALU instructions per
// wavefront instead of 306 with a DPP tree per value.  A fixed pairwise order (deterministic).
typedef unsigned int cis_u32x2 __attribute__((ext_vector_type(2)));
template <bool Half32> __device__ inline void lane_swap(double& x, double& y) {
  const uint64_t ux = __builtin_bit_cast(uint64_t, x), uy = __builtin_bit_cast(uint64_t, y);
  cis_u32x2 lo, hi;
  if (Half32) {
    lo = __builtin_amdgcn_permlane32_swap((uint32_t)ux, (uint32_t)uy, false, false);
    hi = __builtin_amdgcn_permlane32_swap((uint32_t)(ux >> 32), (uint32_t)(uy >> 32), false, false);
  } else {
    lo = __builtin_amdgcn_permlane16_swap((uint32_t)ux, (uint32_t)uy, false, false);
    hi = __builtin_amdgcn_permlane16_swap((uint32_t)(ux >> 32), (uint32_t)(uy >> 32), false, false);
  }
  x = __builtin_bit_cast(double, (uint64_t)lo[0] | ((uint64_t)hi[0] << 32));
  y = __builtin_bit_cast(double, (uint64_t)lo[1] | ((uint64_t)hi[1] << 32));
}
template <int N> __device__ inline void wave_sums(const double* v, double* dst) {
  constexpr int M1 = (N + 1) / 2, M2 = (M1 + 1) / 2;
  // p[j]: lanes 0-31 hold value 2j, lanes 32-63 value 2j+1 (each summed over lanes l and l+32); an odd last
  // value is paired with itself (its copy has index N and is not written)
  double p[M1];
#pragma unroll
  for (int j = 0; j < M1; ++j) {
    double x = v[2 * j], y = 2 * j + 1 < N ? v[2 * j + 1] : v[2 * j];
    lane_swap<true>(x, y);
    p[j] = x + y;
  }
  // q[i]: rows 0, 1, 2, 3 hold values 4i, 4i+2, 4i+1, 4i+3 (each summed over four lanes)
  double q[M2];
#pragma unroll
  for (int i = 0; i < M2; ++i) {
    double x = p[2 * i], y = 2 * i + 1 < M1 ? p[2 * i + 1] : p[2 * i];
    lane_swap<false>(x, y);
    q[i] = x + y;
  }
  const int lane = threadIdx.x & 63, r = lane >> 4;
  const int slot = r == 1 ? 2 : r == 2 ? 1 : r;
#pragma unroll
  for (int i = 0; i < M2; ++i) {
    double x = q[i];
    x += dpp_move<0x128>(x);  // row_ror:8
    x += dpp_move<0x124>(x);  // row_ror:4
    x += dpp_move<0x4E>(x);   // quad_perm [2, 3, 0, 1]
    x += dpp_move<0xB1>(x);   // quad_perm [1, 0, 3, 2]
    const int m = 4 * i + slot;
    if ((lane & 15) == 0 && m < N) dst[m] = x;
  }
}

// N running FP64 sums per thread.  With Comp, every thread's running sum is compensated: the exact rounding
// error of each addition (TwoSum) is accumulated beside it, over the long sequential part of the summation;
// the 64 lanes of a wavefront are combined by a pairwise tree (wave_sums; error O(log2(64) eps)) and the
// wavefronts' results again with compensation.  Without Comp the
// running sums and the merge are plain FP64.
template <int N, bool Comp, int NT> struct Acc {
  static constexpr int NW = NT / 64;
  double s[N], c[Comp ? N : 1];
  __device__ inline void zero() {
#pragma unroll
    for (int m = 0; m < N; ++m) {
      s[m] = 0.0;
      if (Comp) c[m] = 0.0;
    }
  }
  __device__ inline void add(int m, double x) {
    if (Comp) {
      two_sum_add(s[m], c[m], x);
    } else {
      s[m] += x;
    }
  }
  // Block-wide totals, identical in every thread.  red: NW * N doubles of LDS.
  __device__ inline void reduce(double* out, double* red) {
    const int wid = threadIdx.x >> 6;
    double v[N];
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = Comp ? s[m] + c[m] : s[m];
    wave_sums<N>(v, red + wid * N);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < N; ++m) {
      double a = red[m], b = 0.0;
      for (int q = 1; q < NW; ++q) {
        if (Comp) {
          two_sum_add(a, b, red[q * N + m]);
        } else {
          a += red[q * N + m];
        }
      }
      out[m] = Comp ? a + b : a;
    }
    __syncthreads();
  }
  // The same totals written to LDS by thread 0 only (sh_out: N doubles), for a block that hands them to one
  // thread: the totals are then not live in every thread's registers.
  __device__ inline void reduce_to_lds(double* sh_out, double* red) {
    const int wid = threadIdx.x >> 6;
    double v[N];
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = Comp ? s[m] + c[m] : s[m];
    wave_sums<N>(v, red + wid * N);
    __syncthreads();
    if (threadIdx.x < N) {
      const int m = threadIdx.x;
      double a = red[m], b = 0.0;
      for (int q = 1; q < NW; ++q) {
        if (Comp) {
          two_sum_add(a, b, red[q * N + m]);
        } else {
          a += red[q * N + m];
        }
      }
      sh_out[m] = Comp ? a + b : a;
    }
    __syncthreads();
  }
};

// ---------------------------------------------------------------------------
// Gas model (Sec. 2)
// ---------------------------------------------------------------------------

struct Prim {
  double rho, U[3], T, Ttr, Trot;
};

// Eqs. 1-5 with K_tr = 3, K_rot = 2
__device__ inline Prim prim_of(const double* W, double R) {
  Prim p;
  p.rho = W[0];
  double ir = 1.0 / W[0];
  p.U[0] = W[1] * ir;
  p.U[1] = W[2] * ir;
  p.U[2] = W[3] * ir;
  double ke = 0.5 * W[0] * (p.U[0] * p.U[0] + p.U[1] * p.U[1] + p.U[2] * p.U[2]);
  double irR = ir / R;
  p.T = 0.4 * (W[4] - ke) * irR;
  p.Trot = W[5] * irR;
  p.Ttr = (2.0 / 3.0) * (W[4] - ke - W[5]) * irR;
  return p;
}

// Viscosity.  Eq. 13 (VHS), mu_ref (T_tr/T_ref)^omega as exp(omega log(T_tr/T_ref)): a few ulp, and far fewer
// registers than the double-double pow of the math library (the face pass computes it once per face inside a
// wide kernel).  Eq. 14 (Sutherland, C_s > 0): mu_ref x^(3/2) (T_ref + C_s)/(T_tr + C_s), x = T_tr/T_ref.
__device__ inline double visc(double Ttr, const GasC& g) {
  const double x = Ttr / g.T_ref;
  if (g.C_s > 0.0) return g.mu_ref * x * sqrt(x) * (g.T_ref + g.C_s) / (Ttr + g.C_s);
  return g.mu_ref * exp(g.omega_v * log(x));
}
// d ln(mu) / d ln(T_tr): omega (VHS), 3/2 - T_tr/(T_tr + C_s) (Sutherland)
__device__ inline double visc_exponent(double Ttr, const GasC& g) {
  return g.C_s > 0.0 ? 1.5 - Ttr / (Ttr + g.C_s) : g.omega_v;
}

// (2 pi R T)^-3/2
__device__ inline double maxwell_norm(double RT) {
  const double x = 6.283185307179586476925 * RT;
  return 1.0 / (x * sqrt(x));
}

// Coefficients of the reduced Rykov equilibria (Eqs. 17-23) for one macroscopic state.
__device__ inline void eq_coeffs(const Prim& p, const double* q, const GasC& g, double* e) {
  const double R = g.R;
  double RTtr = R * p.Ttr, RT = R * p.T, RTrot = R * p.Trot;
  double ptr = p.rho * RTtr, pp = p.rho * RT, prot = p.rho * RTrot;
  e[0] = p.rho;
  e[1] = p.U[0];
  e[2] = p.U[1];
  e[3] = p.U[2];
  e[4] = p.T;
  e[5] = p.Ttr;
  e[6] = p.Trot;
  for (int d = 0; d < 6; ++d) e[8 + d] = q[d];
  e[14] = p.rho * maxwell_norm(RTtr);
  e[15] = 1.0 / (2.0 * RTtr);
  e[16] = p.rho * maxwell_norm(RT);
  e[17] = 1.0 / (2.0 * RT);
  e[18] = 1.0 / (15.0 * RTtr * ptr);               // Eq. 19
  e[19] = g.omega0 / (15.0 * RT * pp);             // Eq. 20
  e[20] = (1.0 - g.delta) / (RTtr * prot);         // Eq. 21
  e[21] = g.omega1 * (1.0 - g.delta) / (RT * pp);  // Eq. 22
  e[22] = 1.0 / RTtr;
  e[23] = 1.0 / RT;
  e[24] = RTrot;
  e[25] = RT;
  e[26] = 1.0 - 1.0 / g.Z;  // Eqs. 17-18
  e[27] = 1.0 / g.Z;
}

// exp of the equilibrium evaluation.  FP64: the library exp.  FP32: the hardware base-2 exponential of
// t = fl(x log2 e), corrected by the rounding error of that product: with log2 e = L_hi + L_lo (L_hi the FP32
// value nearest log2 e), e = (x L_hi - t) + x L_lo is formed exactly enough by two FMAs (the FMA-based exact
// product error of Dekker's method), and exp(x) = 2^t 2^e ~ 2^t (1 + e ln 2), |e| < 2^-24 |t|.  Without the
// correction the error grows with |x| (3.8e-6 relative at x = -87, which moved the converged mixed wall heat
// flux by 1.3e-5); with it the error is that of the hardware 2^t plus one rounding (about 1.2e-7 relative
// with a correctly rounded 2^t).  Six instructions instead of the library expf's ten; results below the FP32
// normal range may flush to zero (values under 1.2e-38, against O(1) sums).
__device__ inline double eq_exp(double x) { return exp(x); }
__device__ inline float eq_exp(float x) {
  constexpr float kL2eHi = 1.44269502162933349609375f;  // FP32 nearest log2(e)
  constexpr float kL2eLo = 1.925963e-8f;                 // log2(e) - kL2eHi
  constexpr float kLn2 = 0.693147180559945309f;
  const float t = x * kL2eHi;
  const float e = __builtin_fmaf(x, kL2eLo, __builtin_fmaf(x, kL2eHi, -t));
  const float r = __builtin_amdgcn_exp2f(t);
  return __builtin_fmaf(r, e * kLn2, r);
}

// exp(c2 b) for the equilibrium's exponentials, b = -1/(2RT) fixed per cell or face.  FP64: exp(c2 b).  FP32:
// b log2 e is split once, in FP64, into B_hi + B_lo (B_hi its nearest FP32 value); t = fl(c2 B_hi), and the
// rounding error of the whole exponent, e = (c2 B_hi - t) + c2 B_lo, follows from two FMAs as in eq_exp, so
// exp(c2 b) = 2^t (1 + e ln 2).  Folding b into the base-2 constant removes one product and its rounding (the
// error is then that of c2, of the hardware 2^t and of one rounding).
template <class C> struct EqExp;
template <> struct EqExp<double> {
  double b;
  __device__ inline void load(double bnat) { b = bnat; }
  __device__ inline double operator()(double c2) const { return exp(c2 * b); }
};
template <> struct EqExp<float> {
  float hi, lo;
  __device__ inline void load(double bnat) {
    const double b2 = bnat * 1.4426950408889634;
    hi = (float)b2;
    lo = (float)(b2 - (double)hi);
  }
  __device__ inline float operator()(float c2) const {
    constexpr float kLn2 = 0.693147180559945309f;
    const float t = c2 * hi;
    const float e = __builtin_fmaf(c2, lo, __builtin_fmaf(c2, hi, -t));
    const float r = __builtin_amdgcn_exp2f(t);
    return __builtin_fmaf(r, e * kLn2, r);
  }
};

// G*, R* of Eqs. 17-23 times a constant factor c (c = 1, or c = s/(tau+s) in the face step of Eq. 45), with
// the constants combined once per cell or face: c (1-1/Z) a_tr and c a_T/Z as the two exponentials'
// amplitudes, the Shakhov-type factors in the form c^2 k1 - k2 of the peculiar speed, and the R* parts as
// RT_rot G_tr + RT G_rot + (c.q_rot)(m3 g_tr + m4 g_T).  Two exponentials per velocity.
template <class C> struct Eq {
  C Ux, Uy, Uz, qtx, qty, qtz, qrx, qry, qrz, A1, A2, k1, k2, k3, k4, m1, m2, m3, m4;
  EqExp<C> x1, x2;
  __device__ inline void load(const double* e, double c = 1.0) {
    Ux = (C)e[1];
    Uy = (C)e[2];
    Uz = (C)e[3];
    qtx = (C)e[8];
    qty = (C)e[9];
    qtz = (C)e[10];
    qrx = (C)e[11];
    qry = (C)e[12];
    qrz = (C)e[13];
    A1 = (C)(c * e[26] * e[14]);
    x1.load(-e[15]);
    A2 = (C)(c * e[27] * e[16]);
    x2.load(-e[17]);
    k1 = (C)(e[18] * e[22]);
    k2 = (C)(5.0 * e[18]);
    k3 = (C)(e[19] * e[23]);
    k4 = (C)(5.0 * e[19]);
    m1 = (C)e[24];
    m2 = (C)e[25];
    m3 = (C)(e[24] * e[20]);
    m4 = (C)(e[25] * e[21]);
  }
  __device__ inline void eval(C ux, C uy, C uz, C& Gs, C& Rs) const {
    const C cx = ux - Ux, cy = uy - Uy, cz = uz - Uz;
    const C c2 = cx * cx + cy * cy + cz * cz;
    const C cqt = cx * qtx + cy * qty + cz * qtz;
    const C cqr = cx * qrx + cy * qry + cz * qrz;
    const C g1 = A1 * x1(c2);
    const C g2 = A2 * x2(c2);
    const C Gt = g1 + g1 * (cqt * (c2 * k1 - k2));
    const C Gr = g2 + g2 * (cqt * (c2 * k3 - k4));
    Gs = Gt + Gr;
    Rs = m1 * Gt + (m2 * Gr + cqr * (m3 * g1 + m4 * g2));
  }
};

// One discrete velocity (structure-of-arrays DVS, see DVS_* in cis_internal.h)
struct Vel {
  double ux, uy, uz, w, um, h2;
};
__device__ inline Vel vel(const Dev& d, int64_t k) {
  const double* v = d.dvs;
  const int64_t n = d.nv;
  return Vel{v[k], v[n + k], v[2 * n + k], v[3 * n + k], v[4 * n + k], v[5 * n + k]};
}
template <class T> __device__ inline void vel_t(const Dev& d, int64_t k, T& ux, T& uy, T& uz);
template <> __device__ inline void vel_t<double>(const Dev& d, int64_t k, double& ux, double& uy, double& uz) {
  ux = d.dvs[k];
  uy = d.dvs[d.nv + k];
  uz = d.dvs[2 * d.nv + k];
}
template <> __device__ inline void vel_t<float>(const Dev& d, int64_t k, float& ux, float& uy, float& uz) {
  ux = d.dvs_f[k];
  uy = d.dvs_f[d.nv + k];
  uz = d.dvs_f[2 * d.nv + k];
}

// u.n with the tie rule (|u.n| <= snap |u| -> 0)
__device__ inline double udotn(const Vel& v, double nx, double ny, double nz, double snap) {
  double un = v.ux * nx + v.uy * ny + v.uz * nz;
  return fabs(un) <= snap * v.um ? 0.0 : un;
}

__device__ inline double inv_dt_cell(const Dev& d, double h) {
  double v = d.inv_dt;
  if (d.cfl_imp > 0.0) v += d.umax / (d.cfl_imp * h);
  return v;
}

// Euler flux with the rotational-energy row (Eq. 40), p = rho R T
__device__ inline void euler_flux(const double* W, double nx, double ny, double nz, double* out) {
  double ir = 1.0 / W[0];
  double Ux = W[1] * ir, Uy = W[2] * ir, Uz = W[3] * ir;
  double p = 0.4 * (W[4] - 0.5 * W[0] * (Ux * Ux + Uy * Uy + Uz * Uz));
  double Un = Ux * nx + Uy * ny + Uz * nz;
  out[0] = W[0] * Un;
  out[1] = W[1] * Un + p * nx;
  out[2] = W[2] * Un + p * ny;
  out[3] = W[3] * Un + p * nz;
  out[4] = (W[4] + p) * Un;
  out[5] = W[5] * Un;
}

}  // namespace cis
