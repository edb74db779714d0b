// Derivatives used by the adjoint (VJP) of the steady residual: host+device functions, FP64.
//
// theta = (rho, U_x, U_y, U_z, T, T_tr, T_rot, q_tr x3, q_rot x3) parametrises the reduced Rykov
// equilibria G*, R* of Eqs. 17-23.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "cis_internal.h"

namespace cis {

constexpr int NTH = 13;

// G*, R* of one macroscopic state theta and their partial derivatives with respect to theta (Eqs. 17-23).
// setup() once per state, eval() per velocity.
struct EqAd {
  double R, rho, U[3], T, Ttr, Trot, qt[3], qr[3];
  double A, B, ntr, nT, iA2, iB2, k1, k2, ctr, crt, z1, z2;
  __host__ __device__ inline void setup(const double* th, const GasC& g) {
    const double twopi = 6.283185307179586476925;
    R = g.R;
    rho = th[0];
    for (int e = 0; e < 3; ++e) {
      U[e] = th[1 + e];
      qt[e] = th[7 + e];
      qr[e] = th[10 + e];
    }
    T = th[4];
    Ttr = th[5];
    Trot = th[6];
    // translational part: g_tr = n_tr exp(-c2/(2A)), A = R T_tr, k1 = 1/(15 R T_tr p_tr) = 1/(15 rho A^2)
    A = R * Ttr;
    ntr = rho * pow(twopi * A, -1.5);
    iA2 = 0.5 / A;
    k1 = 1.0 / (15.0 * rho * A * A);
    // rotational-relaxation part: g_T with B = R T, k2 = omega0/(15 rho B^2)
    B = R * T;
    nT = rho * pow(twopi * B, -1.5);
    iB2 = 0.5 / B;
    k2 = g.omega0 / (15.0 * rho * B * B);
    // R^tr = R T_rot G^tr + ctr (c.q_rot) g_tr,  R^rot = R T G^rot + crt (c.q_rot) g_T
    ctr = (1.0 - g.delta) / (rho * A);
    crt = g.omega1 * (1.0 - g.delta) / (rho * B);
    z2 = 1.0 / g.Z;
    z1 = 1.0 - z2;
  }
  // Values at u; when dG is not null, also dG/dtheta, dR/dtheta (13 each).
  __host__ __device__ inline void eval(double ux, double uy, double uz, double& Gs, double& Rs, double* dG,
                                       double* dR) const {
    const double c[3] = {ux - U[0], uy - U[1], uz - U[2]};
    const double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    const double cq = c[0] * qt[0] + c[1] * qt[1] + c[2] * qt[2];
    const double cr = c[0] * qr[0] + c[1] * qr[1] + c[2] * qr[2];
    const double gtr = ntr * exp(-c2 * iA2), gT = nT * exp(-c2 * iB2);
    const double mA = c2 / A - 5.0, mB = c2 / B - 5.0;
    const double Ptr = 1.0 + cq * k1 * mA, Prot = 1.0 + cq * k2 * mB;
    const double Gtr = gtr * Ptr, Grot = gT * Prot;
    const double Rtr = R * Trot * Gtr + ctr * cr * gtr;
    const double Rrot = R * T * Grot + crt * cr * gT;
    Gs = z1 * Gtr + z2 * Grot;
    Rs = z1 * Rtr + z2 * Rrot;
    if (!dG) return;
    // rho: g is proportional to rho, k1 and k2 to 1/rho; the c.q_rot terms do not depend on rho
    {
      const double dGtr = (Gtr - gtr * cq * k1 * mA) / rho;
      const double dGrot = (Grot - gT * cq * k2 * mB) / rho;
      dG[0] = z1 * dGtr + z2 * dGrot;
      dR[0] = z1 * R * Trot * dGtr + z2 * R * T * dGrot;
    }
    // U_e: dc/dU_e = -e_e
    for (int e = 0; e < 3; ++e) {
      const double dgtr = gtr * c[e] / A, dgT = gT * c[e] / B;
      const double dPtr = k1 * (-qt[e] * mA - 2.0 * cq * c[e] / A);
      const double dProt = k2 * (-qt[e] * mB - 2.0 * cq * c[e] / B);
      const double dGtr = dgtr * Ptr + gtr * dPtr;
      const double dGrot = dgT * Prot + gT * dProt;
      dG[1 + e] = z1 * dGtr + z2 * dGrot;
      dR[1 + e] = z1 * (R * Trot * dGtr + ctr * (cr * dgtr - qr[e] * gtr)) +
                  z2 * (R * T * dGrot + crt * (cr * dgT - qr[e] * gT));
    }
    // T (enters G^rot, R^rot; crt is proportional to 1/T)
    {
      const double dgT = gT * (c2 * iB2 - 1.5) / T;
      const double dProt = cq * k2 * (10.0 - 3.0 * c2 / B) / T;
      const double dGrot = dgT * Prot + gT * dProt;
      dG[4] = z2 * dGrot;
      dR[4] = z2 * (R * Grot + R * T * dGrot + crt * cr * (dgT - gT / T));
    }
    // T_tr (enters G^tr, R^tr; ctr is proportional to 1/T_tr)
    {
      const double dgtr = gtr * (c2 * iA2 - 1.5) / Ttr;
      const double dPtr = cq * k1 * (10.0 - 3.0 * c2 / A) / Ttr;
      const double dGtr = dgtr * Ptr + gtr * dPtr;
      dG[5] = z1 * dGtr;
      dR[5] = z1 * (R * Trot * dGtr + ctr * cr * (dgtr - gtr / Ttr));
    }
    // T_rot
    dG[6] = 0.0;
    dR[6] = z1 * R * Gtr;
    // q_tr, q_rot
    for (int e = 0; e < 3; ++e) {
      const double dGtr = gtr * c[e] * k1 * mA, dGrot = gT * c[e] * k2 * mB;
      dG[7 + e] = z1 * dGtr + z2 * dGrot;
      dR[7 + e] = z1 * R * Trot * dGtr + z2 * R * T * dGrot;
      dG[10 + e] = 0.0;
      dR[10 + e] = z1 * ctr * c[e] * gtr + z2 * crt * c[e] * gT;
    }
  }
};

// g = J^T v with J = dG_n/dW the Jacobian of the Euler flux along n of the macroscopic system (Eq. 37 with the
// equilibrium closure p = (gamma - 1)(rho E - rho |U|^2 / 2), gamma = 7/5, and rho E_rot carried with U.n), at the
// state W = (rho, rho U, rho E, rho E_rot).  Written out from G_n = (rho U.n, rho U U.n + p n, (rho E + p) U.n,
// rho E_rot U.n): with s = v.G_n, K = (v_m.(rho U) + v_4 (rho E + p) + v_5 rho E_rot)/rho and P = v_m.n + v_4 U.n,
//   ds/drho = -U.n K + (|U|^2/5) P,  ds/d(rho U) = v_0 n + v_m U.n + K n - (2/5) U P,
//   ds/d(rho E) = (2/5) P + v_4 U.n,  ds/d(rho E_rot) = v_5 U.n.
__host__ __device__ inline void euler_flux_vjp(const double* W, double nx, double ny, double nz, const double* v,
                                               double* g) {
  const double ir = 1.0 / W[0];
  const double Ux = W[1] * ir, Uy = W[2] * ir, Uz = W[3] * ir;
  const double U2 = Ux * Ux + Uy * Uy + Uz * Uz;
  const double p = 0.4 * (W[4] - 0.5 * W[0] * U2);
  const double Un = Ux * nx + Uy * ny + Uz * nz;
  const double K = (v[1] * W[1] + v[2] * W[2] + v[3] * W[3] + v[4] * (W[4] + p) + v[5] * W[5]) * ir;
  const double P = v[1] * nx + v[2] * ny + v[3] * nz + v[4] * Un;
  g[0] = -Un * K + 0.2 * U2 * P;
  g[1] = v[0] * nx + v[1] * Un + K * nx - 0.4 * Ux * P;
  g[2] = v[0] * ny + v[2] * Un + K * ny - 0.4 * Uy * P;
  g[3] = v[0] * nz + v[3] * Un + K * nz - 0.4 * Uz * P;
  g[4] = 0.4 * P + v[4] * Un;
  g[5] = v[5] * Un;
}

// Forward-mode dual number with N derivative components (used once per face, on one thread).
template <int N> struct Dual {
  double v;
  double d[N];
  __host__ __device__ Dual() : v(0.0) {
    for (int j = 0; j < N; ++j) d[j] = 0.0;
  }
  __host__ __device__ Dual(double x) : v(x) {
    for (int j = 0; j < N; ++j) d[j] = 0.0;
  }
};
template <int N> __host__ __device__ inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v + b.v);
  for (int j = 0; j < N; ++j) r.d[j] = a.d[j] + b.d[j];
  return r;
}
template <int N> __host__ __device__ inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v - b.v);
  for (int j = 0; j < N; ++j) r.d[j] = a.d[j] - b.d[j];
  return r;
}
template <int N> __host__ __device__ inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v * b.v);
  for (int j = 0; j < N; ++j) r.d[j] = a.d[j] * b.v + a.v * b.d[j];
  return r;
}
template <int N> __host__ __device__ inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v / b.v);
  for (int j = 0; j < N; ++j) r.d[j] = (a.d[j] - r.v * b.d[j]) / b.v;
  return r;
}
template <int N> __host__ __device__ inline Dual<N> powd(const Dual<N>& a, double e) {
  Dual<N> r(pow(a.v, e));
  const double f = e * pow(a.v, e - 1.0);
  for (int j = 0; j < N; ++j) r.d[j] = f * a.d[j];
  return r;
}
__host__ __device__ inline double powd(double a, double e) { return pow(a, e); }

// Face macroscopic state after the collision coupling (Eqs. 47-52) as a function of the moment sums of
// phi_bar: S1 = sum_k w (G, u G, |u|^2/2 G + R, R), S2 = sum_k w (c|c|^2 G, c R) with c = u - U_f.
// Outputs theta (13) and tau.
template <class S>
__host__ __device__ inline void face_state(const S* S1, const S* S2, double s, const GasC& g, S* th, S& tau) {
  const S rho = S1[0];
  const S U[3] = {S1[1] / rho, S1[2] / rho, S1[3] / rho};
  const S ke = S(0.5) * rho * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
  const S E = S1[4], Er = S1[5];
  const S rR = rho * S(g.R);
  const S T = S(0.4) * (E - ke) / rR;
  const S Ttr_bar = S(2.0 / 3.0) * (E - ke - Er) / rR;
  if (g.C_s > 0.0) {
    // Eq. 14
    const S x = Ttr_bar / S(g.T_ref);
    tau = S(g.mu_ref * (g.T_ref + g.C_s)) * powd(x, 1.5) / ((Ttr_bar + S(g.C_s)) * rR * Ttr_bar);
  } else {
    tau = S(g.mu_ref * pow(g.T_ref, -g.omega_v)) * powd(Ttr_bar, g.omega_v) / (rR * Ttr_bar);
  }
  const S Erot = (S(g.Z) * tau * Er + S(s) * rR * T) / (S(g.Z) * tau + S(s));
  const S den_tr = tau + S(s) - S((s / 3.0) * (1.0 - 1.0 / g.Z + g.omega0 / g.Z));
  const S den_rot = tau + S(s) - S(s * (1.0 - g.delta) * (1.0 - 1.0 / g.Z + g.omega1 / g.Z));
  th[0] = rho;
  th[1] = U[0];
  th[2] = U[1];
  th[3] = U[2];
  th[4] = T;
  th[5] = S(2.0 / 3.0) * (E - ke - Erot) / rR;
  th[6] = Erot / rR;
  for (int d = 0; d < 3; ++d) {
    th[7 + d] = tau * S(0.5) * S2[d] / den_tr;
    th[10 + d] = tau * S2[3 + d] / den_rot;
  }
}

// Jacobian of (rho, U, T, T_tr, T_rot) with respect to W = (rho, rho U, rho E, rho E_rot) (Eqs. 1-5),
// applied transposed: gW += (d prim / d W)^T gprim, gprim = (g_rho, g_U[3], g_T, g_Ttr, g_Trot).
__host__ __device__ inline void prim_vjp(const double* W, double R, const double* gp, double* gW) {
  const double r = W[0];
  const double U[3] = {W[1] / r, W[2] / r, W[3] / r};
  const double U2 = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
  const double ke = 0.5 * r * U2;
  const double T = 0.4 * (W[4] - ke) / (r * R);
  const double Trot = W[5] / (r * R);
  const double Ttr = (2.0 / 3.0) * (W[4] - ke - W[5]) / (r * R);
  // rho
  gW[0] += gp[0];
  for (int e = 0; e < 3; ++e) {
    gW[0] += gp[1 + e] * (-U[e] / r);
    gW[1 + e] += gp[1 + e] / r;
  }
  // T = 0.4 (W4 - ke)/(r R): dke/dW0 = -U2/2, dke/dW_e = U_e
  gW[0] += gp[4] * (0.4 * 0.5 * U2 / (r * R) - T / r);
  for (int e = 0; e < 3; ++e) gW[1 + e] += gp[4] * (-0.4 * U[e] / (r * R));
  gW[4] += gp[4] * (0.4 / (r * R));
  // T_tr = (2/3)(W4 - ke - W5)/(r R)
  gW[0] += gp[5] * ((2.0 / 3.0) * 0.5 * U2 / (r * R) - Ttr / r);
  for (int e = 0; e < 3; ++e) gW[1 + e] += gp[5] * (-(2.0 / 3.0) * U[e] / (r * R));
  gW[4] += gp[5] * ((2.0 / 3.0) / (r * R));
  gW[5] += gp[5] * (-(2.0 / 3.0) / (r * R));
  // T_rot = W5/(r R)
  gW[0] += gp[6] * (-Trot / r);
  gW[5] += gp[6] / (r * R);
}

}  // namespace cis
