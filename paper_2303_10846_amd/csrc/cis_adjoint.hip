// gfx950 kernels of the steady residual and its vector-Jacobian product (FP64).
//
// The steady residual R(x; p) of the state x = (G, R, W, q) is the fixed point of one implicit iteration
// (Sec. 3.5) with the predicted state equal to the current one:
//   R_phi = (phi*(W, q) - phi)/tau(W) - F(phi; p)                         (right-hand side of Eq. 33)
//   R_W   = W - [sum_k w Phi (phi - phi*) + M(W)],  M(W) = analytic moments of phi*  (Eqs. 62-65)
//   R_q   = q - [1/2 sum_k w c|c|^2 (G - G*) + a0 q_tr;  sum_k w c (R - R*) + a1 q_rot]   (Eqs. 66-67)
// with p = (T_w of one wall, rho_inf and |U_inf| of the far field).  The objective is the wall heat flux
// J = sum over the wall faces of A sum_k w (u.n)(|u|^2/2 G_f + R_f) (Eq. 72 numerator).
//
// The VJP runs backwards through the steps of the micro flux: the cell terms (one workgroup per cell), the
// face collision coupling of Eqs. 45, 47-52 and the boundary conditions (one workgroup per face), and the
// limited least-squares reconstruction of Eq. 46 (workgroup per (cell, velocity chunk), FP64 atomics into
// the neighbour rows).  The face macroscopic state is a function of 12 moment sums; its 14 x 12 Jacobian
// is taken once per face with forward-mode dual numbers.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "cis_adjoint.h"
#include "cis_adjoint_math.h"
#include "cis_device.h"
#include "cis_internal.h"

namespace cis {

namespace {

// Velocity loop of a per-face / per-cell workgroup.
template <class F> __device__ inline void v_loop(int64_t nv, F&& body) {
  for (int64_t k = threadIdx.x; k < nv; k += kBlock) body(k);
}

// theta = (rho, U, T, T_tr, T_rot, q_tr, q_rot) and tau of a cell state (Eqs. 1-5, 13)
__device__ inline double cell_theta(const double* W, const double* q, const GasC& g, double* th, Prim& p) {
  p = prim_of(W, g.R);
  th[0] = p.rho;
  th[1] = p.U[0];
  th[2] = p.U[1];
  th[3] = p.U[2];
  th[4] = p.T;
  th[5] = p.Ttr;
  th[6] = p.Trot;
  for (int m = 0; m < 6; ++m) th[7 + m] = q[m];
  return visc(p.Ttr, g) / (p.rho * g.R * p.Ttr);
}

}  // namespace

// ---------------------------------------------------------------------------
// Steady residual per cell.  rG, rR hold the micro flux F (Eq. 31) on entry and R_phi on exit.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_cell_steady(Dev d, Bufs b, double* rG, double* rR, double* rW,
                                                        double* rq) {
  __shared__ double red[(kBlock / 64) * 2 * 12];
  const int64_t i = blockIdx.x, nv = d.nv;
  const GasC& g = d.gas;
  const double* W = b.W + 6 * i;
  double th[NTH];
  Prim p;
  const double tau = cell_theta(W, b.q + 6 * i, g, th, p);
  const double it = 1.0 / tau;
  EqAd e;
  e.setup(th, g);
  const double* G = (const double*)b.G + i * nv;
  const double* R = (const double*)b.R + i * nv;
  Acc<12, false, kBlock> acc;
  acc.zero();
  v_loop(nv, [&](int64_t k) {
    const Vel v = vel(d, k);
    double Gs, Rs;
    e.eval(v.ux, v.uy, v.uz, Gs, Rs, nullptr, nullptr);
    const double gk = G[k], rk = R[k];
    rG[i * nv + k] = (Gs - gk) * it - rG[i * nv + k];
    rR[i * nv + k] = (Rs - rk) * it - rR[i * nv + k];
    const double gd = v.w * (gk - Gs), rd = v.w * (rk - Rs);
    const double cx = v.ux - p.U[0], cy = v.uy - p.U[1], cz = v.uz - p.U[2];
    const double c2 = cx * cx + cy * cy + cz * cz;
    acc.add(0, gd);
    acc.add(1, v.ux * gd);
    acc.add(2, v.uy * gd);
    acc.add(3, v.uz * gd);
    acc.add(4, v.h2 * gd + rd);
    acc.add(5, rd);
    acc.add(6, 0.5 * cx * c2 * gd);
    acc.add(7, 0.5 * cy * c2 * gd);
    acc.add(8, 0.5 * cz * c2 * gd);
    acc.add(9, cx * rd);
    acc.add(10, cy * rd);
    acc.add(11, cz * rd);
  });
  double s[12];
  acc.reduce(s, red);
  if (threadIdx.x == 0) {
    for (int m = 0; m < 5; ++m) rW[6 * i + m] = W[m] - (s[m] + W[m]);
    rW[6 * i + 5] = W[5] - (s[5] + p.rho * g.R * ((1.0 - 1.0 / g.Z) * p.Trot + p.T / g.Z));
    const double a0 = (1.0 / 3.0) * (1.0 - (1.0 - g.omega0) / g.Z);
    const double a1 = (1.0 - g.delta) * (1.0 - (1.0 - g.omega1) / g.Z);
    const double* q = b.q + 6 * i;
    for (int m = 0; m < 3; ++m) {
      rq[6 * i + m] = q[m] - (s[6 + m] + q[m] * a0);
      rq[6 * i + 3 + m] = q[3 + m] - (s[9 + m] + q[3 + m] * a1);
    }
  }
}

void launch_cell_steady(const Dev& d, const Bufs& b, double* rG, double* rR, double* rW, double* rq, hipStream_t st) {
  hipLaunchKernelGGL(k_cell_steady, dim3((unsigned)d.nc), dim3(kBlock), 0, st, d, b, rG, rR, rW, rq);
}

// ---------------------------------------------------------------------------
// VJP, cell terms: everything of R_phi, R_W, R_q except the micro flux.  Writes gG, gR (plain stores), gW, gq.
// PhiOnly: the seed is (vG, vR) alone and only gW, gq are written, i.e. (dR_phi/d(W, q))^T v_phi.
// ---------------------------------------------------------------------------

template <bool HasV, bool PhiOnly = false>
__global__ __launch_bounds__(kBlock) void k_cell_vjp(Dev d, Bufs b, AdjArgs a) {
  __shared__ double red[(kBlock / 64) * 2 * 17];
  const int64_t i = blockIdx.x, nv = d.nv;
  const GasC& g = d.gas;
  const double* W = b.W + 6 * i;
  double th[NTH];
  Prim p;
  const double tau = cell_theta(W, b.q + 6 * i, g, th, p);
  const double it = 1.0 / tau;
  EqAd e;
  e.setup(th, g);
  double vW[6], vq[6];
  for (int m = 0; m < 6; ++m) {
    vW[m] = HasV && !PhiOnly ? a.vW[6 * i + m] : 0.0;
    vq[m] = HasV && !PhiOnly ? a.vq[6 * i + m] : 0.0;
  }
  const double* G = (const double*)b.G + i * nv;
  const double* R = (const double*)b.R + i * nv;
  Acc<17, false, kBlock> acc;
  acc.zero();
  v_loop(nv, [&](int64_t k) {
    const Vel v = vel(d, k);
    double Gs, Rs, dG[NTH], dR[NTH];
    e.eval(v.ux, v.uy, v.uz, Gs, Rs, dG, dR);
    const double gk = G[k], rk = R[k];
    const double vg = HasV ? a.vG[i * nv + k] : 0.0, vr = HasV ? a.vR[i * nv + k] : 0.0;
    const double cx = v.ux - p.U[0], cy = v.uy - p.U[1], cz = v.uz - p.U[2];
    const double c2 = cx * cx + cy * cy + cz * cz;
    const double vqc = vq[0] * cx + vq[1] * cy + vq[2] * cz;
    // -(dR/dphi_k)^T v: the collision term, the moments of R_W and the heat-flux sums of R_q
    const double aG = vg * it + v.w * (vW[0] + vW[1] * v.ux + vW[2] * v.uy + vW[3] * v.uz + vW[4] * v.h2 + 0.5 * c2 * vqc);
    const double aR = vr * it + v.w * (vW[4] + vW[5] + vq[3] * cx + vq[4] * cy + vq[5] * cz);
    if (!PhiOnly) {
      a.gG[i * nv + k] = -aG;
      a.gR[i * nv + k] = -aR;
    }
#pragma unroll
    for (int m = 0; m < NTH; ++m) acc.add(m, aG * dG[m] + aR * dR[m]);
    acc.add(13, -(vg * (Gs - gk) + vr * (Rs - rk)) * it * it);
    // c = u - U inside the heat-flux sums of R_q
    const double gd = v.w * (gk - Gs), rd = v.w * (rk - Rs);
    acc.add(14, gd * (0.5 * vq[0] * c2 + vqc * cx) + vq[3] * rd);
    acc.add(15, gd * (0.5 * vq[1] * c2 + vqc * cy) + vq[4] * rd);
    acc.add(16, gd * (0.5 * vq[2] * c2 + vqc * cz) + vq[5] * rd);
  });
  double s[17];
  acc.reduce(s, red);
  if (threadIdx.x == 0) {
    const double a0 = (1.0 / 3.0) * (1.0 - (1.0 - g.omega0) / g.Z);
    const double a1 = (1.0 - g.delta) * (1.0 - (1.0 - g.omega1) / g.Z);
    for (int m = 0; m < 3; ++m) {
      a.gq[6 * i + m] = vq[m] * (1.0 - a0) + s[7 + m];
      a.gq[6 * i + 3 + m] = vq[3 + m] * (1.0 - a1) + s[10 + m];
    }
    const double taubar = s[13];
    const double z2 = 1.0 / g.Z, z1 = 1.0 - z2;
    double gp[7];
    gp[0] = s[0] - taubar * tau / p.rho - vW[5] * g.R * (z1 * p.Trot + z2 * p.T);
    gp[1] = s[1] + s[14];
    gp[2] = s[2] + s[15];
    gp[3] = s[3] + s[16];
    gp[4] = s[4] - vW[5] * p.rho * g.R * z2;
    gp[5] = s[5] + taubar * tau * (visc_exponent(p.Ttr, g) - 1.0) / p.Ttr;
    gp[6] = s[6] - vW[5] * p.rho * g.R * z1;
    double gW[6] = {0, 0, 0, 0, 0, 0};
    prim_vjp(W, g.R, gp, gW);
    gW[5] += vW[5];
    for (int m = 0; m < 6; ++m) a.gW[6 * i + m] = gW[m];
  }
}

// ---------------------------------------------------------------------------
// VJP, face terms.  On entry faceG/faceR hold phi_bar (Eq. 46); on exit the adjoint of phi_bar.
// The seed of the face flux A (u.n) phi_f is -A (u.n)(v_o/V_o - v_n/V_n), plus the objective's.
// ---------------------------------------------------------------------------

template <bool HasV, int NF> __global__ __launch_bounds__(kBlock) void k_face_vjp(Dev d, Bufs b, AdjArgs a) {
  __shared__ double red[(kBlock / 64) * 2 * 14];
  __shared__ double sh_th[NTH + 1], sh_jac[14 * 12], sh_bar[12];
  const int64_t f = blockIdx.x, nv = d.nv;
  const double* fg = d.face_geo + FGW * f;
  const double A = fg[0], nx = fg[1], ny = fg[2], nz = fg[3], s = fg[4];
  const int64_t o = d.face_cell[2 * f], nb = d.face_cell[2 * f + 1];
  const double iVo = d.cell_geo[Lay<NF>::CG * o + 1], iVn = nb >= 0 ? d.cell_geo[Lay<NF>::CG * nb + 1] : 0.0;
  double* rowG = (double*)b.faceG + f * nv;
  double* rowR = (double*)b.faceR + f * nv;
  const int32_t bcs = d.face_bc[f];
  const GasC& g = d.gas;
  const double cJ = (bcs >= 0 && bcs == a.jslot) ? a.cJ : 0.0;
  // adjoint of the face value A (u.n) phi_f
  auto seed = [&](int64_t k, const Vel& v, double un, double& sg, double& sr) {
    double tg = 0.0, tr = 0.0;
    if (HasV) {
      tg = -a.vG[o * nv + k] * iVo;
      tr = -a.vR[o * nv + k] * iVo;
      if (nb >= 0) {
        tg += a.vG[nb * nv + k] * iVn;
        tr += a.vR[nb * nv + k] * iVn;
      }
    }
    sg = A * un * (tg + cJ * v.w * v.h2);
    sr = A * un * (tr + cJ * v.w);
  };

  if (bcs < 0) {
    // forward: moment sums S1 (Eqs. 47-49), heat-flux sums S2 (Eqs. 51-52) and the second moments of G_bar
    Acc<6, false, kBlock> a6;
    a6.zero();
    v_loop(nv, [&](int64_t k) {
      const Vel v = vel(d, k);
      const double wg = v.w * rowG[k], wr = v.w * rowR[k];
      a6.add(0, wg);
      a6.add(1, v.ux * wg);
      a6.add(2, v.uy * wg);
      a6.add(3, v.uz * wg);
      a6.add(4, v.h2 * wg + wr);
      a6.add(5, wr);
    });
    double S1[6];
    a6.reduce(S1, red);
    const double rho = S1[0];
    const double U[3] = {S1[1] / rho, S1[2] / rho, S1[3] / rho};
    Acc<12, false, kBlock> a12;
    a12.zero();
    v_loop(nv, [&](int64_t k) {
      const Vel v = vel(d, k);
      const double cx = v.ux - U[0], cy = v.uy - U[1], cz = v.uz - U[2];
      const double c2 = cx * cx + cy * cy + cz * cz;
      const double wg = v.w * rowG[k], wr = v.w * rowR[k];
      a12.add(0, cx * c2 * wg);
      a12.add(1, cy * c2 * wg);
      a12.add(2, cz * c2 * wg);
      a12.add(3, cx * wr);
      a12.add(4, cy * wr);
      a12.add(5, cz * wr);
      a12.add(6, cx * cx * wg);
      a12.add(7, cy * cy * wg);
      a12.add(8, cz * cz * wg);
      a12.add(9, cx * cy * wg);
      a12.add(10, cx * cz * wg);
      a12.add(11, cy * cz * wg);
    });
    double S2M[12];
    a12.reduce(S2M, red);
    if (threadIdx.x == 0) {
      Dual<12> x1[6], x2[6], th[NTH], tau;
      for (int m = 0; m < 6; ++m) {
        x1[m] = Dual<12>(S1[m]);
        x1[m].d[m] = 1.0;
        x2[m] = Dual<12>(S2M[m]);
        x2[m].d[6 + m] = 1.0;
      }
      face_state(x1, x2, s, g, th, tau);
      for (int m = 0; m < NTH; ++m) {
        sh_th[m] = th[m].v;
        for (int j = 0; j < 12; ++j) sh_jac[12 * m + j] = th[m].d[j];
      }
      sh_th[NTH] = tau.v;
      for (int j = 0; j < 12; ++j) sh_jac[12 * NTH + j] = tau.d[j];
    }
    __syncthreads();
    double th[NTH];
    for (int m = 0; m < NTH; ++m) th[m] = sh_th[m];
    const double tau = sh_th[NTH];
    EqAd e;
    e.setup(th, g);
    const double ct = tau / (tau + s), cs = s / (tau + s), ctau = s / ((tau + s) * (tau + s));
    // reverse of Eq. 45: adjoints of theta and tau
    Acc<14, false, kBlock> a14;
    a14.zero();
    v_loop(nv, [&](int64_t k) {
      const Vel v = vel(d, k);
      const double un = udotn(v, nx, ny, nz, d.snap);
      double sg, sr;
      seed(k, v, un, sg, sr);
      double Gs, Rs, dG[NTH], dR[NTH];
      e.eval(v.ux, v.uy, v.uz, Gs, Rs, dG, dR);
#pragma unroll
      for (int m = 0; m < NTH; ++m) a14.add(m, cs * (sg * dG[m] + sr * dR[m]));
      a14.add(13, ctau * (sg * (rowG[k] - Gs) + sr * (rowR[k] - Rs)));
    });
    double tb[14];
    a14.reduce(tb, red);
    if (threadIdx.x == 0) {
      double Sb[12];
      for (int j = 0; j < 12; ++j) {
        double x = 0.0;
        for (int m = 0; m < 14; ++m) x += sh_jac[12 * m + j] * tb[m];
        Sb[j] = x;
      }
      // U = S1[1..3]/S1[0] inside S2: dS2q_d/dU_e = -(delta_de trM + 2 M_de), dS2r_d/dU_e = -delta_de S1[5]
      const double M[3][3] = {{S2M[6], S2M[9], S2M[10]}, {S2M[9], S2M[7], S2M[11]}, {S2M[10], S2M[11], S2M[8]}};
      const double trM = S2M[6] + S2M[7] + S2M[8];
      // Sb[0..5]: adjoint of S1, Sb[6..8]: of the q_tr sums, Sb[9..11]: of the q_rot sums
      double Ub[3];
      for (int ee = 0; ee < 3; ++ee) {
        double x = -Sb[6 + ee] * trM - Sb[9 + ee] * S1[5];
        for (int dd = 0; dd < 3; ++dd) x -= 2.0 * Sb[6 + dd] * M[dd][ee];
        Ub[ee] = x;
      }
      double s1b[6];
      for (int m = 0; m < 6; ++m) s1b[m] = Sb[m];
      for (int ee = 0; ee < 3; ++ee) {
        s1b[1 + ee] += Ub[ee] / rho;
        s1b[0] -= Ub[ee] * U[ee] / rho;
      }
      for (int m = 0; m < 6; ++m) {
        sh_bar[m] = s1b[m];
        sh_bar[6 + m] = Sb[6 + m];
      }
    }
    __syncthreads();
    double sb[12];
    for (int m = 0; m < 12; ++m) sb[m] = sh_bar[m];
    v_loop(nv, [&](int64_t k) {
      const Vel v = vel(d, k);
      const double un = udotn(v, nx, ny, nz, d.snap);
      double sg, sr;
      seed(k, v, un, sg, sr);
      const double cx = v.ux - U[0], cy = v.uy - U[1], cz = v.uz - U[2];
      const double c2 = cx * cx + cy * cy + cz * cz;
      rowG[k] = ct * sg + v.w * (sb[0] + sb[1] * v.ux + sb[2] * v.uy + sb[3] * v.uz + sb[4] * v.h2 +
                                 c2 * (sb[6] * cx + sb[7] * cy + sb[8] * cz));
      rowR[k] = ct * sr + v.w * (sb[4] + sb[5] + sb[9] * cx + sb[10] * cy + sb[11] * cz);
    });
    if (threadIdx.x == 0) {
      a.gpf[3 * f] = 0.0;
      a.gpf[3 * f + 1] = 0.0;
      a.gpf[3 * f + 2] = 0.0;
    }
    return;
  }

  // boundary face: outgoing velocities carry phi_bar, incoming ones the wall or free-stream Maxwellian
  const double* bc = d.bc + BCW * bcs;
  const bool wall = bc[0] == 1.0;
  const double Ub[3] = {bc[2], bc[3], bc[4]}, Tb = bc[5];
  const double RTb = g.R * Tb;
  const double anorm = pow(6.283185307179586476925 * RTb, -1.5), bexp = 1.0 / (2.0 * RTb);
  auto maxw = [&](const Vel& v, double& c2, double& cU) {
    const double cx = v.ux - Ub[0], cy = v.uy - Ub[1], cz = v.uz - Ub[2];
    c2 = cx * cx + cy * cy + cz * cz;
    cU = cx * Ub[0] + cy * Ub[1] + cz * Ub[2];
    return anorm * exp(-c2 * bexp);
  };
  double gp0 = 0.0, gp1 = 0.0, gp2 = 0.0;
  if (wall) {
    // rho_w = out/in (zero net mass flux); din = d(in)/dT_w
    Acc<3, false, kBlock> a3;
    a3.zero();
    v_loop(nv, [&](int64_t k) {
      const Vel v = vel(d, k);
      const double un = udotn(v, nx, ny, nz, d.snap);
      if (un > 0.0) {
        a3.add(0, v.w * un * rowG[k]);
      } else {
        double c2, cU;
        const double m1 = maxw(v, c2, cU);
        a3.add(1, v.w * (-un) * m1);
        a3.add(2, v.w * (-un) * m1 * (c2 * bexp - 1.5) / Tb);
      }
    });
    double t3[3];
    a3.reduce(t3, red);
    const double in = t3[1], rho_w = t3[0] / in;
    // adjoint of rho_w and the T_w terms of the incoming half
    Acc<3, false, kBlock> b3;
    b3.zero();
    v_loop(nv, [&](int64_t k) {
      const Vel v = vel(d, k);
      const double un = udotn(v, nx, ny, nz, d.snap);
      if (un > 0.0) return;
      double sg, sr, c2, cU;
      seed(k, v, un, sg, sr);
      const double m1 = maxw(v, c2, cU);
      const double dm1 = m1 * (c2 * bexp - 1.5) / Tb;
      b3.add(0, (sg + RTb * sr) * m1);
      b3.add(1, (sg + RTb * sr) * rho_w * dm1);
      b3.add(2, sr * g.R * rho_w * m1);
    });
    double u3[3];
    b3.reduce(u3, red);
    const double rho_wb = u3[0];
    if (bcs == a.wslot) gp0 = u3[1] + u3[2] + rho_wb * (-rho_w / in) * t3[2];
    v_loop(nv, [&](int64_t k) {
      const Vel v = vel(d, k);
      const double un = udotn(v, nx, ny, nz, d.snap);
      if (un > 0.0) {
        double sg, sr;
        seed(k, v, un, sg, sr);
        rowG[k] = sg + rho_wb * v.w * un / in;
        rowR[k] = sr;
      } else {
        rowG[k] = 0.0;
        rowR[k] = 0.0;
      }
    });
  } else {
    const double rho_inf = bc[1];
    const double Um = sqrt(Ub[0] * Ub[0] + Ub[1] * Ub[1] + Ub[2] * Ub[2]);
    if (bcs == a.fslot) {
      Acc<2, false, kBlock> b2;
      b2.zero();
      v_loop(nv, [&](int64_t k) {
        const Vel v = vel(d, k);
        const double un = udotn(v, nx, ny, nz, d.snap);
        if (un > 0.0) return;
        double sg, sr, c2, cU;
        seed(k, v, un, sg, sr);
        const double m1 = maxw(v, c2, cU);
        const double t = (sg + RTb * sr) * m1;
        b2.add(0, t);
        b2.add(1, Um > 0.0 ? t * rho_inf * cU / (Um * RTb) : 0.0);
      });
      double u2[2];
      b2.reduce(u2, red);
      gp1 = u2[0];
      gp2 = u2[1];
    }
    v_loop(nv, [&](int64_t k) {
      const Vel v = vel(d, k);
      const double un = udotn(v, nx, ny, nz, d.snap);
      if (un > 0.0) {
        double sg, sr;
        seed(k, v, un, sg, sr);
        rowG[k] = sg;
        rowR[k] = sr;
      } else {
        rowG[k] = 0.0;
        rowR[k] = 0.0;
      }
    });
  }
  if (threadIdx.x == 0) {
    a.gpf[3 * f] = gp0;
    a.gpf[3 * f + 1] = gp1;
    a.gpf[3 * f + 2] = gp2;
  }
}

// ---------------------------------------------------------------------------
// VJP, reconstruction (Eq. 46): the adjoint of phi_bar on the faces where a cell is upwind goes to the
// cell's own value and, through the limited least-squares gradient, to its face neighbours.
// Workgroup (cell, 256 velocities); contributions are added with FP64 atomics.
// ---------------------------------------------------------------------------

template <int NF>
__device__ inline void recon_vjp_one(const Dev& d, const double* __restrict__ src, const double* __restrict__ fadj,
                                     double* gout, int64_t i, int64_t k, const int32_t* nb, const int32_t* fc,
                                     const double* geo, double kh3, const Vel& v, const double* un,
                                     const double* Lfrozen) {
  const int64_t nv = d.nv;
  // adjoint of phi_bar gathered from the faces of which this cell is the upwind side
  double pself = 0.0, gbx = 0.0, gby = 0.0, gbz = 0.0;
  bool any = false;
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    const double* s = geo + CG_FACE + CG_SLOT * a;
    bool up = nb[a] >= 0 ? (s[0] > 0.0 ? un[a] > 0.0 : un[a] >= 0.0) : un[a] > 0.0;
    if (!up) continue;
    const double pb = fadj[(int64_t)fc[a] * nv + k];
    any = true;
    pself += pb;
    gbx += pb * (s[5] - v.ux * s[8]);
    gby += pb * (s[6] - v.uy * s[8]);
    gbz += pb * (s[7] - v.uz * s[8]);
  }
  if (!any) return;
  // forward: least-squares gradient, extrema of the stencil and the limiter (same branches as Step 2(a))
  const double phi = src[i * nv + k];
  double pn[NF];
#pragma unroll
  for (int a = 0; a < NF; ++a) pn[a] = nb[a] >= 0 ? src[(int64_t)nb[a] * nv + k] : phi;
  double gx = 0, gy = 0, gz = 0, pmax = phi, pmin = phi;
  int imax = -1, imin = -1;
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    if (nb[a] < 0) continue;
    const double* s = geo + CG_FACE + CG_SLOT * a;
    const double dphi = pn[a] - phi;
    gx += s[9] * dphi;
    gy += s[10] * dphi;
    gz += s[11] * dphi;
    if (pn[a] > pmax) {
      pmax = pn[a];
      imax = a;
    }
    if (pn[a] < pmin) {
      pmin = pn[a];
      imin = a;
    }
  }
  double L = 1.0, d1m = 0.0, d2m = 0.0, eps2 = 0.0;
  int amin = -1, isel = -1;
  double psel = 0.0;
  if (d.limiter == 3) {
    L = Lfrozen[i * nv + k];  // frozen values: constants of the linearisation
  } else if (d.limiter) {
    const bool use_max = fabs(pmax) > fabs(pmin);
    psel = use_max ? pmax : pmin;
    isel = use_max ? imax : imin;
    eps2 = kh3 * psel * psel;
#pragma unroll
    for (int a = 0; a < NF; ++a) {
      const double* s = geo + CG_FACE + CG_SLOT * a;
      const double d2 = gx * s[5] + gy * s[6] + gz * s[7];
      if (d2 != 0.0) {
        const double d1 = d2 > 0.0 ? pmax - phi : pmin - phi;
        const double psi = ((d1 * d1 + eps2) * d2 + 2.0 * d2 * d2 * d1) / (d2 * (d1 * d1 + 2.0 * d2 * d2 + d1 * d2 + eps2));
        if (psi < L) {
          L = psi;
          amin = a;
          d1m = d1;
          d2m = d2;
        }
      }
    }
  }
  // reverse: grad_out = L g
  double pnb[NF];
#pragma unroll
  for (int a = 0; a < NF; ++a) pnb[a] = 0.0;
  auto add_to = [&](int idx, double x) {
    if (idx < 0) {
      pself += x;
    } else {
#pragma unroll
      for (int a = 0; a < NF; ++a)
        if (a == idx) pnb[a] += x;
    }
  };
  double grx = L * gbx, gry = L * gby, grz = L * gbz;
  // the limiter's own derivative; limiter = 2 holds L fixed (frozen-limiter linearisation), limiter = 3 stores it
  if (amin >= 0 && d.limiter == 1) {
    const double Lb = gbx * gx + gby * gy + gbz * gz;
    const double d1 = d1m, d2 = d2m;
    const double N = (d1 * d1 + eps2) * d2 + 2.0 * d2 * d2 * d1;
    const double D = d2 * (d1 * d1 + 2.0 * d2 * d2 + d1 * d2 + eps2);
    const double psi = N / D;
    const double p_d1 = ((2.0 * d1 * d2 + 2.0 * d2 * d2) - psi * d2 * (2.0 * d1 + d2)) / D;
    const double p_d2 = ((d1 * d1 + eps2 + 4.0 * d1 * d2) - psi * (d1 * d1 + 6.0 * d2 * d2 + 2.0 * d1 * d2 + eps2)) / D;
    const double p_e = (d2 - psi * d2) / D;
    const double* s = geo + CG_FACE + CG_SLOT * amin;
    grx += Lb * p_d2 * s[5];
    gry += Lb * p_d2 * s[6];
    grz += Lb * p_d2 * s[7];
    const double d1b = Lb * p_d1;
    add_to(d2 > 0.0 ? imax : imin, d1b);
    pself -= d1b;
    add_to(isel, Lb * p_e * 2.0 * kh3 * psel);
  }
#pragma unroll
  for (int a = 0; a < NF; ++a) {
    if (nb[a] < 0) continue;
    const double* s = geo + CG_FACE + CG_SLOT * a;
    const double t = s[9] * grx + s[10] * gry + s[11] * grz;
    pnb[a] += t;
    pself -= t;
  }
  unsafeAtomicAdd(gout + i * nv + k, pself);
#pragma unroll
  for (int a = 0; a < NF; ++a)
    if (nb[a] >= 0 && pnb[a] != 0.0) unsafeAtomicAdd(gout + (int64_t)nb[a] * nv + k, pnb[a]);
}

template <int NF> __global__ __launch_bounds__(kBlock) void k_recon_vjp(Dev d, Bufs b, AdjArgs a) {
  const int64_t i = blockIdx.x, nv = d.nv;
  const int64_t k = (int64_t)blockIdx.y * kBlock + threadIdx.x;
  if (k >= nv) return;
  int32_t nb[NF], fc[NF];
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    nb[q] = d.cell_nb[NF * i + q];
    fc[q] = d.cell_face[NF * i + q];
  }
  const double* geo = d.cell_geo + Lay<NF>::CG * i;
  double kh3 = d.lim_K * geo[2];
  kh3 = kh3 * kh3 * kh3;
  const Vel v = vel(d, k);
  double un[NF];
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    const double* s = geo + CG_FACE + CG_SLOT * q;
    un[q] = udotn(v, s[2], s[3], s[4], d.snap);
  }
  const double* LG = (const double*)d.lim_frozen;
  const double* LR = LG ? LG + d.nc * nv : nullptr;
  recon_vjp_one<NF>(d, (const double*)b.G, (const double*)b.faceG, a.gG, i, k, nb, fc, geo, kh3, v, un, LG);
  recon_vjp_one<NF>(d, (const double*)b.R, (const double*)b.faceR, a.gR, i, k, nb, fc, geo, kh3, v, un, LR);
}

template <int NF> void launch_vjp_nf(const Dev& d, const Bufs& b, const AdjArgs& a, hipStream_t st) {
  const bool hv = a.vG != nullptr;
  launch_recon<double>(d, b, st);
  if (hv) {
    hipLaunchKernelGGL((k_face_vjp<true, NF>), dim3((unsigned)d.nf), dim3(kBlock), 0, st, d, b, a);
    hipLaunchKernelGGL(k_cell_vjp<true>, dim3((unsigned)d.nc), dim3(kBlock), 0, st, d, b, a);
  } else {
    hipLaunchKernelGGL((k_face_vjp<false, NF>), dim3((unsigned)d.nf), dim3(kBlock), 0, st, d, b, a);
    hipLaunchKernelGGL(k_cell_vjp<false>, dim3((unsigned)d.nc), dim3(kBlock), 0, st, d, b, a);
  }
  const unsigned nch = (unsigned)((d.nv + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_recon_vjp<NF>, dim3((unsigned)d.nc, nch), dim3(kBlock), 0, st, d, b, a);
}

void launch_vjp(const Dev& d, const Bufs& b, const AdjArgs& a, hipStream_t st) {
  if (d.mf == 4)
    launch_vjp_nf<4>(d, b, a, st);
  else
    launch_vjp_nf<kMaxFaces>(d, b, a, st);
}

// ---------------------------------------------------------------------------
// Adjoint solve: diagonal preconditioner and the vector kernels of restarted GMRES.
// ---------------------------------------------------------------------------

// out = M^-1 in: the phi rows are divided by -(1/tau_i + sum_f (A_f/V_i) max(u.n_out, 0)), the diagonal of
// dR_phi/dphi with first-order upwind faces; the W and q rows are copied (their blocks are near identity).
template <int NF> __global__ __launch_bounds__(kBlock) void k_precond(Dev d, Bufs b, const double* in, double* out) {
  const int64_t i = blockIdx.x, nv = d.nv;
  const int64_t P = d.nc * nv;
  const double* geo = d.cell_geo + Lay<NF>::CG * i;
  Prim p = prim_of(b.W + 6 * i, d.gas.R);
  const double itau = (p.rho * d.gas.R * p.Ttr) / visc(p.Ttr, d.gas);
  for (int64_t k = (int64_t)blockIdx.y * kBlock + threadIdx.x; k < nv; k += (int64_t)gridDim.y * kBlock) {
    const Vel v = vel(d, k);
    double D = itau;
#pragma unroll
    for (int a = 0; a < NF; ++a) {
      const double* s = geo + CG_FACE + CG_SLOT * a;
      const double un = udotn(v, s[2], s[3], s[4], d.snap);
      if (un > 0.0) D += s[1] * un;
    }
    out[i * nv + k] = -in[i * nv + k] / D;
    out[P + i * nv + k] = -in[P + i * nv + k] / D;
  }
  if (blockIdx.y == 0 && threadIdx.x < 12) {
    const int64_t o = 2 * P + (threadIdx.x < 6 ? 6 * i + threadIdx.x : 6 * d.nc + 6 * i + threadIdx.x - 6);
    out[o] = in[o];
  }
}

void launch_precond(const Dev& d, const Bufs& b, const double* in, double* out, hipStream_t st) {
  const unsigned nch = (unsigned)std::min<int64_t>((d.nv + kBlock - 1) / kBlock, 64);
  if (d.mf == 4)
    hipLaunchKernelGGL(k_precond<4>, dim3((unsigned)d.nc, nch), dim3(kBlock), 0, st, d, b, in, out);
  else
    hipLaunchKernelGGL(k_precond<kMaxFaces>, dim3((unsigned)d.nc, nch), dim3(kBlock), 0, st, d, b, in, out);
}

// ---------------------------------------------------------------------------
// Block preconditioner over (phi, Y = (W, q)).  With x = (phi, Y), dR/dx = [[A, B], [C, E]] where B = dR_phi/dY
// and C = dR_Y/dphi = -M (the moment and heat-flux sums of R_W, R_q) are cell-local and E ~ I.  For
// (dR/dx)^T x = s, eliminating Y gives
//   S x_phi = s_phi + M^T s_Y,  S = (A - B C)^T,   x_Y = s_Y - B^T x_phi.
// A - B C is the collision-coupled transport operator whose slow modes are the macroscopic ones; the implicit
// step of Steps 4-5 linearised, (D + N)^-1 [I + (1/tau) dphi*/dW Mac^-1 M_c] (macro system of Eq. 43, then the
// micro system of Eq. 33 with the predicted equilibrium), approximates -(A - B C)^-1, so
//   x_phi = z + M_c^T Mac^-T B^T z,  z = -(D + N)^-T (s_phi + M^T s_Y),
// with B^T z from the cell VJP.  Mac is the steady macro system: D_i = sum_f (A_f/V_i) r_f / 2 (+ 1/(Z tau_i)
// for rho E_rot), off-diagonal blocks (A_f/V_i)(dG_n/dW (W_j) - r_f I)/2.
// ---------------------------------------------------------------------------

namespace {

// out_phi = in_phi + M^T in_Y (the phi rows of s - C^T s_Y); the Y rows are copied.
__global__ __launch_bounds__(kBlock) void k_adj_expand(Dev d, Bufs b, const double* in, double* out) {
  const int64_t i = blockIdx.x, nv = d.nv, P = d.nc * nv;
  const Prim p = prim_of(b.W + 6 * i, d.gas.R);
  const double* sW = in + 2 * P + 6 * i;
  const double* sq = in + 2 * P + 6 * d.nc + 6 * i;
  double vW[6], vq[6];
  for (int m = 0; m < 6; ++m) {
    vW[m] = sW[m];
    vq[m] = sq[m];
  }
  for (int64_t k = (int64_t)blockIdx.y * kBlock + threadIdx.x; k < nv; k += (int64_t)gridDim.y * kBlock) {
    const Vel v = vel(d, k);
    const double cx = v.ux - p.U[0], cy = v.uy - p.U[1], cz = v.uz - p.U[2];
    const double c2 = cx * cx + cy * cy + cz * cz;
    const double vqc = vq[0] * cx + vq[1] * cy + vq[2] * cz;
    out[i * nv + k] =
        in[i * nv + k] + v.w * (vW[0] + vW[1] * v.ux + vW[2] * v.uy + vW[3] * v.uz + vW[4] * v.h2 + 0.5 * c2 * vqc);
    out[P + i * nv + k] = in[P + i * nv + k] + v.w * (vW[4] + vW[5] + vq[3] * cx + vq[4] * cy + vq[5] * cz);
  }
  if (blockIdx.y == 0 && threadIdx.x < 12) {
    const int64_t o = 2 * P + (threadIdx.x < 6 ? 6 * i + threadIdx.x : 6 * d.nc + 6 * i + threadIdx.x - 6);
    out[o] = in[o];
  }
}

// x_phi += M_c^T u: the conserved-moment rows of the macro residual (rho, rho U, rho E from G; rho E, rho E_rot
// from R) spread back over the velocities.
__global__ __launch_bounds__(kBlock) void k_adj_lift(Dev d, const double* u, double* x) {
  const int64_t i = blockIdx.x, nv = d.nv, P = d.nc * nv;
  double c[6];
  for (int m = 0; m < 6; ++m) c[m] = u[6 * i + m];
  for (int64_t k = (int64_t)blockIdx.y * kBlock + threadIdx.x; k < nv; k += (int64_t)gridDim.y * kBlock) {
    const Vel v = vel(d, k);
    x[i * nv + k] += v.w * (c[0] + c[1] * v.ux + c[2] * v.uy + c[3] * v.uz + c[4] * v.h2);
    x[P + i * nv + k] += v.w * (c[4] + c[5]);
  }
}

// Face spectral radii r_f (Eq. 41, from the cells' own W) and the diagonals of the steady macro system.
template <int NF> __global__ __launch_bounds__(kBlock) void k_adj_macro_prep(Dev d, Bufs b, double* rc, double* mD) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.nc) return;
  const GasC& g = d.gas;
  const double* geo = d.cell_geo + Lay<NF>::CG * i;
  const Prim pa = prim_of(b.W + 6 * i, g.R);
  double acc = 0.0;
  for (int a = 0; a < NF; ++a) {
    const double* s = geo + CG_FACE + CG_SLOT * a;
    const int32_t nb = d.cell_nb[NF * i + a];
    const int32_t fc = d.cell_face[NF * i + a];
    if (fc < 0) {  // unused slot
      rc[NF * i + a] = 0.0;
      continue;
    }
    const Prim pb = nb >= 0 ? prim_of(b.W + 6 * (int64_t)nb, g.R) : pa;
    const double rho = 0.5 * (pa.rho + pb.rho), T = 0.5 * (pa.T + pb.T), Ttr = 0.5 * (pa.Ttr + pb.Ttr);
    const double Un = 0.5 * ((pa.U[0] + pb.U[0]) * s[2] + (pa.U[1] + pb.U[1]) * s[3] + (pa.U[2] + pb.U[2]) * s[4]);
    const double r = fabs(Un) + sqrt(g.gamma * g.R * T) +
                     2.0 * visc(Ttr, g) / (rho * d.face_geo[FGW * (int64_t)fc + 5]);
    rc[NF * i + a] = r;
    acc += 0.5 * s[1] * r;
  }
  const double tau = visc(pa.Ttr, g) / (pa.rho * g.R * pa.Ttr);
  mD[2 * i] = acc;
  mD[2 * i + 1] = acc + 1.0 / (g.Z * tau);
}

// One point relaxation over one colour of Mac^T u = t.  Row i of Mac^T couples the neighbours j through
// Mac_ji^T = -(A_f/V_j)(dG_n/dW (W_i)^T + r_f I)/2 with n out of cell i (the flux Jacobian is odd in n and r_f
// is the same from both sides).  Four lanes per cell, one per face, as in the forward macro sweep.
template <int NF>
__global__ __launch_bounds__(64) void k_adj_macro_sweep(Dev d, Bufs b, const double* rc, const double* mD,
                                                        const double* t, double* u, int64_t c0, int64_t c1) {
  constexpr int NL = NF <= 4 ? 4 : 8, SH = NF <= 4 ? 2 : 3;  // lanes per cell; lanes past NF carry zero
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = c0 + (tid >> SH);
  const int a = (int)(tid & (NL - 1));
  const bool valid = i < c1;
  double term[6] = {0, 0, 0, 0, 0, 0};
  if (valid) {
    const int32_t nb = a < NF ? d.cell_nb[NF * i + a] : kNoFace;
    if (nb >= 0) {
      const double* geo = d.cell_geo + Lay<NF>::CG * i;
      const double* s = geo + CG_FACE + CG_SLOT * a;
      const double half_av = 0.5 * s[1] * geo[0] * d.cell_geo[Lay<NF>::CG * (int64_t)nb + 1];
      double uj[6], gj[6];
      for (int m = 0; m < 6; ++m) uj[m] = u[6 * (int64_t)nb + m];
      euler_flux_vjp(b.W + 6 * i, s[2], s[3], s[4], uj, gj);
      const double r = rc[NF * i + a];
      for (int m = 0; m < 6; ++m) term[m] = half_av * (gj[m] + r * uj[m]);
    }
  }
  double tn[NL][6];
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 1; q < NL; ++q)
    for (int m = 0; m < 6; ++m) tn[q][m] = __shfl(term[m], lane + q, 64);
  if (!valid || a != 0) return;
  const double D = mD[2 * i], D5 = mD[2 * i + 1];
  for (int m = 0; m < 6; ++m) {
    double acc = t[6 * i + m] + term[m];
#pragma unroll
    for (int q = 1; q < NF; ++q) acc += tn[q][m];
    u[6 * i + m] = acc / (m == 5 ? D5 : D);
  }
}

// x_Y = s_Y - (gW, gq)
__global__ __launch_bounds__(kBlock) void k_adj_ysub(int64_t nc, int64_t off, const double* in, const double* gW,
                                                     const double* gq, double* out) {
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < 12 * nc; t += (int64_t)gridDim.x * kBlock)
    out[off + t] = in[off + t] - (t < 6 * nc ? gW[t] : gq[t - 6 * nc]);
}

}  // namespace

void launch_adj_block_precond(const Dev& d, const Bufs& b, const double* in, double* out, double* tmp, double* cell,
                              const int64_t* color_off, int64_t n_colors, int micro_pairs, int macro_pairs,
                              hipStream_t st) {
  const int64_t nc = d.nc, P = d.nc * d.nv;
  double* gW = cell;
  double* gq = gW + 6 * nc;
  double* u = gq + 6 * nc;
  double* rc = u + 6 * nc;
  double* mD = rc + (int64_t)d.mf * nc;
  const unsigned nch = (unsigned)std::min<int64_t>((d.nv + kBlock - 1) / kBlock, 64);
  const unsigned ncb = (unsigned)((nc + kBlock - 1) / kBlock);
  // z = -(D + N)^-T (s_phi + M^T s_Y)
  hipLaunchKernelGGL(k_adj_expand, dim3((unsigned)nc, nch), dim3(kBlock), 0, st, d, b, in, tmp);
  if (micro_pairs > 0)
    launch_adj_sweeps(d, b, tmp, out, color_off, n_colors, micro_pairs, st);
  else
    launch_precond(d, b, tmp, out, st);
  AdjArgs a{out, out + P, nullptr, nullptr, 0.0, -1, -1, -1, nullptr, nullptr, gW, gq, nullptr};
  if (macro_pairs > 0) {
    // t = B^T z (W part), then Mac^T u = t and x_phi = z + M_c^T u
    hipLaunchKernelGGL((k_cell_vjp<true, true>), dim3((unsigned)nc), dim3(kBlock), 0, st, d, b, a);
    if (d.mf == 4)
      hipLaunchKernelGGL(k_adj_macro_prep<4>, dim3(ncb), dim3(kBlock), 0, st, d, b, rc, mD);
    else
      hipLaunchKernelGGL(k_adj_macro_prep<kMaxFaces>, dim3(ncb), dim3(kBlock), 0, st, d, b, rc, mD);
    launch_axpby(6 * nc, 0.0, gW, 0.0, u, st);
    for (const int64_t c : sweep_sequence(color_off, n_colors, macro_pairs)) {
      const int64_t n = color_off[c + 1] - color_off[c];
      if (d.mf == 4)
        hipLaunchKernelGGL(k_adj_macro_sweep<4>, dim3((unsigned)((4 * n + 63) / 64)), dim3(64), 0, st, d, b,
                           (const double*)rc, (const double*)mD, (const double*)gW, u, color_off[c], color_off[c + 1]);
      else
        hipLaunchKernelGGL(k_adj_macro_sweep<kMaxFaces>, dim3((unsigned)((8 * n + 63) / 64)), dim3(64), 0, st, d, b,
                           (const double*)rc, (const double*)mD, (const double*)gW, u, color_off[c], color_off[c + 1]);
    }
    hipLaunchKernelGGL(k_adj_lift, dim3((unsigned)nc, nch), dim3(kBlock), 0, st, d, (const double*)u, out);
  }
  // x_Y = s_Y - B^T x_phi
  hipLaunchKernelGGL((k_cell_vjp<true, true>), dim3((unsigned)nc), dim3(kBlock), 0, st, d, b, a);
  const int64_t tail = 12 * nc;
  hipLaunchKernelGGL(k_adj_ysub, dim3((unsigned)std::min<int64_t>((tail + kBlock - 1) / kBlock, 4096)), dim3(kBlock),
                     0, st, nc, 2 * P, in, (const double*)gW, (const double*)gq, out);
}

namespace {
constexpr int kDotBlocks = 256;

// part[y][blockIdx.x] = partial of <V_y, w>
__global__ __launch_bounds__(kBlock) void k_dots(const double* V, int64_t n, const double* w, double* part) {
  __shared__ double red[(kBlock / 64) * 2];
  const double* vy = V + (int64_t)blockIdx.y * n;
  Acc<1, false, kBlock> acc;
  acc.zero();
  for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < n; x += (int64_t)gridDim.x * kBlock)
    acc.add(0, vy[x] * w[x]);
  double t;
  acc.reduce(&t, red);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_sum_parts(const double* part, int np, double* out) {
  __shared__ double red[(kBlock / 64) * 2];
  Acc<1, false, kBlock> acc;
  acc.zero();
  for (int x = threadIdx.x; x < np; x += kBlock) acc.add(0, part[(int64_t)blockIdx.x * np + x]);
  double t;
  acc.reduce(&t, red);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// w -= sum_j h[j] V_j
__global__ __launch_bounds__(kBlock) void k_gemv_sub(const double* V, int64_t n, int nvec, const double* h, double* w) {
  for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < n; x += (int64_t)gridDim.x * kBlock) {
    double acc = w[x];
    for (int j = 0; j < nvec; ++j) acc -= h[j] * V[(int64_t)j * n + x];
    w[x] = acc;
  }
}

// y = a x + c y
__global__ __launch_bounds__(kBlock) void k_axpby(int64_t n, double a, const double* x, double c, double* y) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    y[i] = (c == 0.0 ? 0.0 : c * y[i]) + (a == 0.0 ? 0.0 : a * x[i]);
}

unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 8192)); }
}  // namespace

void launch_dots(const double* V, int64_t n, int nvec, const double* w, double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dots, dim3(kDotBlocks, nvec), dim3(kBlock), 0, st, V, n, w, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(nvec), dim3(kBlock), 0, st, (const double*)part, kDotBlocks, out);
}

void launch_gemv_sub(const double* V, int64_t n, int nvec, const double* h, double* w, hipStream_t st) {
  hipLaunchKernelGGL(k_gemv_sub, dim3(grid_for(n)), dim3(kBlock), 0, st, V, n, nvec, h, w);
}

void launch_axpby(int64_t n, double a, const double* x, double c, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kBlock), 0, st, n, a, x, c, y);
}

int dot_partials() { return kDotBlocks; }

}  // namespace cis
