// Element assembly and nodal kernels of the Newton step.
//
// Residuals R_m, R_p follow the consistent-linearization appendix written on
// the reference configuration for P1 tetrahedra (F constant per element, so
// the divergence of P~ vanishes; body force b = 0), integrated with the
// symmetric 4-point degree-2 rule.  The tangent blocks are the exact
// derivatives of these residuals along the generalized-alpha kinematics
// (eqs. defining A, B, C, D in section 3.3):
//   A = am dR_m/dv-dot + c2 dR_m/dv + c3 dR_m/du,  B = c2 dR_m/dp,
//   C = am dR_p/dv-dot + c2 dR_p/dv + c3 dR_p/du,  D = am dR_p/dp-dot + c2 dR_p/dp,
// with c2 = alpha_f gamma dt and c3 = c2^2/alpha_m.  The displacement
// derivatives are derived here in closed form (the appendix's listing of the
// C block has one term with the opposite sign to this derivative; the
// residual is taken as the definition).
//
// tau_M = c_m h_e / (c rho0) is frozen per element: h_e = longest reference
// edge, c the bulk (compressible) or shear (incompressible) wave speed.
//
// One thread per element; elements of one colour share no node, so the
// read-modify-write scatter into the block arrays is free of conflicts and the
// summation order is fixed by the colour order (bitwise reproducible).
#include <cmath>

#include "vms_internal.h"

namespace {

constexpr double QA = 0.5854101966249685;  // (5 + 3 sqrt 5)/20
constexpr double QB = 0.1381966011250105;  // (5 - sqrt 5)/20
constexpr double QD = QA - QB;

struct MatP {
  int kind;
  double rho0, mu, kappa, k1, k2, kd, cm, cwave;
};

struct StateP {
  const double *u_n, *p_n, *v_n, *du_n, *dp_n, *dv_n;
  const double *u, *p, *v, *du, *dp, *dv;
};

__device__ __forceinline__ void rho_beta(const MatP &m, double p, double &rho, double &beta,
                                         double &rho_p, double &beta_p) {
  if (m.kind == VMS_NH_COMP) {
    const double s = sqrt(p * p + m.kappa * m.kappa);
    rho = m.rho0 * (s + p) / m.kappa;
    beta = 1.0 / s;
    rho_p = rho * beta;
    beta_p = -p / (s * s * s);
  } else {
    rho = m.rho0;
    beta = 0.0;
    rho_p = 0.0;
    beta_p = 0.0;
  }
}

__device__ __forceinline__ double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// sum_q c_q N_qA N_qB for the symmetric rule (N_qA = QB + QD delta_qA)
__device__ __forceinline__ double qsum2(const double *c, double S, int A, int B) {
  double r = QB * QB * S + QB * QD * (c[A] + c[B]);
  if (A == B) r += QD * QD * c[A];
  return r;
}

template <int FL>
__global__ void __launch_bounds__(128)
k_assemble(int ne, const int32_t *__restrict__ elems, const double *__restrict__ X,
           const int32_t *__restrict__ tets, const double *__restrict__ fibre, MatP mp, vms_ga ga,
           StateP sp, int64_t nnzb, const int32_t *__restrict__ elem_blk, double *KA, double *KB,
           double *KC, double *KD, double *R, double *corr, const double *__restrict__ lam, double *vjp,
           const double *__restrict__ dfibre, int pmask, double *sens, int *inverted) {
  constexpr bool RES = FL & VMS_ASM_RESIDUAL;
  constexpr bool TAN = FL & VMS_ASM_TANGENT;
  constexpr bool COR = FL & VMS_ASM_RKCORR;
  constexpr bool VJP = FL & VMS_ASM_VJP;
  constexpr bool SENS = FL & VMS_ASM_SENS;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ne) return;
  const int e = elems[t];
  int nd[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) nd[a] = tets[4 * (int64_t)e + a];

  // staged nodal values: rates at n+alpha_m, values at n+alpha_f
  double u[4][3], v[4][3], dv[4][3], rk[4][3], p[4], dp[4], Xe[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t o = 3 * (int64_t)nd[a];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Xe[a][i] = X[o + i];
      u[a][i] = sp.u_n[o + i] + ga.af * (sp.u[o + i] - sp.u_n[o + i]);
      v[a][i] = sp.v_n[o + i] + ga.af * (sp.v[o + i] - sp.v_n[o + i]);
      dv[a][i] = sp.dv_n[o + i] + ga.am * (sp.dv[o + i] - sp.dv_n[o + i]);
      if (COR) rk[a][i] = sp.du_n[o + i] + ga.am * (sp.du[o + i] - sp.du_n[o + i]) - v[a][i];
    }
    p[a] = sp.p_n[nd[a]] + ga.af * (sp.p[nd[a]] - sp.p_n[nd[a]]);
    dp[a] = sp.dp_n[nd[a]] + ga.am * (sp.dp[nd[a]] - sp.dp_n[nd[a]]);
  }

  // reference geometry: gradients G_A are the rows of the inverse edge matrix
  double e1[3], e2[3], e3[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    e1[i] = Xe[1][i] - Xe[0][i];
    e2[i] = Xe[2][i] - Xe[0][i];
    e3[i] = Xe[3][i] - Xe[0][i];
  }
  double G[4][3];
  G[1][0] = e2[1] * e3[2] - e2[2] * e3[1];
  G[1][1] = e2[2] * e3[0] - e2[0] * e3[2];
  G[1][2] = e2[0] * e3[1] - e2[1] * e3[0];
  G[2][0] = e3[1] * e1[2] - e3[2] * e1[1];
  G[2][1] = e3[2] * e1[0] - e3[0] * e1[2];
  G[2][2] = e3[0] * e1[1] - e3[1] * e1[0];
  G[3][0] = e1[1] * e2[2] - e1[2] * e2[1];
  G[3][1] = e1[2] * e2[0] - e1[0] * e2[2];
  G[3][2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double det6 = dot3(e1, G[1]);
  const double V = det6 / 6.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    G[1][i] /= det6;
    G[2][i] /= det6;
    G[3][i] /= det6;
    G[0][i] = -(G[1][i] + G[2][i] + G[3][i]);
  }
  double h2 = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a + 1; b < 4; ++b) {
      const double d0 = Xe[a][0] - Xe[b][0], d1 = Xe[a][1] - Xe[b][1], d2 = Xe[a][2] - Xe[b][2];
      h2 = fmax(h2, d0 * d0 + d1 * d1 + d2 * d2);
    }
  const double tau = mp.cm * sqrt(h2) / (mp.cwave * mp.rho0);

  // deformation
  double F[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int I = 0; I < 3; ++I) {
      double s = (i == I) ? 1.0 : 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) s += u[a][i] * G[a][I];
      F[i][I] = s;
    }
  double cof[3][3];  // cofactor matrix: F^-1 = cof^T / J
  cof[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
  cof[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
  cof[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
  cof[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
  cof[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
  cof[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
  cof[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
  cof[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
  cof[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
  const double J = F[0][0] * cof[0][0] + F[0][1] * cof[0][1] + F[0][2] * cof[0][2];
  if (!(J > 0.0)) {
    atomicOr(inverted, 1);
    return;
  }
  double FiT[3][3];  // F^-T (i, I) = cof(i, I) / J
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int I = 0; I < 3; ++I) FiT[i][I] = cof[i][I] / J;

  // spatial gradients g_A = F^-T G_A and nodal-field gradients
  double g[4][3], FG[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      g[a][i] = FiT[i][0] * G[a][0] + FiT[i][1] * G[a][1] + FiT[i][2] * G[a][2];
      FG[a][i] = F[i][0] * G[a][0] + F[i][1] * G[a][1] + F[i][2] * G[a][2];
    }
  double L[3][3], gradp[3], divv = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gradp[i] = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) s += v[a][i] * g[a][j];
      L[i][j] = s;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) gradp[i] += p[a] * g[a][i];
    divv += L[i][i];
  }
  double trC = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int I = 0; I < 3; ++I) trC += F[i][I] * F[i][I];
  const double cJ = cbrt(J);
  const double Jm23 = 1.0 / (cJ * cJ);

  // iso first Piola stress P~ = d(rho0 G_iso)/dF
  double P[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int I = 0; I < 3; ++I) P[i][I] = mp.mu * Jm23 * (F[i][I] - trC / 3.0 * FiT[i][I]);

  // fibre families (HGO): H = kd I + (1 - 3 kd) a (x) a
  double fa[2][3], Fa[2][3], HC[2], W1[2], W2[2];
  const bool hgo = (mp.kind == VMS_HGO_INCOMP);
  if (hgo) {
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
      for (int I = 0; I < 3; ++I) fa[f][I] = fibre[6 * (int64_t)e + 3 * f + I];
#pragma unroll
      for (int i = 0; i < 3; ++i) Fa[f][i] = F[i][0] * fa[f][0] + F[i][1] * fa[f][1] + F[i][2] * fa[f][2];
      HC[f] = mp.kd * trC + (1.0 - 3.0 * mp.kd) * dot3(Fa[f], Fa[f]);
      const double E = Jm23 * HC[f] - 1.0;
      const double ee = exp(mp.k2 * E * E);
      W1[f] = mp.k1 * E * ee;
      W2[f] = mp.k1 * ee * (1.0 + 2.0 * mp.k2 * E * E);
      // P += W1 Q, Q = Jm23 (2 F H - 2/3 HC F^-T)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int I = 0; I < 3; ++I) {
          const double FH = mp.kd * F[i][I] + (1.0 - 3.0 * mp.kd) * Fa[f][i] * fa[f][I];
          P[i][I] += W1[f] * Jm23 * (2.0 * FH - 2.0 / 3.0 * HC[f] * FiT[i][I]);
        }
    }
  }

  // quadrature-point fields
  double pq[4], dpq[4], dvq[4][3], rho[4], beta[4], rhop[4], betap[4];
  const double Sp = p[0] + p[1] + p[2] + p[3];
  const double Sdp = dp[0] + dp[1] + dp[2] + dp[3];
  double Sdv[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) Sdv[i] = dv[0][i] + dv[1][i] + dv[2][i] + dv[3][i];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    pq[q] = QB * Sp + QD * p[q];
    dpq[q] = QB * Sdp + QD * dp[q];
#pragma unroll
    for (int i = 0; i < 3; ++i) dvq[q][i] = QB * Sdv[i] + QD * dv[q][i];
    rho_beta(mp, pq[q], rho[q], beta[q], rhop[q], betap[q]);
  }
  const double w = V / 4.0;
  const double pbar = Sp / 4.0;

  // per-node quadrature sums
  double sA[4][3];   // sum_q w N_qA J rho_q v-dot_q
  double PaA[4];     // sum_q w J N_qA (beta_q p-dot_q + div v)
  double rvq[4][3];  // rho_q v-dot_q
  double Srv[3] = {0, 0, 0};
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      rvq[q][i] = rho[q] * dvq[q][i];
      Srv[i] += rvq[q][i];
    }
  double Sbp = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) Sbp += beta[q] * dpq[q];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int i = 0; i < 3; ++i) sA[a][i] = w * J * (QB * Srv[i] + QD * rvq[a][i]);
    PaA[a] = w * J * (QB * Sbp + QD * beta[a] * dpq[a] + divv);
  }

  if (SENS) {
    // lam_e^T dR_e/dtheta for theta = (mu, kappa, k1, k2, fibre angle phi)
    double Xb[3], Sdr[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) Xb[i] = w * Srv[i] + V * gradp[i];
    const bool comp = (mp.kind == VMS_NH_COMP);
    const double c2w = comp ? (mp.kappa + 4.0 * mp.mu / 3.0) : mp.mu;
    for (int k = 0; k < 5; ++k) {
      double val = 0.0;
      if (pmask & (1 << k)) {
        double dP[3][3] = {}, dtau = 0.0, drho[4] = {0, 0, 0, 0}, dbeta[4] = {0, 0, 0, 0};
        if (k == 0) {           // mu: neo-Hookean stress and tau_M through the wave speed
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int I = 0; I < 3; ++I) dP[i][I] = Jm23 * (F[i][I] - trC / 3.0 * FiT[i][I]);
          dtau = comp ? -tau * (2.0 / 3.0) / c2w : -0.5 * tau / mp.mu;
        } else if (k == 1) {    // kappa: rho(p), beta(p) and tau_M
          if (comp) {
            dtau = -0.5 * tau / c2w;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const double sq = sqrt(pq[q] * pq[q] + mp.kappa * mp.kappa);
              drho[q] = mp.rho0 * (mp.kappa * mp.kappa / sq - sq - pq[q]) / (mp.kappa * mp.kappa);
              dbeta[q] = -mp.kappa / (sq * sq * sq);
            }
          }
        } else if (hgo) {       // fibre families
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            const double E = Jm23 * HC[f] - 1.0;
            if (k == 2 || k == 3) {
              const double sc = (k == 2) ? W1[f] / mp.k1 : W1[f] * E * E;
#pragma unroll
              for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int I = 0; I < 3; ++I) {
                  const double FH = mp.kd * F[i][I] + (1.0 - 3.0 * mp.kd) * Fa[f][i] * fa[f][I];
                  dP[i][I] += sc * Jm23 * (2.0 * FH - 2.0 / 3.0 * HC[f] * FiT[i][I]);
                }
            } else {            // phi: a_f -> a_f + da_f dphi
              double da[3], Fda[3];
#pragma unroll
              for (int I = 0; I < 3; ++I) da[I] = dfibre[6 * (int64_t)e + 3 * f + I];
#pragma unroll
              for (int i = 0; i < 3; ++i) Fda[i] = F[i][0] * da[0] + F[i][1] * da[1] + F[i][2] * da[2];
              const double dHC = (1.0 - 3.0 * mp.kd) * 2.0 * dot3(Fa[f], Fda);
              const double dW1 = W2[f] * Jm23 * dHC;
#pragma unroll
              for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int I = 0; I < 3; ++I) {
                  const double FH = mp.kd * F[i][I] + (1.0 - 3.0 * mp.kd) * Fa[f][i] * fa[f][I];
                  const double FdH = (1.0 - 3.0 * mp.kd) * (Fda[i] * fa[f][I] + Fa[f][i] * da[I]);
                  const double Q = Jm23 * (2.0 * FH - 2.0 / 3.0 * HC[f] * FiT[i][I]);
                  const double dQ = Jm23 * (2.0 * FdH - 2.0 / 3.0 * dHC * FiT[i][I]);
                  dP[i][I] += dW1 * Q + W1[f] * dQ;
                }
            }
          }
        }
        // assemble lam^T dR/dtheta over the element's nodes
        double Sdrv[3] = {0, 0, 0};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i = 0; i < 3; ++i) Sdrv[i] += drho[q] * dvq[q][i];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const double *la = lam + 4 * (int64_t)nd[a];
          double dRp = dtau * J * dot3(g[a], Xb) + tau * J * w * dot3(g[a], Sdrv);
#pragma unroll
          for (int q = 0; q < 4; ++q) dRp += w * J * (QB + (q == a ? QD : 0.0)) * dbeta[q] * dpq[q];
          val += la[3] * dRp;
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            double dRm = V * (dP[i][0] * G[a][0] + dP[i][1] * G[a][1] + dP[i][2] * G[a][2]);
#pragma unroll
            for (int q = 0; q < 4; ++q) dRm += w * J * (QB + (q == a ? QD : 0.0)) * drho[q] * dvq[q][i];
            val += la[i] * dRm;
          }
        }
      }
      sens[5 * (int64_t)e + k] = val;
    }
    (void)Sdr;
  }

  if (RES) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int64_t o = 4 * (int64_t)nd[a];
      double rp = PaA[a];
      double st = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i) st += g[a][i] * (w * Srv[i] + V * gradp[i]);
      rp += tau * J * st;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double pg = P[i][0] * G[a][0] + P[i][1] * G[a][1] + P[i][2] * G[a][2];
        R[o + i] += sA[a][i] + V * pg - V * J * pbar * g[a][i];
      }
      R[o + 3] += rp;
    }
  }

  if (TAN || COR || VJP) {
    // per-quadrature-point weights for the sum_q c_q N_qA N_qB forms
    double cR[4], cB[4], cBp[4];
    double SR = 0, SB = 0, SBp = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cR[q] = w * J * rho[q];
      cB[q] = w * J * beta[q];
      cBp[q] = w * J * betap[q] * dpq[q];
      SR += cR[q];
      SB += cB[q];
      SBp += cBp[q];
    }
    double Xbar[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) Xbar[i] = w * Srv[i] + V * gradp[i];
    double gX[4], cpu[4][3] = {}, cpp[4] = {};
#pragma unroll
    for (int a = 0; a < 4; ++a) gX[a] = dot3(g[a], Xbar);

#pragma unroll
    for (int a = 0; a < 4; ++a) {
      double cu[3] = {0, 0, 0}, cp = 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        // d(R_m)_A / du_B  (3x3, i row, j column)
        const double ab = dot3(G[a], G[b]);
        const double gg = dot3(g[a], g[b]);
        double Ku[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            double m = (i == j ? ab : 0.0) - 2.0 / 3.0 * FG[a][i] * g[b][j] -
                       2.0 / 3.0 * g[a][i] * FG[b][j] + 2.0 / 9.0 * trC * g[a][i] * g[b][j] +
                       trC / 3.0 * g[a][j] * g[b][i];
            Ku[i][j] = V * mp.mu * Jm23 * m + V * J * pbar * (g[a][j] * g[b][i] - g[a][i] * g[b][j]) +
                       sA[a][i] * g[b][j];
          }
        if (hgo) {
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            const double aGa = dot3(fa[f], G[a]), aGb = dot3(fa[f], G[b]);
            const double GHG = mp.kd * ab + (1.0 - 3.0 * mp.kd) * aGa * aGb;
            double FHa[3], FHb[3], Qa[3], Qb[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              FHa[i] = mp.kd * FG[a][i] + (1.0 - 3.0 * mp.kd) * Fa[f][i] * aGa;
              FHb[i] = mp.kd * FG[b][i] + (1.0 - 3.0 * mp.kd) * Fa[f][i] * aGb;
              Qa[i] = Jm23 * (2.0 * FHa[i] - 2.0 / 3.0 * HC[f] * g[a][i]);
              Qb[i] = Jm23 * (2.0 * FHb[i] - 2.0 / 3.0 * HC[f] * g[b][i]);
            }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int j = 0; j < 3; ++j) {
                const double d2E = -2.0 / 3.0 * Jm23 * g[b][j] * (2.0 * FHa[i] - 2.0 / 3.0 * HC[f] * g[a][i]) +
                                   Jm23 * ((i == j ? 2.0 * GHG : 0.0) - 4.0 / 3.0 * g[a][i] * FHb[j] +
                                           2.0 / 3.0 * HC[f] * g[a][j] * g[b][i]);
                Ku[i][j] += V * (W2[f] * Qa[i] * Qb[j] + W1[f] * d2E);
              }
          }
        }
        // d(R_p)_A / du_B (1x3)
        double Lg[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) Lg[j] = L[0][j] * g[b][0] + L[1][j] * g[b][1] + L[2][j] * g[b][2];
        double Kpu[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
          Kpu[j] = g[b][j] * PaA[a] - J * w * Lg[j] +
                   tau * J * (g[b][j] * gX[a] - g[a][j] * gX[b] - V * gg * gradp[j]);

        // remaining partial derivatives of (R_m, R_p)_A with respect to node B's staged fields
        double rpv[3] = {0, 0, 0};  // sum_q w J rho_p,q v-dot_q N_qA N_qB
        double rN = 0.0;             // sum_q w rho_q N_qB
        double st = 0.0;             // sum_q w rho_p,q N_qB (g_A . v-dot_q)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double na = QB + (q == a ? QD : 0.0), nb = QB + (q == b ? QD : 0.0);
#pragma unroll
          for (int i = 0; i < 3; ++i) rpv[i] += w * J * rhop[q] * dvq[q][i] * na * nb;
          rN += w * rho[q] * nb;
          st += w * rhop[q] * nb * dot3(g[a], dvq[q]);
        }
        const double mR = qsum2(cR, SR, a, b);           // dR_m/dv-dot = mR I
        double dRm_dp[3], dRp_dvd[3], dRp_dv[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          dRm_dp[i] = rpv[i] - J * g[a][i] * w;
          dRp_dvd[i] = tau * J * g[a][i] * rN;
          dRp_dv[i] = J * g[b][i] * w;
        }
        const double dRp_dp = qsum2(cBp, SBp, a, b) + tau * J * (V * gg + st);
        const double dRp_dpd = qsum2(cB, SB, a, b);
        if (TAN) {
          const int64_t blk = elem_blk[16 * (int64_t)e + 4 * a + b];
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
              KA[(3 * i + j) * nnzb + blk] += (i == j ? ga.am * mR : 0.0) + ga.c3 * Ku[i][j];
#pragma unroll
          for (int i = 0; i < 3; ++i) KB[i * nnzb + blk] += ga.c2 * dRm_dp[i];
#pragma unroll
          for (int j = 0; j < 3; ++j) KC[j * nnzb + blk] += ga.am * dRp_dvd[j] + ga.c2 * dRp_dv[j] + ga.c3 * Kpu[j];
          KD[blk] += ga.am * dRp_dpd + ga.c2 * dRp_dp;
        }
        if (VJP) {
          // cotangents of node B's staged fields: lam_A^T dR_A / d(field_B)
          const double *la = lam + 4 * (int64_t)nd[a];
          double *ob = vjp + 11 * (int64_t)nd[b];
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            ob[j] += la[0] * Ku[0][j] + la[1] * Ku[1][j] + la[2] * Ku[2][j] + la[3] * Kpu[j];
            ob[4 + j] += la[3] * dRp_dv[j];
            ob[7 + j] += la[j] * mR + la[3] * dRp_dvd[j];
          }
          ob[3] += la[0] * dRm_dp[0] + la[1] * dRm_dp[1] + la[2] * dRm_dp[2] + la[3] * dRp_dp;
          ob[10] += la[3] * dRp_dpd;
        }
        if (COR) {
#pragma unroll
          for (int i = 0; i < 3; ++i) cu[i] += Ku[i][0] * rk[b][0] + Ku[i][1] * rk[b][1] + Ku[i][2] * rk[b][2];
          cp += Kpu[0] * rk[b][0] + Kpu[1] * rk[b][1] + Kpu[2] * rk[b][2];
        }
      }
      if (COR) {
        const double s = ga.c2 / ga.am;
        const int64_t o = 4 * (int64_t)nd[a];
#pragma unroll
        for (int i = 0; i < 3; ++i) cpu[a][i] = s * cu[i];
        cpp[a] = s * cp;
        for (int i = 0; i < 3; ++i) corr[o + i] += cpu[a][i];
        corr[o + 3] += cpp[a];
      }
    }
  }
}

// R = load * f_ext (momentum rows), 0 (mass rows); corr = 0
__global__ void k_init_residual(int n, const double *f_ext, double load, double *R, double *corr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = 4 * (int64_t)i;
  if (R) {
    for (int c = 0; c < 3; ++c) R[o + c] = f_ext ? load * f_ext[3 * (int64_t)i + c] : 0.0;
    R[o + 3] = 0.0;
  }
  if (corr)
    for (int c = 0; c < 4; ++c) corr[o + c] = 0.0;
}

__global__ void k_clear_flag(int *p) {
  if (threadIdx.x == 0) *p = 0;
}

__global__ void k_fill(int64_t n, double *x, double v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_nodal_load(int n, const int32_t *nf_ptr, const int32_t *nf_face, const int32_t *bfaces,
                             const double *X, const double *traction, double *f_ext) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double f0 = 0, f1 = 0, f2 = 0;
  for (int k = nf_ptr[i]; k < nf_ptr[i + 1]; ++k) {
    const int64_t fc = nf_face[k];
    const int32_t a = bfaces[3 * fc], b = bfaces[3 * fc + 1], c = bfaces[3 * fc + 2];
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = X[3 * (int64_t)b + d] - X[3 * (int64_t)a + d];
      e2[d] = X[3 * (int64_t)c + d] - X[3 * (int64_t)a + d];
    }
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    const double area3 = 0.5 * sqrt(cx * cx + cy * cy + cz * cz) / 3.0;
    f0 -= traction[3 * fc] * area3;
    f1 -= traction[3 * fc + 1] * area3;
    f2 -= traction[3 * fc + 2] * area3;
  }
  f_ext[3 * (int64_t)i] = f0;
  f_ext[3 * (int64_t)i + 1] = f1;
  f_ext[3 * (int64_t)i + 2] = f2;
}

__global__ void k_predictor(int n, vms_ga ga, double t_np1, const uint8_t *dir, const double *dir_vel,
                            StateP sp, double *u, double *p, double *v, double *du, double *dp, double *dv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double r = (ga.gm - 1.0) / ga.gm;
  for (int c = 0; c < 3; ++c) {
    const int64_t o = 3 * (int64_t)i + c;
    if (dir[4 * (int64_t)i + c]) {
      u[o] = dir_vel[o] * t_np1;
      v[o] = dir_vel[o];
      du[o] = dir_vel[o];
      dv[o] = 0.0;
    } else {
      u[o] = sp.u_n[o];
      v[o] = sp.v_n[o];
      du[o] = r * sp.du_n[o];
      dv[o] = r * sp.dv_n[o];
    }
  }
  p[i] = sp.p_n[i];
  dp[i] = r * sp.dp_n[i];
}

__global__ void __launch_bounds__(VMS_BLOCK)
k_resnorm(int n, vms_ga ga, const uint8_t *dir, StateP sp, const double *R, vms_dev_status *ds) {
  __shared__ double sm[4];
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    for (int c = 0; c < 3; ++c) {
      if (dir[4 * (int64_t)i + c]) continue;
      const int64_t o = 3 * (int64_t)i + c;
      const double rk = (sp.du_n[o] + ga.am * (sp.du[o] - sp.du_n[o])) - (sp.v_n[o] + ga.af * (sp.v[o] - sp.v_n[o]));
      const double rm = R[4 * (int64_t)i + c];
      acc += rk * rk + rm * rm;
    }
    if (!dir[4 * (int64_t)i + 3]) {
      const double rp = R[4 * (int64_t)i + 3];
      acc += rp * rp;
    }
  }
  acc = block_sum(acc, sm);
  if (threadIdx.x == 0) ds->part[blockIdx.x] = acc;
}

// second pass of the norm: fixed-order sum of the per-workgroup partials
__global__ void __launch_bounds__(VMS_BLOCK) k_resnorm_finalize(int nb, vms_dev_status *ds) {
  __shared__ double sm[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) s += ds->part[k];
  s = block_sum(s, sm);
  if (threadIdx.x == 0) ds->norm2 = s;
}

// W_ii = |K_ii|^(-1/2) (>= eps) else 1; Dirichlet dofs get a unit diagonal and W = 1
__global__ void k_diagW(int n, const int32_t *diag_pos, int64_t nnzb, const double *A, const double *D,
                        const uint8_t *dir, double eps, double *W) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = diag_pos[i];
  for (int c = 0; c < 4; ++c) {
    const double d = (c < 3) ? A[(4 * c) * nnzb + b] : D[b];
    const double ad = fabs(d);
    double wv = 1.0;
    if (!dir[4 * (int64_t)i + c] && ad >= eps) wv = 1.0 / sqrt(ad);
    W[4 * (int64_t)i + c] = wv;
  }
}

// K <- W K W with Dirichlet rows/columns replaced by the identity
__global__ void __launch_bounds__(VMS_BLOCK)
k_scale_blocks(int n, int64_t nnzb, const int32_t *rp, const int32_t *col, const uint8_t *dir,
               const double *W, double *A, double *B, double *C, double *D, float *A32, float *B32,
               float *C32, float *D32) {
  const int lane = threadIdx.x & 15;
  const int row = blockIdx.x * 16 + (threadIdx.x >> 4);
  if (row >= n) return;
  const uint8_t *di = dir + 4 * (int64_t)row;
  const double *Wi = W + 4 * (int64_t)row;
  for (int b = rp[row] + lane; b < rp[row + 1]; b += 16) {
    const int j = col[b];
    const uint8_t *dj = dir + 4 * (int64_t)j;
    const double *Wj = W + 4 * (int64_t)j;
    const bool same = (j == row);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const int64_t k = (3 * r + c) * nnzb + b;
        double val = (di[r] || dj[c]) ? ((same && r == c) ? 1.0 : 0.0) : A[k] * Wi[r] * Wj[c];
        A[k] = val;
        if (A32) A32[k] = (float)val;
      }
    for (int r = 0; r < 3; ++r) {
      const int64_t k = r * nnzb + b;
      double vb = (di[r] || dj[3]) ? 0.0 : B[k] * Wi[r] * Wj[3];
      double vc = (di[3] || dj[r]) ? 0.0 : C[k] * Wi[3] * Wj[r];
      B[k] = vb;
      C[k] = vc;
      if (B32) { B32[k] = (float)vb; C32[k] = (float)vc; }
    }
    double vd = (di[3] || dj[3]) ? (same ? 1.0 : 0.0) : D[b] * Wi[3] * Wj[3];
    D[b] = vd;
    if (D32) D32[b] = (float)vd;
  }
}

__global__ void k_rhs(int n, const uint8_t *dir, const double *W, const double *R, const double *corr,
                      double *rhs) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= 4 * (int64_t)n) return;
  const double r = -R[k] + (corr ? corr[k] : 0.0);
  rhs[k] = dir[k] ? 0.0 : W[k] * r;
}

__global__ void k_update(int n, vms_ga ga, const uint8_t *dir, const double *W, const double *x, StateP sp,
                         double *u, double *p, double *v, double *du, double *dp, double *dv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o4 = 4 * (int64_t)i;
  const double gdt = ga.gm * ga.dt;
  for (int c = 0; c < 3; ++c) {
    const int64_t o = 3 * (int64_t)i + c;
    if (dir[o4 + c]) continue;
    const double ddv = W[o4 + c] * x[o4 + c];
    const double rk = (sp.du_n[o] + ga.am * (du[o] - sp.du_n[o])) - (sp.v_n[o] + ga.af * (v[o] - sp.v_n[o]));
    const double ddu = ga.c2 / ga.am * ddv - rk / ga.am;
    dv[o] += ddv;
    v[o] += gdt * ddv;
    du[o] += ddu;
    u[o] += gdt * ddu;
  }
  if (!dir[o4 + 3]) {
    const double ddp = W[o4 + 3] * x[o4 + 3];
    dp[i] += ddp;
    p[i] += gdt * ddp;
  }
}

inline StateP mk_state(const vms_state *s) {
  StateP p;
  p.u_n = s->u_n; p.p_n = s->p_n; p.v_n = s->v_n; p.du_n = s->du_n; p.dp_n = s->dp_n; p.dv_n = s->dv_n;
  p.u = s->u; p.p = s->p; p.v = s->v; p.du = s->du; p.dp = s->dp; p.dv = s->dv;
  return p;
}

inline int grid1(int64_t n, int bs = VMS_BLOCK) { return (int)((n + bs - 1) / bs); }

}  // namespace

vms_ga vms_genalpha(const vms_timeint *ti) {
  vms_ga g;
  g.am = 0.5 * (3.0 - ti->rho_inf) / (1.0 + ti->rho_inf);
  g.af = 1.0 / (1.0 + ti->rho_inf);
  g.gm = g.af;
  g.dt = ti->dt;
  g.c2 = g.af * g.gm * g.dt;
  g.c3 = g.c2 * g.c2 / g.am;
  const double t = ti->t_n + g.af * ti->dt;
  g.load = (ti->t_load > 0.0) ? fmin(t / ti->t_load, 1.0) : 1.0;
  return g;
}

int vms_check_mesh(vms_ctx *ctx, const vms_mesh *m) {
  if (!m || m->n_nodes <= 0 || m->n_tets < 0 || m->nnzb <= 0 || !m->X || !m->tets || !m->dir_mask ||
      !m->row_ptr || !m->col || !m->tpos || !m->diag_pos || !m->elem_blk || !m->elem_by_colour ||
      !m->colour_ptr || m->n_colours <= 0)
    return vms_set_error(ctx, VMS_ERR_ARG, "incomplete mesh description");
  if (m->colour_ptr[m->n_colours] != m->n_tets)
    return vms_set_error(ctx, VMS_ERR_ARG, "colour_ptr does not cover every element");
  return VMS_OK;
}

int vms_launch_assemble(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat, const vms_ga &ga,
                        const vms_state *st, const double *f_ext, vms_matrix *K, double *R, double *corr,
                        unsigned flags, const double *lam, double *vjp, const double *dfibre, int pmask,
                        double *sens) {
  const int n = mesh->n_nodes;
  const int64_t nnzb = mesh->nnzb;
  MatP mp{mat->kind, mat->rho0, mat->mu, mat->kappa, mat->k1, mat->k2, mat->kd, mat->c_m, 0.0};
  mp.cwave = (mat->kind == VMS_NH_COMP) ? sqrt((mat->kappa + 4.0 * mat->mu / 3.0) / mat->rho0)
                                        : sqrt(mat->mu / mat->rho0);
  if (mat->kind == VMS_HGO_INCOMP && !mesh->fibre)
    return vms_set_error(ctx, VMS_ERR_ARG, "HGO material needs fibre directions");
  const StateP sp = mk_state(st);
  const bool res = flags & VMS_ASM_RESIDUAL, tan = flags & VMS_ASM_TANGENT, cor = flags & VMS_ASM_RKCORR;
  if (tan) {
    hipLaunchKernelGGL(k_fill, dim3(grid1(9 * nnzb)), dim3(VMS_BLOCK), 0, ctx->stream, 9 * nnzb, K->A, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(grid1(3 * nnzb)), dim3(VMS_BLOCK), 0, ctx->stream, 3 * nnzb, K->B, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(grid1(3 * nnzb)), dim3(VMS_BLOCK), 0, ctx->stream, 3 * nnzb, K->C, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(grid1(nnzb)), dim3(VMS_BLOCK), 0, ctx->stream, nnzb, K->D, 0.0);
  }
  const bool vj = flags & VMS_ASM_VJP;
  if ((flags & VMS_ASM_SENS) && (!lam || !sens || ((pmask & 16) && !dfibre)))
    return vms_set_error(ctx, VMS_ERR_ARG, "sensitivity needs lam, an output array (and dfibre for phi)");
  if (vj) {
    if (!lam || !vjp) return vms_set_error(ctx, VMS_ERR_ARG, "VJP needs lam and an output array");
    hipLaunchKernelGGL(k_fill, dim3(grid1(11 * (int64_t)n)), dim3(VMS_BLOCK), 0, ctx->stream, 11 * (int64_t)n, vjp, 0.0);
  }
  if (res || cor)
    hipLaunchKernelGGL(k_init_residual, dim3(grid1(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, f_ext, ga.load,
                       res ? R : nullptr, cor ? corr : nullptr);
  VMS_LAUNCH_CHECK(ctx);
  for (int c = 0; c < mesh->n_colours; ++c) {
    const int c0 = mesh->colour_ptr[c], ne = mesh->colour_ptr[c + 1] - c0;
    if (ne <= 0) continue;
    const int32_t *el = mesh->elem_by_colour + c0;
    dim3 gr((ne + 127) / 128), bl(128);
#define VMS_ASM_CASE(FLV)                                                                                 \
  case FLV:                                                                                               \
    hipLaunchKernelGGL(k_assemble<FLV>, gr, bl, 0, ctx->stream, ne, el, mesh->X, mesh->tets, mesh->fibre, \
                       mp, ga, sp, nnzb, mesh->elem_blk, K ? K->A : nullptr, K ? K->B : nullptr,           \
                       K ? K->C : nullptr, K ? K->D : nullptr, R, corr, lam, vjp, dfibre, pmask, sens,    \
                       &ctx->dstat->inverted);                                                             \
    break;
    switch (flags & 31u) {
      VMS_ASM_CASE(1)
      VMS_ASM_CASE(2)
      VMS_ASM_CASE(3)
      VMS_ASM_CASE(4)
      VMS_ASM_CASE(5)
      VMS_ASM_CASE(6)
      VMS_ASM_CASE(7)
      VMS_ASM_CASE(8)
      VMS_ASM_CASE(16)
      default: return vms_set_error(ctx, VMS_ERR_ARG, "no assembly flag set");
    }
#undef VMS_ASM_CASE
  }
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}

int vms_launch_clear_inverted(vms_ctx *ctx) {
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, ctx->stream, &ctx->dstat->inverted);
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}

int vms_launch_norm(vms_ctx *ctx, const vms_mesh *mesh, const vms_ga &ga, const vms_state *st, const double *R) {
  const int n = mesh->n_nodes;
  const int nb = vms_red_blocks(n);
  hipLaunchKernelGGL(k_resnorm, dim3(nb), dim3(VMS_BLOCK), 0, ctx->stream, n, ga, mesh->dir_mask, mk_state(st),
                     R, ctx->dstat);
  hipLaunchKernelGGL(k_resnorm_finalize, dim3(1), dim3(VMS_BLOCK), 0, ctx->stream, nb, ctx->dstat);
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}

int vms_launch_prepare(vms_ctx *ctx, const vms_mesh *mesh, vms_matrix *K, const double *R, const double *corr,
                       double *rhs, double eps_diag, int mirror32) {
  const int n = mesh->n_nodes;
  const int64_t nnzb = mesh->nnzb;
  if (!K || !K->A || !K->B || !K->C || !K->D || !K->W)
    return vms_set_error(ctx, VMS_ERR_ARG, "matrix arrays missing");
  if (mirror32 && (!K->A32 || !K->B32 || !K->C32 || !K->D32))
    return vms_set_error(ctx, VMS_ERR_ARG, "FP32 mirror arrays missing");
  hipLaunchKernelGGL(k_diagW, dim3(grid1(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, mesh->diag_pos, nnzb, K->A,
                     K->D, mesh->dir_mask, eps_diag, K->W);
  hipLaunchKernelGGL(k_scale_blocks, dim3((n + 15) / 16), dim3(VMS_BLOCK), 0, ctx->stream, n, nnzb,
                     mesh->row_ptr, mesh->col, mesh->dir_mask, K->W, K->A, K->B, K->C, K->D,
                     mirror32 ? K->A32 : nullptr, mirror32 ? K->B32 : nullptr, mirror32 ? K->C32 : nullptr,
                     mirror32 ? K->D32 : nullptr);
  if (rhs)
    hipLaunchKernelGGL(k_rhs, dim3(grid1(4 * (int64_t)n)), dim3(VMS_BLOCK), 0, ctx->stream, n, mesh->dir_mask,
                       K->W, R, corr, rhs);
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}

int vms_launch_update(vms_ctx *ctx, const vms_mesh *mesh, const vms_ga &ga, vms_state *st, const double *W,
                      const double *x) {
  const int n = mesh->n_nodes;
  hipLaunchKernelGGL(k_update, dim3(grid1(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, ga, mesh->dir_mask, W, x,
                     mk_state(st), st->u, st->p, st->v, st->du, st->dp, st->dv);
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}

int vms_launch_predictor(vms_ctx *ctx, const vms_mesh *mesh, const vms_ga &ga, double t_np1, vms_state *st) {
  const int n = mesh->n_nodes;
  if (!mesh->dir_vel) return vms_set_error(ctx, VMS_ERR_ARG, "dir_vel missing");
  hipLaunchKernelGGL(k_predictor, dim3(grid1(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, ga, t_np1, mesh->dir_mask,
                     mesh->dir_vel, mk_state(st), st->u, st->p, st->v, st->du, st->dp, st->dv);
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}

extern "C" int vms_nodal_load(vms_ctx *ctx, const vms_mesh *mesh, double *f_ext) {
  if (!ctx) return VMS_ERR_ARG;
  if (!mesh || mesh->n_nodes <= 0 || !f_ext || !mesh->X || !mesh->nf_ptr ||
      (mesh->n_bfaces > 0 && (!mesh->bfaces || !mesh->traction || !mesh->nf_face)))
    return vms_set_error(ctx, VMS_ERR_ARG, "vms_nodal_load: bad arguments");
  const int n = mesh->n_nodes;
  hipLaunchKernelGGL(k_nodal_load, dim3(grid1(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, mesh->nf_ptr,
                     mesh->nf_face, mesh->bfaces, mesh->X, mesh->traction, f_ext);
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}
