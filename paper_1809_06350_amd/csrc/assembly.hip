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
// Four lanes per element, all elements in one launch.  Each element writes its
// 16 node-pair blocks (16 values each) and its nodal rows to element buffers
// in HBM with plain stores; a gather then sums, for every block (node), the
// contributions listed by setup in element order.  No atomics, no colouring,
// and the sums are bitwise reproducible.
//
// Element buffer layouts (doubles, e = element, a/b = local node):
//   KE[e][4a+b][16] = (A 3x3 row-major, B 3, C 3, D) of block (a, b)
//   RE[e][a][4]     = (R_m, R_p) rows of node a
//   CE[e][a][4]     = R-bar_k correction rows of node a
//   VE[e][a][12]    = cotangents of node a's staged fields (11 used)
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

// Sum over the four lanes of an element (every lane receives the same bits:
// the pairwise sums are commutative and combined in the same order).
// The quad exchanges are DPP moves (quad_perm: lane j of each quad reads lane p_j of the same
// quad), which the VALU executes in a few cycles, instead of LDS-routed permutes.
template <int QPERM>
__device__ __forceinline__ double quad_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), QPERM, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), QPERM, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double qsum4(double v) {
  v += quad_move<0xB1>(v);   // lanes 1, 0, 3, 2
  v += quad_move<0x4E>(v);   // lanes 2, 3, 0, 1
  return v;
}
// lane B of the quad, to every lane of the quad
template <int B>
__device__ __forceinline__ double qbc(double v) { return quad_move<B * 0x55>(v); }
// any lane of the wavefront (a lane number known only at run time)
__device__ __forceinline__ double qget(double v, int src_lane) { return __shfl(v, src_lane, 64); }

// sum_q c_q N_qA N_qB for the symmetric rule (N_qA = QB + QD delta_qA), S = sum_q c_q
__device__ __forceinline__ double qsum2(double ca, double cb, double S, bool same) {
  double r = QB * QB * S + QB * QD * (ca + cb);
  if (same) r += QD * QD * ca;
  return r;
}

// Per-lane (local node a = quadrature point a of the symmetric rule) and
// element quantities of one element at the generalized-alpha stages: what the
// residual, tangent, R-bar_k and adjoint terms are built from.
struct ElemQ {
  double Ga[3], ga_[3], FGa[3], F[3][3], FiT[3][3], L[3][3], gradp[3];
  double fa[2][3], Fa[2][3], HC[2], W1[2], W2[2];
  double J, Jm23, V, w, tau, trC, pbar, PaA, Xbar[3], sA[3], rka[3];
  double rho, beta, rhop, betap, pq, dpq, dvq[3];
  bool ok;
};

// Staged values of one node: X, u, v at n+alpha_f, v-dot at n+alpha_m, R-bar_k = u-dot - v at the
// stages (COR), p at n+alpha_f, p-dot at n+alpha_m -- NODE_STAGE doubles, in this order.
#define NODE_STAGE 17
template <bool COR>
__device__ __forceinline__ void stage_node(int nd, const double *__restrict__ X, const vms_ga &ga, const StateP &sp,
                                           double *out) {
  const int64_t o3 = 3 * (int64_t)nd;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double v = sp.v_n[o3 + i] + ga.af * (sp.v[o3 + i] - sp.v_n[o3 + i]);
    out[i] = X[o3 + i];
    out[3 + i] = sp.u_n[o3 + i] + ga.af * (sp.u[o3 + i] - sp.u_n[o3 + i]);
    out[6 + i] = v;
    out[9 + i] = sp.dv_n[o3 + i] + ga.am * (sp.dv[o3 + i] - sp.dv_n[o3 + i]);
    out[12 + i] = COR ? sp.du_n[o3 + i] + ga.am * (sp.du[o3 + i] - sp.du_n[o3 + i]) - v : 0.0;
  }
  out[15] = sp.p_n[nd] + ga.af * (sp.p[nd] - sp.p_n[nd]);
  out[16] = sp.dp_n[nd] + ga.am * (sp.dp[nd] - sp.dp_n[nd]);
}

// Element prologue of lane a (four lanes per element, lanes base..base+3) from the staged values
// of its node (stage_node): reference geometry, F, J, the stress scalars and the quadrature-point
// values; element sums are quad reductions over the four lanes.
template <bool HGO>
__device__ __forceinline__ void elem_prologue_staged(int e, int a, int base, bool act, const double *nodev,
                                                     const double *__restrict__ fibre, const MatP &mp,
                                                     const vms_ga &ga, int *inverted, ElemQ &q) {
  double Xa[3], ua[3], va[3], dva[3], rka[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Xa[i] = nodev[i];
    ua[i] = nodev[3 + i];
    va[i] = nodev[6 + i];
    dva[i] = nodev[9 + i];
    rka[i] = nodev[12 + i];
  }
  const double pa = nodev[15], dpa = nodev[16];

  // reference geometry: G_A are the rows of the inverse edge matrix
  double Xn[4][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Xn[0][i] = qbc<0>(Xa[i]);
    Xn[1][i] = qbc<1>(Xa[i]);
    Xn[2][i] = qbc<2>(Xa[i]);
    Xn[3][i] = qbc<3>(Xa[i]);
  }
  double e1[3], e2[3], e3[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    e1[i] = Xn[1][i] - Xn[0][i];
    e2[i] = Xn[2][i] - Xn[0][i];
    e3[i] = Xn[3][i] - Xn[0][i];
  }
  double G1[3], G2[3], G3[3];
  G1[0] = e2[1] * e3[2] - e2[2] * e3[1];
  G1[1] = e2[2] * e3[0] - e2[0] * e3[2];
  G1[2] = e2[0] * e3[1] - e2[1] * e3[0];
  G2[0] = e3[1] * e1[2] - e3[2] * e1[1];
  G2[1] = e3[2] * e1[0] - e3[0] * e1[2];
  G2[2] = e3[0] * e1[1] - e3[1] * e1[0];
  G3[0] = e1[1] * e2[2] - e1[2] * e2[1];
  G3[1] = e1[2] * e2[0] - e1[0] * e2[2];
  G3[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double det6 = dot3(e1, G1);
  const double V = det6 / 6.0;
  double Ga[3];
  const double rdet6 = 1.0 / det6;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double g1 = G1[i] * rdet6, g2 = G2[i] * rdet6, g3 = G3[i] * rdet6;
    Ga[i] = (a == 0) ? -(g1 + g2 + g3) : (a == 1) ? g1 : (a == 2) ? g2 : g3;
  }
  double h2 = 0.0;
#pragma unroll
  for (int p0 = 0; p0 < 4; ++p0)
#pragma unroll
    for (int p1 = p0 + 1; p1 < 4; ++p1) {
      const double d0 = Xn[p0][0] - Xn[p1][0], d1 = Xn[p0][1] - Xn[p1][1], d2 = Xn[p0][2] - Xn[p1][2];
      h2 = fmax(h2, d0 * d0 + d1 * d1 + d2 * d2);
    }
  const double tau = mp.cm * sqrt(h2) / (mp.cwave * mp.rho0);

  // deformation gradient F = I + sum_A u_A (x) G_A
  double F[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int I = 0; I < 3; ++I) F[i][I] = (i == I ? 1.0 : 0.0) + qsum4(ua[i] * Ga[I]);
  double cof[3][3];  // cofactors: F^-T = cof / J
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
  const bool ok = act && (J > 0.0);
  if (act && !(J > 0.0) && a == 0) atomicOr(inverted, 1);
  double FiT[3][3];
  const double rJ = 1.0 / J;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int I = 0; I < 3; ++I) FiT[i][I] = cof[i][I] * rJ;

  // spatial gradient g_a = F^-T G_a, F G_a, grad v, grad p
  double ga_[3], FGa[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ga_[i] = FiT[i][0] * Ga[0] + FiT[i][1] * Ga[1] + FiT[i][2] * Ga[2];
    FGa[i] = F[i][0] * Ga[0] + F[i][1] * Ga[1] + F[i][2] * Ga[2];
  }
  double L[3][3], gradp[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) L[i][j] = qsum4(va[i] * ga_[j]);
    gradp[i] = qsum4(pa * ga_[i]);
  }
  const double divv = L[0][0] + L[1][1] + L[2][2];
  double trC = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int I = 0; I < 3; ++I) trC += F[i][I] * F[i][I];
  const double cJ = cbrt(J);
  const double Jm23 = 1.0 / (cJ * cJ);

  // fibre families (HGO): H = kd I + (1 - 3 kd) a (x) a
  double fa[2][3] = {}, Fa[2][3] = {}, HC[2] = {}, W1[2] = {}, W2[2] = {};
  if (HGO) {
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
    }
  }

  // quadrature point a: p, p-dot, v-dot and the constitutive scalars
  const double Sp = qsum4(pa), Sdp = qsum4(dpa);
  double dvq[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) dvq[i] = QB * qsum4(dva[i]) + QD * dva[i];
  const double pq = QB * Sp + QD * pa, dpq = QB * Sdp + QD * dpa;
  double rho, beta, rhop, betap;
  rho_beta(mp, pq, rho, beta, rhop, betap);
  double rv[3], Srv[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    rv[i] = rho * dvq[i];
    Srv[i] = qsum4(rv[i]);
  }
  const double Sbp = qsum4(beta * dpq);
  const double w = V / 4.0;
  const double pbar = Sp / 4.0;
  double sA[3];  // sum_q w N_qa J rho_q v-dot_q
#pragma unroll
  for (int i = 0; i < 3; ++i) sA[i] = w * J * (QB * Srv[i] + QD * rv[i]);
  const double PaA = w * J * (QB * Sbp + QD * beta * dpq + divv);
  double Xbar[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) Xbar[i] = w * Srv[i] + V * gradp[i];

  // hand the quantities the element's terms use to the caller
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    q.Ga[i] = Ga[i]; q.ga_[i] = ga_[i]; q.FGa[i] = FGa[i]; q.gradp[i] = gradp[i];
    q.Xbar[i] = Xbar[i]; q.sA[i] = sA[i]; q.rka[i] = rka[i]; q.dvq[i] = dvq[i];
#pragma unroll
    for (int j = 0; j < 3; ++j) { q.F[i][j] = F[i][j]; q.FiT[i][j] = FiT[i][j]; q.L[i][j] = L[i][j]; }
  }
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    q.HC[f] = HC[f]; q.W1[f] = W1[f]; q.W2[f] = W2[f];
#pragma unroll
    for (int i = 0; i < 3; ++i) { q.fa[f][i] = fa[f][i]; q.Fa[f][i] = Fa[f][i]; }
  }
  q.J = J; q.Jm23 = Jm23; q.V = V; q.w = w; q.tau = tau; q.trC = trC; q.pbar = pbar; q.PaA = PaA;
  q.rho = rho; q.beta = beta; q.rhop = rhop; q.betap = betap; q.pq = pq; q.dpq = dpq; q.ok = ok;
}

// The prologue of lane a from global memory: stage node nda, then the staged prologue.
template <bool HGO, bool COR>
__device__ __forceinline__ void elem_prologue(int e, int a, int nda, int base, bool act,
                                              const double *__restrict__ X, const double *__restrict__ fibre,
                                              const MatP &mp, const vms_ga &ga, const StateP &sp, int *inverted,
                                              ElemQ &q) {
  double nodev[NODE_STAGE];
  stage_node<COR>(nda, X, ga, sp, nodev);
  elem_prologue_staged<HGO>(e, a, base, act, nodev, fibre, mp, ga, inverted, q);
}


// Four lanes per element: lane a owns local node a (and quadrature point a of
// the symmetric rule, whose point q has N_q = QB + QD delta_qA).  Element sums
// (F, grad v, grad p, quadrature sums) are quad reductions; in the pair loop
// lane a computes row a of the element matrix, fetching node b's data from
// lane b by shuffle, so no lane holds the whole element.
template <int FL, bool HGO>
__global__ void __launch_bounds__(256)
k_assemble(int ne, const double *__restrict__ X, const int32_t *__restrict__ tets,
           const double *__restrict__ fibre, MatP mp, vms_ga ga, StateP sp, double *__restrict__ KE,
           double *__restrict__ RE, double *__restrict__ CE, const double *__restrict__ lam,
           double *__restrict__ VE, const double *__restrict__ dfibre, int pmask, double *sens, int *inverted) {
  constexpr bool RES = FL & VMS_ASM_RESIDUAL;
  constexpr bool TAN = FL & VMS_ASM_TANGENT;
  constexpr bool COR = FL & VMS_ASM_RKCORR;
  constexpr bool VJP = FL & VMS_ASM_VJP;
  constexpr bool SENS = FL & VMS_ASM_SENS;
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = gt >> 2;
  const int a = gt & 3;
  const int base = (threadIdx.x & 63) & ~3;
  const bool act = k < ne;
  const int e = act ? k : ne - 1;
  const int nda = tets[4 * (int64_t)e + a];
  ElemQ q;
  elem_prologue<HGO, COR>(e, a, nda, base, act, X, fibre, mp, ga, sp, inverted, q);
  const double(&Ga)[3] = q.Ga, (&ga_)[3] = q.ga_, (&FGa)[3] = q.FGa, (&gradp)[3] = q.gradp;
  const double(&F)[3][3] = q.F, (&FiT)[3][3] = q.FiT, (&L)[3][3] = q.L;
  const double(&fa)[2][3] = q.fa, (&Fa)[2][3] = q.Fa;
  const double(&HC)[2] = q.HC, (&W1)[2] = q.W1, (&W2)[2] = q.W2;
  const double(&Xbar)[3] = q.Xbar, (&sA)[3] = q.sA, (&rka)[3] = q.rka, (&dvq)[3] = q.dvq;
  const double &J = q.J, &Jm23 = q.Jm23, &V = q.V, &w = q.w, &tau = q.tau, &trC = q.trC, &pbar = q.pbar;
  const double &PaA = q.PaA, &rho = q.rho, &beta = q.beta, &rhop = q.rhop, &betap = q.betap;
  const double &pq = q.pq, &dpq = q.dpq;
  const bool ok = q.ok;

  if (RES) {
    double Pg[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double pgi = mp.mu * Jm23 * ((F[i][0] - trC / 3.0 * FiT[i][0]) * Ga[0] + (F[i][1] - trC / 3.0 * FiT[i][1]) * Ga[1] +
                                   (F[i][2] - trC / 3.0 * FiT[i][2]) * Ga[2]);
      if (HGO) {
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          const double aG = dot3(fa[f], Ga);
          const double FHG = mp.kd * FGa[i] + (1.0 - 3.0 * mp.kd) * Fa[f][i] * aG;
          pgi += W1[f] * Jm23 * (2.0 * FHG - 2.0 / 3.0 * HC[f] * ga_[i]);
        }
      }
      Pg[i] = pgi;
    }
    if (act) {
      double2 *o = reinterpret_cast<double2 *>(RE + 4 * (4 * (int64_t)e + a));
      const double r0 = sA[0] + V * Pg[0] - V * J * pbar * ga_[0];
      const double r1 = sA[1] + V * Pg[1] - V * J * pbar * ga_[1];
      const double r2 = sA[2] + V * Pg[2] - V * J * pbar * ga_[2];
      const double r3 = PaA + tau * J * dot3(ga_, Xbar);
      o[0] = ok ? make_double2(r0, r1) : make_double2(0.0, 0.0);
      o[1] = ok ? make_double2(r2, r3) : make_double2(0.0, 0.0);
    }
  }

  if (SENS) {
    // lam_e^T dR_e/dtheta, theta = (mu, kappa, k1, k2, fibre angle); lane a adds node a's rows
    const double *la = lam + 4 * (int64_t)nda;
    const bool comp = (mp.kind == VMS_NH_COMP);
    const double c2w = comp ? (mp.kappa + 4.0 * mp.mu / 3.0) : mp.mu;
    for (int kk = 0; kk < 5; ++kk) {
      double val = 0.0;
      if (pmask & (1 << kk)) {
        double dPg[3] = {0, 0, 0}, dtau = 0.0, drho = 0.0, dbeta = 0.0;   // at quadrature point a
        if (kk == 0) {
#pragma unroll
          for (int i = 0; i < 3; ++i)
            dPg[i] = Jm23 * ((F[i][0] - trC / 3.0 * FiT[i][0]) * Ga[0] + (F[i][1] - trC / 3.0 * FiT[i][1]) * Ga[1] +
                             (F[i][2] - trC / 3.0 * FiT[i][2]) * Ga[2]);
          dtau = comp ? -tau * (2.0 / 3.0) / c2w : -0.5 * tau / mp.mu;
        } else if (kk == 1) {
          if (comp) {
            dtau = -0.5 * tau / c2w;
            const double sq = sqrt(pq * pq + mp.kappa * mp.kappa);
            drho = mp.rho0 * (mp.kappa * mp.kappa / sq - sq - pq) / (mp.kappa * mp.kappa);
            dbeta = -mp.kappa / (sq * sq * sq);
          }
        } else if (HGO) {
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            const double E = Jm23 * HC[f] - 1.0;
            const double aG = dot3(fa[f], Ga);
            if (kk == 2 || kk == 3) {
              const double sc = (kk == 2) ? W1[f] / mp.k1 : W1[f] * E * E;
#pragma unroll
              for (int i = 0; i < 3; ++i) {
                const double FHG = mp.kd * FGa[i] + (1.0 - 3.0 * mp.kd) * Fa[f][i] * aG;
                dPg[i] += sc * Jm23 * (2.0 * FHG - 2.0 / 3.0 * HC[f] * ga_[i]);
              }
            } else {
              double da[3], Fda[3];
#pragma unroll
              for (int I = 0; I < 3; ++I) da[I] = dfibre[6 * (int64_t)e + 3 * f + I];
#pragma unroll
              for (int i = 0; i < 3; ++i) Fda[i] = F[i][0] * da[0] + F[i][1] * da[1] + F[i][2] * da[2];
              const double dHC = (1.0 - 3.0 * mp.kd) * 2.0 * dot3(Fa[f], Fda);
              const double dW1 = W2[f] * Jm23 * dHC;
              const double daG = dot3(da, Ga);
#pragma unroll
              for (int i = 0; i < 3; ++i) {
                const double FHG = mp.kd * FGa[i] + (1.0 - 3.0 * mp.kd) * Fa[f][i] * aG;
                const double FdHG = (1.0 - 3.0 * mp.kd) * (Fda[i] * aG + Fa[f][i] * daG);
                const double QG = Jm23 * (2.0 * FHG - 2.0 / 3.0 * HC[f] * ga_[i]);
                const double dQG = Jm23 * (2.0 * FdHG - 2.0 / 3.0 * dHC * ga_[i]);
                dPg[i] += dW1 * QG + W1[f] * dQG;
              }
            }
          }
        }
        // quadrature sums of the rho / beta derivatives
        double dr[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) dr[i] = drho * dvq[i];
        double Sdr[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) Sdr[i] = qsum4(dr[i]);
        const double Sdb = qsum4(dbeta * dpq);
        double dRp = dtau * J * dot3(ga_, Xbar) + tau * J * w * dot3(ga_, Sdr) + w * J * (QB * Sdb + QD * dbeta * dpq);
        val = la[3] * dRp;
#pragma unroll
        for (int i = 0; i < 3; ++i) val += la[i] * (V * dPg[i] + w * J * (QB * Sdr[i] + QD * dr[i]));
      }
      val = qsum4(val);
      if (ok && a == 0) sens[5 * (int64_t)e + kk] = val;
    }
  }

  if (TAN || COR || VJP) {
    const double cRa = w * J * rho, cBa = w * J * beta, cBpa = w * J * betap * dpq;
    const double SR = qsum4(cRa), SB = qsum4(cBa), SBp = qsum4(cBpa), Srho = qsum4(rho);
    double rpd[3], Srpd[3];   // rho_p v-dot at quadrature point a, and its quadrature sum
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      rpd[i] = rhop * dvq[i];
      Srpd[i] = qsum4(rpd[i]);
    }
    const double gXa = dot3(ga_, Xbar);
    double Lga[3];  // (grad v)^T g_a
#pragma unroll
    for (int j = 0; j < 3; ++j) Lga[j] = L[0][j] * ga_[0] + L[1][j] * ga_[1] + L[2][j] * ga_[2];
    const double *la = VJP ? lam + 4 * (int64_t)nda : nullptr;
    double cu[3] = {0, 0, 0}, cp = 0.0;
#pragma unroll 1
    for (int b = 0; b < 4; ++b) {
      const int src = base + b;
      double Gb[3], gb[3], FGb[3], Lgb[3], rpdb[3], rkb[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        Gb[i] = qget(Ga[i], src);
        gb[i] = qget(ga_[i], src);
        FGb[i] = qget(FGa[i], src);
        Lgb[i] = qget(Lga[i], src);
        rpdb[i] = qget(rpd[i], src);
        rkb[i] = COR ? qget(rka[i], src) : 0.0;
      }
      const double gXb = qget(gXa, src), cRb = qget(cRa, src), cBb = qget(cBa, src), cBpb = qget(cBpa, src);
      const double rhob = qget(rho, src);
      const bool same = (a == b);
      const double ab = dot3(Ga, Gb);
      const double gg = dot3(ga_, gb);
      // d(R_m)_a / du_b
      double Ku[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double m = (i == j ? ab : 0.0) - 2.0 / 3.0 * FGa[i] * gb[j] - 2.0 / 3.0 * ga_[i] * FGb[j] +
                           2.0 / 9.0 * trC * ga_[i] * gb[j] + trC / 3.0 * ga_[j] * gb[i];
          Ku[i][j] = V * mp.mu * Jm23 * m + V * J * pbar * (ga_[j] * gb[i] - ga_[i] * gb[j]) + sA[i] * gb[j];
        }
      if (HGO) {
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          const double aGa = dot3(fa[f], Ga), aGb = dot3(fa[f], Gb);
          const double GHG = mp.kd * ab + (1.0 - 3.0 * mp.kd) * aGa * aGb;
          double FHa[3], FHb[3], Qa[3], Qb[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            FHa[i] = mp.kd * FGa[i] + (1.0 - 3.0 * mp.kd) * Fa[f][i] * aGa;
            FHb[i] = mp.kd * FGb[i] + (1.0 - 3.0 * mp.kd) * Fa[f][i] * aGb;
            Qa[i] = Jm23 * (2.0 * FHa[i] - 2.0 / 3.0 * HC[f] * ga_[i]);
            Qb[i] = Jm23 * (2.0 * FHb[i] - 2.0 / 3.0 * HC[f] * gb[i]);
          }
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              const double d2E = -2.0 / 3.0 * Jm23 * gb[j] * (2.0 * FHa[i] - 2.0 / 3.0 * HC[f] * ga_[i]) +
                                 Jm23 * ((i == j ? 2.0 * GHG : 0.0) - 4.0 / 3.0 * ga_[i] * FHb[j] +
                                         2.0 / 3.0 * HC[f] * ga_[j] * gb[i]);
              Ku[i][j] += V * (W2[f] * Qa[i] * Qb[j] + W1[f] * d2E);
            }
        }
      }
      // d(R_p)_a / du_b
      double Kpu[3];
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Kpu[j] = gb[j] * PaA - J * w * Lgb[j] + tau * J * (gb[j] * gXa - ga_[j] * gXb - V * gg * gradp[j]);
      // remaining partial derivatives with respect to node b's staged fields
      const double mR = qsum2(cRa, cRb, SR, same);
      const double rN = w * (QB * Srho + QD * rhob);
      const double st = w * (QB * dot3(ga_, Srpd) + QD * dot3(ga_, rpdb));
      double dRm_dp[3], dRp_dvd[3], dRp_dv[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double rpv = w * J * (QB * QB * Srpd[i] + QB * QD * (rpd[i] + rpdb[i]) + (same ? QD * QD * rpd[i] : 0.0));
        dRm_dp[i] = rpv - J * ga_[i] * w;
        dRp_dvd[i] = tau * J * ga_[i] * rN;
        dRp_dv[i] = J * gb[i] * w;
      }
      const double dRp_dp = qsum2(cBpa, cBpb, SBp, same) + tau * J * (V * gg + st);
      const double dRp_dpd = qsum2(cBa, cBb, SB, same);
      if (TAN && act) {
        double kv[16];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) kv[3 * i + j] = (i == j ? ga.am * mR : 0.0) + ga.c3 * Ku[i][j];
#pragma unroll
        for (int i = 0; i < 3; ++i) kv[9 + i] = ga.c2 * dRm_dp[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) kv[12 + j] = ga.am * dRp_dvd[j] + ga.c2 * dRp_dv[j] + ga.c3 * Kpu[j];
        kv[15] = ga.am * dRp_dpd + ga.c2 * dRp_dp;
        double2 *o = reinterpret_cast<double2 *>(KE + 16 * (16 * (int64_t)e + 4 * a + b));
#pragma unroll
        for (int q = 0; q < 8; ++q) o[q] = ok ? make_double2(kv[2 * q], kv[2 * q + 1]) : make_double2(0.0, 0.0);
      }
      if (COR) {
#pragma unroll
        for (int i = 0; i < 3; ++i) cu[i] += Ku[i][0] * rkb[0] + Ku[i][1] * rkb[1] + Ku[i][2] * rkb[2];
        cp += Kpu[0] * rkb[0] + Kpu[1] * rkb[1] + Kpu[2] * rkb[2];
      }
      if (VJP) {
        // lam_a^T dR_a/d(field_b), summed over the element's rows a, written by lane b
        double c[11];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          c[j] = la[0] * Ku[0][j] + la[1] * Ku[1][j] + la[2] * Ku[2][j] + la[3] * Kpu[j];
          c[4 + j] = la[3] * dRp_dv[j];
          c[7 + j] = la[j] * mR + la[3] * dRp_dvd[j];
        }
        c[3] = la[0] * dRm_dp[0] + la[1] * dRm_dp[1] + la[2] * dRm_dp[2] + la[3] * dRp_dp;
        c[10] = la[3] * dRp_dpd;
        double *o = VE + 12 * (4 * (int64_t)e + b);
#pragma unroll
        for (int q = 0; q < 11; ++q) {
          const double t = qsum4(c[q]);
          if (act && same) o[q] = ok ? t : 0.0;
        }
      }
    }
    if (COR && act) {
      const double s = ok ? ga.c2 / ga.am : 0.0;
      double2 *o = reinterpret_cast<double2 *>(CE + 4 * (4 * (int64_t)e + a));
      o[0] = make_double2(s * cu[0], s * cu[1]);
      o[1] = make_double2(s * cu[2], s * cp);
    }
  }
}

// K blocks from the element buffer: 16 lanes per block (one per value), the
// contributions summed in the order setup listed them (increasing element).
__global__ void __launch_bounds__(VMS_BLOCK)
k_gather_blocks(int64_t nnzb, const int32_t *__restrict__ ptr, const int32_t *__restrict__ src,
                const double *__restrict__ KE, double *__restrict__ KA, double *__restrict__ KB,
                double *__restrict__ KC, double *__restrict__ KD) {
  const int64_t gt = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t b = gt >> 4;
  const int v = (int)(gt & 15);
  if (b >= nnzb) return;
  const int k0 = ptr[b], k1 = ptr[b + 1];
  double s = 0.0;
  int k = k0;
  for (; k + 4 <= k1; k += 4) {   // four loads in flight, sums in list order
    const int64_t s0 = src[k], s1 = src[k + 1], s2 = src[k + 2], s3 = src[k + 3];
    const double x0 = KE[16 * s0 + v], x1 = KE[16 * s1 + v], x2 = KE[16 * s2 + v], x3 = KE[16 * s3 + v];
    s = (((s + x0) + x1) + x2) + x3;
  }
  for (; k < k1; ++k) s += KE[16 * (int64_t)src[k] + v];
  if (v < 9)
    KA[v * nnzb + b] = s;
  else if (v < 12)
    KB[(v - 9) * nnzb + b] = s;
  else if (v < 15)
    KC[(v - 12) * nnzb + b] = s;
  else
    KD[b] = s;
}

// Row-owner assembly of the tangent (with the residual and the R-bar_k term when asked): sixteen
// lanes per node i, as four element slots of four lanes.  The node's incident elements -- the
// contributions of its diagonal block, in increasing element order -- are taken four at a time;
// each slot runs its element's prologue (lane b = local node b = quadrature point b, as in
// k_assemble) and forms the element-matrix row of node i, lane b holding block (a_i, b).  The
// slots then add their blocks, in element order, into the row's accumulator in LDS, and the row's
// W = 16 slots are written once, lane v storing value v of all of them (one 128-byte line).  Every
// element is computed once per node, so its prologue runs four times, but no element matrix goes
// through HBM.  The sums run in the order of k_gather_blocks / k_gather_nodes (increasing element)
// over the same per-pair formulas, so K, R and the R-bar_k term agree with the element-buffer path
// to rounding (the two kernels' FMA contractions differ) and are bitwise reproducible run to run.
#define ROW_NODES 16
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int FL, bool HGO>
__global__ void __launch_bounds__(256)
k_assemble_rows(int n, const int32_t *__restrict__ col, const int32_t *__restrict__ diag_pos,
                const int32_t *__restrict__ src_ptr, const int32_t *__restrict__ src, int64_t nnzb,
                const double *__restrict__ X, const int32_t *__restrict__ tets, const double *__restrict__ fibre,
                MatP mp, vms_ga ga, StateP sp, double *__restrict__ KA, double *__restrict__ KB,
                double *__restrict__ KC, double *__restrict__ KD, double *__restrict__ Rout,
                double *__restrict__ Cout, const double *__restrict__ f_ext, double load, int *inverted) {
  constexpr bool RES = FL & VMS_ASM_RESIDUAL;
  constexpr bool COR = FL & VMS_ASM_RKCORR;
  constexpr int W = 16;
  __shared__ double acc[ROW_NODES][W][16];   // [node][slot][value]
  __shared__ double accv[ROW_NODES][2][4];   // residual row, R-bar_k row
  __shared__ int cols[ROW_NODES][W];         // the row's block columns
  __shared__ double stg[ROW_NODES][W][NODE_STAGE];   // their staged values
  const int g = threadIdx.x >> 4, l = threadIdx.x & 15;
  const int sub = l >> 2, a = l & 3;
  const int base = (threadIdx.x & 63) & ~3;
  // XCD-aware: each XCD takes a contiguous range of rows, so its L2 holds that range's 1-ring state
  const int node = xcd_block(blockIdx.x, gridDim.x) * ROW_NODES + g;
  const bool nact = node < n;
  const int i = nact ? node : n - 1;
  const int dp = diag_pos[i];
  const int k0 = src_ptr[dp];
  const int cnt = nact ? src_ptr[dp + 1] - k0 : 0;
#pragma unroll
  for (int s = 0; s < W; ++s) acc[g][s][l] = 0.0;
  {   // lane l stages the node of slot l (the padding slots repeat node i)
    const int nd = col[(int64_t)W * i + l];
    cols[g][l] = nd;
    double v[NODE_STAGE];
    stage_node<COR>(nd, X, ga, sp, v);
#pragma unroll
    for (int c = 0; c < NODE_STAGE; ++c) stg[g][l][c] = v[c];
  }
  if (l < 8) {
    const int c = l & 3;
    accv[g][l >> 2][c] = (RES && l < 4 && c < 3 && f_ext) ? load * f_ext[3 * (int64_t)i + c] : 0.0;
  }
  // the wavefront's four nodes run the same number of rounds (shuffles need every lane)
  int rounds = (cnt + 3) >> 2;
  rounds = max(rounds, __shfl_xor(rounds, 16, 64));
  rounds = max(rounds, __shfl_xor(rounds, 32, 64));
  wave_lds_sync();
  // the next round's incidence and node are requested before this round's arithmetic (an inactive
  // slot takes element 0, which exists whenever the wavefront has a round)
  int ent_n = 0, nda_n = 0;
  if (rounds > 0) {
    ent_n = sub < cnt ? src[k0 + sub] : 0;
    nda_n = tets[4 * (int64_t)(ent_n >> 4) + a];
  }
  for (int r = 0; r < rounds; ++r) {
    const int kk = 4 * r + sub;
    const bool act = kk < cnt;
    const int ent = ent_n, nda = nda_n;
    const int e = ent >> 4, ai = (ent >> 2) & 3;   // element and node i's local index in it
    ent_n = kk + 4 < cnt ? src[k0 + kk + 4] : 0;
    // this lane's slot in row i: the column nda among the row's sorted real blocks (every node of
    // an element of node i is a column of row i; an inactive slot reads slot 0 and is discarded)
    int slot = 0;
    for (int s = 0; s < W; ++s)
      if (cols[g][s] == nda) { slot = s; break; }
    ElemQ q;
    elem_prologue_staged<HGO>(e, a, base, act, stg[g][slot], fibre, mp, ga, inverted, q);
    nda_n = tets[4 * (int64_t)(ent_n >> 4) + a];
    const double(&ga_)[3] = q.ga_, (&gradp)[3] = q.gradp, (&L)[3][3] = q.L;
    const double &J = q.J, &Jm23 = q.Jm23, &V = q.V, &w = q.w, &tau = q.tau, &trC = q.trC, &pbar = q.pbar;
    const double &rho = q.rho, &beta = q.beta, &rhop = q.rhop, &betap = q.betap, &dpq = q.dpq;
    const bool ok = q.ok;
    const int src_row = base + ai;
    double resv[4] = {0.0, 0.0, 0.0, 0.0};
    if (RES) {   // the row of local node a, kept by lane a_i
      double Pg[3];
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        double pgi = mp.mu * Jm23 * ((q.F[ii][0] - trC / 3.0 * q.FiT[ii][0]) * q.Ga[0] +
                                     (q.F[ii][1] - trC / 3.0 * q.FiT[ii][1]) * q.Ga[1] +
                                     (q.F[ii][2] - trC / 3.0 * q.FiT[ii][2]) * q.Ga[2]);
        if (HGO) {
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            const double aG = dot3(q.fa[f], q.Ga);
            const double FHG = mp.kd * q.FGa[ii] + (1.0 - 3.0 * mp.kd) * q.Fa[f][ii] * aG;
            pgi += q.W1[f] * Jm23 * (2.0 * FHG - 2.0 / 3.0 * q.HC[f] * ga_[ii]);
          }
        }
        Pg[ii] = pgi;
      }
      resv[0] = q.sA[0] + V * Pg[0] - V * J * pbar * ga_[0];
      resv[1] = q.sA[1] + V * Pg[1] - V * J * pbar * ga_[1];
      resv[2] = q.sA[2] + V * Pg[2] - V * J * pbar * ga_[2];
      resv[3] = q.PaA + tau * J * dot3(ga_, q.Xbar);
    }
    // element sums and this lane's column quantities (node b = a), as in k_assemble
    const double cRb = q.w * J * rho, cBb = w * J * beta, cBpb = w * J * betap * dpq;
    const double SR = qsum4(cRb), SB = qsum4(cBb), SBp = qsum4(cBpb), Srho = qsum4(rho);
    double rpdb[3], Srpd[3];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) {
      rpdb[ii] = rhop * q.dvq[ii];
      Srpd[ii] = qsum4(rpdb[ii]);
    }
    const double gXb = dot3(ga_, q.Xbar);
    double Lgb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) Lgb[j] = L[0][j] * ga_[0] + L[1][j] * ga_[1] + L[2][j] * ga_[2];
    // row quantities of node a_i, from its lane
    double Ga[3], gar[3], FGa[3], rpd[3], sA[3];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) {
      Ga[ii] = qget(q.Ga[ii], src_row);
      gar[ii] = qget(ga_[ii], src_row);
      FGa[ii] = qget(q.FGa[ii], src_row);
      rpd[ii] = qget(rpdb[ii], src_row);
      sA[ii] = qget(q.sA[ii], src_row);
    }
    const double PaA = qget(q.PaA, src_row), gXa = qget(gXb, src_row);
    const double cRa = qget(cRb, src_row), cBa = qget(cBb, src_row), cBpa = qget(cBpb, src_row);
    const double(&Gb)[3] = q.Ga, (&gb)[3] = ga_, (&FGb)[3] = q.FGa;
    const bool same = (ai == a);
    const double ab = dot3(Ga, Gb);
    const double gg = dot3(gar, gb);
    double Ku[3][3];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double m = (ii == j ? ab : 0.0) - 2.0 / 3.0 * FGa[ii] * gb[j] - 2.0 / 3.0 * gar[ii] * FGb[j] +
                         2.0 / 9.0 * trC * gar[ii] * gb[j] + trC / 3.0 * gar[j] * gb[ii];
        Ku[ii][j] = V * mp.mu * Jm23 * m + V * J * pbar * (gar[j] * gb[ii] - gar[ii] * gb[j]) + sA[ii] * gb[j];
      }
    if (HGO) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const double aGa = dot3(q.fa[f], Ga), aGb = dot3(q.fa[f], Gb);
        const double GHG = mp.kd * ab + (1.0 - 3.0 * mp.kd) * aGa * aGb;
        double FHa[3], FHb[3], Qa[3], Qb[3];
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          FHa[ii] = mp.kd * FGa[ii] + (1.0 - 3.0 * mp.kd) * q.Fa[f][ii] * aGa;
          FHb[ii] = mp.kd * FGb[ii] + (1.0 - 3.0 * mp.kd) * q.Fa[f][ii] * aGb;
          Qa[ii] = Jm23 * (2.0 * FHa[ii] - 2.0 / 3.0 * q.HC[f] * gar[ii]);
          Qb[ii] = Jm23 * (2.0 * FHb[ii] - 2.0 / 3.0 * q.HC[f] * gb[ii]);
        }
#pragma unroll
        for (int ii = 0; ii < 3; ++ii)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const double d2E = -2.0 / 3.0 * Jm23 * gb[j] * (2.0 * FHa[ii] - 2.0 / 3.0 * q.HC[f] * gar[ii]) +
                               Jm23 * ((ii == j ? 2.0 * GHG : 0.0) - 4.0 / 3.0 * gar[ii] * FHb[j] +
                                       2.0 / 3.0 * q.HC[f] * gar[j] * gb[ii]);
            Ku[ii][j] += V * (q.W2[f] * Qa[ii] * Qb[j] + q.W1[f] * d2E);
          }
      }
    }
    double Kpu[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Kpu[j] = gb[j] * PaA - J * w * Lgb[j] + tau * J * (gb[j] * gXa - gar[j] * gXb - V * gg * gradp[j]);
    const double mR = qsum2(cRa, cRb, SR, same);
    const double rN = w * (QB * Srho + QD * rho);
    const double st = w * (QB * dot3(gar, Srpd) + QD * dot3(gar, rpdb));
    double dRm_dp[3], dRp_dvd[3], dRp_dv[3];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) {
      const double rpv = w * J * (QB * QB * Srpd[ii] + QB * QD * (rpd[ii] + rpdb[ii]) + (same ? QD * QD * rpd[ii] : 0.0));
      dRm_dp[ii] = rpv - J * gar[ii] * w;
      dRp_dvd[ii] = tau * J * gar[ii] * rN;
      dRp_dv[ii] = J * gb[ii] * w;
    }
    const double dRp_dp = qsum2(cBpa, cBpb, SBp, same) + tau * J * (V * gg + st);
    const double dRp_dpd = qsum2(cBa, cBb, SB, same);
    double kv[16];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
      for (int j = 0; j < 3; ++j) kv[3 * ii + j] = (ii == j ? ga.am * mR : 0.0) + ga.c3 * Ku[ii][j];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) kv[9 + ii] = ga.c2 * dRm_dp[ii];
#pragma unroll
    for (int j = 0; j < 3; ++j) kv[12 + j] = ga.am * dRp_dvd[j] + ga.c2 * dRp_dv[j] + ga.c3 * Kpu[j];
    kv[15] = ga.am * dRp_dpd + ga.c2 * dRp_dp;
    // the R-bar_k term of row a_i: sum over the columns b in order (the lanes of the slot)
    double cv[4] = {0.0, 0.0, 0.0, 0.0};
    if (COR) {
      double tu[3], tp;
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) tu[ii] = Ku[ii][0] * q.rka[0] + Ku[ii][1] * q.rka[1] + Ku[ii][2] * q.rka[2];
      tp = Kpu[0] * q.rka[0] + Kpu[1] * q.rka[1] + Kpu[2] * q.rka[2];
      double cu[3] = {0.0, 0.0, 0.0}, cp = 0.0;
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) cu[ii] = ((qbc<0>(tu[ii]) + qbc<1>(tu[ii])) + qbc<2>(tu[ii])) + qbc<3>(tu[ii]);
      cp = ((qbc<0>(tp) + qbc<1>(tp)) + qbc<2>(tp)) + qbc<3>(tp);
      const double sc = ok ? ga.c2 / ga.am : 0.0;
      cv[0] = sc * cu[0]; cv[1] = sc * cu[1]; cv[2] = sc * cu[2]; cv[3] = sc * cp;
    }
    // add the four elements' contributions in element order
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (sub == t && act) {
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[g][slot][v] += ok ? kv[v] : 0.0;
        if ((RES || COR) && a == ai) {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            if (RES) accv[g][0][c] += ok ? resv[c] : 0.0;
            if (COR) accv[g][1][c] += cv[c];
          }
        }
      }
      wave_lds_sync();
    }
  }
  if (!nact) return;
  const int64_t b0 = (int64_t)W * i;
  double *dst = l < 9 ? KA + l * nnzb : (l < 12 ? KB + (l - 9) * nnzb : (l < 15 ? KC + (l - 12) * nnzb : KD));
#pragma unroll
  for (int s = 0; s < W; ++s) dst[b0 + s] = acc[g][s][l];
  if (RES && l < 4) Rout[4 * (int64_t)i + l] = accv[g][0][l];
  if (COR && l >= 4 && l < 8) Cout[4 * (int64_t)i + (l - 4)] = accv[g][1][l - 4];
}

// Nodal rows from an element buffer E[e][a][ws]: out[i][c] (c < w) = init +
// sum over the (element, local node) incidences of node i, which are the
// contributions of its diagonal block (pairs a*4 + a).  init = load * f_ext
// on the momentum rows when f_ext is given, else 0.
__global__ void __launch_bounds__(VMS_BLOCK)
k_gather_nodes(int n, int w, const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ ptr,
               const int32_t *__restrict__ src, const double *__restrict__ E, int ws, double *__restrict__ out,
               const double *__restrict__ f_ext, double load) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gt >= (int64_t)n * w) return;
  const int i = (int)(gt / w), c = (int)(gt % w);
  const int blk = diag_pos[i];
  double s = (f_ext && c < 3) ? load * f_ext[3 * (int64_t)i + c] : 0.0;
  auto at = [&](int q) { return (4 * (int64_t)(q >> 4) + ((q & 15) >> 2)) * ws + c; };
  const int k1 = ptr[blk + 1];
  int k = ptr[blk];
  for (; k + 4 <= k1; k += 4) {   // four loads in flight, sums in list order
    const int q0 = src[k], q1 = src[k + 1], q2 = src[k + 2], q3 = src[k + 3];
    const double x0 = E[at(q0)], x1 = E[at(q1)], x2 = E[at(q2)], x3 = E[at(q3)];
    s = (((s + x0) + x1) + x2) + x3;
  }
  for (; k < k1; ++k) s += E[at(src[k])];
  out[gt] = s;
}

__global__ void k_clear_flag(int *p) {
  if (threadIdx.x == 0) *p = 0;
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

__global__ void k_predictor(int n, vms_ga ga, double t_np1, const uint8_t *dir, const double *dir_vel, int lift,
                            StateP sp, double *u, double *p, double *v, double *du, double *dp, double *dv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double r = (ga.gm - 1.0) / ga.gm;
  for (int c = 0; c < 3; ++c) {
    const int64_t o = 3 * (int64_t)i + c;
    if (dir[4 * (int64_t)i + c] && lift) {
      u[o] = sp.u_n[o];
      v[o] = sp.v_n[o];
      du[o] = r * sp.du_n[o];
      dv[o] = 0.0;
    } else if (dir[4 * (int64_t)i + c]) {
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
k_scale_blocks(int n, int64_t nnzb, int SW, const int32_t *__restrict__ col, const int32_t *__restrict__ diag_pos,
               const uint8_t *__restrict__ dir, const double *__restrict__ W, double *__restrict__ A,
               double *__restrict__ B, double *__restrict__ C, double *__restrict__ D, float *__restrict__ A32,
               float *__restrict__ B32, float *__restrict__ C32, float *__restrict__ D32) {
  const int lane = threadIdx.x & 15;
  const int row = blockIdx.x * 16 + (threadIdx.x >> 4);
  if (row >= n) return;
  const uint8_t *di = dir + 4 * (int64_t)row;
  const double *Wi = W + 4 * (int64_t)row;
  const int bd = diag_pos[row];
  for (int b = SW * row + lane; b < SW * row + SW; b += 16) {   // padding slots stay zero
    const int j = col[b];
    const uint8_t *dj = dir + 4 * (int64_t)j;
    const double *Wj = W + 4 * (int64_t)j;
    const bool same = (b == bd);
    // every value of the block is loaded before any is stored
    double va[9], vb[3], vc[3];
#pragma unroll
    for (int q = 0; q < 9; ++q) va[q] = A[q * nnzb + b];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      vb[r] = B[r * nnzb + b];
      vc[r] = C[r * nnzb + b];
    }
    double vd = D[b];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        va[3 * r + c] = (di[r] || dj[c]) ? ((same && r == c) ? 1.0 : 0.0) : va[3 * r + c] * Wi[r] * Wj[c];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      vb[r] = (di[r] || dj[3]) ? 0.0 : vb[r] * Wi[r] * Wj[3];
      vc[r] = (di[3] || dj[r]) ? 0.0 : vc[r] * Wi[3] * Wj[r];
    }
    vd = (di[3] || dj[3]) ? (same ? 1.0 : 0.0) : vd * Wi[3] * Wj[3];
#pragma unroll
    for (int q = 0; q < 9; ++q) A[q * nnzb + b] = va[q];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      B[r * nnzb + b] = vb[r];
      C[r * nnzb + b] = vc[r];
    }
    D[b] = vd;
    if (A32) {
#pragma unroll
      for (int q = 0; q < 9; ++q) A32[q * nnzb + b] = (float)va[q];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        B32[r * nnzb + b] = (float)vb[r];
        C32[r * nnzb + b] = (float)vc[r];
      }
      D32[b] = (float)vd;
    }
  }
}

__global__ void k_rhs(int n, const uint8_t *dir, const double *W, const double *R, const double *corr,
                      double *rhs) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= 4 * (int64_t)n) return;
  const double r = -R[k] + (corr ? corr[k] : 0.0);
  rhs[k] = dir[k] ? 0.0 : W[k] * r;
}

__global__ void k_update(int n, vms_ga ga, const uint8_t *dir, const double *W, const double *x, int lift, StateP sp,
                         double *u, double *p, double *v, double *du, double *dp, double *dv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o4 = 4 * (int64_t)i;
  const double gdt = ga.gm * ga.dt;
  for (int c = 0; c < 3; ++c) {
    const int64_t o = 3 * (int64_t)i + c;
    const bool d = dir[o4 + c] != 0;
    if (d && !lift) continue;
    const double ddv = d ? 0.0 : (W ? W[o4 + c] * x[o4 + c] : x[o4 + c]);
    const double rk = (sp.du_n[o] + ga.am * (du[o] - sp.du_n[o])) - (sp.v_n[o] + ga.af * (v[o] - sp.v_n[o]));
    const double ddu = ga.c2 / ga.am * ddv - rk / ga.am;
    dv[o] += ddv;
    v[o] += gdt * ddv;
    du[o] += ddu;
    u[o] += gdt * ddu;
  }
  if (!dir[o4 + 3]) {
    const double ddp = W ? W[o4 + 3] * x[o4 + 3] : x[o4 + 3];
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
  if (!m || m->n_nodes <= 0 || m->n_tets < 0 || m->n_tets > VMS_MAX_TETS || m->nnzb <= 0 || !m->X ||
      (m->n_tets > 0 && !m->tets) ||
      !m->dir_mask || m->slot_width < 16 || (m->slot_width & 15) || m->nnzb != (int64_t)m->slot_width * m->n_nodes ||
      !m->col || !m->tpos || !m->diag_pos || !m->blk_src_ptr || !m->shat_col || m->shat_width < 64 || (m->shat_width & 63) ||
      m->shat_width > VMS_MAX_SHAT_ROW ||
      (m->n_tets > 0 && !m->blk_src))
    return vms_set_error(ctx, VMS_ERR_ARG, "incomplete mesh description");
  return VMS_OK;
}

// The tangent (with the residual and the R-bar_k term) goes by row owners, straight into K, R and
// corr, when every block row has sixteen slots and no VJP or sensitivity is asked.
static bool asm_by_rows(const vms_mesh *mesh, unsigned flags) {
  return (flags & VMS_ASM_TANGENT) && !(flags & (VMS_ASM_VJP | VMS_ASM_SENS)) && mesh->slot_width == 16;
}

size_t vms_asm_scratch_bytes(const vms_mesh *mesh, unsigned flags) {
  if (asm_by_rows(mesh, flags)) return 4 * 256;
  size_t per = 0;   // doubles per element
  if (flags & VMS_ASM_TANGENT) per += 256;
  if (flags & VMS_ASM_RESIDUAL) per += 16;
  if (flags & VMS_ASM_RKCORR) per += 16;
  if (flags & VMS_ASM_VJP) per += 48;
  return per * sizeof(double) * (size_t)(mesh->n_tets > 0 ? mesh->n_tets : 0) + 4 * 256;
}

int vms_launch_assemble(vms_ctx *ctx, const vms_mesh *mesh, const vms_material *mat, const vms_ga &ga,
                        const vms_state *st, const double *f_ext, vms_matrix *K, double *R, double *corr,
                        unsigned flags, void *scratch, size_t scratch_bytes, const double *lam, double *vjp,
                        const double *dfibre, int pmask, double *sens) {
  const int n = mesh->n_nodes, m = mesh->n_tets;
  const int64_t nnzb = mesh->nnzb;
  MatP mp{mat->kind, mat->rho0, mat->mu, mat->kappa, mat->k1, mat->k2, mat->kd, mat->c_m, 0.0};
  mp.cwave = (mat->kind == VMS_NH_COMP) ? sqrt((mat->kappa + 4.0 * mat->mu / 3.0) / mat->rho0)
                                        : sqrt(mat->mu / mat->rho0);
  if (mat->kind == VMS_HGO_INCOMP && !mesh->fibre)
    return vms_set_error(ctx, VMS_ERR_ARG, "HGO material needs fibre directions");
  const StateP sp = mk_state(st);
  const bool res = flags & VMS_ASM_RESIDUAL, tan = flags & VMS_ASM_TANGENT, cor = flags & VMS_ASM_RKCORR;
  const bool vj = flags & VMS_ASM_VJP, sn = flags & VMS_ASM_SENS;
  if (sn && (!lam || !sens || ((pmask & 16) && !dfibre)))
    return vms_set_error(ctx, VMS_ERR_ARG, "sensitivity needs lam, an output array (and dfibre for phi)");
  if (vj && (!lam || !vjp)) return vms_set_error(ctx, VMS_ERR_ARG, "VJP needs lam and an output array");
  if ((res || tan || cor || vj) && (!scratch || scratch_bytes < vms_asm_scratch_bytes(mesh, flags)))
    return vms_set_error(ctx, VMS_ERR_WORKSPACE, "assembly workspace too small: %zu < %zu", scratch_bytes,
                         vms_asm_scratch_bytes(mesh, flags));
  // element buffers, 256-byte aligned
  char *p = (char *)(((uintptr_t)scratch + 255) & ~(uintptr_t)255);
  auto take = [&](size_t per) {
    double *r = (double *)p;
    p += ((per * sizeof(double) * (size_t)m + 255) / 256) * 256;
    return r;
  };
  const bool hgo = (mat->kind == VMS_HGO_INCOMP);
  if (asm_by_rows(mesh, flags)) {   // nodes without elements get zero blocks and load * f_ext
    dim3 gr((unsigned)((n + ROW_NODES - 1) / ROW_NODES)), bl(256);
#define VMS_ROWS_CASE(FLV)                                                                               \
  case FLV: {                                                                                            \
    auto kern = hgo ? (k_assemble_rows<FLV, true>) : (k_assemble_rows<FLV, false>);                      \
    hipLaunchKernelGGL(kern, gr, bl, 0, ctx->stream, n, mesh->col, mesh->diag_pos, mesh->blk_src_ptr,    \
                       mesh->blk_src, nnzb, mesh->X, mesh->tets, mesh->fibre, mp, ga, sp, K->A, K->B, K->C, \
                       K->D, R, corr, f_ext, ga.load, &ctx->dstat->inverted);                            \
  } break;
    switch (flags & 7u) {
      VMS_ROWS_CASE(2)
      VMS_ROWS_CASE(3)
      VMS_ROWS_CASE(6)
      VMS_ROWS_CASE(7)
      default: return vms_set_error(ctx, VMS_ERR_ARG, "unsupported assembly flags");
    }
#undef VMS_ROWS_CASE
    VMS_LAUNCH_CHECK(ctx);
    return VMS_OK;
  }
  double *KE = tan ? take(256) : nullptr;
  double *RE = res ? take(16) : nullptr;
  double *CE = cor ? take(16) : nullptr;
  double *VE = vj ? take(48) : nullptr;
  if (m > 0) {
    dim3 gr((unsigned)((4 * (int64_t)m + 255) / 256)), bl(256);
#define VMS_ASM_CASE(FLV)                                                                                 \
  case FLV: {                                                                                             \
    auto kern = hgo ? (k_assemble<FLV, true>) : (k_assemble<FLV, false>);                                 \
    hipLaunchKernelGGL(kern, gr, bl, 0, ctx->stream, m, mesh->X, mesh->tets, mesh->fibre, mp, ga, sp, KE, \
                       RE, CE, lam, VE, dfibre, pmask, sens, &ctx->dstat->inverted);                      \
  } break;
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
      default: return vms_set_error(ctx, VMS_ERR_ARG, "unsupported assembly flags");
    }
#undef VMS_ASM_CASE
    VMS_LAUNCH_CHECK(ctx);
  }
  if (tan)
    hipLaunchKernelGGL(k_gather_blocks, dim3(grid1(16 * nnzb)), dim3(VMS_BLOCK), 0, ctx->stream, nnzb,
                       mesh->blk_src_ptr, mesh->blk_src, (const double *)KE, K->A, K->B, K->C, K->D);
  if (res)
    hipLaunchKernelGGL(k_gather_nodes, dim3(grid1(4 * (int64_t)n)), dim3(VMS_BLOCK), 0, ctx->stream, n, 4,
                       mesh->diag_pos, mesh->blk_src_ptr, mesh->blk_src, (const double *)RE, 4, R, f_ext, ga.load);
  if (cor)
    hipLaunchKernelGGL(k_gather_nodes, dim3(grid1(4 * (int64_t)n)), dim3(VMS_BLOCK), 0, ctx->stream, n, 4,
                       mesh->diag_pos, mesh->blk_src_ptr, mesh->blk_src, (const double *)CE, 4, corr,
                       (const double *)nullptr, 0.0);
  if (vj)
    hipLaunchKernelGGL(k_gather_nodes, dim3(grid1(11 * (int64_t)n)), dim3(VMS_BLOCK), 0, ctx->stream, n, 11,
                       mesh->diag_pos, mesh->blk_src_ptr, mesh->blk_src, (const double *)VE, 12, vjp,
                       (const double *)nullptr, 0.0);
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
                     mesh->slot_width, mesh->col, mesh->diag_pos, mesh->dir_mask, K->W, K->A, K->B, K->C, K->D,
                     mirror32 ? K->A32 : nullptr, mirror32 ? K->B32 : nullptr, mirror32 ? K->C32 : nullptr,
                     mirror32 ? K->D32 : nullptr);
  if (rhs)
    hipLaunchKernelGGL(k_rhs, dim3(grid1(4 * (int64_t)n)), dim3(VMS_BLOCK), 0, ctx->stream, n, mesh->dir_mask,
                       K->W, R, corr, rhs);
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}

int vms_launch_update(vms_ctx *ctx, const vms_mesh *mesh, const vms_ga &ga, vms_state *st, const double *W,
                      const double *x, int lift) {
  const int n = mesh->n_nodes;
  hipLaunchKernelGGL(k_update, dim3(grid1(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, ga, mesh->dir_mask, W, x,
                     lift ? 1 : 0, mk_state(st), st->u, st->p, st->v, st->du, st->dp, st->dv);
  VMS_LAUNCH_CHECK(ctx);
  return VMS_OK;
}

int vms_launch_predictor(vms_ctx *ctx, const vms_mesh *mesh, const vms_ga &ga, double t_np1, vms_state *st,
                         int lift) {
  const int n = mesh->n_nodes;
  if (!mesh->dir_vel) return vms_set_error(ctx, VMS_ERR_ARG, "dir_vel missing");
  hipLaunchKernelGGL(k_predictor, dim3(grid1(n)), dim3(VMS_BLOCK), 0, ctx->stream, n, ga, t_np1, mesh->dir_mask,
                     mesh->dir_vel, lift ? 1 : 0, mk_state(st), st->u, st->p, st->v, st->du, st->dp, st->dv);
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
