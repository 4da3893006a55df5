// Per-node physics of the fused step, shared by the one-step and the two-step
// kernels: the constants of one replica in the compute type, the 14 normals of
// a node, and the update of one node from its pulled populations and the 3x3
// density stencil (forces, wall rule, barycentric velocity, MRT collision with
// forcing moments and noise).  Both kernels inline the same code, so a step
// computes the same numbers whichever kernel runs it.
//
// Method (arXiv:1808.05168): non-ideal force of Eq. (11), the a_* correction
// of the footnote to Eq. (13), the non-equilibrium acceleration of Eq. (12),
// U_z = 0 on the wall rows (Sec. III.A), the barycentric velocity of Eq. (10),
// relaxation of Eq. (15) in the moment basis of Table I towards m^eq(rho^S, U),
// forcing moments (first order with the factor 1 - lambda_d/2, higher ones
// Guo's, each with 1 - lambda_a/2) and the noise of Eqs. (22)-(23).
#pragma once

#include "fnlb_device.hpp"
#include "fnlb_internal.hpp"

namespace fnlb {

template <typename Real>
struct NodePhys {
  Real G, ne;
  Real lam_d, lam_e, lam_s, lam_q, lam_p;
  Real fac_d, fac_e, fac_s;
  Real sig0d, sig0[5], sig1[5];
  bool loc;
  Real shA1, shA5;  // reference shift of a deviation moving up one row (species A)

  // physics constants in the compute type; the noise amplitudes of the
  // moments 1 and 3..8 are those at the reference densities, or with local
  // noise the factors that multiply the square roots of the local densities
  __device__ __forceinline__ void load(const RepInfo& R) {
    G = (Real)R.G;
    ne = (Real)R.ne_coef;
    lam_d = (Real)R.lam[1];
    lam_e = (Real)R.lam[3];
    lam_s = (Real)R.lam[4];
    lam_q = (Real)R.lam[6];
    lam_p = (Real)R.lam[8];
    fac_d = (Real)R.fac[1];
    fac_e = (Real)R.fac[3];
    fac_s = (Real)R.fac[4];
    loc = (R.flags & FNLB_NOISE_LOC) != 0;
    const double* sgA = loc ? R.sig_base : R.sig[0];
    const double* sgB = loc ? R.sig_base : R.sig[1];
    sig0d = (Real)sgA[1];
    const int q[5] = {3, 4, 5, 6, 8};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      sig0[k] = (Real)sgA[q[k]];
      sig1[k] = (Real)sgB[q[k]];
    }
    // w_l (rho_ref^A(j) - rho_ref^A(j+1)) = -w_l rho_bar grad_c0; species B
    // has the opposite sign
    shA1 = (Real)(-R.rA_step / 9.0);
    shA5 = (Real)(-R.rA_step / 36.0);
  }
};

// The 14 standard normals of a node at time t: species A uses g_0..g_7 from
// Philox calls 0 and 1, species B g_8..g_13 from calls 2 and 3.
template <typename Real>
__device__ __forceinline__ void node_noise(uint32_t node, uint64_t t, uint32_t k0, uint32_t k1,
                                           const BmTables* bmt, Real (&gA0)[4], Real (&gA1)[4],
                                           Real (&gB0)[4], Real (&gB1)[4]) {
  node_normals(node, t, 2u, k0, k1, gB0, bmt);
  node_normals(node, t, 3u, k0, k1, gB1, bmt);
  node_normals(node, t, 0u, k0, k1, gA0, bmt);
  node_normals(node, t, 1u, k0, k1, gA1, bmt);
}

// Update of one node.  dA, dB: on entry the pulled populations of the node as
// deviations from w_l rho_ref^S of its row, on exit the post-collision values
// (before the streaming shift).  aU/aC/aD, bU/bC/bD: density deviations of
// species A and B in the rows above, at and below the node (ghost rows beyond
// the walls repeat the wall row), read at c - 1, c, c + 1.  rAj: rho_ref^A of
// the node's row; szref: the reference part of the z component of
// sum_l w_l c_l rho^A(r + c_l).
template <typename Real, typename DT>
__device__ __forceinline__ void node_update(const NodePhys<Real>& P, int flags, bool top,
                                            bool bot, double rAj, double rho0, double szref,
                                            const DT* aU, const DT* aC, const DT* aD,
                                            const DT* bU, const DT* bC, const DT* bD, int c,
                                            Real (&dA)[9], Real (&dB)[9], Real (&gA0)[4],
                                            Real (&gA1)[4], Real (&gB0)[4], Real (&gB1)[4]) {
  const Real w1 = (Real)(1.0 / 9.0), w5 = (Real)(1.0 / 36.0), w0 = (Real)(4.0 / 9.0);
  const DT dAc = aC[c], dBc = bC[c];
  const DT aWc = aC[c - 1], aEc = aC[c + 1], bWc = bC[c - 1], bEc = bC[c + 1];
  const DT aWp = aU[c - 1], aEp = aU[c + 1];
  const DT dAp = aU[c], dBp = bU[c], bWp = bU[c - 1], bEp = bU[c + 1];
  const DT dAm = aD[c], aWm = aD[c - 1], aEm = aD[c + 1];
  const DT dBm = bD[c], bWm = bD[c - 1], bEm = bD[c + 1];
  const Real rhoA = (Real)rAj + (Real)dAc;
  const Real rhoB = (Real)(rho0 - rAj) + (Real)dBc;
  const Real rho = rhoA + rhoB;
  // FP32: the hardware reciprocal (1 ulp) instead of a correctly rounded
  // division sequence
  Real inv_rho;
  if constexpr (sizeof(Real) == 4)
    inv_rho = __builtin_amdgcn_rcpf(rho);
  else
    inv_rho = (Real)1 / rho;

  // s^S = sum_l w_l c_l rho^S(r + c_l) (deviation part + reference part)
  const Real sAx = w1 * (Real)(aEc - aWc) + w5 * (Real)((aEp - aWp) + (aEm - aWm));
  const Real sBx = w1 * (Real)(bEc - bWc) + w5 * (Real)((bEp - bWp) + (bEm - bWm));
  const Real sAz = w1 * (Real)(dAp - dAm) + w5 * (Real)((aEp + aWp) - (aEm + aWm)) + (Real)szref;
  const Real sBz = w1 * (Real)(dBp - dBm) + w5 * (Real)((bEp + bWp) - (bEm + bWm)) - (Real)szref;

  // non-ideal forces (Eq. (11)); with a_* both species share
  // a_bar = (rho^A a^A_NI + rho^B a^B_NI) / rho
  const Real G = P.G;
  Real FAx, FAz, FBx, FBz;
  if (flags & FNLB_ASTAR) {
    const Real abx = -G * (rhoA * sBx + rhoB * sAx) * inv_rho;
    const Real abz = -G * (rhoA * sBz + rhoB * sAz) * inv_rho;
    FAx = rhoA * abx;
    FAz = rhoA * abz;
    FBx = rhoB * abx;
    FBz = rhoB * abz;
  } else {
    FAx = -G * rhoA * sBx;
    FAz = -G * rhoA * sBz;
    FBx = -G * rhoB * sAx;
    FBz = -G * rhoB * sAz;
  }
  // non-equilibrium forces (Eq. (12)): rho^A grad_c0/(3c) = rho grad_c0/3
  FAz += P.ne * rho;
  FBz -= P.ne * rho;

  // species momenta (Eq. (9)) from deviations (the reference carries none)
  Real jAx = (dA[1] - dA[3]) + (dA[5] - dA[6]) + (dA[8] - dA[7]);
  Real jAz = (dA[2] - dA[4]) + (dA[5] + dA[6]) - (dA[7] + dA[8]);
  Real jBx = (dB[1] - dB[3]) + (dB[5] - dB[6]) + (dB[8] - dB[7]);
  Real jBz = (dB[2] - dB[4]) + (dB[5] + dB[6]) - (dB[7] + dB[8]);

  // U_z = 0 on the wall rows: move the barycentric normal momentum from the
  // bounced-back normal population into the rest population
  if ((flags & FNLB_WALL_UZ_FIX) && (bot || top)) {
    const Real Pi = jAz + jBz + (Real)0.5 * (FAz + FBz);
    const Real delA = rhoA * inv_rho * Pi, delB = rhoB * inv_rho * Pi;
    if (bot) {
      dA[2] -= delA;
      dA[0] += delA;
      dB[2] -= delB;
      dB[0] += delB;
    } else {
      dA[4] += delA;
      dA[0] -= delA;
      dB[4] += delB;
      dB[0] -= delB;
    }
    jAz -= delA;
    jBz -= delB;
  }

  // barycentric velocity (Eq. (10))
  const Real Ux = (jAx + jBx + (Real)0.5 * (FAx + FBx)) * inv_rho;
  const Real Uz = (jAz + jBz + (Real)0.5 * (FAz + FBz)) * inv_rho;
  const Real Uxx = Ux * Ux, Uzz = Uz * Uz, Uxz = Ux * Uz;

  // noise amplitudes: at the reference densities, or with local noise the
  // base amplitudes times the square roots of the local densities, applied to
  // the normals (the amplitudes themselves stay loop-invariant)
  const Real sd = P.sig0d;
  const Real sA3 = P.sig0[0], sA4 = P.sig0[1], sA5 = P.sig0[2], sA6 = P.sig0[3], sA8 = P.sig0[4];
  const Real sB3 = P.sig1[0], sB4 = P.sig1[1], sB5 = P.sig1[2], sB6 = P.sig1[3], sB8 = P.sig1[4];
  if (P.loc) {
    const Real qa = sqrt(rhoA), qb = sqrt(rhoB), qd = sqrt(rhoA * rhoB * inv_rho);
    gA0[0] *= qd;
    gA0[1] *= qd;
    gA0[2] *= qa;
    gA0[3] *= qa;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      gA1[k] *= qa;
      gB0[k] *= qb;
    }
    gB1[0] *= qb;
    gB1[1] *= qb;
  }
  const Real xi1 = sd * gA0[0], xi2 = sd * gA0[1];
  const Real lam_d = P.lam_d, lam_e = P.lam_e, lam_s = P.lam_s, lam_q = P.lam_q, lam_p = P.lam_p;
  const Real fac_d = P.fac_d, fac_e = P.fac_e, fac_s = P.fac_s;

  // collision of one species in moment space: adds the increments
  // R_l = w_l sum_a T_al dm_a / N_a to the populations
  auto collide = [&](Real(&d)[9], Real rs, Real jx, Real jz, Real Fx, Real Fz, Real x1, Real x2,
                     Real x3, Real x4, Real x5, Real x6, Real x7, Real x8) {
    const Real s14 = (d[1] + d[2]) + (d[3] + d[4]);
    const Real s58 = (d[5] + d[6]) + (d[7] + d[8]);
    const Real m3 = -2 * d[0] + s14 + 4 * s58;
    const Real m4 = (d[1] - d[2]) + (d[3] - d[4]);
    const Real m5 = (d[5] - d[6]) + (d[7] - d[8]);
    const Real m6 = (d[3] - d[1]) + 2 * ((d[5] - d[6]) + (d[8] - d[7]));
    const Real m7 = (d[4] - d[2]) + 2 * ((d[5] + d[6]) - (d[7] + d[8]));
    const Real m8 = 2 * d[0] - 4 * s14 + 8 * s58;
    const Real UF = Ux * Fx + Uz * Fz;
    const Real dm1 = lam_d * (rs * Ux - jx) + fac_d * Fx + x1;
    const Real dm2 = lam_d * (rs * Uz - jz) + fac_d * Fz + x2;
    const Real dm3 = lam_e * (3 * rs * (Uxx + Uzz) - m3) + fac_e * 6 * UF + x3;
    const Real dm4 = lam_s * (rs * (Uxx - Uzz) - m4) + fac_s * 2 * (Ux * Fx - Uz * Fz) + x4;
    const Real dm5 = lam_s * (rs * Uxz - m5) + fac_s * (Ux * Fz + Uz * Fx) + x5;
    const Real dm6 = -lam_q * m6 + x6;
    const Real dm7 = -lam_q * m7 + x7;
    const Real dm8 = -lam_p * m8 + x8;
    // e_a = dm_a / N_a with N = (1, 1/3, 1/3, 4, 4/9, 1/9, 2/3, 2/3, 16)
    const Real e1 = 3 * dm1, e2 = 3 * dm2, e3 = (Real)0.25 * dm3, e4 = (Real)2.25 * dm4;
    const Real e5 = 9 * dm5, e6 = (Real)1.5 * dm6, e7 = (Real)1.5 * dm7;
    const Real e8 = (Real)0.0625 * dm8;
    d[0] += w0 * (2 * (e8 - e3));
    const Real a38 = e3 - 4 * e8;
    d[1] += w1 * (a38 + e1 + e4 - e6);
    d[3] += w1 * (a38 - e1 + e4 + e6);
    d[2] += w1 * (a38 + e2 - e4 - e7);
    d[4] += w1 * (a38 - e2 - e4 + e7);
    const Real b38 = 4 * e3 + 8 * e8;
    const Real p1 = e1 + 2 * e6, p2 = e2 + 2 * e7;
    d[5] += w5 * (b38 + p1 + p2 + e5);
    d[7] += w5 * (b38 - p1 - p2 + e5);
    d[6] += w5 * (b38 - p1 + p2 - e5);
    d[8] += w5 * (b38 + p1 - p2 - e5);
  };
  collide(dA, rhoA, jAx, jAz, FAx, FAz, xi1, xi2, sA3 * gA0[2], sA4 * gA0[3], sA5 * gA1[0],
          sA6 * gA1[1], sA6 * gA1[2], sA8 * gA1[3]);
  collide(dB, rhoB, jBx, jBz, FBx, FBz, -xi1, -xi2, sB3 * gB0[0], sB4 * gB0[1], sB5 * gB0[2],
          sB6 * gB0[3], sB6 * gB1[0], sB8 * gB1[1]);
}

}  // namespace fnlb
