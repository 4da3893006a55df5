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
// Philox calls 0 and 1, species B g_8..g_11 from call 2 and g_12, g_13 from
// the words (w12, w13) of the call that steps 2s and 2s + 1 share (gB1[2] and
// gB1[3] are not used).
template <typename Real>
__device__ __forceinline__ void node_noise_words(uint32_t node, uint64_t t, uint32_t k0,
                                                 uint32_t k1, const BmTables* bmt,
                                                 uint32_t w12, uint32_t w13, Real (&gA0)[4],
                                                 Real (&gA1)[4], Real (&gB0)[4],
                                                 Real (&gB1)[4]) {
  node_normals(node, t, 2u, k0, k1, gB0, bmt);
  box_muller(w12, w13, gB1[0], gB1[1], bmt);
  gB1[2] = gB1[3] = (Real)0;
  node_normals(node, t, 0u, k0, k1, gA0, bmt);
  node_normals(node, t, 1u, k0, k1, gA1, bmt);
}

// The same, drawing the shared call itself.
template <typename Real>
__device__ __forceinline__ void node_noise(uint32_t node, uint64_t t, uint32_t k0, uint32_t k1,
                                           const BmTables* bmt, Real (&gA0)[4], Real (&gA1)[4],
                                           Real (&gB0)[4], Real (&gB1)[4]) {
  uint32_t w12, w13, o12, o13;
  shared_words(node, t, k0, k1, w12, w13, o12, o13);
  node_noise_words(node, t, k0, k1, bmt, w12, w13, gA0, gA1, gB0, gB1);
}

// ---- The sample of one node, formed by the sampling step from the values
// its collision reads.
//
// From f(t) as pulled: (delta c, delta rho), the pressure deviation and, with
// velocity sampling, (U_x, U_z), the barycentric velocity of Eq. (10) with the
// total non-ideal force (the a_* and non-equilibrium parts cancel between the
// species) and U_z = 0 on the wall rows when the wall rule is on.  The
// pressure (reading R11: P = rho/3 + (G/4) sum_l w_l |c_l|^2 [rho^A rho^B(r +
// c_l) + rho^B rho^A(r + c_l)], the ghost rows repeating the wall row) is
// split into a part that is constant along a row, G/4 (rho_ref^A s_ref^B +
// rho_ref^B s_ref^A) - P_ref, which the row pass adds in FP64, and the
// deviation formed here,
//   dp = delta rho / 3 + G/4 [rho_ref^A ds^B + rho_ref^B ds^A
//                            + d^A s_ref^B + d^B s_ref^A + d^A ds^B + d^B ds^A],
// with s^S = s_ref^S + ds^S = sum_l w_l |c_l|^2 rho^S(r + c_l) and d^S the
// density deviations: every term is of the size of the fluctuations, so the
// compute type (FP32 with FP32-deviation storage) carries its relative
// rounding, not that of the O(1) reference terms.

// the 3 x 3 density stencil of both species (deviations; W, C, E of the rows
// below, at and above the node)
template <typename DT>
struct Stencil {
  DT aC, aW, aE, aU, aUW, aUE, aD, aDW, aDE;
  DT bC, bW, bE, bU, bUW, bUE, bD, bDW, bDE;
};

template <typename DT>
__device__ __forceinline__ Stencil<DT> load_stencil(const DT* aU, const DT* aC, const DT* aD,
                                                    const DT* bU, const DT* bC, const DT* bD,
                                                    int c) {
  return Stencil<DT>{aC[c], aC[c - 1], aC[c + 1], aU[c], aU[c - 1], aU[c + 1],
                     aD[c], aD[c - 1], aD[c + 1], bC[c], bC[c - 1], bC[c + 1],
                     bU[c], bU[c - 1], bU[c + 1], bD[c], bD[c - 1], bD[c + 1]};
}

// the reference values of one row the sample needs, in the compute type
template <typename Real>
struct SampleRow {
  Real rAj, rBj, c0, sAref, sBref, G4, szref;
  bool wall;  // U_z = 0 on this row
};

// (formed in FP64 and rounded once to the compute type; the kernels read them
// from the replica's row table, which k_row_consts fills with this function)
template <typename Real>
__device__ __forceinline__ SampleRow<Real> sample_row_calc(const RepInfo& R, int j, int jU,
                                                           int jD) {
  const double rho0 = R.rho0;
  const double rAj = R.rA_mid + R.rA_step * j, rBj = rho0 - rAj;
  const double rAu = R.rA_mid + R.rA_step * jU, rAd = R.rA_mid + R.rA_step * jD;
  const double rBu = rho0 - rAu, rBd = rho0 - rAd;
  SampleRow<Real> r;
  r.rAj = (Real)rAj;
  r.rBj = (Real)rBj;
  r.c0 = (Real)(rAj * (1.0 / rho0));
  r.sAref = (Real)((1.0 / 9.0) * (2.0 * rAj + rAu + rAd) + (1.0 / 9.0) * (rAu + rAd));
  r.sBref = (Real)((1.0 / 9.0) * (2.0 * rBj + rBu + rBd) + (1.0 / 9.0) * (rBu + rBd));
  r.G4 = (Real)(0.25 * R.G);
  r.szref = (Real)(R.rA_step * (double)(jU - jD) * (1.0 / 6.0));
  r.wall = (R.flags & FNLB_WALL_UZ_FIX) && (j == 0 || j == R.Lz - 1);
  return r;
}

// Where the sample of one replica goes and the row table it reads: the
// RepInfo fields the sampling code needs, read once at the start of a launch.
// (A kernel that stores to global memory would otherwise read them again
// after its stores, and the wait for such a load also waits for every load
// issued before it, the prefetched rows included.)
template <typename Store, typename Real>
struct SampleDest {
  Store* fld;        // the replica's pairs
  double* ppart;     // the replica's pressure parts
  const Real* rowc;  // the replica's row constants
  int64_t plane;     // Lz Lx
  int Lx, Lz, nparts;
  bool wall_fix;
};
template <typename Store, typename Real>
__device__ __forceinline__ SampleDest<Store, Real> sample_dest(const RepInfo& R, void* fields,
                                                               double* ppart) {
  SampleDest<Store, Real> d;
  d.fld = (Store*)fields + R.field_off;
  d.ppart = ppart + R.ppart_off;
  d.rowc = (const Real*)R.rowc;
  d.plane = (int64_t)R.Lz * R.Lx;
  d.Lx = R.Lx;
  d.Lz = R.Lz;
  d.nparts = pressure_parts(R.Lx);
  d.wall_fix = (R.flags & FNLB_WALL_UZ_FIX) != 0;
  return d;
}

// The sample constants of row j from the replica's row table (read through
// the constant address space: the table does not change during a launch, so
// a wavefront-uniform row is read with scalar loads).
template <typename Store, typename Real>
__device__ __forceinline__ SampleRow<Real> sample_row(const SampleDest<Store, Real>& D, int j) {
  typedef const __attribute__((address_space(4))) Real ConstReal;
  ConstReal* t = (ConstReal*)(D.rowc + (size_t)kRowConsts * j);
  SampleRow<Real> r;
  r.rAj = t[0];
  r.rBj = t[1];
  r.c0 = t[2];
  r.sAref = t[3];
  r.sBref = t[4];
  r.szref = t[5];
  r.G4 = t[6];
  r.wall = D.wall_fix && (j == 0 || j == D.Lz - 1);
  return r;
}

// the part of the pressure deviation that is constant along row j (FP64)
__device__ __forceinline__ double pressure_row_ref(const RepInfo& R, int j) {
  const int Lz = R.Lz, jU = min(j + 1, Lz - 1), jD = max(j - 1, 0);
  const double rho0 = R.rho0;
  const double rAj = R.rA_mid + R.rA_step * j, rBj = rho0 - rAj;
  const double rAu = R.rA_mid + R.rA_step * jU, rAd = R.rA_mid + R.rA_step * jD;
  const double rBu = rho0 - rAu, rBd = rho0 - rAd;
  const double sAref = (1.0 / 9.0) * (2.0 * rAj + rAu + rAd) + (1.0 / 9.0) * (rAu + rAd);
  const double sBref = (1.0 / 9.0) * (2.0 * rBj + rBu + rBd) + (1.0 / 9.0) * (rBu + rBd);
  return 0.25 * R.G * (rAj * sBref + rBj * sAref) - (R.p_ref - rho0 / 3.0);
}

template <typename Real>
struct NodeSample {
  Real dc, drho, dp, ux, uz;
  bool bad;  // a density not positive, c outside (0, 1), or a pressure not finite
};

// jx, jz: total momentum of the pulled populations (before the wall rule);
// G: the coupling
template <typename Real, typename DT>
__device__ __forceinline__ NodeSample<Real> node_sample(const Stencil<DT>& s,
                                                        const SampleRow<Real>& r, Real G, Real jx,
                                                        Real jz, bool velocity) {
  const Real w1 = (Real)(1.0 / 9.0), w2 = (Real)(1.0 / 18.0), w5 = (Real)(1.0 / 36.0);
  const Real aC = (Real)s.aC, bC = (Real)s.bC;
  const Real rhoA = r.rAj + aC, rhoB = r.rBj + bC;
  const Real rho = rhoA + rhoB;
  Real inv_rho;
  if constexpr (sizeof(Real) == 4)
    inv_rho = __builtin_amdgcn_rcpf(rho);
  else
    inv_rho = (Real)1 / rho;
  NodeSample<Real> o;
  o.drho = aC + bC;
  o.dc = (aC - r.c0 * o.drho) * inv_rho;
  const Real sdA = w1 * ((Real)(s.aE + s.aW) + (Real)(s.aU + s.aD)) +
                   w2 * ((Real)(s.aUE + s.aUW) + (Real)(s.aDE + s.aDW));
  const Real sdB = w1 * ((Real)(s.bE + s.bW) + (Real)(s.bU + s.bD)) +
                   w2 * ((Real)(s.bUE + s.bUW) + (Real)(s.bDE + s.bDW));
  o.dp = o.drho * (Real)(1.0 / 3.0) +
         r.G4 * ((r.rAj * sdB + r.rBj * sdA) + (aC * r.sBref + bC * r.sAref) +
                 (aC * sdB + bC * sdA));
  o.bad = !(rhoA > (Real)0) || !(rhoB > (Real)0) || !(o.dc + r.c0 > (Real)0) ||
          !(o.dc + r.c0 < (Real)1) || !isfinite(o.dp);
  o.ux = o.uz = (Real)0;
  if (velocity) {
    // total force -G (rho^A s^B + rho^B s^A), s^S = sum_l w_l c_l rho^S(r + c_l)
    const Real sAx = w1 * (Real)(s.aE - s.aW) + w5 * (Real)((s.aUE - s.aUW) + (s.aDE - s.aDW));
    const Real sBx = w1 * (Real)(s.bE - s.bW) + w5 * (Real)((s.bUE - s.bUW) + (s.bDE - s.bDW));
    const Real sAz =
        w1 * (Real)(s.aU - s.aD) + w5 * (Real)((s.aUE + s.aUW) - (s.aDE + s.aDW)) + r.szref;
    const Real sBz =
        w1 * (Real)(s.bU - s.bD) + w5 * (Real)((s.bUE + s.bUW) - (s.bDE + s.bDW)) - r.szref;
    const Real Fx = -G * (rhoA * sBx + rhoB * sAx);
    const Real Fz = -G * (rhoA * sBz + rhoB * sAz);
    o.ux = (jx + (Real)0.5 * Fx) * inv_rho;
    o.uz = r.wall ? (Real)0 : (jz + (Real)0.5 * Fz) * inv_rho;
  }
  return o;
}

// A copy of v that the compiler cannot tie to v's other uses (an empty asm
// statement; no instruction).  The sample is formed from such copies, so it
// shares no floating-point operation with the collision, whose FP32
// contractions then stay those of the step that does not sample: a sampled
// trajectory stays bit-identical to an unsampled one.
template <typename T>
__device__ __forceinline__ T opaque(T v) {
  asm("" : "+v"(v));
  return v;
}

// The sample of a node with stencil s0 (pulled populations f, for the
// momentum), formed from opaque copies.
template <typename Real, typename DT, typename Store>
__device__ __forceinline__ NodeSample<Real> sample_of(const Stencil<DT>& s0,
                                                      const Store (&f)[18],
                                                      const SampleRow<Real>& r, Real G,
                                                      bool velocity) {
  Stencil<DT> st = s0;
  st = Stencil<DT>{opaque(st.aC), opaque(st.aW), opaque(st.aE), opaque(st.aU), opaque(st.aUW),
                   opaque(st.aUE), opaque(st.aD), opaque(st.aDW), opaque(st.aDE),
                   opaque(st.bC), opaque(st.bW), opaque(st.bE), opaque(st.bU), opaque(st.bUW),
                   opaque(st.bUE), opaque(st.bD), opaque(st.bDW), opaque(st.bDE)};
  Real jx = (Real)0, jz = (Real)0;
  if (velocity) {
    Real d[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) d[l] = opaque((Real)f[l]) + opaque((Real)f[9 + l]);
    jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    jz = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
  }
  return node_sample<Real, DT>(st, r, opaque(G), jx, jz, velocity);
}

// Stores a node's sample at node n = j Lx + x: the pairs (delta c, delta rho)
// [, (U_x, U_z)] in the storage type ([1 or 2][Lz][Lx][2]).
template <typename Store, typename Real>
__device__ __forceinline__ void store_sample(const SampleDest<Store, Real>& D, int32_t* watchdog,
                                             int j, int x, const NodeSample<Real>& o,
                                             bool velocity) {
  Store* fld = D.fld;
  const int64_t n = (int64_t)j * D.Lx + x, plane = D.plane;
  if constexpr (sizeof(Store) == 4) {
    *(float2*)(fld + 2 * n) = make_float2((float)o.dc, (float)o.drho);
    if (velocity) *(float2*)(fld + 2 * plane + 2 * n) = make_float2((float)o.ux, (float)o.uz);
  } else {
    *(double2*)(fld + 2 * n) = make_double2((double)o.dc, (double)o.drho);
    if (velocity) *(double2*)(fld + 2 * plane + 2 * n) = make_double2((double)o.ux, (double)o.uz);
  }
  if (o.bad) atomicOr(watchdog, 1);
}

// x from the lane the DPP pattern CTRL selects (patterns within rows of 16
// lanes, every lane of the wavefront active).
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(
      (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo));
}
__device__ __forceinline__ double readlane_as_f64(float x, int lane) {
  return (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ double readlane_as_f64(double x, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Part `part` of row j's sum of pressure deviations (columns 64 part ..
// 64 part + 63): every lane of a wavefront passes its node's deviation (0 for
// a lane past the row).  In the compute type, within each row of 16 lanes:
// pairs, then quads (lane moves by quad permutation), then the quad sums
// rotated by 4 and by 8 lanes, after which lane 0 of the row holds the row's
// sum; the four row sums are added in FP64 as (r0 + r1) + (r2 + r3) and
// stored by the first lane.  The order is fixed, so the part does not depend
// on how the lanes run.  Called by whole wavefronts with every lane active.
template <typename Store, typename Real>
__device__ __forceinline__ void store_pressure_part(const SampleDest<Store, Real>& D, int j,
                                                    int part, Real v) {
  if constexpr (sizeof(Real) == 4) {
    v += dpp_f32<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f32<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f32<0x124>(v);  // row_ror 4
    v += dpp_f32<0x128>(v);  // row_ror 8
  } else {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x124>(v);
    v += dpp_f64<0x128>(v);
  }
  const double s = (readlane_as_f64(v, 0) + readlane_as_f64(v, 16)) +
                   (readlane_as_f64(v, 32) + readlane_as_f64(v, 48));
  if ((threadIdx.x & 63) == 0) D.ppart[(int64_t)j * D.nparts + part] = s;
}

// Update of one node.  dA, dB: on entry the pulled populations of the node as
// deviations from w_l rho_ref^S of its row, on exit the post-collision values
// (before the streaming shift).  st: the 3 x 3 density deviations of species
// A and B in the rows above, at and below the node (ghost rows beyond the
// walls repeat the wall row; load_stencil).  rAj: rho_ref^A of the node's row;
// szref: the reference part of the z component of sum_l w_l c_l rho^A(r + c_l).
template <typename Real, typename DT>
__device__ __forceinline__ void node_update(const NodePhys<Real>& P, int flags, bool top,
                                            bool bot, double rAj, double rho0, double szref,
                                            const Stencil<DT>& st, Real (&dA)[9], Real (&dB)[9],
                                            Real (&gA0)[4], Real (&gA1)[4], Real (&gB0)[4],
                                            Real (&gB1)[4]) {
  const Real w1 = (Real)(1.0 / 9.0), w5 = (Real)(1.0 / 36.0), w0 = (Real)(4.0 / 9.0);
  const DT dAc = st.aC, dBc = st.bC;
  const DT aWc = st.aW, aEc = st.aE, bWc = st.bW, bEc = st.bE;
  const DT aWp = st.aUW, aEp = st.aUE;
  const DT dAp = st.aU, dBp = st.bU, bWp = st.bUW, bEp = st.bUE;
  const DT dAm = st.aD, aWm = st.aDW, aEm = st.aDE;
  const DT dBm = st.bD, bWm = st.bDW, bEm = st.bDE;
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
