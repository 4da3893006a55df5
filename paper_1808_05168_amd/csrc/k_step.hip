// Fused fluctuating two-species D2Q9 step (one HBM pass per step).
//
// Method (arXiv:1808.05168): LB update of Eq. (6) with the collision of
// Eq. (14) in the moment basis of Table I, MRT relaxation (Eq. (15)) towards
// m^eq(rho^S, U) with the barycentric velocity of Eq. (10), forcing by the
// non-ideal force of Eq. (11), the non-equilibrium acceleration of Eq. (12)
// with the a_* correction of the footnote to Eq. (13), and the thermal noise
// of Eqs. (22)-(23); walls at z = +-L/2 with mid-way bounce-back, U_z = 0 on
// the wall rows, ghost densities equal to the adjacent fluid row, periodic x
// (Sec. III.A).  The first-order forcing moments carry the factor
// (1 - lambda_d/2) and the higher ones are Guo's (each with 1 - lambda_a/2),
// the reading that makes the imposed linear profile an exact fixed point.
//
// Layout and mapping.  Populations are stored structure-of-arrays, one plane
// per (species, link), x fastest, as deviations d_l = f_l - w_l rho_ref^S(z)
// from the imposed profile rho_ref^A = rho_bar c_0(z), rho_ref^B = rho_bar
// (1 - c_0(z)).  A wavefront owns a strip of 64 consecutive columns and
// marches up a range of rows: lanes 1..62 are updated, lanes 0 and 63 only
// supply the x-neighbour densities of the force stencil, exchanged with DPP
// lane shifts; densities of the rows below and above stay in registers, so
// each population is read once per step (plus the two halo lanes and one halo
// row at each end of the row range).  Streaming is a push: post-collision
// populations go straight to their destination node of the other state copy.
// In deviation form, a population that changes row picks up the constant
// shift w_l (rho_ref(z) - rho_ref(z + c_lz)).
#include "fnlb.h"
#include "fnlb_device.hpp"
#include "fnlb_internal.hpp"

#include <type_traits>

namespace fnlb {
namespace {

// Addressing: populations are read and written with buffer instructions on
// one descriptor per replica state block; the plane offset is a scalar and
// the lane offset a 32-bit byte offset, so no per-lane 64-bit address math is
// needed.  Dword 3 of the descriptor is the gfx9-family raw-buffer format.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ Rsrc make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           kRsrcWord3);
}

template <typename Store>
__device__ __forceinline__ Store bload(Rsrc r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float bload<float>(Rsrc r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(Rsrc r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <typename Store>
__device__ __forceinline__ void bstore(Rsrc r, uint32_t voff, uint32_t soff, Store v);
template <>
__device__ __forceinline__ void bstore<float>(Rsrc r, uint32_t voff, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}
template <>
__device__ __forceinline__ void bstore<double>(Rsrc r, uint32_t voff, uint32_t soff, double v) {
  using u2 = __attribute__((ext_vector_type(2))) uint32_t;
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, 0);
}

// Rows are loaded as 18 raw values: species A links 0..8 then species B.
template <typename Store>
__device__ __forceinline__ void load_row(Rsrc r, uint32_t plane_b, uint32_t off, Store (&o)[18]) {
#pragma unroll
  for (int q = 0; q < 18; ++q) o[q] = bload<Store>(r, off, (uint32_t)q * plane_b);
}

template <typename DT, typename Store>
__device__ __forceinline__ void row_density(const Store (&o)[18], DT& da, DT& db) {
  DT a = (DT)o[0], b = (DT)o[9];
#pragma unroll
  for (int l = 1; l < 9; ++l) {
    a += (DT)o[l];
    b += (DT)o[9 + l];
  }
  da = a;
  db = b;
}

template <typename Real, typename Store, int MODE>
__global__ __launch_bounds__(kBlock) void k_step(const StepArgs a) {
  using DT = typename std::conditional<MODE == kStep, Real, double>::type;

  // XCD-aware block order: consecutive hardware blocks go to different XCDs,
  // so give each XCD a contiguous range of work items (neighbouring strips and
  // row ranges share halo data in that XCD's L2).
  const int nb = a.n_blocks;
  const int b = blockIdx.x;
  const int per_xcd = nb >> 3;
  const int blk = (b & 7) * per_xcd + (b >> 3);
  const int wave = blk * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wave >= a.n_items) return;
  const int lane = threadIdx.x & (kWave - 1);

  const Item it = a.items[wave];
  const RepInfo& R = a.reps[it.rep];
  const int Lx = R.Lx, Lz = R.Lz;
  const int64_t plane = R.plane;
  const int pitch = R.pitch;
  constexpr uint32_t SB = sizeof(Store);
  const uint32_t plane_b = (uint32_t)(plane * SB);
  const Rsrc in = make_rsrc((const char*)a.state_in + R.state_off * SB, 18u * plane_b);
  const Rsrc out = make_rsrc((char*)a.state_out + R.state_off * SB, 18u * plane_b);
  const uint32_t row_b = (uint32_t)pitch * SB;
  const int flags = R.flags;

  // columns: lane 0 = strip*62 - 1, ..., wrapped periodically
  const int xc = it.strip * kStrip + lane - 1;
  int xs = xc % Lx;
  if (xs < 0) xs += Lx;
  const bool upd = lane >= 1 && lane <= kStrip && xc < Lx;
  int xe = xs + 1;
  if (xe == Lx) xe = 0;
  int xw = xs - 1;
  if (xw < 0) xw = Lx - 1;
  const uint32_t xs_b = (uint32_t)xs * SB, xe_b = (uint32_t)xe * SB, xw_b = (uint32_t)xw * SB;

  const int64_t t = *a.t_base + a.t_off;
  const uint32_t k0 = R.seed_lo, k1 = R.seed_hi;

  // physics constants in the compute type
  const Real G = (Real)R.G;
  const Real ne = (Real)R.ne_coef;
  const Real lam_d = (Real)R.lam[1], lam_e = (Real)R.lam[3], lam_s = (Real)R.lam[4];
  const Real lam_q = (Real)R.lam[6], lam_p = (Real)R.lam[8];
  const Real fac_d = (Real)R.fac[1], fac_e = (Real)R.fac[3], fac_s = (Real)R.fac[4];
  const Real w1 = (Real)(1.0 / 9.0), w5 = (Real)(1.0 / 36.0), w0 = (Real)(4.0 / 9.0);
  const double rA0 = R.rA_mid, rAs = R.rA_step, rho0 = R.rho0;
  // shift of a deviation moving up one row, species A: w_l (rho_ref^A(j) -
  // rho_ref^A(j+1)) = -w_l rho_bar grad_c0; species B has the opposite sign.
  const Real shA1 = (Real)(-rAs / 9.0), shA5 = (Real)(-rAs / 36.0);

  const int j0 = it.j0, j1 = it.j1;

  // rolling densities (deviations) of rows j-1 (m), j (c), j+1 (p)
  DT dAm, dBm, dAc, dBc, dAp, dBp;
  Store cur[18], nxt[18];
  load_row(in, plane_b, (uint32_t)j0 * row_b + xs_b, cur);
  row_density<DT>(cur, dAc, dBc);
  if (j0 > 0) {
    Store tmp[18];
    load_row(in, plane_b, (uint32_t)(j0 - 1) * row_b + xs_b, tmp);
    row_density<DT>(tmp, dAm, dBm);
  } else {
    dAm = dAc;
    dBm = dBc;
  }

  for (int j = j0; j < j1; ++j) {
    const bool top = (j == Lz - 1), bot = (j == 0);
    if (!top) load_row(in, plane_b, (uint32_t)(j + 1) * row_b + xs_b, nxt);

    // thermal noise of this node: 14 standard normals (independent of loads)
    Real g[14];
    if constexpr (MODE != kSampleOnly) {
      uint32_t wd[16];
      node_words((uint32_t)(j * Lx + xs), (uint64_t)t, k0, k1, wd);
#pragma unroll
      for (int i = 0; i < 7; ++i) box_muller(wd[2 * i], wd[2 * i + 1], g[2 * i], g[2 * i + 1]);
    }

    if (!top) {
      row_density<DT>(nxt, dAp, dBp);
    } else {
      dAp = dAc;  // ghost row above the top wall
      dBp = dBc;
    }

    // x-neighbours of the three rows
    const DT aWm = from_left(dAm), aEm = from_right(dAm);
    const DT bWm = from_left(dBm), bEm = from_right(dBm);
    const DT aWc = from_left(dAc), aEc = from_right(dAc);
    const DT bWc = from_left(dBc), bEc = from_right(dBc);
    const DT aWp = from_left(dAp), aEp = from_right(dAp);
    const DT bWp = from_left(dBp), bEp = from_right(dBp);

    // reference densities of this row and of the rows the stencil reaches
    const double rAj = rA0 + rAs * j;
    const int jU = top ? j : j + 1, jD = bot ? j : j - 1;
    const double szref = rAs * (double)(jU - jD) * (1.0 / 6.0);  // species A

    if constexpr (MODE != kStep) {
      // observables of f(t): delta c, delta rho and the pressure
      const double rhoA = rAj + (double)dAc, rhoB = (rho0 - rAj) + (double)dBc;
      const double rho = rhoA + rhoB;
      const double drho = (double)dAc + (double)dBc;
      const double c0 = rAj / rho0;
      const double dc = ((double)dAc - c0 * drho) / rho;
      // pressure (half trace): rho/3 + (G/4) sum w|c|^2 [rhoA rhoB' + rhoB rhoA']
      const double rAu = rA0 + rAs * jU, rAd = rA0 + rAs * jD;
      const double rBu = rho0 - rAu, rBd = rho0 - rAd, rBj = rho0 - rAj;
      const double sA = (1.0 / 9.0) * ((rAj + (double)aEc) + (rAj + (double)aWc) +
                                       (rAu + (double)dAp) + (rAd + (double)dAm)) +
                        (1.0 / 18.0) * ((rAu + (double)aEp) + (rAu + (double)aWp) +
                                        (rAd + (double)aEm) + (rAd + (double)aWm));
      const double sB = (1.0 / 9.0) * ((rBj + (double)bEc) + (rBj + (double)bWc) +
                                       (rBu + (double)dBp) + (rBd + (double)dBm)) +
                        (1.0 / 18.0) * ((rBu + (double)bEp) + (rBu + (double)bWp) +
                                        (rBd + (double)bEm) + (rBd + (double)bWm));
      const double dP = drho * (1.0 / 3.0) + R.G * 0.25 * (rhoA * sB + rhoB * sA) - (R.p_ref - rho0 / 3.0);
      if (upd) {
        double* fld = a.fields + R.field_off;
        fld[(int64_t)j * Lx + xc] = dc;
        fld[(int64_t)(Lz + j) * Lx + xc] = drho;
        const bool bad = !(rhoA > 0.0) || !(rhoB > 0.0) || !(dc + c0 > 0.0) ||
                         !(dc + c0 < 1.0) || !isfinite(dP);
        if (bad) atomicOr(a.watchdog, 1);
      }
      const double tot = wave_sum(upd ? dP : 0.0);
      if (lane == 0) a.ppart[R.ppart_off + (int64_t)it.strip * Lz + j] = tot;
    }

    if constexpr (MODE != kSampleOnly) {
      Real dA[9], dB[9];
#pragma unroll
      for (int l = 0; l < 9; ++l) {
        dA[l] = (Real)cur[l];
        dB[l] = (Real)cur[9 + l];
      }
      const Real rhoA = (Real)rAj + (Real)dAc;
      const Real rhoB = (Real)(rho0 - rAj) + (Real)dBc;
      const Real rho = rhoA + rhoB;
      const Real inv_rho = (Real)1 / rho;

      // s^S = sum_l w_l c_l rho^S(r + c_l) (deviation part + reference part)
      const Real sAx = w1 * (Real)(aEc - aWc) + w5 * (Real)((aEp - aWp) + (aEm - aWm));
      const Real sBx = w1 * (Real)(bEc - bWc) + w5 * (Real)((bEp - bWp) + (bEm - bWm));
      const Real sAz = w1 * (Real)(dAp - dAm) + w5 * (Real)((aEp + aWp) - (aEm + aWm)) + (Real)szref;
      const Real sBz = w1 * (Real)(dBp - dBm) + w5 * (Real)((bEp + bWp) - (bEm + bWm)) - (Real)szref;

      // non-ideal forces (Eq. (11)); with a_* both species share
      // a_bar = (rho^A a^A_NI + rho^B a^B_NI) / rho
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
      FAz += ne * rho;
      FBz -= ne * rho;

      // species momenta (Eq. (9)) from deviations (the reference carries none)
      Real jAx = (dA[1] - dA[3]) + (dA[5] - dA[6]) + (dA[8] - dA[7]);
      Real jAz = (dA[2] - dA[4]) + (dA[5] + dA[6]) - (dA[7] + dA[8]);
      Real jBx = (dB[1] - dB[3]) + (dB[5] - dB[6]) + (dB[8] - dB[7]);
      Real jBz = (dB[2] - dB[4]) + (dB[5] + dB[6]) - (dB[7] + dB[8]);

      // U_z = 0 on the wall rows: move the barycentric normal momentum from
      // the bounced-back normal population into the rest population
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

      // noise amplitudes (reference densities, or local ones)
      Real sd = (Real)R.sig[0][1];
      Real sA3 = (Real)R.sig[0][3], sA4 = (Real)R.sig[0][4], sA6 = (Real)R.sig[0][6],
           sA8 = (Real)R.sig[0][8];
      Real sB3 = (Real)R.sig[1][3], sB4 = (Real)R.sig[1][4], sB6 = (Real)R.sig[1][6],
           sB8 = (Real)R.sig[1][8];
      Real sA5 = (Real)R.sig[0][5], sB5 = (Real)R.sig[1][5];
      if (flags & FNLB_NOISE_LOC) {
        const Real qa = sqrt(rhoA), qb = sqrt(rhoB);
        sd = (Real)R.sig_base[1] * sqrt(rhoA * rhoB * inv_rho);
        sA3 = (Real)R.sig_base[3] * qa;
        sA4 = (Real)R.sig_base[4] * qa;
        sA5 = (Real)R.sig_base[5] * qa;
        sA6 = (Real)R.sig_base[6] * qa;
        sA8 = (Real)R.sig_base[8] * qa;
        sB3 = (Real)R.sig_base[3] * qb;
        sB4 = (Real)R.sig_base[4] * qb;
        sB5 = (Real)R.sig_base[5] * qb;
        sB6 = (Real)R.sig_base[6] * qb;
        sB8 = (Real)R.sig_base[8] * qb;
      }
      const Real xi1 = sd * g[0], xi2 = sd * g[1];

      // collision of one species in moment space; returns the increments
      // R_l = w_l sum_a T_al dm_a / N_a added to the populations
      auto collide = [&](Real (&d)[9], Real rs, Real jx, Real jz, Real Fx, Real Fz, Real x1,
                         Real x2, Real x3, Real x4, Real x5, Real x6, Real x7, Real x8) {
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
      collide(dA, rhoA, jAx, jAz, FAx, FAz, xi1, xi2, sA3 * g[2], sA4 * g[3], sA5 * g[4],
              sA6 * g[5], sA6 * g[6], sA8 * g[7]);
      collide(dB, rhoB, jBx, jBz, FBx, FBz, -xi1, -xi2, sB3 * g[8], sB4 * g[9], sB5 * g[10],
              sB6 * g[11], sB6 * g[12], sB8 * g[13]);

      // streaming (push) with mid-way bounce-back
      if (upd) {
        const uint32_t rj = (uint32_t)j * row_b;
        const uint32_t ru = rj + row_b, rd = rj - row_b;
        auto emit = [&](int s, const Real (&d)[9], Real sh1, Real sh5) {
          const uint32_t o = (uint32_t)(9 * s) * plane_b;
          bstore<Store>(out, rj + xs_b, o + 0 * plane_b, (Store)d[0]);
          bstore<Store>(out, rj + xe_b, o + 1 * plane_b, (Store)d[1]);
          bstore<Store>(out, rj + xw_b, o + 3 * plane_b, (Store)d[3]);
          if (!top) {
            bstore<Store>(out, ru + xs_b, o + 2 * plane_b, (Store)(d[2] + sh1));
            bstore<Store>(out, ru + xe_b, o + 5 * plane_b, (Store)(d[5] + sh5));
            bstore<Store>(out, ru + xw_b, o + 6 * plane_b, (Store)(d[6] + sh5));
          } else {
            bstore<Store>(out, rj + xs_b, o + 4 * plane_b, (Store)d[2]);
            bstore<Store>(out, rj + xs_b, o + 7 * plane_b, (Store)d[5]);
            bstore<Store>(out, rj + xs_b, o + 8 * plane_b, (Store)d[6]);
          }
          if (!bot) {
            bstore<Store>(out, rd + xs_b, o + 4 * plane_b, (Store)(d[4] - sh1));
            bstore<Store>(out, rd + xw_b, o + 7 * plane_b, (Store)(d[7] - sh5));
            bstore<Store>(out, rd + xe_b, o + 8 * plane_b, (Store)(d[8] - sh5));
          } else {
            bstore<Store>(out, rj + xs_b, o + 2 * plane_b, (Store)d[4]);
            bstore<Store>(out, rj + xs_b, o + 5 * plane_b, (Store)d[7]);
            bstore<Store>(out, rj + xs_b, o + 6 * plane_b, (Store)d[8]);
          }
        };
        emit(0, dA, shA1, shA5);
        emit(1, dB, -shA1, -shA5);
      }
    }

    // rotate the row window
    dAm = dAc;
    dBm = dBc;
    dAc = dAp;
    dBc = dBp;
#pragma unroll
    for (int q = 0; q < 18; ++q) cur[q] = nxt[q];
  }
}

template <typename Real, typename Store>
hipError_t launch_typed(int mode, const StepArgs& a, hipStream_t s) {
  const dim3 grid(a.n_blocks), block(kBlock);
  switch (mode) {
    case kStep:
      hipLaunchKernelGGL((k_step<Real, Store, kStep>), grid, block, 0, s, a);
      break;
    case kStepSample:
      hipLaunchKernelGGL((k_step<Real, Store, kStepSample>), grid, block, 0, s, a);
      break;
    case kSampleOnly:
      hipLaunchKernelGGL((k_step<Real, Store, kSampleOnly>), grid, block, 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(int precision, int mode, const StepArgs& a, hipStream_t stream) {
  if (a.n_items <= 0) return hipSuccess;
  if (precision == FNLB_FP64) return launch_typed<double, double>(mode, a, stream);
  return launch_typed<float, float>(mode, a, stream);
}

}  // namespace fnlb
