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
// Layout.  Populations are stored structure-of-arrays, one plane per
// (species, link), x fastest, rows padded to 64 elements.  What is stored at
// node r for link l is the post-collision population of r (streaming is a
// pull: the next step reads link l of node r from r - c_l, or from the
// opposite link of r itself where c_l leaves through a wall, which is mid-way
// bounce-back).  Values are deviations from w_l rho_ref^S(z_dest) of the row
// they stream to, with rho_ref^A = rho_bar c_0(z), rho_ref^B = rho_bar
// (1 - c_0(z)); the writer adds the constant w_l (rho_ref(z) - rho_ref(z +
// c_lz)) for links that change row.  The state of rest on the imposed profile
// is all zeros.
//
// Mapping.  A block of four wavefronts owns a 256-column segment of one row
// range and marches through its rows, upwards or downwards (neighbouring row
// ranges alternate, so that the halo rows they share are read at the same
// time and served once from HBM).  Every lane pulls its node's 18 populations
// of the row ahead, sums its densities into a four-row ring in LDS (plus the
// two segment-edge columns, pulled by 36 lanes of the first wavefront with one
// load, or wrapped when the segment is a whole periodic row), and after one
// barrier per row reads the eight neighbour densities of the non-local force
// from LDS.  The pulled populations wait in an LDS slot of the lane until
// the row is collided, while the loads of the row after next are in flight.
// Stores are the node's own 18 post-collision values; in the tiled
// layout each link of a wavefront's row is one contiguous 256-byte run.  A
// step that samples also writes, per node, the density deviations of the
// state it pulled (and the momenta for velocity sampling), summed in FP64 and
// stored in the storage type; the transform pass forms the observables from
// them in FP64.
#include "fnlb.h"
#include "fnlb_device.hpp"
#include "fnlb_internal.hpp"
#include "fnlb_state.hpp"

#include <type_traits>

namespace fnlb {
namespace {

template <typename DT, typename Store>
__device__ __forceinline__ void density(const Store (&o)[18], DT& da, DT& db) {
  DT a = (DT)o[0], b = (DT)o[9];
#pragma unroll
  for (int l = 1; l < 9; ++l) {
    a += (DT)o[l];
    b += (DT)o[9 + l];
  }
  da = a;
  db = b;
}

// the 18 populations of one column pulled at row jr (segment-edge column)
template <typename Store>
__device__ __forceinline__ void edge_pull(Rsrc r, uint32_t link_b, uint32_t row_b, int jr,
                                          int Lz, int Lx, int col, Store (&o)[18]) {
  constexpr uint32_t SB = sizeof(Store);
  const int cm = col == 0 ? Lx - 1 : col - 1, cp = col == Lx - 1 ? 0 : col + 1;
  load_pulled(r, link_b, row_b, jr, Lz, col_offset(col, SB), col_offset(cm, SB),
              col_offset(cp, SB), o);
}

// TAB_LDS (FP64 only): the block copies the Box-Muller tables into LDS first,
// which pays off for work items of several rows.
template <typename Real, typename Store, int MODE, bool TAB_LDS>
__global__ __launch_bounds__(kBlock) void k_step(const StepArgs a) {
  // Density ring in LDS (row slot, species, column + 1) in the compute type:
  // the collision reads the same sums whether or not the step samples, so
  // sampling leaves the trajectory bit-identical.
  using DT = Real;
  constexpr int kRow = kSeg + 2;
  __shared__ DT ring[4][2][kRow];
  __shared__ Store edge[2][36];  // pulled populations of the two edge columns
  // A lane parks the pulled populations of the row ahead in LDS (a slot
  // private to the lane) and reads them back at the top of the next iteration.
  // That frees the registers to receive the loads of the row after next while
  // the current row is collided, so a row's loads are in flight for a whole
  // iteration.
  __shared__ Store pbuf[18][kBlock];

  // XCD-aware block order: consecutive hardware blocks go to different XCDs,
  // so give each XCD a contiguous range of work items (neighbouring segments
  // of the same rows share their edge columns in that XCD's L2).
  const int nb = a.n_blocks;
  const int b = blockIdx.x;
  const int per_xcd = nb >> 3;
  const int blk = (b & 7) * per_xcd + (b >> 3);
  if (blk >= a.n_items) return;  // whole block: no barrier is skipped by part of it

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const Item it = a.items[blk];
  const RepInfo& R = a.reps[it.rep];
  const int Lx = R.Lx, Lz = R.Lz;
  constexpr uint32_t SB = sizeof(Store);
  const uint32_t link_b = 64u * SB;                 // tiled layout of the state block
  const uint32_t row_b = (uint32_t)R.pitch * 18u * SB;
  const uint32_t block_b = (uint32_t)(18 * R.plane * SB);
  const Rsrc in = make_rsrc((const char*)a.state_in + R.state_off * SB, block_b);
  const Rsrc out = make_rsrc((char*)a.state_out + R.state_off * SB, block_b);
  const int flags = R.flags;

  // columns of this segment
  const int X0 = it.strip * kSeg;
  const int width = min(kSeg, Lx - X0);
  const bool act = tid < width;
  const int x = act ? X0 + tid : X0;
  const int xm = x == 0 ? Lx - 1 : x - 1, xp = x == Lx - 1 ? 0 : x + 1;
  const uint32_t xb = col_offset(x, SB), xmb = col_offset(xm, SB), xpb = col_offset(xp, SB);
  const bool whole_row = (X0 == 0 && width == Lx);
  const int hl = X0 == 0 ? Lx - 1 : X0 - 1;          // left edge column
  const int hr = X0 + width == Lx ? 0 : X0 + width;  // right edge column
  const int c = tid + 1;                             // ring column of this lane
  // wavefronts entirely beyond the last column of a narrow lattice only take
  // part in the barriers
  const bool wave_act = X0 + kWave * wv < Lx;

  // writes the density deviations of 18 pulled populations into ring column
  // col of row jr
  auto put_col = [&](int jr, int col, const Store(&o)[18]) {
    DT da, db;
    density<DT>(o, da, db);
    ring[jr & 3][0][col] = da;
    ring[jr & 3][1][col] = db;
  };
  // writes the density deviations of row jr of this lane into the ring (and,
  // for a whole periodic row, the wrapped edge columns)
  auto put_row = [&](int jr, const Store(&o)[18]) {
    if (act) {
      put_col(jr, c, o);
      if (whole_row) {
        if (x == Lx - 1) put_col(jr, 0, o);
        if (x == 0) put_col(jr, width + 1, o);
      }
    }
  };

  // Edge columns of a partial segment: lane 18 e + 9 s + l of wavefront 0
  // pulls link l of species s of edge column e (0: left, 1: right) with one
  // load instruction; after the row barrier the lane that needs the edge sums
  // the nine values of each species.
  // c_x + 1, c_z + 1 (2 bits each) and opp(l) (4 bits) of link l, packed
  constexpr uint32_t kCXp = 0x20919u, kCZp = 0x02865u;
  constexpr uint64_t kOppP = 0x658721430ull;
  const bool edge_lane = !whole_row && wv == 0 && lane < 36;
  const int el = lane % 9, es = (lane % 18) / 9;
  const int ecx = (int)((kCXp >> (2 * el)) & 3u) - 1;
  const int ecz = (int)((kCZp >> (2 * el)) & 3u) - 1;
  const int eopp = (int)((kOppP >> (4 * el)) & 15u);
  const int ecol = lane < 18 ? hl : hr;
  int exs = ecol - ecx;
  exs = exs < 0 ? exs + Lx : (exs >= Lx ? exs - Lx : exs);
  // the load is issued here and its value written to LDS only just before the
  // row barrier, so that the noise of the current row overlaps the latency of
  // the next row's loads
  auto pull_edges = [&](int jr) -> Store {
    if (edge_lane) {
      const int js = jr - ecz;
      const bool bounce = js < 0 || js >= Lz;
      const uint32_t pl = (uint32_t)(9 * es + (bounce ? eopp : el)) * link_b;
      const uint32_t off = pl + (uint32_t)(bounce ? jr : js) * row_b +
                           col_offset(bounce ? ecol : exs, SB);
      return bload<Store>(in, off, 0);
    }
    return (Store)0;
  };
  auto put_edges = [&](int jr, Store v) {
    if (edge_lane) edge[jr & 1][lane] = v;
  };
  auto sum_edges = [&](int jr) {
    if (!whole_row && (tid == 0 || tid == width - 1)) {
      const Store* e = edge[jr & 1] + (tid == 0 ? 0 : 18);
      Store o[18];
#pragma unroll
      for (int l = 0; l < 18; ++l) o[l] = e[l];
      put_col(jr, tid == 0 ? 0 : width + 1, o);
    }
  };

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
  // shift of a deviation that moves up one row, species A: w_l (rho_ref^A(j)
  // - rho_ref^A(j+1)) = -w_l rho_bar grad_c0; species B has the opposite sign
  const Real shA1 = (Real)(-rAs / 9.0), shA5 = (Real)(-rAs / 36.0);

  // noise amplitudes of the moments 1 and 3..8, read once before the row loop
  // (reloading them per row cost 5% of the step): those at the reference
  // densities, or with local noise the factors that multiply the square roots
  // of the local densities
  const bool loc = (flags & FNLB_NOISE_LOC) != 0;
  const double* sgA = loc ? R.sig_base : R.sig[0];
  const double* sgB = loc ? R.sig_base : R.sig[1];
  const Real sig0d = (Real)sgA[1];
  const Real sig0[5] = {(Real)sgA[3], (Real)sgA[4], (Real)sgA[5], (Real)sgA[6], (Real)sgA[8]};
  const Real sig1[5] = {(Real)sgB[3], (Real)sgB[4], (Real)sgB[5], (Real)sgB[6], (Real)sgB[8]};

  const int j0 = it.j0, j1 = it.j1;
  // FP64 Box-Muller tables: gathered by table index, from LDS when the item
  // has several rows (the copy is one more barrier before the first row)
  const BmTables* bmt = R.bm;
  if constexpr (TAB_LDS) {
    static_assert(sizeof(Real) == 8, "tables are used by the FP64 form only");
    __shared__ BmTables bm_lds;
    const double2* src = (const double2*)R.bm;
    double2* dst = (double2*)&bm_lds;
    constexpr int n2 = (int)(sizeof(BmTables) / sizeof(double2));
    for (int q = tid; q < n2; q += kBlock) dst[q] = src[q];
    __syncthreads();
    bmt = &bm_lds;
  }
  // Rows whose densities the item needs: its own and one more on each side
  // inside the walls.  The item marches from jfirst in direction dir (items
  // alternate, so that two sharing a boundary read its rows at the same time);
  // "ahead" is the next row in that direction.
  const int dir = it.dir;
  const int lo = max(j0 - 1, 0), hi = min(j1, Lz - 1);
  const int jfirst = dir > 0 ? j0 : j1 - 1;
  auto needed = [&](int jr) { return jr >= lo && jr <= hi; };
  auto park = [&](const Store(&o)[18]) {
#pragma unroll
    for (int q = 0; q < 18; ++q) pbuf[q][tid] = o[q];
  };
  Store cur[18], nxt[18];
  load_pulled(in, link_b, row_b, jfirst, Lz, xb, xmb, xpb, cur);
  put_row(jfirst, cur);
  park(cur);
  if (needed(jfirst - dir)) {  // the row behind the first one
    Store tmp[18];
    load_pulled(in, link_b, row_b, jfirst - dir, Lz, xb, xmb, xpb, tmp);
    put_row(jfirst - dir, tmp);
  }
  if (!whole_row && (tid == 0 || tid == width - 1)) {
    const int col = tid == 0 ? hl : hr, rc = tid == 0 ? 0 : width + 1;
    for (int k = 0; k < 2; ++k) {
      const int jr = k == 0 ? jfirst - dir : jfirst;
      if (!needed(jr)) continue;
      Store o[18];
      edge_pull<Store>(in, link_b, row_b, jr, Lz, Lx, col, o);
      put_col(jr, rc, o);
    }
  }

  Store ev = (Store)0;
  // the first row ahead is in flight before the loop
  if (needed(jfirst + dir)) {
    load_pulled(in, link_b, row_b, jfirst + dir, Lz, xb, xmb, xpb, nxt);
    ev = pull_edges(jfirst + dir);
  }

  for (int i = 0; i < j1 - j0; ++i) {
    const int j = jfirst + dir * i;
    const bool top = (j == Lz - 1), bot = (j == 0);
    const int ja = j + dir;  // the row ahead
    const bool ahead = needed(ja);
    // the populations of this row, parked in the previous iteration (or
    // before the loop)
#pragma unroll
    for (int q = 0; q < 18; ++q) cur[q] = pbuf[q][tid];

    // thermal noise of this node: 14 standard normals, drawn while the next
    // row's loads are in flight (species A uses g_0..g_7 from calls 0 and 1,
    // species B g_8..g_13 from calls 2 and 3)
    const uint32_t node = (uint32_t)(j * Lx + x);
    Real gA0[4], gA1[4], gB0[4], gB1[4];
    if constexpr (MODE != kSampleOnly) {
      if (wave_act) {
        node_normals(node, (uint64_t)t, 2u, k0, k1, gB0, bmt);
        node_normals(node, (uint64_t)t, 3u, k0, k1, gB1, bmt);
        node_normals(node, (uint64_t)t, 0u, k0, k1, gA0, bmt);
        node_normals(node, (uint64_t)t, 1u, k0, k1, gA1, bmt);
      }
    }

    if (ahead) {
      put_row(ja, nxt);
      put_edges(ja, ev);
      park(nxt);
    }
    // the row after next: its loads run through the barrier and the collision
    if (needed(ja + dir)) {
      load_pulled(in, link_b, row_b, ja + dir, Lz, xb, xmb, xpb, nxt);
      ev = pull_edges(ja + dir);
    }
    __syncthreads();
    if (ahead) sum_edges(ja);

    // the 3 x 3 density stencil; ghost rows beyond the walls repeat the wall row
    const int jU = top ? j : j + 1, jD = bot ? j : j - 1;

    // reference densities of this row and of the rows the stencil reaches
    const double rAj = rA0 + rAs * j;
    const double szref = rAs * (double)(jU - jD) * (1.0 / 6.0);  // species A

    if constexpr (MODE != kStep) {
      // sample of f(t): the density deviations of this node and, for velocity
      // sampling, its total momentum, summed in FP64 and stored in the storage
      // type (in FP32 the rounding, 6e-8 relative, stays far inside the
      // 1e-5 bar of that storage form); the transform pass forms the
      // observables from them
      if (act) {
        double da, db;
        density<double>(cur, da, db);
        Store* fld = (Store*)a.fields + R.field_off;
        const int64_t plane = (int64_t)Lz * Lx, n = (int64_t)j * Lx + x;
        fld[n] = (Store)da;
        fld[plane + n] = (Store)db;
        if (flags & FNLB_SAMPLE_VELOCITY) {
          double d[9];
#pragma unroll
          for (int l = 0; l < 9; ++l) d[l] = (double)cur[l] + (double)cur[9 + l];
          fld[2 * plane + n] = (Store)((d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]));
          fld[3 * plane + n] = (Store)((d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]));
        }
      }
    }

    if constexpr (MODE != kSampleOnly) {
     if (wave_act) {
      const DT* aU = ring[jU & 3][0];
      const DT* bU = ring[jU & 3][1];
      const DT* aC = ring[j & 3][0];
      const DT* bC = ring[j & 3][1];
      const DT* aD = ring[jD & 3][0];
      const DT* bD = ring[jD & 3][1];
      const DT dAc = aC[c], dBc = bC[c];
      const DT aWc = aC[c - 1], aEc = aC[c + 1], bWc = bC[c - 1], bEc = bC[c + 1];
      const DT dAp = aU[c], aWp = aU[c - 1], aEp = aU[c + 1];
      const DT dBp = bU[c], bWp = bU[c - 1], bEp = bU[c + 1];
      const DT dAm = aD[c], aWm = aD[c - 1], aEm = aD[c + 1];
      const DT dBm = bD[c], bWm = bD[c - 1], bEm = bD[c + 1];
      Real dA[9], dB[9];
#pragma unroll
      for (int l = 0; l < 9; ++l) {
        dA[l] = (Real)cur[l];
        dB[l] = (Real)cur[9 + l];
      }
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
      const Real sAz =
          w1 * (Real)(dAp - dAm) + w5 * (Real)((aEp + aWp) - (aEm + aWm)) + (Real)szref;
      const Real sBz =
          w1 * (Real)(dBp - dBm) + w5 * (Real)((bEp + bWp) - (bEm + bWm)) - (Real)szref;

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

      // noise amplitudes: at the reference densities, or with local noise the
      // base amplitudes times the square roots of the local densities, applied
      // to the normals (the amplitudes themselves stay loop-invariant)
      const Real sd = sig0d;
      const Real sA3 = sig0[0], sA4 = sig0[1], sA5 = sig0[2], sA6 = sig0[3], sA8 = sig0[4];
      const Real sB3 = sig1[0], sB4 = sig1[1], sB5 = sig1[2], sB6 = sig1[3], sB8 = sig1[4];
      if (loc) {
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

      // collision of one species in moment space: adds the increments
      // R_l = w_l sum_a T_al dm_a / N_a to the populations
      auto collide = [&](Real(&d)[9], Real rs, Real jx, Real jz, Real Fx, Real Fz, Real x1,
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
      collide(dA, rhoA, jAx, jAz, FAx, FAz, xi1, xi2, sA3 * gA0[2], sA4 * gA0[3],
              sA5 * gA1[0], sA6 * gA1[1], sA6 * gA1[2], sA8 * gA1[3]);
      collide(dB, rhoB, jBx, jBz, FBx, FBz, -xi1, -xi2, sB3 * gB0[0], sB4 * gB0[1],
              sB5 * gB0[2], sB6 * gB0[3], sB6 * gB1[0], sB8 * gB1[1]);

      // store the node's post-collision populations, each shifted to the
      // reference of the row it streams to (bounced-back links stay in row)
      if (act) {
        const uint32_t off = (uint32_t)j * row_b + xb;
        const Real up = top ? (Real)0 : (Real)1, dn = bot ? (Real)0 : (Real)1;
        auto emit = [&](int s, const Real(&d)[9], Real sh1, Real sh5) {
          const uint32_t p = (uint32_t)(9 * s) * link_b;
          bstore<Store>(out, off, p, (Store)d[0]);
          bstore<Store>(out, off, p + link_b, (Store)d[1]);
          bstore<Store>(out, off, p + 2 * link_b, (Store)(d[2] + up * sh1));
          bstore<Store>(out, off, p + 3 * link_b, (Store)d[3]);
          bstore<Store>(out, off, p + 4 * link_b, (Store)(d[4] - dn * sh1));
          bstore<Store>(out, off, p + 5 * link_b, (Store)(d[5] + up * sh5));
          bstore<Store>(out, off, p + 6 * link_b, (Store)(d[6] + up * sh5));
          bstore<Store>(out, off, p + 7 * link_b, (Store)(d[7] - dn * sh5));
          bstore<Store>(out, off, p + 8 * link_b, (Store)(d[8] - dn * sh5));
        };
        emit(0, dA, shA1, shA5);
        emit(1, dB, -shA1, -shA5);
      }
     }
    }
  }
}

template <typename Real, typename Store, bool TAB_LDS>
hipError_t launch_typed(int mode, const StepArgs& a, hipStream_t s) {
  const dim3 grid(a.n_blocks), block(kBlock);
  switch (mode) {
    case kStep:
      hipLaunchKernelGGL((k_step<Real, Store, kStep, TAB_LDS>), grid, block, 0, s, a);
      break;
    case kStepSample:
      hipLaunchKernelGGL((k_step<Real, Store, kStepSample, TAB_LDS>), grid, block, 0, s, a);
      break;
    case kSampleOnly:
      hipLaunchKernelGGL((k_step<Real, Store, kSampleOnly, TAB_LDS>), grid, block, 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(int precision, int mode, const StepArgs& a, hipStream_t stream) {
  if (a.n_items <= 0) return hipSuccess;
  if (precision == FNLB_FP64)
    return a.chunk_rows >= 4 ? launch_typed<double, double, true>(mode, a, stream)
                             : launch_typed<double, double, false>(mode, a, stream);
  return launch_typed<float, float, false>(mode, a, stream);
}

}  // namespace fnlb
