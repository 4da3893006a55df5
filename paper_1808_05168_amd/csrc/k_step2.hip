// Two fused fluctuating D2Q9 steps per HBM pass (FP32-deviation storage).
//
// Method (arXiv:1808.05168): each of the two steps is the LB update of
// Eq. (6) with the collision of Eq. (14) exactly as in the one-step kernel
// (the node update is the same inlined code, fnlb_node.hpp): non-ideal force
// of Eq. (11), a_* of the footnote to Eq. (13), non-equilibrium acceleration
// of Eq. (12), the wall rule and walls of Sec. III.A, noise of Eqs. (22)-(23)
// drawn for (node, t) in the first step and (node, t + 1) in the second.
//
// Why: the one-step kernel streams 144 B per node-step at the bandwidth its
// access shape reaches, with the collision and noise hidden under the
// traffic.  Two steps per pass read and write the state once for two steps,
// so the pass is bound by the arithmetic of two collisions instead.
//
// Mapping.  A block of 512 lanes owns whole periodic rows (one lane per
// column), so the halo of the second step in x is the same block's columns;
// narrow lattices share a block (lane width 64, 128, 256 or 512 per work
// item, all items of a block of one width).  Each item marches through its
// row range [j0, j1) in direction dir.  Stage A runs the first step on the
// rows [j0 - 2, j1 + 2) (clipped at the walls), as the one-step kernel does,
// but instead of storing a row's 18 post-collision values it pushes them in
// LDS to where they stream: the node itself for links with c_z = 0, the row
// ahead or behind otherwise (or, at a wall, back into the node's own opposite
// link).  Once a row of time t + 1 is complete, each lane reads its node's 18
// populations of it and their densities go into a second ring; two rows
// later stage B runs the second step on that row (b = a - 3 dir) from those
// populations and that ring, and stores the result (time t + 2) to HBM in the
// layout of the state.  Two barriers per row: the first separates the
// densities of the row ahead from stage A and the densities of t + 1 from
// stage B, the second the pushes from their reads; stage B runs between them,
// after stage A, so that it needs none of its own.
//
// LDS per block: the density rings of t and t + 1 (3 rows each, 12 KiB each)
// and the pushed populations, kept per class of link for as long as each
// class lives: same-row links 2 rows, links moving in the march direction 3,
// links moving against it 2 (84 KiB).  A completed row of t + 1 is read once,
// for its densities, and stays in registers until its second step.  One block
// per compute unit, two wavefronts per SIMD.
#include "fnlb.h"
#include "fnlb_device.hpp"
#include "fnlb_internal.hpp"
#include "fnlb_node.hpp"
#include "fnlb_state.hpp"

namespace fnlb {
namespace {

constexpr int kRingCols = kTBLanes + 2 * kTBMaxSub;  // each item: its columns + 2 wrap columns

__device__ __forceinline__ void density18(const float (&o)[18], float& da, float& db) {
  float a = o[0], b = o[9];
#pragma unroll
  for (int l = 1; l < 9; ++l) {
    a += o[l];
    b += o[9 + l];
  }
  da = a;
  db = b;
}

// non-negative row -> ring slot
__device__ __forceinline__ int mod3(int r) { return (int)((unsigned)r % 3u); }

template <int MODE>
__global__ __launch_bounds__(kTBLanes) void k_step2(const Step2Args a) {
  using Real = float;
  using Store = float;
  using DT = float;
  // Densities of t and of t + 1, rows mod 3.  The two barriers per row keep
  // a slot's readers apart from its next writer.
  __shared__ DT ring[3][2][kRingCols];
  __shared__ DT dring[3][2][kRingCols];
  // Pushed populations of t + 1, [slot][3 s + k][column]: links 0, 1, 3 of
  // each species (pZ, rows mod 2); links 2, 5, 6 or 4, 7, 8, whichever move in
  // the march direction (pAh, rows mod 3) and against it (pBe, rows mod 2).
  // A row is read once, when it is complete (for its densities); the values
  // then stay in registers until its second step, one row later.
  __shared__ Store pZ[2][6][kTBLanes];
  __shared__ Store pAh[3][6][kTBLanes];
  __shared__ Store pBe[2][6][kTBLanes];

  const int nb = a.n_blocks;
  const int b = blockIdx.x;
  const int per_xcd = nb >> 3;
  const int blk = (b & 7) * per_xcd + (b >> 3);
  if (blk >= a.n_items) return;  // whole block

  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const PackItem* pit = a.items + blk;
  const int nsub = pit->nsub, lw = pit->lwidth, niter = pit->niter;
  const int W = 1 << lw;
  // the item of this wavefront (uniform across it: W >= 64)
  const int sub = __builtin_amdgcn_readfirstlane((wv * kWave) >> lw);
  const bool sub_ok = sub < nsub;
  const int rep = sub_ok ? pit->rep[sub] : pit->rep[0];
  const int j0 = sub_ok ? pit->j0[sub] : 0, j1 = sub_ok ? pit->j1[sub] : 0;
  const int dir = sub_ok ? pit->dir[sub] : 1;
  const RepInfo& R = a.reps[rep];
  const int Lx = R.Lx, Lz = R.Lz;
  constexpr uint32_t SB = sizeof(Store);
  const uint32_t link_b = 64u * SB;
  const uint32_t row_b = (uint32_t)R.pitch * 18u * SB;
  const uint32_t block_b = (uint32_t)(18 * R.plane * SB);
  const Rsrc in = make_rsrc((const char*)a.state_in + R.state_off * SB, block_b);
  const Rsrc out = make_rsrc((char*)a.state_out + R.state_off * SB, block_b);
  const int flags = R.flags;
  const SampleDest<Store, Real> SD = sample_dest<Store, Real>(R, a.fields, a.ppart);

  const int xl = tid & (W - 1);  // column within the item
  const bool act = sub_ok && xl < Lx;
  const int x = act ? xl : 0;
  const int xm = x == 0 ? Lx - 1 : x - 1, xp = x == Lx - 1 ? 0 : x + 1;
  const uint32_t xb = col_offset(x, SB), xmb = col_offset(xm, SB), xpb = col_offset(xp, SB);
  const bool wave_act = sub_ok && (((wv * kWave) & (W - 1)) < Lx);
  const int cb = sub * (W + 2);  // ring columns of this item: cb .. cb + Lx + 1
  const int c = cb + x + 1;      // ring column of this lane
  const int pb = sub * W;        // push-buffer columns of this item
  const int pc = pb + x, pm = pb + xm, pp = pb + xp;

  const int64_t t = *a.t_base + a.t_off;
  const uint32_t k0 = R.seed_lo, k1 = R.seed_hi;
  const double rA0 = R.rA_mid, rAs = R.rA_step, rho0 = R.rho0;
  NodePhys<Real> P;
  P.load(R);
  const BmTables* bmt = R.bm;

  // stage A: rows [alo, ahi) of the first step; raw densities needed on
  // [lo, hi]
  const int alo = max(j0 - 2, 0), ahi = min(j1 + 2, Lz);
  const int lo = max(alo - 1, 0), hi = min(ahi, Lz - 1);
  const int afirst = dir > 0 ? alo : ahi - 1;
  auto needed = [&](int jr) { return jr >= lo && jr <= hi; };
  auto a_row = [&](int r) { return r >= alo && r < ahi; };

  auto put_raw = [&](int jr, const Store(&o)[18]) {
    if (act) {
      DT da, db;
      density18(o, da, db);
      const int sl = mod3(jr);
      ring[sl][0][c] = da;
      ring[sl][1][c] = db;
      if (x == Lx - 1) {
        ring[sl][0][cb] = da;
        ring[sl][1][cb] = db;
      }
      if (x == 0) {
        ring[sl][0][cb + Lx + 1] = da;
        ring[sl][1][cb + Lx + 1] = db;
      }
    }
  };

  // slots of the pushed populations of a row r of t + 1, per class
  auto zs = [&](int r) { return r & 1; };
  auto ahs = [&](int r) { return mod3(r); };
  auto bes = [&](int r) { return r & 1; };
  // the class arrays of links moving up (2, 5, 6) and down (4, 7, 8)
  const bool up_march = dir > 0;

  Store cur[18], nxt[18];
  // populations of t + 1 at this lane's node (see the loop)
  Store hp[18], hn[18];
  if (sub_ok && a_row(afirst)) {
    load_pulled(in, link_b, row_b, afirst, Lz, xb, xmb, xpb, cur);
    put_raw(afirst, cur);
    if (needed(afirst - dir)) {
      Store tmp[18];
      load_pulled(in, link_b, row_b, afirst - dir, Lz, xb, xmb, xpb, tmp);
      put_raw(afirst - dir, tmp);
    }
    if (needed(afirst + dir)) load_pulled(in, link_b, row_b, afirst + dir, Lz, xb, xmb, xpb, nxt);
  }

  // With t even the two steps share one noise call per node (words 12 and 13
  // of both steps): stage A draws it and keeps the second step's two words,
  // which its second step uses two rows (two iterations) later.
  const bool odd_t = (t & 1) != 0;
  // kept words of the rows ar - 3 dir, ar - 2 dir and ar - dir (t even)
  uint32_t kw[3][2] = {{0u, 0u}, {0u, 0u}, {0u, 0u}};

  // One row of each stage.  cur: the pulled row ar of t, nxt: the row ahead;
  // hn: the populations of t + 1 of the row whose second step runs now (row
  // ar - 3 dir), then those of the row behind (ar - dir); hp: those of row
  // ar - 2 dir, whose second step runs in the next iteration.  The loop runs
  // two iterations per trip with the register sets swapped in the second, so
  // that no set is copied.
  auto iteration = [&](int i, Store(&cur)[18], Store(&nxt)[18], Store(&hp)[18],
                       Store(&hn)[18]) {
    (void)hp;
    const int ar = afirst + dir * i;  // row of the first step
    const bool doA = sub_ok && a_row(ar);
    const bool topA = ar == Lz - 1, botA = ar == 0;

    // ---- stage A, before the barrier: noise, densities of the row ahead
    Real gA0[4], gA1[4], gB0[4], gB1[4];
    uint32_t nw12 = 0u, nw13 = 0u;  // words 12, 13 of step t + 1 at (ar, x), t even
    if (doA && wave_act) {
      const uint32_t node = (uint32_t)(ar * Lx + x);
      uint32_t w12, w13;
      shared_words(node, (uint64_t)t, k0, k1, w12, w13, nw12, nw13);
      node_noise_words(node, (uint64_t)t, k0, k1, bmt, w12, w13, gA0, gA1, gB0, gB1);
    }
    if (doA && needed(ar + dir)) put_raw(ar + dir, nxt);
    // the sample constants of row ar, read before the barrier, which waits
    // for them
    SampleRow<Real> srow{};
    if constexpr (MODE == kStepSample)
      if (doA) srow = sample_row(SD, ar);
    __syncthreads();

    // ---- stage A: the first step of row ar, pushed to where it streams
    if (doA) {
      const int jU = topA ? ar : ar + 1, jD = botA ? ar : ar - 1;
      const double rAj = rA0 + rAs * ar;
      const double szref = rAs * (double)(jU - jD) * (1.0 / 6.0);
      // sample of f(t) on the item's own rows, formed as the one-step kernel
      // forms it, from the stencil the collision reads (its own read of it)
      if constexpr (MODE == kStepSample) {
        if (wave_act && ar >= j0 && ar < j1) {
          Real dp = (Real)0;
          if (act) {
            const bool vel = (flags & FNLB_SAMPLE_VELOCITY) != 0;
            const NodeSample<Real> smp = sample_of<Real, DT, Store>(
                load_stencil(ring[mod3(jU)][0], ring[mod3(ar)][0], ring[mod3(jD)][0],
                             ring[mod3(jU)][1], ring[mod3(ar)][1], ring[mod3(jD)][1], c),
                cur, srow, P.G, vel);
            store_sample(SD, a.watchdog, ar, x, smp, vel);
            dp = smp.dp;
          }
          store_pressure_part(SD, ar, ((wv * kWave) & (W - 1)) >> 6, dp);
        }
      }
      const Stencil<DT> st =
          load_stencil(ring[mod3(jU)][0], ring[mod3(ar)][0], ring[mod3(jD)][0],
                       ring[mod3(jU)][1], ring[mod3(ar)][1], ring[mod3(jD)][1], c);
      if (wave_act) {
        Real dA[9], dB[9];
#pragma unroll
        for (int l = 0; l < 9; ++l) {
          dA[l] = cur[l];
          dB[l] = cur[9 + l];
        }
        node_update<Real, DT>(P, flags, topA, botA, rAj, rho0, szref, st, dA, dB, gA0, gA1, gB0,
                              gB1);

        if (act) {
          // values as the one-step kernel stores them: each shifted to the
          // reference of the row it streams to (bounced-back links stay)
          const Real upf = topA ? (Real)0 : (Real)1, dnf = botA ? (Real)0 : (Real)1;
          const int z = zs(ar);
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const Real(&d)[9] = s == 0 ? dA : dB;
            const Real sh1 = s == 0 ? P.shA1 : -P.shA1, sh5 = s == 0 ? P.shA5 : -P.shA5;
            pZ[z][3 * s + 0][pc] = d[0];
            pZ[z][3 * s + 1][pp] = d[1];
            pZ[z][3 * s + 2][pm] = d[3];
            const Real u0 = d[2] + upf * sh1, u1 = d[5] + upf * sh5, u2 = d[6] + upf * sh5;
            const Real m0 = d[4] - dnf * sh1, m1 = d[7] - dnf * sh5, m2 = d[8] - dnf * sh5;
            // up-moving links: to row ar + 1, or bounced into the node's own
            // down-moving links at the top wall
            if (!topA) {
              Store* q = up_march ? &pAh[ahs(ar + 1)][0][0] : &pBe[bes(ar + 1)][0][0];
              q[(3 * s + 0) * kTBLanes + pc] = u0;
              q[(3 * s + 1) * kTBLanes + pp] = u1;
              q[(3 * s + 2) * kTBLanes + pm] = u2;
            } else {
              Store* q = up_march ? &pBe[bes(ar)][0][0] : &pAh[ahs(ar)][0][0];
              q[(3 * s + 0) * kTBLanes + pc] = u0;
              q[(3 * s + 1) * kTBLanes + pc] = u1;
              q[(3 * s + 2) * kTBLanes + pc] = u2;
            }
            // down-moving links: to row ar - 1, or bounced into the node's own
            // up-moving links at the bottom wall
            if (!botA) {
              Store* q = up_march ? &pBe[bes(ar - 1)][0][0] : &pAh[ahs(ar - 1)][0][0];
              q[(3 * s + 0) * kTBLanes + pc] = m0;
              q[(3 * s + 1) * kTBLanes + pm] = m1;
              q[(3 * s + 2) * kTBLanes + pp] = m2;
            } else {
              Store* q = up_march ? &pAh[ahs(ar)][0][0] : &pBe[bes(ar)][0][0];
              q[(3 * s + 0) * kTBLanes + pc] = m0;
              q[(3 * s + 1) * kTBLanes + pc] = m1;
              q[(3 * s + 2) * kTBLanes + pc] = m2;
            }
          }
        }
      }
      // the row after next, into the registers of this row (the next
      // iteration sees them as its row ahead): its loads run through stage B
      // and the next noise
      if (needed(ar + 2 * dir)) load_pulled(in, link_b, row_b, ar + 2 * dir, Lz, xb, xmb, xpb, cur);
    }

    // ---- stage B: the second step of row bq = ar - 3 dir, whose populations
    // of t + 1 were read two iterations ago (into hn) and whose densities of
    // t + 1 (rows bq and bq +- 1) are complete since the last iteration; the
    // result is stored to HBM.  Run between the two barriers (after stage A,
    // whose noise is then no longer live), it needs no barrier of its own:
    // the next writes of the density slots it reads follow the second one.
    const int bq = ar - 3 * dir;
    const bool doB = sub_ok && wave_act && bq >= j0 && bq < j1;
    if (doB) {
      Real gA0b[4], gA1b[4], gB0b[4], gB1b[4];
      {
        const uint32_t node = (uint32_t)(bq * Lx + x);
        uint32_t w12 = kw[0][0], w13 = kw[0][1];
        if (odd_t) {  // t + 1 even: its shared call is its own
          uint32_t o12, o13;
          shared_words(node, (uint64_t)(t + 1), k0, k1, w12, w13, o12, o13);
        }
        node_noise_words(node, (uint64_t)(t + 1), k0, k1, bmt, w12, w13, gA0b, gA1b, gB0b,
                         gB1b);
      }
      const bool top = bq == Lz - 1, bot = bq == 0;
      Real dA[9], dB[9];
#pragma unroll
      for (int l = 0; l < 9; ++l) {
        dA[l] = hn[l];
        dB[l] = hn[9 + l];
      }
      const int jU = top ? bq : bq + 1, jD = bot ? bq : bq - 1;
      const double rAj = rA0 + rAs * bq;
      const double szref = rAs * (double)(jU - jD) * (1.0 / 6.0);
      const Stencil<DT> stb =
          load_stencil(dring[mod3(jU)][0], dring[mod3(bq)][0], dring[mod3(jD)][0],
                       dring[mod3(jU)][1], dring[mod3(bq)][1], dring[mod3(jD)][1], c);
      node_update<Real, DT>(P, flags, top, bot, rAj, rho0, szref, stb, dA, dB, gA0b, gA1b, gB0b,
                            gB1b);
      if (act) {
        const uint32_t off = (uint32_t)bq * row_b + xb;
        const Real upf = top ? (Real)0 : (Real)1, dnf = bot ? (Real)0 : (Real)1;
        auto emit = [&](int s, const Real(&d)[9], Real sh1, Real sh5) {
          const uint32_t p = (uint32_t)(9 * s) * link_b;
          bstore<Store>(out, off, p, (Store)d[0]);
          bstore<Store>(out, off, p + link_b, (Store)d[1]);
          bstore<Store>(out, off, p + 2 * link_b, (Store)(d[2] + upf * sh1));
          bstore<Store>(out, off, p + 3 * link_b, (Store)d[3]);
          bstore<Store>(out, off, p + 4 * link_b, (Store)(d[4] - dnf * sh1));
          bstore<Store>(out, off, p + 5 * link_b, (Store)(d[5] + upf * sh5));
          bstore<Store>(out, off, p + 6 * link_b, (Store)(d[6] + upf * sh5));
          bstore<Store>(out, off, p + 7 * link_b, (Store)(d[7] - dnf * sh5));
          bstore<Store>(out, off, p + 8 * link_b, (Store)(d[8] - dnf * sh5));
        };
        emit(0, dA, P.shA1, P.shA5);
        emit(1, dB, -P.shA1, -P.shA5);
      }
    }

    __syncthreads();

    // the populations of row r of t + 1 at this lane's column, in link order
    auto pulled1 = [&](int r, Store(&o)[18]) {
      const int z = zs(r);
      // class arrays of the up-moving (2, 5, 6) and down-moving (4, 7, 8) links
      const Store* qu = up_march ? &pAh[ahs(r)][0][0] : &pBe[bes(r)][0][0];
      const Store* qd = up_march ? &pBe[bes(r)][0][0] : &pAh[ahs(r)][0][0];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        o[9 * s + 0] = pZ[z][3 * s + 0][pc];
        o[9 * s + 1] = pZ[z][3 * s + 1][pc];
        o[9 * s + 3] = pZ[z][3 * s + 2][pc];
        o[9 * s + 2] = qu[(3 * s + 0) * kTBLanes + pc];
        o[9 * s + 5] = qu[(3 * s + 1) * kTBLanes + pc];
        o[9 * s + 6] = qu[(3 * s + 2) * kTBLanes + pc];
        o[9 * s + 4] = qd[(3 * s + 0) * kTBLanes + pc];
        o[9 * s + 7] = qd[(3 * s + 1) * kTBLanes + pc];
        o[9 * s + 8] = qd[(3 * s + 2) * kTBLanes + pc];
      }
    };

    // ---- the row behind is complete: read its populations of t + 1 (kept in
    // registers for its second step two iterations later) and sum its
    // densities
    const int dr = ar - dir;
    const bool doD = sub_ok && act && dr >= max(j0 - 1, 0) && dr <= min(j1, Lz - 1);
    if (doD) pulled1(dr, hn);
    kw[0][0] = kw[1][0];
    kw[0][1] = kw[1][1];
    kw[1][0] = kw[2][0];
    kw[1][1] = kw[2][1];
    kw[2][0] = nw12;
    kw[2][1] = nw13;
    if (doD) {
      DT da, db;
      density18(hn, da, db);
      const int sl = mod3(dr);
      dring[sl][0][c] = da;
      dring[sl][1][c] = db;
      if (x == Lx - 1) {
        dring[sl][0][cb] = da;
        dring[sl][1][cb] = db;
      }
      if (x == 0) {
        dring[sl][0][cb + Lx + 1] = da;
        dring[sl][1][cb + Lx + 1] = db;
      }
    }
  };
  // the host rounds niter up to an even count (trailing iterations do nothing)
  for (int i = 0; i < niter; i += 2) {
    iteration(i, cur, nxt, hp, hn);
    iteration(i + 1, nxt, cur, hn, hp);
  }
}

}  // namespace

hipError_t launch_step2(int mode, const Step2Args& a, hipStream_t stream) {
  if (a.n_items <= 0) return hipSuccess;
  const dim3 grid(a.n_blocks), block(kTBLanes);
  if (mode == kStepSample)
    hipLaunchKernelGGL((k_step2<kStepSample>), grid, block, 0, stream, a);
  else if (mode == kStep)
    hipLaunchKernelGGL((k_step2<kStep>), grid, block, 0, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace fnlb
