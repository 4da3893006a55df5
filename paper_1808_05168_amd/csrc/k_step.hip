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
// step that samples also forms, per node, the sample of the state it pulled
// from the stencil its collision reads (node_sample, in the compute type) and
// stores the pairs the row transform takes and the pressure deviation.
#include "fnlb.h"
#include "fnlb_device.hpp"
#include "fnlb_internal.hpp"
#include "fnlb_node.hpp"
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
  const SampleDest<Store, Real> SD = sample_dest<Store, Real>(R, a.fields, a.ppart);

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
  // (a segment of one column has one lane next to both edges)
  auto sum_edges = [&](int jr) {
    if (!whole_row && (tid == 0 || tid == width - 1)) {
      for (int side = 0; side < 2; ++side) {
        if (side == 0 ? tid != 0 : tid != width - 1) continue;
        const Store* e = edge[jr & 1] + 18 * side;
        Store o[18];
#pragma unroll
        for (int l = 0; l < 18; ++l) o[l] = e[l];
        put_col(jr, side == 0 ? 0 : width + 1, o);
      }
    }
  };

  const int64_t t = *a.t_base + a.t_off;
  const uint32_t k0 = R.seed_lo, k1 = R.seed_hi;

  const double rA0 = R.rA_mid, rAs = R.rA_step, rho0 = R.rho0;
  // physics constants, read once before the row loop (reloading the noise
  // amplitudes per row cost 5% of the step)
  NodePhys<Real> P;
  P.load(R);

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
    for (int side = 0; side < 2; ++side) {
      if (side == 0 ? tid != 0 : tid != width - 1) continue;
      const int col = side == 0 ? hl : hr, rc = side == 0 ? 0 : width + 1;
      for (int k = 0; k < 2; ++k) {
        const int jr = k == 0 ? jfirst - dir : jfirst;
        if (!needed(jr)) continue;
        Store o[18];
        edge_pull<Store>(in, link_b, row_b, jr, Lz, Lx, col, o);
        put_col(jr, rc, o);
      }
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
    // species B g_8..g_11 from call 2 and g_12, g_13 from its half of the
    // call shared with the other step of its pair)
    const uint32_t node = (uint32_t)(j * Lx + x);
    Real gA0[4], gA1[4], gB0[4], gB1[4];
    if constexpr (MODE != kSampleOnly) {
      if (wave_act) node_noise(node, (uint64_t)t, k0, k1, bmt, gA0, gA1, gB0, gB1);
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
    // the sample constants of row j, read before the barrier
    SampleRow<Real> srow{};
    if constexpr (MODE != kStep) srow = sample_row(SD, j);
    __syncthreads();
    if (ahead) sum_edges(ja);

    // the 3 x 3 density stencil; ghost rows beyond the walls repeat the wall row
    const int jU = top ? j : j + 1, jD = bot ? j : j - 1;

    // reference densities of this row and of the rows the stencil reaches
    const double rAj = rA0 + rAs * j;
    const double szref = rAs * (double)(jU - jD) * (1.0 / 6.0);  // species A

    // the full densities of this row's pulled state, on request (FP64: the
    // adjoint's recompute of a segment), from the sums the ring holds
    if constexpr (sizeof(Real) == 8) {
      if (a.dens && act) {
        const int64_t n = (int64_t)j * Lx + x;
        a.dens[n] = rAj + (double)ring[j & 3][0][c];
        a.dens[(int64_t)Lx * Lz + n] = (rho0 - rAj) + (double)ring[j & 3][1][c];
      }
    }

    // sample of f(t) (sampling modes), formed from the stencil the collision
    // reads (the arithmetic shares nothing with the collision) and stored
    // before it, which keeps the sample out of the collision's registers
    // the stencil: the sample reads its own before the collision's (this
    // kernel is bound by its memory traffic, not by LDS; a stencil kept across
    // the sample would cost registers, and in FP64 an occupancy step)
    auto stencil = [&]() {
      return load_stencil(ring[jU & 3][0], ring[j & 3][0], ring[jD & 3][0], ring[jU & 3][1],
                          ring[j & 3][1], ring[jD & 3][1], c);
    };
    if constexpr (MODE != kStep) {
      if (wave_act) {
        Real dp = (Real)0;
        if (act) {
          const bool vel = (flags & FNLB_SAMPLE_VELOCITY) != 0;
          const NodeSample<Real> smp = sample_of<Real, DT, Store>(
              stencil(), cur, srow, P.G, vel);
          store_sample(SD, a.watchdog, j, x, smp, vel);
          dp = smp.dp;
        }
        store_pressure_part(SD, j, (X0 >> 6) + wv, dp);
      }
    }
    const Stencil<DT> st = stencil();

    if constexpr (MODE != kSampleOnly) {
     if (wave_act) {
      Real dA[9], dB[9];
#pragma unroll
      for (int l = 0; l < 9; ++l) {
        dA[l] = (Real)cur[l];
        dB[l] = (Real)cur[9 + l];
      }
      node_update<Real, DT>(P, flags, top, bot, rAj, rho0, szref, st, dA, dB, gA0, gA1, gB0, gB1);

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
        emit(0, dA, P.shA1, P.shA5);
        emit(1, dB, -P.shA1, -P.shA5);
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
