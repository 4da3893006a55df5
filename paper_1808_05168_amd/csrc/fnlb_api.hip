// Host runtime of the fnlb library: parameter validation, the buffer plan,
// replica and work-item tables, the per-step launch sequence and the
// synchronous read/write calls of the C ABI (include/fnlb.h).
#include "fnlb.h"
#include "fnlb_device.hpp"
#include "fnlb_fft.hpp"
#include "fnlb_internal.hpp"
#include "fnlb_state.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace fnlb;

// The static workspace of fnlb_init_static_work: one array per device, part
// of the library's code object, held until the process ends.  In host code
// `scratch` names a host-side stand-in, not device memory; its device address
// comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is handed to kernels.
static __device__ __align__(256) char scratch[FNLB_STATIC_WORK_BYTES];

namespace {

constexpr size_t kAlign = 256;
// option bits that choose how the steps are launched, not what they compute
constexpr int kExecFlags = FNLB_NO_GRAPH | FNLB_TWO_STEP | FNLB_ONE_STEP;
size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }
bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Largest lattice dimension the observable kernels hold in LDS (64 KiB of
// complex doubles per row or column).
constexpr int kMaxDim = 4096;
// the row transform reads a sample plane through 32-bit byte offsets
static_assert((int64_t)kMaxDim * kMaxDim * 8 < ((int64_t)1 << 32), "sample plane offsets");
// Largest non-power-of-two dimension (direct transform, quadratic cost).
constexpr int kMaxDirect = 2048;
// Complex entries of the column-pass LDS tile.
constexpr int kColTile = 2048;  // complex values per column-transform tile (32 KiB)
constexpr int kRowGroup = 1024;  // complex values per row-transform block (short rows share)
// samples per column pass: the row passes of up to this many samples keep
// their spectra, and one column pass adds them all, reading and writing the
// FP64 sums once instead of once per sample
constexpr int kSpecSlots = 16;
constexpr int kTransformThreads = 256;  // threads of a transform block (at least one per row)
// lengths the wavefront transforms take
constexpr bool wave_fft_len(int n) { return n >= kFftMin && n <= kFftMax && (n & (n - 1)) == 0; }

// The two-step kernel takes FP32-deviation storage and whole rows of at most
// kTBLanes columns.
bool two_step_fits(const fnlb_replica_params* reps, int n_rep, int precision) {
  if (precision != FNLB_FP32_DEV) return false;
  for (int r = 0; r < n_rep; ++r)
    if (reps[r].Lx > kTBLanes) return false;
  return true;
}

// lanes per two-step work item: the row length rounded up to a power of two, at
// least one wavefront
int tb_lwidth(int Lx) {
  int lw = 6;
  while ((1 << lw) < Lx) ++lw;
  return lw;
}

int validate(const fnlb_replica_params* reps, int32_t n_rep, const fnlb_options* opt) {
  if (!reps || !opt || n_rep <= 0) return FNLB_EINVAL;
  if (opt->precision != FNLB_FP64 && opt->precision != FNLB_FP32_DEV) return FNLB_EINVAL;
  if (opt->sample_every < 0 || opt->chunk_rows < 0) return FNLB_EINVAL;
  if (opt->flags &
      ~(FNLB_ASTAR | FNLB_WALL_UZ_FIX | FNLB_NOISE_LOC | FNLB_FORCE_LITERAL | FNLB_NO_GRAPH |
        FNLB_SAMPLE_VELOCITY | FNLB_TWO_STEP | FNLB_ONE_STEP))
    return FNLB_EINVAL;
  if ((opt->flags & FNLB_TWO_STEP) && (opt->flags & FNLB_ONE_STEP)) return FNLB_EINVAL;
  if ((opt->flags & FNLB_TWO_STEP) && !two_step_fits(reps, n_rep, opt->precision))
    return FNLB_EINVAL;
  for (int r = 0; r < n_rep; ++r) {
    const fnlb_replica_params& p = reps[r];
    if (p.Lx < 2 || p.Lz < 2 || p.Lx > kMaxDim || p.Lz > kMaxDim) return FNLB_EINVAL;
    const bool p2 = is_pow2(p.Lx) && is_pow2(p.Lz);
    if (!p2 && (p.Lx > kMaxDirect || p.Lz > kMaxDirect)) return FNLB_EINVAL;
    if ((int64_t)p.Lx * p.Lz >= (int64_t)1 << 31) return FNLB_EINVAL;
    if (!(p.rho0 > 0) || !(p.kT >= 0) || !(p.G >= 0) || !std::isfinite(p.kT) ||
        !std::isfinite(p.G) || !std::isfinite(p.rho0))
      return FNLB_EINVAL;
    const double taus[5] = {p.tau_d, p.tau_s, p.tau_e, p.tau_q, p.tau_eps};
    for (double t : taus)
      if (!(t > 0.5) || !std::isfinite(t)) return FNLB_EINVAL;
    if (!(std::fabs(p.grad_c0) * p.Lz < 1.0)) return FNLB_EINVAL;
  }
  return FNLB_OK;
}

// The buffer plan: every offset the kernels use.
struct Plan {
  std::vector<RepInfo> info;
  std::vector<Item> items;
  std::vector<RowRef> rows;  // rows and column tiles of the block transforms
  std::vector<ColRef> cols;
  std::vector<RowTask> frows;  // and of the wavefront transforms (8 to 512 points)
  std::vector<ColTask> fcols;
  size_t store_size = 0;
  size_t state_half = 0;  // bytes of one state copy
  size_t state_bytes = 0, accum_bytes = 0, work_bytes = 0;
  // work-buffer offsets (bytes)
  size_t o_bm = 0;  // FP64 Box-Muller tables
  size_t o_rowc = 0;                 // per-row sample constants of every replica
  std::vector<size_t> rowc_at;       // byte offset of each replica's rows there
  size_t o_reps = 0, o_items = 0, o_rows = 0, o_cols = 0, o_frows = 0, o_fcols = 0, o_misc = 0,
         o_tw = 0, o_fields = 0, o_spec = 0, o_ppart = 0;
  size_t item_capacity = 0;  // items the work buffer holds (row ranges of one row)
  int max_lx = 0, max_lz = 0, max_col_lds = 0, max_row_lds = 0, chunk = 0;
  int n_pairs = 1;  // complex row transforms per row: (dc, drho) [, (Ux, Uz)]
  // samples whose row spectra and pressure parts are kept before one column
  // pass adds them all (slots of spec_slot complex pairs of the storage type
  // and ppart_slot doubles)
  int spec_slots = 1;
  size_t spec_slot = 0, ppart_slot = 0;
  // the two-step kernel: eligibility, its blocks of work items, their capacity
  bool tb_ok = false;
  std::vector<PackItem> pitems;
  size_t pitem_capacity = 0;
  size_t o_pitems = 0;
};

// work items for a row-range length: (replica, row range, segment), with
// neighbouring segments of the same rows adjacent
void make_items(Plan& P, int chunk) {
  P.chunk = chunk;
  P.items.clear();
  for (size_t r = 0; r < P.info.size(); ++r) {
    const RepInfo& R = P.info[r];
    const int nseg = (R.Lx + kSeg - 1) / kSeg;
    for (int j0 = 0; j0 < R.Lz; j0 += chunk)
      for (int s = 0; s < nseg; ++s)
        // every other row range marches downwards, so that neighbouring ranges
        // read their shared boundary rows at the same time (one of the two
        // reads then hits L2)
        P.items.push_back(Item{(int32_t)r, s, j0, std::min(R.Lz, j0 + chunk),
                               ((j0 / chunk) & 1) ? -1 : 1});
  }
}

// Work items of the two-step kernel for a row-range length: per replica its
// row ranges (alternating march direction, as for the one-step kernel), packed
// kTBLanes >> lwidth to a block among replicas of the same lane width.  A
// block's iteration count is its longest item's: the first-step rows (the
// range plus two rows on each side, clipped at the walls) and three more
// (the second step of a row runs three iterations after its first).
void make_pitems(Plan& P, int chunk) {
  P.pitems.clear();
  if (!P.tb_ok) return;
  for (int lw = 6; (1 << lw) <= kTBLanes; ++lw) {
    const int per_block = kTBLanes >> lw;
    PackItem cur{};
    cur.lwidth = lw;
    for (size_t r = 0; r < P.info.size(); ++r) {
      const RepInfo& R = P.info[r];
      if (tb_lwidth(R.Lx) != lw) continue;
      for (int j0 = 0; j0 < R.Lz; j0 += chunk) {
        const int j1 = std::min(R.Lz, j0 + chunk);
        const int dir = ((j0 / chunk) & 1) ? -1 : 1;
        const int alo = std::max(j0 - 2, 0), ahi = std::min(j1 + 2, R.Lz);
        const int niter = dir > 0 ? j1 + 3 - alo : ahi - j0 + 3;
        const int k = cur.nsub++;
        cur.rep[k] = (int32_t)r;
        cur.j0[k] = j0;
        cur.j1[k] = j1;
        cur.dir[k] = dir;
        // the kernel runs two iterations per loop trip
        cur.niter = std::max(cur.niter, (niter + 1) & ~1);
        if (cur.nsub == per_block) {
          P.pitems.push_back(cur);
          cur = PackItem{};
          cur.lwidth = lw;
        }
      }
    }
    if (cur.nsub > 0) P.pitems.push_back(cur);
  }
}

// Row-range lengths found by fnlb_autotune, per precision and set of lattice
// shapes, for the life of the process.
std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;

std::string tune_key(const fnlb_replica_params* reps, int n_rep, int precision) {
  std::map<std::pair<int, int>, int> shapes;
  for (int r = 0; r < n_rep; ++r) ++shapes[{reps[r].Lx, reps[r].Lz}];
  std::string k = std::to_string(precision);
  for (const auto& e : shapes)
    k += "|" + std::to_string(e.first.first) + "x" + std::to_string(e.first.second) + "*" +
         std::to_string(e.second);
  return k;
}

// (a negative value: that many rows with the two-step kernel)
// The tuning file: a header line, comment lines starting with '#', and one
// line per entry,
// "<device architecture>\t<precision|shapes>\t<rows, negative for two steps>".
constexpr char kTuneMagic[] = "fnlb-tune 1";

// the current device's architecture name (e.g. gfx950:sramecc+:xnack-)
std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  return std::string(prop.gcnArchName);
}

int cached_chunk(const fnlb_replica_params* reps, int n_rep, int precision) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune_cache.find(tune_key(reps, n_rep, precision));
  return it == g_tune_cache.end() ? 0 : it->second;
}

int auto_chunk(const fnlb_replica_params* reps, int n_rep) {
  int64_t seg_rows = 0;
  for (int r = 0; r < n_rep; ++r)
    seg_rows += (int64_t)((reps[r].Lx + kSeg - 1) / kSeg) * reps[r].Lz;
  // aim for about 1024 blocks (four per compute unit) when the lattice allows;
  // small lattices get single-row items so that they still spread over the chip
  const int64_t c = seg_rows / 1024;
  int chunk = 1;
  while (chunk * 2 <= c && chunk < 64) chunk *= 2;
  return chunk;
}

// The FP64 Box-Muller tables (see BmTables), computed in extended precision.
void fill_bm_tables(BmTables& T) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < 256; ++j) {
    const long double ang = 2.0L * pi * (long double)j / 256.0L;
    T.sc[j] = make_double2((double)sinl(ang), (double)cosl(ang));
  }
  for (int j = 0; j < 96; ++j) {
    if (j == 31 || j == 32) {
      T.lg[j] = make_double2(1.0, 0.0);
      continue;
    }
    const long double b = 0.75L + ((long double)j + 0.5L) / 128.0L;
    int ex;
    const double m = std::frexp((double)(1.0L / b), &ex);  // 20 significant bits
    const double c = std::ldexp(std::nearbyint(std::ldexp(m, 20)), ex - 20);
    T.lg[j] = make_double2(c, (double)logl((long double)c));
  }
  const long double ln2 = 0.693147180559945309417232121458176568L;
  int ex;
  const double m = std::frexp((double)ln2, &ex);  // 42 significant bits
  const double hi = std::ldexp(std::nearbyint(std::ldexp(m, 42)), ex - 42);
  T.ln2 = make_double2(hi, (double)(ln2 - (long double)hi));
}

void make_plan(const fnlb_replica_params* reps, int n_rep, const fnlb_options* opt, Plan& P,
               int spec_slots) {
  P.store_size = opt->precision == FNLB_FP64 ? 8 : 4;
  P.spec_slots = spec_slots;
  P.tb_ok = two_step_fits(reps, n_rep, opt->precision);
  int chunk = opt->chunk_rows;
  if (chunk <= 0) chunk = std::abs(cached_chunk(reps, n_rep, opt->precision));
  if (chunk <= 0) chunk = auto_chunk(reps, n_rep);
  P.info.assign(n_rep, RepInfo{});
  int64_t state_elems = 0, field_d = 0, spec_c = 0, acc_d = 0, ppart_d = 0, tw_c = 0,
          rowc_c = 0;
  P.rowc_at.assign(n_rep, 0);
  // sampled fields: (delta c, delta rho) and, on request, (U_x, U_z)
  const int nf = n_fields(opt->flags);
  P.n_pairs = nf / 2;
  const int64_t elem_align = (int64_t)(kAlign / P.store_size);
  for (int r = 0; r < n_rep; ++r) {
    const fnlb_replica_params& p = reps[r];
    RepInfo& R = P.info[r];
    R.Lx = p.Lx;
    R.Lz = p.Lz;
    R.pitch = (p.Lx + kRowAlign - 1) / kRowAlign * kRowAlign;
    R.plane = ((int64_t)p.Lz * R.pitch + elem_align - 1) / elem_align * elem_align;
    R.state_off = state_elems;
    state_elems += 18 * R.plane;
    const int nkx = p.Lx / 2 + 1;
    // 256-byte aligned (paired loads of the row pass)
    field_d = (field_d + 256 / P.store_size - 1) / (256 / P.store_size) * (256 / P.store_size);
    R.field_off = field_d;
    field_d += (int64_t)nf * p.Lz * p.Lx;  // the pairs
    // row spectra (complex pairs of the storage type) in whole 128-byte lines
    // per row, so that the column pass reads each tile row as aligned lines
    const int line = 128 / (2 * (int)P.store_size);
    R.spitch = (nkx + line - 1) / line * line;
    spec_c = (spec_c + line - 1) / line * line;
    R.spec_off = spec_c;
    spec_c += (int64_t)nf * p.Lz * R.spitch;
    R.acc_off = acc_d;
    acc_d += 3LL * nf * p.Lz * nkx;
    R.pacc_off = acc_d;
    acc_d += 2 + p.Lz;
    R.ppart_off = ppart_d;
    ppart_d += (int64_t)p.Lz * pressure_parts(p.Lx);
    R.tw_off = tw_c;
    tw_c += p.Lx + p.Lz;
    P.rowc_at[r] = (size_t)rowc_c * P.store_size;
    rowc_c += (int64_t)kRowConsts * p.Lz;
    R.flags = opt->flags;
    R.pow2 = is_pow2(p.Lx) && is_pow2(p.Lz);
    R.seed_lo = (uint32_t)p.seed;
    R.seed_hi = (uint32_t)(p.seed >> 32);
    R.rho0 = p.rho0;
    R.grad = p.grad_c0;
    R.G = p.G;
    R.ne_coef = p.grad_c0 / 3.0;
    R.rA_mid = p.rho0 * (0.5 - 0.5 * (p.Lz - 1) * p.grad_c0);
    R.rA_step = p.rho0 * p.grad_c0;
    const double lam_d = 1.0 / p.tau_d, lam_s = 1.0 / p.tau_s, lam_e = 1.0 / p.tau_e,
                 lam_q = 1.0 / p.tau_q, lam_p = 1.0 / p.tau_eps;
    const double lam[9] = {0.0, lam_d, lam_d, lam_e, lam_s, lam_s, lam_q, lam_q, lam_p};
    // N_a = sum_l w_l T_al^2 of the basis of Table I
    const double N[9] = {1.0, 1.0 / 3, 1.0 / 3, 4.0, 4.0 / 9, 1.0 / 9, 2.0 / 3, 2.0 / 3, 16.0};
    for (int q = 0; q < 9; ++q) {
      R.lam[q] = lam[q];
      R.fac[q] = 1.0 - 0.5 * lam[q];
    }
    if (opt->flags & FNLB_FORCE_LITERAL) R.fac[1] = R.fac[2] = 1.0;
    // Eq. (22): <xi xi>_{1,2} = (2 - lam_d) lam_d kT rho^A rho^B / rho;
    // Eq. (23): <xi^S xi^S>_a = 3 (2 - lam_a) lam_a N_a kT rho^S, a = 3..8;
    // reference densities rho_bar/2 each ("hom" noise).
    const double rbar = 0.5 * p.rho0;
    std::memset(R.sig, 0, sizeof(R.sig));
    std::memset(R.sig_base, 0, sizeof(R.sig_base));
    R.sig_base[1] = std::sqrt((2.0 - lam_d) * lam_d * p.kT);
    R.sig[0][1] = R.sig[1][1] = R.sig_base[1] * std::sqrt(rbar * rbar / p.rho0);
    for (int q = 3; q < 9; ++q) {
      R.sig_base[q] = std::sqrt(3.0 * (2.0 - lam[q]) * lam[q] * N[q] * p.kT);
      R.sig[0][q] = R.sig[1][q] = R.sig_base[q] * std::sqrt(rbar);
    }
    R.p_ref = p.rho0 / 3.0 + p.G * p.rho0 * p.rho0 / 12.0;
    R.inv_norm = 1.0 / std::sqrt((double)p.Lx * (double)p.Lz);
    P.max_lx = std::max(P.max_lx, p.Lx);
    P.max_lz = std::max(P.max_lz, p.Lz);
  }
  make_items(P, chunk);
  make_pitems(P, chunk);
  P.item_capacity = 0;
  P.pitem_capacity = 0;
  for (const RepInfo& R : P.info) {
    P.item_capacity += (size_t)((R.Lx + kSeg - 1) / kSeg) * R.Lz;
    if (P.tb_ok) P.pitem_capacity += (size_t)R.Lz;  // at most one block per row
  }
  // rows and column tiles of the transforms: the wavefront transforms for
  // lengths of 8 to 512 points (powers of two), the block transforms (longer
  // rows or columns, or direct sums for other lengths) otherwise
  P.rows.clear();
  P.cols.clear();
  P.frows.clear();
  P.fcols.clear();
  P.max_col_lds = 0;
  P.max_row_lds = 0;
  for (int r = 0; r < n_rep; ++r) {
    const RepInfo& R = P.info[r];
    const int nkx = R.Lx / 2 + 1;
    if (wave_fft_len(R.Lx)) {
      // rows per wavefront: two halves of 512 / Lx rows for float pairs, one
      // for double pairs
      const int per = (P.store_size == 4 ? 2 : 1) * kFftMax / R.Lx;
      for (int j = 0; j < R.Lz; j += per)
        P.frows.push_back(RowTask{r, j, std::min(per, R.Lz - j), 0});
    } else {
      // short power-of-two rows are transformed several to a block
      const int per = R.pow2 ? std::min(kTransformThreads, std::max(1, kRowGroup / R.Lx)) : 1;
      for (int j = 0; j < R.Lz; j += per) {
        const int nr = std::min(per, R.Lz - j);
        P.rows.push_back(RowRef{r, j, nr, 0});
        // the rows, plus N/2 twiddles for the power-of-two FFT
        P.max_row_lds = std::max(P.max_row_lds, nr * R.Lx + (R.pow2 ? R.Lx / 2 : 0));
      }
    }
    if (wave_fft_len(R.Lz)) {
      const int tile = 4 * kFftMax / R.Lz;  // columns per block
      for (int f = 0; f < nf; ++f)
        for (int k0 = 0; k0 < nkx; k0 += tile)
          P.fcols.push_back(ColTask{r, f, k0, std::min(tile, nkx - k0)});
      continue;
    }
    int lt = 0;  // tile of 2^lt columns: at most 16 and at most kColTile values
    while (lt < 4 && (2 << lt) * R.Lz <= kColTile) ++lt;
    const int tile = 1 << lt;
    for (int f = 0; f < nf; ++f)
      for (int k0 = 0; k0 < nkx; k0 += tile) {
        const int nc = std::min(tile, nkx - k0);
        P.cols.push_back(ColRef{r, f, k0, nc, lt});
        // the tile, plus Lz/2 twiddles for the power-of-two FFT
        P.max_col_lds = std::max(P.max_col_lds, tile * R.Lz + (R.pow2 ? R.Lz / 2 : 0));
      }
  }
  P.state_half = align_up((size_t)state_elems * P.store_size);
  P.state_bytes = 2 * P.state_half;
  P.accum_bytes = align_up((size_t)acc_d * 8);
  size_t o = 0;
  P.o_reps = o;
  o = align_up(o + P.info.size() * sizeof(RepInfo));
  P.o_items = o;
  o = align_up(o + P.item_capacity * sizeof(Item));
  P.o_pitems = o;
  o = align_up(o + P.pitem_capacity * sizeof(PackItem));
  P.o_rows = o;
  o = align_up(o + P.rows.size() * sizeof(RowRef));
  P.o_cols = o;
  o = align_up(o + P.cols.size() * sizeof(ColRef));
  P.o_frows = o;
  o = align_up(o + P.frows.size() * sizeof(RowTask));
  P.o_fcols = o;
  o = align_up(o + P.fcols.size() * sizeof(ColTask));
  P.o_misc = o;  // int64 time base + int32 watchdog
  o = align_up(o + 16);
  P.o_bm = o;
  o = align_up(o + sizeof(BmTables));
  P.o_rowc = o;
  o = align_up(o + (size_t)rowc_c * P.store_size);
  P.o_tw = o;
  o = align_up(o + (size_t)tw_c * 16);
  P.o_fields = o;
  o = align_up(o + (size_t)field_d * P.store_size);
  P.spec_slot = (size_t)spec_c;  // whole 128-byte lines
  P.ppart_slot = (size_t)ppart_d;
  P.o_spec = o;
  o = align_up(o + P.spec_slots * P.spec_slot * 2 * P.store_size);
  P.o_ppart = o;
  o = align_up(o + P.spec_slots * P.ppart_slot * 8);
  P.work_bytes = o;
}

// Device addresses of the tables the replicas share (Box-Muller) or own (row
// constants) in the work buffer at `work`.
void set_table_pointers(Plan& P, char* work) {
  for (size_t r = 0; r < P.info.size(); ++r) {
    P.info[r].bm = (const BmTables*)(work + P.o_bm);
    P.info[r].rowc = work + P.o_rowc + P.rowc_at[r];
  }
}

}  // namespace

struct fnlb_handle {
  std::vector<fnlb_replica_params> reps;
  fnlb_options opt{};
  Plan plan;
  char* state = nullptr;
  char* accum = nullptr;
  char* work = nullptr;
  hipStream_t stream = nullptr;
  int cur = 0;           // which state copy holds f(t)
  int64_t t = 0;         // current time
  int64_t t_dev = 0;     // value held by the device time base
  int64_t nsamples = 0;
  int error = FNLB_OK;   // sticky error
  // sampling periods captured as graphs, per parity of the starting copy:
  // graph[0] holds one period; when sampling, graph[1] holds kgraph periods
  // and graph[2] two, whose samples fill the spectrum slots in turn and share
  // one column pass at the end (a column pass reads and writes every FP64 sum
  // once, whatever number of samples it adds).  In them the transforms of
  // each sample run on a branch of their own (captured from obs_stream)
  // beside the plain steps that follow.
  hipStream_t cap_stream = nullptr, obs_stream = nullptr;
  hipEvent_t ev_fork[kSpecSlots] = {}, ev_join[kSpecSlots] = {};
  hipGraphExec_t graph[3][2] = {};  // [kind][parity]
  int graph_launches[3] = {};       // kernel launches of the state in each kind
  int kgraph = 0;                   // periods of graph[1] (0: no such graph)
  int pending = 0;  // samples in the spectrum slots that no column pass has added yet
  int64_t period = 0;
  bool two_step = false;    // pairs of steps run in the two-step kernel
  int static_dev = -1;   // device whose static workspace this handle holds, or -1
  // the last forward sweep of a misfit, kept for its reverse sweep
  struct {
    bool valid = false;
    const void* d_adj = nullptr;
    size_t bytes = 0;
    int64_t horizon = 0, t0 = 0, nsamp = 0;
    int32_t K = 0, field = 0;
    bool pressure = false;
    bool last_seg_kept = false;  // the segment buffers hold the last segment's states
  } adj;

  RepInfo* d_reps() { return (RepInfo*)(work + plan.o_reps); }
  Item* d_items() { return (Item*)(work + plan.o_items); }
  PackItem* d_pitems() { return (PackItem*)(work + plan.o_pitems); }
  RowRef* d_rows() { return (RowRef*)(work + plan.o_rows); }
  ColRef* d_cols() { return (ColRef*)(work + plan.o_cols); }
  RowTask* d_frows() { return (RowTask*)(work + plan.o_frows); }
  ColTask* d_fcols() { return (ColTask*)(work + plan.o_fcols); }
  int64_t* d_time() { return (int64_t*)(work + plan.o_misc); }
  int32_t* d_watchdog() { return (int32_t*)(work + plan.o_misc + 8); }
  double2* d_tw() { return (double2*)(work + plan.o_tw); }
  void* d_fields() { return (void*)(work + plan.o_fields); }
  void* d_spec(int slot = 0) {
    return work + plan.o_spec + (size_t)slot * plan.spec_slot * 2 * plan.store_size;
  }
  double* d_ppart(int slot = 0) {
    return (double*)(work + plan.o_ppart) + (size_t)slot * plan.ppart_slot;
  }
  char* state_copy(int k) { return state + (size_t)k * plan.state_half; }
};

namespace {

int dev_err(fnlb_handle* h, hipError_t e) {
  if (e == hipSuccess) return FNLB_OK;
  h->error = FNLB_EDEVICE;
  return FNLB_EDEVICE;
}

StepArgs step_args(fnlb_handle* h, int64_t t_off, int slot = 0) {
  StepArgs a{};
  a.reps = h->d_reps();
  a.items = h->d_items();
  a.n_items = (int)h->plan.items.size();
  const int nb = (a.n_items + 7) / 8 * 8;
  a.n_blocks = nb;
  a.chunk_rows = h->plan.chunk;
  a.state_in = h->state_copy(h->cur);
  a.state_out = h->state_copy(1 - h->cur);
  a.t_base = h->d_time();
  a.t_off = t_off;
  a.fields = h->d_fields();
  a.ppart = h->d_ppart(slot);
  a.watchdog = h->d_watchdog();
  return a;
}

Step2Args step2_args(fnlb_handle* h, int64_t t_off, int slot = 0) {
  Step2Args a{};
  a.reps = h->d_reps();
  a.items = h->d_pitems();
  a.n_items = (int)h->plan.pitems.size();
  a.n_blocks = (a.n_items + 7) / 8 * 8;
  a.state_in = h->state_copy(h->cur);
  a.state_out = h->state_copy(1 - h->cur);
  a.t_base = h->d_time();
  a.t_off = t_off;
  a.fields = h->d_fields();
  a.ppart = h->d_ppart(slot);
  a.watchdog = h->d_watchdog();
  return a;
}

// Whether the launch at time t (n steps still to go) takes two steps: the
// handle runs the two-step kernel, two steps remain, and t + 1 is not a
// sample time (a sample of f(t) itself is taken by the two-step kernel).
bool pair_at(const fnlb_handle* h, int64_t t, int64_t n) {
  const int every = h->opt.sample_every;
  return h->two_step && n >= 2 && !(every > 0 && (t + 1) % every == 0);
}

// One launch of the state from time t: two steps or one, sampling f(t) when t
// is a sample time (its pressure sums into spectrum slot `slot`); returns the
// steps taken (0 on error, e set).
int launch_state(fnlb_handle* h, int64_t t_off, bool pair, bool smp, int slot, hipStream_t s,
                 hipError_t& e) {
  if (pair) {
    e = launch_step2(smp ? kStepSample : kStep, step2_args(h, t_off, slot), s);
    return e == hipSuccess ? 2 : 0;
  }
  e = launch_step(h->opt.precision, smp ? kStepSample : kStep, step_args(h, t_off, slot), s);
  return e == hipSuccess ? 1 : 0;
}

// Row passes of one sample into spectrum slot `slot`: the sampled pairs the
// step stored are transformed along x (the step has put the sample's pressure
// sums in the slot).
hipError_t observe_rows(fnlb_handle* h, hipStream_t s, int slot) {
  const Plan& P = h->plan;
  hipError_t e = launch_row_fft(h->d_reps(), h->d_frows(), (int)P.frows.size(), P.n_pairs,
                                h->opt.precision, h->d_fields(), h->d_spec(slot), h->d_tw(), s);
  if (e == hipSuccess)
    e = launch_row_transform(h->d_reps(), h->d_rows(), (int)P.rows.size(), P.n_pairs,
                             P.max_row_lds, h->opt.precision, h->d_fields(), h->d_spec(slot),
                             h->d_tw(), s);
  return e;
}

// Column passes over the samples in slots 0 .. nslots - 1, added to the
// accumulators (or to acc) in slot order.
hipError_t observe_cols(fnlb_handle* h, hipStream_t s, int nslots, double* acc = nullptr) {
  const Plan& P = h->plan;
  if (!acc) acc = (double*)h->accum;
  hipError_t e = launch_col_fft(h->d_reps(), h->d_fcols(), (int)P.fcols.size(),
                                h->opt.precision, h->d_spec(), nslots, P.spec_slot, acc,
                                h->d_tw(), h->d_ppart(), P.ppart_slot, s);
  if (e == hipSuccess)
    e = launch_col_transform(h->d_reps(), h->d_cols(), (int)P.cols.size(), P.max_col_lds,
                             h->opt.precision, h->d_spec(), nslots, P.spec_slot, acc,
                             h->d_tw(), h->d_ppart(), P.ppart_slot, s);
  return e;
}

// Structure-factor transforms and pressure reduction of one sample at once.
hipError_t observe(fnlb_handle* h, hipStream_t s, double* acc = nullptr) {
  hipError_t e = observe_rows(h, s, 0);
  if (e == hipSuccess) e = observe_cols(h, s, 1, acc);
  return e;
}

// The column pass of the samples still kept in the slots (fnlb_step leaves
// none behind, and a graph replay starts from the first slot).
hipError_t flush_samples(fnlb_handle* h) {
  hipError_t e = hipSuccess;
  if (h->pending > 0) e = observe_cols(h, h->stream, h->pending);
  h->pending = 0;
  return e;
}

void drop_graphs(fnlb_handle* h) {
  for (auto& gp : h->graph)
    for (auto& g : gp)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
}

// periods in a graph of kind `which` (0: one, 1: kgraph, 2: two)
int graph_periods(const fnlb_handle* h, int which) {
  return which == 0 ? 1 : which == 1 ? h->kgraph : 2;
}

// the kinds of graph a handle captures: one period; kgraph periods when kgraph
// > 1; two periods when kgraph > 2
bool graph_kind_used(const fnlb_handle* h, int which) {
  return which == 0 || (which == 1 && h->kgraph > 1) || (which == 2 && h->kgraph > 2);
}

// The graph for n steps from a period start: the most periods that n holds.
int graph_kind_for(const fnlb_handle* h, int64_t n) {
  if (graph_kind_used(h, 1) && n >= h->kgraph * h->period) return 1;
  if (graph_kind_used(h, 2) && n >= 2 * h->period) return 2;
  return 0;
}

// Captures `graph_periods(which)` periods of `period` steps starting at a
// period start, from state copy `parity`: the first step of each period
// samples when sampling is on, and the last node advances the device time
// counter by the steps of the graph.  Kernels read their time as counter +
// offset, so one graph serves every start.  The transforms of each sample form
// a branch that forks after the sampling step and joins before the next
// sampling step (which overwrites the sample buffer) or the last node: they
// read only the sample buffer and write only the spectra, pressure sums and
// accumulators, which no step touches.  The sample of period p keeps its row
// spectra in slot p, and the branch of the last sample runs the column pass
// over every slot of the graph.
hipError_t capture_periods(fnlb_handle* h, int which, int parity) {
  hipError_t e = hipSuccess;
  if (!h->cap_stream) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess && !h->obs_stream)
    e = hipStreamCreateWithFlags(&h->obs_stream, hipStreamNonBlocking);
  for (int k = 0; k < kSpecSlots && e == hipSuccess; ++k) {
    if (!h->ev_fork[k]) e = hipEventCreateWithFlags(&h->ev_fork[k], hipEventDisableTiming);
    if (e == hipSuccess && !h->ev_join[k])
      e = hipEventCreateWithFlags(&h->ev_join[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) return e;
  hipStream_t s = h->cap_stream;
  e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const bool sampling = h->opt.sample_every > 0;
  const int nper = graph_periods(h, which);
  const int64_t len = nper * h->period;
  const int saved = h->cur;
  h->cur = parity;
  hipError_t le = hipSuccess;
  int joins = -1;   // the branch that has yet to join (-1: none)
  int forked = -1;  // the sample whose branch has yet to be issued (-1: none)
  int launches = 0;
  // the transforms of the sample of period p, on the side stream from the
  // fork event recorded after its sampling step
  auto branch = [&](int p) {
    le = hipStreamWaitEvent(h->obs_stream, h->ev_fork[p], 0);
    if (le != hipSuccess) return;
    joins = p;
    le = observe_rows(h, h->obs_stream, p);
    if (le == hipSuccess && p == nper - 1) le = observe_cols(h, h->obs_stream, nper);
    // recorded even after a failed launch, so that the branch can join
    const hipError_t re = hipEventRecord(h->ev_join[p], h->obs_stream);
    if (le == hipSuccess) le = re;
  };
  for (int64_t k = 0; k < len && le == hipSuccess;) {
    const int per = (int)(k / h->period);
    // each period starts at a sample time and holds no other
    const bool smp = sampling && k % h->period == 0;
    if (smp && joins >= 0) {
      le = hipStreamWaitEvent(s, h->ev_join[joins], 0);
      joins = -1;
      if (le != hipSuccess) break;
    }
    const int took = launch_state(h, k, pair_at(h, k, len - k), smp, per, s, le);
    k += took > 0 ? took : 1;
    ++launches;
    if (le == hipSuccess && forked >= 0) {
      branch(forked);
      forked = -1;
    }
    if (le == hipSuccess && smp) {
      le = hipEventRecord(h->ev_fork[per], s);
      // The branch is issued after the step that follows, when that step does
      // not sample: the runtime then keeps the chain of steps, the sampling
      // step's first successor, on one hardware queue, and the transforms
      // start beside a step that already holds the compute units (as kernel
      // traces show; captured first, the branch took the sampling step's
      // queue and each sample added two waits between queues).
      if (le == hipSuccess) {
        if (k < len && k % h->period != 0)
          forked = per;
        else
          branch(per);
      }
    }
    h->cur ^= 1;
  }
  h->graph_launches[which] = launches;
  // the branch always joins, so that the capture can end
  if (joins >= 0) {
    const hipError_t je = hipStreamWaitEvent(s, h->ev_join[joins], 0);
    if (le == hipSuccess) le = je;
  }
  if (le == hipSuccess) le = launch_advance_time(h->d_time(), len, s);
  h->cur = saved;
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  if (le != hipSuccess) e = le;
  hipGraphExec_t& x = h->graph[which][parity];
  if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  // upload it now, so that its first launch costs what every launch costs
  if (e == hipSuccess) e = hipGraphUpload(x, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return e;
}

// Graphs of up to this many steps are captured when the handle is created (and
// again after fnlb_autotune changes the work items), so that fnlb_step never
// captures or instantiates a graph; longer periods are captured on first use.
constexpr int64_t kPrecapturePeriod = 1024;

hipError_t prepare_graphs(fnlb_handle* h) {
  if ((h->opt.flags & FNLB_NO_GRAPH) || h->period > kPrecapturePeriod) return hipSuccess;
  hipError_t e = hipSuccess;
  for (int which = 0; which < 3; ++which)
    for (int parity = 0; parity < 2 && e == hipSuccess && graph_kind_used(h, which); ++parity)
      if (!h->graph[which][parity]) e = capture_periods(h, which, parity);
  return e;
}

// Runs one captured graph of kind `which` on the caller's stream.
int replay_periods(fnlb_handle* h, int which) {
  hipError_t e = hipSuccess;
  if (h->t_dev != h->t) {  // bring the device time counter to the period start
    e = launch_advance_time(h->d_time(), h->t - h->t_dev, h->stream);
    h->t_dev = h->t;
  }
  hipGraphExec_t& x = h->graph[which][h->cur];
  if (e == hipSuccess && !x) e = capture_periods(h, which, h->cur);
  if (e == hipSuccess) e = hipGraphLaunch(x, h->stream);
  if (e != hipSuccess) return dev_err(h, e);
  const int nper = graph_periods(h, which);
  h->t += nper * h->period;
  h->t_dev += nper * h->period;
  if (h->graph_launches[which] & 1) h->cur ^= 1;
  if (h->opt.sample_every > 0) h->nsamples += nper;
  return FNLB_OK;
}

int check_watchdog(fnlb_handle* h) {
  int32_t flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, h->d_watchdog(), 4, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return dev_err(h, e);
  if (flag) h->error = FNLB_EWATCHDOG;
  return h->error;
}

const double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
const int kCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int kCZ[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// Where f_l(x, j) of the current state is stored: link l of node
// (x - c_lx, j - c_lz), or link opp(l) of (x, j) itself when that source lies
// beyond a wall (mid-way bounce-back).  Returns the element index of species
// s in the replica's state block (tiled layout, state_index).
size_t pull_source(const RepInfo& R, int s, int l, int j, int x) {
  const int js = j - kCZ[l];
  if (js < 0 || js >= R.Lz) return state_index(9 * s + kOpp[l], j, x, R.pitch);
  int xs = x - kCX[l];
  if (xs < 0) xs += R.Lx;
  if (xs >= R.Lx) xs -= R.Lx;
  return state_index(9 * s + l, js, xs, R.pitch);
}

}  // namespace

extern "C" {

int fnlb_bytes_required(const fnlb_replica_params* reps, int32_t n_rep,
                        const fnlb_options* options, size_t* state_bytes, size_t* accum_bytes,
                        size_t* work_bytes) {
  const int rc = validate(reps, n_rep, options);
  if (rc) return rc;
  Plan P;
  make_plan(reps, n_rep, options, P, kSpecSlots);
  if (state_bytes) *state_bytes = P.state_bytes;
  if (accum_bytes) *accum_bytes = P.accum_bytes;
  if (work_bytes) *work_bytes = P.work_bytes;
  return FNLB_OK;
}

}  // extern "C"

namespace {

// fnlb_init over a given workspace; static_dev >= 0 marks the workspace as the
// static array of that device (released by fnlb_destroy).
int init_handle(const fnlb_replica_params* reps, int32_t n_rep, const fnlb_options* options,
                void* d_state, size_t state_bytes, void* d_accum, size_t accum_bytes,
                void* d_work, size_t work_bytes, void* hip_stream, int static_dev,
                int spec_slots, fnlb_handle** out) {
  if (!out) return FNLB_EINVAL;
  *out = nullptr;
  int rc = validate(reps, n_rep, options);
  if (rc) return rc;
  if (!d_state || !d_accum || !d_work) return FNLB_EINVAL;
  if (((uintptr_t)d_state | (uintptr_t)d_accum | (uintptr_t)d_work) % kAlign) return FNLB_EINVAL;
  fnlb_handle* h = new (std::nothrow) fnlb_handle();
  if (!h) return FNLB_ENOMEM;
  h->reps.assign(reps, reps + n_rep);
  h->opt = *options;
  make_plan(reps, n_rep, options, h->plan, spec_slots);
  const Plan& P = h->plan;
  if (state_bytes < P.state_bytes || accum_bytes < P.accum_bytes || work_bytes < P.work_bytes) {
    delete h;
    return FNLB_ENOMEM;
  }
  h->static_dev = static_dev;
  h->state = (char*)d_state;
  h->accum = (char*)d_accum;
  h->work = (char*)d_work;
  h->stream = (hipStream_t)hip_stream;
  h->period = h->opt.sample_every > 0 ? h->opt.sample_every : 16;
  // the long graph: as many sampling periods as there are slots, within the
  // steps captured in advance
  if (h->opt.sample_every > 0)
    h->kgraph = (int)std::min<int64_t>(P.spec_slots, kPrecapturePeriod / h->period);
  if (h->kgraph < 2) h->kgraph = 0;
  // the kernel: as requested, else as tuned for this shape (a negative cached
  // row count), else one step per launch
  if (h->opt.flags & FNLB_TWO_STEP)
    h->two_step = true;
  else if (!(h->opt.flags & FNLB_ONE_STEP) && options->chunk_rows <= 0)
    h->two_step = P.tb_ok && cached_chunk(reps, n_rep, options->precision) < 0;
  hipStream_t s = h->stream;
  hipError_t e = hipSuccess;
  auto up = [&](size_t off, const void* src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(h->work + off, src, n, hipMemcpyHostToDevice, s);
  };
  static_assert(sizeof(BmTables) % 16 == 0, "table layout");
  BmTables bm;
  fill_bm_tables(bm);
  up(P.o_bm, &bm, sizeof(BmTables));
  set_table_pointers(h->plan, h->work);
  up(P.o_reps, P.info.data(), P.info.size() * sizeof(RepInfo));
  up(P.o_items, P.items.data(), P.items.size() * sizeof(Item));
  up(P.o_pitems, P.pitems.data(), P.pitems.size() * sizeof(PackItem));
  up(P.o_rows, P.rows.data(), P.rows.size() * sizeof(RowRef));
  up(P.o_cols, P.cols.data(), P.cols.size() * sizeof(ColRef));
  up(P.o_frows, P.frows.data(), P.frows.size() * sizeof(RowTask));
  up(P.o_fcols, P.fcols.data(), P.fcols.size() * sizeof(ColTask));
  if (e == hipSuccess) e = launch_fill_zero(h->work + P.o_misc, 16, s);
  if (e == hipSuccess) e = launch_fill_zero(h->work + P.o_ppart, P.work_bytes - P.o_ppart, s);
  if (e == hipSuccess) e = launch_twiddles(h->d_reps(), P.info.data(), n_rep, h->d_tw(), s);
  if (e == hipSuccess)
    e = launch_row_consts(h->d_reps(), P.info.data(), n_rep, h->opt.precision, s);
  // state of rest on the imposed profile: all deviations zero
  if (e == hipSuccess) e = launch_fill_zero(h->state, P.state_bytes, s);
  if (e == hipSuccess) e = launch_fill_zero(h->accum, P.accum_bytes, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = prepare_graphs(h);
  if (e != hipSuccess) {
    h->static_dev = -1;  // the caller still owns the static workspace
    fnlb_destroy(h);
    return FNLB_EDEVICE;
  }
  *out = h;
  return FNLB_OK;
}

constexpr size_t kStaticWorkBytes = (size_t)FNLB_STATIC_WORK_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};
bool g_static_busy[kMaxDevices] = {};

}  // namespace

extern "C" {

int fnlb_init(const fnlb_replica_params* reps, int32_t n_rep, const fnlb_options* options,
              void* d_state, size_t state_bytes, void* d_accum, size_t accum_bytes,
              void* d_work, size_t work_bytes, void* hip_stream, fnlb_handle** out) {
  return init_handle(reps, n_rep, options, d_state, state_bytes, d_accum, accum_bytes, d_work,
                     work_bytes, hip_stream, -1, kSpecSlots, out);
}

int fnlb_init_static_work(const fnlb_replica_params* reps, int32_t n_rep,
                          const fnlb_options* options, void* d_state, size_t state_bytes,
                          void* d_accum, size_t accum_bytes, void* hip_stream,
                          fnlb_handle** out) {
  if (!out) return FNLB_EINVAL;
  *out = nullptr;
  const int rc = validate(reps, n_rep, options);
  if (rc) return rc;
  // the handle launches every step directly on the caller's stream: no graph,
  // stream or event of its own
  fnlb_options opt = *options;
  opt.flags |= FNLB_NO_GRAPH;
  // as many spectrum slots as the array holds (at least one)
  int slots = kSpecSlots;
  for (;; slots /= 2) {
    Plan P;
    make_plan(reps, n_rep, &opt, P, slots);
    if (P.work_bytes <= kStaticWorkBytes) break;
    if (slots == 1) return FNLB_ENOMEM;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return FNLB_EDEVICE;
  if (dev < 0 || dev >= kMaxDevices) return FNLB_EDEVICE;
  void* work = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_busy[dev]) return FNLB_ESTATE;  // one such handle per device
    if (!g_static_ptr[dev]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
        return FNLB_EDEVICE;
      g_static_ptr[dev] = p;
    }
    work = g_static_ptr[dev];
    g_static_busy[dev] = true;
  }
  const int r = init_handle(reps, n_rep, &opt, d_state, state_bytes, d_accum, accum_bytes, work,
                            kStaticWorkBytes, hip_stream, dev, slots, out);
  if (r != FNLB_OK) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    g_static_busy[dev] = false;
  }
  return r;
}

int fnlb_step(fnlb_handle* h, int64_t n) {
  if (!h || n < 0) return FNLB_EINVAL;
  if (h->error) return h->error;
  const int every = h->opt.sample_every;
  const bool use_graph = !(h->opt.flags & FNLB_NO_GRAPH);
  while (n > 0) {
    const int64_t t = h->t;
    // whole sampling periods from a period start replay a captured graph:
    // kgraph periods at once while that many remain, else two, else one
    if (use_graph && n >= h->period && t % h->period == 0 && (every == 0 || t >= 1)) {
      const int which = graph_kind_for(h, n);
      // the graphs fill the slots from the first
      const hipError_t fe = flush_samples(h);
      if (fe != hipSuccess) return dev_err(h, fe);
      const int rc = replay_periods(h, which);
      if (rc) return rc;
      n -= graph_periods(h, which) * h->period;
      continue;
    }
    const bool smp = every > 0 && t >= 1 && t % every == 0;
    hipError_t e = hipSuccess;
    const int took =
        launch_state(h, t - h->t_dev, pair_at(h, t, n), smp, h->pending, h->stream, e);
    if (e == hipSuccess && smp) {
      e = observe_rows(h, h->stream, h->pending++);
      if (e == hipSuccess && h->pending == h->plan.spec_slots) e = flush_samples(h);
    }
    if (e != hipSuccess) return dev_err(h, e);
    if (smp) ++h->nsamples;
    h->cur ^= 1;
    h->t += took;
    n -= took;
  }
  // every sample of the call is in the accumulators when it returns
  const hipError_t e = flush_samples(h);
  if (e != hipSuccess) return dev_err(h, e);
  return FNLB_OK;
}

int fnlb_autotune(fnlb_handle* h, int32_t steps_per_trial, int32_t* chunk_rows_out) {
  if (!h || steps_per_trial < 1) return FNLB_EINVAL;
  if (h->error) return h->error;
  Plan& P = h->plan;
  int max_lz = 0;
  for (const RepInfo& R : P.info) max_lz = std::max(max_lz, R.Lz);
  // candidates: (two-step kernel?, rows per work item).  Lengths above twice
  // the tallest lattice are left out: every replica then gets whole-lattice
  // items, the plan a shorter length already gives.  One length per kernel is
  // kept whatever the lattice (4 and 8), so that a short lattice still gives
  // each kernel a candidate (the two-step list starts at 8).
  struct Cand {
    bool two;
    int rows;
    float ms;  // per step, the faster of two rounds
  };
  std::vector<Cand> cands;
  if (!(h->opt.flags & FNLB_TWO_STEP))
    for (int c : {1, 2, 4, 8, 16, 32, 64, 128})
      if (c <= 2 * max_lz || c == 4) cands.push_back(Cand{false, c, 1e30f});
  if (P.tb_ok && !(h->opt.flags & FNLB_ONE_STEP))
    for (int c : {8, 16, 32, 64, 128, 256})
      if (c <= 2 * max_lz || c == 8) cands.push_back(Cand{true, c, 1e30f});
  if (cands.empty()) return FNLB_EINVAL;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // Two rounds over the candidates, each timed by its faster round, so that
  // neither the order of the trials (clocks still ramping up during the first
  // ones) nor one disturbed trial decides: neighbouring lengths often differ
  // by only a few percent.  Trial launches read the current copy and write
  // the spare one, so the state and the time are unchanged.
  auto upload = [&]() {
    hipError_t u = hipMemcpyAsync(h->d_items(), P.items.data(), P.items.size() * sizeof(Item),
                                  hipMemcpyHostToDevice, h->stream);
    if (u == hipSuccess && !P.pitems.empty())
      u = hipMemcpyAsync(h->d_pitems(), P.pitems.data(), P.pitems.size() * sizeof(PackItem),
                         hipMemcpyHostToDevice, h->stream);
    return u;
  };
  for (int round = 0; round < 2; ++round)
    for (Cand& cd : cands) {
      if (e != hipSuccess) break;
      make_items(P, cd.rows);
      make_pitems(P, cd.rows);
      e = upload();
      const int64_t off = h->t - h->t_dev;
      auto trial = [&]() {
        return cd.two ? launch_step2(kStep, step2_args(h, off), h->stream)
                      : launch_step(h->opt.precision, kStep, step_args(h, off), h->stream);
      };
      for (int w = 0; w < 2 && e == hipSuccess; ++w) e = trial();
      if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
      for (int k = 0; k < steps_per_trial && e == hipSuccess; ++k) e = trial();
      if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess) cd.ms = std::min(cd.ms, ms / (cd.two ? 2.0f : 1.0f));
    }
  Cand best{false, P.chunk, 1e30f};
  for (const Cand& cd : cands)
    if (cd.ms < best.ms) best = cd;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  make_items(P, best.rows);
  make_pitems(P, best.rows);
  P.chunk = best.rows;
  if (e == hipSuccess) e = upload();
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return dev_err(h, e);
  h->two_step = best.two;
  drop_graphs(h);
  e = prepare_graphs(h);
  if (e != hipSuccess) return dev_err(h, e);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[tune_key(h->reps.data(), (int)h->reps.size(), h->opt.precision)] =
        best.two ? -best.rows : best.rows;
  }
  if (chunk_rows_out) *chunk_rows_out = best.rows;
  return FNLB_OK;
}

int fnlb_tune_lookup(const fnlb_replica_params* reps, int32_t n_rep, int32_t precision,
                     int32_t* found, int32_t* steps_per_launch, int32_t* chunk_rows) {
  if (!reps || n_rep <= 0 || !found) return FNLB_EINVAL;
  const int v = cached_chunk(reps, n_rep, precision);
  *found = v != 0;
  if (steps_per_launch) *steps_per_launch = v < 0 ? 2 : 1;
  if (chunk_rows) *chunk_rows = std::abs(v);
  return FNLB_OK;
}

int fnlb_tune_cache_save(const char* path) {
  if (!path) return FNLB_EINVAL;
  const std::string arch = device_arch();
  // entries of other architectures already in the file are kept
  std::vector<std::string> keep;
  if (FILE* f = std::fopen(path, "r")) {
    char line[4096];
    while (std::fgets(line, sizeof line, f)) {
      std::string l(line);
      if (l.rfind(kTuneMagic, 0) == 0 || l.rfind("#", 0) == 0) continue;
      if (l.compare(0, arch.size() + 1, arch + "\t") != 0) keep.push_back(l);
    }
    std::fclose(f);
  }
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return FNLB_EINVAL;
  bool ok = std::fprintf(f, "%s\n# device %s\n", kTuneMagic, arch.c_str()) > 0;
  for (const std::string& l : keep) ok = ok && std::fputs(l.c_str(), f) >= 0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& e : g_tune_cache)
      ok = ok && std::fprintf(f, "%s\t%s\t%d\n", arch.c_str(), e.first.c_str(), e.second) > 0;
  }
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return FNLB_EINVAL;
  }
  return FNLB_OK;
}

int fnlb_tune_cache_load(const char* path) {
  if (!path) return FNLB_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return FNLB_EINVAL;
  const std::string arch = device_arch();
  char line[4096];
  bool first = true, ok = true;
  std::map<std::string, int> entries;
  while (std::fgets(line, sizeof line, f)) {
    std::string l(line);
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
    if (first) {
      ok = l == kTuneMagic;
      first = false;
      if (!ok) break;
      continue;
    }
    if (l.empty() || l[0] == '#') continue;  // comments
    const size_t a = l.find('\t'), b = l.rfind('\t');
    if (a == std::string::npos || b == a) {
      ok = false;
      break;
    }
    if (l.compare(0, a, arch) != 0) continue;  // tuned on another architecture
    char* end = nullptr;
    const long v = std::strtol(l.c_str() + b + 1, &end, 10);
    if (!end || *end != 0 || v == 0) {
      ok = false;
      break;
    }
    entries[l.substr(a + 1, b - a - 1)] = (int)v;
  }
  std::fclose(f);
  if (!ok || first) return FNLB_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& e : entries) g_tune_cache[e.first] = e.second;
  return FNLB_OK;
}

int fnlb_launch_config(const fnlb_handle* h, int32_t* steps_per_launch, int32_t* chunk_rows) {
  if (!h) return FNLB_EINVAL;
  if (steps_per_launch) *steps_per_launch = h->two_step ? 2 : 1;
  if (chunk_rows) *chunk_rows = h->plan.chunk;
  return FNLB_OK;
}

int fnlb_accumulate_structure_factor(fnlb_handle* h) {
  if (!h) return FNLB_EINVAL;
  if (h->error) return h->error;
  StepArgs a = step_args(h, h->t - h->t_dev);
  hipError_t e = launch_step(h->opt.precision, kSampleOnly, a, h->stream);
  if (e == hipSuccess) e = observe(h, h->stream);
  if (e != hipSuccess) return dev_err(h, e);
  ++h->nsamples;
  return FNLB_OK;
}

int fnlb_read_structure_factor(fnlb_handle* h, int32_t rep, int32_t field, double* sum_abs2,
                               double* sum_re, double* sum_im, int64_t* n_samples) {
  if (!h || rep < 0 || rep >= (int)h->reps.size() || field < 0 ||
      field >= n_fields(h->opt.flags))
    return FNLB_EINVAL;
  if (h->error) return h->error;
  const RepInfo& R = h->plan.info[rep];
  const int nkx = R.Lx / 2 + 1, Lz = R.Lz;
  const size_t plane = (size_t)Lz * nkx;
  const double* base = (const double*)h->accum + R.acc_off + (size_t)field * 3 * plane;
  // device layout [kind][k_x][k_z]; the caller's arrays are [k_z][k_x]
  std::vector<double> buf(3 * plane);
  hipError_t e = hipMemcpyAsync(buf.data(), base, 3 * plane * 8, hipMemcpyDeviceToHost,
                                h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return dev_err(h, e);
  double* dst[3] = {sum_abs2, sum_re, sum_im};
  for (int k = 0; k < 3; ++k)
    if (dst[k])
      for (int kx = 0; kx < nkx; ++kx)
        for (int kz = 0; kz < Lz; ++kz)
          dst[k][(size_t)kz * nkx + kx] = buf[k * plane + (size_t)kx * Lz + kz];
  if (n_samples) *n_samples = h->nsamples;
  return check_watchdog(h);
}

int fnlb_read_pressure(fnlb_handle* h, int32_t rep, double* sum_dP, double* sum_dP2,
                       double* profile_sum, int64_t* n_samples) {
  if (!h || rep < 0 || rep >= (int)h->reps.size()) return FNLB_EINVAL;
  if (h->error) return h->error;
  const RepInfo& R = h->plan.info[rep];
  std::vector<double> buf(2 + R.Lz);
  hipError_t e = hipMemcpyAsync(buf.data(), (const double*)h->accum + R.pacc_off,
                                buf.size() * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return dev_err(h, e);
  if (sum_dP) *sum_dP = buf[0];
  if (sum_dP2) *sum_dP2 = buf[1];
  if (profile_sum) std::memcpy(profile_sum, buf.data() + 2, (size_t)R.Lz * 8);
  if (n_samples) *n_samples = h->nsamples;
  return check_watchdog(h);
}

int fnlb_read_populations(fnlb_handle* h, int32_t rep, double* out) {
  if (!h || !out || rep < 0 || rep >= (int)h->reps.size()) return FNLB_EINVAL;
  if (h->error) return h->error;
  const RepInfo& R = h->plan.info[rep];
  const size_t ss = h->plan.store_size;
  const size_t block = 18 * (size_t)R.plane;
  std::vector<char> raw(block * ss);
  const char* src = h->state_copy(h->cur) + (size_t)R.state_off * ss;
  hipError_t e = hipMemcpyAsync(raw.data(), src, raw.size(), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return dev_err(h, e);
  const size_t n = (size_t)R.Lz * R.Lx;
  for (int s = 0; s < 2; ++s)
    for (int l = 0; l < 9; ++l)
      for (int j = 0; j < R.Lz; ++j) {
        const double rA = R.rA_mid + R.rA_step * j;
        const double ref = kW[l] * (s == 0 ? rA : R.rho0 - rA);
        for (int x = 0; x < R.Lx; ++x) {
          const size_t k = pull_source(R, s, l, j, x);
          const double d = ss == 8 ? ((const double*)raw.data())[k]
                                   : (double)((const float*)raw.data())[k];
          out[(size_t)(s * 9 + l) * n + (size_t)j * R.Lx + x] = ref + d;
        }
      }
  return FNLB_OK;
}

int fnlb_write_populations(fnlb_handle* h, int32_t rep, const double* in) {
  if (!h || !in || rep < 0 || rep >= (int)h->reps.size()) return FNLB_EINVAL;
  if (h->error) return h->error;
  const RepInfo& R = h->plan.info[rep];
  const size_t ss = h->plan.store_size;
  const size_t block = 18 * (size_t)R.plane;
  std::vector<char> raw(block * ss, 0);
  const size_t n = (size_t)R.Lz * R.Lx;
  for (int s = 0; s < 2; ++s)
    for (int l = 0; l < 9; ++l)
      for (int j = 0; j < R.Lz; ++j) {
        const double rA = R.rA_mid + R.rA_step * j;
        const double ref = kW[l] * (s == 0 ? rA : R.rho0 - rA);
        for (int x = 0; x < R.Lx; ++x) {
          const size_t k = pull_source(R, s, l, j, x);
          const double d = in[(size_t)(s * 9 + l) * n + (size_t)j * R.Lx + x] - ref;
          if (ss == 8)
            ((double*)raw.data())[k] = d;
          else
            ((float*)raw.data())[k] = (float)d;
        }
      }
  char* dst = h->state_copy(h->cur) + (size_t)R.state_off * ss;
  hipError_t e = hipMemcpyAsync(dst, raw.data(), raw.size(), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return dev_err(h, e);
}

int fnlb_reset_accumulators(fnlb_handle* h) {
  if (!h) return FNLB_EINVAL;
  if (h->error) return h->error;
  hipError_t e = launch_fill_zero(h->accum, h->plan.accum_bytes, h->stream);
  if (e != hipSuccess) return dev_err(h, e);
  h->nsamples = 0;
  return FNLB_OK;
}

int fnlb_reinit(fnlb_handle* h, const fnlb_replica_params* reps, int32_t n_rep) {
  if (!h || !reps) return FNLB_EINVAL;
  if (h->error) return h->error;
  if (n_rep != (int32_t)h->reps.size()) return FNLB_EINVAL;
  for (int r = 0; r < n_rep; ++r)
    if (reps[r].Lx != h->reps[r].Lx || reps[r].Lz != h->reps[r].Lz) return FNLB_EINVAL;
  const int rc = validate(reps, n_rep, &h->opt);
  if (rc) return rc;
  // same shapes and row ranges: the same buffer plan, work items, transform
  // tables and twiddles; only the replica table changes, so the captured
  // graphs stay valid
  fnlb_options o = h->opt;
  o.chunk_rows = h->plan.chunk;
  Plan P;
  make_plan(reps, n_rep, &o, P, h->plan.spec_slots);
  h->reps.assign(reps, reps + n_rep);
  h->plan.info = P.info;
  set_table_pointers(h->plan, h->work);
  h->adj.valid = false;
  const Plan& Q = h->plan;
  hipStream_t s = h->stream;
  hipError_t e = hipMemcpyAsync(h->work + Q.o_reps, Q.info.data(), Q.info.size() * sizeof(RepInfo),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_row_consts(h->d_reps(), Q.info.data(), n_rep, h->opt.precision, s);
  if (e == hipSuccess) e = launch_fill_zero(h->work + Q.o_misc, 16, s);
  if (e == hipSuccess) e = launch_fill_zero(h->work + Q.o_ppart, Q.work_bytes - Q.o_ppart, s);
  if (e == hipSuccess) e = launch_fill_zero(h->state, Q.state_bytes, s);
  if (e == hipSuccess) e = launch_fill_zero(h->accum, Q.accum_bytes, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_err(h, e);
  h->cur = 0;
  h->t = h->t_dev = 0;
  h->nsamples = 0;
  return FNLB_OK;
}

int fnlb_get_time(const fnlb_handle* h, int64_t* t) {
  if (!h || !t) return FNLB_EINVAL;
  *t = h->t;
  return FNLB_OK;
}

int fnlb_set_time(fnlb_handle* h, int64_t t) {
  if (!h || t < 0) return FNLB_EINVAL;
  if (h->error) return h->error;
  h->t = t;
  return FNLB_OK;
}

}  // extern "C"

namespace {

// Checkpoint image: this header, then the current state copy (raw stored
// values), then the accumulators.
struct CkptHeader {
  char magic[8];
  uint32_t version;
  int32_t precision, flags, sample_every, n_rep, reserved;
  int64_t t, nsamples;
  uint64_t state_bytes, accum_bytes, key;
};
constexpr char kCkptMagic[8] = {'F', 'N', 'L', 'B', 'C', 'K', 'P', 'T'};

// FNV-1a over everything that fixes the layout and the dynamics of a handle:
// replica parameters (seeds included), precision, physics flags, sampling.
uint64_t ckpt_key(const fnlb_handle* h) {
  uint64_t k = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) k = (k ^ c[i]) * 1099511628211ull;
  };
  for (const fnlb_replica_params& p : h->reps) {
    mix(&p.Lx, 4);
    mix(&p.Lz, 4);
    const double d[9] = {p.rho0, p.grad_c0, p.kT, p.G, p.tau_d, p.tau_s, p.tau_e, p.tau_q,
                         p.tau_eps};
    mix(d, sizeof d);
    mix(&p.seed, 8);
  }
  const int32_t o[3] = {h->opt.precision, h->opt.flags & ~kExecFlags, h->opt.sample_every};
  mix(o, sizeof o);
  return k;
}

}  // namespace

extern "C" {

int fnlb_checkpoint_bytes(const fnlb_handle* h, size_t* bytes) {
  if (!h || !bytes) return FNLB_EINVAL;
  *bytes = sizeof(CkptHeader) + h->plan.state_half + h->plan.accum_bytes;
  return FNLB_OK;
}

int fnlb_save(fnlb_handle* h, void* host_buf, size_t n) {
  if (!h || !host_buf) return FNLB_EINVAL;
  if (h->error) return h->error;
  const size_t need = sizeof(CkptHeader) + h->plan.state_half + h->plan.accum_bytes;
  if (n < need) return FNLB_ENOMEM;
  CkptHeader hd{};
  std::memcpy(hd.magic, kCkptMagic, 8);
  hd.version = 2;  // 2: tiled state layout
  hd.precision = h->opt.precision;
  hd.flags = h->opt.flags;
  hd.sample_every = h->opt.sample_every;
  hd.n_rep = (int32_t)h->reps.size();
  hd.t = h->t;
  hd.nsamples = h->nsamples;
  hd.state_bytes = h->plan.state_half;
  hd.accum_bytes = h->plan.accum_bytes;
  hd.key = ckpt_key(h);
  char* out = (char*)host_buf;
  std::memcpy(out, &hd, sizeof hd);
  hipError_t e = hipMemcpyAsync(out + sizeof hd, h->state_copy(h->cur), h->plan.state_half,
                                hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out + sizeof hd + h->plan.state_half, h->accum, h->plan.accum_bytes,
                       hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return dev_err(h, e);
  return check_watchdog(h);
}

int fnlb_load(fnlb_handle* h, const void* host_buf, size_t n) {
  if (!h || !host_buf || n < sizeof(CkptHeader)) return FNLB_EINVAL;
  if (h->error) return h->error;
  CkptHeader hd;
  std::memcpy(&hd, host_buf, sizeof hd);
  if (std::memcmp(hd.magic, kCkptMagic, 8) != 0 || hd.version != 2) return FNLB_EINVAL;
  if (hd.state_bytes != h->plan.state_half || hd.accum_bytes != h->plan.accum_bytes ||
      hd.key != ckpt_key(h) || hd.t < 0 || hd.nsamples < 0)
    return FNLB_EINVAL;
  if (n < sizeof hd + hd.state_bytes + hd.accum_bytes) return FNLB_ENOMEM;
  const char* in = (const char*)host_buf + sizeof hd;
  hipError_t e = hipMemcpyAsync(h->state_copy(h->cur), in, h->plan.state_half,
                                hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->accum, in + h->plan.state_half, h->plan.accum_bytes,
                       hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return dev_err(h, e);
  h->t = hd.t;
  h->nsamples = hd.nsamples;
  return FNLB_OK;
}

}  // extern "C"

namespace {

// Device workspace of the adjoint (byte offsets).
struct AdjPlan {
  size_t ckpt = 0, seg = 0, mu = 0, gf = 0, gs = 0, dens = 0, adjf = 0, acc = 0, target = 0,
         weight = 0, Wq = 0, mean = 0, rows = 0, Gq = 0, tpart = 0, jpart = 0, small = 0,
         total = 0;
  int64_t nck = 0;
};

int adj_plan(const fnlb_handle* h, int64_t horizon, int32_t K, AdjPlan& A) {
  if (h->reps.size() != 1 || h->opt.precision != FNLB_FP64) return FNLB_EINVAL;
  if ((h->opt.flags & ~kExecFlags) != (FNLB_ASTAR | FNLB_WALL_UZ_FIX)) return FNLB_EINVAL;
  if (horizon < 1 || K < 1) return FNLB_EINVAL;
  const RepInfo& R = h->plan.info[0];
  const size_t N = (size_t)R.Lx * R.Lz, P = (size_t)R.Lz * (R.Lx / 2 + 1);
  if (N > ((size_t)1 << 20)) return FNLB_EINVAL;  // direct spectral sums
  const size_t SH = h->plan.state_half;
  A.nck = (horizon + K - 1) / K;
  size_t o = 0;
  auto take = [&](size_t& off, size_t bytes) {
    off = o;
    o = align_up(o + bytes);
  };
  take(A.ckpt, (size_t)A.nck * SH);
  take(A.seg, ((size_t)K + 1) * SH);  // a segment's states (and the one after it)
  take(A.mu, 2 * SH);
  take(A.gf, 18 * N * 8);
  take(A.gs, 4 * N * 8);
  take(A.dens, (size_t)K * 2 * N * 8);  // the pulled densities of a segment's states
  take(A.adjf, 2 * N * 8);  // sample term: one field, or the two pressure adjoints
  take(A.acc, h->plan.accum_bytes);
  take(A.target, P * 8);
  take(A.weight, P * 8);
  take(A.Wq, P * 8);
  take(A.mean, P * 16);
  take(A.rows, P * 16);
  take(A.Gq, P * 16);
  take(A.tpart, ((N + 63) / 64) * 3 * 8);  // one partial per 64-thread block
  take(A.jpart, ((P + 255) / 256) * 8);
  take(A.small, 64);  // theta accumulator [3], J
  A.total = o;
  return FNLB_OK;
}

}  // namespace

extern "C" {

int fnlb_adjoint_bytes_required(const fnlb_handle* h, int64_t horizon, int32_t ckpt_every,
                                size_t* bytes) {
  if (!h || !bytes) return FNLB_EINVAL;
  AdjPlan A;
  const int rc = adj_plan(h, horizon, ckpt_every, A);
  if (rc) return rc;
  *bytes = A.total;
  return FNLB_OK;
}

}  // extern "C"

namespace {

// Pointers of the adjoint workspace and of the handle that both sweeps use.
struct AdjCtx {
  fnlb_handle* h;
  AdjPlan A;
  char* W;
  hipStream_t s;
  const RepInfo* R;
  const RepInfo* dR;
  size_t SH, N, P;
  int every;
  double* acc;
  double* theta;  // [0..2] parameter partials, [4] J
  char* mu[2];

  AdjCtx(fnlb_handle* hh, const AdjPlan& a, void* d_adj)
      : h(hh), A(a), W((char*)d_adj), s(hh->stream), R(&hh->plan.info[0]), dR(hh->d_reps()),
        SH(hh->plan.state_half), N((size_t)R->Lx * R->Lz), P((size_t)R->Lz * (R->Lx / 2 + 1)),
        every(hh->opt.sample_every), acc((double*)(W + a.acc)), theta((double*)(W + a.small)) {
    mu[0] = W + A.mu;
    mu[1] = W + A.mu + SH;
  }
  char* ckpt(int64_t k) const { return W + A.ckpt + (size_t)k * SH; }
  char* seg(int64_t k) const { return W + A.seg + (size_t)k * SH; }
  // the pulled densities [2][Lz][Lx] of state k of a segment
  double* dens(int64_t k) const { return (double*)(W + A.dens) + (size_t)k * 2 * N; }
  bool sampled(int64_t t) const { return every > 0 && t >= 1 && t % every == 0; }
  // The step of a sample time runs the sampling variant of the step kernel
  // both in the forward sweep and when a segment is recomputed, so that every
  // recomputed state is bit-identical to the forward one whatever the
  // checkpoint interval (the two kernel variants may round differently).
  // (dens: where the step writes the pulled densities of `in`, or null;
  // slot: the spectrum slot of a sample's pressure parts)
  hipError_t step_from(const char* in, char* out, int64_t t, double* dens = nullptr,
                       int slot = 0) const {
    StepArgs a = step_args(h, t - h->t_dev, slot);
    a.state_in = in;
    a.state_out = out;
    a.dens = dens;
    return launch_step(FNLB_FP64, sampled(t) ? kStepSample : kStep, a, s);
  }
};

// Forward sweep of a misfit over a horizon (the structure factor of `field`,
// or with `pressure` the pressure row profile): populations checkpointed every
// ckpt_every steps and the samples summed privately in the workspace, then J
// and its sensitivities to the sampled spectrum (or row profile).  The handle
// remembers the sweep so that misfit_reverse can differentiate it.
int misfit_forward(fnlb_handle* h, bool pressure, int32_t field, const double* target,
                   const double* weight, int64_t horizon, int32_t ckpt_every, void* d_adj,
                   size_t adj_bytes, double* J) {
  if (!h || !target || !weight || !d_adj || !J) return FNLB_EINVAL;
  if (h->error) return h->error;
  h->adj.valid = false;
  if (h->opt.sample_every <= 0) return FNLB_EINVAL;
  AdjPlan A;
  int rc = adj_plan(h, horizon, ckpt_every, A);
  if (rc) return rc;
  if (adj_bytes < A.total) return FNLB_ENOMEM;
  if ((uintptr_t)d_adj % kAlign) return FNLB_EINVAL;
  const AdjCtx C(h, A, d_adj);
  char* W = C.W;
  hipStream_t s = C.s;
  const int64_t t0 = h->t;
  const int K = ckpt_every;
  double* dJ = C.theta + 4;
  const size_t nt = pressure ? (size_t)C.R->Lz : C.P;  // target and weight entries
  hipError_t e = hipMemcpyAsync(W + A.target, target, nt * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(W + A.weight, weight, nt * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_fill_zero(C.acc, h->plan.accum_bytes, s);
  if (e == hipSuccess) e = launch_fill_zero(W + A.small, 64, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(C.mu[0], h->state_copy(h->cur), C.SH, hipMemcpyDeviceToDevice, s);
  // The states alternate between two buffers; the last segment's states, and
  // the pulled densities of each, go straight to the segment buffers, where
  // the reverse sweep, which differentiates that segment first, finds them
  // without recomputing it.  The samples keep their row spectra in the
  // spectrum slots and one column pass adds up to kSpecSlots of them into the
  // private sums, in time order.
  const int64_t last_ts = (A.nck - 1) * (int64_t)K;
  const int slots = h->plan.spec_slots;
  int64_t nsamp = 0;
  int cur = 0, pend = 0;
  for (int64_t k = 0; k < horizon && e == hipSuccess; ++k) {
    const char* in = C.mu[cur];
    char* out = C.mu[cur ^ 1];
    double* dens = nullptr;
    if (k % K == 0) e = hipMemcpyAsync(C.ckpt(k / K), C.mu[cur], C.SH, hipMemcpyDeviceToDevice, s);
    if (k >= last_ts) {
      if (k == last_ts && e == hipSuccess)
        e = hipMemcpyAsync(C.seg(0), C.mu[cur], C.SH, hipMemcpyDeviceToDevice, s);
      in = C.seg(k - last_ts);
      out = C.seg(k - last_ts + 1);
      dens = C.dens(k - last_ts);
    }
    const bool smp = C.sampled(t0 + k);
    if (e == hipSuccess) e = C.step_from(in, out, t0 + k, dens, smp ? pend : 0);
    if (smp) {
      if (e == hipSuccess) e = observe_rows(h, s, pend);
      if (++pend == slots && e == hipSuccess) {
        e = observe_cols(h, s, pend, C.acc);
        pend = 0;
      }
      ++nsamp;
    }
    cur ^= 1;
  }
  if (pend > 0 && e == hipSuccess) e = observe_cols(h, s, pend, C.acc);
  if (nsamp == 0) return e == hipSuccess ? FNLB_EINVAL : dev_err(h, e);
  const double ns = (double)nsamp;
  if (pressure) {
    // Wq holds lam_j = dJ/d(P - P_ref) of a node of row j in one sample
    if (e == hipSuccess)
      e = launch_adj_pmisfit(C.dR, *C.R, C.acc, (const double*)(W + A.target),
                             (const double*)(W + A.weight), ns, (double*)(W + A.Wq), dJ, s);
  } else {
    if (e == hipSuccess)
      e = launch_adj_misfit(C.dR, *C.R, h->d_tw(), C.acc, (const double*)(W + A.target),
                            (const double*)(W + A.weight), (double*)(W + A.Wq),
                            (double2*)(W + A.mean), (double*)(W + A.jpart), field, ns, s);
    if (e == hipSuccess)
      e = launch_sum((const double*)(W + A.jpart), (int)((C.P + 255) / 256), dJ, s);
  }
  double Jv = 0.0;
  if (e == hipSuccess) e = hipMemcpyAsync(&Jv, dJ, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_err(h, e);
  *J = Jv;
  h->adj.valid = true;
  h->adj.d_adj = d_adj;
  h->adj.bytes = adj_bytes;
  h->adj.horizon = horizon;
  h->adj.t0 = t0;
  h->adj.nsamp = nsamp;
  h->adj.K = K;
  h->adj.field = field;
  h->adj.pressure = pressure;
  h->adj.last_seg_kept = true;
  return FNLB_OK;
}

// Reverse sweep of the last forward sweep over the same workspace: per
// checkpointed segment the states are recomputed with the step kernel, then
// each step is differentiated backwards; dJ/d(tau_s, tau_d, G) into grad.
int misfit_reverse(fnlb_handle* h, void* d_adj, size_t adj_bytes, double* grad) {
  if (!h || !d_adj || !grad) return FNLB_EINVAL;
  if (h->error) return h->error;
  if (!h->adj.valid || h->adj.d_adj != d_adj || h->adj.bytes != adj_bytes ||
      h->t != h->adj.t0)
    return FNLB_ESTATE;
  AdjPlan A;
  const int rc = adj_plan(h, h->adj.horizon, h->adj.K, A);
  if (rc) return rc;
  const AdjCtx C(h, A, d_adj);
  char* W = C.W;
  hipStream_t s = C.s;
  const int64_t t0 = h->adj.t0, horizon = h->adj.horizon;
  const int K = h->adj.K, field = h->adj.field;
  const bool pressure = h->adj.pressure;
  const double ns = (double)h->adj.nsamp;
  // the parameter partials of each block run over the whole sweep and are
  // summed once at its end (J, in theta[4], is kept)
  hipError_t e = launch_fill_zero(C.theta, 32, s);
  if (e == hipSuccess) e = launch_fill_zero(C.mu[0], 2 * C.SH, s);
  if (e == hipSuccess) e = launch_fill_zero(W + A.tpart, ((C.N + 63) / 64) * 3 * 8, s);
  int nx = 0;  // mu[nx] holds dJ/dS_{t+1}
  for (int64_t sgi = A.nck - 1; sgi >= 0 && e == hipSuccess; --sgi) {
    const int64_t ts = sgi * K, te = std::min<int64_t>(horizon, ts + K);
    // the segment's states recomputed from its checkpoint, each step also
    // writing the pulled densities of its input state (the last state's too,
    // by one step past the segment, whose output is not used); the forward
    // sweep left the last segment's in place, until a reverse sweep recomputes
    // another segment there
    if (sgi != A.nck - 1 || !h->adj.last_seg_kept) {
      if (sgi != A.nck - 1) h->adj.last_seg_kept = false;
      e = hipMemcpyAsync(C.seg(0), C.ckpt(sgi), C.SH, hipMemcpyDeviceToDevice, s);
      for (int64_t k = ts; k < te && e == hipSuccess; ++k)
        e = C.step_from(C.seg(k - ts), C.seg(k - ts + 1), t0 + k, C.dens(k - ts));
    }
    for (int64_t k = te - 1; k >= ts && e == hipSuccess; --k) {
      const double* S = (const double*)C.seg(k - ts);
      double* dens = C.dens(k - ts);
      const double* adjf = nullptr;
      if (e == hipSuccess && C.sampled(t0 + k)) {
        if (pressure)
          e = launch_adj_psample(C.dR, *C.R, dens,
                                 (const double*)(W + A.Wq), (double*)(W + A.adjf),
                                 (double*)(W + A.tpart), s);
        else
          e = launch_adj_sample(C.dR, *C.R, h->d_tw(), (const double*)(W + A.Wq),
                                (const double2*)(W + A.mean), field, ns,
                                dens, (double2*)(W + A.rows),
                                (double2*)(W + A.Gq), (double*)(W + A.adjf), s);
        adjf = (const double*)(W + A.adjf);
      }
      if (e == hipSuccess)
        e = launch_adj_step(C.dR, *C.R, S, (const double*)C.mu[nx], (double*)C.mu[nx ^ 1],
                            dens, (double*)(W + A.gf), (double*)(W + A.gs),
                            adjf, pressure ? kAdjPressure : field, t0 + k,
                            (double*)(W + A.tpart), s);
      nx ^= 1;
    }
  }
  if (e == hipSuccess) e = launch_adj_theta(*C.R, (const double*)(W + A.tpart), C.theta, s);
  double out[3] = {0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(out, C.theta, 3 * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_err(h, e);
  // dJ/dlambda -> dJ/dtau with lambda = 1/tau
  const double ls = C.R->lam[4], ld = C.R->lam[1];
  grad[0] = -ls * ls * out[0];
  grad[1] = -ld * ld * out[1];
  grad[2] = out[2];
  return FNLB_OK;
}

// Host conversion between the caller's layout [species][l][z][x] of the
// populations f(t) and the stored elements of one replica: the element that
// holds f_l(x, z) is pull_source(), a bijection, so a cotangent moves between
// the two layouts by the same permutation (the reference shifts of the stored
// deviations are constants and drop out).
void to_stored(const RepInfo& R, const double* user, double* stored) {
  const size_t n = (size_t)R.Lz * R.Lx;
  for (int s = 0; s < 2; ++s)
    for (int l = 0; l < 9; ++l)
      for (int j = 0; j < R.Lz; ++j)
        for (int x = 0; x < R.Lx; ++x)
          stored[pull_source(R, s, l, j, x)] = user[(size_t)(s * 9 + l) * n + (size_t)j * R.Lx + x];
}

void from_stored(const RepInfo& R, const double* stored, double* user) {
  const size_t n = (size_t)R.Lz * R.Lx;
  for (int s = 0; s < 2; ++s)
    for (int l = 0; l < 9; ++l)
      for (int j = 0; j < R.Lz; ++j)
        for (int x = 0; x < R.Lx; ++x)
          user[(size_t)(s * 9 + l) * n + (size_t)j * R.Lx + x] = stored[pull_source(R, s, l, j, x)];
}

}  // namespace

extern "C" {

int fnlb_sq_misfit(fnlb_handle* h, int32_t field, const double* S_target, const double* weight,
                   int64_t horizon, int32_t ckpt_every, void* d_adj, size_t adj_bytes,
                   double* J) {
  if (field != 0 && field != 1) return FNLB_EINVAL;
  return misfit_forward(h, false, field, S_target, weight, horizon, ckpt_every, d_adj, adj_bytes,
                        J);
}

int fnlb_pressure_misfit(fnlb_handle* h, const double* P_target, const double* weight,
                         int64_t horizon, int32_t ckpt_every, void* d_adj, size_t adj_bytes,
                         double* J) {
  return misfit_forward(h, true, 0, P_target, weight, horizon, ckpt_every, d_adj, adj_bytes, J);
}

int fnlb_misfit_backward(fnlb_handle* h, void* d_adj, size_t adj_bytes, double* grad) {
  return misfit_reverse(h, d_adj, adj_bytes, grad);
}

int fnlb_sq_misfit_gradient(fnlb_handle* h, int32_t field, const double* S_target,
                            const double* weight, int64_t horizon, int32_t ckpt_every,
                            void* d_adj, size_t adj_bytes, double* J, double* grad) {
  if (!grad) return FNLB_EINVAL;
  const int rc = fnlb_sq_misfit(h, field, S_target, weight, horizon, ckpt_every, d_adj,
                                adj_bytes, J);
  return rc ? rc : misfit_reverse(h, d_adj, adj_bytes, grad);
}

int fnlb_pressure_misfit_gradient(fnlb_handle* h, const double* P_target, const double* weight,
                                  int64_t horizon, int32_t ckpt_every, void* d_adj,
                                  size_t adj_bytes, double* J, double* grad) {
  if (!grad) return FNLB_EINVAL;
  const int rc = fnlb_pressure_misfit(h, P_target, weight, horizon, ckpt_every, d_adj,
                                      adj_bytes, J);
  return rc ? rc : misfit_reverse(h, d_adj, adj_bytes, grad);
}

int fnlb_step_vjp(fnlb_handle* h, const double* mu_next, double* mu, double* dtheta, void* d_adj,
                  size_t adj_bytes) {
  if (!h || !mu_next || !mu || !dtheta || !d_adj) return FNLB_EINVAL;
  if (h->error) return h->error;
  AdjPlan A;
  const int rc = adj_plan(h, 1, 1, A);
  if (rc) return rc;
  if (adj_bytes < A.total) return FNLB_ENOMEM;
  if ((uintptr_t)d_adj % kAlign) return FNLB_EINVAL;
  const AdjCtx C(h, A, d_adj);
  // this call's layout of the workspace differs from a misfit sweep's
  h->adj.valid = false;
  const RepInfo& R = *C.R;
  const size_t nel = 18 * (size_t)R.plane;  // stored elements of the replica
  std::vector<double> st(nel, 0.0);
  to_stored(R, mu_next, st.data());
  hipStream_t s = C.s;
  const double* S = (const double*)h->state_copy(h->cur);
  hipError_t e = launch_fill_zero(C.mu[0], 2 * C.SH, s);
  if (e == hipSuccess) e = hipMemcpyAsync(C.mu[0], st.data(), nel * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_fill_zero(C.theta, 32, s);
  if (e == hipSuccess) e = launch_fill_zero(C.W + A.tpart, ((C.N + 63) / 64) * 3 * 8, s);
  if (e == hipSuccess) e = launch_adj_density(C.dR, R, S, (double*)(C.W + A.dens), s);
  if (e == hipSuccess)
    e = launch_adj_step(C.dR, R, S, (const double*)C.mu[0], (double*)C.mu[1],
                        (double*)(C.W + A.dens), (double*)(C.W + A.gf), (double*)(C.W + A.gs),
                        nullptr, 0, h->t, (double*)(C.W + A.tpart), s);
  if (e == hipSuccess) e = launch_adj_theta(R, (const double*)(C.W + A.tpart), C.theta, s);
  double out[3] = {0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(st.data(), C.mu[1], nel * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, C.theta, 3 * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_err(h, e);
  from_stored(R, st.data(), mu);
  const double ls = R.lam[4], ld = R.lam[1];
  dtheta[0] = -ls * ls * out[0];
  dtheta[1] = -ld * ld * out[1];
  dtheta[2] = out[2];
  return FNLB_OK;
}

int fnlb_destroy(fnlb_handle* h) {
  if (!h) return FNLB_OK;
  if (h->static_dev >= 0) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    g_static_busy[h->static_dev] = false;
  }
  drop_graphs(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->obs_stream) (void)hipStreamDestroy(h->obs_stream);
  for (int k = 0; k < kSpecSlots; ++k) {
    if (h->ev_fork[k]) (void)hipEventDestroy(h->ev_fork[k]);
    if (h->ev_join[k]) (void)hipEventDestroy(h->ev_join[k]);
  }
  delete h;
  return FNLB_OK;
}

#ifndef FNLB_BUILD_ID
#define FNLB_BUILD_ID "unknown"
#endif

const char* fnlb_build_id(void) { return FNLB_BUILD_ID; }

const char* fnlb_strerror(int code) {
  switch (code) {
    case FNLB_OK: return "ok";
    case FNLB_EINVAL: return "invalid argument or parameter";
    case FNLB_ENOMEM: return "caller buffer smaller than required";
    case FNLB_EDEVICE: return "HIP runtime error";
    case FNLB_EWATCHDOG: return "non-finite or non-physical state detected";
    case FNLB_ESTATE: return "call not valid in the current state";
    default: return "unknown error";
  }
}

}  // extern "C"
