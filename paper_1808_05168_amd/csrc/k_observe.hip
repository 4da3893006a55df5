// Observables of a sample: structure factors of delta c and delta rho, and
// optionally of U_x and U_z (Appendix, Eqs. (A1)-(A4): Phi(q) = (Lx Lz)^{-1/2}
// sum_{x,j} dphi e^{-i q.r}, S(q) = <|Phi(q)|^2> on the lattice; Sec. IV.A for
// S_U) and the mean pressure (Sec. IV.C).
//
// The sampling step forms the fields of a sample and stores them per node as
// complex pairs (z = delta c + i delta rho, and z = U_x + i U_z) in the
// storage type, and sums the nodes' pressure deviations from the row's
// constant part in FP64, per row and 64 columns.  A row pass transforms each
// row's pairs as one complex sequence and splits the result by Hermitian
// symmetry into the half spectra k_x = 0..Lx/2 of the two fields; a column
// pass transforms each k_x column over the Lz rows and adds |Phi|^2, Re Phi
// and Im Phi to the FP64 accumulators, and adds the sample's mean pressure
// and row profile.  Both transforms compute in FP64; the row spectra between
// them are kept in the storage type (complex float pairs for FP32-deviation
// storage, whose fields are float values).  Rows and columns of 8 to 512 points (powers
// of two) use the wavefront transforms; longer power-of-two lengths the
// in-LDS FFT of a block; other lengths a direct sum with exactly reduced
// twiddle indices.  Every sum is formed in a fixed order, so every
// accumulator is deterministic.
#include "fnlb.h"
#include "fnlb_fft.hpp"
#include "fnlb_internal.hpp"
#include "fnlb_node.hpp"

namespace fnlb {
namespace {

// The element of the row spectra: the storage type's complex pair.
template <typename FT>
struct SpecOf {
  using type = double2;
};
template <>
struct SpecOf<float> {
  using type = float2;
};
__device__ __forceinline__ double2 widen(double2 v) { return v; }
__device__ __forceinline__ double2 widen(float2 v) { return make_double2(v.x, v.y); }
template <typename ST>
__device__ __forceinline__ ST narrow(double x, double y) {
  if constexpr (sizeof(ST) == 8)
    return make_float2((float)x, (float)y);
  else
    return make_double2(x, y);
}

__global__ void k_fill_zero(uint32_t* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = i; k < n; k += stride) p[k] = 0u;
}

__global__ void k_advance_time(int64_t* t, int64_t dt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *t += dt;
}

// twiddles of one replica: tw[m] = exp(-2 pi i m / N) for the Lx table then
// the Lz table.
// The per-row sample constants (sample_row_calc), one thread per row; ghost
// rows beyond the walls repeat the wall row, as in the step.
template <typename Real>
__global__ void k_row_consts(const RepInfo* reps) {
  const RepInfo& R = reps[blockIdx.y];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= R.Lz) return;
  const int jU = j == R.Lz - 1 ? j : j + 1, jD = j == 0 ? j : j - 1;
  const SampleRow<Real> r = sample_row_calc<Real>(R, j, jU, jD);
  Real* t = (Real*)R.rowc + (size_t)kRowConsts * j;
  t[0] = r.rAj;
  t[1] = r.rBj;
  t[2] = r.c0;
  t[3] = r.sAref;
  t[4] = r.sBref;
  t[5] = r.szref;
  t[6] = r.G4;
  t[7] = (Real)0;
}

__global__ void k_twiddles(const RepInfo* reps, double2* tw_base) {
  const RepInfo& R = reps[blockIdx.y];
  double2* tw = tw_base + R.tw_off;
  const int total = R.Lx + R.Lz;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int N = i < R.Lx ? R.Lx : R.Lz;
    const int m = i < R.Lx ? i : i - R.Lx;
    double s, c;
    sincospi(2.0 * (double)m / (double)N, &s, &c);
    tw[i] = make_double2(c, -s);
  }
}

// Global loads are issued kBatch per thread before their values are used, so
// that their latencies overlap.
constexpr int kBatch = 8;

// Row pass of a sample (block transforms): one block per group of
// consecutive rows of one replica (several short rows share a block) and field
// pair (blockIdx.y).  The rows' pairs, of type FT, are read into LDS (bit
// reversed for the FFT), transformed and split into the two half spectra.
// LDS: the rows, then (power-of-two rows) the N/2 twiddles the FFT uses.
template <typename FT>
__global__ __launch_bounds__(256) void k_row_transform(const RepInfo* reps, const RowRef* rows,
                                                       const void* fields, void* spec,
                                                       const double2* tw_base) {
  using ST = typename SpecOf<FT>::type;
  extern __shared__ double2 lds[];
  const RowRef rr = rows[blockIdx.x];
  const RepInfo& R = reps[rr.rep];
  const int N = R.Lx, Lz = R.Lz, nkx = N / 2 + 1, nr = rr.nrows;
  const int pair = blockIdx.y;
  const FT* z = (const FT*)fields + R.field_off + (size_t)pair * 2 * Lz * N;
  const double2* tw = tw_base + R.tw_off;
  const size_t orow = (size_t)(2 * pair) * Lz + rr.j0;  // first field of the pair
  ST* out_c = (ST*)spec + R.spec_off + orow * R.spitch;
  ST* out_r = out_c + (size_t)Lz * R.spitch;
  const int total = nr * N;
  const int bits = R.pow2 ? __ffs(N) - 1 : 0;
  // the block's threads split into one group per row
  const int gsz = blockDim.x / nr;
  const int r = threadIdx.x / gsz, t2 = threadIdx.x - r * gsz;
  const bool live = r < nr;
  const int j = rr.j0 + (live ? r : 0);
  if (live)
    for (int x = t2; x < N; x += gsz) {
      const size_t n = (size_t)j * N + x;
      lds[(size_t)r * N + (R.pow2 ? bitrev(x, bits) : x)] =
          make_double2((double)z[2 * n], (double)z[2 * n + 1]);
    }
  if (R.pow2) {
    double2* tws = lds + total;
    for (int m = threadIdx.x; m < N / 2; m += blockDim.x) tws[m] = tw[m];
    lds_fft(lds, bits, nr, tws);
  } else {
    __syncthreads();
  }
  if (!live) return;
  const double2* row = lds + (size_t)r * N;
  for (int k = t2; k < nkx; k += gsz) {
    double2 Z, Zm;
    if (R.pow2) {
      Z = row[k];
      Zm = row[(N - k) & (N - 1)];
    } else {
      // direct sum for Z(k) and Z(N-k)
      double zr = 0, zi = 0, mr = 0, mi = 0;
      const int km = (N - k) % N;
      int ik = 0, im = 0;
      for (int x = 0; x < N; ++x) {
        const double2 a = row[x];
        const double2 w1 = tw[ik], w2 = tw[im];
        zr += a.x * w1.x - a.y * w1.y;
        zi += a.x * w1.y + a.y * w1.x;
        mr += a.x * w2.x - a.y * w2.y;
        mi += a.x * w2.y + a.y * w2.x;
        ik += k;
        if (ik >= N) ik -= N;
        im += km;
        if (im >= N) im -= N;
      }
      Z = make_double2(zr, zi);
      Zm = make_double2(mr, mi);
    }
    // C(k) = (Z(k) + conj Z(N-k)) / 2, Rho(k) = (Z(k) - conj Z(N-k)) / (2i)
    const size_t o = (size_t)r * R.spitch + k;
    out_c[o] = narrow<ST>(0.5 * (Z.x + Zm.x), 0.5 * (Z.y - Zm.y));
    out_r[o] = narrow<ST>(0.5 * (Z.y + Zm.y), 0.5 * (Zm.x - Z.x));
  }
}

// Pressure of a sample for one replica, by one block: each row's sum is its
// parts in order plus Lx times the row's constant part; the row sums go into
// the profile (row means), then a fixed-shape tree over the rows gives the
// spatial mean.  Layout of the replica's block: {sum, sum2, profile[Lz]}.
// rows: LDS scratch of at least the next power of two >= Lz doubles.
__device__ void pressure_reduce(const RepInfo& R, const double* ppart, double* acc,
                                double* rows) {
  const int Lz = R.Lz, np = pressure_parts(R.Lx);
  const double* pp = ppart + R.ppart_off;  // parts of the row sums of P - P_ref
  double* pa = acc + R.pacc_off;
  int P2 = 1;
  while (P2 < Lz) P2 <<= 1;
  for (int j = threadIdx.x; j < P2; j += blockDim.x) {
    double s = 0.0;
    if (j < Lz) {
      const double* part = pp + (size_t)j * np;
      double d = part[0];
      for (int k = 1; k < np; ++k) d += part[k];
      s = d + R.Lx * pressure_row_ref(R, j);
      pa[2 + j] += s / (double)R.Lx;
    }
    rows[j] = s;
  }
  for (int h = P2 >> 1; h >= 1; h >>= 1) {
    __syncthreads();
    for (int j = threadIdx.x; j < h; j += blockDim.x) rows[j] += rows[j + h];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double mean = rows[0] / ((double)R.Lx * (double)Lz);
    pa[0] += mean;
    pa[1] += mean * mean;
  }
}

// Column pass: one block per (replica, field, tile of 2^ltile k_x columns).
// The block of the first tile of the first field also reduces the replica's
// pressure of every sample (from the parts the sampling step wrote).
// LDS: the tile's columns, then (power-of-two columns) the M/2 twiddles.
template <typename ST>
__global__ __launch_bounds__(256) void k_col_transform(const RepInfo* reps, const ColRef* cols,
                                                       const ST* spec0, double* acc,
                                                       const double2* tw_base,
                                                       const double* ppart0, int nslots,
                                                       size_t spec_slot, size_t ppart_slot) {
  extern __shared__ double2 lds[];
  const ColRef cr = cols[blockIdx.x];
  for (int sl = 0; sl < nslots; ++sl) {
    // samples in slot order, each a full pass over the tile
    const ST* spec = spec0 + sl * spec_slot;
    const double* ppart = ppart0 + sl * ppart_slot;
    if (sl > 0) __syncthreads();  // the last sample's tile and sums are done with
    const RepInfo& R = reps[cr.rep];
    const int Lx = R.Lx, M = R.Lz, nkx = Lx / 2 + 1;
    const int nc = cr.ncols, lt = cr.ltile, tmask = (1 << lt) - 1;
    const ST* in = spec + R.spec_off + (size_t)cr.field * M * R.spitch + cr.kx0;
    const double2* tw = tw_base + R.tw_off + Lx;
    const size_t plane = (size_t)M * nkx;
    // accumulators are stored column-major, [k_x][k_z], so a tile's sums are one
    // contiguous run per kind
    double* a2 = acc + R.acc_off + (size_t)cr.field * 3 * plane + (size_t)cr.kx0 * M;
    double* are = a2 + plane;
    double* aim = a2 + 2 * plane;
    const double norm = R.inv_norm;
    const int bits = __ffs(M) - 1;
    const int total = M << lt;
    // load: row-major reads of the tile's consecutive k_x of each row
    for (int base = threadIdx.x; base < total; base += kBatch * blockDim.x) {
      // (two plain arrays: an array of double2 assigned under a condition is
      // kept in scratch memory)
      double vr[kBatch], vi[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int q = base + u * blockDim.x;
        if (q < total && (q & tmask) < nc) {
          const double2 t = widen(in[(size_t)(q >> lt) * R.spitch + (q & tmask)]);
          vr[u] = t.x;
          vi[u] = t.y;
        }
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int q = base + u * blockDim.x;
        const int j = q >> lt, c = q & tmask;
        if (q < total && c < nc)
          lds[(size_t)c * M + (R.pow2 ? bitrev(j, bits) : j)] = make_double2(vr[u], vi[u]);
      }
    }
    if (R.pow2) {
      // The sums of the first batch of entries are loaded before the transform,
      // so that their latency overlaps it (entry q of the tile is column
      // q >> bits, k_z = q & (M - 1), at offset q of each accumulator run).
      const int valid = min(total, nc * M);
      double s2[kBatch], sr[kBatch], si[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int q = threadIdx.x + u * blockDim.x;
        if (q < valid) {
          s2[u] = a2[q];
          sr[u] = are[q];
          si[u] = aim[q];
        }
      }
      double2* tws = lds + ((size_t)M << lt);
      for (int m = threadIdx.x; m < M / 2; m += blockDim.x) tws[m] = tw[m];
      lds_fft(lds, bits, nc, tws);
      for (int base = threadIdx.x; base < valid; base += kBatch * blockDim.x) {
        if (base != (int)threadIdx.x) {
#pragma unroll
          for (int u = 0; u < kBatch; ++u) {
            const int q = base + u * blockDim.x;
            if (q < valid) {
              s2[u] = a2[q];
              sr[u] = are[q];
              si[u] = aim[q];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const int q = base + u * blockDim.x;
          if (q < valid) {
            const double2 P = lds[q];
            const double re = P.x * norm, im = P.y * norm;
            a2[q] = s2[u] + (re * re + im * im);
            are[q] = sr[u] + re;
            aim[q] = si[u] + im;
          }
        }
      }
    } else {
      __syncthreads();
      for (int q = threadIdx.x; q < total; q += blockDim.x) {
        const int c = q / M, kz = q - c * M;
        if (c >= nc) continue;
        const double2* col = lds + (size_t)c * M;
        double re = 0, im = 0;
        int ik = 0;
        for (int j = 0; j < M; ++j) {
          const double2 a = col[j], w = tw[ik];
          re += a.x * w.x - a.y * w.y;
          im += a.x * w.y + a.y * w.x;
          ik += kz;
          if (ik >= M) ik -= M;
        }
        re *= norm;
        im *= norm;
        const size_t o = (size_t)c * M + kz;
        a2[o] += re * re + im * im;
        are[o] += re;
        aim[o] += im;
      }
    }
    if (cr.field == 0 && cr.kx0 == 0) {
      __syncthreads();  // the tile's LDS is free again (it holds >= Lz double2)
      pressure_reduce(R, ppart, acc, (double*)lds);
    }
  }
}

// ---- Wavefront transforms (rows and columns of 8 to 512 points, powers of
// two): one sequence per group of N / 8 lanes, eight points per lane, the
// Stockham passes of wave_fft.

// Row pass of a sample on rows of N = 8 to 512 points (a power of two): each
// wavefront takes one task of up to 2 G consecutive rows of one replica (G =
// 512 / N) in two halves of G rows (float pairs; G rows for double pairs),
// one row per group of S = N / 8 lanes, and one field pair.  Lane t of a
// group loads the pairs of nodes t + S q (q = 0..7), the order the first
// pass of wave_fft takes (each load of a group is one run of S consecutive
// pairs); the row is transformed and split by Hermitian symmetry into the
// half spectra k_x = 0 .. N/2 of the two fields.  With float pairs the second
// half's pairs are loaded before the first half is transformed, so that
// their latency overlaps that transform.
template <typename FT>
struct RowPoints {  // the eight pairs of a lane, as loaded
  float2 p[8];
};

template <typename FT, int N>
__device__ __forceinline__ RowPoints<FT> load_row_points(const RepInfo& R, int pair, int j,
                                                         int t, const void* fields) {
  constexpr int S = N / 8;
  const float2* z = (const float2*)((const FT*)fields + R.field_off) +
                    (size_t)pair * R.Lz * N + (size_t)j * N + t;
  RowPoints<FT> r;
#pragma unroll
  for (int q = 0; q < 8; ++q) r.p[q] = z[S * q];
  return r;
}

// The transform of one row per group from its points (v[q] = node t + S q),
// split into the two half spectra (live groups only store).  buf: the group's
// sequence in LDS, which the previous row's split may still be reading.
template <typename FT, int N>
__device__ __forceinline__ void row_transform(const RepInfo& R, double2 (&v)[8], int pair, int j,
                                              bool live, int t, double2* buf, void* spec,
                                              const double2* tw) {
  using ST = typename SpecOf<FT>::type;
  constexpr int S = N / 8;
  wave_sync();  // the group's earlier reads of buf are done
  wave_fft<N>(v, buf, t, tw);
  // C(k) = (Z(k) + conj Z(N-k)) / 2, Rho(k) = (Z(k) - conj Z(N-k)) / (2i), k <= N/2
  wave_sync();
#pragma unroll
  for (int p = 0; p < 8; ++p) buf[pidx(t + S * p)] = v[p];
  wave_sync();
  if (!live) return;
  const int Lz = R.Lz;
  ST* out_c = (ST*)spec + R.spec_off + ((size_t)(2 * pair) * Lz + j) * R.spitch;
  ST* out_r = out_c + (size_t)Lz * R.spitch;
#pragma unroll
  for (int p = 0; p < 5; ++p) {
    const int k = t + S * p;
    if (k <= N / 2) {
      const double2 Z = v[p], Zm = buf[pidx((N - k) & (N - 1))];
      out_c[k] = narrow<ST>(0.5 * (Z.x + Zm.x), 0.5 * (Z.y - Zm.y));
      out_r[k] = narrow<ST>(0.5 * (Z.y + Zm.y), 0.5 * (Zm.x - Z.x));
    }
  }
}

template <typename FT, int N>
__device__ __forceinline__ void row_fft(const RepInfo& R, const RowTask& T, int pair, int lane,
                                        const void* fields, void* spec,
                                        const double2* tw_base, double2* wlds) {
  constexpr int S = N / 8, G = 64 / S;
  static_assert(G * seq_pitch(N) <= kWaveFftLds, "wavefront LDS");
  const int g = lane / S, t = lane % S;
  double2* buf = wlds + g * seq_pitch(N);
  const double2* tw = tw_base + R.tw_off;
  // rows of the two halves (a dead group loads the task's first row)
  const bool live0 = g < T.nrows, live1 = G + g < T.nrows;
  const bool two = T.nrows > G;  // the whole wavefront
  const int j0 = T.j0 + (live0 ? g : 0), j1 = T.j0 + (live1 ? G + g : 0);
  double2 v[8];
  if constexpr (sizeof(FT) == 4) {
    const RowPoints<FT> a = load_row_points<FT, N>(R, pair, j0, t, fields);
    // (loaded whether or not the task has a second half: a value loaded under
    // a condition would be kept in scratch memory)
    const RowPoints<FT> b = load_row_points<FT, N>(R, pair, j1, t, fields);
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = make_double2(a.p[q].x, a.p[q].y);
    row_transform<FT, N>(R, v, pair, j0, live0, t, buf, spec, tw);
    if (two) {
      // (the twiddles again through a pointer the compiler cannot identify
      // with tw: kept from the first half, they would stay in registers
      // across it)
      const double2* tw1 = tw;
      asm volatile("" : "+v"(tw1));
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = make_double2(b.p[q].x, b.p[q].y);
      row_transform<FT, N>(R, v, pair, j1, live1, t, buf, spec, tw1);
    }
  } else {
    // double pairs: tasks of one half
    const double2* z = (const double2*)((const double*)fields + R.field_off) +
                       (size_t)pair * R.Lz * N + (size_t)j0 * N + t;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = z[S * q];
    row_transform<FT, N>(R, v, pair, j0, live0, t, buf, spec, tw);
  }
}

template <typename FT>
__global__ __launch_bounds__(256) void k_row_fft(const RepInfo* reps, const RowTask* tasks,
                                                 int n_tasks, const void* fields, void* spec,
                                                 const double2* tw_base) {
  __shared__ double2 lds[4 * kWaveFftLds];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  const int task = blockIdx.x * 4 + wv;
  if (task >= n_tasks) return;  // the whole wavefront: nothing below waits on others
  const RowTask T = tasks[task];
  const RepInfo& R = reps[__builtin_amdgcn_readfirstlane(T.rep)];
  const int pair = blockIdx.y;
  double2* w = lds + wv * kWaveFftLds;
#define FNLB_ROW(n) row_fft<FT, n>(R, T, pair, lane, fields, spec, tw_base, w)
  switch (R.Lx) {
    case 8: FNLB_ROW(8); break;
    case 16: FNLB_ROW(16); break;
    case 32: FNLB_ROW(32); break;
    case 64: FNLB_ROW(64); break;
    case 128: FNLB_ROW(128); break;
    case 256: FNLB_ROW(256); break;
    default: FNLB_ROW(512); break;
  }
#undef FNLB_ROW
}

// Column pass on columns of M = 8 to 512 points (Lz a power of two), over the
// spectra of nslots samples (slot s at spec + s spec_slot): a block takes a
// tile of C = 2048 / M consecutive k_x columns of one field's row spectra
// (every row of the tile one run of whole 128-byte lines) per sample, each
// wavefront transforms C / 4 of them (wave_fft, one per group of M / 8 lanes)
// and adds |Phi|^2, Re Phi and Im Phi of entries k_z = t + S p to running FP64
// sums, sample after sample, which it loads before the first and stores after
// the last; the sums therefore round exactly as one pass per sample would.
// The next sample's tile is loaded while the current one is transformed.  The
// block of the first tile of the first field also adds the replica's pressure
// of each sample, in order.
template <typename ST, int M>
__device__ __forceinline__ void col_fft(const RepInfo& R, const ColTask& T, const ST* spec,
                                        int nslots, size_t spec_slot, double* acc,
                                        const double2* tw_base, const double* ppart,
                                        size_t ppart_slot, double2* lds) {
  constexpr int S = M / 8, G = 64 / S, C = 4 * G, pitch = seq_pitch(M);
  constexpr int rp = 256 / C;  // tile rows one load instruction covers
  static_assert(C * pitch <= 4 * kWaveFftLds, "tile");
  const int Lx = R.Lx, nkx = Lx / 2 + 1, spitch = R.spitch;
  const double norm = R.inv_norm;
  const int ncols = T.ncols;
  const size_t plane = (size_t)M * nkx;
  const double2* tw = tw_base + R.tw_off + Lx;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  const int g = lane / S, t = lane % S;
  const int c = wv * G + g;
  const bool live = c < ncols;
  // accumulators are stored column-major, [k_x][k_z]; a dead group reads the
  // tile's first column, so that the sums stay in registers
  double* a2 = acc + R.acc_off + (size_t)T.field * 3 * plane + (size_t)T.kx0 * M +
               (size_t)(live ? c : 0) * M;
  double s2[8], sr[8], si[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int kz = t + S * p;
    s2[p] = a2[kz];
    sr[p] = a2[plane + kz];
    si[p] = a2[2 * plane + kz];
  }
  // the tile: thread i loads column i % C (a column past the tile, whose group
  // is dead, loads a copy of the first column) of rows i / C + rp u, as named
  // values (an array kept across a barrier would be placed in scratch memory)
  const int lc = threadIdx.x % C, lr = threadIdx.x / C;
  const ST* in = spec + R.spec_off + (size_t)T.field * M * spitch + T.kx0 +
                 (size_t)lr * spitch + (lc < ncols ? lc : 0);
  const size_t rs = (size_t)rp * spitch;
  ST l0 = in[0], l1 = in[rs], l2 = in[2 * rs], l3 = in[3 * rs], l4 = in[4 * rs],
     l5 = in[5 * rs], l6 = in[6 * rs], l7 = in[7 * rs];
  double2* tile = lds + lc * pitch;
  double2* col = lds + c * pitch;
  for (int sl = 0; sl < nslots; ++sl) {
    lds_barrier();  // every wavefront is done with the last tile
    tile[pidx(lr)] = widen(l0);
    tile[pidx(lr + rp)] = widen(l1);
    tile[pidx(lr + 2 * rp)] = widen(l2);
    tile[pidx(lr + 3 * rp)] = widen(l3);
    tile[pidx(lr + 4 * rp)] = widen(l4);
    tile[pidx(lr + 5 * rp)] = widen(l5);
    tile[pidx(lr + 6 * rp)] = widen(l6);
    tile[pidx(lr + 7 * rp)] = widen(l7);
    if (sl + 1 < nslots) {
      in += spec_slot;
      l0 = in[0];
      l1 = in[rs];
      l2 = in[2 * rs];
      l3 = in[3 * rs];
      l4 = in[4 * rs];
      l5 = in[5 * rs];
      l6 = in[6 * rs];
      l7 = in[7 * rs];
    }
    lds_barrier();  // (the next tile's loads stay in flight)
    double2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = col[pidx(t + S * q)];
    wave_fft<M>(v, col, t, tw);
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const double re = v[p].x * norm, im = v[p].y * norm;
      s2[p] = s2[p] + (re * re + im * im);
      sr[p] = sr[p] + re;
      si[p] = si[p] + im;
    }
  }
  if (live) {
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int kz = t + S * p;
      a2[kz] = s2[p];
      a2[plane + kz] = sr[p];
      a2[2 * plane + kz] = si[p];
    }
  }
  if (T.field == 0 && T.kx0 == 0) {
    for (int sl = 0; sl < nslots; ++sl) {
      __syncthreads();  // the tile (or the previous sum) is no longer read
      pressure_reduce(R, ppart + sl * ppart_slot, acc, (double*)lds);
    }
  }
}

template <typename ST>
__global__ __launch_bounds__(256) void k_col_fft(const RepInfo* reps, const ColTask* tasks,
                                                 int n_tasks, const ST* spec, int nslots,
                                                 size_t spec_slot, double* acc,
                                                 const double2* tw_base, const double* ppart,
                                                 size_t ppart_slot) {
  __shared__ double2 lds[4 * kWaveFftLds];
  // XCD-aware order: the grid is a multiple of 8 blocks, and block b runs on
  // XCD b % 8, which gets the consecutive tasks (b % 8) per_xcd ...; the
  // tiles of neighbouring columns, which share the 128-byte lines of the
  // spectrum rows, then meet in one L2
  const int per_xcd = (int)(gridDim.x >> 3);
  const int task = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (task >= n_tasks) return;  // whole block
  const ColTask T = tasks[task];
  const RepInfo& R = reps[__builtin_amdgcn_readfirstlane(T.rep)];
#define FNLB_COL(n) \
  col_fft<ST, n>(R, T, spec, nslots, spec_slot, acc, tw_base, ppart, ppart_slot, lds)
  switch (R.Lz) {
    case 8: FNLB_COL(8); break;
    case 16: FNLB_COL(16); break;
    case 32: FNLB_COL(32); break;
    case 64: FNLB_COL(64); break;
    case 128: FNLB_COL(128); break;
    case 256: FNLB_COL(256); break;
    default: FNLB_COL(512); break;
  }
#undef FNLB_COL
}

}  // namespace

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t stream) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, stream, (uint32_t*)p, n);
  return hipGetLastError();
}

hipError_t launch_advance_time(int64_t* t_base, int64_t dt, hipStream_t stream) {
  hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(64), 0, stream, t_base, dt);
  return hipGetLastError();
}

hipError_t launch_twiddles(const RepInfo* d_reps, const RepInfo* h_reps, int n_rep,
                           double2* tw_base, hipStream_t stream) {
  int maxn = 0;
  for (int r = 0; r < n_rep; ++r) maxn = std::max(maxn, h_reps[r].Lx + h_reps[r].Lz);
  const dim3 grid((maxn + 255) / 256, n_rep);
  hipLaunchKernelGGL(k_twiddles, grid, dim3(256), 0, stream, d_reps, tw_base);
  return hipGetLastError();
}

hipError_t launch_row_consts(const RepInfo* d_reps, const RepInfo* h_reps, int n_rep,
                             int precision, hipStream_t stream) {
  int maxz = 0;
  for (int r = 0; r < n_rep; ++r) maxz = std::max(maxz, h_reps[r].Lz);
  const dim3 grid((maxz + 255) / 256, n_rep);
  if (precision == FNLB_FP64)
    hipLaunchKernelGGL(k_row_consts<double>, grid, dim3(256), 0, stream, d_reps);
  else
    hipLaunchKernelGGL(k_row_consts<float>, grid, dim3(256), 0, stream, d_reps);
  return hipGetLastError();
}

hipError_t launch_row_transform(const RepInfo* reps, const RowRef* rows, int n_rows, int n_pairs,
                                int max_row_lds, int precision, const void* fields,
                                void* spec, const double2* tw, hipStream_t stream) {
  if (n_rows <= 0) return hipSuccess;
  const size_t lds = (size_t)max_row_lds * sizeof(double2);
  if (precision == FNLB_FP64)
    hipLaunchKernelGGL(k_row_transform<double>, dim3(n_rows, n_pairs), dim3(256), lds, stream,
                       reps, rows, fields, spec, tw);
  else
    hipLaunchKernelGGL(k_row_transform<float>, dim3(n_rows, n_pairs), dim3(256), lds, stream,
                       reps, rows, fields, spec, tw);
  return hipGetLastError();
}

hipError_t launch_col_transform(const RepInfo* reps, const ColRef* cols, int n_cols,
                                int max_lds_cols, int precision, const void* spec, int nslots,
                                size_t spec_slot, double* acc, const double2* tw,
                                const double* ppart, size_t ppart_slot, hipStream_t stream) {
  if (n_cols <= 0 || nslots <= 0) return hipSuccess;
  const size_t lds = (size_t)max_lds_cols * sizeof(double2);
  if (precision == FNLB_FP64)
    hipLaunchKernelGGL(k_col_transform<double2>, dim3(n_cols), dim3(256), lds, stream, reps,
                       cols, (const double2*)spec, acc, tw, ppart, nslots, spec_slot,
                       ppart_slot);
  else
    hipLaunchKernelGGL(k_col_transform<float2>, dim3(n_cols), dim3(256), lds, stream, reps,
                       cols, (const float2*)spec, acc, tw, ppart, nslots, spec_slot,
                       ppart_slot);
  return hipGetLastError();
}

hipError_t launch_row_fft(const RepInfo* reps, const RowTask* tasks, int n_tasks, int n_pairs,
                          int precision, const void* fields, void* spec, const double2* tw,
                          hipStream_t stream) {
  if (n_tasks <= 0) return hipSuccess;
  const dim3 grid((n_tasks + 3) / 4, n_pairs);
  if (precision == FNLB_FP64)
    hipLaunchKernelGGL(k_row_fft<double>, grid, dim3(256), 0, stream, reps, tasks, n_tasks,
                       fields, spec, tw);
  else
    hipLaunchKernelGGL(k_row_fft<float>, grid, dim3(256), 0, stream, reps, tasks, n_tasks,
                       fields, spec, tw);
  return hipGetLastError();
}

hipError_t launch_col_fft(const RepInfo* reps, const ColTask* tasks, int n_tasks,
                          int precision, const void* spec, int nslots, size_t spec_slot,
                          double* acc, const double2* tw, const double* ppart,
                          size_t ppart_slot, hipStream_t stream) {
  if (n_tasks <= 0 || nslots <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n_tasks + 7) / 8 * 8));  // a multiple of the 8 XCDs
  if (precision == FNLB_FP64)
    hipLaunchKernelGGL(k_col_fft<double2>, grid, dim3(256), 0, stream, reps, tasks, n_tasks,
                       (const double2*)spec, nslots, spec_slot, acc, tw, ppart, ppart_slot);
  else
    hipLaunchKernelGGL(k_col_fft<float2>, grid, dim3(256), 0, stream, reps, tasks, n_tasks,
                       (const float2*)spec, nslots, spec_slot, acc, tw, ppart, ppart_slot);
  return hipGetLastError();
}

}  // namespace fnlb
