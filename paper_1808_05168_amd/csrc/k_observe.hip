// Observables of a sample: structure factors of delta c and delta rho, and
// optionally of U_x and U_z (Appendix, Eqs. (A1)-(A4): Phi(q) = (Lx Lz)^{-1/2}
// sum_{x,j} dphi e^{-i q.r}, S(q) = <|Phi(q)|^2> on the lattice; Sec. IV.A for
// S_U) and the mean pressure (Sec. IV.C).
//
// The step kernel writes the real fields of a sample.  A row pass transforms
// two fields of a row at once as one complex sequence (z = delta c + i delta
// rho, and z = U_x + i U_z) and splits the result by Hermitian symmetry into
// the half spectra k_x = 0..Lx/2; a column pass transforms each k_x column
// over the Lz rows and adds |Phi|^2, Re Phi and Im Phi to the FP64
// accumulators.  Power-of-two lengths use an in-LDS radix-2 FFT; other
// lengths a direct sum with exactly reduced twiddle indices.  Pressure
// partials (one per strip and row) are reduced in a fixed order, so every
// accumulator is deterministic.
#include "fnlb.h"
#include "fnlb_fft.hpp"
#include "fnlb_internal.hpp"

namespace fnlb {
namespace {

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

// Row pass: one block per group of consecutive rows of one replica (several
// short rows share a block) and field pair (blockIdx.y).  LDS: the rows, then
// (power-of-two rows) the N/2 twiddles the FFT uses.
__global__ void k_row_transform(const RepInfo* reps, const RowRef* rows, const double* fields,
                                double2* spec, const double2* tw_base) {
  extern __shared__ double2 lds[];
  const RowRef rr = rows[blockIdx.x];
  const RepInfo& R = reps[rr.rep];
  const int N = R.Lx, Lz = R.Lz, nkx = N / 2 + 1, nr = rr.nrows;
  const size_t row0 = (size_t)(2 * blockIdx.y) * Lz + rr.j0;  // first field of the pair
  const double* fc = fields + R.field_off + row0 * N;
  const double* fr = fc + (size_t)Lz * N;
  const double2* tw = tw_base + R.tw_off;
  double2* out_c = spec + R.spec_off + row0 * nkx;
  double2* out_r = out_c + (size_t)Lz * nkx;
  const int total = nr * N;
  const int bits = R.pow2 ? __ffs(N) - 1 : 0;
  for (int base = threadIdx.x; base < total; base += kBatch * blockDim.x) {
    double vc[kBatch], vr[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int q = base + u * blockDim.x;
      if (q < total) {
        vc[u] = fc[q];
        vr[u] = fr[q];
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int q = base + u * blockDim.x;
      if (q < total) {
        const int d = R.pow2 ? ((q >> bits) << bits) + bitrev(q & (N - 1), bits) : q;
        lds[d] = make_double2(vc[u], vr[u]);
      }
    }
  }
  if (R.pow2) {
    double2* tws = lds + total;
    for (int m = threadIdx.x; m < N / 2; m += blockDim.x) tws[m] = tw[m];
    lds_fft(lds, bits, nr, tws);
  } else {
    __syncthreads();
  }
  // the block's threads split into one group per row
  const int gsz = blockDim.x / nr;
  const int r = threadIdx.x / gsz;
  if (r >= nr) return;
  const double2* row = lds + (size_t)r * N;
  for (int k = threadIdx.x - r * gsz; k < nkx; k += gsz) {
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
    const size_t o = (size_t)r * nkx + k;
    out_c[o] = make_double2(0.5 * (Z.x + Zm.x), 0.5 * (Z.y - Zm.y));
    out_r[o] = make_double2(0.5 * (Z.y + Zm.y), 0.5 * (Zm.x - Z.x));
  }
}

// Column pass: one block per (replica, field, tile of 2^ltile k_x columns).
// LDS: the tile's columns, then (power-of-two columns) the M/2 twiddles.
__global__ void k_col_transform(const RepInfo* reps, const ColRef* cols, const double2* spec,
                                double* acc, const double2* tw_base) {
  extern __shared__ double2 lds[];
  const ColRef cr = cols[blockIdx.x];
  const RepInfo& R = reps[cr.rep];
  const int Lx = R.Lx, M = R.Lz, nkx = Lx / 2 + 1;
  const int nc = cr.ncols, lt = cr.ltile, tmask = (1 << lt) - 1;
  const double2* in = spec + R.spec_off + (size_t)cr.field * M * nkx + cr.kx0;
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
    double2 v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int q = base + u * blockDim.x;
      if (q < total && (q & tmask) < nc) v[u] = in[(size_t)(q >> lt) * nkx + (q & tmask)];
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int q = base + u * blockDim.x;
      const int j = q >> lt, c = q & tmask;
      if (q < total && c < nc) lds[(size_t)c * M + (R.pow2 ? bitrev(j, bits) : j)] = v[u];
    }
  }
  if (R.pow2) {
    double2* tws = lds + ((size_t)M << lt);
    for (int m = threadIdx.x; m < M / 2; m += blockDim.x) tws[m] = tw[m];
    lds_fft(lds, bits, nc, tws);
    // accumulate: the three sums of a batch of entries are read before any is
    // written back
    for (int base = threadIdx.x; base < total; base += kBatch * blockDim.x) {
      double re[kBatch], im[kBatch], s2[kBatch], sr[kBatch], si[kBatch];
      size_t o[kBatch];
      bool ok[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int q = base + u * blockDim.x;
        const int c = q >> bits, kz = q & (M - 1);
        ok[u] = q < total && c < nc;
        o[u] = (size_t)c * M + kz;
        if (ok[u]) {
          const double2 P = lds[(size_t)c * M + kz];
          re[u] = P.x * norm;
          im[u] = P.y * norm;
          s2[u] = a2[o[u]];
          sr[u] = are[o[u]];
          si[u] = aim[o[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        if (ok[u]) {
          a2[o[u]] = s2[u] + (re[u] * re[u] + im[u] * im[u]);
          are[o[u]] = sr[u] + re[u];
          aim[o[u]] = si[u] + im[u];
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
}

// Pressure: one block per replica.  Row sums over strips in strip order, row
// means into the profile, then a fixed-shape tree over rows for the spatial
// mean.  Layout of the replica's block: {sum, sum2, profile[Lz]}.
__global__ void k_pressure_reduce(const RepInfo* reps, const double* ppart, double* acc) {
  extern __shared__ double rows[];
  const RepInfo& R = reps[blockIdx.x];
  const int Lz = R.Lz, ns = R.nstrips;
  const double* pp = ppart + R.ppart_off;
  double* pa = acc + R.pacc_off;
  int P2 = 1;
  while (P2 < Lz) P2 <<= 1;
  for (int j = threadIdx.x; j < P2; j += blockDim.x) {
    double s = 0.0;
    if (j < Lz) {
      for (int k = 0; k < ns; ++k) s += pp[(size_t)k * Lz + j];
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

hipError_t launch_row_transform(const RepInfo* reps, const RowRef* rows, int n_rows, int n_pairs,
                                int max_row_lds, const double* fields, double2* spec,
                                const double2* tw, hipStream_t stream) {
  if (n_rows <= 0) return hipSuccess;
  const size_t lds = (size_t)max_row_lds * sizeof(double2);
  hipLaunchKernelGGL(k_row_transform, dim3(n_rows, n_pairs), dim3(256), lds, stream, reps, rows,
                     fields, spec, tw);
  return hipGetLastError();
}

hipError_t launch_col_transform(const RepInfo* reps, const ColRef* cols, int n_cols,
                                int max_lds_cols, const double2* spec, double* acc,
                                const double2* tw, hipStream_t stream) {
  if (n_cols <= 0) return hipSuccess;
  const size_t lds = (size_t)max_lds_cols * sizeof(double2);
  hipLaunchKernelGGL(k_col_transform, dim3(n_cols), dim3(256), lds, stream, reps, cols, spec,
                     acc, tw);
  return hipGetLastError();
}

hipError_t launch_pressure_reduce(const RepInfo* reps, int n_rep, int max_lz, const double* ppart,
                                  double* acc, hipStream_t stream) {
  int P2 = 1;
  while (P2 < max_lz) P2 <<= 1;
  hipLaunchKernelGGL(k_pressure_reduce, dim3(n_rep), dim3(256), (size_t)P2 * sizeof(double),
                     stream, reps, ppart, acc);
  return hipGetLastError();
}

}  // namespace fnlb
