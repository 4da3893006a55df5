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

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ unsigned bitrev(unsigned v, int bits) {
  return __brev(v) >> (32 - bits);
}

// In-place radix-2 decimation-in-time FFT of `ncol` sequences of length N
// stored column-major in LDS (buf[c * N + k], already in bit-reversed order);
// tw[m] = exp(-2 pi i m / N).
__device__ void lds_fft(double2* buf, int N, int ncol, const double2* tw) {
  const int half = N >> 1;
  const int total = half * ncol;
  for (int len = 2; len <= N; len <<= 1) {
    const int h = len >> 1;
    const int tstep = N / len;
    __syncthreads();
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
      const int c = q / half;
      const int b = q - c * half;
      const int grp = b / h, k = b - grp * h;
      const int i0 = grp * len + k, i1 = i0 + h;
      double2* col = buf + (size_t)c * N;
      const double2 w = tw[k * tstep];
      const double2 u = col[i0];
      const double2 v = cmul(col[i1], w);
      col[i0] = make_double2(u.x + v.x, u.y + v.y);
      col[i1] = make_double2(u.x - v.x, u.y - v.y);
    }
  }
  __syncthreads();
}

// Row pass: one block per (replica, row) and field pair (blockIdx.y).
__global__ void k_row_transform(const RepInfo* reps, const RowRef* rows, const double* fields,
                                double2* spec, const double2* tw_base) {
  extern __shared__ double2 lds[];
  const RowRef rr = rows[blockIdx.x];
  const RepInfo& R = reps[rr.rep];
  const int N = R.Lx, Lz = R.Lz, nkx = N / 2 + 1;
  const size_t row = (size_t)(2 * blockIdx.y) * Lz + rr.j;  // first field of the pair
  const double* fc = fields + R.field_off + row * N;
  const double* fr = fc + (size_t)Lz * N;
  const double2* tw = tw_base + R.tw_off;
  double2* out_c = spec + R.spec_off + row * nkx;
  double2* out_r = out_c + (size_t)Lz * nkx;
  if (R.pow2) {
    const int bits = __ffs(N) - 1;
    for (int x = threadIdx.x; x < N; x += blockDim.x)
      lds[bitrev(x, bits)] = make_double2(fc[x], fr[x]);
    lds_fft(lds, N, 1, tw);
  } else {
    for (int x = threadIdx.x; x < N; x += blockDim.x) lds[x] = make_double2(fc[x], fr[x]);
    __syncthreads();
  }
  for (int k = threadIdx.x; k < nkx; k += blockDim.x) {
    double2 Z, Zm;
    if (R.pow2) {
      Z = lds[k];
      Zm = lds[(N - k) & (N - 1)];
    } else {
      // direct sum for Z(k) and Z(N-k)
      double zr = 0, zi = 0, mr = 0, mi = 0;
      const int km = (N - k) % N;
      int ik = 0, im = 0;
      for (int x = 0; x < N; ++x) {
        const double2 a = lds[x];
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
    out_c[k] = make_double2(0.5 * (Z.x + Zm.x), 0.5 * (Z.y - Zm.y));
    out_r[k] = make_double2(0.5 * (Z.y + Zm.y), 0.5 * (Zm.x - Z.x));
  }
}

// Column pass: one block per (replica, field, tile of k_x columns).
__global__ void k_col_transform(const RepInfo* reps, const ColRef* cols, const double2* spec,
                                double* acc, const double2* tw_base) {
  extern __shared__ double2 lds[];
  const ColRef cr = cols[blockIdx.x];
  const RepInfo& R = reps[cr.rep];
  const int Lx = R.Lx, M = R.Lz, nkx = Lx / 2 + 1;
  const int nc = cr.ncols;
  const double2* in = spec + R.spec_off + (size_t)cr.field * M * nkx;
  const double2* tw = tw_base + R.tw_off + Lx;
  const size_t plane = (size_t)M * nkx;
  double* a2 = acc + R.acc_off + (size_t)cr.field * 3 * plane;
  double* are = a2 + plane;
  double* aim = a2 + 2 * plane;
  const double norm = R.inv_norm;
  const int bits = __ffs(M) - 1;
  // load: row-major reads of nc consecutive k_x per row
  for (int q = threadIdx.x; q < M * nc; q += blockDim.x) {
    const int j = q / nc, c = q - j * nc;
    const double2 v = in[(size_t)j * nkx + cr.kx0 + c];
    lds[(size_t)c * M + (R.pow2 ? bitrev(j, bits) : j)] = v;
  }
  if (R.pow2) {
    lds_fft(lds, M, nc, tw);
    for (int q = threadIdx.x; q < M * nc; q += blockDim.x) {
      const int kz = q / nc, c = q - kz * nc;
      const double2 P = lds[(size_t)c * M + kz];
      const double re = P.x * norm, im = P.y * norm;
      const size_t o = (size_t)kz * nkx + cr.kx0 + c;
      a2[o] += re * re + im * im;
      are[o] += re;
      aim[o] += im;
    }
  } else {
    __syncthreads();
    for (int q = threadIdx.x; q < M * nc; q += blockDim.x) {
      const int kz = q / nc, c = q - kz * nc;
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
      const size_t o = (size_t)kz * nkx + cr.kx0 + c;
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
                                int max_lx, const double* fields, double2* spec,
                                const double2* tw, hipStream_t stream) {
  if (n_rows <= 0) return hipSuccess;
  const size_t lds = (size_t)max_lx * sizeof(double2);
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
