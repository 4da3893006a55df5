// Observables of a sample: structure factors of delta c and delta rho, and
// optionally of U_x and U_z (Appendix, Eqs. (A1)-(A4): Phi(q) = (Lx Lz)^{-1/2}
// sum_{x,j} dphi e^{-i q.r}, S(q) = <|Phi(q)|^2> on the lattice; Sec. IV.A for
// S_U) and the mean pressure (Sec. IV.C).
//
// The step kernel writes the density deviations (and momenta) of a sample in
// the storage type (FP32 with FP32-deviation storage, else FP64).  A row pass forms the real fields and the pressure from them,
// transforms two fields of a row at once as one complex sequence (z = delta c
// + i delta rho, and z = U_x + i U_z) and splits the result by Hermitian
// symmetry into the half spectra k_x = 0..Lx/2; a column pass transforms each
// k_x column over the Lz rows and adds |Phi|^2, Re Phi and Im Phi to the FP64
// accumulators.  Power-of-two lengths use the in-LDS FFT; other lengths a
// direct sum with exactly reduced twiddle indices.  Pressure row sums are
// formed and reduced in a fixed order, so every accumulator is deterministic.
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

// Row pass of a sample: one block per group of consecutive rows of one
// replica (several short rows share a block) and field pair (blockIdx.y).
// The step kernel leaves, per node, the deviations of the two species
// densities from the row references (and, with velocity sampling, the total
// momenta), of type FT; this pass works in FP64.  It forms the sampled fields from them: pair 0 is
// delta c + i delta rho, together with the pressure of every node (reading
// R11: P = rho/3 + (G/4) sum_l w_l |c_l|^2 [rho^A rho^B(r + c_l) + rho^B
// rho^A(r + c_l)], ghost rows repeating the wall row) summed per row in a
// fixed order, and the check of the state; pair 1 is U_x + i U_z, the
// barycentric velocity of Eq. (10) after the wall fix.  Neighbour densities
// are read from global memory (L2) with 32-bit offsets shared by both species.
// Each row is then transformed and split into the two half spectra.  LDS: the
// rows, then (power-of-two rows) the N/2 twiddles the FFT uses.
template <typename FT>
__global__ __launch_bounds__(256) void k_row_transform(const RepInfo* reps, const RowRef* rows,
                                                       const void* fields, double2* spec,
                                                       const double2* tw_base, double* ppart,
                                                       int32_t* watchdog) {
  extern __shared__ double2 lds[];
  __shared__ double red[256 / kWave];
  const RowRef rr = rows[blockIdx.x];
  const RepInfo& R = reps[rr.rep];
  const int N = R.Lx, Lz = R.Lz, nkx = N / 2 + 1, nr = rr.nrows;
  const int pair = blockIdx.y;
  const size_t plane = (size_t)Lz * N;
  const FT* dA = (const FT*)fields + R.field_off;  // density deviations [Lz][Lx]
  const FT* dB = dA + plane;
  const FT* mX = dB + plane;  // total momenta (velocity sampling)
  const FT* mZ = mX + plane;
  const double2* tw = tw_base + R.tw_off;
  const size_t orow = (size_t)(2 * pair) * Lz + rr.j0;  // first field of the pair
  double2* out_c = spec + R.spec_off + orow * nkx;
  double2* out_r = out_c + (size_t)Lz * nkx;
  const int total = nr * N;
  const int bits = R.pow2 ? __ffs(N) - 1 : 0;
  // the block's threads split into one group per row
  const int gsz = blockDim.x / nr;
  const int r = threadIdx.x / gsz, t2 = threadIdx.x - r * gsz;
  const bool live = r < nr;
  const int j = rr.j0 + (live ? r : 0);
  const int jU = min(j + 1, Lz - 1), jD = max(j - 1, 0);
  const double rho0 = R.rho0, G = R.G;
  const double rAj = R.rA_mid + R.rA_step * j, rBj = rho0 - rAj;
  const double rAu = R.rA_mid + R.rA_step * jU, rAd = R.rA_mid + R.rA_step * jD;
  const double rBu = rho0 - rAu, rBd = rho0 - rAd;
  const double szref = R.rA_step * (double)(jU - jD) * (1.0 / 6.0);  // species A
  // reference parts of the weighted neighbour sums s^S of the pressure
  const double sAref = (1.0 / 9.0) * (2.0 * rAj + rAu + rAd) + (1.0 / 9.0) * (rAu + rAd);
  const double sBref = (1.0 / 9.0) * (2.0 * rBj + rBu + rBd) + (1.0 / 9.0) * (rBu + rBd);
  const double c0 = rAj / rho0, dPref = R.p_ref - rho0 / 3.0;
  const bool wall = (R.flags & FNLB_WALL_UZ_FIX) && (j == 0 || j == Lz - 1);
  // byte offsets of the three rows (Lx, Lz <= 4096, so 8 Lx Lz < 2^32: the
  // planes are read through 32-bit offsets from a uniform base); FS bytes per
  // value
  constexpr uint32_t FS = sizeof(FT);
  const uint32_t oC = (uint32_t)j * N * FS, oU = (uint32_t)jU * N * FS, oD = (uint32_t)jD * N * FS;
  auto ld = [](const FT* base, uint32_t off) {
    return (double)*(const FT*)((const char*)base + off);
  };
  double psum = 0.0;
  bool bad = false;
  // The sampled field(s) of node x from its 3 x 3 stencil of density
  // deviations (W, C, E of the rows below, at and above) of both species; c is
  // the node's byte offset (for the momenta).
  struct Stencil {
    double D, DW, DE, C, W, E, U, UW, UE;
  };
  auto eval = [&](int x, uint32_t c, const Stencil& A, const Stencil& B) {
    const double rhoA = rAj + A.C, rhoB = rBj + B.C;
    const double rho = rhoA + rhoB;
    double2 v;
    if (pair == 0) {
      const double drho = A.C + B.C;
      const double dc = (A.C - c0 * drho) / rho;
      const double sA = sAref + (1.0 / 9.0) * ((A.E + A.W) + (A.U + A.D)) +
                        (1.0 / 18.0) * ((A.UE + A.UW) + (A.DE + A.DW));
      const double sB = sBref + (1.0 / 9.0) * ((B.E + B.W) + (B.U + B.D)) +
                        (1.0 / 18.0) * ((B.UE + B.UW) + (B.DE + B.DW));
      const double dP = drho * (1.0 / 3.0) + G * 0.25 * (rhoA * sB + rhoB * sA) - dPref;
      psum += dP;
      bad = bad || !(rhoA > 0.0) || !(rhoB > 0.0) || !(dc + c0 > 0.0) || !(dc + c0 < 1.0) ||
            !isfinite(dP);
      v = make_double2(dc, drho);
    } else {
      // total force -G (rho^A s^B + rho^B s^A) with s^S = sum_l w_l c_l rho^S(r + c_l)
      // (the a_* and non-equilibrium parts cancel between the species)
      const double vAx = (1.0 / 9.0) * (A.E - A.W) + (1.0 / 36.0) * ((A.UE - A.UW) + (A.DE - A.DW));
      const double vBx = (1.0 / 9.0) * (B.E - B.W) + (1.0 / 36.0) * ((B.UE - B.UW) + (B.DE - B.DW));
      const double vAz =
          (1.0 / 9.0) * (A.U - A.D) + (1.0 / 36.0) * ((A.UE + A.UW) - (A.DE + A.DW)) + szref;
      const double vBz =
          (1.0 / 9.0) * (B.U - B.D) + (1.0 / 36.0) * ((B.UE + B.UW) - (B.DE + B.DW)) - szref;
      const double Fx = -G * (rhoA * vBx + rhoB * vAx);
      const double Fz = -G * (rhoA * vBz + rhoB * vAz);
      v = make_double2((ld(mX, c) + 0.5 * Fx) / rho, wall ? 0.0 : (ld(mZ, c) + 0.5 * Fz) / rho);
    }
    lds[(size_t)r * N + (R.pow2 ? bitrev(x, bits) : x)] = v;
  };
  if (live && (N & 1) == 0) {
    // even rows: a thread takes two neighbouring nodes, reading each row of
    // each species as one aligned pair (x and the row length are even) and
    // the pair's two outer neighbours
    auto ld2 = [](const FT* base, uint32_t off) {
      if constexpr (sizeof(FT) == 8) {
        return *(const double2*)((const char*)base + off);
      } else {
        const float2 v = *(const float2*)((const char*)base + off);
        return make_double2((double)v.x, (double)v.y);
      }
    };
    for (int x = 2 * t2; x < N; x += 2 * gsz) {
      const uint32_t x8 = FS * x, xm8 = x == 0 ? FS * (N - 1) : x8 - FS,
                     xq8 = x + 2 == N ? 0u : x8 + 2 * FS;
      Stencil A0, A1, B0, B1;
      auto rows = [&](const FT* base, Stencil& S0, Stencil& S1) {
        const double2 mD = ld2(base, oD + x8), mC = ld2(base, oC + x8), mU = ld2(base, oU + x8);
        const double lD = ld(base, oD + xm8), lC = ld(base, oC + xm8), lU = ld(base, oU + xm8);
        const double rD = ld(base, oD + xq8), rC = ld(base, oC + xq8), rU = ld(base, oU + xq8);
        S0 = Stencil{mD.x, lD, mD.y, mC.x, lC, mC.y, mU.x, lU, mU.y};
        S1 = Stencil{mD.y, mD.x, rD, mC.y, mC.x, rC, mU.y, mU.x, rU};
      };
      rows(dA, A0, A1);
      rows(dB, B0, B1);
      eval(x, oC + x8, A0, B0);
      eval(x + 1, oC + x8 + FS, A1, B1);
    }
  } else if (live) {
    for (int x = t2; x < N; x += gsz) {
      const uint32_t x8 = FS * x, xm8 = x == 0 ? FS * (N - 1) : x8 - FS,
                     xp8 = x == N - 1 ? 0u : x8 + FS;
      auto row3 = [&](const FT* base) {
        return Stencil{ld(base, oD + x8), ld(base, oD + xm8), ld(base, oD + xp8),
                       ld(base, oC + x8), ld(base, oC + xm8), ld(base, oC + xp8),
                       ld(base, oU + x8), ld(base, oU + xm8), ld(base, oU + xp8)};
      };
      eval(x, oC + x8, row3(dA), row3(dB));
    }
  }
  if (pair == 0) {
    // row sums of P - P_ref: a butterfly over the row's lanes within each
    // wavefront (fixed order, every lane receives the sum), then the row's
    // wavefronts in order.  gsz is a power of two: rows are grouped only on
    // power-of-two lattices, where every group holds the same power of two.
    const int w = gsz < kWave ? gsz : kWave;
    double v = psum;
    for (int m = w >> 1; m >= 1; m >>= 1) v += __shfl_xor(v, m, w);
    if (gsz > kWave) {
      if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
      __syncthreads();
      if (live && t2 == 0) {
        double sum = 0.0;
        for (int k = 0; k < gsz / kWave; ++k) sum += red[threadIdx.x / kWave + k];
        ppart[R.ppart_off + j] = sum;
      }
    } else if (live && t2 == 0) {
      ppart[R.ppart_off + j] = v;
    }
    if (bad) atomicOr(watchdog, 1);
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
    const size_t o = (size_t)r * nkx + k;
    out_c[o] = make_double2(0.5 * (Z.x + Zm.x), 0.5 * (Z.y - Zm.y));
    out_r[o] = make_double2(0.5 * (Z.y + Zm.y), 0.5 * (Zm.x - Z.x));
  }
}

// Pressure of a sample for one replica, by one block: the row sums go into the
// profile (row means), then a fixed-shape tree over the rows gives the spatial
// mean.  Layout of the replica's block: {sum, sum2, profile[Lz]}.  rows: LDS
// scratch of at least the next power of two >= Lz doubles.
__device__ void pressure_reduce(const RepInfo& R, const double* ppart, double* acc,
                                double* rows) {
  const int Lz = R.Lz;
  const double* pp = ppart + R.ppart_off;  // row sums of P - P_ref
  double* pa = acc + R.pacc_off;
  int P2 = 1;
  while (P2 < Lz) P2 <<= 1;
  for (int j = threadIdx.x; j < P2; j += blockDim.x) {
    double s = 0.0;
    if (j < Lz) {
      s = pp[j];
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
// pressure (the row pass has written all row sums).
// LDS: the tile's columns, then (power-of-two columns) the M/2 twiddles.
__global__ __launch_bounds__(256) void k_col_transform(const RepInfo* reps, const ColRef* cols,
                                                       const double2* spec, double* acc,
                                                       const double2* tw_base,
                                                       const double* ppart) {
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
    // (two plain arrays: an array of double2 assigned under a condition is
    // kept in scratch memory)
    double vr[kBatch], vi[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int q = base + u * blockDim.x;
      if (q < total && (q & tmask) < nc) {
        const double2 t = in[(size_t)(q >> lt) * nkx + (q & tmask)];
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
                                int max_row_lds, int precision, const void* fields,
                                double2* spec, const double2* tw, double* ppart,
                                int32_t* watchdog, hipStream_t stream) {
  if (n_rows <= 0) return hipSuccess;
  const size_t lds = (size_t)max_row_lds * sizeof(double2);
  if (precision == FNLB_FP64)
    hipLaunchKernelGGL(k_row_transform<double>, dim3(n_rows, n_pairs), dim3(256), lds, stream,
                       reps, rows, fields, spec, tw, ppart, watchdog);
  else
    hipLaunchKernelGGL(k_row_transform<float>, dim3(n_rows, n_pairs), dim3(256), lds, stream,
                       reps, rows, fields, spec, tw, ppart, watchdog);
  return hipGetLastError();
}

hipError_t launch_col_transform(const RepInfo* reps, const ColRef* cols, int n_cols,
                                int max_lds_cols, const double2* spec, double* acc,
                                const double2* tw, const double* ppart, hipStream_t stream) {
  if (n_cols <= 0) return hipSuccess;
  const size_t lds = (size_t)max_lds_cols * sizeof(double2);
  hipLaunchKernelGGL(k_col_transform, dim3(n_cols), dim3(256), lds, stream, reps, cols, spec,
                     acc, tw, ppart);
  return hipGetLastError();
}

}  // namespace fnlb
