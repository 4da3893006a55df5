// In-LDS radix-2 FFT shared by the structure-factor transforms and their
// adjoint.
#pragma once

#include <hip/hip_runtime.h>

namespace fnlb {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ unsigned bitrev(unsigned v, int bits) {
  return __brev(v) >> (32 - bits);
}

// In-place radix-2 decimation-in-time FFT of `ncol` sequences of length
// N = 2^lg stored column-major in LDS (buf[c * N + k], already in bit-reversed
// order); tw[m] = exp(-2 pi i m / N).  Stage s combines pairs h = 2^(s-1)
// apart with the twiddle W_{2h}^k = tw[k << (lg - s)].  Two consecutive
// stages are done by one thread on the four elements they couple (a radix-2^2
// butterfly in registers: the same operations, half the LDS round trips and
// barriers); with an odd number of stages the first runs alone.  All index
// arithmetic is shifts and masks.
__device__ inline void lds_fft(double2* buf, int lg, int ncol, const double2* tw) {
  int s = 1;
  if (lg & 1) {
    // stage 1 (h = 1, twiddle 1): pairs (2b, 2b + 1)
    const int total = ncol << (lg - 1);
    __syncthreads();
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
      double2* p = buf + 2 * q;
      const double2 u = p[0], v = cmul(p[1], tw[0]);
      p[0] = make_double2(u.x + v.x, u.y + v.y);
      p[1] = make_double2(u.x - v.x, u.y - v.y);
    }
    s = 2;
  }
  if (lg >= 2) {
    const int total = ncol << (lg - 2);  // four-element butterflies
    const int qmask = (1 << (lg - 2)) - 1;
    for (; s < lg; s += 2) {
      // stages s and s + 1: elements p0 + {0, h, 2h, 3h} of a 4h block
      const int lgh = s - 1, h = 1 << lgh;
      __syncthreads();
      for (int q = threadIdx.x; q < total; q += blockDim.x) {
        const int c = q >> (lg - 2);
        const int b = q & qmask;
        const int k = b & (h - 1);
        double2* col = buf + ((size_t)c << lg) + ((b >> lgh) << (s + 1)) + k;
        const double2 ws = tw[k << (lg - s)];
        const double2 wt = tw[k << (lg - s - 1)];
        const double2 wu = tw[(k + h) << (lg - s - 1)];
        const double2 a0 = col[0], a1 = col[h], a2 = col[2 * h], a3 = col[3 * h];
        // stage s: (a0, a1) and (a2, a3) with W_{2h}^k
        const double2 v1 = cmul(a1, ws), v3 = cmul(a3, ws);
        const double2 b0 = make_double2(a0.x + v1.x, a0.y + v1.y);
        const double2 b1 = make_double2(a0.x - v1.x, a0.y - v1.y);
        const double2 b2 = make_double2(a2.x + v3.x, a2.y + v3.y);
        const double2 b3 = make_double2(a2.x - v3.x, a2.y - v3.y);
        // stage s + 1: (b0, b2) with W_{4h}^k and (b1, b3) with W_{4h}^(k+h)
        const double2 v2 = cmul(b2, wt), v4 = cmul(b3, wu);
        col[0] = make_double2(b0.x + v2.x, b0.y + v2.y);
        col[2 * h] = make_double2(b0.x - v2.x, b0.y - v2.y);
        col[h] = make_double2(b1.x + v4.x, b1.y + v4.y);
        col[3 * h] = make_double2(b1.x - v4.x, b1.y - v4.y);
      }
    }
  }
  __syncthreads();
}

}  // namespace fnlb

namespace fnlb {

// ---- Wavefront transforms: sequences of 8 to 512 points held in registers.
//
// A sequence of N = 8 S points belongs to S lanes of one wavefront (64 / S
// sequences per wavefront), eight points per lane, and is transformed by
// Stockham passes (one of radix 2 or 4 if N is not a power of 8, then radix
// 8) in registers, with an exchange through the wavefront's own LDS between
// passes.  No block barrier is needed: the LDS operations of a wavefront are
// performed in order, and wave_sync() keeps the compiler from moving them
// across a pass boundary.  In LDS a sequence is padded by one slot per eight
// points (pidx), which spreads the stride-8 writes of a pass over the banks.

constexpr int kFftMin = 8, kFftMax = 512;
// double2 slots of one padded sequence of n points (the extra slot keeps
// neighbouring sequences on different banks)
__host__ __device__ constexpr int seq_pitch(int n) { return n + n / 8 + 1; }
// double2 slots of LDS a wavefront uses for its sequences (any N in range)
constexpr int kWaveFftLds = 640;
// (512 / N sequences of N points: 576 + 512 / N slots, largest at N = 8)
static_assert((512 / kFftMin) * seq_pitch(kFftMin) <= kWaveFftLds &&
                  seq_pitch(kFftMax) <= kWaveFftLds,
              "wavefront LDS");

__device__ __forceinline__ int pidx(int i) { return i + (i >> 3); }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block barrier that orders LDS accesses only: global loads in flight stay
// in flight across it (__syncthreads would wait for them)
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
// -i z
__device__ __forceinline__ double2 cmi(double2 a) { return make_double2(a.y, -a.x); }

// X[p] = sum_q x[q] W_4^{pq}, W_4 = -i, in place
__device__ __forceinline__ void dft4(double2& x0, double2& x1, double2& x2, double2& x3) {
  const double2 b0 = cadd(x0, x2), b1 = csub(x0, x2), b2 = cadd(x1, x3), b3 = cmi(csub(x1, x3));
  x0 = cadd(b0, b2);
  x2 = csub(b0, b2);
  x1 = cadd(b1, b3);
  x3 = csub(b1, b3);
}

// V[p] = sum_q v[q] W_8^{pq}, W_8 = exp(-2 pi i / 8), in place: the four-point
// transforms of the even and odd points, combined with W_8^p
__device__ __forceinline__ void dft8(double2 (&v)[8]) {
  double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  constexpr double h = 0.70710678118654752440;  // 1 / sqrt(2)
  // W_8 o1 = (1 - i) o1 / sqrt(2); W_8^2 o2 = -i o2; W_8^3 o3 = -(1 + i) o3 / sqrt(2)
  const double2 t1 = make_double2(h * (o1.x + o1.y), h * (o1.y - o1.x));
  const double2 t2 = cmi(o2);
  const double2 t3 = make_double2(h * (o3.y - o3.x), -h * (o3.x + o3.y));
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1);
  v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2);
  v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3);
  v[7] = csub(e3, t3);
}

// Forward DFT X[k] = sum_n x[n] W_N^{nk} of one sequence (N a power of two,
// kFftMin <= N <= kFftMax, fixed at compile time), lane t = 0 .. S - 1 of its
// group (S = N / 8).  On entry v[q] = x[t + S q]; on exit v[p] = X[t + S p].
// buf: the sequence's padded LDS slots (seq_pitch(N)); tw[m] = W_N^m =
// exp(-2 pi i m / N).  Stockham pass of radix r over sub-transforms of length
// L: butterfly b takes x[b + (N / r) q], q < r, twiddled by
// W_{rL}^{(b mod L) q}, and writes its r outputs to
// (b - b mod L) r + (b mod L) + L p.
template <int N>
__device__ __forceinline__ void wave_fft(double2 (&v)[8], double2* buf, int t,
                                         const double2* tw) {
  static_assert(N >= kFftMin && N <= kFftMax && (N & (N - 1)) == 0, "length");
  constexpr int lg = N == 8 ? 3 : N == 16 ? 4 : N == 32 ? 5 : N == 64 ? 6 : N == 128 ? 7
                                                                    : N == 256 ? 8 : 9;
  constexpr int S = N / 8, r0 = lg % 3 == 1 ? 2 : lg % 3 == 2 ? 4 : 1, n8 = lg / 3;
  if constexpr (r0 == 2) {
    // first pass of radix 2 (L = 1, no twiddles): lane t holds the
    // butterflies b = t + S i, inputs in its registers i and i + 4
    double2 o[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = cadd(v[i], v[i + 4]);
      o[2 * i + 1] = csub(v[i], v[i + 4]);
    }
    wave_sync();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      buf[pidx(2 * (t + S * i))] = o[2 * i];
      buf[pidx(2 * (t + S * i) + 1)] = o[2 * i + 1];
    }
  } else if constexpr (r0 == 4) {
    // first pass of radix 4: butterflies b = t + S i, inputs i + 2 q
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      double2 x0 = v[i], x1 = v[i + 2], x2 = v[i + 4], x3 = v[i + 6];
      dft4(x0, x1, x2, x3);
      v[i] = x0;
      v[i + 2] = x1;
      v[i + 4] = x2;
      v[i + 6] = x3;
    }
    wave_sync();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int p = 0; p < 4; ++p) buf[pidx(4 * (t + S * i) + p)] = v[i + 2 * p];
  }
  if constexpr (r0 > 1) {
    wave_sync();
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = buf[pidx(t + S * q)];
  }
  // radix-8 passes over L = r0, 8 r0, ..., N / 8; the outputs t + S p of the
  // last stay in registers
#pragma unroll
  for (int ps = 0; ps < n8; ++ps) {
    const int L = r0 << (3 * ps);
    // the pass's twiddles W_{8L}^{kq} = W_N^{kq step} are requested first, so
    // that their loads overlap the exchange
    double2 w[7];
    if (L > 1) {
      const int k = t & (L - 1), step = N / (8 * L);
#pragma unroll
      for (int q = 1; q < 8; ++q) w[q - 1] = tw[k * q * step];
      __builtin_amdgcn_sched_barrier(0);
    }
    if (ps > 0) {
      // the previous pass's outputs, through LDS
      const int Lp = L >> 3, kp = t & (Lp - 1), base = (t - kp) * 8 + kp;
      wave_sync();
#pragma unroll
      for (int p = 0; p < 8; ++p) buf[pidx(base + Lp * p)] = v[p];
      wave_sync();
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = buf[pidx(t + S * q)];
    }
    if (L > 1) {
#pragma unroll
      for (int q = 1; q < 8; ++q) v[q] = cmul(v[q], w[q - 1]);
    }
    dft8(v);
  }
}

}  // namespace fnlb
