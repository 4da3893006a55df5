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
