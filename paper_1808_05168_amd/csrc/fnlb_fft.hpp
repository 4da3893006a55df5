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
// order); tw[m] = exp(-2 pi i m / N).  All index arithmetic is shifts and masks.
__device__ inline void lds_fft(double2* buf, int lg, int ncol, const double2* tw) {
  const int half = 1 << (lg - 1);
  const int total = half * ncol;
  for (int s = 1; s <= lg; ++s) {
    const int lgh = s - 1, h = 1 << lgh, tsh = lg - s;
    __syncthreads();
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
      const int c = q >> (lg - 1);
      const int b = q & (half - 1);
      const int k = b & (h - 1);
      const int i0 = ((b >> lgh) << s) + k, i1 = i0 + h;
      double2* col = buf + ((size_t)c << lg);
      const double2 w = tw[k << tsh];
      const double2 u = col[i0];
      const double2 v = cmul(col[i1], w);
      col[i0] = make_double2(u.x + v.x, u.y + v.y);
      col[i1] = make_double2(u.x - v.x, u.y - v.y);
    }
  }
  __syncthreads();
}

}  // namespace fnlb
