// Device helpers of the fnlb kernels: the counter-based noise generator,
// Box-Muller in FP64 and FP32, and a wavefront sum.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fnlb {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the Philox
// S-box on a 4x32-bit counter under a 2x32-bit key; the key is bumped by the
// Weyl increments between rounds.  Multipliers and increments are the
// published ones.
struct Philox4 {
  uint32_t v[4];
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);  // truth table of a ^ b ^ c
}

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                  uint32_t c3, uint32_t k0, uint32_t k1) {
  constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
  constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t pa = (uint64_t)kMulA * c0;
    const uint64_t pb = (uint64_t)kMulB * c2;
    const uint32_t y0 = xor3((uint32_t)(pb >> 32), c1, k0);
    const uint32_t y2 = xor3((uint32_t)(pa >> 32), c3, k1);
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = y0;
    c2 = y2;
    k0 += kWeylA;
    k1 += kWeylB;
  }
  return Philox4{{c0, c1, c2, c3}};
}

// Tables of the FP64 Box-Muller, filled on the host at init (in extended
// precision) and read through the vector caches.
//  sc[j] = (sin, cos)(2 pi j / 256), j = 0..255.
//  lg[j] = (c_j, ln c_j) for the log reduction over f in [3/4, 3/2) in buckets
//          of width 1/128: c_j is 1 / (3/4 + (j + 1/2) / 128) rounded to 20
//          significant bits (so that f c_j is exact), and exactly 1 for the two
//          buckets next to f = 1 (j = 31, 32), which keeps ln u accurate to a
//          few ulps relative as u -> 1.
//  ln2 = (ln 2 rounded to 42 bits, the rest), so that e ln 2 is exact for the
//        small integers e that occur.
struct BmTables {
  double2 sc[256];
  double2 lg[96];
  double2 ln2;
};

// ln u for u = (w + 1/2) 2^-32: u = 2^e f with f in [3/4, 3/2), then
// ln u = e ln 2 - ln c_j + ln(1 + r) with r = f c_j - 1 (exact, |r| < 1/128)
// and the Taylor series of ln(1 + r) to r^8 (remainder below 1e-20).
__device__ __forceinline__ double bm_log(uint32_t w, const BmTables* __restrict__ tab) {
  const double u = ((double)w + 0.5) * 0x1.0p-32;
  int k;
  const double m = frexp(u, &k);  // u = m 2^k, m in [1/2, 1)
  const bool lo = m < 0.75;
  const double f = lo ? 2.0 * m : m;
  const int e = lo ? k - 1 : k;
  const int j = min((int)((f - 0.75) * 128.0), 95);
  const double2 cl = tab->lg[j];
  const double r = f * cl.x - 1.0;
  const double p =
      r * (1.0 + r * (-1.0 / 2 + r * (1.0 / 3 + r * (-1.0 / 4 + r * (1.0 / 5 + r * (-1.0 / 6 +
                                      r * (1.0 / 7 - r * (1.0 / 8))))))));
  const double2 ln2 = tab->ln2;
  const double ef = (double)e;
  return (ef * ln2.x - cl.y) + (p + ef * ln2.y);
}

// (sin, cos)(2 pi u) for u = (w + 1/2) 2^-32: with the angle in turns an
// exact 33-bit fraction, u = j / 256 + (d + 1/2) 2^-32 with |d + 1/2| <= 2^23,
// and the small angle a = 2 pi (d + 1/2) 2^-32 (|a| <= pi / 256) goes through
// its Taylor series (sin to a^7, 1 - cos to a^6; remainders below 1e-20).
__device__ __forceinline__ void bm_sincos(uint32_t w, const BmTables* __restrict__ tab, double& s,
                                          double& c) {
  const uint32_t jj = (w >> 24) + ((w >> 23) & 1u);  // nearest multiple of 2^24, in 2^24 units
  const int32_t d = (int32_t)(w - (jj << 24));
  const double2 t = tab->sc[jj & 255u];
  const double a = ((double)d + 0.5) * 0x1.921fb54442d18p-30;  // 2 pi 2^-32
  const double a2 = a * a;
  const double sa = a + a * a2 * (-1.0 / 6 + a2 * (1.0 / 120 - a2 * (1.0 / 5040)));
  const double q = a2 * (0.5 + a2 * (-1.0 / 24 + a2 * (1.0 / 720)));  // 1 - cos a
  s = t.x + (t.y * sa - t.x * q);
  c = t.y - (t.x * sa + t.y * q);
}

// Box-Muller (Box and Muller 1958) on u = (w + 1/2) 2^-32:
// g0 = sqrt(-2 ln u_a) cos(2 pi u_b), g1 = sqrt(-2 ln u_a) sin(2 pi u_b).
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double& g0, double& g1,
                                           const BmTables* __restrict__ tab) {
  const double r = sqrt(-2.0 * bm_log(wa, tab));
  double s, c;
  bm_sincos(wb, tab, s, c);
  g0 = r * c;
  g1 = r * s;
}

// FP32 form on the hardware transcendentals (v_log_f32 = log2, v_sqrt_f32,
// v_sin_f32 / v_cos_f32 taking the angle in turns).  -2 ln u_a uses the
// hardware log2 of the rounded u_a for u_a < 15/16; above, where rounding u_a
// to FP32 would lose the small distance to 1, it uses the series
// -ln(1 - v) = v + v^2/2 + ... + v^6/6 (truncation below 1e-8 relative for
// v <= 1/16) in v = 1 - u_a = (~w + 1/2) 2^-32, which FP32 holds to full
// relative precision.  The angle 2 pi u_b is written as pi + 2 pi x with
// x = u_b - 1/2 in (-1/2, 1/2).
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& g0, float& g1,
                                           const BmTables*) {
  constexpr float kMinus2Ln2 = -1.3862943611198906f;
  const float u = fmaf((float)wa, 0x1.0p-32f, 0x1.0p-33f);
  const float nl_log = kMinus2Ln2 * __builtin_amdgcn_logf(u);
  const float v = fmaf((float)(~wa), 0x1.0p-32f, 0x1.0p-33f);
  float p = fmaf(v, 1.0f / 6.0f, 0.2f);
  p = fmaf(v, p, 0.25f);
  p = fmaf(v, p, 1.0f / 3.0f);
  p = fmaf(v, p, 0.5f);
  p = fmaf(v, p, 1.0f);
  const float nl_ser = 2.0f * v * p;
  const float r = __builtin_amdgcn_sqrtf(wa >= 0xF0000000u ? nl_ser : nl_log);
  const float x = fmaf((float)(int)(wb ^ 0x80000000u), 0x1.0p-32f, 0x1.0p-33f);
  g0 = -r * __builtin_amdgcn_cosf(x);
  g1 = -r * __builtin_amdgcn_sinf(x);
}

// Words 4 call .. 4 call + 3 of one node and one step: counter
// (node, t_lo, t_hi, call), key (seed_lo, seed_hi).  A step takes calls 0..2
// of its own and half of call 3 of the even step of its pair (shared_words).
__device__ __forceinline__ Philox4 node_call(uint32_t node, uint64_t t, uint32_t call,
                                             uint32_t k0, uint32_t k1) {
  return philox4x32_10(node, (uint32_t)t, (uint32_t)(t >> 32), call, k0, k1);
}

// The standard normals g_{4c}, ..., g_{4c+3} (Box-Muller on the word pairs of
// call c, c = 0..2).  tab: the FP64 Box-Muller tables (unused by the FP32 form).
template <typename Real>
__device__ __forceinline__ void node_normals(uint32_t node, uint64_t t, uint32_t call,
                                             uint32_t k0, uint32_t k1, Real (&g)[4],
                                             const BmTables* tab) {
  const Philox4 r = node_call(node, t, call, k0, k1);
  box_muller(r.v[0], r.v[1], g[0], g[1], tab);
  box_muller(r.v[2], r.v[3], g[2], g[3], tab);
}

// Call 3 is shared by the steps 2s and 2s + 1 (counter (node, 2s, 3)): its
// words 0 and 1 are words 12 and 13 of step 2s, its words 2 and 3 those of
// step 2s + 1, so that two steps draw seven calls.  This step's two words in
// (w12, w13), the other step's in (o12, o13).
__device__ __forceinline__ void shared_words(uint32_t node, uint64_t t, uint32_t k0, uint32_t k1,
                                             uint32_t& w12, uint32_t& w13, uint32_t& o12,
                                             uint32_t& o13) {
  const Philox4 r = node_call(node, t & ~(uint64_t)1, 3u, k0, k1);
  const bool odd = (t & 1) != 0;
  w12 = odd ? r.v[2] : r.v[0];
  w13 = odd ? r.v[3] : r.v[1];
  o12 = odd ? r.v[0] : r.v[2];
  o13 = odd ? r.v[1] : r.v[3];
}

// Deterministic sum over the 64 lanes of a wavefront (fixed butterfly order);
// every lane receives the total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

}  // namespace fnlb
