// Device access to the population state shared by the step and adjoint
// kernels: buffer descriptors over one replica's state block and the pull of
// a node's 18 populations (streaming with mid-way bounce-back).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fnlb {

// Populations are read and written with buffer instructions on one
// descriptor per replica state block; the plane offset is a scalar and the
// lane offset a 32-bit byte offset.  Dword 3 of the descriptor is the
// gfx9-family raw-buffer format.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ Rsrc make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           kRsrcWord3);
}

template <typename Store>
__device__ __forceinline__ Store bload(Rsrc r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float bload<float>(Rsrc r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(Rsrc r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <typename Store>
__device__ __forceinline__ void bstore(Rsrc r, uint32_t voff, uint32_t soff, Store v);
template <>
__device__ __forceinline__ void bstore<float>(Rsrc r, uint32_t voff, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}
template <>
__device__ __forceinline__ void bstore<double>(Rsrc r, uint32_t voff, uint32_t soff, double v) {
  using u2 = __attribute__((ext_vector_type(2))) uint32_t;
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, 0);
}

// Pull of the 18 populations f_l(x, jr) of one node: link l comes from
// (x - c_lx, jr - c_lz), or, where that lies beyond a wall, from link opp(l)
// of the node itself.  xb, xmb, xpb: byte offsets of columns x, x-1, x+1.
template <typename Store>
__device__ __forceinline__ void load_pulled(Rsrc r, uint32_t plane_b, uint32_t row_b, int jr,
                                            int Lz, uint32_t xb, uint32_t xmb, uint32_t xpb,
                                            Store (&o)[18]) {
  const uint32_t r0 = (uint32_t)jr * row_b;
  const uint32_t rdn = r0 - row_b, rup = r0 + row_b;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const uint32_t p = (uint32_t)(9 * s) * plane_b;
    o[9 * s + 0] = bload<Store>(r, r0 + xb, p);
    o[9 * s + 1] = bload<Store>(r, r0 + xmb, p + plane_b);
    o[9 * s + 3] = bload<Store>(r, r0 + xpb, p + 3 * plane_b);
    if (jr > 0) {
      o[9 * s + 2] = bload<Store>(r, rdn + xb, p + 2 * plane_b);
      o[9 * s + 5] = bload<Store>(r, rdn + xmb, p + 5 * plane_b);
      o[9 * s + 6] = bload<Store>(r, rdn + xpb, p + 6 * plane_b);
    } else {
      o[9 * s + 2] = bload<Store>(r, r0 + xb, p + 4 * plane_b);
      o[9 * s + 5] = bload<Store>(r, r0 + xb, p + 7 * plane_b);
      o[9 * s + 6] = bload<Store>(r, r0 + xb, p + 8 * plane_b);
    }
    if (jr < Lz - 1) {
      o[9 * s + 4] = bload<Store>(r, rup + xb, p + 4 * plane_b);
      o[9 * s + 7] = bload<Store>(r, rup + xpb, p + 7 * plane_b);
      o[9 * s + 8] = bload<Store>(r, rup + xmb, p + 8 * plane_b);
    } else {
      o[9 * s + 4] = bload<Store>(r, r0 + xb, p + 2 * plane_b);
      o[9 * s + 7] = bload<Store>(r, r0 + xb, p + 5 * plane_b);
      o[9 * s + 8] = bload<Store>(r, r0 + xb, p + 6 * plane_b);
    }
  }
}

}  // namespace fnlb
