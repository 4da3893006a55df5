// Access to the population state shared by the step and adjoint kernels and
// the host runtime: the layout of one replica's state block, buffer
// descriptors over it, and the pull of a node's 18 populations (streaming
// with mid-way bounce-back).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fnlb {

// Layout of one replica's state block (elements of the storage type).  Each
// row is cut into tiles of 64 columns (the row pitch is a multiple of 64), and
// a tile holds the 18 values q = 9 s + l (species s, link l) of its 64 columns
// contiguously:
//   element (q, j, x) = ((j * pitch / 64 + x / 64) * 18 + q) * 64 + x % 64.
// A wavefront's 18 loads or stores of one row then fall in a few neighbouring
// 4.6 KiB (FP32) or 9.2 KiB (FP64) blocks instead of 18 planes megabytes
// apart, which streams about 20% faster on HBM3E.  In bytes: link stride
// 64 SB, tile stride 18 * 64 SB, row stride 18 * pitch * SB.
__host__ __device__ inline size_t state_index(int q, int j, int x, int pitch) {
  return ((size_t)j * (size_t)(pitch >> 6) + (size_t)(x >> 6)) * (18 * 64) + (size_t)q * 64 +
         (size_t)(x & 63);
}

// byte offset of column x inside a row
__device__ __forceinline__ uint32_t col_offset(int x, uint32_t SB) {
  return (uint32_t)(x >> 6) * (18u * 64u * SB) + (uint32_t)(x & 63) * SB;
}

// Populations are read and written with buffer instructions on one
// descriptor per replica state block; the (row, link) offset is a scalar and
// the column offset a 32-bit per-lane byte offset.  Dword 3 of the descriptor is the
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

// State stores carry the non-temporal hint (cache-policy bit 1, "nt"): a
// stored population is read once, one whole step later, so it need not stay
// in the caches in between.  Measured on gfx950: 3-10% shorter steps for
// lattices larger than the L2, no change for smaller ones.
constexpr int kStoreNT = 2;

template <typename Store>
__device__ __forceinline__ void bstore(Rsrc r, uint32_t voff, uint32_t soff, Store v);
template <>
__device__ __forceinline__ void bstore<float>(Rsrc r, uint32_t voff, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, kStoreNT);
}
template <>
__device__ __forceinline__ void bstore<double>(Rsrc r, uint32_t voff, uint32_t soff, double v) {
  using u2 = __attribute__((ext_vector_type(2))) uint32_t;
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, kStoreNT);
}

// Pull of the 18 populations f_l(x, jr) of one node: link l comes from
// (x - c_lx, jr - c_lz), or, where that lies beyond a wall, from link opp(l)
// of the node itself.  link_b, row_b: byte strides of a link and a row;
// xb, xmb, xpb: column offsets (col_offset) of x, x-1, x+1.
template <typename Store>
__device__ __forceinline__ void load_pulled(Rsrc r, uint32_t link_b, uint32_t row_b, int jr,
                                            int Lz, uint32_t xb, uint32_t xmb, uint32_t xpb,
                                            Store (&o)[18]) {
  const uint32_t r0 = (uint32_t)jr * row_b;
  const uint32_t rdn = r0 - row_b, rup = r0 + row_b;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const uint32_t p = (uint32_t)(9 * s) * link_b;
    o[9 * s + 0] = bload<Store>(r, r0 + xb, p);
    o[9 * s + 1] = bload<Store>(r, r0 + xmb, p + link_b);
    o[9 * s + 3] = bload<Store>(r, r0 + xpb, p + 3 * link_b);
    if (jr > 0) {
      o[9 * s + 2] = bload<Store>(r, rdn + xb, p + 2 * link_b);
      o[9 * s + 5] = bload<Store>(r, rdn + xmb, p + 5 * link_b);
      o[9 * s + 6] = bload<Store>(r, rdn + xpb, p + 6 * link_b);
    } else {
      o[9 * s + 2] = bload<Store>(r, r0 + xb, p + 4 * link_b);
      o[9 * s + 5] = bload<Store>(r, r0 + xb, p + 7 * link_b);
      o[9 * s + 6] = bload<Store>(r, r0 + xb, p + 8 * link_b);
    }
    if (jr < Lz - 1) {
      o[9 * s + 4] = bload<Store>(r, rup + xb, p + 4 * link_b);
      o[9 * s + 7] = bload<Store>(r, rup + xpb, p + 7 * link_b);
      o[9 * s + 8] = bload<Store>(r, rup + xmb, p + 8 * link_b);
    } else {
      o[9 * s + 4] = bload<Store>(r, r0 + xb, p + 2 * link_b);
      o[9 * s + 7] = bload<Store>(r, r0 + xb, p + 5 * link_b);
      o[9 * s + 8] = bload<Store>(r, r0 + xb, p + 6 * link_b);
    }
  }
}

}  // namespace fnlb
