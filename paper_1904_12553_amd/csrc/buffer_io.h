// buffer_io.h -- state access of the step kernels through buffer
// instructions (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nplbm {

// State access through buffer instructions.  In the row-interleaved layout
// one row of a state group (all its planes) is one contiguous block, so a
// buffer resource is built per (group, row) in scalar registers, and an
// element is addressed by a scalar plane offset plus a per-lane column
// offset shared by all planes: one buffer_load / buffer_store per value
// with no per-access vector address arithmetic.  The resource's size is the
// row block, so an offset outside it reads 0 / drops the store instead of
// touching other memory.
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format

__device__ __forceinline__ Rsrc row_rsrc(const void *base, uint32_t row_bytes, int y) {
  return __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char *>(static_cast<const char *>(base)) + (size_t)y * row_bytes, (short)0,
      (int)row_bytes, kRsrcWord3);
}
template <typename Real>
__device__ __forceinline__ Real bld(Rsrc r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(Real) == 8)
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  else
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
// Stores of the new state are never read again within the step; kNT marks
// them nontemporal (streaming).  Measured faster wherever each wave's row
// of stores covers whole cache lines: every FP64 kernel, the FP32 2-D rows
// of interior lanes (2048^2 N = 5: 62.2% -> 62.9% of the HBM roofline,
// 4096^2 N = 3: 66.9% -> 70.9%) and the D3Q15 passes (256^3 N = 3: 48.1%
// -> 51.0%); slower on the FP32 rows that hold their halo (mixed N = 5:
// 58.4% -> 57.1%).
template <typename Real, bool kNT>
__device__ __forceinline__ void bst(Rsrc r, uint32_t voff, uint32_t soff, Real v) {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  constexpr int kAux = kNT ? 2 : 0;  // cache-policy bit nt of gfx94x/gfx950
  if constexpr (sizeof(Real) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, kAux);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, kAux);
}

}  // namespace nplbm
