// Helpers shared by the fused pair kernels (FP32 and FP64 forms).
#pragma once

#include "kernels.hpp"

namespace fockmi {

// LDS element at a per-thread byte offset plus a compile-time byte offset; the
// constant folds into the instruction's 16-bit immediate when below 64 KiB.
template <unsigned C, typename E>
__device__ __forceinline__ E& lds_at(E* lds, unsigned off) {
  static_assert(C < 65536u, "LDS immediate offset out of range");
  return *reinterpret_cast<E*>(reinterpret_cast<char*>(lds) + off + C);
}

// Hides a value from loop-invariant code motion: addresses derived from it are
// formed where they are used (base register + immediate) instead of being
// hoisted out of the pair loop, one register each, and spilled.
__device__ __forceinline__ unsigned opaque(unsigned x) {
  asm volatile("" : "+v"(x));
  return x;
}

__device__ __forceinline__ double ld_f64(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

}  // namespace fockmi
