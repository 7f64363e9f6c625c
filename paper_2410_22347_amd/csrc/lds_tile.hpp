// Direct copies from global memory into LDS for the workgroup-shared tile
// ring of the scoring kernel.
#pragma once

#include "search_common.hpp"

namespace gv {
namespace scan {

// One lane's 16 bytes from global memory straight into LDS: lane i of the
// wavefront writes lds_base + 16 i (lds_base is the same for every lane).
// Written as asm so that the compiler does not order the ring reads behind
// every copy in flight; the caller waits on the memory counter itself.  The
// instruction writes no register, so nothing of it is left in flight for the
// compiler to reuse; M0 is restored before the block ends.
__device__ __forceinline__ void copy_lds16(const void* g, uint32_t lds_base) {
  const uint32_t base = __builtin_amdgcn_readfirstlane(lds_base);
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n"
      "s_nop 1\n"
      "s_mov_b32 m0, %2\n"
      "s_nop 0\n"
      "global_load_lds_dwordx4 %1, off\n"
      "s_nop 1\n"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "v"(g), "s"(base)
      : "memory");
}

}  // namespace scan
}  // namespace gv
