// gfx950 asynchronous global -> LDS copies and the waits that go with them.
//
// global_load_lds_dwordx4 moves 16 bytes per lane from global memory straight
// into LDS (lane i's bytes land at the wave-uniform base + 16 i), with no
// registers holding the data in flight.  The compiler does not track these
// copies, so completion is waited for explicitly with vmcnt (the count of this
// wave's outstanding vector-memory operations, copies and loads alike, which
// retire in issue order for loads), and a bare s_barrier (no fence, which
// would wait for every copy in flight) publishes every wave's completed
// copies to the workgroup.
#pragma once

#include "common.h"

namespace rise {
namespace async {

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt field is 6 bits");
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
#endif
}

__device__ __forceinline__ void wait_lgkmcnt0() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#endif
}

// workgroup barrier without a memory fence; the scheduling barriers keep the
// compiler from moving any instruction across it
__device__ __forceinline__ void barrier() {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_barrier" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
#endif
}

// 16 bytes per lane, global -> LDS at lds_base + 16 * lane (lds_base wave-uniform).
// Written as inline asm (the LDS base goes to M0 through the operand
// constraint): issued through the builtin, the copy counts for the compiler as
// a memory access that may touch both global memory and LDS, and while one is
// outstanding it can only wait for LDS reads with lgkmcnt(0), which exposes the
// latency of the newest fragment read before every MFMA that needs an older
// one.  Hidden from the compiler, the copies are tracked by the explicit vmcnt
// waits alone (the compiler's own vmcnt waits stay safe: loads retire in
// order, so untracked copies only make them wait longer).
__device__ __forceinline__ void copy16(const void* src, void* lds_base) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t base = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)((__attribute__((address_space(3))) char*)lds_base));
  asm volatile("global_load_lds_dwordx4 %0, off" ::"v"(src), "{m0}"(base) : "memory");
#endif
}
// 4 bytes per lane, global -> LDS at lds_base + 4 * lane, the same way
__device__ __forceinline__ void copy4(const void* src, void* lds_base) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t base = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)((__attribute__((address_space(3))) char*)lds_base));
  asm volatile("global_load_lds_dword %0, off" ::"v"(src), "{m0}"(base) : "memory");
#endif
}

}  // namespace async
}  // namespace rise
