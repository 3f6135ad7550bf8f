// Global → LDS copies through buffer loads (gfx950): the LDS address space
// type and a raw buffer resource whose reads past the end return 0.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace higp {

typedef __attribute__((address_space(3))) void lds_void_t;

// Buffer resource over `bytes` bytes at `base` (reads past the end return 0).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  const int nrec = bytes > 0x7fffffff ? 0x7fffffff : (int)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, nrec, 0x00020000);
}

}  // namespace higp
