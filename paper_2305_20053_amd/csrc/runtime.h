// Host runtime helpers: owning device buffers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "../../include/saa.h"

namespace saa_rt {

// HIP runtime status -> library status.
inline int check_hip(hipError_t e) { return e == hipSuccess ? SAA_OK : SAA_E_DEVICE; }

// Owning device allocation; freed on destruction.
// Pinned host memory (hipHostMalloc), freed with the owner.
struct HostBuf {
  void* p = nullptr;
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
  int alloc(size_t n) {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return SAA_E_OOM;
    }
    return SAA_OK;
  }
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  int alloc(size_t n) {
    release();
    if (n == 0) return SAA_OK;
    if (hipMalloc(&p, n) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return SAA_E_OOM;
    }
    bytes = n;
    return SAA_OK;
  }
  int alloc_zero(size_t n, hipStream_t st) {
    int rc = alloc(n);
    if (rc || !p) return rc;
    if (hipMemsetAsync(p, 0, n, st) != hipSuccess) return SAA_E_DEVICE;
    return SAA_OK;
  }
};

}  // namespace saa_rt
