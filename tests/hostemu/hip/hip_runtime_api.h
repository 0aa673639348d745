// Host emulation of the few HIP runtime declarations libfcfs's host code uses.
// Test infrastructure: lets the kernels be compiled and run on the CPU (one
// std::thread per lane, a barrier per wave) to check their indexing and logic
// under the address sanitizer before they run on a GPU.
#pragma once
#include <cstddef>
typedef void* hipStream_t;
typedef int hipError_t;
#define hipSuccess 0
inline hipError_t hipGetLastError() { return hipSuccess; }
#include <cstring>
inline hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t) {
  std::memset(p, v, n);
  return hipSuccess;
}
