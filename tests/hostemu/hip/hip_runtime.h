// Host emulation of the HIP device-side dialect used by libfcfs kernels (see
// hip_runtime_api.h). Workgroups run one after another; the lanes of a
// workgroup are std::threads; __builtin_amdgcn_wave_barrier is a barrier over
// the 64 lanes of the wave; LDS is one static array shared by the workgroup.
#pragma once
#include <algorithm>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <thread>
#include <vector>

#include "hip_runtime_api.h"

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace hostemu {
inline thread_local dim3 tid_, bid_, grid_;
inline thread_local std::barrier<>* wave_bar_ = nullptr;
inline thread_local std::barrier<>* block_bar_ = nullptr;
constexpr size_t kLdsFloats = 160 * 1024 / 4;
}  // namespace hostemu

// The dynamic LDS arrays: every kernel declares `extern __shared__ float
// smem[]` at block scope, which names an array of its own namespace; the
// emulation main file defines one per kernel namespace and lists them here.
namespace hostemu {
extern float* const lds_arrays[];
extern const int n_lds_arrays;
}  // namespace hostemu

#define threadIdx (hostemu::tid_)
#define blockIdx (hostemu::bid_)
#define gridDim (hostemu::grid_)

template <class T> inline T min(T a, T b) { return a < b ? a : b; }
template <class T> inline T max(T a, T b) { return a > b ? a : b; }
inline float __uint_as_float(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
inline uint32_t __float_as_uint(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
#define __builtin_amdgcn_readfirstlane(x) (x)
#define __builtin_amdgcn_fence(...) ((void)0)
#define __builtin_amdgcn_sched_barrier(...) ((void)0)
#define __builtin_amdgcn_wave_barrier() (hostemu::wave_bar_->arrive_and_wait())
#define __syncthreads() (hostemu::block_bar_->arrive_and_wait())
#define __builtin_nontemporal_store(v, p) (*(p) = (v))
#define __builtin_nontemporal_load(p) (*(p))

// v_dot2 of two pairs of 16-bit values into an FP32 accumulator
template <class V>
inline float hostemu_dot2(V a, V b, float c) { return (float)a[0] * (float)b[0] + (float)a[1] * (float)b[1] + c; }
#define __builtin_amdgcn_fdot2_f32_bf16(a, b, c, clamp) hostemu_dot2(a, b, c)
#define __builtin_amdgcn_fdot2(a, b, c, clamp) hostemu_dot2(a, b, c)
// v_perm_b32: byte i of the result is byte sel[i] of the 8-byte value whose
// low word is b and high word is a (selectors 0..7 only).
inline uint32_t __builtin_amdgcn_perm(uint32_t a, uint32_t b, uint32_t sel) {
  const uint64_t v = ((uint64_t)a << 32) | b;
  uint32_t r = 0;
  for (int i = 0; i < 4; ++i) {
    const uint32_t s = (sel >> (8 * i)) & 0xffu;
    if (s > 7) std::abort();
    r |= (uint32_t)((v >> (8 * s)) & 0xffu) << (8 * i);
  }
  return r;
}

// Raw buffer resources: base and record count; reads past the count return 0.
namespace hostemu {
struct BufferRsrc {
  const char* base;
  int64_t records;
};
inline BufferRsrc make_buffer_rsrc(void* p, int, int num, int) { return BufferRsrc{static_cast<const char*>(p), num}; }
// Out-of-range loads return zero. Only the lane offset is trusted to be range
// checked: a load whose lane offset is in range but whose sum with the scalar
// offset is not would read outside the buffer on the device, so it aborts here.
inline uint32_t raw_buffer_load_b32(BufferRsrc r, int voff, int soff, int) {
  if (voff < 0 || (int64_t)voff + 4 > r.records) return 0u;
  const int64_t off = (int64_t)voff + soff;
  if (soff < 0 || off + 4 > r.records) {
    std::fprintf(stderr, "raw buffer load past the range: voff %d soff %d records %d\n", voff, soff, r.records);
    std::abort();
  }
  uint32_t v;
  std::memcpy(&v, r.base + off, 4);
  return v;
}
inline uint16_t raw_buffer_load_b16(BufferRsrc r, int voff, int soff, int) {
  if (voff < 0 || (int64_t)voff + 2 > r.records) return 0u;
  const int64_t off = (int64_t)voff + soff;
  if (soff < 0 || off + 2 > r.records) {
    std::fprintf(stderr, "raw buffer load past the range: voff %d soff %d records %d\n", voff, soff, r.records);
    std::abort();
  }
  uint16_t v;
  std::memcpy(&v, r.base + off, 2);
  return v;
}
}  // namespace hostemu
typedef hostemu::BufferRsrc __amdgpu_buffer_rsrc_t;
#define __builtin_amdgcn_make_buffer_rsrc(p, stride, num, flags) hostemu::make_buffer_rsrc(p, stride, num, flags)
#define __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, aux) hostemu::raw_buffer_load_b32(r, voff, soff, aux)
#define __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, aux) hostemu::raw_buffer_load_b16(r, voff, soff, aux)

struct uint4 {
  unsigned x, y, z, w;
};
struct uint2 {
  unsigned x, y;
};
inline uint2 make_uint2(unsigned x, unsigned y) { return uint2{x, y}; }
struct float4 {
  float x, y, z, w;
};

#ifndef __clang__
// IEEE binary16 storage with round-to-nearest-even conversion from float
// (clang has the type natively).
struct _Float16 {
  uint16_t bits;
  _Float16() = default;
  explicit _Float16(float f) {
    uint32_t u = __float_as_uint(f);
    uint32_t sign = (u >> 16) & 0x8000u;
    uint32_t a = u & 0x7fffffffu;
    if (a > 0x7f800000u) { bits = (uint16_t)(sign | 0x7e00u); return; }
    if (a >= 0x477ff000u) { bits = (uint16_t)(sign | 0x7c00u); return; }   // rounds to inf
    if (a < 0x38800000u) {                                               // subnormal or zero
      float m = __uint_as_float(a) * 16777216.0f;                        // * 2^24, exact
      bits = (uint16_t)(sign | (uint32_t)std::nearbyint(m));
      return;
    }
    uint32_t mant = a & 0x7fffffu, exp = (a >> 23) - 112;
    uint32_t h = (exp << 10) | (mant >> 13);
    uint32_t rest = mant & 0x1fffu;
    if (rest > 0x1000u || (rest == 0x1000u && (h & 1u))) ++h;
    bits = (uint16_t)(sign | h);
  }
  operator float() const {
    uint32_t sign = (uint32_t)(bits & 0x8000u) << 16;
    uint32_t e = (bits >> 10) & 0x1f, m = bits & 0x3ffu;
    if (e == 0) return (sign ? -1.f : 1.f) * (float)m / 16777216.0f;
    if (e == 31) return __uint_as_float(sign | 0x7f800000u | (m << 13));
    return __uint_as_float(sign | ((e + 112) << 23) | (m << 13));
  }
};
#endif

// Matrix-core instructions, emulated for one wave: every lane publishes its
// A and B fragments, then computes its own D entries. Operand layout of the
// 16x16x32 forms: A lane l = row l%16, k = 8*(l/16)+i; B lane l = column l%16,
// same k; D lane l = column l%16, rows 4*(l/16)+i.
namespace hostemu {
struct WaveScratch {
  float a[64][8], b[64][8];
};
inline thread_local WaveScratch* wave_scratch_ = nullptr;
template <class V8, class F4>
inline F4 mfma_16x16x32(V8 a, V8 b, F4 c) {
  const int l = (int)(tid_.x & 63);
  WaveScratch* s = wave_scratch_;
  for (int i = 0; i < 8; ++i) {
    s->a[l][i] = (float)a[i];
    s->b[l][i] = (float)b[i];
  }
  wave_bar_->arrive_and_wait();
  F4 out = c;
  for (int i = 0; i < 4; ++i) {
    const int m = 4 * (l / 16) + i, n = l % 16;
    float acc = 0.f;
    for (int k = 0; k < 32; ++k) acc += s->a[m + 16 * (k / 8)][k % 8] * s->b[n + 16 * (k / 8)][k % 8];
    out[i] += acc;
  }
  wave_bar_->arrive_and_wait();
  return out;
}
}  // namespace hostemu
// v_mfma_f32_16x16x4_f32: A lane l = row l%16, k = l/16 (one float); B lane
// l = column l%16, same k; D as above.
namespace hostemu {
template <class F4>
inline F4 mfma_16x16x4_f32(float a, float b, F4 c) {
  const int l = (int)(tid_.x & 63);
  WaveScratch* s = wave_scratch_;
  s->a[l][0] = a;
  s->b[l][0] = b;
  wave_bar_->arrive_and_wait();
  F4 out = c;
  for (int i = 0; i < 4; ++i) {
    const int m = 4 * (l / 16) + i, n = l % 16;
    float acc = 0.f;
    for (int k = 0; k < 4; ++k) acc += s->a[m + 16 * k][0] * s->b[n + 16 * k][0];
    out[i] += acc;
  }
  wave_bar_->arrive_and_wait();
  return out;
}
}  // namespace hostemu
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) hostemu::mfma_16x16x4_f32(a, b, c)
#define __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, x, y, z) hostemu::mfma_16x16x32(a, b, c)
#define __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, x, y, z) hostemu::mfma_16x16x32(a, b, c)

template <class K, class... A>
inline void hostemu_launch(K kernel, dim3 grid, dim3 block, size_t lds, A... args) {
  if (lds > hostemu::kLdsFloats * 4) std::abort();
  const unsigned nthreads = block.x, nwaves = (nthreads + 63) / 64;
  // One worker thread per lane, reused for every workgroup; fresh barriers per
  // workgroup (lanes that return early drop out of them).
  std::vector<std::unique_ptr<std::barrier<>>> bars;
  std::unique_ptr<std::barrier<>> block_bar;
  std::barrier<> start((std::ptrdiff_t)nthreads + 1), done((std::ptrdiff_t)nthreads + 1);
  std::vector<hostemu::WaveScratch> scratch(nwaves);
  unsigned long long cur = 0;
  auto prepare = [&](unsigned long long b) {
    bars.clear();
    for (unsigned w = 0; w < nwaves; ++w)
      bars.emplace_back(new std::barrier<>((std::ptrdiff_t)std::min(64u, nthreads - 64 * w)));
    block_bar.reset(new std::barrier<>((std::ptrdiff_t)nthreads));
    for (int i = 0; i < hostemu::n_lds_arrays; ++i)   // stale LDS reads as NaN
      std::memset(hostemu::lds_arrays[i], 0xff, lds);
    cur = b;
  };
  // workgroups in x-fastest order over the whole (x, y, z) grid
  const unsigned long long nblocks = (unsigned long long)grid.x * grid.y * grid.z;
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nthreads; ++t)
    th.emplace_back([&, t] {
      for (unsigned long long b = 0; b < nblocks; ++b) {
        start.arrive_and_wait();
        hostemu::tid_ = dim3(t, 0, 0);
        hostemu::bid_ = dim3(cur % grid.x, (cur / grid.x) % grid.y, cur / ((unsigned long long)grid.x * grid.y));
        hostemu::grid_ = grid;
        hostemu::wave_bar_ = bars[t / 64].get();
        hostemu::block_bar_ = block_bar.get();
        hostemu::wave_scratch_ = &scratch[t / 64];
        kernel(args...);
        hostemu::wave_bar_->arrive_and_drop();
        hostemu::block_bar_->arrive_and_drop();
        done.arrive_and_wait();
      }
    });
  for (unsigned long long b = 0; b < nblocks; ++b) {
    prepare(b);
    start.arrive_and_wait();
    done.arrive_and_wait();
  }
  for (auto& x : th) x.join();
}
#define hipLaunchKernelGGL(k, grid, block, lds, stream, ...) hostemu_launch(k, grid, block, lds, __VA_ARGS__)
