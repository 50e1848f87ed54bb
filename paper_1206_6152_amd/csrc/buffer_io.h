// buffer_io.h -- raw buffer loads and stores for the sweep kernels. A buffer
// resource (base address, size in bytes) lives in scalar registers; each
// access adds a per-lane 32-bit byte offset and a uniform 32-bit byte offset,
// so a lane needs one address register for any number of rows. Accesses past
// the size read zero and write nothing. Device code only.
#pragma once

#include <hip/hip_runtime.h>

namespace vp {
namespace {

// resource word 3 for gfx9-family raw buffers: 32-bit data format, no swizzle
constexpr int kBufWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, unsigned bytes)
{
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufWord3);
}

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <typename T>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, T x);
template <>
__device__ __forceinline__ void buf_store<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float x)
{
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, voff, soff, 0);
}
template <>
__device__ __forceinline__ void buf_store<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double x)
{
  using U2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, x), r, voff, soff, 0);
}

// 8 bytes: the values of two adjacent FP32 cells
__device__ __forceinline__ float2 buf_load_pair(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// 16 bytes: four floats or two doubles. The whole offset is per lane and the
// uniform offset field is the constant 0: with a register there, the
// compiler's check for the hazard of a store wider than 8 bytes whose data
// registers are rewritten right after issue does not fire on this target,
// and an immediately following register write can replace data the store
// has not yet read.
template <typename VT>
__device__ __forceinline__ void buf_store16(__amdgpu_buffer_rsrc_t r, unsigned voff, const VT& x)
{
  static_assert(sizeof(VT) == 16, "16-byte vector");
  using U4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0u, 0u, 0));
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, x), r, voff, 0u, 0);
}

}  // namespace
}  // namespace vp
