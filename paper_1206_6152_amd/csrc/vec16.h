// vec16.h -- 16-byte vectors of the storage type (four floats or two
// doubles), for coalesced staging of f through LDS, and pairs of values of
// adjacent cells (two lines per lane). Device code only.
#pragma once

#include <hip/hip_runtime.h>

namespace vp {
namespace {

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 2;
};

template <typename T>
struct Pair2;
template <>
struct Pair2<float> {
  using type = float2;
};
template <>
struct Pair2<double> {
  using type = double2;
};

template <typename VT, typename T>
__device__ __forceinline__ T lane_of(const VT& v, int q)
{
  return reinterpret_cast<const T*>(&v)[q];
}

}  // namespace
}  // namespace vp
