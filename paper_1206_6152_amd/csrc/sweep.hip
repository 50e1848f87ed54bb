// sweep.hip -- directional PFC advection sweeps of the 6D distribution function
// for gfx950.
//
// Method (Sec. 2.1 of Yoshikawa, Yoshida & Umemura): along one axis every line
// of f moves with one Courant number nu = u tau / D (u is uniform along the
// line: the velocity of the cell for a position axis, the acceleration of the
// spatial cell for a velocity axis). With nu = m + alpha (m = floor |nu|,
// 0 <= alpha < 1) the new average of cell i is the old content of the
// traced-back interval (Eq. (13)), written in flux form (Eq. (16)):
//   g_k = f_k + F_{k-1} - F_k,   f'_i = g_{i-m},
//   F_k = alpha (f_k + c1 Lp_k + c2 Lm_k),
//   c1 = (1 - alpha)(2 - alpha)/6,  c2 = (1 - alpha)(1 + alpha)/6,
// for transport toward increasing index; F_k is the integral over the last
// alpha of cell k of the third-order profile with slope correctors of the PFC
// scheme (Filbet, Sonnendrucker & Bertrand 2001), whose corrected differences
// are, with f_inf the largest value of the line before the sweep,
//   Lp_k = clamp(f_{k+1} - f_k, -2 (f_inf - f_k), 2 f_k),
//   Lm_k = clamp(f_k - f_{k-1}, -2 f_k, 2 (f_inf - f_k)).
// Transport toward decreasing index is the mirror image: the line is reversed,
// updated as above and reversed back (the mapping is exact, also in rounding).
// Ghost cells are zero with zero flux (outflow) or periodic images.
//
// Execution: one lane owns one whole line in registers (the line length is a
// template parameter). Strided axes load the line straight from HBM: lanes of a
// wave hold adjacent lines, so every row access of the wave is one contiguous
// segment. Contiguous lines (the vz axis) are staged through LDS so that the
// HBM traffic stays coalesced, then transposed into registers. The alpha,
// c1, c2 of a line are computed in FP64 and rounded once to the storage type.
#include "vp_internal.h"

namespace vp {
namespace {

template <typename T>
__device__ __forceinline__ T vmin_(T a, T b) { return a < b ? a : b; }
template <typename T>
__device__ __forceinline__ T vmax_(T a, T b) { return a > b ? a : b; }

// Flux F through the right face of a cell with old values (left, centre, right).
template <typename T>
__device__ __forceinline__ T face_flux(T fl, T f0, T fr, T finf, T alpha, T c1, T c2)
{
  const T dp = fr - f0;
  const T dm = f0 - fl;
  const T room = finf - f0;
  const T lp = vmin_(vmax_(dp, T(-2) * room), T(2) * f0);
  const T lm = vmin_(vmax_(dm, T(-2) * f0), T(2) * room);
  return alpha * (f0 + c1 * lp + c2 * lm);
}

// Update one line held in registers by Courant number nu.
template <typename T, int N>
__device__ __forceinline__ void pfc_line(T (&v)[N], double nu, bool periodic)
{
  const bool neg = nu < 0.0;
  const double a = fabs(nu);
  const double fl = floor(a);
  const double alpha_d = a - fl;
  int m;
  if (fl >= (double)N) m = periodic ? (int)fmod(fl, (double)N) : N;
  else m = (int)fl;
  const T alpha = (T)alpha_d;
  const T c1 = (T)((1.0 - alpha_d) * (2.0 - alpha_d) / 6.0);
  const T c2 = (T)((1.0 - alpha_d) * (1.0 + alpha_d) / 6.0);

  // mirror so that transport is toward increasing index
#pragma unroll
  for (int i = 0; i < N / 2; i++) {
    const T x = v[i], y = v[N - 1 - i];
    v[i] = neg ? y : x;
    v[N - 1 - i] = neg ? x : y;
  }

  T finf = T(0);
#pragma unroll
  for (int i = 0; i < N; i++) finf = vmax_(finf, v[i]);

  const T ghost_l = periodic ? v[N - 1] : T(0);
  const T ghost_r = periodic ? v[0] : T(0);
  T fprev = T(0);
  if (periodic) {
    const T left_of_last = (N >= 2) ? v[N >= 2 ? N - 2 : 0] : v[0];
    fprev = face_flux(left_of_last, v[N - 1], v[0], finf, alpha, c1, c2);
  }
  T vprev = ghost_l;
#pragma unroll
  for (int i = 0; i < N; i++) {
    const T vi = v[i];
    const T vn = (i + 1 < N) ? v[i + 1 < N ? i + 1 : 0] : ghost_r;
    const T F = face_flux(vprev, vi, vn, finf, alpha, c1, c2);
    v[i] = vi + fprev - F;
    fprev = F;
    vprev = vi;
  }

  // integer part of the shift: f'_i = g_{i-m} (wrap or zero fill)
  if (m != 0) {
#pragma unroll
    for (int b = 1; b <= N; b <<= 1) {
      if (m & b) {
        T t[N];
#pragma unroll
        for (int i = 0; i < N; i++) t[i] = v[i];
#pragma unroll
        for (int i = 0; i < N; i++) {
          if (i - b >= 0) v[i] = t[i - b >= 0 ? i - b : 0];
          else v[i] = periodic ? t[(i - b + N) % N >= 0 ? (i - b + N) % N : 0] : T(0);
        }
      }
    }
  }

#pragma unroll
  for (int i = 0; i < N / 2; i++) {
    const T x = v[i], y = v[N - 1 - i];
    v[i] = neg ? y : x;
    v[N - 1 - i] = neg ? x : y;
  }
}

__device__ __forceinline__ double line_nu(const SweepArgs& a, long long o, long long c)
{
  if (a.velocity) return a.accel[o / a.sp_div] * a.scale;
  const long long j = (c / a.j_div) % a.j_mod;
  return (a.vmin + ((double)j + 0.5) * a.dv) * a.scale;
}

// Strided lines: lane = line (o, c); cells at (o*N + r)*inner + c.
template <typename T, int N>
__global__ __launch_bounds__(256) void sweep_strided(SweepArgs a)
{
  const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
  if (gid >= a.nlines) return;
  const long long o = gid / a.inner;
  const long long c = gid - o * a.inner;
  T* p = static_cast<T*>(a.f) + o * (long long)N * a.inner + c;
  T v[N];
#pragma unroll
  for (int r = 0; r < N; r++) v[r] = p[(long long)r * a.inner];
  pfc_line<T, N>(v, line_nu(a, o, c), a.periodic != 0);
#pragma unroll
  for (int r = 0; r < N; r++) p[(long long)r * a.inner] = v[r];
}

template <typename T, int N>
struct ContigShape {
  // lines per workgroup: as many as fit 40 KB of LDS (at least 64)
  static constexpr int bytes = (N + 1) * (int)sizeof(T);
  static constexpr int lines = (256 * bytes <= 40960) ? 256 : (128 * bytes <= 40960) ? 128 : 64;
};

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

template <typename VT, typename T>
__device__ __forceinline__ T lane_of(const VT& v, int q)
{
  return reinterpret_cast<const T*>(&v)[q];
}

// Contiguous lines (inner == 1): a workgroup takes LINES consecutive lines
// (one contiguous block of LINES*N elements), copies it into LDS with
// coalesced 16-byte loads (all issued before the first LDS write), gives each
// lane one line in registers, and copies the result back the same way. The LDS
// rows are padded to N+1 elements so the per-line accesses hit distinct banks.
template <typename T, int N>
__global__ __launch_bounds__((ContigShape<T, N>::lines)) void sweep_contig(SweepArgs a)
{
  constexpr int LINES = ContigShape<T, N>::lines;
  constexpr int P = N + 1;
  using VT = typename Vec16<T>::type;
  constexpr int V = Vec16<T>::n;
  constexpr bool VEC = (N % V) == 0;
  constexpr int PER = VEC ? N / V : N;   // loads per lane for a full tile
  __shared__ T tile[LINES * P];
  const int tid = threadIdx.x;
  const long long line0 = (long long)blockIdx.x * LINES;
  const long long left = a.nlines - line0;
  const int nl = left < LINES ? (int)left : LINES;
  T* g = static_cast<T*>(a.f) + line0 * N;
  if (nl == LINES) {
    if constexpr (VEC) {
      const VT* gv = reinterpret_cast<const VT*>(g);
      VT x[PER];
#pragma unroll
      for (int k = 0; k < PER; k++) x[k] = gv[tid + k * LINES];
#pragma unroll
      for (int k = 0; k < PER; k++) {
        const int e = (tid + k * LINES) * V;
#pragma unroll
        for (int q = 0; q < V; q++) tile[((e + q) / N) * P + ((e + q) % N)] = lane_of<VT, T>(x[k], q);
      }
    } else {
      T x[PER];
#pragma unroll
      for (int k = 0; k < PER; k++) x[k] = g[tid + k * LINES];
#pragma unroll
      for (int k = 0; k < PER; k++) {
        const int e = tid + k * LINES;
        tile[(e / N) * P + (e % N)] = x[k];
      }
    }
  } else {
    const int count = nl * N;
    for (int e = tid; e < count; e += LINES) tile[(e / N) * P + (e % N)] = g[e];
  }
  __syncthreads();
  if (tid < nl) {
    T v[N];
#pragma unroll
    for (int r = 0; r < N; r++) v[r] = tile[tid * P + r];
    pfc_line<T, N>(v, line_nu(a, line0 + tid, 0), a.periodic != 0);
#pragma unroll
    for (int r = 0; r < N; r++) tile[tid * P + r] = v[r];
  }
  __syncthreads();
  if (nl == LINES) {
    if constexpr (VEC) {
      VT* gv = reinterpret_cast<VT*>(g);
#pragma unroll
      for (int k = 0; k < PER; k++) {
        const int e = (tid + k * LINES) * V;
        VT x;
        T* xs = reinterpret_cast<T*>(&x);
#pragma unroll
        for (int q = 0; q < V; q++) xs[q] = tile[((e + q) / N) * P + ((e + q) % N)];
        gv[tid + k * LINES] = x;
      }
    } else {
#pragma unroll
      for (int k = 0; k < PER; k++) {
        const int e = tid + k * LINES;
        g[e] = tile[(e / N) * P + (e % N)];
      }
    }
  } else {
    const int count = nl * N;
    for (int e = tid; e < count; e += LINES) g[e] = tile[(e / N) * P + (e % N)];
  }
}

template <typename T, int N>
hipError_t launch_n(const SweepArgs& a, hipStream_t s)
{
  if (a.nlines <= 0) return hipSuccess;
  if (a.inner == 1) {
    constexpr int LINES = ContigShape<T, N>::lines;
    const long long blocks = (a.nlines + LINES - 1) / LINES;
    hipLaunchKernelGGL((sweep_contig<T, N>), dim3((unsigned)blocks), dim3(LINES), 0, s, a);
  } else {
    const long long blocks = (a.nlines + 255) / 256;
    hipLaunchKernelGGL((sweep_strided<T, N>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_t(const SweepArgs& a, hipStream_t s)
{
  switch (a.n) {
    case 1: return launch_n<T, 1>(a, s);
    case 2: return launch_n<T, 2>(a, s);
    case 3: return launch_n<T, 3>(a, s);
    case 4: return launch_n<T, 4>(a, s);
    case 6: return launch_n<T, 6>(a, s);
    case 8: return launch_n<T, 8>(a, s);
    case 12: return launch_n<T, 12>(a, s);
    case 16: return launch_n<T, 16>(a, s);
    case 24: return launch_n<T, 24>(a, s);
    case 32: return launch_n<T, 32>(a, s);
    case 48: return launch_n<T, 48>(a, s);
    case 64: return launch_n<T, 64>(a, s);
    case 96: return launch_n<T, 96>(a, s);
    case 128: return launch_n<T, 128>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool sweep_length_supported(int n)
{
  switch (n) {
    case 1: case 2: case 3: case 4: case 6: case 8: case 12: case 16:
    case 24: case 32: case 48: case 64: case 96: case 128:
      return true;
    default:
      return false;
  }
}

hipError_t launch_sweep(const SweepArgs& a, int dtype, hipStream_t s)
{
  return dtype == 0 ? launch_t<float>(a, s) : launch_t<double>(a, s);
}

}  // namespace vp
