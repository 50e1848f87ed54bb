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
// Transport toward decreasing index is the mirror image: the same update on the
// reversed line, which rounds identically. The plain sweeps reverse by renaming
// registers (a wave whose lines all move one way) or with selects (a wave with
// both signs); the one-pass kernels hold each axis in LDS in the orientation
// of its sweep. Ghost cells are zero with zero flux (outflow) or periodic
// images. Since f_k <= f_inf, the clamp bounds are always ordered, so each
// clamp is one median-of-three.
//
// Execution: one lane owns one whole line in registers (the line length is a
// template parameter). Strided axes load the line straight from HBM: lanes of a
// wave hold adjacent lines, so every row access of the wave is one contiguous
// segment. Contiguous lines (the vz axis) are staged through LDS so that the
// HBM traffic stays coalesced, then transposed into registers. Several sweeps
// share one pass over HBM where their lines fit on chip together: a half kick
// (or two in a row) on a whole velocity block, in LDS or, for FP64 32^3
// blocks, in registers with LDS between axes; two velocity sweeps on slices
// of a block; and T_z T_y on an x index times a chunk of velocity cells. The alpha, c1, c2 of a line are computed in FP64
// and rounded once to the storage type. The whole-cell part m of the shift is
// applied as the line is written out: each cell goes once to its shifted place.
#include "vp_internal.h"

#include "pfc_line.h"
#include "buffer_io.h"

#include "vec16.h"

namespace vp {
namespace {

// Strided lines, general addressing: lane = line (o, c); cells at (o*N + r)*inner + c.
__device__ __forceinline__ double line_nu_wide(const SweepArgs& a, long long o, long long c)
{
  if (a.velocity) return a.accel[o / a.sp_div] * a.scale;
  const long long j = (c / a.j_div) % a.j_mod;
  return (a.vmin + ((double)j + 0.5) * a.dv) * a.scale;
}

template <typename T, int N>
__global__ __launch_bounds__(256) void sweep_strided_wide(SweepArgs a)
{
  const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
  if (gid >= a.nlines) return;
  const long long o = gid / a.inner;
  const long long c = gid - o * a.inner;
  const long long base = o * (long long)N * a.inner + c;
  const T* p = static_cast<const T*>(a.f) + base;
  T* q = static_cast<T*>(a.out ? a.out : a.f) + base;
  const long long inner = a.inner;
  T v[N];
#pragma unroll
  for (int r = 0; r < N; r++) v[r] = p[(long long)r * inner];
  const LineCoef<T> k = pfc_line<T, N>(v, line_nu_wide(a, o, c), a.periodic != 0);
  store_shifted<T, N>(v, k.shift, a.periodic != 0, [&](int r, T x) { q[(long long)r * inner] = x; });
}

// Strided lines, compact addressing: the workgroup's first line is the uniform
// base; a lane's cells sit at base + r*inner + off with a 32-bit offset (the
// host checks that every offset fits), and the line index arithmetic is 32-bit.
// PART (x sweep, 256 lines of one spatial (y, z) column per workgroup): the
// workgroup also sums its lines' new values at each x in FP64, in a fixed
// order, into part[blockIdx.x * N + x], so the density needs no extra pass
// over f.
template <typename T, int N>
struct PartShape {
  // P lanes share one x row's sum: the largest power of two (at most 64)
  // with N*P <= 256; each adds 256/P of the row's values in a fixed order,
  // then the P partial sums meet in a butterfly
  static constexpr int P = N * 64 <= 256 ? 64 : N * 32 <= 256 ? 32 : N * 16 <= 256 ? 16 :
                           N * 8 <= 256 ? 8 : N * 4 <= 256 ? 4 : N * 2 <= 256 ? 2 : 1;
  static constexpr int ROW = 256 + P;    // padded LDS row: the reads below hit distinct banks
  static constexpr bool ok = N >= 1 && N <= 256 && N * ROW * (int)sizeof(T) <= 68 * 1024;
};

template <typename T, int N, bool PART>
__global__ __launch_bounds__(256) void sweep_strided(SweepArgs a)
{
  const long long gid0 = (long long)blockIdx.x * 256;
  const unsigned t = threadIdx.x;
  if (gid0 + t >= a.nlines) return;
  const long long o0 = gid0 / a.inner;
  const unsigned inner = (unsigned)a.inner;
  const unsigned c0 = (unsigned)(gid0 - o0 * a.inner);
  const unsigned cc = c0 + t;
  const unsigned dov = cc / inner;          // slabs past the base line's slab
  const unsigned c = cc - dov * inner;
  const unsigned off = dov * (unsigned)(N * inner) + c - c0;
  const long long b0 = o0 * N * (long long)inner + c0;
  const T* fb = static_cast<const T*>(a.f) + b0;
  T* ob = static_cast<T*>(a.out ? a.out : a.f) + b0;
  double nu;
  if (a.velocity) {
    const long long sp_div = a.sp_div;
    const long long q0 = o0 / sp_div;
    const unsigned r0 = (unsigned)(o0 - q0 * sp_div);
    nu = a.accel[q0 + (r0 + dov) / (unsigned)sp_div] * a.scale;
  } else {
    const unsigned j = (c / (unsigned)a.j_div) % (unsigned)a.j_mod;
    nu = (a.vmin + ((double)j + 0.5) * a.dv) * a.scale;
  }
  T v[N];
#pragma unroll
  for (int r = 0; r < N; r++) v[r] = (fb + (long long)r * inner)[off];
  const LineCoef<T> k = pfc_line<T, N>(v, nu, a.periodic != 0);
  store_shifted<T, N>(v, k.shift, a.periodic != 0, [&](int r, T x) { (ob + (long long)r * inner)[off] = x; });
  if constexpr (PART) {
    // every lane of the workgroup is live here (the host checks it)
    using PS = PartShape<T, N>;
    __shared__ T tile[N * PS::ROW];   // row r: the new values at x = r of the 256 lines
    store_shifted<T, N>(v, k.shift, a.periodic != 0, [&](int r, T x) { tile[r * PS::ROW + t] = x; });
    __syncthreads();
    const int row = t / PS::P, q = t % PS::P;
    if (row < N) {                    // N*P may be under 256: the other lanes idle
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < 256 / PS::P; j++) acc += (double)tile[row * PS::ROW + j * PS::P + q];
#pragma unroll
      for (int o = PS::P / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (q == 0) a.part[(long long)blockIdx.x * N + row] = acc;
    }
  }
}

template <typename T, int N>
struct ContigShape {
  // lines per workgroup: as many as fit 40 KB of LDS (at least 64)
  static constexpr int bytes = (N + 1) * (int)sizeof(T);
  static constexpr int lines = (256 * bytes <= 40960) ? 256 : (128 * bytes <= 40960) ? 128 : 64;
};


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
  const T* g = static_cast<const T*>(a.f) + line0 * N;
  T* go = static_cast<T*>(a.out ? a.out : a.f) + line0 * N;
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
  double nu;
  if (a.velocity) {
    const long long q0 = line0 / a.sp_div;
    const unsigned r0 = (unsigned)(line0 - q0 * a.sp_div);
    nu = a.accel[q0 + (r0 + (unsigned)tid) / (unsigned)a.sp_div] * a.scale;
  } else {
    nu = (a.vmin + 0.5 * a.dv) * a.scale;   // inner == 1: one velocity cell on this axis
  }
  __syncthreads();
  if (tid < nl) {
    T* row = tile + tid * P;
    T v[N];
#pragma unroll
    for (int r = 0; r < N; r++) v[r] = row[r];
    const LineCoef<T> k = pfc_line<T, N>(v, nu, a.periodic != 0);
    store_shifted<T, N>(v, k.shift, a.periodic != 0, [&](int r, T x) { row[r] = x; });
  }
  __syncthreads();
  if (nl == LINES) {
    if constexpr (VEC) {
      VT* gv = reinterpret_cast<VT*>(go);
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
        go[e] = tile[(e / N) * P + (e % N)];
      }
    }
  } else {
    const int count = nl * N;
    for (int e = tid; e < count; e += LINES) go[e] = tile[(e / N) * P + (e % N)];
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
    const bool narrow = narrow_ok(a, N);
    if (narrow && a.part) {
      if constexpr (PartShape<T, N>::ok)
        hipLaunchKernelGGL((sweep_strided<T, N, true>), dim3((unsigned)blocks), dim3(256), 0, s, a);
      else
        return hipErrorInvalidValue;
    } else if (a.part) {
      return hipErrorInvalidValue;
    } else if (narrow)
      hipLaunchKernelGGL((sweep_strided<T, N, false>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((sweep_strided_wide<T, N>), dim3((unsigned)blocks), dim3(256), 0, s, a);
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

// compact addressing when every lane offset from its workgroup's first line
// fits in 31 bits and the index arithmetic fits in 32 bits
bool narrow_ok(const SweepArgs& a, int N)
{
  const bool no_straddle = (a.inner % 256) == 0;
  const long long span = no_straddle ? 256 : (256 / a.inner + 2) * (long long)N * a.inner;
  return a.inner < (1LL << 31) && span < (1LL << 31) && a.j_div < (1LL << 31) && a.j_mod < (1LL << 31) &&
         a.sp_div < (1LL << 31);
}

template <typename T>
bool part_shape_ok(int n)
{
  switch (n) {
    case 1: return PartShape<T, 1>::ok;
    case 2: return PartShape<T, 2>::ok;
    case 3: return PartShape<T, 3>::ok;
    case 4: return PartShape<T, 4>::ok;
    case 6: return PartShape<T, 6>::ok;
    case 8: return PartShape<T, 8>::ok;
    case 12: return PartShape<T, 12>::ok;
    case 16: return PartShape<T, 16>::ok;
    case 24: return PartShape<T, 24>::ok;
    case 32: return PartShape<T, 32>::ok;
    case 48: return PartShape<T, 48>::ok;
    case 64: return PartShape<T, 64>::ok;
    case 96: return PartShape<T, 96>::ok;
    case 128: return PartShape<T, 128>::ok;
    default: return false;
  }
}

bool sweep_part_supported(const SweepArgs& a, int dtype)
{
  // whole workgroups of lines (no lane leaves early), strided lines, compact addressing
  if (a.inner % 256 != 0 || a.nlines % 256 != 0 || !narrow_ok(a, a.n)) return false;
  return dtype == 0 ? part_shape_ok<float>(a.n) : part_shape_ok<double>(a.n);
}

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
