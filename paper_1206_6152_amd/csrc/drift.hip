// drift.hip -- the position sweeps T_z then T_y of Eq. (17) (Sec. 2.1 of
// Yoshikawa, Yoshida & Umemura) in one pass over f, for square (y, z) planes
// that fit on chip with a chunk of velocity cells. The line update is that of
// sweep.hip (pfc_line.h), so the pass rounds like the single sweeps. gfx950.
#include "vp_internal.h"

#include "pfc_line.h"

namespace vp {
namespace {

// ---- one-pass drift along z, then y -----------------------------------------
// A tile is one x index and W consecutive velocity cells of every (y, z) cell
// (W contiguous values per (y, z) cell in HBM, one or more whole cache lines).
// Each z line of a tile is read from HBM by one lane, updated in registers and
// parked in LDS; after a barrier each y line is taken from LDS by one lane,
// updated and written back to HBM. f crosses HBM once for the two sweeps.
// Rows of W are unpadded; planes are padded to SY = W (mod 64) elements so
// both sweep directions are bank-conflict free.
//
// Each line takes the forward form of the update with |nu|: a z line whose
// vz is negative is mirrored in registers after its (storage-order) load and
// parked in LDS in that order; the LDS rows are laid out in the orientation
// of each column's y sweep, and a y line is stored back in storage order.
//
// The Courant-number coefficients of both sweeps depend only on the velocity
// cell, so drift_table_kernel computes them once per call for every velocity
// cell (the same line_coef as every other sweep, so the bits agree) and a lane
// reads its two entries instead of dividing indices and coefficients in FP64.
// Addresses are 32-bit byte offsets from uniform row bases (a tile spans under
// 4 GiB, checked on the host).
//
// The grid is (velocity-chunk groups, x); a workgroup takes TILES consecutive
// chunks. The z lines of the next tile are loaded into registers while the
// current tile's y lines are swept and stored, so that the single workgroup an
// LDS-sized tile leaves on a CU keeps loads in flight while it computes. The
// tile loop is unrolled at compile time, which keeps every memory-counter wait
// exact.
template <typename T, int NY, int NZ, int W>
struct DriftShape {
  static constexpr int SY0 = NZ * W;
  static constexpr int SY = SY0 + ((((W - SY0) % 64) + 64) % 64);
  static constexpr int ELEMS = NY * SY;
  static constexpr int BYTES = ELEMS * (int)sizeof(T);
  static constexpr int LZ = NY * W, LY = NZ * W;
  static constexpr int THREADS = ((LZ > LY ? LZ : LY) + 63) / 64 * 64;
  static constexpr bool fits = BYTES <= 160 * 1024 && THREADS <= 1024 && (W % (16 / (int)sizeof(T))) == 0;
};

// alpha, c1, c2 of one line in the storage type; meta holds the signed whole-
// cell shift in its low 16 bits, bit 16 set where nu_z < 0 and bit 17 where
// nu_y < 0
template <typename T>
struct alignas(16) LineTab {
  T alpha, c1, c2;
  int meta;
};

__device__ __forceinline__ int tab_shift(int meta) { return (int)(short)(meta & 0xffff); }

template <typename T, int NY, int NZ>
__global__ __launch_bounds__(256) void drift_table_kernel(DriftArgs a)
{
  const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
  if (j >= a.nv3) return;
  LineTab<T>* zt = static_cast<LineTab<T>*>(a.tab);
  LineTab<T>* yt = zt + a.nv3;
  const long long jz = j % a.nvz;
  const long long jy = (j / a.nvz) % a.nvy;
  const bool periodic = a.periodic != 0;
  const double nuz = (a.vmin_z + ((double)jz + 0.5) * a.dv_z) * a.scale_z;
  const double nuy = (a.vmin_y + ((double)jy + 0.5) * a.dv_y) * a.scale_y;
  const int flags = (nuz < 0.0 ? 1 << 16 : 0) | (nuy < 0.0 ? 1 << 17 : 0);
  const LineCoef<T> cz = line_coef<T, NZ>(fabs(nuz), periodic);
  const LineCoef<T> cy = line_coef<T, NY>(fabs(nuy), periodic);
  zt[j] = LineTab<T>{cz.alpha, cz.c1, cz.c2, (cz.shift & 0xffff) | flags};
  yt[j] = LineTab<T>{cy.alpha, cy.c1, cy.c2, (cy.shift & 0xffff) | flags};
}

// Chunks narrower than a 128-byte cache line (W sizeof(T) = 128 / G bytes,
// the 48-cell planes) share each line among G consecutive chunks. A
// unit is then G workgroups that take chunks (c TILES + t) G + q, q = 0..G-1,
// tile by tile; with a.xcd_group the G workgroups of a unit are b = 8 (G m +
// q) + x, which the round-robin over the 8 XCDs places on one XCD (x) one
// after another, so that the halves or quarters of each line meet in that
// XCD's L2 instead of being fetched from HBM once per chunk.
template <typename T, int NY, int NZ, int W, int TILES, int G>
__global__ __launch_bounds__((DriftShape<T, NY, NZ, W>::THREADS)) void drift_yz_block(DriftArgs a)
{
  using S = DriftShape<T, NY, NZ, W>;
  static_assert(S::LZ == S::LY, "square planes");
  __shared__ T L[S::ELEMS];
  const int tid = threadIdx.x;
  const long long nchunk = a.nv3 / W;
  const long long upx = (nchunk / G + TILES - 1) / TILES;   // units per x index
  long long unit;
  int q;
  if (G > 1 && a.xcd_group) {
    const long long b = blockIdx.x, x = b & 7, k = b >> 3;
    q = (int)(k % G);
    unit = 8 * (k / G) + x;
  } else {
    q = (int)(blockIdx.x % G);
    unit = blockIdx.x / G;
  }
  const long long ix = unit / upx, cg = unit - ix * upx;
  auto chunk = [&](int t) { return (cg * TILES + t) * G + q; };
  const long long jc0 = chunk(0);
  const bool periodic = a.periodic != 0;
  const LineTab<T>* zt = static_cast<const LineTab<T>*>(a.tab);
  const LineTab<T>* yt = zt + a.nv3;
  // z-line lane (iy, w), y-line lane (iz, w): the same split of the lane index
  const int i0 = tid / W, w = tid - i0 * W;
  const unsigned RB = (unsigned)(a.nv3 * (long long)sizeof(T));   // bytes from one z to the next
  const char* slab = static_cast<const char*>(a.f) + ix * NY * NZ * a.nv3 * (long long)sizeof(T);
  const unsigned zoff = (unsigned)i0 * (unsigned)NZ * RB + (unsigned)w * (unsigned)sizeof(T);
  auto tile = [&](long long jc) { return slab + jc * W * (long long)sizeof(T); };
  T v[NZ];
  if (tid < S::LZ) {
    const char* src = tile(jc0);
#pragma unroll
    for (int r = 0; r < NZ; r++) v[r] = *reinterpret_cast<const T*>(src + (size_t)r * RB + zoff);
  }
#pragma unroll
  for (int k = 0; k < TILES; k++) {
    const long long jc = chunk(k);
    if (jc >= nchunk) break;                      // uniform over the workgroup (ragged ends: G = 1)
    if (tid < S::LZ) {
      // the z line, mirrored where vz < 0, takes the forward update and is
      // parked in LDS in that order, at its y place in the y sweep's
      // orientation
      const LineTab<T> c = zt[jc * W + w];
      const bool rz = (c.meta >> 16) & 1, ry = (c.meta >> 17) & 1;
      const int base = (ry ? NY - 1 - i0 : i0) * S::SY + w;
#pragma unroll
      for (int i = 0; i < NZ / 2; i++) {
        const T x0 = v[i], x1 = v[NZ - 1 - i];
        v[i] = rz ? x1 : x0;
        v[NZ - 1 - i] = rz ? x0 : x1;
      }
      pfc_core<T, NZ>(v, c.alpha, c.c1, c.c2, periodic);
      store_shifted<T, NZ>(v, tab_shift(c.meta), periodic, [&](int r, T x) { L[base + r * W] = x; });
    }
    __syncthreads();
    // the next tile's z lines go into flight before this tile's y lines
    if (k + 1 < TILES && chunk(k + 1) < nchunk && tid < S::LZ) {
      const char* src = tile(chunk(k + 1));
#pragma unroll
      for (int r = 0; r < NZ; r++) v[r] = *reinterpret_cast<const T*>(src + (size_t)r * RB + zoff);
    }
    if (tid < S::LY) {
      // lane (iz, w) takes storage z = iz (so each row a wave stores is whole
      // cache lines), found at LDS z place iz, or NZ-1-iz where vz < 0; the
      // y line comes out of LDS in its sweep orientation and row r goes to
      // storage y = r, or NY-1-r where vy < 0
      const LineTab<T> c = yt[jc * W + w];
      const bool rz = (c.meta >> 16) & 1, ry = (c.meta >> 17) & 1;
      const int base = (rz ? NZ - 1 - i0 : i0) * W + w;
      T u[NY];
#pragma unroll
      for (int r = 0; r < NY; r++) u[r] = L[base + r * S::SY];
      pfc_core<T, NY>(u, c.alpha, c.c1, c.c2, periodic);
      char* dst = const_cast<char*>(tile(jc));
      const unsigned ystep = (unsigned)NZ * RB;
      const unsigned y0 = (unsigned)i0 * RB + (unsigned)w * (unsigned)sizeof(T) + (ry ? (unsigned)(NY - 1) * ystep : 0u);
      const unsigned yst = ry ? 0u - ystep : ystep;
      store_shifted<T, NY>(u, tab_shift(c.meta), periodic, [&](int r, T x) {
        *reinterpret_cast<T*>(dst + (unsigned)(y0 + (unsigned)r * yst)) = x;
      });
    }
    if (k + 1 < TILES) __syncthreads();           // LDS is reused by the next tile
  }
}

template <typename T, int NP, int W, int TILES>
hipError_t launch_drift_yz_sq(const DriftArgs& a0, hipStream_t s)
{
  using S = DriftShape<T, NP, NP, W>;
  static_assert(S::fits, "tile does not fit the LDS");
  constexpr int G = (W * (int)sizeof(T) >= 128) ? 1 : 128 / (W * (int)sizeof(T));
  const long long nchunk = a0.nv3 / W;
  if (a0.nx <= 0 || nchunk <= 0) return hipSuccess;
  if (G > 1 && nchunk % (TILES * G) != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL((drift_table_kernel<T, NP, NP>), dim3((unsigned)((a0.nv3 + 255) / 256)), dim3(256), 0, s, a0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long units = a0.nx * ((nchunk / G + TILES - 1) / TILES);
  DriftArgs a = a0;
  a.xcd_group = (G > 1 && units % 8 == 0) ? 1 : 0;
  hipLaunchKernelGGL((drift_yz_block<T, NP, NP, W, TILES, G>), dim3((unsigned)(units * G)), dim3(S::THREADS), 0, s, a);
  return hipGetLastError();
}

}  // namespace

// (y, z) planes of 16, 24 or 32 cells with whole-cache-line velocity chunks
// Velocity cells per chunk (W), tiles per workgroup, and chunks per cache
// line (G) of the one-pass T_z T_y: whole-line chunks up to 32-cell planes;
// 48-cell planes take half-line chunks (FP32 16 cells, FP64 8), whose
// workgroups are grouped per line (above). 64-cell planes would take quarter
// lines (32 bytes); measured on the 16 x 64 x 64 slab, that pass took 2.7
// times a plain sweep, so those planes keep two plain sweeps.
struct DriftPlan {
  int w, tiles, g;
};

static DriftPlan drift_plan(int dtype, int ny, int nz, long long nv3)
{
  DriftPlan p{0, 0, 1};
  if (ny != nz) return p;
  const int es = dtype == 0 ? 4 : 8;
  if (dtype == 0) {
    switch (ny) {
      case 16: p = {64, 4, 1}; break;
      case 24: case 32: p = {32, 4, 1}; break;
      case 48: p = {16, 4, 2}; break;
      default: return DriftPlan{0, 0, 1};
    }
  } else {
    switch (ny) {
      case 16: p = {32, 2, 1}; break;
      case 24: p = {16, 2, 1}; break;
      case 32: p = {16, 4, 1}; break;
      case 48: p = {8, 2, 2}; break;
      default: return DriftPlan{0, 0, 1};
    }
  }
  if (nv3 % p.w != 0) return DriftPlan{0, 0, 1};
  if (p.g > 1 && (nv3 / p.w) % (p.tiles * p.g) != 0) return DriftPlan{0, 0, 1};
  // 32-bit byte offsets within a tile: the largest is under the tile's span
  if (((long long)ny * nz * nv3 - nv3 + p.w) * es >= (1LL << 32)) return DriftPlan{0, 0, 1};
  return p;
}

size_t drift_table_bytes(int dtype, long long nv3)
{
  return (size_t)(2 * nv3) * (dtype == 0 ? sizeof(LineTab<float>) : sizeof(LineTab<double>));
}

bool drift_yz_supported(int dtype, int ny, int nz, long long nv3) { return drift_plan(dtype, ny, nz, nv3).w != 0; }

// Tiles per workgroup: four, except two for the FP64 16- and 24-planes, whose
// workgroups are small enough that several share a CU anyway, and for the
// FP64 48-planes.
hipError_t launch_drift_yz(const DriftArgs& a, int dtype, hipStream_t s)
{
  if (!a.tab || drift_plan(dtype, a.ny, a.nz, a.nv3).w == 0) return hipErrorInvalidValue;
  if (dtype == 0) {
    switch (a.ny) {
      case 16: return launch_drift_yz_sq<float, 16, 64, 4>(a, s);
      case 24: return launch_drift_yz_sq<float, 24, 32, 4>(a, s);
      case 32: return launch_drift_yz_sq<float, 32, 32, 4>(a, s);
      case 48: return launch_drift_yz_sq<float, 48, 16, 4>(a, s);
      default: break;
    }
  } else {
    switch (a.ny) {
      case 16: return launch_drift_yz_sq<double, 16, 32, 2>(a, s);
      case 24: return launch_drift_yz_sq<double, 24, 16, 2>(a, s);
      case 32: return launch_drift_yz_sq<double, 32, 16, 4>(a, s);
      case 48: return launch_drift_yz_sq<double, 48, 8, 2>(a, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}
}  // namespace vp
