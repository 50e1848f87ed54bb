// drift.hip -- the position sweeps T_z then T_y of Eq. (17) (Sec. 2.1 of
// Yoshikawa, Yoshida & Umemura) in one pass over f, for square (y, z) planes
// that fit on chip with a chunk of velocity cells. The line update is that of
// sweep.hip (pfc_line.h), so the pass rounds like the single sweeps. gfx950.
#include "vp_internal.h"

#include "pfc_line.h"
#include "vec16.h"

namespace vp {
namespace {

// ---- one-pass drift along z, then y -----------------------------------------
// A tile is one x index and W consecutive velocity cells of every (y, z) cell
// (W contiguous values per (y, z) cell in HBM). Each z line of a tile is read
// from HBM by one lane, updated in registers and parked in LDS; after a
// barrier each y line is taken from LDS by one lane, updated and written back
// to HBM. f crosses HBM once for the two sweeps. Two kernels: drift_yz_block
// below (one line per lane, the next tile's z lines prefetched) and
// drift_yz_pairs further down (two lines per lane, half the LDS per tile).
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

// Chunks narrower than a 128-byte cache line (W sizeof(T) = 128 / G bytes:
// FP64 48-cell planes here, FP32 64-cell planes in drift_yz_pairs) share each
// line among G consecutive chunks. A
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

// ---- one-pass drift, two lines per lane -------------------------------------
// The same two sweeps on tiles of W velocity cells, with lane (i, p) of the
// NP x W/2 lanes holding the lines of the adjacent cells 2p and 2p + 1 of the
// tile. The z lines (y = i) come in as 8- or 16-byte pairs, so that a row of
// W/2 lanes reads one whole W-cell run, and are swept in registers; they reach
// the y sweep through LDS in two rounds (cells 2p, then cells 2p + 1) of W/2
// columns, half the LDS that one line per lane needs. In the second phase lane
// (i, p) takes the y lines (z = i) of the same two cells. With nv_z even the
// two cells of a pair share vy, hence the y sweep's coefficients, shift and
// orientation, so the y lines go back to HBM as pairs too. Byte offsets are
// 64-bit: a tile may span more than 4 GiB (64 x 64 planes of 1 MiB blocks).
template <typename T, int NP, int W>
struct DrPairShape {
  static constexpr int H = W / 2;                                  // LDS columns per round
  static constexpr int SY0 = NP * H;
  static constexpr int SY = SY0 + ((((H - SY0) % 64) + 64) % 64);   // = H (mod 64)
  static constexpr int ELEMS = NP * SY;
  static constexpr int BYTES = ELEMS * (int)sizeof(T);
  static constexpr int THREADS = NP * H;
  static constexpr bool fits = BYTES <= 160 * 1024 && THREADS <= 1024 && THREADS % 64 == 0 && W % 2 == 0;
};

template <typename T, int NP, int W, int TILES, int G>
__global__ __launch_bounds__((DrPairShape<T, NP, W>::THREADS)) void drift_yz_pairs(DriftArgs a)
{
  using S = DrPairShape<T, NP, W>;
  using P2 = typename Pair2<T>::type;
  constexpr int H = S::H;
  __shared__ T L[S::ELEMS];
  const int tid = threadIdx.x;
  const int i0 = tid / H, p = tid - i0 * H;
  const long long nchunk = a.nv3 / W;
  const long long upx = (nchunk / G + TILES - 1) / TILES;   // units per x index
  // the G workgroups of a unit take the G chunks of each cache line (grouped
  // on one XCD as in drift_yz_block)
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
  const bool periodic = a.periodic != 0;
  const LineTab<T>* zt = static_cast<const LineTab<T>*>(a.tab);
  const LineTab<T>* yt = zt + a.nv3;
  const long long RB = a.nv3 * (long long)sizeof(T);   // bytes from one z to the next
  char* slab = static_cast<char*>(a.f) + ix * NP * NP * RB;
#pragma unroll 1
  for (int k = 0; k < TILES; k++) {
    const long long jc = (cg * TILES + k) * G + q;
    if (jc >= nchunk) break;                            // uniform over the workgroup (ragged ends: G = 1)
    char* tile = slab + (jc * W + 2 * p) * (long long)sizeof(T);
    T v0[NP], v1[NP];
    {
      const char* src = tile + (long long)i0 * NP * RB;
#pragma unroll
      for (int r = 0; r < NP; r++) {
        const P2 x = *reinterpret_cast<const P2*>(src + r * RB);
        v0[r] = x.x;
        v1[r] = x.y;
      }
    }
    const long long j = jc * W + 2 * p;
    const LineTab<T> cz0 = zt[j], cz1 = zt[j + 1], cy0 = yt[j], cy1 = yt[j + 1];
    // z lines, mirrored where vz < 0, take the forward update
    auto zsweep = [&](T(&v)[NP], const LineTab<T>& c) {
      const bool rz = (c.meta >> 16) & 1;
#pragma unroll
      for (int i = 0; i < NP / 2; i++) {
        const T x0 = v[i], x1 = v[NP - 1 - i];
        v[i] = rz ? x1 : x0;
        v[NP - 1 - i] = rz ? x0 : x1;
      }
      pfc_core<T, NP>(v, c.alpha, c.c1, c.c2, periodic);
    };
    zsweep(v0, cz0);
    zsweep(v1, cz1);
    // one round: the z lines of one cell per lane are parked in LDS (at their
    // y place in the y sweep's orientation), and each lane takes back the y
    // line of storage z = i of the same cell, found at LDS z place i, or
    // NP-1-i where vz < 0
    auto round = [&](T(&v)[NP], const LineTab<T>& cz, const LineTab<T>& cy) {
      const bool ry = (cz.meta >> 17) & 1;
      const int base = (ry ? NP - 1 - i0 : i0) * S::SY + p;
      store_shifted<T, NP>(v, tab_shift(cz.meta), periodic, [&](int r, T x) { L[base + r * H] = x; });
      __syncthreads();
      const bool rz = (cy.meta >> 16) & 1;
      const int yb = (rz ? NP - 1 - i0 : i0) * H + p;
#pragma unroll
      for (int r = 0; r < NP; r++) v[r] = L[yb + r * S::SY];
      pfc_core<T, NP>(v, cy.alpha, cy.c1, cy.c2, periodic);
      __syncthreads();                                  // LDS is reused by the next round
    };
    round(v0, cz0, cy0);
    round(v1, cz1, cy1);
    // row r of the y lines goes to storage y = r, or NP-1-r where vy < 0
    const bool ry = (cy0.meta >> 17) & 1;
    const long long ystep = NP * RB;
    char* dst = tile + (long long)i0 * RB + (ry ? (NP - 1) * ystep : 0LL);
    const long long yst = ry ? -ystep : ystep;
    store_shifted2<T, NP>(v0, v1, tab_shift(cy0.meta), periodic,
                          [&](int r, T x0, T x1) { *reinterpret_cast<P2*>(dst + r * yst) = P2{x0, x1}; });
  }
}

template <typename T, int NP, int W, int TILES, int G>
hipError_t launch_drift_yz_pairs(const DriftArgs& a0, hipStream_t s)
{
  using S = DrPairShape<T, NP, W>;
  static_assert(S::fits, "tile does not fit the LDS");
  const long long nchunk = a0.nv3 / W;
  if (a0.nx <= 0 || nchunk <= 0) return hipSuccess;
  if (a0.nv3 % W != 0 || a0.nvz % 2 != 0) return hipErrorInvalidValue;
  if (G > 1 && nchunk % (TILES * G) != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL((drift_table_kernel<T, NP, NP>), dim3((unsigned)((a0.nv3 + 255) / 256)), dim3(256), 0, s, a0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long units = a0.nx * ((nchunk / G + TILES - 1) / TILES);
  DriftArgs a = a0;
  a.xcd_group = (G > 1 && units % 8 == 0) ? 1 : 0;
  hipLaunchKernelGGL((drift_yz_pairs<T, NP, W, TILES, G>), dim3((unsigned)(units * G)), dim3(S::THREADS), 0, s, a);
  return hipGetLastError();
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

// Velocity cells per chunk (W), tiles per workgroup, chunks per cache line (G)
// and kernel of the one-pass T_z T_y. Two lines per lane (drift_yz_pairs,
// nv_z even): FP32 planes of 32 and 48 cells and FP64 planes of 32 in
// whole-line chunks, FP32 64-cell planes in half-line chunks grouped per line.
// One line per lane (drift_yz_block): whole-line chunks for 16- and 24-cell
// planes, half-line chunks grouped per line for FP64 48-cell planes. FP64
// 64-cell planes, and the rest, take the single sweeps.
struct DriftPlan {
  int w, tiles, g, pairs;
};

static DriftPlan drift_plan(int dtype, int ny, int nz, long long nv3, long long nvz)
{
  DriftPlan p{0, 0, 1, 0};
  if (ny != nz || nv3 <= 0) return p;
  const int es = dtype == 0 ? 4 : 8;
  if (dtype == 0) {
    switch (ny) {
      case 16: p = {64, 4, 1, 0}; break;
      case 24: p = {32, 4, 1, 0}; break;
      case 32: p = {32, 4, 1, 1}; break;
      case 48: p = {32, 4, 1, 1}; break;
      case 64: p = {16, 4, 2, 1}; break;
      default: return DriftPlan{0, 0, 1, 0};
    }
  } else {
    switch (ny) {
      case 16: p = {32, 2, 1, 0}; break;
      case 24: p = {16, 2, 1, 0}; break;
      case 32: p = {16, 4, 1, 1}; break;
      case 48: p = {8, 2, 2, 0}; break;
      default: return DriftPlan{0, 0, 1, 0};
    }
  }
  if (nv3 % p.w != 0) return DriftPlan{0, 0, 1, 0};
  if (p.g > 1 && (nv3 / p.w) % (p.tiles * p.g) != 0) return DriftPlan{0, 0, 1, 0};
  if (p.pairs) return nvz % 2 == 0 ? p : DriftPlan{0, 0, 1, 0};
  // 32-bit byte offsets within a tile: the largest is under the tile's span
  if (((long long)ny * nz * nv3 - nv3 + p.w) * es >= (1LL << 32)) return DriftPlan{0, 0, 1, 0};
  return p;
}

size_t drift_table_bytes(int dtype, long long nv3)
{
  return (size_t)(2 * nv3) * (dtype == 0 ? sizeof(LineTab<float>) : sizeof(LineTab<double>));
}

bool drift_yz_supported(int dtype, int ny, int nz, long long nv3, long long nvz)
{
  return drift_plan(dtype, ny, nz, nv3, nvz).w != 0;
}

hipError_t launch_drift_yz(const DriftArgs& a, int dtype, hipStream_t s)
{
  const DriftPlan p = drift_plan(dtype, a.ny, a.nz, a.nv3, a.nvz);
  if (!a.tab || p.w == 0) return hipErrorInvalidValue;
  if (dtype == 0) {
    switch (a.ny) {
      case 16: return launch_drift_yz_sq<float, 16, 64, 4>(a, s);
      case 24: return launch_drift_yz_sq<float, 24, 32, 4>(a, s);
      case 32: return launch_drift_yz_pairs<float, 32, 32, 4, 1>(a, s);
      case 48: return launch_drift_yz_pairs<float, 48, 32, 4, 1>(a, s);
      case 64: return launch_drift_yz_pairs<float, 64, 16, 4, 2>(a, s);
      default: break;
    }
  } else {
    switch (a.ny) {
      case 16: return launch_drift_yz_sq<double, 16, 32, 2>(a, s);
      case 24: return launch_drift_yz_sq<double, 24, 16, 2>(a, s);
      case 32: return launch_drift_yz_pairs<double, 32, 16, 4, 1>(a, s);
      case 48: return launch_drift_yz_sq<double, 48, 8, 2>(a, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}
}  // namespace vp
