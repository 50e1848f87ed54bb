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
// (or two in a row) on a whole velocity block, two velocity sweeps on half a
// block or on slices of whole (vy, vz) planes, and T_z T_y on an x index times
// a chunk of velocity cells. The alpha, c1, c2 of a line are computed in FP64
// and rounded once to the storage type. The whole-cell part m of the shift is
// applied as the line is written out: each cell goes once to its shifted place.
#include "vp_internal.h"

#include "pfc_line.h"
#include "buffer_io.h"

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

// ---- one-pass half kick -----------------------------------------------------
// The velocity block of one spatial cell (NX*NY*NZ values, contiguous in HBM)
// is read once (the vx lines straight into registers), swept along vx, then
// vy, then vz in LDS (each lane owns one line per sweep, in registers), and
// written back once. The LDS layout pads
// each vz row to NZ+1 and each vx plane to SX = NZ (mod 64) elements, which
// keeps the accesses of all three sweep directions on distinct banks.
template <typename T, int NX, int NY, int NZ>
struct KickShape {
  static constexpr int SY = NZ + 1;
  static constexpr int SX0 = NY * SY;
  static constexpr int SX = SX0 + ((((NZ - SX0) % 64) + 64) % 64);
  static constexpr int ELEMS = NX * SX;
  static constexpr int BYTES = ELEMS * (int)sizeof(T);
  static constexpr int L0 = NY * NZ, L1 = NX * NZ, L2 = NX * NY;
  static constexpr int LINES = L0 > L1 ? (L0 > L2 ? L0 : L2) : (L1 > L2 ? L1 : L2);
  static constexpr int THREADS = ((LINES + 63) / 64) * 64;
  static constexpr int NV3 = NX * NY * NZ;
  static constexpr bool fits = BYTES <= 160 * 1024 && THREADS <= 1024 && (NV3 % (16 / (int)sizeof(T))) == 0;
};

// Each velocity axis of a block is held in LDS in the orientation of its
// sweep: reversed where the acceleration along it is negative, so every line
// update transports toward increasing LDS index (the forward form of the
// line update, with |nu|). The orientation enters only through addresses: the
// row order of the first sweep's HBM loads (a scalar choice), each lane's LDS
// base, and the order in which the block is read back out. One code path
// serves all eight sign combinations, which keeps the register footprint that
// of a single line update.
template <typename T, int NX, int NY, int NZ, int REPS>
__global__ __launch_bounds__((KickShape<T, NX, NY, NZ>::THREADS)) void kick_block(KickArgs a)
{
  using S = KickShape<T, NX, NY, NZ>;
  using VT = typename Vec16<T>::type;
  constexpr int V = Vec16<T>::n;
  constexpr int NVEC = S::NV3 / V;
  constexpr int PER = (NVEC + S::THREADS - 1) / S::THREADS;
  constexpr unsigned ROWB = NY * NZ * (unsigned)sizeof(T);   // bytes between vx rows
  constexpr unsigned BLKB = S::NV3 * (unsigned)sizeof(T);
  __shared__ T L[S::ELEMS];
  const int tid = threadIdx.x;
  const long long s = blockIdx.x;
  const auto rs = buf_rsrc(static_cast<const T*>(a.f) + s * S::NV3, BLKB);
  const double nux = a.a[0][s] * a.scale[0], nuy = a.a[1][s] * a.scale[1], nuz = a.a[2][s] * a.scale[2];
  const bool rx = nux < 0.0, ry = nuy < 0.0, rz = nuz < 0.0;
  const LineCoef<T> cx = line_coef<T, NX>(fabs(nux), false);
  const LineCoef<T> cy = line_coef<T, NY>(fabs(nuy), false);
  const LineCoef<T> cz = line_coef<T, NZ>(fabs(nuz), false);
  // first vx sweep, lane (jy, jz): the line comes from HBM (a row of a wave is
  // 64 consecutive values) and goes to the lane's oriented (vy, vz) place
  if (tid < S::L0) {
    const int jy = tid / NZ, jz = tid - jy * NZ;
    const int base = (ry ? NY - 1 - jy : jy) * S::SY + (rz ? NZ - 1 - jz : jz);
    const unsigned voff = (unsigned)tid * (unsigned)sizeof(T);
    T v[NX];
#pragma unroll
    for (int r = 0; r < NX; r++) v[r] = buf_load<T>(rs, voff, (unsigned)(rx ? NX - 1 - r : r) * ROWB);
    pfc_core<T, NX>(v, cx.alpha, cx.c1, cx.c2, false);
    store_shifted<T, NX>(v, cx.shift, false, [&](int r, T x) { L[base + r * S::SX] = x; });
  }
  __syncthreads();
#pragma unroll
  for (int rep = 0; rep < REPS; rep++) {
    if (rep > 0) {
      if (tid < S::L0) {  // vx lines at LDS (vy, vz) = (tid / NZ, tid % NZ)
        const int base = (tid / NZ) * S::SY + (tid % NZ);
        T u[NX];
#pragma unroll
        for (int r = 0; r < NX; r++) u[r] = L[base + r * S::SX];
        pfc_core<T, NX>(u, cx.alpha, cx.c1, cx.c2, false);
        store_shifted<T, NX>(u, cx.shift, false, [&](int r, T x) { L[base + r * S::SX] = x; });
      }
      __syncthreads();
    }
    if (tid < S::L1) {  // vy lines at LDS (vx, vz)
      const int base = (tid / NZ) * S::SX + (tid % NZ);
      T u[NY];
#pragma unroll
      for (int r = 0; r < NY; r++) u[r] = L[base + r * S::SY];
      pfc_core<T, NY>(u, cy.alpha, cy.c1, cy.c2, false);
      store_shifted<T, NY>(u, cy.shift, false, [&](int r, T x) { L[base + r * S::SY] = x; });
    }
    __syncthreads();
    if (tid < S::L2) {  // vz lines at LDS (vx, vy)
      const int base = (tid / NY) * S::SX + (tid % NY) * S::SY;
      T u[NZ];
#pragma unroll
      for (int r = 0; r < NZ; r++) u[r] = L[base + r];
      pfc_core<T, NZ>(u, cz.alpha, cz.c1, cz.c2, false);
      store_shifted<T, NZ>(u, cz.shift, false, [&](int r, T x) { L[base + r] = x; });
    }
    __syncthreads();
  }
  // back to HBM (over f, or to out) in storage order, 16 bytes per access.
  // Lane t writes chunks t + k*THREADS; as THREADS = NY*NZ, all of a lane's
  // chunks share their (vy, vz) cells and advance by V along vx, so the LDS
  // place of chunk k is the lane's base plus k times a uniform step.
  static_assert(S::THREADS == NY * NZ && NVEC == PER * S::THREADS, "whole chunks per lane");
  const int e0 = tid * V;
  const int jz = e0 % NZ, jy = (e0 / NZ) % NY, jx0 = e0 / (NY * NZ);
  const int yz = (ry ? NY - 1 - jy : jy) * S::SY + (rz ? NZ - V - jz : jz);   // lowest LDS z place of the chunk
  const int b0 = (rx ? NX - 1 - jx0 : jx0) * S::SX + yz;
  const int step = (rx ? -V : V) * S::SX;
  const unsigned vo = (unsigned)tid * 16u;
  const auto ws = a.out ? buf_rsrc(static_cast<const T*>(a.out) + s * S::NV3, BLKB) : rs;
  if (rz) {
#pragma unroll
    for (int k = 0; k < PER; k++) {
      VT x;
      T* xs = reinterpret_cast<T*>(&x);
      const int lo = b0 + k * step;
#pragma unroll
      for (int q = 0; q < V; q++) xs[q] = L[lo + V - 1 - q];
      buf_store16(ws, vo + (unsigned)(k * S::THREADS) * 16u, x);
    }
  } else {
#pragma unroll
    for (int k = 0; k < PER; k++) {
      VT x;
      T* xs = reinterpret_cast<T*>(&x);
      const int lo = b0 + k * step;
#pragma unroll
      for (int q = 0; q < V; q++) xs[q] = L[lo + q];
      buf_store16(ws, vo + (unsigned)(k * S::THREADS) * 16u, x);
    }
  }
}

template <typename T, int NV>
hipError_t launch_kick_cube(const KickArgs& a, hipStream_t s)
{
  using S = KickShape<T, NV, NV, NV>;
  static_assert(S::fits, "velocity block does not fit the LDS");
  static_assert(NV % Vec16<T>::n == 0, "16-byte output chunks stay inside a vz row");
  if (a.np <= 0) return hipSuccess;
  if (a.reps == 2)
    hipLaunchKernelGGL((kick_block<T, NV, NV, NV, 2>), dim3((unsigned)a.np), dim3(S::THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((kick_block<T, NV, NV, NV, 1>), dim3((unsigned)a.np), dim3(S::THREADS), 0, s, a);
  return hipGetLastError();
}

// ---- two velocity sweeps in one pass over half a velocity block --------------
// When a whole velocity block does not fit in LDS but half of it does (FP64
// 32^3: 256 KiB, half 128 KiB), two consecutive sweeps whose lines both lie in
// the half run in one pass: PASS 0 is T_vx then T_vy on the half with vz in
// [c0, c0 + CH); PASS 1 is T_vz then T_vx on the half with vy in the chunk;
// PASS 2 is T_vy then T_vz on the half with vx in the chunk. A half kick is
// PASS 0 and a T_vz sweep; the two half kicks between two drifts (T_vx T_vy
// T_vz T_vx T_vy T_vz) are PASS 0, 1, 2. Each LDS layout keeps the HBM-
// contiguous axis contiguous and pads rows so both sweep directions are
// bank-conflict free; the arithmetic is that of the single sweeps. With CH
// below NV / 2 the same kernel takes slices of CH planes (PASS 2 only, for
// blocks whose half does not fit either).
template <typename T, int NV, int PASS, int CH_ = NV / 2>
struct PairShape {
  static constexpr int CH = CH_;                         // planes across the third axis
  static constexpr int NCH = NV / CH;                    // slices per velocity block
  static constexpr int PAD = 64 / (int)sizeof(T);
  static constexpr int SR = NV + 1;                       // padded vz row (PASS 1, 2)
  // PASS 0: [vx][vy][c], vx stride SA; PASS 1: [vx][c][vz]; PASS 2: [c][vy][vz]
  static constexpr int SA = NV * CH + PAD;
  static constexpr int ELEMS = PASS == 0 ? NV * SA : NV * CH * SR;
  static constexpr int BYTES = ELEMS * (int)sizeof(T);
  static constexpr int THREADS = NV * CH;                  // lines per sweep
  static constexpr int HALF = NV * NV * CH;                // values in one slice
  static constexpr bool fits = BYTES <= 160 * 1024 && THREADS <= 1024 && NV % CH == 0;
};

template <typename T, int NV, int PASS, int CH_>
__device__ __forceinline__ void pair_coords(int e, int& gofs, int& lds, bool fx, bool fy, bool fz)
{
  // element e of the slice in HBM order -> offset in the block, LDS index; a
  // swept axis whose flag is set is held reversed in LDS (the chunk axis never)
  using S = PairShape<T, NV, PASS, CH_>;
  auto fl = [](bool f, int i) { return f ? NV - 1 - i : i; };
  if constexpr (PASS == 0) {          // runs of CH along vz
    const int run = e / S::CH, c = e - run * S::CH;
    gofs = run * NV + c;             // + c0 added by the caller
    lds = fl(fx, run / NV) * S::SA + fl(fy, run % NV) * S::CH + c;
  } else if constexpr (PASS == 1) {   // per vx, CH whole vz rows
    const int vx = e / (S::CH * NV), rem = e - vx * (S::CH * NV);
    const int c = rem / NV, vz = rem - c * NV;
    gofs = vx * NV * NV + rem;       // + c0 * NV
    lds = (fl(fx, vx) * S::CH + c) * S::SR + fl(fz, vz);
  } else {                            // CH whole vx planes
    const int c = e / (NV * NV), rem = e - c * (NV * NV);
    const int vy = rem / NV, vz = rem - vy * NV;
    gofs = e;                         // + c0 * NV * NV
    lds = (c * NV + fl(fy, vy)) * S::SR + fl(fz, vz);
  }
}

// The two swept axes of a slice are held in LDS in the orientation of their
// sweeps (reversed where the acceleration along them is negative), so both
// line updates take the forward form with |nu|; the orientation enters only
// through the LDS places of the loaded and stored pieces.
template <typename T, int NV, int PASS, int CH_>
__global__ __launch_bounds__((PairShape<T, NV, PASS, CH_>::THREADS)) void kick_pair_block(KickArgs a)
{
  using S = PairShape<T, NV, PASS, CH_>;
  constexpr int CH = S::CH;
  __shared__ T L[S::ELEMS];
  const int tid = threadIdx.x;
  const long long s = blockIdx.x / S::NCH;
  const int c0 = (int)(blockIdx.x - s * S::NCH) * CH;
  const long long cofs = PASS == 0 ? c0 : (PASS == 1 ? c0 * NV : c0 * NV * NV);
  T* g = static_cast<T*>(a.f) + s * (long long)(NV * NV * NV) + cofs;
  // the two sweeps: axis A then axis B (0 = vx, 1 = vy, 2 = vz)
  constexpr int AX0 = PASS == 0 ? 0 : (PASS == 1 ? 2 : 1);
  constexpr int AX1 = PASS == 0 ? 1 : (PASS == 1 ? 0 : 2);
  const double nu0 = a.a[AX0][s] * a.scale[AX0], nu1 = a.a[AX1][s] * a.scale[AX1];
  const bool f0 = nu0 < 0.0, f1 = nu1 < 0.0;
  const bool fx = (AX0 == 0 && f0) || (AX1 == 0 && f1);
  const bool fy = (AX0 == 1 && f0) || (AX1 == 1 && f1);
  const bool fz = (AX0 == 2 && f0) || (AX1 == 2 && f1);
  // 16-byte pieces: V consecutive values along vz, adjacent in HBM and in LDS
  // (descending in LDS where vz is held reversed); every load of the lane is
  // issued before the first LDS write
  using VT = typename Vec16<T>::type;
  constexpr int V = Vec16<T>::n;
  constexpr int PER = S::HALF / V / S::THREADS;
  static_assert(S::HALF % (V * S::THREADS) == 0 && S::CH % V == 0, "half block is not whole 16-byte pieces");
  {
    VT x[PER];
#pragma unroll
    for (int k = 0; k < PER; k++) {
      int go, li;
      pair_coords<T, NV, PASS, CH_>((tid + k * S::THREADS) * V, go, li, fx, fy, fz);
      x[k] = *reinterpret_cast<const VT*>(g + go);
    }
    if (fz) {
#pragma unroll
      for (int k = 0; k < PER; k++) {
        int go, li;
        pair_coords<T, NV, PASS, CH_>((tid + k * S::THREADS) * V, go, li, fx, fy, fz);
#pragma unroll
        for (int q = 0; q < V; q++) L[li - q] = lane_of<VT, T>(x[k], q);
      }
    } else {
#pragma unroll
      for (int k = 0; k < PER; k++) {
        int go, li;
        pair_coords<T, NV, PASS, CH_>((tid + k * S::THREADS) * V, go, li, fx, fy, fz);
#pragma unroll
        for (int q = 0; q < V; q++) L[li + q] = lane_of<VT, T>(x[k], q);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 2; q++) {
    const int ax = q == 0 ? AX0 : AX1;
    const double nu = q == 0 ? nu0 : nu1;
    int base, st;
    if constexpr (PASS == 0) {
      // lanes (other in-plane axis, c); vx stride SA, vy stride CH
      const int o = tid / CH, c = tid - o * CH;
      if (ax == 0) { base = o * CH + c; st = S::SA; }
      else { base = o * S::SA + c; st = CH; }
    } else if constexpr (PASS == 1) {
      if (ax == 2) {                 // vz lines, lanes (vx, c)
        const int vx = tid / CH, c = tid - vx * CH;
        base = (vx * CH + c) * S::SR; st = 1;
      } else {                       // vx lines, lanes (c, vz)
        const int c = tid / NV, vz = tid - c * NV;
        base = c * S::SR + vz; st = CH * S::SR;
      }
    } else {
      if (ax == 1) {                 // vy lines, lanes (c, vz)
        const int c = tid / NV, vz = tid - c * NV;
        base = c * NV * S::SR + vz; st = S::SR;
      } else {                       // vz lines, lanes (c, vy)
        const int c = tid / NV, vy = tid - c * NV;
        base = (c * NV + vy) * S::SR; st = 1;
      }
    }
    T v[NV];
#pragma unroll
    for (int r = 0; r < NV; r++) v[r] = L[base + r * st];
    const LineCoef<T> k = line_coef<T, NV>(fabs(nu), false);
    pfc_core<T, NV>(v, k.alpha, k.c1, k.c2, false);
    store_shifted<T, NV>(v, k.shift, false, [&](int r, T x) { L[base + r * st] = x; });
    __syncthreads();
  }
  if (fz) {
#pragma unroll
    for (int k = 0; k < PER; k++) {
      int go, li;
      pair_coords<T, NV, PASS, CH_>((tid + k * S::THREADS) * V, go, li, fx, fy, fz);
      VT x;
      T* xs = reinterpret_cast<T*>(&x);
#pragma unroll
      for (int q = 0; q < V; q++) xs[q] = L[li - q];
      *reinterpret_cast<VT*>(g + go) = x;
    }
  } else {
#pragma unroll
    for (int k = 0; k < PER; k++) {
      int go, li;
      pair_coords<T, NV, PASS, CH_>((tid + k * S::THREADS) * V, go, li, fx, fy, fz);
      VT x;
      T* xs = reinterpret_cast<T*>(&x);
#pragma unroll
      for (int q = 0; q < V; q++) xs[q] = L[li + q];
      *reinterpret_cast<VT*>(g + go) = x;
    }
  }
}

template <typename T, int NV>
hipError_t launch_kick_pair_cube(const KickArgs& a, int pass, hipStream_t s)
{
  if (a.np <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)(2 * a.np);
  switch (pass) {
    case 0:
      static_assert(PairShape<T, NV, 0>::fits, "half block does not fit the LDS");
      hipLaunchKernelGGL((kick_pair_block<T, NV, 0, NV / 2>), dim3(blocks), dim3(PairShape<T, NV, 0>::THREADS), 0, s, a);
      break;
    case 1:
      static_assert(PairShape<T, NV, 1>::fits, "half block does not fit the LDS");
      hipLaunchKernelGGL((kick_pair_block<T, NV, 1, NV / 2>), dim3(blocks), dim3(PairShape<T, NV, 1>::THREADS), 0, s, a);
      break;
    default:
      static_assert(PairShape<T, NV, 2>::fits, "half block does not fit the LDS");
      hipLaunchKernelGGL((kick_pair_block<T, NV, 2, NV / 2>), dim3(blocks), dim3(PairShape<T, NV, 2>::THREADS), 0, s, a);
      break;
  }
  return hipGetLastError();
}

// T_vy then T_vz on slices of CH whole (vy, vz) planes (one slice per
// workgroup): for velocity blocks too large for the half-block passes
template <typename T, int NV, int CH>
hipError_t launch_kick_planes(const KickArgs& a, hipStream_t s)
{
  using S = PairShape<T, NV, 2, CH>;
  static_assert(S::fits, "slice does not fit the LDS");
  if (a.np <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)(S::NCH * a.np);
  hipLaunchKernelGGL((kick_pair_block<T, NV, 2, CH>), dim3(blocks), dim3(S::THREADS), 0, s, a);
  return hipGetLastError();
}

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
// A workgroup takes TILES consecutive tiles. The z lines of the next tile are
// loaded into registers while the current tile's y lines are swept and
// stored, so that the single workgroup an LDS-sized tile leaves on a CU keeps
// loads in flight while it computes. The tile loop is unrolled at compile
// time, which keeps every memory-counter wait exact.
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

template <typename T, int NY, int NZ, int W, int TILES>
__global__ __launch_bounds__((DriftShape<T, NY, NZ, W>::THREADS)) void drift_yz_block(DriftArgs a)
{
  using S = DriftShape<T, NY, NZ, W>;
  __shared__ T L[S::ELEMS];
  const int tid = threadIdx.x;
  const long long nchunk = a.nv3 / W;
  const long long ntiles = a.nx * nchunk;
  const long long t0 = (long long)blockIdx.x * TILES;
  const bool periodic = a.periodic != 0;
  // z-line lane (iy, w), y-line lane (iz, w)
  const int iy = tid / W, wz = tid - iy * W;
  const int iz = tid / W, wy = tid - iz * W;
  auto tile_base = [&](long long t) {   // (y, z, w) = base[(y*NZ + z)*nv3 + w]
    const long long ix = t / nchunk, jc = t - ix * nchunk;
    return static_cast<T*>(a.f) + ix * NY * NZ * a.nv3 + jc * W;
  };
  // lane offsets within a tile are 32-bit (the host checks that a tile spans
  // under 4 GiB); row pointers are uniform
  const unsigned zoff = (unsigned)iy * (unsigned)(NZ * a.nv3) + (unsigned)wz;
  T v[NZ];
  if (tid < S::LZ) {
    const T* src = tile_base(t0);
#pragma unroll
    for (int r = 0; r < NZ; r++) v[r] = (src + (long long)r * a.nv3)[zoff];
  }
#pragma unroll
  for (int k = 0; k < TILES; k++) {
    const long long t = t0 + k;
    if (t >= ntiles) break;                       // uniform over the workgroup
    const long long jc = t % nchunk;
    if (tid < S::LZ) {
      // the z line, mirrored where vz < 0, takes the forward update and is
      // parked in LDS in that order, at its y place in the y sweep's
      // orientation
      const long long jz = (jc * W + wz) % a.nvz;
      const long long jy = ((jc * W + wz) / a.nvz) % a.nvy;
      const double nu = (a.vmin_z + ((double)jz + 0.5) * a.dv_z) * a.scale_z;
      const bool rz = nu < 0.0;
      const bool ry = (a.vmin_y + ((double)jy + 0.5) * a.dv_y) * a.scale_y < 0.0;
      const int base = (ry ? NY - 1 - iy : iy) * S::SY + wz;
#pragma unroll
      for (int i = 0; i < NZ / 2; i++) {
        const T x0 = v[i], x1 = v[NZ - 1 - i];
        v[i] = rz ? x1 : x0;
        v[NZ - 1 - i] = rz ? x0 : x1;
      }
      const LineCoef<T> c = line_coef<T, NZ>(fabs(nu), periodic);
      pfc_core<T, NZ>(v, c.alpha, c.c1, c.c2, periodic);
      store_shifted<T, NZ>(v, c.shift, periodic, [&](int r, T x) { L[base + r * W] = x; });
    }
    __syncthreads();
    // the next tile's z lines go into flight before this tile's y lines
    if (k + 1 < TILES && t + 1 < ntiles && tid < S::LZ) {
      const T* src = tile_base(t + 1);
#pragma unroll
      for (int r = 0; r < NZ; r++) v[r] = (src + (long long)r * a.nv3)[zoff];
    }
    if (tid < S::LY) {
      // lane (iz, w) takes storage z = iz (so each row a wave stores is whole
      // cache lines), found at LDS z place iz, or NZ-1-iz where vz < 0; the
      // y line comes out of LDS in its sweep orientation
      const long long jz = (jc * W + wy) % a.nvz;
      const long long jy = ((jc * W + wy) / a.nvz) % a.nvy;
      const bool rz = (a.vmin_z + ((double)jz + 0.5) * a.dv_z) * a.scale_z < 0.0;
      const double nu = (a.vmin_y + ((double)jy + 0.5) * a.dv_y) * a.scale_y;
      const bool ry = nu < 0.0;
      const int base = (rz ? NZ - 1 - iz : iz) * W + wy;
      T u[NY];
#pragma unroll
      for (int r = 0; r < NY; r++) u[r] = L[base + r * S::SY];
      const LineCoef<T> c = line_coef<T, NY>(fabs(nu), periodic);
      pfc_core<T, NY>(u, c.alpha, c.c1, c.c2, periodic);
      T* dst = tile_base(t);
      const unsigned off = (unsigned)iz * (unsigned)a.nv3 + (unsigned)wy;
      store_shifted<T, NY>(u, c.shift, periodic, [&](int r, T x) {
        (dst + (long long)(ry ? NY - 1 - r : r) * NZ * a.nv3)[off] = x;
      });
    }
    if (k + 1 < TILES) __syncthreads();           // LDS is reused by the next tile
  }
}

template <typename T, int NP, int W, int TILES>
hipError_t launch_drift_yz_sq(const DriftArgs& a, hipStream_t s)
{
  using S = DriftShape<T, NP, NP, W>;
  static_assert(S::fits, "tile does not fit the LDS");
  const long long tiles = a.nx * (a.nv3 / W);
  if (tiles <= 0) return hipSuccess;
  const long long blocks = (tiles + TILES - 1) / TILES;
  hipLaunchKernelGGL((drift_yz_block<T, NP, NP, W, TILES>), dim3((unsigned)blocks), dim3(S::THREADS), 0, s, a);
  return hipGetLastError();
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

// Velocity cubes whose block fits the LDS of one workgroup: FP32 up to 32^3,
// FP64 up to 24^3.
bool kick_fused_supported(int dtype, const int nv[3])
{
  if (nv[0] != nv[1] || nv[1] != nv[2]) return false;
  const int n = nv[0];
  if (dtype == 0) return n == 8 || n == 16 || n == 24 || n == 32;
  return n == 8 || n == 16 || n == 24;
}

// (y, z) planes of 16, 24 or 32 cells with whole-cache-line velocity chunks
static int drift_yz_width(int dtype, int ny, int nz, long long nv3)
{
  if (ny != nz) return 0;
  int w = 0;
  if (dtype == 0) w = (ny == 16) ? 64 : (ny == 24 || ny == 32) ? 32 : 0;
  else w = (ny == 16) ? 32 : (ny == 24 || ny == 32) ? 16 : 0;
  if (w == 0 || nv3 % w != 0) return 0;
  if ((long long)ny * nz * nv3 >= (1LL << 32)) return 0;   // 32-bit lane offsets within a tile
  return w;
}

bool drift_yz_supported(int dtype, int ny, int nz, long long nv3) { return drift_yz_width(dtype, ny, nz, nv3) != 0; }

// Tiles per workgroup: four, except two for the FP64 16- and 24-planes, whose
// workgroups are small enough that several share a CU anyway.
hipError_t launch_drift_yz(const DriftArgs& a, int dtype, hipStream_t s)
{
  const int w = drift_yz_width(dtype, a.ny, a.nz, a.nv3);
  if (dtype == 0) {
    switch (a.ny) {
      case 16: return launch_drift_yz_sq<float, 16, 64, 4>(a, s);
      case 24: return launch_drift_yz_sq<float, 24, 32, 4>(a, s);
      case 32: return launch_drift_yz_sq<float, 32, 32, 4>(a, s);
      default: break;
    }
  } else {
    switch (a.ny) {
      case 16: return launch_drift_yz_sq<double, 16, 32, 2>(a, s);
      case 24: return launch_drift_yz_sq<double, 24, 16, 2>(a, s);
      case 32: return launch_drift_yz_sq<double, 32, 16, 4>(a, s);
      default: break;
    }
  }
  (void)w;
  return hipErrorInvalidValue;
}

bool kick_pair_supported(int dtype, const int nv[3])
{
  return dtype == 1 && nv[0] == 32 && nv[1] == 32 && nv[2] == 32;
}

// 48^3 and 64^3 blocks: slices of 12 and 8 planes in FP32 (110 and 130
// KiB), 6 and 4 in FP64 (110 and 130 KiB)
bool kick_planes_supported(int dtype, const int nv[3])
{
  return (dtype == 0 || dtype == 1) && nv[0] == nv[1] && nv[1] == nv[2] && (nv[0] == 48 || nv[0] == 64);
}

hipError_t launch_kick_planes(const KickArgs& a, int dtype, const int nv[3], hipStream_t s)
{
  if (!kick_planes_supported(dtype, nv)) return hipErrorInvalidValue;
  if (dtype == 0) return nv[0] == 48 ? launch_kick_planes<float, 48, 12>(a, s) : launch_kick_planes<float, 64, 8>(a, s);
  return nv[0] == 48 ? launch_kick_planes<double, 48, 6>(a, s) : launch_kick_planes<double, 64, 4>(a, s);
}

hipError_t launch_kick_pair(const KickArgs& a, int dtype, const int nv[3], int pass, hipStream_t s)
{
  if (!kick_pair_supported(dtype, nv) || pass < 0 || pass > 2) return hipErrorInvalidValue;
  return launch_kick_pair_cube<double, 32>(a, pass, s);
}

hipError_t launch_kick(const KickArgs& a, int dtype, const int nv[3], hipStream_t s)
{
  if (!kick_fused_supported(dtype, nv)) return hipErrorInvalidValue;
  if (dtype == 0) {
    switch (nv[0]) {
      case 8: return launch_kick_cube<float, 8>(a, s);
      case 16: return launch_kick_cube<float, 16>(a, s);
      case 24: return launch_kick_cube<float, 24>(a, s);
      default: return launch_kick_cube<float, 32>(a, s);
    }
  }
  switch (nv[0]) {
    case 8: return launch_kick_cube<double, 8>(a, s);
    case 16: return launch_kick_cube<double, 16>(a, s);
    default: return launch_kick_cube<double, 24>(a, s);
  }
}

}  // namespace vp
