// kick.hip -- the velocity half kicks of Eq. (17) (T_vx, T_vy, T_vz with the
// acceleration of each spatial cell; Sec. 2.1 of Yoshikawa, Yoshida &
// Umemura) in passes that hold a whole velocity block or slices of one on
// chip. The line update is that of sweep.hip
// (pfc_line.h), so every pass rounds like the single sweeps. gfx950.
#include "vp_internal.h"

#include "pfc_line.h"
#include "buffer_io.h"
#include "vec16.h"

namespace vp {
namespace {

// ---- line coefficients of a half kick, per spatial cell ----------------------
// The three velocity sweeps of a spatial cell move with nu_l = a_l tau / dv_l,
// uniform over its velocity block. kick_table_kernel splits each |nu_l| once
// per call (line_coef, as every sweep does, so the bits agree) and the kick
// passes read the entry of their block instead of repeating the FP64
// arithmetic in every lane.
template <typename T>
struct KickTab {
  T alpha[3], c1[3], c2[3];
  int shift[3];
  int neg;      // bit l set where nu_l < 0
};

template <typename T, int NV>
__global__ __launch_bounds__(256) void kick_table_kernel(KickArgs a)
{
  const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
  if (s >= a.np) return;
  KickTab<T> t;
  t.neg = 0;
#pragma unroll
  for (int l = 0; l < 3; l++) {
    const double nu = a.a[l][s] * a.scale[l];
    const LineCoef<T> c = line_coef<T, NV>(fabs(nu), false);
    t.alpha[l] = c.alpha;
    t.c1[l] = c.c1;
    t.c2[l] = c.c2;
    t.shift[l] = c.shift;
    t.neg |= nu < 0.0 ? 1 << l : 0;
  }
  static_cast<KickTab<T>*>(a.tab)[s] = t;
}

template <typename T, int NV>
hipError_t launch_kick_table(const KickArgs& a, hipStream_t s)
{
  if (!a.tab) return hipErrorInvalidValue;
  hipLaunchKernelGGL((kick_table_kernel<T, NV>), dim3((unsigned)((a.np + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

__device__ __forceinline__ bool tab_neg(int neg, int l) { return (neg >> l) & 1; }

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
  static_assert(NX == NY && NY == NZ, "the coefficient table is built for cubic blocks");
  const KickTab<T>* __restrict__ tab = static_cast<const KickTab<T>*>(a.tab) + s;
  const bool rx = tab_neg(tab->neg, 0), ry = tab_neg(tab->neg, 1), rz = tab_neg(tab->neg, 2);
  const LineCoef<T> cx{tab->alpha[0], tab->c1[0], tab->c2[0], tab->shift[0], false};
  const LineCoef<T> cy{tab->alpha[1], tab->c1[1], tab->c2[1], tab->shift[1], false};
  const LineCoef<T> cz{tab->alpha[2], tab->c1[2], tab->c2[2], tab->shift[2], false};
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
  const hipError_t e = launch_kick_table<T, NV>(a, s);
  if (e != hipSuccess) return e;
  if (a.reps == 2)
    hipLaunchKernelGGL((kick_block<T, NV, NV, NV, 2>), dim3((unsigned)a.np), dim3(S::THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((kick_block<T, NV, NV, NV, 1>), dim3((unsigned)a.np), dim3(S::THREADS), 0, s, a);
  return hipGetLastError();
}

// ---- two velocity sweeps in one pass over slices of a velocity block ---------
// When a whole velocity block does not fit in LDS, two consecutive sweeps whose
// lines both lie in a slice of CH planes run in one pass: PASS 0 is T_vx then
// T_vy on the slice with vz in [c0, c0 + CH); PASS 1 is T_vz then T_vx on the
// slice with vy in the chunk; PASS 2 is T_vy then T_vz on the slice with vx in
// the chunk. The two half kicks between two drifts (T_vx T_vy T_vz T_vx T_vy
// T_vz) are PASS 0, 1, 2; a lone half kick is a T_vx sweep and PASS 2 (or
// PASS 0 and a T_vz sweep). Each LDS layout keeps the HBM-contiguous axis
// contiguous and pads rows so both sweep directions are bank-conflict free;
// the arithmetic is that of the single sweeps.
template <typename T, int NV, int PASS, int CH_ = NV / 2>
struct PairShape {
  static constexpr int CH = CH_;                         // planes across the third axis
  static constexpr int NCH = NV / CH;                    // slices per velocity block
  // PASS 0 vx rows of SA = NV CH + PAD elements, SA = CH (mod the 64 banks
  // of 4 bytes), so that the T_vy lanes (vx, c) of a wave take distinct banks
  static constexpr int WD = (int)sizeof(T) / 4;           // banks per element
  static constexpr int PAD = ((CH_ - NV * CH_) * WD % 64 + 64) % 64 / WD;
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
  // workgroup -> (spatial cell s, slice): the slices of one velocity block
  // take consecutive workgroups, or with a.xcd_group (np a multiple of 8) the
  // workgroups b = 8 (NCH m + q) + x, which the hardware's round-robin over
  // the 8 XCDs places on one XCD (x) one after another, so that slices that
  // share cache lines (vz-slices: runs of CH values of each vz row) meet in
  // that XCD's L2
  long long s;
  int slice;
  if (a.xcd_group) {
    const long long b = blockIdx.x, x = b & 7, k = b >> 3, m = k / S::NCH;
    slice = (int)(k - m * S::NCH);
    s = 8 * m + x;
  } else {
    s = blockIdx.x / S::NCH;
    slice = (int)(blockIdx.x - s * S::NCH);
  }
  const int c0 = slice * CH;
  const long long cofs = PASS == 0 ? c0 : (PASS == 1 ? c0 * NV : c0 * NV * NV);
  T* g = static_cast<T*>(a.f) + s * (long long)(NV * NV * NV) + cofs;
  // the two sweeps: axis A then axis B (0 = vx, 1 = vy, 2 = vz)
  constexpr int AX0 = PASS == 0 ? 0 : (PASS == 1 ? 2 : 1);
  constexpr int AX1 = PASS == 0 ? 1 : (PASS == 1 ? 0 : 2);
  const KickTab<T>* __restrict__ tab = static_cast<const KickTab<T>*>(a.tab) + s;
  const bool f0 = tab_neg(tab->neg, AX0), f1 = tab_neg(tab->neg, AX1);
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
    pfc_core<T, NV>(v, tab->alpha[ax], tab->c1[ax], tab->c2[ax], false);
    store_shifted<T, NV>(v, tab->shift[ax], false, [&](int r, T x) { L[base + r * st] = x; });
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

// ---- T_vx then T_vy with two lines per lane, on vz-slices of W cells ---------
// The first of the three slice passes for blocks whose vz-slices of the layout
// above would hold only 32-byte runs (64^3 FP32: 8 values). Lane (i, p) of the
// NV x W/2 lanes holds the lines of the adjacent vz cells 2p and 2p + 1 of the
// slice: the vx lines (vy = i) come in as 8-byte pairs, so that a row of W/2
// lanes reads one whole W-cell run (64 bytes), in the sweep's orientation, and
// are swept in registers. They reach the vy sweep through LDS in two rounds
// (cells 2p, then 2p + 1) of W/2 columns each, parked at their storage vx and
// at the vy place of the vy sweep's orientation; lane (i, p) then takes the vy
// lines (vx = i) of the same two cells, which go back to HBM as pairs. All
// lines of a block share the spatial cell's coefficients, shifts and
// orientations. The slices of a block share cache lines and are grouped per
// XCD as in kick_pair_block.
template <typename T, int NV, int W>
struct KvPairShape {
  static constexpr int H = W / 2;                                   // LDS columns per round
  static constexpr int SX0 = NV * H;
  static constexpr int SX = SX0 + ((((H - SX0) % 64) + 64) % 64);   // = H (mod 64)
  static constexpr int ELEMS = NV * SX;
  static constexpr int BYTES = ELEMS * (int)sizeof(T);
  static constexpr int THREADS = NV * H;
  static constexpr int NCH = NV / W;
  static constexpr bool fits = BYTES <= 160 * 1024 && THREADS <= 1024 && THREADS % 64 == 0 && NV % W == 0;
};

// One round of kick_vxvy_pairs: the lane's swept vx line goes to LDS at its
// storage vx places and at the vy place of the vy sweep's orientation; after
// the barrier the lane takes the vy line of storage vx = i0 of the same cell
// and sweeps it.
template <typename T, int NV, int W>
__device__ __forceinline__ void kv_round(T (&v)[NV], T* L, int i0, int p, bool fx, bool fy,
                                         const KickTab<T>* __restrict__ tab)
{
  using S = KvPairShape<T, NV, W>;
  constexpr int H = S::H;
  const int yb = (fy ? NV - 1 - i0 : i0) * H + p;
  store_shifted<T, NV>(v, tab->shift[0], false, [&](int d, T x) { L[(fx ? NV - 1 - d : d) * S::SX + yb] = x; });
  __syncthreads();
  const int xb = i0 * S::SX + p;
#pragma unroll
  for (int r = 0; r < NV; r++) v[r] = L[xb + r * H];
  pfc_core<T, NV>(v, tab->alpha[1], tab->c1[1], tab->c2[1], false);
  __syncthreads();  // LDS is reused by the next round
}

template <typename T, int NV, int W>
__global__ __launch_bounds__((KvPairShape<T, NV, W>::THREADS)) void kick_vxvy_pairs(KickArgs a)
{
  static_assert(sizeof(T) == 4, "8-byte pairs of FP32 cells");
  using S = KvPairShape<T, NV, W>;
  constexpr int H = S::H;
  constexpr unsigned PLANEB = NV * NV * 4u, ROWB = NV * 4u, BLKB = NV * PLANEB;
  __shared__ T L[S::ELEMS];
  const int tid = threadIdx.x;
  const int i0 = tid / H, p = tid - i0 * H;
  long long s;
  int slice;
  if (a.xcd_group) {
    const long long b = blockIdx.x, x = b & 7, k = b >> 3, m = k / S::NCH;
    slice = (int)(k - m * S::NCH);
    s = 8 * m + x;
  } else {
    s = blockIdx.x / S::NCH;
    slice = (int)(blockIdx.x - s * S::NCH);
  }
  const auto rs = buf_rsrc(static_cast<const T*>(a.f) + s * (long long)(NV * NV * NV), BLKB);
  const unsigned cofs = (unsigned)(slice * W + 2 * p) * 4u;   // the pair's vz cells, bytes
  const KickTab<T>* __restrict__ tab = static_cast<const KickTab<T>*>(a.tab) + s;
  const bool fx = tab_neg(tab->neg, 0), fy = tab_neg(tab->neg, 1);
  T v0[NV], v1[NV];
  {
    // vx lines (vy = i0), rows read in the sweep's orientation
    const unsigned voff = (unsigned)i0 * ROWB + cofs;
#pragma unroll
    for (int r = 0; r < NV; r++) {
      const float2 x = buf_load_pair(rs, voff, (unsigned)(fx ? NV - 1 - r : r) * PLANEB);
      v0[r] = x.x;
      v1[r] = x.y;
    }
  }
  pfc_core<T, NV>(v0, tab->alpha[0], tab->c1[0], tab->c2[0], false);
  pfc_core<T, NV>(v1, tab->alpha[0], tab->c1[0], tab->c2[0], false);
  kv_round<T, NV, W>(v0, L, i0, p, fx, fy, tab);
  kv_round<T, NV, W>(v1, L, i0, p, fx, fy, tab);
  // sweep place d of a vy line (vx = i0) is storage vy = d, or NV-1-d where a_y < 0
  char* wb = static_cast<char*>(a.f) + s * (long long)BLKB + (unsigned)i0 * PLANEB + cofs;
  store_shifted2<T, NV>(v0, v1, tab->shift[1], false, [&](int d, T x0, T x1) {
    *reinterpret_cast<float2*>(wb + (unsigned)(fy ? NV - 1 - d : d) * ROWB) = float2{x0, x1};
  });
}

// vz-slice width of the two-lines-per-lane T_vx T_vy pass, or 0 where the
// slices of kick_pair_block already hold whole 64-byte runs
template <typename T, int NV>
constexpr int vxvy_pair_width()
{
  return (sizeof(T) == 4 && NV == 64) ? 16 : 0;
}

// The three two-sweep passes of two consecutive half kicks (T_vx T_vy on
// slices of CV vz-planes, T_vz T_vx on slices of CY vy-rows, T_vy T_vz on
// slices of CX vx-planes) for velocity blocks whose halves exceed the LDS:
// six sweeps in three passes instead of four (two T_vx sweeps and two
// plane passes)
template <typename T, int NV, int CV, int CY, int CX>
hipError_t launch_kick_slices(const KickArgs& a0, int pass, hipStream_t s)
{
  static_assert(PairShape<T, NV, 0, CV>::fits && PairShape<T, NV, 1, CY>::fits && PairShape<T, NV, 2, CX>::fits,
                "slice does not fit the LDS");
  if (a0.np <= 0) return hipSuccess;
  if (pass == 0) {
    const hipError_t e = launch_kick_table<T, NV>(a0, s);
    if (e != hipSuccess) return e;
  }
  KickArgs a = a0;
  a.xcd_group = (a.np % 8 == 0) ? 1 : 0;
  switch (pass) {
    case 0:
      if constexpr (vxvy_pair_width<T, NV>() > 0) {
        using K = KvPairShape<T, NV, vxvy_pair_width<T, NV>()>;
        static_assert(K::fits, "slice does not fit the LDS");
        hipLaunchKernelGGL((kick_vxvy_pairs<T, NV, vxvy_pair_width<T, NV>()>), dim3((unsigned)(K::NCH * a.np)),
                           dim3(K::THREADS), 0, s, a);
      } else {
        hipLaunchKernelGGL((kick_pair_block<T, NV, 0, CV>), dim3((unsigned)(PairShape<T, NV, 0, CV>::NCH * a.np)),
                           dim3(PairShape<T, NV, 0, CV>::THREADS), 0, s, a);
      }
      break;
    case 1:
      hipLaunchKernelGGL((kick_pair_block<T, NV, 1, CY>), dim3((unsigned)(PairShape<T, NV, 1, CY>::NCH * a.np)),
                         dim3(PairShape<T, NV, 1, CY>::THREADS), 0, s, a);
      break;
    default:
      hipLaunchKernelGGL((kick_pair_block<T, NV, 2, CX>), dim3((unsigned)(PairShape<T, NV, 2, CX>::NCH * a.np)),
                         dim3(PairShape<T, NV, 2, CX>::THREADS), 0, s, a);
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
  const hipError_t e = launch_kick_table<T, NV>(a, s);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)(S::NCH * a.np);
  hipLaunchKernelGGL((kick_pair_block<T, NV, 2, CH>), dim3(blocks), dim3(S::THREADS), 0, s, a);
  return hipGetLastError();
}


// ---- FP64 32^3 blocks: the sweeps of one or two half kicks in one pass ------
// A block of 32^3 doubles (256 KiB) does not fit in LDS, so here it lives in
// registers: each of the 1024 lanes holds one whole line of the block along
// the axis being swept. Between sweeps along different axes the block changes
// hands through LDS in two halves: the lines of one orientation (S) are
// written and those of the next (D) read back. S and D lines share one
// coordinate (the third axis), and each lane holds its S line and its D line
// in the same half of it (both lane maps put that coordinate's top bit on the
// same lane bit), so a lane writes its old line before it reads its new one
// and never holds two. Half 0 trades first; half 1 writes while half 0 sweeps
// its new lines, and lines left unswept by half 1 are swept while half 0 of
// the next exchange writes, so LDS traffic overlaps the arithmetic. Every axis
// is held in its sweep's orientation (reversed where nu < 0), as in
// kick_block, and each sweep's whole-cell shift is applied where its lines
// are written to LDS. LDS layouts, in doubles of oriented (x, y, z):
//   x <-> y (halves of z):  528 x + 16 y + (z & 15)
//   y <-> z (halves of x):  1072 (x & 15) + 33 y + z
//   z <-> x (halves of y):  512 x + 32 (y & 15) + (z ^ g),
//                           g = 16 (y & 1) + 2 ((y & 15) >> 1) + (x & 1),
// so that 32 consecutive lanes touch 32 different bank pairs in every access.
// Lane maps (lane t, t[i:j] its bits i..j):
//   x lines (y, z): z = t[0:3] + 16 t[9], y = t[4:7] + 16 t[8]
//   y lines (x, z): z = t[0:3] + 16 t[9], x = t[4:6] + 8 t[8] + 16 t[7]
//   z lines (x, y): y = t[0:3] + 16 t[8], x = t[4:6] + 8 t[9] + 16 t[7]
// The first x lines come straight from HBM and the last ones go straight back
// (each row of a wave is four runs of 16 values); after the last z sweep one
// more exchange hands the block to x lines for that.
constexpr int KL_N = 32;
constexpr int KL_ELEMS = 1072 * 15 + 33 * 31 + 31 + 1;   // the largest layout's extent

template <int REPS>
__global__ __launch_bounds__(1024) void kick_lines_f64(KickArgs a)
{
  constexpr int N = KL_N;
  constexpr unsigned ROWB = N * N * 8u;                   // bytes between vx planes
  constexpr unsigned BLKB = N * N * N * 8u;
  __shared__ double L[KL_ELEMS];
  const int t = threadIdx.x;
  const long long s = blockIdx.x;
  const auto rs = buf_rsrc(static_cast<const double*>(a.f) + s * (N * N * N), BLKB);
  const auto ws = a.out ? buf_rsrc(static_cast<const double*>(a.out) + s * (N * N * N), BLKB) : rs;
  const KickTab<double>* __restrict__ tab = static_cast<const KickTab<double>*>(a.tab) + s;
  const bool rx = tab_neg(tab->neg, 0), ry = tab_neg(tab->neg, 1), rz = tab_neg(tab->neg, 2);
  const double ax = tab->alpha[0], ay = tab->alpha[1], az = tab->alpha[2];
  const double c1x = tab->c1[0], c1y = tab->c1[1], c1z = tab->c1[2];
  const double c2x = tab->c2[0], c2y = tab->c2[1], c2z = tab->c2[2];
  const int shx = tab->shift[0], shy = tab->shift[1], shz = tab->shift[2];
  const int b7 = (t >> 7) & 1, b8 = (t >> 8) & 1, b9 = (t >> 9) & 1;
  const int lo = t & 15;
  const int xl_z = lo + 16 * b9, xl_y = ((t >> 4) & 15) + 16 * b8;            // x line (y, z)
  const int yl_z = lo + 16 * b9, yl_x = ((t >> 4) & 7) + 8 * b8 + 16 * b7;    // y line (x, z)
  const int zl_y = lo + 16 * b8, zl_x = ((t >> 4) & 7) + 8 * b9 + 16 * b7;    // z line (x, y)
  double v[N];

  auto sweep_x = [&]() { pfc_core<double, N>(v, ax, c1x, c2x, false); };
  auto sweep_y = [&]() { pfc_core<double, N>(v, ay, c1y, c2y, false); };
  auto sweep_z = [&]() { pfc_core<double, N>(v, az, c1z, c2z, false); };
  auto write_x = [&]() {
    const int base = xl_y * 16 + (xl_z & 15);
    store_shifted<double, N>(v, shx, false, [&](int d, double x) { L[base + d * 528] = x; });
  };
  auto read_y = [&]() {
    const int base = yl_x * 528 + (yl_z & 15);
#pragma unroll
    for (int r = 0; r < N; r++) v[r] = L[base + r * 16];
  };
  auto write_y = [&]() {
    const int base = (yl_x & 15) * 1072 + yl_z;
    store_shifted<double, N>(v, shy, false, [&](int d, double x) { L[base + d * 33] = x; });
  };
  auto read_z = [&]() {
    const int base = (zl_x & 15) * 1072 + zl_y * 33;
#pragma unroll
    for (int r = 0; r < N; r++) v[r] = L[base + r];
  };
  auto write_z = [&]() {
    const int yl = zl_y & 15;
    const int base = zl_x * 512 + yl * 32;
    const int g = 16 * (yl & 1) + 2 * (yl >> 1) + (zl_x & 1);
    store_shifted<double, N>(v, shz, false, [&](int d, double x) { L[base + (d ^ g)] = x; });
  };
  auto read_x = [&]() {
    const int yl = xl_y & 15;
    const int zg = xl_z ^ (16 * (yl & 1) + 2 * (yl >> 1));   // z ^ g without the x bit
    const int base = yl * 32;
#pragma unroll
    for (int r = 0; r < N; r++) v[r] = L[r * 512 + base + (zg ^ (r & 1))];
  };
  // one change of orientation, halves by lane bit h; pend: the S line still
  // awaits its sweep
  auto exchange = [&](bool h, bool pend, auto&& sweepS, auto&& writeS, auto&& readD, auto&& sweepD) {
    if (pend) sweepS();
    if (!h) writeS();
    __syncthreads();
    if (!h) readD();
    __syncthreads();
    if (!h) sweepD();
    else writeS();
    __syncthreads();
    if (h) readD();
    __syncthreads();
  };

  // x lines from HBM: lane (y, z) reads rows x in its sweep orientation
  const int ys = ry ? N - 1 - xl_y : xl_y, zs = rz ? N - 1 - xl_z : xl_z;
  const unsigned voff = (unsigned)(ys * N + zs) * 8u;
#pragma unroll
  for (int r = 0; r < N; r++) v[r] = buf_load<double>(rs, voff, (unsigned)(rx ? N - 1 - r : r) * ROWB);
  exchange(b9, true, sweep_x, write_x, read_y, sweep_y);
  exchange(b7, b9, sweep_y, write_y, read_z, sweep_z);
  if constexpr (REPS == 2) {
    exchange(b8, b7, sweep_z, write_z, read_x, sweep_x);
    exchange(b9, b8, sweep_x, write_x, read_y, sweep_y);
    exchange(b7, b9, sweep_y, write_y, read_z, sweep_z);
  }
  // the last z lines go to x lines, which go back to HBM as they arrive
  auto store_x = [&]() {
#pragma unroll
    for (int r = 0; r < N; r++) buf_store<double>(ws, voff, (unsigned)(rx ? N - 1 - r : r) * ROWB, v[r]);
  };
  const bool pend = b7, h = b8;
  if (pend) sweep_z();
  if (!h) write_z();
  __syncthreads();
  if (!h) read_x();
  __syncthreads();
  if (!h) store_x();
  else write_z();
  __syncthreads();
  if (h) {
    read_x();
    store_x();
  }
}

hipError_t launch_kick_lines_f64(const KickArgs& a, hipStream_t s)
{
  static_assert(KL_ELEMS * 8 <= 160 * 1024, "LDS");
  if (a.np <= 0) return hipSuccess;
  const hipError_t e = launch_kick_table<double, KL_N>(a, s);
  if (e != hipSuccess) return e;
  if (a.reps == 2)
    hipLaunchKernelGGL((kick_lines_f64<2>), dim3((unsigned)a.np), dim3(1024), 0, s, a);
  else
    hipLaunchKernelGGL((kick_lines_f64<1>), dim3((unsigned)a.np), dim3(1024), 0, s, a);
  return hipGetLastError();
}

}  // namespace

// Velocity cubes whose block fits the LDS of one workgroup: FP32 up to 32^3,
// FP64 up to 24^3.
bool kick_fused_supported(int dtype, const int nv[3])
{
  if (nv[0] != nv[1] || nv[1] != nv[2]) return false;
  const int n = nv[0];
  if (dtype == 0) return n == 8 || n == 16 || n == 24 || n == 32;
  return n == 8 || n == 16 || n == 24;
}

size_t kick_table_bytes(int dtype, long long np)
{
  return (size_t)np * (dtype == 0 ? sizeof(KickTab<float>) : sizeof(KickTab<double>));
}

bool kick_lines_supported(int dtype, const int nv[3])
{
  return dtype == 1 && nv[0] == KL_N && nv[1] == KL_N && nv[2] == KL_N;
}

hipError_t launch_kick_lines(const KickArgs& a, int dtype, const int nv[3], hipStream_t s)
{
  if (!kick_lines_supported(dtype, nv) || (a.reps != 1 && a.reps != 2)) return hipErrorInvalidValue;
  return launch_kick_lines_f64(a, s);
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

// 48^3 and 64^3 FP32 blocks: vz-slices of 16 planes (48^3; 147 KiB) or the
// two-lines-per-lane pass on 16-cell vz-slices (64^3; 130 KiB), vy-slices of
// 16 and 8 rows, vx-slices of 12 and 8 planes (150, 110 KiB; 130, 130 KiB).
// 48^3 FP64 blocks: slices of 8 planes or rows for all three passes (64-byte
// vz runs, 147 KiB each). FP64 64^3 would leave 32-byte vz runs and keeps the
// four-pass route.
bool kick_slices_supported(int dtype, const int nv[3])
{
  if (nv[0] != nv[1] || nv[1] != nv[2]) return false;
  return dtype == 0 ? (nv[0] == 48 || nv[0] == 64) : nv[0] == 48;
}

hipError_t launch_kick_slices(const KickArgs& a, int dtype, const int nv[3], int pass, hipStream_t s)
{
  if (!kick_slices_supported(dtype, nv) || pass < 0 || pass > 2) return hipErrorInvalidValue;
  if (dtype == 1) return launch_kick_slices<double, 48, 8, 8, 8>(a, pass, s);
  return nv[0] == 48 ? launch_kick_slices<float, 48, 16, 16, 12>(a, pass, s)
                     : launch_kick_slices<float, 64, 8, 8, 8>(a, pass, s);
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
