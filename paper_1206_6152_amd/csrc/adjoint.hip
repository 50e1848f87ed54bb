// adjoint.hip -- reverse mode of the directional PFC sweep (not in the paper;
// it gives gradients of the final field energy for the C ABI's vp_grad).
//
// For one line with forward input f (the sweep's input state), Courant number
// nu = s + sign * alpha and output adjoint lam_out, the lane recomputes the
// forward quantities (f_inf and its first argmax, the one-sided differences
// and which bound of each corrector clamp is active) and runs the flux form
// backwards, in the same mirrored register view as the forward update:
//   lam_g_k = lam_out_{k+s}                     (transpose of the shift)
//   lam_F_k = lam_g_{k+1} - lam_g_k             (F_k leaves cell k, enters k+1)
//   F_k = alpha * (f_k + c1 Lp_k + c2 Lm_k):
//     lam_f_k += alpha lam_F_k, lam_Lp = c1 alpha lam_F_k, lam_Lm = c2 alpha lam_F_k,
//     lam_alpha += lam_F_k (f_k + c1 Lp_k + c2 Lm_k + alpha (c1' Lp_k + c2' Lm_k)),
//     c1' = (2 alpha - 3)/6, c2' = -alpha/3;
//   Lp = clamp(f_{k+1} - f_k, 2 f_k - 2 f_inf, 2 f_k) and
//   Lm = clamp(f_k - f_{k-1}, -2 f_k, 2 f_inf - 2 f_k) pass their adjoint to
//   the operands of the active branch (a bound is active only when the
//   difference is strictly beyond it), f_inf passes its adjoint to the first
//   cell holding the maximum, and lam_nu = sign * lam_alpha.
// A velocity sweep's nu = a_l(x) tau / dv_l sends lam_nu to the acceleration;
// the per-line values are reduced per spatial cell in a fixed order.
#include "pfc_line.h"
#include "vec16.h"
#include "vp_internal.h"

namespace vp {
namespace {

// Reverse of pfc_line + store_shifted for one line; returns d<lam_out, out>/d nu.
// `at(r)` is the offset of storage cell r of the lane's line from both bases.
//
// The view runs along the transport direction: view cell i is storage cell i
// (nu >= 0) or N-1-i (nu < 0); the lane's forward line and lam line are
// mirrored into the view with selects, so every lane follows the same
// instruction stream whatever its sign. In the view the shift is
// m = floor(|nu|) >= 0 and its transpose is lam_g_k = lam_out_{k+m} (zero
// beyond an outflow end, wrapped if periodic). One pass over the cells in view
// order then writes out_{i-1} once cell i is known: cell i sends its own terms
// to out_i, its Lp interior-branch term to out_{i+1} and its Lm interior-branch
// term to out_{i-1}.
// la(r, x) gives the lam value of cell r from its stored value x.
// GATHER (lines in LDS): where the line has a whole-cell shift, lam_g is
// read straight into view order, each view cell from the storage cell that
// the mirror and the transposed shift name, instead of loading lam in
// storage order and permuting registers with selects (N^2 of them for the
// shift); the same values land in the same registers.
template <typename T, int N, bool GATHER = false, typename AT, typename LA>
__device__ __forceinline__ double adj_line(const T* fin, T* lam, double nu, bool periodic, AT at, LA la)
{
#pragma clang fp contract(off)
  const LineCoef<T> k = line_coef<T, N>(nu, periodic);
  const bool neg = k.neg;
  T w[N], l[N];
  if constexpr (GATHER) {
    const int m = neg ? -k.shift : k.shift;   // >= 0, below N when periodic
#pragma unroll
    for (int r = 0; r < N; r++) w[r] = fin[at(r)];
    if (m == 0) {                             // no shift: storage order, then the mirror
#pragma unroll
      for (int r = 0; r < N; r++) l[r] = la(r, lam[at(r)]);
#pragma unroll
      for (int i = 0; i < N / 2; i++) {
        const T p = l[i], q = l[N - 1 - i];
        l[i] = neg ? q : p;
        l[N - 1 - i] = neg ? p : q;
      }
    } else {
#pragma unroll
      for (int i = 0; i < N; i++) {
        int j = i + m;
        if (periodic && j >= N) j -= N;
        const bool in = j < N;                // else past an outflow end: zero
        const int rs = in ? (neg ? N - 1 - j : j) : 0;
        const T x = la(rs, lam[at(rs)]);
        l[i] = in ? x : T(0);
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < N; r++) {
      w[r] = fin[at(r)];
      l[r] = la(r, lam[at(r)]);
    }
  }
  // f_inf and the first storage cell that holds it
  T finf = T(0);
  int am = -1;
#pragma unroll
  for (int r = 0; r < N; r++)
    if (w[r] > finf) {
      finf = w[r];
      am = r;
    }
  const int amv = (neg && am >= 0) ? N - 1 - am : am;   // its view index
#pragma unroll
  for (int i = 0; i < N / 2; i++) {
    const T x = w[i], y = w[N - 1 - i];
    w[i] = neg ? y : x;
    w[N - 1 - i] = neg ? x : y;
    if constexpr (!GATHER) {
      const T p = l[i], q = l[N - 1 - i];
      l[i] = neg ? q : p;
      l[N - 1 - i] = neg ? p : q;
    }
  }
  const int m = neg ? -k.shift : k.shift;
  if (!GATHER && m != 0) {
    T g[N];
#pragma unroll
    for (int i = 0; i < N; i++) {
      int src = i + m;
      if (periodic) src %= N;
      T x = T(0);
#pragma unroll
      for (int j = 0; j < N; j++)
        if (j == src) x = l[j];
      g[i] = x;
    }
#pragma unroll
    for (int i = 0; i < N; i++) l[i] = g[i];
  }
  const double a = fabs(nu);
  const double al = a - floor(a);
  const T dc1 = (T)((2.0 * al - 3.0) / 6.0);
  const T dc2 = (T)(-al / 3.0);
  const T alpha = k.alpha, c1 = k.c1, c2 = k.c2;
  const T twoinf = finf + finf;
  const T lg0 = l[0];
  T dm = periodic ? w[0] - w[N - 1] : w[0];
  // d<lam_out, out>/d alpha = sum_i lam_F_i d F_i / d alpha, first on its own
  T lalpha = T(0);
  {
    T dmq = periodic ? w[0] - w[N - 1] : w[0];
#pragma unroll
    for (int i = 0; i < N; i++) {
      const T f0 = w[i];
      const T fr = (i + 1 < N) ? w[i + 1 < N ? i + 1 : 0] : (periodic ? w[0] : T(0));
      const T dp = fr - f0;
      const T h = f0 + f0;
      const T r = twoinf - h;
      const T lp = clamp_ordered(dp, -r, h);
      const T lm = clamp_ordered(dmq, -h, r);
      const T lgn = (i + 1 < N) ? l[i + 1 < N ? i + 1 : 0] : (periodic ? lg0 : T(0));
      const T lF = lgn - l[i];
      const T q = fma_(c2, lm, fma_(c1, lp, f0));
      lalpha = lalpha + lF * (q + alpha * (dc1 * lp + dc2 * lm));
      dmq = dp;
    }
  }
  // fresh copies, so that nothing of the first pass is kept for the second
#pragma unroll
  for (int i = 0; i < N; i++) asm volatile("" : "+v"(w[i]));
  T lfinf = T(0);
  T carry = T(0), pending = T(0), wrap_back = T(0);
#pragma unroll
  for (int i = 0; i < N; i++) {
    const T f0 = w[i];
    const T fr = (i + 1 < N) ? w[i + 1 < N ? i + 1 : 0] : (periodic ? w[0] : T(0));
    const T dp = fr - f0;
    const T h = f0 + f0;
    const T r = twoinf - h;
    const T lgi = l[i];
    const T lgn = (i + 1 < N) ? l[i + 1 < N ? i + 1 : 0] : (periodic ? lg0 : T(0));
    const T lF = lgn - lgi;                      // lam_F_i = lam_g_{i+1} - lam_g_i
    const T lin = alpha * lF;
    const T llp = c1 * lin;
    const T llm = c2 * lin;
    const bool p_lo = dp < -r, p_hi = dp > h;
    const bool m_lo = dm < -h, m_hi = dm > r;
    const bool p_mid = !(p_lo || p_hi), m_mid = !(m_lo || m_hi);
    T own = lgi + lin;
    own = own + (p_mid ? -llp : T(2) * llp);
    own = own + (m_mid ? llm : -(T(2) * llm));
    own = own + carry;
    lfinf = lfinf - (p_lo ? T(2) * llp : T(0));
    lfinf = lfinf + (m_hi ? T(2) * llm : T(0));
    const T back = m_mid ? -llm : T(0);
    if (i > 0) l[i > 0 ? i - 1 : 0] = pending + back;
    else wrap_back = back;
    pending = own;
    carry = p_mid ? llp : T(0);
    dm = dp;
  }
  l[N - 1] = pending + (periodic ? wrap_back : T(0));
  if (periodic) l[0] = l[0] + carry;
#pragma unroll
  for (int i = 0; i < N; i++) {
    if (i == amv) l[i] = l[i] + lfinf;
  }
  // back to storage order
#pragma unroll
  for (int i = 0; i < N / 2; i++) {
    const T p = l[i], q = l[N - 1 - i];
    l[i] = neg ? q : p;
    l[N - 1 - i] = neg ? p : q;
  }
#pragma unroll
  for (int r = 0; r < N; r++) lam[at(r)] = l[r];
  return neg ? -(double)lalpha : (double)lalpha;
}

template <typename T, int N, bool GATHER = false, typename AT>
__device__ __forceinline__ double adj_line(const T* fin, T* lam, double nu, bool periodic, AT at)
{
  return adj_line<T, N, GATHER>(fin, lam, nu, periodic, at, [](int, T x) { return x; });
}

__device__ __forceinline__ double adj_line_nu(const SweepArgs& a, long long o, long long c)
{
  if (a.velocity) return a.accel[o / a.sp_div] * a.scale;
  const long long j = (c / a.j_div) % a.j_mod;
  return (a.vmin + ((double)j + 0.5) * a.dv) * a.scale;
}

// NARROW: the workgroup's first line is the uniform base and a lane's cells sit
// at base + r*inner + off with a 32-bit offset (the host checks that they fit),
// as in the forward strided sweep; otherwise 64-bit addressing per lane.
template <typename T, int N, bool NARROW, bool ADD = false>
__global__ __launch_bounds__(256) void sweep_adj_kernel(SweepArgs a, const T* fin, T* lam, double* dnu)
{
  const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
  if (gid >= a.nlines) return;
  double d;
  if constexpr (NARROW) {
    const long long gid0 = (long long)blockIdx.x * 256;
    const unsigned t = threadIdx.x;
    const long long o0 = gid0 / a.inner;
    const unsigned inner = (unsigned)a.inner;
    const unsigned c0 = (unsigned)(gid0 - o0 * a.inner);
    const unsigned cc = c0 + t;
    const unsigned dov = cc / inner;
    const unsigned c = cc - dov * inner;
    const unsigned off = dov * (unsigned)(N * inner) + c - c0;
    const long long b0 = o0 * N * (long long)inner + c0;
    double nu;
    if (a.velocity) {
      const long long q0 = o0 / a.sp_div;
      const unsigned r0 = (unsigned)(o0 - q0 * a.sp_div);
      nu = a.accel[q0 + (r0 + dov) / (unsigned)a.sp_div] * a.scale;
    } else {
      const unsigned j = (c / (unsigned)a.j_div) % (unsigned)a.j_mod;
      nu = (a.vmin + ((double)j + 0.5) * a.dv) * a.scale;
    }
    // uniform row base (r * inner) plus the lane's 32-bit offset
    if constexpr (ADD) {
      const long long o = o0 + dov;
      const double* add = a.addend + c / (unsigned)a.add_div;
      d = adj_line<T, N>(fin + b0, lam + b0, nu, a.periodic != 0,
                         [&](int r) { return (long long)r * inner + off; },
                         [&](int r, T x) { return (T)((double)x + a.add_coef * add[(o * N + r) * a.add_stride]); });
    } else {
      d = adj_line<T, N>(fin + b0, lam + b0, nu, a.periodic != 0,
                         [&](int r) { return (long long)r * inner + off; });
    }
  } else {
    const long long o = gid / a.inner;
    const long long c = gid - o * a.inner;
    const long long base = o * (long long)N * a.inner + c;
    const long long inner = a.inner;
    d = adj_line<T, N>(fin + base, lam + base, adj_line_nu(a, o, c), a.periodic != 0,
                       [&](int r) { return (long long)r * inner; });
  }
  if (dnu) dnu[gid] = d;
}

// Contiguous lines (inner == 1, the vz sweep): a workgroup stages LINES
// consecutive lines of the forward input and of lam through LDS with coalesced
// loads (rows padded to N + 1), each lane runs the reverse update of one line
// there, and lam goes back the same way.
template <typename T, int N>
struct AdjContig {
  static constexpr int P = N + 1;
  static constexpr int LINES = (2 * 256 * P * (int)sizeof(T) <= 65536) ? 256
                               : (2 * 128 * P * (int)sizeof(T) <= 65536) ? 128 : 64;
};

template <typename T, int N>
__global__ __launch_bounds__((AdjContig<T, N>::LINES)) void sweep_adj_contig(SweepArgs a, const T* fin, T* lam,
                                                                             double* dnu)
{
  using S = AdjContig<T, N>;
  constexpr int LINES = S::LINES, P = S::P;
  __shared__ T tf[LINES * P];
  __shared__ T tl[LINES * P];
  const int tid = threadIdx.x;
  const long long line0 = (long long)blockIdx.x * LINES;
  const long long left = a.nlines - line0;
  const int nl = left < LINES ? (int)left : LINES;
  const T* gf = fin + line0 * N;
  T* gl = lam + line0 * N;
  if (nl == LINES) {
    T xf[N], xl[N];
#pragma unroll
    for (int k = 0; k < N; k++) {
      xf[k] = gf[tid + k * LINES];
      xl[k] = gl[tid + k * LINES];
    }
#pragma unroll
    for (int k = 0; k < N; k++) {
      const int e = tid + k * LINES;
      tf[(e / N) * P + (e % N)] = xf[k];
      tl[(e / N) * P + (e % N)] = xl[k];
    }
  } else {
    for (int e = tid; e < nl * N; e += LINES) {
      tf[(e / N) * P + (e % N)] = gf[e];
      tl[(e / N) * P + (e % N)] = gl[e];
    }
  }
  __syncthreads();
  if (tid < nl) {
    const long long line = line0 + tid;
    const double nu = a.velocity ? a.accel[line / a.sp_div] * a.scale
                                 : (a.vmin + 0.5 * a.dv) * a.scale;   // one velocity cell on this axis
    const double d = adj_line<T, N>(tf + tid * P, tl + tid * P, nu, a.periodic != 0, [&](int r) { return r; });
    if (dnu) dnu[line] = d;
  }
  __syncthreads();
  if (nl == LINES) {
#pragma unroll
    for (int k = 0; k < N; k++) {
      const int e = tid + k * LINES;
      gl[e] = tl[(e / N) * P + (e % N)];
    }
  } else {
    for (int e = tid; e < nl * N; e += LINES) gl[e] = tl[(e / N) * P + (e % N)];
  }
}

// lam_a[s] += scale * sum of dnu over the lines of spatial cell s (a
// contiguous run of `per` line indices), fixed-order tree per workgroup.
__global__ __launch_bounds__(256) void reduce_lines_kernel(double* lam_a, const double* dnu, long long per,
                                                           double scale)
{
  __shared__ double sh[256];
  const long long s = blockIdx.x;
  double acc = 0.0;
  for (long long i = threadIdx.x; i < per; i += 256) acc += dnu[s * per + i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) lam_a[s] += scale * sh[0];
}

// ---- reverse of one half kick in one pass --------------------------------------
// The adjoint of T_vz T_vy T_vx (tau) for velocity blocks of which two copies
// fit the LDS: the block's forward input x and its adjoint lam are staged
// (16-byte loads, storage order, rows padded to N + 1 and planes to
// SX = N (mod 64)); the forward states the reverse sweeps need are rebuilt in
// LDS with the forward line update, and the reverse line updates run in
// place on lam:
//   B = T_vy T_vx x;  lam <- vz reverse at B;
//   B = T_vx x;       lam <- vy reverse at B;
//   B = x;            lam <- vx reverse at B;
// then lam goes back to HBM. x crosses HBM up to three times (the reloads
// mostly hit in L2) and lam twice, against twelve passes for two regenerated
// states and three separate reverse sweeps. Each reverse line runs adj_line
// on the same inputs as the single reverse sweep, and the per-line nu
// adjoints are added per axis in the order of reduce_lines_kernel, so the
// results are those of the separate passes bit for bit.
template <typename T, int N>
struct AdjKickShape {
  static constexpr int SY = N + 1;
  static constexpr int SX0 = N * SY;
  static constexpr int SX = SX0 + ((((N - SX0) % 64) + 64) % 64);
  static constexpr int ELEMS = N * SX;
  static constexpr int LINES = N * N;
  // at least 256 lanes: the reduction below runs the 256-lane tree of reduce_lines_kernel
  static constexpr int THREADS = (LINES + 63) / 64 * 64 > 256 ? (LINES + 63) / 64 * 64 : 256;
  static constexpr int BYTES = 2 * ELEMS * (int)sizeof(T) + 3 * LINES * (int)sizeof(double) + 3 * 256 * (int)sizeof(double);
  static constexpr bool fits = BYTES <= 160 * 1024 && THREADS <= 1024 && N % (16 / (int)sizeof(T)) == 0;
};

template <typename T, int N>
__global__ __launch_bounds__((AdjKickShape<T, N>::THREADS)) void kick_adj_block(KickAdjArgs a)
{
  using S = AdjKickShape<T, N>;
  using VT = typename Vec16<T>::type;
  constexpr int V = Vec16<T>::n;
  constexpr int NVEC = N * N * N / V;
  __shared__ T B[S::ELEMS];
  __shared__ T C[S::ELEMS];
  __shared__ double dn[3][S::LINES];
  __shared__ double sh[3][256];
  const int tid = threadIdx.x;
  const long long s = blockIdx.x;
  const T* xg = static_cast<const T*>(a.fin) + s * (long long)(N * N * N);
  T* lg = static_cast<T*>(a.lam) + s * (long long)(N * N * N);
  const double nux = a.accel[0][s] * a.scale[0], nuy = a.accel[1][s] * a.scale[1], nuz = a.accel[2][s] * a.scale[2];
  auto place = [](int e) {   // storage element e -> LDS index
    const int jz = e % N, jy = (e / N) % N, jx = e / (N * N);
    return jx * S::SX + jy * S::SY + jz;
  };
  // staging: every 16-byte load of a lane is in flight before its first LDS
  // write (a rolled loop would wait out one load latency per vector); the
  // opaque copies of the lane index keep the compiler from holding the
  // addresses of every staging for the whole kernel
  constexpr int PER = (NVEC + S::THREADS - 1) / S::THREADS;
  auto load = [&](VT (&x)[PER], const T* src) {
    int t0 = tid;
    asm volatile("" : "+v"(t0));
#pragma unroll
    for (int j = 0; j < PER; j++) {
      const int k = t0 + j * S::THREADS;
      if (k < NVEC) x[j] = reinterpret_cast<const VT*>(src)[k];
    }
  };
  auto park = [&](T* dst, const VT (&x)[PER]) {
    int t0 = tid;
    asm volatile("" : "+v"(t0));
#pragma unroll
    for (int j = 0; j < PER; j++) {
      const int k = t0 + j * S::THREADS;
      if (k < NVEC) {
        const int b = place(k * V);
#pragma unroll
        for (int q = 0; q < V; q++) dst[b + q] = lane_of<VT, T>(x[j], q);
      }
    }
  };
  auto stage = [&](T* dst, const T* src) {
    VT x[PER];
    load(x, src);
    park(dst, x);
  };
  // forward sweep of B along vx (lanes (jy, jz)) or vy (lanes (jx, jz)), in place
  // the sweep lambdas are inlined at each call, so that their axis, hence
  // every LDS stride, is a constant there (a shared out-of-line body takes the
  // strides at run time and spills across the calls)
  auto forward = [&](int axis, double nu) __attribute__((always_inline)) {
    if (tid < S::LINES) {
      const int o = tid / N, i = tid - o * N;
      const int base = axis == 0 ? o * S::SY + i : o * S::SX + i;
      const int st = axis == 0 ? S::SX : S::SY;
      T v[N];
#pragma unroll
      for (int r = 0; r < N; r++) v[r] = B[base + r * st];
      const LineCoef<T> k = pfc_line<T, N>(v, nu, false);
      store_shifted<T, N>(v, k.shift, false, [&](int r, T x) { B[base + r * st] = x; });
    }
    __syncthreads();
  };
  // reverse sweep along `axis` at forward input B, lam in C, in place
  auto reverse = [&](int axis, double nu) __attribute__((always_inline)) {
    if (tid < S::LINES) {
      const int o = tid / N, i = tid - o * N;
      int base, st;
      if (axis == 2) { base = o * S::SX + i * S::SY; st = 1; }          // vz lines, lanes (jx, jy)
      else if (axis == 1) { base = o * S::SX + i; st = S::SY; }        // vy lines, lanes (jx, jz)
      else { base = o * S::SY + i; st = S::SX; }                      // vx lines, lanes (jy, jz)
      dn[axis][tid] = adj_line<T, N, true>(B, C, nu, false, [&](int r) { return base + r * st; });
    }
    __syncthreads();
  };
  {
    VT x[PER], l[PER];
    load(x, xg);
    load(l, lg);
    park(B, x);
    park(C, l);
  }
  __syncthreads();
  forward(0, nux);
  forward(1, nuy);
  reverse(2, nuz);
  stage(B, xg);
  __syncthreads();
  forward(0, nux);
  reverse(1, nuy);
  stage(B, xg);
  __syncthreads();
  reverse(0, nux);
#pragma unroll
  for (int j = 0; j < PER; j++) {
    const int k = tid + j * S::THREADS;
    if (k < NVEC) {
      const int b = place(k * V);
      VT x;
      T* xs = reinterpret_cast<T*>(&x);
#pragma unroll
      for (int q = 0; q < V; q++) xs[q] = C[b + q];
      reinterpret_cast<VT*>(lg)[k] = x;
    }
  }
  // lam_a[l][s] += scale_l * sum of the block's line adjoints, in the order of
  // reduce_lines_kernel: lane t < 256 adds lines t, t + 256, ..., then a tree
  // (the three axes' trees side by side, with the same pairs as each alone)
  if (!a.lam_a[0]) return;   // uniform: no acceleration adjoint wanted
  if (tid < 256) {
#pragma unroll
    for (int l = 0; l < 3; l++) {
      double acc = 0.0;
      for (int i = tid; i < S::LINES; i += 256) acc += dn[l][i];
      sh[l][tid] = acc;
    }
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
#pragma unroll
      for (int l = 0; l < 3; l++) sh[l][tid] += sh[l][tid + w];
    }
    __syncthreads();
  }
  if (tid < 3) a.lam_a[tid][s] += a.scale[tid] * sh[tid][0];
}

template <typename T, int N>
hipError_t launch_kick_adj_n(const KickAdjArgs& a, hipStream_t s)
{
  using S = AdjKickShape<T, N>;
  static_assert(S::fits, "two velocity blocks do not fit the LDS");
  if (a.np <= 0) return hipSuccess;
  hipLaunchKernelGGL((kick_adj_block<T, N>), dim3((unsigned)a.np), dim3(S::THREADS), 0, s, a);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t launch_adj_n(const SweepArgs& a, const void* fin, void* lam, double* dnu, hipStream_t s)
{
  if (a.nlines <= 0) return hipSuccess;
  if (a.inner == 1) {
    if (a.addend) return hipErrorInvalidValue;
    constexpr int LINES = AdjContig<T, N>::LINES;
    hipLaunchKernelGGL((sweep_adj_contig<T, N>), dim3((unsigned)((a.nlines + LINES - 1) / LINES)), dim3(LINES), 0, s,
                       a, static_cast<const T*>(fin), static_cast<T*>(lam), dnu);
    return hipGetLastError();
  }
  const long long blocks = (a.nlines + 255) / 256;
  if (a.addend) {
    if (!narrow_ok(a, N)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((sweep_adj_kernel<T, N, true, true>), dim3((unsigned)blocks), dim3(256), 0, s, a,
                       static_cast<const T*>(fin), static_cast<T*>(lam), dnu);
  } else if (narrow_ok(a, N))
    hipLaunchKernelGGL((sweep_adj_kernel<T, N, true>), dim3((unsigned)blocks), dim3(256), 0, s, a,
                       static_cast<const T*>(fin), static_cast<T*>(lam), dnu);
  else
    hipLaunchKernelGGL((sweep_adj_kernel<T, N, false>), dim3((unsigned)blocks), dim3(256), 0, s, a,
                       static_cast<const T*>(fin), static_cast<T*>(lam), dnu);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_t(const SweepArgs& a, const void* fin, void* lam, double* dnu, hipStream_t s)
{
  switch (a.n) {
    case 1: return launch_adj_n<T, 1>(a, fin, lam, dnu, s);
    case 2: return launch_adj_n<T, 2>(a, fin, lam, dnu, s);
    case 3: return launch_adj_n<T, 3>(a, fin, lam, dnu, s);
    case 4: return launch_adj_n<T, 4>(a, fin, lam, dnu, s);
    case 6: return launch_adj_n<T, 6>(a, fin, lam, dnu, s);
    case 8: return launch_adj_n<T, 8>(a, fin, lam, dnu, s);
    case 12: return launch_adj_n<T, 12>(a, fin, lam, dnu, s);
    case 16: return launch_adj_n<T, 16>(a, fin, lam, dnu, s);
    case 24: return launch_adj_n<T, 24>(a, fin, lam, dnu, s);
    case 32: return launch_adj_n<T, 32>(a, fin, lam, dnu, s);
    case 48: return launch_adj_n<T, 48>(a, fin, lam, dnu, s);
    case 64: return launch_adj_n<T, 64>(a, fin, lam, dnu, s);
    case 96: return launch_adj_n<T, 96>(a, fin, lam, dnu, s);
    case 128: return launch_adj_n<T, 128>(a, fin, lam, dnu, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool adjoint_addend_supported(const SweepArgs& a)
{
  return a.inner > 1 && a.add_div > 0 && narrow_ok(a, a.n);
}

hipError_t launch_sweep_adjoint(const SweepArgs& a, int dtype, const void* fin, void* lam, double* dnu,
                                hipStream_t s)
{
  return dtype == 0 ? launch_adj_t<float>(a, fin, lam, dnu, s) : launch_adj_t<double>(a, fin, lam, dnu, s);
}

// Cubic velocity blocks of which two copies fit the LDS: FP32 8^3, 16^3,
// 24^3; FP64 8^3 (FP64 16^3 fits too, but its reverse lines need more
// registers than a lane has and spill).
bool kick_adjoint_supported(int dtype, const int nv[3])
{
  if (nv[0] != nv[1] || nv[1] != nv[2]) return false;
  const int n = nv[0];
  return n == 8 || (dtype == 0 && (n == 16 || n == 24));
}

hipError_t launch_kick_adjoint(const KickAdjArgs& a, int dtype, const int nv[3], hipStream_t s)
{
  if (!kick_adjoint_supported(dtype, nv)) return hipErrorInvalidValue;
  if (dtype == 0) {
    switch (nv[0]) {
      case 8: return launch_kick_adj_n<float, 8>(a, s);
      case 16: return launch_kick_adj_n<float, 16>(a, s);
      default: return launch_kick_adj_n<float, 24>(a, s);
    }
  }
  return launch_kick_adj_n<double, 8>(a, s);
}

hipError_t launch_reduce_lines(double* lam_a, const double* dnu, long long np, long long per, double scale,
                               hipStream_t s)
{
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_lines_kernel, dim3((unsigned)np), dim3(256), 0, s, lam_a, dnu, per, scale);
  return hipGetLastError();
}

}  // namespace vp
