// gravity.hip -- density moment, Fourier-convolution Poisson solve, two-point
// acceleration and FP64 reductions (Sec. 2.2 and Eqs. (18)-(25), (29), (30),
// (41) of Yoshikawa, Yoshida & Umemura) for gfx950.
//
// The transforms are done axis by axis: a workgroup takes one or more lines,
// stages them and the twiddle table in LDS and runs a self-sorting mixed-radix FFT
// (radices 4, 2 and 3, which cover every axis length the library accepts and
// its doubling for the isolated solve); lines of up to 32 cells, and any other
// length, take a direct sum.
// The spatial grids of this method are small (at most a few hundred cells per
// axis), so a line fits one workgroup and no FFT library is needed. All of it
// runs in FP64.
#include "vp_internal.h"

namespace vp {
namespace {

constexpr int RED = 256;  // reduction workgroup size

__device__ __forceinline__ double block_sum(double x, double* sh)
{
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int w = RED / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max(double x, double* sh)
{
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int w = RED / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// rho = dv3 * sum over the contiguous velocity block of one spatial cell.
// 16-byte loads, four independent accumulators per lane so that several loads
// are in flight, then a fixed-order tree over the workgroup (deterministic).
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
};
template <>
struct Vec16<double> {
  using type = double2;
};

template <typename T>
__device__ __forceinline__ double vsum(const float4& v) { return ((double)v.x + (double)v.y) + ((double)v.z + (double)v.w); }
template <typename T>
__device__ __forceinline__ double vsum(const double2& v) { return v.x + v.y; }

template <typename T>
__global__ __launch_bounds__(RED) void density_kernel(const T* f, double* rho, long long nv3, double dv3)
{
  __shared__ double sh[RED];
  using VT = typename Vec16<T>::type;
  constexpr int V = 16 / sizeof(T);
  const T* p = f + (long long)blockIdx.x * nv3;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  long long done = 0;
  if ((nv3 % V) == 0 && (reinterpret_cast<uintptr_t>(p) % 16) == 0) {
    const VT* pv = reinterpret_cast<const VT*>(p);
    const long long nvec = nv3 / V;
    long long i = threadIdx.x;
    for (; i + 3 * RED < nvec; i += 4 * RED) {
      const VT a = pv[i], b = pv[i + RED], c = pv[i + 2 * RED], d = pv[i + 3 * RED];
      acc0 += vsum<T>(a);
      acc1 += vsum<T>(b);
      acc2 += vsum<T>(c);
      acc3 += vsum<T>(d);
    }
    for (; i < nvec; i += RED) acc0 += vsum<T>(pv[i]);
    done = nv3;
  }
  for (long long j = done + threadIdx.x; j < nv3; j += RED) acc0 += (double)p[j];
  const double s = block_sum((acc0 + acc1) + (acc2 + acc3), sh);
  if (threadIdx.x == 0) rho[blockIdx.x] = s * dv3;
}

// out[s] = scale * sum_j a[s*nv3 + j] w[j] (FP64, fixed order per cell): one
// workgroup per spatial cell, four accumulators per lane, then a tree.
template <typename T>
__global__ __launch_bounds__(RED) void weighted_moment_kernel(const T* a, const double* w, double* out,
                                                              long long nv3, double scale)
{
  __shared__ double sh[RED];
  const T* p = a + (long long)blockIdx.x * nv3;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  long long j = threadIdx.x;
  for (; j + 3 * RED < nv3; j += 4 * RED) {
    acc0 += (double)p[j] * w[j];
    acc1 += (double)p[j + RED] * w[j + RED];
    acc2 += (double)p[j + 2 * RED] * w[j + 2 * RED];
    acc3 += (double)p[j + 3 * RED] * w[j + 3 * RED];
  }
  for (; j < nv3; j += RED) acc0 += (double)p[j] * w[j];
  const double s = block_sum((acc0 + acc1) + (acc2 + acc3), sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s * scale;
}

// One workgroup per spatial (y, z) column: lane t takes x = t % n and chunk
// group g = t / n (G = 256 / n groups), adds the chunks k = g, g + G, ... in
// order, and the G group sums of each x are then added in order of g. The
// order is fixed, so the result is deterministic.
__global__ __launch_bounds__(256) void density_from_parts_kernel(double* rho, const double* part, long long nyz,
                                                                 long long nchunk, int n, double dv3)
{
  __shared__ double sums[256];
  const long long yz = blockIdx.x;
  const int t = threadIdx.x;
  const int G = 256 / n;
  const int x = t % n, g = t / n;
  double acc = 0.0;
  if (g < G) {
    const double* p = part + yz * nchunk * n + x;
    for (long long k = g; k < nchunk; k += G) acc += p[k * n];
  }
  sums[t] = acc;
  __syncthreads();
  if (t < n) {
    double tot = 0.0;
    for (int q = 0; q < G; q++) tot += sums[q * n + t];
    rho[(long long)t * nyz + yz] = tot * dv3;
  }
}

__global__ void twiddle_kernel(double2* w, int M)
{
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  double sn, cs;
  sincospi(2.0 * (double)k / (double)M, &sn, &cs);
  w[k] = make_double2(cs, -sn);  // exp(-2 pi i k / M)
}

// One workgroup per line of the axis; lanes compute frequencies.
__global__ __launch_bounds__(128) void dft_kernel(double2* data, long long inner, int M, int sign,
                                                   const double2* tw)
{
  extern __shared__ double2 lds[];
  double2* x = lds;       // M values
  double2* w = lds + M;   // M twiddles
  const long long line = blockIdx.x;
  const long long o = line / inner;
  const long long c = line - o * inner;
  double2* p = data + o * (long long)M * inner + c;
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    x[j] = p[(long long)j * inner];
    const double2 t = tw[j];
    w[j] = make_double2(t.x, sign < 0 ? t.y : -t.y);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < M; k += blockDim.x) {
    double sr = 0.0, si = 0.0;
    int idx = 0;  // (j * k) mod M
    for (int j = 0; j < M; j++) {
      const double2 a = x[j];
      const double2 b = w[idx];
      sr += a.x * b.x - a.y * b.y;
      si += a.x * b.y + a.y * b.x;
      idx += k;
      if (idx >= M) idx -= M;
    }
    p[(long long)k * inner] = make_double2(sr, si);
  }
}

// Radices of the mixed-radix transform: fours, then a two, then threes (every
// axis length this library accepts, and its doubling, factors so).
struct FftPlan {
  int n;
  int r[24];
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// u / d for 0 <= u < 2^24 and d >= 1 through a float reciprocal, corrected to
// the exact quotient (integer division has no instruction of its own)
__device__ __forceinline__ int div_small(int u, int d, float inv)
{
  int q = (int)((float)u * inv);
  q += ((q + 1) * d <= u) ? 1 : 0;
  q -= (q * d > u) ? 1 : 0;
  return q;
}

// A self-sorting (Stockham) mixed-radix FFT of L = 2^lgL lines of the axis
// per workgroup, in LDS with the lines interleaved (element x of line l at
// x L + l, so lanes with adjacent l touch adjacent banks, and adjacent lines,
// adjacent in HBM for every axis but the last, load together). A stage of
// radix R with Ns = product of the earlier radices takes, for t < M/R and
// k = t mod Ns, the R values t + r M/R, turns them by w^(r k M/(Ns R)),
// transforms them with the R-point DFT and writes output q to
// (t / Ns) Ns R + k + q Ns. The twiddle table w is the M-th roots of unity,
// conjugated for the inverse direction; every index into it is below M. Same
// result as the direct sum up to rounding (O(log M) eps).
__global__ __launch_bounds__(64) void fft_kernel(double2* data, long long inner, long long lines, int M, int lgL,
                                                  int sign, const double2* tw, FftPlan plan)
{
  extern __shared__ double2 lds[];
  const int L = 1 << lgL;
  double2* a = lds;
  double2* b = lds + M * L;
  double2* w = lds + 2 * M * L;
  long long* lbase = reinterpret_cast<long long*>(lds + 2 * M * L + M);   // L line offsets
  const long long first = (long long)blockIdx.x * L;
  for (int l = threadIdx.x; l < L; l += blockDim.x) {
    const long long line = first + l, o = line / inner, c = line - o * inner;
    lbase[l] = o * (long long)M * inner + c;
  }
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    const double2 t = tw[j];
    w[j] = make_double2(t.x, sign < 0 ? t.y : -t.y);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < M * L; e += blockDim.x) {
    const int l = e & (L - 1), j = e >> lgL;
    if (first + l < lines) a[e] = data[lbase[l] + (long long)j * inner];
  }
  __syncthreads();
  int ns = 1;
  for (int st = 0; st < plan.n; st++) {
    const int R = plan.r[st], step = M / R, tws = M / (ns * R);
    const float inv = 1.0f / (float)ns;
    for (int u = threadIdx.x; u < step * L; u += blockDim.x) {
      const int l = u & (L - 1), t = u >> lgL;
      const int tq = div_small(t, ns, inv), k = t - tq * ns;
      double2 v[4];
#pragma unroll
      for (int r = 0; r < 4; r++)
        if (r < R) v[r] = cmul(a[(t + r * step) * L + l], w[r * k * tws]);
      const int base = tq * ns * R + k;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        if (q >= R) break;
        double2 y = v[0];
#pragma unroll
        for (int r = 1; r < 4; r++)
          if (r < R) {
            // (q r) mod R for q, r < R <= 4: q r < 3R
            const int qr = q * r, m = qr - (qr >= R ? R : 0) - (qr >= 2 * R ? R : 0);
            const double2 z = cmul(v[r], w[m * step]);
            y.x += z.x;
            y.y += z.y;
          }
        b[(base + q * ns) * L + l] = y;
      }
    }
    __syncthreads();
    double2* x = a;
    a = b;
    b = x;
    ns *= R;
  }
  for (int e = threadIdx.x; e < M * L; e += blockDim.x) {
    const int l = e & (L - 1), j = e >> lgL;
    if (first + l < lines) data[lbase[l] + (long long)j * inner] = a[e];
  }
}

__global__ void load_rho_kernel(double2* data, Grid3 g, const double* rho, Grid3 n)
{
  const long long tot = (long long)g.m[0] * g.m[1] * g.m[2];
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < tot;
       s += (long long)gridDim.x * blockDim.x) {
    const int i2 = (int)(s % g.m[2]);
    const int i1 = (int)((s / g.m[2]) % g.m[1]);
    const int i0 = (int)(s / ((long long)g.m[2] * g.m[1]));
    double v = 0.0;
    if (i0 < n.m[0] && i1 < n.m[1] && i2 < n.m[2]) v = rho[((long long)i0 * n.m[1] + i1) * n.m[2] + i2];
    data[s] = make_double2(v, 0.0);
  }
}

// G_hat(k) = -pi G / sum_l sin^2(pi k_l / M_l) / d_l^2 (Eq. (20), unequal
// spacings), zero at k = 0.
__global__ void green_periodic_kernel(double2* data, Grid3 g, double G, double d0, double d1, double d2)
{
  const long long tot = (long long)g.m[0] * g.m[1] * g.m[2];
  const double pi = 3.14159265358979323846;
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < tot;
       s += (long long)gridDim.x * blockDim.x) {
    const int k2 = (int)(s % g.m[2]);
    const int k1 = (int)((s / g.m[2]) % g.m[1]);
    const int k0 = (int)(s / ((long long)g.m[2] * g.m[1]));
    const double s0 = sinpi((double)k0 / g.m[0]);
    const double s1 = sinpi((double)k1 / g.m[1]);
    const double s2 = sinpi((double)k2 / g.m[2]);
    const double den = s0 * s0 / (d0 * d0) + s1 * s1 / (d1 * d1) + s2 * s2 / (d2 * d2);
    const double gk = (k0 == 0 && k1 == 0 && k2 == 0) ? 0.0 : -pi * G / den;
    const double2 v = data[s];
    data[s] = make_double2(v.x * gk, v.y * gk);
  }
}

__global__ void mul_spectrum_kernel(double2* data, const double2* spec, long long count)
{
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < count;
       s += (long long)gridDim.x * blockDim.x) {
    const double2 a = data[s], b = spec[s];
    data[s] = make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
  }
}

// Isolated Green's function of the doubled grid: K(r) = -G d0 d1 d2 / |r| at
// the mirrored offset, self_value at the origin.
__global__ void green_isolated_kernel(double2* data, Grid3 g, double G, double d0, double d1, double d2,
                                      double self_value)
{
  const long long tot = (long long)g.m[0] * g.m[1] * g.m[2];
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < tot;
       s += (long long)gridDim.x * blockDim.x) {
    int o2 = (int)(s % g.m[2]);
    int o1 = (int)((s / g.m[2]) % g.m[1]);
    int o0 = (int)(s / ((long long)g.m[2] * g.m[1]));
    o0 = min(o0, g.m[0] - o0);
    o1 = min(o1, g.m[1] - o1);
    o2 = min(o2, g.m[2] - o2);
    double v;
    if (o0 == 0 && o1 == 0 && o2 == 0) {
      v = self_value;
    } else {
      const double x = o0 * d0, y = o1 * d1, z = o2 * d2;
      v = -G * d0 * d1 * d2 / sqrt(x * x + y * y + z * z);
    }
    data[s] = make_double2(v, 0.0);
  }
}

__global__ void extract_phi_kernel(double* phi, Grid3 n, const double2* data, Grid3 g, double scale)
{
  const int e0 = n.m[0] + 2, e1 = n.m[1] + 2, e2 = n.m[2] + 2;
  const long long tot = (long long)e0 * e1 * e2;
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < tot;
       s += (long long)gridDim.x * blockDim.x) {
    const int t2 = (int)(s % e2) - 1;
    const int t1 = (int)((s / e2) % e1) - 1;
    const int t0 = (int)(s / ((long long)e2 * e1)) - 1;
    const int w0 = (t0 + g.m[0]) % g.m[0];
    const int w1 = (t1 + g.m[1]) % g.m[1];
    const int w2 = (t2 + g.m[2]) % g.m[2];
    phi[s] = data[((long long)w0 * g.m[1] + w1) * g.m[2] + w2].x * scale;
  }
}

__global__ void gradient_kernel(double* a, const double* phi, Grid3 n, double d0, double d1, double d2)
{
  const long long np = (long long)n.m[0] * n.m[1] * n.m[2];
  const long long e1 = n.m[1] + 2, e2 = n.m[2] + 2;
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < np;
       s += (long long)gridDim.x * blockDim.x) {
    const long long i2 = s % n.m[2];
    const long long i1 = (s / n.m[2]) % n.m[1];
    const long long i0 = s / ((long long)n.m[2] * n.m[1]);
    const long long c = ((i0 + 1) * e1 + (i1 + 1)) * e2 + (i2 + 1);
    a[s] = -(phi[c + e1 * e2] - phi[c - e1 * e2]) / (2.0 * d0);
    a[np + s] = -(phi[c + e2] - phi[c - e2]) / (2.0 * d1);
    a[2 * np + s] = -(phi[c + 1] - phi[c - 1]) / (2.0 * d2);
  }
}

// Cell counters (i0, i1, i2) of a row-major box m0 x m1 x m2, advanced by a
// fixed stride without integer division. The stride is split once into its
// own counters, whose i2 part is below m2 and i1 part below m1, so each step
// carries at most once per axis. Counters past the end of the box are never
// read.
struct Idx3 {
  int i0, i1, i2;
  static __device__ __forceinline__ Idx3 split(long long e, int m1, int m2)
  {
    Idx3 c;
    c.i2 = (int)(e % m2);
    const long long r = e / m2;
    c.i1 = (int)(r % m1);
    c.i0 = (int)(r / m1);
    return c;
  }
  __device__ __forceinline__ void step(const Idx3& d, int m1, int m2)
  {
    i2 += d.i2;
    if (i2 >= m2) {
      i2 -= m2;
      ++i1;
    }
    i1 += d.i1;
    if (i1 >= m1) {
      i1 -= m1;
      ++i0;
    }
    i0 += d.i0;
  }
};

template <typename T, int V>
struct alignas(sizeof(T) * V) Pack {
  T v[V];
};

// Per spatial cell: sum_j f_j and sum_j f_j |v_j|^2 over its velocity block
// (Eqs. (29), (30) before the dx^3 dv^3 factor). A lane loads V consecutive
// cells of one vz-line at a time (16 bytes when nv_z is a multiple of V, else
// V = 1), four loads in flight, and walks the velocity indices with Idx3.
template <typename T, int V>
__global__ __launch_bounds__(RED) void energy_partial_kernel(const T* f, double* part, VelGrid vg)
{
  __shared__ double sh[RED];
  const int ny = vg.nv[1], nz = vg.nv[2];
  const long long nv3 = (long long)vg.nv[0] * ny * nz;
  const long long ngrp = nv3 / V;
  const Pack<T, V>* p = reinterpret_cast<const Pack<T, V>*>(f + (long long)blockIdx.x * nv3);
  Idx3 c = Idx3::split((long long)threadIdx.x * V, ny, nz);
  const Idx3 d = Idx3::split((long long)RED * V, ny, nz);
  double m[4] = {0.0, 0.0, 0.0, 0.0}, k[4] = {0.0, 0.0, 0.0, 0.0};
  auto add = [&](const Pack<T, V>& q, int a) {
    const double vx = vg.vmin[0] + (c.i0 + 0.5) * vg.dv[0];
    const double vy = vg.vmin[1] + (c.i1 + 0.5) * vg.dv[1];
    const double wxy = vx * vx + vy * vy;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const double vz = vg.vmin[2] + (c.i2 + e + 0.5) * vg.dv[2];
      const double x = (double)q.v[e];
      m[a] += x;
      k[a] += x * (wxy + vz * vz);
    }
    c.step(d, ny, nz);
  };
  long long g = threadIdx.x;
  for (; g + 3 * RED < ngrp; g += 4 * RED) {
    const Pack<T, V> q0 = p[g], q1 = p[g + RED], q2 = p[g + 2 * RED], q3 = p[g + 3 * RED];
    add(q0, 0);
    add(q1, 1);
    add(q2, 2);
    add(q3, 3);
  }
  for (; g < ngrp; g += RED) add(p[g], 0);
  const double ms = block_sum((m[0] + m[1]) + (m[2] + m[3]), sh);
  const double ks = block_sum((k[0] + k[1]) + (k[2] + k[3]), sh);
  if (threadIdx.x == 0) {
    part[2 * (long long)blockIdx.x] = ms;
    part[2 * (long long)blockIdx.x + 1] = ks;
  }
}

// Whole-grid reductions in two stages: REDUCE_BLOCKS workgroups (fewer for a
// small grid) each reduce a fixed grid-stride share of the spatial cells into
// out[RED_PART + ...], then one workgroup combines the partials in order. The
// grid size depends only on the cell count, so the sums are deterministic.
__host__ __device__ constexpr int reduce_blocks(long long np)
{
  return (int)(np / RED + 1 < REDUCE_BLOCKS ? np / RED + 1 : REDUCE_BLOCKS);
}

// stage 1 of vp_energy: per workgroup sums of M, K (from the per-cell
// partials) and of rho phi over its cells
__global__ __launch_bounds__(RED) void energy_stage_kernel(double* out, const double* part, const double* rho,
                                                           const double* phi, Grid3 n)
{
  __shared__ double sh[RED];
  const long long np = (long long)n.m[0] * n.m[1] * n.m[2];
  const long long e1 = n.m[1] + 2, e2 = n.m[2] + 2;
  const long long s0 = (long long)blockIdx.x * RED + threadIdx.x, st = (long long)gridDim.x * RED;
  Idx3 c = Idx3::split(s0, n.m[1], n.m[2]);
  const Idx3 d = Idx3::split(st, n.m[1], n.m[2]);
  double m = 0.0, k = 0.0, u = 0.0;
  for (long long s = s0; s < np; s += st) {
    m += part[2 * s];
    k += part[2 * s + 1];
    u += rho[s] * phi[((c.i0 + 1) * e1 + (c.i1 + 1)) * e2 + (c.i2 + 1)];
    c.step(d, n.m[1], n.m[2]);
  }
  const double ms = block_sum(m, sh);
  const double ks = block_sum(k, sh);
  const double us = block_sum(u, sh);
  if (threadIdx.x == 0) {
    double* o = out + RED_PART + 3 * (long long)blockIdx.x;
    o[0] = ms;
    o[1] = ks;
    o[2] = us;
  }
}

__global__ __launch_bounds__(RED) void energy_final_kernel(double* out, int nb, double dx3, double dv3)
{
  __shared__ double sh[RED];
  double m = 0.0, k = 0.0, u = 0.0;
  for (int b = threadIdx.x; b < nb; b += RED) {
    const double* o = out + RED_PART + 3 * (long long)b;
    m += o[0];
    k += o[1];
    u += o[2];
  }
  const double ms = block_sum(m, sh);
  const double ks = block_sum(k, sh);
  const double us = block_sum(u, sh);
  if (threadIdx.x == 0) {
    const double K = 0.5 * ks * dx3 * dv3;
    const double U = 0.5 * us * dx3;
    out[0] = K;
    out[1] = U;
    out[2] = ms * dx3 * dv3;
    out[3] = K + U;
  }
}

__global__ __launch_bounds__(RED) void accel_max_stage_kernel(double* out, const double* a, long long np, double i0,
                                                              double i1, double i2)
{
  __shared__ double sh[RED];
  double m = 0.0;
  for (long long s = (long long)blockIdx.x * RED + threadIdx.x; s < np; s += (long long)gridDim.x * RED) {
    m = fmax(m, fabs(a[s]) * i0);
    m = fmax(m, fabs(a[np + s]) * i1);
    m = fmax(m, fabs(a[2 * np + s]) * i2);
  }
  const double r = block_max(m, sh);
  if (threadIdx.x == 0) out[RED_PART + blockIdx.x] = r;
}

__global__ __launch_bounds__(RED) void max_final_kernel(double* out, int nb)
{
  __shared__ double sh[RED];
  double m = 0.0;
  for (int b = threadIdx.x; b < nb; b += RED) m = fmax(m, out[RED_PART + b]);
  const double r = block_max(m, sh);
  if (threadIdx.x == 0) out[0] = r;
}

// ---- transposes for the reverse mode ---------------------------------------

// lam_phi(t), t in -1..N per axis, of a_l(i) = -(phi(i+e_l) - phi(i-e_l)) / (2 d_l):
// lam_phi(t) = sum_l (lam_a_l(t+e_l) - lam_a_l(t-e_l)) / (2 d_l), lam_a zero outside.
__global__ void gradient_adj_kernel(double* lphi, const double* la, Grid3 n, double d0, double d1, double d2)
{
  const int e0 = n.m[0] + 2, e1 = n.m[1] + 2, e2 = n.m[2] + 2;
  const long long tot = (long long)e0 * e1 * e2;
  const long long np = (long long)n.m[0] * n.m[1] * n.m[2];
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < tot;
       s += (long long)gridDim.x * blockDim.x) {
    const int t2 = (int)(s % e2) - 1;
    const int t1 = (int)((s / e2) % e1) - 1;
    const int t0 = (int)(s / ((long long)e2 * e1)) - 1;
    auto A = [&](int l, int i0, int i1, int i2) -> double {
      if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= n.m[0] || i1 >= n.m[1] || i2 >= n.m[2]) return 0.0;
      return la[(long long)l * np + ((long long)i0 * n.m[1] + i1) * n.m[2] + i2];
    };
    double v = (A(0, t0 + 1, t1, t2) - A(0, t0 - 1, t1, t2)) / (2.0 * d0);
    v += (A(1, t0, t1 + 1, t2) - A(1, t0, t1 - 1, t2)) / (2.0 * d1);
    v += (A(2, t0, t1, t2 + 1) - A(2, t0, t1, t2 - 1)) / (2.0 * d2);
    lphi[s] = v;
  }
}

// Transposed ghost fill of the periodic potential: out(i) = sum of lam_phi(t)
// over the cells t in -1..N that are periodic images of i.
__global__ void fold_periodic_kernel(double* out, const double* lphi, Grid3 n)
{
  const long long np = (long long)n.m[0] * n.m[1] * n.m[2];
  const long long e1 = n.m[1] + 2, e2 = n.m[2] + 2;
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < np;
       s += (long long)gridDim.x * blockDim.x) {
    const int i2 = (int)(s % n.m[2]);
    const int i1 = (int)((s / n.m[2]) % n.m[1]);
    const int i0 = (int)(s / ((long long)n.m[2] * n.m[1]));
    int t[3][3], c[3];
    const int ii[3] = {i0, i1, i2};
    for (int l = 0; l < 3; l++) {
      c[l] = 0;
      t[l][c[l]++] = ii[l];
      if (ii[l] == n.m[l] - 1) t[l][c[l]++] = -1;
      if (ii[l] == 0) t[l][c[l]++] = n.m[l];
    }
    double acc = 0.0;
    for (int a = 0; a < c[0]; a++)
      for (int b = 0; b < c[1]; b++)
        for (int d = 0; d < c[2]; d++)
          acc += lphi[((long long)(t[0][a] + 1) * e1 + (t[1][b] + 1)) * e2 + (t[2][d] + 1)];
    out[s] = acc;
  }
}

// Place lam_phi(t), t in -1..N per axis, on the doubled grid at t mod 2N
// (summing where two targets share a position, which happens only for N = 1).
__global__ void load_ext_kernel(double2* data, Grid3 g, const double* lphi, Grid3 n)
{
  const long long tot = (long long)g.m[0] * g.m[1] * g.m[2];
  const long long e1 = n.m[1] + 2, e2 = n.m[2] + 2;
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < tot;
       s += (long long)gridDim.x * blockDim.x) {
    const int p2 = (int)(s % g.m[2]);
    const int p1 = (int)((s / g.m[2]) % g.m[1]);
    const int p0 = (int)(s / ((long long)g.m[2] * g.m[1]));
    const int pp[3] = {p0, p1, p2};
    int t[3][2], c[3];
    for (int l = 0; l < 3; l++) {
      c[l] = 0;
      if (pp[l] <= n.m[l]) t[l][c[l]++] = pp[l];
      if (pp[l] == g.m[l] - 1) t[l][c[l]++] = -1;
    }
    double acc = 0.0;
    for (int a = 0; a < c[0]; a++)
      for (int b = 0; b < c[1]; b++)
        for (int d = 0; d < c[2]; d++)
          acc += lphi[((long long)(t[0][a] + 1) * e1 + (t[1][b] + 1)) * e2 + (t[2][d] + 1)];
    data[s] = make_double2(acc, 0.0);
  }
}

// out(i) = scale * Re data(i) for the cells i of the n-grid inside the g-grid
__global__ void extract_interior_kernel(double* out, const double2* data, Grid3 g, Grid3 n, double scale)
{
  const long long np = (long long)n.m[0] * n.m[1] * n.m[2];
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < np;
       s += (long long)gridDim.x * blockDim.x) {
    const int i2 = (int)(s % n.m[2]);
    const int i1 = (int)((s / n.m[2]) % n.m[1]);
    const int i0 = (int)(s / ((long long)n.m[2] * n.m[1]));
    out[s] = data[((long long)i0 * g.m[1] + i1) * g.m[2] + i2].x * scale;
  }
}

// lam[s, j] += coef * x[s] (broadcast over the velocity block)
template <typename T>
__global__ void broadcast_add_kernel(T* lam, const double* x, long long np, long long nv3, double coef)
{
  const long long tot = np * nv3;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x)
    lam[e] = (T)((double)lam[e] + coef * x[e / nv3]);
}

// lam[s, j] = coef * phi(interior cell s)
template <typename T>
__global__ void seed_kernel(T* lam, const double* phi, Grid3 n, long long nv3, double coef)
{
  const long long np = (long long)n.m[0] * n.m[1] * n.m[2];
  const long long e1 = n.m[1] + 2, e2 = n.m[2] + 2;
  const long long tot = np * nv3;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const long long s = e / nv3;
    const long long i2 = s % n.m[2];
    const long long i1 = (s / n.m[2]) % n.m[1];
    const long long i0 = s / ((long long)n.m[2] * n.m[1]);
    lam[e] = (T)(coef * phi[((i0 + 1) * e1 + (i1 + 1)) * e2 + (i2 + 1)]);
  }
}

// out[0] = 1/2 sum rho phi dx3 (the potential energy, fixed order)
__global__ __launch_bounds__(RED) void potential_stage_kernel(double* out, const double* rho, const double* phi,
                                                              Grid3 n)
{
  __shared__ double sh[RED];
  const long long np = (long long)n.m[0] * n.m[1] * n.m[2];
  const long long e1 = n.m[1] + 2, e2 = n.m[2] + 2;
  const long long s0 = (long long)blockIdx.x * RED + threadIdx.x, st = (long long)gridDim.x * RED;
  Idx3 c = Idx3::split(s0, n.m[1], n.m[2]);
  const Idx3 d = Idx3::split(st, n.m[1], n.m[2]);
  double u = 0.0;
  for (long long s = s0; s < np; s += st) {
    u += rho[s] * phi[((c.i0 + 1) * e1 + (c.i1 + 1)) * e2 + (c.i2 + 1)];
    c.step(d, n.m[1], n.m[2]);
  }
  const double us = block_sum(u, sh);
  if (threadIdx.x == 0) out[RED_PART + blockIdx.x] = us;
}

__global__ __launch_bounds__(RED) void sum_final_kernel(double* out, int nb, double scale)
{
  __shared__ double sh[RED];
  double u = 0.0;
  for (int b = threadIdx.x; b < nb; b += RED) u += out[RED_PART + b];
  const double us = block_sum(u, sh);
  if (threadIdx.x == 0) out[0] = scale * us;
}

unsigned grid_for(long long n, int block)
{
  long long b = (n + block - 1) / block;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_gradient_adj(double* lphi, const double* la, Grid3 n, double d0, double d1, double d2,
                               hipStream_t s)
{
  const long long tot = (long long)(n.m[0] + 2) * (n.m[1] + 2) * (n.m[2] + 2);
  hipLaunchKernelGGL(gradient_adj_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, s, lphi, la, n, d0, d1, d2);
  return hipGetLastError();
}

hipError_t launch_fold_periodic(double* out, const double* lphi, Grid3 n, hipStream_t s)
{
  const long long np = (long long)n.m[0] * n.m[1] * n.m[2];
  hipLaunchKernelGGL(fold_periodic_kernel, dim3(grid_for(np, 256)), dim3(256), 0, s, out, lphi, n);
  return hipGetLastError();
}

hipError_t launch_load_ext(double2* data, Grid3 g, const double* lphi, Grid3 n, hipStream_t s)
{
  const long long tot = (long long)g.m[0] * g.m[1] * g.m[2];
  hipLaunchKernelGGL(load_ext_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, s, data, g, lphi, n);
  return hipGetLastError();
}

hipError_t launch_extract_interior(double* out, const double2* data, Grid3 g, Grid3 n, double scale, hipStream_t s)
{
  const long long np = (long long)n.m[0] * n.m[1] * n.m[2];
  hipLaunchKernelGGL(extract_interior_kernel, dim3(grid_for(np, 256)), dim3(256), 0, s, out, data, g, n, scale);
  return hipGetLastError();
}

hipError_t launch_broadcast_add(void* lam, int dtype, const double* x, long long np, long long nv3, double coef,
                                hipStream_t s)
{
  const long long tot = np * nv3;
  if (dtype == 0)
    hipLaunchKernelGGL(broadcast_add_kernel<float>, dim3(grid_for(tot, 256)), dim3(256), 0, s, (float*)lam, x, np,
                       nv3, coef);
  else
    hipLaunchKernelGGL(broadcast_add_kernel<double>, dim3(grid_for(tot, 256)), dim3(256), 0, s, (double*)lam, x,
                       np, nv3, coef);
  return hipGetLastError();
}

hipError_t launch_seed(void* lam, int dtype, const double* phi_ext, Grid3 n, long long nv3, double coef,
                       hipStream_t s)
{
  const long long tot = (long long)n.m[0] * n.m[1] * n.m[2] * nv3;
  if (dtype == 0)
    hipLaunchKernelGGL(seed_kernel<float>, dim3(grid_for(tot, 256)), dim3(256), 0, s, (float*)lam, phi_ext, n, nv3,
                       coef);
  else
    hipLaunchKernelGGL(seed_kernel<double>, dim3(grid_for(tot, 256)), dim3(256), 0, s, (double*)lam, phi_ext, n,
                       nv3, coef);
  return hipGetLastError();
}

hipError_t launch_potential_energy(double* out, const double* rho, const double* phi_ext, Grid3 n, double dx3,
                                   hipStream_t s)
{
  const int nb = reduce_blocks((long long)n.m[0] * n.m[1] * n.m[2]);
  hipLaunchKernelGGL(potential_stage_kernel, dim3(nb), dim3(RED), 0, s, out, rho, phi_ext, n);
  hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(RED), 0, s, out, nb, 0.5 * dx3);
  return hipGetLastError();
}

hipError_t launch_density(const void* f, int dtype, double* rho, long long np, long long nv3, double dv3,
                          hipStream_t s)
{
  if (dtype == 0)
    hipLaunchKernelGGL(density_kernel<float>, dim3((unsigned)np), dim3(RED), 0, s, (const float*)f, rho, nv3, dv3);
  else
    hipLaunchKernelGGL(density_kernel<double>, dim3((unsigned)np), dim3(RED), 0, s, (const double*)f, rho, nv3, dv3);
  return hipGetLastError();
}

// dst = src, one 16-byte vector per lane per round: the plain read-and-write
// stream that the sweep passes are measured against. A dispatch holds under
// 2^32 work-items, so the grid is capped and larger copies loop.
__global__ __launch_bounds__(256) void copy16_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     long long n)
{
  const long long stride = (long long)gridDim.x * 256;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_copy16(const void* src, void* dst, long long n16, hipStream_t s)
{
  if (n16 <= 0) return hipSuccess;
  const long long blocks = (n16 + 255) / 256;
  const unsigned grid = (unsigned)(blocks < (1LL << 20) ? blocks : (1LL << 20));
  hipLaunchKernelGGL(copy16_kernel, dim3(grid), dim3(256), 0, s, static_cast<const float4*>(src),
                     static_cast<float4*>(dst), n16);
  return hipGetLastError();
}

hipError_t launch_weighted_moment(const void* a, int dtype, const double* w, double* out, long long np,
                                  long long nv3, double scale, hipStream_t s)
{
  if (np <= 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(weighted_moment_kernel<float>, dim3((unsigned)np), dim3(RED), 0, s, (const float*)a, w, out,
                       nv3, scale);
  else
    hipLaunchKernelGGL(weighted_moment_kernel<double>, dim3((unsigned)np), dim3(RED), 0, s, (const double*)a, w,
                       out, nv3, scale);
  return hipGetLastError();
}

hipError_t launch_density_from_parts(double* rho, const double* part, long long nyz, long long nchunk, int n,
                                     double dv3, hipStream_t s)
{
  const long long cells = nyz * n;
  if (cells <= 0) return hipSuccess;
  hipLaunchKernelGGL(density_from_parts_kernel, dim3((unsigned)nyz), dim3(256), 0, s, rho, part, nyz, nchunk, n,
                     dv3);
  return hipGetLastError();
}

hipError_t launch_twiddles(double2* w, int M, hipStream_t s)
{
  hipLaunchKernelGGL(twiddle_kernel, dim3((M + 127) / 128), dim3(128), 0, s, w, M);
  return hipGetLastError();
}

// The transform of every line along one axis: the mixed-radix FFT for lines
// longer than 32 cells whose length factors into 4s, 2s and 3s (all lengths
// this library accepts, and their doubling), else the direct sum. Up to 32
// cells the direct sum, with one lane per output and a single barrier, is the
// faster of the two (32 cells: 4.8 against 7.1 us per axis of 32^3).
hipError_t launch_dft_axis(double2* data, Grid3 g, int axis, int sign, const double2* tw, hipStream_t s)
{
  long long inner = 1;
  for (int q = 2; q > axis; q--) inner *= g.m[q];
  const long long tot = (long long)g.m[0] * g.m[1] * g.m[2];
  const int M = g.m[axis];
  const long long lines = tot / M;
  if (M == 1) return hipSuccess;
  FftPlan plan{};
  int m = M;
  while (m % 4 == 0 && plan.n < 24) {
    plan.r[plan.n++] = 4;
    m /= 4;
  }
  while (m % 2 == 0 && plan.n < 24) {
    plan.r[plan.n++] = 2;
    m /= 2;
  }
  while (m % 3 == 0 && plan.n < 24) {
    plan.r[plan.n++] = 3;
    m /= 3;
  }
  if (m == 1 && M > 32) {
    // lines per workgroup: a power of two, at most 512 / M values' worth, and
    // few enough that the grid keeps about 512 workgroups
    int lgL = 0;
    while ((2LL << lgL) * M <= 512 && (lines >> (lgL + 1)) >= 512) lgL++;
    const int L = 1 << lgL;
    const size_t lds = (2 * (size_t)M * L + M) * sizeof(double2) + (size_t)L * sizeof(long long);
    hipLaunchKernelGGL(fft_kernel, dim3((unsigned)((lines + L - 1) / L)), dim3(64), lds, s, data, inner, lines, M,
                       lgL, sign, tw, plan);
  } else {
    const size_t lds = 2 * (size_t)M * sizeof(double2);
    hipLaunchKernelGGL(dft_kernel, dim3((unsigned)lines), dim3(128), lds, s, data, inner, M, sign, tw);
  }
  return hipGetLastError();
}

hipError_t launch_load_rho(double2* data, Grid3 g, const double* rho, Grid3 n, hipStream_t s)
{
  const long long tot = (long long)g.m[0] * g.m[1] * g.m[2];
  hipLaunchKernelGGL(load_rho_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, s, data, g, rho, n);
  return hipGetLastError();
}

hipError_t launch_green_periodic(double2* data, Grid3 g, double G, double d0, double d1, double d2, hipStream_t s)
{
  const long long tot = (long long)g.m[0] * g.m[1] * g.m[2];
  hipLaunchKernelGGL(green_periodic_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, s, data, g, G, d0, d1, d2);
  return hipGetLastError();
}

hipError_t launch_mul_spectrum(double2* data, const double2* spec, long long count, hipStream_t s)
{
  hipLaunchKernelGGL(mul_spectrum_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, data, spec, count);
  return hipGetLastError();
}

hipError_t launch_green_isolated(double2* data, Grid3 g, double G, double d0, double d1, double d2,
                                 double self_value, hipStream_t s)
{
  const long long tot = (long long)g.m[0] * g.m[1] * g.m[2];
  hipLaunchKernelGGL(green_isolated_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, s, data, g, G, d0, d1, d2,
                     self_value);
  return hipGetLastError();
}

hipError_t launch_extract_phi(double* phi_ext, Grid3 n, const double2* data, Grid3 g, double scale, hipStream_t s)
{
  const long long tot = (long long)(n.m[0] + 2) * (n.m[1] + 2) * (n.m[2] + 2);
  hipLaunchKernelGGL(extract_phi_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, s, phi_ext, n, data, g, scale);
  return hipGetLastError();
}

hipError_t launch_gradient(double* accel, const double* phi_ext, Grid3 n, double d0, double d1, double d2,
                           hipStream_t s)
{
  const long long np = (long long)n.m[0] * n.m[1] * n.m[2];
  hipLaunchKernelGGL(gradient_kernel, dim3(grid_for(np, 256)), dim3(256), 0, s, accel, phi_ext, n, d0, d1, d2);
  return hipGetLastError();
}

hipError_t launch_energy_partials(const void* f, int dtype, double* part, long long np, VelGrid vg, hipStream_t s)
{
  // 16-byte groups need whole groups per vz-line and a 16-byte aligned base
  // (every block then starts aligned, its length being a multiple of V).
  const bool a16 = (reinterpret_cast<uintptr_t>(f) % 16) == 0;
  if (dtype == 0) {
    if (a16 && vg.nv[2] % 4 == 0)
      hipLaunchKernelGGL((energy_partial_kernel<float, 4>), dim3((unsigned)np), dim3(RED), 0, s,
                         static_cast<const float*>(f), part, vg);
    else
      hipLaunchKernelGGL((energy_partial_kernel<float, 1>), dim3((unsigned)np), dim3(RED), 0, s,
                         static_cast<const float*>(f), part, vg);
  } else {
    if (a16 && vg.nv[2] % 2 == 0)
      hipLaunchKernelGGL((energy_partial_kernel<double, 2>), dim3((unsigned)np), dim3(RED), 0, s,
                         static_cast<const double*>(f), part, vg);
    else
      hipLaunchKernelGGL((energy_partial_kernel<double, 1>), dim3((unsigned)np), dim3(RED), 0, s,
                         static_cast<const double*>(f), part, vg);
  }
  return hipGetLastError();
}

hipError_t launch_energy_final(double* out, const double* part, const double* rho, const double* phi_ext, Grid3 n,
                               double dx3, double dv3, hipStream_t s)
{
  const int nb = reduce_blocks((long long)n.m[0] * n.m[1] * n.m[2]);
  hipLaunchKernelGGL(energy_stage_kernel, dim3(nb), dim3(RED), 0, s, out, part, rho, phi_ext, n);
  hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(RED), 0, s, out, nb, dx3, dv3);
  return hipGetLastError();
}

hipError_t launch_accel_max(double* out, const double* accel, long long np, double i0, double i1, double i2,
                            hipStream_t s)
{
  const int nb = reduce_blocks(np);
  hipLaunchKernelGGL(accel_max_stage_kernel, dim3(nb), dim3(RED), 0, s, out, accel, np, i0, i1, i2);
  hipLaunchKernelGGL(max_final_kernel, dim3(1), dim3(RED), 0, s, out, nb);
  return hipGetLastError();
}

}  // namespace vp
