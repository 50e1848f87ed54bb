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
#include "vp_internal.h"

namespace vp {
namespace {

template <typename T, int N, bool REV>
__device__ __forceinline__ T pfc_core_adj(const T (&v)[N], T (&lam)[N], T alpha, T c1, T c2, T dc1, T dc2,
                                          bool periodic)
{
#pragma clang fp contract(off)
#define AT(a, i) a[REV ? (N - 1 - (i)) : (i)]
  T finf = T(0);
  int am = -1;
#pragma unroll
  for (int i = 0; i < N; i++)
    if (v[i] > finf) {
      finf = v[i];
      am = i;
    }
  const T twoinf = finf + finf;
  T lg[N];
#pragma unroll
  for (int i = 0; i < N; i++) lg[i] = lam[i];
  T lfinf = T(0);
  T lalpha = T(0);
  T dm = periodic ? AT(v, 0) - AT(v, N - 1) : AT(v, 0);
  const T ghost_r = periodic ? AT(v, 0) : T(0);
#pragma unroll
  for (int i = 0; i < N; i++) {
    const T f0 = AT(v, i);
    const T fr = (i + 1 < N) ? AT(v, i + 1 < N ? i + 1 : 0) : ghost_r;
    const T dp = fr - f0;
    const T h = f0 + f0;
    const T r = twoinf - h;
    const T lp = clamp_ordered(dp, -r, h);
    const T lm = clamp_ordered(dm, -h, r);
    // lam_F_i = lam_g_{i+1} - lam_g_i (the last face leaves the line unless periodic)
    const T gnext = (i + 1 < N) ? AT(lg, i + 1 < N ? i + 1 : 0) : (periodic ? AT(lg, 0) : T(0));
    const T lF = gnext - AT(lg, i);
    const T inner = fma_(c2, lm, fma_(c1, lp, f0));
    lalpha = lalpha + lF * (inner + alpha * (dc1 * lp + dc2 * lm));
    const T lin = alpha * lF;
    AT(lam, i) = AT(lam, i) + lin;
    const T llp = c1 * lin;
    const T llm = c2 * lin;
    // Lp branch
    if (dp < -r) {
      AT(lam, i) = AT(lam, i) + T(2) * llp;
      lfinf = lfinf - T(2) * llp;
    } else if (dp > h) {
      AT(lam, i) = AT(lam, i) + T(2) * llp;
    } else {
      if (i + 1 < N) AT(lam, i + 1 < N ? i + 1 : 0) = AT(lam, i + 1 < N ? i + 1 : 0) + llp;
      else if (periodic) AT(lam, 0) = AT(lam, 0) + llp;
      AT(lam, i) = AT(lam, i) - llp;
    }
    // Lm branch
    if (dm < -h) {
      AT(lam, i) = AT(lam, i) - T(2) * llm;
    } else if (dm > r) {
      lfinf = lfinf + T(2) * llm;
      AT(lam, i) = AT(lam, i) - T(2) * llm;
    } else {
      AT(lam, i) = AT(lam, i) + llm;
      if (i > 0) AT(lam, i > 0 ? i - 1 : 0) = AT(lam, i > 0 ? i - 1 : 0) - llm;
      else if (periodic) AT(lam, N - 1) = AT(lam, N - 1) - llm;
    }
    dm = dp;
  }
#pragma unroll
  for (int i = 0; i < N; i++)
    if (i == am) lam[i] = lam[i] + lfinf;
#undef AT
  return lalpha;
}

// Reverse of pfc_line + apply_shift for one line; returns d<lam_out, out>/d nu.
template <typename T, int N, typename ST, typename LD>
__device__ __forceinline__ double pfc_line_adj(const T (&v)[N], T (&lam)[N], double nu, bool periodic, ST st,
                                               LD ld)
{
  const LineCoef<T> k = line_coef<T, N>(nu, periodic);
  const double alpha_d = (double)k.alpha;
  (void)alpha_d;
  // transpose of f'_i = g_{i-s}: lam_g_k = lam_out_{k+s}
  apply_shift<T, N>(lam, -k.shift, periodic, st, ld);
  const double a = fabs(nu);
  const double al = a - floor(a);
  const T dc1 = (T)((2.0 * al - 3.0) / 6.0);
  const T dc2 = (T)(-al / 3.0);
  T lalpha;
  if (k.neg) lalpha = pfc_core_adj<T, N, true>(v, lam, k.alpha, k.c1, k.c2, dc1, dc2, periodic);
  else lalpha = pfc_core_adj<T, N, false>(v, lam, k.alpha, k.c1, k.c2, dc1, dc2, periodic);
  return k.neg ? -(double)lalpha : (double)lalpha;
}

__device__ __forceinline__ double adj_line_nu(const SweepArgs& a, long long o, long long c)
{
  if (a.velocity) return a.accel[o / a.sp_div] * a.scale;
  const long long j = (c / a.j_div) % a.j_mod;
  return (a.vmin + ((double)j + 0.5) * a.dv) * a.scale;
}

template <typename T, int N>
__global__ __launch_bounds__(256) void sweep_adj_kernel(SweepArgs a, const T* fin, T* lam, double* dnu)
{
  const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
  if (gid >= a.nlines) return;
  const long long o = gid / a.inner;
  const long long c = gid - o * a.inner;
  const long long base = o * (long long)N * a.inner + c;
  const long long inner = a.inner;
  T v[N], l[N];
#pragma unroll
  for (int r = 0; r < N; r++) {
    v[r] = fin[base + r * inner];
    l[r] = lam[base + r * inner];
  }
  T* p = lam + base;
  const double d = pfc_line_adj<T, N>(v, l, adj_line_nu(a, o, c), a.periodic != 0,
                                      [&](int r, T x) { p[(long long)r * inner] = x; },
                                      [&](int r) { return p[(long long)r * inner]; });
#pragma unroll
  for (int r = 0; r < N; r++) p[(long long)r * inner] = l[r];
  if (dnu) dnu[gid] = d;
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

template <typename T, int N>
hipError_t launch_adj_n(const SweepArgs& a, const void* fin, void* lam, double* dnu, hipStream_t s)
{
  if (a.nlines <= 0) return hipSuccess;
  const long long blocks = (a.nlines + 255) / 256;
  hipLaunchKernelGGL((sweep_adj_kernel<T, N>), dim3((unsigned)blocks), dim3(256), 0, s, a,
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

hipError_t launch_sweep_adjoint(const SweepArgs& a, int dtype, const void* fin, void* lam, double* dnu,
                                hipStream_t s)
{
  return dtype == 0 ? launch_adj_t<float>(a, fin, lam, dnu, s) : launch_adj_t<double>(a, fin, lam, dnu, s);
}

hipError_t launch_reduce_lines(double* lam_a, const double* dnu, long long np, long long per, double scale,
                               hipStream_t s)
{
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_lines_kernel, dim3((unsigned)np), dim3(256), 0, s, lam_a, dnu, per, scale);
  return hipGetLastError();
}

}  // namespace vp
