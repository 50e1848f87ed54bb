// pfc_line.h -- the one-line PFC update shared by the sweep kernels and by
// their reverse mode (Sec. 2.1 of Yoshikawa, Yoshida & Umemura; the formulas
// are stated in sweep.hip). Device code only.
#pragma once

#include <hip/hip_runtime.h>

namespace vp {
namespace {

__device__ __forceinline__ float clamp_ordered(float x, float lo, float hi)
{
  return __builtin_amdgcn_fmed3f(x, lo, hi);
}
__device__ __forceinline__ double clamp_ordered(double x, double lo, double hi)
{
  return fmin(fmax(x, lo), hi);
}
__device__ __forceinline__ float max_(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double max_(double a, double b) { return fmax(a, b); }

template <typename T>
struct LineCoef {
  T alpha, c1, c2;
  int shift;  // signed whole-cell shift s: f'_i = g_{i-s}
  bool neg;
};

template <typename T, int N>
__device__ __forceinline__ LineCoef<T> line_coef(double nu, bool periodic)
{
  LineCoef<T> k;
  k.neg = nu < 0.0;
  const double a = fabs(nu);
  const double fl = floor(a);
  const double alpha = a - fl;
  int m;
  if (fl >= (double)N) m = periodic ? (int)fmod(fl, (double)N) : N;
  else m = (int)fl;
  k.alpha = (T)alpha;
  k.c1 = (T)((1.0 - alpha) * (2.0 - alpha) / 6.0);
  k.c2 = (T)((1.0 - alpha) * (1.0 + alpha) / 6.0);
  k.shift = k.neg ? -m : m;
  return k;
}

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Fractional update g of one line held in registers, transport toward
// increasing index. Every rounding
// step is written out (automatic contraction is off), so all kernels that use
// this routine produce the same bits:
//   h = 2 f_k, r = 2 f_inf - h (= 2 (f_inf - f_k) exactly),
//   Lp = med3(f_{k+1} - f_k, -r, h), Lm = med3(f_k - f_{k-1}, -h, r),
//   q_k = fma(c2, Lm, fma(c1, Lp, f_k))   (the face flux is F_k = alpha q_k),
//   g_k = fma(alpha, q_{k-1} - q_k, f_k)   (= f_k + F_{k-1} - F_k).
template <typename T, int N>
__device__ __forceinline__ void pfc_core(T (&v)[N], T alpha, T c1, T c2, bool periodic)
{
#pragma clang fp contract(off)
#define AT(i) v[i]
  T finf = T(0);
#pragma unroll
  for (int i = 0; i < N; i++) finf = max_(finf, v[i]);
  const T twoinf = finf + finf;

  // flux through the left face of cell 0: zero (outflow) or that of cell N-1
  T qprev = T(0);
  T dm = periodic ? AT(0) - AT(N - 1) : AT(0);   // f_0 - f_{-1}
  if (periodic) {
    const T fl = AT(N >= 2 ? N - 2 : 0), f0 = AT(N - 1), fr = AT(0);
    const T h = f0 + f0;
    const T r = twoinf - h;
    const T lp = clamp_ordered(fr - f0, -r, h);
    const T lm = clamp_ordered(f0 - fl, -h, r);
    qprev = fma_(c2, lm, fma_(c1, lp, f0));
  }
  const T ghost_r = periodic ? AT(0) : T(0);
#pragma unroll
  for (int i = 0; i < N; i++) {
    const T f0 = AT(i);
    const T fr = (i + 1 < N) ? AT(i + 1 < N ? i + 1 : 0) : ghost_r;
    const T dp = fr - f0;
    const T h = f0 + f0;
    const T r = twoinf - h;
    const T lp = clamp_ordered(dp, -r, h);
    const T lm = clamp_ordered(dm, -h, r);
    const T q = fma_(c2, lm, fma_(c1, lp, f0));
    AT(i) = fma_(alpha, qprev - q, f0);
    qprev = q;
    dm = dp;
  }
#undef AT
}

// Fractional update of one line by Courant number nu; returns the coefficients
// (whose signed shift the caller applies, with store_shifted). A lane whose
// line moves toward decreasing index mirrors its data with selects around the
// forward update. One code path serves both directions: separate branches per
// direction make the compiler hoist the work the branches share and keep both
// sets of values alive, which costs far more registers than the two selects
// per cell. Every route does the same arithmetic in the same order, so all
// kernels agree bit for bit.
template <typename T, int N>
__device__ __forceinline__ LineCoef<T> pfc_line(T (&v)[N], double nu, bool periodic)
{
  const LineCoef<T> k = line_coef<T, N>(nu, periodic);
#pragma unroll
  for (int i = 0; i < N / 2; i++) {
    const T x = v[i], y = v[N - 1 - i];
    v[i] = k.neg ? y : x;
    v[N - 1 - i] = k.neg ? x : y;
  }
  pfc_core<T, N>(v, k.alpha, k.c1, k.c2, periodic);
#pragma unroll
  for (int i = 0; i < N / 2; i++) {
    const T x = v[i], y = v[N - 1 - i];
    v[i] = k.neg ? y : x;
    v[N - 1 - i] = k.neg ? x : y;
  }
  return k;
}

// Writes the shifted line f'_i = g_{i-s} (periodic wrap, or zero where the
// source lies beyond an outflow boundary) of the fractional result g held in
// v to the line's storage; st(i, x) sets cell i. Each cell is written once
// with its final value.
template <typename T, int N, typename ST>
__device__ __forceinline__ void store_shifted(const T (&v)[N], int shift, bool periodic, ST st)
{
  if (shift == 0) {
#pragma unroll
    for (int r = 0; r < N; r++) st(r, v[r]);
    return;
  }
  // a per-lane copy: the bounds tests below stay inside this rarely taken
  // branch instead of being precomputed as scalar masks for the whole kernel
  asm volatile("" : "+v"(shift));
#pragma unroll
  for (int r = 0; r < N; r++) {
    int d = r + shift;
    if (periodic) {
      d %= N;
      if (d < 0) d += N;
      st(d, v[r]);
    } else if (d >= 0 && d < N) {
      st(d, v[r]);
    }
  }
  if (!periodic) {
    for (int i = 0; i < N; i++) {
      const int src = i - shift;
      if (src < 0 || src >= N) st(i, T(0));
    }
  }
}

// store_shifted for two lines that take the same shift: st(i, x0, x1) sets
// cell i of both, so that the caller can write the pair with one access.
template <typename T, int N, typename ST>
__device__ __forceinline__ void store_shifted2(const T (&v0)[N], const T (&v1)[N], int shift, bool periodic, ST st)
{
  if (shift == 0) {
#pragma unroll
    for (int r = 0; r < N; r++) st(r, v0[r], v1[r]);
    return;
  }
  asm volatile("" : "+v"(shift));
#pragma unroll
  for (int r = 0; r < N; r++) {
    int d = r + shift;
    if (periodic) {
      d %= N;
      if (d < 0) d += N;
      st(d, v0[r], v1[r]);
    } else if (d >= 0 && d < N) {
      st(d, v0[r], v1[r]);
    }
  }
  if (!periodic) {
    for (int i = 0; i < N; i++) {
      const int src = i - shift;
      if (src < 0 || src >= N) st(i, T(0), T(0));
    }
  }
}

}  // namespace
}  // namespace vp
