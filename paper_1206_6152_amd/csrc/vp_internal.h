// vp_internal.h -- declarations shared by the library's HIP translation units
// (kernels and the host C-ABI). Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vp {

// Geometry and Courant-number rule of one directional sweep. The array is
// viewed as [outer][n][inner]: a line is (o, c) and its cells sit at
// (o*n + r)*inner + c for r = 0..n-1.
struct SweepArgs {
  void* f;
  long long outer;     // number of slabs
  long long inner;     // stride between consecutive cells of a line
  long long nlines;    // outer * inner
  int n;               // line length
  int velocity;        // 1: nu = accel[o / sp_div] * scale; 0: nu = v_j * scale
  int periodic;        // 1: periodic ghosts; 0: outflow ghosts
  int pad0;
  double scale;        // tau / dv (velocity) or tau / dx (position)
  const double* accel; // acceleration component (velocity sweeps)
  long long sp_div;    // spatial cell of slab o is o / sp_div (velocity sweeps)
  long long j_div;     // velocity index j = (c / j_div) % j_mod (position sweeps)
  long long j_mod;
  double vmin, dv;     // cell-centre velocity v_j = vmin + (j + 1/2) dv
  double* part;        // optional: per-workgroup sums of the new line values (see below)
  void* out;           // optional: write the result here (same layout) instead of over f
  // reverse sweeps only, optional: each lam value is first raised by
  // add_coef * addend[spatial cell] (the spatial cell of line (o, c), cell r is
  // (o*n + r) * add_stride + c / add_div)
  const double* addend;
  double add_coef;
  long long add_stride, add_div;
};

// Launch one sweep on the stream; dtype 0 = float, 1 = double.
hipError_t launch_sweep(const SweepArgs& a, int dtype, hipStream_t s);

// True when a workgroup of 256 consecutive lines of length N can be addressed
// from its first line with 32-bit lane offsets (and 32-bit index arithmetic).
bool narrow_ok(const SweepArgs& a, int N);

// With part set, workgroup b (256 consecutive lines) also writes
// part[b * n + r] = sum over its lines of the new value at cell r, in FP64.
// True when the sweep supports that for these arguments.
bool sweep_part_supported(const SweepArgs& a, int dtype);

// True when n is a line length the sweep kernels are instantiated for.
bool sweep_length_supported(int n);

// Half kick T_vz T_vy T_vx(tau) of every spatial cell's velocity block in one
// pass: the block of cell s is f[s*nv3 .. (s+1)*nv3) and moves with
// nu_l = a_l[s] * scale_l.
struct KickArgs {
  void* f;
  long long np;
  const double* a[3];
  double scale[3];
  int reps;   // 1: one half kick; 2: two consecutive half kicks with the same acceleration
  void* out;  // one-pass kick only: write the result here (same layout) instead of over f
  // per-spatial-cell line coefficients of the three velocity sweeps, filled by
  // the launch functions before the pass: kick_table_bytes(dtype, np) bytes
  void* tab;
  int xcd_group;  // set by the launch functions: slices of one block on one XCD
};
size_t kick_table_bytes(int dtype, long long np);

// True when a one-pass kernel exists for this velocity grid and element type.
bool kick_fused_supported(int dtype, const int nv[3]);
hipError_t launch_kick(const KickArgs& a, int dtype, const int nv[3], hipStream_t s);

// FP64 32^3 blocks: one half kick (reps 1) or two with the same acceleration
// (reps 2) in one pass, the block held in registers (one line per lane) and
// changing orientation through LDS in halves.
bool kick_lines_supported(int dtype, const int nv[3]);
hipError_t launch_kick_lines(const KickArgs& a, int dtype, const int nv[3], hipStream_t s);

// The six sweeps of two consecutive half kicks in three passes over slices
// (T_vx T_vy on vz-slices, T_vz T_vx on vy-slices, T_vy T_vz on vx-slices),
// for FP32 48^3 and 64^3 and FP64 48^3 blocks; pass 0 also fills the
// coefficient table.
bool kick_slices_supported(int dtype, const int nv[3]);
hipError_t launch_kick_slices(const KickArgs& a, int dtype, const int nv[3], int pass, hipStream_t s);
// T_vy then T_vz in one pass over slices of whole (vy, vz) planes, for
// velocity blocks too large for the passes above (48^3 and 64^3: 12 and 8
// planes in FP32, 6 and 4 in FP64, 110 and 130 KiB per slice). A half kick is
// a T_vx sweep and this pass.
bool kick_planes_supported(int dtype, const int nv[3]);
hipError_t launch_kick_planes(const KickArgs& a, int dtype, const int nv[3], hipStream_t s);

// T_y T_z(tau) (z first) in one pass: tile = one x index x W velocity cells of
// every (y, z) cell. Position sweeps: nu = v_l(j) tau / dx_l.
struct DriftArgs {
  void* f;
  long long nx, nv3;
  int ny, nz;
  long long nvy, nvz;
  int periodic;
  double vmin_y, dv_y, scale_y;
  double vmin_z, dv_z, scale_z;
  // per-velocity-cell line coefficients of the two sweeps, filled by
  // launch_drift_yz before the pass: drift_table_bytes(dtype, nv3) bytes
  void* tab;
  int xcd_group;  // set by launch_drift_yz: chunks that share cache lines on one XCD
};
size_t drift_table_bytes(int dtype, long long nv3);
bool drift_yz_supported(int dtype, int ny, int nz, long long nv3, long long nvz);
hipError_t launch_drift_yz(const DriftArgs& a, int dtype, hipStream_t s);

// ---- gravity and reductions (FP64) ----------------------------------------

// rho[s] = dv3 * sum_j f[s*nv3 + j]
hipError_t launch_density(const void* f, int dtype, double* rho, long long np, long long nv3,
                          double dv3, hipStream_t s);

// dst = src for n16 16-byte vectors (16-byte aligned, not overlapping)
hipError_t launch_copy16(const void* src, void* dst, long long n16, hipStream_t s);

// out[s] = scale * sum_j a[s*nv3 + j] w[j]
hipError_t launch_weighted_moment(const void* a, int dtype, const double* w, double* out, long long np,
                                  long long nv3, double scale, hipStream_t s);

// rho from the x sweep's workgroup sums: spatial column yz (of nyz) has
// nchunk workgroups, each with n sums (one per x);
// rho[x*nyz + yz] = dv3 * sum_k part[(yz*nchunk + k)*n + x]. With G = 256/n
// chunk groups, group g adds the chunks k = g, g + G, ... in order, and the G
// group sums are then added in order of g (a fixed order, deterministic).
hipError_t launch_density_from_parts(double* rho, const double* part, long long nyz, long long nchunk, int n,
                                     double dv3, hipStream_t s);

struct Grid3 {
  int m[3];
};

// Twiddle table w[k] = exp(-2 pi i k / M), k = 0..M-1, as (cos, sin) pairs.
hipError_t launch_twiddles(double2* w, int M, hipStream_t s);

// In-place DFT along one axis of a complex field of shape g (C order);
// sign -1 forward, +1 inverse (no scaling). tw is the table for g.m[axis].
hipError_t launch_dft_axis(double2* data, Grid3 g, int axis, int sign, const double2* tw,
                           hipStream_t s);

// data = rho (imag 0) on an n-grid (periodic) or zero-padded into the 2n-grid.
hipError_t launch_load_rho(double2* data, Grid3 g, const double* rho, Grid3 n, hipStream_t s);

// data *= G_hat(k) of the periodic discrete Green's function; zero mode -> 0.
hipError_t launch_green_periodic(double2* data, Grid3 g, double G, double d0, double d1,
                                 double d2, hipStream_t s);

// data *= spec (complex, same grid)
hipError_t launch_mul_spectrum(double2* data, const double2* spec, long long count, hipStream_t s);

// Real-space isolated Green's function on the doubled grid (offsets mirrored).
hipError_t launch_green_isolated(double2* data, Grid3 g, double G, double d0, double d1,
                                 double d2, double self_value, hipStream_t s);

// phi_ext[t] (t in -1..n per axis) = scale * Re data[t mod g]
hipError_t launch_extract_phi(double* phi_ext, Grid3 n, const double2* data, Grid3 g,
                              double scale, hipStream_t s);

// a_l = -(phi(i+e_l) - phi(i-e_l)) / (2 d_l) from the ghost-padded potential.
hipError_t launch_gradient(double* accel, const double* phi_ext, Grid3 n, double d0, double d1,
                           double d2, hipStream_t s);

// Partial sums per spatial cell: part[2*s] = sum f, part[2*s+1] = sum f |v|^2.
struct VelGrid {
  int nv[3];
  double vmin[3];
  double dv[3];
};
hipError_t launch_energy_partials(const void* f, int dtype, double* part, long long np,
                                  VelGrid vg, hipStream_t s);

// The whole-grid reductions below take a device buffer `out` of
// RED_PART + 3 REDUCE_BLOCKS doubles: results in out[0..3], per-workgroup
// partials from out[RED_PART] on.
constexpr int REDUCE_BLOCKS = 1024;
constexpr int RED_PART = 8;
constexpr int RED_DOUBLES = RED_PART + 3 * REDUCE_BLOCKS;

// out[0..3] = K, U, M, E from the partials, rho and phi_ext (deterministic).
hipError_t launch_energy_final(double* out, const double* part, const double* rho,
                               const double* phi_ext, Grid3 n, double dx3, double dv3,
                               hipStream_t s);

// out[0] = max over cells and axes of |a_l| * inv_dv[l].
hipError_t launch_accel_max(double* out, const double* accel, long long np, double i0, double i1,
                            double i2, hipStream_t s);

// ---- reverse mode -------------------------------------------------------------

// lam <- J^T lam for the sweep described by a at forward input fin; the
// per-line d<lam, out>/d nu goes to dnu[line] when dnu is not null. With
// a.addend set, lam is first raised by the addend (strided lines with compact
// addressing only: adjoint_addend_supported).
hipError_t launch_sweep_adjoint(const SweepArgs& a, int dtype, const void* fin, void* lam, double* dnu,
                                hipStream_t s);
bool adjoint_addend_supported(const SweepArgs& a);
// lam_a[s] += scale * sum_{i < per} dnu[s*per + i], s < np
// Reverse of one half kick T_vz T_vy T_vx in one pass (see adjoint.hip): lam
// <- J^T lam at forward input fin, and lam_a[l][s] += scale[l] * (the block's
// summed line adjoints), for the grids kick_adjoint_supported accepts.
struct KickAdjArgs {
  const void* fin;
  void* lam;
  long long np;
  const double* accel[3];
  double scale[3];    // tau / dv_l
  double* lam_a[3];   // all NULL: no acceleration adjoint
};
bool kick_adjoint_supported(int dtype, const int nv[3]);
hipError_t launch_kick_adjoint(const KickAdjArgs& a, int dtype, const int nv[3], hipStream_t s);
hipError_t launch_reduce_lines(double* lam_a, const double* dnu, long long np, long long per, double scale,
                               hipStream_t s);
hipError_t launch_gradient_adj(double* lphi_ext, const double* lam_a, Grid3 n, double d0, double d1, double d2,
                               hipStream_t s);
hipError_t launch_fold_periodic(double* out, const double* lphi_ext, Grid3 n, hipStream_t s);
hipError_t launch_load_ext(double2* data, Grid3 g, const double* lphi_ext, Grid3 n, hipStream_t s);
hipError_t launch_extract_interior(double* out, const double2* data, Grid3 g, Grid3 n, double scale,
                                   hipStream_t s);
hipError_t launch_broadcast_add(void* lam, int dtype, const double* x, long long np, long long nv3, double coef,
                                hipStream_t s);
hipError_t launch_seed(void* lam, int dtype, const double* phi_ext, Grid3 n, long long nv3, double coef,
                       hipStream_t s);
hipError_t launch_potential_energy(double* out, const double* rho, const double* phi_ext, Grid3 n, double dx3,
                                   hipStream_t s);

}  // namespace vp
