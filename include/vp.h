/*
 * vp.h -- C ABI of the MI355X (gfx950) six-dimensional Vlasov-Poisson library.
 *
 * The library advances a distribution function f(x, y, z, vx, vy, vz) of a
 * collisionless self-gravitating system with the directionally split
 * positive-flux-conservative (PFC) scheme of Yoshikawa, Yoshida & Umemura
 * (arXiv:1206.6152), Sec. 2: one-dimensional PFC advections along each phase-
 * space axis (Sec. 2.1, Eqs. (5)-(16)), composed as the leapfrog product of
 * Eq. (17), with the density of Eq. (18), the FFT-convolution Poisson solve of
 * Sec. 2.2 (periodic, Eqs. (19)-(20); isolated by grid doubling, Eq. (21)) and
 * the two-point acceleration of Eq. (22).
 *
 * Conventions shared by every entry point
 *   - Grid (Sec. 2, Eqs. (3)-(4)): space is [-L/2, L/2) per axis with cell
 *     centres x_i = -L/2 + (i + 1/2) L/N; velocity is [vmin, vmax] per axis
 *     with centres v_j = vmin + (j + 1/2) dv, dv = (vmax - vmin)/Nv.
 *   - f layout: one C-order array f[Nx][Ny][Nz][Nvx][Nvy][Nvz] (vz fastest)
 *     of float (VP_F32) or double (VP_F64) in device memory. The element type
 *     is the storage and sweep precision; density, potential, acceleration and
 *     diagnostics are always FP64.
 *   - Spatial fields (rho, accel components) are C-order [Nx][Ny][Nz] FP64.
 *     The potential is returned with one ghost layer, [Nx+2][Ny+2][Nz+2]
 *     (index 0 holds cell -1).
 *   - Every call returns 0 (VP_OK) or a negative VP_E* code; vp_last_error()
 *     then describes the failure. Arguments are validated before any device
 *     work, so VP_EINVAL leaves the state untouched.
 *   - Work is enqueued asynchronously on the HIP stream given to vp_init.
 *     Only vp_energy and vp_dt wait for the stream (they return host values).
 *   - The library is not re-entrant per context: calls on one context must
 *     not overlap. Distinct contexts are independent.
 *
 * Boundary conditions (Sec. 2.1): velocity axes are always outflow (matter
 * pushed past vmin/vmax is lost). VP_BC_PERIODIC makes the spatial sweeps and
 * the Poisson solve periodic; VP_BC_ISOLATED makes the spatial sweeps outflow
 * and the Poisson solve isolated.
 */
#ifndef VP_H
#define VP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VP_OK 0
#define VP_EINVAL (-1)        /* bad argument or configuration */
#define VP_ENOMEM (-2)        /* device allocation failed */
#define VP_EHIP (-3)          /* HIP runtime or kernel launch failure */
#define VP_ENONFINITE (-4)    /* a diagnostic sum is not finite */
#define VP_EUNSUPPORTED (-5)  /* valid request the library does not implement */

#define VP_BC_PERIODIC 0
#define VP_BC_ISOLATED 1

#define VP_F32 0
#define VP_F64 1

/* Problem statement of Sec. 2. All lengths >= 1. Every one of the six axis
 * lengths must be one of the line lengths the sweep kernels are built for:
 * 1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128. VP_BC_ISOLATED needs
 * equal spacings dx = dy = dz. */
typedef struct vp_config {
  int32_t n[3];       /* spatial cells Nx, Ny, Nz */
  int32_t nv[3];      /* velocity cells Nvx, Nvy, Nvz */
  double L[3];        /* box lengths (> 0) */
  double vmin[3];     /* V^- per axis */
  double vmax[3];     /* V^+ per axis (> vmin) */
  double G;           /* gravitational constant (>= 0) */
  int32_t bc;         /* VP_BC_PERIODIC or VP_BC_ISOLATED */
  int32_t dtype;      /* VP_F32 or VP_F64: element type of f */
  int32_t flags;      /* must be 0 */
  int32_t reserved;   /* must be 0 */
} vp_config;

typedef struct vp_ctx vp_ctx;  /* opaque */

/* sizeof(vp_config) as compiled into the library (binding self-check). */
int vp_config_size(void);

/* Pure host validation of a configuration; touches no device. */
int vp_config_validate(const vp_config* cfg);

/* Create a context on the current HIP device for the f array at f_dev (device
 * pointer, 16-byte aligned, layout and type above, caller-owned). The library BORROWS f: it
 * updates it in place and the caller keeps it alive, and does not modify it
 * behind the library's back, until vp_free. hip_stream is a hipStream_t (NULL
 * for the null stream). Allocates the FP64 work fields and computes the
 * initial acceleration from f (density, Poisson, gradient). On success *out
 * receives the context; on failure *out is NULL and nothing stays allocated. */
int vp_init(const vp_config* cfg, void* f_dev, void* hip_stream, vp_ctx** out);

/* One step of Eq. (17): T_vx, T_vy, T_vz at dt/2 with the current
 * acceleration; T_z, T_y, T_x at dt; density, Poisson solve and acceleration;
 * T_vx, T_vy, T_vz at dt/2 with the new acceleration. The acceleration left in
 * the context serves the first half kick of the next step, so the Poisson
 * equation is solved once per step, after the position sweeps as the paper
 * states. When Nv^3 is a multiple of 256 and Nx is at most 64 (VP_F32) or 32
 * (VP_F64), the T_x sweep also sums its new values over velocity in FP64 and
 * the density of Eq. (18) comes from those sums (same value as vp_density up
 * to the order of the FP64 additions). dt must be finite and > 0. */
int vp_step(vp_ctx* ctx, double dt);

/* n consecutive vp_step calls with the same dt (n >= 0), with the same result
 * bit for bit. The closing half kick of one step and the opening half kick of
 * the next use the same acceleration; they run as one pass over f. */
int vp_run(vp_ctx* ctx, int32_t nsteps, double dt);

/* A single one-dimensional PFC advection T_axis(tau) of every line of f
 * (Sec. 2.1, Eqs. (11)-(16)): axis 0, 1, 2 = x, y, z move with the cell's
 * velocity v_axis; axis 3, 4, 5 = vx, vy, vz move with the stored
 * acceleration a_{axis-3} of the spatial cell. tau must be finite (any sign;
 * any Courant number). */
int vp_sweep(vp_ctx* ctx, int32_t axis, double tau);

/* The two halves of Eq. (17). vp_kick: T_vz T_vy T_vx(tau) with the stored
 * acceleration (T_vx first). vp_drift: T_x T_y T_z(tau) (T_z first). Each is
 * exactly the corresponding vp_sweep calls in that order (same arithmetic, same
 * result bit for bit); vp_kick runs the three velocity sweeps of a spatial
 * cell in one pass over f when that cell's velocity block fits on chip
 * (cubic velocity grids: FP32 up to 32^3 and FP64 up to 24^3 in LDS, FP64
 * 32^3 in registers with one line per lane; 48^3 and 64^3 as a T_vx sweep
 * then T_vy T_vz in one pass over slices of whole (vy, vz) planes), and
 * vp_drift runs T_z and T_y in one pass when a (y, z) plane of a chunk of
 * velocity cells fits on chip (square planes of 16, 24, 32 or 48 cells, and
 * 64 in FP32), then T_x. */
int vp_kick(vp_ctx* ctx, double tau);
int vp_drift(vp_ctx* ctx, double tau);

/* Recompute the stored acceleration from the current f (Eqs. (18)-(22)). */
int vp_accel(vp_ctx* ctx);

/* Copy the stored acceleration to a_dev ([3][Nx][Ny][Nz] FP64, device), or
 * replace it from a_dev. */
int vp_get_accel(vp_ctx* ctx, double* a_dev);
int vp_set_accel(vp_ctx* ctx, const double* a_dev);

/* rho = integral of f over velocity (Eq. (18)) of the current f, written to
 * rho_dev ([Nx][Ny][Nz] FP64, device, caller-owned). Asynchronous. */
int vp_density(vp_ctx* ctx, double* rho_dev);

/* Velocity moment of an array a_dev with the layout and type of f, against
 * weights w_dev ([Nvx][Nvy][Nvz] FP64, device): out_dev[s] = scale *
 * sum_j a[s][j] w[j] for every spatial cell s ([Nx][Ny][Nz] FP64, device,
 * caller-owned), accumulated in FP64 in a fixed order. With w = 1 and
 * scale = dv^3 it is the density of Eq. (18); with w = M(v) and scale = rho0
 * it carries a gradient dL/df0 of an initial condition f0 = rho0 (1 + delta(x))
 * M(v) to dL/d delta(x). Asynchronous. */
int vp_moment(vp_ctx* ctx, const void* a_dev, const double* w_dev, double scale, double* out_dev);

/* Potential of the current f (Eqs. (18)-(21)) with one ghost layer, written to
 * phi_dev ([Nx+2][Ny+2][Nz+2] FP64, device, caller-owned). Periodic: the
 * k = 0 mode is zero and ghosts are periodic images. Isolated: ghosts hold
 * the convolution evaluated one cell outside the box. Asynchronous. */
int vp_potential(vp_ctx* ctx, double* phi_dev);

/* Kinetic, potential and total energy and mass of the current f
 * (Eqs. (29), (30), (41)), out_host[0..3] = K, U, M, E, with cell-centre
 * velocities. Synchronises the stream. VP_ENONFINITE if a sum is not finite. */
int vp_energy(vp_ctx* ctx, double out_host[4]);

/* dt = cfl * min(dt_p, dt_v) of Eqs. (23)-(25) from the stored acceleration,
 * with V^max = max(|vmin|, |vmax|) per axis; an axis with no velocity extent
 * or no acceleration imposes no limit. Synchronises the stream. */
int vp_dt(vp_ctx* ctx, double cfl, double* dt_host);

/* Per-phase timing, the breakdown of the paper's Table 1 (Sec. 4): when
 * enabled, every sweep and every gravity solve issued by vp_step, vp_run,
 * vp_sweep and vp_accel is bracketed by HIP events on the context's stream.
 * vp_profile_enable(ctx, 1) clears the totals and starts recording;
 * vp_profile_enable(ctx, 0) stops. vp_profile_read synchronises the stream and
 * returns, per phase, the summed event time in milliseconds and the number of
 * launches: phases 0..5 are the sweeps along x, y, z, vx, vy, vz, phase 6 the
 * gravity solve (density, or the reduction of the T_x sums, Poisson,
 * acceleration), phase 7 the one-pass half
 * kick, phase 8 the one-pass pair of half kicks of vp_run, phase 9 the
 * one-pass T_y T_z, phase 10 the reverse sweeps and phase 11 the reverse
 * gravity map of vp_grad and vp_*_adjoint, phase 12 a pass of two velocity
 * sweeps over slices of 48^3 or 64^3 velocity blocks (too large for one
 * pass), phase 13 the one-pass reverse half kick (vp_kick_adjoint, vp_grad).
 * Arrays have VP_NPHASE entries and are caller-owned host memory. */
#define VP_NPHASE 14
int vp_profile_enable(vp_ctx* ctx, int32_t on);
int vp_profile_read(vp_ctx* ctx, double ms_out[VP_NPHASE], int64_t count_out[VP_NPHASE]);

/* Measurement aid, no context: dst_dev = src_dev for nbytes bytes on the HIP
 * stream hip_stream (NULL = default stream), one 16-byte vector per lane. Its
 * read-and-write rate is the practical HBM ceiling that the sweep passes are
 * compared with. Both pointers are device memory, 16-byte aligned, and the
 * ranges must not overlap; nbytes >= 0 is a multiple of 16. Invalid arguments
 * return VP_EINVAL before any device work. Asynchronous. */
int vp_stream_copy(const void* src_dev, void* dst_dev, int64_t nbytes, void* hip_stream);

/* Integral of 1/|r| over one cell of widths dx, dy, dz centred on the origin.
 * The paper's isolated Green's function (Sec. 2.2, Eq. (21)) is G/r and says
 * nothing of the cell's own offset; this library reads the kernel as
 * -G dx dy dz / |r| away from zero and -G times this integral at zero (the
 * potential of a uniform cell at its centre). Pure host arithmetic, no device
 * and no context; returns NaN, with a message for vp_last_error, unless all
 * three widths are finite and > 0. */
double vp_cell_self_integral(double dx, double dy, double dz);

/* ---- reverse mode (gradients; an extension beyond the paper) -------------
 *
 * The loss is the field energy of the final state, L = -U (U of Eq. (41)),
 * after nsteps steps of Eq. (17) with a fixed dt. The limited update is a
 * piecewise-smooth map: the reverse mode differentiates the branch that the
 * forward input selects (a corrector bound counts as active only when the
 * one-sided difference is strictly beyond it; f_inf's adjoint goes to the
 * first cell holding the line maximum).
 *
 * vp_sweep_adjoint: lam <- J^T lam for the single sweep T_axis(tau) taken at
 * the forward input f_in (device, layout and type of f; lam likewise, updated
 * in place). For a velocity axis, when lam_accel ([3][Nx][Ny][Nz] FP64, device)
 * is not NULL, the adjoint of the stored acceleration component a_{axis-3} is
 * added to it (the sweep moves with nu = a tau / dv).
 *
 * vp_kick_adjoint: lam <- J^T lam for the half kick T_vz T_vy T_vx (tau) of
 * Eq. (17) with the stored acceleration, taken at the forward input f_in
 * (arguments as for vp_sweep_adjoint; lam_accel, when not NULL, gains the
 * adjoint of all three acceleration components). One pass per velocity
 * block that rebuilds the two intermediate states on chip; the result equals
 * vp_sweep_adjoint along vz, vy and vx at those states bit for bit. Available
 * where two velocity blocks fit on chip (cubic grids of 8, 16 or 24 cells in
 * VP_F32, 8 in VP_F64); VP_EUNSUPPORTED elsewhere, before any device work.
 *
 * vp_accel_adjoint: lam += dv^3 G^T D^T lam_accel, the transpose of the linear
 * map f -> density -> potential -> acceleration of Eqs. (18)-(22).
 *
 * vp_grad: from the current f = f0 (with the acceleration the context holds
 * for it), runs nsteps steps forward, keeping a copy of f every ckpt_every
 * steps and the acceleration of every step, so that the reverse sweep
 * recomputes one segment at a time; writes dL/df0 to grad_f0_dev (device,
 * layout and type of f, caller-owned, 16-byte aligned) and L to *loss_host.
 * On return f holds the final state and the context its acceleration, as after
 * vp_run(nsteps, dt). Allocates ceil(nsteps/ckpt_every) + ckpt_every + 1
 * copies of f for the call (checkpoints, the states of one segment, and two
 * arrays in which each step's sweep inputs are regenerated from the step's
 * start), plus the acceleration of every step, and frees them before
 * returning (VP_ENOMEM if they do not fit). Synchronises the stream. */
int vp_sweep_adjoint(vp_ctx* ctx, int32_t axis, double tau, const void* f_in_dev, void* lam_dev,
                     double* lam_accel_dev);
int vp_kick_adjoint(vp_ctx* ctx, double tau, const void* f_in_dev, void* lam_dev, double* lam_accel_dev);
int vp_accel_adjoint(vp_ctx* ctx, const double* lam_accel_dev, void* lam_dev);
int vp_grad(vp_ctx* ctx, int32_t nsteps, double dt, int32_t ckpt_every, void* grad_f0_dev, double* loss_host);

/* vp_sweep_adjoint_noalloc: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same arguments, same kernels and the same result bit for bit as
 * vp_sweep_adjoint, but it calls no hipMalloc, hipFree or other allocating
 * routine: the per-line adjoints of a velocity sweep's Courant numbers live
 * in a static device array of VP_NOALLOC_MAX_LINES doubles (32 MiB), which
 * each device the library runs on holds until the process ends (its address
 * is resolved per device by vp_init). A velocity sweep with lam_accel_dev set
 * and more lines than that (N_cells / Nv_axis > VP_NOALLOC_MAX_LINES) returns
 * VP_EINVAL before any device work. The array is shared by every call on a
 * device and keeps the last call's contents (each call overwrites every entry
 * it reads, so nothing has to start at zero); calls that overlap in time on
 * one device, from any contexts or streams, race on it. No phase timing is
 * recorded for this call. */
#define VP_NOALLOC_MAX_LINES 4194304
int vp_sweep_adjoint_noalloc(vp_ctx* ctx, int32_t axis, double tau, const void* f_in_dev, void* lam_dev,
                             double* lam_accel_dev);

/* Release everything the context owns (never f). NULL is accepted. */
int vp_free(vp_ctx* ctx);

/* Description of the last failure on the calling thread ("" if none); valid
 * until the next vp_* call on the thread. */
const char* vp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VP_H */
