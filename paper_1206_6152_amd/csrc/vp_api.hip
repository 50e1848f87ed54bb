// vp_api.hip -- host side of the C ABI declared in include/vp.h: configuration
// checks, the context and its FP64 work fields, and the sequencing of the
// kernels of one step of Eq. (17) (Yoshikawa, Yoshida & Umemura, Sec. 2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "vp.h"
#include "vp_internal.h"

using vp::Grid3;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...)
{
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

bool debug_sync()
{
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("VP_DEBUG_SYNC");
    v = (e && e[0] == '1') ? 1 : 0;
  }
  return v == 1;
}

}  // namespace

struct vp_ctx {
  vp_config cfg;
  void* f = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  long long np = 0, nv3 = 0;
  double dx[3] = {0, 0, 0}, dv[3] = {0, 0, 0};
  Grid3 ng{};           // spatial grid
  Grid3 wg{};           // transform grid: ng (periodic) or 2 ng (isolated)
  double* rho = nullptr;
  double* phi = nullptr;      // (N+2)^3
  double* accel = nullptr;    // [3][np]
  double2* work = nullptr;    // wg cells
  double2* kspec = nullptr;   // isolated Green's function spectrum
  double2* tw[3] = {nullptr, nullptr, nullptr};
  double* part = nullptr;     // 2 * np
  double* red = nullptr;      // vp::RED_DOUBLES doubles on the device: results, then partials
  double* host = nullptr;     // 8 pinned doubles
  // reverse-mode work fields (allocated on first use)
  double* lphi = nullptr;     // (N+2)^3
  double* radj = nullptr;     // np
  double* dnu = nullptr;      // one value per line of a sweep
  long long dnu_len = 0;
  // workgroup sums of the x sweep (density without another pass over f);
  // null when the x sweep of this grid cannot produce them
  double* xsum = nullptr;
  // per-velocity-cell line coefficients of the one-pass T_z T_y (null when
  // the grid has no such pass)
  void* dtab = nullptr;
  // per-spatial-cell line coefficients of the kick passes (null when the
  // velocity grid has none)
  void* ktab = nullptr;
  // phase timing (vp_profile_*): pending event pairs per phase
  bool profiling = false;
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  double phase_ms[VP_NPHASE] = {};
  long long phase_n[VP_NPHASE] = {};
  // this device's address of the static scratch array (vp_sweep_adjoint_noalloc)
  double* scratch = nullptr;
};

// Scratch of vp_sweep_adjoint_noalloc: the per-line adjoint of the Courant
// number of one velocity sweep, one double per line, VP_NOALLOC_MAX_LINES lines
// (32 MiB). It is a static device array, so every device the library runs on
// holds its own copy from code-object load until the process ends. In host
// code the name is a host-side stand-in, never a device address: host code
// uses only the per-device address from hipGetSymbolAddress (scratch_address).
__device__ __align__(256) double scratch[VP_NOALLOC_MAX_LINES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxDevices] = {};

// The current device's address of `scratch`, resolved once per device (the
// caller has made `device` current). Called from vp_init.
int scratch_address(int device, double** out)
{
  if (device < 0 || device >= kMaxDevices) return fail(VP_EUNSUPPORTED, "device index %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(VP_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_addr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_addr[device];
  return VP_OK;
}

}  // namespace

namespace {

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(VP_EHIP, "%s: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

int check_launch(vp_ctx* c, hipError_t e, const char* what)
{
  if (e != hipSuccess) return fail(VP_EHIP, "%s: %s", what, hipGetErrorString(e));
  if (debug_sync()) {
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(VP_EHIP, "%s (sync): %s", what, hipGetErrorString(e));
  }
  return VP_OK;
}

#define LAUNCH(c, expr)                                 \
  do {                                                  \
    int r_ = check_launch((c), (expr), #expr);          \
    if (r_ != VP_OK) return r_;                         \
  } while (0)

// Gauss-Legendre rule of order n on [-1, 1]: nodes are the roots of P_n,
// found by Newton's method from the estimate cos(pi (i + 3/4) / (n + 1/2)),
// with P_n and P_n' from Bonnet's three-term recurrence; weights
// 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, double* x, double* w)
{
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; i++) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; it++) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; k++) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace

// Integral of 1/|r| over the cell of widths dx, dy, dz centred on the origin: the
// potential of a unit-density cell at its own centre, which is the isolated
// kernel's value at zero offset. Since div(r/|r|) = 2/|r|, the divergence
// theorem makes the volume integral half the outward flux of r/|r|; on the two
// faces normal to axis l, r.n = h_l (the half width), so
//   I = sum_l h_l int_{face l} dA / |r|.
// Across one face coordinate the integrand has the antiderivative asinh, so
//   int_face dA/|r| = 4 int_0^{h_b} asinh(h_c / sqrt(h_l^2 + y^2)) dy,
// a smooth integrand (its nearest complex singularity is at y = i h_l),
// integrated with 16-point Gauss-Legendre panels no wider than h_l / 2.
double vp_cell_self_integral(double dx, double dy, double dz)
{
  g_err.clear();
  if (!(dx > 0.0) || !(dy > 0.0) || !(dz > 0.0) || !std::isfinite(dx + dy + dz)) {
    fail(VP_EINVAL, "cell widths must be finite and > 0");
    return NAN;
  }
  const int NG = 16;
  double gx[NG], gw[NG];
  gauss_legendre(NG, gx, gw);
  const double h[3] = {0.5 * dx, 0.5 * dy, 0.5 * dz};
  double total = 0.0;
  for (int l = 0; l < 3; l++) {
    const double hl = h[l];
    for (int t = 0; t < 2; t++) {  // (hb, hc) and (hc, hb): the face integral both ways, averaged
      const double hb = h[(l + 1 + t) % 3], hc = h[(l + 2 - t) % 3];
      const long panels = std::max(1L, (long)std::ceil(2.0 * hb / hl));
      const double width = hb / panels;
      double face = 0.0;
      for (long p = 0; p < panels; p++) {
        const double mid = (p + 0.5) * width;
        double acc = 0.0;
        for (int g = 0; g < NG; g++) {
          const double y = mid + 0.5 * width * gx[g];
          acc += gw[g] * std::asinh(hc / std::sqrt(hl * hl + y * y));
        }
        face += 0.5 * width * acc;
      }
      total += 0.5 * hl * 4.0 * face;
    }
  }
  return total;
}

namespace {

void release(vp_ctx* c)
{
  if (!c) return;
  hipFree(c->rho);
  hipFree(c->phi);
  hipFree(c->accel);
  hipFree(c->work);
  hipFree(c->kspec);
  for (auto& t : c->tw) hipFree(t);
  hipFree(c->part);
  hipFree(c->xsum);
  hipFree(c->dtab);
  hipFree(c->ktab);
  hipFree(c->red);
  hipFree(c->lphi);
  hipFree(c->radj);
  hipFree(c->dnu);
  if (c->host) hipHostFree(c->host);
  for (auto& p : c->ev_pending) {
    hipEventDestroy(p.second.first);
    hipEventDestroy(p.second.second);
  }
  for (auto e : c->ev_free) hipEventDestroy(e);
  delete c;
}

template <typename P>
int dalloc(P** p, size_t bytes, const char* what)
{
  hipError_t e = hipMalloc((void**)p, bytes ? bytes : 16);
  if (e != hipSuccess) {
    *p = nullptr;
    hipGetLastError();
    return fail(VP_ENOMEM, "hipMalloc(%s, %zu bytes): %s", what, bytes, hipGetErrorString(e));
  }
  return VP_OK;
}

long long prod3(const int m[3]) { return (long long)m[0] * m[1] * m[2]; }

hipEvent_t take_event(vp_ctx* c)
{
  if (!c->ev_free.empty()) {
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one phase with events when profiling is on.
struct PhaseScope {
  vp_ctx* c;
  int phase;
  hipEvent_t a = nullptr, b = nullptr;
  PhaseScope(vp_ctx* c_, int p) : c(c_), phase(p)
  {
    if (!c->profiling) return;
    a = take_event(c);
    b = take_event(c);
    if (a) hipEventRecord(a, c->stream);
  }
  ~PhaseScope()
  {
    if (!c->profiling || !a || !b) return;
    hipEventRecord(b, c->stream);
    c->ev_pending.push_back({phase, {a, b}});
  }
};

// Fold finished event pairs into the totals (synchronises the stream).
int drain_events(vp_ctx* c)
{
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (auto& p : c->ev_pending) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p.second.first, p.second.second));
    c->phase_ms[p.first] += ms;
    c->phase_n[p.first] += 1;
    c->ev_free.push_back(p.second.first);
    c->ev_free.push_back(p.second.second);
  }
  c->ev_pending.clear();
  return VP_OK;
}

// potential (with ghosts) of the density held in rho_in
int poisson_from(vp_ctx* c, const double* rho_in, double* phi_out)
{
  const bool iso = c->cfg.bc == VP_BC_ISOLATED;
  LAUNCH(c, vp::launch_load_rho(c->work, c->wg, rho_in, c->ng, c->stream));
  for (int ax = 0; ax < 3; ax++) LAUNCH(c, vp::launch_dft_axis(c->work, c->wg, ax, -1, c->tw[ax], c->stream));
  if (iso)
    LAUNCH(c, vp::launch_mul_spectrum(c->work, c->kspec, prod3(c->wg.m), c->stream));
  else
    LAUNCH(c, vp::launch_green_periodic(c->work, c->wg, c->cfg.G, c->dx[0], c->dx[1], c->dx[2], c->stream));
  for (int ax = 0; ax < 3; ax++) LAUNCH(c, vp::launch_dft_axis(c->work, c->wg, ax, +1, c->tw[ax], c->stream));
  LAUNCH(c, vp::launch_extract_phi(phi_out, c->ng, c->work, c->wg, 1.0 / (double)prod3(c->wg.m), c->stream));
  return VP_OK;
}

// density -> rho, Poisson -> phi (with ghosts)
int potential_into(vp_ctx* c, double* phi_out)
{
  LAUNCH(c, vp::launch_density(c->f, c->cfg.dtype, c->rho, c->np, c->nv3,
                               c->dv[0] * c->dv[1] * c->dv[2], c->stream));
  return poisson_from(c, c->rho, phi_out);
}

int compute_accel(vp_ctx* c)
{
  PhaseScope scope(c, 6);
  int r = potential_into(c, c->phi);
  if (r != VP_OK) return r;
  LAUNCH(c, vp::launch_gradient(c->accel, c->phi, c->ng, c->dx[0], c->dx[1], c->dx[2], c->stream));
  return VP_OK;
}

// acceleration of the density held in c->rho
int accel_from_rho(vp_ctx* c)
{
  int r = poisson_from(c, c->rho, c->phi);
  if (r != VP_OK) return r;
  LAUNCH(c, vp::launch_gradient(c->accel, c->phi, c->ng, c->dx[0], c->dx[1], c->dx[2], c->stream));
  return VP_OK;
}

vp::SweepArgs sweep_args(vp_ctx* c, int axis, double tau)
{
  const auto& k = c->cfg;
  long long d[6] = {k.n[0], k.n[1], k.n[2], k.nv[0], k.nv[1], k.nv[2]};
  vp::SweepArgs a{};
  a.f = c->f;
  a.n = (int)d[axis];
  a.inner = 1;
  for (int q = 5; q > axis; q--) a.inner *= d[q];
  a.outer = 1;
  for (int q = 0; q < axis; q++) a.outer *= d[q];
  a.nlines = a.outer * a.inner;
  if (axis >= 3) {
    const int l = axis - 3;
    a.velocity = 1;
    a.periodic = 0;
    a.accel = c->accel + (long long)l * c->np;
    a.scale = tau / c->dv[l];
    a.sp_div = 1;
    for (int q = 3; q < axis; q++) a.sp_div *= d[q];
    a.j_div = 1;
    a.j_mod = 1;
  } else {
    a.velocity = 0;
    a.periodic = (k.bc == VP_BC_PERIODIC) ? 1 : 0;
    a.scale = tau / c->dx[axis];
    a.j_div = 1;
    for (int q = 5; q > axis + 3; q--) a.j_div *= d[q];
    a.j_mod = d[axis + 3];
    a.vmin = k.vmin[axis];
    a.dv = c->dv[axis];
    a.sp_div = 1;
  }
  return a;
}

int sweep(vp_ctx* c, int axis, double tau)
{
  const vp::SweepArgs a = sweep_args(c, axis, tau);
  PhaseScope scope(c, axis);
  LAUNCH(c, vp::launch_sweep(a, c->cfg.dtype, c->stream));
  return VP_OK;
}

// T_axis(tau) of the array at src, result written to dst (same layout, another array)
int sweep_to(vp_ctx* c, int axis, double tau, const void* src, void* dst)
{
  vp::SweepArgs a = sweep_args(c, axis, tau);
  a.f = const_cast<void*>(src);
  a.out = dst;
  PhaseScope scope(c, axis);
  LAUNCH(c, vp::launch_sweep(a, c->cfg.dtype, c->stream));
  return VP_OK;
}

// True when the x sweep can leave per-workgroup density sums: every
// workgroup's 256 lines lie in one spatial (y, z) column.
bool x_sweep_sums(vp_ctx* c)
{
  const vp::SweepArgs a = sweep_args(c, 0, 1.0);
  return c->nv3 % 256 == 0 && vp::sweep_part_supported(a, c->cfg.dtype);
}

// lam <- J^T lam of T_axis(tau) at forward input fin; velocity axes add the
// acceleration adjoint to lam_a (if not null).
int sweep_adjoint(vp_ctx* c, int axis, double tau, const void* fin, void* lam, double* lam_a,
                  const double* rho_adj = nullptr)
{
  vp::SweepArgs a = sweep_args(c, axis, tau);
  if (rho_adj) {   // lam += dv^3 rho_adj(spatial cell) first: fused into the loads where supported
    const double dv3 = c->dv[0] * c->dv[1] * c->dv[2];
    a.addend = rho_adj;
    a.add_coef = dv3;
    a.add_stride = a.inner / c->nv3;
    a.add_div = c->nv3;
    if (axis >= 3 || a.inner % c->nv3 != 0 || !vp::adjoint_addend_supported(a)) {
      a.addend = nullptr;
      PhaseScope scope(c, 11);
      LAUNCH(c, vp::launch_broadcast_add(lam, c->cfg.dtype, rho_adj, c->np, c->nv3, dv3, c->stream));
    }
  }
  const bool want = axis >= 3 && lam_a;
  if (want && a.nlines > c->dnu_len) {
    hipFree(c->dnu);
    c->dnu = nullptr;
    c->dnu_len = 0;
    int r = dalloc(&c->dnu, sizeof(double) * a.nlines, "line adjoints");
    if (r) return r;
    c->dnu_len = a.nlines;
  }
  PhaseScope scope(c, 10);
  LAUNCH(c, vp::launch_sweep_adjoint(a, c->cfg.dtype, fin, lam, want ? c->dnu : nullptr, c->stream));
  if (want) {
    const int l = axis - 3;
    LAUNCH(c, vp::launch_reduce_lines(lam_a + (long long)l * c->np, c->dnu, c->np, a.nlines / c->np,
                                      tau / c->dv[l], c->stream));
  }
  return VP_OK;
}

// lam <- adjoint of the half kick T_vz T_vy T_vx (tau) at forward input fin,
// with c->accel, in one pass; lam_a[l] gains the acceleration adjoint
int kick_adjoint(vp_ctx* c, double tau, const void* fin, void* lam, double* lam_a)
{
  vp::KickAdjArgs a{};
  a.fin = fin;
  a.lam = lam;
  a.np = c->np;
  for (int l = 0; l < 3; l++) {
    a.accel[l] = c->accel + (long long)l * c->np;
    a.scale[l] = tau / c->dv[l];
    a.lam_a[l] = lam_a ? lam_a + (long long)l * c->np : nullptr;
  }
  const int nv[3] = {c->cfg.nv[0], c->cfg.nv[1], c->cfg.nv[2]};
  PhaseScope scope(c, 13);
  LAUNCH(c, vp::launch_kick_adjoint(a, c->cfg.dtype, nv, c->stream));
  return VP_OK;
}

// c->radj = G^T D^T lam_a: transpose of potential -> acceleration, per spatial
// cell (the density adjoint; lam then gains dv^3 times it)
int density_adjoint(vp_ctx* c, const double* lam_a)
{
  const long long ext = (long long)(c->cfg.n[0] + 2) * (c->cfg.n[1] + 2) * (c->cfg.n[2] + 2);
  int r;
  if (!c->lphi && (r = dalloc(&c->lphi, sizeof(double) * ext, "potential adjoint"))) return r;
  if (!c->radj && (r = dalloc(&c->radj, sizeof(double) * c->np, "density adjoint"))) return r;
  PhaseScope scope(c, 11);
  LAUNCH(c, vp::launch_gradient_adj(c->lphi, lam_a, c->ng, c->dx[0], c->dx[1], c->dx[2], c->stream));
  if (c->cfg.bc == VP_BC_ISOLATED) {
    LAUNCH(c, vp::launch_load_ext(c->work, c->wg, c->lphi, c->ng, c->stream));
    for (int ax = 0; ax < 3; ax++) LAUNCH(c, vp::launch_dft_axis(c->work, c->wg, ax, -1, c->tw[ax], c->stream));
    LAUNCH(c, vp::launch_mul_spectrum(c->work, c->kspec, prod3(c->wg.m), c->stream));
    for (int ax = 0; ax < 3; ax++) LAUNCH(c, vp::launch_dft_axis(c->work, c->wg, ax, +1, c->tw[ax], c->stream));
    LAUNCH(c, vp::launch_extract_interior(c->radj, c->work, c->wg, c->ng, 1.0 / (double)prod3(c->wg.m), c->stream));
  } else {
    LAUNCH(c, vp::launch_fold_periodic(c->radj, c->lphi, c->ng, c->stream));
    LAUNCH(c, vp::launch_load_rho(c->work, c->wg, c->radj, c->ng, c->stream));
    for (int ax = 0; ax < 3; ax++) LAUNCH(c, vp::launch_dft_axis(c->work, c->wg, ax, -1, c->tw[ax], c->stream));
    LAUNCH(c, vp::launch_green_periodic(c->work, c->wg, c->cfg.G, c->dx[0], c->dx[1], c->dx[2], c->stream));
    for (int ax = 0; ax < 3; ax++) LAUNCH(c, vp::launch_dft_axis(c->work, c->wg, ax, +1, c->tw[ax], c->stream));
    LAUNCH(c, vp::launch_extract_interior(c->radj, c->work, c->wg, c->ng, 1.0 / (double)prod3(c->wg.m), c->stream));
  }
  return VP_OK;
}

// lam += dv^3 G^T D^T lam_a: transpose of density -> potential -> acceleration
int accel_adjoint(vp_ctx* c, const double* lam_a, void* lam)
{
  int r = density_adjoint(c, lam_a);
  if (r) return r;
  PhaseScope scope(c, 11);
  LAUNCH(c, vp::launch_broadcast_add(lam, c->cfg.dtype, c->radj, c->np, c->nv3, c->dv[0] * c->dv[1] * c->dv[2],
                                     c->stream));
  return VP_OK;
}

// T_vz T_vy T_vx(tau), reps times in a row with the same acceleration: one
// pass over f when the velocity block fits on chip.
int kick_n(vp_ctx* c, double tau, int reps)
{
  const int nv[3] = {c->cfg.nv[0], c->cfg.nv[1], c->cfg.nv[2]};
  if (vp::kick_fused_supported(c->cfg.dtype, nv)) {
    vp::KickArgs a{};
    a.tab = c->ktab;
    a.f = c->f;
    a.np = c->np;
    a.reps = reps;
    for (int l = 0; l < 3; l++) {
      a.a[l] = c->accel + (long long)l * c->np;
      a.scale[l] = tau / c->dv[l];
    }
    PhaseScope scope(c, reps == 2 ? 8 : 7);
    LAUNCH(c, vp::launch_kick(a, c->cfg.dtype, nv, c->stream));
    return VP_OK;
  }
  if (vp::kick_lines_supported(c->cfg.dtype, nv)) {   // FP64 32^3: one line per lane, LDS between axes
    vp::KickArgs a{};
    a.tab = c->ktab;
    a.f = c->f;
    a.np = c->np;
    a.reps = reps;
    for (int l = 0; l < 3; l++) {
      a.a[l] = c->accel + (long long)l * c->np;
      a.scale[l] = tau / c->dv[l];
    }
    PhaseScope scope(c, reps == 2 ? 8 : 7);
    LAUNCH(c, vp::launch_kick_lines(a, c->cfg.dtype, nv, c->stream));
    return VP_OK;
  }
  int r;
  if (vp::kick_planes_supported(c->cfg.dtype, nv)) {   // T_vx | T_vy T_vz per half kick
    vp::KickArgs a{};
    a.tab = c->ktab;
    a.f = c->f;
    a.np = c->np;
    a.reps = 1;
    for (int l = 0; l < 3; l++) {
      a.a[l] = c->accel + (long long)l * c->np;
      a.scale[l] = tau / c->dv[l];
    }
    if (reps == 2 && vp::kick_slices_supported(c->cfg.dtype, nv)) {   // T_vx T_vy | T_vz T_vx | T_vy T_vz
      for (int pass = 0; pass < 3; pass++) {
        PhaseScope scope(c, 12);
        LAUNCH(c, vp::launch_kick_slices(a, c->cfg.dtype, nv, pass, c->stream));
      }
      return VP_OK;
    }
    for (int i = 0; i < reps; i++) {
      if ((r = sweep(c, 3, tau))) return r;
      PhaseScope scope(c, 12);
      LAUNCH(c, vp::launch_kick_planes(a, c->cfg.dtype, nv, c->stream));
    }
    return VP_OK;
  }
  for (int i = 0; i < reps; i++)
    if ((r = sweep(c, 3, tau)) || (r = sweep(c, 4, tau)) || (r = sweep(c, 5, tau))) return r;
  return VP_OK;
}

int kick(vp_ctx* c, double tau) { return kick_n(c, tau, 1); }

// T_x T_y T_z(tau): z and y in one pass when the (y, z) plane fits on chip;
// with x_sums the x sweep also writes its workgroup sums to c->xsum
int drift(vp_ctx* c, double tau, bool x_sums = false)
{
  int r;
  const auto& k = c->cfg;
  if (vp::drift_yz_supported(k.dtype, k.n[1], k.n[2], c->nv3, k.nv[2])) {
    vp::DriftArgs a{};
    a.f = c->f;
    a.nx = k.n[0];
    a.nv3 = c->nv3;
    a.ny = k.n[1];
    a.nz = k.n[2];
    a.nvy = k.nv[1];
    a.nvz = k.nv[2];
    a.periodic = (k.bc == VP_BC_PERIODIC) ? 1 : 0;
    a.vmin_y = k.vmin[1];
    a.dv_y = c->dv[1];
    a.scale_y = tau / c->dx[1];
    a.vmin_z = k.vmin[2];
    a.dv_z = c->dv[2];
    a.scale_z = tau / c->dx[2];
    a.tab = c->dtab;
    {
      PhaseScope scope(c, 9);
      LAUNCH(c, vp::launch_drift_yz(a, k.dtype, c->stream));
    }
  } else if ((r = sweep(c, 2, tau)) || (r = sweep(c, 1, tau))) {
    return r;
  }
  if (!x_sums) return sweep(c, 0, tau);
  vp::SweepArgs a = sweep_args(c, 0, tau);
  a.part = c->xsum;
  PhaseScope scope(c, 0);
  LAUNCH(c, vp::launch_sweep(a, c->cfg.dtype, c->stream));
  return VP_OK;
}

// drift, then the acceleration of the drifted f (one step's middle): the x
// sweep sums its new values per workgroup when it can, which replaces the
// density pass over f by a reduction of those sums
int drift_accel(vp_ctx* c, double tau)
{
  if (!c->xsum) {
    int r = drift(c, tau);
    return r ? r : compute_accel(c);
  }
  int r = drift(c, tau, /*x_sums=*/true);
  if (r) return r;
  PhaseScope scope(c, 6);
  const long long nyz = (long long)c->cfg.n[1] * c->cfg.n[2];
  LAUNCH(c, vp::launch_density_from_parts(c->rho, c->xsum, nyz, c->nv3 / 256, c->cfg.n[0],
                                          c->dv[0] * c->dv[1] * c->dv[2], c->stream));
  return accel_from_rho(c);
}

int check_ctx(vp_ctx* c)
{
  if (!c) return fail(VP_EINVAL, "null context");
  return VP_OK;
}

}  // namespace

extern "C" {

int vp_config_size(void) { return (int)sizeof(vp_config); }

int vp_config_validate(const vp_config* cfg)
{
  g_err.clear();
  if (!cfg) return fail(VP_EINVAL, "null config");
  for (int l = 0; l < 3; l++) {
    if (cfg->n[l] < 1 || cfg->nv[l] < 1) return fail(VP_EINVAL, "axis %d: cell counts must be >= 1", l);
    if (!vp::sweep_length_supported(cfg->n[l]))
      return fail(VP_EUNSUPPORTED, "n[%d] = %d is not a supported line length", l, cfg->n[l]);
    if (!vp::sweep_length_supported(cfg->nv[l]))
      return fail(VP_EUNSUPPORTED, "nv[%d] = %d is not a supported line length", l, cfg->nv[l]);
    if (!(std::isfinite(cfg->L[l]) && cfg->L[l] > 0)) return fail(VP_EINVAL, "L[%d] must be finite and > 0", l);
    if (!(std::isfinite(cfg->vmin[l]) && std::isfinite(cfg->vmax[l]) && cfg->vmax[l] > cfg->vmin[l]))
      return fail(VP_EINVAL, "velocity range of axis %d must be finite with vmax > vmin", l);
  }
  if (!(std::isfinite(cfg->G) && cfg->G >= 0)) return fail(VP_EINVAL, "G must be finite and >= 0");
  if (cfg->bc != VP_BC_PERIODIC && cfg->bc != VP_BC_ISOLATED) return fail(VP_EINVAL, "unknown bc %d", cfg->bc);
  if (cfg->dtype != VP_F32 && cfg->dtype != VP_F64) return fail(VP_EINVAL, "unknown dtype %d", cfg->dtype);
  if (cfg->flags != 0 || cfg->reserved != 0) return fail(VP_EINVAL, "flags and reserved must be 0");
  const double np = (double)cfg->n[0] * cfg->n[1] * cfg->n[2];
  const double nv = (double)cfg->nv[0] * cfg->nv[1] * cfg->nv[2];
  if (np * nv > 9.0e18 / 8) return fail(VP_EINVAL, "grid too large");
  if (np > 2.0e9 || nv > 2.0e9) return fail(VP_EINVAL, "spatial or velocity grid too large");
  if (cfg->bc == VP_BC_ISOLATED) {
    const double d0 = cfg->L[0] / cfg->n[0], d1 = cfg->L[1] / cfg->n[1], d2 = cfg->L[2] / cfg->n[2];
    if (std::fabs(d0 - d1) > 1e-12 * d0 || std::fabs(d0 - d2) > 1e-12 * d0)
      return fail(VP_EUNSUPPORTED, "isolated Poisson needs equal spacings");
  }
  return VP_OK;
}

int vp_init(const vp_config* cfg, void* f_dev, void* hip_stream, vp_ctx** out)
{
  g_err.clear();
  if (!out) return fail(VP_EINVAL, "null output pointer");
  *out = nullptr;
  int r = vp_config_validate(cfg);
  if (r != VP_OK) return r;
  if (!f_dev) return fail(VP_EINVAL, "null f pointer");
  if (reinterpret_cast<uintptr_t>(f_dev) % 16 != 0) return fail(VP_EINVAL, "f must be 16-byte aligned");
  vp_ctx* c = new (std::nothrow) vp_ctx;
  if (!c) return fail(VP_ENOMEM, "host allocation failed");
  c->cfg = *cfg;
  c->f = f_dev;
  c->stream = (hipStream_t)hip_stream;
  const hipError_t de = hipGetDevice(&c->device);
  if (de != hipSuccess) {
    delete c;
    return fail(VP_EHIP, "device query: %s", hipGetErrorString(de));
  }
  if ((r = scratch_address(c->device, &c->scratch))) {
    delete c;
    return r;
  }
  for (int l = 0; l < 3; l++) {
    c->dx[l] = cfg->L[l] / cfg->n[l];
    c->dv[l] = (cfg->vmax[l] - cfg->vmin[l]) / cfg->nv[l];
    c->ng.m[l] = cfg->n[l];
    c->wg.m[l] = cfg->bc == VP_BC_ISOLATED ? 2 * cfg->n[l] : cfg->n[l];
  }
  c->np = prod3(c->ng.m);
  c->nv3 = (long long)cfg->nv[0] * cfg->nv[1] * cfg->nv[2];
  const long long ext = (long long)(cfg->n[0] + 2) * (cfg->n[1] + 2) * (cfg->n[2] + 2);
  const long long wn = prod3(c->wg.m);
  if ((r = dalloc(&c->rho, sizeof(double) * c->np, "rho")) ||
      (r = dalloc(&c->phi, sizeof(double) * ext, "phi")) ||
      (r = dalloc(&c->accel, sizeof(double) * 3 * c->np, "accel")) ||
      (r = dalloc(&c->work, sizeof(double2) * wn, "transform work")) ||
      (r = dalloc(&c->part, sizeof(double) * 2 * c->np, "partials")) ||
      (r = dalloc(&c->red, sizeof(double) * vp::RED_DOUBLES, "reduction"))) {
    release(c);
    return r;
  }
  for (int ax = 0; ax < 3; ax++) {
    if ((r = dalloc(&c->tw[ax], sizeof(double2) * c->wg.m[ax], "twiddles"))) {
      release(c);
      return r;
    }
  }
  if (cfg->bc == VP_BC_ISOLATED && (r = dalloc(&c->kspec, sizeof(double2) * wn, "green spectrum"))) {
    release(c);
    return r;
  }
  if (x_sweep_sums(c)) {   // n_x sums per 256 lines of the x sweep
    const long long nsum = (long long)cfg->n[1] * cfg->n[2] * (c->nv3 / 256) * cfg->n[0];
    if ((r = dalloc(&c->xsum, sizeof(double) * nsum, "x sweep sums"))) {
      release(c);
      return r;
    }
  }
  {
    const int nv[3] = {cfg->nv[0], cfg->nv[1], cfg->nv[2]};
    if ((vp::kick_fused_supported(cfg->dtype, nv) || vp::kick_lines_supported(cfg->dtype, nv) ||
         vp::kick_planes_supported(cfg->dtype, nv)) &&
        (r = dalloc(&c->ktab, vp::kick_table_bytes(cfg->dtype, c->np), "kick coefficients"))) {
      release(c);
      return r;
    }
  }
  if (vp::drift_yz_supported(cfg->dtype, cfg->n[1], cfg->n[2], c->nv3, cfg->nv[2]) &&
      (r = dalloc(&c->dtab, vp::drift_table_bytes(cfg->dtype, c->nv3), "drift coefficients"))) {
    release(c);
    return r;
  }
  hipError_t he = hipHostMalloc((void**)&c->host, sizeof(double) * 8, hipHostMallocDefault);
  if (he != hipSuccess) {
    c->host = nullptr;
    release(c);
    return fail(VP_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(he));
  }
  for (int ax = 0; ax < 3; ax++) {
    if ((r = check_launch(c, vp::launch_twiddles(c->tw[ax], c->wg.m[ax], c->stream), "twiddles"))) {
      release(c);
      return r;
    }
  }
  if (cfg->bc == VP_BC_ISOLATED) {
    const double self = -cfg->G * vp_cell_self_integral(c->dx[0], c->dx[1], c->dx[2]);
    r = check_launch(c, vp::launch_green_isolated(c->kspec, c->wg, cfg->G, c->dx[0], c->dx[1], c->dx[2], self,
                                                  c->stream), "green");
    for (int ax = 0; ax < 3 && r == VP_OK; ax++)
      r = check_launch(c, vp::launch_dft_axis(c->kspec, c->wg, ax, -1, c->tw[ax], c->stream), "green dft");
    if (r != VP_OK) {
      release(c);
      return r;
    }
  }
  r = compute_accel(c);
  if (r != VP_OK) {
    hipStreamSynchronize(c->stream);
    release(c);
    return r;
  }
  *out = c;
  return VP_OK;
}

int vp_sweep(vp_ctx* c, int32_t axis, double tau)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (axis < 0 || axis > 5) return fail(VP_EINVAL, "axis must be 0..5");
  if (!std::isfinite(tau)) return fail(VP_EINVAL, "tau must be finite");
  return sweep(c, axis, tau);
}

int vp_step(vp_ctx* c, double dt)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!(std::isfinite(dt) && dt > 0)) return fail(VP_EINVAL, "dt must be finite and > 0");
  const double h = 0.5 * dt;
  if ((r = kick(c, h)) || (r = drift_accel(c, dt)) || (r = kick(c, h))) return r;
  return VP_OK;
}

int vp_run(vp_ctx* c, int32_t nsteps, double dt)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (nsteps < 0) return fail(VP_EINVAL, "nsteps must be >= 0");
  if (!(std::isfinite(dt) && dt > 0)) return fail(VP_EINVAL, "dt must be finite and > 0");
  if (nsteps == 0) return VP_OK;
  // the closing half kick of a step and the opening half kick of the next use
  // the same acceleration and run back to back: one pass does both
  const double h = 0.5 * dt;
  if ((r = kick(c, h))) return r;
  for (int i = 0; i < nsteps; i++) {
    if ((r = drift_accel(c, dt))) return r;
    if ((r = kick_n(c, h, i + 1 < nsteps ? 2 : 1))) return r;
  }
  return VP_OK;
}

int vp_kick(vp_ctx* c, double tau)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!std::isfinite(tau)) return fail(VP_EINVAL, "tau must be finite");
  return kick(c, tau);
}

int vp_drift(vp_ctx* c, double tau)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!std::isfinite(tau)) return fail(VP_EINVAL, "tau must be finite");
  return drift(c, tau);
}

int vp_accel(vp_ctx* c)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  return compute_accel(c);
}

int vp_get_accel(vp_ctx* c, double* a_dev)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!a_dev) return fail(VP_EINVAL, "null pointer");
  HIP_TRY(hipMemcpyAsync(a_dev, c->accel, sizeof(double) * 3 * c->np, hipMemcpyDeviceToDevice, c->stream));
  return VP_OK;
}

int vp_set_accel(vp_ctx* c, const double* a_dev)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!a_dev) return fail(VP_EINVAL, "null pointer");
  HIP_TRY(hipMemcpyAsync(c->accel, a_dev, sizeof(double) * 3 * c->np, hipMemcpyDeviceToDevice, c->stream));
  return VP_OK;
}

int vp_density(vp_ctx* c, double* rho_dev)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!rho_dev) return fail(VP_EINVAL, "null pointer");
  LAUNCH(c, vp::launch_density(c->f, c->cfg.dtype, rho_dev, c->np, c->nv3, c->dv[0] * c->dv[1] * c->dv[2],
                               c->stream));
  return VP_OK;
}

int vp_moment(vp_ctx* c, const void* a_dev, const double* w_dev, double scale, double* out_dev)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!a_dev || !w_dev || !out_dev) return fail(VP_EINVAL, "null pointer");
  if (!std::isfinite(scale)) return fail(VP_EINVAL, "scale must be finite");
  LAUNCH(c, vp::launch_weighted_moment(a_dev, c->cfg.dtype, w_dev, out_dev, c->np, c->nv3, scale, c->stream));
  return VP_OK;
}

int vp_potential(vp_ctx* c, double* phi_dev)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!phi_dev) return fail(VP_EINVAL, "null pointer");
  return potential_into(c, phi_dev);
}

int vp_energy(vp_ctx* c, double out_host[4])
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!out_host) return fail(VP_EINVAL, "null pointer");
  if ((r = potential_into(c, c->phi))) return r;
  vp::VelGrid vg{};
  for (int l = 0; l < 3; l++) {
    vg.nv[l] = c->cfg.nv[l];
    vg.vmin[l] = c->cfg.vmin[l];
    vg.dv[l] = c->dv[l];
  }
  LAUNCH(c, vp::launch_energy_partials(c->f, c->cfg.dtype, c->part, c->np, vg, c->stream));
  LAUNCH(c, vp::launch_energy_final(c->red, c->part, c->rho, c->phi, c->ng, c->dx[0] * c->dx[1] * c->dx[2],
                                    c->dv[0] * c->dv[1] * c->dv[2], c->stream));
  HIP_TRY(hipMemcpyAsync(c->host, c->red, sizeof(double) * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int i = 0; i < 4; i++) out_host[i] = c->host[i];
  for (int i = 0; i < 4; i++)
    if (!std::isfinite(out_host[i])) return fail(VP_ENONFINITE, "diagnostic %d is not finite", i);
  return VP_OK;
}

int vp_dt(vp_ctx* c, double cfl, double* dt_host)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!dt_host) return fail(VP_EINVAL, "null pointer");
  if (!(std::isfinite(cfl) && cfl > 0)) return fail(VP_EINVAL, "cfl must be finite and > 0");
  LAUNCH(c, vp::launch_accel_max(c->red, c->accel, c->np, 1.0 / c->dv[0], 1.0 / c->dv[1], 1.0 / c->dv[2],
                                 c->stream));
  HIP_TRY(hipMemcpyAsync(c->host, c->red, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  double dtp = INFINITY;
  for (int l = 0; l < 3; l++) {
    const double vm = std::fmax(std::fabs(c->cfg.vmin[l]), std::fabs(c->cfg.vmax[l]));
    if (vm > 0) dtp = std::fmin(dtp, c->dx[l] / vm);
  }
  const double amax = c->host[0];
  const double dtv = amax > 0 ? 1.0 / amax : INFINITY;
  *dt_host = cfl * std::fmin(dtp, dtv);
  return VP_OK;
}

int vp_sweep_adjoint(vp_ctx* c, int32_t axis, double tau, const void* f_in_dev, void* lam_dev,
                     double* lam_accel_dev)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (axis < 0 || axis > 5) return fail(VP_EINVAL, "axis must be 0..5");
  if (!std::isfinite(tau)) return fail(VP_EINVAL, "tau must be finite");
  if (!f_in_dev || !lam_dev) return fail(VP_EINVAL, "null pointer");
  return sweep_adjoint(c, axis, tau, f_in_dev, lam_dev, lam_accel_dev);
}

int vp_kick_adjoint(vp_ctx* c, double tau, const void* f_in_dev, void* lam_dev, double* lam_accel_dev)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!std::isfinite(tau)) return fail(VP_EINVAL, "tau must be finite");
  if (!f_in_dev || !lam_dev) return fail(VP_EINVAL, "null pointer");
  const int nv[3] = {c->cfg.nv[0], c->cfg.nv[1], c->cfg.nv[2]};
  if (!vp::kick_adjoint_supported(c->cfg.dtype, nv))
    return fail(VP_EUNSUPPORTED, "no one-pass reverse half kick for this velocity grid");
  return kick_adjoint(c, tau, f_in_dev, lam_dev, lam_accel_dev);
}

int vp_sweep_adjoint_noalloc(vp_ctx* c, int32_t axis, double tau, const void* f_in_dev, void* lam_dev,
                             double* lam_accel_dev)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (axis < 0 || axis > 5) return fail(VP_EINVAL, "axis must be 0..5");
  if (!std::isfinite(tau)) return fail(VP_EINVAL, "tau must be finite");
  if (!f_in_dev || !lam_dev) return fail(VP_EINVAL, "null pointer");
  const vp::SweepArgs a = sweep_args(c, axis, tau);
  const bool want = axis >= 3 && lam_accel_dev;
  if (want && a.nlines > VP_NOALLOC_MAX_LINES)
    return fail(VP_EINVAL, "velocity sweep of %lld lines exceeds the %d-line device scratch of the "
                           "allocation-free reverse sweep", a.nlines, VP_NOALLOC_MAX_LINES);
  if (want && !c->scratch) return fail(VP_EHIP, "device scratch address not resolved");
  // every line writes its own entry before the reduction reads it, so the
  // scratch needs no clearing; no phase timing here (it would create events)
  LAUNCH(c, vp::launch_sweep_adjoint(a, c->cfg.dtype, f_in_dev, lam_dev, want ? c->scratch : nullptr, c->stream));
  if (want) {
    const int l = axis - 3;
    LAUNCH(c, vp::launch_reduce_lines(lam_accel_dev + (long long)l * c->np, c->scratch, c->np, a.nlines / c->np,
                                      tau / c->dv[l], c->stream));
  }
  return VP_OK;
}

int vp_accel_adjoint(vp_ctx* c, const double* lam_accel_dev, void* lam_dev)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!lam_accel_dev || !lam_dev) return fail(VP_EINVAL, "null pointer");
  return accel_adjoint(c, lam_accel_dev, lam_dev);
}

namespace {

struct GradWork {
  vp_ctx* c;
  std::vector<void*> bufs;
  std::vector<double*> dbufs;
  ~GradWork()
  {
    for (void* p : bufs) hipFree(p);
    for (double* p : dbufs) hipFree(p);
  }
  int f(void** p, size_t bytes)
  {
    int r = dalloc(p, bytes, "gradient work");
    if (!r) bufs.push_back(*p);
    return r;
  }
  int d(double** p, size_t bytes)
  {
    int r = dalloc(p, bytes, "gradient work");
    if (!r) dbufs.push_back(*p);
    return r;
  }
};

int copy_f(vp_ctx* c, void* dst, const void* src, size_t bytes)
{
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
  return VP_OK;
}

// dst = T_vz T_vy T_vx(tau) src (dst may not alias src): one pass when the
// velocity block fits on chip (in LDS, or in registers for FP64 32^3), else a
// copy and the kick in place. c->f is left pointing at dst.
int kick_to(vp_ctx* c, double tau, const void* src, void* dst, size_t fbytes)
{
  const int nv[3] = {c->cfg.nv[0], c->cfg.nv[1], c->cfg.nv[2]};
  const bool lines = vp::kick_lines_supported(c->cfg.dtype, nv);
  if (lines || vp::kick_fused_supported(c->cfg.dtype, nv)) {
    vp::KickArgs a{};
    a.tab = c->ktab;
    a.f = const_cast<void*>(src);
    a.out = dst;
    a.np = c->np;
    a.reps = 1;
    for (int l = 0; l < 3; l++) {
      a.a[l] = c->accel + (long long)l * c->np;
      a.scale[l] = tau / c->dv[l];
    }
    c->f = dst;
    PhaseScope scope(c, 7);
    LAUNCH(c, lines ? vp::launch_kick_lines(a, c->cfg.dtype, nv, c->stream)
                    : vp::launch_kick(a, c->cfg.dtype, nv, c->stream));
    return VP_OK;
  }
  int r = copy_f(c, dst, src, fbytes);
  if (r) return r;
  c->f = dst;
  return kick(c, tau);
}

// T_axis(tau) in place on the array at buf (left as c->f)
int sweep_on(vp_ctx* c, int axis, double tau, void* buf)
{
  c->f = buf;
  return sweep(c, axis, tau);
}

// Reverse mode of nsteps steps of Eq. (17) with checkpoints; see vp.h.
//
// Device memory: every k-th state of the forward run (ceil(nsteps/k) copies of
// f), the other k-1 states of the segment being reversed, and two work arrays
// in which the inputs of a step's nine sweeps are regenerated from the step's
// start, in the order the reverse sweeps need them:
//   closing half kick (a_{n+1}):  in8 = T_vy T_vx in6, then in7 = T_vx in6,
//                                 with in6 = drift(kick(x0)) kept throughout;
//   drift:                        in5 = T_y T_z in3, then in4 = T_z in3,
//                                 with in3 = kick(x0) kept throughout;
//   opening half kick (a_n):      in1 = T_vx x0 and in2 = T_vy in1.
// Every regenerated input is computed by the kernels of the forward run, so it
// is the forward input bit for bit; the price is twelve sweep passes per step
// instead of eight. Where two velocity blocks fit the LDS
// (kick_adjoint_supported), each reverse half kick is one pass at its input
// (in6, or x0) that rebuilds in7, in8 (in1, in2) on chip: seven regenerating
// passes and five reverse passes per step instead of twelve and nine, with the
// same bits.
int grad_impl(vp_ctx* c, int nsteps, double dt, int k, void* lam, double* loss)
{
  const size_t fb = (size_t)c->np * (size_t)c->nv3 * (c->cfg.dtype == VP_F32 ? 4 : 8);
  const size_t ab = sizeof(double) * 3 * (size_t)c->np;
  const int nck = (nsteps + k - 1) / k;
  void* user_f = c->f;
  GradWork w{c};
  // ck: every k-th state of the forward run; st[1..k-1]: the other states of
  // one segment, recomputed; b1, b2: regenerated sweep inputs of one step
  std::vector<void*> ck(nck), st(k, nullptr);
  void *b1 = nullptr, *b2 = nullptr;
  double *ahist = nullptr, *lam_a = nullptr, *lam_p = nullptr;
  int r;
  for (int i = 0; i < nck; i++)
    if ((r = w.f(&ck[i], fb))) return r;
  for (int i = 1; i < k; i++)
    if ((r = w.f(&st[i], fb))) return r;
  if ((r = w.f(&b1, fb)) || (r = w.f(&b2, fb))) return r;
  if ((r = w.d(&ahist, ab * (size_t)(nsteps + 1))) || (r = w.d(&lam_a, ab)) || (r = w.d(&lam_p, ab))) return r;
  auto A = [&](int n) { return ahist + (size_t)n * 3 * c->np; };
  const int nv[3] = {c->cfg.nv[0], c->cfg.nv[1], c->cfg.nv[2]};
  const bool fused_adj = vp::kick_adjoint_supported(c->cfg.dtype, nv);
  auto set_accel = [&](int n) { return copy_f(c, c->accel, A(n), ab); };

  // forward pass from f0, keeping checkpoints and every step's acceleration
  if ((r = copy_f(c, A(0), c->accel, ab))) return r;
  const double h = 0.5 * dt;
  // between checkpoints the closing half kick of step n-1 and the opening one
  // of step n (same acceleration) run as one pass, as in vp_run
  bool closing = false;   // the closing half kick of the previous step is still due
  for (int n = 0; n < nsteps; n++) {
    if (n % k == 0) {
      if (closing && (r = kick(c, h))) return r;
      closing = false;
      if ((r = copy_f(c, ck[n / k], user_f, fb))) return r;
    }
    if ((r = kick_n(c, h, closing ? 2 : 1)) || (r = drift_accel(c, dt))) return r;
    if ((r = copy_f(c, A(n + 1), c->accel, ab))) return r;
    closing = true;
  }
  if (closing && (r = kick(c, h))) return r;
  // user_f now holds the final state; the reverse pass leaves it alone
  // loss = -U of the final state, seed lam = dL/df = -dx^3 dv^3 phi(x)
  if ((r = potential_into(c, c->phi))) return r;
  const double dx3 = c->dx[0] * c->dx[1] * c->dx[2], dv3 = c->dv[0] * c->dv[1] * c->dv[2];
  LAUNCH(c, vp::launch_potential_energy(c->red, c->rho, c->phi, c->ng, dx3, c->stream));
  HIP_TRY(hipMemcpyAsync(c->host, c->red, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LAUNCH(c, vp::launch_seed(lam, c->cfg.dtype, c->phi, c->ng, c->nv3, -dx3 * dv3, c->stream));
  HIP_TRY(hipMemsetAsync(lam_p, 0, ab, c->stream));

  for (int seg = nck - 1; seg >= 0 && r == VP_OK; seg--) {
    const int s0 = seg * k, s1 = (s0 + k < nsteps) ? s0 + k : nsteps;
    st[0] = ck[seg];
    for (int n = s0; n + 1 < s1 && r == VP_OK; n++) {   // recompute the segment's states
      if ((r = set_accel(n))) break;
      if ((r = kick_to(c, h, st[n - s0], st[n - s0 + 1], fb)) || (r = drift_accel(c, dt)) || (r = kick(c, h))) break;
    }
    for (int n = s1 - 1; n >= s0 && r == VP_OK; n--) {
      void* x0 = st[n - s0];
      // closing half kick, acceleration a_{n+1}: in6 in b1, in8 then in7 in b2
      // (or the whole reverse half kick in one pass at in6)
      if ((r = set_accel(n)) || (r = kick_to(c, h, x0, b1, fb))) break;
      if ((r = drift(c, dt))) break;                                     // b1 = in6
      if ((r = set_accel(n + 1)) || (r = copy_f(c, lam_a, lam_p, ab))) break;
      if (fused_adj) {
        if ((r = kick_adjoint(c, h, b1, lam, lam_a))) break;
      } else {
        if ((r = sweep_to(c, 3, h, b1, b2)) || (r = sweep_on(c, 4, h, b2))) break;
        if ((r = sweep_adjoint(c, 5, h, b2, lam, lam_a))) break;          // at in8
        if ((r = sweep_to(c, 3, h, b1, b2)) || (r = sweep_adjoint(c, 4, h, b2, lam, lam_a))) break;   // at in7
        if ((r = sweep_adjoint(c, 3, h, b1, lam, lam_a))) break;          // at in6
      }
      // a_{n+1} = A(state after the drift): the density adjoint's contribution
      // to lam rides on the loads of the reverse x sweep that follows
      if ((r = density_adjoint(c, lam_a))) break;
      // drift: in3 in b1, in5 then in4 in b2
      if ((r = set_accel(n)) || (r = kick_to(c, h, x0, b1, fb))) break;  // b1 = in3
      if ((r = sweep_to(c, 2, dt, b1, b2)) || (r = sweep_on(c, 1, dt, b2))) break;   // b2 = in5
      if ((r = sweep_adjoint(c, 0, dt, b2, lam, nullptr, c->radj))) break;
      if ((r = sweep_to(c, 2, dt, b1, b2)) || (r = sweep_adjoint(c, 1, dt, b2, lam, nullptr))) break;   // at in4
      if ((r = sweep_adjoint(c, 2, dt, b1, lam, nullptr))) break;         // at in3
      // opening half kick, acceleration a_n: in1 in b1, in2 in b2 (or one pass at x0)
      HIP_TRY(hipMemsetAsync(lam_p, 0, ab, c->stream));
      if (fused_adj) {
        if ((r = kick_adjoint(c, h, x0, lam, lam_p))) break;
        continue;
      }
      if ((r = sweep_to(c, 3, h, x0, b1)) || (r = sweep_to(c, 4, h, b1, b2))) break;
      if ((r = sweep_adjoint(c, 5, h, b2, lam, lam_p)) || (r = sweep_adjoint(c, 4, h, b1, lam, lam_p)) ||
          (r = sweep_adjoint(c, 3, h, x0, lam, lam_p)))
        break;
    }
  }
  c->f = user_f;
  if (r) return r;
  // a_0 = A(f0)
  if ((r = accel_adjoint(c, lam_p, lam))) return r;
  if ((r = set_accel(nsteps))) return r;
  HIP_TRY(hipStreamSynchronize(c->stream));
  *loss = -c->host[0];
  return VP_OK;
}

}  // namespace

int vp_grad(vp_ctx* c, int32_t nsteps, double dt, int32_t ckpt_every, void* grad_f0_dev, double* loss_host)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (nsteps < 0) return fail(VP_EINVAL, "nsteps must be >= 0");
  if (!(std::isfinite(dt) && dt > 0)) return fail(VP_EINVAL, "dt must be finite and > 0");
  if (ckpt_every < 1) return fail(VP_EINVAL, "ckpt_every must be >= 1");
  if (!grad_f0_dev || !loss_host) return fail(VP_EINVAL, "null pointer");
  if (reinterpret_cast<uintptr_t>(grad_f0_dev) % 16 != 0) return fail(VP_EINVAL, "gradient must be 16-byte aligned");
  r = grad_impl(c, nsteps, dt, ckpt_every, grad_f0_dev, loss_host);
  if (r) hipStreamSynchronize(c->stream);
  return r;
}

int vp_profile_enable(vp_ctx* c, int32_t on)
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if ((r = drain_events(c))) return r;
  c->profiling = on != 0;
  if (c->profiling) {
    for (int i = 0; i < VP_NPHASE; i++) {
      c->phase_ms[i] = 0;
      c->phase_n[i] = 0;
    }
  }
  return VP_OK;
}

int vp_profile_read(vp_ctx* c, double ms_out[VP_NPHASE], int64_t count_out[VP_NPHASE])
{
  g_err.clear();
  int r = check_ctx(c);
  if (r) return r;
  if (!ms_out || !count_out) return fail(VP_EINVAL, "null pointer");
  if ((r = drain_events(c))) return r;
  for (int i = 0; i < VP_NPHASE; i++) {
    ms_out[i] = c->phase_ms[i];
    count_out[i] = c->phase_n[i];
  }
  return VP_OK;
}

int vp_stream_copy(const void* src, void* dst, int64_t nbytes, void* hip_stream)
{
  g_err.clear();
  if (!src || !dst) return fail(VP_EINVAL, "null pointer");
  if (nbytes < 0 || nbytes % 16 != 0) return fail(VP_EINVAL, "nbytes must be a non-negative multiple of 16");
  const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
  if (a % 16 != 0 || b % 16 != 0) return fail(VP_EINVAL, "pointers must be 16-byte aligned");
  if (nbytes > 0 && a < b + (uintptr_t)nbytes && b < a + (uintptr_t)nbytes)
    return fail(VP_EINVAL, "source and destination overlap");
  const hipError_t e = vp::launch_copy16(src, dst, nbytes / 16, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(VP_EHIP, "copy: %s", hipGetErrorString(e));
  return VP_OK;
}

int vp_free(vp_ctx* c)
{
  g_err.clear();
  if (!c) return VP_OK;
  hipStreamSynchronize(c->stream);
  release(c);
  return VP_OK;
}

const char* vp_last_error(void) { return g_err.c_str(); }

}  // extern "C"
