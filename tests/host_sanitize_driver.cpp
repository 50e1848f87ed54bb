// Drives every host-side validation path of the C ABI (config checks, null
// pointers, null contexts, copy arguments, the self-integral) for a build of
// the library's host code with AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_sanitized_builds.py). No call reaches a device: each one fails
// its host checks first, or is pure host arithmetic. Exits non-zero when a
// call returns another code than the one expected.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "vp.h"

static int failures = 0;

static void expect(const char* what, int got, int want)
{
  if (got != want) {
    std::printf("FAIL %s: got %d want %d (%s)\n", what, got, want, vp_last_error());
    failures++;
  }
}

static vp_config good()
{
  vp_config c;
  std::memset(&c, 0, sizeof c);
  for (int l = 0; l < 3; l++) {
    c.n[l] = 8;
    c.nv[l] = 16;
    c.L[l] = 1.0;
    c.vmin[l] = -1.0;
    c.vmax[l] = 1.0;
  }
  c.G = 1.0;
  c.bc = VP_BC_PERIODIC;
  c.dtype = VP_F32;
  return c;
}

int main()
{
  expect("config size", vp_config_size(), (int)sizeof(vp_config));
  vp_config c = good();
  expect("good config", vp_config_validate(&c), VP_OK);
  c.bc = VP_BC_ISOLATED;
  c.dtype = VP_F64;
  expect("good isolated FP64 config", vp_config_validate(&c), VP_OK);
  expect("null config", vp_config_validate(nullptr), VP_EINVAL);

  struct Bad {
    const char* what;
    void (*edit)(vp_config&);
    int want;
  };
  const Bad bad[] = {
      {"n = 0", [](vp_config& x) { x.n[0] = 0; }, VP_EINVAL},
      {"nv < 0", [](vp_config& x) { x.nv[1] = -1; }, VP_EINVAL},
      {"n = 10", [](vp_config& x) { x.n[0] = 10; }, VP_EUNSUPPORTED},
      {"nv = 20", [](vp_config& x) { x.nv[2] = 20; }, VP_EUNSUPPORTED},
      {"L = 0", [](vp_config& x) { x.L[1] = 0.0; }, VP_EINVAL},
      {"L = nan", [](vp_config& x) { x.L[1] = NAN; }, VP_EINVAL},
      {"L = inf", [](vp_config& x) { x.L[2] = INFINITY; }, VP_EINVAL},
      {"vmax < vmin", [](vp_config& x) { x.vmax[1] = -1.0; }, VP_EINVAL},
      {"vmin = nan", [](vp_config& x) { x.vmin[0] = NAN; }, VP_EINVAL},
      {"G < 0", [](vp_config& x) { x.G = -1.0; }, VP_EINVAL},
      {"G = nan", [](vp_config& x) { x.G = NAN; }, VP_EINVAL},
      {"bc = 7", [](vp_config& x) { x.bc = 7; }, VP_EINVAL},
      {"dtype = 2", [](vp_config& x) { x.dtype = 2; }, VP_EINVAL},
      {"flags = 1", [](vp_config& x) { x.flags = 1; }, VP_EINVAL},
      {"isolated, unequal spacing", [](vp_config& x) { x.bc = VP_BC_ISOLATED; x.L[1] = 2.0; }, VP_EUNSUPPORTED},
  };
  for (const Bad& b : bad) {
    vp_config x = good();
    b.edit(x);
    expect(b.what, vp_config_validate(&x), b.want);
    if (std::strlen(vp_last_error()) == 0) {
      std::printf("FAIL %s: no error message\n", b.what);
      failures++;
    }
  }

  // null pointers to vp_init fail before any device work
  c = good();
  vp_ctx* ctx = nullptr;
  expect("init null f", vp_init(&c, nullptr, nullptr, &ctx), VP_EINVAL);
  expect("init left ctx null", ctx == nullptr ? 0 : 1, 0);
  expect("init null out", vp_init(&c, reinterpret_cast<void*>(4096), nullptr, nullptr), VP_EINVAL);
  expect("init null config", vp_init(nullptr, reinterpret_cast<void*>(4096), nullptr, &ctx), VP_EINVAL);

  // every entry point rejects a null context
  double d4[4], d1 = 0.0;
  double ms[VP_NPHASE];
  int64_t cnt[VP_NPHASE];
  expect("sweep", vp_sweep(nullptr, 0, 0.1), VP_EINVAL);
  expect("step", vp_step(nullptr, 0.1), VP_EINVAL);
  expect("run", vp_run(nullptr, 2, 0.1), VP_EINVAL);
  expect("kick", vp_kick(nullptr, 0.1), VP_EINVAL);
  expect("drift", vp_drift(nullptr, 0.1), VP_EINVAL);
  expect("accel", vp_accel(nullptr), VP_EINVAL);
  expect("get_accel", vp_get_accel(nullptr, nullptr), VP_EINVAL);
  expect("set_accel", vp_set_accel(nullptr, nullptr), VP_EINVAL);
  expect("density", vp_density(nullptr, nullptr), VP_EINVAL);
  expect("moment", vp_moment(nullptr, nullptr, nullptr, 1.0, nullptr), VP_EINVAL);
  expect("potential", vp_potential(nullptr, nullptr), VP_EINVAL);
  expect("energy", vp_energy(nullptr, d4), VP_EINVAL);
  expect("dt", vp_dt(nullptr, 0.5, &d1), VP_EINVAL);
  expect("sweep_adjoint", vp_sweep_adjoint(nullptr, 3, 0.1, nullptr, nullptr, nullptr), VP_EINVAL);
  expect("sweep_adjoint_noalloc", vp_sweep_adjoint_noalloc(nullptr, 3, 0.1, nullptr, nullptr, nullptr), VP_EINVAL);
  expect("kick_adjoint", vp_kick_adjoint(nullptr, 0.1, nullptr, nullptr, nullptr), VP_EINVAL);
  expect("accel_adjoint", vp_accel_adjoint(nullptr, nullptr, nullptr), VP_EINVAL);
  expect("grad", vp_grad(nullptr, 2, 0.1, 1, nullptr, &d1), VP_EINVAL);
  expect("profile_enable", vp_profile_enable(nullptr, 1), VP_EINVAL);
  expect("profile_read", vp_profile_read(nullptr, ms, cnt), VP_EINVAL);
  expect("free", vp_free(nullptr), VP_OK);

  // copy arguments: the addresses are never dereferenced
  char* p = reinterpret_cast<char*>(4096);
  expect("copy null src", vp_stream_copy(nullptr, p, 64, nullptr), VP_EINVAL);
  expect("copy null dst", vp_stream_copy(p, nullptr, 64, nullptr), VP_EINVAL);
  expect("copy size", vp_stream_copy(p, p + 4096, 24, nullptr), VP_EINVAL);
  expect("copy negative", vp_stream_copy(p, p + 4096, -16, nullptr), VP_EINVAL);
  expect("copy misaligned", vp_stream_copy(p + 8, p + 4096, 64, nullptr), VP_EINVAL);
  expect("copy overlap", vp_stream_copy(p, p + 16, 64, nullptr), VP_EINVAL);

  // the self term: pure host arithmetic
  const double w = vp_cell_self_integral(1.0, 2.0, 0.5);
  expect("self integral finite", std::isfinite(w) && w > 0.0 ? 0 : 1, 0);
  expect("self integral rejects", std::isnan(vp_cell_self_integral(-1.0, 1.0, 1.0)) ? 0 : 1, 0);
  expect("self integral rejects nan", std::isnan(vp_cell_self_integral(1.0, NAN, 1.0)) ? 0 : 1, 0);

  std::printf("host checks done, %d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
