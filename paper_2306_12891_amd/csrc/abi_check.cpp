// Host-side checks of the C ABI (include/dg.h) under the address and
// undefined-behaviour sanitizers.  Built by sanitize.py with the host part of
// libdgmi (dg_host.cpp) instrumented; runs on the CPU.  Every entry point is
// called with the invalid arguments its declaration rejects (NULL context or
// pointers, host pointers, out-of-range sizes and options, bad time steps) and
// must return the documented error code without touching memory it does not
// own.  A valid dg_init builds the basis and the neighbour table on the host;
// without a GPU it then fails in the device allocation and must release
// everything (the sanitizer reports a use after free or a double free); with a
// GPU the context is used for the pointer and option checks and finalized.
// Exit status 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "dg.h"

static int g_fail = 0;

#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "abi_check: line %d: %s\n", __LINE__, #cond); \
      ++g_fail;                                                        \
    }                                                                  \
  } while (0)

static dg_mesh box(int nx, int ny, int nz) {
  dg_mesh m;
  m.nelem[0] = nx;
  m.nelem[1] = ny;
  m.nelem[2] = nz;
  for (int d = 0; d < 3; ++d) {
    m.lo[d] = 0.0;
    m.hi[d] = 1.0;
  }
  return m;
}

int main() {
  dg_options opt;
  dg_default_options(&opt);
  EXPECT(opt.equations == DG_EULER && opt.alpha_min == 0.01 && opt.alpha_max == 0.7 && opt.alpha_spread == 0.5);
  EXPECT(opt.lifting == DG_LIFT_SPLIT);
  dg_ctx* c = nullptr;
  dg_mesh m = box(2, 2, 2);
  // dg_init argument checks (no allocation happens for any of them)
  EXPECT(dg_init(&m, 3, 1.4, 0.0, nullptr) == DG_EINVAL);
  EXPECT(dg_init(nullptr, 3, 1.4, 0.0, &c) == DG_EINVAL && c == nullptr);
  EXPECT(dg_init(&m, 0, 1.4, 0.0, &c) == DG_EINVAL && c == nullptr);
  EXPECT(dg_init(&m, 8, 1.4, 0.0, &c) == DG_EINVAL && c == nullptr);
  EXPECT(dg_init(&m, 3, 1.0, 0.0, &c) == DG_EINVAL);
  EXPECT(dg_init(&m, 3, NAN, 0.0, &c) == DG_EINVAL);
  EXPECT(dg_init(&m, 3, 1.4, -1.0, &c) == DG_EINVAL);
  EXPECT(dg_init(&m, 3, 1.4, INFINITY, &c) == DG_EINVAL);
  dg_mesh bad = box(0, 2, 2);
  EXPECT(dg_init(&bad, 3, 1.4, 0.0, &c) == DG_EINVAL);
  bad = box(2, 2, 2);
  bad.hi[1] = bad.lo[1];
  EXPECT(dg_init(&bad, 3, 1.4, 0.0, &c) == DG_EINVAL);
  bad = box(1 << 10, 1 << 10, 1 << 10);
  EXPECT(dg_init(&bad, 3, 1.4, 0.0, &c) == DG_EINVAL);
  EXPECT(std::strlen(dg_last_error(nullptr)) > 0);
  // every call on a NULL context
  double s5[5], dt = 0.0, ms[5];
  int64_t l5[5], a = 0, b = 0;
  EXPECT(dg_set_options(nullptr, &opt) == DG_EINVAL);
  EXPECT(dg_get_options(nullptr, &opt) == DG_EINVAL);
  EXPECT(dg_set_stream(nullptr, nullptr) == DG_EINVAL);
  EXPECT(dg_time_derivative(nullptr, nullptr, nullptr) == DG_EINVAL);
  EXPECT(rk_step(nullptr, nullptr, 1e-3) == DG_EINVAL);
  EXPECT(dg_rk_steps(nullptr, nullptr, 1e-3, 1) == DG_EINVAL);
  EXPECT(dg_vjp(nullptr, nullptr, nullptr, nullptr) == DG_EINVAL);
  EXPECT(dg_vjp_noalloc(nullptr, nullptr, nullptr, nullptr) == DG_EINVAL);
  EXPECT(rk_step_vjp(nullptr, nullptr, 1e-3, nullptr, nullptr) == DG_EINVAL);
  EXPECT(rk_step_record(nullptr, nullptr, 1e-3, nullptr) == DG_EINVAL);
  EXPECT(rk_step_vjp_recorded(nullptr, nullptr, 1e-3, nullptr, nullptr) == DG_EINVAL);
  EXPECT(dg_max_dt(nullptr, nullptr, 0.5, &dt) == DG_EINVAL);
  EXPECT(dg_integrals(nullptr, nullptr, s5) == DG_EINVAL);
  EXPECT(dg_alpha(nullptr, nullptr, nullptr) == DG_EINVAL);
  EXPECT(dg_check_finite(nullptr, nullptr) == DG_EINVAL);
  EXPECT(dg_set_profiling(nullptr, 1) == DG_EINVAL);
  EXPECT(dg_profile_read(nullptr, ms, l5) == DG_EINVAL);
  EXPECT(dg_node_weights(nullptr, s5) == DG_EINVAL);
  EXPECT(dg_sizes(nullptr, &a, &b) == DG_EINVAL);
  EXPECT(dg_set_cs_field(nullptr, nullptr) == DG_EINVAL);
  EXPECT(dg_set_geometry(nullptr, nullptr) == DG_EINVAL);
  EXPECT(dg_set_connectivity(nullptr, nullptr) == DG_EINVAL);
  EXPECT(dg_set_wall_model(nullptr, -1, 1.0, 0.0) == DG_EINVAL);
  EXPECT(dg_finalize(nullptr) == DG_OK);
  // a valid context: every degree builds its basis and neighbour table on the
  // host; without a device the allocation fails and nothing stays behind
  for (int N = 1; N <= 7; ++N) {
    dg_mesh mm = box(3, 2, 1);
    const int rc = dg_init(&mm, N, 1.4, 1e-3, &c);
    if (rc != DG_OK) {
      EXPECT(c == nullptr && (rc == DG_ENOMEM || rc == DG_EHIP));
      EXPECT(std::strlen(dg_last_error(nullptr)) > 0);
      continue;
    }
    // with a GPU: host pointers, bad sizes and options are refused
    std::vector<double> host(size_t(6) * 5 * (N + 1) * (N + 1) * (N + 1), 1.0), hout(host.size());
    EXPECT(dg_time_derivative(c, host.data(), hout.data()) == DG_EINVAL);
    EXPECT(rk_step(c, host.data(), 1e-3) == DG_EINVAL);
    EXPECT(dg_max_dt(c, host.data(), 0.5, &dt) == DG_EINVAL);
    EXPECT(dg_set_cs_field(c, host.data()) == DG_EINVAL);
    EXPECT(dg_set_geometry(c, host.data()) == DG_EINVAL);
    EXPECT(dg_set_wall_model(c, 3, 1.0, 0.0) == DG_EINVAL);
    std::vector<int32_t> conn(size_t(6) * 18, 0);
    EXPECT(dg_set_connectivity(c, conn.data()) == DG_EINVAL);
    dg_options o = opt;
    o.Cs = -1.0;
    EXPECT(dg_set_options(c, &o) == DG_EINVAL);
    o = opt;
    o.lifting = 2;
    EXPECT(dg_set_options(c, &o) == DG_EINVAL);
    EXPECT(dg_sizes(c, &a, &b) == DG_OK && a == 6 && b == (N + 1) * (N + 1) * (N + 1));
    EXPECT(dg_finalize(c) == DG_OK);
    c = nullptr;
  }
  if (g_fail) return 1;
  std::printf("abi_check: ok\n");
  return 0;
}
