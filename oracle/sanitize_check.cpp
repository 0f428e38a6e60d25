// Address/undefined-behaviour sanitizer run of the CPU oracle (TEST
// INFRASTRUCTURE, like the oracle itself).  Built by oracle.sanitize_check()
// with g++ -fsanitize=address,undefined and run as a separate program: every
// extern "C" entry point of the oracle is called on small meshes that reach
// each code path (Euler and Navier-Stokes with all volume and surface fluxes,
// the Smagorinsky model, DG/FV blending with both reconstructions, curved
// elements with structured and general connectivity, wall-modelled faces,
// the dense brute-force variant, dual-number products and rollouts, the
// indicator, the reductions).  Exits 0 when every call returns normally; the
// sanitizers abort with a report on any out-of-bounds access, use after free,
// signed overflow or other undefined behaviour.
#include "dg_oracle.cpp"

#include <cstdio>

using namespace oracle;

namespace {

int g_fail = 0;

void check(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "sanitize_check: %s failed\n", what);
    ++g_fail;
  }
}

Setup base(int N, int nx, int ny, int nz) {
  Setup s;
  std::memset(&s, 0, sizeof(s));
  s.N = N;
  s.nx = nx;
  s.ny = ny;
  s.nz = nz;
  for (int d = 0; d < 3; ++d) {
    s.lo[d] = 0.0;
    s.hi[d] = 6.283185307179586;
  }
  s.gamma = 1.4;
  s.mu = 1e-2;
  s.Pr = 0.72;
  s.alpha_min = 0.01;
  s.alpha_max = 0.7;
  s.alpha_spread = 0.5;
  s.Prt = 0.9;
  s.fv_recon = FV_MINMOD;
  s.wall_dir = -1;
  return s;
}

// Smooth state with a jump in x (exercises the blending) at the nodes of the
// box mesh: rho, u, v, w, p from sines of the node coordinates.
std::vector<double> state(const Setup& s, bool jump) {
  const int n1 = s.N + 1, nn = n1 * n1 * n1, ne = s.nx * s.ny * s.nz;
  std::vector<double> xi(n1), w(n1), D(n1 * n1), Dh(n1 * n1), Vi(n1 * n1), ed(n1 + 1);
  or_basis(s.N, xi.data(), w.data(), D.data(), Dh.data(), Vi.data(), ed.data());
  std::vector<double> U(size_t(ne) * 5 * nn);
  for (int e = 0; e < ne; ++e) {
    const int ex = e % s.nx, ey = (e / s.nx) % s.ny, ez = e / (s.nx * s.ny);
    for (int n = 0; n < nn; ++n) {
      const int i = n % n1, j = (n / n1) % n1, k = n / (n1 * n1);
      const double x = (ex + 0.5 * (xi[i] + 1.0)) * (s.hi[0] - s.lo[0]) / s.nx;
      const double y = (ey + 0.5 * (xi[j] + 1.0)) * (s.hi[1] - s.lo[1]) / s.ny;
      const double z = (ez + 0.5 * (xi[k] + 1.0)) * (s.hi[2] - s.lo[2]) / s.nz;
      double rho = 1.0 + 0.2 * std::sin(x + 2.0 * y) * std::cos(z);
      double p = 1.0 + 0.1 * std::cos(x - y + z);
      if (jump && ex >= s.nx / 2) {
        rho *= 0.25;
        p *= 0.2;
      }
      const double u = 0.3 * std::sin(y), v = -0.2 * std::cos(z + x), ww = 0.1 * std::sin(x);
      double* Ue = &U[size_t(e) * 5 * nn];
      Ue[n] = rho;
      Ue[nn + n] = rho * u;
      Ue[2 * nn + n] = rho * v;
      Ue[3 * nn + n] = rho * ww;
      Ue[4 * nn + n] = p / (s.gamma - 1.0) + 0.5 * rho * (u * u + v * v + ww * ww);
    }
  }
  return U;
}

// Operator, products, rollout and reductions of one setup.
void run_all(const Setup& s, bool jump, const char* what) {
  const int n1 = s.N + 1, nn = n1 * n1 * n1, ne = s.nx * s.ny * s.nz;
  const size_t n = size_t(ne) * 5 * nn;
  std::vector<double> U = state(s, jump), Ut(n), Vd(n), JV(n), dg(n), fv(n), al(ne);
  for (size_t i = 0; i < n; ++i) Vd[i] = std::sin(0.37 * double(i));
  check(or_time_derivative(&s, U.data(), Ut.data(), nullptr, dg.data(), fv.data(), al.data()) == 0, what);
  check(or_jvp(&s, U.data(), Vd.data(), Ut.data(), JV.data()) == 0, what);
  const double dt = 0.25 * or_max_dt(&s, U.data(), 0.5);
  check(dt > 0.0, what);
  std::vector<double> U1 = U, V1 = Vd;
  check(or_rk_steps(&s, U1.data(), dt, 2) == 0, what);
  check(or_rk_jvp(&s, U.data(), V1.data(), dt, 1) == 0, what);
  double I[5];
  check(or_integrals(&s, Ut.data(), I) == 0, what);
  if (s.N >= 2) {
    std::vector<double> E(ne), a1(ne), a(ne);
    check(or_alpha(&s, U1.data(), E.data(), a1.data(), a.data()) == 0, what);
  }
  if (s.equations == EQ_NS) {
    std::vector<double> g(size_t(ne) * 12 * nn);
    check(or_gradient(&s, U.data(), g.data()) == 0, what);
  }
  if (!s.blending && !s.xnodes) {
    const int32_t sel[2] = {0, ne - 1};
    std::vector<double> us(size_t(2) * 5 * nn);
    check(or_time_derivative_elems(&s, U.data(), sel, 2, us.data()) == 0, what);
  }
}

// Node coordinates of the box mesh displaced by a smooth periodic field.
std::vector<double> warped(const Setup& s) {
  const int n1 = s.N + 1, nn = n1 * n1 * n1, ne = s.nx * s.ny * s.nz;
  std::vector<double> xi(n1), w(n1), D(n1 * n1), Dh(n1 * n1), Vi(n1 * n1), ed(n1 + 1);
  or_basis(s.N, xi.data(), w.data(), D.data(), Dh.data(), Vi.data(), ed.data());
  std::vector<double> X(size_t(ne) * 3 * nn);
  for (int e = 0; e < ne; ++e) {
    const int ex = e % s.nx, ey = (e / s.nx) % s.ny, ez = e / (s.nx * s.ny);
    for (int q = 0; q < nn; ++q) {
      const int i = q % n1, j = (q / n1) % n1, k = q / (n1 * n1);
      const double x = (ex + 0.5 * (xi[i] + 1.0)) * 6.283185307179586 / s.nx;
      const double y = (ey + 0.5 * (xi[j] + 1.0)) * 6.283185307179586 / s.ny;
      const double z = (ez + 0.5 * (xi[k] + 1.0)) * 6.283185307179586 / s.nz;
      const double a = 0.05 * std::sin(x) * std::sin(y) * std::sin(z);
      double* Xe = &X[size_t(e) * 3 * nn];
      Xe[q] = x + a;
      Xe[nn + q] = y + 0.7 * a;
      Xe[2 * nn + q] = z - 0.5 * a;
    }
  }
  return X;
}

}  // namespace

int main() {
  or_set_threads(2);
  // basis, fluxes and closed-form helpers
  for (int N = 1; N <= 7; ++N) {
    const int n1 = N + 1;
    std::vector<double> xi(n1), w(n1), D(n1 * n1), Dh(n1 * n1), Vi(n1 * n1), ed(n1 + 1);
    check(or_basis(N, xi.data(), w.data(), D.data(), Dh.data(), Vi.data(), ed.data()) == 0, "basis");
    (void)or_threshold(N);
  }
  {
    Setup s = base(3, 1, 1, 1);
    const double a[5] = {1.0, 0.2, -0.1, 0.3, 2.6}, b[5] = {0.8, -0.1, 0.2, 0.0, 2.1};
    const double nv[3] = {0.6, 0.0, 0.8};
    double f[5];
    for (int vf = 0; vf < 4; ++vf)
      for (int sf = 0; sf < 3; ++sf) {
        s.vol_flux = vf;
        s.surf_flux = sf;
        for (int d = 0; d < 3; ++d) {
          or_two_point_flux(&s, d, a, b, f);
          or_surface_flux(&s, d, a, b, f);
          or_physical_flux(&s, d, a, f);
        }
        or_surface_flux_n(&s, nv, a, b, f);
      }
    s.equations = EQ_NS;
    s.wall_dir = 1;
    (void)or_wall_friction_velocity(&s, 1.0, 2e-5, 0.1);
    (void)or_spalding(12.0);
    double A5[5], B5[5];
    or_rk_coefficients(A5, B5);
    double Ad[4] = {-1.0, 0.5, 0.0, -2.0}, u2[2] = {1.0, 1.0};
    or_lserk4_linear(2, Ad, u2, 0.01, 3);
  }
  // Euler and Navier-Stokes, every flux pair, on the box
  for (int eq = 0; eq < 2; ++eq)
    for (int vf = 0; vf < 4; ++vf)
      for (int sf = 0; sf < 3; ++sf) {
        Setup s = base(3, 3, 2, 2);
        s.equations = eq;
        s.vol_flux = vf;
        s.surf_flux = sf;
        run_all(s, false, "box operator");
      }
  {  // dense brute force on one and two elements
    for (int nx = 1; nx <= 2; ++nx) {
      Setup s = base(2, nx, 1, 1);
      s.equations = EQ_NS;
      s.vol_flux = VF_PI;
      s.surf_flux = SF_ROE;
      std::vector<double> U = state(s, false), Ut(U.size());
      check(or_dense_time_derivative(&s, U.data(), Ut.data()) == 0, "dense");
    }
  }
  {  // Smagorinsky model, constant and per-element coefficient
    Setup s = base(3, 2, 2, 2);
    s.equations = EQ_NS;
    s.vol_flux = VF_PI;
    s.surf_flux = SF_ROE;
    s.Cs = 0.17;
    run_all(s, false, "les");
    std::vector<double> cs(8);
    for (int e = 0; e < 8; ++e) cs[e] = 0.05 + 0.02 * e;
    s.cs_elem = cs.data();
    run_all(s, false, "les per element");
  }
  for (int recon = 0; recon < 2; ++recon)  // blending, Euler and Navier-Stokes
    for (int eq = 0; eq < 2; ++eq) {
      Setup s = base(4, 6, 1, 1);
      s.blending = 1;
      s.fv_recon = recon;
      s.equations = eq;
      s.indicator = recon;
      run_all(s, true, "blended");
    }
  {  // wall-modelled faces, with the blending and with the model
    Setup s = base(3, 2, 3, 2);
    s.equations = EQ_NS;
    s.vol_flux = VF_PI;
    s.surf_flux = SF_ROE;
    s.mu = 2e-4;
    s.wall_dir = 1;
    s.wm_uinf = 1.0;
    s.wm_mainf = 0.7;
    run_all(s, false, "walls");
    s.Cs = 0.17;
    s.blending = 1;
    s.vol_flux = VF_KG;
    s.surf_flux = SF_LLF;
    run_all(s, true, "walls blended les");
  }
  {  // curved elements: structured and general connectivity (identity faces)
    Setup s = base(3, 2, 2, 2);
    s.equations = EQ_NS;
    s.vol_flux = VF_PI;
    s.surf_flux = SF_ROE;
    const std::vector<double> X = warped(s);
    s.xnodes = X.data();
    run_all(s, false, "curved");
    const int ne = 8, nn = 64;
    std::vector<double> Ja(size_t(ne) * 9 * nn), J(size_t(ne) * nn);
    check(or_metrics(&s, Ja.data(), J.data()) == 0, "metrics");
    std::vector<int32_t> nb(size_t(ne) * 6), conn(size_t(ne) * 18);
    check(or_neighbors(&s, nb.data()) == 0, "neighbours");
    for (int e = 0; e < ne; ++e)
      for (int f = 0; f < 6; ++f) {
        conn[size_t(e) * 18 + 3 * f] = nb[size_t(e) * 6 + f];
        conn[size_t(e) * 18 + 3 * f + 1] = f ^ 1;
        conn[size_t(e) * 18 + 3 * f + 2] = 0;
      }
    s.conn = conn.data();
    s.Cs = 0.1;
    run_all(s, false, "curved general connectivity");
  }
  if (g_fail) return 1;
  std::printf("sanitize_check: ok\n");
  return 0;
}
