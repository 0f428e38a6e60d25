// HIP kernels of the split-form DGSEM operator for one polynomial degree.
// This file is compiled once per degree N (1..7) with -DDG_N=<N>; each
// translation unit exports dgmi::table_N<N>() with its launchers.
//
// Work decomposition: one workgroup per element, one thread per node
// ((N+1)^3 nodes, rounded up to whole 64-wide wavefronts).  The element's
// state is staged through LDS as primitive variables; face fluxes are
// computed by the workgroup for all six faces of its element from its own
// face layer and the neighbour's (read from global memory, mostly L2/MALL
// hits), so no second kernel or face buffer is needed for the advective part.
// Both elements sharing a face evaluate f*(U-, U+) with the same operand
// order and the same code, which gives bitwise-identical interface fluxes and
// hence discrete conservation to round-off.
//
// Equations (paper: Blind et al., FLEXI; Sec. 2 and Sec. 4.1 for the split
// form on LGL nodes and the DG/FV blend, Sec. 4.2 for the alpha bounds):
//   advective:  U_t = -sum_d (2/dx_d) [ sum_l Dhat_{i_d l} F#_d(U_n, U_l)
//                         + (1/w_{i_d}) (delta_{i_d N} f*_+ - delta_{i_d 0} f*_-) ]
//   viscous (BR1): g_d' = (2/dx_d') [ sum_l Dw_{i l} q_l + (1/w_i)(delta_iN q*_+ - delta_i0 q*_-) ]
//               U_t += sum_d (2/dx_d) [ sum_l Dw_{i_d l} Fv_{d,l} + (1/w)(delta_N Fv*_+ - delta_0 Fv*_-) ]
//   with Dw = D - W^-1 B (strong form with the boundary term folded in).
//   blend:      U_t = (1 - a) U_t^DG + a U_t^FV.
#include "dg_internal.hpp"

#ifndef DG_N
#error "compile with -DDG_N=<polynomial degree>"
#endif

namespace dgmi {
namespace {

constexpr int N = DG_N;
constexpr int n1 = N + 1;
constexpr int nn = n1 * n1 * n1;
constexpr int nf = n1 * n1;
constexpr int NT = ((nn + 63) / 64) * 64;
// smallest power of two >= NT (tree reductions over NT threads)
constexpr int NTP2 = NT <= 64 ? 64 : (NT <= 128 ? 128 : (NT <= 256 ? 256 : 512));
constexpr BasisLayout BL(n1);
constexpr int NB_STAGE = 2 * n1 * n1 + 3 * n1 + 1;  // Dhat, Dw, winv, xi, edge

enum { VF_KG = 0, VF_PI = 1, VF_CH = 2, VF_STD = 3 };
enum { SF_LLF = 0, SF_ROE = 1, SF_CENTRAL = 2 };

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of elements so that x/y/z neighbours share its L2.
__device__ __forceinline__ int element_of_block(int b, int chunk) { return (b & 7) * chunk + (b >> 3); }

__device__ __forceinline__ int face_node(int d, int l, int a) {
  const int t1 = a % n1, t2 = a / n1;
  return d == 0 ? l + n1 * t1 + nf * t2 : (d == 1 ? t1 + n1 * l + nf * t2 : t1 + n1 * t2 + nf * l);
}

// ---------------------------------------------------------------------------
// Pointwise physics
// ---------------------------------------------------------------------------
// Primitive set kept per node: rho, u, v, w, p, x, theta with x = e (KG),
// h (PI, STD) or beta = rho / (2p) (CH); theta = p / rho (Navier-Stokes).
template <int VF>
__device__ __forceinline__ void primitives(const double U[5], double gm1, double P[7]) {
  const double rho = U[0];
  const double ir = 1.0 / rho;
  const double vx = U[1] * ir, vy = U[2] * ir, vz = U[3] * ir;
  const double p = gm1 * (U[4] - 0.5 * (U[1] * vx + U[2] * vy + U[3] * vz));
  P[0] = rho; P[1] = vx; P[2] = vy; P[3] = vz; P[4] = p;
  if (VF == VF_KG) P[5] = U[4] * ir;
  else if (VF == VF_CH) P[5] = 0.5 * rho / p;
  else P[5] = (U[4] + p) * ir;
  P[6] = p * ir;
}

__device__ __forceinline__ double logmean(double a, double b) {
  const double zeta = a / b;
  const double f = (zeta - 1.0) / (zeta + 1.0);
  const double u = f * f;
  const double F = (u < 1e-4) ? 1.0 + u * (1.0 / 3.0 + u * (1.0 / 5.0 + u * (1.0 / 7.0))) : log(zeta) / (2.0 * f);
  return (a + b) / (2.0 * F);
}

// Two-point flux in a frame rotated so that the normal velocity is component 0.
// Inputs: rho, (un, ut1, ut2), p, E of both states; output (f_rho, f_mn, f_mt1, f_mt2, f_E).
template <int VF>
__device__ __forceinline__ void twopoint_rot(const double ra, const double ua[3], const double pa, const double Ea,
                                             const double rb, const double ub[3], const double pb, const double Eb,
                                             double gm1, double f[5]) {
  if (VF == VF_STD) {
    const double ha = (Ea + pa) / ra, hb = (Eb + pb) / rb;
    const double ma = ra * ua[0], mb = rb * ub[0];
    f[0] = 0.5 * (ma + mb);
    f[1] = 0.5 * (ma * ua[0] + pa + mb * ub[0] + pb);
    f[2] = 0.5 * (ma * ua[1] + mb * ub[1]);
    f[3] = 0.5 * (ma * ua[2] + mb * ub[2]);
    f[4] = 0.5 * (ma * ha + mb * hb);
    return;
  }
  const double um0 = 0.5 * (ua[0] + ub[0]), um1 = 0.5 * (ua[1] + ub[1]), um2 = 0.5 * (ua[2] + ub[2]);
  if (VF == VF_KG || VF == VF_PI) {
    const double rm = 0.5 * (ra + rb), pm = 0.5 * (pa + pb);
    const double fr = rm * um0;
    f[0] = fr;
    f[1] = fr * um0 + pm;
    f[2] = fr * um1;
    f[3] = fr * um2;
    if (VF == VF_KG) f[4] = fr * (0.5 * (Ea / ra + Eb / rb)) + pm * um0;
    else f[4] = fr * (0.5 * ((Ea + pa) / ra + (Eb + pb) / rb));
    return;
  }
  // Chandrashekar (entropy conservative)
  const double ba = ra / (2.0 * pa), bb = rb / (2.0 * pb);
  const double rln = logmean(ra, rb), bln = logmean(ba, bb);
  const double rm = 0.5 * (ra + rb), bm = 0.5 * (ba + bb);
  const double fr = rln * um0;
  f[0] = fr;
  f[1] = fr * um0 + rm / (2.0 * bm);
  f[2] = fr * um1;
  f[3] = fr * um2;
  const double usq = 0.5 * (ua[0] * ua[0] + ua[1] * ua[1] + ua[2] * ua[2] + ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
  f[4] = fr * (1.0 / (2.0 * gm1 * bln) - 0.5 * usq) + um0 * f[1] + um1 * f[2] + um2 * f[3];
}

// Surface flux f*_D(L, R) = F#_D(L, R) - Dis/2 of conservative states; the
// Riemann solver is chosen at run time (uniform across the workgroup).
template <int VF, int D>
__device__ __forceinline__ void surface_flux(int sf, const double L[5], const double R[5], double gamma,
                                             double f[5]) {
  constexpr int kn = 1 + D, k1 = 1 + (D + 1) % 3, k2 = 1 + (D + 2) % 3;  // (n, t1, t2) cyclic
  const double gm1 = gamma - 1.0;
  const double mLn = L[kn], mL1 = L[k1], mL2 = L[k2];
  const double mRn = R[kn], mR1 = R[k1], mR2 = R[k2];
  const double rL = L[0], rR = R[0];
  const double iL = 1.0 / rL, iR = 1.0 / rR;
  const double uL[3] = {mLn * iL, mL1 * iL, mL2 * iL};
  const double uR[3] = {mRn * iR, mR1 * iR, mR2 * iR};
  const double pL = gm1 * (L[4] - 0.5 * (mLn * uL[0] + mL1 * uL[1] + mL2 * uL[2]));
  const double pR = gm1 * (R[4] - 0.5 * (mRn * uR[0] + mR1 * uR[1] + mR2 * uR[2]));
  double g[5];
  twopoint_rot<VF>(rL, uL, pL, L[4], rR, uR, pR, R[4], gm1, g);
  if (sf == SF_LLF) {
    const double cL = sqrt(gamma * pL * iL), cR = sqrt(gamma * pR * iR);
    const double lam = fmax(fabs(uL[0]) + cL, fabs(uR[0]) + cR);
    const double hl = 0.5 * lam;
    g[0] -= hl * (rR - rL);
    g[1] -= hl * (mRn - mLn);
    g[2] -= hl * (mR1 - mL1);
    g[3] -= hl * (mR2 - mL2);
    g[4] -= hl * (R[4] - L[4]);
  } else if (sf == SF_ROE) {
    const double sL = sqrt(rL), sR = sqrt(rR);
    const double inv = 1.0 / (sL + sR);
    const double ut0 = (sL * uL[0] + sR * uR[0]) * inv;
    const double ut1 = (sL * uL[1] + sR * uR[1]) * inv;
    const double ut2 = (sL * uL[2] + sR * uR[2]) * inv;
    const double HL = (L[4] + pL) * iL, HR = (R[4] + pR) * iR;
    const double Ht = (sL * HL + sR * HR) * inv;
    const double rt = sL * sR;
    const double q2 = ut0 * ut0 + ut1 * ut1 + ut2 * ut2;
    const double c2 = gm1 * (Ht - 0.5 * q2);
    const double ct = sqrt(c2);
    const double drho = rR - rL, dp = pR - pL;
    const double dun = uR[0] - uL[0], dt1 = uR[1] - uL[1], dt2 = uR[2] - uL[2];
    const double i2c2 = 1.0 / (2.0 * c2);
    const double a1 = (dp - rt * ct * dun) * i2c2;
    const double a5 = (dp + rt * ct * dun) * i2c2;
    const double a2 = drho - dp / c2;
    const double l1 = fabs(ut0 - ct), l5 = fabs(ut0 + ct), l2 = fabs(ut0);
    const double w1 = l1 * a1, w5 = l5 * a5;
    const double D0 = w1 + w5 + l2 * a2;
    const double Dn = w1 * (ut0 - ct) + w5 * (ut0 + ct) + l2 * (a2 * ut0);
    const double D1 = w1 * ut1 + w5 * ut1 + l2 * (a2 * ut1 + rt * dt1);
    const double D2 = w1 * ut2 + w5 * ut2 + l2 * (a2 * ut2 + rt * dt2);
    const double D4 = w1 * (Ht - ct * ut0) + w5 * (Ht + ct * ut0) + l2 * (a2 * 0.5 * q2 + rt * (ut1 * dt1 + ut2 * dt2));
    g[0] -= 0.5 * D0;
    g[1] -= 0.5 * Dn;
    g[2] -= 0.5 * D1;
    g[3] -= 0.5 * D2;
    g[4] -= 0.5 * D4;
  }
  f[0] = g[0];
  f[kn] = g[1];
  f[k1] = g[2];
  f[k2] = g[3];
  f[4] = g[4];
}

// Direction given as a (loop-unrolled) constant: dispatch to the specialised flux.
template <int VF>
__device__ __forceinline__ void surface_flux_dir(int d, int sf, const double L[5], const double R[5], double gamma,
                                                 double f[5]) {
  if (d == 0) surface_flux<VF, 0>(sf, L, R, gamma, f);
  else if (d == 1) surface_flux<VF, 1>(sf, L, R, gamma, f);
  else surface_flux<VF, 2>(sf, L, R, gamma, f);
}

// ---------------------------------------------------------------------------
// Volume integral along direction D for node n (index id along D).
// ---------------------------------------------------------------------------
template <int VF, int D>
__device__ __forceinline__ void volume_dir(const double (*sP)[nn], const double* sDhat, int n, int id,
                                           const double me[7], double invJ, double gm1, double acc[5]) {
  constexpr int st = D == 0 ? 1 : (D == 1 ? n1 : nf);
  const int base = n - id * st;
  const double* crow = sDhat + id * n1;
  if (VF == VF_KG || VF == VF_PI) {
    // f_rho = fr4/4, f_m = fr4 us/8 + ps/2 e_D, f_E = fr4 xs/8 (+ ps und/4 for KG)
    // with sums s = a + b and fr4 = rho_s und_s.
    double s_fr = 0.0, s_m0 = 0.0, s_m1 = 0.0, s_m2 = 0.0, s_p = 0.0, s_E1 = 0.0, s_E2 = 0.0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      const int m = base + l * st;
      const double c = crow[l];
      const double rs = me[0] + sP[0][m];
      const double us = me[1] + sP[1][m];
      const double vs = me[2] + sP[2][m];
      const double ws = me[3] + sP[3][m];
      const double ps = me[4] + sP[4][m];
      const double xs = me[5] + sP[5][m];
      const double und = D == 0 ? us : (D == 1 ? vs : ws);
      const double cf = c * (rs * und);
      s_fr += cf;
      s_m0 = fma(cf, us, s_m0);
      s_m1 = fma(cf, vs, s_m1);
      s_m2 = fma(cf, ws, s_m2);
      const double cp = c * ps;
      s_p += cp;
      s_E1 = fma(cf, xs, s_E1);
      if (VF == VF_KG) s_E2 = fma(cp, und, s_E2);
    }
    acc[0] -= invJ * (0.25 * s_fr);
    acc[1] -= invJ * (0.125 * s_m0 + (D == 0 ? 0.5 * s_p : 0.0));
    acc[2] -= invJ * (0.125 * s_m1 + (D == 1 ? 0.5 * s_p : 0.0));
    acc[3] -= invJ * (0.125 * s_m2 + (D == 2 ? 0.5 * s_p : 0.0));
    acc[4] -= invJ * (0.125 * s_E1 + (VF == VF_KG ? 0.25 * s_E2 : 0.0));
  } else if (VF == VF_STD) {
    // F# = (F(a) + F(b))/2 with F_rho = rho u_D, F_m = rho u_D u + p e_D, F_E = rho h u_D
    const double mA = me[0] * me[1 + D];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0, sp = 0.0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      const int m = base + l * st;
      const double c = crow[l];
      const double mB = sP[0][m] * sP[1 + D][m];
      s0 = fma(c, mA + mB, s0);
      s1 = fma(c, mA * me[1] + mB * sP[1][m], s1);
      s2 = fma(c, mA * me[2] + mB * sP[2][m], s2);
      s3 = fma(c, mA * me[3] + mB * sP[3][m], s3);
      sp = fma(c, me[4] + sP[4][m], sp);
      s4 = fma(c, mA * me[5] + mB * sP[5][m], s4);
    }
    acc[0] -= invJ * (0.5 * s0);
    acc[1] -= invJ * (0.5 * (s1 + (D == 0 ? sp : 0.0)));
    acc[2] -= invJ * (0.5 * (s2 + (D == 1 ? sp : 0.0)));
    acc[3] -= invJ * (0.5 * (s3 + (D == 2 ? sp : 0.0)));
    acc[4] -= invJ * (0.5 * s4);
  } else {
    // Chandrashekar: general pairwise evaluation (test flux)
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      const int m = base + l * st;
      const double c = crow[l];
      const double ua[3] = {me[1 + D], me[1 + (D + 1) % 3], me[1 + (D + 2) % 3]};
      const double ub[3] = {sP[1 + D][m], sP[1 + (D + 1) % 3][m], sP[1 + (D + 2) % 3][m]};
      double f[5];
      twopoint_rot<VF_CH>(me[0], ua, me[4], 0.0, sP[0][m], ub, sP[4][m], 0.0, gm1, f);
      s[0] = fma(c, f[0], s[0]);
      s[1 + D] = fma(c, f[1], s[1 + D]);
      s[1 + (D + 1) % 3] = fma(c, f[2], s[1 + (D + 1) % 3]);
      s[1 + (D + 2) % 3] = fma(c, f[3], s[1 + (D + 2) % 3]);
      s[4] = fma(c, f[4], s[4]);
    }
    for (int v = 0; v < 5; ++v) acc[v] -= invJ * s[v];
  }
}

// ---------------------------------------------------------------------------
// BR1 lifted gradient at node n: g[d][c] = d q_c / d x_d, q = (u, v, w, theta).
// sQ holds the interface values q* on the six faces of the element.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lifted_gradient(const double (*sP)[nn], const double (*sQ)[4][nf], const double* sDw,
                                                const double* swinv, int n, const int ijk[3], const double invJ[3],
                                                double g[3][4]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
    const int id = ijk[d];
    const int base = n - id * st;
    const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
    const double* crow = sDw + id * n1;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      const int m = base + l * st;
      const double c = crow[l];
      s0 = fma(c, sP[1][m], s0);
      s1 = fma(c, sP[2][m], s1);
      s2 = fma(c, sP[3][m], s2);
      s3 = fma(c, sP[6][m], s3);
    }
    if (id == N) {
      const double wN = swinv[N];
      s0 = fma(wN, sQ[2 * d + 1][0][a], s0);
      s1 = fma(wN, sQ[2 * d + 1][1][a], s1);
      s2 = fma(wN, sQ[2 * d + 1][2][a], s2);
      s3 = fma(wN, sQ[2 * d + 1][3][a], s3);
    }
    if (id == 0) {
      const double w0 = swinv[0];
      s0 = fma(-w0, sQ[2 * d][0][a], s0);
      s1 = fma(-w0, sQ[2 * d][1][a], s1);
      s2 = fma(-w0, sQ[2 * d][2][a], s2);
      s3 = fma(-w0, sQ[2 * d][3][a], s3);
    }
    g[d][0] = invJ[d] * s0;
    g[d][1] = invJ[d] * s1;
    g[d][2] = invJ[d] * s2;
    g[d][3] = invJ[d] * s3;
  }
}

// Viscous flux in direction d (momentum x, y, z and energy components):
// tau = mu (grad u + grad u^T - 2/3 div u I), F_E = u . tau_d + kappa dtheta/dx_d.
template <int D>
__device__ __forceinline__ void viscous_flux(const double g[3][4], double vx, double vy, double vz, double mu,
                                             double kappa, double F[4]) {
  const double div = g[0][0] + g[1][1] + g[2][2];
  const double dv = (2.0 / 3.0) * mu * div;
  F[0] = mu * (g[D][0] + g[0][D]) - (D == 0 ? dv : 0.0);
  F[1] = mu * (g[D][1] + g[1][D]) - (D == 1 ? dv : 0.0);
  F[2] = mu * (g[D][2] + g[2][D]) - (D == 2 ? dv : 0.0);
  F[3] = vx * F[0] + vy * F[1] + vz * F[2] + kappa * g[D][3];
}

__device__ __forceinline__ double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return a > 0.0 ? fmin(a, b) : fmax(a, b);
}

// Reconstructed face states of FV subcell m along a line (primitive w = rho,u,v,w,p):
// slopes by minmod of divided differences between node positions for interior
// subcells (outer subcells first order), first-order fallback if a face state
// has rho <= 0 or p <= 0.  Returns the state at the right (plus) or left face.
__device__ __forceinline__ void subcell_face_state(const double (*sP)[nn], int base, int st, int m, bool right,
                                                   int recon, const double* sxi, const double* sedge, double w[5]) {
  const int mm = base + m * st;
  double c[5];
  const int pidx[5] = {0, 1, 2, 3, 4};
#pragma unroll
  for (int v = 0; v < 5; ++v) c[v] = sP[pidx[v]][mm];
  if (recon == 1 && m >= 1 && m <= N - 1) {
    double sg[5];
    const double hl = 1.0 / (sxi[m] - sxi[m - 1]);
    const double hr = 1.0 / (sxi[m + 1] - sxi[m]);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double wl = sP[v][mm - st], wr = sP[v][mm + st];
      sg[v] = minmod((c[v] - wl) * hl, (wr - c[v]) * hr);
    }
    const double dp = sedge[m + 1] - sxi[m], dm = sedge[m] - sxi[m];
    const bool ok = (c[0] + sg[0] * dp > 0.0) && (c[4] + sg[4] * dp > 0.0) && (c[0] + sg[0] * dm > 0.0) &&
                    (c[4] + sg[4] * dm > 0.0);
    if (ok) {
      const double dx = right ? dp : dm;
#pragma unroll
      for (int v = 0; v < 5; ++v) c[v] = c[v] + sg[v] * dx;
    }
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) w[v] = c[v];
}

__device__ __forceinline__ void prim_to_cons(const double w[5], double gm1, double U[5]) {
  U[0] = w[0];
  U[1] = w[0] * w[1];
  U[2] = w[0] * w[2];
  U[3] = w[0] * w[3];
  U[4] = w[4] / gm1 + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
}

// Interface values of face item q (face f, face-local index a) into LDS:
// advective f* and, for Navier-Stokes, q* = (q- + q+)/2.  D = f / 2.
template <int VF, bool NS, int D>
__device__ __forceinline__ void face_item(const StageArgs& A, int e, const double* Ue, int q, double (*sF)[5][nf],
                                          double (*sQ)[4][nf]) {
  const int f = q / nf;
  const int a = q - f * nf;
  const int side = f & 1;
  const int nb = A.nbr[6 * e + f];
  const double* Un = A.U + (size_t)nb * 5 * nn;
  const int nown = face_node(D, side ? N : 0, a);
  const int nnb = face_node(D, side ? 0 : N, a);
  double L[5], R[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double xo = Ue[v * nn + nown];
    const double xn = Un[v * nn + nnb];
    L[v] = side ? xo : xn;
    R[v] = side ? xn : xo;
  }
  double fs[5];
  surface_flux<VF, D>(A.sf, L, R, A.gamma, fs);
#pragma unroll
  for (int v = 0; v < 5; ++v) sF[f][v][a] = fs[v];
  if (NS) {
    double PL[7], PR[7];
    primitives<VF>(L, A.gamma - 1.0, PL);
    primitives<VF>(R, A.gamma - 1.0, PR);
    sQ[f][0][a] = 0.5 * (PL[1] + PR[1]);
    sQ[f][1][a] = 0.5 * (PL[2] + PR[2]);
    sQ[f][2][a] = 0.5 * (PL[3] + PR[3]);
    sQ[f][3][a] = 0.5 * (PL[6] + PR[6]);
  }
}

// Face items 0 .. 6 nf - 1 spread over the workgroup; items of one direction
// run a direction-specialised code path.
template <int VF, bool NS>
__device__ __forceinline__ void all_face_items(const StageArgs& A, int e, const double* Ue, int t,
                                               double (*sF)[5][nf], double (*sQ)[4][nf]) {
  for (int q = t; q < 6 * nf; q += NT) {
    if (q < 2 * nf) face_item<VF, NS, 0>(A, e, Ue, q, sF, sQ);
    else if (q < 4 * nf) face_item<VF, NS, 1>(A, e, Ue, q, sF, sQ);
    else face_item<VF, NS, 2>(A, e, Ue, q, sF, sQ);
  }
}

// ---------------------------------------------------------------------------
// Stage kernel: operator (+ FV blend) and either U_t output or RK update.
// EQ: 0 Euler, 1 Navier-Stokes.
// ---------------------------------------------------------------------------
template <int VF, int EQ, bool BLEND>
__global__ __launch_bounds__(NT) void k_stage(StageArgs A) {
  constexpr bool NS = (EQ == 1);
  constexpr int NPV = NS ? 7 : 6;
  __shared__ double sB[NB_STAGE];
  __shared__ double sP[7][nn];
  __shared__ double sF[6][5][nf];
  __shared__ double sQ[NS ? 6 : 1][4][nf];
  __shared__ double sX[BLEND ? 5 : 1][BLEND ? nn : 1];
  (void)NPV;

  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const int t = threadIdx.x;
  const double gm1 = A.gamma - 1.0;
  for (int q = t; q < NB_STAGE; q += NT) sB[q] = A.basis[q];
  const double* sDhat = sB + BL.Dhat();
  const double* sDw = sB + BL.Dw();
  const double* swinv = sB + BL.winv();
  const double* sxi = sB + BL.xi();
  const double* sedge = sB + BL.edge();

  const double* Ue = A.U + (size_t)e * 5 * nn;
  double u[5], me[7];
  int ijk[3] = {0, 0, 0};
  if (t < nn) {
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = Ue[v * nn + t];
    primitives<VF>(u, gm1, me);
#pragma unroll
    for (int k = 0; k < 7; ++k)
      if (k < 6 || NS) sP[k][t] = me[k];
    ijk[0] = t % n1;
    ijk[1] = (t / n1) % n1;
    ijk[2] = t / nf;
  }
  all_face_items<VF, NS>(A, e, Ue, t, sF, sQ);
  __syncthreads();

  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double Fv[3][4];
  if (t < nn) {
    volume_dir<VF, 0>(sP, sDhat, t, ijk[0], me, A.invJ[0], gm1, acc);
    volume_dir<VF, 1>(sP, sDhat, t, ijk[1], me, A.invJ[1], gm1, acc);
    volume_dir<VF, 2>(sP, sDhat, t, ijk[2], me, A.invJ[2], gm1, acc);
    // advective surface terms
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int id = ijk[d];
      const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
      if (id == N) {
        const double c = A.invJ[d] * swinv[N];
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] -= c * sF[2 * d + 1][v][a];
      }
      if (id == 0) {
        const double c = A.invJ[d] * swinv[0];
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] += c * sF[2 * d][v][a];
      }
    }
    if (NS) {
      double g[3][4];
      lifted_gradient(sP, sQ, sDw, swinv, t, ijk, A.invJ, g);
      viscous_flux<0>(g, me[1], me[2], me[3], A.mu, A.kappa, Fv[0]);
      viscous_flux<1>(g, me[1], me[2], me[3], A.mu, A.kappa, Fv[1]);
      viscous_flux<2>(g, me[1], me[2], me[3], A.mu, A.kappa, Fv[2]);
    }
  }

  if (BLEND) {
    double al = 0.0;
    {
      double m = 0.0;
#pragma unroll
      for (int f = 0; f < 6; ++f) m = fmax(m, A.alpha1[A.nbr[6 * e + f]]);
      al = fmax(A.alpha1[e], A.aspread * m);
      if (al < A.amin) al = 0.0;
      if (t == 0 && A.alpha_out) A.alpha_out[e] = al;
    }
    if (al > 0.0) {  // uniform over the workgroup
      double fv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
        __syncthreads();
        if (t < nn && ijk[d] < N) {
          const int base = t - ijk[d] * st;
          double wl[5], wr[5], UL[5], UR[5], fs[5];
          subcell_face_state(sP, base, st, ijk[d], true, A.recon, sxi, sedge, wl);
          subcell_face_state(sP, base, st, ijk[d] + 1, false, A.recon, sxi, sedge, wr);
          prim_to_cons(wl, gm1, UL);
          prim_to_cons(wr, gm1, UR);
          surface_flux_dir<VF>(d, A.sf, UL, UR, A.gamma, fs);
#pragma unroll
          for (int v = 0; v < 5; ++v) sX[v][t] = fs[v];
        }
        __syncthreads();
        if (t < nn) {
          const int id = ijk[d];
          const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
          const double c = A.invJ[d] * swinv[id];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const double Fr = (id == N) ? sF[2 * d + 1][v][a] : sX[v][t];
            const double Fl = (id == 0) ? sF[2 * d][v][a] : sX[v][t - st];
            fv[v] -= c * (Fr - Fl);
          }
        }
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[v] = (1.0 - al) * acc[v] + al * fv[v];
    }
  }

  if (NS) {
    // viscous divergence, one direction at a time through LDS (reuses sP)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      __syncthreads();
      if (t < nn) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sP[c][t] = Fv[d][c];
      }
      __syncthreads();
      if (t < nn) {
        const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
        const int id = ijk[d];
        const int base = t - id * st;
        const double* crow = sDw + id * n1;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int l = 0; l < n1; ++l) {
          const int m = base + l * st;
          const double c = crow[l];
          s0 = fma(c, sP[0][m], s0);
          s1 = fma(c, sP[1][m], s1);
          s2 = fma(c, sP[2][m], s2);
          s3 = fma(c, sP[3][m], s3);
        }
        const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
        if (id == N) {
          const int nb = A.nbr[6 * e + 2 * d + 1];
          const double* Fn = A.Fvf + ((size_t)nb * 6 + 2 * d) * 4 * nf;
          const double wN = swinv[N];
          s0 = fma(wN, 0.5 * (Fv[d][0] + Fn[0 * nf + a]), s0);
          s1 = fma(wN, 0.5 * (Fv[d][1] + Fn[1 * nf + a]), s1);
          s2 = fma(wN, 0.5 * (Fv[d][2] + Fn[2 * nf + a]), s2);
          s3 = fma(wN, 0.5 * (Fv[d][3] + Fn[3 * nf + a]), s3);
        }
        if (id == 0) {
          const int nb = A.nbr[6 * e + 2 * d];
          const double* Fn = A.Fvf + ((size_t)nb * 6 + 2 * d + 1) * 4 * nf;
          const double w0 = swinv[0];
          s0 = fma(-w0, 0.5 * (Fv[d][0] + Fn[0 * nf + a]), s0);
          s1 = fma(-w0, 0.5 * (Fv[d][1] + Fn[1 * nf + a]), s1);
          s2 = fma(-w0, 0.5 * (Fv[d][2] + Fn[2 * nf + a]), s2);
          s3 = fma(-w0, 0.5 * (Fv[d][3] + Fn[3 * nf + a]), s3);
        }
        acc[1] = fma(A.invJ[d], s0, acc[1]);
        acc[2] = fma(A.invJ[d], s1, acc[2]);
        acc[3] = fma(A.invJ[d], s2, acc[3]);
        acc[4] = fma(A.invJ[d], s3, acc[4]);
      }
    }
  }

  if (t < nn) {
    const size_t o = (size_t)e * 5 * nn + t;
    if (A.mode == MODE_UT) {
#pragma unroll
      for (int v = 0; v < 5; ++v) A.Ut[o + v * nn] = acc[v];
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        double gv = acc[v];
        if (A.A != 0.0) gv = A.A * A.G[o + v * nn] + acc[v];
        if (A.writeG) A.G[o + v * nn] = gv;
        A.Uout[o + v * nn] = u[v] + A.Bdt * gv;
      }
    }
  }
}

// Normal viscous flux at face node q of the element (face f = q / nf, D = f / 2).
template <int D>
__device__ __forceinline__ void lift_face_node(const StageArgs& A, int e, int q, const double (*sP)[nn],
                                               const double (*sQ)[4][nf], const double* sB) {
  const int f = q / nf;
  const int a = q - f * nf;
  const int n = face_node(D, (f & 1) ? N : 0, a);
  const int ijk[3] = {n % n1, (n / n1) % n1, n / nf};
  double g[3][4], F[4];
  lifted_gradient(sP, sQ, sB + BL.Dw(), sB + BL.winv(), n, ijk, A.invJ, g);
  viscous_flux<D>(g, sP[1][n], sP[2][n], sP[3][n], A.mu, A.kappa, F);
  double* out = A.Fvf + ((size_t)e * 6 + f) * 4 * nf;
#pragma unroll
  for (int c = 0; c < 4; ++c) out[c * nf + a] = F[c];
}

// ---------------------------------------------------------------------------
// BR1 lifting pass (Navier-Stokes): normal viscous flux at the element's own
// face nodes -> Fvf[e][f][c][a], read by the neighbours' stage kernels.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_lift(StageArgs A) {
  __shared__ double sB[NB_STAGE];
  __shared__ double sP[7][nn];
  __shared__ double sF[1][5][nf];
  __shared__ double sQ[6][4][nf];
  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const int t = threadIdx.x;
  const double gm1 = A.gamma - 1.0;
  for (int q = t; q < NB_STAGE; q += NT) sB[q] = A.basis[q];
  const double* Ue = A.U + (size_t)e * 5 * nn;
  if (t < nn) {
    double u[5], P[7];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = Ue[v * nn + t];
    primitives<VF_PI>(u, gm1, P);
#pragma unroll
    for (int k = 0; k < 7; ++k) sP[k][t] = P[k];
  }
  for (int q = t; q < 6 * nf; q += NT) {
    const int f = q / nf;
    const int a = q - f * nf;
    const int d = f >> 1;
    const int side = f & 1;
    const int nb = A.nbr[6 * e + f];
    const double* Un = A.U + (size_t)nb * 5 * nn;
    const int nown = face_node(d, side ? N : 0, a);
    const int nnb = face_node(d, side ? 0 : N, a);
    double L[5], R[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double xo = Ue[v * nn + nown];
      const double xn = Un[v * nn + nnb];
      L[v] = side ? xo : xn;
      R[v] = side ? xn : xo;
    }
    double PL[7], PR[7];
    primitives<VF_PI>(L, gm1, PL);
    primitives<VF_PI>(R, gm1, PR);
    sQ[f][0][a] = 0.5 * (PL[1] + PR[1]);
    sQ[f][1][a] = 0.5 * (PL[2] + PR[2]);
    sQ[f][2][a] = 0.5 * (PL[3] + PR[3]);
    sQ[f][3][a] = 0.5 * (PL[6] + PR[6]);
  }
  __syncthreads();
  (void)sF;
  for (int q = t; q < 6 * nf; q += NT) {
    if (q < 2 * nf) lift_face_node<0>(A, e, q, sP, sQ, sB);
    else if (q < 4 * nf) lift_face_node<1>(A, e, q, sP, sQ, sB);
    else lift_face_node<2>(A, e, q, sP, sQ, sB);
  }
}

// ---------------------------------------------------------------------------
// Modal indicator -> clipped blending coefficient a1 per element (FP64).
// q = rho p; qhat = (Vinv x Vinv x Vinv) q on orthonormal Legendre modes;
// E_N = energy of modes with max index N over all; E_{N-1} likewise over the
// modes up to N-1; E = max (or E_N only); a0 = 1/(1 + exp(-s/T (E - T)));
// a1 = min(a0, a_max), 0 below a_min.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_alpha1(StageArgs A) {
  __shared__ double sV[nf];
  __shared__ double sq[nn];
  __shared__ double st[nn];
  __shared__ double sred[3][NT];
  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const int t = threadIdx.x;
  for (int q = t; q < nf; q += NT) sV[q] = A.basis[BL.Vinv() + q];
  const double* Ue = A.U + (size_t)e * 5 * nn;
  const double gm1 = A.gamma - 1.0;
  int ijk[3] = {0, 0, 0};
  if (t < nn) {
    double u[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = Ue[v * nn + t];
    const double ir = 1.0 / u[0];
    const double p = gm1 * (u[4] - 0.5 * ir * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]));
    sq[t] = u[0] * p;
    ijk[0] = t % n1;
    ijk[1] = (t / n1) % n1;
    ijk[2] = t / nf;
  }
  __syncthreads();
  if (t < nn) {  // x: st[a,j,k] = sum_i Vinv[a][i] q[i,j,k]
    const int base = t - ijk[0];
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < n1; ++i) s = fma(sV[ijk[0] * n1 + i], sq[base + i], s);
    st[t] = s;
  }
  __syncthreads();
  if (t < nn) {  // y
    const int base = t - ijk[1] * n1;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < n1; ++j) s = fma(sV[ijk[1] * n1 + j], st[base + j * n1], s);
    sq[t] = s;
  }
  __syncthreads();
  double e2 = 0.0;
  int mx = 0;
  if (t < nn) {  // z
    const int base = t - ijk[2] * nf;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < n1; ++k) s = fma(sV[ijk[2] * n1 + k], sq[base + k * nf], s);
    e2 = s * s;
    mx = max(ijk[0], max(ijk[1], ijk[2]));
  }
  sred[0][t] = e2;
  sred[1][t] = (mx == N) ? e2 : 0.0;
  sred[2][t] = (mx == N - 1) ? e2 : 0.0;
  __syncthreads();
  for (int h = NTP2 / 2; h > 0; h >>= 1) {
    if (t < h && t + h < NT) {
      sred[0][t] += sred[0][t + h];
      sred[1][t] += sred[1][t + h];
      sred[2][t] += sred[2][t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double S = sred[0][0], SN = sred[1][0], SN1 = sred[2][0];
    const double EN = S > 0.0 ? SN / S : 0.0;
    const double rest = S - SN;
    const double EN1 = rest > 0.0 ? SN1 / rest : 0.0;
    const double E = A.indicator == 1 ? EN : fmax(EN, EN1);
    const double a0 = 1.0 / (1.0 + exp(-(A.sharp / A.thresh) * (E - A.thresh)));
    double a1 = fmin(a0, A.amax);
    if (a1 < A.amin) a1 = 0.0;
    const_cast<double*>(A.alpha1)[e] = a1;
  }
}

__global__ void k_spread(StageArgs A) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= A.nelem) return;
  double m = 0.0;
  for (int f = 0; f < 6; ++f) m = fmax(m, A.alpha1[A.nbr[6 * e + f]]);
  double al = fmax(A.alpha1[e], A.aspread * m);
  if (al < A.amin) al = 0.0;
  A.alpha_out[e] = al;
}

// ---------------------------------------------------------------------------
// Reductions (grid-stride over elements, fixed order => deterministic).
// ---------------------------------------------------------------------------
constexpr int RED_BLOCKS = 1024;

__global__ __launch_bounds__(NT) void k_max_rate(ReduceArgs R) {
  __shared__ double s0[NT], s1[NT];
  const int t = threadIdx.x;
  double ma = 0.0, mv = 0.0;
  const double gm1 = R.gamma - 1.0;
  for (int e = blockIdx.x; e < R.nelem; e += gridDim.x) {
    if (t < nn) {
      const double* Ue = R.X + (size_t)e * 5 * nn;
      double u[5];
      for (int v = 0; v < 5; ++v) u[v] = Ue[v * nn + t];
      const double ir = 1.0 / u[0];
      const double vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
      const double p = gm1 * (u[4] - 0.5 * (u[1] * vx + u[2] * vy + u[3] * vz));
      const double c = sqrt(R.gamma * p * ir);
      const double ra = (fabs(vx) + c) * R.invdx[0] + (fabs(vy) + c) * R.invdx[1] + (fabs(vz) + c) * R.invdx[2];
      const double rv = R.nu_fac * ir *
                        (R.invdx[0] * R.invdx[0] + R.invdx[1] * R.invdx[1] + R.invdx[2] * R.invdx[2]);
      ma = fmax(ma, ra);
      mv = fmax(mv, rv);
    }
  }
  s0[t] = ma;
  s1[t] = mv;
  __syncthreads();
  for (int h = NTP2 / 2; h > 0; h >>= 1) {
    if (t < h && t + h < NT) {
      s0[t] = fmax(s0[t], s0[t + h]);
      s1[t] = fmax(s1[t], s1[t + h]);
    }
    __syncthreads();
  }
  if (t == 0) {
    R.partial[2 * blockIdx.x] = s0[0];
    R.partial[2 * blockIdx.x + 1] = s1[0];
  }
}

__global__ __launch_bounds__(NT) void k_integrals(ReduceArgs R) {
  __shared__ double s[5][NT];
  const int t = threadIdx.x;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double wq = 0.0;
  if (t < nn) {
    const double* w = R.basis + BL.w();
    wq = w[t % n1] * w[(t / n1) % n1] * w[t / nf] * R.Jac;
  }
  for (int e = blockIdx.x; e < R.nelem; e += gridDim.x) {
    if (t < nn) {
      const double* Xe = R.X + (size_t)e * 5 * nn;
      for (int v = 0; v < 5; ++v) acc[v] = fma(wq, Xe[v * nn + t], acc[v]);
    }
  }
  for (int v = 0; v < 5; ++v) s[v][t] = acc[v];
  __syncthreads();
  for (int h = NTP2 / 2; h > 0; h >>= 1) {
    if (t < h && t + h < NT)
      for (int v = 0; v < 5; ++v) s[v][t] += s[v][t + h];
    __syncthreads();
  }
  if (t == 0)
    for (int v = 0; v < 5; ++v) R.partial[5 * blockIdx.x + v] = s[v][0];
}

__global__ __launch_bounds__(NT) void k_nonfinite(ReduceArgs R) {
  __shared__ double s[NT];
  const int t = threadIdx.x;
  double cnt = 0.0;
  for (int e = blockIdx.x; e < R.nelem; e += gridDim.x) {
    if (t < nn) {
      const double* Xe = R.X + (size_t)e * 5 * nn;
      for (int v = 0; v < 5; ++v) cnt += isfinite(Xe[v * nn + t]) ? 0.0 : 1.0;
    }
  }
  s[t] = cnt;
  __syncthreads();
  for (int h = NTP2 / 2; h > 0; h >>= 1) {
    if (t < h && t + h < NT) s[t] += s[t + h];
    __syncthreads();
  }
  if (t == 0) R.partial[blockIdx.x] = s[0];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
inline int blocks_for(const StageArgs& A) { return 8 * A.chunk; }

template <int VF>
hipError_t launch_stage_vf(const StageArgs& A, int eq, hipStream_t s) {
  const dim3 grid(blocks_for(A)), block(NT);
  if (eq == 1) hipLaunchKernelGGL((k_stage<VF, 1, false>), grid, block, 0, s, A);
  else if (A.blend) hipLaunchKernelGGL((k_stage<VF, 0, true>), grid, block, 0, s, A);
  else hipLaunchKernelGGL((k_stage<VF, 0, false>), grid, block, 0, s, A);
  return hipGetLastError();
}

hipError_t launch_stage(const StageArgs& A, int eq, hipStream_t s) {
  switch (A.vf) {
    case VF_KG: return launch_stage_vf<VF_KG>(A, eq, s);
    case VF_PI: return launch_stage_vf<VF_PI>(A, eq, s);
    case VF_CH: return launch_stage_vf<VF_CH>(A, eq, s);
    default: return launch_stage_vf<VF_STD>(A, eq, s);
  }
}

hipError_t launch_lift(const StageArgs& A, hipStream_t s) {
  hipLaunchKernelGGL(k_lift, dim3(blocks_for(A)), dim3(NT), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_alpha1(const StageArgs& A, hipStream_t s) {
  hipLaunchKernelGGL(k_alpha1, dim3(blocks_for(A)), dim3(NT), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_spread(const StageArgs& A, hipStream_t s) {
  hipLaunchKernelGGL(k_spread, dim3((A.nelem + 255) / 256), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_max_rate(const ReduceArgs& R, hipStream_t s) {
  hipLaunchKernelGGL(k_max_rate, dim3(RED_BLOCKS), dim3(NT), 0, s, R);
  return hipGetLastError();
}

hipError_t launch_integrals(const ReduceArgs& R, hipStream_t s) {
  hipLaunchKernelGGL(k_integrals, dim3(RED_BLOCKS), dim3(NT), 0, s, R);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const ReduceArgs& R, hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite, dim3(RED_BLOCKS), dim3(NT), 0, s, R);
  return hipGetLastError();
}

const KernelTable kTable = {
    NT, launch_stage, nullptr, launch_lift, nullptr, launch_alpha1, launch_spread,
    launch_max_rate, launch_integrals, launch_nonfinite, nullptr, nullptr,
};

}  // namespace

#define DG_CAT2(a, b) a##b
#define DG_CAT(a, b) DG_CAT2(a, b)
const KernelTable* DG_CAT(table_N, DG_N)() { return &kTable; }

}  // namespace dgmi
