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
// The Navier-Stokes stage kernel is bound by LDS traffic and issue rate, not
// by HBM: the BR1 gradient is accumulated inside the split-form partner loop
// (off the diagonal Dw = Dhat / 2, so partner values and coefficients are
// shared), the twelve viscous-flux components are exchanged through LDS once,
// and all global loads of a workgroup are issued in two rounds (indices,
// state and basis; then the neighbours' face states) before any arithmetic.
//
// Equations (paper: Blind et al., FLEXI; Sec. 2 and Sec. 4.1 for the split
// form on LGL nodes and the DG/FV blend, Sec. 4.2 for the alpha bounds):
//   advective:  U_t = -sum_d (2/dx_d) [ sum_l Dhat_{i_d l} F#_d(U_n, U_l)
//                         + (1/w_{i_d}) (delta_{i_d N} f*_+ - delta_{i_d 0} f*_-) ]
//   viscous (BR1): g_d' = (2/dx_d') [ sum_l Dw_{i l} q_l + (1/w_i)(delta_iN q*_+ - delta_i0 q*_-) ]
//               U_t += sum_d (2/dx_d) [ sum_l Dw_{i_d l} Fv_{d,l} + (1/w)(delta_N Fv*_+ - delta_0 Fv*_-) ]
//   with Dw = D - W^-1 B (strong form with the boundary term folded in).
//   blend:      U_t = (1 - a) U_t^DG + a U_t^FV.
//
// Precision: every flux/derivative routine is templated on the arithmetic
// type R.  R = double is the FP64 operator.  R = float is the mixed operator:
// the state, the Runge-Kutta register and update stay FP64; node primitives,
// interface values, fluxes, derivatives and U_t accumulate in FP32 after
// subtracting a constant reference (p0, h0, theta0) from pressure, total
// enthalpy and temperature.  For the Pirozzoli (or arithmetic-mean) flux the
// shift is exact in real arithmetic: the momentum flux changes by the constant
// p0 e_d, which the operator annihilates, and the energy flux by h0 times the
// mass flux, which is added back as U_t,E += h0 U_t,rho in FP64.
#include <algorithm>

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
// Row stride of the stage kernel's node arrays in LDS: a multiple of 64
// doubles (N >= 3), so that one base address reaches every row through the
// 512-byte offset units of paired LDS reads.
constexpr int nnp = N <= 2 ? nn : ((nn + 63) / 64) * 64;
// smallest power of two >= NT (tree reductions over NT threads)
constexpr int NTP2 = NT <= 64 ? 64 : (NT <= 128 ? 128 : (NT <= 256 ? 256 : 512));
constexpr BasisLayout BL(n1);
constexpr int NB_STAGE = 2 * n1 * n1 + 3 * n1 + 1;  // Dhat, Dw, winv, xi, edge

// Tuning: minimum waves per SIMD requested from the register allocator for
// the stage kernel (0 = compiler default), and whether the volume loop skips
// the zero diagonal of Dhat.
#ifndef DG_STAGE_MIN_WAVES
#define DG_STAGE_MIN_WAVES 0
#endif
#ifndef DG_SKIP_DIAG
#define DG_SKIP_DIAG 0
#endif
// Accumulate the BR1 gradient inside the split-form volume loop, reusing its
// partner values and coefficients (1), or in a separate pass (0).  The fused
// loop is kept rolled: fully unrolled, the partner loads in flight need more
// than 200 registers.
#ifndef DG_VDIV_LINES
#define DG_VDIV_LINES 0
#endif
#ifndef DG_FUSED_GRAD
#define DG_FUSED_GRAD 1
#endif

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
// Arithmetic helpers
// ---------------------------------------------------------------------------
// FP64 reciprocal and square root: hardware approximations refined by Newton
// iterations, for positive normal arguments; within an ulp of the correctly
// rounded result at a third of the instructions of the IEEE expansions.
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ double sqrt64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  const double r = fma(-h, s, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  double d = fma(-s, s, x);
  s = fma(d, h, s);
  d = fma(-s, s, x);
  return fma(d, h, s);
}

// Square root of a non-negative argument (0 and tiny values give 0).
__device__ __forceinline__ double sqrt_nonneg(double x) { return x > 1e-300 ? sqrt64(x) : 0.0; }
__device__ __forceinline__ float sqrt_nonneg(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ __forceinline__ double rcpR(double x) { return rcp64(x); }
__device__ __forceinline__ float rcpR(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double sqrtR(double x) { return sqrt64(x); }
__device__ __forceinline__ float sqrtR(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmaR(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double absR(double a) { return fabs(a); }
__device__ __forceinline__ float absR(float a) { return fabsf(a); }
__device__ __forceinline__ double maxR(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float maxR(float a, float b) { return fmaxf(a, b); }

// Constant reference state subtracted in the mixed-precision operator
// (all zero for FP64): pressure, total enthalpy h = (E + p)/rho, theta = p/rho.
struct Ref {
  double p, h, th;
};

// Reference of the mixed operator: the state at node 0 of element 0.  Any
// constant is exact in real arithmetic; a state value keeps the shifted
// quantities small for FP32.
__device__ __forceinline__ Ref reference_state(const double* U, double gm1) {
  const double r = U[0], ir = rcp64(r);
  const double mx = U[nn], my = U[2 * nn], mz = U[3 * nn], E = U[4 * nn];
  const double p = gm1 * (E - 0.5 * ir * (mx * mx + my * my + mz * mz));
  Ref ref;
  ref.p = p;
  ref.h = (E + p) * ir;
  ref.th = p * ir;
  return ref;
}

// ---------------------------------------------------------------------------
// Pointwise physics
// ---------------------------------------------------------------------------
// Primitive set kept per node: rho, u, v, w, p, x, theta with x = e (KG),
// h (PI, STD) or beta = rho / (2p) (CH); theta = p / rho.  Computed in FP64,
// shifted by the reference (mixed) and rounded to R.
template <int VF, class R, bool MX>
__device__ __forceinline__ void primitives(const double U[5], double gm1, const Ref& ref, R P[7]) {
  const double rho = U[0];
  const double ir = rcp64(rho);
  const double vx = U[1] * ir, vy = U[2] * ir, vz = U[3] * ir;
  const double p = gm1 * (U[4] - 0.5 * (U[1] * vx + U[2] * vy + U[3] * vz));
  double x;
  if (VF == VF_KG) x = U[4] * ir;
  else if (VF == VF_CH) x = 0.5 * rho * rcp64(p);
  else x = (U[4] + p) * ir;
  const double th = p * ir;
  P[0] = (R)rho;
  P[1] = (R)vx;
  P[2] = (R)vy;
  P[3] = (R)vz;
  P[4] = (R)(MX ? p - ref.p : p);
  P[5] = (R)(MX ? x - ref.h : x);
  P[6] = (R)(MX ? th - ref.th : th);
}

__device__ __forceinline__ double logmean(double a, double b) {
  const double zeta = a * rcp64(b);
  const double f = (zeta - 1.0) * rcp64(zeta + 1.0);
  const double u = f * f;
  const double F = (u < 1e-4) ? 1.0 + u * (1.0 / 3.0 + u * (1.0 / 5.0 + u * (1.0 / 7.0))) : log(zeta) / (2.0 * f);
  return (a + b) * rcp64(2.0 * F);
}

template <int D>
struct Axes {
  static constexpr int kn = 1 + D, k1 = 1 + (D + 1) % 3, k2 = 1 + (D + 2) % 3;
};

// A state in the frame rotated to direction D: normal component first, then
// the two tangential ones in cyclic order (D+1, D+2).  p and h are shifted by
// the reference in the mixed operator; e = E/rho (KG only).
template <class R>
struct RotState {
  R r, ir, un, u1, u2, p, h, e, mn;
};

// Jumps R - L of an interface (computed in FP64, then rounded), the LLF wave
// speed and the reference enthalpy.
template <class R>
struct Jumps {
  R dr, dmn, dm1, dm2, dE, dp, dun, du1, du2, lam, h0;
};

struct State64 {
  double r, ir, un, u1, u2, p, h, e, mn, m1, m2, E;
};

template <int D>
__device__ __forceinline__ State64 state64(const double U[5], double gm1) {
  State64 s;
  s.r = U[0];
  s.ir = rcp64(U[0]);
  s.mn = U[Axes<D>::kn];
  s.m1 = U[Axes<D>::k1];
  s.m2 = U[Axes<D>::k2];
  s.E = U[4];
  s.un = s.mn * s.ir;
  s.u1 = s.m1 * s.ir;
  s.u2 = s.m2 * s.ir;
  s.p = gm1 * (s.E - 0.5 * (s.mn * s.un + s.m1 * s.u1 + s.m2 * s.u2));
  s.h = (s.E + s.p) * s.ir;
  s.e = s.E * s.ir;
  return s;
}

template <class R, bool MX>
__device__ __forceinline__ RotState<R> to_rot(const State64& s, const Ref& ref) {
  RotState<R> o;
  o.r = (R)s.r;
  o.ir = (R)s.ir;
  o.un = (R)s.un;
  o.u1 = (R)s.u1;
  o.u2 = (R)s.u2;
  o.p = (R)(MX ? s.p - ref.p : s.p);
  o.h = (R)(MX ? s.h - ref.h : s.h);
  o.e = (R)s.e;
  o.mn = (R)s.mn;
  return o;
}

// Jumps of an interface; the energy jump of the mixed operator is
// E_R - E_L - h0 (rho_R - rho_L), the jump of the shifted energy flux variable.
template <class R, bool MX>
__device__ __forceinline__ Jumps<R> jumps(const State64& L, const State64& Rt, double gamma, const Ref& ref,
                                          int sf) {
  Jumps<R> j;
  const double dr = Rt.r - L.r;
  j.dr = (R)dr;
  j.dmn = (R)(Rt.mn - L.mn);
  j.dm1 = (R)(Rt.m1 - L.m1);
  j.dm2 = (R)(Rt.m2 - L.m2);
  j.dE = (R)(MX ? (Rt.E - L.E) - ref.h * dr : Rt.E - L.E);
  j.dp = (R)(Rt.p - L.p);
  j.dun = (R)(Rt.un - L.un);
  j.du1 = (R)(Rt.u1 - L.u1);
  j.du2 = (R)(Rt.u2 - L.u2);
  j.h0 = (R)(MX ? ref.h : 0.0);
  j.lam = (R)0;
  if (sf == SF_LLF) {
    const double cL = sqrt64(gamma * L.p * L.ir), cR = sqrt64(gamma * Rt.p * Rt.ir);
    j.lam = (R)fmax(fabs(L.un) + cL, fabs(Rt.un) + cR);
  }
  return j;
}

// Two-point flux in the rotated frame: (f_rho, f_mn, f_mt1, f_mt2, f_E).
template <int VF, class R>
__device__ __forceinline__ void twopoint_rot(const RotState<R>& a, const RotState<R>& b, R gm1, R f[5]) {
  const R half = (R)0.5;
  if (VF == VF_STD) {
    f[0] = half * (a.mn + b.mn);
    f[1] = half * (a.mn * a.un + a.p + b.mn * b.un + b.p);
    f[2] = half * (a.mn * a.u1 + b.mn * b.u1);
    f[3] = half * (a.mn * a.u2 + b.mn * b.u2);
    f[4] = half * (a.mn * a.h + b.mn * b.h);
    return;
  }
  const R um0 = half * (a.un + b.un), um1 = half * (a.u1 + b.u1), um2 = half * (a.u2 + b.u2);
  if (VF == VF_KG || VF == VF_PI) {
    const R rm = half * (a.r + b.r), pm = half * (a.p + b.p);
    const R fr = rm * um0;
    f[0] = fr;
    f[1] = fr * um0 + pm;
    f[2] = fr * um1;
    f[3] = fr * um2;
    if (VF == VF_KG) f[4] = fr * (half * (a.e + b.e)) + pm * um0;
    else f[4] = fr * (half * (a.h + b.h));
    return;
  }
  // Chandrashekar (entropy conservative; FP64 only)
  const double ba = 0.5 * a.r * rcp64(a.p), bb = 0.5 * b.r * rcp64(b.p);
  const double rln = logmean(a.r, b.r), bln = logmean(ba, bb);
  const double rm = 0.5 * (a.r + b.r), bm = 0.5 * (ba + bb);
  const double fr = rln * um0;
  f[0] = fr;
  f[1] = fr * um0 + rm * rcp64(2.0 * bm);
  f[2] = fr * um1;
  f[3] = fr * um2;
  const double usq = 0.5 * (a.un * a.un + a.u1 * a.u1 + a.u2 * a.u2 + b.un * b.un + b.u1 * b.u1 + b.u2 * b.u2);
  f[4] = fr * (rcp64(2.0 * gm1 * bln) - 0.5 * usq) + um0 * f[1] + um1 * f[2] + um2 * f[3];
}

// Interface flux f* = F#(L, R) - Dis/2 in the rotated frame; the Riemann
// solver is chosen at run time (uniform across the workgroup).  In the mixed
// operator the energy component is that of the shifted flux, f*_E - h0 f*_rho.
template <int VF, class R>
__device__ __forceinline__ void riemann_rot(int sf, const RotState<R>& L, const RotState<R>& Rs, const Jumps<R>& J,
                                            R gamma, R g[5]) {
  const R gm1 = gamma - (R)1;
  const R half = (R)0.5;
  twopoint_rot<VF, R>(L, Rs, gm1, g);
  if (sf == SF_LLF) {
    const R hl = half * J.lam;
    g[0] -= hl * J.dr;
    g[1] -= hl * J.dmn;
    g[2] -= hl * J.dm1;
    g[3] -= hl * J.dm2;
    g[4] -= hl * J.dE;
  } else if (sf == SF_ROE) {
    const R sL = sqrtR(L.r), sR = sqrtR(Rs.r);
    const R inv = rcpR(sL + sR);
    const R ut0 = (sL * L.un + sR * Rs.un) * inv;
    const R ut1 = (sL * L.u1 + sR * Rs.u1) * inv;
    const R ut2 = (sL * L.u2 + sR * Rs.u2) * inv;
    const R Hs = (sL * L.h + sR * Rs.h) * inv;  // Roe-averaged (shifted) total enthalpy
    const R Ht = Hs + J.h0;
    const R rt = sL * sR;
    const R q2 = ut0 * ut0 + ut1 * ut1 + ut2 * ut2;
    const R c2 = gm1 * (Ht - half * q2);
    const R ct = sqrtR(c2);
    const R ic2 = rcpR(c2);
    const R a1 = half * (J.dp - rt * ct * J.dun) * ic2;
    const R a5 = half * (J.dp + rt * ct * J.dun) * ic2;
    const R a2 = J.dr - J.dp * ic2;
    const R l1 = absR(ut0 - ct), l5 = absR(ut0 + ct), l2 = absR(ut0);
    const R w1 = l1 * a1, w5 = l5 * a5;
    const R D0 = w1 + w5 + l2 * a2;
    const R Dn = w1 * (ut0 - ct) + w5 * (ut0 + ct) + l2 * (a2 * ut0);
    const R D1 = w1 * ut1 + w5 * ut1 + l2 * (a2 * ut1 + rt * J.du1);
    const R D2 = w1 * ut2 + w5 * ut2 + l2 * (a2 * ut2 + rt * J.du2);
    const R D4 = w1 * (Hs - ct * ut0) + w5 * (Hs + ct * ut0) +
                 l2 * (a2 * (half * q2 - J.h0) + rt * (ut1 * J.du1 + ut2 * J.du2));
    g[0] -= half * D0;
    g[1] -= half * Dn;
    g[2] -= half * D1;
    g[3] -= half * D2;
    g[4] -= half * D4;
  }
}

// Rotated-frame 5-vector back to (rho, x, y, z, E) order.
template <int D, class R>
__device__ __forceinline__ void unrotate(const R g[5], R f[5]) {
  f[0] = g[0];
  f[Axes<D>::kn] = g[1];
  f[Axes<D>::k1] = g[2];
  f[Axes<D>::k2] = g[3];
  f[4] = g[4];
}

// Lifted interface value q* = (q- + q+)/2, q = (u, v, w, theta), from FP64
// rotated states (theta shifted by the reference in the mixed operator).
template <int D, class R, bool MX>
__device__ __forceinline__ void interface_q(const State64& L, const State64& Rt, const Ref& ref, R q[4]) {
  double a[4], b[4];
  a[Axes<D>::kn - 1] = L.un; a[Axes<D>::k1 - 1] = L.u1; a[Axes<D>::k2 - 1] = L.u2; a[3] = L.p * L.ir;
  b[Axes<D>::kn - 1] = Rt.un; b[Axes<D>::k1 - 1] = Rt.u1; b[Axes<D>::k2 - 1] = Rt.u2; b[3] = Rt.p * Rt.ir;
  if (MX) {
    a[3] -= ref.th;
    b[3] -= ref.th;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) q[c] = (R)(0.5 * (a[c] + b[c]));
}

// FP64 surface flux f*_D(L, R) of conservative states (minus side L).
template <int VF, int D>
__device__ __forceinline__ void surface_flux(int sf, const double L[5], const double R[5], double gamma,
                                             double f[5]) {
  const Ref ref{0.0, 0.0, 0.0};
  const State64 a = state64<D>(L, gamma - 1.0), b = state64<D>(R, gamma - 1.0);
  const Jumps<double> J = jumps<double, false>(a, b, gamma, ref, sf);
  double g[5];
  riemann_rot<VF, double>(sf, to_rot<double, false>(a, ref), to_rot<double, false>(b, ref), J, gamma, g);
  unrotate<D, double>(g, f);
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
// Dhat has a zero diagonal, so partner l = id is skipped: the loop visits
// l = id + 1, ..., id + N (mod N + 1).
__device__ __forceinline__ int partner(int id, int k) {
  if (!DG_SKIP_DIAG) return k - 1;
  const int l = id + k;
  return l >= n1 ? l - n1 : l;
}
constexpr int kPartners = DG_SKIP_DIAG ? N : N + 1;

// Calls body(l, m) for the partners l of node n (index id along a line of
// stride ST starting at node base) in the order above.  ROLLED: a rolled loop
// with the partner index and node advanced incrementally (one wrap test per
// partner instead of the modulo and two address products).
template <bool ROLLED, int ST, class F>
__device__ __forceinline__ void partner_loop(int id, int n, int base, F&& body) {
  if (!DG_SKIP_DIAG) {  // every l; the zero diagonal term is evaluated too
    if (ROLLED) {
#pragma unroll 1
      for (int l = 0; l < n1; ++l) body(l, base + l * ST);
    } else {
#pragma unroll
      for (int l = 0; l < n1; ++l) body(l, base + l * ST);
    }
  } else if (ROLLED) {
    int l = id, m = n;
#pragma unroll 1
    for (int k = 1; k <= kPartners; ++k) {
      ++l;
      m += ST;
      if (l == n1) {
        l = 0;
        m = base;
      }
      body(l, m);
    }
  } else {
#pragma unroll
    for (int k = 1; k <= kPartners; ++k) {
      const int l = partner(id, k);
      body(l, base + l * ST);
    }
  }
}

// With GRAD, also returns gs[c] = sum_{l != id} Dw_{id l} q_c(l) along the line
// (q = u, v, w, theta): the off-diagonal part of the BR1 gradient, which
// reuses the partner values and coefficients the flux loop reads anyway
// (off the diagonal Dw = D = Dhat / 2 exactly).
template <int VF, int D, class R, bool GRAD = false>
__device__ __forceinline__ void volume_dir(const R (*sP)[nnp], const R* sDhat, R wb, int n, int id, const R me[7],
                                           R invJ, R gm1, R acc[5], const R* sDw = nullptr, R* gs = nullptr) {
  constexpr int st = D == 0 ? 1 : (D == 1 ? n1 : nf);
  const int base = n - id * st;
  const R* crow = sDhat + id * n1;
  R g0 = 0, g1 = 0, g2 = 0, g3 = 0;
  auto grad_acc = [&](R c, int m) {
    if (GRAD) {
      g0 = fmaR(c, sP[1][m], g0);
      g1 = fmaR(c, sP[2][m], g1);
      g2 = fmaR(c, sP[3][m], g2);
      g3 = fmaR(c, sP[6][m], g3);
    }
  };
  if (VF == VF_KG || VF == VF_PI) {
    // Per partner l the pair weight a_l = c_l (rho_n + rho_l)(und_n + und_l);
    // the node's own factor of each product is taken out of the sum:
    //   sum_l a_l (u_n + u_l) = u_n sum_l a_l + sum_l a_l u_l   (u, v, w, x),
    //   sum_l c_l (p_n + p_l) = p_n rowsum + sum_l c_l p_l,
    // rowsum = sum_l Dhat_{id l} (1/w_0 in row 0, -1/w_N in row N, 0 inside).
    // Then f_rho = A/4, f_m = (u_n A + s_u)/8 + P/2 e_D, f_E = (x_n A + s_x)/8
    // (+ sum_l c_l (p_n + p_l)(und_n + und_l)/4 for KG).  Every partner
    // including l = id (Dhat has a zero diagonal) is visited with a
    // compile-time offset from the line start.
    const R und_n = me[1 + D];
    R s_A = 0, s_u = 0, s_v = 0, s_w = 0, s_x = 0, s_p = 0, s_E2 = 0;
    auto pair = [&](int l, int m) {
      const R c = crow[l];
      grad_acc(c, m);
      const R rl = sP[0][m], ul = sP[1][m], vl = sP[2][m], wl = sP[3][m], pl = sP[4][m], xl = sP[5][m];
      const R undl = D == 0 ? ul : (D == 1 ? vl : wl);
      const R unds = und_n + undl;
      const R a = c * ((me[0] + rl) * unds);
      s_A += a;
      s_u = fmaR(a, ul, s_u);
      s_v = fmaR(a, vl, s_v);
      s_w = fmaR(a, wl, s_w);
      s_x = fmaR(a, xl, s_x);
      if (VF == VF_KG) {
        const R cp = c * (me[4] + pl);
        s_p += cp;
        s_E2 = fmaR(cp, unds, s_E2);
      } else {
        s_p = fmaR(c, pl, s_p);
      }
    };
    partner_loop<GRAD, st>(id, n, base, pair);
    const R q4 = (R)0.25, q8 = (R)0.125, h2 = (R)0.5;
    R P = s_p;
    if (VF != VF_KG) {
      const R rowsum = id == 0 ? wb : (id == N ? -wb : (R)0);
      P = fmaR(me[4], rowsum, s_p);
    }
    acc[0] -= invJ * (q4 * s_A);
    acc[1] -= invJ * (q8 * fmaR(me[1], s_A, s_u) + (D == 0 ? h2 * P : (R)0));
    acc[2] -= invJ * (q8 * fmaR(me[2], s_A, s_v) + (D == 1 ? h2 * P : (R)0));
    acc[3] -= invJ * (q8 * fmaR(me[3], s_A, s_w) + (D == 2 ? h2 * P : (R)0));
    acc[4] -= invJ * (q8 * fmaR(me[5], s_A, s_x) + (VF == VF_KG ? q4 * s_E2 : (R)0));
  } else if (VF == VF_STD) {
    // F# = (F(a) + F(b))/2 with F_rho = rho u_D, F_m = rho u_D u + p e_D, F_E = rho h u_D
    // with the node's own terms taken out of the sums (rowsum as above)
    const R mA = me[0] * me[1 + D];
    R s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, sp = 0;
    auto pair = [&](int l, int m) {
      const R c = crow[l];
      grad_acc(c, m);
      const R cB = c * (sP[0][m] * sP[1 + D][m]);
      s0 += cB;
      s1 = fmaR(cB, sP[1][m], s1);
      s2 = fmaR(cB, sP[2][m], s2);
      s3 = fmaR(cB, sP[3][m], s3);
      s4 = fmaR(cB, sP[5][m], s4);
      sp = fmaR(c, sP[4][m], sp);
    };
    partner_loop<GRAD, st>(id, n, base, pair);
    const R rowsum = id == 0 ? wb : (id == N ? -wb : (R)0);
    const R mr = mA * rowsum;
    s0 += mr;
    s1 = fmaR(mr, me[1], s1);
    s2 = fmaR(mr, me[2], s2);
    s3 = fmaR(mr, me[3], s3);
    s4 = fmaR(mr, me[5], s4);
    sp = fmaR(me[4], rowsum, sp);
    const R h2 = (R)0.5;
    acc[0] -= invJ * (h2 * s0);
    acc[1] -= invJ * (h2 * (s1 + (D == 0 ? sp : (R)0)));
    acc[2] -= invJ * (h2 * (s2 + (D == 1 ? sp : (R)0)));
    acc[3] -= invJ * (h2 * (s3 + (D == 2 ? sp : (R)0)));
    acc[4] -= invJ * (h2 * s4);
  } else {
    // Chandrashekar: general pairwise evaluation (FP64 test flux)
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    RotState<double> a;
    a.r = me[0]; a.un = me[1 + D]; a.u1 = me[1 + (D + 1) % 3]; a.u2 = me[1 + (D + 2) % 3]; a.p = me[4];
#pragma unroll
    for (int k = 1; k <= kPartners; ++k) {
      const int l = partner(id, k);
      const int m = base + l * st;
      const double c = crow[l];
      grad_acc((R)c, m);
      RotState<double> b;
      b.r = sP[0][m]; b.un = sP[1 + D][m]; b.u1 = sP[1 + (D + 1) % 3][m]; b.u2 = sP[1 + (D + 2) % 3][m];
      b.p = sP[4][m];
      double f[5];
      twopoint_rot<VF_CH, double>(a, b, gm1, f);
      s[0] = fma(c, f[0], s[0]);
      s[1 + D] = fma(c, f[1], s[1 + D]);
      s[1 + (D + 1) % 3] = fma(c, f[2], s[1 + (D + 1) % 3]);
      s[1 + (D + 2) % 3] = fma(c, f[3], s[1 + (D + 2) % 3]);
      s[4] = fma(c, f[4], s[4]);
    }
    for (int v = 0; v < 5; ++v) acc[v] -= invJ * (R)s[v];
  }
  if (GRAD) {
    const R h2 = (R)0.5;
    gs[0] = h2 * g0;
    gs[1] = h2 * g1;
    gs[2] = h2 * g2;
    gs[3] = h2 * g3;
  }
}

// ---------------------------------------------------------------------------
// BR1 lifted gradient at node n: g[d][c] = d q_c / d x_d, q = (u, v, w, theta).
// sQ holds the interface values q* on the six faces of the element.
// ---------------------------------------------------------------------------
template <class R, int ROW = nn>
__device__ __forceinline__ void lifted_gradient(const R (*sP)[ROW], const R (*sQ)[4][nf], const R* sDw, const R* swinv,
                                                int n, const int ijk[3], const R invJ[3], R g[3][4]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
    const int id = ijk[d];
    const int base = n - id * st;
    const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
    const R* crow = sDw + id * n1;
    R s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      const int m = base + l * st;
      const R c = crow[l];
      s0 = fmaR(c, sP[1][m], s0);
      s1 = fmaR(c, sP[2][m], s1);
      s2 = fmaR(c, sP[3][m], s2);
      s3 = fmaR(c, sP[6][m], s3);
    }
    if (id == 0 || id == N) {  // one branch for both faces (N >= 1)
      const int f = 2 * d + (id == N);
      const R w = id == N ? swinv[N] : -swinv[0];
      s0 = fmaR(w, sQ[f][0][a], s0);
      s1 = fmaR(w, sQ[f][1][a], s1);
      s2 = fmaR(w, sQ[f][2][a], s2);
      s3 = fmaR(w, sQ[f][3][a], s3);
    }
    g[d][0] = invJ[d] * s0;
    g[d][1] = invJ[d] * s1;
    g[d][2] = invJ[d] * s2;
    g[d][3] = invJ[d] * s3;
  }
}

// Viscous flux in direction D (momentum x, y, z and energy components):
// tau = mu (grad u + grad u^T - 2/3 div u I), F_E = u . tau_D + kappa dtheta/dx_D.
template <int D, class R>
__device__ __forceinline__ void viscous_flux(const R g[3][4], R vx, R vy, R vz, R mu, R kappa, R F[4]) {
  const R div = g[0][0] + g[1][1] + g[2][2];
  const R dv = (R)(2.0 / 3.0) * mu * div;
  F[0] = mu * (g[D][0] + g[0][D]) - (D == 0 ? dv : (R)0);
  F[1] = mu * (g[D][1] + g[1][D]) - (D == 1 ? dv : (R)0);
  F[2] = mu * (g[D][2] + g[2][D]) - (D == 2 ? dv : (R)0);
  F[3] = vx * F[0] + vy * F[1] + vz * F[2] + kappa * g[D][3];
}

// Smagorinsky eddy viscosity at a node from its lifted gradient g[d][c]
// (c = u, v, w): mu_t = rho (C_s Delta)^2 |S|, |S|^2 = 2 S_ij S_ij.
template <class R>
__device__ __forceinline__ R eddy_viscosity(const R g[3][4], R rho, R csd2) {
  const R a = g[0][1] + g[1][0], b = g[0][2] + g[2][0], c = g[1][2] + g[2][1];
  const R S2 = (R)2 * (g[0][0] * g[0][0] + g[1][1] * g[1][1] + g[2][2] * g[2][2]) + a * a + b * b + c * c;
  return rho * csd2 * sqrt_nonneg(S2);
}

__device__ __forceinline__ double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return a > 0.0 ? fmin(a, b) : fmax(a, b);
}

// Reconstructed face states of FV subcell m along a line (primitive w = rho,u,v,w,p):
// slopes by minmod of divided differences between node positions for interior
// subcells (outer subcells first order), first-order fallback if a face state
// has rho <= 0 or p <= 0.  Returns the state at the right (plus) or left face.
__device__ __forceinline__ void subcell_face_state(const double (*sP)[nnp], int base, int st, int m, bool right,
                                                   int recon, const double* sxi, const double* sedge, double w[5]) {
  const int mm = base + m * st;
  double c[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) c[v] = sP[v][mm];
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

// Geometry of face item q: face f (0:-x 1:+x 2:-y 3:+y 4:-z 5:+z), normal
// direction d, face-local index a, the own and the neighbour's volume node on
// the face.  One code path serves all directions (no branch divergence): the
// direction only enters address arithmetic.
struct FaceItem {
  int f, a, d, side, nb, nown, nnb, k1, k2;  // k1, k2: tangential momentum components
};

// The six neighbours of an element that is the same for the whole workgroup,
// read with scalar loads (short latency, no vector memory round trip before
// the face-state loads that need them); pick() selects face f's.
struct Nbr6 {
  int n[6];
  __device__ __forceinline__ int pick(int f) const {  // selects, not an indexed (scratch) array
    const bool odd = (f & 1) != 0;
    const int a01 = odd ? n[1] : n[0], a23 = odd ? n[3] : n[2], a45 = odd ? n[5] : n[4];
    return f < 2 ? a01 : (f < 4 ? a23 : a45);
  }
};
__device__ __forceinline__ Nbr6 uniform_nbr6(const int32_t* nbr, int e) {
  const int eu = __builtin_amdgcn_readfirstlane(e);
  Nbr6 r;
#pragma unroll
  for (int f = 0; f < 6; ++f) r.n[f] = nbr[6 * eu + f];
  return r;
}

__device__ __forceinline__ FaceItem face_item_geometry_nb(int nb, int q) {
  FaceItem it;
  it.f = q / nf;
  it.a = q - it.f * nf;
  it.d = it.f >> 1;
  it.side = it.f & 1;
  it.nb = nb;
  const int t1 = it.a % n1, t2 = it.a / n1;
  const int sn = it.d == 0 ? 1 : (it.d == 1 ? n1 : nf);
  const int s1 = it.d == 0 ? n1 : 1;
  const int s2 = it.d == 2 ? n1 : nf;
  const int tang = t1 * s1 + t2 * s2;
  it.nown = (it.side ? N : 0) * sn + tang;
  it.nnb = (it.side ? 0 : N) * sn + tang;
  it.k1 = it.d == 2 ? 1 : it.d + 2;  // 1 + (d+1) % 3
  it.k2 = it.d == 0 ? 3 : it.d;      // 1 + (d+2) % 3
  return it;
}

__device__ __forceinline__ FaceItem face_item_geometry(const int32_t* nbr, int e, int q) {
  return face_item_geometry_nb(nbr[6 * e + q / nf], q);
}

// Face item q of a workgroup-uniform element with neighbours b.
__device__ __forceinline__ FaceItem face_item_geometry(const Nbr6& b, int q) {
  return face_item_geometry_nb(b.pick(q / nf), q);
}

// Conservative state of node n with the momentum rotated to (normal, t1, t2).
__device__ __forceinline__ void load_rotated(const double* Ux, int n, const FaceItem& it, double X[5]) {
  X[0] = Ux[n];
  X[1] = Ux[(1 + it.d) * nn + n];
  X[2] = Ux[it.k1 * nn + n];
  X[3] = Ux[it.k2 * nn + n];
  X[4] = Ux[4 * nn + n];
}

// Conservative minus (L) and plus (R) states of the face item, rotated (the
// side only selects the two addresses).
__device__ __forceinline__ void face_loads(const double* U, int e, const FaceItem& it, double L[5], double R[5]) {
  const int eL = it.side ? e : it.nb, eR = it.side ? it.nb : e;
  const int nL = it.side ? it.nown : it.nnb, nR = it.side ? it.nnb : it.nown;
  load_rotated(U + (size_t)eL * 5 * nn, nL, it, L);
  load_rotated(U + (size_t)eR * 5 * nn, nR, it, R);
}

// ---------------------------------------------------------------------------
// Wall-modelled boundaries (paper Sec. 3).  A face without neighbour (nbr -1)
// is a wall.  Its advective flux and its BR1 interface value take the mirror
// image of the own face state (normal momentum reversed) as the other side; its
// viscous flux comes from the wall model: Spalding's law of the wall
//   y+ = u+ + c [e^(k u+) - 1 - (k u+) - (k u+)^2/2 - (k u+)^3/6 - (k u+)^4/24],
//   k = 0.4, c = 0.1108,
// solved for the friction velocity with the wall-parallel velocity of the
// element's node on the opposite face (distance h = the element size) as input,
// optionally van Driest transformed first.  The shear stress rho_w u_tau^2
// acts against that velocity; mass, normal momentum and energy see no flux.
// The solve runs in its own kernel over the wall face nodes (k_wall_flux),
// which writes the flux into the wall face's own slot of Fvf; the stage
// kernel reads it there, so that the Newton iteration (transcendental
// functions in FP64) does not raise the register count of the stage kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wm_bracket(double k, double ek) {
  // e^k minus its Taylor polynomial of degree four
  return ek - (1.0 + k * (1.0 + k * (0.5 + k * (1.0 / 6.0 + k * (1.0 / 24.0)))));
}

// u_tau for wall-parallel speed u > 0 at distance h, kinematic viscosity nu.
// With x = u / u_tau the law reads x y+(x) = Re_h = h u / nu.  Newton's method
// in s = ln x on ln(x y+(x)) - ln(Re_h), which is increasing and convex in s,
// converges monotonically from any start right of the root; x = sqrt(Re_h)
// is one (y+(x) >= x), capped at 1700 where e^(0.4 x) is still finite.  A
// final Newton step on y+(u/u_tau) - h u_tau / nu polishes the root.
__device__ double wm_friction_velocity(double u, double nu, double h) {
  const double lre = log(h * u / nu);
  double s = fmin(0.5 * lre, log(1700.0));
  double x = exp(s);
  for (int it = 0; it < 100; ++it) {
    const double k = 0.4 * x, ek = exp(k);
    const double y = x + 0.1108 * wm_bracket(k, ek);
    const double dy = 1.0 + 0.1108 * 0.4 * (ek - (1.0 + k * (1.0 + k * (0.5 + k * (1.0 / 6.0)))));
    const double step = (s + log(y) - lre) / (1.0 + x * dy / y);
    s -= step;
    x = exp(s);
    if (fabs(step) <= 1e-15) break;
  }
  const double ut = u / x;
  const double k = 0.4 * x, ek = exp(k);
  const double y = x + 0.1108 * wm_bracket(k, ek);
  const double dy = 1.0 + 0.1108 * 0.4 * (ek - (1.0 + k * (1.0 + k * (0.5 + k * (1.0 / 6.0)))));
  const double F = y - h * ut / nu;
  const double dF = -dy * x / ut - h / nu;
  return ut - F / dF;
}

// Wall-model viscous flux of a wall face item along +d in the rotated frame
// (normal, t1, t2, energy): rhow = density at the wall node, (rx, mt1, mt2) =
// density and tangential momenta of the exchange node, sg = -1 on the
// element's + face.
__device__ __forceinline__ void wall_model_flux(const StageArgs& A, double rhow, double rx, double mt1, double mt2,
                                                double sg, double g[4]) {
  g[0] = g[1] = g[2] = g[3] = 0.0;
  const double ir = 1.0 / rx;
  const double v1 = mt1 * ir, v2 = mt2 * ir;
  const double sp2 = v1 * v1 + v2 * v2;
  if (!(sp2 > 0.0)) return;
  const double sp = sqrt(sp2);
  double ueq = sp;
  if (A.wm_b > 0.0) ueq = (A.wm_uinf / A.wm_b) * asin(fmin(A.wm_b * sp / A.wm_uinf, 1.0));
  const double ut = wm_friction_velocity(ueq, A.mu / rhow, A.wm_h);
  const double c = sg * rhow * ut * ut / sp;
  g[1] = c * v1;
  g[2] = c * v2;
}

// Face item without neighbour: the own face node (minus side if it lies on the
// element's + face) and its mirror image.
__device__ __forceinline__ void wall_face_loads(const double* U, int e, const FaceItem& it, double L[5],
                                                double R[5]) {
  double X[5];
  load_rotated(U + (size_t)e * 5 * nn, it.nown, it, X);
#pragma unroll
  for (int v = 0; v < 5; ++v) L[v] = R[v] = X[v];
  if (it.side) R[1] = -X[1];
  else L[1] = -X[1];
}

template <bool WALL>
__device__ __forceinline__ void face_loads_w(const double* U, int e, const FaceItem& it, double L[5], double R[5]) {
  if (WALL && it.nb < 0) wall_face_loads(U, e, it, L, R);
  else face_loads(U, e, it, L, R);
}

// Elements per workgroup (EPB) of the stage and lifting kernels.  With one
// element per workgroup, N = 5 fills 216 of 256 lanes (the last wave is 3/8
// full) and a wave instruction costs the same whatever its active lanes; two
// elements fill 432 of 448.  Each element owns a slot of TPE consecutive
// threads (node t and face item t of slot s is thread s TPE + t); the slots
// share the basis in LDS and every barrier.  Measured at N = 5: the lifting
// kernel gains 6 % with two elements; the stage kernel loses 17 % (its LDS then
// admits two workgroups per CU instead of four), so it keeps one.
#ifndef DG_EPB_STAGE
#define DG_EPB_STAGE 1
#endif
#ifndef DG_EPB_LIFT
#define DG_EPB_LIFT (DG_N == 5 ? 2 : 1)
#endif
template <int E>
struct Pack {
  static constexpr int EPB = E;
  static constexpr int TPE = E == 1 ? NT : (nn > 6 * nf ? nn : 6 * nf);
  static constexpr int NTB = ((E * TPE + 63) / 64) * 64;
  // face items handled by one thread of a slot (item q = t + k TPE, k < FI)
  static constexpr int FI = (6 * nf + TPE - 1) / TPE;
  static_assert(E >= 1 && NTB <= 1024, "workgroup size");
};
using PS = Pack<DG_EPB_STAGE>;
using PL = Pack<DG_EPB_LIFT>;

// Slot of the calling thread: element e (clamped to a valid one), its thread
// index t within the slot, and t = TPE (beyond every per-thread bound: nodes,
// face items) for threads without an element: the padding of the last wave
// and the second slot of a workgroup past the last element.
struct Slot {
  int s, e, t, traw;
  bool live;
};
template <class P>
__device__ __forceinline__ Slot slot_of_thread(int e0, int nelem) {
  Slot r;
  const int tid = threadIdx.x;
  const int s0 = P::EPB == 1 ? 0 : tid / P::TPE;
  r.s = s0 < P::EPB ? s0 : P::EPB - 1;
  r.live = s0 < P::EPB && e0 + r.s < nelem;
  r.e = r.live ? e0 + r.s : e0;
  r.traw = tid - s0 * P::TPE;
  r.t = r.live ? r.traw : P::TPE;
  return r;
}

// Loads of one face item, issued together before any of them is used: both
// rotated states and (Navier-Stokes) the neighbour's normal viscous flux.
// At a wall (WALL variant, neighbour -1) fn is the wall-model flux, read from
// the element's own slot of the wall face.
// Split BR1 (StageArgs.split): at a face node of the element's face f (normal
// direction d, side s), the neighbour n's lifted gradient differs from its own
// part (the one n's Fvf holds) by the other halves of the interface values at
// that node: across the shared face the element's own q (normal derivative,
// weight c_d), and across n's lateral faces where the node lies on an edge
// of the face, the q of the diagonal element (n's neighbour there; weight
// c_g).  On the structured periodic box the diagonal element across n's
// lateral face is n shifted as the element is by its own neighbour there
// (n + nbr(e, lateral) - e; the shift along the lateral direction does not
// depend on the coordinate along d), and its node is n's face node moved to
// the other side along the lateral direction; each edge face item loads the
// density and momenta of its one or two diagonal nodes with the face states.
struct Lateral {
  int dir, side;  // n's lateral face (direction, side) through the node
};
template <bool SPLIT>
struct SplitLoads {
  int nlat = 0;
  Lateral lat[2];
  double dg[2][3];  // rho, m_d, m_dg of the diagonal nodes (d: the face normal)
};
template <>
struct SplitLoads<false> {};

// The (up to two) lateral faces of the neighbour across face item it, and the
// loads of the diagonal nodes (element e with the neighbours nb6).
__device__ __forceinline__ void split_issue(const StageArgs& A, const FaceItem& it, const Nbr6& nb6, int e,
                                            SplitLoads<true>& sp) {
  const int da = it.d == 0 ? 1 : 0, db = it.d == 2 ? 1 : 2;  // tangential directions, t1 along da
  const int t1 = it.a % n1, t2 = it.a / n1;
  // slots filled with fixed indices (selects, no indexed scratch array)
  const bool e1 = t1 == 0 || t1 == N, e2 = t2 == 0 || t2 == N;
  sp.nlat = (e1 ? 1 : 0) + (e2 ? 1 : 0);
  sp.lat[0] = Lateral{e1 ? da : db, e1 ? (t1 == N ? 1 : 0) : (t2 == N ? 1 : 0)};
  sp.lat[1] = Lateral{db, t2 == N ? 1 : 0};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (j >= sp.nlat) break;
    const int dg = sp.lat[j].dir, sg = sp.lat[j].side;
    const int diag = it.nb + nb6.pick(2 * dg + sg) - e;
    const int node = it.nnb + (sg ? -N : N) * (dg == 0 ? 1 : (dg == 1 ? n1 : nf));
    const double* Ud = A.U + (size_t)diag * 5 * nn + node;
    sp.dg[j][0] = Ud[0];
    sp.dg[j][1] = Ud[(1 + it.d) * nn];
    sp.dg[j][2] = Ud[(1 + dg) * nn];
  }
}

__device__ __forceinline__ double pick3(const double v[3], int d) { return d == 0 ? v[0] : (d == 1 ? v[1] : v[2]); }

// The neighbour-dependent rest of the neighbour's normal viscous flux at face
// item it (split BR1), added to fn (in the face frame: normal, t1, t2 and
// energy components): the viscous flux (linear in the gradient for constant
// viscosity) of the gradient made of the other halves, with the neighbour's
// velocity at the node, written out for its few non-zero terms.  own / nb:
// the element's and the neighbour's face states (rotated frame, FP64).
//   normal half g_d = c_d q_e:   tau_nn = 4/3 mu c_d u_n,e, tau_tn = mu c_d u_t,e;
//   lateral half g_dg = c_g u_g: tau_dg,n += mu c_g u_n,g, tau_nn -= 2/3 mu c_g u_dg,g;
//   F_E = u_nb . tau_n + kappa c_d theta_e.
__device__ __forceinline__ void split_rest(const StageArgs& A, const FaceItem& it, const State64& own,
                                           const State64& nb, const SplitLoads<true>& sp, double fn[4]) {
  // (1/w_0) / 2, w_0 = w_N: a uniform load through the constant address space
  const double hw = 0.5 * ((const double __attribute__((address_space(4)))*)(uintptr_t)A.basis)[BL.winv()];
  const double mu = A.mu;
  const double cd = pick3(A.invJ, it.d) * (it.side ? -hw : hw);
  double tnn = (4.0 / 3.0) * mu * cd * own.un;
  double t1 = mu * cd * own.u1, t2 = mu * cd * own.u2;
  double fe = A.kappa * cd * own.p * own.ir;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (j >= sp.nlat) break;
    const int dg = sp.lat[j].dir;
    const double cg = pick3(A.invJ, dg) * (sp.lat[j].side ? hw : -hw) * rcp64(sp.dg[j][0]);
    const double sh = mu * cg * sp.dg[j][1];                    // tau_dg,n
    const double dv = (2.0 / 3.0) * mu * cg * sp.dg[j][2];     // from the divergence
    tnn -= dv;
    const bool first = dg == (it.d == 2 ? 0 : it.d + 1);        // dg is the t1 direction
    if (first) t1 += sh;
    else t2 += sh;
  }
  fe += nb.un * tnn + nb.u1 * t1 + nb.u2 * t2;
  fn[0] += tnn;  // fn in the face frame
  fn[1] += t1;
  fn[2] += t2;
  fn[3] += fe;
}

template <bool NS, class R, bool WALL = false, bool SPLIT = false>
struct FaceData {
  FaceItem it;
  double L[5], R_[5];
  R fn[4];
  SplitLoads<SPLIT> sp;
};

template <bool NS, class R, bool WALL = false, bool SPLIT = false>
__device__ __forceinline__ void face_issue(const StageArgs& A, int e, FaceData<NS, R, WALL, SPLIT>& fd,
                                           const Nbr6* nb6 = nullptr) {
  const FaceItem& it = fd.it;
  if constexpr (SPLIT) {
    split_issue(A, it, *nb6, e, fd.sp);
  }
  if (WALL && it.nb < 0) {
    wall_face_loads(A.U, e, it, fd.L, fd.R_);
    const R* Fn = reinterpret_cast<const R*>(A.Fvf) + ((size_t)e * 6 + it.f) * 4 * nf + it.a;
#pragma unroll
    for (int c = 0; c < 4; ++c) fd.fn[c] = Fn[c * nf];
    return;
  }
  face_loads(A.U, e, it, fd.L, fd.R_);
  if (NS) {
    const R* Fn = reinterpret_cast<const R*>(A.Fvf) + ((size_t)it.nb * 6 + (it.f ^ 1)) * 4 * nf + it.a;
    if (SPLIT) {  // in the face frame (normal, t1, t2, energy), as the rest is formed
      fd.fn[0] = Fn[it.d * nf];
      fd.fn[1] = Fn[(it.k1 - 1) * nf];
      fd.fn[2] = Fn[(it.k2 - 1) * nf];
      fd.fn[3] = Fn[3 * nf];
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) fd.fn[c] = Fn[c * nf];
    }
  }
}

template <class R>
__device__ __forceinline__ void store_q(const FaceItem& it, const R qs[4], R (*sQ)[4][nf]) {
  sQ[it.f][it.d][it.a] = qs[0];
  sQ[it.f][it.k1 - 1][it.a] = qs[1];
  sQ[it.f][it.k2 - 1][it.a] = qs[2];
  sQ[it.f][3][it.a] = qs[3];
}

// Interface values of a face item into LDS: advective f*, and for
// Navier-Stokes q* = (q- + q+)/2 and the neighbour's normal viscous flux.
template <int VF, bool NS, class R, bool MX, bool WALL = false, bool SPLIT = false>
__device__ __forceinline__ void face_item(const StageArgs& A, const FaceData<NS, R, WALL, SPLIT>& fd, const Ref& ref,
                                          R (*sF)[5][nf], R (*sQ)[4][nf], R (*sFn)[4][nf]) {
  const FaceItem& it = fd.it;
  const State64 sL = state64<0>(fd.L, A.gamma - 1.0), sR = state64<0>(fd.R_, A.gamma - 1.0);
  if (NS) {
    R fn[4] = {fd.fn[0], fd.fn[1], fd.fn[2], fd.fn[3]};
    if constexpr (SPLIT) {
      static_assert(sizeof(R) == 8, "split BR1: FP64");
      __builtin_amdgcn_sched_barrier(0);
      split_rest(A, it, it.side ? sL : sR, it.side ? sR : sL, fd.sp, fn);
      __builtin_amdgcn_sched_barrier(0);
      store_q(it, fn, sFn);  // from the face frame
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) sFn[it.f][c][it.a] = fn[c];
    }
  }
  const Jumps<R> J = jumps<R, MX>(sL, sR, A.gamma, ref, A.sf);
  R g[5];
  riemann_rot<VF, R>(A.sf, to_rot<R, MX>(sL, ref), to_rot<R, MX>(sR, ref), J, (R)A.gamma, g);
  sF[it.f][0][it.a] = g[0];
  sF[it.f][1 + it.d][it.a] = g[1];
  sF[it.f][it.k1][it.a] = g[2];
  sF[it.f][it.k2][it.a] = g[3];
  sF[it.f][4][it.a] = g[4];
  if (NS) {
    R qs[4];
    interface_q<0, R, MX>(sL, sR, ref, qs);
    store_q(it, qs, sQ);
  }
}

// ---------------------------------------------------------------------------
// Stage kernel: operator (+ FV blend) and either U_t output or RK update.
// EQ: 0 Euler, 1 Navier-Stokes, 2 Navier-Stokes with the Smagorinsky eddy
// viscosity.  R: arithmetic type (double, or float for the mixed operator, MX).
// ---------------------------------------------------------------------------
// Several elements per workgroup: two workgroups per CU need 4 waves per SIMD
// (at most 128 registers); not imposed on the CH flux, which would spill.
#if DG_STAGE_MIN_WAVES > 0
#define DG_STAGE_BOUNDS __launch_bounds__(PS::NTB, DG_STAGE_MIN_WAVES)
#elif DG_EPB_STAGE > 1
#define DG_STAGE_BOUNDS __launch_bounds__(PS::NTB, VF == VF_CH ? 1 : 4)
#else
#define DG_STAGE_BOUNDS __launch_bounds__(PS::NTB)
#endif
// Indicator quantity q = rho p of a conservative node state.
__device__ __forceinline__ double indicator_q(const double u[5], double gm1) {
  const double ir = 1.0 / u[0];
  const double p = gm1 * (u[4] - 0.5 * ir * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]));
  return u[0] * p;
}

// First-stage blending coefficient of one element (Sec. 4.1): modal energies
// of q (node t holds qt) by the three 1-D V^-1 contractions through LDS (sq,
// st: nn doubles each, sVi: V^-1 already written), the three energy sums by
// lane shuffles within each wave and the per-wave partials (sred: 3 NT/64
// doubles) in a fixed order, then the sigmoid, the clip at alpha_max and the
// cut-off below alpha_min.  Every thread of the workgroup (NT threads, one
// element) calls it; the result is valid in thread 0.
constexpr int NWAVE = NT / 64;
__device__ __forceinline__ double element_alpha1(const StageArgs& A, const double* sVi, double* sq, double* st,
                                                 double* sred, int t, const int ijk[3], double qt) {
  if (t < nn) sq[t] = qt;
  __syncthreads();
  if (t < nn) {  // x: st[a,j,k] = sum_i Vinv[a][i] q[i,j,k]
    const int base = t - ijk[0];
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < n1; ++i) s = fma(sVi[ijk[0] * n1 + i], sq[base + i], s);
    st[t] = s;
  }
  __syncthreads();
  if (t < nn) {  // y
    const int base = t - ijk[1] * n1;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < n1; ++j) s = fma(sVi[ijk[1] * n1 + j], st[base + j * n1], s);
    sq[t] = s;
  }
  __syncthreads();
  double e2 = 0.0;
  int mx = 0;
  if (t < nn) {  // z
    const int base = t - ijk[2] * nf;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < n1; ++k) s = fma(sVi[ijk[2] * n1 + k], sq[base + k * nf], s);
    e2 = s * s;
    mx = max(ijk[0], max(ijk[1], ijk[2]));
  }
  double r0 = e2, r1 = (mx == N) ? e2 : 0.0, r2 = (mx == N - 1) ? e2 : 0.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    r0 += __shfl_xor(r0, o);
    r1 += __shfl_xor(r1, o);
    r2 += __shfl_xor(r2, o);
  }
  if ((t & 63) == 0) {
    sred[t >> 6] = r0;
    sred[NWAVE + (t >> 6)] = r1;
    sred[2 * NWAVE + (t >> 6)] = r2;
  }
  __syncthreads();
  double a1 = 0.0;
  if (t == 0) {
    double S = 0.0, SN = 0.0, SN1 = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) {
      S += sred[w];
      SN += sred[NWAVE + w];
      SN1 += sred[2 * NWAVE + w];
    }
    const double EN = S > 0.0 ? SN / S : 0.0;
    const double rest = S - SN;
    const double EN1 = rest > 0.0 ? SN1 / rest : 0.0;
    const double E = A.indicator == 1 ? EN : fmax(EN, EN1);
    const double a0 = 1.0 / (1.0 + exp(-(A.sharp / A.thresh) * (E - A.thresh)));
    a1 = fmin(a0, A.amax);
    if (a1 < A.amin) a1 = 0.0;
  }
  return a1;
}

// The blended Euler stage kernel's epilogue computes the next stage's first
// coefficient (StageArgs.alpha1_next) when its LDS pool holds the indicator's
// scratch and one pass of threads loads the basis with V^-1.
constexpr bool kFusedAlpha1 = N >= 2 && DG_EPB_STAGE == 1 && 7 * nnp + 30 * nf >= 2 * nn + 3 * NWAVE &&
                               NB_STAGE + nf <= NT;

// Viscous fluxes at a node from its lifted gradient g (with the Smagorinsky
// eddy viscosity when LES).
template <bool LES, class R>
__device__ __forceinline__ void node_viscous_flux(const StageArgs& A, int e, const R g[3][4], const R* me,
                                                  R Fv[3][4]) {
  R mu = (R)A.mu, kap = (R)A.kappa;
  if (LES) {
    const double cs = A.cs_elem ? A.cs_elem[e] : A.cs;
    const R mut = eddy_viscosity<R>(g, me[0], (R)(cs * cs * A.delta2));
    mu += mut;
    kap = fmaR((R)A.ktf, mut, kap);
  }
  viscous_flux<0, R>(g, me[1], me[2], me[3], mu, kap, Fv[0]);
  viscous_flux<1, R>(g, me[1], me[2], me[3], mu, kap, Fv[1]);
  viscous_flux<2, R>(g, me[1], me[2], me[3], mu, kap, Fv[2]);
}

__device__ __forceinline__ int axis_stride(int j) { return j == 0 ? 1 : (j == 1 ? n1 : nf); }

// Padded node layout of the split lifting's LDS copy of (u, v, w, theta): one
// double after every x-row, so that the lines read across a wavefront (x-lines
// of different rows, y-lines of different planes) fall on different LDS banks.
constexpr int SQP = nn + nn / n1;  // doubles per variable
__device__ __forceinline__ constexpr int pstride(int j) { return j == 0 ? 1 : (j == 1 ? n1 + 1 : n1 * (n1 + 1)); }
__device__ __forceinline__ int padded(int m) { return m + m / n1; }  // node m = i0 + n1 i1 + nf i2

// The four lifted variables of node t into the padded layout (P: primitives).
__device__ __forceinline__ void store_own_q(double* sq, int t, const double P[7]) {
  const int m = padded(t);
  sq[m] = P[1];
  sq[SQP + m] = P[2];
  sq[2 * SQP + m] = P[3];
  sq[3 * SQP + m] = P[6];
}

// Split BR1: the own part of the normal viscous flux at every face node of
// the element (into Fout, laid out as StageArgs.Fvf), from sq = (u, v, w,
// theta) at its nodes (LDS, padded layout), by lines rather than one face
// node at a time:
//   pass 1: each normal line (3 nf of them) gives the derivatives of
//     (u, v, w, theta) along it at both end nodes, and each line of a face
//     plane along one of the plane's axes j (6 faces x 2 axes x n1 lines)
//     those of u_d and of u_j (d: the face normal; one task per variable, so
//     that the tasks' work is about even and the code is the same for both)
//     at its nodes, into the LDS scratch sW (48 nf doubles);
//   pass 2: each face node forms its flux from these and its velocity.
// Each line's values are read from LDS once; the differentiation matrix comes
// with uniform loads from the constant address space.  The interface values
// are the node's own half, q / 2.  The caller synchronises the workgroup
// before (sq written, sW free); the function synchronises between the passes.
using cdouble_ptr = const double __attribute__((address_space(4)))*;
template <int TPE>
__device__ __forceinline__ void own_part_by_lines(const StageArgs& A, int e, int t, const double* sq, double* sW,
                                                  double* Fout) {
  const cdouble_ptr cb = (cdouble_ptr)(uintptr_t)A.basis;
  const cdouble_ptr Dw = cb + BL.Dw();
  const double h0 = -0.5 * cb[BL.winv()], hN = 0.5 * cb[BL.winv() + N];  // own-half weights at the ends
  double* sGn = sW;            // [3 d][2 side][4 v][nf]
  double* sT = sW + 24 * nf;   // [6 f][2 jj][2 c][nf]
  constexpr int NTASK = 3 * nf + 24 * n1;
  for (int task = t; task < NTASK; task += TPE) {
    if (task < 3 * nf) {  // normal line
      const int d = task / nf, a = task - d * nf;
      const int ja = d == 0 ? 1 : 0, jb = d == 2 ? 1 : 2;
      const int sd = pstride(d);
      const int base = (a % n1) * pstride(ja) + (a / n1) * pstride(jb);
      double g0[4] = {0, 0, 0, 0}, gN[4] = {0, 0, 0, 0};
#pragma unroll
      for (int l = 0; l < n1; ++l) {
        const double c0 = Dw[l], cN = Dw[N * n1 + l];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double q = sq[v * SQP + base + l * sd];
          g0[v] = fma(c0, q, g0[v]);
          gN[v] = fma(cN, q, gN[v]);
        }
      }
      const double J = A.invJ[0] * (d == 0) + A.invJ[1] * (d == 1) + A.invJ[2] * (d == 2);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        g0[v] = J * fma(h0, sq[v * SQP + base], g0[v]);
        gN[v] = J * fma(hN, sq[v * SQP + base + N * sd], gN[v]);
        sGn[((2 * d) * 4 + v) * nf + a] = g0[v];
        sGn[((2 * d + 1) * 4 + v) * nf + a] = gN[v];
      }
    } else {  // one variable (u_d or u_j) along a line of a face plane
      const int u = task - 3 * nf;
      const int c = u / (12 * n1), w = u - c * 12 * n1;  // c: the variable; the code does not branch on it
      const int f = w / (2 * n1), r = w - f * 2 * n1, jj = r / n1, pos = r - jj * n1;
      const int d = f >> 1, id = (f & 1) ? N : 0;
      const int ja = d == 0 ? 1 : 0, jb = d == 2 ? 1 : 2;
      const int j = jj ? jb : ja, o = jj ? ja : jb;
      const int sj = pstride(j);
      const double* src = sq + (c ? j : d) * SQP + id * pstride(d) + pos * pstride(o);
      double q[n1];
#pragma unroll
      for (int l = 0; l < n1; ++l) q[l] = src[l * sj];
      const double J = A.invJ[0] * (j == 0) + A.invJ[1] * (j == 1) + A.invJ[2] * (j == 2);
      double* out = sT + ((f * 2 + jj) * 2 + c) * nf;
#pragma unroll
      for (int i = 0; i < n1; ++i) {
        double tv = 0;
#pragma unroll
        for (int l = 0; l < n1; ++l) tv = fma(Dw[i * n1 + l], q[l], tv);
        if (i == 0) tv = fma(h0, q[0], tv);
        if (i == N) tv = fma(hN, q[N], tv);
        out[jj ? pos + n1 * i : i + n1 * pos] = J * tv;
      }
    }
  }
  __syncthreads();
  const double mu = A.mu, kap = A.kappa;
  for (int q = t; q < 6 * nf; q += TPE) {
    const int f = q / nf, a = q - f * nf, d = f >> 1;
    const int ja = d == 0 ? 1 : 0, jb = d == 2 ? 1 : 2;
    const int n = (f & 1 ? N : 0) * pstride(d) + (a % n1) * pstride(ja) + (a / n1) * pstride(jb);
    const double* gn = sGn + f * 4 * nf + a;  // f = 2 d + side
    const double dn_ud = gn[d * nf], dn_ua = gn[ja * nf], dn_ub = gn[jb * nf], dn_th = gn[3 * nf];
    const double* tt = sT + f * 4 * nf + a;
    const double da_ud = tt[0], da_ua = tt[nf], db_ud = tt[2 * nf], db_ub = tt[3 * nf];
    const double dv = (2.0 / 3.0) * mu * (dn_ud + da_ua + db_ub);
    const double Fd = mu * (dn_ud + dn_ud) - dv;
    const double Fa = mu * (dn_ua + da_ud);
    const double Fb = mu * (dn_ub + db_ud);
    const double FE = sq[d * SQP + n] * Fd + sq[ja * SQP + n] * Fa + sq[jb * SQP + n] * Fb + kap * dn_th;
    double* o = Fout + ((size_t)e * 6 + f) * 4 * nf + a;
    // streaming stores: read once, by the neighbours' next stage kernel
    __builtin_nontemporal_store(Fd, &o[d * nf]);
    __builtin_nontemporal_store(Fa, &o[ja * nf]);
    __builtin_nontemporal_store(Fb, &o[jb * nf]);
    __builtin_nontemporal_store(FE, &o[3 * nf]);
  }
}

// Split BR1 lifting: the own part of the normal viscous flux at every face
// node of the element (into StageArgs.Fvf), from the element's own nodes
// only; one element per workgroup.  The stage kernel's epilogue does the same
// for its output state.
__global__ __launch_bounds__(PS::NTB) void k_lift_split(StageArgs A) {
  static_assert(PS::EPB == 1 && PS::TPE == PS::NTB, "one element per workgroup");
  __shared__ double sW[4 * SQP + 48 * nf];
  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;  // uniform over the workgroup
  const int t = threadIdx.x;
  if (t < nn) {
    const double* Ue = A.U + (size_t)e * 5 * nn;
    double u[5], P[7];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = Ue[v * nn + t];
    primitives<VF_PI, double, false>(u, A.gamma - 1.0, Ref{0.0, 0.0, 0.0}, P);
    store_own_q(sW, t, P);
  }
  __syncthreads();
  own_part_by_lines<PS::TPE>(A, e, t, sW, sW + 4 * SQP, A.Fvf);
}

// With BLEND (FP64) only the advective operator is blended: the viscous terms
// enter unweighted, and MODE_DIFF leaves them out.  SPLIT: the split BR1
// variant (StageArgs.split; FP64 Navier-Stokes without the eddy viscosity,
// walls or blending).
template <int VF, int EQ, bool BLEND, class R, bool WALL = false, bool SPLIT = false>
__global__ DG_STAGE_BOUNDS void k_stage(StageArgs A) {
  constexpr bool NS = (EQ >= 1);
  constexpr bool LES = (EQ == 2);
  constexpr bool MX = sizeof(R) == 4;
  static_assert(!(BLEND && MX), "the blended operator is FP64 only");
  static_assert(!WALL || (NS && !MX), "walls: FP64 Navier-Stokes");
  // LDS pool: primitives sP[7][nnp], face fluxes sF[6][5][nf], and for
  // Navier-Stokes the interface values sQ[6][4][nf] and the neighbours' normal
  // viscous fluxes sFn[6][4][nf].  The twelve viscous-flux components of all
  // nodes are later exchanged through sV[12][nnp], which overlays sP, sF and sQ
  // (all consumed by then) but not sFn.
  constexpr int oF = 7 * nnp, oQ = oF + 30 * nf, oFn = std::max(oQ + 24 * nf, 12 * nnp);
  constexpr int POOL = NS ? oFn + 24 * nf : oQ;
  static_assert(!NS || 12 * nnp <= oFn, "viscous exchange must not overlay sFn");
  constexpr int EPB = PS::EPB, TPE = PS::TPE, FI = PS::FI;
  __shared__ R sPoolAll[EPB][POOL];
  __shared__ R sB[NB_STAGE];
  __shared__ double sXAll[EPB][BLEND ? 5 : 1][BLEND ? nn : 1];
  __shared__ double sB64[BLEND ? NB_STAGE + nf : 1];  // with V^-1 (Vinv follows edge in the basis)

  const int e0 = EPB * element_of_block(blockIdx.x, A.chunk);
  if (e0 >= A.nelem) return;  // uniform over the workgroup
  const Slot sl = slot_of_thread<PS>(e0, A.nelem);
  const int e = sl.e, t = sl.t, tid = threadIdx.x;
  R* sPool = sPoolAll[sl.s];
  double (*sX)[BLEND ? nn : 1] = sXAll[sl.s];
  R (*sP)[nnp] = reinterpret_cast<R (*)[nnp]>(sPool);
  R (*sF)[5][nf] = reinterpret_cast<R (*)[5][nf]>(sPool + oF);
  R (*sQ)[4][nf] = reinterpret_cast<R (*)[4][nf]>(sPool + (NS ? oQ : 0));
  R (*sFn)[4][nf] = reinterpret_cast<R (*)[4][nf]>(sPool + (NS ? oFn : 0));
  R (*sV)[nnp] = reinterpret_cast<R (*)[nnp]>(sPool);
  const double gm1 = A.gamma - 1.0;
  // Memory round trip 1: neighbour indices of the thread's face items, the
  // node state and the basis.
  static_assert(EPB == 1, "one element per workgroup: its neighbours are uniform");
  const Nbr6 nb6 = uniform_nbr6(A.nbr, e);
  static_assert(!SPLIT || (EQ == 1 && !BLEND && !WALL && !MX), "split BR1: FP64 Navier-Stokes on the box");
  FaceData<NS, R, WALL, SPLIT> fd[FI];
#pragma unroll
  for (int k = 0; k < FI; ++k)
    if (t + k * TPE < 6 * nf) fd[k].it = face_item_geometry(nb6, t + k * TPE);
  // wall faces of the element (bit f): at most the two normal to wall_dir
  int wmask = 0;
  if (WALL) {
#pragma unroll
    for (int f = 0; f < 6; ++f) wmask |= nb6.n[f] < 0 ? 1 << f : 0;
  }
  const double* Ue = A.U + (size_t)e * 5 * nn;
  double u[5], gprev[5];
  if (t < nn) {
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = Ue[v * nn + t];
  }
  static_assert(NB_STAGE <= PS::NTB, "one basis entry per thread");
  const double bval = tid < NB_STAGE ? A.basis[tid] : 0.0;
  // V^-1 for the indicator of the stage output (blended Euler runs)
  const double vval = (BLEND && !NS && kFusedAlpha1 && tid >= NB_STAGE && tid < NB_STAGE + nf) ? A.basis[tid] : 0.0;
  const Ref ref = MX ? reference_state(A.U, gm1) : Ref{0.0, 0.0, 0.0};
  // Round trip 2: the face states (needs the neighbour indices).
#pragma unroll
  for (int k = 0; k < FI; ++k)
    if (t + k * TPE < 6 * nf) face_issue<NS, R, WALL, SPLIT>(A, e, fd[k], &nb6);
  if (tid < NB_STAGE) {
    sB[tid] = (R)bval;
    if (BLEND) sB64[tid] = bval;
  }
  if constexpr (BLEND && !NS && kFusedAlpha1)
    if (tid >= NB_STAGE && tid < NB_STAGE + nf) sB64[tid] = vval;
  const R* sDhat = sB + BL.Dhat();
  const R* sDw = sB + BL.Dw();
  const R* swinv = sB + BL.winv();
  const R invJ[3] = {(R)A.invJ[0], (R)A.invJ[1], (R)A.invJ[2]};

  R me[7];
  int ijk[3] = {0, 0, 0};
  if (t < nn) {
    primitives<VF, R, MX>(u, gm1, ref, me);
#pragma unroll
    for (int k = 0; k < 7; ++k)
      if (k < 6 || NS) sP[k][t] = me[k];
    ijk[0] = t % n1;
    ijk[1] = (t / n1) % n1;
    ijk[2] = t / nf;
  }
#pragma unroll
  for (int k = 0; k < FI; ++k)
    if (t + k * TPE < 6 * nf) face_item<VF, NS, R, MX, WALL, SPLIT>(A, fd[k], ref, sF, sQ, sFn);
  __syncthreads();

  R acc[5] = {0, 0, 0, 0, 0};
  R Fv[3][4];
  if (t < nn) {
    constexpr bool FG = NS && DG_FUSED_GRAD && !BLEND;
    R gs[3][4];
    volume_dir<VF, 0, R, FG>(sP, sDhat, swinv[0], t, ijk[0], me, invJ[0], (R)gm1, acc, sDw, gs[0]);
    volume_dir<VF, 1, R, FG>(sP, sDhat, swinv[0], t, ijk[1], me, invJ[1], (R)gm1, acc, sDw, gs[1]);
    volume_dir<VF, 2, R, FG>(sP, sDhat, swinv[0], t, ijk[2], me, invJ[2], (R)gm1, acc, sDw, gs[2]);
    // advective surface terms
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int id = ijk[d];
      const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
      if (id == 0 || id == N) {  // one branch for both faces (N >= 1)
        const int f = 2 * d + (id == N);
        const R c = invJ[d] * (id == N ? -swinv[N] : swinv[0]);
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] = fmaR(c, sF[f][v][a], acc[v]);
      }
    }
    if (NS && !BLEND) {  // blended: after the subcell pass (registers)
      R g[3][4];
      if (!FG) {
        lifted_gradient<R, nnp>(sP, sQ, sDw, swinv, t, ijk, invJ, g);
      } else {
      // BR1 gradient: line sums from the volume loop + diagonal + interface values
      const R qo[4] = {me[1], me[2], me[3], me[6]};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int id = ijk[d];
        const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
        R s[4] = {gs[d][0], gs[d][1], gs[d][2], gs[d][3]};
        if (id == 0 || id == N) {  // diagonal of Dw (zero inside) and the lifting term
          const int f = 2 * d + (id == N);
          const R cd = sDw[id * n1 + id];
          const R w = id == N ? swinv[N] : -swinv[0];
#pragma unroll
          for (int c = 0; c < 4; ++c) s[c] = fmaR(w, sQ[f][c][a], fmaR(cd, qo[c], s[c]));
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) g[d][c] = invJ[d] * s[c];
      }
      }
      node_viscous_flux<LES, R>(A, e, g, me, Fv);
    }
  }

  if (BLEND) {
    // (FP64 only: R = double)
    double al = 0.0;
    {
      double m = 0.0;
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const int nb = nb6.n[f];
        if (!WALL || nb >= 0) m = fmax(m, A.alpha1[nb]);  // a wall face spreads nothing
      }
      al = fmax(A.alpha1[e], A.aspread * m);
      if (al < A.amin) al = 0.0;
      if (t == 0 && A.alpha_out) A.alpha_out[e] = al;
    }
    // The subcell pass holds barriers: it runs when any element of the
    // workgroup is blended, each slot doing its work only if its own is.
    bool run = al > 0.0;
    if (EPB > 1) {
      __shared__ int sAny[EPB];
      if (sl.traw == 0 && threadIdx.x < EPB * TPE) sAny[sl.s] = sl.live && al > 0.0;
      __syncthreads();
      run = false;
#pragma unroll
      for (int k = 0; k < EPB; ++k) run = run || sAny[k] != 0;
    }
    if (run) {  // uniform over the workgroup
      const double* sxi = sB64 + BL.xi();
      const double* sedge = sB64 + BL.edge();
      const double* swinv64 = sB64 + BL.winv();
      const double (*sP64)[nnp] = reinterpret_cast<const double (*)[nnp]>(sP);
      const double (*sF64)[5][nf] = reinterpret_cast<const double (*)[5][nf]>(sF);
      double fv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
        __syncthreads();
        if (t < nn && ijk[d] < N && al > 0.0) {
          const int base = t - ijk[d] * st;
          double wl[5], wr[5], UL[5], UR[5], fs[5];
          subcell_face_state(sP64, base, st, ijk[d], true, A.recon, sxi, sedge, wl);
          subcell_face_state(sP64, base, st, ijk[d] + 1, false, A.recon, sxi, sedge, wr);
          prim_to_cons(wl, gm1, UL);
          prim_to_cons(wr, gm1, UR);
          surface_flux_dir<VF>(d, A.sf, UL, UR, A.gamma, fs);
#pragma unroll
          for (int v = 0; v < 5; ++v) sX[v][t] = fs[v];
        }
        __syncthreads();
        if (t < nn && al > 0.0) {
          const int id = ijk[d];
          const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
          const double c = A.invJ[d] * swinv64[id];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const double Fr = (id == N) ? sF64[2 * d + 1][v][a] : sX[v][t];
            const double Fl = (id == 0) ? sF64[2 * d][v][a] : sX[v][t - st];
            fv[v] -= c * (Fr - Fl);
          }
        }
      }
      if (!(al > 0.0)) {
        if (A.mode == MODE_DIFF) {
#pragma unroll
          for (int v = 0; v < 5; ++v) acc[v] = (R)0;
        }
      } else if (A.mode == MODE_DIFF) {
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] = (R)(fv[v] - (double)acc[v]);
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] = (R)((1.0 - al) * (double)acc[v] + al * fv[v]);
      }
    } else if (A.mode == MODE_DIFF) {
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[v] = (R)0;
    }
    if (NS && t < nn) {  // sP and sQ are intact: the subcell pass writes sX only
      R g[3][4];
      lifted_gradient<R, nnp>(sP, sQ, sDw, swinv, t, ijk, invJ, g);
      node_viscous_flux<LES, R>(A, e, g, me, Fv);
    }
  }

  // Runge-Kutta register (stages 2-5), loaded ahead of the viscous phase so
  // that its latency is hidden (earlier, its registers would be live across
  // the volume loop, the kernel's register peak).
  if (t < nn && A.mode != MODE_UT && A.A != 0.0) {
#pragma unroll
    for (int v = 0; v < 5; ++v) gprev[v] = __builtin_nontemporal_load(&A.G[(size_t)e * 5 * nn + t + v * nn]);
  }
  if (NS && !(BLEND && A.mode == MODE_DIFF)) {  // uniform over the workgroup
    // viscous divergence: all twelve flux components exchanged through LDS
    // once; with DG_VDIV_LINES a line pass (one thread per line of each
    // direction, 3 (N+1)^2 lines) replaces the n1 values of every line and
    // component by sum_l Dw_il Fv_l, in place (lines of one direction are
    // disjoint and each direction owns four rows), with the coefficients
    // uniform over the workgroup; each node then reads its 12 sums, instead
    // of reading n1 partners and coefficients per component.
    __syncthreads();
    if (t < nn) {
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < 4; ++c) sV[4 * d + c][t] = Fv[d][c];
    }
    __syncthreads();
#if DG_VDIV_LINES
    // one task per (line, pair of components): 6 (N+1)^2 tasks
    for (int q = tid; q < 6 * nf; q += PS::NTB) {
      const int cp = q & 1, ql = q >> 1;
      const int d = ql / nf, a = ql - d * nf;
      const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
      const int base = face_node(d, 0, a);
      R* r0 = sV[4 * d + 2 * cp];
      R* r1 = sV[4 * d + 2 * cp + 1];
      R v0[n1], v1[n1];
#pragma unroll
      for (int l = 0; l < n1; ++l) {
        v0[l] = r0[base + l * st];
        v1[l] = r1[base + l * st];
      }
#pragma unroll
      for (int i = 0; i < n1; ++i) {
        R s0 = 0, s1 = 0;
#pragma unroll
        for (int l = 0; l < n1; ++l) {
          const R c = sDw[i * n1 + l];  // the same address in every lane (broadcast)
          s0 = fmaR(c, v0[l], s0);
          s1 = fmaR(c, v1[l], s1);
        }
        r0[base + i * st] = s0;
        r1[base + i * st] = s1;
      }
    }
    __syncthreads();
#endif
    if (t < nn) {
      const R h2 = (R)0.5;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int id = ijk[d];
#if DG_VDIV_LINES
        R s0 = sV[4 * d + 0][t], s1 = sV[4 * d + 1][t], s2 = sV[4 * d + 2][t], s3 = sV[4 * d + 3][t];
#else
        const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
        const int base = t - id * st;
        const R* crow = sDw + id * n1;
        R s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
        for (int l = 0; l < n1; ++l) {
          const int m = base + l * st;
          const R c = crow[l];
          s0 = fmaR(c, sV[4 * d + 0][m], s0);
          s1 = fmaR(c, sV[4 * d + 1][m], s1);
          s2 = fmaR(c, sV[4 * d + 2][m], s2);
          s3 = fmaR(c, sV[4 * d + 3][m], s3);
        }
#endif
        const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
        if (id == 0 || id == N) {  // F*v = mean with the neighbour's normal viscous flux (sFn)
          const int f = 2 * d + (id == N);
          const bool wf = WALL && ((wmask >> f) & 1);  // wall: sFn is F*v itself
          const R w = (wf ? (R)1 : h2) * (id == N ? swinv[N] : -swinv[0]);
          const R o = wf ? (R)0 : (R)1;
          s0 = fmaR(w, fmaR(o, Fv[d][0], sFn[f][0][a]), s0);
          s1 = fmaR(w, fmaR(o, Fv[d][1], sFn[f][1][a]), s1);
          s2 = fmaR(w, fmaR(o, Fv[d][2], sFn[f][2][a]), s2);
          s3 = fmaR(w, fmaR(o, Fv[d][3], sFn[f][3][a]), s3);
        }
        acc[1] = fmaR(invJ[d], s0, acc[1]);
        acc[2] = fmaR(invJ[d], s1, acc[2]);
        acc[3] = fmaR(invJ[d], s2, acc[3]);
        acc[4] = fmaR(invJ[d], s3, acc[4]);
      }
    }
  }

  if (t < nn) {
    double ut[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) ut[v] = (double)acc[v];
    if (MX) ut[4] += ref.h * ut[0];  // undo the energy-flux shift h0 * (mass flux)
    const size_t o = (size_t)e * 5 * nn + t;
    if (A.mode != MODE_RK) {  // MODE_UT, MODE_DIFF
#pragma unroll
      for (int v = 0; v < 5; ++v) A.Ut[o + v * nn] = ut[v];
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        double gv = ut[v];
        if (A.A != 0.0) gv = A.A * gprev[v] + ut[v];
        // streaming stores (the register is read once, by this element's next
        // stage; the state by the next stage kernel)
        if (A.writeG) __builtin_nontemporal_store(gv, &A.G[o + v * nn]);
        u[v] = u[v] + A.Bdt * gv;  // the stage output, kept for the indicator below
        __builtin_nontemporal_store(u[v], &A.Uout[o + v * nn]);
      }
    }
  }
  // Split BR1, Runge-Kutta stage: the own part of the normal viscous flux of
  // the stage output at the element's face nodes, for the next stage (what
  // k_lift_split computes, here from the values just written and still in
  // registers).
  if constexpr (SPLIT) {
    if (A.Fvf_next && A.mode == MODE_RK) {  // uniform over the workgroup
      static_assert(4 * SQP + 48 * nf <= POOL, "lifted variables and line sums in the LDS pool");
      double* sq = reinterpret_cast<double*>(sPool);
      __syncthreads();  // the pool's last readers (the viscous pass) are done
      if (t < nn) {
        double P[7];
        primitives<VF_PI, double, false>(u, gm1, Ref{0.0, 0.0, 0.0}, P);
        store_own_q(sq, t, P);
      }
      __syncthreads();
      own_part_by_lines<TPE>(A, e, t, sq, sq + 4 * SQP, A.Fvf_next);
    }
  }
  // Euler only: measured on the blended Navier-Stokes stage (N = 4, its
  // occupancy limited by LDS) the epilogue's barriers cost more than the
  // separate indicator launch it saves.
  if constexpr (BLEND && !NS && kFusedAlpha1) {
    if (A.alpha1_next && A.mode == MODE_RK) {  // uniform over the workgroup
      static_assert(POOL >= 2 * nn + 3 * NWAVE && PS::NTB == NT && BL.Vinv() == NB_STAGE,
                    "indicator scratch in the LDS pool, V^-1 after the stage basis");
      double* sq = reinterpret_cast<double*>(sPool);
      double* st = sq + nn;
      double* sred = st + nn;
      const double* sVi = sB64 + NB_STAGE;
      __syncthreads();  // the pool's last readers (subcell and viscous passes) are done
      const double qt = t < nn ? indicator_q(u, gm1) : 0.0;
      const double a1 = element_alpha1(A, sVi, sq, st, sred, t, ijk, qt);
      if (t == 0) A.alpha1_next[e] = a1;
    }
  }
}

// ---------------------------------------------------------------------------
// BR1 lifting pass (Navier-Stokes): normal viscous flux at the element's own
// face nodes -> Fvf[e][f][c][a] (type R), read by the neighbours' stage kernels.
// ---------------------------------------------------------------------------
template <class R, bool MX>
__device__ __forceinline__ void lift_face_q(const StageArgs& A, const FaceItem& it, const double L[5],
                                            const double Rr[5], const Ref& ref, R (*sQ)[4][nf]) {
  const State64 sL = state64<0>(L, A.gamma - 1.0), sR = state64<0>(Rr, A.gamma - 1.0);
  R qs[4];
  interface_q<0, R, MX>(sL, sR, ref, qs);
  store_q(it, qs, sQ);
}



// Index of volume node n on the face of axis j (lower remaining axis first).
__device__ __forceinline__ int face_index(int j, int i0, int i1, int i2) {
  return j == 0 ? i1 + n1 * i2 : (j == 1 ? i0 + n1 * i2 : i0 + n1 * i1);
}

// Derivative along tangential axis j of the normal velocity u_d and of u_j at
// node n (BR1: line sum with Dw plus the lifting term of axis j's faces); with
// THIRD also that of u_o (o: the other tangential axis).
template <class R, bool THIRD = false>
__device__ __forceinline__ void tangential_pair(const R (*sq)[nn], const R (*sQ)[4][nf], const R* sDw,
                                                const R* swinv, int n, int d, int j, int i0, int i1, int i2,
                                                R invJj, R& dud, R& duj, int o = 0, R* duo = nullptr) {
  const int sj = axis_stride(j);
  const int id = j == 0 ? i0 : (j == 1 ? i1 : i2);
  const int base = n - id * sj;
  const R* crow = sDw + id * n1;
  const R* qd = sq[d];
  const R* qj = sq[j];
  const R* qo = sq[o];
  R s0 = 0, s1 = 0, s2 = 0;
#pragma unroll 2
  for (int l = 0; l < n1; ++l) {
    const R c = crow[l];
    s0 = fmaR(c, qd[base + l * sj], s0);
    s1 = fmaR(c, qj[base + l * sj], s1);
    if (THIRD) s2 = fmaR(c, qo[base + l * sj], s2);
  }
  if (id == 0 || id == N) {
    const int f = 2 * j + (id == N);
    const R w = id == N ? swinv[N] : -swinv[0];
    const int a = face_index(j, i0, i1, i2);
    s0 = fmaR(w, sQ[f][d][a], s0);
    s1 = fmaR(w, sQ[f][j][a], s1);
    if (THIRD) s2 = fmaR(w, sQ[f][o][a], s2);
  }
  dud = invJj * s0;
  duj = invJj * s1;
  if (THIRD) *duo = invJj * s2;
}

// Normal viscous flux at face node q of the element (face f = q / nf, normal
// axis d), from sq = (u, v, w, theta[, rho]) at the nodes and the interface
// values sQ.  Only the gradient components it needs are formed: the
// derivatives along d of (u, v, w, theta) and, along each tangential axis j,
// those of u_d and u_j (with the eddy viscosity also the third velocity
// component, for the full strain rate).
template <class R, bool LES>
__device__ __forceinline__ void lift_face_node(const StageArgs& A, int e, const FaceItem& it, const R (*sq)[nn],
                                               const R (*sQ)[4][nf], const R* sB, const R invJ[3]) {
  const int n = it.nown, d = it.d;
  const int i0 = n % n1, i1 = (n / n1) % n1, i2 = n / nf;
  const R* sDw = sB + BL.Dw();
  const R* swinv = sB + BL.winv();
  const int ja = d == 0 ? 1 : 0, jb = d == 2 ? 1 : 2;  // tangential axes
  // normal line: derivatives of u, v, w, theta along d
  const int sn = axis_stride(d);
  const int id = it.side ? N : 0;
  const int base = n - id * sn;
  const R* crow = sDw + id * n1;
  R g0 = 0, g1 = 0, g2 = 0, g3 = 0;
#pragma unroll 2
  for (int l = 0; l < n1; ++l) {
    const int m = base + l * sn;
    const R c = crow[l];
    g0 = fmaR(c, sq[0][m], g0);
    g1 = fmaR(c, sq[1][m], g1);
    g2 = fmaR(c, sq[2][m], g2);
    g3 = fmaR(c, sq[3][m], g3);
  }
  {
    const R w = it.side ? swinv[N] : -swinv[0];
    g0 = fmaR(w, sQ[it.f][0][it.a], g0);
    g1 = fmaR(w, sQ[it.f][1][it.a], g1);
    g2 = fmaR(w, sQ[it.f][2][it.a], g2);
    g3 = fmaR(w, sQ[it.f][3][it.a], g3);
  }
  const R Jd = d == 0 ? invJ[0] : (d == 1 ? invJ[1] : invJ[2]);
  g0 *= Jd;
  g1 *= Jd;
  g2 *= Jd;
  g3 *= Jd;
  R da_ud, da_ua, db_ud, db_ub, da_ub = 0, db_ua = 0;
  tangential_pair<R, LES>(sq, sQ, sDw, swinv, n, d, ja, i0, i1, i2, ja == 0 ? invJ[0] : invJ[1], da_ud, da_ua, jb,
                          &da_ub);
  tangential_pair<R, LES>(sq, sQ, sDw, swinv, n, d, jb, i0, i1, i2, jb == 1 ? invJ[1] : invJ[2], db_ud, db_ub, ja,
                          &db_ua);
  const R dn_ud = d == 0 ? g0 : (d == 1 ? g1 : g2);
  const R dn_ua = ja == 0 ? g0 : g1;
  const R dn_ub = jb == 1 ? g1 : g2;
  R mu = (R)A.mu, kap = (R)A.kappa;
  if (LES) {  // strain rate from the full velocity gradient in the face frame
    const R sa = dn_ua + da_ud, sb = dn_ub + db_ud, sc = da_ub + db_ua;
    const R S2 = (R)2 * (dn_ud * dn_ud + da_ua * da_ua + db_ub * db_ub) + sa * sa + sb * sb + sc * sc;
    const double cs = A.cs_elem ? A.cs_elem[e] : A.cs;
    const R mut = sq[LES ? 4 : 0][n] * (R)(cs * cs * A.delta2) * sqrt_nonneg(S2);
    mu += mut;
    kap = fmaR((R)A.ktf, mut, kap);
  }
  const R dv = (R)(2.0 / 3.0) * mu * (dn_ud + da_ua + db_ub);
  const R Fd = mu * (dn_ud + dn_ud) - dv;
  const R Fa = mu * (dn_ua + da_ud);
  const R Fb = mu * (dn_ub + db_ud);
  const R ud = sq[d][n], ua = sq[ja][n], ub = sq[jb][n];
  const R FE = ud * Fd + ua * Fa + ub * Fb + kap * g3;
  R* out = reinterpret_cast<R*>(A.Fvf) + ((size_t)e * 6 + it.f) * 4 * nf + it.a;
  __builtin_nontemporal_store(Fd, &out[d * nf]);  // streaming: read once, by the neighbour
  __builtin_nontemporal_store(Fa, &out[ja * nf]);
  __builtin_nontemporal_store(Fb, &out[jb * nf]);
  __builtin_nontemporal_store(FE, &out[3 * nf]);
}

// Register budget of the lifting kernel: 8 waves per SIMD (64 VGPRs) with one
// face item per thread, else 4; the line sums with run-time strides are only
// partly unrolled so that the partner loads in flight fit in it.
template <class R, bool LES, bool WALL = false>
__global__ __launch_bounds__(PL::NTB, PL::FI == 1 && N >= 2 ? 8 : 4) void k_lift(StageArgs A) {
  constexpr bool MX = sizeof(R) == 4;
  constexpr int EPB = PL::EPB, TPE = PL::TPE, FI = PL::FI;
  __shared__ R sB[NB_STAGE];
  __shared__ R sqAll[EPB][LES ? 5 : 4][nn];  // u, v, w, theta (, rho)
  __shared__ R sQAll[EPB][6][4][nf];
  const int e0 = EPB * element_of_block(blockIdx.x, A.chunk);
  if (e0 >= A.nelem) return;  // uniform over the workgroup
  const Slot sl = slot_of_thread<PL>(e0, A.nelem);
  const int e = sl.e, t = sl.t, tid = threadIdx.x;
  R (*sq)[nn] = sqAll[sl.s];
  R (*sQ)[4][nf] = sQAll[sl.s];
  const double gm1 = A.gamma - 1.0;
  // Round trip 1: neighbour indices, node state, basis; round trip 2: face states.
  // neighbours of the workgroup's elements (scalar loads), then the slot's
  Nbr6 nbs[EPB];
#pragma unroll
  for (int k = 0; k < EPB; ++k) nbs[k] = uniform_nbr6(A.nbr, min(e0 + k, A.nelem - 1));
  Nbr6 nb6 = nbs[0];
#pragma unroll
  for (int k = 1; k < EPB; ++k)
    if (sl.s == k) nb6 = nbs[k];
  FaceItem its[FI];
#pragma unroll
  for (int k = 0; k < FI; ++k)
    if (t + k * TPE < 6 * nf) its[k] = face_item_geometry(nb6, t + k * TPE);
  const double* Ue = A.U + (size_t)e * 5 * nn;
  double u[5];
  if (t < nn) {
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = Ue[v * nn + t];
  }
  const double bval = tid < NB_STAGE ? A.basis[tid] : 0.0;
  const Ref ref = MX ? reference_state(A.U, gm1) : Ref{0.0, 0.0, 0.0};
  double FL[FI][5], FR[FI][5];
#pragma unroll
  for (int k = 0; k < FI; ++k)
    if (t + k * TPE < 6 * nf) face_loads_w<WALL>(A.U, e, its[k], FL[k], FR[k]);
  if (tid < NB_STAGE) sB[tid] = (R)bval;
  const R invJ[3] = {(R)A.invJ[0], (R)A.invJ[1], (R)A.invJ[2]};
  if (t < nn) {
    R P[7];
    primitives<VF_PI, R, MX>(u, gm1, ref, P);
    sq[0][t] = P[1];
    sq[1][t] = P[2];
    sq[2][t] = P[3];
    sq[3][t] = P[6];
    if (LES) sq[LES ? 4 : 0][t] = P[0];
  }
#pragma unroll
  for (int k = 0; k < FI; ++k)
    if (t + k * TPE < 6 * nf) lift_face_q<R, MX>(A, its[k], FL[k], FR[k], ref, sQ);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < FI; ++k)
    if (t + k * TPE < 6 * nf && !(WALL && its[k].nb < 0)) lift_face_node<R, LES>(A, e, its[k], sq, sQ, sB, invJ);
}

// Wall-model flux at every wall face node (FP64): thread -> (side p, element
// of the wall plane, face node a); the flux goes into Fvf[e][f][c][a] of the
// wall face f = 2 wall_dir + p, in the global components (x, y, z momentum,
// energy), read by the stage kernel of the same element.
__global__ __launch_bounds__(256) void k_wall_flux(StageArgs A) {
  const int wd = A.wall_dir;
  const int da = wd == 0 ? 1 : 0, db = wd == 2 ? 1 : 2;  // the plane's directions
  const int na = A.ne[da], nb = A.ne[db];
  const long long total = 2LL * na * nb * nf;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int a = (int)(id % nf);
  const long long r = id / nf;
  const int ia = (int)(r % na), ib = (int)((r / na) % nb), p = (int)(r / ((long long)na * nb));
  int ix[3];
  ix[wd] = p ? A.ne[wd] - 1 : 0;
  ix[da] = ia;
  ix[db] = ib;
  const int e = ix[0] + A.ne[0] * (ix[1] + A.ne[1] * ix[2]);
  const int f = 2 * wd + p;
  const FaceItem it = face_item_geometry(A.nbr, e, f * nf + a);
  const double* Ue = A.U + (size_t)e * 5 * nn;
  double g[4];
  wall_model_flux(A, Ue[it.nown], Ue[it.nnb], Ue[it.k1 * nn + it.nnb], Ue[it.k2 * nn + it.nnb], p ? -1.0 : 1.0, g);
  double* out = A.Fvf + ((size_t)e * 6 + f) * 4 * nf + a;
  out[it.d * nf] = g[0];
  out[(it.k1 - 1) * nf] = g[1];
  out[(it.k2 - 1) * nf] = g[2];
  out[3 * nf] = g[3];
}

// ===========================================================================
// Reverse mode: vector-Jacobian product of the FP64 operator (the blending,
// curved meshes, the eddy viscosity and the wall model further below or as
// variants of these kernels).
//
//   U_bar = (dL/dU)^T lambda,   lambda = cotangent of U_t.
//
// * Volume integral: F# is symmetric, so node n's cotangent is
//     sum_d sum_l (d1 F#_d(U_n, U_l))^T w_nl,
//     w_nl = -(2/dx_d)(Dhat_{i l} lambda_n + Dhat_{l i} lambda_l),
//   evaluated by hand-derived reverse mode of the two-point flux in primitive
//   variables, then pulled back to conservative variables once per node.
// * Interface fluxes: each element pulls the flux cotangent (which collects
//   lambda of both elements) back to its own face state by a hand-derived
//   reverse sweep of f*(U-, U+) (riemann_vjp), one per face node.
// * BR1 viscous terms: reverse of Fv(U, g), of g(q, q*) and of q(U).  The
//   interface value q* couples the lifted gradients of both elements, so a
//   first pass (k_vjp_lift) writes the cotangent of each element's normal
//   gradient at its own face nodes, which the neighbours read.
// Non-smooth points use the same conventions as the oracle's dual numbers:
// d|x|/dx = 0 at 0 and max(a, b) takes the mean derivative at a tie.
// ===========================================================================
// sign(x) with 0 at 0: the derivative of |x| under the adjoint's convention.
__device__ __forceinline__ double sgn0(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// Reverse mode of the interface flux f* = F#(L, R) - Dis/2 of riemann_rot
// (FP64, rotated frame: normal momentum in slot 1), from conservative states:
// for the flux cotangent gb, the cotangents Lb and Rb of both states, in one
// hand-derived sweep.  Non-smooth points as in the oracle's dual numbers:
// |x|' = 0 at 0, max(a, b) takes half of each derivative at a tie.
template <int VF>
__device__ __forceinline__ void riemann_vjp(int sf, const double L[5], const double R[5], double gamma,
                                            const double gb[5], double Lb[5], double Rb[5]) {
  const double gm1 = gamma - 1.0;
  const double iL = rcp64(L[0]), iR = rcp64(R[0]);
  const double unL = L[1] * iL, u1L = L[2] * iL, u2L = L[3] * iL;
  const double unR = R[1] * iR, u1R = R[2] * iR, u2R = R[3] * iR;
  const double pL = gm1 * (L[4] - 0.5 * (L[1] * unL + L[2] * u1L + L[3] * u2L));
  const double pR = gm1 * (R[4] - 0.5 * (R[1] * unR + R[2] * u1R + R[3] * u2R));
  const double hL = (L[4] + pL) * iL, hR = (R[4] + pR) * iR;
  // cotangents of the primitive intermediates of each side (normal and
  // tangential velocities, pressure, enthalpy, 1/rho)
  double bunL = 0.0, bu1L = 0.0, bu2L = 0.0, bpL = 0.0, bhL = 0.0, biL = 0.0;
  double bunR = 0.0, bu1R = 0.0, bu2R = 0.0, bpR = 0.0, bhR = 0.0, biR = 0.0;
#pragma unroll
  for (int v = 0; v < 5; ++v) Lb[v] = Rb[v] = 0.0;
  // central part
  if (VF == VF_STD) {
    Lb[1] += 0.5 * (gb[0] + gb[1] * unL + gb[2] * u1L + gb[3] * u2L + gb[4] * hL);
    Rb[1] += 0.5 * (gb[0] + gb[1] * unR + gb[2] * u1R + gb[3] * u2R + gb[4] * hR);
    bunL += 0.5 * gb[1] * L[1];
    bunR += 0.5 * gb[1] * R[1];
    bpL += 0.5 * gb[1];
    bpR += 0.5 * gb[1];
    bu1L += 0.5 * gb[2] * L[1];
    bu1R += 0.5 * gb[2] * R[1];
    bu2L += 0.5 * gb[3] * L[1];
    bu2R += 0.5 * gb[3] * R[1];
    bhL += 0.5 * gb[4] * L[1];
    bhR += 0.5 * gb[4] * R[1];
  } else {
    const double um0 = 0.5 * (unL + unR), um1 = 0.5 * (u1L + u1R), um2 = 0.5 * (u2L + u2R);
    const double rm = 0.5 * (L[0] + R[0]), pm = 0.5 * (pL + pR);
    const double fr = rm * um0;
    double bfr = gb[0] + gb[1] * um0 + gb[2] * um1 + gb[3] * um2;
    double bum0 = gb[1] * fr, bpm = gb[1];
    const double bum1 = gb[2] * fr, bum2 = gb[3] * fr;
    if (VF == VF_KG) {
      const double xm = 0.5 * (L[4] * iL + R[4] * iR);
      bfr += gb[4] * xm;
      bpm += gb[4] * um0;
      bum0 += gb[4] * pm;
      const double bxm = 0.5 * gb[4] * fr;
      Lb[4] += bxm * iL;
      Rb[4] += bxm * iR;
      biL += bxm * L[4];
      biR += bxm * R[4];
    } else {
      bfr += gb[4] * 0.5 * (hL + hR);
      bhL += 0.5 * gb[4] * fr;
      bhR += 0.5 * gb[4] * fr;
    }
    bum0 += bfr * rm;
    const double brm = bfr * um0;
    Lb[0] += 0.5 * brm;
    Rb[0] += 0.5 * brm;
    bpL += 0.5 * bpm;
    bpR += 0.5 * bpm;
    bunL += 0.5 * bum0;
    bunR += 0.5 * bum0;
    bu1L += 0.5 * bum1;
    bu1R += 0.5 * bum1;
    bu2L += 0.5 * bum2;
    bu2R += 0.5 * bum2;
  }
  if (sf == SF_LLF) {
    const double cL = sqrt64(gamma * pL * iL), cR = sqrt64(gamma * pR * iR);
    const double aL = fabs(unL) + cL, aR = fabs(unR) + cR;
    const double hl = 0.5 * fmax(aL, aR);
    double bhl = 0.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      bhl -= gb[v] * (R[v] - L[v]);
      Lb[v] += hl * gb[v];
      Rb[v] -= hl * gb[v];
    }
    const double baL = aL > aR ? 0.5 * bhl : (aR > aL ? 0.0 : 0.25 * bhl);
    const double baR = aR > aL ? 0.5 * bhl : (aL > aR ? 0.0 : 0.25 * bhl);
    bunL += baL * sgn0(unL);
    bunR += baR * sgn0(unR);
    const double kL = 0.5 * gamma * baL * rcp64(cL), kR = 0.5 * gamma * baR * rcp64(cR);
    bpL += kL * iL;
    biL += kL * pL;
    bpR += kR * iR;
    biR += kR * pR;
  } else if (sf == SF_ROE) {
    const double sL = sqrt64(L[0]), sR = sqrt64(R[0]);
    const double inv = rcp64(sL + sR);
    const double ut0 = (sL * unL + sR * unR) * inv;
    const double ut1 = (sL * u1L + sR * u1R) * inv;
    const double ut2 = (sL * u2L + sR * u2R) * inv;
    const double Ht = (sL * hL + sR * hR) * inv;
    const double rt = sL * sR;
    const double q2 = ut0 * ut0 + ut1 * ut1 + ut2 * ut2;
    const double c2 = gm1 * (Ht - 0.5 * q2);
    const double ct = sqrt64(c2);
    const double ic2 = rcp64(c2);
    const double dp = pR - pL;
    const double dun = unR - unL, dt1 = u1R - u1L, dt2 = u2R - u2L;
    const double a1 = 0.5 * (dp - rt * ct * dun) * ic2;
    const double a5 = 0.5 * (dp + rt * ct * dun) * ic2;
    const double a2 = (R[0] - L[0]) - dp * ic2;
    const double l1 = fabs(ut0 - ct), l5 = fabs(ut0 + ct), l2 = fabs(ut0);
    const double w1 = l1 * a1, w5 = l5 * a5;
    // cotangents of the dissipation terms (f = g - D/2)
    const double bD0 = -0.5 * gb[0], bDn = -0.5 * gb[1], bD1 = -0.5 * gb[2], bD2 = -0.5 * gb[3],
                 bD4 = -0.5 * gb[4];
    const double tt = ut1 * dt1 + ut2 * dt2;
    double bw1 = bD0 + bDn * (ut0 - ct) + (bD1 * ut1 + bD2 * ut2) + bD4 * (Ht - ct * ut0);
    double bw5 = bD0 + bDn * (ut0 + ct) + (bD1 * ut1 + bD2 * ut2) + bD4 * (Ht + ct * ut0);
    double bl2 = bD0 * a2 + bDn * a2 * ut0 + bD1 * (a2 * ut1 + rt * dt1) + bD2 * (a2 * ut2 + rt * dt2) +
                 bD4 * (a2 * 0.5 * q2 + rt * tt);
    double ba2 = l2 * (bD0 + bDn * ut0 + bD1 * ut1 + bD2 * ut2 + bD4 * 0.5 * q2);
    const double wsum = w1 + w5 + l2 * a2;
    double but0 = bDn * wsum + bD4 * ct * (w5 - w1);
    double but1 = bD1 * wsum + bD4 * l2 * rt * dt1;
    double but2 = bD2 * wsum + bD4 * l2 * rt * dt2;
    double bct = bDn * (w5 - w1) + bD4 * ut0 * (w5 - w1);
    double bHt = bD4 * (w1 + w5);
    double bq2 = bD4 * l2 * a2 * 0.5;
    double brt = l2 * (bD1 * dt1 + bD2 * dt2 + bD4 * tt);
    const double bdt1 = l2 * rt * (bD1 + bD4 * ut1);
    const double bdt2 = l2 * rt * (bD2 + bD4 * ut2);
    // w1 = l1 a1, w5 = l5 a5; the absolute values
    const double bl1 = bw1 * a1, ba1 = bw1 * l1;
    const double bl5 = bw5 * a5, ba5 = bw5 * l5;
    const double s1 = sgn0(ut0 - ct), s5 = sgn0(ut0 + ct);
    but0 += bl1 * s1 + bl5 * s5 + bl2 * sgn0(ut0);
    bct += -bl1 * s1 + bl5 * s5;
    // wave strengths
    const double bdr = ba2;
    double bdp = -ba2 * ic2 + 0.5 * (ba1 + ba5) * ic2;
    double bic2 = -ba2 * dp + ba1 * 0.5 * (dp - rt * ct * dun) + ba5 * 0.5 * (dp + rt * ct * dun);
    const double kd = 0.5 * (ba5 - ba1) * ic2;
    brt += kd * ct * dun;
    bct += kd * rt * dun;
    const double bdun = kd * rt * ct;
    // sound speed and Roe averages
    double bc2 = -bic2 * ic2 * ic2 + bct * 0.5 * rcp64(ct);
    bHt += gm1 * bc2;
    bq2 -= 0.5 * gm1 * bc2;
    but0 += 2.0 * ut0 * bq2;
    but1 += 2.0 * ut1 * bq2;
    but2 += 2.0 * ut2 * bq2;
    double bsL = brt * sR, bsR = brt * sL;
    const double binv = but0 * (sL * unL + sR * unR) + but1 * (sL * u1L + sR * u1R) + but2 * (sL * u2L + sR * u2R) +
                        bHt * (sL * hL + sR * hR);
    bsL += inv * (but0 * unL + but1 * u1L + but2 * u2L + bHt * hL);
    bsR += inv * (but0 * unR + but1 * u1R + but2 * u2R + bHt * hR);
    bunL += but0 * sL * inv;
    bunR += but0 * sR * inv;
    bu1L += but1 * sL * inv;
    bu1R += but1 * sR * inv;
    bu2L += but2 * sL * inv;
    bu2R += but2 * sR * inv;
    bhL += bHt * sL * inv;
    bhR += bHt * sR * inv;
    const double bS = -binv * inv * inv;
    bsL += bS;
    bsR += bS;
    Lb[0] += bsL * 0.5 * rcp64(sL) - bdr;
    Rb[0] += bsR * 0.5 * rcp64(sR) + bdr;
    bpL -= bdp;
    bpR += bdp;
    bunL -= bdun;
    bunR += bdun;
    bu1L -= bdt1;
    bu1R += bdt1;
    bu2L -= bdt2;
    bu2R += bdt2;
  }
  // primitives -> conservative state, each side: h = (E + p)/rho,
  // p = (g-1)(E - (m . u)/2), u = m/rho
  {
    Lb[4] += bhL * iL;
    bpL += bhL * iL;
    biL += bhL * (L[4] + pL);
    Lb[4] += gm1 * bpL;
    const double kp = -0.5 * gm1 * bpL;
    Lb[1] += kp * unL;
    Lb[2] += kp * u1L;
    Lb[3] += kp * u2L;
    bunL += kp * L[1];
    bu1L += kp * L[2];
    bu2L += kp * L[3];
    Lb[1] += bunL * iL;
    Lb[2] += bu1L * iL;
    Lb[3] += bu2L * iL;
    biL += bunL * L[1] + bu1L * L[2] + bu2L * L[3];
    Lb[0] -= biL * iL * iL;
  }
  {
    Rb[4] += bhR * iR;
    bpR += bhR * iR;
    biR += bhR * (R[4] + pR);
    Rb[4] += gm1 * bpR;
    const double kp = -0.5 * gm1 * bpR;
    Rb[1] += kp * unR;
    Rb[2] += kp * u1R;
    Rb[3] += kp * u2R;
    bunR += kp * R[1];
    bu1R += kp * R[2];
    bu2R += kp * R[3];
    Rb[1] += bunR * iR;
    Rb[2] += bu1R * iR;
    Rb[3] += bu2R * iR;
    biR += bunR * R[1] + bu1R * R[2] + bu2R * R[3];
    Rb[0] -= biR * iR * iR;
  }
}

// Cotangent of the lifted viscous flux at node m in all three directions,
// Fvb[d][c] (c = momentum x, y, z, energy), from lambda along the three lines
// through m (sLam, components 1..4) and lambda of the neighbours on the faces
// containing m (sLn[f][c][a], components 1..4):
//   Fvb_d(m) = (2/dx_d) [ sum_n Dw_{i(n) i(m)} lambda_n
//                         + 1/2 delta_{i N}(lambda_m / w_N - lambda_nb+ / w_0)
//                         + 1/2 delta_{i 0}(lambda_nb- / w_N - lambda_m / w_0) ].
// wmask: bit f set for wall faces, whose surface term is the wall model's
// flux (no own or neighbour share of the lifted viscous flux).
__device__ __forceinline__ void viscous_flux_cotangent(const double (*sLam)[nn], const double (*sLn)[4][nf],
                                                       const double* sDw, const double* swinv, int m,
                                                       const int ijk[3], const double invJ[3], double Fvb[3][4],
                                                       int wmask = 0) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
    const int id = ijk[d];
    const int base = m - id * st;
    const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      const double c = sDw[l * n1 + id];  // Dw transposed
      const int k = base + l * st;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) s[cc] = fma(c, sLam[1 + cc][k], s[cc]);
    }
    if (id == N && !((wmask >> (2 * d + 1)) & 1)) {
#pragma unroll
      for (int cc = 0; cc < 4; ++cc)
        s[cc] += 0.5 * (swinv[N] * sLam[1 + cc][m] - swinv[0] * sLn[2 * d + 1][cc][a]);
    }
    if (id == 0 && !((wmask >> (2 * d)) & 1)) {
#pragma unroll
      for (int cc = 0; cc < 4; ++cc)
        s[cc] += 0.5 * (swinv[N] * sLn[2 * d][cc][a] - swinv[0] * sLam[1 + cc][m]);
    }
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) Fvb[d][cc] = invJ[d] * s[cc];
  }
}

// Cotangent of the lifted gradient g[a][b] (b = u, v, w, theta) from the
// viscous-flux cotangent: with taub_jd = Fvb_d[j] + u_j Fvb_d[E],
//   gb[a][b] = mu (taub_ba + taub_ab) - 2/3 mu delta_ab sum_j taub_jj,  gb[a][3] = kappa Fvb_a[E].
__device__ __forceinline__ void gradient_cotangent(const double Fvb[3][4], const double u[3], double mu,
                                                   double kappa, double gb[3][4]) {
  double tb[3][3];  // tb[j][d]
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int d = 0; d < 3; ++d) tb[j][d] = fma(u[j], Fvb[d][3], Fvb[d][j]);
  const double tr = (2.0 / 3.0) * mu * (tb[0][0] + tb[1][1] + tb[2][2]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int b = 0; b < 3; ++b) gb[a][b] = mu * (tb[b][a] + tb[a][b]) - (a == b ? tr : 0.0);
    gb[a][3] = kappa * Fvb[a][3];
  }
}

// With the Smagorinsky model: the cotangent of the lifted gradient with the
// effective coefficients mu + mu_t, kappa + ktf mu_t (mu_t = rho csd2 |S|,
// |S|^2 = 2 S_ij S_ij), plus the pullback of mu_t through |S| (derivative 0
// where |S| = 0) into gb and through rho into rhob:
//   mub = sum_d [ sum_j taub_jd tauhat_dj + ktf Fvb_d[E] g[d][3] ],
//   tauhat_dj = g[d][j] + g[j][d] - 2/3 delta_dj div.
__device__ __forceinline__ void les_gradient_cotangent(const double Fvb[3][4], const double u[3],
                                                       const double g[3][4], double rho, double mu, double kappa,
                                                       double csd2, double ktf, double gb[3][4], double& rhob) {
  const double a = g[0][1] + g[1][0], b = g[0][2] + g[2][0], c = g[1][2] + g[2][1];
  const double S2 = 2.0 * (g[0][0] * g[0][0] + g[1][1] * g[1][1] + g[2][2] * g[2][2]) + a * a + b * b + c * c;
  const double Sm = sqrt_nonneg(S2);
  const double mut = rho * csd2 * Sm;
  gradient_cotangent(Fvb, u, mu + mut, fma(ktf, mut, kappa), gb);
  const double tr = (2.0 / 3.0) * (g[0][0] + g[1][1] + g[2][2]);
  double mub = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double th = g[d][j] + g[j][d] - (j == d ? tr : 0.0);
      mub = fma(fma(u[j], Fvb[d][3], Fvb[d][j]), th, mub);
    }
    mub = fma(ktf * Fvb[d][3], g[d][3], mub);
  }
  rhob = fma(mub * csd2, Sm, rhob);
  if (Sm > 0.0) {
    const double k = mub * rho * csd2 * rcp64(Sm);  // d|S| = dS2 / (2|S|)
    gb[0][0] = fma(2.0 * k, g[0][0], gb[0][0]);
    gb[1][1] = fma(2.0 * k, g[1][1], gb[1][1]);
    gb[2][2] = fma(2.0 * k, g[2][2], gb[2][2]);
    gb[0][1] = fma(k, a, gb[0][1]);
    gb[1][0] = fma(k, a, gb[1][0]);
    gb[0][2] = fma(k, b, gb[0][2]);
    gb[2][0] = fma(k, b, gb[2][0]);
    gb[1][2] = fma(k, c, gb[1][2]);
    gb[2][1] = fma(k, c, gb[2][1]);
  }
}

__device__ __forceinline__ double vjp_csd2(const VjpArgs& A, int e) {
  const double cs = A.cs_elem ? A.cs_elem[e] : A.cs;
  return cs * cs * (A.delta2_elem ? A.delta2_elem[e] : A.delta2);
}

// Wall faces of element e (bit f), at most the two normal to wall_dir.
__device__ __forceinline__ int vjp_wall_mask(const VjpArgs& A, int e) {
  if (A.wall_dir < 0) return 0;
  const int f0 = 2 * A.wall_dir;
  return (A.nbr[6 * e + f0] < 0 ? 1 << f0 : 0) | (A.nbr[6 * e + f0 + 1] < 0 ? 2 << f0 : 0);
}

// Reverse of wall_model_flux: the cotangents gb1, gb2 of its two tangential
// components pulled back to the wall node's density and the exchange node's
// density and tangential momenta (added).  u_tau depends on the (van Driest
// transformed) speed and on nu = mu / rho_w through Spalding's law
// F(u_tau) = y+(u/u_tau) - h u_tau / nu = 0: du_tau = -(F_u du + F_nu dnu) / F_utau.
__device__ void wall_model_flux_vjp(const VjpArgs& A, double rhow, double rx, double mt1, double mt2, double sg,
                                    double gb1, double gb2, double& rhowb, double& rxb, double& mt1b,
                                    double& mt2b) {
  const double ir = 1.0 / rx;
  const double v1 = mt1 * ir, v2 = mt2 * ir;
  const double sp2 = v1 * v1 + v2 * v2;
  if (!(sp2 > 0.0)) return;  // zero flux
  const double sp = sqrt(sp2);
  double ueq = sp, dueq = 1.0;
  if (A.wm_b > 0.0) {
    const double arg = A.wm_b * sp / A.wm_uinf;
    if (arg > 1.0) {  // capped: constant
      ueq = (A.wm_uinf / A.wm_b) * asin(1.0);
      dueq = 0.0;
    } else {
      ueq = (A.wm_uinf / A.wm_b) * asin(arg);
      dueq = 1.0 / sqrt(1.0 - arg * arg);
    }
  }
  const double nu = A.mu / rhow, h = A.wm_h;
  const double ut = wm_friction_velocity(ueq, nu, h);
  const double x = ueq / ut;
  const double k = 0.4 * x, ek = exp(k);
  const double dy = 1.0 + 0.1108 * 0.4 * (ek - (1.0 + k * (1.0 + k * (0.5 + k * (1.0 / 6.0)))));
  const double Fut = -dy * x / ut - h / nu, Fu = dy / ut, Fnu = h * ut / (nu * nu);
  const double c = sg * rhow * ut * ut / sp;
  const double cb = gb1 * v1 + gb2 * v2;
  double v1b = gb1 * c, v2b = gb2 * c;
  rhowb += cb * sg * ut * ut / sp;
  const double utb = cb * sg * rhow * 2.0 * ut / sp;
  double spb = -cb * c / sp;
  const double nub = -utb * Fnu / Fut;
  spb += -utb * Fu / Fut * dueq;
  rhowb -= nub * A.mu / (rhow * rhow);
  v1b += spb * v1 / sp;
  v2b += spb * v2 / sp;
  mt1b += v1b * ir;
  mt2b += v2b * ir;
  rxb -= (v1b * v1 + v2b * v2) * ir;
}

// Neighbour lambda (components 1..4) on face item q into sLn (zero at walls).
template <int D>
__device__ __forceinline__ void neighbour_lambda(const VjpArgs& A, int e, int q, double (*sLn)[4][nf]) {
  const int f = q / nf;
  const int a = q - f * nf;
  const int side = f & 1;
  if (A.nbr[6 * e + f] < 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) sLn[f][c][a] = 0.0;
    return;
  }
  const double* Ln = A.Lbar + (size_t)A.nbr[6 * e + f] * 5 * nn;
  const int nnb = face_node(D, side ? 0 : N, a);
#pragma unroll
  for (int c = 0; c < 4; ++c) sLn[f][c][a] = Ln[(1 + c) * nn + nnb];
}

// Pass 1 of the viscous reverse: cotangent of each element's normal lifted
// gradient at its own face nodes -> Gbf[e][f][c][a].
template <int D>
__device__ __forceinline__ void vjp_lift_face_node(const VjpArgs& A, int e, int q, const double (*sLam)[nn],
                                                   const double (*sLn)[4][nf], const double (*sU)[nn],
                                                   const double* sDw, const double* swinv, int wmask) {
  const int f = q / nf;
  const int a = q - f * nf;
  const int m = face_node(D, (f & 1) ? N : 0, a);
  const int ijk[3] = {m % n1, (m / n1) % n1, m / nf};
  double Fvb[3][4], gb[3][4];
  viscous_flux_cotangent(sLam, sLn, sDw, swinv, m, ijk, A.invJ, Fvb, wmask);
  const double u[3] = {sU[0][m], sU[1][m], sU[2][m]};
  gradient_cotangent(Fvb, u, A.mu, A.kappa, gb);
  double* out = A.Gbf + ((size_t)e * 6 + f) * 4 * nf;
#pragma unroll
  for (int c = 0; c < 4; ++c) out[c * nf + a] = gb[D][c];
}

__global__ __launch_bounds__(NT) void k_vjp_lift(VjpArgs A) {
  __shared__ double sB[NB_STAGE];
  __shared__ double sLam[5][nn];
  __shared__ double sU[3][nn];
  __shared__ double sLn[6][4][nf];
  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const int t = threadIdx.x;
  for (int q = t; q < NB_STAGE; q += NT) sB[q] = A.basis[q];
  if (t < nn) {
    const double* Ue = A.U + (size_t)e * 5 * nn;
    const double* Le = A.Lbar + (size_t)e * 5 * nn;
    const double ir = rcp64(Ue[t]);
#pragma unroll
    for (int j = 0; j < 3; ++j) sU[j][t] = Ue[(1 + j) * nn + t] * ir;
#pragma unroll
    for (int v = 0; v < 5; ++v) sLam[v][t] = Le[v * nn + t];
  }
  for (int q = t; q < 6 * nf; q += NT) {
    if (q < 2 * nf) neighbour_lambda<0>(A, e, q, sLn);
    else if (q < 4 * nf) neighbour_lambda<1>(A, e, q, sLn);
    else neighbour_lambda<2>(A, e, q, sLn);
  }
  __syncthreads();
  const int wmask = vjp_wall_mask(A, e);
  for (int q = t; q < 6 * nf; q += NT) {
    if (q < 2 * nf) vjp_lift_face_node<0>(A, e, q, sLam, sLn, sU, sB + BL.Dw(), sB + BL.winv(), wmask);
    else if (q < 4 * nf) vjp_lift_face_node<1>(A, e, q, sLam, sLn, sU, sB + BL.Dw(), sB + BL.winv(), wmask);
    else vjp_lift_face_node<2>(A, e, q, sLam, sLn, sU, sB + BL.Dw(), sB + BL.winv(), wmask);
  }
}

// Interface part of face item q: the cotangent of the element's own face
// state, (d f*/d U_own)^T fbar with fbar = -(2/dx_d)(lambda_- / w_N -
// lambda_+ / w_0), by the reverse sweep of the interface flux (riemann_vjp).
// One code path for all directions: states and cotangent are rotated by
// address (normal component first).
// At a wall face (WALL, neighbour -1): the interface flux with the mirror
// state (normal momentum reversed) as the other side, so its cotangent reaches
// the own state through both arguments; plus the reverse of the wall model's
// viscous flux, whose exchange-node part goes to sWx[side][variable][a]
// (density and momenta).
template <int VF, bool WALL = false>
__device__ __forceinline__ void vjp_face_item(const VjpArgs& A, int e, int q, const double* swinv,
                                              double (*sSF)[5][nf], double (*sWx)[4][nf] = nullptr) {
  const FaceItem it = face_item_geometry(A.nbr, e, q);
  if (WALL && it.nb < 0) {
    const int row[5] = {0, 1 + it.d, it.k1, it.k2, 4};
    const double* Ue = A.U + (size_t)e * 5 * nn;
    const double* Le = A.Lbar + (size_t)e * 5 * nn;
    const double invJd = it.d == 0 ? A.invJ[0] : (it.d == 1 ? A.invJ[1] : A.invJ[2]);
    const double cw = it.side ? -invJd * swinv[N] : invJd * swinv[0];
    double L[5], R[5], fb[5], Lb[5], Rb[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      const double X = Ue[row[r] * nn + it.nown];
      L[r] = (r == 1 && !it.side) ? -X : X;
      R[r] = (r == 1 && it.side) ? -X : X;
      fb[r] = cw * Le[row[r] * nn + it.nown];
    }
    riemann_vjp<VF>(A.sf, L, R, A.gamma, fb, Lb, Rb);
    double ob[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) ob[r] = (it.side ? Lb[r] : Rb[r]) + (r == 1 ? -1.0 : 1.0) * (it.side ? Rb[r] : Lb[r]);
    const double cv = invJd * (it.side ? swinv[N] : -swinv[0]);
    double rhowb = 0.0, rxb = 0.0, m1b = 0.0, m2b = 0.0;
    wall_model_flux_vjp(A, L[0], Ue[it.nnb], Ue[it.k1 * nn + it.nnb], Ue[it.k2 * nn + it.nnb],
                        it.side ? -1.0 : 1.0, cv * Le[it.k1 * nn + it.nown], cv * Le[it.k2 * nn + it.nown], rhowb,
                        rxb, m1b, m2b);
    ob[0] += rhowb;
#pragma unroll
    for (int r = 0; r < 5; ++r) sSF[it.f][row[r]][it.a] = ob[r];
    sWx[it.side][0][it.a] = rxb;
    sWx[it.side][1 + it.d][it.a] = 0.0;
    sWx[it.side][it.k1][it.a] = m1b;
    sWx[it.side][it.k2][it.a] = m2b;
    return;
  }
  const int eL = it.side ? e : it.nb, eR = it.side ? it.nb : e;
  const int nL = it.side ? it.nown : it.nnb, nR = it.side ? it.nnb : it.nown;
  const int row[5] = {0, 1 + it.d, it.k1, it.k2, 4};  // rotated position -> variable
  const double* UL = A.U + (size_t)eL * 5 * nn;
  const double* UR = A.U + (size_t)eR * 5 * nn;
  const double* LL = A.Lbar + (size_t)eL * 5 * nn;
  const double* LR = A.Lbar + (size_t)eR * 5 * nn;
  const double invJd = it.d == 0 ? A.invJ[0] : (it.d == 1 ? A.invJ[1] : A.invJ[2]);
  const double cm = -invJd * swinv[N], cp = invJd * swinv[0];
  double L[5], R[5], fb[5], Lb[5], Rb[5];
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    const int v = row[r];
    L[r] = UL[v * nn + nL];
    R[r] = UR[v * nn + nR];
    fb[r] = fma(cm, LL[v * nn + nL], cp * LR[v * nn + nR]);
  }
  riemann_vjp<VF>(A.sf, L, R, A.gamma, fb, Lb, Rb);
#pragma unroll
  for (int r = 0; r < 5; ++r) sSF[it.f][row[r]][it.a] = it.side ? Lb[r] : Rb[r];
}

// Navier-Stokes data of face item q: q* (forward gradient), the neighbour's
// lambda and its normal-gradient cotangent.
template <int D, bool GN = true>
__device__ __forceinline__ void vjp_face_ns(const VjpArgs& A, int e, int q, double (*sQ)[4][nf],
                                            double (*sLn)[4][nf], double (*sGn)[4][nf]) {
  const int f = q / nf;
  const int a = q - f * nf;
  const int side = f & 1;
  const int nb = A.nbr[6 * e + f];
  const int eL = side ? e : nb, eR = side ? nb : e;
  const int nL = face_node(D, N, a), nR = face_node(D, 0, a), nnb = side ? nR : nL;
  double L[5], R[5];
  if (nb < 0) {  // wall: the own face state and its mirror image
    const int no = side ? nL : nR;
#pragma unroll
    for (int v = 0; v < 5; ++v) L[v] = R[v] = A.U[((size_t)e * 5 + v) * nn + no];
    if (side) R[1 + D] = -R[1 + D];
    else L[1 + D] = -L[1 + D];
    const double gm1 = A.gamma - 1.0;
    double qs[4];
    interface_q<D, double, false>(state64<D>(L, gm1), state64<D>(R, gm1), Ref{0.0, 0.0, 0.0}, qs);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sQ[f][c][a] = qs[c];
      sLn[f][c][a] = 0.0;
      if (GN) sGn[f][c][a] = 0.0;
    }
    return;
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    L[v] = A.U[((size_t)eL * 5 + v) * nn + nL];
    R[v] = A.U[((size_t)eR * 5 + v) * nn + nR];
  }
  const double gm1 = A.gamma - 1.0;
  const Ref ref{0.0, 0.0, 0.0};
  double qs[4];
  interface_q<D, double, false>(state64<D>(L, gm1), state64<D>(R, gm1), ref, qs);
  const double* Ln = A.Lbar + (size_t)nb * 5 * nn;
  const double* Gn = A.Gbf + ((size_t)nb * 6 + (f ^ 1)) * 4 * nf;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    sQ[f][c][a] = qs[c];
    sLn[f][c][a] = Ln[(1 + c) * nn + nnb];
    if (GN) sGn[f][c][a] = Gn[c * nf + a];
  }
}

// Pass 1 with the Smagorinsky model: the gradient cotangent at a face node
// depends on the eddy viscosity there, so the kernel forms the forward lifted
// gradient (interface values q* of all six faces) and the density at its own
// face nodes first.
__global__ __launch_bounds__(NT) void k_vjp_lift_les(VjpArgs A) {
  __shared__ double sB[NB_STAGE];
  __shared__ double sP[7][nn];
  __shared__ double sLam[5][nn];
  __shared__ double sQ[6][4][nf];
  __shared__ double sLn[6][4][nf];
  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const int t = threadIdx.x;
  const double gm1 = A.gamma - 1.0;
  for (int q = t; q < NB_STAGE; q += NT) sB[q] = A.basis[q];
  if (t < nn) {
    const double* Ue = A.U + (size_t)e * 5 * nn;
    const double* Le = A.Lbar + (size_t)e * 5 * nn;
    double u[5], me[7];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      u[v] = Ue[v * nn + t];
      sLam[v][t] = Le[v * nn + t];
    }
    primitives<VF_PI, double, false>(u, gm1, Ref{0.0, 0.0, 0.0}, me);
#pragma unroll
    for (int k = 0; k < 7; ++k) sP[k][t] = me[k];
  }
  for (int q = t; q < 6 * nf; q += NT) {
    if (q < 2 * nf) vjp_face_ns<0, false>(A, e, q, sQ, sLn, nullptr);
    else if (q < 4 * nf) vjp_face_ns<1, false>(A, e, q, sQ, sLn, nullptr);
    else vjp_face_ns<2, false>(A, e, q, sQ, sLn, nullptr);
  }
  __syncthreads();
  const double* sDw = sB + BL.Dw();
  const double* swinv = sB + BL.winv();
  const double csd2 = vjp_csd2(A, e);
  const int wmask = vjp_wall_mask(A, e);
  for (int q = t; q < 6 * nf; q += NT) {
    const int f = q / nf, a = q - f * nf, d = f >> 1;
    const int m = face_node(d, (f & 1) ? N : 0, a);
    const int ijk[3] = {m % n1, (m / n1) % n1, m / nf};
    double g[3][4], Fvb[3][4], gb[3][4], rhob = 0.0;
    lifted_gradient<double>(sP, sQ, sDw, swinv, m, ijk, A.invJ, g);
    viscous_flux_cotangent(sLam, sLn, sDw, swinv, m, ijk, A.invJ, Fvb, wmask);
    const double u[3] = {sP[1][m], sP[2][m], sP[3][m]};
    les_gradient_cotangent(Fvb, u, g, sP[0][m], A.mu, A.kappa, csd2, A.ktf, gb, rhob);
    double* out = A.Gbf + ((size_t)e * 6 + f) * 4 * nf;
#pragma unroll
    for (int c = 0; c < 4; ++c) out[c * nf + a] = d == 0 ? gb[0][c] : (d == 1 ? gb[1][c] : gb[2][c]);
  }
}

// Hand-derived reverse mode of the two-point volume flux with respect to its
// first argument, in primitive variables (rho, u, p, x), for the flux
// cotangent w (unrotated components).  x = h (PI, STD) or e (KG).
template <int VF, int D>
__device__ __forceinline__ void twopoint_vjp(const double me[7], double rl, const double ul[3], double pl,
                                             double xl, const double w[5], double pb[6]) {
  if (VF == VF_STD) {
    // d1 F# = (1/2) dF(a)/da; F = (rho u_D, rho u_D u + p e_D, rho h u_D)
    const double r = me[0], uD = me[1 + D];
    const double s = w[0] + w[1] * me[1] + w[2] * me[2] + w[3] * me[3] + w[4] * me[5];
    pb[0] += 0.5 * uD * s;
#pragma unroll
    for (int j = 0; j < 3; ++j) pb[1 + j] += 0.5 * w[1 + j] * r * uD;
    pb[1 + D] += 0.5 * r * s;
    pb[4] += 0.5 * w[1 + D];
    pb[5] += 0.5 * w[4] * r * uD;
    return;
  }
  const double rm = 0.5 * (me[0] + rl);
  const double um[3] = {0.5 * (me[1] + ul[0]), 0.5 * (me[2] + ul[1]), 0.5 * (me[3] + ul[2])};
  const double xm = 0.5 * (me[5] + xl);
  const double fr = rm * um[D];
  double wr = w[0] + w[1] * um[0] + w[2] * um[1] + w[3] * um[2] + w[4] * xm;  // total cotangent of f_rho
  pb[0] += 0.5 * wr * um[D];
#pragma unroll
  for (int j = 0; j < 3; ++j) pb[1 + j] += 0.5 * w[1 + j] * fr;
  pb[1 + D] += 0.5 * wr * rm;
  pb[4] += 0.5 * w[1 + D];
  pb[5] += 0.5 * w[4] * fr;
  if (VF == VF_KG) {  // + p_m u_m,D in the energy flux
    const double pm = 0.5 * (me[4] + pl);
    pb[4] += 0.5 * w[4] * um[D];
    pb[1 + D] += 0.5 * w[4] * pm;
  }
}

template <int VF, int D>
__device__ __forceinline__ void volume_vjp_dir(const double (*sP)[nn], const double (*sLam)[nn], const double* sDhat,
                                               int n, int id, const double me[7], const double lam[5], double invJ,
                                               double pb[6]) {
  constexpr int st = D == 0 ? 1 : (D == 1 ? n1 : nf);
  const int base = n - id * st;
#pragma unroll 1
  for (int k = 1; k <= kPartners; ++k) {
    const int l = partner(id, k);
    const int m = base + l * st;
    const double c1 = -invJ * sDhat[id * n1 + l], c2 = -invJ * sDhat[l * n1 + id];
    double w[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) w[v] = fma(c1, lam[v], c2 * sLam[v][m]);
    const double ul[3] = {sP[1][m], sP[2][m], sP[3][m]};
    twopoint_vjp<VF, D>(me, sP[0][m], ul, sP[4][m], sP[5][m], w, pb);
  }
}

// Main reverse kernel.  Writes U_bar (or U_acc + U_bar when A.Uacc is set).
// EQ: 0 Euler, 1 Navier-Stokes, 2 with the Smagorinsky eddy viscosity; WALL:
// wall-modelled faces (neighbour -1).
// Three waves per SIMD (at most 168 registers; a few spill) run the reverse
// kernel faster than two without spills; the wall variants keep their
// registers, and so does N = 7, where the LDS admits one workgroup per CU.
template <int VF, int EQ, bool WALL = false>
__global__ __launch_bounds__(NT, WALL || N > 6 ? 1 : 3) void k_vjp(VjpArgs A) {
  constexpr bool NS = (EQ >= 1);
  constexpr bool LES = (EQ == 2);
  static_assert(!WALL || EQ >= 1, "walls: Navier-Stokes");
  __shared__ double sWx[WALL ? 2 : 1][4][nf];
  __shared__ double sB[NB_STAGE];
  __shared__ double sP[7][nn];
  __shared__ double sLam[5][nn];
  __shared__ double sSF[6][5][nf];
  __shared__ double sQ[NS ? 6 : 1][4][nf];
  __shared__ double sLn[NS ? 6 : 1][4][nf];
  __shared__ double sGn[NS ? 6 : 1][4][nf];
  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const int t = threadIdx.x;
  const double gm1 = A.gamma - 1.0;
  for (int q = t; q < NB_STAGE; q += NT) sB[q] = A.basis[q];
  const double* sDhat = sB + BL.Dhat();
  const double* sDw = sB + BL.Dw();
  const double* swinv = sB + BL.winv();
  const Ref ref{0.0, 0.0, 0.0};
  double u[5], me[7], lam[5];
  int ijk[3] = {0, 0, 0};
  if (t < nn) {
    const double* Ue = A.U + (size_t)e * 5 * nn;
    const double* Le = A.Lbar + (size_t)e * 5 * nn;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      u[v] = Ue[v * nn + t];
      lam[v] = Le[v * nn + t];
      sLam[v][t] = lam[v];
    }
    primitives<VF, double, false>(u, gm1, ref, me);
#pragma unroll
    for (int k = 0; k < 7; ++k) sP[k][t] = me[k];
    ijk[0] = t % n1;
    ijk[1] = (t / n1) % n1;
    ijk[2] = t / nf;
  }
  __syncthreads();  // the face items read the basis (swinv)
  const int wmask = WALL ? vjp_wall_mask(A, e) : 0;
#pragma unroll 1
  for (int q = t; q < 6 * nf; q += NT) vjp_face_item<VF, WALL>(A, e, q, swinv, sSF, sWx);
  if (NS) {
    for (int q = t; q < 6 * nf; q += NT) {
      if (q < 2 * nf) vjp_face_ns<0>(A, e, q, sQ, sLn, sGn);
      else if (q < 4 * nf) vjp_face_ns<1>(A, e, q, sQ, sLn, sGn);
      else vjp_face_ns<2>(A, e, q, sQ, sLn, sGn);
    }
  }
  __syncthreads();

  // primitive cotangents: rho, u, v, w, p, x (= h or e); theta added below
  double pb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double thb = 0.0;
  double gb[3][4];
  if (t < nn) {
    volume_vjp_dir<VF, 0>(sP, sLam, sDhat, t, ijk[0], me, lam, A.invJ[0], pb);
    volume_vjp_dir<VF, 1>(sP, sLam, sDhat, t, ijk[1], me, lam, A.invJ[1], pb);
    volume_vjp_dir<VF, 2>(sP, sLam, sDhat, t, ijk[2], me, lam, A.invJ[2], pb);
    if (A.alpha) {  // blended: the DG advective volume term enters with weight 1 - alpha
      const double wv = 1.0 - A.alpha[e];
#pragma unroll
      for (int i = 0; i < 6; ++i) pb[i] *= wv;
    }
    if (NS) {
      double Fvb[3][4], g[3][4];
      viscous_flux_cotangent(sLam, sLn, sDw, swinv, t, ijk, A.invJ, Fvb, wmask);
      lifted_gradient<double>(sP, sQ, sDw, swinv, t, ijk, A.invJ, g);
      const double csd2 = LES ? vjp_csd2(A, e) : 0.0;
      const double mue = LES ? A.mu + eddy_viscosity<double>(g, me[0], csd2) : A.mu;
      // u enters the energy flux u . tau_d
      const double div = g[0][0] + g[1][1] + g[2][2];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double tau = mue * (g[d][j] + g[j][d]) - (j == d ? (2.0 / 3.0) * mue * div : 0.0);
          s = fma(tau, Fvb[d][3], s);
        }
        pb[1 + j] += s;
      }
      const double uu[3] = {me[1], me[2], me[3]};
      if (LES) les_gradient_cotangent(Fvb, uu, g, me[0], A.mu, A.kappa, csd2, A.ktf, gb, pb[0]);
      else gradient_cotangent(Fvb, uu, A.mu, A.kappa, gb);
    }
  }
  if (NS) {
    // q_bar = sum_d' (2/dx_d') [ Dw^T gb_d' along the d' line + interface terms ]
    double (*sX)[nn] = sLam;  // lambda is no longer needed
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      __syncthreads();
      if (t < nn) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sX[c][t] = gb[d][c];
      }
      __syncthreads();
      if (t < nn) {
        const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
        const int id = ijk[d];
        const int base = t - id * st;
        const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
        double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int l = 0; l < n1; ++l) {
          const double c = sDw[l * n1 + id];
          const int k = base + l * st;
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) s[cc] = fma(c, sX[cc][k], s[cc]);
        }
        // interface value q* = (q + q_nb)/2; at a wall (q + M q)/2, M the
        // mirror (normal velocity reversed)
        if (id == N) {
          if (WALL && ((wmask >> (2 * d + 1)) & 1)) {
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) s[cc] += cc == d ? 0.0 : swinv[N] * gb[d][cc];
          } else {
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) s[cc] += 0.5 * (swinv[N] * gb[d][cc] - swinv[0] * sGn[2 * d + 1][cc][a]);
          }
        }
        if (id == 0) {
          if (WALL && ((wmask >> (2 * d)) & 1)) {
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) s[cc] -= cc == d ? 0.0 : swinv[0] * gb[d][cc];
          } else {
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) s[cc] += 0.5 * (swinv[N] * sGn[2 * d][cc][a] - swinv[0] * gb[d][cc]);
          }
        }
        pb[1] += A.invJ[d] * s[0];
        pb[2] += A.invJ[d] * s[1];
        pb[3] += A.invJ[d] * s[2];
        thb += A.invJ[d] * s[3];
      }
    }
  }
  if (t < nn) {
    // primitive cotangents -> conservative: u = m/rho, p = (g-1)(E - |m|^2/(2 rho)),
    // x = h = (E + p)/rho (PI, STD) or e = E/rho (KG), theta = p/rho
    const double ir = rcp64(u[0]);
    double rb = pb[0], ub[3] = {pb[1], pb[2], pb[3]}, pbar = pb[4], Eb = 0.0;
    if (VF == VF_KG) {
      Eb += pb[5] * ir;
      rb -= pb[5] * me[5] * ir;
    } else {
      Eb += pb[5] * ir;
      pbar += pb[5] * ir;
      rb -= pb[5] * me[5] * ir;
    }
    pbar += thb * ir;
    rb -= thb * me[6] * ir;
    const double q2 = me[1] * me[1] + me[2] * me[2] + me[3] * me[3];
    Eb += gm1 * pbar;
    rb += gm1 * pbar * 0.5 * q2;
    double mb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      mb[j] = -gm1 * pbar * me[1 + j] + ub[j] * ir;
      rb -= ub[j] * me[1 + j] * ir;
    }
    double out[5] = {rb, mb[0], mb[1], mb[2], Eb};
    // interface contributions of the faces containing this node
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int id = ijk[d];
      const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
      if (id == N)
#pragma unroll
        for (int v = 0; v < 5; ++v) out[v] += sSF[2 * d + 1][v][a];
      if (id == 0)
#pragma unroll
        for (int v = 0; v < 5; ++v) out[v] += sSF[2 * d][v][a];
    }
    if (WALL) {  // exchange nodes of the wall faces: the wall model's pullback
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (d != A.wall_dir) continue;
        const int id = ijk[d];
        const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
        if (id == 0 && ((wmask >> (2 * d + 1)) & 1))
#pragma unroll
          for (int v = 0; v < 4; ++v) out[v] += sWx[1][v][a];
        if (id == N && ((wmask >> (2 * d)) & 1))
#pragma unroll
          for (int v = 0; v < 4; ++v) out[v] += sWx[0][v][a];
      }
    }
    const size_t o = (size_t)e * 5 * nn + t;
#pragma unroll
    for (int v = 0; v < 5; ++v) A.Ubar[o + v * nn] = A.Uacc ? A.Uacc[o + v * nn] + out[v] : out[v];
  }
}

// ===========================================================================
// Reverse mode through the DG/FV blending (Euler).  The surface terms of the
// DG and FV operators coincide (outer subcells first order), so
//   U_t = (1 - a) V_DG + a V_FV + S(f*),
//   U_bar = V_DG^T((1 - a) lambda) + V_FV^T(a lambda) + S^T lambda + (da/dU)^T abar,
//   abar_e = sum over the nodes of e of lambda . (U_t^FV - U_t^DG).
// k_vjp weights its volume part by 1 - a; the kernels below give the
// coefficient and FV parts.  Conventions at switches as in the forward-mode
// reference: clip when a0 > alpha_max, cut-off when a < alpha_min (derivative
// 0), maxima with the mean derivative at ties in the order evaluated, minmod
// through the selected slope (mean at ties), positivity fallback through the
// selected branch.
// ===========================================================================
__global__ __launch_bounds__(NT) void k_vjp_alpha_bar(VjpArgs A) {
  __shared__ double sred[NT];
  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const int t = threadIdx.x;
  if (A.alpha[e] == 0.0) {  // uniform over the workgroup
    if (t == 0) A.abar[e] = 0.0;
    return;
  }
  double s = 0.0;
  if (t < nn) {
    const size_t o = (size_t)e * 5 * nn + t;
#pragma unroll
    for (int v = 0; v < 5; ++v) s = fma(A.Lbar[o + v * nn], A.Dfd[o + v * nn], s);
  }
  sred[t] = s;
  __syncthreads();
  for (int h = NTP2 / 2; h > 0; h >>= 1) {
    if (t < h && t + h < NT) sred[t] += sred[t + h];
    __syncthreads();
  }
  if (t == 0) A.abar[e] = sred[0];
}

// d alpha_j / d alpha1_e (j, e: elements; j is e or a face neighbour of e).
__device__ double spread_weight(const VjpArgs& A, int j, int e) {
  if (A.alpha[j] == 0.0) return 0.0;  // cut off: flat
  double m = 0.0, w[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int nb = A.nbr[6 * j + f];
    if (nb < 0) continue;  // wall face: not part of the maximum
    const double x = A.alpha1[nb];
    if (x > m) {
#pragma unroll
      for (int g = 0; g < 6; ++g) w[g] = g == f ? 1.0 : 0.0;
      m = x;
    } else if (!(m > x)) {  // tie
#pragma unroll
      for (int g = 0; g < 6; ++g) w[g] = g == f ? 0.5 : 0.5 * w[g];
    }
  }
  const double a1 = A.alpha1[j], sm = A.aspread * m;
  const double ws = a1 > sm ? 1.0 : (sm > a1 ? 0.0 : 0.5);
  double r = j == e ? ws : 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f)
    if (A.nbr[6 * j + f] == e) r += (1.0 - ws) * A.aspread * w[f];
  return r;
}

// U_bar = [Uacc +] (d alpha / d U)^T abar: pullback through the spread (a
// gather over the element and its neighbours), the clip, the sigmoid, the
// modal energies E_N, E_{N-1} of q = rho p and q(U).
__global__ __launch_bounds__(NT) void k_vjp_alpha(VjpArgs A) {
  __shared__ double sV[nf];
  __shared__ double sq[nn];
  __shared__ double st[nn];
  __shared__ double sred[3][NT];
  __shared__ double sa1b;
  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const int t = threadIdx.x;
  for (int q = t; q < nf; q += NT) sV[q] = A.basis[BL.Vinv() + q];
  if (t == 0) {
    int cand[7] = {e, A.nbr[6 * e], A.nbr[6 * e + 1], A.nbr[6 * e + 2], A.nbr[6 * e + 3], A.nbr[6 * e + 4],
                   A.nbr[6 * e + 5]};
    double r = 0.0;
    for (int i = 0; i < 7; ++i) {
      bool dup = cand[i] < 0;  // wall face
      for (int k = 0; k < i; ++k) dup = dup || cand[k] == cand[i];
      if (!dup) r += A.abar[cand[i]] * spread_weight(A, cand[i], e);
    }
    sa1b = r;
  }
  const double* Ue = A.U + (size_t)e * 5 * nn;
  const double gm1 = A.gamma - 1.0;
  int ijk[3] = {0, 0, 0};
  double u[5], rho = 1.0, p = 0.0;
  if (t < nn) {
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = Ue[v * nn + t];
    const double ir = 1.0 / u[0];
    p = gm1 * (u[4] - 0.5 * ir * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]));
    rho = u[0];
    sq[t] = u[0] * p;
    ijk[0] = t % n1;
    ijk[1] = (t / n1) % n1;
    ijk[2] = t / nf;
  }
  __syncthreads();
  // forward modal transform (as k_alpha1), keeping the node's coefficient
  if (t < nn) {
    const int base = t - ijk[0];
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < n1; ++i) s = fma(sV[ijk[0] * n1 + i], sq[base + i], s);
    st[t] = s;
  }
  __syncthreads();
  if (t < nn) {
    const int base = t - ijk[1] * n1;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < n1; ++j) s = fma(sV[ijk[1] * n1 + j], st[base + j * n1], s);
    sq[t] = s;
  }
  __syncthreads();
  double qh = 0.0, e2 = 0.0;
  int mx = 0;
  if (t < nn) {
    const int base = t - ijk[2] * nf;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < n1; ++k) s = fma(sV[ijk[2] * n1 + k], sq[base + k * nf], s);
    qh = s;
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
  const double S = sred[0][0], SN = sred[1][0], SN1 = sred[2][0];
  const double EN = S > 0.0 ? SN / S : 0.0;
  const double Rr = S - SN;
  const double EN1 = Rr > 0.0 ? SN1 / Rr : 0.0;
  const double E = A.indicator == 1 ? EN : fmax(EN, EN1);
  const double k = A.sharp / A.thresh;
  const double a0 = 1.0 / (1.0 + exp(-k * (E - A.thresh)));
  // uniform: no derivative when cut off or clipped
  const bool live = sa1b != 0.0 && A.alpha1[e] != 0.0 && !(a0 > A.amax);
  const double Eb = live ? sa1b * k * a0 * (1.0 - a0) : 0.0;
  const double wN = A.indicator == 1 ? 1.0 : (EN > EN1 ? 1.0 : (EN1 > EN ? 0.0 : 0.5));
  const double ENb = Eb * wN, EN1b = Eb * (1.0 - wN);
  double e2b = 0.0;
  if (S > 0.0) e2b += ENb * ((mx == N ? 1.0 : 0.0) - EN) / S;
  if (Rr > 0.0) e2b += EN1b * ((mx == N - 1 ? 1.0 : 0.0) - (mx <= N - 1 ? EN1 : 0.0)) / Rr;
  __syncthreads();
  // transposed modal transform of qhat_bar = 2 qhat e2_bar: z, y, x
  if (t < nn) sq[t] = 2.0 * qh * e2b;
  __syncthreads();
  if (t < nn) {
    const int base = t - ijk[2] * nf;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < n1; ++c) s = fma(sV[c * n1 + ijk[2]], sq[base + c * nf], s);
    st[t] = s;
  }
  __syncthreads();
  if (t < nn) {
    const int base = t - ijk[1] * n1;
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < n1; ++b) s = fma(sV[b * n1 + ijk[1]], st[base + b * n1], s);
    sq[t] = s;
  }
  __syncthreads();
  if (t < nn) {
    const int base = t - ijk[0];
    double qb = 0.0;
#pragma unroll
    for (int a = 0; a < n1; ++a) qb = fma(sV[a * n1 + ijk[0]], sq[base + a], qb);
    // q = rho p, p = (g-1)(E - |m|^2 / (2 rho))
    const double rb = qb * p, pb = qb * rho;
    const double ir = 1.0 / rho;
    const double vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
    const double out[5] = {rb + gm1 * pb * 0.5 * (vx * vx + vy * vy + vz * vz), -gm1 * pb * vx, -gm1 * pb * vy,
                           -gm1 * pb * vz, gm1 * pb};
    const size_t o = (size_t)e * 5 * nn + t;
#pragma unroll
    for (int v = 0; v < 5; ++v) A.Ubar[o + v * nn] = A.Uacc ? A.Uacc[o + v * nn] + out[v] : out[v];
  }
}

// FV subcell part: U_bar += V_FV^T(a lambda) for blended elements.  Per
// direction: the interior subcell fluxes F_{m+1/2} = f*(w+_m, w-_{m+1}) are
// pulled back to the ten primitive components of their two reconstructed
// states by one reverse sweep of the interface flux (riemann_vjp) per
// subcell interface node (rotated frame, one code path for all directions);
// the reconstruction (minmod, positivity fallback) is pulled back along each
// line per variable.
template <int VF>
__global__ __launch_bounds__(NT) void k_vjp_fv(VjpArgs A) {
  __shared__ double sB[NB_STAGE];
  __shared__ double sW[5][nnp];  // primitives rho, u, v, w, p
  __shared__ double sL[5][nn];   // lambda
  __shared__ double sWb[5][nn];  // primitive cotangent
  __shared__ double sG[N * nf][10];
  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const double al = A.alpha[e];
  if (al == 0.0) return;  // uniform: pure DG element
  const int t = threadIdx.x;
  const double gm1 = A.gamma - 1.0;
  for (int q = t; q < NB_STAGE; q += NT) sB[q] = A.basis[q];
  const double* sxi = sB + BL.xi();
  const double* sedge = sB + BL.edge();
  const double* swinv = sB + BL.winv();
  const Ref ref{0.0, 0.0, 0.0};
  double u[5], me[7];
  if (t < nn) {
    const size_t o = (size_t)e * 5 * nn + t;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      u[v] = A.U[o + v * nn];
      sL[v][t] = A.Lbar[o + v * nn];
      sWb[v][t] = 0.0;
    }
    primitives<VF, double, false>(u, gm1, ref, me);
#pragma unroll
    for (int v = 0; v < 5; ++v) sW[v][t] = me[v];
  }
  for (int d = 0; d < 3; ++d) {
    const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
    const int c1 = d == 2 ? 0 : d + 1, c2 = d == 0 ? 2 : (d == 1 ? 0 : 1);  // tangential velocity (cyclic)
    __syncthreads();
#pragma unroll 1
    for (int i = t; i < N * nf; i += NT) {
      const int m = i / nf, a = i - m * nf;
      const int nm = face_node(d, m, a), base = nm - m * st;
      double W[2][5];
      subcell_face_state(sW, base, st, m, true, A.recon, sxi, sedge, W[0]);
      subcell_face_state(sW, base, st, m + 1, false, A.recon, sxi, sedge, W[1]);
      // flux cotangent (conservative, rotated): a (2/dx_d)(lambda_{m+1}/w_{m+1} - lambda_m/w_m)
      const double invJd = d == 0 ? A.invJ[0] : (d == 1 ? A.invJ[1] : A.invJ[2]);
      const int np = nm + st;
      const int row[5] = {0, 1 + d, 1 + c1, 1 + c2, 4};
      double fb[5];
#pragma unroll
      for (int r = 0; r < 5; ++r)
        fb[r] = al * invJd * (sL[row[r]][np] * swinv[m + 1] - sL[row[r]][nm] * swinv[m]);
      // conservative states in the rotated frame, the reverse sweep of the
      // interface flux, and the pullback to both primitive face states
      double C[2][5], Cb[2][5];
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const double r = W[sd][0];
        const double un = d == 0 ? W[sd][1] : (d == 1 ? W[sd][2] : W[sd][3]);
        const double u1 = c1 == 0 ? W[sd][1] : (c1 == 1 ? W[sd][2] : W[sd][3]);
        const double u2 = c2 == 0 ? W[sd][1] : (c2 == 1 ? W[sd][2] : W[sd][3]);
        C[sd][0] = r;
        C[sd][1] = r * un;
        C[sd][2] = r * u1;
        C[sd][3] = r * u2;
        C[sd][4] = W[sd][4] * (1.0 / gm1) + 0.5 * r * (W[sd][1] * W[sd][1] + W[sd][2] * W[sd][2] +
                                                       W[sd][3] * W[sd][3]);
      }
      riemann_vjp<VF>(A.sf, C[0], C[1], A.gamma, fb, Cb[0], Cb[1]);
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const double r = W[sd][0];
        const double un = d == 0 ? W[sd][1] : (d == 1 ? W[sd][2] : W[sd][3]);
        const double u1 = c1 == 0 ? W[sd][1] : (c1 == 1 ? W[sd][2] : W[sd][3]);
        const double u2 = c2 == 0 ? W[sd][1] : (c2 == 1 ? W[sd][2] : W[sd][3]);
        const double* B = Cb[sd];
        const double q2h = 0.5 * (W[sd][1] * W[sd][1] + W[sd][2] * W[sd][2] + W[sd][3] * W[sd][3]);
        sG[i][5 * sd + 0] = B[0] + B[1] * un + B[2] * u1 + B[3] * u2 + B[4] * q2h;
#pragma unroll
        for (int j = 0; j < 3; ++j)
          sG[i][5 * sd + 1 + j] = (j == d ? B[1] : (j == c1 ? B[2] : B[3])) * r + B[4] * r * W[sd][1 + j];
        sG[i][5 * sd + 4] = B[4] * (1.0 / gm1);
      }
    }
    __syncthreads();
    // pullback of the reconstruction, per (line, variable)
    for (int w = t; w < 5 * nf; w += NT) {
      const int v = w / nf, a = w - v * nf;
      const int base = face_node(d, 0, a);
      double wb[n1];
#pragma unroll
      for (int m = 0; m < n1; ++m) wb[m] = 0.0;
#pragma unroll
      for (int m = 0; m < n1; ++m) {
        const double gp = m < N ? sG[m * nf + a][v] : 0.0;       // cotangent of w+_m
        const double gmv = m > 0 ? sG[(m - 1) * nf + a][5 + v] : 0.0;  // of w-_m
        wb[m] += gp + gmv;
        if (A.recon == 1 && m >= 1 && m <= N - 1) {
          const int mm = base + m * st;
          const double hl = 1.0 / (sxi[m] - sxi[m - 1]);
          const double hr = 1.0 / (sxi[m + 1] - sxi[m]);
          const double dp = sedge[m + 1] - sxi[m], dm = sedge[m] - sxi[m];
          // positivity flag of subcell m (as in subcell_face_state)
          const double c0 = sW[0][mm], c4 = sW[4][mm];
          const double s0 = minmod((c0 - sW[0][mm - st]) * hl, (sW[0][mm + st] - c0) * hr);
          const double s4 = minmod((c4 - sW[4][mm - st]) * hl, (sW[4][mm + st] - c4) * hr);
          const bool ok = (c0 + s0 * dp > 0.0) && (c4 + s4 * dp > 0.0) && (c0 + s0 * dm > 0.0) && (c4 + s4 * dm > 0.0);
          if (ok) {
            const double sb = gp * dp + gmv * dm;  // cotangent of the slope
            const double cv = sW[v][mm];
            const double sl = (cv - sW[v][mm - st]) * hl, sr = (sW[v][mm + st] - cv) * hr;
            double bl = 0.0, br = 0.0;
            if (sl * sr > 0.0) {
              const bool pick_l = sl > 0.0 ? sl < sr : sl > sr;
              const bool pick_r = sl > 0.0 ? sr < sl : sr > sl;
              if (pick_l) bl = sb;
              else if (pick_r) br = sb;
              else {
                bl = 0.5 * sb;
                br = 0.5 * sb;
              }
            }
            wb[m] += bl * hl - br * hr;
            wb[m - 1] -= bl * hl;
            wb[m + 1] += br * hr;
          }
        }
      }
#pragma unroll
      for (int m = 0; m < n1; ++m) sWb[v][base + m * st] += wb[m];
    }
  }
  __syncthreads();
  if (t < nn) {
    // primitives (rho, u, v, w, p) -> conservative
    const double ir = rcp64(u[0]);
    const double vx = me[1], vy = me[2], vz = me[3];
    const double pb = sWb[4][t];
    const double ub[3] = {sWb[1][t], sWb[2][t], sWb[3][t]};
    double out[5];
    out[0] = sWb[0][t] - (ub[0] * vx + ub[1] * vy + ub[2] * vz) * ir + gm1 * pb * 0.5 * (vx * vx + vy * vy + vz * vz);
    out[1] = ub[0] * ir - gm1 * pb * vx;
    out[2] = ub[1] * ir - gm1 * pb * vy;
    out[3] = ub[2] * ir - gm1 * pb * vz;
    out[4] = gm1 * pb;
    const size_t o = (size_t)e * 5 * nn + t;
#pragma unroll
    for (int v = 0; v < 5; ++v) A.Ubar[o + v * nn] += out[v];
  }
}

__global__ void k_axpby(double* y, double a, const double* x, double b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = (a == 0.0 ? 0.0 : a * y[i]) + b * x[i];
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
  __shared__ double sred[3 * NWAVE];
  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const int t = threadIdx.x;
  for (int q = t; q < nf; q += NT) sV[q] = A.basis[BL.Vinv() + q];
  const double* Ue = A.U + (size_t)e * 5 * nn;
  int ijk[3] = {0, 0, 0};
  double qt = 0.0;
  if (t < nn) {
    double u[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = Ue[v * nn + t];
    qt = indicator_q(u, A.gamma - 1.0);
    ijk[0] = t % n1;
    ijk[1] = (t / n1) % n1;
    ijk[2] = t / nf;
  }
  const double a1 = element_alpha1(A, sV, sq, st, sred, t, ijk, qt);
  if (t == 0) const_cast<double*>(A.alpha1)[e] = a1;
}

__global__ void k_spread(StageArgs A) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= A.nelem) return;
  double m = 0.0;
  for (int f = 0; f < 6; ++f) {
    const int nb = A.nbr[6 * e + f];
    if (nb >= 0) m = fmax(m, A.alpha1[nb]);  // a wall face spreads nothing
  }
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
      double ra, rv;
      if (R.M) {
        // curved: 1/dx_d -> |Ja^d|/(2J), |u_d| -> |u.Ja^d|/|Ja^d| at the node
        const double* Me = R.M + (size_t)e * 10 * nn + t;
        const double iJ = Me[9 * nn];
        ra = 0.0;
        double h2 = 0.0;
        for (int d = 0; d < 3; ++d) {
          const double jx = Me[(3 * d) * nn], jy = Me[(3 * d + 1) * nn], jz = Me[(3 * d + 2) * nn];
          const double jn = sqrt(jx * jx + jy * jy + jz * jz);
          const double h = 0.5 * jn * iJ;
          ra += (fabs(vx * jx + vy * jy + vz * jz) / jn + c) * h;
          h2 += h * h;
        }
        rv = R.nu_fac * ir * h2;
      } else {
        ra = (fabs(vx) + c) * R.invdx[0] + (fabs(vy) + c) * R.invdx[1] + (fabs(vz) + c) * R.invdx[2];
        rv = R.nu_fac * ir * (R.invdx[0] * R.invdx[0] + R.invdx[1] * R.invdx[1] + R.invdx[2] * R.invdx[2]);
      }
      // a node that is not finite or has rho <= 0 or p <= 0 makes the rate
      // infinite (fmax would drop a NaN), so the host reports it
      const bool ok = u[0] > 0.0 && p > 0.0 && isfinite(ra) && isfinite(rv);
      ma = fmax(ma, ok ? ra : INFINITY);
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
      // curved: the node's Jacobian in place of the constant one
      const double wJ = R.M ? wq / (R.Jac * R.M[((size_t)e * 10 + 9) * nn + t]) : wq;
      for (int v = 0; v < 5; ++v) acc[v] = fma(wJ, Xe[v * nn + t], acc[v]);
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

// ===========================================================================
// Curved elements: the split form with metric terms (FP64).
//
// Metric array M[e][10][nn]: Ja^i_m (contravariant direction i, Cartesian
// component m) at slot 3 i + m, 1/J at slot 9.  Computed once from the node
// coordinates in the conservative curl form, which satisfies the discrete
// metric identities (a uniform state stays uniform):
//   Ja^i_m = -( d_j (X_l d_k X_n) - d_k (X_l d_j X_n) ),
// (j, k) = (i+1, i+2) mod 3, (n, l) = (m+1, m+2) mod 3, d_j the LGL
// derivative along reference direction j of nodal values.
//   J U_t = - sum_i [ sum_l Dhat_il Ft#_i(U_n, U_l) + lifted surface flux ],
//   Ft#_i(a, b) = F#(a, b) . (Ja^i(a) + Ja^i(b)) / 2,
// with the interface flux ft* = |Ja_f| f*(U-, U+; Ja_f / |Ja_f|) and the face
// metric Ja_f the mean of both elements' node metrics (both elements form the
// same value, so conservation holds to round-off as on the box).  The
// Navier-Stokes terms use the BR1 gradient by the chain rule,
// grad q = (1/J) sum_i Ja^i (d_i q + lifting), and the contravariant viscous
// flux sum_m Ja^i_m Fv_m, at faces Ja_f . (Fv- + Fv+)/2.
// ===========================================================================
constexpr int MS = 10;  // metric slots per node

__device__ __forceinline__ int node_along(int n, int id, int st, int l) { return n + (l - id) * st; }

// Metric terms of one element per workgroup; *bad counts nodes whose
// Jacobian is not positive and finite.  Coordinates are taken relative to
// c = (X_first + X_last)/2 of the element (the curl form is translation
// invariant; small products keep the round-off of its differences small).
// Also the squared filter width of the eddy viscosity per element, d2[e] =
// ((element volume)^(1/3) / (N + 1))^2, the volume the quadrature sum of J.
__global__ __launch_bounds__(NT) void k_metrics(const double* X, const double* basis, double* M, int* bad,
                                                 double* d2, int nelem, int chunk) {
  __shared__ double sD[nf];
  __shared__ double sX[3][nn];
  __shared__ double sG[2][nn];
  __shared__ double sW[nn];
  const int e = element_of_block(blockIdx.x, chunk);
  if (e >= nelem) return;
  const int t = threadIdx.x;
  for (int q = t; q < nf; q += NT) sD[q] = basis[BL.D() + q];
  if (t < nn)
    for (int m = 0; m < 3; ++m) {
      const double* Xm = X + ((size_t)e * 3 + m) * nn;
      sX[m][t] = Xm[t] - 0.5 * (Xm[0] + Xm[nn - 1]);
    }
  __syncthreads();
  int ijk[3] = {0, 0, 0};
  const int st[3] = {1, n1, nf};
  double dX[3][3];
  if (t < nn) {
    ijk[0] = t % n1;
    ijk[1] = (t / n1) % n1;
    ijk[2] = t / nf;
    for (int m = 0; m < 3; ++m)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int l = 0; l < n1; ++l) s = fma(sD[ijk[j] * n1 + l], sX[m][node_along(t, ijk[j], st[j], l)], s);
        dX[m][j] = s;
      }
    const double J = dX[0][0] * (dX[1][1] * dX[2][2] - dX[1][2] * dX[2][1]) -
                     dX[0][1] * (dX[1][0] * dX[2][2] - dX[1][2] * dX[2][0]) +
                     dX[0][2] * (dX[1][0] * dX[2][1] - dX[1][1] * dX[2][0]);
    if (!(J > 0.0) || !isfinite(J)) atomicAdd(bad, 1);
    M[((size_t)e * MS + 9) * nn + t] = 1.0 / J;
    const double* w = basis + BL.winv();
    sW[t] = J / (w[ijk[0]] * w[ijk[1]] * w[ijk[2]]);
  }
  __syncthreads();
  if (t == 0) {  // element volume in node order
    double vol = 0.0;
    for (int n = 0; n < nn; ++n) vol += sW[n];
    const double delta = cbrt(vol) / (double)n1;
    d2[e] = delta * delta;
  }
  for (int i = 0; i < 3; ++i) {
    const int j = (i + 1) % 3, k = (i + 2) % 3;
    for (int m = 0; m < 3; ++m) {
      const int mn = (m + 1) % 3, ml = (m + 2) % 3;
      __syncthreads();
      if (t < nn) {
        sG[0][t] = sX[ml][t] * dX[mn][k];
        sG[1][t] = sX[ml][t] * dX[mn][j];
      }
      __syncthreads();
      if (t < nn) {
        double dp = 0.0, dq = 0.0;
        for (int l = 0; l < n1; ++l) {
          dp = fma(sD[ijk[j] * n1 + l], sG[0][node_along(t, ijk[j], st[j], l)], dp);
          dq = fma(sD[ijk[k] * n1 + l], sG[1][node_along(t, ijk[k], st[k], l)], dq);
        }
        M[((size_t)e * MS + 3 * i + m) * nn + t] = -(dp - dq);
      }
    }
  }
}

// Interface flux along the unit normal n: the momentum is rotated into an
// orthonormal frame (n, t1, t2), the rotated-frame flux evaluated and rotated
// back (the two-point fluxes and both dissipations are rotationally
// invariant).  t1 is n crossed with the coordinate axis of its smallest
// component.  L: minus side.
template <int VF>
__device__ __forceinline__ void surface_flux_normal(int sf, const double L[5], const double R[5], const double n[3],
                                                    double gamma, double f[5]) {
  const double ax = fabs(n[0]), ay = fabs(n[1]), az = fabs(n[2]);
  double t1[3];
  if (ax <= ay && ax <= az) {
    t1[0] = 0.0; t1[1] = n[2]; t1[2] = -n[1];
  } else if (ay <= az) {
    t1[0] = -n[2]; t1[1] = 0.0; t1[2] = n[0];
  } else {
    t1[0] = n[1]; t1[1] = -n[0]; t1[2] = 0.0;
  }
  const double it = rcp64(sqrt64(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]));
  t1[0] *= it; t1[1] *= it; t1[2] *= it;
  const double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
  double a[5], b[5];
  a[0] = L[0]; a[4] = L[4];
  b[0] = R[0]; b[4] = R[4];
  a[1] = n[0] * L[1] + n[1] * L[2] + n[2] * L[3];
  a[2] = t1[0] * L[1] + t1[1] * L[2] + t1[2] * L[3];
  a[3] = t2[0] * L[1] + t2[1] * L[2] + t2[2] * L[3];
  b[1] = n[0] * R[1] + n[1] * R[2] + n[2] * R[3];
  b[2] = t1[0] * R[1] + t1[1] * R[2] + t1[2] * R[3];
  b[3] = t2[0] * R[1] + t2[1] * R[2] + t2[2] * R[3];
  const Ref ref{0.0, 0.0, 0.0};
  const State64 sa = state64<0>(a, gamma - 1.0), sb = state64<0>(b, gamma - 1.0);
  const Jumps<double> J = jumps<double, false>(sa, sb, gamma, ref, sf);
  double g[5];
  riemann_rot<VF, double>(sf, to_rot<double, false>(sa, ref), to_rot<double, false>(sb, ref), J, gamma, g);
  f[0] = g[0];
  f[1] = g[1] * n[0] + g[2] * t1[0] + g[3] * t2[0];
  f[2] = g[1] * n[1] + g[2] * t1[1] + g[3] * t2[1];
  f[3] = g[1] * n[2] + g[2] * t1[2] + g[3] * t2[2];
  f[4] = g[4];
}

// Face item q of element e on a curved mesh: own face f (normal reference
// direction d), face index a and volume node; the neighbour, its local face
// fb, face index ab (the orientation code maps a to ab: bit 0 swaps the two
// face-local indices, bit 1 reverses the first, bit 2 the second) and volume
// node.  Every face is evaluated from its minus to its plus side: the side
// whose face is a + face when the other's is a - face (on a structured mesh
// the element whose + face it is), else the smaller (element, face).
struct CFaceItem {
  int f, a, d, side, nown, nb, fb, ab, nnb;
  bool own_minus;
};

__device__ __forceinline__ int face_vol_node(int f, int a) {
  const int d = f >> 1;
  const int t1 = a % n1, t2 = a / n1;
  const int sn = d == 0 ? 1 : (d == 1 ? n1 : nf);
  const int s1 = d == 0 ? n1 : 1;
  const int s2 = d == 2 ? n1 : nf;
  return ((f & 1) ? N : 0) * sn + t1 * s1 + t2 * s2;
}

__device__ __forceinline__ CFaceItem cface(const int32_t* conn, const int32_t* nbr, int e, int q) {
  CFaceItem it;
  it.f = q / nf;
  it.a = q - it.f * nf;
  it.d = it.f >> 1;
  it.side = it.f & 1;
  it.nown = face_vol_node(it.f, it.a);
  int o = 0;
  if (conn) {
    const int32_t* c = conn + ((size_t)e * 6 + it.f) * 3;
    it.nb = c[0];
    it.fb = c[1];
    o = c[2];
  } else {
    it.nb = nbr[6 * e + it.f];
    it.fb = it.f ^ 1;
  }
  const int t1 = it.a % n1, t2 = it.a / n1;
  int u = (o & 1) ? t2 : t1, v = (o & 1) ? t1 : t2;
  if (o & 2) u = N - u;
  if (o & 4) v = N - v;
  it.ab = u + n1 * v;
  it.nnb = face_vol_node(it.fb, it.ab);
  const bool pb = it.fb & 1;
  it.own_minus = (it.side && !pb) || ((it.side != 0) == pb && (e < it.nb || (e == it.nb && it.f < it.fb)));
  return it;
}

__device__ __forceinline__ CFaceItem curved_face_item(const StageArgs& A, int e, int q) {
  return cface(A.conn, A.nbr, e, q);
}

// Loads of a curved face item: both conservative states in Cartesian
// components (L the minus, R the plus side), the metric row of each side's
// face direction at its node, signed by its face side (s Ja, s = +1 on +
// faces), and (Navier-Stokes) the neighbour's projected viscous flux.
struct CurvedFace {
  CFaceItem it;
  double L[5], R[5], jm[3], jp[3], fn[4];
};

template <bool NS>
__device__ __forceinline__ void curved_face_issue(const StageArgs& A, int e, CurvedFace& cf) {
  const CFaceItem& it = cf.it;
  const int eL = it.own_minus ? e : it.nb, eR = it.own_minus ? it.nb : e;
  const int nL = it.own_minus ? it.nown : it.nnb, nR = it.own_minus ? it.nnb : it.nown;
  const int fL = it.own_minus ? it.f : it.fb, fR = it.own_minus ? it.fb : it.f;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    cf.L[v] = A.U[((size_t)eL * 5 + v) * nn + nL];
    cf.R[v] = A.U[((size_t)eR * 5 + v) * nn + nR];
  }
  const double sL = (fL & 1) ? 1.0 : -1.0, sR = (fR & 1) ? 1.0 : -1.0;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    cf.jm[m] = sL * A.M[((size_t)eL * MS + 3 * (fL >> 1) + m) * nn + nL];
    cf.jp[m] = sR * A.M[((size_t)eR * MS + 3 * (fR >> 1) + m) * nn + nR];
  }
  if (NS) {
    const double* Fn = A.Fvf + ((size_t)it.nb * 6 + it.fb) * 4 * nf + it.ab;
#pragma unroll
    for (int c = 0; c < 4; ++c) cf.fn[c] = Fn[c * nf];
  }
}

// Face normal from the minus to the plus side, N = (s_m Ja_m - s_p Ja_p)/2
// (both elements form it bitwise alike), and the sign that turns values
// along N into values along the own face's reference direction +xi:
// s_own (own_minus ? +1 : -1).
__device__ __forceinline__ double curved_face_normal(const CurvedFace& cf, double Nv[3]) {
#pragma unroll
  for (int m = 0; m < 3; ++m) Nv[m] = 0.5 * (cf.jm[m] - cf.jp[m]);
  return (cf.it.side ? 1.0 : -1.0) * (cf.it.own_minus ? 1.0 : -1.0);
}

// Face metric and lifted interface value q* = (q- + q+)/2, q = (u, v, w, theta).
__device__ __forceinline__ void curved_face_q(const CurvedFace& cf, double gm1, double q[4]) {
  const double iL = rcp64(cf.L[0]), iR = rcp64(cf.R[0]);
  const double uL = cf.L[1] * iL, vL = cf.L[2] * iL, wL = cf.L[3] * iL;
  const double uR = cf.R[1] * iR, vR = cf.R[2] * iR, wR = cf.R[3] * iR;
  const double pL = gm1 * (cf.L[4] - 0.5 * (cf.L[1] * uL + cf.L[2] * vL + cf.L[3] * wL));
  const double pR = gm1 * (cf.R[4] - 0.5 * (cf.R[1] * uR + cf.R[2] * vR + cf.R[3] * wR));
  q[0] = 0.5 * (uL + uR);
  q[1] = 0.5 * (vL + vR);
  q[2] = 0.5 * (wL + wR);
  q[3] = 0.5 * (pL * iL + pR * iR);
}

// Split-form volume sum along reference direction D with the averaged metric
// (sums s = a + b of the node and partner values, js = Ja^D(a) + Ja^D(b)):
//   KG/PI: f_rho = rs un/8, f_m = rs un us/16 + ps js/4, f_E = rs un xs/16
//          (+ ps un/8 for KG), un = us.js;
//   STD:   (F(a).js + F(b).js)/4.
// Adds -(sum) to acc; with GRAD also returns the off-diagonal line sums of
// the BR1 gradient (Dhat/2 = D off the diagonal).
template <int VF, int D, bool GRAD>
__device__ __forceinline__ void volume_dir_curved(const double (*sP)[nnp], const double (*sM)[nn],
                                                  const double* sDhat, int n, int id, const double me[7],
                                                  const double jo[3], double acc[5], double* gs) {
  constexpr int st = D == 0 ? 1 : (D == 1 ? n1 : nf);
  const int base = n - id * st;
  const double* crow = sDhat + id * n1;
  double g0 = 0, g1 = 0, g2 = 0, g3 = 0;
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, px = 0, py = 0, pz = 0, s5 = 0;
  auto pair = [&](int l, int m) {
    const double c = crow[l];
    if (GRAD) {
      g0 = fma(c, sP[1][m], g0);
      g1 = fma(c, sP[2][m], g1);
      g2 = fma(c, sP[3][m], g2);
      g3 = fma(c, sP[6][m], g3);
    }
    const double jx = jo[0] + sM[3 * D + 0][m], jy = jo[1] + sM[3 * D + 1][m], jz = jo[2] + sM[3 * D + 2][m];
    if (VF == VF_STD) {
      const double ra = me[0], rb = sP[0][m];
      const double ua = me[1] * jx + me[2] * jy + me[3] * jz;
      const double ub = sP[1][m] * jx + sP[2][m] * jy + sP[3][m] * jz;
      const double fa = c * (ra * ua), fb = c * (rb * ub);
      s0 += fa + fb;
      s1 = fma(fa, me[1], fma(fb, sP[1][m], s1));
      s2 = fma(fa, me[2], fma(fb, sP[2][m], s2));
      s3 = fma(fa, me[3], fma(fb, sP[3][m], s3));
      s4 = fma(fa, me[5], fma(fb, sP[5][m], s4));
      const double cp = c * (me[4] + sP[4][m]);
      px = fma(cp, jx, px);
      py = fma(cp, jy, py);
      pz = fma(cp, jz, pz);
    } else {
      const double rs = me[0] + sP[0][m];
      const double us = me[1] + sP[1][m], vs = me[2] + sP[2][m], ws = me[3] + sP[3][m];
      const double ps = me[4] + sP[4][m], xs = me[5] + sP[5][m];
      const double un = us * jx + vs * jy + ws * jz;
      const double cf = c * (rs * un);
      s0 += cf;
      s1 = fma(cf, us, s1);
      s2 = fma(cf, vs, s2);
      s3 = fma(cf, ws, s3);
      s4 = fma(cf, xs, s4);
      const double cp = c * ps;
      px = fma(cp, jx, px);
      py = fma(cp, jy, py);
      pz = fma(cp, jz, pz);
      if (VF == VF_KG) s5 = fma(cp, un, s5);
    }
  };
  partner_loop<true, st>(id, n, base, pair);
  if (VF == VF_STD) {
    acc[0] -= 0.25 * s0;
    acc[1] -= 0.25 * (s1 + px);
    acc[2] -= 0.25 * (s2 + py);
    acc[3] -= 0.25 * (s3 + pz);
    acc[4] -= 0.25 * s4;
  } else {
    acc[0] -= 0.125 * s0;
    acc[1] -= 0.0625 * s1 + 0.25 * px;
    acc[2] -= 0.0625 * s2 + 0.25 * py;
    acc[3] -= 0.0625 * s3 + 0.25 * pz;
    acc[4] -= 0.0625 * s4 + (VF == VF_KG ? 0.125 * s5 : 0.0);
  }
  if (GRAD) {
    gs[0] = 0.5 * g0;
    gs[1] = 0.5 * g1;
    gs[2] = 0.5 * g2;
    gs[3] = 0.5 * g3;
  }
}

// Stage kernel on curved elements (one element per workgroup).  LDS:
// primitives sP[7][nnp] and node metrics sM[9][nn] (overlaid later by the
// twelve contravariant viscous fluxes sV[12][nnp]), interface fluxes
// sF[6][5][nf], and for Navier-Stokes q* sQ[6][4][nf], which the face metrics
// sJf[6][3][nf] overlay once the gradient is formed, and the neighbours'
// projected viscous fluxes sFn[6][4][nf].  At N = 5 this is 53 KB: three
// workgroups per CU, with at most 168 registers (3 waves per SIMD).
template <int VF, int EQ>
__global__ __launch_bounds__(NT, DG_N == 5 ? 3 : 1) void k_stage_curved(StageArgs A) {
  constexpr bool NS = EQ >= 1;
  constexpr int oM = 7 * nnp, oF = oM + 9 * nn, oQ = oF + 30 * nf, oFn = oQ + 24 * nf;
  constexpr int POOL = NS ? oFn + 24 * nf : oQ;
  static_assert(12 * nnp <= oF, "viscous exchange overlays primitives and metrics only");
  __shared__ double sPool[POOL];
  __shared__ double sB[NB_STAGE];
  double (*sP)[nnp] = reinterpret_cast<double (*)[nnp]>(sPool);
  double (*sM)[nn] = reinterpret_cast<double (*)[nn]>(sPool + oM);
  double (*sF)[5][nf] = reinterpret_cast<double (*)[5][nf]>(sPool + oF);
  double (*sQ)[4][nf] = reinterpret_cast<double (*)[4][nf]>(sPool + (NS ? oQ : 0));
  double (*sFn)[4][nf] = reinterpret_cast<double (*)[4][nf]>(sPool + (NS ? oFn : 0));
  double (*sJf)[3][nf] = reinterpret_cast<double (*)[3][nf]>(sPool + (NS ? oQ : 0));
  double (*sV)[nnp] = reinterpret_cast<double (*)[nnp]>(sPool);

  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const int t = threadIdx.x;
  const double gm1 = A.gamma - 1.0;
  constexpr int FIC = (6 * nf + NT - 1) / NT;
  CurvedFace cf[FIC];
#pragma unroll
  for (int k = 0; k < FIC; ++k)
    if (t + k * NT < 6 * nf) cf[k].it = curved_face_item(A, e, t + k * NT);
  const double* Ue = A.U + (size_t)e * 5 * nn;
  const double* Me = A.M + (size_t)e * MS * nn;
  double u[5], gprev[5], mt[MS];
  if (t < nn) {
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = Ue[v * nn + t];
#pragma unroll
    for (int k = 0; k < MS; ++k) mt[k] = Me[k * nn + t];
  }
  const double bval = t < NB_STAGE ? A.basis[t] : 0.0;
#pragma unroll
  for (int k = 0; k < FIC; ++k)
    if (t + k * NT < 6 * nf) curved_face_issue<NS>(A, e, cf[k]);
  if (t < NB_STAGE) sB[t] = bval;
  const double* sDhat = sB + BL.Dhat();
  const double* sDw = sB + BL.Dw();
  const double* swinv = sB + BL.winv();
  const Ref ref0{0.0, 0.0, 0.0};

  double me[7];
  double jfk[FIC][3];  // face metric along the own +xi, written to LDS after the gradient
  int ijk[3] = {0, 0, 0};
  if (t < nn) {
    primitives<VF, double, false>(u, gm1, ref0, me);
#pragma unroll
    for (int k = 0; k < 7; ++k)
      if (k < 6 || NS) sP[k][t] = me[k];
#pragma unroll
    for (int k = 0; k < 9; ++k) sM[k][t] = mt[k];
    ijk[0] = t % n1;
    ijk[1] = (t / n1) % n1;
    ijk[2] = t / nf;
  }
#pragma unroll
  for (int k = 0; k < FIC; ++k)
    if (t + k * NT < 6 * nf) {
      const CurvedFace& c = cf[k];
      const CFaceItem& it = c.it;
      double Nv[3];
      const double so = curved_face_normal(c, Nv);
      const double sh = sqrt64(Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2]);
      const double ish = rcp64(sh);
      const double nv[3] = {Nv[0] * ish, Nv[1] * ish, Nv[2] * ish};
      double f[5];
      surface_flux_normal<VF>(A.sf, c.L, c.R, nv, A.gamma, f);
      const double sc = so * sh;  // flux along the own face's +xi
#pragma unroll
      for (int v = 0; v < 5; ++v) sF[it.f][v][it.a] = sc * f[v];
      if (NS) {
        double q[4];
        curved_face_q(c, gm1, q);
        // the neighbour projected its flux on its own face metric: along
        // the own +xi that is -s_own s_nb times its value
        const double sn = ((it.side != 0) == ((it.fb & 1) != 0)) ? -1.0 : 1.0;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          sQ[it.f][cc][it.a] = q[cc];
          sFn[it.f][cc][it.a] = sn * c.fn[cc];
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) jfk[k][m] = so * Nv[m];
      }
    }
  __syncthreads();

  double acc[5] = {0, 0, 0, 0, 0};
  double Fv[3][4];
  if (t < nn) {
    double gs[3][4];
    volume_dir_curved<VF, 0, NS>(sP, sM, sDhat, t, ijk[0], me, mt + 0, acc, gs[0]);
    volume_dir_curved<VF, 1, NS>(sP, sM, sDhat, t, ijk[1], me, mt + 3, acc, gs[1]);
    volume_dir_curved<VF, 2, NS>(sP, sM, sDhat, t, ijk[2], me, mt + 6, acc, gs[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int id = ijk[d];
      const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
      if (id == 0 || id == N) {
        const int f = 2 * d + (id == N);
        const double c = id == N ? -swinv[N] : swinv[0];
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] = fma(c, sF[f][v][a], acc[v]);
      }
    }
    if (NS) {
      // reference-direction derivatives of q with the lifting, then the chain rule
      const double qo[4] = {me[1], me[2], me[3], me[6]};
      double s[3][4];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int id = ijk[d];
        const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
#pragma unroll
        for (int c = 0; c < 4; ++c) s[d][c] = gs[d][c];
        if (id == 0 || id == N) {
          const int f = 2 * d + (id == N);
          const double cd = sDw[id * n1 + id];
          const double w = id == N ? swinv[N] : -swinv[0];
#pragma unroll
          for (int c = 0; c < 4; ++c) s[d][c] = fma(w, sQ[f][c][a], fma(cd, qo[c], s[d][c]));
        }
      }
      const double iJ = mt[9];
      double g[3][4];
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          g[m][c] = iJ * (mt[m] * s[0][c] + mt[3 + m] * s[1][c] + mt[6 + m] * s[2][c]);
      double mu = A.mu, kap = A.kappa;
      if (EQ == 2) {  // Smagorinsky eddy viscosity with the element's filter width
        const double cs = A.cs_elem ? A.cs_elem[e] : A.cs;
        const double mut = eddy_viscosity<double>(g, me[0], cs * cs * A.delta2_elem[e]);
        mu += mut;
        kap = fma(A.ktf, mut, kap);
      }
      viscous_flux<0, double>(g, me[1], me[2], me[3], mu, kap, Fv[0]);
      viscous_flux<1, double>(g, me[1], me[2], me[3], mu, kap, Fv[1]);
      viscous_flux<2, double>(g, me[1], me[2], me[3], mu, kap, Fv[2]);
    }
  }

  if (t < nn && A.mode != MODE_UT && A.A != 0.0) {
#pragma unroll
    for (int v = 0; v < 5; ++v) gprev[v] = __builtin_nontemporal_load(&A.G[(size_t)e * 5 * nn + t + v * nn]);
  }
  if (NS) {
    __syncthreads();  // sP, sM and sQ consumed
    if (t < nn) {
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          sV[4 * d + c][t] = mt[3 * d] * Fv[0][c] + mt[3 * d + 1] * Fv[1][c] + mt[3 * d + 2] * Fv[2][c];
    }
#pragma unroll
    for (int k = 0; k < FIC; ++k)
      if (t + k * NT < 6 * nf)
#pragma unroll
        for (int m = 0; m < 3; ++m) sJf[cf[k].it.f][m][cf[k].it.a] = jfk[k][m];
    __syncthreads();
    if (t < nn) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
        const int id = ijk[d];
        const int base = t - id * st;
        const double* crow = sDw + id * n1;
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
        for (int l = 0; l < n1; ++l) {
          const int m = base + l * st;
          const double c = crow[l];
          s0 = fma(c, sV[4 * d + 0][m], s0);
          s1 = fma(c, sV[4 * d + 1][m], s1);
          s2 = fma(c, sV[4 * d + 2][m], s2);
          s3 = fma(c, sV[4 * d + 3][m], s3);
        }
        const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
        if (id == 0 || id == N) {  // Gt* = Ja_f . (Fv(own) + Fv(nb)) / 2, the neighbour's part in sFn
          const int f = 2 * d + (id == N);
          const double w = 0.5 * (id == N ? swinv[N] : -swinv[0]);
          const double jx = sJf[f][0][a], jy = sJf[f][1][a], jz = sJf[f][2][a];
          s0 = fma(w, jx * Fv[0][0] + jy * Fv[1][0] + jz * Fv[2][0] + sFn[f][0][a], s0);
          s1 = fma(w, jx * Fv[0][1] + jy * Fv[1][1] + jz * Fv[2][1] + sFn[f][1][a], s1);
          s2 = fma(w, jx * Fv[0][2] + jy * Fv[1][2] + jz * Fv[2][2] + sFn[f][2][a], s2);
          s3 = fma(w, jx * Fv[0][3] + jy * Fv[1][3] + jz * Fv[2][3] + sFn[f][3][a], s3);
        }
        acc[1] += s0;
        acc[2] += s1;
        acc[3] += s2;
        acc[4] += s3;
      }
    }
  }

  if (t < nn) {
    const double iJ = mt[9];
    const size_t o = (size_t)e * 5 * nn + t;
    if (A.mode != MODE_RK) {
#pragma unroll
      for (int v = 0; v < 5; ++v) A.Ut[o + v * nn] = acc[v] * iJ;
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double ut = acc[v] * iJ;
        double gv = ut;
        if (A.A != 0.0) gv = A.A * gprev[v] + ut;
        if (A.writeG) __builtin_nontemporal_store(gv, &A.G[o + v * nn]);  // streaming, as in k_stage
        __builtin_nontemporal_store(u[v] + A.Bdt * gv, &A.Uout[o + v * nn]);
      }
    }
  }
}

// BR1 lifting pass on curved elements: at each own face node the full
// lifted gradient (reference derivatives of q along the three directions with
// their lifting terms, chain rule with the node metric), the Cartesian viscous
// fluxes and their projection on the face metric, Ja_f . Fv -> Fvf[e][f][c][a].
// One element per workgroup (measured at N = 5: two elements per workgroup,
// which speeds up the Cartesian lifting kernel, make this one 9 % slower).
using PLC = Pack<1>;
template <bool LES>
__global__ __launch_bounds__(PLC::NTB) void k_lift_curved(StageArgs A) {
  constexpr int EPB = PLC::EPB, TPE = PLC::TPE, FIC = PLC::FI;
  __shared__ double sB[NB_STAGE];
  __shared__ double sqAll[EPB][LES ? 5 : 4][nn];
  __shared__ double sQAll[EPB][6][4][nf];
  const int e0 = EPB * element_of_block(blockIdx.x, A.chunk);
  if (e0 >= A.nelem) return;  // uniform over the workgroup
  const Slot sl = slot_of_thread<PLC>(e0, A.nelem);
  const int e = sl.e, t = sl.t, tid = threadIdx.x;
  double (*sq)[nn] = sqAll[sl.s];
  double (*sQ)[4][nf] = sQAll[sl.s];
  const double gm1 = A.gamma - 1.0;
  CurvedFace cf[FIC];
#pragma unroll
  for (int k = 0; k < FIC; ++k)
    if (t + k * TPE < 6 * nf) cf[k].it = curved_face_item(A, e, t + k * TPE);
  const double* Ue = A.U + (size_t)e * 5 * nn;
  double u[5];
  if (t < nn) {
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = Ue[v * nn + t];
  }
  const double bval = tid < NB_STAGE ? A.basis[tid] : 0.0;
#pragma unroll
  for (int k = 0; k < FIC; ++k)
    if (t + k * TPE < 6 * nf) curved_face_issue<false>(A, e, cf[k]);
  if (tid < NB_STAGE) sB[tid] = bval;
  if (t < nn) {
    const double ir = rcp64(u[0]);
    const double vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
    const double p = gm1 * (u[4] - 0.5 * (u[1] * vx + u[2] * vy + u[3] * vz));
    sq[0][t] = vx;
    sq[1][t] = vy;
    sq[2][t] = vz;
    sq[3][t] = p * ir;
    if (LES) sq[LES ? 4 : 0][t] = u[0];
  }
#pragma unroll
  for (int k = 0; k < FIC; ++k)
    if (t + k * TPE < 6 * nf) {
      double q[4];
      curved_face_q(cf[k], gm1, q);
#pragma unroll
      for (int c = 0; c < 4; ++c) sQ[cf[k].it.f][c][cf[k].it.a] = q[c];
    }
  __syncthreads();
  const double* sDw = sB + BL.Dw();
  const double* swinv = sB + BL.winv();
#pragma unroll
  for (int k = 0; k < FIC; ++k)
    if (t + k * TPE < 6 * nf) {
      const CFaceItem& it = cf[k].it;
      const int n = it.nown;
      const int ijk[3] = {n % n1, (n / n1) % n1, n / nf};
      const double* Mn = A.M + (size_t)e * MS * nn + n;
      double s[3][4];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
        const int id = ijk[d];
        const int base = n - id * st;
        const double* crow = sDw + id * n1;
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll 2
        for (int l = 0; l < n1; ++l) {
          const int m = base + l * st;
          const double c = crow[l];
          a0 = fma(c, sq[0][m], a0);
          a1 = fma(c, sq[1][m], a1);
          a2 = fma(c, sq[2][m], a2);
          a3 = fma(c, sq[3][m], a3);
        }
        if (id == 0 || id == N) {
          const int f = 2 * d + (id == N);
          const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
          const double w = id == N ? swinv[N] : -swinv[0];
          a0 = fma(w, sQ[f][0][a], a0);
          a1 = fma(w, sQ[f][1][a], a1);
          a2 = fma(w, sQ[f][2][a], a2);
          a3 = fma(w, sQ[f][3][a], a3);
        }
        s[d][0] = a0;
        s[d][1] = a1;
        s[d][2] = a2;
        s[d][3] = a3;
      }
      double mt[MS];
#pragma unroll
      for (int kk = 0; kk < MS; ++kk) mt[kk] = Mn[kk * nn];
      double g[3][4];
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          g[m][c] = mt[9] * (mt[m] * s[0][c] + mt[3 + m] * s[1][c] + mt[6 + m] * s[2][c]);
      double F[3][4];
      double mu = A.mu, kap = A.kappa;
      if (LES) {  // Smagorinsky eddy viscosity with the element's filter width
        const double cs = A.cs_elem ? A.cs_elem[e] : A.cs;
        const double mut = eddy_viscosity<double>(g, sq[LES ? 4 : 0][n], cs * cs * A.delta2_elem[e]);
        mu += mut;
        kap = fma(A.ktf, mut, kap);
      }
      viscous_flux<0, double>(g, sq[0][n], sq[1][n], sq[2][n], mu, kap, F[0]);
      viscous_flux<1, double>(g, sq[0][n], sq[1][n], sq[2][n], mu, kap, F[1]);
      viscous_flux<2, double>(g, sq[0][n], sq[1][n], sq[2][n], mu, kap, F[2]);
      double Nv[3];
      const double so = curved_face_normal(cf[k], Nv);
      const double Jf[3] = {so * Nv[0], so * Nv[1], so * Nv[2]};  // face metric along the own +xi
      double* out = A.Fvf + ((size_t)e * 6 + it.f) * 4 * nf + it.a;
#pragma unroll
      for (int c = 0; c < 4; ++c)  // streaming: read once, by the neighbour
        __builtin_nontemporal_store(Jf[0] * F[0][c] + Jf[1] * F[1][c] + Jf[2] * F[2][c], &out[c * nf]);
    }
}

// ===========================================================================
// Reverse mode on curved elements (FP64; Euler and Navier-Stokes; KG, PI and
// STD fluxes).  U_t = (1/J)(...) at every node, so with lt = lambda / J the
// Cartesian reverse formulas hold with the two-point flux along the averaged
// metric vector (Ja^i(n) + Ja^i(l))/2, the interface flux along the face
// normal N in its canonical orientation (its cotangent collects lt of both
// elements), the chain-rule gradient and the contravariant viscous flux.
// Pass 1 (k_vjp_lift_curved) writes, at each own face node, the cotangent of
// the reference derivative along the face direction times its lifting weight,
// which the neighbour's pass 2 (k_vjp_curved) reads.
// ===========================================================================

// Reverse mode of the interface flux along the unit normal n: the cotangent
// rotated into the frame (n, t1, t2), the rotated-frame reverse sweep
// (riemann_vjp), the state cotangents rotated back.
template <int VF>
__device__ __forceinline__ void flux_normal_vjp(int sf, const double L[5], const double R[5], const double n[3],
                                                double gamma, const double fb[5], double Lb[5], double Rb[5]) {
  const double ax = fabs(n[0]), ay = fabs(n[1]), az = fabs(n[2]);
  double t1[3];
  if (ax <= ay && ax <= az) {
    t1[0] = 0.0; t1[1] = n[2]; t1[2] = -n[1];
  } else if (ay <= az) {
    t1[0] = -n[2]; t1[1] = 0.0; t1[2] = n[0];
  } else {
    t1[0] = n[1]; t1[1] = -n[0]; t1[2] = 0.0;
  }
  const double it = rcp64(sqrt64(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]));
  t1[0] *= it; t1[1] *= it; t1[2] *= it;
  const double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
  double a[5], b[5], gb[5], ab[5], bb[5];
  a[0] = L[0]; a[4] = L[4];
  b[0] = R[0]; b[4] = R[4];
  a[1] = n[0] * L[1] + n[1] * L[2] + n[2] * L[3];
  a[2] = t1[0] * L[1] + t1[1] * L[2] + t1[2] * L[3];
  a[3] = t2[0] * L[1] + t2[1] * L[2] + t2[2] * L[3];
  b[1] = n[0] * R[1] + n[1] * R[2] + n[2] * R[3];
  b[2] = t1[0] * R[1] + t1[1] * R[2] + t1[2] * R[3];
  b[3] = t2[0] * R[1] + t2[1] * R[2] + t2[2] * R[3];
  gb[0] = fb[0];
  gb[1] = n[0] * fb[1] + n[1] * fb[2] + n[2] * fb[3];
  gb[2] = t1[0] * fb[1] + t1[1] * fb[2] + t1[2] * fb[3];
  gb[3] = t2[0] * fb[1] + t2[1] * fb[2] + t2[2] * fb[3];
  gb[4] = fb[4];
  riemann_vjp<VF>(sf, a, b, gamma, gb, ab, bb);
  Lb[0] = ab[0]; Lb[4] = ab[4];
  Rb[0] = bb[0]; Rb[4] = bb[4];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    Lb[1 + j] = n[j] * ab[1] + t1[j] * ab[2] + t2[j] * ab[3];
    Rb[1 + j] = n[j] * bb[1] + t1[j] * bb[2] + t2[j] * bb[3];
  }
}

// The minus (L) and plus (R) side of a curved face item and its normal
// N = (s_L Ja_L - s_R Ja_R)/2.
struct CurvedSides {
  int eL, eR, nL, nR, fL, fR;
};
__device__ __forceinline__ CurvedSides curved_sides(const CFaceItem& it, int e) {
  CurvedSides c;
  c.eL = it.own_minus ? e : it.nb;
  c.eR = it.own_minus ? it.nb : e;
  c.nL = it.own_minus ? it.nown : it.nnb;
  c.nR = it.own_minus ? it.nnb : it.nown;
  c.fL = it.own_minus ? it.f : it.fb;
  c.fR = it.own_minus ? it.fb : it.f;
  return c;
}
__device__ __forceinline__ void curved_normal(const double* M, const CurvedSides& c, double Nv[3]) {
  const double sL = (c.fL & 1) ? 1.0 : -1.0, sR = (c.fR & 1) ? 1.0 : -1.0;
#pragma unroll
  for (int m = 0; m < 3; ++m)
    Nv[m] = 0.5 * (sL * M[((size_t)c.eL * MS + 3 * (c.fL >> 1) + m) * nn + c.nL] -
                   sR * M[((size_t)c.eR * MS + 3 * (c.fR >> 1) + m) * nn + c.nR]);
}

// Reverse of the two-point flux along the direction vector nv (not unit) with
// respect to its first argument, in primitive variables (rho, u, p, x).
template <int VF>
__device__ __forceinline__ void twopoint_vjp_n(const double me[7], double rl, const double ul[3], double pl,
                                               double xl, const double nv[3], const double w[5], double pb[6]) {
  const double wn = w[1] * nv[0] + w[2] * nv[1] + w[3] * nv[2];
  if (VF == VF_STD) {
    const double r = me[0];
    const double un = me[1] * nv[0] + me[2] * nv[1] + me[3] * nv[2];
    const double s = w[0] + w[1] * me[1] + w[2] * me[2] + w[3] * me[3] + w[4] * me[5];
    pb[0] += 0.5 * un * s;
#pragma unroll
    for (int j = 0; j < 3; ++j) pb[1 + j] += 0.5 * (w[1 + j] * r * un + nv[j] * r * s);
    pb[4] += 0.5 * wn;
    pb[5] += 0.5 * w[4] * r * un;
    return;
  }
  const double rm = 0.5 * (me[0] + rl);
  const double um[3] = {0.5 * (me[1] + ul[0]), 0.5 * (me[2] + ul[1]), 0.5 * (me[3] + ul[2])};
  const double xm = 0.5 * (me[5] + xl);
  const double Un = um[0] * nv[0] + um[1] * nv[1] + um[2] * nv[2];
  const double fr = rm * Un;
  const double wr = w[0] + w[1] * um[0] + w[2] * um[1] + w[3] * um[2] + w[4] * xm;
  pb[0] += 0.5 * wr * Un;
#pragma unroll
  for (int j = 0; j < 3; ++j) pb[1 + j] += 0.5 * (w[1 + j] * fr + wr * rm * nv[j]);
  pb[4] += 0.5 * wn;
  pb[5] += 0.5 * w[4] * fr;
  if (VF == VF_KG) {
    const double pm = 0.5 * (me[4] + pl);
    pb[4] += 0.5 * w[4] * Un;
#pragma unroll
    for (int j = 0; j < 3; ++j) pb[1 + j] += 0.5 * w[4] * pm * nv[j];
  }
}

template <int VF, int D>
__device__ __forceinline__ void volume_vjp_dir_curved(const double (*sP)[nn], const double (*sM)[nn],
                                                      const double (*sLt)[nn], const double* sDhat, int n, int id,
                                                      const double me[7], const double jo[3], const double lt[5],
                                                      double pb[6]) {
  constexpr int st = D == 0 ? 1 : (D == 1 ? n1 : nf);
  const int base = n - id * st;
#pragma unroll 1
  for (int k = 1; k <= kPartners; ++k) {
    const int l = partner(id, k);
    const int m = base + l * st;
    const double c1 = -sDhat[id * n1 + l], c2 = -sDhat[l * n1 + id];
    double w[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) w[v] = fma(c1, lt[v], c2 * sLt[v][m]);
    const double nv[3] = {0.5 * (jo[0] + sM[3 * D][m]), 0.5 * (jo[1] + sM[3 * D + 1][m]),
                          0.5 * (jo[2] + sM[3 * D + 2][m])};
    const double ul[3] = {sP[1][m], sP[2][m], sP[3][m]};
    twopoint_vjp_n<VF>(me, sP[0][m], ul, sP[4][m], sP[5][m], nv, w, pb);
  }
}

// Interface part of curved face item q: (d ft*/d U_own)^T fbar, ft* the face
// flux |N| f*(U_L, U_R; N/|N|) in its canonical orientation and fbar its
// cotangent, sum over both elements of (lifting coefficient) x (orientation
// sign) x lt at their face node (flux_normal_vjp).
template <int VF>
__device__ __forceinline__ void vjp_face_item_curved(const VjpArgs& A, int e, int q, const double* swinv,
                                                     double (*sSF)[5][nf]) {
  const CFaceItem it = cface(A.conn, A.nbr, e, q);
  const CurvedSides c = curved_sides(it, e);
  double Nv[3];
  curved_normal(A.M, c, Nv);
  const double sh = sqrt64(Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2]);
  const double ish = rcp64(sh);
  const double nv[3] = {Nv[0] * ish, Nv[1] * ish, Nv[2] * ish};
  const double so = (it.side ? 1.0 : -1.0) * (it.own_minus ? 1.0 : -1.0);
  const double sb = ((it.fb & 1) ? 1.0 : -1.0) * (it.own_minus ? -1.0 : 1.0);
  const double co = so * (it.side ? -swinv[N] : swinv[0]) * A.M[((size_t)e * MS + 9) * nn + it.nown];
  const double cb = sb * ((it.fb & 1) ? -swinv[N] : swinv[0]) * A.M[((size_t)it.nb * MS + 9) * nn + it.nnb];
  const double* UL = A.U + (size_t)c.eL * 5 * nn;
  const double* UR = A.U + (size_t)c.eR * 5 * nn;
  const double* Lo = A.Lbar + (size_t)e * 5 * nn;
  const double* Lb = A.Lbar + (size_t)it.nb * 5 * nn;
  double L[5], R[5], fb[5], Lc[5], Rc[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    L[v] = UL[v * nn + c.nL];
    R[v] = UR[v * nn + c.nR];
    fb[v] = fma(co, Lo[v * nn + it.nown], cb * Lb[v * nn + it.nnb]);
  }
  flux_normal_vjp<VF>(A.sf, L, R, nv, A.gamma, fb, Lc, Rc);
#pragma unroll
  for (int v = 0; v < 5; ++v) sSF[it.f][v][it.a] = sh * (it.own_minus ? Lc[v] : Rc[v]);
}

// Navier-Stokes face data of face item q: the face metric along the own +xi
// (sJo), the neighbour's lt at its node scaled by -s_own s_nb w_nb (sLn; w the
// lifting weight of the neighbour's face), and, with Q, q* (forward gradient)
// and the neighbour's pass-1 output (sGn).
template <bool Q, bool GN = Q>
__device__ __forceinline__ void vjp_face_ns_curved(const VjpArgs& A, int e, int q, const double* swinv,
                                                   double (*sJo)[3][nf], double (*sLn)[4][nf], double (*sQ)[4][nf],
                                                   double (*sGn)[4][nf]) {
  const CFaceItem it = cface(A.conn, A.nbr, e, q);
  const CurvedSides c = curved_sides(it, e);
  double Nv[3];
  curved_normal(A.M, c, Nv);
  const double so = (it.side ? 1.0 : -1.0) * (it.own_minus ? 1.0 : -1.0);
#pragma unroll
  for (int m = 0; m < 3; ++m) sJo[it.f][m][it.a] = so * Nv[m];
  const double sameside = ((it.side != 0) == ((it.fb & 1) != 0)) ? -1.0 : 1.0;  // -s_own s_nb
  const double wb = (it.fb & 1) ? swinv[N] : -swinv[0];
  const double lb = sameside * wb * A.M[((size_t)it.nb * MS + 9) * nn + it.nnb];
  const double* Lb = A.Lbar + (size_t)it.nb * 5 * nn;
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) sLn[it.f][cc][it.a] = lb * Lb[(1 + cc) * nn + it.nnb];
  if (Q) {
    double L[5], R[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      L[v] = A.U[((size_t)c.eL * 5 + v) * nn + c.nL];
      R[v] = A.U[((size_t)c.eR * 5 + v) * nn + c.nR];
    }
    const double gm1 = A.gamma - 1.0;
    const double iL = rcp64(L[0]), iR = rcp64(R[0]);
    const double uL = L[1] * iL, vL = L[2] * iL, wL = L[3] * iL, uR = R[1] * iR, vR = R[2] * iR, wR = R[3] * iR;
    const double pL = gm1 * (L[4] - 0.5 * (L[1] * uL + L[2] * vL + L[3] * wL));
    const double pR = gm1 * (R[4] - 0.5 * (R[1] * uR + R[2] * vR + R[3] * wR));
    sQ[it.f][0][it.a] = 0.5 * (uL + uR);
    sQ[it.f][1][it.a] = 0.5 * (vL + vR);
    sQ[it.f][2][it.a] = 0.5 * (wL + wR);
    sQ[it.f][3][it.a] = 0.5 * (pL * iL + pR * iR);
    if (GN) {
      const double* Gn = A.Gbf + ((size_t)it.nb * 6 + it.fb) * 4 * nf;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) sGn[it.f][cc][it.a] = Gn[cc * nf + it.ab];
    }
  }
}

// Cotangent of the Cartesian viscous fluxes Fvb[m][c] at node p: the
// contravariant cotangents from lt along the three lines (Dw transposed),
// mapped by the node metric, plus the face terms Jo (w_own lt_own + sLn)/2 of
// the faces containing p.
__device__ __forceinline__ void viscous_flux_cotangent_curved(const double (*sLt)[nn], const double (*sLn)[4][nf],
                                                              const double (*sJo)[3][nf], const double* sDw,
                                                              const double* swinv, int p, const int ijk[3],
                                                              const double mt[MS], double Fvb[3][4]) {
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) Fvb[m][cc] = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
    const int id = ijk[d];
    const int base = p - id * st;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      const double c = sDw[l * n1 + id];
      const int k = base + l * st;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) s[cc] = fma(c, sLt[1 + cc][k], s[cc]);
    }
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) Fvb[m][cc] = fma(mt[3 * d + m], s[cc], Fvb[m][cc]);
    if (id == 0 || id == N) {
      const int f = 2 * d + (id == N);
      const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
      const double wo = id == N ? swinv[N] : -swinv[0];
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const double tt = 0.5 * fma(wo, sLt[1 + cc][p], sLn[f][cc][a]);
#pragma unroll
        for (int m = 0; m < 3; ++m) Fvb[m][cc] = fma(sJo[f][m][a], tt, Fvb[m][cc]);
      }
    }
  }
}

// Pass 1: at each own face node, the cotangent of the reference derivative of
// q along the face direction times the face's lifting weight -> Gbf[e][f][c][a].
// With the Smagorinsky model (LES) the gradient cotangent at a face node
// depends on the eddy viscosity there: the kernel then also forms the forward
// chain-rule gradient at its own face nodes (q at all nodes, q* of all faces).
template <bool LES>
__global__ __launch_bounds__(NT) void k_vjp_lift_curved(VjpArgs A) {
  __shared__ double sB[NB_STAGE];
  __shared__ double sLt[5][nn];
  __shared__ double sU[LES ? 5 : 3][nn];  // u, v, w (, theta, rho)
  __shared__ double sLn[6][4][nf];
  __shared__ double sJo[6][3][nf];
  __shared__ double sQ[LES ? 6 : 1][4][nf];
  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const int t = threadIdx.x;
  for (int q = t; q < NB_STAGE; q += NT) sB[q] = A.basis[q];
  const double* swinv = sB + BL.winv();
  if (t < nn) {
    const double* Ue = A.U + (size_t)e * 5 * nn;
    const double* Le = A.Lbar + (size_t)e * 5 * nn;
    const double ir = rcp64(Ue[t]);
    const double iJ = A.M[((size_t)e * MS + 9) * nn + t];
#pragma unroll
    for (int j = 0; j < 3; ++j) sU[j][t] = Ue[(1 + j) * nn + t] * ir;
    if (LES) {
      const double p = (A.gamma - 1.0) * (Ue[4 * nn + t] - 0.5 * (Ue[nn + t] * sU[0][t] + Ue[2 * nn + t] * sU[1][t] +
                                                                 Ue[3 * nn + t] * sU[2][t]));
      sU[LES ? 3 : 0][t] = p * ir;
      sU[LES ? 4 : 0][t] = Ue[t];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) sLt[v][t] = Le[v * nn + t] * iJ;
  }
  __syncthreads();  // swinv
  for (int q = t; q < 6 * nf; q += NT) {
    if (LES) vjp_face_ns_curved<true, false>(A, e, q, swinv, sJo, sLn, sQ, nullptr);
    else vjp_face_ns_curved<false>(A, e, q, swinv, sJo, sLn, nullptr, nullptr);
  }
  __syncthreads();
  const double csd2 = LES ? vjp_csd2(A, e) : 0.0;
  for (int q = t; q < 6 * nf; q += NT) {
    const int f = q / nf, a = q - f * nf, d = f >> 1;
    const int p = face_vol_node(f, a);
    const int ijk[3] = {p % n1, (p / n1) % n1, p / nf};
    double mt[MS];
#pragma unroll
    for (int k = 0; k < MS; ++k) mt[k] = A.M[((size_t)e * MS + k) * nn + p];
    double Fvb[3][4], gb[3][4];
    viscous_flux_cotangent_curved(sLt, sLn, sJo, sB + BL.Dw(), swinv, p, ijk, mt, Fvb);
    const double u[3] = {sU[0][p], sU[1][p], sU[2][p]};
    if (LES) {  // forward chain-rule gradient at p: reference derivatives with lifting
      const double* sDw = sB + BL.Dw();
      double sr[3][4];
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) {
        const int st = dd == 0 ? 1 : (dd == 1 ? n1 : nf);
        const int id = ijk[dd];
        const int base = p - id * st;
        const double* crow = sDw + id * n1;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int l = 0; l < n1; ++l) {
          const double c = crow[l];
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) acc[cc] = fma(c, sU[cc][base + l * st], acc[cc]);
        }
        if (id == 0 || id == N) {
          const int ff = 2 * dd + (id == N);
          const int aa = dd == 0 ? ijk[1] + n1 * ijk[2] : (dd == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
          const double w = id == N ? swinv[N] : -swinv[0];
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) acc[cc] = fma(w, sQ[ff][cc][aa], acc[cc]);
        }
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) sr[dd][cc] = acc[cc];
      }
      double g[3][4];
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int c = 0; c < 4; ++c) g[m][c] = mt[9] * (mt[m] * sr[0][c] + mt[3 + m] * sr[1][c] + mt[6 + m] * sr[2][c]);
      double rhob = 0.0;
      les_gradient_cotangent(Fvb, u, g, sU[LES ? 4 : 0][p], A.mu, A.kappa, csd2, A.ktf, gb, rhob);
    } else {
      gradient_cotangent(Fvb, u, A.mu, A.kappa, gb);
    }
    const double w = (f & 1) ? swinv[N] : -swinv[0];
    double* out = A.Gbf + ((size_t)e * 6 + f) * 4 * nf;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      out[c * nf + a] = w * mt[9] * (mt[3 * d] * gb[0][c] + mt[3 * d + 1] * gb[1][c] + mt[3 * d + 2] * gb[2][c]);
  }
}

// Pass 2: U_bar (or U_acc + U_bar) on curved elements.
template <int VF, int EQ>
__global__ __launch_bounds__(NT) void k_vjp_curved(VjpArgs A) {
  constexpr bool NS = (EQ >= 1);
  constexpr bool LES = (EQ == 2);
  __shared__ double sB[NB_STAGE];
  __shared__ double sP[7][nn];
  __shared__ double sM[9][nn];
  __shared__ double sLt[5][nn];
  __shared__ double sSF[6][5][nf];
  __shared__ double sQ[NS ? 6 : 1][4][nf];
  __shared__ double sLn[NS ? 6 : 1][4][nf];
  __shared__ double sGn[NS ? 6 : 1][4][nf];
  __shared__ double sJo[NS ? 6 : 1][3][nf];
  const int e = element_of_block(blockIdx.x, A.chunk);
  if (e >= A.nelem) return;
  const int t = threadIdx.x;
  const double gm1 = A.gamma - 1.0;
  for (int q = t; q < NB_STAGE; q += NT) sB[q] = A.basis[q];
  const double* sDhat = sB + BL.Dhat();
  const double* sDw = sB + BL.Dw();
  const double* swinv = sB + BL.winv();
  const Ref ref{0.0, 0.0, 0.0};
  double u[5], me[7], lt[5], mt[MS];
  int ijk[3] = {0, 0, 0};
  if (t < nn) {
    const double* Ue = A.U + (size_t)e * 5 * nn;
    const double* Le = A.Lbar + (size_t)e * 5 * nn;
#pragma unroll
    for (int k = 0; k < MS; ++k) mt[k] = A.M[((size_t)e * MS + k) * nn + t];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      u[v] = Ue[v * nn + t];
      lt[v] = Le[v * nn + t] * mt[9];
      sLt[v][t] = lt[v];
    }
    primitives<VF, double, false>(u, gm1, ref, me);
#pragma unroll
    for (int k = 0; k < 7; ++k) sP[k][t] = me[k];
#pragma unroll
    for (int k = 0; k < 9; ++k) sM[k][t] = mt[k];
    ijk[0] = t % n1;
    ijk[1] = (t / n1) % n1;
    ijk[2] = t / nf;
  }
  __syncthreads();  // swinv
#pragma unroll 1
  for (int q = t; q < 6 * nf; q += NT) vjp_face_item_curved<VF>(A, e, q, swinv, sSF);
  if (NS)
    for (int q = t; q < 6 * nf; q += NT) vjp_face_ns_curved<true>(A, e, q, swinv, sJo, sLn, sQ, sGn);
  __syncthreads();

  double pb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double thb = 0.0;
  double sb[3][4];  // cotangents of the reference derivatives of q
  if (t < nn) {
    volume_vjp_dir_curved<VF, 0>(sP, sM, sLt, sDhat, t, ijk[0], me, mt + 0, lt, pb);
    volume_vjp_dir_curved<VF, 1>(sP, sM, sLt, sDhat, t, ijk[1], me, mt + 3, lt, pb);
    volume_vjp_dir_curved<VF, 2>(sP, sM, sLt, sDhat, t, ijk[2], me, mt + 6, lt, pb);
    if (NS) {
      double Fvb[3][4];
      viscous_flux_cotangent_curved(sLt, sLn, sJo, sDw, swinv, t, ijk, mt, Fvb);
      // forward gradient: reference derivatives with lifting, chain rule
      double s[3][4];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
        const int id = ijk[d];
        const int base = t - id * st;
        const double* crow = sDw + id * n1;
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
        for (int l = 0; l < n1; ++l) {
          const int m = base + l * st;
          const double c = crow[l];
          a0 = fma(c, sP[1][m], a0);
          a1 = fma(c, sP[2][m], a1);
          a2 = fma(c, sP[3][m], a2);
          a3 = fma(c, sP[6][m], a3);
        }
        if (id == 0 || id == N) {
          const int f = 2 * d + (id == N);
          const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
          const double w = id == N ? swinv[N] : -swinv[0];
          a0 = fma(w, sQ[f][0][a], a0);
          a1 = fma(w, sQ[f][1][a], a1);
          a2 = fma(w, sQ[f][2][a], a2);
          a3 = fma(w, sQ[f][3][a], a3);
        }
        s[d][0] = a0;
        s[d][1] = a1;
        s[d][2] = a2;
        s[d][3] = a3;
      }
      double g[3][4];
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int c = 0; c < 4; ++c) g[m][c] = mt[9] * (mt[m] * s[0][c] + mt[3 + m] * s[1][c] + mt[6 + m] * s[2][c]);
      const double csd2 = LES ? vjp_csd2(A, e) : 0.0;
      const double mue = LES ? A.mu + eddy_viscosity<double>(g, me[0], csd2) : A.mu;
      const double div = g[0][0] + g[1][1] + g[2][2];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double tau = mue * (g[d][j] + g[j][d]) - (j == d ? (2.0 / 3.0) * mue * div : 0.0);
          acc = fma(tau, Fvb[d][3], acc);
        }
        pb[1 + j] += acc;
      }
      double gb[3][4];
      const double uu[3] = {me[1], me[2], me[3]};
      if (LES) les_gradient_cotangent(Fvb, uu, g, me[0], A.mu, A.kappa, csd2, A.ktf, gb, pb[0]);
      else gradient_cotangent(Fvb, uu, A.mu, A.kappa, gb);
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          sb[d][c] = mt[9] * (mt[3 * d] * gb[0][c] + mt[3 * d + 1] * gb[1][c] + mt[3 * d + 2] * gb[2][c]);
    }
  }
  if (NS) {
    // q_bar = sum_d [ Dw^T sb_d along the d line + (w_own sb_d + neighbour's) / 2 at faces ]
    double (*sX)[nn] = sLt;  // lt is no longer needed
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      __syncthreads();
      if (t < nn) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sX[c][t] = sb[d][c];
      }
      __syncthreads();
      if (t < nn) {
        const int st = d == 0 ? 1 : (d == 1 ? n1 : nf);
        const int id = ijk[d];
        const int base = t - id * st;
        double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int l = 0; l < n1; ++l) {
          const double c = sDw[l * n1 + id];
          const int k = base + l * st;
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) s[cc] = fma(c, sX[cc][k], s[cc]);
        }
        if (id == 0 || id == N) {
          const int f = 2 * d + (id == N);
          const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
          const double wo = id == N ? swinv[N] : -swinv[0];
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) s[cc] += 0.5 * fma(wo, sb[d][cc], sGn[f][cc][a]);
        }
        pb[1] += s[0];
        pb[2] += s[1];
        pb[3] += s[2];
        thb += s[3];
      }
    }
  }
  if (t < nn) {
    const double ir = rcp64(u[0]);
    double rb = pb[0], ub[3] = {pb[1], pb[2], pb[3]}, pbar = pb[4], Eb = 0.0;
    if (VF == VF_KG) {
      Eb += pb[5] * ir;
      rb -= pb[5] * me[5] * ir;
    } else {
      Eb += pb[5] * ir;
      pbar += pb[5] * ir;
      rb -= pb[5] * me[5] * ir;
    }
    pbar += thb * ir;
    rb -= thb * me[6] * ir;
    const double q2 = me[1] * me[1] + me[2] * me[2] + me[3] * me[3];
    Eb += gm1 * pbar;
    rb += gm1 * pbar * 0.5 * q2;
    double mb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      mb[j] = -gm1 * pbar * me[1 + j] + ub[j] * ir;
      rb -= ub[j] * me[1 + j] * ir;
    }
    double out[5] = {rb, mb[0], mb[1], mb[2], Eb};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int id = ijk[d];
      const int a = d == 0 ? ijk[1] + n1 * ijk[2] : (d == 1 ? ijk[0] + n1 * ijk[2] : ijk[0] + n1 * ijk[1]);
      if (id == N)
#pragma unroll
        for (int v = 0; v < 5; ++v) out[v] += sSF[2 * d + 1][v][a];
      if (id == 0)
#pragma unroll
        for (int v = 0; v < 5; ++v) out[v] += sSF[2 * d][v][a];
    }
    const size_t o = (size_t)e * 5 * nn + t;
#pragma unroll
    for (int v = 0; v < 5; ++v) A.Ubar[o + v * nn] = A.Uacc ? A.Uacc[o + v * nn] + out[v] : out[v];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
inline int blocks_for(const StageArgs& A) { return 8 * A.chunk; }

// Stage and lifting kernels: P::EPB elements per workgroup, the groups of
// consecutive elements split into 8 XCD-contiguous ranges.
template <class P>
inline StageArgs grouped(const StageArgs& A) {
  StageArgs B = A;
  B.chunk = ((A.nelem + P::EPB - 1) / P::EPB + 7) / 8;
  return B;
}

template <int VF, class R>
hipError_t launch_stage_vf(const StageArgs& A0, int eq, hipStream_t s) {
  const StageArgs A = grouped<PS>(A0);
  const dim3 grid(blocks_for(A)), block(PS::NTB);
  if (A.wall_dir >= 0) {  // walls: FP64 Navier-Stokes (checked on the host)
    if constexpr (sizeof(R) == 8) {
      if (eq == 2) {
        if constexpr (VF != VF_CH) {
          if (A.blend) hipLaunchKernelGGL((k_stage<VF, 2, true, double, true>), grid, block, 0, s, A);
          else hipLaunchKernelGGL((k_stage<VF, 2, false, double, true>), grid, block, 0, s, A);
        } else {
          return hipErrorInvalidValue;
        }
      } else if (eq == 1) {
        if (A.blend) hipLaunchKernelGGL((k_stage<VF, 1, true, double, true>), grid, block, 0, s, A);
        else hipLaunchKernelGGL((k_stage<VF, 1, false, double, true>), grid, block, 0, s, A);
      } else {
        return hipErrorInvalidValue;
      }
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (A.blend && eq >= 1) {  // FP64 (checked on the host)
    if constexpr (sizeof(R) == 8) {
      if (eq == 2) {
        if constexpr (VF != VF_CH) hipLaunchKernelGGL((k_stage<VF, 2, true, double>), grid, block, 0, s, A);
        else return hipErrorInvalidValue;
      } else {
        hipLaunchKernelGGL((k_stage<VF, 1, true, double>), grid, block, 0, s, A);
      }
    } else {
      return hipErrorInvalidValue;
    }
  } else if (eq == 2) {
    if constexpr (VF != VF_CH) hipLaunchKernelGGL((k_stage<VF, 2, false, R>), grid, block, 0, s, A);
    else return hipErrorInvalidValue;
  } else if (eq == 1) {
    if constexpr (sizeof(R) == 8) {
      if (A.split) {
        hipLaunchKernelGGL((k_stage<VF, 1, false, double, false, true>), grid, block, 0, s, A);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_stage<VF, 1, false, R>), grid, block, 0, s, A);
  } else if (A.blend) {
    if constexpr (sizeof(R) == 8) hipLaunchKernelGGL((k_stage<VF, 0, true, double>), grid, block, 0, s, A);
    else return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((k_stage<VF, 0, false, R>), grid, block, 0, s, A);
  }
  return hipGetLastError();
}

hipError_t launch_stage(const StageArgs& A, int eq, hipStream_t s) {
  switch (A.vf) {
    case VF_KG: return launch_stage_vf<VF_KG, double>(A, eq, s);
    case VF_PI: return launch_stage_vf<VF_PI, double>(A, eq, s);
    case VF_CH: return launch_stage_vf<VF_CH, double>(A, eq, s);
    default: return launch_stage_vf<VF_STD, double>(A, eq, s);
  }
}

// Mixed operator: flux forms whose reference shift is exact (PI, STD).
hipError_t launch_stage_mixed(const StageArgs& A, int eq, hipStream_t s) {
  switch (A.vf) {
    case VF_PI: return launch_stage_vf<VF_PI, float>(A, eq, s);
    case VF_STD: return launch_stage_vf<VF_STD, float>(A, eq, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_lift(const StageArgs& A0, int eq, hipStream_t s) {
  const StageArgs A = grouped<PL>(A0);
  if (A.wall_dir >= 0) {
    if (eq == 2) hipLaunchKernelGGL((k_lift<double, true, true>), dim3(blocks_for(A)), dim3(PL::NTB), 0, s, A);
    else hipLaunchKernelGGL((k_lift<double, false, true>), dim3(blocks_for(A)), dim3(PL::NTB), 0, s, A);
    return hipGetLastError();
  }
  if (eq == 2) hipLaunchKernelGGL((k_lift<double, true>), dim3(blocks_for(A)), dim3(PL::NTB), 0, s, A);
  else if (A.split) {
    const StageArgs B = grouped<PS>(A0);
    hipLaunchKernelGGL(k_lift_split, dim3(blocks_for(B)), dim3(PS::NTB), 0, s, B);
  } else {
    hipLaunchKernelGGL((k_lift<double, false>), dim3(blocks_for(A)), dim3(PL::NTB), 0, s, A);
  }
  return hipGetLastError();
}

hipError_t launch_wall_flux(const StageArgs& A, hipStream_t s) {
  const int wd = A.wall_dir;
  if (wd < 0 || wd > 2) return hipErrorInvalidValue;
  const long long total = 2LL * A.ne[wd == 0 ? 1 : 0] * A.ne[wd == 2 ? 1 : 2] * nf;
  hipLaunchKernelGGL(k_wall_flux, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_lift_mixed(const StageArgs& A0, int eq, hipStream_t s) {
  const StageArgs A = grouped<PL>(A0);
  if (A.wall_dir >= 0) return hipErrorInvalidValue;
  if (eq == 2) hipLaunchKernelGGL((k_lift<float, true>), dim3(blocks_for(A)), dim3(PL::NTB), 0, s, A);
  else hipLaunchKernelGGL((k_lift<float, false>), dim3(blocks_for(A)), dim3(PL::NTB), 0, s, A);
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

template <int VF>
hipError_t launch_vjp_vf(const VjpArgs& A, int eq, hipStream_t s) {
  const dim3 grid(8 * A.chunk), block(NT);
  if (A.wall_dir >= 0) {  // walls: Navier-Stokes (checked on the host)
    if (eq == 2) hipLaunchKernelGGL((k_vjp<VF, 2, true>), grid, block, 0, s, A);
    else if (eq == 1) hipLaunchKernelGGL((k_vjp<VF, 1, true>), grid, block, 0, s, A);
    else return hipErrorInvalidValue;
  } else if (eq == 2) hipLaunchKernelGGL((k_vjp<VF, 2>), grid, block, 0, s, A);
  else if (eq == 1) hipLaunchKernelGGL((k_vjp<VF, 1>), grid, block, 0, s, A);
  else hipLaunchKernelGGL((k_vjp<VF, 0>), grid, block, 0, s, A);
  return hipGetLastError();
}

hipError_t launch_vjp(const VjpArgs& A, int eq, hipStream_t s) {
  switch (A.vf) {
    case VF_KG: return launch_vjp_vf<VF_KG>(A, eq, s);
    case VF_PI: return launch_vjp_vf<VF_PI>(A, eq, s);
    case VF_STD: return launch_vjp_vf<VF_STD>(A, eq, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_vjp_alpha_bar(const VjpArgs& A, hipStream_t s) {
  hipLaunchKernelGGL(k_vjp_alpha_bar, dim3(8 * A.chunk), dim3(NT), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_vjp_alpha(const VjpArgs& A, hipStream_t s) {
  hipLaunchKernelGGL(k_vjp_alpha, dim3(8 * A.chunk), dim3(NT), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_vjp_fv(const VjpArgs& A, hipStream_t s) {
  const dim3 grid(8 * A.chunk), block(NT);
  switch (A.vf) {
    case VF_KG: hipLaunchKernelGGL(k_vjp_fv<VF_KG>, grid, block, 0, s, A); break;
    case VF_PI: hipLaunchKernelGGL(k_vjp_fv<VF_PI>, grid, block, 0, s, A); break;
    case VF_STD: hipLaunchKernelGGL(k_vjp_fv<VF_STD>, grid, block, 0, s, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_vjp_lift(const VjpArgs& A, hipStream_t s) {
  if (A.les) hipLaunchKernelGGL(k_vjp_lift_les, dim3(8 * A.chunk), dim3(NT), 0, s, A);
  else hipLaunchKernelGGL(k_vjp_lift, dim3(8 * A.chunk), dim3(NT), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_axpby(double* y, double a, const double* x, double b, size_t n, hipStream_t s) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)blocks), dim3(256), 0, s, y, a, x, b, n);
  return hipGetLastError();
}

template <int VF>
hipError_t launch_stage_curved_vf(const StageArgs& A, int eq, hipStream_t s) {
  const dim3 grid(blocks_for(A)), block(NT);
  if (eq == 2) hipLaunchKernelGGL((k_stage_curved<VF, 2>), grid, block, 0, s, A);
  else if (eq == 1) hipLaunchKernelGGL((k_stage_curved<VF, 1>), grid, block, 0, s, A);
  else hipLaunchKernelGGL((k_stage_curved<VF, 0>), grid, block, 0, s, A);
  return hipGetLastError();
}

// Curved elements: KG, PI and STD volume fluxes.
hipError_t launch_stage_curved(const StageArgs& A, int eq, hipStream_t s) {
  switch (A.vf) {
    case VF_KG: return launch_stage_curved_vf<VF_KG>(A, eq, s);
    case VF_PI: return launch_stage_curved_vf<VF_PI>(A, eq, s);
    case VF_STD: return launch_stage_curved_vf<VF_STD>(A, eq, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_lift_curved(const StageArgs& A0, int eq, hipStream_t s) {
  const StageArgs A = grouped<PLC>(A0);
  if (eq == 2) hipLaunchKernelGGL((k_lift_curved<true>), dim3(blocks_for(A)), dim3(PLC::NTB), 0, s, A);
  else hipLaunchKernelGGL((k_lift_curved<false>), dim3(blocks_for(A)), dim3(PLC::NTB), 0, s, A);
  return hipGetLastError();
}

template <int VF>
hipError_t launch_vjp_curved_vf(const VjpArgs& A, int eq, hipStream_t s) {
  const dim3 grid(8 * A.chunk), block(NT);
  if (eq == 2) hipLaunchKernelGGL((k_vjp_curved<VF, 2>), grid, block, 0, s, A);
  else if (eq == 1) hipLaunchKernelGGL((k_vjp_curved<VF, 1>), grid, block, 0, s, A);
  else hipLaunchKernelGGL((k_vjp_curved<VF, 0>), grid, block, 0, s, A);
  return hipGetLastError();
}

hipError_t launch_vjp_curved(const VjpArgs& A, int eq, hipStream_t s) {
  switch (A.vf) {
    case VF_KG: return launch_vjp_curved_vf<VF_KG>(A, eq, s);
    case VF_PI: return launch_vjp_curved_vf<VF_PI>(A, eq, s);
    case VF_STD: return launch_vjp_curved_vf<VF_STD>(A, eq, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_vjp_lift_curved(const VjpArgs& A, hipStream_t s) {
  if (A.les) hipLaunchKernelGGL((k_vjp_lift_curved<true>), dim3(8 * A.chunk), dim3(NT), 0, s, A);
  else hipLaunchKernelGGL((k_vjp_lift_curved<false>), dim3(8 * A.chunk), dim3(NT), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_metrics(const double* X, const double* basis, double* M, int* bad, double* d2, int nelem,
                          int chunk, hipStream_t s) {
  hipLaunchKernelGGL(k_metrics, dim3(8 * chunk), dim3(NT), 0, s, X, basis, M, bad, d2, nelem, chunk);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const ReduceArgs& R, hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite, dim3(RED_BLOCKS), dim3(NT), 0, s, R);
  return hipGetLastError();
}

const KernelTable kTable = {
    NT, kFusedAlpha1 ? 1 : 0, launch_stage, launch_stage_mixed, launch_lift, launch_lift_mixed, launch_alpha1, launch_spread,
    launch_max_rate, launch_integrals, launch_nonfinite, launch_vjp, launch_vjp_lift, launch_vjp_alpha_bar,
    launch_vjp_alpha, launch_vjp_fv, launch_axpby, launch_metrics, launch_stage_curved, launch_lift_curved,
    launch_vjp_curved, launch_vjp_lift_curved, launch_wall_flux,
};

}  // namespace

#define DG_CAT2(a, b) a##b
#define DG_CAT(a, b) DG_CAT2(a, b)
const KernelTable* DG_CAT(table_N, DG_N)() { return &kTable; }

}  // namespace dgmi
