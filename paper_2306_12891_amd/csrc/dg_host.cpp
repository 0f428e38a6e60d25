// Host side of libdgmi: argument validation, context and scratch management,
// the 1-D Legendre-Gauss-Lobatto basis, the periodic neighbour table, the
// Runge-Kutta stage loop and the C ABI declared in include/dg.h.
// No arithmetic of the operator runs here: every step is a HIP kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "dg.h"
#include "dg_internal.hpp"

using namespace dgmi;

// Device scratch of dg_vjp_noalloc: a file-scope array instead of allocations,
// for callers that cannot allocate device memory.  Every GPU the library runs
// on holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device
// (kept per device in g_scratch), never through the array's name.
static __device__ __align__(256) double scratch[(size_t(64) << 20) / sizeof(double)];

namespace {

constexpr int kRedBlocks = 1024;  // must match the reduction grid of the kernels

// Carpenter-Kennedy five-stage fourth-order 2N-storage coefficients (the
// explicit Runge-Kutta scheme of the paper's Sec. 2, whose stages enter the PID).
const double kA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                      -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                      1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                      2277821191437.0 / 14882151754819.0};

char g_init_error[256] = "";

constexpr size_t kScratchBytes = size_t(64) << 20;  // the scratch array below
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mutex;
static_assert(sizeof(scratch) == kScratchBytes, "scratch size");

const KernelTable* table_for(int N) {
  switch (N) {
    case 1: return table_N1();
    case 2: return table_N2();
    case 3: return table_N3();
    case 4: return table_N4();
    case 5: return table_N5();
    case 6: return table_N6();
    case 7: return table_N7();
    default: return nullptr;
  }
}

// Legendre P_n and P_n' at x by the three-term recurrence.
void legendre_pd(int n, double x, double& P, double& dP) {
  double pm1 = 1.0, p = x;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    const double pn = ((2 * k + 1) * x * p - k * pm1) / (k + 1);
    pm1 = p;
    p = pn;
  }
  P = p;
  dP = (std::fabs(x) < 1.0) ? n * (pm1 - x * p) / (1.0 - x * x) : 0.5 * n * (n + 1) * std::pow(x, n + 1);
}

// Packed basis for degree N (see BasisLayout).
std::vector<double> build_basis(int N) {
  const int n1 = N + 1;
  const BasisLayout L(n1);
  std::vector<double> b(L.size(), 0.0);
  std::vector<double> x(n1), w(n1), PN(n1);
  // LGL points: +-1 and the zeros of P_N'; Newton on P_N' using the Legendre
  // ODE for P_N'' = (2x P_N' - N(N+1) P_N)/(1 - x^2), symmetric pairs.
  x[0] = -1.0;
  x[N] = 1.0;
  for (int i = 1; i <= N / 2; ++i) {
    double z = -std::cos(M_PI * i / N);
    for (int it = 0; it < 60; ++it) {
      double P, dP;
      legendre_pd(N, z, P, dP);
      const double d2P = (2.0 * z * dP - N * (N + 1.0) * P) / (1.0 - z * z);
      const double step = dP / d2P;
      z -= step;
      if (std::fabs(step) <= 1e-17) break;
    }
    x[i] = z;
    x[N - i] = -z;
  }
  if (N % 2 == 0) x[N / 2] = 0.0;
  for (int i = 0; i < n1; ++i) {
    double P, dP;
    legendre_pd(N, x[i], P, dP);
    PN[i] = P;
    w[i] = 2.0 / (N * (N + 1.0) * P * P);
  }
  // Lagrange derivative matrix on the LGL points.
  std::vector<double> D(n1 * n1, 0.0);
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j)
      if (i != j) D[i * n1 + j] = PN[i] / (PN[j] * (x[i] - x[j]));
  D[0] = -0.25 * N * (N + 1.0);
  D[N * n1 + N] = 0.25 * N * (N + 1.0);
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      // split form: 2D with the SBP boundary terms removed at the two corners
      double dh = 2.0 * D[i * n1 + j];
      if (i == j && (i == 0 || i == N)) dh = 0.0;
      b[L.Dhat() + i * n1 + j] = dh;
      // strong form with the boundary term folded in: D - W^-1 B
      double dw = D[i * n1 + j];
      if (i == j && i == 0) dw += 1.0 / w[0];
      if (i == j && i == N) dw -= 1.0 / w[N];
      b[L.Dw() + i * n1 + j] = dw;
    }
  for (int i = 0; i < n1; ++i) {
    b[L.winv() + i] = 1.0 / w[i];
    b[L.xi() + i] = x[i];
    b[L.w() + i] = w[i];
  }
  for (int k = 0; k < n1 * n1; ++k) b[L.D() + k] = D[k];
  double s = -1.0;
  b[L.edge()] = -1.0;
  for (int m = 0; m < n1; ++m) {
    s += w[m];
    b[L.edge() + m + 1] = s;
  }
  // Inverse of the orthonormal Legendre Vandermonde V_ij = sqrt(j + 1/2) P_j(x_i)
  // (Gauss-Jordan with partial pivoting).
  std::vector<double> V(n1 * n1), Vi(n1 * n1, 0.0);
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      double P, dP;
      legendre_pd(j, x[i], P, dP);
      V[i * n1 + j] = std::sqrt(j + 0.5) * P;
    }
  for (int i = 0; i < n1; ++i) Vi[i * n1 + i] = 1.0;
  for (int c = 0; c < n1; ++c) {
    int p = c;
    for (int r = c + 1; r < n1; ++r)
      if (std::fabs(V[r * n1 + c]) > std::fabs(V[p * n1 + c])) p = r;
    for (int k = 0; k < n1; ++k) {
      std::swap(V[c * n1 + k], V[p * n1 + k]);
      std::swap(Vi[c * n1 + k], Vi[p * n1 + k]);
    }
    const double piv = V[c * n1 + c];
    for (int k = 0; k < n1; ++k) {
      V[c * n1 + k] /= piv;
      Vi[c * n1 + k] /= piv;
    }
    for (int r = 0; r < n1; ++r) {
      if (r == c) continue;
      const double f = V[r * n1 + c];
      for (int k = 0; k < n1; ++k) {
        V[r * n1 + k] -= f * V[c * n1 + k];
        Vi[r * n1 + k] -= f * Vi[c * n1 + k];
      }
    }
  }
  for (int k = 0; k < n1 * n1; ++k) b[L.Vinv() + k] = Vi[k];
  return b;
}

}  // namespace

struct dg_ctx {
  int N = 0, n1 = 0, nn = 0, nf = 0;
  int ne[3] = {0, 0, 0};
  int nelem = 0, chunk = 0;
  double lo[3], hi[3], dx[3], invJ[3], Jac = 1.0;
  double gamma = 1.4, mu = 0.0;
  dg_options opt;
  hipStream_t stream = nullptr;
  int device = 0;
  const KernelTable* kt = nullptr;
  size_t nstate = 0;  // doubles per state
  int32_t* nbr = nullptr;
  double* basis = nullptr;
  double* G = nullptr;
  double* U2 = nullptr;
  double* alpha1 = nullptr;
  double* alpha1b = nullptr;  // the other of the pair the fused indicator ping-pongs
  double* alpha = nullptr;
  double* Fvf = nullptr;
  double* Fvf2 = nullptr;  // split BR1: the own part of the next stage state (allocated on first use)
  double* cs_field = nullptr;  // per-element Smagorinsky coefficients (dg_set_cs_field)
  int has_cs_field = 0;
  double* M = nullptr;         // curved mesh metrics [nelem][10][nn] (dg_set_geometry), NULL: box
  double* d2e = nullptr;       // curved mesh: squared filter width of the eddy viscosity per element
  int* d_bad = nullptr;        // count of invalid Jacobians (dg_set_geometry)
  int32_t* conn = nullptr;     // general connectivity [nelem][6][3] (dg_set_connectivity), NULL: structured
  int wall_dir = -1;           // wall-modelled faces normal to this direction (dg_set_wall_model), -1: none
  double wm_uinf = 1.0, wm_mainf = 0.0;
  double* partial = nullptr;
  double* h_partial = nullptr;
  // reverse mode (allocated on first use): stage states Y_0..Y_4, the
  // register and state cotangents, and the face buffer of gradient cotangents
  double* Y[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double* Gbar = nullptr;
  double* Ybar = nullptr;
  double* Gbf = nullptr;
  // reverse mode through the blending: U_t^FV - U_t^DG and the cotangent of alpha
  double* Dfd = nullptr;
  double* abar = nullptr;
  // this device's copy of the file-scope scratch (dg_vjp_noalloc), or NULL
  // when its address could not be obtained
  char* scratch = nullptr;
  char err[256] = "";
  // kernel timing (dg_set_profiling)
  int profiling = 0;
  std::vector<hipEvent_t> ev_pool;
  struct Rec { int kind; int a, b; };
  std::vector<Rec> recs;
};

namespace {

int fail(dg_ctx* c, int code, const char* fmt, ...) {
  char* buf = c ? c->err : g_init_error;
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, 256, fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(dg_ctx* c, hipError_t e, const char* where) {
  return fail(c, DG_EHIP, "%s: %s", where, hipGetErrorString(e));
}

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

void release(dg_ctx* c) {
  if (!c) return;
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  c->ev_pool.clear();
  hipFree(c->nbr);
  hipFree(c->basis);
  hipFree(c->G);
  hipFree(c->U2);
  hipFree(c->alpha1);
  hipFree(c->alpha1b);
  hipFree(c->alpha);
  hipFree(c->Fvf);
  hipFree(c->Fvf2);
  hipFree(c->cs_field);
  hipFree(c->M);
  hipFree(c->d2e);
  hipFree(c->d_bad);
  hipFree(c->conn);
  hipFree(c->partial);
  if (c->h_partial) hipHostFree(c->h_partial);
  for (double* y : c->Y) hipFree(y);
  hipFree(c->Gbar);
  hipFree(c->Ybar);
  hipFree(c->Gbf);
  hipFree(c->Dfd);
  hipFree(c->abar);
}

StageArgs stage_args(const dg_ctx* c) {
  StageArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nbr = c->nbr;
  a.basis = c->basis;
  a.alpha1 = c->alpha1;
  a.Fvf = c->Fvf;
  for (int d = 0; d < 3; ++d) a.invJ[d] = c->invJ[d];
  a.gamma = c->gamma;
  a.mu = c->mu;
  a.kappa = c->mu * c->gamma / ((c->gamma - 1.0) * c->opt.Pr);
  a.amin = c->opt.alpha_min;
  a.amax = c->opt.alpha_max;
  a.aspread = c->opt.alpha_spread;
  a.thresh = 0.5 * std::pow(10.0, -1.8 * std::pow(c->N + 1.0, 0.25));
  a.sharp = std::log(9999.0);  // alpha0(E = 0) = 1e-4
  a.nelem = c->nelem;
  a.chunk = c->chunk;
  a.vf = c->opt.vol_flux;
  a.sf = c->opt.surf_flux;
  a.blend = c->opt.blending;
  a.indicator = c->opt.indicator;
  a.recon = c->opt.fv_recon;
  a.cs_elem = c->has_cs_field ? c->cs_field : nullptr;
  a.M = c->M;
  a.conn = c->conn;
  a.delta2_elem = c->d2e;
  a.cs = c->opt.Cs;
  a.wall_dir = c->wall_dir;
  for (int d = 0; d < 3; ++d) a.ne[d] = c->ne[d];
  if (c->wall_dir >= 0) {
    a.wm_h = c->dx[c->wall_dir];
    a.wm_uinf = c->wm_uinf;
    // van Driest: b = sqrt(r / (1 + r)), r = (gamma - 1)/2 Ma^2 Pr^(1/3)
    const double r = 0.5 * (c->gamma - 1.0) * c->wm_mainf * c->wm_mainf * std::cbrt(c->opt.Pr);
    a.wm_b = c->wm_mainf > 0.0 ? std::sqrt(r / (1.0 + r)) : 0.0;
  }
  const double delta = std::cbrt(c->dx[0] * c->dx[1] * c->dx[2]) / (c->N + 1.0);
  a.delta2 = delta * delta;
  a.ktf = c->gamma / ((c->gamma - 1.0) * c->opt.Prt);
  return a;
}

// Kernel variant of the equations: 0 Euler, 1 Navier-Stokes, 2 Navier-Stokes
// with the Smagorinsky eddy viscosity (constant C_s > 0 or a per-element field).
int eq_code(const dg_ctx* c) {
  if (c->opt.equations != DG_NS) return 0;
  return (c->has_cs_field || c->opt.Cs > 0.0) ? 2 : 1;
}

ReduceArgs reduce_args(const dg_ctx* c, const double* X) {
  ReduceArgs r;
  std::memset(&r, 0, sizeof(r));
  r.X = X;
  r.partial = c->partial;
  r.basis = c->basis;
  for (int d = 0; d < 3; ++d) r.invdx[d] = 1.0 / c->dx[d];
  r.gamma = c->gamma;
  r.nu_fac = c->opt.equations == DG_NS ? c->mu * c->gamma / c->opt.Pr : 0.0;
  r.Jac = c->Jac;
  r.nelem = c->nelem;
  r.M = c->M;
  return r;
}

int check_ctx(dg_ctx* c) {
  if (!c || !c->kt) return DG_EINVAL;
  return DG_OK;
}

// Event pair around one launch when profiling; returns the pool index or -1.
int prof_event(dg_ctx* c) {
  const int used = 2 * (int)c->recs.size();
  if ((int)c->ev_pool.size() < used + 2) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      c->ev_pool.push_back(e);
    }
  }
  return used;
}

template <class F>
hipError_t timed(dg_ctx* c, int kind, F&& launch) {
  if (!c->profiling) return launch();
  const int i = prof_event(c);
  if (i < 0) return launch();
  hipEventRecord(c->ev_pool[i], c->stream);
  const hipError_t e = launch();
  hipEventRecord(c->ev_pool[i + 1], c->stream);
  c->recs.push_back({kind, i, i + 1});
  return e;
}

// Split BR1 (see StageArgs.split): used for the FP64 Navier-Stokes operator
// without the eddy viscosity, blending, walls or curved geometry when the
// options ask for it.
bool split_on(const dg_ctx* c) {
  return c->opt.lifting == DG_LIFT_SPLIT && eq_code(c) == 1 && c->opt.precision == DG_FP64 && !c->opt.blending &&
         c->wall_dir < 0 && !c->M && !c->conn;
}

// Chaining of the split lifting through the stages of one Runge-Kutta step:
// CHAIN_IN: c->Fvf already holds the own part of X_in (the previous stage
// wrote it), so no lifting launch; CHAIN_OUT: the stage kernel writes the own
// part of X_out for the next stage.  Ignored unless split_on.
enum { CHAIN_IN = 1, CHAIN_OUT = 2 };

// Chain flags of stage k of a step whose last stage that chains is klast.
int chain_flags(int k, int klast) { return (k > 0 ? CHAIN_IN : 0) | (k < klast ? CHAIN_OUT : 0); }

int ensure_split_buffer(dg_ctx* c) {
  if (!split_on(c) || c->Fvf2) return DG_OK;
  const hipError_t e = hipMalloc((void**)&c->Fvf2, (size_t)c->nelem * 6 * 4 * c->nf * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c->Fvf2 = nullptr;
    return fail(c, (e == hipErrorOutOfMemory) ? DG_ENOMEM : DG_EHIP, "split lifting buffer: %s", hipGetErrorString(e));
  }
  return DG_OK;
}

// One evaluation of the operator on X_in: [indicator], [BR1 lifting], stage.
// alpha1_next (blending, MODE_RK): the stage kernel writes the coefficients of
// X_out there, and the indicator of X_in is taken as already in c->alpha1.
// chain: CHAIN_* flags (split BR1, MODE_RK; needs ensure_split_buffer).
int run_stage(dg_ctx* c, const double* Xin, double* Xout, double* Ut, int mode, double A, double Bdt, int writeG,
              double* alpha_out, double* alpha1_next = nullptr, int chain = 0) {
  StageArgs a = stage_args(c);
  a.U = Xin;
  a.Uout = Xout;
  a.G = c->G;
  a.Ut = Ut;
  a.mode = mode;
  a.A = A;
  a.Bdt = Bdt;
  a.writeG = writeG;
  a.alpha_out = alpha_out;
  a.alpha1_next = alpha1_next;
  hipError_t e;
  if (c->opt.blending && !alpha1_next) {
    e = timed(c, DG_K_INDICATOR, [&] { return c->kt->alpha1(a, c->stream); });
    if (e != hipSuccess) return hip_fail(c, e, "indicator kernel");
  }
  const int eq = eq_code(c);
  if (c->conn && !c->M)
    return fail(c, DG_ESTATE, "general connectivity needs curved elements: call dg_set_geometry first");
  if (c->wall_dir >= 0 && (eq == 0 || c->opt.precision != DG_FP64 || c->M))
    return fail(c, DG_ESTATE, "wall-modelled boundaries need the FP64 Navier-Stokes operator on the box");
  if (c->M) {  // curved mesh (FP64, no blending: checked when set)
    if (eq >= 1) {
      e = timed(c, DG_K_LIFT, [&] { return c->kt->lift_curved(a, eq, c->stream); });
      if (e != hipSuccess) return hip_fail(c, e, "lifting kernel (curved)");
    }
    e = timed(c, DG_K_STAGE, [&] { return c->kt->stage_curved(a, eq, c->stream); });
    if (e != hipSuccess) return hip_fail(c, e, "stage kernel (curved)");
    return DG_OK;
  }
  const bool mixed = c->opt.precision == DG_MIXED;
  const bool split = split_on(c);
  if (!split || mode != MODE_RK) chain = 0;
  if (split) {
    a.split = 1;
    if ((chain & CHAIN_OUT) && !c->Fvf2) return fail(c, DG_ESTATE, "split lifting buffer missing");
    a.Fvf_next = (chain & CHAIN_OUT) ? c->Fvf2 : nullptr;
  }
  if (eq >= 1 && !(chain & CHAIN_IN)) {
    e = timed(c, DG_K_LIFT,
              [&] { return mixed ? c->kt->lift_mixed(a, eq, c->stream) : c->kt->lift(a, eq, c->stream); });
    if (e != hipSuccess) return hip_fail(c, e, "lifting kernel");
  }
  if (c->wall_dir >= 0) {  // FP64 Navier-Stokes (checked above)
    e = timed(c, DG_K_LIFT, [&] { return c->kt->wall_flux(a, c->stream); });
    if (e != hipSuccess) return hip_fail(c, e, "wall-model kernel");
  }
  e = timed(c, DG_K_STAGE,
            [&] { return mixed ? c->kt->stage_mixed(a, eq, c->stream) : c->kt->stage(a, eq, c->stream); });
  if (e != hipSuccess) return hip_fail(c, e, "stage kernel");
  if (a.Fvf_next) std::swap(c->Fvf, c->Fvf2);  // the own part of X_out is now c->Fvf
  return DG_OK;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Options a curved mesh supports: the FP64 operator with the KG, PI or STD
// volume flux, Euler or Navier-Stokes (also with the eddy viscosity), no
// blending.
int curved_compatible(dg_ctx* c, const dg_options* o, int cs_field, const char* where) {
  (void)cs_field;
  if (o->blending) return fail(c, DG_EUNSUPPORTED, "%s: no blending on curved meshes", where);
  if (o->precision != DG_FP64) return fail(c, DG_EUNSUPPORTED, "%s: curved meshes use the FP64 operator", where);
  if (o->vol_flux == DG_VF_CH) return fail(c, DG_EUNSUPPORTED, "%s: curved meshes: KG, PI or STD flux", where);
  return DG_OK;
}

// Options wall-modelled boundaries support: the FP64 Navier-Stokes operator
// (with or without eddy viscosity), no blending, on the Cartesian box.
int wall_compatible(dg_ctx* c, const dg_options* o, const char* where) {
  if (o->equations != DG_NS) return fail(c, DG_EUNSUPPORTED, "%s: walls need the Navier-Stokes equations", where);
  if (o->precision != DG_FP64) return fail(c, DG_EUNSUPPORTED, "%s: walls use the FP64 operator", where);
  if (c->M || c->conn) return fail(c, DG_EUNSUPPORTED, "%s: walls are built for the Cartesian box", where);
  return DG_OK;
}

int vjp_supported(dg_ctx* c) {
  if (c->conn && !c->M)
    return fail(c, DG_ESTATE, "general connectivity needs curved elements: call dg_set_geometry first");
  if (c->opt.precision != DG_FP64) return fail(c, DG_EUNSUPPORTED, "vjp: FP64 operator only");
  if (c->opt.vol_flux == DG_VF_CH) return fail(c, DG_EUNSUPPORTED, "vjp: not available for the CH flux");
  return DG_OK;
}

// Reverse-mode scratch, allocated on first use (stages: the five stage states
// that rk_step_vjp recomputes).
int ensure_reverse_buffers(dg_ctx* c, bool rk, bool stages = true) {
  hipError_t e = hipSuccess;
  const size_t bytes = c->nstate * sizeof(double);
  if (!c->Gbf) e = hipMalloc((void**)&c->Gbf, (size_t)c->nelem * 6 * 4 * c->nf * sizeof(double));
  if (e == hipSuccess && c->opt.blending && !c->Dfd) e = hipMalloc((void**)&c->Dfd, bytes);
  if (e == hipSuccess && c->opt.blending && !c->abar) e = hipMalloc((void**)&c->abar, (size_t)c->nelem * sizeof(double));
  if (rk) {
    for (int k = 0; k < 5 && e == hipSuccess && stages; ++k)
      if (!c->Y[k]) e = hipMalloc((void**)&c->Y[k], bytes);
    if (e == hipSuccess && !c->Gbar) e = hipMalloc((void**)&c->Gbar, bytes);
    if (e == hipSuccess && !c->Ybar) e = hipMalloc((void**)&c->Ybar, bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, (e == hipErrorOutOfMemory) ? DG_ENOMEM : DG_EHIP, "reverse-mode buffers: %s", hipGetErrorString(e));
  }
  return DG_OK;
}

// U_bar = [Uacc +] (dL/dU)^T lambda on the context's stream, with the given
// reverse-mode buffers: the face buffer of gradient cotangents Gbf
// (Navier-Stokes), and with blending U_t^FV - U_t^DG (Dfd) and the cotangent
// of alpha (abar).  Every entry of them is written before it is read.
int run_vjp_buffers(dg_ctx* c, const double* U, const double* lambda, double* U_bar, const double* Uacc,
                    double* Gbf, double* Dfd, double* abar) {
  int rc = 0;
  VjpArgs v;
  std::memset(&v, 0, sizeof(v));
  v.U = U;
  v.Lbar = lambda;
  v.Ubar = U_bar;
  v.Uacc = Uacc;
  v.nbr = c->nbr;
  v.basis = c->basis;
  v.Gbf = Gbf;
  for (int d = 0; d < 3; ++d) v.invJ[d] = c->invJ[d];
  v.gamma = c->gamma;
  v.mu = c->mu;
  v.kappa = c->mu * c->gamma / ((c->gamma - 1.0) * c->opt.Pr);
  v.nelem = c->nelem;
  v.chunk = c->chunk;
  v.vf = c->opt.vol_flux;
  v.sf = c->opt.surf_flux;
  v.M = c->M;
  v.conn = c->conn;
  {
    const StageArgs a = stage_args(c);
    v.les = eq_code(c) == 2;
    v.cs_elem = a.cs_elem;
    v.cs = a.cs;
    v.delta2 = a.delta2;
    v.ktf = a.ktf;
    v.wall_dir = a.wall_dir;
    v.wm_h = a.wm_h;
    v.wm_uinf = a.wm_uinf;
    v.wm_b = a.wm_b;
    v.delta2_elem = a.delta2_elem;
  }
  hipError_t e;
  if (c->M) {  // curved mesh (FP64, no blending: checked when set)
    if (c->opt.equations == DG_NS) {
      e = timed(c, DG_K_VJP_LIFT, [&] { return c->kt->vjp_lift_curved(v, c->stream); });
      if (e != hipSuccess) return hip_fail(c, e, "vjp lifting kernel (curved)");
    }
    e = timed(c, DG_K_VJP, [&] { return c->kt->vjp_curved(v, eq_code(c), c->stream); });
    if (e != hipSuccess) return hip_fail(c, e, "vjp kernel (curved)");
    return DG_OK;
  }
  if (c->opt.blending) {
    // forward at U: blending coefficients and U_t^FV - U_t^DG
    if ((rc = run_stage(c, U, nullptr, Dfd, MODE_DIFF, 0.0, 0.0, 0, c->alpha))) return rc;
    const StageArgs a = stage_args(c);
    v.alpha = c->alpha;
    v.alpha1 = c->alpha1;
    v.Dfd = Dfd;
    v.abar = abar;
    v.amin = a.amin;
    v.amax = a.amax;
    v.aspread = a.aspread;
    v.thresh = a.thresh;
    v.sharp = a.sharp;
    v.indicator = a.indicator;
    v.recon = a.recon;
    e = timed(c, DG_K_VJP, [&] { return c->kt->vjp_alpha_bar(v, c->stream); });
    if (e != hipSuccess) return hip_fail(c, e, "vjp blending-coefficient kernel");
    e = timed(c, DG_K_VJP, [&] { return c->kt->vjp_alpha(v, c->stream); });  // U_bar = [Uacc +] alpha part
    if (e != hipSuccess) return hip_fail(c, e, "vjp blending-coefficient kernel");
    e = timed(c, DG_K_VJP, [&] { return c->kt->vjp_fv(v, c->stream); });  // U_bar += FV part
    if (e != hipSuccess) return hip_fail(c, e, "vjp FV subcell kernel");
    v.Uacc = U_bar;  // the DG part accumulates on top
  }
  if (c->opt.equations == DG_NS) {
    e = timed(c, DG_K_VJP_LIFT, [&] { return c->kt->vjp_lift(v, c->stream); });
    if (e != hipSuccess) return hip_fail(c, e, "vjp lifting kernel");
  }
  e = timed(c, DG_K_VJP, [&] { return c->kt->vjp(v, eq_code(c), c->stream); });
  if (e != hipSuccess) return hip_fail(c, e, "vjp kernel");
  return DG_OK;
}

// U_bar = [Uacc +] (dL/dU)^T lambda with the context's reverse-mode buffers
// (allocated on first use).
int run_vjp(dg_ctx* c, const double* U, const double* lambda, double* U_bar, const double* Uacc) {
  const int rc = ensure_reverse_buffers(c, false);
  if (rc) return rc;
  return run_vjp_buffers(c, U, lambda, U_bar, Uacc, c->Gbf, c->Dfd, c->abar);
}

// Structured periodic neighbour table of the context's mesh.
std::vector<int32_t> structured_nbr(const dg_ctx* c) {
  std::vector<int32_t> nbr((size_t)c->nelem * 6);
  const int nx = c->ne[0], ny = c->ne[1], nz = c->ne[2];
  for (int ez = 0; ez < nz; ++ez)
    for (int ey = 0; ey < ny; ++ey)
      for (int ex = 0; ex < nx; ++ex) {
        const size_t e = ex + (size_t)nx * (ey + (size_t)ny * ez);
        nbr[6 * e + 0] = ((ex + nx - 1) % nx) + nx * (ey + ny * ez);
        nbr[6 * e + 1] = ((ex + 1) % nx) + nx * (ey + ny * ez);
        nbr[6 * e + 2] = ex + nx * (((ey + ny - 1) % ny) + ny * ez);
        nbr[6 * e + 3] = ex + nx * (((ey + 1) % ny) + ny * ez);
        nbr[6 * e + 4] = ex + nx * (ey + ny * ((ez + nz - 1) % nz));
        nbr[6 * e + 5] = ex + nx * (ey + ny * ((ez + 1) % nz));
      }
  return nbr;
}

// Neighbour table of the box: periodic, with -1 on the wall faces normal to
// the context's wall direction.
std::vector<int32_t> box_nbr(const dg_ctx* c, int wall_dir) {
  std::vector<int32_t> nbr = structured_nbr(c);
  if (wall_dir < 0) return nbr;
  const int nx = c->ne[0], ny = c->ne[1];
  for (size_t e = 0; e < (size_t)c->nelem; ++e) {
    const int ix[3] = {(int)(e % nx), (int)((e / nx) % ny), (int)(e / ((size_t)nx * ny))};
    if (ix[wall_dir] == 0) nbr[6 * e + 2 * wall_dir] = -1;
    if (ix[wall_dir] == c->ne[wall_dir] - 1) nbr[6 * e + 2 * wall_dir + 1] = -1;
  }
  return nbr;
}

// New device neighbour table (and connectivity) filled on the context's
// stream behind its queued work, swapped in only when complete, so that a
// failure leaves the context unchanged.
int swap_tables(dg_ctx* c, const std::vector<int32_t>& nbr, const int32_t* conn, const char* where) {
  int32_t *dnbr = nullptr, *dconn = nullptr;
  const size_t cbytes = (size_t)c->nelem * 18 * sizeof(int32_t);
  hipError_t e = hipMalloc((void**)&dnbr, nbr.size() * sizeof(int32_t));
  if (e == hipSuccess && conn) e = hipMalloc((void**)&dconn, cbytes);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dnbr, nbr.data(), nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && conn) e = hipMemcpyAsync(dconn, conn, cbytes, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // the host arrays are the caller's
  if (e != hipSuccess) {
    (void)hipGetLastError();
    hipFree(dnbr);
    hipFree(dconn);
    return fail(c, (e == hipErrorOutOfMemory) ? DG_ENOMEM : DG_EHIP, "%s: %s", where, hipGetErrorString(e));
  }
  hipFree(c->nbr);
  c->nbr = dnbr;
  hipFree(c->conn);
  c->conn = dconn;
  return DG_OK;
}

// Face-local index a mapped by orientation code o (bit 0 swap, bit 1 reverse
// the first, bit 2 the second index).
int orient_face_index(int N, int o, int a) {
  const int n1 = N + 1, t1 = a % n1, t2 = a / n1;
  int u = (o & 1) ? t2 : t1, v = (o & 1) ? t1 : t2;
  if (o & 2) u = N - u;
  if (o & 4) v = N - v;
  return u + n1 * v;
}

}  // namespace

extern "C" {

void dg_default_options(dg_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->equations = DG_EULER;
  o->vol_flux = DG_VF_KG;
  o->surf_flux = DG_SF_LLF;
  o->blending = 0;
  o->indicator = DG_IND_HENNEMANN;
  o->fv_recon = DG_FV_MINMOD;
  o->precision = DG_FP64;
  o->lifting = DG_LIFT_SPLIT;
  o->Pr = 0.72;
  o->alpha_min = 0.01;
  o->alpha_max = 0.7;
  o->alpha_spread = 0.5;
  o->Cs = 0.0;
  o->Prt = 0.9;
}

int dg_init(const dg_mesh* mesh, int N, double gamma, double mu, dg_ctx** out) {
  if (!out) return fail(nullptr, DG_EINVAL, "dg_init: out is NULL");
  *out = nullptr;
  if (!mesh) return fail(nullptr, DG_EINVAL, "dg_init: mesh is NULL");
  if (N < 1 || N > 7) return fail(nullptr, DG_EINVAL, "dg_init: N = %d outside 1..7", N);
  if (!(gamma > 1.0) || !std::isfinite(gamma)) return fail(nullptr, DG_EINVAL, "dg_init: gamma must be > 1");
  if (!(mu >= 0.0) || !std::isfinite(mu)) return fail(nullptr, DG_EINVAL, "dg_init: mu must be >= 0");
  long long ne = 1;
  for (int d = 0; d < 3; ++d) {
    if (mesh->nelem[d] < 1) return fail(nullptr, DG_EINVAL, "dg_init: nelem[%d] < 1", d);
    if (!(mesh->hi[d] > mesh->lo[d]) || !std::isfinite(mesh->hi[d] - mesh->lo[d]))
      return fail(nullptr, DG_EINVAL, "dg_init: hi[%d] must exceed lo[%d]", d, d);
    ne *= mesh->nelem[d];
  }
  if (ne > (1LL << 28)) return fail(nullptr, DG_EINVAL, "dg_init: too many elements");
  dg_ctx* c = new (std::nothrow) dg_ctx();
  if (!c) return fail(nullptr, DG_ENOMEM, "dg_init: host allocation failed");
  c->N = N;
  c->n1 = N + 1;
  c->nn = c->n1 * c->n1 * c->n1;
  c->nf = c->n1 * c->n1;
  c->nelem = (int)ne;
  c->chunk = (c->nelem + 7) / 8;
  c->gamma = gamma;
  c->mu = mu;
  c->kt = table_for(N);
  dg_default_options(&c->opt);
  for (int d = 0; d < 3; ++d) {
    c->ne[d] = mesh->nelem[d];
    c->lo[d] = mesh->lo[d];
    c->hi[d] = mesh->hi[d];
    c->dx[d] = (mesh->hi[d] - mesh->lo[d]) / mesh->nelem[d];
    c->invJ[d] = 2.0 / c->dx[d];
    c->Jac *= 0.5 * c->dx[d];
  }
  hipGetDevice(&c->device);
  c->nstate = (size_t)c->nelem * 5 * c->nn;
  const std::vector<double> basis = build_basis(N);
  std::vector<int32_t> nbr((size_t)c->nelem * 6);
  const int nx = c->ne[0], ny = c->ne[1], nz = c->ne[2];
  for (int ez = 0; ez < nz; ++ez)
    for (int ey = 0; ey < ny; ++ey)
      for (int ex = 0; ex < nx; ++ex) {
        const size_t e = ex + (size_t)nx * (ey + (size_t)ny * ez);
        nbr[6 * e + 0] = ((ex + nx - 1) % nx) + nx * (ey + ny * ez);
        nbr[6 * e + 1] = ((ex + 1) % nx) + nx * (ey + ny * ez);
        nbr[6 * e + 2] = ex + nx * (((ey + ny - 1) % ny) + ny * ez);
        nbr[6 * e + 3] = ex + nx * (((ey + 1) % ny) + ny * ez);
        nbr[6 * e + 4] = ex + nx * (ey + ny * ((ez + nz - 1) % nz));
        nbr[6 * e + 5] = ex + nx * (ey + ny * ((ez + 1) % nz));
      }
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  alloc((void**)&c->nbr, nbr.size() * sizeof(int32_t));
  alloc((void**)&c->basis, basis.size() * sizeof(double));
  alloc((void**)&c->G, c->nstate * sizeof(double));
  alloc((void**)&c->U2, c->nstate * sizeof(double));
  alloc((void**)&c->alpha1, (size_t)c->nelem * sizeof(double));
  alloc((void**)&c->alpha1b, (size_t)c->nelem * sizeof(double));
  alloc((void**)&c->alpha, (size_t)c->nelem * sizeof(double));
  alloc((void**)&c->Fvf, (size_t)c->nelem * 6 * 4 * c->nf * sizeof(double));
  alloc((void**)&c->partial, kRedBlocks * 5 * sizeof(double));
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_partial, kRedBlocks * 5 * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemcpy(c->nbr, nbr.data(), nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->basis, basis.data(), basis.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->alpha1, 0, (size_t)c->nelem * sizeof(double));
  if (e != hipSuccess) {
    const bool oom = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation);
    fail(nullptr, oom ? DG_ENOMEM : DG_EHIP, "dg_init: %s", hipGetErrorString(e));
    (void)hipGetLastError();
    release(c);
    delete c;
    return oom ? DG_ENOMEM : DG_EHIP;
  }
  if (c->device >= 0 && c->device < kMaxDevices) {  // with the device current (dg_init's)
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[c->device]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch[c->device] = p;
      else (void)hipGetLastError();
    }
    c->scratch = static_cast<char*>(g_scratch[c->device]);
  }
  *out = c;
  return DG_OK;
}

int dg_set_options(dg_ctx* c, const dg_options* o) {
  if (check_ctx(c) || !o) return fail(c, DG_EINVAL, "dg_set_options: NULL argument");
  if (o->equations < 0 || o->equations > 1) return fail(c, DG_EINVAL, "dg_set_options: equations");
  if (o->vol_flux < 0 || o->vol_flux > 3) return fail(c, DG_EINVAL, "dg_set_options: vol_flux");
  if (o->surf_flux < 0 || o->surf_flux > 2) return fail(c, DG_EINVAL, "dg_set_options: surf_flux");
  if (o->indicator < 0 || o->indicator > 1) return fail(c, DG_EINVAL, "dg_set_options: indicator");
  if (o->fv_recon < 0 || o->fv_recon > 1) return fail(c, DG_EINVAL, "dg_set_options: fv_recon");
  if (o->precision < 0 || o->precision > 1) return fail(c, DG_EINVAL, "dg_set_options: precision");
  if (o->lifting < 0 || o->lifting > 1) return fail(c, DG_EINVAL, "dg_set_options: lifting");
  if (!finite_pos(o->Pr)) return fail(c, DG_EINVAL, "dg_set_options: Pr must be > 0");
  if (!(o->alpha_min >= 0.0 && o->alpha_min <= o->alpha_max && o->alpha_max <= 1.0) ||
      !(o->alpha_spread >= 0.0 && o->alpha_spread <= 1.0))
    return fail(c, DG_EINVAL, "dg_set_options: need 0 <= alpha_min <= alpha_max <= 1, 0 <= spread <= 1");
  if (o->blending && c->N < 2) return fail(c, DG_EUNSUPPORTED, "dg_set_options: blending needs N >= 2");
  if (o->precision == DG_MIXED && !c->kt->stage_mixed)
    return fail(c, DG_EUNSUPPORTED, "dg_set_options: mixed precision not built for this degree");
  if (o->precision == DG_MIXED && o->blending)
    return fail(c, DG_EUNSUPPORTED, "dg_set_options: mixed precision without blending only");
  if (o->precision == DG_MIXED && o->vol_flux != DG_VF_PI && o->vol_flux != DG_VF_STD)
    return fail(c, DG_EUNSUPPORTED, "dg_set_options: mixed precision needs the PI or STD volume flux");
  if (!(o->Cs >= 0.0) || !std::isfinite(o->Cs) || !finite_pos(o->Prt))
    return fail(c, DG_EINVAL, "dg_set_options: need Cs >= 0 and Prt > 0");
  if ((o->Cs > 0.0 || c->has_cs_field) && o->equations == DG_NS && o->vol_flux == DG_VF_CH)
    return fail(c, DG_EUNSUPPORTED, "dg_set_options: the Smagorinsky model is built for the KG, PI and STD fluxes");
  if (c->M) {
    const int rc = curved_compatible(c, o, c->has_cs_field, "dg_set_options");
    if (rc) return rc;
  }
  if (c->wall_dir >= 0) {
    const int rc = wall_compatible(c, o, "dg_set_options");
    if (rc) return rc;
  }
  c->opt = *o;
  return DG_OK;
}

int dg_set_connectivity(dg_ctx* c, const int32_t* conn) {
  if (check_ctx(c)) return DG_EINVAL;
  std::vector<int32_t> nbr;
  if (!conn) {
    nbr = box_nbr(c, c->wall_dir);
  } else {
    if (c->wall_dir >= 0)
      return fail(c, DG_EUNSUPPORTED, "dg_set_connectivity: walls are built for the Cartesian box");
    // every face must name an existing neighbour face that names it back,
    // with the inverse orientation
    const int ne = c->nelem;
    for (int e = 0; e < ne; ++e)
      for (int f = 0; f < 6; ++f) {
        const int32_t* q = conn + ((size_t)e * 6 + f) * 3;
        if (q[0] < 0 || q[0] >= ne || q[1] < 0 || q[1] > 5 || q[2] < 0 || q[2] > 7)
          return fail(c, DG_EINVAL, "dg_set_connectivity: element %d face %d out of range", e, f);
        const int32_t* r = conn + ((size_t)q[0] * 6 + q[1]) * 3;
        if (r[0] != e || r[1] != f)
          return fail(c, DG_EINVAL, "dg_set_connectivity: element %d face %d is not named back", e, f);
        for (int a = 0; a < c->nf; ++a)
          if (orient_face_index(c->N, r[2], orient_face_index(c->N, q[2], a)) != a)
            return fail(c, DG_EINVAL, "dg_set_connectivity: orientations of element %d face %d do not match", e,
                        f);
      }
    nbr.resize((size_t)ne * 6);
    for (size_t k = 0; k < nbr.size(); ++k) nbr[k] = conn[3 * k];
  }
  // the neighbour table (used by the indicator spread and the structured
  // kernels) follows the connectivity
  return swap_tables(c, nbr, conn, "dg_set_connectivity");
}

int dg_set_wall_model(dg_ctx* c, int wall_dir, double u_inf, double ma_inf) {
  if (check_ctx(c)) return DG_EINVAL;
  if (wall_dir < -1 || wall_dir > 2) return fail(c, DG_EINVAL, "dg_set_wall_model: wall_dir must be -1, 0, 1 or 2");
  if (wall_dir >= 0) {
    if (!(ma_inf >= 0.0) || !std::isfinite(ma_inf))
      return fail(c, DG_EINVAL, "dg_set_wall_model: need a finite ma_inf >= 0");
    if (ma_inf > 0.0 && !finite_pos(u_inf))
      return fail(c, DG_EINVAL, "dg_set_wall_model: the van Driest transformation needs u_inf > 0");
    if (!(c->mu > 0.0)) return fail(c, DG_EUNSUPPORTED, "dg_set_wall_model: the wall model needs mu > 0");
    const int rc = wall_compatible(c, &c->opt, "dg_set_wall_model");
    if (rc) return rc;
  } else if (c->wall_dir < 0) {
    return DG_OK;  // no walls to remove (and any general connectivity stays)
  }
  const int rc = swap_tables(c, box_nbr(c, wall_dir), nullptr, "dg_set_wall_model");
  if (rc) return rc;
  c->wall_dir = wall_dir;
  c->wm_uinf = wall_dir >= 0 && ma_inf > 0.0 ? u_inf : 1.0;
  c->wm_mainf = wall_dir >= 0 ? ma_inf : 0.0;
  return DG_OK;
}

int dg_set_geometry(dg_ctx* c, const double* X) {
  if (check_ctx(c)) return DG_EINVAL;
  if (!X) {
    hipFree(c->M);
    c->M = nullptr;
    hipFree(c->d2e);
    c->d2e = nullptr;
    return DG_OK;
  }
  if (!is_device_ptr(X)) return fail(c, DG_EINVAL, "dg_set_geometry: X must be a device pointer");
  if (c->wall_dir >= 0) return fail(c, DG_EUNSUPPORTED, "dg_set_geometry: walls are built for the Cartesian box");
  const int rc = curved_compatible(c, &c->opt, c->has_cs_field, "dg_set_geometry");
  if (rc) return rc;
  // metric terms into a new array, swapped in only when complete and valid:
  // a failure leaves the context's geometry unchanged
  double *M = nullptr, *d2 = nullptr;
  hipError_t e = hipMalloc((void**)&M, (size_t)c->nelem * 10 * c->nn * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&d2, (size_t)c->nelem * sizeof(double));
  if (e == hipSuccess && !c->d_bad) e = hipMalloc((void**)&c->d_bad, sizeof(int));
  int bad = 0;
  if (e == hipSuccess) e = hipMemsetAsync(c->d_bad, 0, sizeof(int), c->stream);
  if (e == hipSuccess) e = c->kt->metrics(X, c->basis, M, c->d_bad, d2, c->nelem, c->chunk, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, c->d_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    hipFree(M);
    hipFree(d2);
    return fail(c, (e == hipErrorOutOfMemory) ? DG_ENOMEM : DG_EHIP, "dg_set_geometry: %s", hipGetErrorString(e));
  }
  if (bad) {
    hipFree(M);
    hipFree(d2);
    return fail(c, DG_EINVAL, "dg_set_geometry: %d nodes with a non-positive or non-finite Jacobian", bad);
  }
  hipFree(c->M);
  c->M = M;
  hipFree(c->d2e);
  c->d2e = d2;
  return DG_OK;
}

int dg_set_cs_field(dg_ctx* c, const double* cs) {
  if (check_ctx(c)) return DG_EINVAL;
  if (!cs) {
    c->has_cs_field = 0;
    return DG_OK;
  }
  if (!is_device_ptr(cs)) return fail(c, DG_EINVAL, "dg_set_cs_field: cs must be a device pointer");
  if (c->opt.vol_flux == DG_VF_CH)
    return fail(c, DG_EUNSUPPORTED, "dg_set_cs_field: the Smagorinsky model is built for the KG, PI and STD fluxes");
  hipError_t e = hipSuccess;
  if (!c->cs_field) e = hipMalloc((void**)&c->cs_field, (size_t)c->nelem * sizeof(double));
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->cs_field, cs, (size_t)c->nelem * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, (e == hipErrorOutOfMemory) ? DG_ENOMEM : DG_EHIP, "dg_set_cs_field: %s", hipGetErrorString(e));
  }
  c->has_cs_field = 1;
  return DG_OK;
}

int dg_get_options(const dg_ctx* c, dg_options* o) {
  if (!c || !o) return DG_EINVAL;
  *o = c->opt;
  return DG_OK;
}

int dg_set_stream(dg_ctx* c, void* s) {
  if (check_ctx(c)) return DG_EINVAL;
  c->stream = (hipStream_t)s;
  return DG_OK;
}

int dg_time_derivative(dg_ctx* c, const double* U, double* Ut) {
  if (check_ctx(c)) return DG_EINVAL;
  if (!is_device_ptr(U) || !is_device_ptr(Ut))
    return fail(c, DG_EINVAL, "dg_time_derivative: U and Ut must be device pointers");
  if ((const void*)U == (const void*)Ut) return fail(c, DG_EINVAL, "dg_time_derivative: Ut aliases U");
  return run_stage(c, U, nullptr, Ut, MODE_UT, 0.0, 0.0, 0, nullptr);
}

int dg_rk_steps(dg_ctx* c, double* U, double dt, int nsteps) {
  if (check_ctx(c)) return DG_EINVAL;
  if (!is_device_ptr(U)) return fail(c, DG_EINVAL, "rk_step: U must be a device pointer");
  if (!finite_pos(dt)) return fail(c, DG_EINVAL, "rk_step: dt must be finite and > 0");
  if (nsteps < 0) return fail(c, DG_EINVAL, "rk_step: nsteps < 0");
  if (const int rc = ensure_split_buffer(c)) return rc;
  double* cur = U;
  // blended Euler operator: the indicator of the start state once, then each
  // stage kernel writes that of its output for the next stage (alpha1 /
  // alpha1b ping-pong); Navier-Stokes keeps the separate indicator launch
  const bool fuse = c->opt.blending && c->opt.equations == DG_EULER && c->kt->fused_alpha1 && nsteps > 0;
  if (fuse) {
    StageArgs a = stage_args(c);
    a.U = U;
    const hipError_t e = timed(c, DG_K_INDICATOR, [&] { return c->kt->alpha1(a, c->stream); });
    if (e != hipSuccess) return hip_fail(c, e, "indicator kernel");
  }
  for (int s = 0; s < nsteps; ++s)
    for (int k = 0; k < 5; ++k) {
      double* nxt = (cur == U) ? c->U2 : U;
      const int writeG = (k < 4) ? 1 : 0;  // the last stage's register is never read again
      // every step starts from a lifting of its start state, so that n steps
      // in one call and n calls of one step agree bitwise
      const int rc = run_stage(c, cur, nxt, nullptr, MODE_RK, kA[k], kB[k] * dt, writeG, nullptr,
                               fuse ? c->alpha1b : nullptr, chain_flags(k, 4));
      if (rc) return rc;
      if (fuse) std::swap(c->alpha1, c->alpha1b);
      cur = nxt;
    }
  if (cur != U) {
    hipError_t e = hipMemcpyAsync(U, cur, c->nstate * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "rk_step copy");
  }
  return DG_OK;
}

int rk_step(dg_ctx* c, double* U, double dt) { return dg_rk_steps(c, U, dt, 1); }

int dg_vjp(dg_ctx* c, const double* U, const double* Ut_bar, double* U_bar) {
  if (check_ctx(c)) return DG_EINVAL;
  if (!is_device_ptr(U) || !is_device_ptr(Ut_bar) || !is_device_ptr(U_bar))
    return fail(c, DG_EINVAL, "dg_vjp: device pointers required");
  if ((const void*)U_bar == (const void*)U || (const void*)U_bar == (const void*)Ut_bar)
    return fail(c, DG_EINVAL, "dg_vjp: U_bar must not alias U or Ut_bar");
  int rc = vjp_supported(c);
  if (rc) return rc;
  return run_vjp(c, U, Ut_bar, U_bar, nullptr);
}

int dg_vjp_noalloc(dg_ctx* c, const double* U, const double* Ut_bar, double* U_bar) {
  if (check_ctx(c)) return DG_EINVAL;
  if (!is_device_ptr(U) || !is_device_ptr(Ut_bar) || !is_device_ptr(U_bar))
    return fail(c, DG_EINVAL, "dg_vjp_noalloc: device pointers required");
  if ((const void*)U_bar == (const void*)U || (const void*)U_bar == (const void*)Ut_bar)
    return fail(c, DG_EINVAL, "dg_vjp_noalloc: U_bar must not alias U or Ut_bar");
  int rc = vjp_supported(c);
  if (rc) return rc;
  if (!c->scratch) return fail(c, DG_EHIP, "dg_vjp_noalloc: no device scratch on this device");
  // the reverse-mode buffers carved from the scratch, 256-byte aligned
  auto round = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t b_gbf = c->opt.equations == DG_NS ? round((size_t)c->nelem * 6 * 4 * c->nf * sizeof(double)) : 0;
  const size_t b_dfd = c->opt.blending ? round(c->nstate * sizeof(double)) : 0;
  const size_t b_abar = c->opt.blending ? round((size_t)c->nelem * sizeof(double)) : 0;
  if (b_gbf + b_dfd + b_abar > kScratchBytes)
    return fail(c, DG_EINVAL, "dg_vjp_noalloc: the mesh needs %zu bytes of scratch, at most %zu are available",
                b_gbf + b_dfd + b_abar, kScratchBytes);
  char* p = c->scratch;
  double* Gbf = b_gbf ? reinterpret_cast<double*>(p) : nullptr;
  double* Dfd = b_dfd ? reinterpret_cast<double*>(p + b_gbf) : nullptr;
  double* abar = b_abar ? reinterpret_cast<double*>(p + b_gbf + b_dfd) : nullptr;
  return run_vjp_buffers(c, U, Ut_bar, U_bar, nullptr, Gbf, Dfd, abar);
}

}  // extern "C"

namespace {

bool overlaps(const double* a, size_t na, const double* b, size_t nb) { return a < b + nb && b < a + na; }

// Reverse 2N-storage recurrence over the stage states Ys[0..4] of one step:
//   Gbar <- A_{k+1} Gbar + B_k dt Ybar,  Ybar <- Ybar + VJP(Y_k, Gbar), k = 4..0.
int rk_reverse(dg_ctx* c, const double* const Ys[5], double dt, const double* U_bar_np1, double* U_bar_n,
               const char* where) {
  const size_t bytes = c->nstate * sizeof(double);
  hipError_t e = hipMemcpyAsync(c->Ybar, U_bar_np1, bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, where);
  for (int k = 4; k >= 0; --k) {
    const double a = (k == 4) ? 0.0 : kA[k + 1];
    e = c->kt->axpby(c->Gbar, a, c->Ybar, kB[k] * dt, c->nstate, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, where);
    const int rc = run_vjp(c, Ys[k], c->Gbar, c->Ybar, c->Ybar);
    if (rc) return rc;
  }
  e = hipMemcpyAsync(U_bar_n, c->Ybar, bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, where);
  return DG_OK;
}

}  // namespace

extern "C" {

int rk_step_record(dg_ctx* c, double* U, double dt, double* Y) {
  if (check_ctx(c)) return DG_EINVAL;
  if (!is_device_ptr(U) || !is_device_ptr(Y)) return fail(c, DG_EINVAL, "rk_step_record: device pointers required");
  if (!finite_pos(dt)) return fail(c, DG_EINVAL, "rk_step_record: dt must be finite and > 0");
  const size_t n = c->nstate;
  if (overlaps(U, n, Y, 5 * n)) return fail(c, DG_EINVAL, "rk_step_record: Y overlaps U");
  if (const int rc = ensure_split_buffer(c)) return rc;
  hipError_t e = hipMemcpyAsync(Y, U, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "rk_step_record copy");
  for (int k = 0; k < 4; ++k) {
    const int rc = run_stage(c, Y + k * n, Y + (k + 1) * n, nullptr, MODE_RK, kA[k], kB[k] * dt, 1, nullptr, nullptr,
                             chain_flags(k, 4));
    if (rc) return rc;
  }
  return run_stage(c, Y + 4 * n, U, nullptr, MODE_RK, kA[4], kB[4] * dt, 0, nullptr, nullptr, chain_flags(4, 4));
}

int rk_step_vjp_recorded(dg_ctx* c, const double* Y, double dt, const double* U_bar_np1, double* U_bar_n) {
  if (check_ctx(c)) return DG_EINVAL;
  if (!is_device_ptr(Y) || !is_device_ptr(U_bar_np1) || !is_device_ptr(U_bar_n))
    return fail(c, DG_EINVAL, "rk_step_vjp_recorded: device pointers required");
  if (!finite_pos(dt)) return fail(c, DG_EINVAL, "rk_step_vjp_recorded: dt must be finite and > 0");
  const size_t n = c->nstate;
  if (overlaps(U_bar_n, n, Y, 5 * n) || overlaps(U_bar_np1, n, Y, 5 * n))
    return fail(c, DG_EINVAL, "rk_step_vjp_recorded: a cotangent overlaps Y");
  int rc = vjp_supported(c);
  if (rc) return rc;
  if ((rc = ensure_reverse_buffers(c, true, false))) return rc;
  const double* Ys[5] = {Y, Y + n, Y + 2 * n, Y + 3 * n, Y + 4 * n};
  return rk_reverse(c, Ys, dt, U_bar_np1, U_bar_n, "rk_step_vjp_recorded");
}

int rk_step_vjp(dg_ctx* c, const double* U_n, double dt, const double* U_bar_np1, double* U_bar_n) {
  if (check_ctx(c)) return DG_EINVAL;
  if (!is_device_ptr(U_n) || !is_device_ptr(U_bar_np1) || !is_device_ptr(U_bar_n))
    return fail(c, DG_EINVAL, "rk_step_vjp: device pointers required");
  if (!finite_pos(dt)) return fail(c, DG_EINVAL, "rk_step_vjp: dt must be finite and > 0");
  if ((const void*)U_bar_n == (const void*)U_n) return fail(c, DG_EINVAL, "rk_step_vjp: U_bar_n aliases U_n");
  int rc = vjp_supported(c);
  if (rc) return rc;
  if ((rc = ensure_reverse_buffers(c, true))) return rc;
  if ((rc = ensure_split_buffer(c))) return rc;
  const size_t bytes = c->nstate * sizeof(double);
  hipError_t e = hipMemcpyAsync(c->Y[0], U_n, bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "rk_step_vjp copy");
  // forward: stage states Y_1..Y_4 (Y_5 = U_{n+1} is not needed)
  for (int k = 0; k < 4; ++k)
    if ((rc = run_stage(c, c->Y[k], c->Y[k + 1], nullptr, MODE_RK, kA[k], kB[k] * dt, 1, nullptr, nullptr,
                        chain_flags(k, 3))))
      return rc;
  const double* Ys[5] = {c->Y[0], c->Y[1], c->Y[2], c->Y[3], c->Y[4]};
  return rk_reverse(c, Ys, dt, U_bar_np1, U_bar_n, "rk_step_vjp");
}

int dg_max_dt(dg_ctx* c, const double* U, double cfl, double* dt_out) {
  if (check_ctx(c) || !dt_out) return fail(c, DG_EINVAL, "dg_max_dt: NULL argument");
  if (!is_device_ptr(U)) return fail(c, DG_EINVAL, "dg_max_dt: U must be a device pointer");
  if (!finite_pos(cfl)) return fail(c, DG_EINVAL, "dg_max_dt: cfl must be finite and > 0");
  ReduceArgs r = reduce_args(c, U);
  hipError_t e = c->kt->max_rate(r, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->h_partial, c->partial, 2 * kRedBlocks * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "dg_max_dt");
  double la = 0.0, lv = 0.0;
  for (int b = 0; b < kRedBlocks; ++b) {
    la = std::max(la, c->h_partial[2 * b]);
    lv = std::max(lv, c->h_partial[2 * b + 1]);
  }
  if (!(la > 0.0) || !std::isfinite(la) || !std::isfinite(lv))
    return fail(c, DG_ENONFINITE, "dg_max_dt: non-finite or zero wave speed");
  double dt = cfl / ((c->N + 1.0) * la);
  if (lv > 0.0) dt = std::min(dt, cfl / ((c->N + 1.0) * (c->N + 1.0) * lv));
  *dt_out = dt;
  return DG_OK;
}

int dg_integrals(dg_ctx* c, const double* X, double out[5]) {
  if (check_ctx(c) || !out) return fail(c, DG_EINVAL, "dg_integrals: NULL argument");
  if (!is_device_ptr(X)) return fail(c, DG_EINVAL, "dg_integrals: X must be a device pointer");
  ReduceArgs r = reduce_args(c, X);
  hipError_t e = c->kt->integrals(r, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->h_partial, c->partial, 5 * kRedBlocks * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "dg_integrals");
  for (int v = 0; v < 5; ++v) {
    double s = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) s += c->h_partial[5 * b + v];
    out[v] = s;
  }
  return DG_OK;
}

int dg_alpha(dg_ctx* c, const double* U, double* alpha) {
  if (check_ctx(c)) return DG_EINVAL;
  if (!is_device_ptr(U) || !is_device_ptr(alpha)) return fail(c, DG_EINVAL, "dg_alpha: device pointers required");
  if (c->N < 2) return fail(c, DG_EUNSUPPORTED, "dg_alpha: needs N >= 2");
  StageArgs a = stage_args(c);
  a.U = U;
  a.alpha_out = alpha;
  hipError_t e = c->kt->alpha1(a, c->stream);
  if (e == hipSuccess) e = c->kt->spread(a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "dg_alpha");
  return DG_OK;
}

int dg_check_finite(dg_ctx* c, const double* X) {
  if (check_ctx(c)) return DG_EINVAL;
  if (!is_device_ptr(X)) return fail(c, DG_EINVAL, "dg_check_finite: X must be a device pointer");
  ReduceArgs r = reduce_args(c, X);
  hipError_t e = c->kt->nonfinite(r, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->h_partial, c->partial, kRedBlocks * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "dg_check_finite");
  double s = 0.0;
  for (int b = 0; b < kRedBlocks; ++b) s += c->h_partial[b];
  if (s > 0.0) return fail(c, DG_ENONFINITE, "dg_check_finite: %.0f non-finite entries", s);
  return DG_OK;
}

int dg_set_profiling(dg_ctx* c, int on) {
  if (check_ctx(c)) return DG_EINVAL;
  c->profiling = on ? 1 : 0;
  c->recs.clear();
  return DG_OK;
}

int dg_profile_read(dg_ctx* c, double ms[5], int64_t launches[5]) {
  if (check_ctx(c) || !ms || !launches) return fail(c, DG_EINVAL, "dg_profile_read: NULL argument");
  for (int k = 0; k < 5; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "dg_profile_read");
  for (const auto& r : c->recs) {
    float t = 0.0f;
    e = hipEventElapsedTime(&t, c->ev_pool[r.a], c->ev_pool[r.b]);
    if (e != hipSuccess) return hip_fail(c, e, "dg_profile_read");
    ms[r.kind] += t;
    launches[r.kind] += 1;
  }
  c->recs.clear();
  return DG_OK;
}

int dg_node_weights(const dg_ctx* c, double* w) {
  if (!c || !w) return DG_EINVAL;
  if (c->M) return DG_EUNSUPPORTED;  // per-node Jacobians: use dg_integrals
  const std::vector<double> b = build_basis(c->N);
  const BasisLayout L(c->n1);
  for (int k = 0; k < c->n1; ++k)
    for (int j = 0; j < c->n1; ++j)
      for (int i = 0; i < c->n1; ++i)
        w[i + c->n1 * (j + c->n1 * k)] = b[L.w() + i] * b[L.w() + j] * b[L.w() + k] * c->Jac;
  return DG_OK;
}

int dg_sizes(const dg_ctx* c, int64_t* n_elems, int64_t* nodes_per_elem) {
  if (!c) return DG_EINVAL;
  if (n_elems) *n_elems = c->nelem;
  if (nodes_per_elem) *nodes_per_elem = c->nn;
  return DG_OK;
}

int dg_finalize(dg_ctx* c) {
  if (!c) return DG_OK;
  release(c);
  delete c;
  return DG_OK;
}

const char* dg_last_error(const dg_ctx* c) { return c ? c->err : g_init_error; }

}  // extern "C"
