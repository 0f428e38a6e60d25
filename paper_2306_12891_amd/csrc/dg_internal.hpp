// Internal interface between the host side of libdgmi (dg_host.cpp) and the
// per-degree kernel translation units (dg_kernels.hip compiled once per N).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgmi {

// MODE_DIFF (blended Euler operator): U_t^FV - U_t^DG of blended elements
// (zero elsewhere) into Ut, for the reverse mode through the blending.
enum { MODE_UT = 0, MODE_RK = 1, MODE_DIFF = 2 };

// Packed 1-D basis, built on the host and read into LDS by the kernels.
// Offsets in doubles for n1 = N + 1.
struct BasisLayout {
  int n1;
  __host__ __device__ constexpr BasisLayout(int n) : n1(n) {}
  __host__ __device__ constexpr int Dhat() const { return 0; }            // split-form volume matrix
  __host__ __device__ constexpr int Dw() const { return n1 * n1; }        // D - W^-1 B  (= -W^-1 D^T W)
  __host__ __device__ constexpr int winv() const { return 2 * n1 * n1; }  // 1 / w_i
  __host__ __device__ constexpr int xi() const { return 2 * n1 * n1 + n1; }
  __host__ __device__ constexpr int edge() const { return 2 * n1 * n1 + 2 * n1; }  // n1 + 1 subcell edges
  __host__ __device__ constexpr int Vinv() const { return 2 * n1 * n1 + 3 * n1 + 1; }
  __host__ __device__ constexpr int w() const { return 3 * n1 * n1 + 3 * n1 + 1; }
  __host__ __device__ constexpr int D() const { return 3 * n1 * n1 + 4 * n1 + 1; }  // plain LGL derivative
  __host__ __device__ constexpr int size() const { return 4 * n1 * n1 + 4 * n1 + 1; }
};

struct StageArgs {
  const double* U;      // stage input state
  double* Uout;         // RK: output state (ping-pong, never aliases U)
  double* G;            // RK register
  double* Ut;           // MODE_UT output
  const int32_t* nbr;   // [nelem][6]: -x +x -y +y -z +z
  const double* basis;  // BasisLayout
  const double* alpha1; // per element, clipped coefficient before spreading
  double* alpha_out;    // optional: final blending coefficient per element
  double* Fvf;          // NS: [nelem][6][4][nf] normal viscous flux on own faces
  double invJ[3];       // 2 / dx_d
  double gamma, mu, kappa;  // kappa = mu gamma / ((gamma - 1) Pr)
  double A, Bdt;        // RK stage coefficients (A_k, B_k dt)
  double amin, amax, aspread;
  double thresh, sharp;  // T(N) and s
  // Smagorinsky model (stage/lift kernels with EQ 2): per-element C_s (or
  // NULL: the constant cs), squared filter width, gamma / ((gamma - 1) Pr_t)
  const double* cs_elem;
  double cs, delta2, ktf;
  int nelem, chunk;      // chunk = ceil(nelem / 8): XCD-contiguous element ranges
  int vf, sf, blend, mode, writeG, indicator, recon;
  // curved mesh: M[e][10][nn], Ja^i_m at slot 3 i + m, 1/J at slot 9 (NULL:
  // the Cartesian box)
  const double* M;
  // curved mesh with general connectivity: conn[e][f] = (neighbour, its local
  // face, orientation 0..7), validated on the host; NULL: structured (nbr)
  const int32_t* conn;
  // wall-modelled boundaries on the two box faces normal to wall_dir (-1:
  // none; those faces have neighbour -1 in nbr): exchange distance wm_h (the
  // element size along wall_dir), van Driest freestream velocity wm_uinf and
  // factor wm_b (0: the untransformed law)
  int wall_dir;
  double wm_h, wm_uinf, wm_b;
  int ne[3];  // elements per direction of the box
  // curved mesh with the eddy viscosity: squared filter width per element
  const double* delta2_elem;
  // blended Euler operator, MODE_RK: the stage kernel also writes the
  // first-stage coefficient of its output state per element here (NULL: not;
  // only where KernelTable.fused_alpha1 is set)
  double* alpha1_next;
  // Split BR1 (FP64 Navier-Stokes without the eddy viscosity, walls or
  // blending, on the box): split != 0 makes Fvf hold each element's "own
  // part" of its normal viscous flux at its face nodes -- the flux of the
  // lifted gradient whose interface values q* = (q- + q+)/2 keep only the
  // element's own half -- and the stage kernel adds the neighbour-dependent
  // rest itself (it is linear in the other halves: the own element's face
  // values and, at the face's edges, those of the diagonal elements).  In
  // MODE_RK the stage kernel then also writes the own part of its output
  // state into Fvf_next (NULL: not), so that a Runge-Kutta run needs the
  // lifting kernel only before its first stage.  The lifting kernel with
  // split != 0 writes the own part.
  double* Fvf_next;
  int split;
};

struct ReduceArgs {
  const double* X;
  double* partial;  // per block
  const double* basis;
  double invdx[3];
  double gamma, nu_fac;  // nu_fac = mu gamma / Pr (0 for Euler)
  double Jac;
  int nelem;
  const double* M;  // curved mesh metrics (see StageArgs), or NULL
};

// Vector-Jacobian product arguments (reverse mode of the FP64 operator).
struct VjpArgs {
  const double* U;      // state at which the operator is linearised
  const double* Lbar;   // cotangent of U_t (lambda)
  double* Ubar;         // output: (dL/dU)^T lambda, or Uacc + that
  const double* Uacc;   // optional: accumulate into this array (may alias Ubar)
  const int32_t* nbr;
  const double* basis;
  double* Gbf;          // NS: [nelem][6][4][nf] cotangent of the normal lifted gradient at own face nodes
  // Smagorinsky model (les != 0): per-element C_s (or NULL: the constant cs),
  // squared filter width, gamma / ((gamma - 1) Pr_t), as in StageArgs
  int les;
  const double* cs_elem;
  double cs, delta2, ktf;
  // wall-modelled boundaries (see StageArgs); wall_dir -1: none
  int wall_dir;
  double wm_h, wm_uinf, wm_b;
  // curved mesh with the eddy viscosity: squared filter width per element
  const double* delta2_elem;
  double invJ[3];
  double gamma, mu, kappa;
  int nelem, chunk;
  int vf, sf;
  // blending (Euler): final and first-stage coefficients of the linearisation
  // state, the differences U_t^FV - U_t^DG (MODE_DIFF) and the per-element
  // cotangent of alpha; all NULL without blending
  const double* alpha;
  const double* alpha1;
  const double* Dfd;
  double* abar;
  double amin, amax, aspread, thresh, sharp;
  int indicator, recon;
  // curved mesh: metric terms and general connectivity (see StageArgs), or NULL
  const double* M;
  const int32_t* conn;
};

struct KernelTable {
  int nt;  // threads per block
  int fused_alpha1;  // the blended Euler stage kernels honour StageArgs.alpha1_next
  hipError_t (*stage)(const StageArgs&, int eq, hipStream_t);
  hipError_t (*stage_mixed)(const StageArgs&, int eq, hipStream_t);
  hipError_t (*lift)(const StageArgs&, int eq, hipStream_t);
  hipError_t (*lift_mixed)(const StageArgs&, int eq, hipStream_t);
  hipError_t (*alpha1)(const StageArgs&, hipStream_t);
  hipError_t (*spread)(const StageArgs&, hipStream_t);
  hipError_t (*max_rate)(const ReduceArgs&, hipStream_t);
  hipError_t (*integrals)(const ReduceArgs&, hipStream_t);
  hipError_t (*nonfinite)(const ReduceArgs&, hipStream_t);
  // reverse operator (eq 0 Euler, 1 Navier-Stokes, 2 with the eddy viscosity;
  // walls per VjpArgs.wall_dir) and its BR1 pass 1 (the eddy-viscosity
  // variant per VjpArgs.les)
  hipError_t (*vjp)(const VjpArgs&, int eq, hipStream_t);
  hipError_t (*vjp_lift)(const VjpArgs&, hipStream_t);
  // reverse mode through the blending: per-element cotangent of alpha, its
  // pullback to the state (writes Ubar = [Uacc +] ...), and the FV subcell
  // part (adds to Ubar)
  hipError_t (*vjp_alpha_bar)(const VjpArgs&, hipStream_t);
  hipError_t (*vjp_alpha)(const VjpArgs&, hipStream_t);
  hipError_t (*vjp_fv)(const VjpArgs&, hipStream_t);
  // y <- a y + b x over n doubles
  hipError_t (*axpby)(double* y, double a, const double* x, double b, size_t n, hipStream_t);
  // curved mesh: metric terms from node coordinates X[e][3][nn] into M
  // (counts non-positive or non-finite Jacobians into *bad), and the
  // operator kernels with metric terms (FP64; eq 0 Euler, 1 Navier-Stokes,
  // 2 with the eddy viscosity; the metric kernel also writes the squared
  // filter width per element into d2)
  hipError_t (*metrics)(const double* X, const double* basis, double* M, int* bad, double* d2, int nelem,
                        int chunk, hipStream_t);
  hipError_t (*stage_curved)(const StageArgs&, int eq, hipStream_t);
  hipError_t (*lift_curved)(const StageArgs&, int eq, hipStream_t);
  // reverse mode on curved elements (FP64, no blending; eq as for vjp, the
  // pass-1 variant per VjpArgs.les)
  hipError_t (*vjp_curved)(const VjpArgs&, int eq, hipStream_t);
  hipError_t (*vjp_lift_curved)(const VjpArgs&, hipStream_t);
  // wall-model flux at the wall face nodes into Fvf (FP64, after the lift)
  hipError_t (*wall_flux)(const StageArgs&, hipStream_t);
};

const KernelTable* table_N1();
const KernelTable* table_N2();
const KernelTable* table_N3();
const KernelTable* table_N4();
const KernelTable* table_N5();
const KernelTable* table_N6();
const KernelTable* table_N7();

}  // namespace dgmi
