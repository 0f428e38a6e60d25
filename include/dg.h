/* dg.h - C ABI of the MI355X split-form DGSEM library (libdgmi.so).
 *
 * The library evaluates the discontinuous Galerkin spectral element operator
 * of the compressible Euler / Navier-Stokes equations on hexahedral meshes
 * (the periodic Cartesian box of dg_init; curved elements with structured or
 * general face connectivity, dg_set_geometry / dg_set_connectivity; two box
 * faces as wall-modelled boundaries, dg_set_wall_model) and advances it with
 * a five-stage, fourth-order, two-register (2N-storage) explicit Runge-Kutta
 * scheme.  All arithmetic runs in HIP kernels on one GPU; the host side only
 * validates arguments and enqueues work.
 *
 * Method (paper: Blind et al., "Towards Exascale CFD Simulations Using the
 * Discontinuous Galerkin Solver FLEXI"):
 *   - split-form DG on Legendre-Gauss-Lobatto nodes in flux-differencing form
 *     (Sec. 2, Sec. 4.1);
 *   - element-wise convex blending with a finite-volume subcell operator,
 *     U_t = a U_t^FV + (1 - a) U_t^DG (Sec. 4.1, blending equation), first
 *     order in the outer subcells (Sec. 4.1); with Navier-Stokes only the
 *     advective operator is blended, the viscous terms enter unweighted;
 *   - blending coefficient from a modal indicator through the sigmoid with
 *     threshold T(N) = 0.5 * 10^(-1.8 (N+1)^0.25) (Sec. 4.1, indicator
 *     equation), spread to face neighbours by 1/2 (Sec. 4.1), and kept in
 *     {0} U [0.01, 0.7] (Sec. 4.2);
 *   - explicit Runge-Kutta time stepping whose stages enter the performance
 *     index (Sec. 2, eq. (pid)).
 * The paper leaves open the two-point fluxes (Kennedy-Gruber, Pirozzoli),
 * the Riemann solvers (LLF, Roe), the viscous lifting (BR1) and the
 * Runge-Kutta coefficients (Carpenter-Kennedy (5,4) 2N-storage); the library
 * implements those standard choices.
 *
 * Data layout (every state-sized array):
 *   double, contiguous, [nElems][5][N+1 (z,k)][N+1 (y,j)][N+1 (x,i)], x fastest;
 *   variables (rho, rho*u, rho*v, rho*w, E); element e = ex + nx*(ey + ny*ez);
 *   node positions x_d = lo_d + (e_d + (xi+1)/2) * dx_d, dx_d = (hi_d-lo_d)/n_d,
 *   xi the Legendre-Gauss-Lobatto points.  "DOF" counts nodes, not variables.
 *
 * Ownership: the caller owns every array passed in (U, Ut, ...), which must
 * be device memory on the context's device and is never freed or retained.
 * The context owns all scratch (Runge-Kutta register, ping-pong state, face
 * buffers, blending arrays, reduction partials); dg_init allocates it (the
 * reverse-mode buffers and the split lifting's second face buffer on first
 * use, as noted at those calls) and dg_finalize releases it.
 *
 * Errors: every function returns DG_OK (0) or a negative code; it never
 * aborts or prints.  dg_last_error() gives a message.  Errors of asynchronous
 * kernels surface at the next synchronising call as DG_EHIP.
 *
 * Streams: every call enqueues on the context's stream (default: the null
 * stream) and returns without synchronising, except the calls that return
 * host scalars (dg_max_dt, dg_integrals, dg_check_finite).  A context is not
 * thread-safe; use one context per stream.
 */
#ifndef DG_H
#define DG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DG_OK = 0,
  DG_EINVAL = -1,        /* bad argument (null/host pointer, alias, range)   */
  DG_ENOMEM = -2,        /* device allocation failed in dg_init              */
  DG_EHIP = -3,          /* HIP runtime error (launch or earlier kernel)     */
  DG_EUNSUPPORTED = -4,  /* valid but unsupported combination of options     */
  DG_ENONFINITE = -5,    /* dg_check_finite found a NaN or Inf               */
  DG_ESTATE = -6         /* call not valid in the context's current state    */
};

enum { DG_EULER = 0, DG_NS = 1 };
enum { DG_VF_KG = 0, DG_VF_PI = 1, DG_VF_CH = 2, DG_VF_STD = 3 };
enum { DG_SF_LLF = 0, DG_SF_ROE = 1, DG_SF_CENTRAL = 2 };
enum { DG_IND_HENNEMANN = 0, DG_IND_PERSSON = 1 };
enum { DG_FV_FIRST = 0, DG_FV_MINMOD = 1 };
enum { DG_FP64 = 0, DG_MIXED = 1 };
/* BR1 lifting of the Navier-Stokes operator (the standard choice for the
 * gradients, which the paper leaves open: the lifted gradient takes the
 * interface values q* = (q- + q+)/2 of the primitive variables q = (u, v, w,
 * p/rho) on every face).
 *   TWO_PASS: every stage first lifts the normal viscous flux at all face
 *     nodes (one kernel), then evaluates the operator.
 *   SPLIT: the same operator up to rounding, with the lifting split into each
 *     element's own half of q*, which the stage kernel of a Runge-Kutta stage
 *     writes for the next stage, and the rest, which the stage kernel adds
 *     where it reads the neighbour's face data; a step lifts only before its
 *     first stage.  Applies to the FP64 operator without the eddy viscosity,
 *     blending, walls or curved geometry; elsewhere TWO_PASS runs. */
enum { DG_LIFT_TWO_PASS = 0, DG_LIFT_SPLIT = 1 };

typedef struct dg_ctx dg_ctx; /* opaque, library-owned */

/* Periodic box: nelem[d] elements over [lo[d], hi[d]] in direction d. */
typedef struct {
  int32_t nelem[3];
  double lo[3], hi[3];
} dg_mesh;

/* Operator options (dg_default_options fills the defaults noted here). */
typedef struct {
  int32_t equations;    /* DG_EULER | DG_NS                          (EULER)   */
  int32_t vol_flux;     /* two-point volume flux: DG_VF_*            (KG)      */
  int32_t surf_flux;    /* Riemann solver: DG_SF_*                   (LLF)     */
  int32_t blending;     /* 0 | 1: DG/FV blending of the advective terms (0)    */
  int32_t indicator;    /* DG_IND_HENNEMANN | DG_IND_PERSSON         (HENNEMANN) */
  int32_t fv_recon;     /* DG_FV_FIRST | DG_FV_MINMOD                (MINMOD)  */
  int32_t precision;    /* DG_FP64 | DG_MIXED                        (FP64)    */
  int32_t lifting;      /* DG_LIFT_*                                 (SPLIT)   */
  double Pr;            /* Prandtl number                            (0.72)    */
  double alpha_min;     /* below: pure DG (paper Sec. 4.2)           (0.01)    */
  double alpha_max;     /* upper clip (paper Sec. 4.2)               (0.7)     */
  double alpha_spread;  /* neighbour factor (paper Sec. 4.1)         (0.5)     */
  double Cs;            /* Smagorinsky coefficient, DG_NS only; 0 = no
                           eddy viscosity (paper Sec. 5)             (0)       */
  double Prt;           /* turbulent Prandtl number of the model     (0.9)     */
} dg_options;

/* Fills *opt with the defaults above. */
void dg_default_options(dg_options* opt);

/* Creates a context for polynomial degree N (1..7) on the mesh, ratio of
 * specific heats gamma (> 1) and dynamic viscosity mu (>= 0; used only by
 * DG_NS).  Uses the current HIP device.  Allocates all scratch; on failure
 * nothing stays allocated and *out is set to NULL. */
int dg_init(const dg_mesh* mesh, int N, double gamma, double mu, dg_ctx** out);

/* Replaces the options.  Validated here: DG_EUNSUPPORTED for blending with
 * N < 2, DG_MIXED with blending, or the Smagorinsky
 * model (Cs > 0) with the DG_VF_CH flux; DG_EINVAL for Cs < 0 or Prt <= 0. */
int dg_set_options(dg_ctx* ctx, const dg_options* opt);
int dg_get_options(const dg_ctx* ctx, dg_options* opt);

/* Smagorinsky eddy viscosity with one coefficient per element (paper Sec. 5:
 * the standard model uses a constant C_s; the learned model sets C_s per
 * element and the eddy viscosity is evaluated at every solution point of the
 * element).  With DG_NS, at every node of element e:
 *   mu_t = rho (C_s(e) Delta)^2 |S|,  |S| = sqrt(2 S_ij S_ij) of the lifted
 *   velocity gradient, Delta = (dx dy dz)^(1/3) / (N + 1) (on curved meshes
 *   (element volume)^(1/3) / (N + 1), see dg_set_geometry),
 * added to mu in the viscous stress, and mu_t gamma / ((gamma - 1) Prt) added
 * to the heat-flux coefficient mu gamma / ((gamma - 1) Pr).
 * cs: device pointer to nElems doubles (element order of the state), copied
 * into the context on its stream (the caller may free it afterwards); it
 * replaces opt.Cs until dg_set_cs_field(ctx, NULL) restores the constant.
 * Errors: DG_EINVAL for a host pointer, DG_EUNSUPPORTED with DG_VF_CH,
 * DG_ENOMEM.  dg_vjp and rk_step_vjp differentiate through the model (mu_t
 * through |S|, with derivative 0 where |S| = 0, and through rho), on the
 * Cartesian box and on curved meshes.  The
 * time-step estimate dg_max_dt uses the molecular viscosity only. */
int dg_set_cs_field(dg_ctx* ctx, const double* cs);

/* Curved hexahedral mesh (the paper's applications in Secs. 3-5 run on
 * unstructured curvilinear meshes; the split form keeps its free-stream,
 * conservation and kinetic-energy/entropy properties there when the metric
 * terms satisfy the discrete metric identities).  X: device pointer to the
 * node coordinates, X[e][m][k][j][i] (nElems x 3 x (N+1)^3 doubles, m = x, y,
 * z; element order and face connectivity of the periodic structured mesh
 * given to dg_init, each element a smooth image of the reference cube with
 * faces shared by two elements holding the same points).  Read once: the
 * library computes and keeps the metric terms (conservative curl form,
 * 10 doubles per node: Ja^i_m and 1/J), after which every operator call
 * (dg_time_derivative, dg_rk_steps, rk_step, dg_max_dt, dg_integrals) uses
 * them:
 *   J U_t = - sum_i [ sum_l Dhat_il F#(U_n, U_l).(Ja^i_n + Ja^i_l)/2 + lifted
 *            face flux |Ja_f| f*(U-, U+; Ja_f/|Ja_f|) ],
 * Ja_f the mean of both elements' metric at a face node; Navier-Stokes with
 * the BR1 gradient (1/J) sum_i Ja^i (d_i q + lifting) and the contravariant
 * viscous flux; with the Smagorinsky model the filter width of an element is
 * (element volume)^(1/3) / (N + 1), the volume the quadrature sum of J (on
 * the box the Cartesian (dx dy dz)^(1/3) / (N + 1)).  X = NULL returns to the
 * Cartesian box of dg_init.
 * Errors (the context's geometry is then unchanged): DG_EINVAL for a host
 * pointer or a non-positive / non-finite Jacobian at any node; DG_EUNSUPPORTED with
 * blending, DG_MIXED or DG_VF_CH (and later dg_set_options calls that would
 * enable them return it); DG_ENOMEM.  dg_vjp and rk_step_vjp work on curved
 * meshes (also with general connectivity and the Smagorinsky model);
 * dg_node_weights returns DG_EUNSUPPORTED there
 * (per-node Jacobians: use dg_integrals). */
int dg_set_geometry(dg_ctx* ctx, const double* X);

/* General connectivity of a curved mesh (unstructured hexahedra, as the
 * paper's meshes in Secs. 3-5 are).  conn: host pointer to nElems x 6 x 3
 * int32, for element e and local face f (0:-xi 1:+xi 2:-eta 3:+eta 4:-zeta
 * 5:+zeta): the neighbour element, its local face that is shared, and the
 * orientation o in 0..7 mapping the face-local node index a = t1 + (N+1) t2
 * (t1 along the lower of the face's two reference axes) to the neighbour's:
 * bit 0 swaps (t1, t2), then bit 1 reverses the first and bit 2 the second
 * index.  Copied.  Every face is evaluated from a minus to a plus side (the
 * + face of a (+,-) pair, else the smaller (element, face)), so both
 * elements use the same interface values.  The node coordinates of
 * dg_set_geometry must follow the same element-local labelling; the operator
 * returns DG_ESTATE while general connectivity is set without curved
 * geometry.  NULL restores the structured periodic mesh of dg_init.
 * Errors: DG_EINVAL for an out-of-range entry, a face that is not named back
 * by its neighbour, or orientations of a face pair that are not inverse to
 * each other (nothing is changed then); DG_ENOMEM. */
int dg_set_connectivity(dg_ctx* ctx, const int32_t* conn);

/* Wall-modelled boundaries (paper Sec. 3): the two faces of the box normal to
 * direction wall_dir (0 x, 1 y, 2 z) become walls, the other directions stay
 * periodic; wall_dir = -1 restores the periodic box.  At a wall the advective
 * flux and the BR1 interface value take the mirror image of the own face state
 * (normal momentum reversed) as the other side.  The viscous flux through the
 * wall is the wall model's: the wall-parallel velocity u of the element's node
 * on the opposite face (the exchange location, h = the element size along
 * wall_dir) gives the friction velocity u_tau by Spalding's law of the wall
 *   y+ = u+ + 0.1108 [e^(0.4 u+) - 1 - 0.4 u+ - (0.4 u+)^2/2 - (0.4 u+)^3/6
 *        - (0.4 u+)^4/24],  y+ = h u_tau / nu,  u+ = u / u_tau,
 * nu = mu / rho at the wall node, solved by Newton's method to full precision;
 * with ma_inf > 0 u is first van Driest transformed,
 *   u_eq = (u_inf / b) asin(min(b u / u_inf, 1)),  b = sqrt(r / (1 + r)),
 *   r = (gamma - 1)/2 ma_inf^2 Pr^(1/3).
 * The wall shear stress rho u_tau^2 acts against that velocity in the
 * tangential momentum; mass, normal momentum and energy see no flux through
 * the wall (adiabatic wall at rest).  Needs the FP64 Navier-Stokes operator
 * (also with the Smagorinsky model and with blending: a wall face spreads no
 * blending coefficient, and the FV subcells of a wall element take the wall's
 * advective flux there), mu > 0, the Cartesian box;
 * while walls are set, dg_set_options, dg_set_geometry and dg_set_connectivity
 * calls that would break this return DG_EUNSUPPORTED.  dg_vjp and rk_step_vjp
 * differentiate through the walls (mirror states, and the wall shear through
 * the Newton solution by the implicit function theorem and through the van
 * Driest transformation, derivative 0 where its argument is capped), also
 * together with the Smagorinsky model.
 * Errors (nothing is changed then): DG_EINVAL for wall_dir outside -1..2,
 * ma_inf < 0 or non-finite, or ma_inf > 0 with u_inf <= 0; DG_EUNSUPPORTED as
 * above; DG_ENOMEM. */
int dg_set_wall_model(dg_ctx* ctx, int wall_dir, double u_inf, double ma_inf);

/* Sets the HIP stream (hipStream_t) all later calls enqueue on; NULL = null
 * stream. */
int dg_set_stream(dg_ctx* ctx, void* hip_stream);

/* Ut = L(U): the semi-discrete time derivative (paper Sec. 4.1: the solution's
 * time derivative of the DG, FV or blended operator).  A pure function of U:
 * the blending coefficient is recomputed from U.  Overwrites all of Ut.
 * Ut must not alias U. */
int dg_time_derivative(dg_ctx* ctx, const double* U, double* Ut);

/* One Runge-Kutta step of size dt (> 0, finite), in place: five stages
 * G <- A_k G + L(U), U <- U + B_k dt G (A_1 = 0).  The paper fixes only an
 * explicit Runge-Kutta scheme whose stages are counted in the performance
 * index (Sec. 2, eq. (pid)); the coefficients A_k, B_k are those of the
 * Carpenter-Kennedy five-stage fourth-order 2N-storage scheme (a reading).
 * U: device, state layout above, read and overwritten.  The blending
 * coefficient is recomputed at every stage.  Errors: DG_EINVAL for a host or
 * NULL pointer or dt not finite and > 0; DG_EHIP for launch failures. */
int rk_step(dg_ctx* ctx, double* U, double dt);

/* nsteps Runge-Kutta steps in place (same result as nsteps rk_step calls).
 * With the split lifting (dg_options.lifting) rk_step, dg_rk_steps,
 * rk_step_record and rk_step_vjp allocate a second face buffer of
 * nElems * 6 * 4 * (N+1)^2 doubles on first use (DG_ENOMEM if that fails). */
int dg_rk_steps(dg_ctx* ctx, double* U, double dt, int nsteps);

/* Vector-Jacobian product of the operator: U_bar = (dL/dU)^T Ut_bar (the
 * reverse mode of dg_time_derivative, for gradients of functionals of the
 * solution).  Overwrites U_bar, which must not alias U or Ut_bar.  With
 * blending the product includes the dependence of the blending
 * coefficient on U (paper Sec. 4.1: indicator sigmoid, clip and neighbour
 * spread) and of the FV subcell reconstruction; at their switches the
 * one-sided rules are: derivative 0 where the coefficient is clipped or cut
 * off, the mean derivative at ties of a maximum, the selected slope of the
 * minmod limiter.  On curved meshes (dg_set_geometry, also with general
 * connectivity) the product is that of the curved operator; with the
 * Smagorinsky model it includes the eddy viscosity's dependence on the
 * lifted gradient and the density (derivative of |S| taken as 0 where
 * |S| = 0); with wall-modelled boundaries it includes the wall model.  Not
 * available with DG_MIXED or the CH flux (DG_EUNSUPPORTED).
 * Allocates the reverse-mode face buffer (and with blending two more buffers)
 * on first use. */
int dg_vjp(dg_ctx* ctx, const double* U, const double* Ut_bar, double* U_bar);

/* dg_vjp for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same product with the same kernels, bitwise equal to dg_vjp, but its
 * reverse-mode buffers (the face buffer of gradient cotangents for DG_NS, and
 * with blending U_t^FV - U_t^DG and the cotangent of the blending
 * coefficient) are carved from a fixed 64 MiB device array of the library
 * (one per GPU, held until the process ends; its address is looked up in
 * dg_init) instead of being allocated on first use.  The call itself
 * allocates nothing.  Limit: nElems * (6 * 4 * (N+1)^2 [DG_NS] + 5 (N+1)^3 + 1
 * [blending]) doubles must fit in 64 MiB (e.g. 2.8 M nodes of DG_NS without
 * blending); larger meshes return DG_EINVAL with the required size.  Every
 * entry of the array is written before it is read in a call, so nothing needs
 * clearing; calls that overlap on one GPU (several contexts or streams at
 * once) race on the array.  Errors as dg_vjp, DG_EHIP if the array's address
 * could not be obtained. */
int dg_vjp_noalloc(dg_ctx* ctx, const double* U, const double* Ut_bar, double* U_bar);

/* Vector-Jacobian product of one rk_step (the step of Sec. 2, eq. (pid), with
 * the 2N-storage coefficients of rk_step): U_bar_n = (dU_{n+1}/dU_n)^T
 * U_bar_np1, with U_n the state before the step.  All three arrays are
 * device memory in the state layout; U_n is read only.  Recomputes the five stage states from
 * U_n and runs the reverse 2N-storage recurrence
 *   Gbar <- A_{k+1} Gbar + B_k dt Ybar,  Ybar <- Ybar + VJP(Y_{k-1}, Gbar),
 * k = 5..1.  Overwrites U_bar_n (may alias U_bar_np1, not U_n).  Same
 * restrictions as dg_vjp; allocates seven state-sized buffers on first use. */
int rk_step_vjp(dg_ctx* ctx, const double* U_n, double dt, const double* U_bar_np1, double* U_bar_n);

/* One rk_step in place on U that also records its five stage states: Y is a
 * device pointer to 5 x (nElems x 5 x (N+1)^3) doubles owned by the caller,
 * filled with Y_0 = U_n, Y_1, ..., Y_4 (the inputs of the five stages; paper
 * Sec. 4: the explicit Runge-Kutta scheme).  U ends as U_{n+1}, bitwise the
 * same as rk_step.  For checkpointed reverse sweeps that keep the stage states
 * of a segment instead of recomputing them in rk_step_vjp.  Errors: DG_EINVAL
 * for host pointers, dt not finite and > 0, or Y overlapping U. */
int rk_step_record(dg_ctx* ctx, double* U, double dt, double* Y);

/* rk_step_vjp from the stage states recorded by rk_step_record (Y, read
 * only): the same reverse recurrence without recomputing the stages, so the
 * same result bitwise.  U_bar_n may alias U_bar_np1; neither may overlap Y.
 * Same restrictions as dg_vjp; allocates two state-sized buffers on first
 * use. */
int rk_step_vjp_recorded(dg_ctx* ctx, const double* Y, double dt, const double* U_bar_np1, double* U_bar_n);

/* Stable time step.  The paper states no time-step rule; the reading used
 * here is the usual convective and viscous CFL estimate over all nodes:
 *   dt = cfl * min(1/((N+1) max sum_d (|u_d|+c)/dx_d),
 *                  1/((N+1)^2 max nu_eff sum_d 1/dx_d^2)),
 * nu_eff = mu gamma/(rho Pr) for DG_NS (on curved meshes |Ja^d|/(2J) in
 * place of 1/dx_d and the contravariant velocity).  U: device state; dt_out:
 * host.  Synchronises.  Errors: DG_EINVAL for bad pointers or cfl not finite
 * and > 0; DG_ENONFINITE if any node is not finite or has rho <= 0 or p <= 0
 * (no time step is returned then). */
int dg_max_dt(dg_ctx* ctx, const double* U, double cfl, double* dt_out);

/* Conservation integrals (the quadrature that makes the split form
 * conservative, Sec. 2): out[v] = sum_e J sum_ijk w_i w_j w_k X[e][v][ijk],
 * FP64, J = dx dy dz / 8 on the box (the node Jacobian on curved meshes),
 * w the LGL weights.  X: device, state layout; out: host, 5 doubles.  The
 * sum is taken in a fixed order (deterministic).  Synchronises.  Errors:
 * DG_EINVAL for bad pointers; DG_EHIP. */
int dg_integrals(dg_ctx* ctx, const double* X, double out[5]);

/* Blending coefficient per element of state U (paper Sec. 4.1: modal
 * indicator of rho*p, sigmoid with threshold T(N), spread of 1/2 to the face
 * neighbours; Sec. 4.2: clip at alpha_max, zero below alpha_min), exactly the
 * coefficient the blended operator uses at that state.  U: device, state
 * layout; alpha: device, nElems doubles, overwritten.  Errors: DG_EINVAL for
 * bad pointers; DG_EUNSUPPORTED without blending. */
int dg_alpha(dg_ctx* ctx, const double* U, double* alpha);

/* DG_OK if every entry of the state-sized array X is finite, else
 * DG_ENONFINITE.  Synchronises. */
int dg_check_finite(dg_ctx* ctx, const double* X);

/* Per-kernel timing for benchmarks.  While enabled (on != 0), every kernel
 * launch of the operator is bracketed by two HIP events recorded on the
 * context's stream.  dg_profile_read synchronises the stream, writes the
 * summed milliseconds and the number of launches per kernel kind
 * (DG_K_STAGE: operator + Runge-Kutta stage, DG_K_LIFT: BR1 lifting and
 * the wall-model pass of dg_set_wall_model,
 * DG_K_INDICATOR: modal indicator, DG_K_VJP: reverse operator,
 * DG_K_VJP_LIFT: reverse BR1 lifting) into ms[5] and launches[5], and clears
 * the records.  Disabling also clears them. */
enum { DG_K_STAGE = 0, DG_K_LIFT = 1, DG_K_INDICATOR = 2, DG_K_VJP = 3, DG_K_VJP_LIFT = 4 };
int dg_set_profiling(dg_ctx* ctx, int on);
int dg_profile_read(dg_ctx* ctx, double ms[5], int64_t launches[5]);

/* Quadrature weight of every node of an element, w_i w_j w_k J (host array
 * of (N+1)^3 doubles, x index fastest), so that sum_e sum_n w_n X[e][v][n]
 * is the integral of X_v (used to build functionals for the adjoint). */
int dg_node_weights(const dg_ctx* ctx, double* w);

/* Sizes: number of elements and nodes per element. */
int dg_sizes(const dg_ctx* ctx, int64_t* n_elems, int64_t* nodes_per_elem);

/* Releases the context and all its scratch (NULL is allowed). */
int dg_finalize(dg_ctx* ctx);

/* Message of the last error on ctx (or of the last failed dg_init when ctx
 * is NULL). */
const char* dg_last_error(const dg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* DG_H */
