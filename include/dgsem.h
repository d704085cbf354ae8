/*
 * dgsem.h -- C ABI of the MI355X (gfx950) DGSEM library libdgsem.so.
 *
 * The library evaluates the semi-discrete residual dU/dt of the compressible Euler /
 * Navier-Stokes equations (HORSES3D paper, arXiv 2206.09733, section "Compressible
 * Navier-Stokes", eqs. compressibleNScompact and viscousfluxes) on curvilinear hexahedral
 * Gauss-Lobatto spectral elements (section "Spatial discretisation: discontinuous Galerkin",
 * eqs. compressibleNScompact_transformed and NS2-NS5): an entropy-conserving split-form
 * volume term (section "Energy/Entropy stable versions"), Riemann fluxes with surface lifting
 * (Roe, local Lax-Friedrichs, EC, central; box of convective fluxes), BR1 viscous terms (box
 * of viscous fluxes), and advances it with Williamson's low-storage explicit RK3 (section
 * "Time advancement").  Every step runs in hand-written HIP kernels.
 *
 * Conventions
 *  - Status: every int-returning call returns DG_OK (0) or a negative DG_E* code; the message
 *    of the last failure on the calling thread is returned by dg_last_error().  Nothing
 *    aborts or throws across the ABI.
 *  - Ownership: dg_mesh / dg_solver / dg_batch handles are owned by the library and freed by
 *    the matching *_destroy.  Device memory is owned by the caller: dg_solver_required_bytes
 *    states the size, the caller allocates it (any device allocator) and passes it to
 *    dg_solver_bind; the library sub-allocates inside it and never frees it.  The buffer must
 *    stay valid until dg_solver_destroy.
 *  - Streams: all device work of a solver is enqueued on the HIP stream given to
 *    dg_solver_bind (NULL = the default stream).  Calls that return host data synchronise that
 *    stream; dg_rk_step and dg_residual with a NULL host pointer only enqueue.
 *  - Threading: a handle may be used by one host thread at a time.
 *  - Layout of every nodal array (state U, residual R): element-major, then conserved variable
 *    (rho, rho v1, rho v2, rho v3, rho e), then node with i fastest:
 *        U[(off_e * 5) + v * nn_e + i + n1 * (j + n2 * k)]
 *    where nn_e = n1 n2 n3 nodes, n_d = N_d + 1, off_e = sum of nn over elements before e.
 *    For uniform order all elements have nn = (N+1)^3 and off_e = e nn.
 *    Element e of an ex*ey*ez box sits at cell (e % ex, (e / ex) % ey, e / (ex ey)).
 *  - Nondimensionalisation: rho_0 = |v_0| = L = 1, gas constant 1 (T = p/rho), p_0 =
 *    1/(gamma Ma^2) for the Taylor-Green state, mu = 1/Re (constant), kappa = mu gamma /
 *    ((gamma-1) Pr).  Re <= 0 selects the Euler equations.
 */
#ifndef DGSEM_H
#define DGSEM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
#define DG_OK 0
#define DG_EINVAL (-1)       /* invalid argument or configuration                       */
#define DG_ENOMEM (-2)       /* device buffer too small, or host allocation failed        */
#define DG_EHIP (-3)         /* a HIP runtime call failed (message holds the HIP error)   */
#define DG_ENONFINITE (-4)   /* a state given to the library holds NaN/Inf or rho,p <= 0   */
#define DG_EUNSUPPORTED (-5) /* valid request outside what this library implements        */
#define DG_ESTATE (-6)       /* call out of order (e.g. solver not bound)                 */

/* ------------------------------------------------------------------ options */
enum { DG_DEFORM_NONE = 0, DG_DEFORM_SINSIN = 1 };
/* quadrature / collocation points (section "Spatial discretisation" allows both): Gauss-Lobatto
 * (every split form, every viscous flux, mixed orders, FP32-bulk), or Gauss-Legendre (more
 * accurate; no boundary nodes, so the plain weak form with face traces interpolated to the
 * element boundaries: uniform-order boxes, undeformed or deformed, FP64, volume flux
 * DG_VOL_CENTRAL, any surface flux, every viscous flux).  On Gauss-Legendre points the map and
 * its metric terms are those of the Lobatto grid of the same order (isoparametric there, curl
 * form there) evaluated at the Gauss points, and each face takes the metric of the element on
 * its -xi side interpolated to the face: a uniform state stays steady on curvilinear meshes.
 * The paper leaves these geometry rules to its references; this is the library's reading. */
enum { DG_NODES_LOBATTO = 0, DG_NODES_GAUSS = 1 };
/* volume two-point flux (the list of split forms of section "Energy/Entropy stable versions"):
 * Chandrashekar's entropy-conserving, kinetic-energy-preserving flux; the central average;
 * Ismail and Roe's entropy-conserving flux; the kinetic-energy-preserving forms of
 * Kennedy-Gruber, Pirozzoli, Ducros and Morinishi (products of arithmetic means of the two
 * states, e.g. Kennedy-Gruber's mass flux {rho}{v.n}) */
enum { DG_VOL_EC = 0, DG_VOL_CENTRAL = 1, DG_VOL_IR = 2, DG_VOL_KENNEDY_GRUBER = 3, DG_VOL_PIROZZOLI = 4,
       DG_VOL_DUCROS = 5, DG_VOL_MORINISHI = 6 };
/* surface numerical flux (box of convective fluxes in section "Spatial discretisation"): Roe
 * (evaluated with Roe and Pike's wave strengths), local Lax-Friedrichs (Rusanov),
 * Chandrashekar's EC flux, central, entropy stable (Chandrashekar's flux minus local
 * Lax-Friedrichs dissipation), Ismail-Roe, entropy stable with matrix dissipation
 * (Chandrashekar's flux minus R|Lambda|T R^T times the jump of the entropy variables),
 * low-dissipation Roe (the velocity jump scaled by the larger local Mach number, at most 1),
 * Lax-Friedrichs with the global wave speed (the largest |v| + c of the stage's state, reduced
 * on the device before each stage; DG_SURF_LLF is the local form, Rusanov).
 * Only DG_VOL_EC / DG_VOL_CENTRAL and the first four surface fluxes have an FP32-bulk form. */
enum { DG_SURF_ROE = 0, DG_SURF_LLF = 1, DG_SURF_EC = 2, DG_SURF_CENTRAL = 3, DG_SURF_ES = 4, DG_SURF_IR = 5,
       DG_SURF_ES_MATRIX = 6, DG_SURF_LOW_DISS_ROE = 7, DG_SURF_LF_GLOBAL = 8 };
/* precision: all-FP64, or FP32 flux/derivative arithmetic with FP64 metrics, RK state and
 * reductions */
enum { DG_FP64 = 0, DG_FP32_BULK = 1 };
/* initial conditions, evaluated on the device at the node coordinates; params:
 *   UNIFORM        rho, v1, v2, v3, p
 *   TGV            (none) Taylor-Green vortex on [0,2pi]^3: v = (sin x cos y cos z,
 *                  -cos x sin y cos z, 0), p = p_0 + (cos 2x + cos 2y)(cos 2z + 2)/16,
 *                  rho = p/p_0
 *   VORTEX         beta, x0, y0, u_inf, v_inf: isentropic vortex (z-uniform) on the free
 *                  stream rho = p = 1
 *   DENSITY_WAVE   amp, v1, v2, v3, p, k1, k2, k3, phase: rho = 1 + amp sin(k.x + phase) */
enum { DG_IC_UNIFORM = 0, DG_IC_TGV = 1, DG_IC_VORTEX = 2, DG_IC_DENSITY_WAVE = 3 };

typedef struct dg_mesh dg_mesh;
typedef struct dg_solver dg_solver;
typedef struct dg_batch dg_batch;

/* Periodic box of ex*ey*ez hexahedra on [lo, hi]; with DG_DEFORM_SINSIN each node is moved by
 * (a sin y sin z, a sin z sin x, a sin x sin y) evaluated at its undeformed position
 * (a = deform_amp).  Uniform order n_uniform in every direction, or per-element anisotropic
 * orders orders[3 e + d] (NULL for uniform).
 * halo = 1 (uniform-order Gauss-Lobatto boxes): the box is treated as one block of a domain split
 * across GPUs whose neighbours across every box face are the block's own periodic images.  Each
 * element face on the box boundary then reads a ghost element instead of its periodic partner,
 * and every stage first exchanges the block's boundary face values: the state's face nodes (and,
 * with viscosity, the face viscous fluxes after the gradient pass; with spectral vanishing
 * viscosity, the filtered flux's components of the face's direction after its flux kernel) are
 * packed into a contiguous send buffer, moved to the receive buffer (a device copy here, the
 * inter-GPU transfer of a split run) and unpacked into the ghosts.  Results equal those of the
 * direct periodic box bit for bit.  The face metrics of the -d faces take the owner's, and the
 * ghosts' faces the Jacobian (read by the interior penalty), once, at set-up. */
typedef struct {
  int ex, ey, ez;
  double lo[3], hi[3];
  int deform;
  double deform_amp;
  int n_uniform;
  const int* orders;
  int nodes;  /* DG_NODES_LOBATTO (default) or DG_NODES_GAUSS */
  int halo;   /* 0 (default) or 1: periodic neighbours through ghost elements and a halo exchange */
} dg_box_desc;

/* face viscous flux (box of viscous fluxes in section "Spatial discretisation"), all with the
 * BR1-lifted gradient of (v, T) in the volume terms:
 *   BR1  average of the two sides' viscous fluxes with their lifted gradients;
 *   BR2  the same with each side's broken (unlifted) gradient plus visc_eta times the lift of
 *        this face's jump alone (visc_eta = 0: 2);
 *   IP   symmetric interior penalty: the same with the broken gradients, plus the penalty
 *        sigma F_v(v_mean, [g] n^) . S, sigma = visc_eta (N+1)^2 / h, h = 2 min(J_-, J_+)/|S|
 *        (visc_eta = 0: 1).
 * On Gauss-Legendre points the values on a face are traces (sum_i l_i(+-1) along the line): the
 * broken gradient's, the lift's (of g* - g(+-1), with g(+-1) the trace of the element's
 * interpolant of g, the split of BR1's weak-form gradient that Gauss quadrature makes exact),
 * U's and J's.
 * The choice is this library's reading: the paper names the three fluxes, not their constants. */
enum { DG_VISC_BR1 = 0, DG_VISC_BR2 = 1, DG_VISC_IP = 2 };

/* Spectral vanishing viscosity (section "Shock capturing"), an artificial-viscosity term added
 * to the residual when svv_mu > 0:
 *   F_a  the Navier-Stokes viscous flux with viscosity svv_mu and conductivity
 *        svv_mu gamma / ((gamma-1) Pr), written in the entropy variables w as B grad w
 *        (eq. shock:fluxmatrix), grad w the BR1 gradient;
 *   B = L^T D L  with L grad w the symmetric traceless part of Z_kj = d_j w_{k+1} + v_k d_j w_5
 *        (D = 2 svv_mu p/rho) and grad w_5 (D = kappa (p/rho)^2);
 *   filtered flux J^{-1/2} L^T D^{1/2} F*(sqrt(J D) L grad w) (eq. shock:filteredflux), F* the
 *        Legendre modal filter of each element: mode (a,b,c) times 1 - (1-s_a)(1-s_b)(1-s_c),
 *        s_k = 0 for k <= svv_cutoff, and for k above it 1 (DG_SVV_TADMOR) or
 *        exp(-((k-N)/(k-svv_cutoff))^2) (DG_SVV_MADAY);
 *   sensor: an element whose s = sum_nodes w_i w_j w_k J |grad_xi rho|^2 exceeds svv_sensor
 *        (>= 0) takes the unfiltered flux B grad w; svv_sensor < 0: no sensor;
 *   residual: the divergence of the filtered flux with BR1 face terms (average of the two
 *        sides' fluxes).
 * The paper leaves the factorisation, the 3D kernel and the sensor's use to cited works: these
 * are this library's readings.  Uniform-order Gauss-Lobatto meshes.  The filtered flux is formed
 * in FP64 in both precisions; an FP32-bulk Navier-Stokes solver adds it to its FP32 viscous flux
 * (rounded once), an FP32-bulk Euler solver adds its divergence in FP64 after the stage. */
enum { DG_SVV_TADMOR = 0, DG_SVV_MADAY = 1 };

/* Explicit LES closure (section on turbulence models, which names the Smagorinsky, WALE, Vreman
 * and SVV-Smagorinsky models and leaves their definitions to its references): with les_cs > 0
 * the artificial viscosity of the term above becomes, node by node, svv_mu + rho nu_t, the eddy
 * viscosity of model les_model with constant C = les_cs, from g = grad v of the same BR1 gradient
 * and the filter width Delta = 2 (J/(N+1)^3)^(1/3) (the cube root of the element volume per
 * node):
 *   DG_LES_SMAGORINSKY  nu_t = (C Delta)^2 |S|, S = (g + g^T)/2, |S| = sqrt(2 S:S);
 *   DG_LES_WALE         nu_t = (C Delta)^2 (Sd:Sd)^(3/2) / ((S:S)^(5/2) + (Sd:Sd)^(5/4)),
 *                       Sd = (g^2 + (g^2)^T)/2 - tr(g^2) I/3 (Nicoud and Ducros);
 *   DG_LES_VREMAN       nu_t = C sqrt(B / (g:g)), b = Delta^2 g g^T,
 *                       B = b11 b22 - b12^2 + b11 b33 - b13^2 + b22 b33 - b23^2 (Vreman);
 * each zero where its denominator vanishes, and the conductivity that viscosity times
 * gamma/((gamma-1) Pr).  Filtered by the SVV kernel, Smagorinsky's is the SVV-Smagorinsky
 * closure; with DG_SVV_TADMOR and svv_cutoff -1 (every mode kept) the plain model.  The filter
 * width and the turbulent Prandtl number (= Pr) are this library's readings.  The step-size
 * estimates count svv_mu, not the eddy viscosity. */
enum { DG_LES_SMAGORINSKY = 0, DG_LES_WALE = 1, DG_LES_VREMAN = 2 };

/* Physics of a solver.  Zero-initialise it (dg_physics p = {0}) before setting fields: every
 * option above is off or at its default when zero. */
typedef struct {
  double gamma, Pr, Ma, Re;
  int vol_flux, surf_flux, precision;
  int visc_flux;    /* DG_VISC_*; used when Re > 0 */
  double visc_eta;  /* BR2 lifting factor or interior-penalty factor; 0 = the default above */
  double svv_mu;    /* spectral vanishing viscosity: artificial viscosity, 0 = off */
  int svv_kernel;   /* DG_SVV_TADMOR or DG_SVV_MADAY */
  int svv_cutoff;   /* cutoff mode, -1..N (-1 with DG_SVV_TADMOR: no filtering) */
  double svv_sensor; /* troubled-element threshold of the density sensor; < 0: none */
  double les_cs;    /* constant of the explicit LES closure; 0 = off */
  int les_model;    /* DG_LES_SMAGORINSKY, DG_LES_WALE or DG_LES_VREMAN */
} dg_physics;

/* Diagnostics, all FP64 with Gauss-Lobatto quadrature w_i w_j w_k J, reduced in a fixed order
 * (bitwise reproducible).  entropy = integral of -rho s/(gamma-1), entropy_paper = integral
 * of -rho s (s = ln p - gamma ln rho, eq. shock:entropy); ke and enstrophy are volume means of
 * rho|v|^2/2 and rho|curl v|^2/2 (element-local derivative of v). */
typedef struct {
  double mass[5];
  double entropy_paper, entropy;
  double ke, enstrophy;
  double lambda_max, rho_min, p_min;
  double volume;
  long long nonfinite;
} dg_diag;

/* ------------------------------------------------------------------ mesh */
/* Build the host-side mesh (connectivity, per-element orders).  A mesh whose orders[] are not
 * all equal is a mixed-order mesh (section "Spatial p-adaptation": every element carries its
 * own order per direction, and faces whose two sides differ in tangential order are coupled
 * through a mortar of the larger orders; the fluxes are L2-projected back, which conserves
 * their integral).  Errors: DG_EINVAL for non-positive sizes, hi <= lo, orders outside
 * [1, 7]; DG_EUNSUPPORTED for a mixed-order mesh with an order above 6 or 2^31 nodes or
 * more. */
int dg_mesh_create_box(const dg_box_desc* d, dg_mesh** out);
void dg_mesh_destroy(dg_mesh* m);
/* n_elements, total nodes and the largest order of the mesh. */
int dg_mesh_info(const dg_mesh* m, long long* n_elements, long long* n_nodes, int* n_max);

/* ------------------------------------------------------------------ solver */
/* Create a solver for the mesh (the mesh may be destroyed afterwards).  Errors: DG_EINVAL for
 * gamma <= 1, Pr <= 0, unknown flux or precision codes; DG_EUNSUPPORTED for an order without
 * a compiled kernel (uniform orders 1..7 are compiled), for a mixed-order mesh with Re > 0
 * (mixed-order meshes are evaluated for the Euler equations, in FP64 or FP32-bulk), and for
 * DG_FP32_BULK with a volume flux other than DG_VOL_EC / DG_VOL_CENTRAL or a surface flux other
 * than DG_SURF_ROE / LLF / EC / CENTRAL.  Spectral vanishing viscosity (svv_mu > 0 or
 * les_cs > 0): DG_EINVAL for an unknown kernel or LES model, a cutoff outside [-1, N], Pr <= 0
 * or a NaN threshold; DG_EUNSUPPORTED on a mixed-order or Gauss-Legendre mesh; svv_mu or
 * les_cs < 0 or non-finite: DG_EINVAL. */
int dg_solver_create(const dg_mesh* m, const dg_physics* p, dg_solver** out);
/* Bytes of device memory the solver needs (host-only; used for admission control). */
int dg_solver_required_bytes(const dg_solver* s, size_t* bytes);
/* Hand the solver a caller-owned device buffer of at least required_bytes bytes and the HIP
 * stream (hipStream_t, NULL = default) for all its work.  Uploads the Gauss-Lobatto tables and
 * connectivity and runs the FP64 geometry kernels (node coordinates, curl-form metric terms
 * Ja^d_n, J, 1/J).  Errors: DG_ENOMEM if bytes is too small, DG_EINVAL for a NULL pointer,
 * DG_ESTATE if already bound, DG_EHIP on a HIP failure. */
int dg_solver_bind(dg_solver* s, void* dev_ptr, size_t bytes, void* hip_stream);
/* Evaluate an initial condition on the device; params as listed at DG_IC_*.  Resets the RK
 * register. */
int dg_set_initial_condition(dg_solver* s, int ic, const double* params);
/* Copy a host state (n = 5 * total nodes doubles, layout above) to the device.  Resets the RK
 * register.  DG_ENONFINITE if any value is non-finite or rho or p is not positive (the device
 * state is then left unchanged). */
int dg_set_state(dg_solver* s, const double* host_U, size_t n);
/* Copy the current state to the host (synchronises the stream). */
int dg_get_state(const dg_solver* s, double* host_U, size_t n);
/* R = dU/dt of the current state.  R stays on the device; if host_R is not NULL it is also
 * copied there (n doubles, layout above; synchronises). */
int dg_residual(dg_solver* s, double* host_R, size_t n);
/* Advance nsteps steps of the solver's low-storage explicit Runge-Kutta scheme (section "Time
 * advancement") with the fixed step dt: per stage k, dU <- A_k dU + dt R(U); U <- U + B_k dU.
 * Default: Williamson's RK3, A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15); see
 * dg_solver_set_scheme.  Only enqueues work on the solver's stream. */
int dg_rk_step(dg_solver* s, double dt, int nsteps);
/* Advance nsteps steps of the solver's scheme with a step size chosen before every step from the
 * state it starts from, on the device: dt = cfl h_min/((N+1)^2 lambda_max), lambda_max the largest
 * |v| + c over the nodes, and with viscosity at most 0.25 h_min^2 Pr rho_min/((N+1)^4 gamma mu)
 * (mu = 1/Re plus svv_mu) --
 * dg_suggest_dt's formula, so a step equals dg_rk_step with dg_suggest_dt(cfl) of the same state,
 * bit for bit.  A max/min reduction and a one-block kernel compute dt, and the stage kernels read
 * it from device memory, so the steps need no host round trip (and replay one captured graph).
 * The paper does not state how the step is chosen; the formula is this library's reading.
 * t_advanced (may be NULL) receives the simulated time advanced.  Synchronises the stream once,
 * at the end.  DG_EINVAL for cfl <= 0 or nsteps < 0; DG_ENONFINITE if a step started from a
 * non-finite or non-physical state (that step and the later ones then had size 0). */
int dg_rk_step_adaptive(dg_solver* s, double cfl, int nsteps, double* t_advanced);
/* Time schemes: Williamson's three-stage RK3 (the default), or Carpenter and Kennedy's five-stage
 * fourth-order low-storage scheme (the paper's RK4 option; their published coefficients). */
enum { DG_RK3_WILLIAMSON = 0, DG_RK4_CARPENTER_KENNEDY = 1 };
/* Select the scheme of dg_rk_step (and of batches the solver joins: all members of a batch must
 * use one scheme).  Errors: DG_EINVAL for an unknown scheme. */
int dg_solver_set_scheme(dg_solver* s, int scheme);
/* Graph replay of RK steps (on by default).  When dg_rk_step runs several steps, or the same
 * dt as its previous call, the launches of one step, and of 8 steps while at least 8 remain,
 * are captured once per starting state buffer into HIP graphs (on a stream the library owns;
 * no memory operations are recorded) and replayed on the solver's stream; the results equal
 * those of eager launches bit for bit.  Graphs are dropped when the state or its FP32
 * reference changes, after dg_autotune and when disabled; steps inside a profile region run
 * eagerly.  enable = 0 disables replay. */
int dg_solver_use_graphs(dg_solver* s, int enable);
/* Mixed-order meshes: the stage runs one launch per bucket of elements with 64 b < nodes <=
 * 64 (b + 1), b = 0..5 (a bucket of fewer than 2048 elements joins the launch of the next larger
 * one), one node per lane, or two nodes per lane when bit b of the tile mask is set.  dg_autotune times both shapes of every occupied bucket on the current state (residual
 * mode, five launches each) and keeps the faster; *tiles receives the mask and *us the summed
 * launch time of the chosen shapes in microseconds (either pointer may be NULL).  The residual
 * buffer is overwritten; the state is not changed.  Uniform-order meshes have one launch shape:
 * *tiles = 0, *us = 0.  Synchronises. */
int dg_autotune(dg_solver* s, int* tiles, double* us);
/* Set the tile mask by hand (default 0).  The result does not depend on it: every node's sums
 * are taken in the same order with either shape.  Uniform-order meshes accept only 0.
 * Errors: DG_EINVAL for a value outside [0, 63]. */
int dg_solver_set_tiles(dg_solver* s, int tiles);
/* Diagnostics of the current state (synchronises). */
int dg_diagnostics(dg_solver* s, dg_diag* out);
/* For callers that cannot allocate (code under HIP graph capture, tight serving loops): the
 * diagnostics of dg_diagnostics, written as a dg_diag record to the device memory dev_out
 * (112 bytes, caller-owned, 8-byte aligned, on the solver's device), enqueued on the solver's stream
 * without synchronising; the values equal dg_diagnostics's bit for bit.  The per-element partial
 * sums live in a static device array of the library (4.2 MB per device, held until the process
 * ends), so the call allocates no memory of any kind.  That array limits the mesh to 32768
 * elements: larger meshes get DG_EUNSUPPORTED.  Calls on one device share the array: calls whose
 * work overlaps on one device (e.g. on two streams) race and must be ordered by the caller.
 * Errors: DG_EINVAL for a NULL output, DG_ESTATE for an unbound solver, DG_EHIP on a HIP failure. */
int dg_diagnostics_noalloc(dg_solver* s, dg_diag* dev_out);
/* dt = cfl h_min / ((N_max+1)^2 lambda_max), and with viscosity the smaller of that and
 * 0.25 h_min^2 / ((N_max+1)^4 gamma mu / (Pr rho_min)), mu = 1/Re plus svv_mu; h_min = smallest
 * undeformed element edge; lambda_max, rho_min from dg_diagnostics of the current state. */
int dg_suggest_dt(dg_solver* s, double cfl, double* dt);
/* Copy the geometry to the host: X (3 per node, layout [off*3 + c*nn + node]), Ja (9 per
 * node, [off*9 + (3 d + c)*nn + node] = component c of Ja^d), J (1 per node).  Any pointer may
 * be NULL.  Synchronises. */
int dg_get_geometry(dg_solver* s, double* host_X, double* host_Ja, double* host_J);
/* Device addresses of the current state and of the last residual (valid until the next
 * dg_rk_step, which moves the state between two buffers). */
int dg_device_pointers(dg_solver* s, void** dev_U, void** dev_R);
/* Wait for all work enqueued by the solver. */
int dg_synchronize(dg_solver* s);

/* Kernel timing.  Between dg_profile_begin and dg_profile_end every kernel the solver launches
 * is bracketed by two HIP events recorded on the solver's stream; dg_profile_end synchronises
 * and returns, per kernel class, the summed elapsed milliseconds and the number of launches.
 * Classes: DG_K_GRADIENT (Navier-Stokes pass computing the BR1 gradient and face viscous
 * fluxes), DG_K_STAGE (residual + RK update), DG_K_DIAGNOSTICS, DG_K_OTHER (geometry, initial
 * condition).  Recording adds the event overhead to the timed region. */
enum { DG_K_GRADIENT = 0, DG_K_STAGE = 1, DG_K_DIAGNOSTICS = 2, DG_K_OTHER = 3, DG_K_CLASSES = 4 };
typedef struct {
  double ms[DG_K_CLASSES];
  long long launches[DG_K_CLASSES];
} dg_profile;
int dg_profile_begin(dg_solver* s);
int dg_profile_end(dg_solver* s, dg_profile* out);
void dg_solver_destroy(dg_solver* s);

/* ------------------------------------------------------------------ batches
 * Independent solvers advanced together (ensembles, parameter sweeps, the solves admitted by a
 * serving loop).  Members of one polynomial order and precision (and all viscous or all
 * inviscid) are advanced by one launch per kernel and stage that covers the elements of all of
 * them (at most 32 members per launch), so that many small solves fill the GPU together;
 * mixed-order, Gauss-Legendre and spectral-vanishing-viscosity members are launched one by one.  Each member keeps its own state, step size and
 * buffer parity; the result of a member is bitwise the same as when it is stepped alone.
 *
 * Create a batch of n bound solvers whose steps are enqueued on hip_stream (hipStream_t, NULL =
 * default).  The members may be bound to other streams: the caller orders the batch's steps
 * after the work the members have pending there (e.g. by synchronising those streams) and does
 * not use a member on its own stream while batch steps are pending.  The solvers stay owned by
 * the caller and must outlive the batch.  Errors: DG_EINVAL for NULL, n < 1 or a repeated
 * member or members with different time schemes; DG_ESTATE for an unbound member. */
int dg_batch_create(dg_solver* const* solvers, int n, void* hip_stream, dg_batch** out);
/* Advance every member nsteps steps of the members' scheme, member i with step dts[i] (n
 * doubles).  Only enqueues work on the batch's stream.  Like dg_rk_step, the launches of one
 * step (and of 8 steps while at least 8 remain) are captured into HIP graphs and replayed when
 * several steps are taken or the same dts recur (a few graphs are kept, keyed by dts, the step
 * count and the members' buffer parities). */
int dg_batch_rk_step(dg_batch* b, const double* dts, int nsteps);
/* enable = 0 disables graph replay of the batch (and drops its graphs). */
int dg_batch_use_graphs(dg_batch* b, int enable);
/* Kernel launches per RK stage of the batch (the one-launch-per-group structure made visible):
 * one per batched group (two with viscous terms), plus one for each mixed-order or
 * Gauss-Legendre member, which runs its own launches within the batch's stages. */
int dg_batch_launches(const dg_batch* b, int* launches_per_stage);
void dg_batch_destroy(dg_batch* b);

/* Message of the last failure on the calling thread ("" if none). */
const char* dg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DGSEM_H */
