/*
 * dgsem_oracle.h -- plain CPU oracle for the DGSEM residual and its low-storage RK3 update.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct reference against
 * which the HIP path is checked.  Only tests/, __graft_entry__.smoke() and the cpu_baseline
 * leg of bench.py may load it.  It shares no code, header, table or helper with the HIP path.
 *
 * What it computes (HORSES3D paper, section "Numerical methods"):
 *   u_t + div F_e = div F_v          (eq. compressibleNScompact, viscous fluxes eq. viscousfluxes)
 * transformed to curvilinear hexahedra (eq. compressibleNScompact_transformed), discretised by
 * the Gauss-Lobatto DGSEM weak form (eqs. NS2-NS4) in its SBP strong form, with the
 * entropy-conserving split-form volume term (section "Energy/Entropy stable versions"), a
 * Riemann flux at faces (box listing convective fluxes), BR1 viscous terms, and Williamson's
 * low-storage RK3 (section "Time advancement").
 *
 * Every floating-point operation is done in the type `real`: double for liborc64.so, long
 * double (x87 80-bit) for liborc80.so, built from the same source.  The fp80 build exists only
 * to measure the fp64 build's own rounding error; all arrays crossing the ABI are double.
 *
 * Layout of every per-node array: element-major, then field, then node (i fastest):
 *   U[off_e*5 + v*nn_e + i + n1*(j + n2*k)]
 * Error handling: functions return 0 on success, negative on invalid input.
 */
#ifndef DGSEM_ORACLE_H
#define DGSEM_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NMAX 8

enum { ORC_VOL_EC = 0, ORC_VOL_CENTRAL = 1, ORC_VOL_IR = 2, ORC_VOL_KG = 3, ORC_VOL_PIROZZOLI = 4,
       ORC_VOL_DUCROS = 5, ORC_VOL_MORINISHI = 6 };
enum { ORC_SURF_ROE = 0, ORC_SURF_LLF = 1, ORC_SURF_EC = 2, ORC_SURF_CENTRAL = 3, ORC_SURF_ES = 4, ORC_SURF_IR = 5,
       ORC_SURF_ES_MATRIX = 6, ORC_SURF_LOW_DISS_ROE = 7, ORC_SURF_LF_GLOBAL = 8 };
enum { ORC_VISC_BR1 = 0, ORC_VISC_BR2 = 1, ORC_VISC_IP = 2 };
enum { ORC_SVV_TADMOR = 0, ORC_SVV_MADAY = 1 };
enum { ORC_IC_UNIFORM = 0, ORC_IC_TGV = 1, ORC_IC_VORTEX = 2, ORC_IC_DENSITY_WAVE = 3 };

typedef struct orc_solver orc_solver;

/* Gauss-Lobatto nodes xi[N+1], weights w[N+1] and derivative matrix D[(N+1)*(N+1)] (row-major). */
int orc_gll(int N, double* xi, double* w, double* D);
/* Gauss-Legendre points xi[N+1], weights w, derivative matrix D (row-major) and the Lagrange
 * basis at the ends, lb[0..N] at xi = -1 and lb[N+1..2N+1] at xi = +1. */
int orc_gl(int N, double* xi, double* w, double* D, double* lb);

/* Mortar operators: I[(M+1)x(N+1)] interpolates order N to order M Lobatto nodes;
 * P[(N+1)x(M+1)] is the exactly integrated L2 projection from order M back to order N. */
int orc_mortar_matrices(int N, int M, double* I, double* P);

/* Periodic box of ex*ey*ez hexahedra on [lo,hi]; deform=1 applies the sin*sin displacement of
 * amplitude amp to every node.  orders: 3*E ints (N1,N2,N3) per element, or NULL for n_uniform. */
orc_solver* orc_create(int ex, int ey, int ez, const double* lo, const double* hi, int deform,
                       double amp, int n_uniform, const int* orders, double gamma, double Pr,
                       double Ma, double Re, int vol_flux, int surf_flux);
/* The same box (uniform order N, optionally deformed) on Gauss-Legendre nodes: plain (non-split)
 * weak form, face traces interpolated to the element boundaries; Re > 0 adds viscous terms (BR1,
 * or BR2 / the interior penalty through orc_set_viscous_flux).  The map and its metric terms are
 * the Lobatto grid's, evaluated at the Gauss points. */
orc_solver* orc_create_gauss(int ex, int ey, int ez, const double* lo, const double* hi, int deform, double amp,
                             int N, double gamma, double Pr, double Ma, double Re, int surf_flux);
void orc_destroy(orc_solver* s);
/* Face viscous flux: BR1 (default), BR2 with lifting factor eta, or the symmetric interior
 * penalty with penalty factor eta (sigma = eta (N+1)^2 / h); eta = 0 takes 2 (BR2), 1 (IP). */
int orc_set_viscous_flux(orc_solver* s, int kind, double eta);
/* Gauss-Legendre meshes: the broken gradient of g = (v, T) and the sum of its six face lifts at
 * every node (layout of orc_gradients), whose sum is the BR1 gradient; and (Navier-Stokes) the
 * face viscous flux of the current state, F[((e*6 + f)*5 + v)*nf + q], f = 2 d + side. */
int orc_gauss_gradient_parts(const orc_solver* s, double* Gb, double* Gl);
int orc_gauss_face_viscous(orc_solver* s, double* F);
long orc_num_nodes(const orc_solver* s);
int orc_num_elements(const orc_solver* s);
int orc_elem_info(const orc_solver* s, int e, int* n3, long* off);
void orc_set_threads(int n);

int orc_get_coords(const orc_solver* s, double* X);           /* [off*3 + n*nn + node]       */
int orc_get_metrics(const orc_solver* s, double* Ja, double* J); /* Ja[off*9+(3d+n)*nn+node] */
int orc_set_ic(orc_solver* s, int ic, const double* params);
int orc_set_state(orc_solver* s, const double* U);
int orc_get_state(const orc_solver* s, double* U);
int orc_residual(orc_solver* s, double* R);                   /* R = dU/dt of current state  */
int orc_gradients(orc_solver* s, double* G);                  /* BR1 lifted grad of (v,T)    */
int orc_rk3(orc_solver* s, double dt, int nsteps);
int orc_rk(orc_solver* s, int scheme, double dt, int nsteps); /* 0 = Williamson RK3, 1 = CK RK4 */
double orc_suggest_dt(const orc_solver* s, double cfl);
int orc_diagnostics(const orc_solver* s, double* out);        /* 14 doubles, see .c          */
double orc_entropy_production(const orc_solver* s, const double* R); /* sum wJ w(U).R      */

/* Point functions (pins). U,F: 5 doubles; n: 3 doubles. */
int orc_euler_flux(const double* U, const double* n, double gamma, double* F);
int orc_two_point_ec(const double* UL, const double* UR, const double* n, double gamma, double* F);
int orc_two_point_ir(const double* UL, const double* UR, const double* n, double gamma, double* F);
int orc_two_point_central(const double* UL, const double* UR, const double* n, double gamma, double* F);
int orc_two_point(int vol_kind, const double* UL, const double* UR, const double* n, double gamma, double* F);
int orc_riemann(int kind, const double* UL, const double* UR, const double* S, double gamma, double* F);
/* Lax-Friedrichs with a given (global) wave speed lam. */
int orc_lax_friedrichs(const double* UL, const double* UR, const double* S, double gamma, double lam, double* F);
int orc_roe_waves(const double* UL, const double* UR, const double* nhat, double gamma, int absval,
                  double* W);
int orc_entropy_vars(const double* U, double gamma, double* w);
double orc_entropy(const double* U, double gamma);            /* -rho s/(gamma-1)            */
double orc_logmean(double a, double b);
int orc_viscous_flux(const double* U, const double* grad, double gamma, double Pr, double Re,
                     double* Fv);                             /* Fv[n*5+v], 3 directions      */

/* Spectral vanishing viscosity (section "Shock capturing"): the Navier-Stokes viscous flux with
 * viscosity mu_a (conductivity from Pr) in entropy variables, half-filtered in the Legendre modal
 * space by Tadmor's or Maday's kernel with cutoff mode M (-1..N), and unfiltered in elements whose
 * density sensor exceeds sensor_threshold (< 0: no sensor).  Added to the residual of Lobatto
 * solvers with conforming faces; mu_a = 0 switches it off. */
int orc_set_svv(orc_solver* s, double mu_a, int kernel, int cutoff, double sensor_threshold);
/* explicit LES closure: the artificial viscosity of the SVV term gains the eddy viscosity
 * rho nu_t of the model (Smagorinsky, WALE or Vreman; constant cs) node by node; cs = 0: off.
 * Set before orc_set_svv. */
enum { ORC_LES_SMAGORINSKY = 0, ORC_LES_WALE = 1, ORC_LES_VREMAN = 2 };
int orc_set_les(orc_solver* s, int model, double cs);
int orc_les_viscosity(const double* U, const double* Gw, double gamma, int model, double cs, double J, int n,
                      double* mu);
int orc_les_flux(const double* U, const double* Gw, double gamma, double Pr, double mu_a, int model, double cs,
                 double J, int n, double* F);
int orc_svv_residual(orc_solver* s, double* Ra, double* form); /* SVV part alone; entropy form */
int orc_svv_sensor(orc_solver* s, double* sens);              /* s_rho of every element       */
int orc_svv_filter(int N, int kernel, int cutoff, const double* f, double* out); /* one field */
int orc_svv_flux(const double* U, const double* Gw, double gamma, double Pr, double mu_a,
                 double* F);                                  /* unfiltered L^T D L G, F[5x+v] */

#ifdef __cplusplus
}
#endif
#endif
