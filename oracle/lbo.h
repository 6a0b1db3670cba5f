/*
 * lbo.h -- C interface of the reference oracle (TEST INFRASTRUCTURE ONLY).
 *
 * A plain, serial, FP64 CPU implementation of one time step of the LBsoft
 * two-component lattice-BGK fluid coupled to rigid colloidal spheres
 * (Bonaccorso et al., "LBsoft: a parallel open-source software for simulation
 * of colloidal systems", Sec. 2 and the eight-step sequence of Sec. 3.1).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library. It shares no code, header, table or
 * constant with the HIP implementation and must never be used as a fallback
 * for it.
 *
 * Conventions
 *   node index       n = x + nx*(y + ny*z)
 *   populations      [k][i][n] (component, oracle direction order, node), FP64,
 *                    full values f_i (not deviations); solid nodes hold 0
 *   direction order  the oracle's own, returned by lbo_lattice()
 *   owner map        0 = fluid, p+1 = solid node of particle p, -1 = wall
 */
#ifndef LBO_H
#define LBO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBO_OK = 0,
  LBO_E_ARG = -1,      /* invalid parameter                                   */
  LBO_E_SPEED = -6     /* a particle moved more than half a node in one step  */
};

typedef struct lbo_params {
  int32_t nx, ny, nz;
  int32_t walls;            /* 0: periodic in z; 1: solid layers z=0 and z=nz-1 */
  double  wall_u_lo[3];     /* velocity of the z=0 wall layer                   */
  double  wall_u_hi[3];     /* velocity of the z=nz-1 wall layer                */
  int32_t ncomp;            /* 1 or 2 fluid components                          */
  double  tau[2];           /* BGK relaxation times                             */
  double  G;                /* Shan-Chen inter-component coupling               */
  double  sc_norm;          /* stencil normalisation of the Shan-Chen sum       */
  double  g[3];             /* body acceleration (force density rho_k * g)      */
  double  radius;           /* sphere radius R                                  */
  double  particle_density; /* mass m = density * 4/3 pi R^3                    */
  double  hertz_K, hertz_d0, hertz_rcap;
  double  zeta[2];          /* wetting constants of the virtual solid density   */
  double  rho_fallback[2];  /* density of a created node with no fluid neighbour */
  int32_t rotate;           /* integrate the rotational degrees of freedom      */
  int32_t particles_fixed;  /* spheres are static obstacles: no map updates,
                               no pair forces, no integration                  */
  /* Janus wetting (Sec. 4, benchmark input): on a sphere's frontier node at
   * angle theta (degrees) from the sphere's body x axis, zeta_k of Eq.
   * soliddens is +janus_zeta[0] S(theta) for component A and
   * -janus_zeta[1] S(theta) for B, with the switching function S going
   * smoothly from +1 (theta <= theta0 - width/2) to -1 (theta >= theta0 +
   * width/2). janus = 0 keeps the constant zeta[k]. */
  int32_t janus;
  double  janus_theta0, janus_width, janus_zeta[2];
  /* Lubrication between sphere pairs (Eq. libric), lub_mu > 0 switches it on:
   * F_i = -6 pi lub_mu R^2/4 (1/h - 1/lub_hn) ((v_i - v_j) . r_ij/|r_ij|) r_ij/|r_ij|
   * for gaps h = |r_ij| - 2R below lub_hn, with h held at lub_hcap below it. */
  double  lub_mu, lub_hn, lub_hcap;
  /* Boundary type of the two z faces (walls = 1), [0] at z = 0, [1] at
   * z = nz-1 (Sec. 2.2, Eq. bb, bbv, bbp and the input directive "bound open"):
   *   0 moving wall: Eq. bbv with the local density and wall_u_lo/hi;
   *   1 pressure (Dirichlet): anti-bounce-back Eq. bbp with the density
   *     wall_rho[face][k] and the velocity extrapolated from the fluid;
   *   2 velocity (Neumann): Eq. bbv with wall_u_lo/hi and the density
   *     extrapolated from the fluid;
   *   3 equilibrium: f_eq(wall_rho[face][k], wall_u) enters from the face.
   * Extrapolation to the face: X_w = X(r_b) + (X(r_b) - X(r_b+1)) / 2 with
   * r_b the fluid node next to the face and r_b+1 the next one inwards. */
  int32_t wall_type[2];
  double  wall_rho[2][2];
} lbo_params;

/* per-particle record returned by lbo_get_particles, in this order */
#define LBO_PREC 50
/*  0 x[3]  3 v[3] (t-1/2)  6 w[3] (t-1/2)  9 q[4]
 * 13 Fliq_prev[3]  16 Tliq_prev[3]
 * last completed step:  19 Fd[3] 22 Td[3] 25 Fc[3] 28 Tc[3] 31 FH[3]
 *                       34 FSC[3] 37 TSC[3] 40 Fliq[3] 43 Tliq[3]
 * 46 sum over links of |F_link|   47 mass  48 inertia
 * 49 1 when Fliq_prev/Tliq_prev hold a previous half-step value, else 0 */

/* observables, lbo_observables() */
#define LBO_NOBS 36
/*  0 mass A   1 mass B   2..4 bare fluid momentum sum_k j_k
 *  5 rho min A  6 rho min B  7 rho max A  8 rho max B  9 max |u|
 * 10 fluid node count  11..13 particle momentum  14 particle KE (transl.)
 * 15 particle KE (rot.)
 * ledger of the last completed step:
 * 16,17 mass removed by destroyed nodes (A,B)  18,19 mass added by created nodes
 * 20,21 mass change from the moving-link corrections (A,B)
 * 22..24 body force sum_n sum_k rho_k g on the fluid nodes after the map update
 * 25..27 Shan-Chen force summed over fluid nodes
 * 28..30 link force sum_links F_link over wall links   31 step counter
 * 32..34 physical fluid momentum sum_fluid sum_k (j_k + F_k / 2), F_k the
 *        Shan-Chen plus body force density of the current state
 * 35     sum over spheres and links of |F_link| of the last step */

void*   lbo_create(const lbo_params* p, const double* rho0 /* [ncomp][N] */,
                   const double* u0 /* [N][3] or NULL */);
void    lbo_destroy(void* s);
int     lbo_add_particles(void* s, int32_t n, const double* x, const double* v,
                          const double* w, const double* q);
int     lbo_step(void* s, int32_t nsteps);
void    lbo_lattice(int32_t* c /* [19][3] */, double* w /* [19] */);
void    lbo_get_f(const void* s, double* f);
void    lbo_set_f(void* s, const double* f);
void    lbo_get_rho(const void* s, double* rho /* [ncomp][N] */);
/* pseudo-potential of the current state: rho_k on fluid nodes, the virtual
 * densities of Eq. soliddens on frontier solid nodes, 0 elsewhere */
void    lbo_get_psi(const void* s, double* psi /* [ncomp][N] */);
void    lbo_get_u(const void* s, double* u /* [N][3] */);
void    lbo_get_owner(const void* s, int32_t* owner);
void    lbo_set_owner(void* s, const int32_t* owner);
int32_t lbo_num_particles(const void* s);
void    lbo_get_particles(const void* s, double* out /* [P][LBO_PREC] */);
void    lbo_set_particle_state(void* s, const double* in /* [P][LBO_PREC] */);
void    lbo_observables(const void* s, double* out /* [LBO_NOBS] */);
double  lbo_loss(const void* s);

/* Test hook: apply nsteps of the rotational update to q at constant w. */
void    lbo_test_rotate(double* q /* [4] */, const double* w /* [3] */, int32_t nsteps);

/* Forward-mode (dual number) run from the initial state f = f_eq(rho0, 0):
 * returns L after nsteps and the directional derivative
 *   dL = dL/dG * dG + dL/dg . dg + sum_n dL/drho0_A(n) * drhoA(n).
 * Particles (optional) are static obstacles; requires particles_fixed = 1
 * when np > 0. */
int     lbo_loss_tangent(const lbo_params* p, const double* rho0, int32_t np,
                         const double* x, int32_t nsteps, double dG,
                         const double* dg /* [3] */, const double* drhoA /* [N] or NULL */,
                         double* L, double* dL);

/* Forward-mode run as lbo_loss_tangent, returning instead the pseudo-potential
 * psi_k(n) of the final state (as lbo_get_psi) and its directional derivative
 * dpsi_k(n), both [ncomp][N]: the tangent-linear map of the whole run applied
 * to (dG, dg, drhoA). */
int     lbo_psi_tangent(const lbo_params* p, const double* rho0, int32_t np,
                        const double* x, int32_t nsteps, double dG,
                        const double* dg /* [3] */, const double* drhoA /* [N] or NULL */,
                        double* psi, double* dpsi);

#ifdef __cplusplus
}
#endif
#endif
