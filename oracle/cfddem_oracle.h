/*
 * cfddem_oracle.h -- plain FP64 CPU oracle for the particle-side hot path of
 * unresolved CFD-DEM as defined in El Geitani, Golshan & Blais, "Towards
 * High-Order CFD-DEM: Development and Validation" (arXiv 2211.01185).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no source, header, table or helper with the HIP library.
 *
 * Conventions: SI units, FP64 everywhere.  Per-particle vectors are stored
 * component-major ("SoA"): x[c*n + i] is component c of particle i.  Particle
 * identity is the array index given at creation; it never changes.
 *
 * What pins each routine (and what stays unpinned) is stated at the top of
 * cfddem_oracle.c.
 */
#ifndef CFDDEM_ORACLE_H
#define CFDDEM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Error flags (bitwise OR, sticky inside an orc_dem). */
#define ORC_OK 0
#define ORC_ERR_DOMAIN 1 /* a particle centre left the box [lo, hi] */
#define ORC_ERR_NAN 2    /* a NaN appeared in the state */

/* DEM parameters (Section 2.2, Table "tab:viscoelastic"). */
typedef struct {
  double box_lo[3], box_hi[3]; /* six planar walls of the container */
  double gravity[3];
  double dt;                   /* DEM time step */
  double E, nu, e, mu;         /* particle-particle: Young, Poisson, restitution, Coulomb */
  double E_w, nu_w, e_w, mu_w; /* particle-wall: wall Young, wall Poisson, restitution, Coulomb */
  double mu_r, mu_r_w;         /* rolling friction, particle-particle and particle-wall (0: none) */
} orc_params;

/* Fluid / mesh parameters of the coupling (Section 2.3).  The structured hex
 * mesh spans the DEM box. */
typedef struct {
  int order;      /* velocity element order: 1 (Q1-Q1) or 2 (Q2-Q1) */
  int n_el[3];    /* elements per axis */
  double rho_f;   /* fluid density */
  double mu_f;    /* fluid DYNAMIC viscosity (Pa s) */
  int model;      /* 0 = VANS model A, 1 = model B */
  double eps_min; /* lower clamp of the void fraction seen by the drag closure */
  int drag;       /* ORC_DRAG_*: closure of the momentum-exchange coefficient */
  int beta_over_eps; /* 1: beta_B = beta_A / eps (Eq. "beta"), 0: the same beta for both models */
  int shear;      /* 1: shear force -V_p div(tau_f) on the particles (Eqs. "fa", "fb") */
} orc_fluid;

/* Drag closures of Section 2.3.2. */
#define ORC_DRAG_DIFELICE 0
#define ORC_DRAG_DALLAVALLE 1
#define ORC_DRAG_RONG 2
#define ORC_DRAG_KOCH_HILL 3
#define ORC_DRAG_BEETSTRA 4
#define ORC_DRAG_GIDASPOW 5

typedef struct orc_dem orc_dem;

/* Threads of the parallel loops (OpenMP; 1 when built without it).  Results
 * are bit-identical for every thread count: only independent per-particle,
 * per-contact and per-element work runs in parallel, and every sum is then
 * accumulated by one thread in the serial order. */
void orc_set_threads(int n);
int orc_get_threads(void);

/* ---- stand-alone building blocks (also used by the whole-step routines) ---- */

/* Hierarchical binning: element index e_a = clamp(floor((x_a-lo_a)*inv_he_a)),
 * then sub-cell s_a = clamp(floor((x_a-(lo_a+e_a*he_a))*inv_hc_a), 0, k_a-1).
 * he_a = (hi_a-lo_a)/n_el_a, inv_he_a = n_el_a/(hi_a-lo_a),
 * inv_hc_a = (k_a*n_el_a)/(hi_a-lo_a).  Linear element index
 * (ez*ney+ey)*nex+ex; linear cell index elem*(kx*ky*kz)+(sz*ky+sy)*kx+sx.
 * Returns the number of particles outside [lo, hi]. */
long orc_bin(long n, const double *x, const double lo[3], const double hi[3],
             const int n_el[3], const int k[3], int *elem, long *cell);

/* All contacting pairs (i<j) at positions x: (R_i+R_j)^2 - |x_j-x_i|^2 > 0,
 * found with a linked cell list.  Writes up to cap pairs sorted by (i,j) and
 * returns the total count. */
long orc_find_pairs(long n, const double *x, const double *r, const double lo[3],
                    const double hi[3], long cap, long *pi, long *pj);

/* Lagrange shape function k of order p (nodes equispaced on [0,1]) and its
 * derivative, at t. */
double orc_lagrange(int p, int k, double t);
double orc_lagrange_deriv(int p, int k, double t);

/* Interpolate the nodal velocity (Q_order) and the Q1 pressure gradient at n
 * points.  U is 3 x n_v (component-major), P is n_p.  Outputs are 3 x n. */
void orc_interpolate(const orc_fluid *f, const double lo[3], const double hi[3], long n,
                     const double *x, const double *U, const double *P, double *u_out,
                     double *gradp_out);

/* Di Felice momentum-exchange coefficient of one particle:
 * beta_p = 0.5 rho_f C_D pi r^2 |slip|. */
double orc_difelice_beta(double rho_f, double mu_f, double eps, double d, double slip);

/* Momentum-exchange coefficient beta_p of one particle (f_D = beta_p slip)
 * for closure `drag` (ORC_DRAG_*) at fluid fraction eps, diameter d and slip
 * speed |slip| >= 0; finite limits at zero slip.  Returns NaN for an unknown
 * closure. */
double orc_drag_beta(int drag, double rho_f, double mu_f, double eps, double d, double slip);
/* Second derivative of Lagrange polynomial k of degree p on nodes m/p. */
double orc_lagrange_deriv2(int p, int k, double t);
/* div(tau_f) of Eq. "stress" at each of n points x (3 x n) from the nodal
 * velocities U (3 x n_v); out: 3 x n. */
void orc_stress_divergence(const orc_fluid *f, const double lo[3], const double hi[3], long n,
                           const double *x, const double *U, double *out);

/* ---- whole-step routines ---- */

/* Copies the initial state and "primes" the stored contact force/torque with
 * one contact evaluation at the initial state with zero tangential overlap. */
orc_dem *orc_dem_create(const orc_params *p, long n, const double *x, const double *v,
                        const double *w, const double *r, const double *rho);
int orc_dem_step(orc_dem *s, long nsteps);
int orc_dem_couple(orc_dem *s, const orc_fluid *f, const double *U, const double *P,
                   double *eps_q, double *beta_q, double *fpf_q, double *elem_sums);
/* The same with a continuous void-fraction field: eps_nodes holds its values
 * at the velocity nodes (the smoothed projection of the element PCM values);
 * the closure sees it interpolated at each particle and eps_q is its value
 * at each quadrature point.  eps_nodes = NULL is orc_dem_couple. */
int orc_dem_couple_field(orc_dem *s, const orc_fluid *f, const double *U, const double *P,
                         const double *eps_nodes, double *eps_q, double *beta_q, double *fpf_q,
                         double *elem_sums);
void orc_dem_get(const orc_dem *s, double *x, double *v, double *w, double *ffp,
                 double *Fc, double *Tc);
void orc_dem_set_ffp(orc_dem *s, const double *ffp);
long orc_dem_ncontacts(const orc_dem *s);
/* Contacts of the last evaluation, sorted by (i, j); j = -1-w for wall w
 * (w = 0..5: x-lo, x-hi, y-lo, y-hi, z-lo, z-hi).  dt is 3 x count, AoS. */
void orc_dem_contacts(const orc_dem *s, long *i, long *j, double *dt);
int orc_dem_error(const orc_dem *s);
void orc_dem_free(orc_dem *s);

#ifdef __cplusplus
}
#endif
#endif
