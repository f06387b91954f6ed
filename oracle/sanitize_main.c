/*
 * sanitize_main.c -- exercises every entry point of the CPU oracle on small
 * beds, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py compiles it together with cfddem_oracle.c
 * with gcc -fsanitize=address,undefined and runs it).  TEST INFRASTRUCTURE
 * ONLY, like the oracle itself.
 *
 * The beds are generated here from a fixed linear congruential sequence (no
 * method arithmetic): a slightly compressed cubic lattice with random
 * velocities and spins, so that pairs, walls, history and sliding all occur,
 * and a sparse random bed; both are coupled with every drag closure, both
 * models, the shear force and a nodal void-fraction field.  Exit status 0
 * when every call returned without error.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "cfddem_oracle.h"

static unsigned long long lcg_state = 0x2211011850ULL;
static double unit(void) {
  lcg_state = lcg_state * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

/* n_side^3 spheres of diameter d on a cubic lattice of spacing f*d in a box
 * whose walls overlap the outer layers by 1 um (when jitter j is zero), the
 * interior jittered by +-j. */
static long lattice(int n_side, double d, double f, double j, double *x, double *lo, double *hi) {
  const long n = (long)n_side * n_side * n_side;
  const double s = f * d, o = 0.5 * d - 1e-6;
  for (int c = 0; c < 3; ++c) {
    lo[c] = 0.0;
    hi[c] = 2.0 * o + (n_side - 1) * s;
  }
  long m = 0;
  for (int k = 0; k < n_side; ++k)
    for (int jy = 0; jy < n_side; ++jy)
      for (int i = 0; i < n_side; ++i) {
        const int g[3] = {i, jy, k};
        for (int c = 0; c < 3; ++c) {
          const int inner = g[c] > 0 && g[c] < n_side - 1;
          x[c * n + m] = o + g[c] * s + (inner ? j * (2.0 * unit() - 1.0) : 0.0);
        }
        ++m;
      }
  return n;
}

static int run_bed(long n, const double *x, double d, const double lo[3], const double hi[3], int order,
                   const int n_el[3], int spins) {
  int bad = 0;
  double *v = malloc(sizeof(double) * 3 * n), *w = malloc(sizeof(double) * 3 * n);
  double *r = malloc(sizeof(double) * n), *rho = malloc(sizeof(double) * n);
  for (long i = 0; i < n; ++i) {
    r[i] = 0.5 * d;
    rho[i] = 2500.0;
    for (int c = 0; c < 3; ++c) {
      v[c * n + i] = 0.05 * (2.0 * unit() - 1.0);
      w[c * n + i] = spins ? 20.0 * (2.0 * unit() - 1.0) : 0.0;
    }
  }
  orc_params p = {{lo[0], lo[1], lo[2]}, {hi[0], hi[1], hi[2]}, {0.0, 0.0, -9.81}, 1e-6,
                  1e6, 0.3, 0.9, 0.3, 2e6, 0.25, 0.8, 0.4, 0.05, 0.02};
  orc_dem *s = orc_dem_create(&p, n, x, v, w, r, rho);

  /* binning and the stand-alone pair search */
  const int k[3] = {2, 2, 2};
  int *elem = malloc(sizeof(int) * n);
  long *cell = malloc(sizeof(long) * n);
  if (orc_bin(n, x, lo, hi, n_el, k, elem, cell) != 0) bad |= 1;
  const long cap = 64 * n;
  long *pi = malloc(sizeof(long) * cap), *pj = malloc(sizeof(long) * cap);
  const long np = orc_find_pairs(n, x, r, lo, hi, cap, pi, pj);
  if (np < 0 || np > cap) bad |= 2;

  /* fluid field on the nodes of the mesh */
  long nv = 1, npn = 1;
  for (int a = 0; a < 3; ++a) {
    nv *= (long)order * n_el[a] + 1;
    npn *= (long)n_el[a] + 1;
  }
  double *U = malloc(sizeof(double) * 3 * nv), *P = malloc(sizeof(double) * npn);
  double *epsn = malloc(sizeof(double) * nv);
  for (long q = 0; q < nv; ++q) {
    U[q] = 0.1 * (2.0 * unit() - 1.0);
    U[nv + q] = 0.1 * (2.0 * unit() - 1.0);
    U[2 * nv + q] = 0.5 + 0.1 * (2.0 * unit() - 1.0);
    epsn[q] = 0.3 + 0.7 * unit();
  }
  for (long q = 0; q < npn; ++q) P[q] = 10.0 * unit();
  long nel = (long)n_el[0] * n_el[1] * n_el[2];
  long nq = (long)(order + 1) * (order + 1) * (order + 1);
  double *eps_q = malloc(sizeof(double) * nel * nq), *beta_q = malloc(sizeof(double) * nel * nq);
  double *fpf_q = malloc(sizeof(double) * 3 * nel * nq), *sums = malloc(sizeof(double) * 12 * nel);

  for (int drag = ORC_DRAG_DIFELICE; drag <= ORC_DRAG_GIDASPOW; ++drag) {
    orc_fluid f = {order, {n_el[0], n_el[1], n_el[2]}, 1.2, 1.8e-5, drag % 2, 0.1, drag, drag % 2,
                   drag >= ORC_DRAG_BEETSTRA};
    if (orc_dem_couple(s, &f, U, P, eps_q, beta_q, fpf_q, sums) != 0) bad |= 4;
    if (orc_dem_step(s, 3) != 0) bad |= 8;
    if (orc_dem_couple_field(s, &f, U, P, epsn, eps_q, beta_q, fpf_q, sums) != 0) bad |= 16;
    if (orc_dem_step(s, 3) != 0) bad |= 32;
    for (double slip = 0.0; slip < 5.0; slip += 0.7)
      for (double eps = 0.15; eps <= 1.0; eps += 0.1)
        if (!isfinite(orc_drag_beta(drag, 1.2, 1.8e-5, eps, d, slip))) bad |= 64;
  }
  double *xi = malloc(sizeof(double) * 3 * n), *uf = malloc(sizeof(double) * 3 * n);
  double *gp = malloc(sizeof(double) * 3 * n), *dtau = malloc(sizeof(double) * 3 * n);
  double *ffp = malloc(sizeof(double) * 3 * n);
  orc_fluid f0 = {order, {n_el[0], n_el[1], n_el[2]}, 1.2, 1.8e-5, 0, 0.1, 0, 0, 1};
  orc_dem_get(s, xi, v, w, ffp, uf, gp);
  orc_interpolate(&f0, lo, hi, n, xi, U, P, uf, gp);
  orc_stress_divergence(&f0, lo, hi, n, xi, U, dtau);
  for (int pp = 1; pp <= 2; ++pp)
    for (int kk = 0; kk <= pp; ++kk)
      for (double t = 0.0; t <= 1.0; t += 0.125)
        if (!isfinite(orc_lagrange(pp, kk, t) + orc_lagrange_deriv(pp, kk, t) + orc_lagrange_deriv2(pp, kk, t)))
          bad |= 128;
  orc_dem_set_ffp(s, ffp);
  if (orc_dem_step(s, 5) != 0) bad |= 256;
  const long nc = orc_dem_ncontacts(s);
  long *ci = malloc(sizeof(long) * (nc ? nc : 1)), *cj = malloc(sizeof(long) * (nc ? nc : 1));
  double *cdt = malloc(sizeof(double) * 3 * (nc ? nc : 1));
  orc_dem_contacts(s, ci, cj, cdt);
  if (orc_dem_error(s) != 0) bad |= 512;
  printf("n %ld pairs %ld contacts %ld status %d\n", n, np, nc, bad);
  orc_dem_free(s);
  free(v), free(w), free(r), free(rho), free(elem), free(cell), free(pi), free(pj), free(U), free(P);
  free(epsn), free(eps_q), free(beta_q), free(fpf_q), free(sums), free(xi), free(uf), free(gp), free(dtau);
  free(ffp), free(ci), free(cj), free(cdt);
  return bad;
}

int main(void) {
  int bad = 0;
  orc_set_threads(2);
  const int n_side = 6;
  const double d = 3e-3;
  double lo[3], hi[3];
  double *x = malloc(sizeof(double) * 3 * n_side * n_side * n_side);
  long n = lattice(n_side, d, 0.99, 0.0, x, lo, hi);
  const int n_el2[3] = {2, 2, 2}, n_el1[3] = {3, 3, 3};
  bad |= run_bed(n, x, d, lo, hi, 2, n_el2, 1);
  bad |= run_bed(n, x, d, lo, hi, 1, n_el1, 0);
  /* a sparse bed: lattice at spacing 2d, the interior jittered */
  n = lattice(n_side, d, 2.0, 0.3 * d, x, lo, hi);
  bad |= run_bed(n, x, d, lo, hi, 2, n_el2, 1);
  free(x);
  printf("%s\n", bad ? "FAIL" : "OK");
  return bad ? 1 : 0;
}
