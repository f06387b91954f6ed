/*
 * cfddem_oracle.c -- plain, slow, FP64 CPU oracle of the particle-side hot path
 * of unresolved CFD-DEM (El Geitani, Golshan & Blais, arXiv 2211.01185).
 *
 * TEST INFRASTRUCTURE ONLY: this file is the checker of the HIP library, never
 * part of it.  Built with gcc -O2 -ffp-contract=off (no FMA contraction).
 *
 * One DEM step (Section 2.2, Eqs. "newton_law" and "angular_momentum", Table
 * "tab:viscoelastic", the contact-force equation, velocity Verlet):
 *   1. a = (F_c + f_fp)/m + g,  alpha = T_c/I
 *   2. v_h = v + dt/2 a,  w_h = w + dt/2 alpha,  x' = x + dt v_h
 *   3. contacts at x': pairs with (R_i+R_j)^2 - |x_j-x_i|^2 > 0, walls with
 *      R_i - dist > 0
 *   4. per contact: Table 1 constants, f_n = -k_n dn n - eta_n v_rn,
 *      f_t = -k_t dt_t - eta_t v_rt with the stored tangential overlap
 *      projected onto the new tangent plane and incremented by v_rt dt,
 *      Coulomb limit |f_t| <= mu |f_n|
 *   5. F_c, T_c = sums over contacts; v = v_h + dt/2 a', w = w_h + dt/2 alpha'
 * One coupling step (Section 2.3): particle-centroid void fraction per element
 * (Eq. "void_fraction"), Q_n interpolation of the fluid velocity and the Q1
 * pressure gradient at each particle, a drag closure (Di Felice, Dallavalle,
 * Rong, Koch-Hill, Beetstra or Gidaspow; optionally beta_B = beta_A / eps), buoyancy and
 * pressure-gradient forces on the particles, and the per-element reduction of
 * the drag back onto the quadrature points (Eqs. "fa", "fb").
 *
 * Pins (tests/test_oracle_*.py), all independent of this file's arithmetic:
 *   binning / contact search  brute force over all pairs, invariance under box
 *                             translation of the cell grid
 *   normal law + Verlet       Hertz two-sphere impact: contact time vs the
 *                             closed form, restitution 1 at e = 1 and e at e < 1
 *   tangential law + Coulomb  sphere sliding on a wall: v(t) = v0 - mu g t and
 *                             rolling at 5/7 v0; static overlap on a wall
 *   force gather              Newton's third law (total contact force zero)
 *   Verlet                    free fall (exact for constant acceleration)
 *   PCM                       solid-volume conservation, per-element counts
 *   interpolation             Q2 reproduces per-axis quadratics, Q1 gradient of
 *                             linear pressure exact
 *   Di Felice                 terminal velocity printed in Section 3.1
 *                             (0.2328 m/s) and its closed form; 0.96 x Stokes at
 *                             vanishing Reynolds number; the voidage exponent
 *                             measured at fixed Reynolds number: 3.7 in both
 *                             limits, minimum 3.05 at Re = 10^1.5, symmetric in
 *                             log10 Re, 3.7 - 0.65/e at 10^(1.5 +- sqrt 2)
 *   other closures            Stokes' 3 pi mu d for a lone sphere at vanishing
 *                             Reynolds number (Koch-Hill, Beetstra, Gidaspow;
 *                             0.96 of it for Dallavalle and Rong); Di Felice and
 *                             Rong equal Dallavalle at eps = 1; Rong's exponent
 *                             at full and vanishing bump; Beetstra's lone-sphere
 *                             Reynolds term, dense Stokes limit and large-Re
 *                             asymptote; Gidaspow's dense branch equals the
 *                             textbook Ergun pressure drop; near-continuity of
 *                             the Gidaspow (Re = 1000) and Koch-Hill
 *                             (eps_p = 0.4) branch joins
 *   pair spin terms           a spin equals the translation with the same
 *                             contact-point velocity; meshing spins slide
 *                             nothing; co-rotating spins are braked; the stored
 *                             tangential overlap stays in the turning tangent
 *                             plane; pair angular momentum about the centre of
 *                             mass
 *   qpt reduction             momentum balance of the drag (and pressure force
 *                             for model B) over the quadrature weights, for
 *                             every closure; beta_B = beta_A / eps per element
 *   threads                   results bit-identical at one and several threads
 * Parity unpinned: long chaotic trajectories, and the form of the rolling
 * torque (named by the paper without a form).
 */
#include "cfddem_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* small vector helpers                                                       */
/* ------------------------------------------------------------------------- */
static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double out[3]) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

static void *xmalloc(size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p) abort();
  return p;
}
static void *xcalloc(size_t count, size_t size) {
  void *p = calloc(count ? count : 1, size ? size : 1);
  if (!p) abort();
  return p;
}

/* Threads: loops whose iterations are independent run in parallel (OpenMP);
 * every sum over particles or contacts is accumulated afterwards by one thread
 * in the same order as a serial run, so results do not depend on the thread
 * count. */
static int orc_nthreads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
static int orc_thread_id(void) {
#ifdef _OPENMP
  return omp_get_thread_num();
#else
  return 0;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

int orc_get_threads(void) { return orc_nthreads(); }

/* ------------------------------------------------------------------------- */
/* Binning (broad search)                                                     */
/* ------------------------------------------------------------------------- */
/* clamp(floor(t), 0, n-1) as an integer; NaN goes to 0. */
static long floor_clamp(double t, long n) {
  double f = floor(t);
  if (!(f >= 0.0)) return 0;
  if (f > (double)(n - 1)) return n - 1;
  return (long)f;
}

long orc_bin(long n, const double *x, const double lo[3], const double hi[3],
             const int n_el[3], const int k[3], int *elem, long *cell) {
  long outside = 0;
  double he[3], inv_he[3], inv_hc[3];
  for (int a = 0; a < 3; ++a) {
    he[a] = (hi[a] - lo[a]) / (double)n_el[a];
    inv_he[a] = (double)n_el[a] / (hi[a] - lo[a]);
    inv_hc[a] = (double)(k[a] * n_el[a]) / (hi[a] - lo[a]);
  }
  for (long i = 0; i < n; ++i) {
    long e[3], sub[3];
    for (int a = 0; a < 3; ++a) {
      double xa = x[a * n + i];
      if (!(xa >= lo[a] && xa <= hi[a])) outside++;
      e[a] = floor_clamp((xa - lo[a]) * inv_he[a], n_el[a]);
      double origin = lo[a] + (double)e[a] * he[a];
      sub[a] = floor_clamp((xa - origin) * inv_hc[a], k[a]);
    }
    long e_lin = (e[2] * n_el[1] + e[1]) * n_el[0] + e[0];
    long s_lin = (sub[2] * k[1] + sub[1]) * k[0] + sub[0];
    if (elem) elem[i] = (int)e_lin;
    if (cell) cell[i] = e_lin * (long)(k[0] * k[1] * k[2]) + s_lin;
  }
  return outside;
}

/* ------------------------------------------------------------------------- */
/* Contact search                                                             */
/* ------------------------------------------------------------------------- */
typedef struct {
  long a, b;
} pair_t;

static int cmp_pair(const void *p, const void *q) {
  const pair_t *u = (const pair_t *)p, *w = (const pair_t *)q;
  if (u->a != w->a) return u->a < w->a ? -1 : 1;
  if (u->b != w->b) return u->b < w->b ? -1 : 1;
  return 0;
}

/* The fine-search predicate: strictly positive overlap, written as
 * (R_i+R_j)^2 - (dx^2+dy^2+dz^2) > 0, summed left to right. */
static int touching(const double xi[3], const double xj[3], double ri, double rj) {
  double dx = xj[0] - xi[0], dy = xj[1] - xi[1], dz = xj[2] - xi[2];
  double rs = ri + rj;
  double d2 = dx * dx + dy * dy + dz * dz;
  return rs * rs - d2 > 0.0;
}

/* Every pair i<j in contact, sorted by (i, j).  A uniform linked cell list
 * whose cells are at least one maximum diameter wide, so that any contacting
 * pair lies in the same or in adjacent cells. */
static long find_pairs_alloc(long n, const double *x, const double *r, const double lo[3],
                             const double hi[3], pair_t **out) {
  double rmax = 0.0;
  for (long i = 0; i < n; ++i)
    if (r[i] > rmax) rmax = r[i];
  long nc[3];
  double inv[3];
  for (int a = 0; a < 3; ++a) {
    double len = hi[a] - lo[a];
    double want = (rmax > 0.0) ? floor(len / (2.0 * rmax)) : 1.0;
    nc[a] = (want > 1048576.0) ? 1048576 : (long)want;
    if (nc[a] < 1) nc[a] = 1;
  }
  /* Fewer, wider cells are still correct; keep the grid within 64 cells per
   * particle so that sparse boxes do not allocate huge grids. */
  long limit = 64 * n > 4096 ? 64 * n : 4096;
  while (nc[0] * nc[1] * nc[2] > limit)
    for (int a = 0; a < 3; ++a) nc[a] = nc[a] * 3 / 4 > 1 ? nc[a] * 3 / 4 : 1;
  for (int a = 0; a < 3; ++a) inv[a] = (double)nc[a] / (hi[a] - lo[a]);
  long ncell = nc[0] * nc[1] * nc[2];
  long *head = (long *)xmalloc(sizeof(long) * ncell);
  long *next = (long *)xmalloc(sizeof(long) * (n ? n : 1));
  long *cc = (long *)xmalloc(sizeof(long) * 3 * (n ? n : 1));
  for (long c = 0; c < ncell; ++c) head[c] = -1;
  for (long i = n - 1; i >= 0; --i) {
    for (int a = 0; a < 3; ++a) cc[3 * i + a] = floor_clamp((x[a * n + i] - lo[a]) * inv[a], nc[a]);
    long c = (cc[3 * i + 2] * nc[1] + cc[3 * i + 1]) * nc[0] + cc[3 * i];
    next[i] = head[c];
    head[c] = i;
  }
  /* each thread collects the pairs of its own range of i; the lists are
   * concatenated and sorted, so the result does not depend on the split */
  int nt = orc_nthreads();
  pair_t **tl = (pair_t **)xcalloc((size_t)nt, sizeof(pair_t *));
  long *tc = (long *)xcalloc((size_t)nt, sizeof(long));
#pragma omp parallel num_threads(nt)
  {
    int t = orc_thread_id();
    long cap = 1024, cnt = 0;
    pair_t *list = (pair_t *)xmalloc(sizeof(pair_t) * cap);
#pragma omp for schedule(static)
    for (long i = 0; i < n; ++i) {
      double xi[3] = {x[i], x[n + i], x[2 * n + i]};
      for (long dz = -1; dz <= 1; ++dz)
        for (long dy = -1; dy <= 1; ++dy)
          for (long dx = -1; dx <= 1; ++dx) {
            long cx = cc[3 * i] + dx, cy = cc[3 * i + 1] + dy, cz = cc[3 * i + 2] + dz;
            if (cx < 0 || cy < 0 || cz < 0 || cx >= nc[0] || cy >= nc[1] || cz >= nc[2]) continue;
            for (long j = head[(cz * nc[1] + cy) * nc[0] + cx]; j >= 0; j = next[j]) {
              if (j <= i) continue;
              double xj[3] = {x[j], x[n + j], x[2 * n + j]};
              if (!touching(xi, xj, r[i], r[j])) continue;
              if (cnt == cap) {
                cap *= 2;
                list = (pair_t *)realloc(list, sizeof(pair_t) * cap);
                if (!list) abort();
              }
              list[cnt].a = i;
              list[cnt].b = j;
              cnt++;
            }
          }
    }
    tl[t] = list;
    tc[t] = cnt;
  }
  long cnt = 0;
  for (int t = 0; t < nt; ++t) cnt += tc[t];
  pair_t *list = (pair_t *)xmalloc(sizeof(pair_t) * (cnt ? cnt : 1));
  for (long t = 0, at = 0; t < nt; at += tc[t], ++t) {
    memcpy(list + at, tl[t], sizeof(pair_t) * tc[t]);
    free(tl[t]);
  }
  free(tl);
  free(tc);
  qsort(list, (size_t)cnt, sizeof(pair_t), cmp_pair);
  free(head);
  free(next);
  free(cc);
  *out = list;
  return cnt;
}

long orc_find_pairs(long n, const double *x, const double *r, const double lo[3],
                    const double hi[3], long cap, long *pi, long *pj) {
  pair_t *list = NULL;
  long cnt = find_pairs_alloc(n, x, r, lo, hi, &list);
  for (long c = 0; c < cnt && c < cap; ++c) {
    pi[c] = list[c].a;
    pj[c] = list[c].b;
  }
  free(list);
  return cnt;
}

/* ------------------------------------------------------------------------- */
/* Contact law (Table "tab:viscoelastic" and the contact-force equation)      */
/* ------------------------------------------------------------------------- */
typedef struct {
  double Ye, Ge, beta, mu; /* effective Young, effective shear, beta(e), Coulomb */
  double mu_r;             /* rolling friction coefficient */
} material_t;

/* 1/Y_e = (1-nu_i^2)/Y_i + (1-nu_j^2)/Y_j */
static double effective_young(double Yi, double nui, double Yj, double nuj) {
  return 1.0 / ((1.0 - nui * nui) / Yi + (1.0 - nuj * nuj) / Yj);
}
/* 1/G_e = 2(2-nu_i)(1+nu_i)/Y_i + 2(2-nu_j)(1+nu_j)/Y_j */
static double effective_shear(double Yi, double nui, double Yj, double nuj) {
  return 1.0 / (2.0 * (2.0 - nui) * (1.0 + nui) / Yi + 2.0 * (2.0 - nuj) * (1.0 + nuj) / Yj);
}
/* beta = ln e / sqrt(ln^2 e + pi^2) */
static double restitution_beta(double e) {
  double l = log(e);
  return l / sqrt(l * l + PI * PI);
}

/* Normal and tangential force of one contact, in the orientation of n (n points
 * from the first body to the second; the returned force acts on the first).
 *   dn      normal overlap (> 0)
 *   vij     relative velocity of the contact point, first minus second
 *   Re, me  effective radius and mass
 *   dt_old  stored tangential overlap (canonical orientation), or zeros
 *   advance 1: project onto the tangent plane and add v_rt*dt; 0: use dt_old
 * Outputs f (normal + tangential), ft, the updated tangential overlap and the
 * magnitude of the normal force. */
static void contact_law(const material_t *mat, const double n[3], double dn, const double vij[3],
                        double Re, double me, double dt, const double dt_old[3], int advance,
                        double f[3], double ft[3], double dt_new[3], double *fn_out) {
  double sq = sqrt(Re * dn);
  double kn = 4.0 / 3.0 * mat->Ye * sq;
  double kt = 8.0 * mat->Ge * sq;
  double Sn = 2.0 * mat->Ye * sq;
  double St = 8.0 * mat->Ge * sq;
  double etan = -2.0 * sqrt(5.0 / 6.0) * mat->beta * sqrt(Sn * me);
  double etat = -2.0 * sqrt(5.0 / 6.0) * mat->beta * sqrt(St * me);

  double vn = dot3(vij, n);
  double vrn[3], vrt[3];
  for (int c = 0; c < 3; ++c) {
    vrn[c] = vn * n[c];
    vrt[c] = vij[c] - vrn[c];
  }
  if (advance) {
    double along = dot3(dt_old, n);
    for (int c = 0; c < 3; ++c) dt_new[c] = (dt_old[c] - along * n[c]) + vrt[c] * dt;
  } else {
    for (int c = 0; c < 3; ++c) dt_new[c] = dt_old[c];
  }
  double fn[3];
  for (int c = 0; c < 3; ++c) {
    fn[c] = -kn * dn * n[c] - etan * vrn[c];
    ft[c] = -kt * dt_new[c] - etat * vrt[c];
  }
  /* Coulomb limit: sliding when |f_t| > mu |f_n| (a tie sticks). */
  double fn_mag = norm3(fn), ft_mag = norm3(ft);
  if (ft_mag > mat->mu * fn_mag) {
    double scale = mat->mu * fn_mag / ft_mag;
    for (int c = 0; c < 3; ++c) {
      ft[c] = ft[c] * scale;
      dt_new[c] = -ft[c] / kt;
    }
  }
  for (int c = 0; c < 3; ++c) f[c] = fn[c] + ft[c];
  *fn_out = fn_mag;
}

/* Rolling friction torque on the first body of a contact (Eq.
 * "angular_momentum" names M^r_ij without giving its form): the constant
 * torque -mu_r R_e |f_n| w/|w| opposing the relative angular velocity
 * w = w_i - w_j (w_i against a wall), zero when w = 0.  The second body
 * receives its negation. */
static void rolling_torque(double mu_r, double Re, double fn_mag, const double w[3], double M[3]) {
  double wm = norm3(w);
  for (int c = 0; c < 3; ++c) M[c] = 0.0;
  if (mu_r > 0.0 && wm > 0.0)
    for (int c = 0; c < 3; ++c) M[c] = -mu_r * Re * fn_mag * w[c] / wm;
}

/* ------------------------------------------------------------------------- */
/* DEM state                                                                  */
/* ------------------------------------------------------------------------- */
struct orc_dem {
  long n;
  orc_params p;
  material_t pp, pw;
  double *x, *v, *w;      /* 3n each */
  double *Fc, *Tc, *ffp;  /* 3n each */
  double *r, *m, *inertia; /* n each */
  long nh;                 /* history: contacts of the last evaluation */
  long *ha, *hb;           /* sorted by (ha, hb); hb = -1-wall for walls */
  double *hdt;             /* 3 per contact */
  int err;
};

/* Stored tangential overlap of contact (a, b), or zero when absent. */
static void history_lookup(const orc_dem *s, long a, long b, double out[3]) {
  long lo = 0, hi = s->nh - 1;
  while (lo <= hi) {
    long mid = (lo + hi) / 2;
    if (s->ha[mid] == a && s->hb[mid] == b) {
      for (int c = 0; c < 3; ++c) out[c] = s->hdt[3 * mid + c];
      return;
    }
    if (s->ha[mid] < a || (s->ha[mid] == a && s->hb[mid] < b))
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  out[0] = out[1] = out[2] = 0.0;
}

static void load3(const double *arr, long n, long i, double out[3]) {
  out[0] = arr[i];
  out[1] = arr[n + i];
  out[2] = arr[2 * n + i];
}

/* Evaluate every contact at the current positions with velocities v, w.
 * advance = 1 for a DEM step (history carried and incremented); 0 for the
 * priming evaluation at creation (zero tangential overlap, history stays
 * empty).  Overwrites F_c, T_c and (when advancing) the history. */
static void evaluate_contacts(orc_dem *s, const double *v, const double *w, int advance) {
  long n = s->n;
  const double *lo = s->p.box_lo, *hi = s->p.box_hi;
  memset(s->Fc, 0, sizeof(double) * 3 * n);
  memset(s->Tc, 0, sizeof(double) * 3 * n);

  pair_t *pairs = NULL;
  long np = find_pairs_alloc(n, s->x, s->r, lo, hi, &pairs);
  /* wall contacts: distance from the centre to each of the six planes */
  long nw_cap = 16, nw = 0;
  pair_t *walls = (pair_t *)xmalloc(sizeof(pair_t) * nw_cap);
  for (long i = 0; i < n; ++i) {
    for (int wall = 0; wall < 6; ++wall) {
      int a = wall / 2;
      double xa = s->x[a * n + i];
      double dist = (wall % 2 == 0) ? xa - lo[a] : hi[a] - xa;
      if (s->r[i] - dist > 0.0) {
        if (nw == nw_cap) {
          nw_cap *= 2;
          walls = (pair_t *)realloc(walls, sizeof(pair_t) * nw_cap);
          if (!walls) abort();
        }
        walls[nw].a = i;
        walls[nw].b = -1 - wall;
        nw++;
      }
    }
  }
  long nc = np + nw;
  pair_t *all = (pair_t *)xmalloc(sizeof(pair_t) * (nc ? nc : 1));
  memcpy(all, pairs, sizeof(pair_t) * np);
  memcpy(all + np, walls, sizeof(pair_t) * nw);
  qsort(all, (size_t)nc, sizeof(pair_t), cmp_pair);
  free(pairs);
  free(walls);

  long *na = (long *)xmalloc(sizeof(long) * (nc ? nc : 1));
  long *nb = (long *)xmalloc(sizeof(long) * (nc ? nc : 1));
  double *ndt = (double *)xmalloc(sizeof(double) * 3 * (nc ? nc : 1));

  /* per-contact force and torques in parallel; F_c and T_c summed below in
   * contact order */
  double *cf = (double *)xmalloc(sizeof(double) * 3 * (nc ? nc : 1));
  double *cti = (double *)xmalloc(sizeof(double) * 3 * (nc ? nc : 1));
  double *ctj = (double *)xmalloc(sizeof(double) * 3 * (nc ? nc : 1));
#pragma omp parallel for schedule(static)
  for (long c = 0; c < nc; ++c) {
    long i = all[c].a, j = all[c].b;
    double xi[3], vi[3], wi[3];
    load3(s->x, n, i, xi);
    load3(v, n, i, vi);
    load3(w, n, i, wi);
    double Ri = s->r[i];
    double dt_old[3] = {0.0, 0.0, 0.0};
    if (advance) history_lookup(s, i, j, dt_old);
    double f[3], ft[3], dt_new[3], nrm[3], vij[3], cr[3];
    if (j >= 0) {
      double xj[3], vj[3], wj[3];
      load3(s->x, n, j, xj);
      load3(v, n, j, vj);
      load3(w, n, j, wj);
      double Rj = s->r[j];
      double d[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
      double dist = norm3(d);
      for (int k = 0; k < 3; ++k) nrm[k] = d[k] / dist;
      double dn = (Ri + Rj) - dist;
      /* v_ij = v_i - v_j + (R_i w_i + R_j w_j) x n */
      double rw[3] = {Ri * wi[0] + Rj * wj[0], Ri * wi[1] + Rj * wj[1], Ri * wi[2] + Rj * wj[2]};
      cross3(rw, nrm, cr);
      for (int k = 0; k < 3; ++k) vij[k] = vi[k] - vj[k] + cr[k];
      double Re = 1.0 / (1.0 / Ri + 1.0 / Rj);
      double me = 1.0 / (1.0 / s->m[i] + 1.0 / s->m[j]);
      double fn_mag;
      contact_law(&s->pp, nrm, dn, vij, Re, me, s->p.dt, dt_old, advance, f, ft, dt_new, &fn_mag);
      double ti[3], tj[3], nxft[3], Mr[3];
      double wrel[3] = {wi[0] - wj[0], wi[1] - wj[1], wi[2] - wj[2]};
      rolling_torque(s->pp.mu_r, Re, fn_mag, wrel, Mr);
      cross3(nrm, ft, nxft);
      for (int k = 0; k < 3; ++k) {
        ti[k] = Ri * nxft[k];
        tj[k] = Rj * nxft[k];
        cf[3 * c + k] = f[k];
        cti[3 * c + k] = ti[k] + Mr[k];
        ctj[3 * c + k] = tj[k] - Mr[k];
      }
    } else {
      int wall = -1 - (int)j;
      int a = wall / 2;
      double dist = (wall % 2 == 0) ? xi[a] - lo[a] : hi[a] - xi[a];
      nrm[0] = nrm[1] = nrm[2] = 0.0;
      nrm[a] = (wall % 2 == 0) ? -1.0 : 1.0; /* from the particle towards the wall */
      double dn = Ri - dist;
      double rw[3] = {Ri * wi[0], Ri * wi[1], Ri * wi[2]};
      cross3(rw, nrm, cr);
      for (int k = 0; k < 3; ++k) vij[k] = vi[k] + cr[k];
      double fn_mag;
      contact_law(&s->pw, nrm, dn, vij, Ri, s->m[i], s->p.dt, dt_old, advance, f, ft, dt_new, &fn_mag);
      double nxft[3], Mr[3];
      rolling_torque(s->pw.mu_r, Ri, fn_mag, wi, Mr);
      cross3(nrm, ft, nxft);
      for (int k = 0; k < 3; ++k) {
        cf[3 * c + k] = f[k];
        cti[3 * c + k] = Ri * nxft[k] + Mr[k];
      }
    }
    na[c] = i;
    nb[c] = j;
    for (int k = 0; k < 3; ++k) ndt[3 * c + k] = dt_new[k];
  }
  /* F_i = sum of f over the contacts of i, T_i likewise (contact order) */
  for (long c = 0; c < nc; ++c) {
    long i = na[c], j = nb[c];
    for (int k = 0; k < 3; ++k) {
      s->Fc[k * n + i] += cf[3 * c + k];
      s->Tc[k * n + i] += cti[3 * c + k];
      if (j >= 0) {
        s->Fc[k * n + j] -= cf[3 * c + k];
        s->Tc[k * n + j] += ctj[3 * c + k];
      }
    }
  }
  free(cf);
  free(cti);
  free(ctj);
  free(all);
  free(s->ha);
  free(s->hb);
  free(s->hdt);
  s->ha = na;
  s->hb = nb;
  s->hdt = ndt;
  s->nh = nc;
  if (!advance) {
    /* priming leaves no tangential history behind, only the contact list */
    for (long c = 0; c < 3 * nc; ++c) s->hdt[c] = 0.0;
  }
}

static void check_state(orc_dem *s) {
  long n = s->n;
  int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
  for (long i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) {
      double xa = s->x[a * n + i];
      if (xa != xa || s->v[a * n + i] != s->v[a * n + i] || s->w[a * n + i] != s->w[a * n + i])
        err |= ORC_ERR_NAN;
      else if (xa < s->p.box_lo[a] || xa > s->p.box_hi[a])
        err |= ORC_ERR_DOMAIN;
    }
  }
  s->err |= err;
}

orc_dem *orc_dem_create(const orc_params *p, long n, const double *x, const double *v,
                        const double *w, const double *r, const double *rho) {
  orc_dem *s = (orc_dem *)xcalloc(1, sizeof(orc_dem));
  s->n = n;
  s->p = *p;
  s->pp.Ye = effective_young(p->E, p->nu, p->E, p->nu);
  s->pp.Ge = effective_shear(p->E, p->nu, p->E, p->nu);
  s->pp.beta = restitution_beta(p->e);
  s->pp.mu = p->mu;
  s->pp.mu_r = p->mu_r;
  s->pw.Ye = effective_young(p->E, p->nu, p->E_w, p->nu_w);
  s->pw.Ge = effective_shear(p->E, p->nu, p->E_w, p->nu_w);
  s->pw.beta = restitution_beta(p->e_w);
  s->pw.mu = p->mu_w;
  s->pw.mu_r = p->mu_r_w;
  size_t v3 = sizeof(double) * 3 * (n ? n : 1);
  s->x = (double *)xmalloc(v3);
  s->v = (double *)xmalloc(v3);
  s->w = (double *)xmalloc(v3);
  s->Fc = (double *)xcalloc(3 * (n ? n : 1), sizeof(double));
  s->Tc = (double *)xcalloc(3 * (n ? n : 1), sizeof(double));
  s->ffp = (double *)xcalloc(3 * (n ? n : 1), sizeof(double));
  s->r = (double *)xmalloc(sizeof(double) * (n ? n : 1));
  s->m = (double *)xmalloc(sizeof(double) * (n ? n : 1));
  s->inertia = (double *)xmalloc(sizeof(double) * (n ? n : 1));
  memcpy(s->x, x, sizeof(double) * 3 * n);
  memcpy(s->v, v, sizeof(double) * 3 * n);
  memcpy(s->w, w, sizeof(double) * 3 * n);
  for (long i = 0; i < n; ++i) {
    s->r[i] = r[i];
    /* solid sphere: m = rho 4/3 pi R^3, I = 2/5 m R^2 */
    s->m[i] = rho[i] * (4.0 / 3.0 * PI * r[i] * r[i] * r[i]);
    s->inertia[i] = 0.4 * s->m[i] * r[i] * r[i];
  }
  check_state(s);
  evaluate_contacts(s, s->v, s->w, 0);
  return s;
}

int orc_dem_step(orc_dem *s, long nsteps) {
  long n = s->n;
  const double dt = s->p.dt;
  const double *g = s->p.gravity;
  double *vh = (double *)xmalloc(sizeof(double) * 3 * (n ? n : 1));
  double *wh = (double *)xmalloc(sizeof(double) * 3 * (n ? n : 1));
  for (long step = 0; step < nsteps; ++step) {
    /* half kick and drift with the stored forces */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
      for (int a = 0; a < 3; ++a) {
        long k = a * n + i;
        double acc = (s->Fc[k] + s->ffp[k]) / s->m[i] + g[a];
        double alpha = s->Tc[k] / s->inertia[i];
        vh[k] = s->v[k] + 0.5 * dt * acc;
        wh[k] = s->w[k] + 0.5 * dt * alpha;
        s->x[k] = s->x[k] + dt * vh[k];
      }
    }
    /* contacts and forces at the new positions, half-step velocities */
    evaluate_contacts(s, vh, wh, 1);
    /* second half kick */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
      for (int a = 0; a < 3; ++a) {
        long k = a * n + i;
        double acc = (s->Fc[k] + s->ffp[k]) / s->m[i] + g[a];
        double alpha = s->Tc[k] / s->inertia[i];
        s->v[k] = vh[k] + 0.5 * dt * acc;
        s->w[k] = wh[k] + 0.5 * dt * alpha;
      }
    }
    check_state(s);
  }
  free(vh);
  free(wh);
  return s->err;
}

/* ------------------------------------------------------------------------- */
/* Coupling (Section 2.3)                                                     */
/* ------------------------------------------------------------------------- */
/* Lagrange polynomial k of degree p on the equispaced nodes t_m = m/p. */
double orc_lagrange(int p, int k, double t) {
  double val = 1.0;
  for (int m = 0; m <= p; ++m) {
    if (m == k) continue;
    double tm = (double)m / p, tk = (double)k / p;
    val *= (t - tm) / (tk - tm);
  }
  return val;
}

/* Derivative: sum over the dropped factor of the product rule. */
double orc_lagrange_deriv(int p, int k, double t) {
  double tk = (double)k / p;
  double sum = 0.0;
  for (int q = 0; q <= p; ++q) {
    if (q == k) continue;
    double term = 1.0 / (tk - (double)q / p);
    for (int m = 0; m <= p; ++m) {
      if (m == k || m == q) continue;
      double tm = (double)m / p;
      term *= (t - tm) / (tk - tm);
    }
    sum += term;
  }
  return sum;
}

/* Second derivative: sum over ordered pairs (q, r) of dropped factors. */
double orc_lagrange_deriv2(int p, int k, double t) {
  double tk = (double)k / p;
  double sum = 0.0;
  for (int q = 0; q <= p; ++q) {
    if (q == k) continue;
    for (int r = 0; r <= p; ++r) {
      if (r == k || r == q) continue;
      double term = 1.0 / (tk - (double)q / p) / (tk - (double)r / p);
      for (int m = 0; m <= p; ++m) {
        if (m == k || m == q || m == r) continue;
        double tm = (double)m / p;
        term *= (t - tm) / (tk - tm);
      }
      sum += term;
    }
  }
  return sum;
}

/* Element of a point and its reference coordinates xi in [0,1]^3. */
static void locate(const orc_fluid *f, const double lo[3], const double hi[3], const double xp[3],
                   long e[3], double xi[3]) {
  for (int a = 0; a < 3; ++a) {
    double he = (hi[a] - lo[a]) / (double)f->n_el[a];
    double inv_he = (double)f->n_el[a] / (hi[a] - lo[a]);
    e[a] = floor_clamp((xp[a] - lo[a]) * inv_he, f->n_el[a]);
    xi[a] = (xp[a] - (lo[a] + (double)e[a] * he)) * inv_he;
  }
}

/* Global index of local node (ia, ib, ic) of element e for order p. */
static long node_index(int p, const int n_el[3], const long e[3], int ia, int ib, int ic) {
  long nx = (long)p * n_el[0] + 1, ny = (long)p * n_el[1] + 1;
  long gx = p * e[0] + ia, gy = p * e[1] + ib, gz = p * e[2] + ic;
  return (gz * ny + gy) * nx + gx;
}

/* u = sum_k N_k(xi) U_k over the (p+1)^3 velocity nodes of element e. */
static void interp_velocity(const orc_fluid *f, const long e[3], const double xi[3], const double *U,
                            long n_v, double u[3]) {
  int p = f->order;
  u[0] = u[1] = u[2] = 0.0;
  for (int ic = 0; ic <= p; ++ic)
    for (int ib = 0; ib <= p; ++ib)
      for (int ia = 0; ia <= p; ++ia) {
        double N = orc_lagrange(p, ia, xi[0]) * orc_lagrange(p, ib, xi[1]) * orc_lagrange(p, ic, xi[2]);
        long node = node_index(p, f->n_el, e, ia, ib, ic);
        for (int c = 0; c < 3; ++c) u[c] += N * U[c * n_v + node];
      }
}

/* grad p = sum_k grad N_k^{Q1}(xi) P_k; d/dx = (1/h_x) d/dxi. */
static void interp_pressure_gradient(const orc_fluid *f, const double lo[3], const double hi[3],
                                     const long e[3], const double xi[3], const double *P,
                                     double gp[3]) {
  double inv_he[3];
  for (int a = 0; a < 3; ++a) inv_he[a] = (double)f->n_el[a] / (hi[a] - lo[a]);
  gp[0] = gp[1] = gp[2] = 0.0;
  for (int ic = 0; ic <= 1; ++ic)
    for (int ib = 0; ib <= 1; ++ib)
      for (int ia = 0; ia <= 1; ++ia) {
        double Pk = P[node_index(1, f->n_el, e, ia, ib, ic)];
        double dx = orc_lagrange_deriv(1, ia, xi[0]) * orc_lagrange(1, ib, xi[1]) * orc_lagrange(1, ic, xi[2]);
        double dy = orc_lagrange(1, ia, xi[0]) * orc_lagrange_deriv(1, ib, xi[1]) * orc_lagrange(1, ic, xi[2]);
        double dz = orc_lagrange(1, ia, xi[0]) * orc_lagrange(1, ib, xi[1]) * orc_lagrange_deriv(1, ic, xi[2]);
        gp[0] += dx * inv_he[0] * Pk;
        gp[1] += dy * inv_he[1] * Pk;
        gp[2] += dz * inv_he[2] * Pk;
      }
}

static long velocity_node_count(const orc_fluid *f) {
  long p = f->order;
  return (p * f->n_el[0] + 1) * (p * f->n_el[1] + 1) * (p * f->n_el[2] + 1);
}

/* d^0, d^1 or d^2 of the 1D basis k at t. */
static double lagrange_d(int p, int k, int order, double t) {
  if (order == 0) return orc_lagrange(p, k, t);
  if (order == 1) return orc_lagrange_deriv(p, k, t);
  return orc_lagrange_deriv2(p, k, t);
}

/* div(tau_f) at a point (Eq. "stress"):
 *   tau_cj = mu_f (d_j u_c + d_c u_j) - 2/3 mu_f (div u) delta_cj,
 *   (div tau)_c = sum_j d_j tau_cj,
 * from the Hessians H[c][a][b] = d_a d_b u_c of the Q_n field. */
static void stress_divergence(const orc_fluid *f, const double lo[3], const double hi[3],
                              const long e[3], const double xi[3], const double *U, long n_v,
                              double out[3]) {
  int p = f->order;
  double inv_he[3];
  for (int a = 0; a < 3; ++a) inv_he[a] = (double)f->n_el[a] / (hi[a] - lo[a]);
  double H[3][3][3];
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) H[c][a][b] = 0.0;
  for (int ic = 0; ic <= p; ++ic)
    for (int ib = 0; ib <= p; ++ib)
      for (int ia = 0; ia <= p; ++ia) {
        long node = node_index(p, f->n_el, e, ia, ib, ic);
        int loc[3] = {ia, ib, ic};
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            int ord[3] = {0, 0, 0};
            ord[a] += 1;
            ord[b] += 1;
            double d2N = inv_he[a] * inv_he[b];
            for (int ax = 0; ax < 3; ++ax) d2N *= lagrange_d(p, loc[ax], ord[ax], xi[ax]);
            for (int c = 0; c < 3; ++c) H[c][a][b] += d2N * U[c * n_v + node];
          }
      }
  double mu = f->mu_f;
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
    for (int j = 0; j < 3; ++j) {
      double d_tau = mu * (H[c][j][j] + H[j][c][j]); /* d_j of mu (d_j u_c + d_c u_j) */
      if (j == c) {
        double d_div = 0.0; /* d_c (div u) */
        for (int k = 0; k < 3; ++k) d_div += H[k][k][c];
        d_tau -= 2.0 / 3.0 * mu * d_div;
      }
      s += d_tau;
    }
    out[c] = s;
  }
}

void orc_stress_divergence(const orc_fluid *f, const double lo[3], const double hi[3], long n,
                           const double *x, const double *U, double *out) {
  long n_v = velocity_node_count(f);
  for (long i = 0; i < n; ++i) {
    double xp[3] = {x[i], x[n + i], x[2 * n + i]}, xi[3], dv[3];
    long e[3];
    locate(f, lo, hi, xp, e, xi);
    stress_divergence(f, lo, hi, e, xi, U, n_v, dv);
    for (int c = 0; c < 3; ++c) out[c * n + i] = dv[c];
  }
}

void orc_interpolate(const orc_fluid *f, const double lo[3], const double hi[3], long n,
                     const double *x, const double *U, const double *P, double *u_out,
                     double *gradp_out) {
  long n_v = velocity_node_count(f);
  for (long i = 0; i < n; ++i) {
    double xp[3] = {x[i], x[n + i], x[2 * n + i]}, xi[3], u[3], gp[3];
    long e[3];
    locate(f, lo, hi, xp, e, xi);
    interp_velocity(f, e, xi, U, n_v, u);
    interp_pressure_gradient(f, lo, hi, e, xi, P, gp);
    for (int c = 0; c < 3; ++c) {
      if (u_out) u_out[c * n + i] = u[c];
      if (gradp_out) gradp_out[c * n + i] = gp[c];
    }
  }
}

/* Di Felice: Re = rho_f eps |slip| d / mu_f,
 * chi = 3.7 - 0.65 exp(-(1.5 - log10 Re)^2 / 2),
 * C_D = (0.63 + 4.8/sqrt(Re))^2 eps^(2 - chi),  beta = 1/2 rho_f C_D pi r^2 |slip|.
 * At zero slip the product C_D |slip| has the finite limit
 * (4.8)^2 mu_f / (rho_f eps d) with chi = 3.7 (log10 Re -> -inf). */
double orc_difelice_beta(double rho_f, double mu_f, double eps, double d, double slip) {
  double r = 0.5 * d;
  double area = PI * r * r;
  if (slip > 0.0) {
    double Re = rho_f * eps * slip * d / mu_f;
    double lg = 1.5 - log10(Re);
    double chi = 3.7 - 0.65 * exp(-(lg * lg) / 2.0);
    double root = 0.63 + 4.8 / sqrt(Re);
    double CD = root * root * pow(eps, 2.0 - chi);
    return 0.5 * rho_f * CD * area * slip;
  }
  double lim = 4.8 * 4.8 * mu_f / (rho_f * eps * d);
  return 0.5 * rho_f * lim * pow(eps, 2.0 - 3.7) * area;
}

/* The other closures of Section 2.3.2, with eps the fluid fraction,
 * eps_p = 1 - eps, Re = rho_f eps |slip| d / mu_f (the particle Reynolds
 * number of the section) and V_p = pi d^3 / 6:
 *  Dallavalle  C_D = (0.63 + 4.8/sqrt(Re))^2, beta = 1/2 rho_f C_D pi r^2 |slip|
 *  Rong        C_D = (0.63 + 4.8/sqrt(Re))^2 eps^(2 - [2.65 (eps + 1)
 *                    - (5.3 - 3.5 eps) eps^2 exp(-(1.5 - log10 Re)^2 / 2)])
 *  Koch-Hill   beta = 18 mu_f eps^2 eps_p / d^2 (F0 + F3 Re / 2) V_p / eps_p,
 *              F0 = (1 + 3 sqrt(eps_p/2) + 135/64 eps_p ln eps_p + 16.14 eps_p)
 *                   / (1 + 0.681 eps_p - 8.48 eps_p^2 + 8.14 eps_p^3) (eps_p < 0.4),
 *                   10 eps_p / eps^3 (eps_p >= 0.4);
 *              F3 = 0.0673 + 0.212 eps_p + 0.0232 / eps^5
 *  Beetstra    f_D = 3 pi mu_f d eps F slip, i.e. beta = 3 pi mu_f d eps F, with
 *              F = 10 eps_p / eps^2 + eps^2 (1 + 1.5 sqrt(eps_p))
 *                  + 0.413 Re / (24 eps^2) (1/eps + 3 eps_p eps + 8.4 Re^-0.343)
 *                    / (1 + 10^(3 eps_p) Re^(-(1 + 4 eps_p)/2))
 *              (the printed force multiplies the fluid velocity; the slip is
 *              read, as in every other closure)
 *  Gidaspow    per unit mixture volume: eps < 0.8 (Ergun)
 *              150 eps_p^2 mu_f / (eps d^2) + 1.75 eps_p rho_f |slip| / d,
 *              eps >= 0.8 (Wen-Yu) 3/4 C_D eps |slip| rho_f eps_p / d eps^-2.65,
 *              C_D = 24/Re (1 + 0.15 Re^0.687) (Re < 1000), 0.44 (Re >= 1000);
 *              per particle times V_p / eps_p (as the Koch-Hill expression
 *              writes out), the |slip| of the Ergun term read as a magnitude.
 * Zero slip: every product C_D |slip| or Re-dependent factor is replaced by
 * its limit. */
static double koch_hill_F0(double ep, double ef) {
  if (ep < 0.4) {
    double lnterm = ep > 0.0 ? 135.0 / 64.0 * ep * log(ep) : 0.0;
    return (1.0 + 3.0 * sqrt(ep / 2.0) + lnterm + 16.14 * ep) /
           (1.0 + 0.681 * ep - 8.48 * ep * ep + 8.14 * ep * ep * ep);
  }
  return 10.0 * ep / (ef * ef * ef);
}

double orc_drag_beta(int drag, double rho_f, double mu_f, double eps, double d, double slip) {
  double r = 0.5 * d;
  double area = PI * r * r;
  double Vp = PI * d * d * d / 6.0;
  double ep = 1.0 - eps;
  double Re = rho_f * eps * slip * d / mu_f;
  switch (drag) {
    case ORC_DRAG_DIFELICE:
      return orc_difelice_beta(rho_f, mu_f, eps, d, slip);
    case ORC_DRAG_DALLAVALLE:
    case ORC_DRAG_RONG: {
      double cds; /* C_D |slip| without the voidage factor */
      double expo = 0.0;
      if (slip > 0.0) {
        double root = 0.63 + 4.8 / sqrt(Re);
        cds = root * root * slip;
      } else {
        cds = 4.8 * 4.8 * mu_f / (rho_f * eps * d);
      }
      if (drag == ORC_DRAG_RONG) {
        double bump = 0.0;
        if (slip > 0.0) {
          double lg = 1.5 - log10(Re);
          bump = exp(-(lg * lg) / 2.0);
        }
        expo = 2.0 - (2.65 * (eps + 1.0) - (5.3 - 3.5 * eps) * eps * eps * bump);
      }
      return 0.5 * rho_f * cds * pow(eps, expo) * area;
    }
    case ORC_DRAG_KOCH_HILL: {
      double F0 = koch_hill_F0(ep, eps);
      double F3 = 0.0673 + 0.212 * ep + 0.0232 / pow(eps, 5.0);
      return 18.0 * mu_f * eps * eps / (d * d) * (F0 + 0.5 * F3 * Re) * Vp;
    }
    case ORC_DRAG_BEETSTRA: {
      double F = 10.0 * ep / (eps * eps) + eps * eps * (1.0 + 1.5 * sqrt(ep));
      if (slip > 0.0) {
        double num = 1.0 / eps + 3.0 * ep * eps + 8.4 * pow(Re, -0.343);
        double den = 1.0 + pow(10.0, 3.0 * ep) * pow(Re, -(1.0 + 4.0 * ep) / 2.0);
        F += 0.413 * Re / (24.0 * eps * eps) * num / den;
      }
      return 3.0 * PI * mu_f * d * eps * F;
    }
    case ORC_DRAG_GIDASPOW: {
      if (eps < 0.8)
        return Vp * (150.0 * ep * mu_f / (eps * d * d) + 1.75 * rho_f * slip / d);
      double cds; /* C_D |slip| */
      if (slip > 0.0) {
        double CD = Re < 1000.0 ? 24.0 / Re * (1.0 + 0.15 * pow(Re, 0.687)) : 0.44;
        cds = CD * slip;
      } else {
        cds = 24.0 * mu_f / (rho_f * eps * d);
      }
      return Vp * 0.75 * cds * eps * rho_f / d * pow(eps, -2.65);
    }
    default:
      return NAN;
  }
}

/* Gauss-Legendre points and weights mapped to [0,1]. */
static void gauss_rule(int npts, double *pt, double *wt) {
  if (npts == 2) {
    double a = 0.5 / sqrt(3.0);
    pt[0] = 0.5 - a;
    pt[1] = 0.5 + a;
    wt[0] = wt[1] = 0.5;
  } else {
    double a = 0.5 * sqrt(3.0 / 5.0);
    pt[0] = 0.5 - a;
    pt[1] = 0.5;
    pt[2] = 0.5 + a;
    wt[0] = wt[2] = 5.0 / 18.0;
    wt[1] = 8.0 / 18.0;
  }
}

/* Element sums layout (component-major over elements, 12 rows):
 *   0 count, 1 sum V_p, 2 sum beta_p, 3-5 sum beta_p u_p, 6-8 sum f_D,
 *   9-11 sum of the undisturbed-flow forces f_gradp (+ f_shear when enabled). */
#define ES_ROWS 12

/* Value of a scalar nodal field of order p at xi in element e. */
static double interp_scalar(const orc_fluid *f, const long e[3], const double xi[3], const double *vals) {
  int p = f->order;
  double out = 0.0;
  for (int ic = 0; ic <= p; ++ic)
    for (int ib = 0; ib <= p; ++ib)
      for (int ia = 0; ia <= p; ++ia) {
        double N = orc_lagrange(p, ia, xi[0]) * orc_lagrange(p, ib, xi[1]) * orc_lagrange(p, ic, xi[2]);
        out += N * vals[node_index(p, f->n_el, e, ia, ib, ic)];
      }
  return out;
}

int orc_dem_couple(orc_dem *s, const orc_fluid *f, const double *U, const double *P,
                   double *eps_q, double *beta_q, double *fpf_q, double *elem_sums) {
  return orc_dem_couple_field(s, f, U, P, NULL, eps_q, beta_q, fpf_q, elem_sums);
}

int orc_dem_couple_field(orc_dem *s, const orc_fluid *f, const double *U, const double *P,
                         const double *eps_nodes, double *eps_q, double *beta_q, double *fpf_q,
                         double *elem_sums) {
  long n = s->n;
  const double *lo = s->p.box_lo, *hi = s->p.box_hi;
  const double *g = s->p.gravity;
  long nel = (long)f->n_el[0] * f->n_el[1] * f->n_el[2];
  int nq1 = f->order + 1; /* 2 Gauss points per axis for Q1, 3 for Q2 */
  long nq = (long)nq1 * nq1 * nq1;
  long n_v = velocity_node_count(f);
  double he[3];
  for (int a = 0; a < 3; ++a) he[a] = (hi[a] - lo[a]) / (double)f->n_el[a];
  double Ve = he[0] * he[1] * he[2];

  double *sums = (double *)xcalloc((size_t)ES_ROWS * nel, sizeof(double));
  long *pe = (long *)xmalloc(sizeof(long) * (n ? n : 1));
  double *pxi = (double *)xmalloc(sizeof(double) * 3 * (n ? n : 1));

  /* per-particle terms of the element sums (rows 2-11), added in particle
   * order after the parallel loops */
  double *pt = (double *)xmalloc(sizeof(double) * 10 * (n ? n : 1));

  /* 1. locate and particle-centroid solid volume per element */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i) {
    double xp[3], xi[3];
    long e[3];
    load3(s->x, n, i, xp);
    locate(f, lo, hi, xp, e, xi);
    pe[i] = (e[2] * f->n_el[1] + e[1]) * f->n_el[0] + e[0];
    for (int a = 0; a < 3; ++a) pxi[3 * i + a] = xi[a];
  }
  for (long i = 0; i < n; ++i) {
    double Vp = 4.0 / 3.0 * PI * s->r[i] * s->r[i] * s->r[i];
    sums[0 * nel + pe[i]] += 1.0;
    sums[1 * nel + pe[i]] += Vp;
  }
  /* 2. per-particle forces */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i) {
    long el = pe[i];
    long e[3] = {el % f->n_el[0], (el / f->n_el[0]) % f->n_el[1], el / ((long)f->n_el[0] * f->n_el[1])};
    double xi[3] = {pxi[3 * i], pxi[3 * i + 1], pxi[3 * i + 2]};
    double uf[3], gp[3], up[3];
    interp_velocity(f, e, xi, U, n_v, uf);
    interp_pressure_gradient(f, lo, hi, e, xi, P, gp);
    load3(s->v, n, i, up);
    double eps = eps_nodes ? interp_scalar(f, e, xi, eps_nodes) : 1.0 - sums[1 * nel + el] / Ve;
    double eps_c = eps;
    if (eps_c < f->eps_min) eps_c = f->eps_min;
    if (eps_c > 1.0) eps_c = 1.0;
    double slip[3] = {uf[0] - up[0], uf[1] - up[1], uf[2] - up[2]};
    double d = 2.0 * s->r[i];
    double Vp = 4.0 / 3.0 * PI * s->r[i] * s->r[i] * s->r[i];
    double beta = orc_drag_beta(f->drag, f->rho_f, f->mu_f, eps_c, d, norm3(slip));
    if (f->beta_over_eps) beta /= eps_c; /* beta_B = beta_A / eps (Eq. "beta") */
    double dtau[3] = {0.0, 0.0, 0.0};
    if (f->shear) stress_divergence(f, lo, hi, e, xi, U, n_v, dtau);
    for (int c = 0; c < 3; ++c) {
      double fD = beta * slip[c];
      double fB = -f->rho_f * Vp * g[c];
      double fG = -Vp * gp[c];
      double fS = -Vp * dtau[c]; /* shear force (zero unless enabled) */
      s->ffp[c * n + i] = fD + fB + fG + fS;
      pt[10 * i + 1 + c] = beta * up[c];
      pt[10 * i + 4 + c] = fD;
      pt[10 * i + 7 + c] = fG + fS; /* undisturbed-flow forces */
    }
    pt[10 * i] = beta;
  }
  for (long i = 0; i < n; ++i) {
    long el = pe[i];
    for (int c = 0; c < 3; ++c) {
      sums[(3 + c) * nel + el] += pt[10 * i + 1 + c];
      sums[(6 + c) * nel + el] += pt[10 * i + 4 + c];
      sums[(9 + c) * nel + el] += pt[10 * i + 7 + c];
    }
    sums[2 * nel + el] += pt[10 * i];
  }
  free(pt);
  /* 3. quadrature-point outputs */
  double gpt[3], gwt[3];
  gauss_rule(nq1, gpt, gwt);
#pragma omp parallel for schedule(static)
  for (long el = 0; el < nel; ++el) {
    long e[3] = {el % f->n_el[0], (el / f->n_el[0]) % f->n_el[1], el / ((long)f->n_el[0] * f->n_el[1])};
    double eps = 1.0 - sums[1 * nel + el] / Ve;
    double sb = sums[2 * nel + el];
    double bq = sb / Ve;
    double ubar[3] = {0.0, 0.0, 0.0};
    if (sums[0 * nel + el] > 0.0 && sb > 0.0)
      for (int c = 0; c < 3; ++c) ubar[c] = sums[(3 + c) * nel + el] / sb;
    for (int qz = 0; qz < nq1; ++qz)
      for (int qy = 0; qy < nq1; ++qy)
        for (int qx = 0; qx < nq1; ++qx) {
          long q = el * nq + ((long)qz * nq1 + qy) * nq1 + qx;
          double xi[3] = {gpt[qx], gpt[qy], gpt[qz]}, uq[3];
          interp_velocity(f, e, xi, U, n_v, uq);
          if (eps_q) eps_q[q] = eps_nodes ? interp_scalar(f, e, xi, eps_nodes) : eps;
          if (beta_q) beta_q[q] = bq;
          for (int c = 0; c < 3; ++c) {
            double F = -bq * (uq[c] - ubar[c]);
            if (f->model == 1) F -= sums[(9 + c) * nel + el] / Ve;
            if (fpf_q) fpf_q[c * nel * nq + q] = F;
          }
        }
  }
  if (elem_sums) memcpy(elem_sums, sums, sizeof(double) * ES_ROWS * nel);
  free(sums);
  free(pe);
  free(pxi);
  return s->err;
}

/* ------------------------------------------------------------------------- */
/* accessors                                                                  */
/* ------------------------------------------------------------------------- */
void orc_dem_get(const orc_dem *s, double *x, double *v, double *w, double *ffp, double *Fc,
                 double *Tc) {
  size_t b = sizeof(double) * 3 * s->n;
  if (x) memcpy(x, s->x, b);
  if (v) memcpy(v, s->v, b);
  if (w) memcpy(w, s->w, b);
  if (ffp) memcpy(ffp, s->ffp, b);
  if (Fc) memcpy(Fc, s->Fc, b);
  if (Tc) memcpy(Tc, s->Tc, b);
}

void orc_dem_set_ffp(orc_dem *s, const double *ffp) {
  memcpy(s->ffp, ffp, sizeof(double) * 3 * s->n);
}

long orc_dem_ncontacts(const orc_dem *s) { return s->nh; }

void orc_dem_contacts(const orc_dem *s, long *i, long *j, double *dt) {
  for (long c = 0; c < s->nh; ++c) {
    if (i) i[c] = s->ha[c];
    if (j) j[c] = s->hb[c];
    if (dt)
      for (int k = 0; k < 3; ++k) dt[3 * c + k] = s->hdt[3 * c + k];
  }
}

int orc_dem_error(const orc_dem *s) { return s->err; }

void orc_dem_free(orc_dem *s) {
  if (!s) return;
  free(s->x);
  free(s->v);
  free(s->w);
  free(s->Fc);
  free(s->Tc);
  free(s->ffp);
  free(s->r);
  free(s->m);
  free(s->inertia);
  free(s->ha);
  free(s->hb);
  free(s->hdt);
  free(s);
}
