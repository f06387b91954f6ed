// couple_kernels.hip -- one coupling step on gfx950 (Section 2.3 of El
// Geitani, Golshan & Blais, arXiv 2211.01185) in two kernels.  A fluidized or
// settled bed fills a small fraction of the mesh, so the step is a
// bandwidth-bound write of the outputs of every empty element (eps = 1, no
// drag, nothing handed to the fluid) and a few long, latency-bound element
// computations.
//
// couple_classify: one wavefront per kClassElems consecutive elements reads
// their cell counts (coalesced), writes the outputs of the empty ones as
// contiguous runs and appends the occupied ones to a list (one atomic per
// block).
//
// couple_occupied: one group of 16, 32, 64 or 128 threads per listed element
// (a tuning choice: groups smaller than a wavefront let one wavefront
// instruction serve several elements of few particles):
//   1. gathers the element's particles from its nested DEM cells (the grid
//      built at the current positions), cell by cell, each cell's particles
//      ordered by index, so that every sum below has an order fixed by the
//      set of particles alone; a cell holding more particles than were
//      loaded with its count (large elements of few cells) is copied by the
//      whole group and ordered by a rank sort,
//   2. particle-centroid void fraction eps_e = 1 - sum V_p / V_e
//      (Eq. "void_fraction"),
//   3. per particle (one per thread): Q_n interpolation of the fluid
//      velocity and the Q1 pressure gradient from the element's nodal values
//      staged in LDS, drag closure, f_fp = f_D + f_B + f_gradp (held by
//      the DEM steps),
//   4. element sums reduced across the group (fixed order), then the
//      quadrature-point outputs eps_q, beta_q and the force density on the
//      fluid F_pf,q = -beta_q (u_q - u_bar) [- sum f_gradp / V_e for model B]
//      (Eqs. "fa", "fb"), one (point, component) per thread.
// No float atomics: every output element is written by exactly one thread and
// every f_fp by the block of the particle's element.
#include "device.h"

namespace cfddem {

constexpr int kWave = 64;
constexpr int kPressLane = 32;      // first lane loading the element's pressure corners
constexpr int kClassElems = 8;      // elements per wavefront of the classify pass
constexpr int kClassBlock = 1024;  // 16 wavefronts: one list append per 128 elements
constexpr int kMaxCoupleBlocks = 4096;  // grid of the occupied-element pass
constexpr int kSlotPre = 4;         // slot entries per cell loaded with the counts

// LDS written by some lanes of a wavefront becomes visible to the others.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
constexpr double kPi = 3.14159265358979323846;

// Transcendentals of the drag closures: the library functions in FP64; in
// FP32 the hardware log2, exp2, 1/sqrt and 1/x (each within about 1 ulp),
// with log10 x = log2 x log10 2, e^x = 2^(x log2 e) and a^b = 2^(b log2 a).
template <typename R>
struct Tr;
template <>
struct Tr<double> {
  static __device__ inline double log10_(double x) { return log10(x); }
  static __device__ inline double log_(double x) { return log(x); }
  static __device__ inline double exp_(double x) { return exp(x); }
  static __device__ inline double pow_(double a, double b) { return pow(a, b); }
  static __device__ inline double rsqrt_(double x) { return 1.0 / sqrt(x); }
  static __device__ inline double rcp_(double x) { return 1.0 / x; }
};
template <>
struct Tr<float> {
  static constexpr float kLog10of2 = 0.30102999566398119521f;
  static constexpr float kLn2 = 0.69314718055994530942f;
  static constexpr float kLog2e = 1.44269504088896340736f;
  static __device__ inline float log10_(float x) { return __builtin_amdgcn_logf(x) * kLog10of2; }
  static __device__ inline float log_(float x) { return __builtin_amdgcn_logf(x) * kLn2; }
  static __device__ inline float exp_(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
  static __device__ inline float pow_(float a, float b) { return __builtin_amdgcn_exp2f(b * __builtin_amdgcn_logf(a)); }
  static __device__ inline float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
  static __device__ inline float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
};

// Momentum-exchange coefficient beta_p of one particle (f_D = beta_p slip) for
// the closures of Section 2.3.2 (Eq. "drag" and the per-particle drag
// expression), fluid fraction eps, diameter d, slip speed >= 0.  Re is the
// section's particle Reynolds number rho_f eps |slip| d / mu_f.  At zero slip
// every Re-dependent factor takes its limit.
//   0 Di Felice   C_D = (0.63 + 4.8 Re^-1/2)^2 eps^(2 - chi),
//                 chi = 3.7 - 0.65 exp(-(1.5 - log10 Re)^2 / 2)
//   1 Dallavalle  C_D = (0.63 + 4.8 Re^-1/2)^2
//   2 Rong        C_D = (0.63 + 4.8 Re^-1/2)^2 eps^(2 - [2.65 (eps + 1)
//                       - (5.3 - 3.5 eps) eps^2 exp(-(1.5 - log10 Re)^2 / 2)])
//                 (these three: beta = 1/2 rho_f C_D pi r^2 |slip|)
//   3 Koch-Hill   beta = 18 mu_f eps^2 / d^2 (F0 + F3 Re / 2) V_p
//   4 Beetstra    beta = 3 pi mu_f d eps F (the slip read for the printed
//                 fluid velocity)
//   5 Gidaspow    Ergun (eps < 0.8) or Wen-Yu (eps >= 0.8) per unit mixture
//                 volume, times V_p / (1 - eps)
//
// The piecewise closures choose a branch by comparing eps, eps_p or Re with a
// threshold, and the branches do not meet there (Gidaspow's two laws differ
// by O(1) at eps = 0.8).  The choice is made once in FP64 by closure_branches
// and passed in as bits, so that the FP32 path takes the branch the FP64
// definition takes; only the arithmetic inside a branch runs in R.
enum : unsigned {
  kBrMoving = 1,     // slip > 0 (else every Re-dependent factor takes its limit)
  kBrKochHillLo = 2, // Koch-Hill: eps_p < 0.4 (the rational F0)
  kBrErgun = 4,      // Gidaspow: eps < 0.8 (Ergun; else Wen-Yu)
  kBrReLo = 8        // Gidaspow, Wen-Yu: Re < 1000 (else C_D = 0.44)
};
__device__ inline unsigned closure_branches(double rho_f, double mu_f, double eps, double d,
                                            double slip) {
#pragma clang fp contract(off)
  unsigned b = 0;
  // R = float: a slip that vanishes in single precision takes the zero-slip
  // limit, which the moving form approaches continuously
  if (slip > 0.0 && (float)slip > 0.0f && (float)(rho_f * eps * slip * d / mu_f) > 0.0f) b |= kBrMoving;
  if (1.0 - eps < 0.4) b |= kBrKochHillLo;
  if (eps < 0.8) b |= kBrErgun;
  if (rho_f * eps * slip * d / mu_f < 1000.0) b |= kBrReLo;
  return b;
}

template <typename R>
__device__ inline R drag_beta(int drag, R rho_f, R mu_f, R eps, R d, R slip, unsigned br) {
  using T = Tr<R>;
  const R r = R(0.5) * d;
  const R area = R(kPi) * r * r;
  const R vp = R(kPi / 6.0) * d * d * d;
  const R ep = R(1) - eps;
  const R inv_mu = T::rcp_(mu_f);
  const R Re = rho_f * eps * slip * d * inv_mu;
  const bool moving = (br & kBrMoving) != 0;
  switch (drag) {
    case 0:
    case 1:
    case 2: {
      // C_D |slip| without the voidage factor; zero slip: 4.8^2 mu_f / (rho_f eps d)
      R cds;
      if (moving) {
        const R root = R(0.63) + R(4.8) * T::rsqrt_(Re);
        cds = root * root * slip;
      } else {
        cds = R(4.8 * 4.8) * mu_f * T::rcp_(rho_f * eps * d);
      }
      R expo = R(0);
      if (drag != 1) {
        R bump = R(0);  // exp(-(1.5 - log10 Re)^2 / 2), 0 at zero slip
        if (moving) {
          const R lg = R(1.5) - T::log10_(Re);
          bump = T::exp_(-(lg * lg) * R(0.5));
        }
        expo = drag == 0 ? R(2) - (R(3.7) - R(0.65) * bump)
                         : R(2) - (R(2.65) * (eps + R(1)) - (R(5.3) - R(3.5) * eps) * eps * eps * bump);
      }
      return R(0.5) * rho_f * cds * (drag == 1 ? R(1) : T::pow_(eps, expo)) * area;
    }
    case 3: {
      R F0;
      if (br & kBrKochHillLo) {
        const R lnterm = ep > R(0) ? R(135.0 / 64.0) * ep * T::log_(ep) : R(0);
        F0 = (R(1) + R(3) * sqrt(ep * R(0.5)) + lnterm + R(16.14) * ep) /
             (R(1) + R(0.681) * ep - R(8.48) * ep * ep + R(8.14) * ep * ep * ep);
      } else {
        F0 = R(10) * ep / (eps * eps * eps);
      }
      const R e2 = eps * eps;
      const R F3 = R(0.0673) + R(0.212) * ep + R(0.0232) / (e2 * e2 * eps);
      return R(18) * mu_f * e2 / (d * d) * (F0 + R(0.5) * F3 * Re) * vp;
    }
    case 4: {
      const R e2 = eps * eps;
      R F = R(10) * ep / e2 + e2 * (R(1) + R(1.5) * sqrt(ep));
      if (moving) {
        const R num = R(1) / eps + R(3) * ep * eps + R(8.4) * T::pow_(Re, R(-0.343));
        const R den = R(1) + T::pow_(R(10), R(3) * ep) * T::pow_(Re, -(R(1) + R(4) * ep) * R(0.5));
        F += R(0.413) * Re / (R(24) * e2) * num / den;
      }
      return R(3.0 * kPi) * mu_f * d * eps * F;
    }
    default: {  // 5
      if (br & kBrErgun) return vp * (R(150) * ep * mu_f / (eps * d * d) + R(1.75) * rho_f * slip / d);
      R cds;  // C_D |slip|; zero slip: 24 mu_f / (rho_f eps d)
      if (moving)
        cds = ((br & kBrReLo) ? R(24) * T::rcp_(Re) * (R(1) + R(0.15) * T::pow_(Re, R(0.687))) : R(0.44)) * slip;
      else
        cds = R(24) * mu_f * T::rcp_(rho_f * eps * d);
      return vp * R(0.75) * cds * eps * rho_f / d * T::pow_(eps, R(-2.65));
    }
  }
}

// Butterfly sums over aligned groups of W lanes (W a power of two <= 64),
// level by level so that the lane exchanges of a level are in flight
// together.  Only the first `active` lanes of the group may hold nonzero
// values: the levels whose partners all lie past them only add zeros to the
// first lanes and are skipped, so lane 0 of the group gets the same sum.
template <int W, int N>
__device__ inline void group_sum_n(double (&v)[N], int active) {
#pragma unroll
  for (int off = W / 2; off >= 1; off >>= 1) {
    if (off >= active) continue;
    double t[N];
#pragma unroll
    for (int j = 0; j < N; ++j) t[j] = __shfl_xor(v[j], off, kWave);
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] += t[j];
  }
}

// Inclusive scan over aligned groups of W lanes; lane is the index in the group.
template <int W>
__device__ inline int group_incl_scan(int v, int lane) {
#pragma unroll
  for (int off = 1; off < W; off <<= 1) {
    const int t = __shfl_up(v, off, W);
    if (lane >= off) v += t;
  }
  return v;
}

// 1D Lagrange basis on equispaced nodes of [0,1] and its derivative (Q1).
__device__ inline void basis1d(int order, double t, double L[3]) {
  if (order == 2) {
    L[0] = 2.0 * (t - 0.5) * (t - 1.0);
    L[1] = -4.0 * t * (t - 1.0);
    L[2] = 2.0 * t * (t - 0.5);
  } else {
    L[0] = 1.0 - t;
    L[1] = t;
    L[2] = 0.0;
  }
}

// First and second derivatives of the 1D basis with respect to t.
__device__ inline void basis1d_deriv(int order, double t, double d1[3], double d2[3]) {
  if (order == 2) {
    d1[0] = 4.0 * t - 3.0;
    d1[1] = 4.0 - 8.0 * t;
    d1[2] = 4.0 * t - 1.0;
    d2[0] = 4.0;
    d2[1] = -8.0;
    d2[2] = 4.0;
  } else {
    d1[0] = -1.0;
    d1[1] = 1.0;
    d1[2] = 0.0;
    d2[0] = d2[1] = d2[2] = 0.0;
  }
}

// Divergence of the fluid stress (Eq. "stress") at local coordinates xi of an
// element whose nodal velocities are sU:
//   div tau = mu_f (lap u + grad(div u) / 3),
// from the second derivatives of the Q_n field, sum-factorized axis by axis.
template <int ORD>
__device__ inline void div_tau(const double xi[3], const double (*sU)[27], const double inv_he[3],
                               double mu_f, double out[3]) {
  constexpr int p1 = ORD + 1;
  double V[3][3], D1[3][3], D2[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    basis1d(ORD, xi[a], V[a]);
    basis1d_deriv(ORD, xi[a], D1[a], D2[a]);
  }
  // per component c the second derivatives of u_c; kept are its Laplacian
  // and its terms of grad(div u) (d_a d_c u_c for each axis a)
  double lap[3], gdiv[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double hxx = 0.0, hyy = 0.0, hzz = 0.0, hxy = 0.0, hxz = 0.0, hyz = 0.0;
#pragma unroll
    for (int ic = 0; ic < p1; ++ic) {
      double sxx = 0.0, syy = 0.0, s00 = 0.0, sxy = 0.0, s10 = 0.0, s01 = 0.0;
#pragma unroll
      for (int ib = 0; ib < p1; ++ib) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int ia = 0; ia < p1; ++ia) {
          const double u = sU[c][(ic * p1 + ib) * p1 + ia];
          a0 += V[0][ia] * u;
          a1 += D1[0][ia] * u;
          a2 += D2[0][ia] * u;
        }
        sxx += V[1][ib] * a2;
        syy += D2[1][ib] * a0;
        s00 += V[1][ib] * a0;
        sxy += D1[1][ib] * a1;
        s10 += V[1][ib] * a1;
        s01 += D1[1][ib] * a0;
      }
      hxx += V[2][ic] * sxx;
      hyy += V[2][ic] * syy;
      hzz += D2[2][ic] * s00;
      hxy += V[2][ic] * sxy;
      hxz += D1[2][ic] * s10;
      hyz += D1[2][ic] * s01;
    }
    hxx *= inv_he[0] * inv_he[0];
    hyy *= inv_he[1] * inv_he[1];
    hzz *= inv_he[2] * inv_he[2];
    hxy *= inv_he[0] * inv_he[1];
    hxz *= inv_he[0] * inv_he[2];
    hyz *= inv_he[1] * inv_he[2];
    lap[c] = hxx + hyy + hzz;
    gdiv[0] += c == 0 ? hxx : (c == 1 ? hxy : hxz);
    gdiv[1] += c == 0 ? hxy : (c == 1 ? hyy : hyz);
    gdiv[2] += c == 0 ? hxz : (c == 1 ? hyz : hzz);
    // one component's nodal values in flight at a time (bounds the registers)
    __asm__ volatile("" ::: "memory");
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c] = mu_f * (lap[c] + gdiv[c] / 3.0);
}


// Di Felice (closure 0), the default.  The element kernels are instantiated
// per MODE: 0 when every bed uses Di Felice without the shear force, 1 for
// any closure, 2 for any closure with the shear force, so that each path
// keeps only the code and registers it needs.
template <typename R>
__device__ inline R difelice_beta(R rho_f, R mu_f, R eps, R d, R slip, unsigned br) {
  using T = Tr<R>;
  const R r = R(0.5) * d;
  const R area = R(kPi) * r * r;
  R cds, expo;
  if (br & kBrMoving) {
    const R Re = rho_f * eps * slip * d * T::rcp_(mu_f);
    const R root = R(0.63) + R(4.8) * T::rsqrt_(Re);
    const R lg = R(1.5) - T::log10_(Re);
    cds = root * root * slip;
    expo = R(2) - (R(3.7) - R(0.65) * T::exp_(-(lg * lg) * R(0.5)));
  } else {
    cds = R(4.8 * 4.8) * mu_f * T::rcp_(rho_f * eps * d);
    expo = R(2.0 - 3.7);
  }
  return R(0.5) * rho_f * cds * T::pow_(eps, expo) * area;
}

// Per-particle step 3 of one element: interpolation, closure, f_fp, and the
// thread's running element sums.
template <typename R, int ORD, int MODE>
__device__ inline void particle_force(const Dev &D, const Cpl &C, int k, const int ee[3],
                                      const double xp[3], const double up[3], double r,
                                      double eps_c, const double (*sU)[27], const double *sP,
                                      const double *sE,
                                      double sums[10]) {
  const Grid &G = D.grid;
  const int n = D.n;
  constexpr int p1 = ORD + 1;
  double xi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) xi[a] = (xp[a] - (G.lo[a] + (double)ee[a] * G.he[a])) * G.inv_he[a];
  double Lx[3], Ly[3], Lz[3];
  basis1d(ORD, xi[0], Lx);
  basis1d(ORD, xi[1], Ly);
  basis1d(ORD, xi[2], Lz);
  double uf[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int ic = 0; ic < p1; ++ic) {
      double acc_c = 0.0;
#pragma unroll
      for (int ib = 0; ib < p1; ++ib) {
        double acc_b = 0.0;
#pragma unroll
        for (int ia = 0; ia < p1; ++ia) acc_b += Lx[ia] * sU[c][(ic * p1 + ib) * p1 + ia];
        acc_c += Ly[ib] * acc_b;
      }
      uf[c] += Lz[ic] * acc_c;
      // one layer of nodal values in flight at a time (bounds the registers)
      __asm__ volatile("" ::: "memory");
    }
  }
  // Q1 pressure gradient, d/dx = inv_he d/dxi, from the differences of the
  // corner values along each axis
  double gp[3];
  {
    const double q0[2] = {1.0 - xi[0], xi[0]}, q1[2] = {1.0 - xi[1], xi[1]}, q2[2] = {1.0 - xi[2], xi[2]};
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        g0 += q1[i] * q2[j] * (sP[1 + 2 * i + 4 * j] - sP[2 * i + 4 * j]);
        g1 += q0[i] * q2[j] * (sP[i + 2 + 4 * j] - sP[i + 4 * j]);
        g2 += q0[i] * q1[j] * (sP[i + 2 * j + 4] - sP[i + 2 * j]);
      }
    gp[0] = g0 * G.inv_he[0];
    gp[1] = g1 * G.inv_he[1];
    gp[2] = g2 * G.inv_he[2];
  }
  const double Vp = 4.0 / 3.0 * kPi * r * r * r;
  const double sl[3] = {uf[0] - up[0], uf[1] - up[1], uf[2] - up[2]};
  const double slip = sqrt(sl[0] * sl[0] + sl[1] * sl[1] + sl[2] * sl[2]);
  constexpr bool GEN = MODE >= 1;
  if (MODE == 2 && C.smooth) {
    // smoothed void fraction: the continuous field at the particle
    double ev = 0.0;
#pragma unroll
    for (int ic = 0; ic < p1; ++ic) {
      double acc_c = 0.0;
#pragma unroll
      for (int ib = 0; ib < p1; ++ib) {
        double acc_b = 0.0;
#pragma unroll
        for (int ia = 0; ia < p1; ++ia) acc_b += Lx[ia] * sE[(ic * p1 + ib) * p1 + ia];
        acc_c += Ly[ib] * acc_b;
      }
      ev += Lz[ic] * acc_c;
    }
    eps_c = fmin(1.0, fmax(ev, C.eps_min));
  }
  const unsigned br = closure_branches(C.rho_f, C.mu_f, eps_c, 2.0 * r, slip);
  double beta = GEN ? (double)drag_beta<R>(C.drag, R(C.rho_f), R(C.mu_f), R(eps_c), R(2.0 * r), R(slip), br)
                    : (double)difelice_beta<R>(R(C.rho_f), R(C.mu_f), R(eps_c), R(2.0 * r), R(slip), br);
  if (C.beta_over_eps) beta /= eps_c;  // beta_B = beta_A / eps (Eq. "beta")
  // shear force -V_p div tau (Eqs. "fa", "fb"), when enabled; added as a
  // separate term, so that a bed without it computes the same arithmetic in
  // every instantiation
  const bool shear = MODE == 2 && C.shear;
  double dtau[3] = {0.0, 0.0, 0.0};
  if (shear) div_tau<ORD>(xi, sU, G.inv_he, C.mu_f, dtau);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double fD = beta * sl[c];
    const double fB = -C.rho_f * Vp * D.g[c];
    const double fG = -Vp * gp[c];
    double f = fD + fB + fG;
    double g = sums[7 + c] + fG;  // undisturbed-flow forces
    if (shear) {
      const double fS = -Vp * dtau[c];
      f += fS;
      g += fS;
    }
    glb(D.ffp)[c * n + k] = f;
    sums[1 + c] += beta * up[c];
    sums[4 + c] += fD;
    sums[7 + c] = g;
  }
  sums[0] += beta;
}

// Sorts a few register values ascending (odd-even transposition).
template <int N>
__device__ inline void sort_small(int (&v)[N]) {
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int i = r & 1; i + 1 < N; i += 2) {
      const int a = v[i], b = v[i + 1];
      v[i] = a < b ? a : b;
      v[i + 1] = a < b ? b : a;
    }
}

// Inserts the slot entries [from, m) of a cell into the sorted run ids[w, w+from).
__device__ inline void insert_rest(int *ids, int w, gptr<const int> sl, int from, int m) {
  for (int s = from; s < m; ++s) {
    const int v = sl[s];
    int k = w + s;
    while (k > w && ids[k - 1] > v) {
      ids[k] = ids[k - 1];
      --k;
    }
    ids[k] = v;
  }
}

// Cell of entry j of the gathered list: the last cell whose run starts at or
// before j (runs of empty cells have no entries, so that cell's run holds j).
__device__ inline int cell_of_entry(const int *coff, int kk, int j) {
  int lo = 0, hi = kk - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (coff[mid] <= j)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Particles one element may hold when computed by NT threads (more raise the
// capacity error): groups smaller than a wavefront share its LDS.
template <int NT>
constexpr int elem_capacity() {
  return NT >= kWave ? kElemMaxParticles : 16 * NT;
}

// Wavefronts of the NT threads computing one element (1 for a group of a
// wavefront).
template <int NT>
constexpr int elem_waves() {
  return NT > kWave ? NT / kWave : 1;
}

// LDS of one element computed by NT threads.
template <int NT>
struct CplShared {
  int ids[elem_capacity<NT>()];
  int raw[elem_capacity<NT>()];  // slot entries in slot order (cooperative gather)
  int coff[NT];                  // offset of each cell's run in ids (cooperative gather)
  double sU[3][27];
  double sP[8];
  double sE[27];     // smoothed void fraction at the element's velocity nodes
  double red[elem_waves<NT>()][11];
  int scan[elem_waves<NT>()];
  int longc[elem_waves<NT>()];
};

// Barrier of the NT threads computing an element: the block for 128, else a
// wavefront barrier (the group is a wavefront or a part of one; the groups of
// a wavefront may be on different branches, which a wavefront executes one
// after the other).
template <int NT>
__device__ inline void cpl_sync() {
  if constexpr (NT <= kWave)
    wave_sync();
  else
    __syncthreads();
}

// One occupied element, computed by NT threads (16, 32, 64 or 128, a tuning
// choice): a group of 16 or 32 lanes, so that a wavefront computes 4 or 2
// elements of few particles at once (every wavefront instruction serves all
// of them), a whole wavefront, or a 128-thread block taking up to 128
// particles in one pass.  Particle t of the element's ordered list is
// handled by thread t mod NT.  The latency is a short chain of memory round
// trips: counts, slot entries and nodal values are loaded together, then the
// particles' state, then the outputs are stored.
template <typename R, int ORD, int MODE, int NT>
__device__ __forceinline__ void couple_element(const Dev &D, const Cpl &C, int e, const double *__restrict__ U,
                               const double *__restrict__ P, double *__restrict__ eps_q,
                               double *__restrict__ beta_q, double *__restrict__ fpf_q,
                               double *__restrict__ esums, int p2, int p3, CplShared<NT> &sh,
                               const double (&sLq)[3][3]) {
  constexpr int kCplThreads = NT;
  constexpr int kCplWaves = elem_waves<NT>();
  constexpr int GW = NT < kWave ? NT : kWave;  // lanes of this element in one wavefront
  const Grid &G = D.grid;
  const int n = D.n;
  const int tid = threadIdx.x & (NT - 1);
  const int lane = tid & (GW - 1);
  const int wave = tid / kWave;
  const int gbase = (int)threadIdx.x & (kWave - 1) & ~(GW - 1);  // first lane of the group
  const int ex = e % G.n_el[0], ey = (e / G.n_el[0]) % G.n_el[1], ez = e / (G.n_el[0] * G.n_el[1]);
  const int ee[3] = {ex, ey, ez};
  // every array through a global-typed pointer: in the batched kernels the
  // pointers come from device tables, and generic ones would give FLAT
  // instructions
  const gptr<const double> Ug = glb(U), Pg = glb(P);
  const gptr<double> eps_g = glb(eps_q), beta_g = glb(beta_q), fpf_g = glb(fpf_q), esums_g = glb(esums);
  constexpr int p1 = ORD + 1;
  constexpr int nnode = p1 * p1 * p1;
  constexpr int nq = p1 * p1 * p1;  // Gauss points: order + 1 per axis
  const long nqtot = (long)G.n_elem * nq;

  // ---- nodal values of the element (at most 27): velocity on the first
  // threads (twice round for 16), pressure corners on threads 32..39 when
  // there are that many, else on the first 8
  constexpr int kNodeIter = (nnode + NT - 1) / NT;
  double un[kNodeIter][3], pk = 0.0;
#pragma unroll
  for (int k = 0; k < kNodeIter; ++k) {
    const int t = tid + k * NT;
    un[k][0] = un[k][1] = un[k][2] = 0.0;
    if (t < nnode) {
      const long nv = (long)C.nvx * C.nvy * ((long)ORD * G.n_el[2] + 1);
      const int ia = t % p1, ib = (t / p1) % p1, ic = t / (p1 * p1);
      const long node = (((long)ORD * ez + ic) * C.nvy + (long)ORD * ey + ib) * C.nvx + (long)ORD * ex + ia;
      un[k][0] = Ug[node];
      un[k][1] = Ug[nv + node];
      un[k][2] = Ug[2 * nv + node];
      if (MODE == 2 && C.smooth) sh.sE[t] = glb(C.eps_nodes)[node];  // read after the barrier below
    }
  }
  constexpr int kPL = NT >= kPressLane + 8 ? kPressLane : 0;
  static_assert(nnode <= kPressLane && NT >= 8, "nodal loads by lane");
  const int pc = tid - kPL;  // pressure corner of this thread
  if (pc >= 0 && pc < 8) {
    const int ia = pc & 1, ib = (pc >> 1) & 1, ic = pc >> 2;
    pk = Pg[((long)(ez + ic) * C.npy + (ey + ib)) * C.npx + (ex + ia)];
  }

  // ---- 1. particles of this element.  The thread owning cell c of the
  // element (c = tid first) loads its count and its first slot entries at once.
  const gptr<const int> cnt = gsel(D.cnt, p3);
  const gptr<const int> slot = gsel(D.slot, p2);
  const int base = e * G.kk;
  const int pre = D.cap < kSlotPre ? D.cap : kSlotPre;
  int m0 = 0;
  int v0[kSlotPre] = {0, 0, 0, 0};
  if (tid < G.kk) {
    m0 = cnt[base + tid];
    const gptr<const int> sl = slot + (size_t)(base + tid) * D.cap;
#pragma unroll
    for (int s = 0; s < kSlotPre; ++s) v0[s] = s < pre ? sl[s] : 0;
  }
  if (m0 > D.cap) m0 = D.cap;
  int mine = m0;
  for (int c = tid + kCplThreads; c < G.kk; c += kCplThreads) {
    const int m = cnt[base + c];
    mine += m < D.cap ? m : D.cap;
  }
  // exclusive scan of the per-thread counts over the element's threads
  const int incl = group_incl_scan<GW>(mine, lane);
  // does any cell hold more entries than were prefetched with the counts?
  const unsigned long long lmask = GW == kWave ? ~0ull : (((1ull << GW) - 1ull) << gbase);
  const bool long_cell = (__ballot(m0 > kSlotPre) & lmask) != 0ull;
  if (lane == GW - 1) {
    sh.scan[wave] = incl;
    sh.longc[wave] = long_cell ? 1 : 0;
  }
#pragma unroll
  for (int k = 0; k < kNodeIter; ++k) {
    const int t = tid + k * NT;
    if (t < nnode) {
      sh.sU[0][t] = un[k][0];
      sh.sU[1][t] = un[k][1];
      sh.sU[2][t] = un[k][2];
    }
  }
  if (pc >= 0 && pc < 8) sh.sP[pc] = pk;
  cpl_sync<NT>();
  int off = incl - mine, total = 0, any_long = 0;
#pragma unroll
  for (int w = 0; w < kCplWaves; ++w) {
    if (w < wave) off += sh.scan[w];
    total += sh.scan[w];
    any_long |= sh.longc[w];
  }
  const bool over = total > elem_capacity<NT>();
  if (over && tid == 0) __hip_atomic_fetch_or(glb(D.err), kErrCapacity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (over) total = 0;
  if (total > 0 && any_long && G.kk <= kCplThreads) {
    // one cell per thread: the slot entries are copied by the whole block
    // (entries past the prefetched ones in one round trip, whatever the
    // number of particles per cell), then each cell's run is ordered by
    // index by a rank sort (particle indices are distinct)
    if (tid < G.kk) {
      sh.coff[tid] = off;
#pragma unroll
      for (int s = 0; s < kSlotPre; ++s)
        if (s < m0) sh.raw[off + s] = v0[s];
    }
    cpl_sync<NT>();
    for (int j = tid; j < total; j += kCplThreads) {
      const int c = cell_of_entry(sh.coff, G.kk, j);
      const int s = j - sh.coff[c];
      if (s >= kSlotPre) sh.raw[j] = slot[(size_t)(base + c) * D.cap + s];
    }
    cpl_sync<NT>();
    for (int j = tid; j < total; j += kCplThreads) {
      const int c = cell_of_entry(sh.coff, G.kk, j);
      const int lo = sh.coff[c], hi = c + 1 < G.kk ? sh.coff[c + 1] : total;
      const int v = sh.raw[j];
      int r = 0;
      for (int k = lo; k < hi; ++k) r += sh.raw[k] < v ? 1 : 0;
      sh.ids[lo + r] = v;
    }
  } else if (total > 0) {
    // each thread writes its cells' particles ordered by index, so the order
    // of ids depends on the set of particles alone
    int w = off;
    if (tid < G.kk) {
#pragma unroll
      for (int s = 0; s < kSlotPre; ++s)
        if (s >= m0) v0[s] = 0x7fffffff;
      sort_small(v0);
#pragma unroll
      for (int s = 0; s < kSlotPre; ++s)
        if (s < m0) sh.ids[w + s] = v0[s];
      insert_rest(sh.ids, w, slot + (size_t)(base + tid) * D.cap, kSlotPre, m0);
      w += m0;
    }
    for (int c = tid + kCplThreads; c < G.kk; c += kCplThreads) {
      int m = cnt[base + c];
      if (m > D.cap) m = D.cap;
      insert_rest(sh.ids, w, slot + (size_t)(base + c) * D.cap, 0, m);
      w += m;
    }
  }
  cpl_sync<NT>();

  // ---- 2. void fraction; the state of the thread's first particle is
  // loaded in the same round trip as its radius
  const gptr<const dvec4> X = gsel(D.pr, p2);
  const int k0 = tid < total ? sh.ids[tid] : -1;
  double x0[3] = {0.0, 0.0, 0.0}, u0[3] = {0.0, 0.0, 0.0}, r0 = 0.0;
  if (k0 >= 0) {
    const dvec4 p = X[k0];
    x0[0] = p.x;
    x0[1] = p.y;
    x0[2] = p.z;
    r0 = p.w;
#pragma unroll
    for (int c = 0; c < 3; ++c) u0[c] = glb(D.v)[c * n + k0];
  }
  double vsum = k0 >= 0 ? 4.0 / 3.0 * kPi * r0 * r0 * r0 : 0.0;
  for (int t = tid + kCplThreads; t < total; t += kCplThreads) {
    const double r = glb(D.rad)[sh.ids[t]];
    vsum += 4.0 / 3.0 * kPi * r * r * r;
  }
  // lanes of this wavefront holding particles (the others hold zeros)
  const int active = min(GW, max(0, total - wave * kWave));
  {
    double vs[1] = {vsum};
    group_sum_n<GW>(vs, active);
    vsum = vs[0];
  }
  if (lane == 0) sh.red[wave][10] = vsum;
  cpl_sync<NT>();
  vsum = 0.0;
#pragma unroll
  for (int w = 0; w < kCplWaves; ++w) vsum += sh.red[w][10];
  const double eps = 1.0 - vsum / C.Ve;

  // ---- 3. per-particle forces
  double sums[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // beta, beta u_p, f_D, f_gradp
  const double eps_c = fmin(1.0, fmax(eps, C.eps_min));
  if (k0 >= 0) particle_force<R, ORD, MODE>(D, C, k0, ee, x0, u0, r0, eps_c, sh.sU, sh.sP, sh.sE, sums);
  for (int t = tid + kCplThreads; t < total; t += kCplThreads) {
    const int k = sh.ids[t];
    const dvec4 p = X[k];
    double xp[3] = {p.x, p.y, p.z}, up[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) up[c] = glb(D.v)[c * n + k];
    particle_force<R, ORD, MODE>(D, C, k, ee, xp, up, p.w, eps_c, sh.sU, sh.sP, sh.sE, sums);
  }
  group_sum_n<GW>(sums, active);
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < 10; ++j) sh.red[wave][j] = sums[j];
  cpl_sync<NT>();
#pragma unroll
  for (int j = 0; j < 10; ++j) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kCplWaves; ++w) v += sh.red[w][j];
    sums[j] = v;
  }

  // ---- 4. quadrature-point outputs.  With 4 nq + 1 threads or more, item
  // t < 3 nq is component t / nq of F at point t % nq; otherwise item q < nq
  // is the three components at point q (same arithmetic per component).  The
  // next nq items write eps and beta, the one after them the element sums.
  // Items go round the element's threads (more than one pass only for groups
  // of 16 or 32).
  constexpr bool kPerComp = 4 * nq + 1 <= NT;
  constexpr int kFThreads = kPerComp ? 3 * nq : nq;
  constexpr int kItems = kFThreads + nq + 1;
  const double s_beta = sums[0];
  const double bq = s_beta / C.Ve;
#pragma unroll 1
  for (int t = tid; t < kItems; t += NT) {
    if (t < kFThreads) {
      const int q = kPerComp ? t % nq : t;
      const int qi[3] = {q % p1, (q / p1) % p1, q / (p1 * p1)};
      // basis values at this item's Gauss point (staged in LDS: a per-thread
      // index into the kernel arguments would turn every use into a memory
      // round trip)
      double Lg[3][p1];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < p1; ++b) Lg[a][b] = sLq[b][qi[a]];
      const int c0 = kPerComp ? t / nq : 0, c1 = kPerComp ? c0 + 1 : 3;
      for (int c = c0; c < c1; ++c) {
        double F = 0.0;
        if (total > 0) {
          double uq = 0.0;
#pragma unroll
          for (int ic = 0; ic < p1; ++ic) {
            double acc_c = 0.0;
#pragma unroll
            for (int ib = 0; ib < p1; ++ib) {
              double acc_b = 0.0;
#pragma unroll
              for (int ia = 0; ia < p1; ++ia) acc_b += Lg[0][ia] * sh.sU[c][(ic * p1 + ib) * p1 + ia];
              acc_c += Lg[1][ib] * acc_b;
            }
            uq += Lg[2][ic] * acc_c;
            __asm__ volatile("" ::: "memory");
          }
          const double ubar = s_beta > 0.0 ? sums[1 + c] / s_beta : 0.0;
          F = -bq * (uq - ubar);
          if (C.model == 1) F -= sums[7 + c] / C.Ve;
        }
        fpf_g[(long)c * nqtot + (long)e * nq + q] = F;
      }
    } else if (t < kFThreads + nq) {
      const long qg = (long)e * nq + (t - kFThreads);
      eps_g[qg] = eps;
      beta_g[qg] = bq;
    } else if (esums) {
      const int ne = G.n_elem;
      esums_g[0 * ne + e] = (double)total;
      esums_g[1 * ne + e] = vsum;
#pragma unroll
      for (int j = 0; j < 10; ++j) esums_g[(2 + j) * ne + e] = sums[j];
    }
  }
  cpl_sync<NT>();  // the LDS is reused for the next element
}

// Classification of kClassElems consecutive elements starting at e0 by one
// wavefront: empty ones get their outputs, occupied ones are appended to
// list (cap entries; entries tag | element) through the counter at cnt_word,
// which is zero before the pass, so that no element is listed twice and the
// count stays within cap; the stores are bounded by cap all the same.  The
// counter takes one atomic per block (a device-wide counter is a single
// address that every XCD contends for: one atomic per wavefront serializes a
// large mesh).
// Called by every thread of the block; s_cnt is LDS of kClassBlock / kWave + 1
// ints.  The order of the list does not matter: each listed element is
// computed on its own.
__device__ __forceinline__ void couple_classify_body(const Dev &D, const Cpl &C, int e0, int p3,
                                                     int *cnt_word, unsigned *list, long long cap,
                                                     unsigned tag,
                                                     double *__restrict__ eps_q,
                                                     double *__restrict__ beta_q,
                                                     double *__restrict__ fpf_q,
                                                     double *__restrict__ esums, int *s_cnt) {
  constexpr int kWaves = kClassBlock / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const Grid &G = D.grid;
  const int ne = e0 >= G.n_elem ? 0 : (G.n_elem - e0 < kClassElems ? G.n_elem - e0 : kClassElems);
  unsigned occupied = 0;
  if (ne > 0) {  // whole wavefront
    const gptr<const int> cnt = gsel(D.cnt, p3);
    for (int c = lane; c - lane < G.kk; c += kWave) {
      int m[kClassElems];
#pragma unroll
      for (int j = 0; j < kClassElems; ++j)
        m[j] = (j < ne && c < G.kk) ? cnt[(size_t)(e0 + j) * G.kk + c] : 0;
#pragma unroll
      for (int j = 0; j < kClassElems; ++j)
        if (__ballot(m[j] != 0)) occupied |= 1u << j;
    }
    // empty elements: eps = 1, no drag, nothing handed to the fluid; their
    // quadrature points form contiguous runs
    const int nq = C.nq;
    const long nqtot = (long)G.n_elem * nq;
    const long q0 = (long)e0 * nq;
    for (int t = lane; t < ne * nq; t += kWave) {
      if ((occupied >> (t / nq)) & 1u) continue;
      const long qg = q0 + t;
      glb(eps_q)[qg] = 1.0;
      glb(beta_q)[qg] = 0.0;
      glb(fpf_q)[qg] = 0.0;
      glb(fpf_q)[nqtot + qg] = 0.0;
      glb(fpf_q)[2 * nqtot + qg] = 0.0;
    }
    if (esums && lane < ne && !((occupied >> lane) & 1u))
      for (int k = 0; k < 12; ++k) glb(esums)[(long)k * G.n_elem + e0 + lane] = 0.0;
  }
  if (lane == 0) s_cnt[wave] = __popc(occupied);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < kWaves; ++w) tot += s_cnt[w];
    s_cnt[kWaves] = tot > 0 ? __hip_atomic_fetch_add(glb(cnt_word), tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
  }
  __syncthreads();
  if (occupied) {
    int base = s_cnt[kWaves];
    for (int w = 0; w < wave; ++w) base += s_cnt[w];
    const int at = base + __popc(occupied & ((1u << lane) - 1u));
    if (lane < ne && ((occupied >> lane) & 1u) && at < cap) glb(list)[at] = tag | (unsigned)(e0 + lane);
  }
}

// Single bed.  Occupied-element counts live in two words selected by the
// parity of the coupling call: call k appends to word k&1 and clears word
// (k+1)&1 for the next call, which nothing reads during call k.
__global__ __launch_bounds__(kClassBlock) void couple_classify(Dev D, Cpl C, int p3, int parity,
                                                               double *__restrict__ eps_q,
                                                               double *__restrict__ beta_q,
                                                               double *__restrict__ fpf_q,
                                                               double *__restrict__ esums) {
  __shared__ int s_cnt[kClassBlock / kWave + 1];
  const int gw = (blockIdx.x * kClassBlock + threadIdx.x) / kWave;
  if (gw == 0 && threadIdx.x == 0) D.err[kOccWord + (parity ^ 1)] = 0;
  couple_classify_body(D, C, gw * kClassElems, p3, D.err + kOccWord + parity, (unsigned *)D.occ,
                       D.grid.n_elem, 0u, eps_q, beta_q, fpf_q, esums, s_cnt);
}

// Elements a block computes at once (the groups of a wavefront for 16 or 32
// threads per element) and its threads.
template <int NT>
constexpr int elems_per_block() {
  return NT < kWave ? kWave / NT : 1;
}
template <int NT>
constexpr int block_threads() {
  return NT < kWave ? kWave : NT;
}
// Wavefronts per SIMD the element kernels are compiled for: 3 (168 VGPRs) for
// Di Felice alone; 2 (256 VGPRs) for the general closures, the shear force and
// the smoothed void fraction, whose extra state would otherwise spill.
template <int MODE>
constexpr int occ_waves() {
  return MODE == 0 ? 3 : 2;
}
template <int NT>
int occ_grid(long long elems) {
  const long long b = (elems + elems_per_block<NT>() - 1) / elems_per_block<NT>();
  return (int)(b < kMaxCoupleBlocks ? b : kMaxCoupleBlocks);
}

// Each group of NT threads takes one listed element at a time, up to
// kMaxCoupleBlocks blocks (blocks past the list exit at once; dispatching one
// block per mesh element would cost more than the work).  Longer lists are
// strided over the grid.
template <typename R, int ORD, int MODE, int NT>
__global__ __launch_bounds__(block_threads<NT>(), occ_waves<MODE>()) void couple_occupied(Dev D, Cpl C, int p2, int p3,
                                                                            int parity,
                                                                            const double *__restrict__ U,
                                                                            const double *__restrict__ P,
                                                                            double *__restrict__ eps_q,
                                                                            double *__restrict__ beta_q,
                                                                            double *__restrict__ fpf_q,
                                                                            double *__restrict__ esums) {
  constexpr int kG = elems_per_block<NT>();
  __shared__ CplShared<NT> sh[kG];
  __shared__ double sLq[3][3];  // 1D velocity basis at the Gauss points
  const int g = (int)threadIdx.x / NT;
  const int first = (int)blockIdx.x * kG + g;
  const int last = D.grid.n_elem - 1;
  // the list entry is read in the same round trip as the list length (the
  // list has n_elem entries)
  const int nocc = min(D.err[kOccWord + parity], D.grid.n_elem);
  const int e = D.occ[first < last ? first : last];
  __asm__ volatile("" ::: "memory");
  if ((int)blockIdx.x * kG >= nocc) return;  // whole block
  const int tid = threadIdx.x;
  if (tid < 9) sLq[tid / 3][tid % 3] = C.Lq[tid / 3][tid % 3];  // read after the element's first barrier
  if (first >= nocc) return;  // whole group (a group of a wavefront: no block barrier follows)
  couple_element<R, ORD, MODE, NT>(D, C, e, U, P, eps_q, beta_q, fpf_q, esums, p2, p3, sh[g], sLq);
  // more occupied elements than groups: the rest, strided over the grid
  for (int i = first + (int)gridDim.x * kG; i < nocc; i += (int)gridDim.x * kG)
    couple_element<R, ORD, MODE, NT>(D, C, D.occ[i], U, P, eps_q, beta_q, fpf_q, esums, p2, p3, sh[g], sLq);
}

// ---------------------------------------------------------------------------
// batched coupling: every bed of a batch, one occupied-element list
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kClassBlock) void couple_classify_batch(
    const Dev *__restrict__ tab, const Cpl *__restrict__ ctab, const CplIO *__restrict__ iot,
    const BedRun *__restrict__ run, const unsigned *__restrict__ map, int *cnt_words, unsigned *list,
    ModeLists ml, long long list_len) {
  __shared__ int s_cnt[kClassBlock / kWave + 1];
  const unsigned mb = map[blockIdx.x];
  const int b = (int)(mb >> kBedShift), blk = (int)(mb & kBlockMask);
  const Dev &D = tab[b];
  const Cpl &C = ctab[b];
  const CplIO &io = iot[b];
  const int p3 = (int)(run[b].s % 3);
  const int gw = blk * (kClassBlock / kWave) + (int)(threadIdx.x / kWave);
  // occupied elements go to the list of the bed's element-kernel variant
  const int m = cpl_mode_of(C.drag, C.shear || C.smooth);
  const long long cap = (m < 2 ? ml.off[m + 1] : list_len) - ml.off[m];
  couple_classify_body(D, C, gw * kClassElems, p3, cnt_words + m, list + ml.off[m], cap,
                       (unsigned)b << kBedShift, io.eps_q, io.beta_q, io.fpf_q, io.esums, s_cnt);
}

template <typename R, int ORD, int MODE, int NT>
__device__ __forceinline__ void couple_listed(const Dev *__restrict__ tab, const Cpl *__restrict__ ctab,
                                              const CplIO *__restrict__ iot,
                                              const BedRun *__restrict__ run, unsigned ent,
                                              CplShared<NT> &sh, double (&sLq)[3][3]) {
  const int b = (int)(ent >> kBedShift), e = (int)(ent & kBlockMask);
  const Dev &D = tab[b];
  const Cpl &C = ctab[b];
  const CplIO &io = iot[b];
  const long long s = run[b].s;
  const int tid = threadIdx.x;
  if (tid < 9) sLq[tid / 3][tid % 3] = C.Lq[tid / 3][tid % 3];  // read after the element's first barrier
  couple_element<R, ORD, MODE, NT>(D, C, e, io.U, io.P, io.eps_q, io.beta_q, io.fpf_q, io.esums, (int)(s & 1),
                                   (int)(s % 3), sh, sLq);
}

template <typename R, int ORD, int MODE, int NT>
__global__ __launch_bounds__(block_threads<NT>(), occ_waves<MODE>()) void couple_occupied_batch(
    const Dev *__restrict__ tab, const Cpl *__restrict__ ctab, const CplIO *__restrict__ iot,
    const BedRun *__restrict__ run, const int *cnt_word, const unsigned *list, long long cap) {
  constexpr int kG = elems_per_block<NT>();
  __shared__ CplShared<NT> sh[kG];
  __shared__ double sLq[3][3];
  const int g = (int)threadIdx.x / NT;
  const long long first = (long long)blockIdx.x * kG + g;
  const int nocc = (int)min((long long)*cnt_word, cap);
  unsigned ent = list[first < cap ? first : cap - 1];  // the list region has cap entries
  __asm__ volatile("" ::: "memory");
  // one call site (the element computation is inlined once); the first entry
  // is read in the same round trip as the list length.  The groups of a block
  // hold consecutive entries, so the first group has an element whenever
  // another has (it stages the basis values).
  for (long long i = first; i < nocc; i += (long long)gridDim.x * kG) {
    if (i != first) ent = list[i];
    // with a whole wavefront per element the entry is the same on every lane:
    // said so, the bed's tables are read with scalar loads into scalar
    // registers instead of into vector registers on every lane
    if (NT >= kWave) ent = __builtin_amdgcn_readfirstlane(ent);
    couple_listed<R, ORD, MODE, NT>(tab, ctab, iot, run, ent, sh[g], sLq);
  }
}

__global__ void reset_count(int *cnt_words) {
  if (blockIdx.x == 0 && threadIdx.x < 3) cnt_words[threadIdx.x] = 0;
}

// Launch of an occupied-element kernel variant: precision, velocity order,
// element-kernel mode (run time values) and threads per element.
#define CFDDEM_DISPATCH(KERNEL_CALL, fp32, order, mode, nt)                                   \
  do {                                                                                         \
    if (nt == 16) {                                                                            \
      constexpr int NT_ = 16;                                                                  \
      CFDDEM_DISPATCH_RT(KERNEL_CALL, fp32, order, mode);                                      \
    } else if (nt == 32) {                                                                     \
      constexpr int NT_ = 32;                                                                  \
      CFDDEM_DISPATCH_RT(KERNEL_CALL, fp32, order, mode);                                      \
    } else if (nt == 64) {                                                                     \
      constexpr int NT_ = 64;                                                                  \
      CFDDEM_DISPATCH_RT(KERNEL_CALL, fp32, order, mode);                                      \
    } else {                                                                                   \
      constexpr int NT_ = 128;                                                                 \
      CFDDEM_DISPATCH_RT(KERNEL_CALL, fp32, order, mode);                                      \
    }                                                                                          \
  } while (0)
#define CFDDEM_DISPATCH_RT(KERNEL_CALL, fp32, order, mode)                                     \
  do {                                                                                         \
    if (fp32) {                                                                                \
      using RT_ = float;                                                                       \
      CFDDEM_DISPATCH_O(KERNEL_CALL, order, mode);                                             \
    } else {                                                                                   \
      using RT_ = double;                                                                      \
      CFDDEM_DISPATCH_O(KERNEL_CALL, order, mode);                                             \
    }                                                                                          \
  } while (0)
#define CFDDEM_DISPATCH_O(KERNEL_CALL, order, mode)                                            \
  do {                                                                                         \
    if (order == 2) {                                                                          \
      constexpr int O_ = 2;                                                                    \
      CFDDEM_DISPATCH_M(KERNEL_CALL, mode);                                                    \
    } else {                                                                                   \
      constexpr int O_ = 1;                                                                    \
      CFDDEM_DISPATCH_M(KERNEL_CALL, mode);                                                    \
    }                                                                                          \
  } while (0)
#define CFDDEM_DISPATCH_M(KERNEL_CALL, mode)                                                   \
  do {                                                                                         \
    if (mode == 2) {                                                                           \
      constexpr int M_ = 2;                                                                    \
      KERNEL_CALL;                                                                             \
    } else if (mode == 1) {                                                                    \
      constexpr int M_ = 1;                                                                    \
      KERNEL_CALL;                                                                             \
    } else {                                                                                   \
      constexpr int M_ = 0;                                                                    \
      KERNEL_CALL;                                                                             \
    }                                                                                          \
  } while (0)

// Every bed of a batch (all of velocity order `order`, all with `nt` threads
// per element).  Occupied elements are listed per element-kernel variant
// (mode_elems[m] elements of beds in mode m, region m of the list at
// ml.off[m], counted in cnt_words[m]), and each variant present runs its own
// launch, so that every bed computes the arithmetic of its own variant
// whatever the other beds are.  The counters are zero on entry and on return.
hipError_t launch_couple_batch(const Dev *tab, const Cpl *ctab, const CplIO *iot, const BedRun *run,
                               const unsigned *map_class, int blocks_class, int *cnt_words,
                               unsigned *list, const long long mode_elems[3], int order, bool fp32, int nt,
                               hipStream_t st) {
  if (blocks_class <= 0) return hipGetLastError();
  ModeLists ml;
  ml.off[0] = 0;
  ml.off[1] = mode_elems[0];
  ml.off[2] = mode_elems[0] + mode_elems[1];
  couple_classify_batch<<<blocks_class, kClassBlock, 0, st>>>(
      tab, ctab, iot, run, map_class, cnt_words, list, ml, mode_elems[0] + mode_elems[1] + mode_elems[2]);
  for (int m = 0; m < 3; ++m) {
    if (mode_elems[m] <= 0) continue;
    CFDDEM_DISPATCH((couple_occupied_batch<RT_, O_, M_, NT_><<<occ_grid<NT_>(mode_elems[m]), block_threads<NT_>(), 0,
                                                               st>>>(tab, ctab, iot, run, cnt_words + M_,
                                                                     list + ml.off[M_], mode_elems[M_])),
                    fp32, order, m, nt);
  }
  return hipGetLastError();
}

// The occupied-element counters of a batch back to zero before a coupling
// step (after a run of steps the batch's step-advance launch does it).
hipError_t launch_reset_count(int *cnt_words, hipStream_t st) {
  reset_count<<<1, 64, 0, st>>>(cnt_words);
  return hipGetLastError();
}

// Elements of one bed covered by one block of the classify pass.
int couple_class_elems_per_block() { return kClassElems * (kClassBlock / kWave); }

hipError_t launch_couple(const Dev &D, const Cpl &C, long long s, long long call, const double *U,
                         const double *P, double *eps_q, double *beta_q, double *fpf_q,
                         double *esums, bool fp32, hipStream_t st) {
  const int p2 = (int)(s & 1), p3 = (int)(s % 3), parity = (int)(call & 1);
  const int ne = D.grid.n_elem;
  const int waves_c = (ne + kClassElems - 1) / kClassElems;
  const int grid_c = (waves_c + kClassBlock / kWave - 1) / (kClassBlock / kWave);
  couple_classify<<<grid_c, kClassBlock, 0, st>>>(D, C, p3, parity, eps_q, beta_q, fpf_q, esums);
  const int mode = cpl_mode_of(C.drag, C.shear || C.smooth);
  CFDDEM_DISPATCH((couple_occupied<RT_, O_, M_, NT_><<<occ_grid<NT_>(ne), block_threads<NT_>(), 0, st>>>(
                      D, C, p2, p3, parity, U, P, eps_q, beta_q, fpf_q, esums)),
                  fp32, C.order, mode, C.elem_threads);
  return hipGetLastError();
}

#undef CFDDEM_DISPATCH_M
#undef CFDDEM_DISPATCH_O
#undef CFDDEM_DISPATCH_RT
#undef CFDDEM_DISPATCH

}  // namespace cfddem
