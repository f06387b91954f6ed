// couple_kernels.hip -- one coupling step on gfx950 (Section 2.3 of El
// Geitani, Golshan & Blais, arXiv 2211.01185), fused into one element-centric
// kernel.  One 64-lane wavefront owns one mesh element (four per block, each
// with its own LDS region, synchronized at wavefront scope only):
//   1. gathers the element's particles from its nested DEM cells (the grid
//      built at the current positions), sorts their indices in LDS so that
//      every sum below has a fixed order,
//   2. particle-centroid void fraction eps_e = 1 - sum V_p / V_e
//      (Eq. "void_fraction"),
//   3. per particle: Q_n interpolation of the fluid velocity and the Q1
//      pressure gradient from the element's nodal values staged in LDS, Di
//      Felice closure, f_fp = f_D + f_B + f_gradp (held by the DEM steps),
//   4. element sums reduced across the wave (fixed butterfly order), then the
//      quadrature-point outputs eps_q, beta_q and the force density on the
//      fluid F_pf,q = -beta_q (u_q - u_bar) [- sum f_gradp / V_e for model B]
//      (Eqs. "fa", "fb").
// No float atomics: every output element is written by exactly one wave and
// every f_fp by the wave of the particle's element.
#include "device.h"

namespace cfddem {

constexpr int kWave = 64;
constexpr int kElemPerBlock = 4;  // one wavefront per element

// LDS written by some lanes of a wavefront becomes visible to the others.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
constexpr double kPi = 3.14159265358979323846;

template <typename R>
__device__ inline R difelice_beta(R rho_f, R mu_f, R eps, R d, R slip) {
  const R r = R(0.5) * d;
  const R area = R(kPi) * r * r;
  if (slip > R(0)) {
    const R Re = rho_f * eps * slip * d / mu_f;
    const R lg = R(1.5) - log10(Re);
    const R chi = R(3.7) - R(0.65) * exp(-(lg * lg) / R(2));
    const R root = R(0.63) + R(4.8) / sqrt(Re);
    const R CD = root * root * pow(eps, R(2) - chi);
    return R(0.5) * rho_f * CD * area * slip;
  }
  // zero slip: C_D |slip| -> 4.8^2 mu_f / (rho_f eps d), chi -> 3.7
  const R lim = R(4.8 * 4.8) * mu_f / (rho_f * eps * d);
  return R(0.5) * rho_f * lim * pow(eps, R(2.0 - 3.7)) * area;
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline int wave_excl_scan(int v, int lane, int &total) {
  int incl = v;
  for (int off = 1; off < kWave; off <<= 1) {
    const int t = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += t;
  }
  total = __shfl(incl, kWave - 1, kWave);
  return incl - v;
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

template <typename R>
__global__ __launch_bounds__(kWave * kElemPerBlock) void couple_elements(Dev D, Cpl C, int p2, int p3,
                                                         const double *__restrict__ U,
                                                         const double *__restrict__ P,
                                                         double *__restrict__ eps_q,
                                                         double *__restrict__ beta_q,
                                                         double *__restrict__ fpf_q,
                                                         double *__restrict__ esums) {
  __shared__ int ids_all[kElemPerBlock][kElemMaxParticles];
  __shared__ double sU_all[kElemPerBlock][3][27];
  __shared__ double sP_all[kElemPerBlock][8];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int e = blockIdx.x * kElemPerBlock + wave;
  const Grid &G = D.grid;
  if (e >= G.n_elem) return;  // whole wavefront
  int *ids = ids_all[wave];
  double(*sU)[27] = sU_all[wave];
  double *sP = sP_all[wave];
  const int n = D.n;
  const int ex = e % G.n_el[0], ey = (e / G.n_el[0]) % G.n_el[1], ez = e / (G.n_el[0] * G.n_el[1]);
  const int nqtot = G.n_elem * C.nq;

  // ---- 1. particles of this element: counts of its cells, scan, gather
  const int *cnt = D.cnt[p3];
  const int *slot = D.slot[p2];
  const double *X = D.xs[p2];
  const int base = e * G.kk;
  int mine = 0;
  for (int c = lane; c < G.kk; c += kWave) {
    int m = cnt[base + c];
    mine += m < D.cap ? m : D.cap;
  }
  int total;
  const int off = wave_excl_scan(mine, lane, total);
  if (total > kElemMaxParticles) {
    if (lane == 0) atomicOr(D.err, kErrCapacity);
    total = 0;
  }
  if (total == 0) {
    // empty element: eps = 1, no drag, nothing handed to the fluid
    for (int q = lane; q < C.nq; q += kWave) {
      const long qg = (long)e * C.nq + q;
      eps_q[qg] = 1.0;
      beta_q[qg] = 0.0;
      for (int c = 0; c < 3; ++c) fpf_q[(long)c * nqtot + qg] = 0.0;
    }
    if (esums && lane < 12) esums[lane * G.n_elem + e] = 0.0;
    return;
  }
  {
    int w = off;
    for (int c = lane; c < G.kk; c += kWave) {
      int m = cnt[base + c];
      if (m > D.cap) m = D.cap;
      const int *sl = slot + (size_t)(base + c) * D.cap;
      for (int s = 0; s < m; ++s) ids[w++] = sl[s];
    }
  }
  // pad to a power of two for the bitonic sort
  int np2 = 1;
  while (np2 < total) np2 <<= 1;
  for (int t = total + lane; t < np2; t += kWave) ids[t] = 0x7fffffff;
  wave_sync();
  for (int size = 2; size <= np2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = lane; t < np2; t += kWave) {
        const int partner = t ^ stride;
        if (partner > t) {
          const int u = ids[t], v = ids[partner];
          const bool up = (t & size) == 0;
          if ((u > v) == up) {
            ids[t] = v;
            ids[partner] = u;
          }
        }
      }
      wave_sync();
    }
  }

  // ---- 2. void fraction
  double vsum = 0.0;
  for (int t = lane; t < total; t += kWave) {
    const double r = D.rad[ids[t]];
    vsum += 4.0 / 3.0 * kPi * r * r * r;
  }
  vsum = wave_sum(vsum);
  const double eps = 1.0 - vsum / C.Ve;

  // ---- 3. per-particle forces
  const int p1 = C.order + 1;
  const int nnode = p1 * p1 * p1;
  double s_beta = 0.0, s_bu[3] = {0, 0, 0}, s_fd[3] = {0, 0, 0}, s_fg[3] = {0, 0, 0};
  if (total > 0) {
    for (int t = lane; t < nnode; t += kWave) {
      const int ia = t % p1, ib = (t / p1) % p1, ic = t / (p1 * p1);
      const long gx = (long)C.order * ex + ia, gy = (long)C.order * ey + ib, gz = (long)C.order * ez + ic;
      const long node = (gz * C.nvy + gy) * C.nvx + gx;
      const long nv = (long)C.nvx * C.nvy * ((long)C.order * G.n_el[2] + 1);
      sU[0][t] = U[node];
      sU[1][t] = U[nv + node];
      sU[2][t] = U[2 * nv + node];
    }
    if (lane < 8) {
      const int ia = lane & 1, ib = (lane >> 1) & 1, ic = lane >> 2;
      sP[lane] = P[((long)(ez + ic) * C.npy + (ey + ib)) * C.npx + (ex + ia)];
    }
    wave_sync();
    const double eps_c = fmin(1.0, fmax(eps, C.eps_min));
    for (int t = lane; t < total; t += kWave) {
      const int k = ids[t];
      double xp[3], up[3], xi[3];
      for (int c = 0; c < 3; ++c) {
        xp[c] = X[c * n + k];
        up[c] = D.v[c * n + k];
      }
      const int ee[3] = {ex, ey, ez};
      for (int a = 0; a < 3; ++a) xi[a] = (xp[a] - (G.lo[a] + (double)ee[a] * G.he[a])) * G.inv_he[a];
      double Lx[3], Ly[3], Lz[3];
      basis1d(C.order, xi[0], Lx);
      basis1d(C.order, xi[1], Ly);
      basis1d(C.order, xi[2], Lz);
      double uf[3] = {0.0, 0.0, 0.0};
      for (int ic = 0; ic < p1; ++ic)
        for (int ib = 0; ib < p1; ++ib) {
          const double wyz = Ly[ib] * Lz[ic];
          for (int ia = 0; ia < p1; ++ia) {
            const double N = Lx[ia] * wyz;
            const int t2 = (ic * p1 + ib) * p1 + ia;
            uf[0] += N * sU[0][t2];
            uf[1] += N * sU[1][t2];
            uf[2] += N * sU[2][t2];
          }
        }
      // Q1 pressure gradient: d/dx = inv_he d/dxi
      double gp[3] = {0.0, 0.0, 0.0};
      {
        const double q0[2] = {1.0 - xi[0], xi[0]}, q1[2] = {1.0 - xi[1], xi[1]}, q2[2] = {1.0 - xi[2], xi[2]};
        const double dq[2] = {-1.0, 1.0};
        for (int c8 = 0; c8 < 8; ++c8) {
          const int ia = c8 & 1, ib = (c8 >> 1) & 1, ic = c8 >> 2;
          const double Pk = sP[c8];
          gp[0] += dq[ia] * q1[ib] * q2[ic] * G.inv_he[0] * Pk;
          gp[1] += q0[ia] * dq[ib] * q2[ic] * G.inv_he[1] * Pk;
          gp[2] += q0[ia] * q1[ib] * dq[ic] * G.inv_he[2] * Pk;
        }
      }
      const double r = D.rad[k];
      const double Vp = 4.0 / 3.0 * kPi * r * r * r;
      const double sl[3] = {uf[0] - up[0], uf[1] - up[1], uf[2] - up[2]};
      const double slip = sqrt(sl[0] * sl[0] + sl[1] * sl[1] + sl[2] * sl[2]);
      const double beta =
          (double)difelice_beta<R>(R(C.rho_f), R(C.mu_f), R(eps_c), R(2.0 * r), R(slip));
      for (int c = 0; c < 3; ++c) {
        const double fD = beta * sl[c];
        const double fB = -C.rho_f * Vp * D.g[c];
        const double fG = -Vp * gp[c];
        D.ffp[c * n + k] = fD + fB + fG;
        s_bu[c] += beta * up[c];
        s_fd[c] += fD;
        s_fg[c] += fG;
      }
      s_beta += beta;
    }
  }
  s_beta = wave_sum(s_beta);
  for (int c = 0; c < 3; ++c) {
    s_bu[c] = wave_sum(s_bu[c]);
    s_fd[c] = wave_sum(s_fd[c]);
    s_fg[c] = wave_sum(s_fg[c]);
  }

  // ---- 4. quadrature-point outputs
  const double bq = s_beta / C.Ve;
  double ubar[3] = {0.0, 0.0, 0.0};
  if (total > 0 && s_beta > 0.0)
    for (int c = 0; c < 3; ++c) ubar[c] = s_bu[c] / s_beta;
  for (int q = lane; q < C.nq; q += kWave) {
    const long qg = (long)e * C.nq + q;
    const int qx = q % C.nq1, qy = (q / C.nq1) % C.nq1, qz = q / (C.nq1 * C.nq1);
    double F[3] = {0.0, 0.0, 0.0};
    if (total > 0) {
      double uq[3] = {0.0, 0.0, 0.0};
      for (int ic = 0; ic < p1; ++ic)
        for (int ib = 0; ib < p1; ++ib)
          for (int ia = 0; ia < p1; ++ia) {
            const double N = C.Lq[ia][qx] * C.Lq[ib][qy] * C.Lq[ic][qz];
            const int t2 = (ic * p1 + ib) * p1 + ia;
            uq[0] += N * sU[0][t2];
            uq[1] += N * sU[1][t2];
            uq[2] += N * sU[2][t2];
          }
      for (int c = 0; c < 3; ++c) {
        F[c] = -bq * (uq[c] - ubar[c]);
        if (C.model == 1) F[c] -= s_fg[c] / C.Ve;
      }
    }
    eps_q[qg] = eps;
    beta_q[qg] = bq;
    for (int c = 0; c < 3; ++c) fpf_q[(long)c * nqtot + qg] = F[c];
  }
  if (esums && lane == 0) {
    const int ne = G.n_elem;
    esums[0 * ne + e] = (double)total;
    esums[1 * ne + e] = vsum;
    esums[2 * ne + e] = s_beta;
    for (int c = 0; c < 3; ++c) {
      esums[(3 + c) * ne + e] = s_bu[c];
      esums[(6 + c) * ne + e] = s_fd[c];
      esums[(9 + c) * ne + e] = s_fg[c];
    }
  }
}

hipError_t launch_couple(const Dev &D, const Cpl &C, long long s, const double *U, const double *P,
                         double *eps_q, double *beta_q, double *fpf_q, double *esums, bool fp32,
                         hipStream_t st) {
  const int grid = (D.grid.n_elem + kElemPerBlock - 1) / kElemPerBlock;
  const int p2 = (int)(s & 1), p3 = (int)(s % 3);
  if (fp32)
    couple_elements<float><<<grid, kWave * kElemPerBlock, 0, st>>>(D, C, p2, p3, U, P, eps_q, beta_q,
                                                                    fpf_q, esums);
  else
    couple_elements<double><<<grid, kWave * kElemPerBlock, 0, st>>>(D, C, p2, p3, U, P, eps_q, beta_q,
                                                                     fpf_q, esums);
  return hipGetLastError();
}

}  // namespace cfddem
