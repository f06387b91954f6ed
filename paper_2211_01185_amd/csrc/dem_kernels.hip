// dem_kernels.hip -- one DEM step on gfx950 (Section 2.2 of El Geitani,
// Golshan & Blais, arXiv 2211.01185):
//   drift_bin   : half kick + drift with the stored forces, binning of the new
//                 centre into the nested cell grid (atomic slot insertion)
//   force_kick  : 27-cell broad search + fine search, Hertz-Mindlin contact
//                 law (Table "tab:viscoelastic", contact-force equation) with
//                 tangential history and Coulomb limit, per-particle gather of
//                 force and torque (no float atomics), second half kick
// Both kernels are one thread per particle over SoA FP64 arrays.  A pair is
// evaluated by both of its particles in the canonical orientation (lower
// original ID first), so both sides compute bit-identical forces and
// tangential overlaps and each stores its own copy of the history.
#include "device.h"

namespace cfddem {

// ---------------------------------------------------------------------------
// drift + binning
// ---------------------------------------------------------------------------
template <bool DRIFT>
__global__ __launch_bounds__(256) void drift_bin(Dev D, int par) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D.n) return;
  const int n = D.n;
  double xp[3];
  if (DRIFT) {
    const double m = D.mass[k];
    const double r = D.rad[k];
    const double inertia = 0.4 * m * r * r;
    for (int c = 0; c < 3; ++c) {
      const int i = c * n + k;
      const double acc = (D.Fc[i] + D.ffp[i]) / m + D.g[c];
      const double alpha = D.Tc[i] / inertia;
      const double vh = D.v[i] + 0.5 * D.dt * acc;
      const double wh = D.w[i] + 0.5 * D.dt * alpha;
      xp[c] = D.x[i] + D.dt * vh;
      D.vh[i] = vh;
      D.wh[i] = wh;
      D.x[i] = xp[c];
    }
  } else {
    for (int c = 0; c < 3; ++c) {
      const int i = c * n + k;
      xp[c] = D.x[i];
      D.vh[i] = D.v[i];
      D.wh[i] = D.w[i];
    }
  }
  int elem, cell;
  bool inside;
  bin_point(D.grid, xp, elem, cell, inside);
  int bits = 0;
  if (!inside) bits |= kErrDomain;
  if (xp[0] != xp[0] || xp[1] != xp[1] || xp[2] != xp[2]) bits |= kErrNan;
  D.cell_prev[k] = D.cell[k];
  D.cell[k] = cell;
  const int s = atomicAdd(&D.cnt[par][cell], 1);
  if (s < D.cap)
    D.slot[(size_t)cell * D.cap + s] = k;
  else
    bits |= kErrCapacity;
  if (bits) atomicOr(D.err, bits);
}

// ---------------------------------------------------------------------------
// contact law
// ---------------------------------------------------------------------------
// One contact in the orientation of the unit normal n (from the first body to
// the second; the force returned acts on the first).  Kinematics and the
// tangential history are FP64; the spring-dashpot arithmetic runs in R.
//   dn   normal overlap, vij relative contact-point velocity (first - second)
//   dto  stored tangential overlap (zeros for a new contact)
// Outputs: f = f_n + f_t, nxft = n x f_t, dtn = updated tangential overlap.
template <typename R, bool ADVANCE>
__device__ inline void contact_law(const Material &M, const double n[3], double dn,
                                   const double vij[3], double Re, double me, double dt,
                                   const double dto[3], double f[3], double nxft[3],
                                   double dtn[3]) {
  const double vn = vij[0] * n[0] + vij[1] * n[1] + vij[2] * n[2];
  double vrn[3], vrt[3];
  for (int c = 0; c < 3; ++c) {
    vrn[c] = vn * n[c];
    vrt[c] = vij[c] - vrn[c];
  }
  if (ADVANCE) {
    const double along = dto[0] * n[0] + dto[1] * n[1] + dto[2] * n[2];
    for (int c = 0; c < 3; ++c) dtn[c] = (dto[c] - along * n[c]) + vrt[c] * dt;
  } else {
    for (int c = 0; c < 3; ++c) dtn[c] = 0.0;
  }
  const R sq = sqrt(R(Re) * R(dn));
  const R kn = R(4.0 / 3.0) * R(M.Ye) * sq;
  const R kt = R(8.0) * R(M.Ge) * sq;
  const R Sn = R(2.0) * R(M.Ye) * sq;
  const R etan = R(M.eta_coef) * sqrt(Sn * R(me));
  const R etat = R(M.eta_coef) * sqrt(kt * R(me));  // S_t = k_t = 8 G_e sqrt(R_e dn)
  R fn[3], ft[3];
  for (int c = 0; c < 3; ++c) {
    fn[c] = -kn * R(dn) * R(n[c]) - etan * R(vrn[c]);
    ft[c] = -kt * R(dtn[c]) - etat * R(vrt[c]);
  }
  const R fn2 = fn[0] * fn[0] + fn[1] * fn[1] + fn[2] * fn[2];
  const R ft2 = ft[0] * ft[0] + ft[1] * ft[1] + ft[2] * ft[2];
  const R fn_mag = sqrt(fn2), ft_mag = sqrt(ft2);
  if (ft_mag > R(M.mu) * fn_mag) {  // sliding (a tie sticks)
    const R scale = R(M.mu) * fn_mag / ft_mag;
    for (int c = 0; c < 3; ++c) {
      ft[c] = ft[c] * scale;
      if (ADVANCE) dtn[c] = -(double)ft[c] / (double)kt;
    }
  }
  for (int c = 0; c < 3; ++c) f[c] = (double)(fn[c] + ft[c]);
  nxft[0] = (double)(R(n[1]) * ft[2] - R(n[2]) * ft[1]);
  nxft[1] = (double)(R(n[2]) * ft[0] - R(n[0]) * ft[2]);
  nxft[2] = (double)(R(n[0]) * ft[1] - R(n[1]) * ft[0]);
}

// ---------------------------------------------------------------------------
// contact search + forces + second half kick
// ---------------------------------------------------------------------------
// par: grid buffer built by the preceding drift_bin; the other count buffer is
// cleared at the cells of the previous binning (it is the next step's buffer).
// hold: history buffer to read; hnew: buffer to write.
template <typename R, bool ADVANCE>
__global__ __launch_bounds__(kForceBlock) void force_kick(Dev D, int par, int hold, int hnew) {
  __shared__ unsigned long long lst[kMaxContacts][kForceBlock];
  const int tx = threadIdx.x;
  const int a = blockIdx.x * kForceBlock + tx;
  if (a >= D.n) return;
  const int n = D.n;
  const Grid &G = D.grid;

  const double xa0 = D.x[a], xa1 = D.x[n + a], xa2 = D.x[2 * n + a];
  const double ra = D.rad[a];
  const int oa = D.oid[a];
  const int ca = D.cell[a];
  int g3[3];
  {
    const int el = ca / G.kk, sub = ca - el * G.kk;
    const int e0 = el % G.n_el[0], e1 = (el / G.n_el[0]) % G.n_el[1], e2 = el / (G.n_el[0] * G.n_el[1]);
    const int s0 = sub % G.k[0], s1 = (sub / G.k[0]) % G.k[1], s2 = sub / (G.k[0] * G.k[1]);
    g3[0] = e0 * G.k[0] + s0;
    g3[1] = e1 * G.k[1] + s1;
    g3[2] = e2 * G.k[2] + s2;
  }

  // ---- broad search over the 27-cell stencil, fine search, sorted insert
  int nc = 0;
  int bits = 0;
  const int *cnt = D.cnt[par];
  for (int dz = -1; dz <= 1; ++dz) {
    const int gz = g3[2] + dz;
    if (gz < 0 || gz >= G.gc[2]) continue;
    const int ez = gz / G.k[2], sz = gz - ez * G.k[2];
    for (int dy = -1; dy <= 1; ++dy) {
      const int gy = g3[1] + dy;
      if (gy < 0 || gy >= G.gc[1]) continue;
      const int ey = gy / G.k[1], sy = gy - ey * G.k[1];
      for (int dx = -1; dx <= 1; ++dx) {
        const int gx = g3[0] + dx;
        if (gx < 0 || gx >= G.gc[0]) continue;
        const int ex = gx / G.k[0], sx = gx - ex * G.k[0];
        const int c2 = ((ez * G.n_el[1] + ey) * G.n_el[0] + ex) * G.kk + (sz * G.k[1] + sy) * G.k[0] + sx;
        int m = cnt[c2];
        if (m > D.cap) m = D.cap;
        const int *sl = D.slot + (size_t)c2 * D.cap;
        for (int s = 0; s < m; ++s) {
          const int b = sl[s];
          if (b == a) continue;
          if (!touching(xa0, xa1, xa2, D.x[b], D.x[n + b], D.x[2 * n + b], ra, D.rad[b])) continue;
          const unsigned long long key =
              ((unsigned long long)(unsigned)(D.oid[b] + kWalls) << 32) | (unsigned)b;
          if (nc < D.maxc) {
            int p = nc;
            while (p > 0 && lst[p - 1][tx] > key) {
              lst[p][tx] = lst[p - 1][tx];
              --p;
            }
            lst[p][tx] = key;
            ++nc;
          } else {
            bits |= kErrCapacity;
          }
        }
      }
    }
  }
  // walls: codes 0..5 sort before every particle code
  {
    int nw = 0;
    unsigned long long wk[kWalls];
    const double xa[3] = {xa0, xa1, xa2};
    for (int wall = 0; wall < kWalls; ++wall) {
      const int ax = wall >> 1;
      const double dist = (wall & 1) ? G.hi[ax] - xa[ax] : xa[ax] - G.lo[ax];
      if (ra - dist > 0.0) wk[nw++] = (unsigned long long)wall << 32;
    }
    if (nw) {
      if (nc + nw > D.maxc) {
        bits |= kErrCapacity;
        nc = D.maxc - nw > 0 ? D.maxc - nw : 0;
      }
      for (int p = nc - 1; p >= 0; --p) lst[p + nw][tx] = lst[p][tx];
      for (int p = 0; p < nw && p < D.maxc; ++p) lst[p][tx] = wk[p];
      nc = nc + nw > D.maxc ? D.maxc : nc + nw;
    }
  }

  // ---- forces, history carried by merging the sorted old and new lists
  const double va0 = D.vh[a], va1 = D.vh[n + a], va2 = D.vh[2 * n + a];
  const double wa0 = D.wh[a], wa1 = D.wh[n + a], wa2 = D.wh[2 * n + a];
  const double ma = D.mass[a];
  const int hn_old = ADVANCE ? D.hn[hold][a] : 0;
  const int *hid_old = D.hid[hold];
  const double *hdt_old = D.hdt[hold];
  int *hid_new = D.hid[hnew];
  double *hdt_new = D.hdt[hnew];
  const size_t mn = (size_t)D.maxc * n;
  int p = 0;
  int old_code = (p < hn_old) ? hid_old[(size_t)p * n + a] : 0x7fffffff;
  double F[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};

  for (int t = 0; t < nc; ++t) {
    const unsigned long long key = lst[t][tx];
    const int code = (int)(key >> 32);
    const int b = (int)(unsigned)(key & 0xffffffffu);
    while (old_code < code) {
      ++p;
      old_code = (p < hn_old) ? hid_old[(size_t)p * n + a] : 0x7fffffff;
    }
    double dto[3] = {0.0, 0.0, 0.0};
    if (ADVANCE && old_code == code) {
      for (int c = 0; c < 3; ++c) dto[c] = hdt_old[(size_t)c * mn + (size_t)p * n + a];
    }
    double f[3], nxft[3], dtn[3], nrm[3], vij[3];
    if (code < kWalls) {
      const int ax = code >> 1;
      const double xa[3] = {xa0, xa1, xa2};
      const double dist = (code & 1) ? G.hi[ax] - xa[ax] : xa[ax] - G.lo[ax];
      nrm[0] = nrm[1] = nrm[2] = 0.0;
      nrm[ax] = (code & 1) ? 1.0 : -1.0;
      const double dn = ra - dist;
      const double rw0 = ra * wa0, rw1 = ra * wa1, rw2 = ra * wa2;
      vij[0] = va0 + (rw1 * nrm[2] - rw2 * nrm[1]);
      vij[1] = va1 + (rw2 * nrm[0] - rw0 * nrm[2]);
      vij[2] = va2 + (rw0 * nrm[1] - rw1 * nrm[0]);
      contact_law<R, ADVANCE>(D.pw, nrm, dn, vij, ra, ma, D.dt, dto, f, nxft, dtn);
      for (int c = 0; c < 3; ++c) {
        F[c] += f[c];
        T[c] += ra * nxft[c];
      }
    } else {
      const double xb0 = D.x[b], xb1 = D.x[n + b], xb2 = D.x[2 * n + b];
      const double vb0 = D.vh[b], vb1 = D.vh[n + b], vb2 = D.vh[2 * n + b];
      const double wb0 = D.wh[b], wb1 = D.wh[n + b], wb2 = D.wh[2 * n + b];
      const double rb = D.rad[b], mb = D.mass[b];
      const bool first = oa < D.oid[b];  // canonical: lower original ID is "i"
      const double xi0 = first ? xa0 : xb0, xi1 = first ? xa1 : xb1, xi2 = first ? xa2 : xb2;
      const double xj0 = first ? xb0 : xa0, xj1 = first ? xb1 : xa1, xj2 = first ? xb2 : xa2;
      const double vi0 = first ? va0 : vb0, vi1 = first ? va1 : vb1, vi2 = first ? va2 : vb2;
      const double vj0 = first ? vb0 : va0, vj1 = first ? vb1 : va1, vj2 = first ? vb2 : va2;
      const double wi0 = first ? wa0 : wb0, wi1 = first ? wa1 : wb1, wi2 = first ? wa2 : wb2;
      const double wj0 = first ? wb0 : wa0, wj1 = first ? wb1 : wa1, wj2 = first ? wb2 : wa2;
      const double ri = first ? ra : rb, rj = first ? rb : ra;
      const double mi = first ? ma : mb, mj = first ? mb : ma;
      const double d0 = xj0 - xi0, d1 = xj1 - xi1, d2 = xj2 - xi2;
      const double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      nrm[0] = d0 / dist;
      nrm[1] = d1 / dist;
      nrm[2] = d2 / dist;
      const double dn = (ri + rj) - dist;
      const double rw0 = ri * wi0 + rj * wj0, rw1 = ri * wi1 + rj * wj1, rw2 = ri * wi2 + rj * wj2;
      vij[0] = vi0 - vj0 + (rw1 * nrm[2] - rw2 * nrm[1]);
      vij[1] = vi1 - vj1 + (rw2 * nrm[0] - rw0 * nrm[2]);
      vij[2] = vi2 - vj2 + (rw0 * nrm[1] - rw1 * nrm[0]);
      const double Re = 1.0 / (1.0 / ri + 1.0 / rj);
      const double me = 1.0 / (1.0 / mi + 1.0 / mj);
      contact_law<R, ADVANCE>(D.pp, nrm, dn, vij, Re, me, D.dt, dto, f, nxft, dtn);
      const double lever = first ? ri : rj;  // torque on i: R_i n x f_t, on j: R_j n x f_t
      const double sgn = first ? 1.0 : -1.0;
      for (int c = 0; c < 3; ++c) {
        F[c] += sgn * f[c];
        T[c] += lever * nxft[c];
      }
    }
    hid_new[(size_t)t * n + a] = code;
    for (int c = 0; c < 3; ++c) hdt_new[(size_t)c * mn + (size_t)t * n + a] = dtn[c];
  }
  D.hn[hnew][a] = nc;

  for (int c = 0; c < 3; ++c) {
    D.Fc[c * n + a] = F[c];
    D.Tc[c * n + a] = T[c];
  }
  if (ADVANCE) {
    const double inertia = 0.4 * ma * ra * ra;
    double vnew[3];
    for (int c = 0; c < 3; ++c) {
      const int i = c * n + a;
      const double acc = (F[c] + D.ffp[i]) / ma + D.g[c];
      const double alpha = T[c] / inertia;
      vnew[c] = D.vh[i] + 0.5 * D.dt * acc;
      D.v[i] = vnew[c];
      D.w[i] = D.wh[i] + 0.5 * D.dt * alpha;
    }
    if (vnew[0] != vnew[0] || vnew[1] != vnew[1] || vnew[2] != vnew[2]) bits |= kErrNan;
  }
  if (F[0] != F[0] || F[1] != F[1] || F[2] != F[2]) bits |= kErrNan;
  // the other count buffer becomes the next binning's: clear what it holds
  D.cnt[par ^ 1][D.cell_prev[a]] = 0;
  if (bits) atomicOr(D.err, bits);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_drift_bin(const Dev &D, int par, bool drift, hipStream_t st) {
  const int grid = (D.n + 255) / 256;
  if (drift)
    drift_bin<true><<<grid, 256, 0, st>>>(D, par);
  else
    drift_bin<false><<<grid, 256, 0, st>>>(D, par);
  return hipGetLastError();
}

hipError_t launch_force_kick(const Dev &D, int par, int hold, int hnew, bool advance, bool fp32,
                             hipStream_t st) {
  const int grid = (D.n + kForceBlock - 1) / kForceBlock;
  if (fp32) {
    if (advance)
      force_kick<float, true><<<grid, kForceBlock, 0, st>>>(D, par, hold, hnew);
    else
      force_kick<float, false><<<grid, kForceBlock, 0, st>>>(D, par, hold, hnew);
  } else {
    if (advance)
      force_kick<double, true><<<grid, kForceBlock, 0, st>>>(D, par, hold, hnew);
    else
      force_kick<double, false><<<grid, kForceBlock, 0, st>>>(D, par, hold, hnew);
  }
  return hipGetLastError();
}

}  // namespace cfddem
