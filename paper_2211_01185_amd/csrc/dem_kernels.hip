// dem_kernels.hip -- DEM steps on gfx950 (Section 2.2 of El Geitani, Golshan
// & Blais, arXiv 2211.01185), one kernel launch per step:
//   drift_bin   : opens a run of steps: half kick + drift from the boundary
//                 state, binning of the new centres into the nested cell grid
//                 (atomic slot insertion; inside a run only for particles
//                 away from the cell they were sorted into, the others being
//                 listed by their sorted index range), displacement test that
//                 requests a new broad search
//   force_kick  : step s: broad search when requested (cell-list neighbour
//                 list over the 27-cell stencil: every pair within
//                 R_i + R_j + skin, the candidates shared out over the lanes
//                 of the particle's group and tested on their position
//                 records; sorted by partner original ID, history carried
//                 over by a binary search of the new list in LDS),
//                 fine search (exact overlap test over the list and the six
//                 walls), Hertz-Mindlin contact law (Table "tab:viscoelastic",
//                 contact-force equation) with tangential history and Coulomb
//                 limit, per-particle gather of force and torque (no float
//                 atomics), second half kick; when another step follows, also
//                 its half kick, drift, binning and displacement test
// The per-step state is kept as 32-byte records per particle (position and
// radius; half-step velocity and mass; half-step angular velocity), so that a
// partner costs a few 16-byte loads from three addresses.  A pair is
// evaluated by both of its particles, each from its own side; every quantity
// one side computes is the exact negation of, or identical to, the other
// side's, so the forces are exactly opposite and each particle keeps its own
// copy of the tangential history in its own list slot.
//
// Each kernel body takes the bed's Dev and the block index explicitly: the
// single-bed kernels pass their argument and blockIdx.x, the batched kernels
// (many independent beds in one launch) look both up in device tables.
#include <hip/hip_ext.h>

#include "device.h"

namespace cfddem {

// Binning of x into the grid of a step (counts cnt, slots sl, cells cl) and
// the displacement test against the last broad-search positions.  In a grid
// that is not exact, a particle in its home cell (home_k) takes no slot.
__device__ inline void bin_and_test(const Dev &D, int k, const double xp[3], const double xbk[3], gptr<int> cnt,
                                    gptr<int> sl, gptr<int> cl, gptr<int> flag, bool force_flag, bool exact,
                                    int home_k, int &bits) {
  int elem, cell;
  bool inside;
  bin_point(D.grid, xp, elem, cell, inside);
  if (!inside) bits |= kErrDomain;
  if (xp[0] != xp[0] || xp[1] != xp[1] || xp[2] != xp[2]) bits |= kErrNan;
  cl[k] = cell;
  if (exact || cell != home_k) {
    const int s = __hip_atomic_fetch_add(&cnt[cell], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (s >= 0 && s < D.cap)
      sl[(size_t)cell * D.cap + s] = k;
    else
      bits |= kErrCapacity;
  }
  // a list built at xb stays complete while every particle is within skin/2
  const double d0 = xp[0] - xbk[0], d1 = xp[1] - xbk[1], d2 = xp[2] - xbk[2];
  if (force_flag ? k == 0 : !(d0 * d0 + d1 * d1 + d2 * d2 <= D.trig2)) __hip_atomic_fetch_or(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// drift + binning (first step of a run; also the creation-time binning)
// ---------------------------------------------------------------------------
// p2 = s & 1, p3 = s % 3 of the step being opened; exact: the kind of its
// grid.  DRIFT = false bins the positions already in pr[p2] (creation,
// restore) and writes the step's velocity records from the boundary
// velocities.
template <bool DRIFT>
__device__ __forceinline__ void drift_bin_body(const Dev &D, int k, int p2, int p3, int force_flag, bool exact) {
  if (k >= D.n) return;
  const int n = D.n;
  double xp[3];
  const gptr<dvec4> x1 = gsel(D.pr, p2), vh = gsel(D.vm, p2), wh = gsel(D.ws, p2);
  const double m = glb(D.mass)[k];
  const double r = glb(D.rad)[k];
  if (DRIFT) {
    const dvec4 xo = gsel(D.pr, p2 ^ 1)[k];
    const double x0[3] = {xo.x, xo.y, xo.z};
    const double inertia = 0.4 * m * r * r;
    double vhc[3], whc[3];
    for (int c = 0; c < 3; ++c) {
      const int i = c * n + k;
      const double acc = (glb(D.Fc)[i] + glb(D.ffp)[i]) / m + D.g[c];
      const double alpha = glb(D.Tc)[i] / inertia;
      vhc[c] = glb(D.v)[i] + 0.5 * D.dt * acc;
      whc[c] = glb(D.w)[i] + 0.5 * D.dt * alpha;
      xp[c] = x0[c] + D.dt * vhc[c];
    }
    x1[k] = dvec4{xp[0], xp[1], xp[2], r};
    vh[k] = dvec4{vhc[0], vhc[1], vhc[2], m};
    wh[k] = dvec4{whc[0], whc[1], whc[2], 0.0};
  } else {
    const dvec4 xo = x1[k];
    xp[0] = xo.x;
    xp[1] = xo.y;
    xp[2] = xo.z;
    vh[k] = dvec4{glb(D.v)[k], glb(D.v)[n + k], glb(D.v)[2 * n + k], m};
    wh[k] = dvec4{glb(D.w)[k], glb(D.w)[n + k], glb(D.w)[2 * n + k], 0.0};
  }
  int bits = 0;
  const double xbk[3] = {glb(D.xb)[k], glb(D.xb)[n + k], glb(D.xb)[2 * n + k]};
  const int home_k = exact ? -1 : glb(D.home)[k];
  bin_and_test(D, k, xp, xbk, gsel(D.cnt, p3), gsel(D.slot, p2), gsel(D.cell, p3), glb(D.flag) + p3, force_flag != 0,
               exact, home_k, bits);
  if (bits) __hip_atomic_fetch_or(glb(D.err), bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool DRIFT>
__global__ __launch_bounds__(256) void drift_bin(Dev D, int p2, int p3, int force_flag, int exact) {
  drift_bin_body<DRIFT>(D, blockIdx.x * 256 + threadIdx.x, p2, p3, force_flag, exact != 0);
}

// Clear the counts of grid p3 at the cells its particles were binned into
// (every cell a grid of either kind can count).
__global__ void clear_grid(Dev D, int p3) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D.n) return;
  gsel(D.cnt, p3)[gsel(D.cell, p3)[k]] = 0;
  if (k == 0) glb(D.flag)[p3] = 0;
}

// ---------------------------------------------------------------------------
// contact law
// ---------------------------------------------------------------------------
// One contact in the orientation of the unit normal n (from the first body to
// the second; the force returned acts on the first).  Kinematics and the
// tangential history are FP64; the spring-dashpot arithmetic runs in R.
//   dn   normal overlap, vij relative contact-point velocity (first - second)
//   dto  stored tangential overlap (zeros for a new contact)
//   wr   relative angular velocity (first - second; the first's against a wall)
// Outputs: f = f_n + f_t, nxft = n x f_t, dtn = updated tangential overlap,
// mr = rolling torque on the first body, -mu_r R_e |f_n| wr/|wr| (zero when
// mu_r = 0 or wr = 0; Eq. "angular_momentum" names it without a form).
template <typename R, bool ADVANCE, bool ROLL>
__device__ inline void contact_law(const Material &M, const double n[3], double dn,
                                   const double vij[3], double Re, double me, double dt,
                                   const double dto[3], const double wr[3], double f[3],
                                   double nxft[3], double dtn[3], double mr[3]) {
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
  mr[0] = mr[1] = mr[2] = 0.0;
  if (ROLL && M.mu_r > 0.0) {
    const R w0 = R(wr[0]), w1 = R(wr[1]), w2 = R(wr[2]);
    const R wm = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    if (wm > R(0.0)) {
      const R s = -R(M.mu_r) * R(Re) * fn_mag / wm;
      mr[0] = (double)(s * w0);
      mr[1] = (double)(s * w1);
      mr[2] = (double)(s * w2);
    }
  }
}

// R_a w_a + R_b w_b without contraction, so that both particles of a pair
// round it identically (an FMA would fuse a different product on each side).
__device__ inline void lever_sum(double ra, double wa0, double wa1, double wa2, double rb,
                                 double wb0, double wb1, double wb2, double rw[3]) {
#pragma clang fp contract(off)
  rw[0] = ra * wa0 + rb * wb0;
  rw[1] = ra * wa1 + rb * wb1;
  rw[2] = ra * wa2 + rb * wb2;
}

// ---------------------------------------------------------------------------
// one DEM step (plus the opening of the next one when CONT)
// ---------------------------------------------------------------------------
// L consecutive lanes of a wavefront share one particle: lane l walks the list
// entries t = l, l + L, ..., lane L-1 also the walls, and the partial force
// and torque are summed over the L lanes in a fixed butterfly order.  When a
// broad search is due the group's lanes share its candidates and build the
// list in LDS; every lane then stores its own entries.  Lane 0 finishes the
// step.  p2 = s & 1, p3 = s % 3.  The grid p3 / slot buffer p2 hold x_s.
// ADVANCE = false: creation-time evaluation (no history advance, no kick).
// src: after a re-sort, the index each particle had when its list was built
//      (NULL otherwise).
// gmode: kGrid* bits, the kinds of the grids of steps s, s+1 and s-1.
template <int L>
__device__ inline double group_sum(double v) {
  for (int off = 1; off < L; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}
template <int L>
__device__ inline unsigned long long group_or(unsigned long long v) {
  for (int off = 1; off < L; off <<= 1) {
    const unsigned lo = __shfl_xor((unsigned)(v & 0xffffffffu), off, 64);
    const unsigned hi = __shfl_xor((unsigned)(v >> 32), off, 64);
    v |= ((unsigned long long)hi << 32) | lo;
  }
  return v;
}

// LDS writes of one lane become visible to the other lanes of its wavefront.
__device__ inline void wave_publish() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Broad search of particle a by the L lanes of its group over the 27-cell
// stencil of grid p3 / slot buffer p2.  Plane by plane, the nine cell counts
// are loaded together, and the plane's candidates are dealt out to the lanes
// four at a time: their slot entries in one round trip, their position
// records and original IDs in a second, then the exact test
// |x_b - x_a| < R_a + R_b + skin; the lanes then insert their passing
// candidates into the group's LDS list, sorted by partner original ID, one
// lane after the other.  Returns the list length, the same on every lane of
// the group.
// When the grid is not exact, a cell's candidates are first its home range
// (particles sorted into it at the last re-sort, whether or not they are
// still there: the exact test decides) and then its slots (particles away
// from their home cell).  A particle within the cut-off lies in the stencil,
// so every such pair is found; one listed both in its home range and in a
// slot is inserted once.
template <int L>
__device__ inline int broad_search(const Dev &D, int a, int lane, int p2, int p3, bool exact, double xa0,
                                   double xa1, double xa2, double ra, unsigned long long *my_list, int &bits) {
  constexpr int kGroups = kForceBlock / L;
  const Grid &G = D.grid;
  const int ca = gsel(D.cell, p3)[a];
  const int el = ca / G.kk, sub = ca - el * G.kk;
  const int g0 = (el % G.n_el[0]) * G.k[0] + sub % G.k[0];
  const int g1 = ((el / G.n_el[0]) % G.n_el[1]) * G.k[1] + (sub / G.k[0]) % G.k[1];
  const int g2 = (el / (G.n_el[0] * G.n_el[1])) * G.k[2] + sub / (G.k[0] * G.k[1]);
  // the index of a stencil cell is a sum of one term per axis (element part
  // plus sub-cell part); -1 marks a term outside the grid
  int tx[3], ty[3], tz[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int gx = g0 + d - 1, gy = g1 + d - 1, gz = g2 + d - 1;
    tx[d] = (gx >= 0 && gx < G.gc[0]) ? (gx / G.k[0]) * G.kk + gx % G.k[0] : -1;
    ty[d] = (gy >= 0 && gy < G.gc[1]) ? (gy / G.k[1]) * G.n_el[0] * G.kk + (gy % G.k[1]) * G.k[0] : -1;
    tz[d] = (gz >= 0 && gz < G.gc[2])
                ? (gz / G.k[2]) * G.n_el[1] * G.n_el[0] * G.kk + (gz % G.k[2]) * G.k[1] * G.k[0]
                : -1;
  }
  const gptr<const int> cnt = gsel(D.cnt, p3);
  const gptr<const int> slot = gsel(D.slot, p2);
  const gptr<const int> hbase = glb(D.base), hstart = glb(D.start);
  const gptr<const dvec4> P = gsel(D.pr, p2);
  const double rsk = ra + D.skin;
  constexpr int kCand = 4;
  const int first_lane = (threadIdx.x & 63) & ~(L - 1);
  int m = 0;
#pragma unroll
  for (int dz = 0; dz < 3; ++dz) {
    // the plane's candidates are numbered 0 .. tot-1 across its nine cells;
    // those of cell j are pf[j] .. hl[j]-1 (home range: particle q + ho[j])
    // and hl[j] .. pf[j+1]-1 (slot q - hl[j] of cell cc[j])
    int cc[9], pf[10], hl[9], ho[9];
    pf[0] = 0;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const int z = tz[dz], y = ty[j / 3], x = tx[j % 3];
      const bool in = z >= 0 && y >= 0 && x >= 0;
      cc[j] = in ? z + y + x : 0;
      const int cj = cnt[cc[j]];
      const bool imp = in && !exact;
      const int bj = imp ? hbase[cc[j]] : 0;
      const int sj = imp ? hstart[cc[j]] : 0;
      hl[j] = pf[j] + bj;
      ho[j] = sj - pf[j];
      pf[j + 1] = hl[j] + (in ? min(cj, D.cap) : 0);
    }
    const int tot = pf[9];
#pragma unroll 1
    for (int q0 = 0; q0 < tot; q0 += kCand * L) {
      // round trip 1: the candidates' slot entries; round trip 2: their
      // position records and original IDs, then the exact test
      // |x_b - x_a| < R_a + R_b + skin
      int bq[kCand];
      bool ok[kCand];
#pragma unroll
      for (int i = 0; i < kCand; ++i) {
        const int q = q0 + lane + L * i;
        ok[i] = q < tot;
        // the last cell whose first candidate is at or before q holds q
        int c = cc[0], lim = hl[0], off = ho[0];
#pragma unroll
        for (int j = 1; j < 9; ++j)
          if (q >= pf[j]) {
            c = cc[j];
            lim = hl[j];
            off = ho[j];
          }
        const bool home = q < lim;
        const size_t at = (ok[i] && !home) ? (size_t)c * D.cap + (q - lim) : 0;
        bq[i] = home ? q + off : slot[at];
        ok[i] = ok[i] && bq[i] != a;
      }
      // every candidate's loads are issued before any is tested: a test
      // written next to its load lets the compiler sink each load into the
      // test's branch, which then waits for it before the next one is issued
      unsigned oq[kCand];
      dvec4 pbq[kCand];
#pragma unroll
      for (int i = 0; i < kCand; ++i) {
        const int b = ok[i] ? bq[i] : a;
        pbq[i] = P[b];
        oq[i] = (unsigned)glb(D.oid)[b];
      }
      __asm__ __volatile__("" ::: "memory");
#pragma unroll
      for (int i = 0; i < kCand; ++i) {
        const double d0 = pbq[i].x - xa0, d1 = pbq[i].y - xa1, d2 = pbq[i].z - xa2;
        const double cut = rsk + pbq[i].w;
        ok[i] = ok[i] & (d0 * d0 + d1 * d1 + d2 * d2 < cut * cut);
      }
      // insertion by partner original ID, one lane of the group after the
      // other; the list length follows each lane's turn
#pragma unroll
      for (int l = 0; l < L; ++l) {
        if (lane == l) {
#pragma unroll
          for (int i = 0; i < kCand; ++i) {
            if (!ok[i]) continue;
            const unsigned long long key = ((unsigned long long)oq[i] << 32) | (unsigned)bq[i];
            int p = m;
            while (p > 0 && my_list[(p - 1) * kGroups] > key) --p;
            if (p > 0 && my_list[(p - 1) * kGroups] == key) continue;  // listed twice
            if (m < D.maxn) {
              for (int t = m; t > p; --t) my_list[t * kGroups] = my_list[(t - 1) * kGroups];
              my_list[p * kGroups] = key;
              ++m;
            } else {
              bits |= kErrCapacity;
            }
          }
        }
        if (L > 1) {
          wave_publish();
          m = __shfl(m, first_lane + l, 64);
        }
      }
    }
  }
  return m;
}

// One neighbour-list entry's data: the partner's position, velocity and
// spin records and the entry's stored tangential overlap.
struct Entry {
  dvec4 p, v, w;
  double h[3];
};
// b comes from a list entry; an index outside [0, n) (only a slot past the
// list's length can hold one) reads the particle itself.
__device__ __forceinline__ Entry load_entry(gptr<const dvec4> P, gptr<const dvec4> VM, gptr<const dvec4> WS,
                                            gptr<const double> hdt, int n, int a, int b, int t) {
  b = (unsigned)b < (unsigned)n ? b : a;
  Entry e;
  e.p = P[b];
  e.v = VM[b];
  e.w = WS[b];
  const size_t i = hist_at(t, n, a);
  e.h[0] = hdt[i];
  e.h[1] = hdt[i + 1];
  e.h[2] = hdt[i + 2];
  return e;
}

// ROLL: some rolling friction coefficient is nonzero (a separate
// instantiation, so that the kernels without it keep their registers).
template <typename R, bool ADVANCE, bool CONT, int L, bool ROLL>
__device__ __forceinline__ void force_kick_body(const Dev &D, int blk, int p2, int p3, const int *src, int gmode) {
  const int gid = blk * kForceBlock + threadIdx.x;
  const int a = gid / L;
  const int lane = gid % L;
  if (a >= D.n) return;  // whole groups leave together
  const int n = D.n;
  const Grid &G = D.grid;
  const int q3 = p3 == 2 ? 0 : p3 + 1;  // (s + 1) % 3
  const int r3 = p3 == 0 ? 2 : p3 - 1;  // (s - 1) % 3
  const gptr<const dvec4> P = gsel(D.pr, p2);
  const gptr<const dvec4> VM = gsel(D.vm, p2);
  const gptr<const dvec4> WS = gsel(D.ws, p2);
  const int lold = glb(D.lbuf)[p3];
  const bool rebuild = !ADVANCE || src != nullptr || glb(D.flag)[p3] != 0;
  const int cur = rebuild ? (lold ^ 1) : lold;

  const dvec4 pa = P[a];
  const double xa0 = pa.x, xa1 = pa.y, xa2 = pa.z, ra = pa.w;
  // walls touched at the last step, the cell of x_{s-1} whose count this
  // particle clears at the end and its home cell: loaded first, so that
  // waiting for them later waits for nothing else
  const unsigned wmask_a = glb(D.wmask)[a];
  const int c_old = gsel(D.cell, r3)[a];
  const int home_a = glb(D.home)[a];
  constexpr int kCand8 = 8;     // old list entries per lane and round trip
  int bits = 0;
  int m_new = 0;                // list length after a broad search
  unsigned long long carried = 0;  // entries of this lane with carried history

  // the group's list (maxn keys, stride kGroups) and, while the history is
  // carried after a broad search, the old position each new entry takes its
  // history from (maxn bytes, stride kGroups)
  extern __shared__ unsigned long long sh_list[];
  constexpr int kGroups = kForceBlock / L;
  unsigned long long *my_list = sh_list + threadIdx.x / L;
  unsigned char *my_from =
      reinterpret_cast<unsigned char *>(sh_list + (size_t)D.maxn * kGroups) + threadIdx.x / L;

  if (rebuild) {
    const int m = broad_search<L>(D, a, lane, p2, p3, (gmode & kGridCurExact) != 0, xa0, xa1, xa2, ra, my_list,
                                  bits);
    m_new = m;
    if (lane == 0) {
      gsel(D.ln, cur)[a] = m;
      glb(D.xb)[a] = xa0;
      glb(D.xb)[n + a] = xa1;
      glb(D.xb)[2 * n + a] = xa2;
    }
    // ---- tangential history of the pairs that touched at the last step:
    //      each lane finds its share of the old touching entries in the new
    //      (sorted) list by binary search in LDS and notes where each new
    //      entry's history comes from; then every lane stores its own new
    //      entries and copies their history
    const int s = src ? glb(src)[a] : a;
    const int mo = gsel(D.ln, lold)[s];
    const unsigned long long mask_old = gsel(D.hmask, lold)[s];
    const gptr<const unsigned long long> olst = gsel(D.nbr, lold);
    for (int t = lane; t < m; t += L) my_from[t * kGroups] = 0;
    wave_publish();
    if (ADVANCE) {
#pragma unroll 1
      for (int q0 = 0; q0 < mo; q0 += kCand8 * L) {
        unsigned ok_old[kCand8];
#pragma unroll
        for (int i = 0; i < kCand8; ++i) {
          const int qo = q0 + lane + L * i;
          const bool live = qo < mo && ((mask_old >> qo) & 1ull);
          ok_old[i] = live ? (unsigned)(olst[(size_t)qo * n + s] >> 32) : 0xffffffffu;
        }
#pragma unroll
        for (int i = 0; i < kCand8; ++i) {
          if (ok_old[i] == 0xffffffffu) continue;
          int lo = 0, hi = m - 1;
          while (lo <= hi) {
            const int mid = (lo + hi) >> 1;
            const unsigned om = (unsigned)(my_list[mid * kGroups] >> 32);
            if (om == ok_old[i]) {
              my_from[mid * kGroups] = (unsigned char)(q0 + lane + L * i + 1);
              break;
            }
            if (om < ok_old[i])
              lo = mid + 1;
            else
              hi = mid - 1;
          }
        }
      }
      wave_publish();
    }
    const gptr<unsigned long long> lst_new = gsel(D.nbr, cur);
    for (int t = lane; t < m; t += L) {
      lst_new[(size_t)t * n + a] = my_list[t * kGroups];
      const int from = my_from[t * kGroups];
      if (from) {
        for (int c = 0; c < 3; ++c)
          gsel(D.hdt, cur)[hist_at(t, n, a) + c] = gsel(D.hdt, lold)[hist_at(from - 1, n, s) + c];
        carried |= 1ull << t;
      }
    }
  }
  // keep the fast path's loads below the (rare) broad search, so that their
  // registers are not live across it
  __asm__ __volatile__("" ::: "memory");

  // ---- one round trip: the list header, this lane's first entry (after a
  //      broad search this lane stored its own entries and their history
  //      itself), the last broad search's position, the particle's own
  //      half-step state and held fluid force, and, on the walls' lane, the
  //      history of the first wall touched last step.  Every load is
  //      unconditional (a stale value is replaced by a select), so that no
  //      branch makes the wavefront wait for the others.
  const gptr<const unsigned long long> lst = gsel(D.nbr, cur);
  const gptr<double> hdt = gsel(D.hdt, cur);
  const unsigned long long hm = gsel(D.hmask, cur)[a];
  const int lnv = gsel(D.ln, cur)[a];
  unsigned long long key = lst[(size_t)min(lane, D.maxn - 1) * n + a];
  const dvec4 va = VM[a], wa = WS[a];
  const double va0 = va.x, va1 = va.y, va2 = va.z, ma = va.w;
  const double wa0 = wa.x, wa1 = wa.y, wa2 = wa.z;
  const unsigned wold = (ADVANCE && lane == L - 1) ? wmask_a : 0u;
  const int m = rebuild ? m_new : lnv;
  unsigned long long mask_prev = rebuild ? carried : hm;

  // ---- fine search and forces over this lane's list entries
  double F[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};
  // rolling torques, summed apart and added to T only for a bed with rolling
  // friction, so that a bed without it gets the same arithmetic in either
  // instantiation
  double Tr[3] = {0.0, 0.0, 0.0};
  unsigned long long mask_new = 0;
  const int last = D.maxn - 1;
  for (int t = lane; t < m; t += L) {
    // one round trip per entry: the partner's records, this entry's stored
    // tangential overlap and the next entry's key (its slot clamped to the
    // list capacity; past the list's length its value is not used)
    const Entry cur_e = load_entry(P, VM, WS, hdt, n, a, (int)(unsigned)(key & 0xffffffffu), t);
    key = lst[(size_t)min(t + L, last) * n + a];
    const dvec4 pb = cur_e.p, vb = cur_e.v, wb = cur_e.w;
    const double rb = pb.w;
    if (!touching(xa0, xa1, xa2, pb.x, pb.y, pb.z, ra, rb)) continue;
    const bool had = ADVANCE && ((mask_prev >> t) & 1ull);
    const double dto[3] = {had ? cur_e.h[0] : 0.0, had ? cur_e.h[1] : 0.0, had ? cur_e.h[2] : 0.0};
    const double mb = vb.w;
    // Evaluated from this particle's side.  Every quantity the partner
    // computes from its side is the exact negation (d, n, relative velocity,
    // tangential overlap, force) or identical (|d|, dn, R_e, m_e, n x f_t), so
    // the two sides stay bit-consistent: force on b = -force on a exactly.
    const double d0 = pb.x - xa0, d1 = pb.y - xa1, d2 = pb.z - xa2;
    const double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    double nrm[3], vij[3], rw[3], f[3], nxft[3], dtn[3], mr[3];
    nrm[0] = d0 / dist;
    nrm[1] = d1 / dist;
    nrm[2] = d2 / dist;
    const double dn = (ra + rb) - dist;
    lever_sum(ra, wa0, wa1, wa2, rb, wb.x, wb.y, wb.z, rw);
    vij[0] = va0 - vb.x + (rw[1] * nrm[2] - rw[2] * nrm[1]);
    vij[1] = va1 - vb.y + (rw[2] * nrm[0] - rw[0] * nrm[2]);
    vij[2] = va2 - vb.z + (rw[0] * nrm[1] - rw[1] * nrm[0]);
    const double Re = 1.0 / (1.0 / ra + 1.0 / rb);
    const double me = 1.0 / (1.0 / ma + 1.0 / mb);
    const double wr[3] = {wa0 - wb.x, wa1 - wb.y, wa2 - wb.z};
    contact_law<R, ADVANCE, ROLL>(D.pp, nrm, dn, vij, Re, me, D.dt, dto, wr, f, nxft, dtn, mr);
    for (int c = 0; c < 3; ++c) {
      F[c] += f[c];
      T[c] += ra * nxft[c];  // R_a n x f_t (n x f_t is the same from both sides)
      if (ROLL) Tr[c] += mr[c];  // the partner's is the exact negation
      hdt[hist_at(t, n, a) + c] = dtn[c];
    }
    mask_new |= 1ull << t;
  }
  // ---- walls (last lane of the group)
  if (lane == L - 1) {
    unsigned wnew = 0;
    for (int wall = 0; wall < kWalls; ++wall) {
      // axis quantities by selection (no run-time index into the grid)
      const int ax = wall >> 1;
      const double xax = ax == 0 ? xa0 : (ax == 1 ? xa1 : xa2);
      const double face = (wall & 1) ? (ax == 0 ? G.hi[0] : (ax == 1 ? G.hi[1] : G.hi[2]))
                                     : (ax == 0 ? G.lo[0] : (ax == 1 ? G.lo[1] : G.lo[2]));
      const double dist = (wall & 1) ? face - xax : xax - face;
      if (!(ra - dist > 0.0)) continue;
      const double sgn = (wall & 1) ? 1.0 : -1.0;
      double nrm[3], vij[3], dto[3] = {0.0, 0.0, 0.0}, f[3], nxft[3], dtn[3], mr[3];
      nrm[0] = ax == 0 ? sgn : 0.0;
      nrm[1] = ax == 1 ? sgn : 0.0;
      nrm[2] = ax == 2 ? sgn : 0.0;
      const double dn = ra - dist;
      const double rw0 = ra * wa0, rw1 = ra * wa1, rw2 = ra * wa2;
      vij[0] = va0 + (rw1 * nrm[2] - rw2 * nrm[1]);
      vij[1] = va1 + (rw2 * nrm[0] - rw0 * nrm[2]);
      vij[2] = va2 + (rw0 * nrm[1] - rw1 * nrm[0]);
      if ((wold >> wall) & 1u)
        for (int c = 0; c < 3; ++c) dto[c] = glb(D.whdt)[hist_at(wall, n, a) + c];
      const double wr[3] = {wa0, wa1, wa2};
      contact_law<R, ADVANCE, ROLL>(D.pw, nrm, dn, vij, ra, ma, D.dt, dto, wr, f, nxft, dtn, mr);
      for (int c = 0; c < 3; ++c) {
        F[c] += f[c];
        T[c] += ra * nxft[c];
        if (ROLL) Tr[c] += mr[c];
        glb(D.whdt)[hist_at(wall, n, a) + c] = dtn[c];
      }
      wnew |= 1u << wall;
    }
    if (wnew != wold || !ADVANCE) glb(D.wmask)[a] = (unsigned char)wnew;
  }
  for (int c = 0; c < 3; ++c) {
    F[c] = group_sum<L>(F[c]);
    T[c] = group_sum<L>(T[c]);
  }
  if (ROLL && (D.pp.mu_r > 0.0 || D.pw.mu_r > 0.0))
    for (int c = 0; c < 3; ++c) T[c] += group_sum<L>(Tr[c]);
  mask_new = group_or<L>(mask_new);
  mask_prev = group_or<L>(mask_prev);
  if (lane != 0) {
    if (bits) __hip_atomic_fetch_or(glb(D.err), bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }

  // ---- lane 0: store the step, open the next one.  Inside a run the
  //      boundary velocities and the stored force/torque are never read, so
  //      only the last step of a run stores them.
  if (rebuild || mask_new != mask_prev) gsel(D.hmask, cur)[a] = mask_new;
  if (!CONT) {
    for (int c = 0; c < 3; ++c) {
      glb(D.Fc)[c * n + a] = F[c];
      glb(D.Tc)[c * n + a] = T[c];
    }
  }
  if (F[0] != F[0] || F[1] != F[1] || F[2] != F[2]) bits |= kErrNan;
  // the grid of step s-1 is free: clear it for step s+2 (where it was not
  // exact, only particles away from their home cell were counted)
  if ((gmode & kGridPrevExact) || c_old != home_a) gsel(D.cnt, r3)[c_old] = 0;

  if (ADVANCE) {
    const double fa[3] = {glb(D.ffp)[a], glb(D.ffp)[n + a], glb(D.ffp)[2 * n + a]};
    const double xbl[3] = {glb(D.xb)[a], glb(D.xb)[n + a], glb(D.xb)[2 * n + a]};
    const double xba[3] = {rebuild ? xa0 : xbl[0], rebuild ? xa1 : xbl[1], rebuild ? xa2 : xbl[2]};
    const double inertia = 0.4 * ma * ra * ra;
    double vb[3], wb[3], acc[3], alpha[3];
    for (int c = 0; c < 3; ++c) {
      const int i = c * n + a;
      acc[c] = (F[c] + fa[c]) / ma + D.g[c];
      alpha[c] = T[c] / inertia;
      vb[c] = (c == 0 ? va0 : (c == 1 ? va1 : va2)) + 0.5 * D.dt * acc[c];
      wb[c] = (c == 0 ? wa0 : (c == 1 ? wa1 : wa2)) + 0.5 * D.dt * alpha[c];
      if (!CONT) {
        glb(D.v)[i] = vb[c];
        glb(D.w)[i] = wb[c];
      }
    }
    if (vb[0] != vb[0] || vb[1] != vb[1] || vb[2] != vb[2]) bits |= kErrNan;
    if (CONT) {
      // open step s+1 with the same held fluid force
      double xp[3], vh[3], wh[3];
      const double xa[3] = {xa0, xa1, xa2};
      for (int c = 0; c < 3; ++c) {
        vh[c] = vb[c] + 0.5 * D.dt * acc[c];
        wh[c] = wb[c] + 0.5 * D.dt * alpha[c];
        xp[c] = xa[c] + D.dt * vh[c];
      }
      gsel(D.pr, p2 ^ 1)[a] = dvec4{xp[0], xp[1], xp[2], ra};
      gsel(D.vm, p2 ^ 1)[a] = dvec4{vh[0], vh[1], vh[2], ma};
      gsel(D.ws, p2 ^ 1)[a] = dvec4{wh[0], wh[1], wh[2], 0.0};
      bin_and_test(D, a, xp, xba, gsel(D.cnt, q3), gsel(D.slot, p2 ^ 1), gsel(D.cell, q3), glb(D.flag) + q3, false,
                   (gmode & kGridNextExact) != 0, home_a, bits);
    }
  }
  if (a == 0) {
    glb(D.flag)[r3] = 0;
    if (!CONT) glb(D.flag)[q3] = 0;
    glb(D.lbuf)[q3] = cur;
  }
  if (bits) __hip_atomic_fetch_or(glb(D.err), bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroups go to the eight XCDs in turn (workgroup i to XCD i % 8), and
// each XCD has its own L2.  Block i takes the particle block that gives every
// XCD one contiguous range of the cell-sorted particles, so that a particle's
// neighbours are mostly read through the L2 that already holds them.
constexpr int kXcds = 8;
__device__ inline int xcd_block(int i, int nb) {
  const int q = nb / kXcds, r = nb % kXcds, x = i % kXcds;
  return x * q + min(x, r) + i / kXcds;
}

// Runs of C consecutive blocks dealt to the XCDs in turn (the k-th run of XCD
// x is run 8k + x), the ragged end of the grid in the single bed's XCD order:
// spatial neighbours stay in one L2 within a run, while the runs spread work
// of unequal cost (the beds of a batch) over every XCD.  On a 64-bed ensemble
// in blocks of two wavefronts (48,234 blocks) runs of 8, 32, 128, 256 and
// 1,024 blocks measured 0.304, 0.302, 0.302, 0.308 and 0.320 ms per step, the
// map's own order 0.305 and one contiguous eighth of the map per XCD 0.327;
// in blocks of one wavefront, runs of 128, 256 and 512 blocks 0.294, 0.294
// and 0.300 ms.
constexpr int kBatchXcdRun = 128;
__device__ inline int xcd_run_block(int i, int nb, int C) {
  const int full = nb / (kXcds * C) * (kXcds * C);
  if (i >= full) return full + xcd_block(i - full, nb - full);  // full is a multiple of 8
  const int x = i % kXcds, j = i / kXcds;
  return ((j / C) * kXcds + x) * C + j % C;
}

template <typename R, bool ADVANCE, bool CONT, int L, bool ROLL>
__global__ __launch_bounds__(kForceBlock, 4) void force_kick(Dev D, int p2, int p3, const int *src, int gmode) {
  force_kick_body<R, ADVANCE, CONT, L, ROLL>(D, xcd_block(blockIdx.x, gridDim.x), p2, p3, src, gmode);
}

// ---------------------------------------------------------------------------
// batched kernels: one launch over every bed of a batch
// ---------------------------------------------------------------------------
// Dynamic LDS of the contact-force kernel: per group, maxn list keys and
// maxn history-source bytes.
static size_t force_lds_bytes(int maxn, int L) {
  return (sizeof(unsigned long long) + 1) * (size_t)maxn * (kForceBlock / L);
}

__device__ inline void bed_of_block(const unsigned *__restrict__ map, int &bed, int &blk) {
  const unsigned m = map[blockIdx.x];
  bed = (int)(m >> kBedShift);
  blk = (int)(m & kBlockMask);
}

// Opens step run.s + 1 of every bed (a run of n steps).
__global__ __launch_bounds__(256) void drift_bin_batch(const Dev *__restrict__ tab,
                                                       const BedRun *__restrict__ run,
                                                       const unsigned *__restrict__ map, int n) {
  int b, blk;
  bed_of_block(map, b, blk);
  const Dev &D = tab[b];
  const long long s = run[b].s + 1;
  drift_bin_body<true>(D, blk * 256 + threadIdx.x, (int)(s & 1), (int)(s % 3),
                       run[b].src != nullptr, n == 1);
}

// Step run.s + i of every bed, of a run of n steps (i = 1 applies the bed's
// pending permutation).
template <typename R, bool CONT, int L, bool ROLL>
__global__ __launch_bounds__(kForceBlock, 4) void force_kick_batch(const Dev *__restrict__ tab,
                                                                   const BedRun *__restrict__ run,
                                                                   const unsigned *__restrict__ map,
                                                                   int i, int n) {
  const unsigned m = map[xcd_run_block(blockIdx.x, gridDim.x, kBatchXcdRun)];
  const int b = (int)(m >> kBedShift), blk = (int)(m & kBlockMask);
  const Dev &D = tab[b];
  const long long s = run[b].s + i;
  force_kick_body<R, true, CONT, L, ROLL>(D, blk, (int)(s & 1), (int)(s % 3),
                                          i == 1 ? run[b].src : nullptr, grid_mode(i, n));
}

// After a run of n steps: every bed's step index advances, pending
// permutations have been applied, and the occupied-element counters of the
// coupling step that opened the run (cnt, 3 words) are cleared for the next.
__global__ void batch_advance(BedRun *run, int nb, int n, int *cnt) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0 && cnt) cnt[0] = cnt[1] = cnt[2] = 0;
  if (b >= nb) return;
  run[b].s += n;
  run[b].src = nullptr;
}

// Writes one bed's table entries (stream-ordered, so that a re-sort's new
// arrays take effect exactly at the next batched launch).
__global__ void batch_set_bed(Dev *tab, BedRun *run, int b, Dev D, long long s, const int *src) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  tab[b] = D;
  run[b].s = s;
  run[b].src = src;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// n: steps of the run this launch opens
hipError_t launch_drift_bin_batch(const Dev *tab, const BedRun *run, const unsigned *map, int blocks, int n,
                                  hipStream_t st) {
  if (blocks > 0) drift_bin_batch<<<blocks, 256, 0, st>>>(tab, run, map, n);
  return hipGetLastError();
}

template <int L, bool ROLL>
static void launch_fkb(const Dev *tab, const BedRun *run, const unsigned *map, int blocks, int i, int n,
                       bool fp32, int maxn, hipStream_t st) {
  const size_t lds = force_lds_bytes(maxn, L);
  const bool cont = i < n;
  if (fp32) {
    if (cont)
      force_kick_batch<float, true, L, ROLL><<<blocks, kForceBlock, lds, st>>>(tab, run, map, i, n);
    else
      force_kick_batch<float, false, L, ROLL><<<blocks, kForceBlock, lds, st>>>(tab, run, map, i, n);
  } else {
    if (cont)
      force_kick_batch<double, true, L, ROLL><<<blocks, kForceBlock, lds, st>>>(tab, run, map, i, n);
    else
      force_kick_batch<double, false, L, ROLL><<<blocks, kForceBlock, lds, st>>>(tab, run, map, i, n);
  }
}

template <bool ROLL>
static void launch_fkb_lanes(const Dev *tab, const BedRun *run, const unsigned *map, int blocks, int i, int n,
                             bool fp32, int maxn, int lanes, hipStream_t st) {
  if (lanes == 1)
    launch_fkb<1, ROLL>(tab, run, map, blocks, i, n, fp32, maxn, st);
  else if (lanes == 4)
    launch_fkb<4, ROLL>(tab, run, map, blocks, i, n, fp32, maxn, st);
  else
    launch_fkb<2, ROLL>(tab, run, map, blocks, i, n, fp32, maxn, st);
}

// Step i (1 .. n) of a run of n steps.  lanes: 1, 2 or 4 (the same for every
// bed of the batch); roll: some bed has a nonzero rolling friction coefficient
hipError_t launch_force_kick_batch(const Dev *tab, const BedRun *run, const unsigned *map, int blocks,
                                   int i, int n, bool fp32, int maxn, int lanes, bool roll, hipStream_t st) {
  if (blocks <= 0) return hipGetLastError();
  if (roll)
    launch_fkb_lanes<true>(tab, run, map, blocks, i, n, fp32, maxn, lanes, st);
  else
    launch_fkb_lanes<false>(tab, run, map, blocks, i, n, fp32, maxn, lanes, st);
  return hipGetLastError();
}

hipError_t launch_batch_advance(BedRun *run, int nb, int n, int *cnt, hipStream_t st) {
  batch_advance<<<(nb + 255) / 256, 256, 0, st>>>(run, nb, n, cnt);
  return hipGetLastError();
}

hipError_t launch_batch_set_bed(Dev *tab, BedRun *run, int b, const Dev &D, long long s, const int *src,
                                hipStream_t st) {
  batch_set_bed<<<1, 64, 0, st>>>(tab, run, b, D, s, src);
  return hipGetLastError();
}

// Writes one bed's coupling constants and buffers into the batch tables.
__global__ void batch_set_cpl(Cpl *ctab, CplIO *iot, int b, Cpl C, CplIO io) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  ctab[b] = C;
  iot[b] = io;
}

hipError_t launch_batch_set_cpl(Cpl *ctab, CplIO *iot, int b, const Cpl &C, const CplIO &io, hipStream_t st) {
  batch_set_cpl<<<1, 64, 0, st>>>(ctab, iot, b, C, io);
  return hipGetLastError();
}

// exact: the kind of the grid of step s
hipError_t launch_drift_bin(const Dev &D, long long s, bool drift, bool force_flag, bool exact, hipStream_t st) {
  const int grid = (D.n + 255) / 256;
  const int p2 = (int)(s & 1), p3 = (int)(s % 3);
  if (drift)
    drift_bin<true><<<grid, 256, 0, st>>>(D, p2, p3, force_flag ? 1 : 0, exact ? 1 : 0);
  else
    drift_bin<false><<<grid, 256, 0, st>>>(D, p2, p3, force_flag ? 1 : 0, exact ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_clear_grid(const Dev &D, long long s, hipStream_t st) {
  clear_grid<<<(D.n + 255) / 256, 256, 0, st>>>(D, (int)(s % 3));
  return hipGetLastError();
}

template <typename R, bool ADVANCE, bool CONT, int L, bool ROLL>
static void launch_fk(const Dev &D, int p2, int p3, const int *src, int gmode, hipStream_t st, hipEvent_t e0,
                      hipEvent_t e1) {
  const int grid = (int)(((long long)D.n * L + kForceBlock - 1) / kForceBlock);
  const size_t lds = force_lds_bytes(D.maxn, L);
  if (e0)
    hipExtLaunchKernelGGL(force_kick<R, ADVANCE, CONT, L, ROLL>, dim3(grid), dim3(kForceBlock), lds, st,
                          e0, e1, 0, D, p2, p3, src, gmode);
  else
    force_kick<R, ADVANCE, CONT, L, ROLL><<<grid, kForceBlock, lds, st>>>(D, p2, p3, src, gmode);
}

template <int L, bool ROLL>
static void launch_fk_lanes(const Dev &D, int p2, int p3, const int *src, int gmode, bool advance, bool cont,
                            bool fp32, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (!advance) {
    if (fp32)
      launch_fk<float, false, false, L, ROLL>(D, p2, p3, src, gmode, st, e0, e1);
    else
      launch_fk<double, false, false, L, ROLL>(D, p2, p3, src, gmode, st, e0, e1);
  } else if (fp32) {
    if (cont)
      launch_fk<float, true, true, L, ROLL>(D, p2, p3, src, gmode, st, e0, e1);
    else
      launch_fk<float, true, false, L, ROLL>(D, p2, p3, src, gmode, st, e0, e1);
  } else {
    if (cont)
      launch_fk<double, true, true, L, ROLL>(D, p2, p3, src, gmode, st, e0, e1);
    else
      launch_fk<double, true, false, L, ROLL>(D, p2, p3, src, gmode, st, e0, e1);
  }
}

template <bool ROLL>
static void launch_fk_roll(const Dev &D, int p2, int p3, const int *src, int gmode, bool advance, bool cont,
                           bool fp32, int lanes, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (lanes == 1)
    launch_fk_lanes<1, ROLL>(D, p2, p3, src, gmode, advance, cont, fp32, st, e0, e1);
  else if (lanes == 4)
    launch_fk_lanes<4, ROLL>(D, p2, p3, src, gmode, advance, cont, fp32, st, e0, e1);
  else
    launch_fk_lanes<2, ROLL>(D, p2, p3, src, gmode, advance, cont, fp32, st, e0, e1);
}

// e0/e1: when non-NULL, events recorded at the kernel's own start and end.
// lanes: 1, 2 or 4.  gmode: kGrid* bits.
hipError_t launch_force_kick(const Dev &D, long long s, const int *src, int gmode, bool advance, bool cont,
                             bool fp32, int lanes, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const int p2 = (int)(s & 1), p3 = (int)(s % 3);
  if (D.pp.mu_r > 0.0 || D.pw.mu_r > 0.0)
    launch_fk_roll<true>(D, p2, p3, src, gmode, advance, cont, fp32, lanes, st, e0, e1);
  else
    launch_fk_roll<false>(D, p2, p3, src, gmode, advance, cont, fp32, lanes, st, e0, e1);
  return hipGetLastError();
}

}  // namespace cfddem
