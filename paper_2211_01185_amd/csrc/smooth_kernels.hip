// smooth_kernels.hip -- smoothed void fraction on gfx950 (Eq. "void_fraction"
// of El Geitani, Golshan & Blais, arXiv 2211.01185, with the smoothing length
// L^2 of Tables "tab:setup2" and "tab:setup4").
//
// The element PCM values eps_e are projected onto the continuous velocity
// space: eps_h with
//     int eps_h phi_i + L^2 int grad eps_h . grad phi_i = int eps_PCM phi_i
// for every basis function phi_i (natural boundary conditions).  On the
// structured mesh the global matrix is a sum of Kronecker products of 1D
// banded matrices (mass M_a, stiffness K_a of each axis),
//     A = Mx My Mz + L^2 (Kx My Mz + Mx Ky Mz + Mx My Kz),
// so it is applied node by node as a (2 order + 1)^3 stencil whose weights
// are products of 1D band entries; the system is solved by Jacobi-
// preconditioned conjugate gradients.  Every reduction has a fixed order
// (per 256-node block, then one wave over the blocks), so the iterates do not
// depend on timing.
//   pcm_elements   eps_e per element, the particle volumes summed exactly in
//                  fixed point (2^-50 of the element volume), so the sum does
//                  not depend on the order of the cell slots
//   smooth_rhs     b_i = sum over the elements around node i of eps_e int phi_i
//   smooth_*       the CG steps
//   eps_q_field    eps_h at every quadrature point
#include "device.h"

namespace cfddem {

namespace {
constexpr int kSB = 256;  // threads per block of the node kernels
constexpr double kPi = 3.14159265358979323846;

// Lattice coordinates of node i (x fastest).
__device__ inline void node_xyz(const SmoothOp &S, long i, int &gx, int &gy, int &gz) {
  gx = (int)(i % S.nn[0]);
  const long r = i / S.nn[0];
  gy = (int)(r % S.nn[1]);
  gz = (int)(r / S.nn[1]);
}

// y_i = (A x)_i over the stencil of node i.
__device__ inline double apply_row(const SmoothOp &S, const double *__restrict__ x, int gx, int gy, int gz) {
  const int b = S.order;
  const double *mx = S.band_m[0] + (size_t)gx * 5, *kx = S.band_k[0] + (size_t)gx * 5;
  const double *my = S.band_m[1] + (size_t)gy * 5, *ky = S.band_k[1] + (size_t)gy * 5;
  const double *mz = S.band_m[2] + (size_t)gz * 5, *kz = S.band_k[2] + (size_t)gz * 5;
  double y = 0.0;
  for (int dz = -b; dz <= b; ++dz) {
    const int jz = gz + dz;
    if (jz < 0 || jz >= S.nn[2]) continue;
    for (int dy = -b; dy <= b; ++dy) {
      const int jy = gy + dy;
      if (jy < 0 || jy >= S.nn[1]) continue;
      const double m_yz = my[dy + 2] * mz[dz + 2];
      const double k_yz = ky[dy + 2] * mz[dz + 2] + my[dy + 2] * kz[dz + 2];
      const double *row = x + ((long)jz * S.nn[1] + jy) * S.nn[0];
      for (int dx = -b; dx <= b; ++dx) {
        const int jx = gx + dx;
        if (jx < 0 || jx >= S.nn[0]) continue;
        const double w = mx[dx + 2] * m_yz + S.L2 * (kx[dx + 2] * m_yz + mx[dx + 2] * k_yz);
        y += w * row[jx];
      }
    }
  }
  return y;
}

// Fixed-order block sum of one value per thread; thread 0 gets the total.
__device__ inline double block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int h = kSB / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  const double t = sh[0];
  __syncthreads();
  return t;
}
}  // namespace

__global__ __launch_bounds__(256) void pcm_elements(Dev D, double Ve, int p2, int p3, double *eps_e) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const Grid &G = D.grid;
  if (e >= G.n_elem) return;
  const int *cnt = sel(D.cnt, p3);
  const int *slot = sel(D.slot, p2);
  const double scale = 0x1p50 / Ve;
  long long acc = 0;
  for (int c = e * G.kk; c < (e + 1) * G.kk; ++c) {
    int m = cnt[c];
    if (m > D.cap) m = D.cap;
    for (int s = 0; s < m; ++s) {
      const double r = D.rad[slot[(size_t)c * D.cap + s]];
      acc += llrint(4.0 / 3.0 * kPi * r * r * r * scale);
    }
  }
  eps_e[e] = 1.0 - (double)acc * 0x1p-50;
}

__global__ __launch_bounds__(kSB) void smooth_rhs(SmoothOp S, const double *__restrict__ eps_e,
                                                  double *__restrict__ b) {
  const long i = (long)blockIdx.x * kSB + threadIdx.x;
  if (i >= S.nv) return;
  int g[3];
  node_xyz(S, i, g[0], g[1], g[2]);
  // per axis: the (element, local node) pairs this lattice index belongs to
  int el[3][2], lc[3][2], ne[3];
  for (int a = 0; a < 3; ++a) {
    const int p = S.order, q = g[a] / p, l = g[a] % p;
    ne[a] = 0;
    if (l != 0) {
      el[a][0] = q;
      lc[a][0] = l;
      ne[a] = 1;
    } else {
      if (q - 1 >= 0) {
        el[a][ne[a]] = q - 1;
        lc[a][ne[a]] = p;
        ++ne[a];
      }
      if (q < S.n_el[a]) {
        el[a][ne[a]] = q;
        lc[a][ne[a]] = 0;
        ++ne[a];
      }
    }
  }
  double acc = 0.0;
  for (int kz = 0; kz < ne[2]; ++kz)
    for (int ky = 0; ky < ne[1]; ++ky)
      for (int kx = 0; kx < ne[0]; ++kx) {
        const long e = ((long)el[2][kz] * S.n_el[1] + el[1][ky]) * S.n_el[0] + el[0][kx];
        acc += eps_e[e] * (S.load[0][lc[0][kx]] * S.load[1][lc[1][ky]] * S.load[2][lc[2][kz]]);
      }
  b[i] = acc;
}

// r = b - A x, z = r / diag, p = z; partial sums of r.z and r.r (and b.b).
__global__ __launch_bounds__(kSB) void smooth_init(SmoothOp S, const double *__restrict__ b,
                                                   const double *__restrict__ x, double *__restrict__ r,
                                                   double *__restrict__ z, double *__restrict__ p,
                                                   double *__restrict__ part) {
  __shared__ double sh[kSB];
  const long i = (long)blockIdx.x * kSB + threadIdx.x;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  if (i < S.nv) {
    int gx, gy, gz;
    node_xyz(S, i, gx, gy, gz);
    const double ri = b[i] - apply_row(S, x, gx, gy, gz);
    const double zi = ri / S.diag[i];
    r[i] = ri;
    z[i] = zi;
    p[i] = zi;
    rz = ri * zi;
    rr = ri * ri;
    bb = b[i] * b[i];
  }
  rz = block_sum(rz, sh);
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = rz;
    part[3 * blockIdx.x + 1] = rr;
    part[3 * blockIdx.x + 2] = bb;
  }
}

// Ap and the partial sums of p.Ap.
__global__ __launch_bounds__(kSB) void smooth_apply(SmoothOp S, const double *__restrict__ p,
                                                    double *__restrict__ Ap, double *__restrict__ part) {
  __shared__ double sh[kSB];
  const long i = (long)blockIdx.x * kSB + threadIdx.x;
  double pAp = 0.0;
  if (i < S.nv) {
    int gx, gy, gz;
    node_xyz(S, i, gx, gy, gz);
    const double y = apply_row(S, p, gx, gy, gz);
    Ap[i] = y;
    pAp = p[i] * y;
  }
  pAp = block_sum(pAp, sh);
  if (threadIdx.x == 0) part[3 * blockIdx.x] = pAp;
}

// Totals of the block partials (three slots per block, the first k used),
// one wave in fixed order: out[j] = sum over blocks of part[3 blk + j].
__global__ __launch_bounds__(64) void smooth_total(int nb, int k, const double *__restrict__ part,
                                                   double *__restrict__ out) {
  for (int j = 0; j < k; ++j) {
    double v = 0.0;
    for (int i = (int)threadIdx.x; i < nb; i += 64) v += part[(size_t)3 * i + j];
    for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    if (threadIdx.x == 0) out[j] = v;
  }
}

// alpha = rz / pAp; x += alpha p; r -= alpha Ap; z = r / diag; partial r.z
// and r.r.  sc: [0] r.z of the current direction, [1] p.Ap.
__global__ __launch_bounds__(kSB) void smooth_update(SmoothOp S, const double *__restrict__ sc,
                                                     double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ z, const double *__restrict__ p,
                                                     const double *__restrict__ Ap, double *__restrict__ part) {
  __shared__ double sh[kSB];
  const long i = (long)blockIdx.x * kSB + threadIdx.x;
  const double pAp = sc[1];
  const double alpha = pAp != 0.0 ? sc[0] / pAp : 0.0;
  double rz = 0.0, rr = 0.0;
  if (i < S.nv) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * Ap[i];
    const double zi = ri / S.diag[i];
    r[i] = ri;
    z[i] = zi;
    rz = ri * zi;
    rr = ri * ri;
  }
  rz = block_sum(rz, sh);
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = rz;
    part[3 * blockIdx.x + 1] = rr;
  }
}

// p = z + beta p, beta = rz_new / rz_old (sc[2] / sc[0]).
__global__ __launch_bounds__(kSB) void smooth_direction(SmoothOp S, const double *__restrict__ sc,
                                                        const double *__restrict__ z, double *__restrict__ p) {
  const long i = (long)blockIdx.x * kSB + threadIdx.x;
  const double beta = sc[0] != 0.0 ? sc[2] / sc[0] : 0.0;
  if (i < S.nv) p[i] = z[i] + beta * p[i];
}

// sc[0] = sc[2]: the new r.z becomes the current one (one thread, after the
// direction update has read both).
__global__ void smooth_shift(double *sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sc[0] = sc[2];
}

// After the initial residual: sc[0] = r.z, sc[3] = r.r, sc[4] = b.b from the
// totals in sc[5..7].
__global__ void smooth_init_scalars(double *sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc[0] = sc[5];
    sc[3] = sc[6];
    sc[4] = sc[7];
  }
}

// eps_h at every quadrature point: thread per point, element-major numbering.
__global__ __launch_bounds__(256) void eps_q_field(SmoothOp S, Cpl C, const double *__restrict__ eps_nodes,
                                                   double *__restrict__ eps_q) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  const long ne = (long)S.n_el[0] * S.n_el[1] * S.n_el[2];
  if (t >= ne * C.nq) return;
  const long e = t / C.nq;
  const int q = (int)(t % C.nq);
  const int p = S.order, p1 = p + 1;
  const int qx = q % p1, qy = (q / p1) % p1, qz = q / (p1 * p1);
  const int ex = (int)(e % S.n_el[0]), ey = (int)((e / S.n_el[0]) % S.n_el[1]),
            ez = (int)(e / ((long)S.n_el[0] * S.n_el[1]));
  double v = 0.0;
  for (int ic = 0; ic < p1; ++ic) {
    double acc_c = 0.0;
    for (int ib = 0; ib < p1; ++ib) {
      double acc_b = 0.0;
      const double *row = eps_nodes + ((long)(p * ez + ic) * S.nn[1] + (p * ey + ib)) * S.nn[0] + p * ex;
      for (int ia = 0; ia < p1; ++ia) acc_b += C.Lq[ia][qx] * row[ia];
      acc_c += C.Lq[ib][qy] * acc_b;
    }
    v += C.Lq[ic][qz] * acc_c;
  }
  eps_q[t] = v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int smooth_blocks(long nv) { return (int)((nv + kSB - 1) / kSB); }

hipError_t launch_pcm_rhs(const Dev &D, const Cpl &C, const SmoothOp &S, long long s, double *eps_e,
                          double *b, hipStream_t st) {
  const int p2 = (int)(s & 1), p3 = (int)(s % 3);
  pcm_elements<<<(D.grid.n_elem + 255) / 256, 256, 0, st>>>(D, C.Ve, p2, p3, eps_e);
  smooth_rhs<<<smooth_blocks(S.nv), kSB, 0, st>>>(S, eps_e, b);
  return hipGetLastError();
}

// sc (device, 8 doubles): [0] r.z of the current direction, [1] p.Ap, [2] the
// new r.z, [3] r.r, [4] b.b, [5..7] scratch of the initial totals
hipError_t launch_smooth_init(const SmoothOp &S, const double *b, const double *x, double *r, double *z,
                              double *p, double *part, double *sc, hipStream_t st) {
  const int nb = smooth_blocks(S.nv);
  smooth_init<<<nb, kSB, 0, st>>>(S, b, x, r, z, p, part);
  smooth_total<<<1, 64, 0, st>>>(nb, 3, part, sc + 5);
  smooth_init_scalars<<<1, 64, 0, st>>>(sc);
  return hipGetLastError();
}

hipError_t launch_smooth_iteration(const SmoothOp &S, double *x, double *r, double *z, double *p, double *Ap,
                                   double *part, double *sc, hipStream_t st) {
  const int nb = smooth_blocks(S.nv);
  smooth_apply<<<nb, kSB, 0, st>>>(S, p, Ap, part);
  smooth_total<<<1, 64, 0, st>>>(nb, 1, part, sc + 1);
  smooth_update<<<nb, kSB, 0, st>>>(S, sc, x, r, z, p, Ap, part);
  smooth_total<<<1, 64, 0, st>>>(nb, 2, part, sc + 2);  // sc[2] = new r.z, sc[3] = r.r
  smooth_direction<<<nb, kSB, 0, st>>>(S, sc, z, p);
  smooth_shift<<<1, 64, 0, st>>>(sc);
  return hipGetLastError();
}

hipError_t launch_eps_q_field(const SmoothOp &S, const Cpl &C, const double *eps_nodes, double *eps_q,
                              hipStream_t st) {
  const long nq = (long)S.n_el[0] * S.n_el[1] * S.n_el[2] * C.nq;
  eps_q_field<<<(int)((nq + 255) / 256), 256, 0, st>>>(S, C, eps_nodes, eps_q);
  return hipGetLastError();
}

}  // namespace cfddem
