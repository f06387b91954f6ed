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
// so it is diagonalized by the generalized eigenvectors of the 1D pairs
// (K_a, M_a) (fast diagonalization): the solve is exact up to rounding, six
// 1D transforms and a diagonal scaling, with no iteration and no history.
//   pcm_cells      the particle volumes of each element summed exactly in
//                  fixed point (2^-50 of the element volume), so the sum does
//                  not depend on the order of the cell slots or of the cells
//   smooth_rhs     b_i = sum over the elements around node i of eps_e int phi_i
//   fd_transform   the 1D transforms of the solve
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

}  // namespace

// Zeroes the fixed-point solid-volume accumulators of the elements.
__global__ __launch_bounds__(256) void pcm_clear(int n_elem, unsigned long long *acc) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < n_elem) acc[e] = 0ull;
}

// One thread per cell: the volumes of its particles in fixed point (2^-50 of
// the element volume), added to its element's accumulator.  Integer sums do
// not depend on the order of the additions.
__device__ __forceinline__ void pcm_cells_body(const Dev &D, double Ve, int p2, int p3, unsigned long long *acc) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  const Grid &G = D.grid;
  if (c >= G.ncells) return;
  int m = sel(D.cnt, p3)[c];
  if (m > D.cap) m = D.cap;
  if (m == 0) return;
  const int *sl = sel(D.slot, p2) + (size_t)c * D.cap;
  const double scale = 0x1p50 / Ve;
  unsigned long long sum = 0;
  for (int s = 0; s < m; ++s) {
    const double r = D.rad[sl[s]];
    sum += (unsigned long long)llrint(4.0 / 3.0 * kPi * r * r * r * scale);
  }
  atomicAdd(acc + c / G.kk, sum);
}

__global__ __launch_bounds__(256) void pcm_cells(Dev D, double Ve, int p2, int p3, unsigned long long *acc) {
  pcm_cells_body(D, Ve, p2, p3, acc);
}

// The same, with the step index read on the device from run[b]: a batch
// replays its coupling step from a graph while its steps advance there.
__global__ __launch_bounds__(256) void pcm_cells_run(Dev D, double Ve, const BedRun *__restrict__ run, int b,
                                                     unsigned long long *acc) {
  const long long s = run[b].s;
  pcm_cells_body(D, Ve, (int)(s & 1), (int)(s % 3), acc);
}

__global__ __launch_bounds__(kSB) void smooth_rhs(SmoothOp S, const unsigned long long *__restrict__ acc,
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
  double sum = 0.0;
  for (int kz = 0; kz < ne[2]; ++kz)
    for (int ky = 0; ky < ne[1]; ++ky)
      for (int kx = 0; kx < ne[0]; ++kx) {
        const long e = ((long)el[2][kz] * S.n_el[1] + el[1][ky]) * S.n_el[0] + el[0][kx];
        const double eps_e = 1.0 - (double)acc[e] * 0x1p-50;  // element PCM value
        sum += eps_e * (S.load[0][lc[0][kx]] * S.load[1][lc[1][ky]] * S.load[2][lc[2][kz]]);
      }
  b[i] = sum;
}

// Fast diagonalization.  Per axis a, V_a holds the generalized eigenvectors of
// (K_a, M_a) (V^T M V = I, V^T K V = diag(lam_a)), so
//     A^-1 = (Vx Vy Vz) diag(1 / (1 + L^2 (lam_x + lam_y + lam_z))) (Vx Vy Vz)^T
// and the solve is three 1D transforms with V^T, the diagonal scaling, and
// three with V.  One pass: out[.., i, ..] = sum_j T[i][j] in[.., j, ..] along
// axis a (T = V^T or V, n_a x n_a row-major), optionally scaled by the
// diagonal.
__global__ __launch_bounds__(kSB) void fd_transform(SmoothOp S, int axis, const double *__restrict__ T,
                                                    const double *__restrict__ in, double *__restrict__ out,
                                                    int scale) {
  const long i = (long)blockIdx.x * kSB + threadIdx.x;
  if (i >= S.nv) return;
  int g[3];
  node_xyz(S, i, g[0], g[1], g[2]);
  const int n = S.nn[axis];
  const long stride = axis == 0 ? 1L : (axis == 1 ? (long)S.nn[0] : (long)S.nn[0] * S.nn[1]);
  const int gi = axis == 0 ? g[0] : (axis == 1 ? g[1] : g[2]);
  const double *line = in + (i - gi * stride);
  const double *row = T + (size_t)gi * n;
  double v = 0.0;
  for (int j = 0; j < n; ++j) v += row[j] * line[j * stride];
  if (scale) v /= 1.0 + S.L2 * (S.lam[0][g[0]] + S.lam[1][g[1]] + S.lam[2][g[2]]);
  out[i] = v;
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

hipError_t launch_pcm_rhs(const Dev &D, const Cpl &C, const SmoothOp &S, long long s, double *acc,
                          double *b, hipStream_t st) {
  const int p2 = (int)(s & 1), p3 = (int)(s % 3);
  unsigned long long *a = reinterpret_cast<unsigned long long *>(acc);
  pcm_clear<<<(D.grid.n_elem + 255) / 256, 256, 0, st>>>(D.grid.n_elem, a);
  pcm_cells<<<(D.grid.ncells + 255) / 256, 256, 0, st>>>(D, C.Ve, p2, p3, a);
  smooth_rhs<<<smooth_blocks(S.nv), kSB, 0, st>>>(S, a, b);
  return hipGetLastError();
}

// x = A^-1 b: transforms with V^T along x, y, z (the last one scaled by the
// inverse diagonal), then with V along z, y, x; t1, t2 are scratch vectors.
// As launch_pcm_rhs for bed b of a batch (step index from run[b]).
hipError_t launch_pcm_rhs_run(const Dev &D, const Cpl &C, const SmoothOp &S, const BedRun *run, int bed,
                              double *acc, double *b, hipStream_t st) {
  unsigned long long *a = reinterpret_cast<unsigned long long *>(acc);
  pcm_clear<<<(D.grid.n_elem + 255) / 256, 256, 0, st>>>(D.grid.n_elem, a);
  pcm_cells_run<<<(D.grid.ncells + 255) / 256, 256, 0, st>>>(D, C.Ve, run, bed, a);
  smooth_rhs<<<smooth_blocks(S.nv), kSB, 0, st>>>(S, a, b);
  return hipGetLastError();
}

hipError_t launch_smooth_solve(const SmoothOp &S, const double *b, double *x, double *t1, double *t2,
                               hipStream_t st) {
  const int nb = smooth_blocks(S.nv);
  fd_transform<<<nb, kSB, 0, st>>>(S, 0, S.Vt[0], b, t1, 0);
  fd_transform<<<nb, kSB, 0, st>>>(S, 1, S.Vt[1], t1, t2, 0);
  fd_transform<<<nb, kSB, 0, st>>>(S, 2, S.Vt[2], t2, t1, 1);
  fd_transform<<<nb, kSB, 0, st>>>(S, 2, S.V[2], t1, t2, 0);
  fd_transform<<<nb, kSB, 0, st>>>(S, 1, S.V[1], t2, t1, 0);
  fd_transform<<<nb, kSB, 0, st>>>(S, 0, S.V[0], t1, x, 0);
  return hipGetLastError();
}

hipError_t launch_eps_q_field(const SmoothOp &S, const Cpl &C, const double *eps_nodes, double *eps_q,
                              hipStream_t st) {
  const long nq = (long)S.n_el[0] * S.n_el[1] * S.n_el[2] * C.nq;
  eps_q_field<<<(int)((nq + 255) / 256), 256, 0, st>>>(S, C, eps_nodes, eps_q);
  return hipGetLastError();
}

}  // namespace cfddem
