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
//   pcm_elems      the particle volumes of each element summed exactly in
//                  fixed point (2^-50 of the element volume), so the sum does
//                  not depend on the order of the cell slots or of the cells
//   smooth_rhs     b_i = sum over the elements around node i of eps_e int phi_i
//   fd_transform   the 1D transforms of the solve (FP64 MFMA products)
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

// One wavefront per element: the volumes of the particles in its cells (kk
// consecutive cells) in fixed point, 2^-50 of the element volume, summed over
// the lanes and written once.  Integer sums do not depend on the order of the
// additions, and nothing needs clearing first.
__device__ __forceinline__ void pcm_elems_body(const Dev &D, double Ve, int p2, int p3, unsigned long long *acc) {
  const Grid &G = D.grid;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (e >= G.n_elem) return;  // whole wavefronts
  const double scale = 0x1p50 / Ve;
  unsigned long long sum = 0;
  for (int i = lane; i < G.kk; i += 64) {
    const int c = e * G.kk + i;
    int m = gsel(D.cnt, p3)[c];
    if (m > D.cap) m = D.cap;
    const gptr<const int> sl = gsel(D.slot, p2) + (size_t)c * D.cap;
    for (int s = 0; s < m; ++s) {
      const double r = glb(D.rad)[sl[s]];
      sum += (unsigned long long)llrint(4.0 / 3.0 * kPi * r * r * r * scale);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if (lane == 0) acc[e] = sum;
}

__global__ __launch_bounds__(256) void pcm_elems(Dev D, double Ve, int p2, int p3, unsigned long long *acc) {
  pcm_elems_body(D, Ve, p2, p3, acc);
}

// The same for bed b of a batch, with the bed's arrays and step index read on
// the device (tab[b], run[b]): a batch replays its coupling step from a graph
// while its steps advance and its re-sorts swap its per-particle arrays.
__global__ __launch_bounds__(256) void pcm_elems_run(const Dev *__restrict__ tab, double Ve,
                                                     const BedRun *__restrict__ run, int b,
                                                     unsigned long long *acc) {
  const long long s = run[b].s;
  pcm_elems_body(tab[b], Ve, (int)(s & 1), (int)(s % 3), acc);
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
// three with V.  One pass applies T (V^T or V, n x n row-major, n = nodes
// along the axis) to every line of the lattice along that axis:
// out[line c, i] = sum_j T[i][j] in[line c, j], optionally scaled by the
// diagonal: a (n x n) x (n x lines) product on the FP64 matrix cores.  A block
// of four wavefronts computes kTI outputs along the axis for kTC lines; each
// wavefront a 16 x 16 part of it as one tile of v_mfma_f64_16x16x4f64 (zero
// padding past n adds exact zeros).  Tiles of 32 x 32 give the 100k bed's
// 161 x 41 x 41 lattice 318 to 414 blocks per pass where 32 x 64 gave 162 to
// 208, fewer than the chip's 256 CUs (the three passes 11.7, 8.2 and 5.6 us
// against 11.0, 6.9 and 5.1 us; a 96-wide k chunk was slower).  The next
// kTK-wide chunk of T and of the lines is loaded into registers while the
// current one is summed, and the result tile is staged through LDS, so that
// loads and stores follow the order of memory on every axis (along the line
// for x, across lines otherwise).
namespace {
constexpr int kTI = 32, kTC = 32, kTK = 64, kTT = 256;
constexpr int kAL = kTI * kTK / kTT, kBL = kTK * kTC / kTT, kOL = kTI * kTC / kTT;  // per thread
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int AX>
__device__ inline long line_base(const SmoothOp &S, int c) {
  if (AX == 0) return (long)c * S.nn[0];
  if (AX == 1) return (long)(c % S.nn[0]) + (long)(c / S.nn[0]) * S.nn[0] * S.nn[1];
  return (long)c;
}

template <int AX>
__device__ inline long axis_stride(const SmoothOp &S) {
  return AX == 0 ? 1L : (AX == 1 ? (long)S.nn[0] : (long)S.nn[0] * S.nn[1]);
}

// Position of element e of a K x Q tile (k along the axis, q across lines)
// in the order of memory.
template <int AX, int K, int Q>
__device__ inline void tile_pos(int e, int &k, int &q) {
  if (AX == 0) {
    k = e % K;
    q = e / K;
  } else {
    k = e / Q;
    q = e % Q;
  }
}
}  // namespace

template <int AX>
__global__ __launch_bounds__(kTT) void fd_transform(SmoothOp S, const double *__restrict__ T,
                                                    const double *__restrict__ in, double *__restrict__ out,
                                                    int scale) {
  __shared__ double As[kTI][kTK + 1];
  __shared__ double Bs[kTK][kTC + 1];
  __shared__ double Os[kTI][kTC + 1];
  const int n = S.nn[AX];
  const int lines = (int)(S.nv / n);
  const int i0 = blockIdx.y * kTI, c0 = blockIdx.x * kTC;
  const int t = threadIdx.x;
  const long stride = axis_stride<AX>(S);
  // the lines this thread loads, fixed over the chunks
  long bb[kBL];
#pragma unroll
  for (int m = 0; m < kBL; ++m) {
    int k, q;
    tile_pos<AX, kTK, kTC>(t + kTT * m, k, q);
    bb[m] = c0 + q < lines ? line_base<AX>(S, c0 + q) : -1;
  }
  double ar[kAL], br[kBL];
  auto load = [&](int j0) {
#pragma unroll
    for (int m = 0; m < kAL; ++m) {
      const int e = t + kTT * m, r = e / kTK, j = j0 + e % kTK;
      ar[m] = (i0 + r < n && j < n) ? T[(size_t)(i0 + r) * n + j] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < kBL; ++m) {
      int k, q;
      tile_pos<AX, kTK, kTC>(t + kTT * m, k, q);
      const int j = j0 + k;
      br[m] = (bb[m] >= 0 && j < n) ? in[bb[m] + (long)j * stride] : 0.0;
    }
  };
  // this wavefront's part: rows wr .. wr+15, lines wc .. wc+15; the lane's
  // operand row / line lr and k offset lk (A: T[row][k], B: line tile[k][line])
  const int lane = t & 63, w = t >> 6;
  const int wr = 16 * (w & 1), wc = 16 * (w >> 1);
  const int lr = lane & 15, lk = lane >> 4;
  dbl4 d0 = {0.0, 0.0, 0.0, 0.0};
  load(0);
  for (int j0 = 0; j0 < n; j0 += kTK) {
#pragma unroll
    for (int m = 0; m < kAL; ++m) {
      const int e = t + kTT * m;
      As[e / kTK][e % kTK] = ar[m];
    }
#pragma unroll
    for (int m = 0; m < kBL; ++m) {
      int k, q;
      tile_pos<AX, kTK, kTC>(t + kTT * m, k, q);
      Bs[k][q] = br[m];
    }
    __syncthreads();
    if (j0 + kTK < n) load(j0 + kTK);
    const int kmax = min(kTK, n - j0);
    for (int kk = 0; kk < kmax; kk += 4) {
      const double av = As[wr + lr][kk + lk];
      const double b0 = Bs[kk + lk][wc + lr];
      d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, d0, 0, 0, 0);
    }
    __syncthreads();
  }
  // result r of a lane: row wr + 4 r + lane / 16, line wc + lane % 16
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    Os[wr + 4 * r + lk][wc + lr] = d0[r];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < kOL; ++m) {
    int k, q;
    tile_pos<AX, kTI, kTC>(t + kTT * m, k, q);
    const int i = i0 + k, c = c0 + q;
    if (i >= n || c >= lines) continue;
    double v = Os[k][q];
    if (scale) {
      const int nx = S.nn[0], ny = S.nn[1];
      int g[3];
      if (AX == 0) {
        g[0] = i; g[1] = c % ny; g[2] = c / ny;
      } else if (AX == 1) {
        g[0] = c % nx; g[1] = i; g[2] = c / nx;
      } else {
        g[0] = c % nx; g[1] = c / nx; g[2] = i;
      }
      v /= 1.0 + S.L2 * (S.lam[0][g[0]] + S.lam[1][g[1]] + S.lam[2][g[2]]);
    }
    out[line_base<AX>(S, c) + (long)i * stride] = v;
  }
}

// eps_h at every quadrature point, element-major numbering: one thread per
// element evaluates the tensor-product interpolation of its (ORD+1)^3 nodal
// values at its (ORD+1)^3 Gauss points (sums over x, then y, then z), staged
// through LDS so that the block writes its points contiguously.
template <int ORD>
__global__ __launch_bounds__(64) void eps_q_field(SmoothOp S, Cpl C, const double *__restrict__ eps_nodes,
                                                  double *__restrict__ eps_q, int ne) {
  constexpr int P1 = ORD + 1, NQ = P1 * P1 * P1;
  __shared__ double out_s[64 * NQ];
  const int e0 = blockIdx.x * 64, e = e0 + threadIdx.x;
  if (e < ne) {
    const int ex = e % S.n_el[0], ey = (e / S.n_el[0]) % S.n_el[1], ez = e / (S.n_el[0] * S.n_el[1]);
    double nod[P1][P1][P1], L[P1][P1];
#pragma unroll
    for (int ic = 0; ic < P1; ++ic)
#pragma unroll
      for (int ib = 0; ib < P1; ++ib) {
        const double *row = eps_nodes + ((long)(ORD * ez + ic) * S.nn[1] + (ORD * ey + ib)) * S.nn[0] + ORD * ex;
#pragma unroll
        for (int ia = 0; ia < P1; ++ia) nod[ic][ib][ia] = row[ia];
      }
#pragma unroll
    for (int a = 0; a < P1; ++a)
#pragma unroll
      for (int i = 0; i < P1; ++i) L[a][i] = C.Lq[a][i];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int qx = q % P1, qy = (q / P1) % P1, qz = q / (P1 * P1);
      double v = 0.0;
#pragma unroll
      for (int ic = 0; ic < P1; ++ic) {
        double acc_c = 0.0;
#pragma unroll
        for (int ib = 0; ib < P1; ++ib) {
          double acc_b = 0.0;
#pragma unroll
          for (int ia = 0; ia < P1; ++ia) acc_b += L[ia][qx] * nod[ic][ib][ia];
          acc_c += L[ib][qy] * acc_b;
        }
        v += L[ic][qz] * acc_c;
      }
      out_s[threadIdx.x * NQ + q] = v;
    }
  }
  __syncthreads();
  const int cnt = min(64, ne - e0) * NQ;
  for (int k = threadIdx.x; k < cnt; k += 64) eps_q[(long)e0 * NQ + k] = out_s[k];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int smooth_blocks(long nv) { return (int)((nv + kSB - 1) / kSB); }

hipError_t launch_pcm_rhs(const Dev &D, const Cpl &C, const SmoothOp &S, long long s, double *acc,
                          double *b, hipStream_t st) {
  const int p2 = (int)(s & 1), p3 = (int)(s % 3);
  unsigned long long *a = reinterpret_cast<unsigned long long *>(acc);
  pcm_elems<<<(D.grid.n_elem + 3) / 4, 256, 0, st>>>(D, C.Ve, p2, p3, a);
  smooth_rhs<<<smooth_blocks(S.nv), kSB, 0, st>>>(S, a, b);
  return hipGetLastError();
}

// x = A^-1 b: transforms with V^T along x, y, z (the last one scaled by the
// inverse diagonal), then with V along z, y, x; t1, t2 are scratch vectors.
// As launch_pcm_rhs for bed b of a batch (step index from run[b]).
hipError_t launch_pcm_rhs_run(const Dev *tab, int n_elem, const Cpl &C, const SmoothOp &S, const BedRun *run,
                              int bed, double *acc, double *b, hipStream_t st) {
  unsigned long long *a = reinterpret_cast<unsigned long long *>(acc);
  pcm_elems_run<<<(n_elem + 3) / 4, 256, 0, st>>>(tab, C.Ve, run, bed, a);
  smooth_rhs<<<smooth_blocks(S.nv), kSB, 0, st>>>(S, a, b);
  return hipGetLastError();
}

static dim3 fd_grid(const SmoothOp &S, int axis) {
  const long n = S.nn[axis], lines = S.nv / n;
  return dim3((unsigned)((lines + kTC - 1) / kTC), (unsigned)((n + kTI - 1) / kTI));
}

hipError_t launch_smooth_solve(const SmoothOp &S, const double *b, double *x, double *t1, double *t2,
                               hipStream_t st) {
  fd_transform<0><<<fd_grid(S, 0), kTT, 0, st>>>(S, S.Vt[0], b, t1, 0);
  fd_transform<1><<<fd_grid(S, 1), kTT, 0, st>>>(S, S.Vt[1], t1, t2, 0);
  fd_transform<2><<<fd_grid(S, 2), kTT, 0, st>>>(S, S.Vt[2], t2, t1, 1);
  fd_transform<2><<<fd_grid(S, 2), kTT, 0, st>>>(S, S.V[2], t1, t2, 0);
  fd_transform<1><<<fd_grid(S, 1), kTT, 0, st>>>(S, S.V[1], t2, t1, 0);
  fd_transform<0><<<fd_grid(S, 0), kTT, 0, st>>>(S, S.V[0], t1, x, 0);
  return hipGetLastError();
}

hipError_t launch_eps_q_field(const SmoothOp &S, const Cpl &C, const double *eps_nodes, double *eps_q,
                              hipStream_t st) {
  const int ne = S.n_el[0] * S.n_el[1] * S.n_el[2];
  if (S.order == 1)
    eps_q_field<1><<<(ne + 63) / 64, 64, 0, st>>>(S, C, eps_nodes, eps_q, ne);
  else
    eps_q_field<2><<<(ne + 63) / 64, 64, 0, st>>>(S, C, eps_nodes, eps_q, ne);
  return hipGetLastError();
}

}  // namespace cfddem
