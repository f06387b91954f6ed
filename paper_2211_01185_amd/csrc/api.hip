// api.hip -- host side of the libcfddem C ABI (include/cfddem.h): parameter
// validation, workspace layout, the step / couple sequencing on the caller's
// stream, accessors in original-ID order, and the periodic re-sort of the
// particle arrays by cell.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "cfddem.h"
#include "device.h"

namespace cfddem {
hipError_t launch_drift_bin(const Dev &D, long long s, bool drift, bool force_flag, bool exact, hipStream_t st);
hipError_t launch_clear_grid(const Dev &D, long long s, hipStream_t st);
hipError_t launch_force_kick(const Dev &D, long long s, const int *src, int gmode, bool advance, bool cont,
                             bool fp32, int lanes, hipStream_t st, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_couple(const Dev &D, const Cpl &C, long long s, long long call, const double *U,
                         const double *P, double *eps_q, double *beta_q, double *fpf_q,
                         double *esums, bool fp32, hipStream_t st);
int smooth_blocks(long nv);
hipError_t launch_pcm_rhs(const Dev &D, const Cpl &C, const SmoothOp &S, long long s, double *acc,
                          double *b, hipStream_t st);
hipError_t launch_pcm_rhs_run(const Dev *tab, int n_elem, const Cpl &C, const SmoothOp &S, const BedRun *run,
                              int bed, double *acc, double *b, hipStream_t st);
hipError_t launch_smooth_solve(const SmoothOp &S, const double *b, double *x, double *t1, double *t2,
                               hipStream_t st);
hipError_t launch_eps_q_field(const SmoothOp &S, const Cpl &C, const double *eps_nodes, double *eps_q,
                              hipStream_t st);
hipError_t launch_drift_bin_batch(const Dev *tab, const BedRun *run, const unsigned *map, int blocks, int n,
                                  hipStream_t st);
hipError_t launch_force_kick_batch(const Dev *tab, const BedRun *run, const unsigned *map, int blocks,
                                   int i, int n, bool fp32, int maxn, int lanes, bool roll, hipStream_t st);
hipError_t launch_batch_advance(BedRun *run, int nb, int n, int *cnt, hipStream_t st);
hipError_t launch_reset_count(int *cnt_words, hipStream_t st);
hipError_t launch_batch_set_bed(Dev *tab, BedRun *run, int b, const Dev &D, long long s, const int *src,
                                hipStream_t st);
hipError_t launch_batch_set_cpl(Cpl *ctab, CplIO *iot, int b, const Cpl &C, const CplIO &io, hipStream_t st);
hipError_t launch_couple_batch(const Dev *tab, const Cpl *ctab, const CplIO *iot, const BedRun *run,
                               const unsigned *map_class, int blocks_class, int *cnt_words,
                               unsigned *list, const long long mode_elems[3], int order, bool fp32, int nt,
                               hipStream_t st);
int couple_class_elems_per_block();
}  // namespace cfddem

using namespace cfddem;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr size_t kAlign = 256;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// ---------------------------------------------------------------------------
// derived sizes
// ---------------------------------------------------------------------------
struct Sizes {
  int n, maxn, cap;
  int lanes;  // lanes per particle in the contact-force kernel
  int smooth;     // smoothed void fraction
  int order;      // velocity element order (1 or 2)
  int nn[3];      // velocity nodes per axis
  long nv;        // velocity nodes
  double skin;
  Grid grid;
  int scan_blocks;  // blocks of the device scan over max(ncells, n) items
};

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

// Generalized symmetric eigenproblem K v = lam M v, M positive definite (n x n
// row-major, n up to a few hundred; set-up only): Cholesky M = L L^T, the
// symmetric C = L^-1 K L^-T diagonalized by cyclic Jacobi rotations
// (C = Q diag(lam) Q^T), then V = L^-T Q, so that V^T M V = I and
// V^T K V = diag(lam).  V is returned row-major with the eigenvectors as
// columns.  False if M is not positive definite.
bool gen_eig(int n, const std::vector<double> &M, const std::vector<double> &K, std::vector<double> &V,
             std::vector<double> &lam) {
  const size_t N = (size_t)n;
  std::vector<double> L(N * N, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = M[j * N + j];
    for (int k = 0; k < j; ++k) d -= L[j * N + k] * L[j * N + k];
    if (!(d > 0.0)) return false;
    L[j * N + j] = sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double v = M[i * N + j];
      for (int k = 0; k < j; ++k) v -= L[i * N + k] * L[j * N + k];
      L[i * N + j] = v / L[j * N + j];
    }
  }
  // W = L^-1 K (column by column), C^T = L^-1 W^T
  std::vector<double> W(N * N), C(N * N);
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double v = K[i * N + c];
      for (int k = 0; k < i; ++k) v -= L[i * N + k] * W[k * N + c];
      W[i * N + c] = v / L[i * N + i];
    }
  for (int r = 0; r < n; ++r)
    for (int i = 0; i < n; ++i) {
      double v = W[r * N + i];
      for (int k = 0; k < i; ++k) v -= L[i * N + k] * C[r * N + k];
      C[r * N + i] = v / L[i * N + i];
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double v = 0.5 * (C[i * N + j] + C[j * N + i]);
      C[i * N + j] = C[j * N + i] = v;
    }
  std::vector<double> Q(N * N, 0.0);
  for (int i = 0; i < n; ++i) Q[i * N + i] = 1.0;
  double norm = 0.0;
  for (size_t i = 0; i < N * N; ++i) norm += C[i] * C[i];
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += C[i * N + j] * C[i * N + j];
    if (off <= 1e-32 * norm) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = C[p * N + q];
        if (apq == 0.0) continue;
        const double theta = (C[q * N + q] - C[p * N + p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double a = C[k * N + p], b = C[k * N + q];
          C[k * N + p] = cs * a - sn * b;
          C[k * N + q] = sn * a + cs * b;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double a = C[p * N + k], b = C[q * N + k];
          C[p * N + k] = cs * a - sn * b;
          C[q * N + k] = sn * a + cs * b;
        }
        for (int k = 0; k < n; ++k) {
          const double a = Q[k * N + p], b = Q[k * N + q];
          Q[k * N + p] = cs * a - sn * b;
          Q[k * N + q] = sn * a + cs * b;
        }
      }
  }
  lam.resize(N);
  for (int i = 0; i < n; ++i) lam[i] = C[i * N + i];
  // V = L^-T Q: back substitution, column by column
  V.assign(N * N, 0.0);
  for (int c = 0; c < n; ++c)
    for (int i = n - 1; i >= 0; --i) {
      double v = Q[i * N + c];
      for (int k = i + 1; k < n; ++k) v -= L[k * N + i] * V[k * N + c];
      V[i * N + c] = v / L[i * N + i];
    }
  return true;
}

// DEM_OK when the parameters are valid; fills the derived grid / capacity.
dem_status derive(const dem_params *dp, const cfd_params *cp, Sizes &S) {
  if (!dp || !cp) return DEM_E_ARG;
  if (dp->abi_version != CFDDEM_ABI_VERSION) return DEM_E_ABI;
  if (dp->n < 1 || dp->n > (int64_t)0x7ffffff0) return DEM_E_ARG;
  if (dp->precision != DEM_FP64 && dp->precision != DEM_FP32_FORCES) return DEM_E_ARG;
  if (!finite_pos(dp->dt) || !finite_pos(dp->E) || !finite_pos(dp->E_w)) return DEM_E_ARG;
  if (!(dp->nu > -1.0 && dp->nu < 0.5) || !(dp->nu_w > -1.0 && dp->nu_w < 0.5)) return DEM_E_ARG;
  if (!(dp->e > 0.0 && dp->e <= 1.0) || !(dp->e_w > 0.0 && dp->e_w <= 1.0)) return DEM_E_ARG;
  if (!(dp->mu >= 0.0) || !(dp->mu_w >= 0.0)) return DEM_E_ARG;
  if (!(dp->mu_r >= 0.0) || !(dp->mu_r_w >= 0.0) || !isfinite(dp->mu_r) || !isfinite(dp->mu_r_w))
    return DEM_E_ARG;
  if (!finite_pos(dp->d_max) || !finite_pos(dp->d_min) || dp->d_min > dp->d_max) return DEM_E_ARG;
  if (dp->max_neighbors < 0 || dp->max_neighbors > kMaxNeighbors) return DEM_E_ARG;
  if (!(dp->skin >= 0.0) || !isfinite(dp->skin)) return DEM_E_ARG;
  if (dp->cell_capacity < 0 || dp->cell_capacity > 1024) return DEM_E_ARG;
  if (dp->resort_every < 0) return DEM_E_ARG;
  if (dp->lanes != 0 && dp->lanes != 1 && dp->lanes != 2 && dp->lanes != 4) return DEM_E_ARG;
  S.lanes = dp->lanes ? dp->lanes : kForceLanes;
  for (int a = 0; a < 3; ++a) {
    if (!isfinite(dp->box_lo[a]) || !isfinite(dp->box_hi[a]) || !(dp->box_hi[a] > dp->box_lo[a]))
      return DEM_E_ARG;
    if (!isfinite(dp->gravity[a])) return DEM_E_ARG;
    if (cp->n_el[a] < 1) return DEM_E_ARG;
  }
  if (cp->order != 1 && cp->order != 2) return DEM_E_ARG;
  if (!finite_pos(cp->rho_f) || !finite_pos(cp->mu_f)) return DEM_E_ARG;
  if (!(cp->eps_min > 0.0 && cp->eps_min <= 1.0)) return DEM_E_ARG;
  if (cp->model != DEM_MODEL_A && cp->model != DEM_MODEL_B) return DEM_E_ARG;
  if (cp->shear != 0 && cp->shear != 1) return DEM_E_ARG;
  if (cp->elem_threads != 0 && cp->elem_threads != 16 && cp->elem_threads != 32 && cp->elem_threads != 64 &&
      cp->elem_threads != 128)
    return DEM_E_ARG;
  if ((cp->smooth != 0 && cp->smooth != 1) || !(cp->smooth_L2 >= 0.0) || !isfinite(cp->smooth_L2))
    return DEM_E_ARG;
  if ((cp->drag & ~(0xff | DEM_DRAG_BETA_OVER_EPS)) != 0 || (cp->drag & 0xff) > DEM_DRAG_GIDASPOW)
    return DEM_E_UNSUPPORTED;

  S.n = (int)dp->n;
  S.smooth = cp->smooth;
  S.order = cp->order;
  S.nv = 1;
  for (int a = 0; a < 3; ++a) {
    S.nn[a] = cp->order * cp->n_el[a] + 1;
    S.nv *= S.nn[a];
  }
  S.maxn = dp->max_neighbors ? dp->max_neighbors : 32;
  S.skin = dp->skin > 0.0 ? dp->skin : 0.1 * dp->d_min;
  // the broad search needs cells at least d_max + skin wide; an element
  // narrower than that caps the skin
  for (int a = 0; a < 3; ++a) {
    const double he = (dp->box_hi[a] - dp->box_lo[a]) / (double)cp->n_el[a];
    const double room = he / (1.0 + 1e-9) - dp->d_max;
    if (room < S.skin) S.skin = room > 0.0 ? room : 0.0;
  }
  Grid &G = S.grid;
  double hc_max = 0.0;
  long long n_elem = 1, ncells = 1;
  for (int a = 0; a < 3; ++a) {
    const double len = dp->box_hi[a] - dp->box_lo[a];
    G.lo[a] = dp->box_lo[a];
    G.hi[a] = dp->box_hi[a];
    G.n_el[a] = cp->n_el[a];
    G.he[a] = len / (double)cp->n_el[a];
    G.inv_he[a] = (double)cp->n_el[a] / len;
    // cells strictly wider than the largest diameter, nested in the element
    double kd = floor(G.he[a] / ((dp->d_max + S.skin) * (1.0 + 1e-9)));
    if (kd < 1.0) kd = 1.0;
    if (kd > 64.0) kd = 64.0;
    G.k[a] = (int)kd;
    G.inv_hc[a] = (double)(G.k[a] * cp->n_el[a]) / len;
    G.gc[a] = G.k[a] * cp->n_el[a];
    if (G.he[a] / G.k[a] > hc_max) hc_max = G.he[a] / G.k[a];
    n_elem *= cp->n_el[a];
    ncells *= (long long)G.gc[a];
  }
  // every element must hold at least one maximum diameter per axis
  for (int a = 0; a < 3; ++a)
    if (G.he[a] < dp->d_max) return DEM_E_UNSUPPORTED;
  if (ncells > 0x7fffffffLL || n_elem > 0x7fffffffLL) return DEM_E_ARG;
  if (S.smooth && S.nv > 0x7fffffffL) return DEM_E_ARG;  // the transforms index lattice lines with int
  G.kk = G.k[0] * G.k[1] * G.k[2];
  G.n_elem = (int)n_elem;
  G.ncells = (int)ncells;
  if (dp->cell_capacity) {
    S.cap = dp->cell_capacity;
  } else {
    // centres at mutual distance >= 0.9 d_min: the balls of that diameter are
    // disjoint and lie in the cell grown by half of it; bound by the densest
    // sphere packing fraction.
    const double del = 0.9 * dp->d_min;
    const double grown = hc_max + del;
    double c = 0.7405 * grown * grown * grown / (kPi / 6.0 * del * del * del);
    c = ceil(c);
    if (c < 8.0) c = 8.0;
    if (c > 1024.0) c = 1024.0;
    S.cap = (int)c;
  }
  const long long items = G.ncells > S.n ? G.ncells : S.n;
  S.scan_blocks = (int)((items + kScanTile - 1) / kScanTile);
  return DEM_OK;
}

// Workspace carving: every array 256-byte aligned.
struct Carver {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct Buffers {
  Dev D;
  // alternates for the re-sort (swapped with D's arrays)
  dvec4 *x2;
  double *v2, *w2, *Fc2, *Tc2, *ffp2, *rad2, *mass2, *whdt2;
  int *oid2, *cell2;
  unsigned char *wmask2;
  int *perm;                    // new index -> old index of the last re-sort
  int *start;                   // first sorted index of each cell (re-sort)
  long long *cnt64, *off64;     // per-particle contact counts / offsets
  long long *bsum;              // per-block partial sums of the device scan
  unsigned long long *scalars;  // [0] contact count, [1] radius max bits, [2] radius min bits
  double *energy;               // per-block kinetic energies, then the two totals
  double *metrics;              // per-block metric partials, then the seven results
  // smoothed void fraction (only when enabled): fixed-point element volume
  // sums, the right-hand side, the field, two scratch vectors, and per axis
  // the generalized eigenvectors (and transpose) and eigenvalues
  double *eps_e, *sb, *sx, *st1, *st2;
  double *fdV[3], *fdVt[3], *fdlam[3];
};

size_t carve(const Sizes &S, char *base, Buffers &B) {
  Carver c{base};
  const size_t n = (size_t)S.n, mn = (size_t)S.maxn;
  Dev &D = B.D;
  D.err = c.take<int>(64);
  if (base) {
    D.flag = D.err + kFlagWord;
    D.lbuf = D.err + kLbufWord;
  }
  B.scalars = c.take<unsigned long long>(8);
  B.energy = c.take<double>(2 * ((n + 255) / 256) + 2);
  {
    const size_t nq1 = (size_t)S.order + 1;
    const size_t nqt = (size_t)S.grid.n_elem * nq1 * nq1 * nq1;
    B.metrics = c.take<double>(6 * ((n + 255) / 256) + (nqt + 255) / 256 + 8);
  }
  if (S.smooth) {
    const size_t nv = (size_t)S.nv;
    B.eps_e = c.take<double>((size_t)S.grid.n_elem);
    B.sb = c.take<double>(nv);
    B.sx = c.take<double>(nv);
    B.st1 = c.take<double>(nv);
    B.st2 = c.take<double>(nv);
    for (int a = 0; a < 3; ++a) {
      const size_t m = (size_t)S.nn[a];
      B.fdV[a] = c.take<double>(m * m);
      B.fdVt[a] = c.take<double>(m * m);
      B.fdlam[a] = c.take<double>(m);
    }
  }
  for (int b = 0; b < 2; ++b) {
    D.pr[b] = c.take<dvec4>(n);
    D.vm[b] = c.take<dvec4>(n);
    D.ws[b] = c.take<dvec4>(n);
    D.slot[b] = c.take<int>((size_t)S.grid.ncells * S.cap);
  }
  for (int b = 0; b < 3; ++b) {
    D.cell[b] = c.take<int>(n);
    D.cnt[b] = c.take<int>((size_t)S.grid.ncells);
  }
  D.v = c.take<double>(3 * n);
  D.w = c.take<double>(3 * n);
  D.Fc = c.take<double>(3 * n);
  D.Tc = c.take<double>(3 * n);
  D.ffp = c.take<double>(3 * n);
  D.rad = c.take<double>(n);
  D.mass = c.take<double>(n);
  D.xb = c.take<double>(3 * n);
  D.oid = c.take<int>(n);
  for (int b = 0; b < 2; ++b) {
    D.ln[b] = c.take<int>(n);
    D.nbr[b] = c.take<unsigned long long>(mn * n);
    D.hmask[b] = c.take<unsigned long long>(n);
    D.hdt[b] = c.take<double>(3 * mn * n);
  }
  D.wmask = c.take<unsigned char>(n);
  D.whdt = c.take<double>(3 * kWalls * n);
  D.occ = c.take<int>((size_t)S.grid.n_elem);
  D.home = c.take<int>(n);
  D.base = c.take<int>((size_t)S.grid.ncells);
  B.x2 = c.take<dvec4>(n);
  B.v2 = c.take<double>(3 * n);
  B.w2 = c.take<double>(3 * n);
  B.Fc2 = c.take<double>(3 * n);
  B.Tc2 = c.take<double>(3 * n);
  B.ffp2 = c.take<double>(3 * n);
  B.rad2 = c.take<double>(n);
  B.mass2 = c.take<double>(n);
  B.oid2 = c.take<int>(n);
  B.cell2 = c.take<int>(n);
  B.wmask2 = c.take<unsigned char>(n);
  B.whdt2 = c.take<double>(3 * kWalls * n);
  B.perm = c.take<int>(n);
  B.start = c.take<int>((size_t)S.grid.ncells);
  D.start = B.start;
  B.cnt64 = c.take<long long>(n + 1);
  B.off64 = c.take<long long>(n + 1);
  B.bsum = c.take<long long>((size_t)S.scan_blocks + 1);
  return c.off + kAlign;
}

// ---------------------------------------------------------------------------
// small kernels: state copy-in, scatter to original order, re-sort gathers
// ---------------------------------------------------------------------------
__global__ void k_init(Dev D, const double *x, const double *v, const double *w, const double *r,
                       const double *rho, unsigned long long *rbits) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D.n) return;
  const int n = D.n;
  D.pr[0][k] = dvec4{x[k], x[n + k], x[2 * n + k], r[k]};
  for (int c = 0; c < 3; ++c) {
    D.v[c * n + k] = v[c * n + k];
    D.w[c * n + k] = w[c * n + k];
    D.Fc[c * n + k] = 0.0;
    D.Tc[c * n + k] = 0.0;
    D.ffp[c * n + k] = 0.0;
  }
  const double rk = r[k];
  D.rad[k] = rk;
  D.mass[k] = rho[k] * (4.0 / 3.0 * kPi * rk * rk * rk);
  D.oid[k] = k;
  for (int b = 0; b < 3; ++b) D.cell[b][k] = 0;
  for (int c = 0; c < 3; ++c) D.xb[c * n + k] = x[c * n + k];
  D.ln[0][k] = 0;
  D.ln[1][k] = 0;
  D.hmask[0][k] = 0;
  D.hmask[1][k] = 0;
  D.wmask[k] = 0;
  // radius and density checks: NaN or non-positive values poison the max
  unsigned long long bits = (rk > 0.0 && rho[k] > 0.0 && isfinite(rk) && isfinite(rho[k]))
                                ? (unsigned long long)__double_as_longlong(rk)
                                : 0x7ff8000000000000ULL;
  atomicMax(&rbits[0], bits);
  atomicMin(&rbits[1], bits);
}

__global__ void k_scatter_pos(int n, const int *oid, const dvec4 *src, double *dst) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int o = oid[k];
  const dvec4 p = src[k];
  dst[o] = p.x;
  dst[n + o] = p.y;
  dst[2 * n + o] = p.z;
}

__global__ void k_scatter3(int n, const int *oid, const double *src, double *dst) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int o = oid[k];
  for (int c = 0; c < 3; ++c) dst[c * n + o] = src[c * n + k];
}

__global__ void k_scatter_cells(int n, int kk, const int *oid, const int *cell, int *elem_out,
                                int *cell_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int o = oid[k];
  if (elem_out) elem_out[o] = cell[k] / kk;
  if (cell_out) cell_out[o] = cell[k];
}

__global__ void k_iota(int n, int *vals) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  vals[k] = k;
}

// Device exclusive scan in three passes: tile-local scan + tile totals, scan
// of the tile totals in one block, add the tile offsets.  `clamp` > 0 caps
// every input at that value (cell counts are capped at the slot capacity).
template <typename TI, typename TO>
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(long long n, const TI *in, int clamp,
                                                             TO *out, long long *bsum) {
  __shared__ long long part[kScanThreads];
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  long long v[kScanItems];
  long long s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    long long t = (base + i < n) ? (long long)in[base + i] : 0;
    if (clamp > 0 && t > clamp) t = clamp;
    v[i] = s;
    s += t;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const long long add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  const long long excl = part[threadIdx.x] - s;
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) out[base + i] = (TO)(v[i] + excl);
  if (threadIdx.x == kScanThreads - 1) bsum[blockIdx.x] = part[threadIdx.x];
}

// exclusive scan of the tile totals; bsum[nb] receives the grand total
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(int nb, long long *bsum) {
  __shared__ long long part[kScanThreads];
  long long carry = 0;
  for (int base = 0; base < nb; base += kScanThreads) {
    const int i = base + threadIdx.x;
    const long long s = i < nb ? bsum[i] : 0;
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
      const long long add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + part[threadIdx.x] - s;
    const long long tile_total = part[kScanThreads - 1];
    __syncthreads();
    carry += tile_total;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

template <typename TO>
__global__ __launch_bounds__(kScanThreads) void k_scan_add(long long n, TO *out, const long long *bsum) {
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  const long long add = bsum[blockIdx.x];
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) out[base + i] = (TO)((long long)out[base + i] + add);
}

template <typename TI, typename TO>
hipError_t device_exclusive_scan(long long n, const TI *in, int clamp, TO *out, long long *bsum,
                                 hipStream_t st) {
  const int nb = (int)((n + kScanTile - 1) / kScanTile);
  if (nb == 0) return hipSuccess;
  k_scan_tiles<TI, TO><<<nb, kScanThreads, 0, st>>>(n, in, clamp, out, bsum);
  k_scan_totals<<<1, kScanThreads, 0, st>>>(nb, bsum);
  k_scan_add<TO><<<nb, kScanThreads, 0, st>>>(n, out, bsum);
  return hipGetLastError();
}

// New position of every particle when the arrays are ordered by cell: the
// cell's first index plus the particle's rank among the cell's particles by
// original ID (independent of the atomic insertion order).
__global__ void k_rank(Dev D, int p2, int p3, const int *start, int *perm) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D.n) return;
  const int c = D.cell[p3][k];
  int m = D.cnt[p3][c];
  if (m > D.cap) m = D.cap;
  const int o = D.oid[k];
  int rank = 0;
  const int *sl = D.slot[p2] + (size_t)c * D.cap;
  for (int s = 0; s < m; ++s) rank += D.oid[sl[s]] < o;
  const int dst = start[c] + rank;
  if (dst >= 0 && dst < D.n) perm[dst] = k;
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long a, unsigned long long b) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    p[0] = a;
    p[1] = b;
  }
}

struct PermSrc {
  const dvec4 *x;
  const double *v, *w, *Fc, *Tc, *ffp, *rad, *mass, *whdt;
  const int *oid, *cell;
  const unsigned char *wmask;
};
struct PermDst {
  dvec4 *x;
  double *v, *w, *Fc, *Tc, *ffp, *rad, *mass, *whdt;
  int *oid, *cell, *home;
  unsigned char *wmask;
};

// Gather every per-particle array into cell order.  Neighbour lists are not
// moved: the broad search that follows a re-sort reads them through perm.
__global__ void k_permute(int n, const int *perm, PermSrc s, PermDst d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int o = perm[k];
  if (o < 0 || o >= n) o = k;  // only after a capacity error (already flagged)
  d.x[k] = s.x[o];
  for (int c = 0; c < 3; ++c) {
    d.v[c * n + k] = s.v[c * n + o];
    d.w[c * n + k] = s.w[c * n + o];
    d.Fc[c * n + k] = s.Fc[c * n + o];
    d.Tc[c * n + k] = s.Tc[c * n + o];
    d.ffp[c * n + k] = s.ffp[c * n + o];
  }
  d.rad[k] = s.rad[o];
  d.mass[k] = s.mass[o];
  d.oid[k] = s.oid[o];
  d.cell[k] = s.cell[o];
  d.home[k] = s.cell[o];
  d.wmask[k] = s.wmask[o];
  for (int wall = 0; wall < kWalls; ++wall)
    for (int c = 0; c < 3; ++c) d.whdt[hist_at(wall, n, k) + c] = s.whdt[hist_at(wall, n, o) + c];
}

// Kinetic energy of the boundary state: translational sum 1/2 m v^2 and
// rotational sum 1/2 I w^2 (I = 2/5 m R^2).  Each block adds its particles in
// a fixed tree order into part[2 block], part[2 block + 1]; one wave then adds
// the block partials (lane l takes blocks l, l + 64, ... in order, then a fixed
// butterfly), so the totals do not depend on timing.
__global__ __launch_bounds__(256) void k_energy_partials(Dev D, double *part) {
  __shared__ double sh[2][256];
  const int k = blockIdx.x * 256 + threadIdx.x;
  double et = 0.0, er = 0.0;
  if (k < D.n) {
    const int n = D.n;
    const double m = D.mass[k], r = D.rad[k];
    double v2 = 0.0, w2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      v2 += D.v[c * n + k] * D.v[c * n + k];
      w2 += D.w[c * n + k] * D.w[c * n + k];
    }
    et = 0.5 * m * v2;
    er = 0.5 * (0.4 * m * r * r) * w2;
  }
  sh[0][threadIdx.x] = et;
  sh[1][threadIdx.x] = er;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0][0];
    part[2 * blockIdx.x + 1] = sh[1][0];
  }
}

__global__ __launch_bounds__(64) void k_energy_total(int nb, const double *part, double *out) {
  double et = 0.0, er = 0.0;
  for (int i = (int)threadIdx.x; i < nb; i += 64) {
    et += part[2 * i];
    er += part[2 * i + 1];
  }
  for (int off = 1; off < 64; off <<= 1) {
    et += __shfl_xor(et, off, 64);
    er += __shfl_xor(er, off, 64);
  }
  if (threadIdx.x == 0) {
    out[0] = et;
    out[1] = er;
  }
}

// Metrics of the current state, per block of 256 particles: momentum (3),
// solid volume, largest overlap ratio, largest speed.  lbw: word of the lbuf
// array holding the list buffer of the last evaluation; p2: position buffer
// of the last completed step.
__global__ __launch_bounds__(256) void k_metrics_partials(Dev D, int lbw, int p2, double *part) {
  __shared__ double sh[6][256];
  const int k = blockIdx.x * 256 + threadIdx.x;
  double q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (k < D.n) {
    const int n = D.n;
    const double m = D.mass[k], r = D.rad[k];
    double v2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double vc = D.v[c * n + k];
      q[c] = m * vc;
      v2 += vc * vc;
    }
    q[3] = 4.0 / 3.0 * kPi * r * r * r;
    q[5] = sqrt(v2);
    // normal overlaps of the touching list entries and walls, at the
    // positions the last evaluation used
    const int lb = D.lbuf[lbw];
    const dvec4 *X = D.pr[p2];
    const dvec4 xa = X[k];
    const unsigned long long mask = D.hmask[lb][k];
    const int len = D.ln[lb][k];
    double worst = 0.0;
    for (int t = 0; t < len; ++t) {
      if (!((mask >> t) & 1ull)) continue;
      const int b = (int)(D.nbr[lb][(size_t)t * n + k] & 0xffffffffull);
      const dvec4 xb = X[b];
      const double d0 = xb.x - xa.x, d1 = xb.y - xa.y, d2 = xb.z - xa.z;
      const double dn = (xa.w + xb.w) - sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      worst = fmax(worst, dn / fmin(xa.w, xb.w));
    }
    const unsigned wm = D.wmask[k];
    for (int w = 0; w < kWalls; ++w) {
      if (!((wm >> w) & 1u)) continue;
      const int ax = w >> 1;
      const double xax = ax == 0 ? xa.x : (ax == 1 ? xa.y : xa.z);
      const double lo = ax == 0 ? D.grid.lo[0] : (ax == 1 ? D.grid.lo[1] : D.grid.lo[2]);
      const double hi = ax == 0 ? D.grid.hi[0] : (ax == 1 ? D.grid.hi[1] : D.grid.hi[2]);
      const double dist = (w & 1) ? hi - xax : xax - lo;
      worst = fmax(worst, (xa.w - dist) / xa.w);
    }
    q[4] = worst;
  }
  for (int j = 0; j < 6; ++j) sh[j][threadIdx.x] = q[j];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + h];
      for (int j = 4; j < 6; ++j) sh[j][threadIdx.x] = fmax(sh[j][threadIdx.x], sh[j][threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// Solid volume seen at the quadrature points, per block of 256 points:
// sum of w_q (1 - eps_q), w_q = Ve times the product of the 1D Gauss weights
// (points ordered element-major, then z, y, x inside an element).
__global__ __launch_bounds__(256) void k_qsolid_partials(const double *eps_q, long long nqt, int nq1, double wa,
                                                         double wb, double Ve, double *part) {
  __shared__ double sh[256];
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (i < nqt) {
    const int nq = nq1 * nq1 * nq1;
    const int l = (int)(i % nq);
    const int qx = l % nq1, qy = (l / nq1) % nq1, qz = l / (nq1 * nq1);
    // 1D weight: wa at the end points, wb at the middle one (three points)
    const double w = (qx == 1 && nq1 == 3 ? wb : wa) * (qy == 1 && nq1 == 3 ? wb : wa) *
                     (qz == 1 && nq1 == 3 ? wb : wa);
    v = Ve * w * (1.0 - eps_q[i]);
  }
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// The seven metrics from the block partials, in a fixed order.
__global__ __launch_bounds__(64) void k_metrics_total(int nb, const double *part, int nbq, const double *qpart,
                                                      double *out) {
  double q[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = (int)threadIdx.x; i < nb; i += 64) {
    for (int j = 0; j < 4; ++j) q[j] += part[6 * i + j];
    q[4] = fmax(q[4], part[6 * i + 4]);
    q[6] = fmax(q[6], part[6 * i + 5]);
  }
  for (int i = (int)threadIdx.x; i < nbq; i += 64) q[5] += qpart[i];
  for (int off = 1; off < 64; off <<= 1) {
    for (int j = 0; j < 4; ++j) q[j] += __shfl_xor(q[j], off, 64);
    q[5] += __shfl_xor(q[5], off, 64);
    q[4] = fmax(q[4], __shfl_xor(q[4], off, 64));
    q[6] = fmax(q[6], __shfl_xor(q[6], off, 64));
  }
  if (threadIdx.x == 0) {
    out[0] = q[0];
    out[1] = q[1];
    out[2] = q[2];
    out[3] = q[4];
    out[4] = q[3];
    out[5] = nbq > 0 ? q[5] : __builtin_nan("");
    out[6] = q[6];
  }
}

// Contacts of the last evaluation that particle k reports: its walls, and the
// touching list entries whose partner has a larger original ID.
__global__ void k_contact_count(Dev D, int lb, long long *cnt, unsigned long long *total) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D.n) return;
  const int n = D.n;
  const int o = D.oid[k];
  int m = __popc((unsigned)D.wmask[k]);
  const unsigned long long mask = D.hmask[lb][k];
  for (int t = 0; t < D.ln[lb][k]; ++t)
    if (((mask >> t) & 1ull) && (int)(D.nbr[lb][(size_t)t * n + k] >> 32) > o) ++m;
  cnt[o] = m;
  if (total) atomicAdd(total, (unsigned long long)m);
}

__global__ void k_contact_write(Dev D, int lb, const long long *off, long long cap, long long *pairs,
                                double *dt_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= D.n) return;
  const int n = D.n;
  const int o = D.oid[k];
  long long w = off[o];
  // walls in descending face index (ascending -1-w), then partners by oid
  const unsigned wm = D.wmask[k];
  for (int wall = kWalls - 1; wall >= 0; --wall) {
    if (!((wm >> wall) & 1u)) continue;
    if (w < cap) {
      pairs[w] = o;
      pairs[cap + w] = -1 - wall;
      for (int c = 0; c < 3; ++c) dt_out[(size_t)c * cap + w] = D.whdt[hist_at(wall, n, k) + c];
    }
    ++w;
  }
  const unsigned long long mask = D.hmask[lb][k];
  for (int t = 0; t < D.ln[lb][k]; ++t) {
    const int ob = (int)(D.nbr[lb][(size_t)t * n + k] >> 32);
    if (!((mask >> t) & 1ull) || ob <= o) continue;
    if (w < cap) {
      pairs[w] = o;
      pairs[cap + w] = ob;
      for (int c = 0; c < 3; ++c) dt_out[(size_t)c * cap + w] = D.hdt[lb][hist_at(t, n, k) + c];
    }
    ++w;
  }
}

inline int blocks(int n, int b) { return (n + b - 1) / b; }

// Device words of a context restored from a checkpoint: the list buffer the
// next step reads, the sticky error bits; broad-search flags and the
// occupied-element counters start cleared.
__global__ void k_restore_words(int *err, int lb_word, int cur, int bits) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (int i = 0; i < 3; ++i) err[kFlagWord + i] = 0;
  err[kOccWord] = 0;
  err[kOccWord + 1] = 0;
  err[kLbufWord + lb_word] = cur;
  err[0] = bits;
}

// Checkpoint blob: a 256-byte header, then the state arrays in the context's
// internal (cell-sorted) order, each at a 256-byte aligned offset.
constexpr uint64_t kCkptMagic = 0x4b43424d45444643ULL;  // "CFDEMBCK"
constexpr int kCkptVersion = 3;
struct CkptHeader {
  uint64_t magic;
  int32_t abi, version;
  int64_t n;
  int32_t maxn, lbuf;       // neighbour-list capacity; list buffer of the next step
  int32_t since_sort, err;  // steps since the last re-sort; sticky error bits
  int64_t s, n_couple;      // completed steps; coupling calls issued
  uint64_t shape;           // hash of the structural parameters
};
static_assert(sizeof(CkptHeader) <= 256, "checkpoint header");

struct Span {
  void *p;
  size_t bytes;
};

dem_status err_to_status(int bits) {
  if (bits & kErrNan) return DEM_E_NAN;
  if (bits & kErrDomain) return DEM_E_DOMAIN;
  if (bits & kErrCapacity) return DEM_E_CAPACITY;
  return DEM_OK;
}

}  // namespace

struct dem_ctx {
  dem_params dp;
  cfd_params cp;
  Sizes S;
  Buffers B;
  Cpl C;
  bool fp32;
  long long s = 0;  // index of the last completed step (0 = creation)
  const int *pending_src = nullptr;  // permutation to apply at the next broad search
  int since_sort = 0;
  long long n_couple = 0;  // coupling steps issued
  dem_status poisoned = DEM_OK;
  bool timing = false;
  SmoothOp SO{};           // smoothed void fraction operator (smooth = 1)
  int in_batch = 0;        // batches holding this bed
  std::vector<hipEvent_t> ev;  // pairs (start, stop) of timed launches
  size_t ev_used = 0;
};

#define HIP_TRY(...)                        \
  do {                                      \
    if ((__VA_ARGS__) != hipSuccess) return DEM_E_HIP; \
  } while (0)

// ---------------------------------------------------------------------------
// scratch of the allocation-free kinetic-energy call
// ---------------------------------------------------------------------------
// Per-block partial sums (2 per block of 256 particles) of
// dem_kinetic_energy_noalloc live in this fixed array, which every GPU the
// library runs on holds for the life of the process (1 MiB), instead of in a
// bed's workspace.  Host code reaches it only through the device address that
// hipGetSymbolAddress returns for the device current at the first call there.
constexpr int kEnergyScratchBlocks = 65536;  // beds of up to 256 x 65536 particles
static __device__ __align__(256) double scratch[2 * kEnergyScratchBlocks];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
dem_status scratch_of_current_device(double **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return DEM_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DEM_E_HIP;
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return DEM_OK;
}
}  // namespace

// Particles per cell of the grid just sorted (at most cap): with start and
// home, the listing the following runs take as their cells' home ranges.
namespace {
__global__ void k_home_base(int ncells, const int *cnt, int cap, int *base) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncells) base[c] = min(cnt[c], cap);
}
}  // namespace

// No home cells (before the first re-sort, after a restore): every grid
// lists all of its particles in its slots.
static hipError_t clear_epoch(const Dev &D, hipStream_t st) {
  hipError_t e = hipMemsetAsync(D.base, 0, sizeof(int) * (size_t)D.grid.ncells, st);
  if (e == hipSuccess) e = hipMemsetAsync(D.home, 0xff, sizeof(int) * (size_t)D.n, st);
  return e;
}

static dem_status resort(dem_ctx *ctx, hipStream_t st) {
  Buffers &B = ctx->B;
  Dev &D = B.D;
  const int n = D.n;
  const int p2 = (int)(ctx->s & 1), p3 = (int)(ctx->s % 3);
  // the grid of the last step holds every particle at its current cell
  HIP_TRY(device_exclusive_scan<int, int>(D.grid.ncells, D.cnt[p3], D.cap, B.start, B.bsum, st));
  k_rank<<<blocks(n, 256), 256, 0, st>>>(D, p2, p3, B.start, B.perm);
  HIP_TRY(hipGetLastError());
  PermSrc src{D.pr[p2], D.v, D.w, D.Fc, D.Tc, D.ffp, D.rad, D.mass, D.whdt, D.oid, D.cell[p3],
              D.wmask};
  PermDst dst{B.x2, B.v2, B.w2, B.Fc2, B.Tc2, B.ffp2, B.rad2, B.mass2, B.whdt2, B.oid2, B.cell2,
              D.home, B.wmask2};
  k_permute<<<blocks(n, 256), 256, 0, st>>>(n, B.perm, src, dst);
  HIP_TRY(hipGetLastError());
  k_home_base<<<blocks(D.grid.ncells, 256), 256, 0, st>>>(D.grid.ncells, D.cnt[p3], D.cap, D.base);
  HIP_TRY(hipGetLastError());
  std::swap(D.pr[p2], B.x2);
  std::swap(D.v, B.v2);
  std::swap(D.w, B.w2);
  std::swap(D.Fc, B.Fc2);
  std::swap(D.Tc, B.Tc2);
  std::swap(D.ffp, B.ffp2);
  std::swap(D.rad, B.rad2);
  std::swap(D.mass, B.mass2);
  std::swap(D.oid, B.oid2);
  std::swap(D.cell[p3], B.cell2);
  std::swap(D.whdt, B.whdt2);
  std::swap(D.wmask, B.wmask2);
  ctx->pending_src = B.perm;
  ctx->since_sort = 0;
  return DEM_OK;
}

// Launch step s (or the creation-time evaluation when !advance).
static dem_status force_launch(dem_ctx *ctx, long long s, bool advance, bool cont, int gmode, hipStream_t st) {
  const int *src = advance ? ctx->pending_src : nullptr;
  ctx->pending_src = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->timing) {
    if (ctx->ev_used + 2 > ctx->ev.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        ctx->ev.push_back(e);
      }
    }
    e0 = ctx->ev[ctx->ev_used];
    e1 = ctx->ev[ctx->ev_used + 1];
    ctx->ev_used += 2;
  }
  HIP_TRY(launch_force_kick(ctx->B.D, s, src, gmode, advance, cont, ctx->fp32, ctx->S.lanes, st, e0, e1));
  return DEM_OK;
}

// ---------------------------------------------------------------------------
// checkpoints
// ---------------------------------------------------------------------------
// The structural parameters a checkpoint depends on (array sizes, the meaning
// of the neighbour lists and of the cell indices), hashed (FNV-1a) over their
// values.
static uint64_t ckpt_shape(const dem_ctx *ctx) {
  uint64_t h = 1469598103934665603ULL;
  auto mix = [&h](const void *p, size_t b) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < b; ++i) {
      h ^= c[i];
      h *= 1099511628211ULL;
    }
  };
  const Sizes &S = ctx->S;
  const int32_t ints[4] = {S.n, S.maxn, S.cap, ctx->fp32 ? 1 : 0};
  mix(ints, sizeof ints);
  mix(&S.skin, sizeof S.skin);
  mix(S.grid.lo, sizeof S.grid.lo);
  mix(S.grid.hi, sizeof S.grid.hi);
  mix(S.grid.n_el, sizeof S.grid.n_el);
  mix(S.grid.k, sizeof S.grid.k);
  return h;
}

// The arrays of a checkpoint, in the context's internal order: positions of
// the last completed step, boundary velocities, stored contact force and
// torque, held fluid force, radii, masses, positions at the last broad
// search, original IDs, wall contacts and their history, and the neighbour
// list (buffer cur) with its touching masks and tangential history.
static int ckpt_spans(dem_ctx *ctx, int cur, Span *sp) {
  Dev &D = ctx->B.D;
  const size_t n = (size_t)D.n, mn = (size_t)D.maxn * n;
  int k = 0;
  sp[k++] = {D.pr[ctx->s & 1], 32 * n};
  sp[k++] = {D.v, 24 * n};
  sp[k++] = {D.w, 24 * n};
  sp[k++] = {D.Fc, 24 * n};
  sp[k++] = {D.Tc, 24 * n};
  sp[k++] = {D.ffp, 24 * n};
  sp[k++] = {D.rad, 8 * n};
  sp[k++] = {D.mass, 8 * n};
  sp[k++] = {D.xb, 24 * n};
  sp[k++] = {D.oid, 4 * n};
  sp[k++] = {D.wmask, n};
  sp[k++] = {D.whdt, 8 * 3 * kWalls * n};
  sp[k++] = {D.ln[cur], 4 * n};
  sp[k++] = {D.nbr[cur], 8 * mn};
  sp[k++] = {D.hmask[cur], 8 * n};
  sp[k++] = {D.hdt[cur], 24 * mn};
  return k;
}

static size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

static size_t ckpt_size(dem_ctx *ctx) {
  Span sp[24];
  const int k = ckpt_spans(ctx, 0, sp);
  size_t off = kAlign;  // header
  for (int i = 0; i < k; ++i) off = align_up(off) + sp[i].bytes;
  return align_up(off);
}

extern "C" {

size_t dem_checkpoint_bytes(dem_ctx *ctx) { return ctx ? ckpt_size(ctx) : 0; }

dem_status dem_read_checkpoint(dem_ctx *ctx, void *dst, size_t bytes, void *stream) {
  if (!ctx || !dst || ((uintptr_t)dst % kAlign) != 0) return DEM_E_ARG;
  if (bytes < ckpt_size(ctx)) return DEM_E_WORKSPACE;
  if (ctx->poisoned) return ctx->poisoned;
  hipStream_t st = (hipStream_t)stream;
  Dev &D = ctx->B.D;
  int words[2] = {0, 0};  // list buffer of the next step, sticky error bits
  HIP_TRY(hipMemcpyAsync(&words[0], D.lbuf + (ctx->s + 1) % 3, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&words[1], D.err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (err_to_status(words[1]) != DEM_OK) {
    ctx->poisoned = err_to_status(words[1]);
    return ctx->poisoned;
  }
  CkptHeader h{};
  h.magic = kCkptMagic;
  h.abi = CFDDEM_ABI_VERSION;
  h.version = kCkptVersion;
  h.n = ctx->S.n;
  h.maxn = ctx->S.maxn;
  h.lbuf = words[0];
  h.since_sort = ctx->since_sort;
  h.err = words[1];
  h.s = ctx->s;
  h.n_couple = ctx->n_couple;
  h.shape = ckpt_shape(ctx);
  char *out = static_cast<char *>(dst);
  HIP_TRY(hipMemcpyAsync(out, &h, sizeof h, hipMemcpyHostToDevice, st));
  Span sp[24];
  const int k = ckpt_spans(ctx, h.lbuf, sp);
  size_t off = kAlign;
  for (int i = 0; i < k; ++i) {
    off = align_up(off);
    HIP_TRY(hipMemcpyAsync(out + off, sp[i].p, sp[i].bytes, hipMemcpyDeviceToDevice, st));
    off += sp[i].bytes;
  }
  HIP_TRY(hipStreamSynchronize(st));  // the header lives on this call's stack
  return DEM_OK;
}

dem_status dem_write_state(dem_ctx *ctx, const void *src, size_t bytes, void *stream) {
  if (!ctx || !src || ((uintptr_t)src % kAlign) != 0 || bytes < kAlign) return DEM_E_ARG;
  if (ctx->in_batch) return DEM_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  CkptHeader h{};
  HIP_TRY(hipMemcpyAsync(&h, src, sizeof h, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h.magic != kCkptMagic || h.abi != CFDDEM_ABI_VERSION || h.version != kCkptVersion) return DEM_E_ABI;
  if (h.n != ctx->S.n || h.maxn != ctx->S.maxn || h.shape != ckpt_shape(ctx) || h.lbuf < 0 || h.lbuf > 1 ||
      h.s < 0 || h.n_couple < 0 || h.since_sort < 0)
    return DEM_E_ARG;
  if (bytes < ckpt_size(ctx)) return DEM_E_WORKSPACE;
  Dev &D = ctx->B.D;
  // empty every cell grid (at the cells the context's particles were binned
  // into), then take the checkpoint's arrays, then bin its positions into
  // the grid of its step: the grid of a completed step is the only one that
  // holds particles between calls, and the order of the particles in a cell's
  // slots is not part of the result
  for (int b = 0; b < 3; ++b) HIP_TRY(launch_clear_grid(D, b, st));
  ctx->s = h.s;
  Span sp[24];
  const int k = ckpt_spans(ctx, h.lbuf, sp);
  const char *in = static_cast<const char *>(src);
  size_t off = kAlign;
  for (int i = 0; i < k; ++i) {
    off = align_up(off);
    HIP_TRY(hipMemcpyAsync(sp[i].p, in + off, sp[i].bytes, hipMemcpyDeviceToDevice, st));
    off += sp[i].bytes;
  }
  k_restore_words<<<1, 64, 0, st>>>(D.err, (int)((h.s + 1) % 3), h.lbuf, h.err);
  HIP_TRY(hipGetLastError());
  // the checkpoint's particle order is not a re-sort's: no home cells
  HIP_TRY(clear_epoch(D, st));
  HIP_TRY(launch_drift_bin(D, h.s, false, false, true, st));
  ctx->since_sort = h.since_sort;
  ctx->n_couple = h.n_couple;
  ctx->pending_src = nullptr;
  ctx->poisoned = err_to_status(h.err);
  HIP_TRY(hipStreamSynchronize(st));
  return DEM_OK;
}

size_t dem_workspace_bytes(const dem_params *dp, const cfd_params *cp) {
  Sizes S;
  if (derive(dp, cp, S) != DEM_OK) return 0;
  Buffers B;
  return carve(S, nullptr, B);
}

dem_status dem_create(const dem_params *dp, const cfd_params *cp, const double *x,
                      const double *v, const double *omega, const double *radius,
                      const double *density, void *workspace, size_t ws_bytes, void *stream,
                      dem_ctx **out) {
  if (!out) return DEM_E_ARG;
  *out = nullptr;
  Sizes S;
  dem_status s = derive(dp, cp, S);
  if (s != DEM_OK) return s;
  if (!x || !v || !omega || !radius || !density) return DEM_E_ARG;
  Buffers B;
  const size_t need = carve(S, nullptr, B);
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || ws_bytes < need) return DEM_E_WORKSPACE;
  dem_ctx *ctx = new (std::nothrow) dem_ctx();
  if (!ctx) return DEM_E_ARG;
  ctx->dp = *dp;
  ctx->cp = *cp;
  ctx->S = S;
  ctx->fp32 = dp->precision == DEM_FP32_FORCES;
  carve(S, (char *)workspace, ctx->B);
  Dev &D = ctx->B.D;
  D.n = S.n;
  D.cap = S.cap;
  D.maxn = S.maxn;
  D.skin = S.skin;
  D.trig2 = (0.499 * S.skin) * (0.499 * S.skin);
  D.dt = dp->dt;
  for (int a = 0; a < 3; ++a) D.g[a] = dp->gravity[a];
  D.grid = S.grid;
  auto material = [](double Y1, double nu1, double Y2, double nu2, double e, double mu) {
    Material m;
    m.Ye = 1.0 / ((1.0 - nu1 * nu1) / Y1 + (1.0 - nu2 * nu2) / Y2);
    m.Ge = 1.0 / (2.0 * (2.0 - nu1) * (1.0 + nu1) / Y1 + 2.0 * (2.0 - nu2) * (1.0 + nu2) / Y2);
    const double l = log(e);
    const double beta = l / sqrt(l * l + kPi * kPi);
    m.eta_coef = -2.0 * sqrt(5.0 / 6.0) * beta;
    m.mu = mu;
    return m;
  };
  D.pp = material(dp->E, dp->nu, dp->E, dp->nu, dp->e, dp->mu);
  D.pw = material(dp->E, dp->nu, dp->E_w, dp->nu_w, dp->e_w, dp->mu_w);
  D.pp.mu_r = dp->mu_r;
  D.pw.mu_r = dp->mu_r_w;
  // coupling constants
  Cpl &C = ctx->C;
  C.order = cp->order;
  C.nq1 = cp->order + 1;
  C.nq = C.nq1 * C.nq1 * C.nq1;
  C.nvx = cp->order * cp->n_el[0] + 1;
  C.nvy = cp->order * cp->n_el[1] + 1;
  C.npx = cp->n_el[0] + 1;
  C.npy = cp->n_el[1] + 1;
  C.rho_f = cp->rho_f;
  C.mu_f = cp->mu_f;
  C.eps_min = cp->eps_min;
  C.model = cp->model;
  C.drag = cp->drag & 0xff;
  C.beta_over_eps = (cp->drag & DEM_DRAG_BETA_OVER_EPS) ? 1 : 0;
  C.shear = cp->shear;
  C.smooth = cp->smooth;
  C.elem_threads = cp->elem_threads ? cp->elem_threads : 128;
  C.eps_nodes = cp->smooth ? ctx->B.sx : nullptr;
  C.Ve = S.grid.he[0] * S.grid.he[1] * S.grid.he[2];
  {
    double gp[3];
    if (C.nq1 == 2) {
      gp[0] = 0.5 - 0.5 / sqrt(3.0);
      gp[1] = 0.5 + 0.5 / sqrt(3.0);
      gp[2] = 0.0;
    } else {
      gp[0] = 0.5 - 0.5 * sqrt(0.6);
      gp[1] = 0.5;
      gp[2] = 0.5 + 0.5 * sqrt(0.6);
    }
    for (int i = 0; i < 3; ++i) {
      const double t = gp[i];
      if (cp->order == 2) {
        C.Lq[0][i] = 2.0 * (t - 0.5) * (t - 1.0);
        C.Lq[1][i] = -4.0 * t * (t - 1.0);
        C.Lq[2][i] = 2.0 * t * (t - 0.5);
      } else {
        C.Lq[0][i] = 1.0 - t;
        C.Lq[1][i] = t;
        C.Lq[2][i] = 0.0;
      }
      C.Lq1[0][i] = 1.0 - t;
      C.Lq1[1][i] = t;
    }
  }

  hipStream_t st = (hipStream_t)stream;
  const int n = S.n;
  auto fail = [&](dem_status code) {
    delete ctx;
    return code;
  };
  if (hipMemsetAsync(D.err, 0, sizeof(int) * 64, st) != hipSuccess) return fail(DEM_E_HIP);
  if (S.smooth) {
    // 1D element matrices on an element of length h (Lagrange basis on
    // equally spaced nodes): Q1 mass h/6 [2 1; 1 2], stiffness 1/h [1 -1; -1 1],
    // load h/2 [1 1]; Q2 mass h/30 [4 2 -1; 2 16 2; -1 2 4], stiffness
    // 1/(3h) [7 -8 1; -8 16 -8; 1 -8 7], load h [1/6 2/3 1/6].  Assembled per
    // axis, then diagonalized together.
    static const double m1[2][2] = {{2.0 / 6.0, 1.0 / 6.0}, {1.0 / 6.0, 2.0 / 6.0}};
    static const double k1[2][2] = {{1.0, -1.0}, {-1.0, 1.0}};
    static const double m2[3][3] = {{4.0 / 30.0, 2.0 / 30.0, -1.0 / 30.0},
                                    {2.0 / 30.0, 16.0 / 30.0, 2.0 / 30.0},
                                    {-1.0 / 30.0, 2.0 / 30.0, 4.0 / 30.0}};
    static const double k2[3][3] = {{7.0 / 3.0, -8.0 / 3.0, 1.0 / 3.0},
                                    {-8.0 / 3.0, 16.0 / 3.0, -8.0 / 3.0},
                                    {1.0 / 3.0, -8.0 / 3.0, 7.0 / 3.0}};
    static const double l1[2] = {0.5, 0.5}, l2[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
    const int p = cp->order;
    SmoothOp &SO = ctx->SO;
    SO.order = p;
    SO.nv = S.nv;
    SO.L2 = cp->smooth_L2;
    std::vector<double> V[3], Vt[3], lam[3];
    for (int a = 0; a < 3; ++a) {
      const int m = S.nn[a];
      SO.nn[a] = m;
      SO.n_el[a] = cp->n_el[a];
      SO.V[a] = ctx->B.fdV[a];
      SO.Vt[a] = ctx->B.fdVt[a];
      SO.lam[a] = ctx->B.fdlam[a];
      const double h = S.grid.he[a];
      std::vector<double> M((size_t)m * m, 0.0), K((size_t)m * m, 0.0);
      for (int e = 0; e < cp->n_el[a]; ++e)
        for (int i = 0; i <= p; ++i)
          for (int j = 0; j <= p; ++j) {
            const size_t at = (size_t)(p * e + i) * m + (p * e + j);
            M[at] += h * (p == 1 ? m1[i][j] : m2[i][j]);
            K[at] += (p == 1 ? k1[i][j] : k2[i][j]) / h;
          }
      if (!gen_eig(m, M, K, V[a], lam[a])) return fail(DEM_E_ARG);
      Vt[a].resize((size_t)m * m);
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Vt[a][(size_t)j * m + i] = V[a][(size_t)i * m + j];
      for (int l = 0; l < 3; ++l) SO.load[a][l] = l <= p ? h * (p == 1 ? l1[l] : l2[l]) : 0.0;
    }
    bool ok = true;
    for (int a = 0; a < 3; ++a)
      ok = ok &&
           hipMemcpyAsync(ctx->B.fdV[a], V[a].data(), sizeof(double) * V[a].size(), hipMemcpyHostToDevice, st) ==
               hipSuccess &&
           hipMemcpyAsync(ctx->B.fdVt[a], Vt[a].data(), sizeof(double) * Vt[a].size(), hipMemcpyHostToDevice,
                          st) == hipSuccess &&
           hipMemcpyAsync(ctx->B.fdlam[a], lam[a].data(), sizeof(double) * lam[a].size(), hipMemcpyHostToDevice,
                          st) == hipSuccess;
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (!ok) return fail(DEM_E_HIP);
  }
  k_fill_u64<<<1, 64, 0, st>>>(ctx->B.scalars, 0ULL, ~0ULL);
  if (hipGetLastError() != hipSuccess) return fail(DEM_E_HIP);
  for (int b = 0; b < 3; ++b)
    if (hipMemsetAsync(D.cnt[b], 0, sizeof(int) * (size_t)S.grid.ncells, st) != hipSuccess)
      return fail(DEM_E_HIP);
  k_init<<<blocks(n, 256), 256, 0, st>>>(D, x, v, omega, radius, density, ctx->B.scalars);
  k_iota<<<blocks(n, 256), 256, 0, st>>>(n, ctx->B.perm);
  if (hipGetLastError() != hipSuccess) return fail(DEM_E_HIP);
  unsigned long long rb[2];
  if (hipMemcpyAsync(rb, ctx->B.scalars, sizeof(rb), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(DEM_E_HIP);
  double rmax, rmin;
  memcpy(&rmax, &rb[0], sizeof(double));
  memcpy(&rmin, &rb[1], sizeof(double));
  if (!(rmax > 0.0) || isnan(rmax) || isnan(rmin) || 2.0 * rmax > dp->d_max * (1.0 + 1e-12) ||
      2.0 * rmin < dp->d_min * (1.0 - 1e-12))
    return fail(DEM_E_ARG);

  // priming: bin the initial positions, optionally sort by cell, evaluate
  ctx->s = 0;
  if (clear_epoch(D, st) != hipSuccess) return fail(DEM_E_HIP);
  if (launch_drift_bin(D, 0, false, false, true, st) != hipSuccess) return fail(DEM_E_HIP);
  if (dp->resort_every > 0) {
    if (resort(ctx, st) != DEM_OK) return fail(DEM_E_HIP);
    ctx->pending_src = nullptr;  // nothing to carry at creation
    if (launch_clear_grid(ctx->B.D, 0, st) != hipSuccess) return fail(DEM_E_HIP);
    if (launch_drift_bin(ctx->B.D, 0, false, false, true, st) != hipSuccess) return fail(DEM_E_HIP);
  }
  if (force_launch(ctx, 0, false, false, kGridCurExact | kGridPrevExact, st) != DEM_OK) return fail(DEM_E_HIP);
  *out = ctx;
  return DEM_OK;
}

dem_status dem_step(dem_ctx *ctx, int32_t n_steps, void *stream) {
  if (!ctx || n_steps < 0) return DEM_E_ARG;
  if (ctx->poisoned) return ctx->poisoned;
  if (n_steps == 0) return DEM_OK;
  hipStream_t st = (hipStream_t)stream;
  if (ctx->dp.resort_every > 0 && ctx->since_sort >= ctx->dp.resort_every) {
    dem_status r = resort(ctx, st);
    if (r != DEM_OK) return r;
  }
  // the held fluid force may have changed since the last step: open the run
  // with a separate half kick + drift, then one kernel per step
  const long long s0 = ctx->s + 1;
  HIP_TRY(launch_drift_bin(ctx->B.D, s0, true, ctx->pending_src != nullptr, n_steps == 1, st));
  for (int i = 0; i < n_steps; ++i) {
    dem_status r = force_launch(ctx, s0 + i, true, i + 1 < n_steps, grid_mode(i + 1, n_steps), st);
    if (r != DEM_OK) return r;
  }
  ctx->s += n_steps;
  ctx->since_sort += n_steps;
  return DEM_OK;
}

// Smoothed void fraction of the current state into B.sx: element PCM values
// (fixed-point accumulators in B.eps_e), right-hand side, direct solve.
static dem_status smooth_solve(dem_ctx *ctx, hipStream_t st) {
  Buffers &B = ctx->B;
  HIP_TRY(launch_pcm_rhs(B.D, ctx->C, ctx->SO, ctx->s, B.eps_e, B.sb, st));
  HIP_TRY(launch_smooth_solve(ctx->SO, B.sb, B.sx, B.st1, B.st2, st));
  return DEM_OK;
}

dem_status cfd_dem_couple(dem_ctx *ctx, const double *u_nodes, const double *p_nodes,
                          double *eps_q, double *beta_q, double *fpf_q, double *elem_sums,
                          void *stream) {
  if (!ctx || !u_nodes || !p_nodes || !eps_q || !beta_q || !fpf_q) return DEM_E_ARG;
  if (ctx->poisoned) return ctx->poisoned;
  hipStream_t st = (hipStream_t)stream;
  if (ctx->C.smooth) {
    dem_status r = smooth_solve(ctx, st);
    if (r != DEM_OK) return r;
  }
  HIP_TRY(launch_couple(ctx->B.D, ctx->C, ctx->s, ctx->n_couple, u_nodes, p_nodes, eps_q, beta_q,
                        fpf_q, elem_sums, ctx->fp32, st));
  if (ctx->C.smooth) HIP_TRY(launch_eps_q_field(ctx->SO, ctx->C, ctx->B.sx, eps_q, st));
  ++ctx->n_couple;
  return DEM_OK;
}


dem_status dem_read_state(dem_ctx *ctx, double *x, double *v, double *omega, double *f_fp,
                          void *stream) {
  if (!ctx) return DEM_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const Dev &D = ctx->B.D;
  if (x) {
    k_scatter_pos<<<blocks(D.n, 256), 256, 0, st>>>(D.n, D.oid, D.pr[ctx->s & 1], x);
    HIP_TRY(hipGetLastError());
  }
  const double *src[4] = {nullptr, D.v, D.w, D.ffp};
  double *dst[4] = {nullptr, v, omega, f_fp};
  for (int i = 1; i < 4; ++i) {
    if (!dst[i]) continue;
    k_scatter3<<<blocks(D.n, 256), 256, 0, st>>>(D.n, D.oid, src[i], dst[i]);
    HIP_TRY(hipGetLastError());
  }
  return DEM_OK;
}

dem_status dem_read_forces(dem_ctx *ctx, double *F_c, double *T_c, void *stream) {
  if (!ctx) return DEM_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const Dev &D = ctx->B.D;
  if (F_c) k_scatter3<<<blocks(D.n, 256), 256, 0, st>>>(D.n, D.oid, D.Fc, F_c);
  if (T_c) k_scatter3<<<blocks(D.n, 256), 256, 0, st>>>(D.n, D.oid, D.Tc, T_c);
  HIP_TRY(hipGetLastError());
  return DEM_OK;
}

dem_status dem_kinetic_energy(dem_ctx *ctx, double *out, void *stream) {
  if (!ctx || !out) return DEM_E_ARG;
  if (ctx->poisoned) return ctx->poisoned;
  hipStream_t st = (hipStream_t)stream;
  const Dev &D = ctx->B.D;
  const int nb = blocks(D.n, 256);
  double *part = ctx->B.energy;
  k_energy_partials<<<nb, 256, 0, st>>>(D, part);
  k_energy_total<<<1, 64, 0, st>>>(nb, part, part + 2 * nb);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out, part + 2 * nb, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return DEM_OK;
}

dem_status dem_kinetic_energy_noalloc(dem_ctx *ctx, double *out, void *stream) {
  if (!ctx || !out) return DEM_E_ARG;
  if (ctx->poisoned) return ctx->poisoned;
  const Dev &D = ctx->B.D;
  const int nb = blocks(D.n, 256);
  if (nb > kEnergyScratchBlocks) return DEM_E_CAPACITY;
  double *part = nullptr;
  const dem_status r = scratch_of_current_device(&part);
  if (r != DEM_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  // every block writes its partials before the total reads them: nothing to clear
  k_energy_partials<<<nb, 256, 0, st>>>(D, part);
  k_energy_total<<<1, 64, 0, st>>>(nb, part, out);
  HIP_TRY(hipGetLastError());
  return DEM_OK;
}

dem_status dem_metrics(dem_ctx *ctx, const double *eps_q, double *out, void *stream) {
  if (!ctx || !out) return DEM_E_ARG;
  if (ctx->poisoned) return ctx->poisoned;
  hipStream_t st = (hipStream_t)stream;
  const Dev &D = ctx->B.D;
  const int nb = blocks(D.n, 256);
  const long long nqt = (long long)D.grid.n_elem * ctx->C.nq;
  const int nbq = eps_q ? (int)((nqt + 255) / 256) : 0;
  double *part = ctx->B.metrics;
  double *qpart = part + 6 * (size_t)nb;
  double *res = qpart + (nqt + 255) / 256;
  k_metrics_partials<<<nb, 256, 0, st>>>(D, (int)((ctx->s + 1) % 3), (int)(ctx->s & 1), part);
  if (nbq) {
    // Gauss-Legendre weights on [0, 1]: 1/2, 1/2 (two points); 5/18, 8/18, 5/18 (three)
    const double wa = ctx->C.nq1 == 2 ? 0.5 : 5.0 / 18.0, wb = ctx->C.nq1 == 2 ? 0.5 : 8.0 / 18.0;
    k_qsolid_partials<<<nbq, 256, 0, st>>>(eps_q, nqt, ctx->C.nq1, wa, wb, ctx->C.Ve, qpart);
  }
  k_metrics_total<<<1, 64, 0, st>>>(nb, part, nbq, qpart, res);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out, res, 7 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return DEM_OK;
}

dem_status dem_read_cells(dem_ctx *ctx, int32_t *elem, int32_t *cell, int32_t *k, void *stream) {
  if (!ctx) return DEM_E_ARG;
  const Dev &D = ctx->B.D;
  if (k)
    for (int a = 0; a < 3; ++a) k[a] = D.grid.k[a];
  if (elem || cell) {
    k_scatter_cells<<<blocks(D.n, 256), 256, 0, (hipStream_t)stream>>>(
        D.n, D.grid.kk, D.oid, D.cell[ctx->s % 3], elem, cell);
    HIP_TRY(hipGetLastError());
  }
  return DEM_OK;
}

dem_status dem_read_contacts(dem_ctx *ctx, int64_t *pairs, double *delta_t, int64_t cap,
                             int64_t *n_out, void *stream) {
  if (!ctx || !n_out || cap < 0 || (cap > 0 && (!pairs || !delta_t))) return DEM_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  Buffers &B = ctx->B;
  const Dev &D = B.D;
  const int n = D.n;
  int lb = 0;
  HIP_TRY(hipMemcpyAsync(&lb, D.lbuf + (ctx->s + 1) % 3, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  k_contact_count<<<blocks(n, 256), 256, 0, st>>>(D, lb, B.cnt64, nullptr);
  HIP_TRY(hipGetLastError());
  HIP_TRY(device_exclusive_scan<long long, long long>(n, B.cnt64, 0, B.off64, B.bsum, st));
  long long total = 0;
  const int nb = (n + kScanTile - 1) / kScanTile;
  HIP_TRY(hipMemcpyAsync(&total, B.bsum + nb, sizeof(long long), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *n_out = total;
  if (cap > 0) {
    k_contact_write<<<blocks(n, 256), 256, 0, st>>>(D, lb, B.off64, cap, (long long *)pairs, delta_t);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
  }
  return DEM_OK;
}

dem_status dem_poll(dem_ctx *ctx, int32_t *sticky_error, int64_t *n_contacts, void *stream) {
  if (!ctx) return DEM_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  Buffers &B = ctx->B;
  const Dev &D = B.D;
  HIP_TRY(hipMemsetAsync(B.scalars, 0, sizeof(unsigned long long), st));
  int lb = 0;
  HIP_TRY(hipMemcpyAsync(&lb, D.lbuf + (ctx->s + 1) % 3, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  k_contact_count<<<blocks(D.n, 256), 256, 0, st>>>(D, lb, B.cnt64, B.scalars);
  HIP_TRY(hipGetLastError());
  int bits = 0;
  unsigned long long total = 0;
  HIP_TRY(hipMemcpyAsync(&bits, D.err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&total, B.scalars, sizeof(total), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const dem_status e = err_to_status(bits);
  if (e != DEM_OK && ctx->poisoned == DEM_OK) ctx->poisoned = e;
  if (sticky_error) *sticky_error = ctx->poisoned;
  if (n_contacts) *n_contacts = (int64_t)total;
  return ctx->poisoned;
}

dem_status dem_kernel_timing(dem_ctx *ctx, int32_t enable) {
  if (!ctx) return DEM_E_ARG;
  ctx->timing = enable != 0;
  return DEM_OK;
}

dem_status dem_kernel_timing_read(dem_ctx *ctx, int64_t *launches, double *total_ms, void *stream) {
  if (!ctx) return DEM_E_ARG;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  double sum = 0.0;
  for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]));
    sum += ms;
  }
  if (launches) *launches = (int64_t)(ctx->ev_used / 2);
  if (total_ms) *total_ms = sum;
  ctx->ev_used = 0;
  return DEM_OK;
}

dem_status dem_destroy(dem_ctx *ctx) {
  if (!ctx || ctx->in_batch) return DEM_E_ARG;
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  delete ctx;
  return DEM_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
}  // extern "C"

struct dem_batch {
  // slots: the beds held (nullptr = free), their coupling buffers
  int n_slots = 0;
  long long max_particles = 0, max_elements = 0;
  bool couples = false;
  std::vector<dem_ctx *> slot;
  std::vector<CplIO> io_host;
  int held = 0;  // occupied slots
  long long held_particles = 0, held_elements = 0;
  // shared by every bed held (fixed while the batch is not empty)
  bool fp32 = false;
  int order = 2;
  int lanes = kForceLanes;
  int elem_threads = 128;  // threads per occupied element of the coupling step
  int maxn = 1;
  // launch layout, rebuilt when the slots change.  Beds are grouped by kernel
  // variant, each group with its own launches, so that a bed's arithmetic
  // never depends on the other beds: the force map holds the blocks of the
  // beds without rolling friction first (nb_force_plain of them), then those
  // of the beds with it; the coupling lists occupied elements per
  // element-kernel variant (mode_elems[m] elements of the beds in mode m)
  bool dirty = true;
  int nb_force_plain = 0;
  long long mode_elems[3] = {0, 0, 0};
  int nb_drift = 0, nb_force = 0, nb_class = 0;
  // device tables and maps (carved from the caller's workspace)
  Dev *tab = nullptr;
  Cpl *ctab = nullptr;
  CplIO *iot = nullptr;
  BedRun *run = nullptr;
  unsigned *map_drift = nullptr, *map_force = nullptr, *map_class = nullptr, *list = nullptr;
  long long cap_drift = 0, cap_force = 0, cap_class = 0;
  int *cnt = nullptr;
  // the counters hold the counts of a coupling step not yet followed by a run
  // of steps (whose last launch clears them)
  bool cnt_dirty = false;
  // pinned host staging of the maps, reused once its last upload is done
  unsigned *stage = nullptr;
  hipEvent_t stage_ev = nullptr;
  bool stage_pending = false;
  // graphs of a chunk: the coupling step, and g_steps DEM steps; graphs of
  // an older layout wait for their last replay before they are destroyed
  hipStream_t cap = nullptr;
  hipGraphExec_t g_cpl = nullptr;
  hipGraphExec_t g_step = nullptr;
  int g_steps = -1;
  // both in one graph, for the chunks with no re-sort due (a graph launch
  // costs the device a few microseconds of its own)
  hipGraphExec_t g_chunk = nullptr;
  int g_chunk_steps = -1;
  std::vector<std::pair<hipGraphExec_t, hipEvent_t>> stale;
};

namespace {

int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Capacity of the maps and lists of a batch of these limits (force blocks
// sized for four lanes per particle, the most a bed may use).
struct SlotCaps {
  long long drift, force, cls, elems;
};
SlotCaps slot_caps(const dem_batch_limits &L) {
  SlotCaps c;
  c.drift = L.max_particles / 256 + L.slots;
  c.force = L.max_particles * 4 / kForceBlock + L.slots;
  c.cls = L.couples ? L.max_elements / couple_class_elems_per_block() + L.slots : 0;
  c.elems = L.couples ? L.max_elements : 0;
  return c;
}

bool limits_ok(const dem_batch_limits *L) {
  return L && L->slots >= 1 && L->slots <= kMaxBeds && L->max_particles >= 1 &&
         L->max_particles <= 0x7ffffff0LL && L->max_elements >= 0 && L->max_elements <= 0x7ffffff0LL &&
         (L->couples == 0 || L->couples == 1);
}

size_t batch_carve(const dem_batch_limits &L, char *base, dem_batch *B) {
  const SlotCaps k = slot_caps(L);
  Carver c{base};
  Dev *tab = c.take<Dev>((size_t)L.slots);
  Cpl *ctab = c.take<Cpl>((size_t)L.slots);
  CplIO *iot = c.take<CplIO>((size_t)L.slots);
  BedRun *run = c.take<BedRun>((size_t)L.slots);
  unsigned *md = c.take<unsigned>((size_t)k.drift);
  unsigned *mf = c.take<unsigned>((size_t)k.force);
  unsigned *mc = c.take<unsigned>((size_t)(k.cls > 0 ? k.cls : 1));
  unsigned *list = c.take<unsigned>((size_t)(k.elems > 0 ? k.elems : 1));
  int *cnt = c.take<int>(64);
  if (B) {
    B->tab = tab;
    B->ctab = ctab;
    B->iot = iot;
    B->run = run;
    B->map_drift = md;
    B->map_force = mf;
    B->map_class = mc;
    B->list = list;
    B->cnt = cnt;
    B->cap_drift = k.drift;
    B->cap_force = k.force;
    B->cap_class = k.cls;
  }
  return c.off + kAlign;
}

void fill_map(unsigned *m, long long &at, int bed, int blocks) {
  for (int k = 0; k < blocks; ++k) m[at++] = ((unsigned)bed << kBedShift) | (unsigned)k;
}

// Graphs of the old layout are destroyed once their last replay has run.
void retire_graphs(dem_batch *B, hipStream_t st) {
  for (hipGraphExec_t *g : {&B->g_cpl, &B->g_step, &B->g_chunk}) {
    if (!*g) continue;
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess && hipEventRecord(e, st) == hipSuccess) {
      B->stale.emplace_back(*g, e);
    } else {
      if (e) (void)hipEventDestroy(e);
      (void)hipStreamSynchronize(st);
      (void)hipGraphExecDestroy(*g);
    }
    *g = nullptr;
  }
  B->g_steps = -1;
  B->g_chunk_steps = -1;
  for (size_t i = 0; i < B->stale.size();) {
    if (hipEventQuery(B->stale[i].second) == hipSuccess) {
      (void)hipGraphExecDestroy(B->stale[i].first);
      (void)hipEventDestroy(B->stale[i].second);
      B->stale[i] = B->stale.back();
      B->stale.pop_back();
    } else {
      ++i;
    }
  }
}

// Rebuilds the launch layout from the held beds and uploads the maps (from
// pinned staging, stream-ordered: launches already enqueued keep reading the
// maps they were enqueued with).
dem_status batch_layout(dem_batch *B, hipStream_t st) {
  if (!B->dirty) return DEM_OK;
  if (B->stage_pending) {
    HIP_TRY(hipEventSynchronize(B->stage_ev));  // the last upload has left the staging
    B->stage_pending = false;
  }
  unsigned *md = B->stage;
  unsigned *mf = md + B->cap_drift;
  unsigned *mc = mf + B->cap_force;
  long long nd = 0, nf = 0, nc = 0;
  B->mode_elems[0] = B->mode_elems[1] = B->mode_elems[2] = 0;
  B->maxn = 1;
  for (int pass = 0; pass < 2; ++pass)  // force blocks: beds without rolling friction first
    for (int b = 0; b < B->n_slots; ++b) {
      const dem_ctx *ctx = B->slot[b];
      if (!ctx) continue;
      const bool roll = ctx->B.D.pp.mu_r > 0.0 || ctx->B.D.pw.mu_r > 0.0;
      if (roll != (pass == 1)) continue;
      fill_map(mf, nf, b, ceil_div((long long)ctx->S.n * ctx->S.lanes, kForceBlock));
    }
  B->nb_force_plain = 0;
  for (int b = 0; b < B->n_slots; ++b) {
    const dem_ctx *ctx = B->slot[b];
    if (!ctx) continue;
    if (!(ctx->B.D.pp.mu_r > 0.0 || ctx->B.D.pw.mu_r > 0.0))
      B->nb_force_plain += ceil_div((long long)ctx->S.n * ctx->S.lanes, kForceBlock);
    fill_map(md, nd, b, ceil_div(ctx->S.n, 256));
    if (B->couples) {
      fill_map(mc, nc, b, ceil_div(ctx->S.grid.n_elem, couple_class_elems_per_block()));
      B->mode_elems[cpl_mode_of(ctx->C.drag, ctx->C.shear || ctx->C.smooth)] += ctx->S.grid.n_elem;
    }
    if (ctx->S.maxn > B->maxn) B->maxn = ctx->S.maxn;
  }
  B->nb_drift = (int)nd;
  B->nb_force = (int)nf;
  B->nb_class = (int)nc;
  if (nd) HIP_TRY(hipMemcpyAsync(B->map_drift, md, sizeof(unsigned) * nd, hipMemcpyHostToDevice, st));
  if (nf) HIP_TRY(hipMemcpyAsync(B->map_force, mf, sizeof(unsigned) * nf, hipMemcpyHostToDevice, st));
  if (nc) HIP_TRY(hipMemcpyAsync(B->map_class, mc, sizeof(unsigned) * nc, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(B->stage_ev, st));
  B->stage_pending = true;
  retire_graphs(B, st);
  B->dirty = false;
  return DEM_OK;
}

// Whether some bed's re-sort is due before its next steps.
bool batch_resort_due(const dem_batch *B) {
  for (const dem_ctx *ctx : B->slot)
    if (ctx && ctx->dp.resort_every > 0 && ctx->since_sort >= ctx->dp.resort_every) return true;
  return false;
}

// Re-sorts the beds whose re-sort is due and refreshes their table entries.
dem_status batch_resorts(dem_batch *B, hipStream_t st) {
  for (int b = 0; b < B->n_slots; ++b) {
    dem_ctx *ctx = B->slot[b];
    if (ctx && ctx->dp.resort_every > 0 && ctx->since_sort >= ctx->dp.resort_every) {
      dem_status r = resort(ctx, st);
      if (r != DEM_OK) return r;
      HIP_TRY(launch_batch_set_bed(B->tab, B->run, b, ctx->B.D, ctx->s, ctx->pending_src, st));
    }
  }
  return DEM_OK;
}

// Enqueues n steps of every bed (no re-sorts).
dem_status batch_enqueue_steps(dem_batch *B, int n, hipStream_t st) {
  HIP_TRY(launch_drift_bin_batch(B->tab, B->run, B->map_drift, B->nb_drift, n, st));
  const int nb_roll = B->nb_force - B->nb_force_plain;
  for (int i = 1; i <= n; ++i) {
    if (B->nb_force_plain > 0)
      HIP_TRY(launch_force_kick_batch(B->tab, B->run, B->map_force, B->nb_force_plain, i, n, B->fp32,
                                      B->maxn, B->lanes, false, st));
    if (nb_roll > 0)
      HIP_TRY(launch_force_kick_batch(B->tab, B->run, B->map_force + B->nb_force_plain, nb_roll, i, n,
                                      B->fp32, B->maxn, B->lanes, true, st));
  }
  HIP_TRY(launch_batch_advance(B->run, B->n_slots, n, B->cnt, st));
  return DEM_OK;
}

dem_status batch_enqueue_couple(dem_batch *B, hipStream_t st) {
  // beds with the smoothed void fraction: their field first (per bed: each
  // has its own mesh and transforms), their quadrature-point values after the
  // shared launches, as a single bed's coupling step orders them
  for (int b = 0; b < B->n_slots; ++b) {
    dem_ctx *ctx = B->slot[b];
    if (!ctx || !ctx->C.smooth) continue;
    HIP_TRY(launch_pcm_rhs_run(B->tab, ctx->S.grid.n_elem, ctx->C, ctx->SO, B->run, b, ctx->B.eps_e,
                               ctx->B.sb, st));
    HIP_TRY(launch_smooth_solve(ctx->SO, ctx->B.sb, ctx->B.sx, ctx->B.st1, ctx->B.st2, st));
  }
  HIP_TRY(launch_couple_batch(B->tab, B->ctab, B->iot, B->run, B->map_class, B->nb_class, B->cnt, B->list,
                              B->mode_elems, B->order, B->fp32, B->elem_threads, st));
  for (int b = 0; b < B->n_slots; ++b) {
    dem_ctx *ctx = B->slot[b];
    if (ctx && ctx->C.smooth) HIP_TRY(launch_eps_q_field(ctx->SO, ctx->C, ctx->B.sx, B->io_host[b].eps_q, st));
  }
  return DEM_OK;
}

void batch_mirror_steps(dem_batch *B, int n) {
  for (dem_ctx *ctx : B->slot) {
    if (!ctx) continue;
    ctx->s += n;
    ctx->since_sort += n;
    ctx->pending_src = nullptr;
  }
}

dem_status batch_poisoned(const dem_batch *B) {
  for (const dem_ctx *ctx : B->slot)
    if (ctx && ctx->poisoned) return ctx->poisoned;
  return DEM_OK;
}

// Whether bed ctx may join the beds the batch holds (same precision, lanes
// and threads per element; for coupling, the same velocity order), and fits
// the block-map encoding.
dem_status bed_fits(const dem_batch *B, const dem_ctx *ctx) {
  const long long n = ctx->S.n;
  const int bd = ceil_div(n, 256), bf = ceil_div(n * ctx->S.lanes, kForceBlock);
  const int ne = ctx->S.grid.n_elem;
  if (bd > (int)kBlockMask || bf > (int)kBlockMask) return DEM_E_UNSUPPORTED;
  if (B->couples && (ne > (int)kBlockMask || ceil_div(ne, couple_class_elems_per_block()) > (int)kBlockMask))
    return DEM_E_UNSUPPORTED;
  if (B->held > 0) {
    if (ctx->fp32 != B->fp32 || ctx->S.lanes != B->lanes || ctx->C.elem_threads != B->elem_threads)
      return DEM_E_UNSUPPORTED;
    if (B->couples && ctx->cp.order != B->order) return DEM_E_UNSUPPORTED;
  }
  if (B->held_particles + n > B->max_particles) return DEM_E_CAPACITY;
  if (B->couples && B->held_elements + ne > B->max_elements) return DEM_E_CAPACITY;
  return DEM_OK;
}

}  // namespace

extern "C" {

size_t dem_batch_slots_workspace_bytes(const dem_batch_limits *limits) {
  if (!limits_ok(limits)) return 0;
  return batch_carve(*limits, nullptr, nullptr);
}

dem_status dem_batch_create_slots(const dem_batch_limits *limits, void *workspace, size_t ws_bytes, void *stream,
                                  dem_batch **out) {
  if (!out) return DEM_E_ARG;
  *out = nullptr;
  if (!limits_ok(limits)) return DEM_E_ARG;
  const size_t need = batch_carve(*limits, nullptr, nullptr);
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || ws_bytes < need) return DEM_E_WORKSPACE;
  dem_batch *B = new (std::nothrow) dem_batch();
  if (!B) return DEM_E_ARG;
  batch_carve(*limits, (char *)workspace, B);
  B->n_slots = limits->slots;
  B->max_particles = limits->max_particles;
  B->max_elements = limits->max_elements;
  B->couples = limits->couples != 0;
  B->slot.assign((size_t)B->n_slots, nullptr);
  B->io_host.assign((size_t)B->n_slots, CplIO{});
  hipStream_t st = (hipStream_t)stream;
  const size_t stage_words = (size_t)(B->cap_drift + B->cap_force + B->cap_class);
  bool ok = hipHostMalloc((void **)&B->stage, sizeof(unsigned) * stage_words, hipHostMallocDefault) == hipSuccess &&
            hipEventCreateWithFlags(&B->stage_ev, hipEventDisableTiming) == hipSuccess &&
            hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) == hipSuccess &&
            hipMemsetAsync(B->cnt, 0, sizeof(int) * 64, st) == hipSuccess;
  if (!ok) {
    dem_batch_destroy(B);
    return DEM_E_HIP;
  }
  *out = B;
  return DEM_OK;
}

dem_status dem_batch_admit(dem_batch *B, int32_t slot, dem_ctx *bed, const double *u_nodes, const double *p_nodes,
                           double *eps_q, double *beta_q, double *fpf_q, double *elem_sums, void *stream) {
  if (!B || !bed || slot < 0 || slot >= B->n_slots || B->slot[slot] || bed->in_batch) return DEM_E_ARG;
  if (B->couples && (!u_nodes || !p_nodes || !eps_q || !beta_q || !fpf_q)) return DEM_E_ARG;
  if (bed->poisoned) return bed->poisoned;
  const dem_status f = bed_fits(B, bed);
  if (f != DEM_OK) return f;
  hipStream_t st = (hipStream_t)stream;
  const CplIO io = B->couples ? CplIO{u_nodes, p_nodes, eps_q, beta_q, fpf_q, elem_sums} : CplIO{};
  HIP_TRY(launch_batch_set_bed(B->tab, B->run, slot, bed->B.D, bed->s, bed->pending_src, st));
  HIP_TRY(launch_batch_set_cpl(B->ctab, B->iot, slot, bed->C, io, st));
  if (B->held == 0) {
    B->fp32 = bed->fp32;
    B->lanes = bed->S.lanes;
    B->elem_threads = bed->C.elem_threads;
    B->order = bed->cp.order;
  }
  B->slot[slot] = bed;
  B->io_host[slot] = io;
  ++B->held;
  B->held_particles += bed->S.n;
  B->held_elements += bed->S.grid.n_elem;
  ++bed->in_batch;
  B->dirty = true;
  return DEM_OK;
}

dem_status dem_batch_retire(dem_batch *B, int32_t slot) {
  if (!B || slot < 0 || slot >= B->n_slots || !B->slot[slot]) return DEM_E_ARG;
  dem_ctx *bed = B->slot[slot];
  B->slot[slot] = nullptr;
  B->io_host[slot] = CplIO{};
  --B->held;
  B->held_particles -= bed->S.n;
  B->held_elements -= bed->S.grid.n_elem;
  --bed->in_batch;
  B->dirty = true;
  return DEM_OK;
}

size_t dem_batch_workspace_bytes(int32_t n_beds, dem_ctx *const *beds) {
  if (n_beds < 1 || n_beds > kMaxBeds || !beds) return 0;
  dem_batch_limits L{n_beds, 1, 0, 0};
  for (int b = 0; b < n_beds; ++b) {
    if (!beds[b]) return 0;
    L.max_particles += beds[b]->S.n;
    L.max_elements += beds[b]->S.grid.n_elem;
  }
  return limits_ok(&L) ? batch_carve(L, nullptr, nullptr) : 0;
}

dem_status dem_batch_create(int32_t n_beds, dem_ctx *const *beds, const double *const *u_nodes,
                            const double *const *p_nodes, double *const *eps_q,
                            double *const *beta_q, double *const *fpf_q,
                            double *const *elem_sums, void *workspace, size_t ws_bytes,
                            void *stream, dem_batch **out) {
  if (!out) return DEM_E_ARG;
  *out = nullptr;
  if (n_beds < 1 || n_beds > kMaxBeds || !beds) return DEM_E_ARG;
  const bool couples = u_nodes != nullptr;
  if (couples && (!p_nodes || !eps_q || !beta_q || !fpf_q)) return DEM_E_ARG;
  dem_batch_limits L{n_beds, couples ? 1 : 0, 0, 0};
  for (int b = 0; b < n_beds; ++b) {
    if (!beds[b]) return DEM_E_ARG;
    for (int j = 0; j < b; ++j)
      if (beds[j] == beds[b]) return DEM_E_ARG;
    if (beds[b]->poisoned) return beds[b]->poisoned;
    L.max_particles += beds[b]->S.n;
    L.max_elements += beds[b]->S.grid.n_elem;
  }
  if (!limits_ok(&L)) return DEM_E_UNSUPPORTED;
  dem_batch *B = nullptr;
  dem_status r = dem_batch_create_slots(&L, workspace, ws_bytes, stream, &B);
  if (r != DEM_OK) return r;
  for (int b = 0; b < n_beds && r == DEM_OK; ++b)
    r = couples ? dem_batch_admit(B, b, beds[b], u_nodes[b], p_nodes[b], eps_q[b], beta_q[b], fpf_q[b],
                                  elem_sums ? elem_sums[b] : nullptr, stream)
                : dem_batch_admit(B, b, beds[b], nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, stream);
  if (r == DEM_OK) r = batch_layout(B, (hipStream_t)stream);
  if (r == DEM_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) r = DEM_E_HIP;
  if (r != DEM_OK) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    dem_batch_destroy(B);
    return r;
  }
  *out = B;
  return DEM_OK;
}

dem_status dem_batch_step(dem_batch *B, int32_t n_steps, void *stream) {
  if (!B || n_steps < 0) return DEM_E_ARG;
  dem_status r = batch_poisoned(B);
  if (r != DEM_OK) return r;
  if (n_steps == 0 || B->held == 0) return DEM_OK;
  hipStream_t st = (hipStream_t)stream;
  r = batch_layout(B, st);
  if (r != DEM_OK) return r;
  r = batch_resorts(B, st);
  if (r != DEM_OK) return r;
  r = batch_enqueue_steps(B, n_steps, st);
  if (r != DEM_OK) return r;
  B->cnt_dirty = false;
  batch_mirror_steps(B, n_steps);
  return DEM_OK;
}

dem_status dem_batch_couple(dem_batch *B, void *stream) {
  if (!B) return DEM_E_ARG;
  if (!B->couples) return DEM_E_ARG;
  dem_status r = batch_poisoned(B);
  if (r != DEM_OK) return r;
  if (B->held == 0) return DEM_OK;
  hipStream_t st = (hipStream_t)stream;
  r = batch_layout(B, st);
  if (r != DEM_OK) return r;
  if (B->cnt_dirty) HIP_TRY(launch_reset_count(B->cnt, st));
  r = batch_enqueue_couple(B, st);
  B->cnt_dirty = r == DEM_OK;
  return r;
}

dem_status dem_batch_run(dem_batch *B, int32_t n_chunks, int32_t steps_per_chunk, int32_t couple,
                         void *stream) {
  if (!B || n_chunks < 0 || steps_per_chunk < 0 || (couple && !B->couples)) return DEM_E_ARG;
  dem_status r = batch_poisoned(B);
  if (r != DEM_OK) return r;
  if (n_chunks == 0 || (steps_per_chunk == 0 && !couple) || B->held == 0) return DEM_OK;
  hipStream_t st = (hipStream_t)stream;
  r = batch_layout(B, st);
  if (r != DEM_OK) return r;
  // capture what this call needs and is not captured yet
  auto capture = [&](bool cpl, int steps, hipGraphExec_t *exec) -> dem_status {
    HIP_TRY(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    dem_status cr = cpl ? batch_enqueue_couple(B, B->cap) : DEM_OK;
    if (cr == DEM_OK && steps > 0) cr = batch_enqueue_steps(B, steps, B->cap);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(B->cap, &g);
    if (cr != DEM_OK || ec != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return cr != DEM_OK ? cr : DEM_E_HIP;
    }
    const hipError_t ei = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      *exec = nullptr;
      return DEM_E_HIP;
    }
    return DEM_OK;
  };
  if (couple && !B->g_cpl) {
    r = capture(true, 0, &B->g_cpl);
    if (r != DEM_OK) return r;
  }
  if (steps_per_chunk > 0 && (!B->g_step || B->g_steps != steps_per_chunk)) {
    if (B->g_step) {
      HIP_TRY(hipStreamSynchronize(st));  // its replays are done
      HIP_TRY(hipGraphExecDestroy(B->g_step));
      B->g_step = nullptr;
    }
    r = capture(false, steps_per_chunk, &B->g_step);
    if (r != DEM_OK) return r;
    B->g_steps = steps_per_chunk;
  }
  if (couple && steps_per_chunk > 0 && (!B->g_chunk || B->g_chunk_steps != steps_per_chunk)) {
    if (B->g_chunk) {
      HIP_TRY(hipStreamSynchronize(st));
      HIP_TRY(hipGraphExecDestroy(B->g_chunk));
      B->g_chunk = nullptr;
    }
    r = capture(true, steps_per_chunk, &B->g_chunk);
    if (r != DEM_OK) return r;
    B->g_chunk_steps = steps_per_chunk;
  }
  // per chunk, the order of dem_batch_couple + dem_batch_step: couple, due
  // re-sorts, steps
  for (int c = 0; c < n_chunks; ++c) {
    if (couple && steps_per_chunk > 0 && !batch_resort_due(B)) {
      if (B->cnt_dirty) HIP_TRY(launch_reset_count(B->cnt, st));
      HIP_TRY(hipGraphLaunch(B->g_chunk, st));
      B->cnt_dirty = false;
      batch_mirror_steps(B, steps_per_chunk);
      continue;
    }
    if (couple) {
      if (B->cnt_dirty) HIP_TRY(launch_reset_count(B->cnt, st));
      HIP_TRY(hipGraphLaunch(B->g_cpl, st));
      B->cnt_dirty = true;
    }
    if (steps_per_chunk > 0) {
      r = batch_resorts(B, st);
      if (r != DEM_OK) return r;
      HIP_TRY(hipGraphLaunch(B->g_step, st));
      B->cnt_dirty = false;
      batch_mirror_steps(B, steps_per_chunk);
    }
  }
  return DEM_OK;
}

dem_status dem_batch_destroy(dem_batch *B) {
  if (!B) return DEM_E_ARG;
  for (dem_ctx *ctx : B->slot)
    if (ctx) --ctx->in_batch;
  for (auto &g : B->stale) {
    (void)hipEventSynchronize(g.second);
    (void)hipGraphExecDestroy(g.first);
    (void)hipEventDestroy(g.second);
  }
  if (B->g_cpl) (void)hipGraphExecDestroy(B->g_cpl);
  if (B->g_step) (void)hipGraphExecDestroy(B->g_step);
  if (B->g_chunk) (void)hipGraphExecDestroy(B->g_chunk);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  if (B->stage_ev) {
    (void)hipEventSynchronize(B->stage_ev);
    (void)hipEventDestroy(B->stage_ev);
  }
  if (B->stage) (void)hipHostFree(B->stage);
  delete B;
  return DEM_OK;
}

const char *dem_status_string(dem_status s) {
  switch (s) {
    case DEM_OK: return "ok";
    case DEM_E_ARG: return "invalid argument";
    case DEM_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case DEM_E_HIP: return "HIP runtime error";
    case DEM_E_DOMAIN: return "particle outside the box";
    case DEM_E_CAPACITY: return "cell or contact capacity exceeded";
    case DEM_E_NAN: return "NaN in the particle state";
    case DEM_E_UNSUPPORTED: return "unsupported option";
    case DEM_E_ABI: return "ABI version mismatch";
    default: return "unknown status";
  }
}

}  // extern "C"
