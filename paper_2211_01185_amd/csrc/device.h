// device.h -- device-side data layout and small helpers shared by the HIP
// kernels of libcfddem (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cfddem {

constexpr int kMaxNeighbors = 64;  // bound of dem_params.max_neighbors (one 64-bit mask)
// Threads per block of the contact-force kernel: one wavefront.  Against 128
// and 256 threads (same registers, four wavefronts per SIMD): fluidized and
// packed 100k beds about 1 % faster, 500k spouted bed 3 %, 64-bed ensemble
// 0.302 -> 0.294 ms per step (finer blocks give each XCD's contiguous ranges
// and the work of unequal beds a finer grain).
constexpr int kForceBlock = 64;
constexpr int kForceLanes = 2;     // default lanes sharing one particle in the contact-force kernel
constexpr int kElemMaxParticles = 1024;  // particles one coupling wave can hold
constexpr int kWalls = 6;          // partner codes 0..5 are the box faces

// sticky device error bits
enum : int { kErrDomain = 1, kErrCapacity = 2, kErrNan = 4 };
// word offsets in the int block at err: [0] error bits, [16..18] broad-search
// flags, [32..34] list buffer, [48..49] occupied-element counts by call parity
enum : int { kFlagWord = 16, kLbufWord = 32, kOccWord = 48 };

// Four doubles as a native vector (32-byte aligned): loads and stores of a
// record are 16-byte vector accesses through pointers of any address space.
typedef double dvec4 __attribute__((ext_vector_type(4)));

struct Material {
  double Ye;        // effective Young's modulus
  double Ge;        // effective shear modulus
  double eta_coef;  // -2 sqrt(5/6) beta(e)  (>= 0)
  double mu;        // Coulomb coefficient
  double mu_r;      // rolling friction coefficient (0: no rolling torque)
};

// Structured grid: mesh elements split into k[a] DEM cells per axis.
struct Grid {
  double lo[3], hi[3];
  double he[3];      // element size
  double inv_he[3];  // n_el / (hi - lo)
  double inv_hc[3];  // (k n_el) / (hi - lo)
  int n_el[3];
  int k[3];
  int kk;            // k0 k1 k2: cells per element
  int gc[3];         // cells per axis, k n_el
  int n_elem;        // n_el0 n_el1 n_el2
  int ncells;        // n_elem kk
};

// Everything a DEM kernel needs, passed by value.  Arrays are indexed by the
// internal (sorted) particle index; vectors are component-major (c*n + k).
// Step s keeps its position and half-step velocity records in buffer s&1 and its
// cell grid counts in buffer s%3, so that one kernel can read step s while it
// prepares step s+1 and clears what step s-1 left behind.
struct Dev {
  int n;
  int cap;    // slots per cell
  int maxn;   // neighbour-list entries per particle
  double dt;
  double g[3];
  double skin;        // neighbour-list skin
  double trig2;       // squared displacement that triggers a new broad search
  Material pp, pw;
  Grid grid;
  // Per-step records, by step parity, one 32-byte record per particle so
  // that a partner's state is a few 16-byte loads from one address each:
  dvec4 *pr[2];          // (x, y, z, R): position x_s and radius
  dvec4 *vm[2];          // (vx, vy, vz, m): half-step velocity of step s and mass
  dvec4 *ws[2];          // (wx, wy, wz, 0): half-step angular velocity of step s
  double *v, *w;         // boundary velocities (end of the last step)
  double *Fc, *Tc;       // stored contact force / torque
  double *ffp;           // held fluid force
  double *rad, *mass;
  double *xb;            // positions at the last broad search
  int *oid;              // original ID of each internal index
  int *cell[3];          // cell of x_s, by step mod 3
  int *cnt[3];           // particles per cell, by step mod 3
  int *slot[2];          // ncells x cap particle indices, by step parity
  int *flag;             // [3] broad search requested, by step mod 3
  int *lbuf;             // [3] neighbour-list buffer in use, by step mod 3
  // neighbour lists (buffer lbuf): entries sorted by partner original ID
  int *ln[2];                    // entries per particle
  unsigned long long *nbr[2];    // maxn x n: (partner oid << 32) | partner index
  unsigned long long *hmask[2];  // bit t: entry t touched at the last evaluation
  double *hdt[2];                // maxn x n tangential overlaps of the entries (hist_at)
  unsigned char *wmask;          // bit w: wall w touched at the last evaluation
  double *whdt;                  // 6 x n tangential overlaps against the walls (hist_at)
  // Re-sort epoch: the particles of cell c were given the sorted indices
  // start[c] .. start[c] + base[c] - 1 at the last re-sort.  Inside a run of
  // steps a cell grid may list them implicitly: such a grid counts (and slots)
  // only the particles away from their home cell, and the broad search takes
  // the home range of each cell besides its slots.
  int *home;             // n: cell at the last re-sort (-1: no re-sort yet)
  int *base;             // ncells: particles sorted into each cell (at most cap)
  int *start;            // ncells: sorted index of each cell's first particle
  int *occ;              // mesh elements holding particles (coupling step)
  int *err;              // sticky error bits
};

// First of the three components of the tangential overlap of entry (or wall)
// t of particle a: the components of one contact are adjacent, so that a
// contact's history is one line, read and written together.
__host__ __device__ inline size_t hist_at(int t, int n, int a) { return ((size_t)t * n + a) * 3; }

// Kind of the cell grids around one step (bits of a launch argument): a
// grid lists every particle in its slots (exact) or only the particles away
// from their home cell.  The last step of a run bins exactly, so that
// everything read between runs (coupling, smoothing, re-sort) sees exact grids.
enum : int {
  kGridCurExact = 1,   // the grid of step s
  kGridNextExact = 2,  // the grid of step s + 1 (binned by this launch)
  kGridPrevExact = 4,  // the grid of step s - 1 (cleared by this launch)
};
__host__ __device__ inline int grid_mode(int i, int n) {
  return (i == n ? kGridCurExact : 0) | (i + 1 == n ? kGridNextExact : 0) | (i == 1 ? kGridPrevExact : 0);
}

// Batched launches: many independent beds in one launch.  Each block of a
// batched kernel looks up (bed << kBedShift) | block-of-the-bed in a block
// map, and the bed's Dev, Cpl, run state and coupling buffers in device
// tables indexed by bed.
constexpr int kBedShift = 20;
constexpr unsigned kBlockMask = (1u << kBedShift) - 1u;
constexpr int kMaxBeds = 4096;

// Run state of one bed of a batch, advanced on the device.
struct BedRun {
  long long s;     // index of the last completed step
  const int *src;  // after a re-sort: index each particle had when its list was built
};

// Occupied-element lists of a batched coupling step, one per element-kernel
// variant (mode 0: Di Felice, 1: other closures, 2: shear force): region m
// starts at off[m] of the list, its length is counted in word m.
struct ModeLists {
  long long off[3];
};

// Element-kernel variant of a bed's coupling step: 2 for the shear force or
// the smoothed void fraction, 1 for a closure other than Di Felice, else 0.
__host__ __device__ inline int cpl_mode_of(int drag, int extended) { return extended ? 2 : (drag != 0 ? 1 : 0); }

// Solver of the smoothed void fraction (smooth_kernels.hip): the global
// matrix M + L^2 K of the velocity space, a Kronecker sum of the 1D mass and
// stiffness matrices of each axis, diagonalized by their generalized
// eigenvectors.
struct SmoothOp {
  int order;
  int nn[3];     // velocity nodes per axis
  int n_el[3];
  long nv;       // velocity nodes
  double L2;     // smoothing length squared
  const double *V[3], *Vt[3];  // per axis: eigenvectors (columns) and their transpose, nn x nn
  const double *lam[3];        // per axis: eigenvalues
  double load[3][3];           // integral of local basis l over an element of axis a
};

// Coupling buffers of one bed of a batch.
struct CplIO {
  const double *U, *P;
  double *eps_q, *beta_q, *fpf_q, *esums;
};

// Coupling constants.
struct Cpl {
  int order;        // 1 or 2
  int nq1;          // quadrature points per axis (order + 1)
  int nq;           // per element
  int nvx, nvy;     // velocity node lattice (x, y extents)
  int npx, npy;     // pressure node lattice
  double rho_f, mu_f, eps_min;
  int model;
  int drag;           // closure (DEM_DRAG_* without the flag bits)
  int beta_over_eps;  // 1: beta divided by the fluid fraction
  int shear;          // 1: shear force -V_p div(tau) added to the particle force
  int smooth;         // 1: the closure sees the smoothed void-fraction field
  const double *eps_nodes;  // that field at the velocity nodes (smooth = 1)
  int elem_threads;   // threads per occupied element in the coupling step: 64 or 128
  double Ve;        // element volume
  double Lq[3][3];  // Lq[a][i]: 1D velocity basis a at Gauss point i
  double Lq1[2][3]; // 1D Q1 basis at Gauss point i (unused for order 2)
};

// Pointers typed as global memory: loads and stores through them are global
// instructions (with an SGPR base where the address allows), whereas a
// generic pointer read from device memory (a batch table) would give FLAT
// instructions, which also hold up every wait for scalar loads.
template <typename T>
using gptr = T __attribute__((address_space(1))) *;
template <typename T>
__device__ __forceinline__ gptr<T> glb(T *p) {
  return (gptr<T>)p;
}

// Buffer i of a double- or triple-buffered array, with constant indices only
// (so that a Dev copied into registers stays in registers).
template <typename T>
__device__ __forceinline__ T *sel(T *const (&a)[2], int i) {
  return i ? a[1] : a[0];
}
template <typename T>
__device__ __forceinline__ T *sel(T *const (&a)[3], int i) {
  return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]);
}
template <typename T, int K>
__device__ __forceinline__ gptr<T> gsel(T *const (&a)[K], int i) {
  return glb(sel(a, i));
}

__device__ inline int floor_clamp(double t, int n) {
  double f = floor(t);
  if (!(f >= 0.0)) return 0;
  if (f > (double)(n - 1)) return n - 1;
  return (int)f;
}

// Hierarchical binning, evaluated without FMA contraction so that the indices
// are a pure function of the IEEE operations written here.
__device__ inline void bin_point(const Grid &G, const double xp[3], int &elem, int &cell,
                                 bool &inside) {
#pragma clang fp contract(off)
  int e[3], s[3];
  inside = true;
  for (int a = 0; a < 3; ++a) {
    const double xa = xp[a];
    if (!(xa >= G.lo[a] && xa <= G.hi[a])) inside = false;
    e[a] = floor_clamp((xa - G.lo[a]) * G.inv_he[a], G.n_el[a]);
    const double origin = G.lo[a] + (double)e[a] * G.he[a];
    s[a] = floor_clamp((xa - origin) * G.inv_hc[a], G.k[a]);
  }
  elem = (e[2] * G.n_el[1] + e[1]) * G.n_el[0] + e[0];
  cell = elem * G.kk + (s[2] * G.k[1] + s[1]) * G.k[0] + s[0];
}

// Fine-search predicate (R_i+R_j)^2 - (dx^2+dy^2+dz^2) > 0, no contraction.
__device__ inline bool touching(double xi0, double xi1, double xi2, double xj0, double xj1,
                                double xj2, double ri, double rj) {
#pragma clang fp contract(off)
  const double dx = xj0 - xi0, dy = xj1 - xi1, dz = xj2 - xi2;
  const double rs = ri + rj;
  const double d2 = dx * dx + dy * dy + dz * dz;
  return rs * rs - d2 > 0.0;
}

}  // namespace cfddem
