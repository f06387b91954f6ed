/*
 * cfddem.h -- C ABI of the MI355X (gfx950) particle-side hot path of
 * unresolved CFD-DEM (El Geitani, Golshan & Blais, "Towards High-Order
 * CFD-DEM: Development and Validation", arXiv 2211.01185).
 *
 * One DEM step (Section 2.2): cell-list broad search, fine contact search,
 * Hertz-Mindlin nonlinear spring-dashpot normal and tangential forces
 * (Table "tab:viscoelastic" and the contact-force equation) with a Coulomb
 * limit, velocity-Verlet integration of Eqs. "newton_law" and
 * "angular_momentum".  One coupling step (Section 2.3): particle-centroid
 * void fraction (Eq. "void_fraction") at the quadrature points of a given
 * Q1/Q2 hex mesh, drag (Eq. "drag" and the per-particle drag expression,
 * with the Di Felice, Dallavalle, Rong, Koch-Hill, Beetstra or Gidaspow
 * closure), buoyancy and pressure-gradient forces on the particles, and the
 * drag (plus, for model B, the pressure-gradient force) reduced back to the
 * quadrature points (Eqs. "fa" / "fb").
 *
 * Conventions for every entry point
 *  - SI units; FP64 in and out.
 *  - Per-particle vectors are component-major: x[c*n + i], c = 0,1,2.
 *  - Particle i is the i-th particle given to dem_create ("original ID").
 *    Every output is in original-ID order; the library's internal order
 *    (re-sorted by cell) is never exposed.
 *  - Pointers are DEVICE pointers unless the comment says "host".
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *    on it and return without waiting, except where "synchronizes" is stated.
 *  - The caller owns every buffer, including the workspace; the library never
 *    allocates device memory and never frees caller memory.  A context must
 *    be used from one host thread at a time.
 *  - Errors: argument errors return at once without enqueuing work.  Errors
 *    found on the device (a particle outside the box, a capacity overflow, a
 *    NaN) set a sticky device flag; dem_poll reports it, and from then on
 *    every call on the context returns that error (the context is poisoned)
 *    until dem_destroy.
 */
#ifndef CFDDEM_H
#define CFDDEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CFDDEM_ABI_VERSION 5

typedef struct dem_ctx dem_ctx;
typedef int32_t dem_status;

enum {
  DEM_OK = 0,
  DEM_E_ARG = -1,         /* invalid argument or parameter */
  DEM_E_WORKSPACE = -2,   /* workspace NULL, misaligned (256 B) or too small */
  DEM_E_HIP = -3,         /* a HIP runtime call failed */
  DEM_E_DOMAIN = -4,      /* a particle centre left the box */
  DEM_E_CAPACITY = -5,    /* cell, neighbour-list or element capacity exceeded */
  DEM_E_NAN = -6,         /* NaN in the particle state */
  DEM_E_UNSUPPORTED = -7, /* valid but not implemented (e.g. another drag law) */
  DEM_E_ABI = -8          /* abi_version mismatch */
};

enum { DEM_FP64 = 0, DEM_FP32_FORCES = 1 };
/* Drag closures of Section 2.3.2 (cfd_params.drag).  DEM_DRAG_BETA_OVER_EPS
 * may be OR-ed in: the coefficient is divided by the fluid fraction,
 * beta_B = beta_A / eps (Eq. "beta"); without it both models use the same
 * coefficient. */
enum {
  DEM_DRAG_DIFELICE = 0,
  DEM_DRAG_DALLAVALLE = 1,
  DEM_DRAG_RONG = 2,
  DEM_DRAG_KOCH_HILL = 3,
  DEM_DRAG_BEETSTRA = 4,  /* the printed force multiplies the fluid velocity: the slip is read */
  DEM_DRAG_GIDASPOW = 5,  /* per-particle coefficient = mixture coefficient x V_p / (1 - eps) */
  DEM_DRAG_BETA_OVER_EPS = 0x100
};
enum { DEM_MODEL_A = 0, DEM_MODEL_B = 1 };

/* DEM parameters (host struct).  Material constants follow Table
 * "tab:viscoelastic": the particle-particle contact uses (E, nu) for both
 * bodies, the particle-wall contact combines the particle's (E, nu) with the
 * wall's (E_w, nu_w).  e must be in (0, 1]; mu >= 0. */
typedef struct {
  int32_t abi_version;   /* must be CFDDEM_ABI_VERSION */
  int32_t precision;     /* DEM_FP64, or DEM_FP32_FORCES: pair-force and drag
                            arithmetic in FP32; positions, velocities,
                            tangential history, overlaps/normals and every
                            accumulation stay FP64 */
  int64_t n;             /* particle count, >= 1 */
  double box_lo[3];      /* the six box faces are the walls */
  double box_hi[3];
  double gravity[3];
  double dt;             /* DEM time step, > 0 */
  double E, nu, e, mu;   /* particle: Young, Poisson; pair restitution, Coulomb friction */
  double E_w, nu_w, e_w, mu_w; /* wall: Young, Poisson; particle-wall restitution, friction */
  int32_t max_neighbors; /* neighbour-list capacity per particle: partners closer
                            than R_i + R_j + skin, 1..64; 0 = 32 */
  int32_t cell_capacity; /* particles per DEM cell, 1..1024; 0 = derived from sizes.
                            Between re-sorts, inside a run of steps, only the
                            particles away from the cell they were sorted into
                            take a slot; the last step of every run lists all */
  int32_t resort_every;  /* DEM steps between re-sorts of the particle arrays by
                            cell; 0 = never (order of creation) */
  int32_t lanes;         /* lanes of a wavefront sharing one particle in the
                            contact-force kernel (each walks every lanes-th
                            list entry): 1, 2 or 4; 0 = 2.  A tuning choice:
                            contact sets do not depend on it, force sums only
                            in their rounding */
  double d_max;          /* largest particle diameter (sizes the DEM cells:
                            cells are at least this wide) */
  double d_min;          /* smallest particle diameter (sizes cell_capacity);
                            dem_create rejects radii outside [d_min, d_max]/2 */
  double skin;           /* neighbour-list skin (m), >= 0; 0 = 0.1 d_min.  The
                            broad search lists partners within R_i + R_j + skin
                            and is redone on the device as soon as a particle
                            has moved more than skin/2 since the last one */
  double mu_r, mu_r_w;   /* rolling friction coefficients, particle-particle and
                            particle-wall, >= 0 (0 = no rolling torque).  The
                            rolling torque M^r of Eq. "angular_momentum" (its
                            form is not given in the paper) is the constant
                            torque -mu_r R_e |f_n| w/|w| with w = w_i - w_j the
                            relative angular velocity at the half step (w_i
                            against a wall) and f_n the full normal force; it
                            acts on i, its negation on j, and is zero when
                            w = 0 */
} dem_params;

/* Coupling parameters (host struct).  The structured hex mesh spans the DEM
 * box: n_el[a] equal elements along axis a.  Velocity nodes form the
 * (order*n_el[a]+1)-per-axis lattice, pressure nodes the Q1 lattice
 * (n_el[a]+1 per axis); both are numbered x fastest, then y, then z.
 * Quadrature: Gauss-Legendre, (order+1) points per axis, numbered x fastest
 * within an element; element index (ez*n_el[1]+ey)*n_el[0]+ex; quadrature
 * arrays are element-major: q_global = element*(order+1)^3 + q_local. */
typedef struct {
  int32_t order;   /* 1 = Q1-Q1, 2 = Q2-Q1 */
  int32_t n_el[3]; /* >= 1 each */
  double rho_f;    /* fluid density, > 0 */
  double mu_f;     /* fluid DYNAMIC viscosity (Pa s), > 0 */
  int32_t drag;    /* DEM_DRAG_* closure, optionally | DEM_DRAG_BETA_OVER_EPS */
  int32_t model;   /* DEM_MODEL_A or DEM_MODEL_B (decides what is handed to
                      the fluid, Eqs. "fa" / "fb") */
  double eps_min;  /* the drag closure sees clamp(eps, eps_min, 1); (0, 1] */
  int32_t shear;   /* 1: add the shear force f = -V_p div(tau_f) (Section 2.3.2,
                      Eqs. "fa" / "fb"), with tau_f the stress of Eq. "stress"
                      evaluated from the Q_n velocity field at the particle
                      (div tau = mu_f (lap u + grad(div u) / 3)); model B also
                      hands it to the fluid.  0: no shear force */
  int32_t smooth;  /* 1: smoothed void fraction.  The element PCM values (Eq.
                      "void_fraction") are projected onto the continuous
                      velocity space: eps_h with int eps_h phi + smooth_L2 int
                      grad eps_h . grad phi = int eps_PCM phi for every basis
                      function phi (natural boundary conditions; the scheme
                      with smoothing length L^2 of Tables "tab:setup2" and
                      "tab:setup4" is described in a companion paper; this
                      weak form is the reading).  eps_q is then eps_h at the
                      quadrature points and the closure sees eps_h at each
                      particle.  Solved directly at every coupling step (the
                      matrix is a Kronecker sum of 1D mass and stiffness
                      matrices, diagonalized at creation by their generalized
                      eigenvectors).  In a batch, each bed with it runs
                      its own solve inside the batch's coupling step.  A
                      velocity lattice of more than 2^31 - 1 nodes is
                      rejected (DEM_E_ARG).
                      0: element PCM values (eps_q constant per element) */
  double smooth_L2; /* smoothing length squared (m^2), >= 0 (0: the plain
                       projection) */
  int32_t elem_threads; /* threads computing one occupied element in the
                       coupling step: 16 or 32 (a group of a wavefront: 4 or
                       2 elements per wavefront instruction, for elements of
                       few particles; an element may then hold at most 256
                       or 512 particles, more raise DEM_E_CAPACITY), 64
                       (one wavefront) or 128 (up to 128 particles in one
                       pass); 0 = 128.  A tuning choice: outputs depend on it
                       only in the rounding of the element sums.  Every bed
                       of a batch must have the same value */
} cfd_params;

/* Bytes of device workspace dem_create needs for these parameters.  Pure host
 * function: no HIP call.  Returns 0 when the parameters are invalid. */
size_t dem_workspace_bytes(const dem_params *dp, const cfd_params *cp);

/* Create a bed.  x, v, omega: 3 x n (component-major); radius, density: n.
 * All five are device arrays, read during the call's stream work and copied
 * into the workspace (the caller may reuse them once the stream reaches this
 * point).  workspace: device memory of ws_bytes >= dem_workspace_bytes(),
 * 256-byte aligned, owned by the caller and kept alive until dem_destroy.
 * The DEM cell grid is nested in the mesh elements (each element is split
 * into k_a >= 1 cells per axis, cells at least one maximum diameter wide), so
 * the mesh is fixed at creation.
 * Creation "primes" the stored contact force and torque with one contact
 * evaluation at the initial state with zero tangential overlap; the held
 * fluid force starts at zero.  *out receives the context (host pointer). */
dem_status dem_create(const dem_params *dp, const cfd_params *cp, const double *x,
                      const double *v, const double *omega, const double *radius,
                      const double *density, void *workspace, size_t ws_bytes,
                      void *stream, dem_ctx **out);

/* Advance n_steps >= 0 DEM steps with the held fluid force (Section 2.3.1:
 * the coupling force is computed once per CFD step and held during the
 * f_coupling DEM sub-steps).  Per step: half kick and drift, binning of the
 * new positions into the cell grid, broad search (cell-list neighbour lists,
 * only when some particle moved more than skin/2 since the last one), fine
 * search (exact overlap test over the lists and the six walls), contact
 * forces at the half-step velocities, second half kick. */
dem_status dem_step(dem_ctx *ctx, int32_t n_steps, void *stream);

/* One coupling step at the current particle state with the given fluid field
 * (Section 2.3: locate and PCM void fraction, Q_n interpolation at the
 * particles, drag closure, particle forces, reduction to quadrature points;
 * F_pf of Eqs. "fa" / "fb").
 *   u_nodes: 3 x n_v nodal velocity (component-major over velocity nodes)
 *   p_nodes: n_p nodal pressure (Q1); must not contain the hydrostatic part
 *            rho_f g.x, since buoyancy is applied to the particles explicitly
 *   eps_q, beta_q: n_el*n_q outputs (void fraction, beta_q = sum beta_p / V_e)
 *   fpf_q: 3 x (n_el*n_q) force density on the fluid (component-major)
 *   elem_sums: NULL, or 12 x n_el (component-major over elements):
 *     0 particle count, 1 sum V_p, 2 sum beta_p, 3-5 sum beta_p u_p,
 *     6-8 sum f_D, 9-11 sum of the undisturbed-flow forces f_gradp (+ f_shear
 *     when cfd_params.shear is set)
 * Also stores f_fp = f_D + f_B + f_gradp (+ f_shear) per particle, held by the
 * following dem_step calls. */
dem_status cfd_dem_couple(dem_ctx *ctx, const double *u_nodes, const double *p_nodes,
                          double *eps_q, double *beta_q, double *fpf_q, double *elem_sums,
                          void *stream);

/* Copy the state out in original-ID order (each argument may be NULL):
 * positions, velocities, angular velocities, held fluid force, all 3 x n. */
dem_status dem_read_state(dem_ctx *ctx, double *x, double *v, double *omega, double *f_fp,
                          void *stream);

/* Stored contact force and torque (sums over the contacts of the last
 * evaluation), 3 x n, original-ID order.  Either may be NULL. */
dem_status dem_read_forces(dem_ctx *ctx, double *F_c, double *T_c, void *stream);

/* Kinetic energy of the current (boundary) state: out[0] = sum 1/2 m v^2,
 * out[1] = sum 1/2 I w^2 with I = 2/5 m R^2 (solid spheres, Eq.
 * "angular_momentum"), host array of 2.  The sums are formed in a fixed order
 * (per 256-particle block, then over blocks), so repeated calls on the same
 * state agree bit for bit.  Used to detect a bed at rest, e.g. when a bed is
 * filled and left to settle by DEM steps alone before coupled runs (Section
 * 3.2).  Synchronizes the stream; returns the sticky error of a poisoned
 * context without computing. */
dem_status dem_kinetic_energy(dem_ctx *ctx, double *out, void *stream);

/* For callers that cannot allocate or synchronize: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The same
 * sums as dem_kinetic_energy, bit for bit, with its per-block partial sums in
 * a fixed device array of the library (1 MiB per GPU, held until the process
 * ends) instead of the bed's workspace; calls no allocating routine and does
 * not synchronize.  out: DEVICE array of 2 doubles, written on the stream.
 * Beds of more than 256 x 65536 = 16,777,216 particles are refused with
 * DEM_E_CAPACITY.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (other streams or host threads) race; calls on one
 * stream are ordered.  Returns the sticky error of a poisoned context. */
dem_status dem_kinetic_energy_noalloc(dem_ctx *ctx, double *out, void *stream);

/* Monitoring metrics of the current state, for checking a run against the
 * conservation properties of the method: Newton's third law makes the
 * contact forces conserve total momentum (Section 2.2, Eq. "newton_law");
 * the contact-force equation needs normal overlaps small against the radii;
 * the particle-centroid void fraction (Eq. "void_fraction") conserves the
 * solid volume, sum over elements of (1 - eps_e) V_e = sum of V_p.
 * out (host, 7 doubles):
 *   [0..2] total linear momentum, sum of m v over the particles (boundary
 *          velocities of the last completed step);
 *   [3]    largest normal overlap of the last evaluation's contacts over the
 *          smaller radius of the pair (the particle's radius for a wall);
 *          0 without contacts;
 *   [4]    total solid volume, sum of 4/3 pi R^3;
 *   [5]    the same volume seen by the fluid: sum over the quadrature points
 *          of w_q (1 - eps_q), with eps_q as cfd_dem_couple wrote it (device,
 *          n_elem x (order+1)^3, may be NULL: then NaN) and w_q the Gauss
 *          weights times the element volume;
 *   [6]    largest particle speed |v|.
 * Sums are reduced in a fixed order (the same bits on every call).  Uses the
 * workspace and synchronizes the stream.  Errors: DEM_E_ARG (ctx or out
 * NULL), the sticky error of a poisoned context. */
dem_status dem_metrics(dem_ctx *ctx, const double *eps_q, double *out, void *stream);

/* Element and DEM-cell index of every particle at its last binning, original-ID
 * order.  Element index as in cfd_params; cell index
 * element*(kx*ky*kz) + (sz*ky+sy)*kx + sx with sub-cell s_a in [0, k_a).
 * k (host, 3 ints, may be NULL) receives the cells per element per axis. */
dem_status dem_read_cells(dem_ctx *ctx, int32_t *elem, int32_t *cell, int32_t *k, void *stream);

/* Contacts of the last evaluation as pairs (i, j): particle pairs with i < j
 * (original IDs) and wall contacts (i, -1-w), w = 0..5 for the x-lo, x-hi,
 * y-lo, y-hi, z-lo, z-hi faces; sorted by (i, j).  pairs: 2 x cap int64
 * (row 0 = i, row 1 = j), delta_t: 3 x cap (component-major) tangential
 * overlap of each contact.  Synchronizes the stream; *n_out (host) receives
 * the total count, which may exceed cap (then only cap are written). */
dem_status dem_read_contacts(dem_ctx *ctx, int64_t *pairs, double *delta_t, int64_t cap,
                             int64_t *n_out, void *stream);

/* ---- Checkpoint / resume ----
 *
 * A checkpoint is the complete state that a DEM step and a coupling step
 * read (Sections 2.2 and 2.3): positions, velocities and angular velocities
 * of the last completed step, the stored contact force and torque, the held
 * fluid force, radii and masses, every contact's tangential overlap
 * (particle pairs and walls) with the neighbour lists that carry it, the
 * positions of the last broad search, the step and coupling-call counters
 * and the internal particle order.  Restoring it into a context created with
 * the same structural parameters (n, max_neighbors, cell_capacity,
 * precision, skin and the mesh/box) and then running the same calls gives
 * the same results bit for bit as the run that wrote it.  The blob is plain
 * bytes (no pointers): it may be copied to the host, stored and brought back.
 *
 * Bytes of a checkpoint of this context (host function; 0 for NULL). */
size_t dem_checkpoint_bytes(dem_ctx *ctx);

/* Write the checkpoint into dst: device memory of >= dem_checkpoint_bytes
 * bytes, 256-byte aligned, owned by the caller.  Synchronizes the stream.
 * Returns the sticky error (and writes nothing) for a poisoned context,
 * DEM_E_WORKSPACE when bytes is too small. */
dem_status dem_read_checkpoint(dem_ctx *ctx, void *dst, size_t bytes, void *stream);

/* Restore a checkpoint (device memory, 256-byte aligned, as written by
 * dem_read_checkpoint) into ctx, replacing its whole state.  ctx must have
 * been created with the same structural parameters as the context that wrote
 * it (else DEM_E_ARG; DEM_E_ABI for a blob of another library version) and
 * must not belong to a batch.  Material constants, the time step, gravity,
 * the fluid parameters and the tuning choices (lanes, threads per element,
 * re-sort interval) are the context's own.  Synchronizes the stream; src may
 * be reused once the call returns. */
dem_status dem_write_state(dem_ctx *ctx, const void *src, size_t bytes, void *stream);

/* Synchronizes the stream; reports the sticky device error (0 or a negative
 * DEM_E_* code, host out) and the number of contacts of the last evaluation
 * (host out).  Either pointer may be NULL. */
dem_status dem_poll(dem_ctx *ctx, int32_t *sticky_error, int64_t *n_contacts, void *stream);

/* Per-kernel timing of the dominant DEM kernel: when enabled, every launch of
 * the contact-force kernel is bracketed by HIP events on its stream.
 * dem_kernel_timing_read synchronizes the stream and returns (host outs) the
 * number of timed launches and their summed duration in milliseconds, and
 * restarts the count. */
dem_status dem_kernel_timing(dem_ctx *ctx, int32_t enable);
dem_status dem_kernel_timing_read(dem_ctx *ctx, int64_t *launches, double *total_ms,
                                  void *stream);

/* Release the context (host memory and HIP events).  The workspace stays the
 * caller's.  Work already enqueued must have completed or be on the stream
 * that the caller synchronizes before freeing the workspace.  DEM_E_ARG (and
 * nothing released) while the bed belongs to a batch. */
dem_status dem_destroy(dem_ctx *ctx);

/* ---- Batches: many independent beds advanced by the same launches ----
 *
 * A batch groups beds already created with dem_create (each with its own
 * particles, box, materials, time step, mesh and fluid parameters) so that
 * every DEM step and coupling step of all of them runs as one launch per
 * kernel: each block of a batched kernel finds its bed and its block within
 * the bed in a block map, and the bed's arrays and constants in device
 * tables.  The arithmetic of a bed does not depend on the other beds of the
 * batch.  Requirements: 1..4096 beds, all of the same precision, lanes and
 * elem_threads; for coupling, all of the same velocity order and each with
 * fewer than 2^20 elements.  A bed with the smoothed void fraction has its
 * field solved on its own mesh within the batch's coupling step (launches
 * per such bed, before the shared ones, and its quadrature-point values
 * after them).  A bed belongs to at most one batch at a time; while it does
 * it must be advanced only through the batch (dem_read_*, dem_poll,
 * dem_kernel_timing and dem_read_checkpoint stay valid; dem_step,
 * dem_write_state and dem_destroy do not; errors are reported per bed by
 * dem_poll).  Destroying the batch, or retiring the bed from its slot,
 * leaves the bed usable on its own.  The same algorithm as dem_step / cfd_dem_couple
 * (Sections 2.2 and 2.3) runs on every bed. */
typedef struct dem_batch dem_batch;

/* Device workspace of a batch of these beds (host function; 0 on invalid
 * arguments).  beds: host array of n_beds contexts. */
size_t dem_batch_workspace_bytes(int32_t n_beds, dem_ctx *const *beds);

/* Build the batch (slots 0..n_beds-1 of a batch of exactly these beds' size,
 * see dem_batch_create_slots).  The coupling buffers are host arrays of n_beds device
 * pointers with the meaning and layout of cfd_dem_couple's arguments, bed by
 * bed; u_nodes == NULL builds a batch without coupling (the other five
 * arrays are then ignored), elem_sums may be NULL or hold NULL entries.
 * The buffers stay registered for the batch's lifetime: dem_batch_couple
 * reads the current contents of u_nodes/p_nodes and overwrites the outputs.
 * workspace: >= dem_batch_workspace_bytes, 256-byte aligned, caller-owned.
 * Synchronizes the stream (the tables are uploaded once).  *out (host)
 * receives the batch. */
dem_status dem_batch_create(int32_t n_beds, dem_ctx *const *beds, const double *const *u_nodes,
                            const double *const *p_nodes, double *const *eps_q,
                            double *const *beta_q, double *const *fpf_q,
                            double *const *elem_sums, void *workspace, size_t ws_bytes,
                            void *stream, dem_batch **out);

/* dem_step(bed, n_steps) for every bed of the batch, as one drift launch, one
 * contact-force launch per step and one bookkeeping launch; beds whose
 * re-sort is due are re-sorted first (per bed). */
dem_status dem_batch_step(dem_batch *batch, int32_t n_steps, void *stream);

/* cfd_dem_couple on every bed of the batch with its registered buffers: one
 * classify launch over all beds' elements and one launch over the occupied
 * elements of all beds. */
dem_status dem_batch_couple(dem_batch *batch, void *stream);

/* n_chunks times: [dem_batch_couple if couple != 0] then
 * dem_batch_step(steps_per_chunk), with the same results.  The coupling step
 * and the run of steps_per_chunk steps are each replayed from a HIP graph
 * captured at their first use (the step graph again when steps_per_chunk
 * changes); due re-sorts run between the two, outside the graphs. */
dem_status dem_batch_run(dem_batch *batch, int32_t n_chunks, int32_t steps_per_chunk,
                         int32_t couple, void *stream);

/* Release the batch (host memory, its graphs, capture stream and pinned map
 * staging); the beds and the workspace stay the caller's, and every bed it
 * held is usable on its own again. */
dem_status dem_batch_destroy(dem_batch *batch);

/* ---- Batch slots: beds join and leave a running batch ----
 *
 * For serving a stream of jobs (continuous batching): a batch with a fixed
 * number of slots and limits on the particles and mesh elements it holds at
 * once; beds are admitted into free slots and retired from them between
 * calls, while the other beds keep their state on the device.  Each bed
 * computes exactly what it computes alone (the arithmetic of a bed does not
 * depend on the others).  The launch layout (block maps, coupling lists) is
 * rebuilt at the next dem_batch_step / dem_batch_couple / dem_batch_run after
 * a change, uploaded stream-ordered from pinned host staging that the batch
 * allocates (launches already enqueued keep the maps they were enqueued
 * with), and the captured graphs are re-captured then (graphs of the old
 * layout are destroyed once their last replay has run). */
typedef struct {
  int32_t slots;          /* beds held at once, 1..4096 */
  int32_t couples;        /* 1: beds are admitted with coupling buffers */
  int64_t max_particles;  /* sum of the held beds' particle counts, >= 1 */
  int64_t max_elements;   /* sum of the held beds' mesh elements (coupling) */
} dem_batch_limits;

/* Device workspace of an empty batch with these limits (host function; 0 on
 * invalid limits). */
size_t dem_batch_slots_workspace_bytes(const dem_batch_limits *limits);

/* An empty batch.  workspace: >= dem_batch_slots_workspace_bytes bytes,
 * 256-byte aligned, caller-owned until dem_batch_destroy.  *out (host)
 * receives the batch. */
dem_status dem_batch_create_slots(const dem_batch_limits *limits, void *workspace, size_t ws_bytes,
                                  void *stream, dem_batch **out);

/* Put bed into free slot `slot`, with its coupling buffers (meaning and
 * layout of cfd_dem_couple's arguments; required when the batch couples,
 * elem_sums may be NULL; ignored otherwise).  The bed continues from its
 * current state and step counter.  Errors: DEM_E_ARG (slot out of range or
 * taken, bed already in a batch, missing buffers), DEM_E_UNSUPPORTED (another
 * precision, lanes, threads per element or velocity order than the beds
 * held), DEM_E_CAPACITY (the limits would be exceeded), or the bed's sticky
 * error.  Enqueues the slot's table entries on the stream. */
dem_status dem_batch_admit(dem_batch *batch, int32_t slot, dem_ctx *bed, const double *u_nodes,
                           const double *p_nodes, double *eps_q, double *beta_q, double *fpf_q,
                           double *elem_sums, void *stream);

/* Free slot `slot`; its bed is usable on its own again (dem_read_*,
 * dem_step, dem_destroy).  Work already enqueued on the batch's stream still
 * reads the bed's workspace: the caller keeps it until the stream has passed
 * that point.  Host-only call. */
dem_status dem_batch_retire(dem_batch *batch, int32_t slot);

/* Static description of a status code. */
const char *dem_status_string(dem_status s);

#ifdef __cplusplus
}
#endif
#endif
