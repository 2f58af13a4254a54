/*
 * lbm.h -- C ABI of the sparse-tile lattice Boltzmann library (liblbm.so).
 *
 * Method: Tomczak & Szafran, "Sparse geometries handling in lattice
 * Boltzmann method implementation for graphic processors" (arXiv 1703.08015).
 * The geometry is covered by a uniform mesh of fixed-size tiles; tiles with
 * no non-solid node are dropped (Sec. 3); a tile map with -1 for empty tiles
 * locates neighbour tiles during propagation (two-copy method, Sec. 3).  One
 * time step fuses gather propagation, half-way bounce-back (propagation only
 * between non-solid nodes, Sec. 3.2) and the BGK collision, Eqs. (2) and (7),
 * with Guo forcing for a body acceleration g, in one of the paper's two fluid
 * models: quasi-compressible, Eqs. (3) and (5), or incompressible, Eqs. (4)
 * and (6).
 *
 * Conventions for every call
 *   - Return value: LBM_OK (0) or a negative LBM_ERR_* code.  Nothing throws
 *     across the ABI.  lbm_last_error() returns a thread-local description of
 *     the most recent failure on the calling thread.
 *   - Dense host or device arrays are x-fastest: element (x, y, z) of an
 *     (nx, ny, nz) lattice is at x + nx*(y + ny*z) (a torch tensor of shape
 *     (nz, ny, nx)).  Vector fields are [component][z][y][x]; PDF fields are
 *     [i][z][y][x] with the velocity order given by lbm_lattice().  For a
 *     batch (lbm_tiles_concat) dense arrays are the concatenation, sample
 *     after sample, of each sample's own dense array.
 *   - The caller owns every host and device buffer and must keep the solver's
 *     workspace alive until lbm_destroy.  The library owns only the opaque
 *     lbm_tiles and lbm_solver objects; it never allocates device memory.
 *   - Device work is enqueued on the HIP stream given to lbm_create (NULL =
 *     the default stream) and is asynchronous unless a call says otherwise.
 *   - A solver is not thread-safe; distinct solvers may be used concurrently.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------- */
#define LBM_OK 0
#define LBM_ERR_ARG (-1)         /* bad argument (NULL, tau <= 1/2, ...) */
#define LBM_ERR_SHAPE (-2)       /* periodic axis not a multiple of the tile edge, bad size */
#define LBM_ERR_UNSUPPORTED (-3) /* lattice / tile / storage combination not built */
#define LBM_ERR_HIP (-4)         /* a HIP runtime call or kernel launch failed */
#define LBM_ERR_NONFINITE (-5)   /* a reduction met a NaN or infinity */
#define LBM_ERR_STATE (-6)       /* call out of order (e.g. step before init) */
#define LBM_ERR_NOMEM (-7)       /* workspace too small, host allocation failed */

/* ---- PDF storage forms ---------------------------------------------- */
#define LBM_F64 0        /* f_i as IEEE binary64, arithmetic in FP64 */
#define LBM_F32_OFFSET 1 /* f_i - w_i rho0 as binary32, arithmetic in FP32 */
#define LBM_F16_OFFSET 2 /* (f_i - w_i rho0) * 2^s as binary16, arithmetic in FP32 */

typedef struct lbm_tiles lbm_tiles;
typedef struct lbm_solver lbm_solver;

/* Statistics of a tiling (Sec. 2.3, Eqs. 11 and 17). */
typedef struct {
  int32_t shape[3];      /* lattice size given to lbm_tiles_build (one sample) */
  int32_t grid[3];       /* size after padding non-periodic axes with solid */
  int32_t tile[3];       /* tile edges (ax, ay, az) */
  int32_t tgrid[3];      /* tiles per axis */
  uint32_t periodic;     /* bit 0 x, bit 1 y, bit 2 z */
  int32_t words;         /* 64-bit fluid-mask words per tile = ax*ay*az/64 */
  int32_t n_samples;     /* 1, or the number of concatenated samples */
  int32_t reserved;
  int64_t n_tiles;       /* N_tiles: all tiles (summed over samples) */
  int64_t n_ftiles;      /* N_ftiles: non-empty tiles */
  int64_t n_fluid;       /* non-solid nodes */
  int64_t n_nodes;       /* nodes of the unpadded lattice (summed over samples) */
  double phi;            /* porosity, Eq. (11) */
  double phi_t;          /* average tile porosity, Eq. (17) */
  double tiles_ratio;    /* N_tiles / N_ftiles (Sec. 3.1.1.1) */
  double alpha_m;        /* alpha_M, the input of Eqs. (27)-(32) (Sec. 3.1.1.2): the share of the faces of
                            non-empty tiles across which the neighbour tile is non-empty (a face buffer of
                            the ghost-buffer method is needed only there), over the axes along which the
                            lattice has more than one node; 0 without non-empty tiles */
} lbm_tiles_info_t;

/* Solver parameters. */
typedef struct {
  int32_t lattice;         /* 9 = D2Q9 (tile 16x16x1) or 19 = D3Q19 (tile 4x4x4 or 4x4x8) */
  int32_t storage;         /* LBM_F64, LBM_F32_OFFSET or LBM_F16_OFFSET */
  double tau;              /* BGK relaxation time, Eq. (2): > 1/2, or +inf = pure streaming */
  double g[3];             /* body acceleration (every sample; see lbm_set_sample_force) */
  double rho0;             /* reference density: cold start and offset storage */
  int32_t f16_scale_log2;  /* s of LBM_F16_OFFSET (0..24) */
  int32_t tiles_per_block; /* waves per workgroup for the D3Q19 step: 1, 2, 4 or 8 (0 = 4) */
  int32_t tile_order;      /* LBM_ORDER_*: order in which tiles are stored and processed */
  int32_t step_kernel;     /* LBM_KERNEL_*: which step kernel runs */
  int32_t store_policy;    /* LBM_STORE_*: cache policy of the step's PDF stores */
  int32_t persistent;      /* 1: the D3Q19 4x4x4 step runs as one persistent grid striding over the
                              active tile list; 0: one wavefront per tile */
  int32_t graph_steps;     /* K > 0: lbm_step replays captured HIP graphs of K steps; 0: plain launches */
  int32_t model;           /* LBM_MODEL_*: fluid model of the collision (0 = quasi-compressible) */
  int32_t pattern;         /* LBM_PATTERN_*: PDF buffers and streaming pattern (0 = two copies) */
  int32_t collision;       /* LBM_COLLISION_*: BGK (0) or MRT */
  int32_t reserved;        /* set to 0 */
  double mrt_rates[5];     /* MRT: s_e, s_eps, s_q, s_pi, s_m (0 = published default) */
} lbm_params;

/* Fluid model of the collision (Sec. 2.1).
 *   QUASI_COMPRESSIBLE: f_eq_i = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u),
 *     Eq. (3); u = sum c_i f_i / rho + g/2, Eq. (5); Guo force density rho g.
 *   INCOMPRESSIBLE: f_eq_i = w_i (rho + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u),
 *     Eq. (4); u = sum c_i f_i + g/2, Eq. (6); the reference density of the
 *     velocity terms is 1 in lattice units, so the force density is g.
 * Both use the source F_i = w_i d [3 (c_i - u).g + 9 (c_i.u)(c_i.g)] with d the
 * force density's factor (rho or 1), scaled by (1 - 1/(2 tau)). */
#define LBM_MODEL_QUASI_COMPRESSIBLE 0
#define LBM_MODEL_INCOMPRESSIBLE 1

/* PDF storage pattern.
 *   TWO_COPY: the paper's two-copy method (Sec. 3): each step gathers from one
 *     copy and writes the other.
 *   SINGLE_COPY: one copy, updated in place (the "AA" access pattern), with
 *     half the PDF memory; it stands where the paper's ghost-buffer method
 *     (Sec. 3, Fig. 4) saves memory.  Steps alternate between a gather/scatter
 *     step, which reads f*_i(x - c_i) and writes f*_i(x) into the slot that
 *     x + c_i reads next, and a step local to each node.  Every step does the
 *     arithmetic of the two-copy step on the same values, so the results are
 *     identical.  With lbm_set_active, the active set may change only after an
 *     even number of steps since lbm_init or lbm_pdfs_import (LBM_ERR_STATE
 *     otherwise). */
#define LBM_PATTERN_TWO_COPY 0
#define LBM_PATTERN_SINGLE_COPY 1

/* Collision operator.
 *   BGK: single relaxation time, Eqs. (2) and (7).
 *   MRT: multiple relaxation times, Eq. (8), with the collision matrix
 *     diagonal in an orthogonal moment basis (the paper does not give it):
 *     Lallemand & Luo (2000) for D2Q9, d'Humieres et al. (2002) for D3Q19:
 *       f* = f + M^-1 [-S M (f - f_eq) + (I - S/2) M F],
 *     f_eq and F of the chosen fluid model.  The shear-stress moments relax
 *     with 1/tau; the energy e, energy square eps, energy flux q, and (D3Q19)
 *     the fourth-order pi and third-order m moments with mrt_rates =
 *     {s_e, s_eps, s_q, s_pi, s_m}, each in (0, 2); an entry 0 takes the
 *     published default (D3Q19 1.19, 1.4, 1.2, 1.4, 1.98; D2Q9 1.64, 1.54,
 *     1.9, and s_pi, s_m unused).  Equal rates 1/tau give the BGK collision. */
#define LBM_COLLISION_BGK 0
#define LBM_COLLISION_MRT 1  /* built for tiles_per_block 0 or 4 and non-regular store policy */

/* Cache policy of the PDF stores of the step: a stored value is next read one
 * step later, after the whole working set has streamed through the caches, so
 * the default writes it non-temporally and leaves L2 to the halo reads. */
#define LBM_STORE_AUTO 0
#define LBM_STORE_REGULAR 1
#define LBM_STORE_NONTEMPORAL 2

/* Tile order inside the solver (the exported tiling is always row-major).
 * Morton order keeps neighbour tiles close in memory and in time. */
#define LBM_ORDER_MORTON 0
#define LBM_ORDER_ROWMAJOR 1

/* Step kernel: AUTO picks the scalar-mask D3Q19 kernel for 4x4x4 tiles and
 * the generic kernel (LDS-staged neighbour records) otherwise.  SHUFFLE is
 * the scalar-mask kernel in its shuffle form (two-copy step, 4x4x4 tiles):
 * each lane loads its own node's values coalesced, sources inside the tile
 * come from other lanes of the wavefront (DPP row shifts, ds_bpermute), and
 * only sources in neighbour tiles are gathered from memory (the in-tile
 * streaming of the paper's Fig. 5 done with wavefront shuffles instead of
 * shared memory).  Same results, bit for bit, as SCALAR_MASK. */
#define LBM_KERNEL_AUTO 0
#define LBM_KERNEL_GENERIC 1
#define LBM_KERNEL_SCALAR_MASK 2
#define LBM_KERNEL_SHUFFLE 3

/* Velocity set and weights of a lattice (q = 9 or 19): c[3*q] (x, y, z per
 * direction), w[q], opp[q].  Standard D2Q9 / D3Q19 sets; the paper's Fig. 1
 * shows the D2Q9 set, the weights are those of Eq. (3) with c_s^2 = 1/3. */
int lbm_lattice(int32_t q, int32_t *c, double *w, int32_t *opp);

/* ---- tiling (host only, once per geometry: Sec. 3) ------------------
 * solid: host uint8 [nz][ny][nx], nonzero = solid.  shape = {nx, ny, nz}
 * (nz = 1 in 2D).  tile = {4,4,4}, {4,4,8} or {16,16,1}.  Non-periodic axes
 * are padded at the high end with solid nodes; a periodic axis must be a
 * multiple of its tile edge (else LBM_ERR_SHAPE).  Non-empty tiles are
 * numbered row-major over tile coordinates, tx fastest.  *out is owned by
 * the caller and released with lbm_tiles_free. */
int lbm_tiles_build(const uint8_t *solid, const int32_t shape[3], const int32_t tile[3],
                    uint32_t periodic, lbm_tiles **out);

int lbm_tiles_info(const lbm_tiles *t, lbm_tiles_info_t *out);

/* Copy the tiling into caller-sized host arrays (any pointer may be NULL):
 *   tile_map   int32 [n_tiles]     index of the non-empty tile or -1 (the paper's tileMap)
 *   tile_coord int32 [3*n_ftiles]  (tx, ty, tz) of each non-empty tile
 *   nbr        int32 [27*n_ftiles] neighbour row, entry (dx+1)+3(dy+1)+9(dz+1),
 *                                  wrapped on periodic axes, -1 outside or empty
 *   fluid      uint64 [words*n_ftiles] node l = lx + ax*(ly + ay*lz) of a tile is
 *                                  bit l%64 of word l/64, set = non-solid
 * For a batch, tile_map holds each sample's map in turn and all tile indices
 * are global (into the concatenated list). */
int lbm_tiles_export(const lbm_tiles *t, int32_t *tile_map, int32_t *tile_coord, int32_t *nbr,
                     uint64_t *fluid);

/* Concatenate k tilings (same tile shape) into one tile list for a batched
 * run: neighbour rows are offset, no link crosses samples.  The parts stay
 * owned by the caller. */
int lbm_tiles_concat(const lbm_tiles *const *parts, int32_t k, lbm_tiles **out);

void lbm_tiles_free(lbm_tiles *t);

/* ---- solver ----------------------------------------------------------
 * Device workspace size for a tiling and parameters (both PDF copies of the
 * two-copy method, Sec. 3, plus tile tables and reduction scratch). */
int lbm_workspace_bytes(const lbm_tiles *t, const lbm_params *p, size_t *bytes);

/* Create a solver.  ws: device memory of at least lbm_workspace_bytes bytes,
 * 256-byte aligned, kept alive by the caller until lbm_destroy.  stream: a
 * hipStream_t (NULL = default stream).  Uploads the tile tables (blocking). */
int lbm_create(const lbm_tiles *t, const lbm_params *p, void *ws, size_t bytes, void *stream,
               lbm_solver **out);

void lbm_destroy(lbm_solver *s);

/* Change the stream later calls enqueue on. */
int lbm_set_stream(lbm_solver *s, void *stream);

/* Moving wall: the face of the box along `axis` (0 x, 1 y, 2 z) beyond the
 * last node (side 1) or before the first (side 0) moves with velocity
 * u[3] (host), as the lid of a driven cavity (the paper's dense workload,
 * Sec. 4.1, whose boundary rule it does not state).  A pull from beyond that
 * face returns the half-way bounce-back value plus 6 w_i rho_w (c_i . u),
 * with rho_w = rho0 (quasi-compressible) or 1 (incompressible) (Ladd's
 * moving-wall rule); the face decides also for diagonal links that cross a
 * second face.  The axis must be non-periodic in every sample (LBM_ERR_ARG
 * otherwise).  axis = -1 removes the lid.  Applies to every sample of a
 * batch and to every later step. */
int lbm_set_lid(lbm_solver *s, int32_t axis, int32_t side, const double *u);

/* Per-sample body acceleration g[3*n_samples] (host), for batches. */
int lbm_set_sample_force(lbm_solver *s, const double *g);

/* Batches: restrict the steps to the samples whose flag is nonzero
 * (active[n_samples], host).  A deactivated sample keeps its state (both PDF
 * copies hold it), so it can be read or reactivated later; moments,
 * reductions and exports still cover every sample.  Needs the scalar-mask
 * D3Q19 kernel (LBM_ERR_UNSUPPORTED otherwise).  With LBM_PATTERN_SINGLE_COPY
 * the set may change only after an even number of steps (LBM_ERR_STATE
 * otherwise).  Synchronises the stream. */
int lbm_set_active(lbm_solver *s, const uint8_t *active);

/* Initial state, Eq. (3) or (4) by the model: on every non-solid node the
 * stored post-collision PDFs become f_eq(rho, u).  rho: device dense FP64 (NULL = rho0 everywhere);
 * u: device dense FP64 [3][...] (NULL = 0).  Resets the step counter. */
int lbm_init(lbm_solver *s, const double *rho, const double *u);

/* n >= 0 time steps: gather propagation with half-way bounce-back, then the
 * BGK collision of Eqs. (2) and (7) with Guo forcing in the solver's model
 * (Eqs. (3), (5) or (4), (6)); the two PDF copies swap roles after each step
 * (Sec. 3).  Asynchronous. */
int lbm_step(lbm_solver *s, int32_t n);

/* Macroscopic fields of the current state: rho = sum f*_i and
 * u = (sum c_i f*_i)/rho - g/2, or sum c_i f*_i - g/2 in the incompressible
 * model (the velocity the last collision used).
 * rho: device dense FP64, u: device dense FP64 [3][...]; solid nodes get 0.
 * Either pointer may be NULL.  Asynchronous. */
int lbm_moments(lbm_solver *s, double *rho, double *u);

/* FP64 totals over non-solid nodes, per sample: out_host[4*sample + k] =
 * mass, then momentum x, y, z (sum of rho u with u as in lbm_moments; sum of
 * u in the incompressible model, whose reference density is 1).
 * Fixed-order reduction (run-to-run identical).  Synchronises the stream.
 * LBM_ERR_NONFINITE if any total is not finite. */
int lbm_reduce(lbm_solver *s, double *out_host);

/* Steady-state residual per sample: out_host[sample] =
 * ||u - u_ref||_2 / ||u||_2 over non-solid nodes, where u_ref is the velocity
 * recorded at the previous lbm_residual or lbm_init call; then records the
 * current velocity as the new reference.  FP64, fixed order.  Synchronises.
 * LBM_ERR_NONFINITE if a residual is not finite. */
int lbm_residual(lbm_solver *s, double *out_host);

/* Dense FP64 copy of the stored PDFs, [i][z][y][x] (solid entries 0), device
 * pointer.  Offset storage forms are expanded as f = w_i rho0 + offset. */
int lbm_pdfs_export(lbm_solver *s, double *dev_dense);

/* Load stored PDFs from a dense FP64 device array of the same layout (solid
 * entries ignored); offset forms round to their storage type. */
int lbm_pdfs_import(lbm_solver *s, const double *dev_dense);

/* Number of steps taken since lbm_init. */
int64_t lbm_step_count(const lbm_solver *s);

/* ---- invariants of the discrete dynamics (starting states) ----------
 * The step (Eqs. 2, 3, 5, 7 with Guo forcing; propagation only between
 * non-solid nodes, Sec. 3.2) conserves the mass of every set of non-solid
 * nodes joined by lattice links, and a family of staggered momenta: for
 * every field beta with c.beta(x + c) = -c.beta(x) on each link between
 * non-solid nodes, L = sum_x beta(x).j(x) (j = sum_i c_i f*_i) obeys
 * L(t+1) = -L(t) + sum_x beta(x).g rho(x).  Collision keeps j at each node
 * (the force adds rho*g); streaming and bounce-back both flip the sign of
 * every term.  These are never damped.  beta_k = (-1)^{x_k} over a set
 * joined by links with c_k != 0 is one such field; nodes that touch only
 * diagonally add more.  A start from rest has L = 0 for all of them and
 * rho0 per node; any other starting state reaches a long-time state that
 * differs unless it is projected first (lbm_project_invariants). */

/* Connected components of the non-solid nodes of one lattice under the
 * links of the D2Q9 (q = 9, shape[2] = 1) or D3Q19 (q = 19) set that join
 * two non-solid nodes; axis = -1 keeps every link, axis = k in {0, 1, 2}
 * (x, y, z; k < 2 for q = 9) only links with c_k != 0.  solid: host uint8
 * [nz][ny][nx], nonzero = solid; shape = {nx, ny, nz}; periodic bits as in
 * lbm_tiles_build (a non-periodic edge is a wall).  labels: host int32
 * [nz][ny][nx], -1 on solid nodes, else the component number, numbered
 * from 0 in order of first appearance, x fastest.  *count = number of
 * components.  Host only, synchronous; LBM_ERR_ARG / LBM_ERR_UNSUPPORTED
 * for bad arguments, LBM_ERR_NOMEM if host memory runs out. */
int lbm_components(int32_t q, const uint8_t *solid, const int32_t shape[3], uint32_t periodic, int32_t axis,
                   int32_t *labels, int32_t *count);

/* lbm_components on the device, with the same labels and count: solid
 * device uint8 [nz][ny][nx]; labels device int32 [nz][ny][nx] (out: -1 on
 * solid nodes, components numbered from 0 in order of first appearance, x
 * fastest); scratch device int32 of lbm_components_device_scratch(shape)
 * entries (overwritten; must not overlap labels); *count host, written before
 * return.  Lock-free union-find over the links on the given stream, then a
 * fixed-order numbering of the roots; synchronises the stream to return the
 * count.  LBM_ERR_ARG / LBM_ERR_UNSUPPORTED for bad arguments, LBM_ERR_HIP if
 * a launch fails. */
int lbm_components_device(int32_t q, const uint8_t *solid, const int32_t shape[3], uint32_t periodic,
                          int32_t axis, int32_t *labels, int32_t *count, int32_t *scratch, void *stream);
/* Scratch entries (int32) lbm_components_device needs for a shape; -1 for a
 * bad shape. */
int64_t lbm_components_device_scratch(const int32_t shape[3]);

/* lbm_components_device for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same labels and count, with the scratch taken from a fixed
 * device array inside the library instead of a caller buffer.  The array
 * holds lbm_components_noalloc_max_scratch() int32 entries (2^22, 16 MiB;
 * each GPU the library runs on keeps its own copy until the process ends),
 * so a shape whose lbm_components_device_scratch(shape) exceeds it (more
 * than 4,193,280 nodes) fails with LBM_ERR_ARG.  Nothing is allocated:
 * the array's device address is looked up once per device on the first
 * call.  Every call on one GPU shares the array and leaves its contents
 * behind (nothing in it needs clearing: every entry used is written before
 * it is read), so calls that overlap on one GPU race; the stream is
 * synchronised before return.  Errors as for lbm_components_device. */
int lbm_components_device_noalloc(int32_t q, const uint8_t *solid, const int32_t shape[3], uint32_t periodic,
                                  int32_t axis, int32_t *labels, int32_t *count, void *stream);
/* Size of that fixed array, in int32 entries. */
int64_t lbm_components_noalloc_max_scratch(void);

/* Give a starting state (rho, u) for lbm_init the invariants of a start
 * from rest.
 *   q, shape, periodic  the lattice, as for lbm_components;
 *   labels  device int32 [nz][ny][nx]: lbm_components(axis = -1) of the
 *           geometry (negative = solid), count components;
 *   rho, u  device dense FP64, rho [nz][ny][nx] and u [3][nz][ny][nx],
 *           updated in place on non-solid nodes (solid entries untouched);
 *   scratch device FP64, 2 * count + 6 * nx * ny * nz entries, overwritten;
 *           must not overlap rho or u.
 * First rho is scaled per component so that it holds rho0 per node.  Then,
 * with the link operator
 *   (T j)(x) = 3 sum_{i: x + c_i non-solid} w_i c_i [c_i.(j(x) + j(x + c_i))] / 2,
 * whose range is orthogonal to every staggered invariant, `iterations`
 * (1..1000) sweeps j <- j + T(rho u - j) from j = 0 replace rho u, and
 * u = j / rho.  T is the identity on smooth fields away from walls, so a
 * few sweeps keep a smooth prediction while removing every invariant.
 * A component whose mass is zero or not finite yields non-finite values.
 * Asynchronous on the given stream; LBM_ERR_ARG for bad arguments,
 * LBM_ERR_HIP if a launch fails. */
int lbm_project_invariants(int32_t q, const int32_t shape[3], uint32_t periodic, const int32_t *labels,
                           int32_t count, double rho0, int32_t iterations, double *rho, double *u, double *scratch,
                           void *stream);

/* Measurement reference, not part of the method: copy `bytes` bytes from
 * src to dst on the device (both device pointers, 16-byte aligned, not
 * overlapping, bytes a multiple of 16) with one 16-byte non-temporal load
 * and store per thread over a grid that covers the buffer: the rate one
 * read and one write stream reach on this device, against which the step's
 * bandwidth is compared.  Asynchronous on the given stream; LBM_ERR_ARG for
 * bad arguments (or more than 2^31 - 1 workgroups of 256 threads),
 * LBM_ERR_HIP if the launch fails. */
int lbm_device_copy(void *dst, const void *src, size_t bytes, void *stream);

const char *lbm_strerror(int code);
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
