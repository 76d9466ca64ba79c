/*
 * cgks.h -- C ABI of the MI355X p-multigrid compact gas-kinetic scheme
 * (CGKS) library, libcgks.so.
 *
 * The library computes the two-level p-multigrid cycle of "A p-multigrid
 * compact gas-kinetic scheme for steady-state acceleration" (Ji, Shyy, Xu):
 * on the high-order level the compact reconstruction, the smooth-flow
 * gas-kinetic flux at every face Gauss point and the Gauss-Green update of
 * cell averages and cell-averaged gradients under two-stage fourth-order
 * (S2O4) or one-step second-order (S1O2) time marching (Secs. 2.1-2.4);
 * on the low-order level the first-order KFVS residual with forcing and
 * the implicit backward-Euler point-relaxation smoother with local time
 * steps (Sec. 3, Algorithm 1), run in a multicolour order.
 *
 * Conventions (every entry point):
 *  - All functions are extern "C", return a cgks_status and never throw.
 *  - Pointers named *_host are host memory; *_dev are device (HBM) pointers;
 *    stream is a hipStream_t passed as void* (NULL = default stream).
 *  - The caller owns every device buffer.  The library copies what it needs
 *    from host inputs during the call; handles own only host memory.
 *  - Device work is stream ordered; host outputs of *_download calls are
 *    valid when the call returns (they synchronise the stream).
 *  - Host state arrays are structure-of-arrays, variable-major: W[v][cell]
 *    (v = 0..dim+1: rho, rho U_1..rho U_dim, rho E) and dW[a][v][cell]
 *    (a = axis), in the caller's cell order.  Device residual arrays are
 *    [v][batch cells] in the library order (cgks_mesh_permutation); the
 *    device state is cell-major (cgks_state_device).
 *  - Handles are not thread safe.  Distinct batches on distinct streams are.
 */
#ifndef CGKS_H
#define CGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CGKS_OK = 0,
    CGKS_EINVAL = 1,      /* bad argument (null pointer, size, index, state of the handle) */
    CGKS_ENOMEM = 2,      /* host allocation failed or device buffer too small */
    CGKS_EDEVICE = 3,     /* a HIP call failed */
    CGKS_EMESH = 4,       /* invalid mesh: non-positive volume, face shared by > 2 cells,
                             unmatched face, unsupported face shape, stencil that cannot fix the
                             quadratic reconstruction, invalid colouring */
    CGKS_ENONPHYS = 5,    /* density or pressure <= 0 met during a cycle */
    CGKS_EDIVERGED = 6,   /* residual grew to 1e3 times its first value (the start-up rise of an
                             impulsive start stays well below that) */
    CGKS_ENOTCONV = 7,    /* cgks_solve hit max_cycles before the tolerance */
    CGKS_EUNSUPPORTED = 8 /* valid but not implemented (e.g. more colours than the sweep supports) */
} cgks_status;

/* boundary tags of boundary faces (interior faces carry 0) */
enum {
    CGKS_BC_INTERIOR = 0,
    CGKS_BC_SLIP_WALL = 1,          /* inviscid reflecting wall: mirror state, normal velocity reversed */
    CGKS_BC_NOSLIP_ISOTHERMAL = 2,  /* no-slip wall at temperature T_wall: wall state (p_L / T_wall, 0,
                                       p_L), interior gradient, no mass flux.  Not a wall of the
                                       paper's cases; stable only on near-wall cells of about
                                       0.1 D at Re 40; went non-physical on 0.05 D ones */
    CGKS_BC_NOSLIP_ADIABATIC = 3,   /* no-slip adiabatic wall (Sec. 4 viscous cases): mirror state
                                       with every velocity component reversed; zero velocity and
                                       zero heat flux at the wall */
    CGKS_BC_FARFIELD = 4,           /* characteristic (Riemann invariant) far field */
    CGKS_BC_PERIODIC = 5            /* cell-based meshes only: joined to its partner face (bface_pair) */
};

enum { CGKS_S2O4 = 0, CGKS_S1O2 = 1 };
enum { CGKS_LOW_KFVS = 0, CGKS_LOW_LF = 1 };
enum { CGKS_FLUX_SMOOTH = 0, CGKS_FLUX_FULL = 1 };
enum { CGKS_FP64 = 0, CGKS_MIXED32 = 1, CGKS_MIXED32_R64 = 2 };
enum { CGKS_RESIDUAL_HIGH = 0, CGKS_RESIDUAL_LOW = 1, CGKS_RESIDUAL_NORM = 2 };

/*
 * Hybrid mesh, cell based (Sec. 2.1: linear elements; a cell's boundary is a
 * union of N_f triangle or quadrilateral faces, edges in 2-D).  Cells are
 * given by type and a CSR list of vertex ids in the local order below; the
 * library builds the faces (shared faces matched by their vertex sets),
 * orients each face outward from its owner, and tags the faces that no two
 * cells share from the boundary-face list.  POLY cells (split-face cells,
 * cells with collapsed vertices) list their faces explicitly: cell_vert
 * holds the face count, then per face its vertex count (2 in 2-D, 3 or 4 in
 * 3-D) and ids.
 */
enum {
    CGKS_CELL_TRI = 1,    /* 2-D, vertices 0 1 2: edges 01 12 20 */
    CGKS_CELL_QUAD = 2,   /* 2-D, vertices 0 1 2 3 in cyclic order: edges 01 12 23 30 */
    CGKS_CELL_TET = 3,    /* faces 012 013 123 023 */
    CGKS_CELL_PYR = 4,    /* base 0123 (cyclic), apex 4: faces 0123 014 124 234 304 */
    CGKS_CELL_PRISM = 5,  /* triangles 012 and 345, edges 03 14 25: faces 012 345 0143 1254 2035 */
    CGKS_CELL_HEX = 6,    /* quads 0123 and 4567 (cyclic), edges 04 15 26 37: faces 0123 4567 0154 1265
                             2376 3047 */
    CGKS_CELL_POLY = 7    /* explicit faces (see above) */
};

/*
 * dim 2 or 3; xyz [n_vert][dim]; cell_type [n_cell], cell_vert_ptr
 * [n_cell + 1], cell_vert: the cells.  n_bface boundary faces:
 * bface_vert_ptr [n_bface + 1], bface_vert (vertex ids in any order),
 * bface_tag [n_bface] (CGKS_BC_*).  A CGKS_BC_PERIODIC face b is joined to
 * the face bface_pair[b] (which must be periodic and pair back to b) as one
 * interior face; their centroid offset is the period.  bface_pair may be
 * NULL without periodic faces.  colour [n_cell] (NULL: the library's
 * largest-degree-first greedy colouring) sets the classes of the
 * multicolour relaxation: ids 0..15, no two face neighbours alike
 * (CGKS_EMESH otherwise); the sweeps visit them in id order.  order_tile:
 * as in cgks_face_mesh_desc.  Every cell face must be shared by exactly
 * one other cell or listed once as a boundary face (CGKS_EMESH otherwise).
 * All arrays are host memory, read during the call only.
 */
typedef struct {
    int dim;
    int64_t n_vert;
    const double *xyz;
    int64_t n_cell;
    const int32_t *cell_type;
    const int64_t *cell_vert_ptr;
    const int64_t *cell_vert;
    int64_t n_bface;
    const int64_t *bface_vert_ptr;
    const int64_t *bface_vert;
    const int32_t *bface_tag;
    const int64_t *bface_pair;      /* [n_bface] or NULL */
    const int32_t *colour;          /* [n_cell] or NULL */
    int64_t order_tile;
} cgks_mesh_desc;

/*
 * Face-based mesh (the second way in; the same mesh gives the same results
 * bitwise either way).  2-D faces are straight edges (2 vertex ids), 3-D
 * faces are planar triangles (3 ids) or bilinear quadrilaterals (4 ids,
 * cyclic).  The vertex order makes the normal point out of face_owner
 * (counter-clockwise owner boundary in 2-D, right-hand rule in 3-D).
 * face_neigh = -1 marks a boundary face, whose face_bc is one of the
 * CGKS_BC_* wall or far-field tags.  face_shift (may be NULL) holds, per
 * face, the translation [dim] that carries the neighbour next to the owner
 * across a periodic seam (zero elsewhere).  The library puts faces into a
 * canonical form first (owner the smaller cell id, vertex cycle starting
 * at its smallest id, faces sorted by owner, neighbour and vertices), so
 * results depend on the mesh only, not on the order the faces are listed
 * in.  colour: as in cgks_mesh_desc.  order_tile sets the library cell
 * order: the cells are put on a Morton (Z-order) curve of their centroids
 * and cut into tiles of order_tile consecutive cells, each tile
 * colour-major inside (0 = the library default, CGKS_ORDER_TILE_DEFAULT;
 * >= n_cell gives one tile, i.e. the whole mesh colour-major).  Cells of
 * one colour are independent, so the order changes no result beyond the
 * rounding of the residual norm's sum; tiles keep a cell's neighbours close
 * in memory and on one XCD.  All arrays are host memory, read during the
 * call only.
 */
typedef struct {
    int dim;                        /* 2 or 3 */
    int64_t n_vert;
    const double *xyz;              /* [n_vert][dim] */
    int64_t n_cell;
    int64_t n_face;
    const int64_t *face_vert_ptr;   /* [n_face + 1] CSR offsets into face_vert */
    const int64_t *face_vert;
    const int64_t *face_owner;      /* [n_face] in [0, n_cell) */
    const int64_t *face_neigh;      /* [n_face] in [0, n_cell) or -1 */
    const int32_t *face_bc;         /* [n_face] */
    const double *face_shift;       /* [n_face][dim] or NULL */
    const int32_t *colour;          /* [n_cell] or NULL */
    int64_t order_tile;             /* cells per ordering tile; 0 = default; < 0 is CGKS_EINVAL */
} cgks_face_mesh_desc;

#define CGKS_ORDER_TILE_DEFAULT 4096

typedef struct {
    int dim, n_colour;
    int64_t n_cell, n_face, n_gp, n_boundary_face;
    int64_t n_planar_faces;         /* faces whose Gauss points share one normal (all 2-D edges and
                                       triangles; flat quads): their face records are shorter */
} cgks_mesh_info;

/*
 * Flow and solver parameters of one case.  Non-dimensional gas with R = 1:
 * T = p / rho.  mu is the constant dynamic viscosity (0 = inviscid); the
 * collision time is tau = mu / p at each Gauss point (Sec. 2.2).  Pr != 1
 * adds (1/Pr - 1) times the Fourier heat flux of the interface state to the
 * energy flux (BGK alone gives Pr = 1).  cfl_high sets the global explicit
 * step dt = cfl_high min_i h_i / (|U_i| + c_i + 2 mu / (rho_i h_i)); cfl_low
 * sets the local steps of the low level (the paper uses 0.3-0.5 and 1000,
 * Sec. 4).  n_implicit backward-Euler steps of n_sweeps point-relaxation
 * sweeps each (6 and 2 in the paper, Sec. 3).  dt_fixed > 0 replaces the
 * CFL rule by a fixed global step.  explicit_only = 1 runs the high-order
 * level alone (the explicit CGKS the paper compares against).
 */
typedef struct {
    double gamma, mu, Pr, T_wall;
    double W_inf[5];                /* free-stream conservative state (first dim+2 used) */
    double cfl_high, cfl_low;
    int32_t n_implicit, n_sweeps;
    int32_t time_scheme;            /* CGKS_S2O4 or CGKS_S1O2 */
    int32_t explicit_only;
    double dt_fixed;
    int32_t low_flux;               /* first-order flux of the low-order level (Sec. 3; Sec. 4 compares
                                       the two): CGKS_LOW_KFVS (0, the paper's default) or CGKS_LOW_LF,
                                       1/2 (F_n(U_L) + F_n(U_R)) - 1/2 lam_f (U_R - U_L) with the face's
                                       spectral radius lam_f of the implicit operator; per case */
    int32_t flux_kind;              /* high-order flux (Sec. 2.2): CGKS_FLUX_SMOOTH (0), the simplified
                                       solution for smooth flow (Eq. 2nd-smooth-flux), or CGKS_FLUX_FULL,
                                       the full time-dependent solution (Eq. 2nd-flux) that Sec. 4 uses for
                                       transonic and supersonic flow: an exp(-t/tau_n) blend of the
                                       equilibrium part and the left/right free-transport parts with
                                       tau_n = tau + |p_l - p_r| / (p_l + p_r) dt; the time marching takes
                                       its flux and interface state as linear fits in t over [0, dt/2] and
                                       [0, dt].  Equal left and right data give the smooth solution. */
    double weno_eps;                /* 0: linear reconstruction weights (smooth flow, Sec. 4); > 0:
                                       nonlinear WENO-type weights with this epsilon (the paper uses 1e-2
                                       and 1e-6): candidates are the quadratic fit and one linear fit per
                                       face neighbour (its average and gradient), weights proportional to
                                       gamma_k / (eps + beta_k)^2 with gamma_0 = 0.95 */
    double area_ref;                /* reference area of the drag coefficient (Sec. 4: the sphere's
                                       pi D^2 / 4, the cylinder's D per unit span); 0: none */
} cgks_params;

typedef struct cgks_mesh cgks_mesh;
typedef struct cgks_batch cgks_batch;

/* Build the faces (cell-based form) and their Gauss points (3 per
   triangle, 4 per quadrilateral with a normal at each point, 2 per 2-D
   edge), cell volumes, centroids and second moments, the reconstruction
   operators, the multicolour classes (the caller's, or largest-degree-first
   greedy colouring with classes numbered by size) and the library cell
   order (tiles of order_tile cells along a Morton curve of the centroids,
   colour-major inside each tile).  Host work only.  *out receives a handle
   (free with cgks_mesh_destroy).  Errors: CGKS_EINVAL (null/size/type),
   CGKS_EMESH (face shared by more than two cells, cell face neither shared
   nor listed as boundary, boundary face matching no cell face, bad
   periodic pairing, non-positive volume, a reconstruction stencil that
   cannot fix the quadratic, an invalid caller colouring), CGKS_ENOMEM. */
cgks_status cgks_mesh_create(const cgks_mesh_desc *desc, cgks_mesh **out);
/* The same from a face-based description. */
cgks_status cgks_mesh_create_faces(const cgks_face_mesh_desc *desc, cgks_mesh **out);
cgks_status cgks_mesh_query(const cgks_mesh *mesh, cgks_mesh_info *info);
/* lib_to_caller[n_cell]: caller cell id of each library cell; colour[n_cell]
   (may be NULL): colour of each caller cell. Host arrays. */
cgks_status cgks_mesh_permutation(const cgks_mesh *mesh, int64_t *lib_to_caller, int32_t *colour);
/* Cell geometry in caller order (host arrays, any may be NULL): vol[n_cell],
   centroid[n_cell][dim], h[n_cell] = 2 dim |V| / sum_f S_f. */
cgks_status cgks_mesh_geometry(const cgks_mesh *mesh, double *vol, double *centroid, double *h);
cgks_status cgks_mesh_destroy(cgks_mesh *mesh);

/* A batch is n_case (mesh, params) pairs stepped together: every kernel
   launch covers all cases; per-case reductions (dt, Res) never mix cases.
   The meshes must outlive the batch.  precision: CGKS_FP64 (everything in
   FP64); CGKS_MIXED32: reconstruction coefficients, interface states, the
   gas-kinetic flux, the face sums and the relaxation sweeps (increments dU
   and their flux changes) in FP32; cell averages, gradients, the stage
   accumulation, R1's accumulation, the low-level state U, its KFVS flux and
   right-hand side, Res and dt in FP64; CGKS_MIXED32_R64: as CGKS_MIXED32,
   but the residual pass R1 (reconstruction, flux, face sums) in FP64, so
   the FP32 parts no longer perturb the cycle's fixed point (R1 = 0) and
   the residual falls below the FP32 noise floor.  Errors: CGKS_EINVAL,
   CGKS_ENOMEM. */
cgks_status cgks_batch_create(const cgks_mesh *const *meshes, const cgks_params *params, int32_t n_case,
                              int32_t precision, cgks_batch **out);
/* A pool: a batch with capacities instead of cases, for continuous
   batching.  Up to max_cases cases live in it at once; each admitted case
   holds one contiguous range of cells, faces, Gauss points and boundary
   faces (the counts cgks_mesh_query reports) until it is released, so the
   capacities are the pool's HBM footprint (cgks_batch_query gives the
   bytes).  Every launch covers all admitted cases; entities of free ranges
   are skipped.  A case gives bitwise the same results in a pool, alone or
   among others admitted and released around it (no reduction or sweep
   block spans two cases, and their shapes depend only on the case).  All
   cases of a pool share dim, precision, n_implicit, n_sweeps, time_scheme
   and explicit_only.  Arrays the library exposes in library cell order
   ([nv][cells] residuals) use max_cells as the row length. */
typedef struct {
    int32_t dim, precision, max_cases;
    int64_t max_cells, max_faces, max_gauss_points, max_boundary_faces;
    int32_t n_implicit, n_sweeps, time_scheme, explicit_only;
} cgks_pool_desc;
cgks_status cgks_pool_create(const cgks_pool_desc *desc, cgks_batch **out);
/* Admit a case into a free slot of a bound pool (the mesh must outlive its
   stay): uploads its geometry into free ranges found first-fit, zeroes its
   state and marks it active; *slot receives the case index to use with the
   state, residual and report calls.  Upload an initial state next.
   CGKS_ENOMEM when no slot or no free range of some entity type is large
   enough (the caller keeps the request waiting; nothing changed),
   CGKS_EINVAL on a dim or parameter mismatch, CGKS_EUNSUPPORTED for a mesh
   with more than 16 colours.  Synchronous on stream; drops a captured
   graph. */
cgks_status cgks_batch_admit(cgks_batch *batch, const cgks_mesh *mesh, const cgks_params *params, int32_t *slot,
                             void *stream);
/* Stop and remove the case in slot; its ranges become free.  Download its
   state first if needed.  Synchronous on stream; drops a captured graph.
   CGKS_EINVAL for a free slot. */
cgks_status cgks_batch_release(cgks_batch *batch, int32_t slot, void *stream);

/* Slots and cell capacity of a batch or pool (the row length of the
   [nv][cells] library-order arrays). */
cgks_status cgks_batch_capacity(const cgks_batch *batch, int32_t *max_cases, int64_t *max_cells);
/* Whether slot holds a case, the library index of its first cell (-1 when
   free) and its cell count. */
cgks_status cgks_batch_slot_info(const cgks_batch *batch, int32_t slot, int32_t *live, int64_t *cell_offset,
                                 int64_t *n_cell);

/* Device bytes the batch needs (geometry, state, work arrays). */
cgks_status cgks_batch_query(const cgks_batch *batch, size_t *device_bytes);
/* Bind a caller-owned device buffer of at least cgks_batch_query bytes
   (256-byte aligned) and upload the geometry into it on stream. */
cgks_status cgks_batch_bind(cgks_batch *batch, void *dev_buf, size_t bytes, void *stream);
cgks_status cgks_batch_destroy(cgks_batch *batch);

/* Set / read the state of case c from host arrays in caller cell order:
   W_host [dim+2][n_cell], dW_host [dim][dim+2][n_cell] (NULL = zero on
   upload, skipped on download).  Synchronous on stream.  The copy goes
   through a pinned host buffer that the batch keeps, grown to the largest
   case transferred and freed with the batch (CGKS_EDEVICE if it cannot be
   allocated). */
cgks_status cgks_state_upload(cgks_batch *batch, int32_t c, const double *W_host, const double *dW_host,
                              void *stream);
cgks_status cgks_state_download(cgks_batch *batch, int32_t c, double *W_host, double *dW_host, void *stream);
/* Device pointer to case c's state records: n_cell records (library order)
   of rec_len = (dim+2)(dim+1) doubles each, W[v] then dW[axis][v].  The
   records of a batch are contiguous, case after case. */
cgks_status cgks_state_device(cgks_batch *batch, int32_t c, double **rec, int32_t *rec_len, int64_t *n_cell);

/* One high-order stage on every case, in place (Secs. 2.2-2.4).  stage 0
   first computes the global step dt of each case from W, keeps W^n, and
   applies the first S2O4 stage (or the whole S1O2 step); stage 1 applies the
   second S2O4 stage (CGKS_EINVAL for S1O2 cases). */
cgks_status cgks_highorder_stage(cgks_batch *batch, int32_t stage, void *stream);

/* Residuals (Sec. 3).  kind = CGKS_RESIDUAL_HIGH: R1 = -sum_f s sum_g wJ
   (F0 + dt/2 F_t), the time-averaged high-order net flux at the current
   state with the dt of the last stage 0 (step 2 of the cycle), extensive.
   kind = CGKS_RESIDUAL_LOW: R0 = -sum_f s S_f F_KFVS, the first-order net
   flux at the current state.  Both write out_dev [batch cells][dim+2] in the
   library's batch-concatenated layout (case c starts at its cell offset,
   variable-major within the case: out_dev + 5*off_c is [nv][n_c]).
   kind = CGKS_RESIDUAL_NORM: out_dev[c] = Res of the last cycle of case c,
   sum |rho_new - rho_old| / sum rho_old (Sec. 4). */
cgks_status cgks_residual(cgks_batch *batch, int32_t kind, double *out_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, serving loops or harnesses that forbid hipMalloc): the
   transferred residual R1 of cgks_residual(CGKS_RESIDUAL_HIGH), from the
   same kernels and bitwise the same, but the residual pass's work arrays
   (boundary ghost data, reconstruction records, face sums) live in a fixed
   64 MiB array of the library on the current device instead of the batch
   arena.  Batches whose launch extents need more get CGKS_ENOMEM (the pass
   needs about 1.2 KB per cell in 3-D FP64, 0.5 KB in 2-D, less in
   MIXED32).  The batch must be bound on the current device (CGKS_EINVAL
   otherwise).  out_dev: [dim+2][max_cells] as for cgks_residual; entries of
   cells outside any case are left untouched.  Calls no hipMalloc, hipFree
   or other allocating routine (kernel timing is not recorded for this
   call).  Each device holds one copy of the array, shared by every call on
   it: calls that overlap on one device race, so serialise them (one stream,
   or events).  The first call on a device looks up the array's address
   (CGKS_EDEVICE if that fails). */
cgks_status cgks_residual_high_noalloc(cgks_batch *batch, double *out_dev, void *stream);

/* Low level of the cycle (Sec. 3 steps 2-5) on every case: W_p0 = W,
   forcing S = R1 - R0(W_p0), n_implicit backward-Euler steps solved by
   multicolour point relaxation, W += U - W_p0.  R1_dev as written by
   cgks_residual(CGKS_RESIDUAL_HIGH).  Also computes Res (cgks_residual
   CGKS_RESIDUAL_NORM) against W^n of the last stage 0. */
cgks_status cgks_lowlevel_smooth(cgks_batch *batch, const double *R1_dev, void *stream);

/* One full two-level cycle on every case (stage 0, stage 1 for S2O4, R1,
   low level; high-order step only when explicit_only).  res_dev (may be
   NULL) receives Res per case. */
cgks_status cgks_cycle(cgks_batch *batch, double *res_dev, void *stream);

/* Capture n_cycles (1..64) consecutive cycles of every case into a HIP
   graph held by the batch (replacing any previous one).  Capture runs on a
   private stream after the work queued on `stream`; the captured kernels
   read dt, Res and the parameters from device memory, so replays need no
   host work.  The graph also records each cycle's Res per case. */
cgks_status cgks_graph_create(cgks_batch *batch, int32_t n_cycles, void *stream);
/* Replay the captured cycles on stream.  res_history_dev (may be NULL)
   receives [n_cycles][n_case] Res values (device).  CGKS_EINVAL when no
   graph has been captured. */
cgks_status cgks_graph_launch(cgks_batch *batch, double *res_history_dev, void *stream);
cgks_status cgks_graph_destroy(cgks_batch *batch);

typedef struct {
    int32_t max_cycles;
    double tol;            /* stop a case when Res_k / Res_1 <= tol (tol_abs = 0) ... */
    int32_t tol_abs;       /* ... or when Res_k <= tol (tol_abs = 1) */
    int32_t check_every;   /* cycles between host checks of Res (>= 1) */
    double *res_history;   /* optional host [n_case][max_cycles] */
} cgks_solve_opts;

typedef struct {
    int32_t cycles;        /* cycles applied to the case's state: the stop is
                              taken at a check, so this is a multiple of
                              check_every (or max_cycles) */
    int32_t converged;     /* the tolerance was met at some cycle of the last block */
    double res_first, res_last;
    cgks_status status;    /* CGKS_OK, CGKS_ENOTCONV, CGKS_ENONPHYS, CGKS_EDIVERGED */
    double force[3];       /* wall force at the start of the case's last cycle (see cgks_wall_force) */
    double cd;             /* drag coefficient of that force (see cgks_wall_force; NaN without area_ref) */
} cgks_solve_report;

/* Cycle until every case meets its tolerance or max_cycles; report[n_case]
   (host).  Res is checked on the host every check_every cycles; with
   2 <= check_every <= 8 those cycles run as one captured graph (this
   replaces a graph made by cgks_graph_create).  A case that meets its tolerance, or is
   found non-physical or diverging, at any cycle of a block stops being
   updated at the check that ends the block; res_history holds every cycle
   it ran. */
cgks_status cgks_solve(cgks_batch *batch, const cgks_solve_opts *opts, cgks_solve_report *report, void *stream);

/* Force of the gas on the walls of each case (Sec. 4, sphere and cylinder
   drag): the sum over slip and no-slip boundary faces of the face-quadrature
   sum of the momentum components of the flux at t = 0 (F0), that is pressure
   plus viscous stress, with the face normal pointing out of the fluid.  It
   is taken in the first high-order pass (stage 0) of every cycle, at the
   state the cycle starts from; a case frozen by cgks_solve keeps the force
   of its last cycle.  force: host [n_case][3] (the z entry is 0 in 2-D);
   cd (may be NULL): host [n_case], the drag coefficient
   force . e_inf / (1/2 rho_inf |U_inf|^2 area_ref) with e_inf the
   free-stream direction (Sec. 4 tables), NaN where area_ref is 0 or the
   free stream is at rest.  Written after the work queued on stream has
   finished.  MIXED32 batches sum FP32 face sums (in FP64).  CGKS_EINVAL on
   a NULL force or an unbound batch. */
cgks_status cgks_wall_force(cgks_batch *batch, double *force, double *cd, void *stream);

/* Pick the launch shapes of this batch by measurement (the batching
   autotuner): threads per block of the face Gauss-point flux, the cell
   gather and update, the low-level face flux and the low-level cell setup
   (64, 128 or 256 each), and cells per block of the relaxation sweep (16,
   32 or 64), each the fastest of three timed launches on the batch's own
   data and current state.  Results never depend on these shapes (no
   reduction crosses a face's or cell's lane group), so a tuned batch steps
   bitwise like an untuned one.  The timed launches write only work arrays
   (reconstruction records, face sums, R1, the low-level arrays), never W or
   grad W.  choice (host, may be NULL) receives the five picks in that
   order.  Synchronous on stream; drops a captured graph.  CGKS_EINVAL for
   an unbound batch or a pool without cases. */
cgks_status cgks_batch_autotune(cgks_batch *batch, int32_t *choice, void *stream);

/* Kernel timing.  enable = 1 brackets the kernel launches of the batch with
   pairs of HIP events recorded on the launch stream: one pair per launch,
   except that the back-to-back colour passes of one implicit step share
   one pair (their span, gaps between the passes included).  The reduction
   kinds count their final per-case kernel with them, and RECON counts the
   boundary ghost pre-pass with the reconstruction.  cgks_timing_read
   synchronises those events and returns, per kernel kind, the summed
   duration in milliseconds and the number of launches of the kind's main
   kernel since the previous read (then starts a new interval).  ms and
   launches are host arrays of CGKS_KERNEL_KINDS entries. */
enum {
    CGKS_K_DT = 0,        /* global time-step reduction */
    CGKS_K_RECON = 1,     /* compact reconstruction */
    CGKS_K_FLUX = 2,      /* gas-kinetic flux at face Gauss points */
    CGKS_K_CELL = 3,      /* Gauss-Green gather, stage update, R1 */
    CGKS_K_LOWFACE = 4,   /* first-order KFVS face flux and spectral radius */
    CGKS_K_LOWCELL = 5,   /* forcing and implicit-step setup */
    CGKS_K_SWEEP = 6,     /* one colour pass of point relaxation */
    CGKS_K_PROLONG = 7,   /* prolongation and residual norm */
    CGKS_KERNEL_KINDS = 8
};
cgks_status cgks_timing_enable(cgks_batch *batch, int32_t enable);
cgks_status cgks_timing_read(cgks_batch *batch, double *ms, int64_t *launches);

const char *cgks_status_string(cgks_status s);

#ifdef __cplusplus
}
#endif
#endif /* CGKS_H */
