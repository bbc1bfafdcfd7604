/*
 * fk.h -- C ABI of the MI355X stochastic interface solver (libfk.so).
 *
 * The library evaluates, at interface nodes of a sub-domain decomposition of
 * the unit square, the Feynman-Kac (probabilistic) representation of the
 * relaxed Winslow mesh equations
 *
 *     xi_t  = -(1/w) grad w . grad xi  + Laplacian xi,
 *     eta_t = -(1/w) grad w . grad eta + Laplacian eta        (Sect. 2, eq. (3))
 *
 * by Monte-Carlo: each node launches n_paths Euler-Maruyama paths of
 * dX = -(grad w / w) ds + sqrt(2) dW (eq. (7a)); a path scores the boundary
 * data where it first leaves the square, or the initial data where it is at
 * the end of the time horizon (eqs. (5), (7b); Sect. 4).  One path set serves
 * xi and eta, which share the drift.  Sub-domain meshes are then obtained by
 * implicit finite-difference solves with the interface values as Dirichlet
 * data (Sect. 4, deterministic single-domain solver).
 *
 * Conventions, for every call:
 *  - Arrays marked "device" are caller-owned device memory; arrays marked
 *    "host" are caller-owned host memory read before the call returns.  The
 *    library keeps no pointer after a call returns, except inside the opaque
 *    handles documented below.
 *  - Calls are asynchronous and ordered on the given HIP stream, unless
 *    stated otherwise.  Outputs are valid once the stream is synchronised.
 *  - Every call returns an int status.  Arguments are validated before any
 *    work is queued; on error nothing is queued, outputs are unspecified and
 *    fk_last_error() describes the failure.  No C++ exception crosses the ABI.
 *  - Errors of work already queued (device faults) surface as FK_E_DEVICE at
 *    the next call that synchronises (fk_sync).
 */
#ifndef FK_H
#define FK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FK_OK 0
#define FK_E_INVAL (-1)        /* bad shape, t < 0, dt <= 0, n_paths < 2, NaN parameter, host node outside
                                  the square (device nodes are checked by the kernels: NaN results) */
#define FK_E_NODEVICE (-2)     /* no usable GPU */
#define FK_E_NOMEM (-3)        /* workspace too small / allocation failed */
#define FK_E_DEVICE (-4)       /* HIP runtime error (launch failure, fault) */
#define FK_E_UNSUPPORTED (-5)  /* valid request this build does not implement */

/* Density kinds: w(tau, x, y) of the mesh equations (Sect. 2; Sect. 5). */
#define FK_DENSITY_CONST 0        /* w = 1 */
#define FK_DENSITY_BUMP 1         /* w = 1 + amp exp(-|X - (cx,cy)|^2 / width2) */
#define FK_DENSITY_MOVING_BUMP 2  /* centre (cx + orbit_r cos(omega tau), cy + orbit_r sin(omega tau)) */
#define FK_DENSITY_TWO_BUMPS 3    /* w = 1 + amp (e1 + e2); e2 centred at (cx - orbit_r cos, cy + orbit_r sin) */
#define FK_DENSITY_RING 4         /* w = 1/rho, rho = 1 + amp exp(width2 |r^2 - 1/100|), r the distance to
                                     the moving centre: the paper's ring (Sect. 5; amp = alpha, width2 = beta) */
#define FK_DENSITY_RIDGE 5        /* w = 1 + amp exp(-(x - cx)^2 / width2) */
#define FK_DENSITY_GRID 6         /* w known only at the nodes of a grid (Sect. 4): samples grid_w; grad w by
                                     finite differences at the nodes (central inside, second-order one-sided
                                     on the edges), b = -grad w / w there, and b bilinear between the nodes
                                     (table grid_b from fk_density_grid_drift).  Static: the time mode and
                                     the analytic parameters are ignored */

/* Time argument of w along a path. */
#define FK_TIME_BACKWARD 0  /* w(t_init + t - s): the time reversal of the Feynman-Kac formula (eq. (5)) */
#define FK_TIME_FROZEN 1    /* w(t_freeze): held fixed over one mesh time step (Sect. 4) */

/* Initial / boundary data kinds (Sect. 3). */
#define FK_DATA_IDENTITY 0  /* xi = x, eta = y: the initial uniform mesh and its boundary data */
#define FK_DATA_SIN 1       /* test mode: phi = sin(pi x) sin(pi y) for both components; boundary
                               data exp(-2 pi^2 (t - s)) phi(X) extended off the square */
#define FK_DATA_ZERO 2      /* boundary data 0 */
#define FK_DATA_GRID 3      /* initial data: bilinear in (grid_n+1)^2 nodal FP64 grids; as boundary data
                               (with grid initial data and FK_SCORE_PROJECT / FK_SCORE_BRIDGE) the same
                               grids at the projected exit point, i.e. their edge nodes' data */
#define FK_DATA_EQUIDISTRIBUTED 4  /* subdomain_solve's outer boundary only: xi = 0 / 1 on the left / right
                                      edges, eta = 0 / 1 on the bottom / top edges, and on the other edges
                                      the 1-D equidistribution of w along the edge, xi(x) = int_0^x w /
                                      int_0^1 w (Sect. 3: the 1-D version of eq. (2)); the interface solve
                                      reads it from the mesh grid with FK_SCORE_EXTEND */

#define FK_SCORE_UNCLAMPED 0  /* boundary data at the first point outside the square */
#define FK_SCORE_PROJECT 1    /* ... after clamping that point onto the square */
#define FK_SCORE_EXTEND 2     /* the FK_DATA_GRID initial data continued bilinearly from its edge cells to
                                 that point: for a grid whose edge nodes hold the boundary data, the data
                                 extended by the grid's own normal slope (a first-order correction of the
                                 overshoot of the discrete exit test); needs grid initial data */
#define FK_SCORE_BRIDGE 3     /* the Brownian-bridge exit test within every step that ends inside, on top
                                 of the discrete one: the diffusion pinned at the step's two ends crosses
                                 a side at distances d0, d1 with probability exp(-d0 d1 / dt); the four
                                 sides combine as independent, a side with d0 d1 / dt > 17 counts as 0;
                                 the step's uniform is word (k & 1) of Philox(k/2, path, node,
                                 ctr3 | 4), u = ((r >> 8) + 1) 2^-24, and u < p ends the path within the
                                 step at its end point projected onto the side of largest probability.
                                 Every exit is scored at the point clamped onto the square.  For w = 1
                                 the killed chain then has the law of the killed diffusion at any step
                                 size.  Plain solves (fk_interface_solve, batches) and the martingale
                                 forms of fk_interface_solve_cv (the Dynkin form: FK_E_UNSUPPORTED) */
#define FK_SCORE_EXPONENTIAL 4  /* exponential time-stepping (Sect. 4's alternative to the fixed steps,
                                 after Jansons & Lythe 2003): step lengths D_k exponentially distributed
                                 with mean dt, D_k = -dt ln u with u = ((r >> 8) + 1) 2^-24 from word
                                 2 + (k & 1) of Philox(k/2, path, node, ctr3 | 4), the step that would
                                 pass the horizon cut at it (a path that stays inside takes
                                 1 + Poisson(t/dt) steps); given D_k the Euler-Maruyama step of that
                                 length and the bridge test of FK_SCORE_BRIDGE with D_k for dt; exits
                                 scored at the projected point.  Single solves only (the batched and
                                 control-variate solves return FK_E_UNSUPPORTED) */

/* Density parameters (plain values; for FK_DENSITY_GRID also two device arrays). */
typedef struct fk_density {
    int32_t kind;       /* FK_DENSITY_* */
    int32_t time_mode;  /* FK_TIME_* */
    double amp, width2, cx, cy, orbit_r, omega, t_freeze;
    /* FK_DENSITY_GRID only (0 / NULL otherwise): */
    int32_t grid_n;          /* grid cells per side, >= 2 */
    int32_t grid_reserved;   /* 0 */
    const double *grid_w;    /* device [(grid_n+1)^2] FP64 samples of w (> 0), row-major [j][i] at
                                (i/grid_n, j/grid_n) */
    const float *grid_b;     /* device [(grid_n+1)^2][2] FP32 nodal drift (b_x, b_y) of grid_w, written by
                                fk_density_grid_drift; 8-byte aligned.  Both arrays are read by every call
                                that takes the density and must stay unchanged until those calls finish */
} fk_density;

/* Initial and boundary data. */
typedef struct fk_data {
    int32_t init_kind;   /* FK_DATA_* */
    int32_t bdry_kind;   /* FK_DATA_IDENTITY, FK_DATA_SIN, FK_DATA_ZERO or FK_DATA_GRID (see there) */
    int32_t score_mode;  /* FK_SCORE_* */
    int32_t grid_n;      /* FK_DATA_GRID: grid cells per side, else 0 */
    double t_init;       /* PDE time at which the initial data hold */
    const double *grid_xi;   /* device, [(grid_n+1)^2] row-major [j][i], x = i/grid_n; or NULL */
    const double *grid_eta;  /* device, same layout; or NULL */
} fk_data;

/* Launch plan of the path kernel (see fk_plan_autotune).  Zero fields take defaults:
 * block 256; blocks_per_cu the kernel's occupancy (the grid is cut to no more
 * wavefronts than there are chunks); chunk 128, or for horizons of at most 64
 * steps: in fk_interface_solve (and the plain pass of fk_interface_solve_cv)
 * the largest of 256, 512, 1024, 2048 that leaves at least 8 chunks per
 * resident wavefront (28 per CU), 256 with a node mask, and 256 in the network
 * forms of fk_interface_solve_cv; for longer horizons in the control-variate
 * passes of fk_interface_solve_cv, the largest of 128, 64, 32 that leaves at
 * least 64 chunks per CU; chunk at most 2048 (FK_E_INVAL beyond);
 * node_tile 1.  The plan changes speed
 * only: results depend on the counters alone. */
typedef struct fk_plan {
    int32_t block;          /* threads per workgroup: 64, 128, 192 or 256 */
    int32_t blocks_per_cu;  /* resident workgroups per compute unit for the persistent grid */
    int32_t chunk;          /* paths handed to a wavefront per queue grab (>= 1) */
    int32_t node_tile;      /* work order: the chunks of this many consecutive nodes (in the queue's
                               cost order) interleaved, a power of two 1..256 (FK_E_INVAL otherwise);
                               1 = node by node; a last, partial tile runs node by node */
} fk_plan;

/*
 * Plan handle (launch plan + captured graph).  fk_plan_autotune times
 * fk_interface_solve on the caller's problem (with probe_paths paths per node)
 * for each candidate shape -- block 64 / 128 / 256 x chunk 32 / 128 / 512 x
 * full / half occupancy x node tile 1 / 8 -- and keeps the fastest in the
 * handle.  Results are cached per process by the device's signature and a
 * hash of the problem's shape (kinds, modes, node count, paths, steps); with
 * the environment variable FK_TUNE_CACHE naming a file they also persist
 * there.  Synchronous; allocates and frees a probe output buffer.  Every
 * candidate gives the same result: the plan changes the schedule only.
 * Pass the tuned plan to the solves with fk_plan_get.
 *
 * fk_plan_capture_begin / _end bracket any sequence of library calls on a
 * non-default stream (e.g. a whole mesh step: density samples, key points,
 * the interface solve, interpolation, the sub-domain solves, quality) and
 * keep it as the handle's executable HIP graph; nothing runs during capture.
 * A later capture of the same sequence with other arguments (another time
 * level, the other ping-pong buffers) updates the executable graph in place
 * when its topology allows (fk_plan_graph_updates counts those), else
 * replaces it.  fk_plan_replay launches it.  The captured calls must not
 * allocate (pass workspaces and outputs) and must not synchronise with the
 * host; the library records no memset into a graph.  create / set / get /
 * autotune check their arguments (FK_E_INVAL); destroy synchronises the
 * device first when a graph is held.
 */
typedef struct fk_plan_handle *fk_plan_t;
int fk_plan_create(const fk_plan *initial, fk_plan_t *out);
int fk_plan_set(fk_plan_t p, const fk_plan *plan);
int fk_plan_get(fk_plan_t p, fk_plan *out);
int fk_plan_autotune(fk_plan_t p, const fk_density *w, const fk_data *d, const double *pts, const uint8_t *mask,
                     int64_t n_nodes, double t, double dt, int64_t probe_paths, uint64_t seed, void *workspace,
                     size_t workspace_bytes, hipStream_t stream);
int fk_plan_capture_begin(fk_plan_t p, hipStream_t stream);
int fk_plan_capture_end(fk_plan_t p, hipStream_t stream);
int fk_plan_replay(fk_plan_t p, hipStream_t stream);
int fk_plan_graph_updates(fk_plan_t p);
void fk_plan_destroy(fk_plan_t p);

/*
 * Samples of an analytic density at the nodes of an n-cell grid (for the
 * grid data path of Sect. 4: w available at grid points only).
 *
 *   w      analytic density (kind FK_DENSITY_CONST .. FK_DENSITY_RIDGE)
 *   tau    PDE time at which w is sampled (the time mode is ignored)
 *   n      cells per side, >= 1
 *   w_out  device [(n+1)^2] FP64, row-major [j][i]: w(tau, i/n, j/n)
 *
 * FK_E_INVAL for a grid density, n < 1 or NULL output.
 */
int fk_density_sample(const fk_density *w, double tau, int32_t n, double *w_out, hipStream_t stream);

/*
 * Nodal drift table of a grid density (Sect. 4: the derivatives in grad w
 * are approximated by finite differences at the grid points): at node
 * (i, j), w_x by the central difference (w[i+1] - w[i-1]) / 2h for
 * 0 < i < n and by the second-order one-sided differences
 * (-3 w[0] + 4 w[1] - w[2]) / 2h, (3 w[n] - 4 w[n-1] + w[n-2]) / 2h on the
 * edges (the same in y), h = 1/n; b = -grad w / w, computed in FP64 and
 * stored as FP32 pairs.
 *
 *   grid_w  device [(n+1)^2] FP64 samples, row-major [j][i]
 *   n       cells per side, >= 2
 *   grid_b  device [(n+1)^2][2] FP32, 8-byte aligned (output)
 *
 * FK_E_INVAL for n < 2, NULL or misaligned arrays.  Samples <= 0 give
 * non-finite or sign-flipped drifts: the caller supplies w > 0.
 */
int fk_density_grid_drift(const double *grid_w, int32_t n, float *grid_b, hipStream_t stream);

/*
 * Bytes of device workspace fk_interface_solve needs for n_nodes nodes (queue
 * counters, the level and node tables and the per-node estimator sums: about
 * 144 B per node, whatever n_paths).  Returns 0 for invalid sizes.
 */
size_t fk_interface_workspace_bytes(int64_t n_nodes, int64_t n_paths);

/*
 * Monte-Carlo interface solve (eqs. (5)-(7); Sect. 4).
 *
 * For node i (0 <= i < n_nodes) at pts[2i], pts[2i+1] (device, FP64, in the
 * closed unit square), and with mask != NULL only where mask[i] != 0, the
 * library runs n_paths Euler-Maruyama
 * paths over the horizon t with step dt (K = ceil(t/dt) steps, the last one
 * t - (K-1) dt), drawing normals from Philox4x32-10 with key = seed and
 * counter (step/2, path, i, (level_id << 4) | 0), two normals per step from
 * one Box-Muller transform.  Path arithmetic is FP32.  The estimator (Sect. 4:
 * the expectation replaced by the mean over the paths) is summed inside the
 * path kernel as exact fixed-point integers -- each score s (relative to the
 * node's shift, see scores) rounded to a multiple of 2^-48 and s^2 to one of
 * 2^-45 -- so results are bitwise independent of the launch plan and of which
 * lane ran which path; mean, sample variance (N - 1) and standard error are
 * then formed in FP64.  Scores must satisfy |s| < 512 (every data kind of
 * this header keeps them within ~1.5); a node with a non-finite or larger
 * score gets NaN outputs.
 *
 *   pts            device [n_nodes][2] FP64, 8-byte aligned.  The coordinates
 *                  stay on the device (the node tables are built there, nodes
 *                  queued in decreasing expected cost), so a caller can solve
 *                  for node lists it computed on the device without a host
 *                  synchronisation.  They are checked by the kernels: a node
 *                  outside the closed square, or with a NaN coordinate, gets
 *                  NaN means and standard errors (and no paths)
 *   mask           device [n_nodes] uint8 or NULL: solve only the nodes with
 *                  mask[i] != 0; the other nodes' outputs (means, standard
 *                  errors, steps, per-path rows) are left untouched.  Node i
 *                  keeps its Philox counter word i, so a masked solve gives
 *                  bitwise the full solve's results at its nodes
 *   xi, eta        device [n_nodes] FP64  sample means
 *   se_xi, se_eta  device [n_nodes] FP64  standard errors sqrt(var/n_paths)
 *   exit_step      device [n_nodes][n_paths] int32 or NULL: step after which
 *                  the path left the square (1..K), -1 if it never did
 *   scores         device [n_nodes][n_paths][2] FP32 or NULL: per-path score
 *                  minus the node's shift (the FP32 rounding of the node
 *                  coordinates when initial and boundary data are both the
 *                  identity, 0 otherwise); written only when given (the
 *                  estimator itself keeps no per-path data)
 *   steps          device [n_nodes] int64 or NULL: Euler-Maruyama steps taken
 *                  per node
 *   total_steps    device [1] uint64 or NULL: steps taken over all nodes
 *   plan           launch plan or NULL for the default
 *   workspace      device, at least fk_interface_workspace_bytes() bytes,
 *                  256-byte aligned; owned by the caller, must not be used by
 *                  other work until the stream passes this call
 */
int fk_interface_solve(const fk_density *w, const fk_data *d,
                       const double *pts, const uint8_t *mask, int64_t n_nodes,
                       double t, double dt, int64_t n_paths, uint64_t seed, uint32_t level_id,
                       double *xi, double *eta, double *se_xi, double *se_eta,
                       int32_t *exit_step, float *scores, int64_t *steps, uint64_t *total_steps,
                       const fk_plan *plan, void *workspace, size_t workspace_bytes,
                       hipStream_t stream);

/*
 * fk_interface_solve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments and results, without the workspace.  Its
 * tables and sums live in a fixed device array inside the library (8 MiB per
 * GPU, held until the process ends; fk_interface_noalloc_max_bytes() returns
 * its size), which bounds n_nodes to about 58,000 -- larger requests fail
 * with FK_E_NOMEM before anything is queued.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine); what must start at
 * zero is cleared by kernels on the stream.  Every call on one GPU uses that
 * GPU's one array: calls that overlap on a GPU (other streams, other host
 * threads) race and corrupt each other's results; the array keeps the last
 * call's contents.
 */
size_t fk_interface_noalloc_max_bytes(void);
int fk_interface_solve_noalloc(const fk_density *w, const fk_data *d, const double *pts, const uint8_t *mask,
                               int64_t n_nodes, double t, double dt, int64_t n_paths, uint64_t seed,
                               uint32_t level_id, double *xi, double *eta, double *se_xi, double *se_eta,
                               int32_t *exit_step, float *scores, int64_t *steps, uint64_t *total_steps,
                               const fk_plan *plan, hipStream_t stream);

/*
 * Batched interface solves: several time levels, each with its own density
 * parameters, horizon and node slice (e.g. a different sub-domain layout),
 * run as one persistent launch over one work queue.  Every level has the
 * semantics of one fk_interface_solve call on its nodes with the same seed,
 * dt, n_paths and data, and its own level_id, so the per-node results are
 * bitwise those of the single calls.  All levels must share the density kind
 * and time mode (FK_E_UNSUPPORTED otherwise).
 */
typedef struct fk_level {
    fk_density w;         /* density of the level */
    double t;             /* horizon of the level */
    double t_init;        /* PDE time of the level's initial data */
    int64_t node_offset;  /* first node of the level in pts and in the outputs */
    int64_t n_nodes;      /* nodes of the level; the slices must tile [0, n_total) */
    uint32_t level_id;    /* Philox counter tag, < 2^28 */
    uint32_t reserved;
} fk_level;

typedef struct fk_batch *fk_batch_t;

/* Builds the device tables (cost-ordered nodes, level constants) once, on the
 * host: pts is host [n_total][2] here (checked: FK_E_INVAL for a node outside
 * the closed square); the data's grid pointers must outlive the batch.
 * Allocates device memory for the tables (freed by fk_batch_destroy). */
int fk_batch_create(const fk_level *levels, int32_t n_levels, const double *pts, int64_t n_total,
                    const fk_data *d, double dt, int64_t n_paths, uint64_t seed, fk_batch_t *out);
/* Device workspace of fk_batch_run: counters and per-node estimator sums (0 for NULL). */
size_t fk_batch_workspace_bytes(fk_batch_t b);
int fk_batch_set_plan(fk_batch_t b, const fk_plan *plan);
int fk_batch_get_plan(fk_batch_t b, fk_plan *plan);
/* Times the launch with probe_paths paths per node for each candidate shape
 * (as fk_plan_autotune: block x chunk x occupancy x node tile; chunk 32 only
 * when the batch's n_paths is below 16 x probe_paths, since a short probe
 * does not show the queue traffic of small grabs at full size), keeps the
 * fastest as the batch's plan and returns it in *chosen (may be NULL).
 * Results are cached like fk_plan_autotune's (device signature + shape hash;
 * FK_TUNE_CACHE).  Synchronous; allocates and frees a small probe output
 * buffer.  Every candidate computes the same result: the plan only changes
 * the schedule. */
int fk_batch_autotune(fk_batch_t b, int64_t probe_paths, void *workspace, size_t workspace_bytes,
                      hipStream_t stream, fk_plan *chosen);
/* Outputs as in fk_interface_solve, over n_total nodes in node-list order. */
int fk_batch_run(fk_batch_t b, double *xi, double *eta, double *se_xi, double *se_eta, int32_t *exit_step,
                 float *scores, uint64_t *total_steps, void *workspace, size_t workspace_bytes,
                 hipStream_t stream);
/* Captures fk_batch_run with these buffers into a HIP graph (stream must not
 * be the default stream; nothing runs during capture); fk_batch_replay
 * launches it.  The captured sequence clears its counters with a kernel, so
 * replays are independent. */
int fk_batch_capture(fk_batch_t b, double *xi, double *eta, double *se_xi, double *se_eta, int32_t *exit_step,
                     float *scores, uint64_t *total_steps, void *workspace, size_t workspace_bytes,
                     hipStream_t stream);
int fk_batch_replay(fk_batch_t b, hipStream_t stream);
void fk_batch_destroy(fk_batch_t b);

/*
 * Deterministic sub-domain solves (Sect. 4): the unit square's nodal grid
 * x = i/N, y = j/N is split into px x py sub-domains of mx x my cells
 * (mx = N/px, my = N/py; px and py divide N, mx, my >= 2).  With the
 * interface values as Dirichlet data, every sub-domain takes one
 * backward-Euler step of length dt_mesh of the relaxed Winslow system (Sect.
 * 2, eq. (3)), central differences, density frozen at t_w:
 *   (u - u^n)/dt_mesh = Laplacian_h u + b . grad_h u,  b = -grad w / w.
 * dt_mesh = +INFINITY solves the steady (elliptic) system of eq. (2),
 * Laplacian_h u + b . grad_h u = 0; xi_n / eta_n are then not read (may be
 * NULL).
 * Each sub-domain system is solved by banded LU without pivoting, in FP64
 * (unknowns numbered along the shorter side first, so the half-bandwidth is
 * min(mx, my) - 1); xi and eta share the factorisation.  Requires
 * |b| h / 2 < 1 (checked from the density's bound; FK_E_UNSUPPORTED
 * otherwise) and min(mx, my) <= 128 (FK_E_UNSUPPORTED).  A grid density
 * (FK_DENSITY_GRID) must be sampled on this mesh's grid (grid_n == N, else
 * FK_E_INVAL): its FP64 finite-difference drift is taken at the nodes, the
 * equidistributed edge data integrates w as linear between the nodes, and
 * |b| h / 2 = |w[i+1] - w[i-1]| / (4 w[i]) < 1 is the caller's to ensure (the
 * samples stay in device memory).
 *   xi_n, eta_n        device [(N+1)^2] FP64, row-major [j][i]: the mesh at t^n
 *   iface_xi/eta       device FP64 [(px-1)(N-1) + (py-1)(N-px)], interface
 *                      nodes in canonical order (vertical lines x = a/px with
 *                      y = j/N ascending, then horizontal lines y = c/py with
 *                      x = i/N ascending, without their crossings)
 *   bdry_kind          FK_DATA_IDENTITY (xi = x, eta = y), FK_DATA_ZERO or
 *                      FK_DATA_EQUIDISTRIBUTED (at t_w) on the outer boundary
 *   xi_out, eta_out    device [(N+1)^2] FP64: the new mesh (boundary, interface
 *                      and sub-domain interiors); must not alias xi_n / eta_n
 *   workspace          device, subdomain_workspace_bytes_rect(px, py, N)
 *                      bytes, 256-B aligned (0 for an unsupported layout)
 * FK_E_INVAL for px, py < 1, N outside [2, 65535], px or py not dividing N,
 * sub-domains under 2 cells a side, NULL arrays.
 */
size_t subdomain_workspace_bytes_rect(int32_t px, int32_t py, int32_t n_cells);
int subdomain_solve_rect(const fk_density *w, double t_w, double dt_mesh, int32_t px, int32_t py, int32_t n_cells,
                         int32_t bdry_kind, const double *xi_n, const double *eta_n, const double *iface_xi,
                         const double *iface_eta, double *xi_out, double *eta_out, void *workspace,
                         size_t workspace_bytes, hipStream_t stream);
/* The square layout: px x px sub-domains of m x m cells, N = px m. */
size_t subdomain_workspace_bytes(int32_t px, int32_t m);
int subdomain_solve(const fk_density *w, double t_w, double dt_mesh, int32_t px, int32_t m, int32_t bdry_kind,
                    const double *xi_n, const double *eta_n, const double *iface_xi, const double *iface_eta,
                    double *xi_out, double *eta_out, void *workspace, size_t workspace_bytes,
                    hipStream_t stream);

/*
 * Outer boundary data of one mesh step on an n-cell grid (the values the
 * sub-domain solve writes to the boundary nodes): the 4n edge nodes of
 * xi_out / eta_out (device [(n+1)^2] FP64, row-major [j][i]) are set, the
 * rest is untouched.  bdry_kind as for subdomain_solve (FK_DATA_IDENTITY,
 * FK_DATA_ZERO, FK_DATA_EQUIDISTRIBUTED with w frozen at t_w); a grid density
 * must have grid_n == n.  The equidistributed data needs a device workspace
 * of fk_boundary_workspace_bytes(n) bytes, 256-byte aligned (else it may be
 * NULL).  Used to supply the line ends of fk_interface_interpolate.
 */
size_t fk_boundary_workspace_bytes(int32_t n);
int fk_boundary_data(const fk_density *w, double t_w, int32_t n, int32_t bdry_kind, double *xi_out, double *eta_out,
                     void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Key points on the interfaces (Sect. 4, further speed-up; Sect. 5): the
 * stochastic solution is needed only near the maxima and minima of rho_x,
 * rho_xx along horizontal interfaces and rho_y, rho_yy along vertical ones;
 * here rho = 1/w.  On each interface line of px x px sub-domains
 * (N = px m), from rho at the line's nodes k = 0 .. N, the unscaled central
 * differences f1_k = rho_{k+1} - rho_{k-1} and
 * f2_k = (rho_{k+1} + rho_{k-1}) - 2 rho_k at k = 1 .. N-1; node k
 * (2 <= k <= N-2) is a key point where f1 or f2 has a discrete extremum
 * (f_k > f_{k-1} and f_k >= f_{k+1}, or f_k < f_{k-1} and f_k <= f_{k+1}) with
 * |f_k| >= tol max |f| over the line.  Crossings of interface lines are key
 * points, and a gap of g > max_gap positions between consecutive knots (key
 * points and the line's two ends) gets ceil(g / max_gap) - 1 more key points
 * at prev + floor(r g / q).
 *
 *   grid_w   device [(N+1)^2] FP64 samples of w > 0 at the step's density time,
 *            row-major [j][i] (fk_density_sample, or a grid density's samples)
 *   mask     device [n_iface] uint8, canonical interface order (output):
 *            1 at key points, 0 elsewhere
 *
 * FK_E_INVAL for px < 2, m < 2, px m > 8192, tol < 0 or not finite,
 * max_gap < 1, NULL arrays.
 */
int fk_key_points(const double *grid_w, int32_t px, int32_t m, double tol, int32_t max_gap, uint8_t *mask,
                  hipStream_t stream);

/*
 * Interface values from key points (Sect. 4; Sect. 5 uses piecewise cubic
 * Hermite interpolation): on each interface line, the monotone piecewise
 * cubic Hermite interpolant (Fritsch & Carlson 1980; slopes of Fritsch &
 * Butland 1984: 0 at an interior knot whose secants differ in sign, else
 * their weighted harmonic mean with weights 2 h_right + h_left and
 * h_right + 2 h_left; at an end the three-point formula, 0 if its sign
 * differs from the end secant's and limited to 3 times it where the secants
 * change sign; two knots give a straight line) through the boundary data at
 * the line's two ends and its key points, in the node coordinate k/N,
 * evaluated at the other nodes of the line.
 *
 *   slot               device [n_iface] int32, canonical order: the node's
 *                      index into key_xi / key_eta, or -1 (not a key point);
 *                      indices >= n_keys yield NaN
 *   key_xi, key_eta    device [n_keys] FP64: the key points' values
 *   edge_xi, edge_eta  device [(N+1)^2] FP64 grids whose edge nodes hold the
 *                      boundary data (fk_boundary_data)
 *   iface_xi/eta       device [n_iface] FP64 (output): every interface node
 *
 * FK_E_INVAL for px < 2, m < 2, px m > 65535, n_keys < 0, NULL arrays.
 */
int fk_interface_interpolate(int32_t px, int32_t m, const int32_t *slot, int64_t n_keys, const double *key_xi,
                             const double *key_eta, const double *edge_xi, const double *edge_eta, double *iface_xi,
                             double *iface_eta, hipStream_t stream);

/*
 * The same interpolant in place, for a solve restricted by a mask (the
 * mask argument of fk_interface_solve): iface_xi / iface_eta (device
 * [n_iface] FP64, canonical order) hold the key points' values at the nodes
 * with mask[i] != 0 on entry; the other nodes are overwritten with the
 * interpolant through those values and the line ends (edge_xi / edge_eta as
 * above).  Key points are read only, so the call needs no second buffer
 * and no host copy of the mask.
 *
 * FK_E_INVAL for px < 2, m < 2, px m > 65535, NULL arrays.
 */
int fk_interface_interpolate_mask(int32_t px, int32_t m, const uint8_t *mask, const double *edge_xi,
                                  const double *edge_eta, double *iface_xi, double *iface_eta, hipStream_t stream);

/*
 * Mesh quality of a nodal map (xi, eta) on an (n+1)^2 grid: out[0] = minimum
 * over cells of the Jacobian xi_x eta_y - xi_y eta_x, out[1] = maximum of the
 * skewness |grad xi . grad eta| / (|grad xi| |grad eta|), both from
 * cell-centred differences.  out is device FP64 [2], 8-byte aligned
 * (FK_E_INVAL otherwise); it also holds the reduction's 64-bit keys between
 * the call's three kernels, so it must not be read on another stream before
 * they finish.  Cells whose skewness is 0/0 (a zero gradient) are passed over.
 */
int fk_mesh_quality(const double *xi, const double *eta, int32_t n, double *out, hipStream_t stream);

/*
 * Learned control variate.  A tanh MLP u_hat(t, x, y) -> (xi_hat, eta_hat),
 * 3 -> 64 -> 64 -> 64 -> 2 with linear outputs, on the normalised input
 * z = (2 t / t_scale - 1, 2 x - 1, 2 y - 1).  Parameters (8706 FP32, in the
 * order W1[64][3] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[2][64] b4[2],
 * row-major) are kept as FP32 master weights with Adam moments; every kernel
 * uses their BF16 rounding ("the network").  Training and evaluation run on
 * BF16 MFMA with FP32 accumulation.  Handles own device memory (freed by
 * fk_cv_destroy); create/get/set/destroy synchronise the device.
 */
typedef struct fk_cv *fk_cv_t;
#define FK_CV_N_PARAMS 8706

int fk_cv_create(const float *params /* host [8706] */, double t_scale, fk_cv_t *out);
void fk_cv_destroy(fk_cv_t cv);
/* params: host [8706] FP32 master weights or NULL; bf16_params: host [8706]
 * BF16 bit patterns of the network or NULL. */
int fk_cv_get_params(fk_cv_t cv, float *params, uint16_t *bf16_params);
/* The identity base: with on = 1 the control is u_hat = (x, y) + network --
 * the network fits the deviation of the mesh map from the identity.  Training
 * then fits target - (x, y), and every evaluation (fk_cv_eval, the node value
 * and the path evaluations of fk_interface_solve_cv) adds x to xi, y to eta
 * and the identity to their gradients.  Applies to all later calls; 0 (the
 * default) is the plain network. */
int fk_cv_set_identity_base(fk_cv_t cv, int32_t on);
/* The base of the control: FK_CV_BASE_NONE (the network itself),
 * FK_CV_BASE_IDENTITY (as fk_cv_set_identity_base(cv, 1)) or FK_CV_BASE_GRID:
 * u_hat = the bilinear interpolant of the solve's grid initial data (the mesh
 * at the step's start) + network, in the martingale form of
 * fk_interface_solve_cv (which then needs FK_DATA_GRID initial data; the
 * Dynkin form is FK_E_UNSUPPORTED since the interpolant has no Laplacian).
 * Over one mesh step the solution stays close to the mesh it starts from, so
 * the network only carries the step's change; it is trained on targets minus
 * the base, which the caller forms (fk_cv_train and fk_cv_eval see the network
 * alone under the grid base).  The martingale blocks then close every 2 steps,
 * with G = the interpolant's gradient there plus the network's gradient taken
 * every `stride` steps and held (each G still fixed before its increments). */
#define FK_CV_BASE_NONE 0
#define FK_CV_BASE_IDENTITY 1
#define FK_CV_BASE_GRID 2
int fk_cv_set_base(fk_cv_t cv, int32_t base);
int fk_cv_set_params(fk_cv_t cv, const float *params /* host [8706] */);
/* Forward-mode evaluation at n points txy (device [n][3]: t, x, y):
 * out (device [n][2][5]) = for each output: value, d/dx, d/dy, d/dt,
 * Laplacian in (x, y). */
int fk_cv_eval(fk_cv_t cv, const float *txy, int64_t n, float *out, hipStream_t stream);
/* Precision of the network's (x, y) gradient in the martingale forms of
 * fk_interface_solve_cv (FK_CV_MARTINGALE, and the network part under
 * FK_CV_BASE_GRID).  FK_CV_GRAD_SPLIT (the default): every activation enters
 * the BF16 products as a hi + lo pair, two products each, and the gradient
 * matches the FP64 evaluation of the same BF16 weights to ~1e-5 relative.
 * FK_CV_GRAD_BF16: activations are rounded to BF16 once (half the products
 * and conversions), ~1e-2 relative.  The martingale estimator is unbiased
 * for any gradient fixed before the increments it multiplies, so both give
 * the same expectation; the rounding only moves each path's score a little
 * (and the variance with it).  The Dynkin form and fk_cv_eval always use
 * the split form.  Applies to later calls; FK_E_INVAL for other modes. */
#define FK_CV_GRAD_SPLIT 0
#define FK_CV_GRAD_BF16 1
int fk_cv_set_grad_precision(fk_cv_t cv, int32_t mode);
/* The network's (x, y) gradient at n points txy (device [n][3]: t, x, y) as
 * the martingale path kernels take it (the handle's gradient precision and
 * base): out (device [n][2][2]) = (dxi/dx, dxi/dy, deta/dx, deta/dy).
 * Parity hook. */
int fk_cv_eval_grad(fk_cv_t cv, const float *txy, int64_t n, float *out, hipStream_t stream);
/* Gradient of the mean-squared error over all n samples (device txy [n][3],
 * target [n][2]) at the current network: grad device [8706], loss device [1]
 * (mean over samples and both outputs) or NULL.  Parity hook. */
int fk_cv_grad(fk_cv_t cv, const float *txy, const float *target, int64_t n, float *grad, float *loss,
               hipStream_t stream);
/* One Adam step (lr; beta = 0.9, 0.999; eps = 1e-8; bias-corrected) with a
 * given gradient (device [8706]).  Parity hook. */
int fk_cv_adam_apply(fk_cv_t cv, const float *grad, float lr, hipStream_t stream);
/* `steps` Adam steps on minibatches of `batch` samples drawn with
 * Philox4x32-10 (key = seed, counter (j, step, 0, 2)) modulo n; loss_out
 * (device [steps] or NULL) receives each step's minibatch loss.  The loop
 * runs as a HIP graph, captured on the first call with this (steps, batch)
 * and replayed afterwards (the call's arrays and scalars reach the kernels
 * through a small device record written on the stream first, so the same
 * graph serves every call).  The arrays must stay unchanged until the stream
 * passes the call. */
int fk_cv_train(fk_cv_t cv, const float *txy, const float *target, int64_t n, int32_t steps, int32_t batch, float lr,
                uint64_t seed, float *loss_out, hipStream_t stream);

/*
 * Control-variate interface solve: the paths of fk_interface_solve (same
 * counters; pts and mask as there: device coordinates, optional mask), each
 * scored with a control variate built from the network u_hat.
 * Two forms of one estimator (they agree in continuous time by Ito's formula
 * applied to u_hat along the path; u_hat's time argument runs backward from
 * t_init + t like the density's):
 *   FK_CV_DYNKIN       u(P) = u_hat(t_init + t, P) + E[ g - u_hat(tau_end, X_end) + sum_j r_j ds_j ],
 *                      r = Laplacian u_hat + b . grad u_hat - d_t u_hat taken at
 *                      the path state every `stride` steps and at the path's
 *                      end, integrated by the trapezoidal rule between those
 *                      points (a quadrature bias that grows with stride dt);
 *   FK_CV_MARTINGALE   u(P) = E[ g - sum_j grad u_hat(X_{k_j}) . dB_j ], dB_j the
 *                      Brownian part sqrt(2 dt) z of the steps from k_j (every
 *                      `stride` steps from the start) to the next k_j or the
 *                      path's end: mean zero for the discrete chain at any stride
 *                      and for any gradient, so also
 *   FK_CV_MARTINGALE_GRID  with the gradient of the grid initial data in place
 *                      of the network's (over one mesh step the solution stays
 *                      close to the mesh it starts from).
 * stride is even, >= 2.  xi/eta/se_*: the CV estimate; plain_*: the plain
 * estimate from the same paths (all four or none: the plain path kernel is run
 * on the same counters after the control-variate kernel, bitwise the plain
 * solve's result); exit_step and cv_scores (device [n][N][2], the per-path CV
 * scores whose mean, plus u_hat(t_init + t, P) in the Dynkin form, is the
 * estimate) optional.  The CV scores are summed in the kernel as in
 * fk_interface_solve (|score| < 512).
 * workspace: fk_interface_cv_workspace_bytes(n_nodes, n_paths) (per-node
 * tables and sums, independent of n_paths).
 */
#define FK_CV_DYNKIN 0
#define FK_CV_MARTINGALE 1
#define FK_CV_MARTINGALE_GRID 2   /* the martingale form with G = gradient of the bilinear interpolant of the
                                     grid initial data at the path's position (no network: cv may be NULL;
                                     needs FK_DATA_GRID initial data); every `stride` steps of each path */
size_t fk_interface_cv_workspace_bytes(int64_t n_nodes, int64_t n_paths);
/* Workspace for FK_CV_MARTINGALE_GRID on a grid_n-cell grid with room for a per-cell FP32
 * gradient table (32 B per cell, built on the stream by the solve): the path kernel then reads
 * one cell entry per component instead of four FP64 grid values, with bitwise the same
 * results.  A workspace of fk_interface_cv_workspace_bytes still works, reading the grids.
 * Returns 0 for n_paths < 2, negative n_nodes or grid_n outside 1..65535. */
size_t fk_interface_cv_grid_workspace_bytes(int64_t n_nodes, int64_t n_paths, int32_t grid_n);
int fk_interface_solve_cv(const fk_density *w, const fk_data *d, const double *pts, const uint8_t *mask,
                          int64_t n_nodes, double t, double dt, int64_t n_paths, uint64_t seed, uint32_t level_id,
                          fk_cv_t cv, int32_t stride,
                          int32_t form, double *xi, double *eta, double *se_xi, double *se_eta, double *plain_xi,
                          double *plain_eta, double *plain_se_xi, double *plain_se_eta, int32_t *exit_step,
                          float *cv_scores, uint64_t *total_steps, const fk_plan *plan, void *workspace,
                          size_t workspace_bytes, hipStream_t stream);

/*
 * Kernel timing.  While enabled (per calling thread), fk_interface_solve
 * records HIP events on its stream around the path kernel and around the
 * reduction kernel (fk_interface_solve_cv: around its start-point network
 * kernel plus path kernel, and around its reductions); fk_timing_last waits
 * for the last recorded events and returns their durations in milliseconds.  Disabled by default (no events
 * are recorded).  fk_timing_last returns FK_E_INVAL if nothing was recorded.
 */
int fk_timing_enable(int enable);
int fk_timing_last(double *path_kernel_ms, double *reduce_kernel_ms);

/*
 * The path kernels' generator on its own, for bitwise checks.
 * fk_philox_words: Philox4x32-10 (Salmon et al., SC'11) of n counters
 *   ctr (device, [n][4] uint32) under the key (seed low word, seed high
 *   word); out (device, [n][4] uint32).
 * fk_normals: for word pairs (ra[i], rb[i]) (device uint32 [n]) the FP32
 *   Brownian increments sqrt(2 D) (z0, z1) of the Box-Muller transform of
 *   u1 = 1 - (ra mod 2^23) 2^-23 and u2 = (rb mod 2^23) 2^-23 (Sect. 4: increments
 *   are sqrt(step) times standard normals; sqrt(2) from the diffusion);
 *   out (device, [n][2] FP32).
 */
int fk_philox_words(const uint32_t *ctr, int64_t n, uint64_t seed, uint32_t *out, hipStream_t stream);
int fk_normals(const uint32_t *ra, const uint32_t *rb, int64_t n, double D, float *out, hipStream_t stream);

/* Wait for the stream; report queued device errors as FK_E_DEVICE. */
int fk_sync(hipStream_t stream);

/* Description of the last error on the calling thread ("" if none). */
const char *fk_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int fk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FK_H */
