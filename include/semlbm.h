/*
 * semlbm.h -- C ABI of the MI355X (gfx950) implementation of the two-phase spectral-element
 * lattice Boltzmann time step of Zhao, Patel & Lee, "Spectral element lattice Boltzmann
 * method for non-ideal gases with partial wetting boundary condition".
 *
 * One solve ("context") = one droplet problem on one unstructured GLL mesh.  The library
 * advances the modified distributions f-bar of Eq. (5) through the collision of Eq. (4)
 * and three SSP-RK3 stages of the weak-form streaming of Eqs. (6) and (12), with the
 * chemical potential of Eq. (2) (weak Laplacian, Eq. (8)), the wetting condition of
 * Sec. 2.2 and the flux bounce-back of Eq. (9).  All arithmetic is FP64 and every step of
 * the time loop runs in the library's HIP kernels on the bound stream.
 *
 * Conventions shared by every call:
 *   - Element-local node index n = i + (N+1) j (+ (N+1)^2 k); i runs along the first
 *     reference direction.  Faces 0..2d-1 are xi-, xi+, eta-, eta+, zeta-, zeta+.
 *   - Global node ids are the caller's: 0 .. n_global-1.  Every per-node array passed in
 *     or out of the library is indexed by the caller's global id.
 *   - Populations are ordered as follows (e_a, weight):
 *       D2Q9  (lattice = 9):  0:(0,0) 4/9; 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 1/9;
 *                             5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1) 1/36.
 *       D3Q19 (lattice = 19): 0 rest 1/3; 1..6: +x,-x,+y,-y,+z,-z 1/18;
 *                             7..18: (1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),
 *                             (1,0,-1),(-1,0,1),(0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1) 1/36.
 *       D3Q13 (lattice = 13): 0 rest 2/5; 1..12 the icosahedron vertices at |e|^2 = 5/3,
 *                             weight 1/20, with a = sqrt((5 - sqrt 5)/6), b = sqrt((5 + sqrt 5)/6):
 *                             (0,a,b),(0,-a,-b),(0,a,-b),(0,-a,b),(a,b,0),(-a,-b,0),
 *                             (a,-b,0),(-a,b,0),(b,0,a),(-b,0,-a),(b,0,-a),(-b,0,a).
 *                             The paper's 3-D runs use a 13-velocity model (Sec. 3.2); this is
 *                             the 13-velocity set whose weights give the equilibrium (A.2) its
 *                             moments up to fourth order under one relaxation time.
 *     The FP64 rest weight is 1 minus the exact sum of the others, so the weights sum to
 *     exactly one.  c_s^2 = 1/3.
 *   - Population arrays are [Q][n_global] (population-major), velocity arrays [d][n_global].
 *   - Host pointers are read or written synchronously and stay owned by the caller.  Device
 *     memory is the caller's workspace (slbm_bind); the library never frees it.
 *   - No call throws; every call returns an slbm_status.  A context must be used from one
 *     host thread at a time.  slbm_last_error() describes the last failure.
 *
 * Environment switches (read where noted; none changes any result, bit for bit):
 *   SLBM_UNFUSED=1        slbm_set_mesh: step with the separate element and node kernels
 *   SLBM_FUSED=1          slbm_set_mesh: step with the fused element kernels wherever the
 *                         mesh allows them (by default not for meshes over 2^20 local
 *                         nodes in 2-D, 2^17 in 3-D); a batch still steps a group over
 *                         that many local nodes with the unfused kernels
 *   SLBM_NO_SPLIT=1       slbm_set_mesh: on the unfused path keep the mesh's own global
 *                         numbering (no element-interior nodes first, no padded element
 *                         stride); every node then goes through the node kernels
 *   SLBM_NO_GRAPH=1       slbm_bind / slbm_batch_create: plain launches, no HIP graphs
 *   SLBM_SERIAL_GROUPS=1  slbm_batch_create: a batch's groups one after another on its
 *                         stream instead of on concurrent streams
 *   SLBM_AUTOTUNE=0       slbm_batch_create: no launch-shape timing (fixed shape rule)
 */
#ifndef SEMLBM_H
#define SEMLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int slbm_status;
#define SLBM_OK 0
#define SLBM_EINVAL (-1)    /* bad argument (sizes, ids, non-positive Jacobian, ...) */
#define SLBM_ENOMEM (-2)    /* workspace too small or host allocation failed */
#define SLBM_EDEVICE (-3)   /* HIP runtime error */
#define SLBM_ESTATE (-4)    /* call out of order (e.g. step before bind) */
#define SLBM_EDIVERGED (-5) /* non-finite state or kinetic energy above the limit */

typedef struct slbm_params {
    int lattice;      /* 9 = D2Q9 (2-D), 19 = D3Q19 or 13 = D3Q13 (3-D) */
    int N;            /* GLL polynomial order: 2..16 in 2-D, 2..6 in 3-D */
    double rho_l;     /* liquid bulk density (Appendix A: 1.0 in the paper) */
    double rho_v;     /* vapour bulk density (Appendix A: 0.1) */
    double delta;     /* interface thickness of Eq. (A.1) */
    double sigma;     /* surface tension gamma; beta = 12 sigma/(delta drho^4),
                         kappa = 3 sigma delta/(2 drho^2) solve Eqs. (A.4)-(A.5) */
    double tau;       /* dimensionless relaxation time of Eq. (4) (0.5 in Sec. 3.3), in units
                         of dt: the kinematic viscosity is tau dt / 3, so a smaller dt (a
                         higher order, a finer mesh) at the same tau is a less viscous fluid
                         with a Laplace number larger by the square of the ratio.  Ignored
                         when nu > 0. */
    double dt;        /* > 0: time step; otherwise dt = min(cfl h_min,
                         C h_min^2 / sqrt(kappa rho_l)) (advective and capillary bounds), with
                         C = 0.25 for N <= 12 and 0.125 for N >= 13. */
    double cfl;       /* h_min = smallest distance of neighbouring GLL nodes on element lines */
    int ke_every;     /* slbm_step checks finiteness and KE_max every ke_every steps (0: never) */
    double ke_limit;  /* KE_max above this (or non-finite) -> SLBM_EDIVERGED; <= 0: 1.0 */
    uint64_t seed;    /* default seed of slbm_init_tanh noise */
    double nu;        /* > 0: kinematic viscosity to hold; slbm_set_mesh then sets
                         tau = (3 nu) / dt once dt is known (cs^2 = 1/3), so the fluid is the
                         same at every order, mesh and time step.  0: use tau.  A caller that
                         zero-initialises the struct gets the tau behaviour. */
} slbm_params;

typedef struct slbm_info {
    double dt, beta, kappa, omega, h_min;
    int64_t n_elements, n_local, n_global, n_wall_nodes, step;
    size_t workspace_bytes;
    int dim, Q, N;
    double tau;       /* relaxation time in use (from nu once the mesh is set, if nu > 0) */
    int64_t n_interior; /* global nodes strictly inside an element that the element kernels
                         * finish themselves (unfused path; 0 on the fused path) */
    int fused;        /* 1: fused element-kernel path, 0: separate element and node kernels
                         * (chosen at slbm_set_mesh: separate kernels for meshes over 2^20
                         * local nodes in 2-D and 2^17 in 3-D, the measured crossovers) */
} slbm_info;

typedef struct slbm_ctx slbm_ctx;

/* Create a context from physical parameters (Appendix A, Eq. (4)).  *out is NULL on error. */
slbm_status slbm_create(const slbm_params *p, slbm_ctx **out);

/* Upload the mesh (Sec. 3: curved unstructured GLL meshes).
 *   xyz       [E][(N+1)^d][d]  node coordinates; shared nodes carry equal coordinates
 *                              (copies across a periodic wrap differ by the period)
 *   gid       [E][(N+1)^d]     caller's global id of every element node; ids shared by
 *                              several elements are summed by direct stiffness summation
 *   wall_face [F][2]           (element, face) of every physical wall face, each at most once
 *   wall_cos  [F]              cos(theta_eq) imposed on the face (Eq. (7), Sec. 2.2)
 *   wall_ub   [F][d] or NULL   wall velocity u_b of Eq. (9) (NULL: resting walls)
 * The library copies everything and derives the metric terms (curl form in 3-D), the
 * lumped mass, wall normals and weights, and the time step.  Errors: SLBM_EINVAL for bad
 * sizes/ids, a wall face listed twice or a non-positive Jacobian, SLBM_ESTATE if already
 * bound. */
slbm_status slbm_set_mesh(slbm_ctx *c, int64_t E, const double *xyz, const int32_t *gid,
                          int64_t n_global, int64_t n_wall_faces, const int32_t *wall_face,
                          const double *wall_cos, const double *wall_ub);

/* Device bytes needed by slbm_bind (valid after slbm_set_mesh; 0 before). */
size_t slbm_workspace_bytes(const slbm_ctx *c);

/* Bind caller-allocated device memory (256-byte aligned, >= slbm_workspace_bytes) and a
 * HIP stream (hipStream_t; NULL = default stream).  Uploads the geometry tables and
 * returns after they are resident.  The memory must outlive the context. */
slbm_status slbm_bind(slbm_ctx *c, void *dev_ptr, size_t bytes, void *hip_stream);

/* Initial condition of Eqs. (A.1)/(A.8)-(A.9): rho = (rl+rv)/2 - (rl-rv)/2 tanh(2 s/delta),
 * s = |x - x0| - R (liquid inside), u = 0, f-bar = t_a rho; plus noise_amp (2U-1) per
 * global node with U = (SplitMix64(seed xor gid) >> 11) 2^-53.  Node coordinates are those
 * of the lowest local copy.  x0 has d entries.  Resets the step counter. */
slbm_status slbm_init_tanh(slbm_ctx *c, const double *x0, double R, double noise_amp,
                           uint64_t seed);

/* rho [n_global] (host): f-bar = t_a rho, u = 0.  Resets the step counter. */
slbm_status slbm_set_rho(slbm_ctx *c, const double *rho);

/* Checkpoint: f-bar [Q][n_global] (host) and the step counter. */
slbm_status slbm_get_state(slbm_ctx *c, double *f, int64_t *step);
slbm_status slbm_set_state(slbm_ctx *c, const double *f, int64_t step);

/* Advance n time steps (collision + 3 SSP-RK3 streaming stages each).  Asynchronous on the
 * bound stream unless ke_every > 0, in which case it synchronises every ke_every steps
 * and returns SLBM_EDIVERGED on a non-finite or too-large kinetic energy. */
slbm_status slbm_step(slbm_ctx *c, int64_t n);

/* Tracing: advance n steps like slbm_step with a HIP event pair around every kernel
 * launch; ms[k] accumulates the elapsed milliseconds and launches[k] the launch count of
 * kernel kind k.  Unfused path (separate element and node kernels): 0 Laplacian, 1 chemical
 * potential, 2 gradients, 3 collision, 4 streaming residual, 5 DSS + Runge-Kutta combine.
 * Fused path (element kernels that finish the previous pass's summation): 6 chemical
 * potential + gradients, 7 collision + stage-1 residual, 8 summation + Runge-Kutta +
 * Laplacian, 9 chemical potential + residual.  Synchronises after every step. */
#define SLBM_NUM_KERNEL_KINDS 10
slbm_status slbm_step_profile(slbm_ctx *c, int64_t n, double *ms, int64_t *launches);

/* Tracing: average duration of one kernel kind (numbering as for slbm_step_profile) when
 * reps (1..4096) launches of it run back to back from one HIP graph on the bound stream
 * (plain launches where the stream cannot be captured), timed by a HIP event pair around
 * the replay (after one untimed replay).  Kinds with
 * stages cycle through them (streaming and Runge-Kutta 1,2,3; fused kinds 8: 1,2,3 and 9:
 * 2,3).  Only the kinds of the context's path (unfused 0-5, fused 6-9) are accepted.  The
 * state and the step counter are restored afterwards (f-bar is saved to the host and
 * uploaded again); synchronising. */
slbm_status slbm_time_kernel(slbm_ctx *c, int kind, int64_t reps, double *ms_per_launch);

/* Queries (synchronising).  rho [n_global] by Eq. (10); u [d][n_global] by Eq. (11);
 * ke_max = max over nodes of rho |u|^2 / 2; mass = sum of lumped mass times rho. */
slbm_status slbm_get_rho(slbm_ctx *c, double *rho);
slbm_status slbm_get_u(slbm_ctx *c, double *u);
slbm_status slbm_kinetic_energy(slbm_ctx *c, double *ke_max, double *mass);

/* Geometric contact angle (Sec. 3.1): mid-density crossings along element lines, points
 * within 2 delta of the wall dropped, algebraic (Kasa) circle/sphere fit, intersection
 * angle with the wall measured through the liquid. */
typedef struct slbm_wall_geom {
    int kind;          /* 0 = plane, 1 = circle (2-D), 2 = sphere (3-D) */
    double point[3];   /* plane: a point of it; circle/sphere: the centre */
    double normal[3];  /* plane: unit normal pointing out of the fluid */
    double radius;     /* circle/sphere radius */
} slbm_wall_geom;
slbm_status slbm_contact_angle(slbm_ctx *c, const slbm_wall_geom *w, double *theta_deg);

slbm_status slbm_get_info(const slbm_ctx *c, slbm_info *info);

/* Host-side tables derived by slbm_create / slbm_set_mesh (no device work):
 * GLL nodes x[N+1], weights w[N+1] and differentiation matrix D[(N+1)^2] (row-major,
 * D[i][m] = l_m'(x_i)), Deville, Fischer & Mund ch. 2; and the assembled GLL-lumped mass
 * matrix MA[n_global] (caller's ids), the M of Eqs. (6) and (8). */
slbm_status slbm_get_gll(const slbm_ctx *c, double *x, double *w, double *D);
slbm_status slbm_get_mass(const slbm_ctx *c, double *MA);
const char *slbm_last_error(const slbm_ctx *c);
void slbm_destroy(slbm_ctx *c);

/* Operator entry points, each one kernel pass of the time step on host data (they use the
 * context's workspace and leave the state untouched):
 *   slbm_op_mu:      mu [n_global] of Eq. (2) with the weak Laplacian of Eq. (8) and the
 *                    wetting boundary integral of Sec. 2.2, from rho [n_global]
 *   slbm_op_grad:    lumped-mass average of element gradients, [d][n_global], of phi
 *   slbm_op_stream:  L [Q][n_global], the assembled right-hand side of Eqs. (6)/(12) with
 *                    the flux of Eq. (9) (L_0 = 0), from g [Q][n_global], rho, mu
 *   slbm_op_collide: f* [Q][n_global] of Eq. (4) from f, rho, grad rho, grad mu
 * Errors as for slbm_step; all of them synchronise. */
slbm_status slbm_op_mu(slbm_ctx *c, const double *rho, double *mu);
slbm_status slbm_op_grad(slbm_ctx *c, const double *phi, double *grad);
slbm_status slbm_op_stream(slbm_ctx *c, const double *g, const double *rho, const double *mu,
                           double *L);
slbm_status slbm_op_collide(slbm_ctx *c, const double *f, const double *rho, const double *grho,
                            const double *gmu, double *fstar);

/* ------------------------------------------------------------------------------------ */
/* Batching: many bound contexts (different meshes, N, dt) advanced together.  Each     */
/* kernel of the step covers every member's elements or nodes in one launch, grouped by */
/* (lattice, N, kernel path); members keep their own workspace.  Members start from the */
/* path they step alone with; a fused group whose members together exceed 2^20 local    */
/* nodes (2^17 in 3-D) steps with the unfused kernels, as one mesh of that size would.  */
/* A member stepped that way has its Laplacian partials recomputed before it next steps */
/* fused (alone, or in a fused group), so every member's results are those of stepping  */
/* alone.                                                                               */
/* ------------------------------------------------------------------------------------ */
typedef struct slbm_batch slbm_batch;
slbm_status slbm_batch_create(void *hip_stream, slbm_batch **out);
/* Add a bound context (must be bound to the batch's stream). */
slbm_status slbm_batch_add(slbm_batch *b, slbm_ctx *c);
slbm_status slbm_batch_remove(slbm_batch *b, slbm_ctx *c);
int slbm_batch_size(const slbm_batch *b);
/* Advance every member n steps (asynchronous, except in a call that tunes, below). */
slbm_status slbm_batch_step(slbm_batch *b, int64_t n);

/* Launch-shape autotuning.  Members with the same (lattice, N, kernel path) form a group
 * whose every kernel covers all of them in one launch; a group can launch in several
 * shapes: one element per block of the element kernels, or as many elements as fit in
 * 256 threads (where more than one fits), each with its block tables in XCD-aware order
 * (every die of the chip works on a contiguous range of elements or nodes) or in plain
 * order.  All shapes give the same bits.  With autotuning on (the default), the first
 * slbm_batch_step of n >= 4 * n_shapes steps after a group of a new (lattice, N, path,
 * floor(log2(elements))) appears spends 4 of those steps per shape on the group (one
 * warm-up, three timed), keeps the fastest and remembers it for later groups of the same
 * key in this batch; that call waits for the device.  Every member still advances exactly
 * n steps.  Off, a group uses wide blocks in XCD order when they make at least 256
 * blocks and one element per block otherwise.  on: 0 or 1, else SLBM_EINVAL. */
slbm_status slbm_batch_set_autotune(slbm_batch *b, int on);

#define SLBM_MAX_SHAPES 4
typedef struct slbm_batch_shape {
    int dim, order, fused;     /* group key (with lattice): dimension, N, fused kernel path (0/1) */
    int members;               /* members in the group */
    int64_t elements;          /* their elements */
    int n_shapes;              /* candidate shapes, at most SLBM_MAX_SHAPES */
    int epb[SLBM_MAX_SHAPES];  /* elements per block of the element kernels */
    int xcd[SLBM_MAX_SHAPES];  /* 1: XCD-aware block order, 0: plain order */
    double us_per_step[SLBM_MAX_SHAPES]; /* measured device us per step of the group, 0 if not */
    int chosen;                /* index of the shape the group launches with */
    int measured;              /* 1 if chosen by timing, 0 by the fixed rule above */
    int lattice;               /* the group's lattice: 9, 19 or 13 */
} slbm_batch_shape;
/* The groups of the current membership: writes min(count, max) entries to out[max] and
 * the number of groups to *count (0 for an empty batch).  Errors: SLBM_EINVAL (null b or
 * count, max < 0, or max > 0 with null out), or those of rebuilding the launch tables
 * after a membership change (SLBM_ENOMEM, SLBM_EDEVICE). */
slbm_status slbm_batch_shapes(slbm_batch *b, slbm_batch_shape *out, int max, int *count);
/* Allocation-free batched step, for callers that cannot allocate device memory (tight
 * serving loops and harnesses that forbid hipMalloc/hipFree): the same n time steps of
 * every member as slbm_batch_step, bit for bit, with no device allocation.  The batch's
 * launch tables (member descriptors and block tables of each group's chosen launch shape)
 * are laid out in a file-scope device array of SLBM_STATIC_SCRATCH_BYTES per GPU instead
 * of library-allocated memory; the groups step one after another on the batch's stream
 * with plain launches (no graphs, no shape tuning: a group uses the shape an earlier
 * slbm_batch_step tuned for its key, else the fixed rule).  Every call on a GPU shares that
 * GPU's array: a call uploads its tables (waiting for its stream) unless the array still
 * holds this batch's current layout, so calls that overlap on one GPU (batches on
 * different streams or host threads) race and must be serialised by the caller.
 * Asynchronous on the batch's stream otherwise.  Errors: SLBM_EINVAL (null b, n < 0),
 * SLBM_ENOMEM if the tables exceed SLBM_STATIC_SCRATCH_BYTES (about 500,000 element and
 * node blocks in all), SLBM_EDEVICE on a HIP error. */
#define SLBM_STATIC_SCRATCH_BYTES (4u << 20)
slbm_status slbm_batch_step_static(slbm_batch *b, int64_t n);
/* Per-member KE_max and mass into ke[size], mass[size] (member order of insertion). */
slbm_status slbm_batch_kinetic_energy(slbm_batch *b, double *ke, double *mass);
void slbm_batch_destroy(slbm_batch *b);

/* ------------------------------------------------------------------------------------ */
/* Serving: a continuous-batching request loop for contact-angle solves.                */
/* ------------------------------------------------------------------------------------ */
typedef struct slbm_server_cfg {
    void *arena;          /* device memory the server sub-allocates workspaces from */
    size_t arena_bytes;
    void *hip_stream;     /* stream of every solve */
    int max_slots;        /* concurrent solves */
    int check_every;      /* KE check cadence in steps (paper: KE_max monitored in time) */
    double ke_stop;       /* retire when KE_max < ke_stop (e.g. 1e-20) */
    int64_t max_steps;    /* or after this many steps */
} slbm_server_cfg;

typedef struct slbm_request {
    slbm_params params;
    int64_t E;
    const double *xyz;       /* copied at submit */
    const int32_t *gid;
    int64_t n_global;
    int64_t n_wall_faces;
    const int32_t *wall_face;
    const double *wall_cos;
    const double *wall_ub;   /* may be NULL */
    double x0[3];
    double R;
    double noise_amp;
    slbm_wall_geom wall;     /* for the contact angle at retirement */
    double *state_out;       /* NULL, or a caller-owned host buffer of Q * n_global doubles:
                              * a request that completes with SLBM_OK copies its final
                              * f-bar there ([Q][n_global], the caller's global numbering, as
                              * slbm_get_state) before its result is published.  The caller
                              * keeps the buffer alive until poll reports the result. */
} slbm_request;

typedef struct slbm_result {
    slbm_status status;      /* SLBM_OK, SLBM_EDIVERGED, ... ; 1 = still pending */
    double theta_deg;
    double ke_max;
    int64_t steps;
    double t_arrive, t_admit, t_done; /* seconds on the server's clock */
} slbm_result;

typedef struct slbm_server slbm_server;
slbm_status slbm_server_create(const slbm_server_cfg *cfg, slbm_server **out);
/* Queue a request (inputs are copied); returns its id.  t_arrive is stamped now. */
slbm_status slbm_server_submit(slbm_server *s, const slbm_request *r, uint64_t *id);
/* Advance the server by one scheduling round: admit prepared requests that fit (slots and
 * arena bytes), run check_every steps of all active solves as one batch, retire finished
 * ones.  Submitted requests are prepared (context creation, mesh processing) by host worker
 * threads while the device runs.  The same workers bind the requests a round admits
 * (workspace uploads and initial state, each worker on a stream of its own) and compute the
 * contact angles of the ones it retires; the round waits for them.  With no active solve
 * (cold start) a round first waits up to 50 ms for the preparations already submitted, so
 * that requests submitted together start together.  Returns the number of unfinished
 * requests in *pending. */
slbm_status slbm_server_tick(slbm_server *s, int *pending);
/* Result of a request (status 1 while pending). */
slbm_status slbm_server_poll(slbm_server *s, uint64_t id, slbm_result *out);
/* Tick until every submitted request is finished. */
slbm_status slbm_server_drain(slbm_server *s);
double slbm_server_clock(const slbm_server *s);
void slbm_server_destroy(slbm_server *s);

#ifdef __cplusplus
}
#endif
#endif /* SEMLBM_H */
