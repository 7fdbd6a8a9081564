/*
 * lbmdvm: high-order lattice Boltzmann (discrete velocity model) channel and
 * duct solver for AMD Instinct MI355X (gfx950).
 *
 * The method is the one of Feuchter & Schleifenbaum, "High-order lattice
 * Boltzmann models for wall-bounded flows at finite Knudsen numbers"
 * (arXiv:1510.08886): an on-lattice DVM for the Boltzmann-BGK equation with an
 * order-N Hermite equilibrium, a Hermite-expanded body force, the trapezoidal
 * (modified population) time integration, and the diffuse Maxwell wall on the
 * unknown populations of half-way walls.
 *
 * Conventions
 *   - Every call returns an int: LBM_OK (0) or a negative LBM_E_* code.
 *     lbm_last_error() returns a thread-local message for the last failure.
 *   - The caller owns every device buffer and the HIP stream. The library never
 *     allocates or frees caller memory; it owns only opaque host handles.
 *     "dev" pointers are device pointers, "host" pointers are host pointers.
 *   - A handle is single-threaded; distinct handles may run concurrently on
 *     distinct streams. No exception crosses this interface.
 *   - Units follow the paper: channel width l0 = 1, isothermal sound speed
 *     c0 = 1, theta = 1. Nodes sit at y_j = (j + 1/2) dx, dx = 1/ny; walls are
 *     half a spacing outside the first and last node (y = 0 and y = 1).
 *   - 2D problems have walls normal to y and a periodic x; 3D ducts have walls
 *     normal to y and z and a periodic x.
 */
#ifndef LBMDVM_H
#define LBMDVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_E_INVALID (-1)         /* bad argument or inconsistent sizes */
#define LBM_E_UNSUPPORTED (-2)     /* valid request the library has no kernel for */
#define LBM_E_NO_MEMORY (-3)       /* caller buffer / pool too small */
#define LBM_E_QUADRATURE (-4)      /* velocity set is not a quadrature of the stated order */
#define LBM_E_DEVICE (-5)          /* HIP runtime error */
#define LBM_E_NOT_CONVERGED (-6)   /* step limit reached before the tolerance */

typedef struct lbm_dvm lbm_dvm_t;
typedef struct lbm_solver lbm_solver_t;
typedef struct lbm_batch lbm_batch_t;

/* Population storage. The collision is FP64 for LBM_F64 and LBM_F32SR and
 * FP32 otherwise; the wall-flux balance and the mass-flux reductions are FP64
 * in every mode. Every post-collision population is rounded to the storage
 * type every step. */
enum lbm_storage {
    LBM_F64 = 0,     /* fbar in double */
    LBM_F32 = 1,     /* fbar as the FP32 deviation fbar - w rho0 (round to nearest) */
    LBM_F16DEV = 2,  /* half-precision scaled deviation fbar / (w rho0) - 1, rounded
                        stochastically with a counter-based hash of (node, velocity,
                        step): unbiased, deterministic and reproducible */
    LBM_F32RAW = 3,  /* fbar itself in FP32 (round to nearest); its rounding step is
                        ~6e-8 of w rho0, so slow relaxations stagnate early */
    LBM_F32SR = 4    /* the FP32 deviation of LBM_F32, collided in FP64 and rounded
                        stochastically (key as for LBM_F16DEV): the same bytes, no
                        bias that accumulates over a long relaxation (round to
                        nearest repeats the same error at a steady state every
                        step). 2D channels of D2V17 and D2V37 (LBM_E_UNSUPPORTED
                        otherwise) */
};

/* Population layout in HBM. Both give identical results; the choice only
 * moves the memory traffic. LBM_LAYOUT_AUTO keeps one array stepped in place
 * up to 512 MiB per copy (it stays largely in the 256 MB last-level cache) and
 * two ping-pong copies above that; 2D problems in LBM_F32 or LBM_F64 whose
 * velocity set has the two-step kernel (lbm_solver_set_pair_steps) take two
 * ping-pong copies from 64 MiB per copy, stepped two steps per launch. */
enum lbm_layout {
    LBM_LAYOUT_AUTO = 0,
    LBM_LAYOUT_IN_PLACE = 1,  /* one array; steps alternate two in-place kinds */
    LBM_LAYOUT_PING_PONG = 2  /* two copies; each step pulls from one into the other */
};

/* Problem statement (Section V / VI of the paper). */
typedef struct {
    int dim;              /* 2: channel (walls at y); 3: duct (walls at y and z) */
    int nx, ny, nz;       /* nodes; nx periodic; nz ignored (1) in 2D */
    double kn;            /* Knudsen number; tau = kn * sqrt(2/pi) (Eq. nm.13) */
    double ma;            /* used when g_set == 0: g = 8 tau ma along x, i.e. the
                             Navier-Stokes no-slip centreline speed is ma */
    int g_set;            /* 1: take g[] as given */
    double g[3];          /* body-force acceleration (Eq. nm.4); g.n must be 0 */
    int hermite_order;    /* N of the equilibrium (Eq. equi.hermite), 2..(Q+1)/2 */
    double accommodation; /* Maxwell's accommodation alpha in [0, 1]: the fraction of
                             the populations reaching a wall that is re-emitted
                             diffusely (the paper's wall is alpha = 1); the rest is
                             reflected specularly. alpha < 1: 2D channels only,
                             stepped ping-pong (LBM_LAYOUT_IN_PLACE is refused) */
    double rho0;          /* reference density (deviation storage, initial state) */
    int storage;          /* enum lbm_storage */
    int layout;           /* enum lbm_layout: how the populations are kept in HBM */
} lbm_problem_t;

/* Derived per-solve scalars. */
typedef struct {
    double tau;           /* relaxation time, Eq. nm.13 */
    double dt;            /* time step 1 / (c * ny): xi dt = e dx */
    double omega;         /* dt / (tau + dt/2), Eq. nm.8 */
    double g[3];          /* body force */
    double u_c;           /* centreline speed g / (8 tau) used to normalise mass flow */
    double mdot_scale;    /* 1 / (4 u_c kn): mdot = mdot_scale * <u_x> (Eq. pf.1) */
    int V;                /* velocities */
    int halo;             /* max |e_i| over the velocity set */
} lbm_params_t;

const char *lbm_last_error(void);

/* ---- discrete velocity models (Section II) -------------------------------- */

/* Solve the weights of a minimal DVM: the velocity groups are the signed
 * permutations of the n_groups generators gen[n_groups * dim] (Eq. wdach); the
 * moment conditions to degree Q (Eqs. genQua / orth) admit a solution only at
 * isolated lattice speeds c* (Eq. dimker). Returns the smallest c* in
 * [c_lo, c_hi] whose group weights are all positive, in *c_out, the weights in
 * w_group_out[n_groups] and the velocity count in *n_vel_out (any output may be
 * NULL). LBM_E_QUADRATURE if there is none. Host only. */
int lbm_dvm_solve(int dim, int n_groups, const int32_t *gen, int Q, double c_lo,
                  double c_hi, double *c_out, double *w_group_out, int *n_vel_out);

/* One minimal DVM found by lbm_dvm_enumerate. */
#define LBM_MAX_GROUPS 16
typedef struct {
    int dim;
    int V;                               /* velocities */
    int E;                               /* stencil energy (1/2c^2) sum |xi|^2 = (1/2) sum |e|^2 */
    int n_groups;
    int32_t gen[LBM_MAX_GROUPS * 3];     /* generators, dim entries each: 0 <= g_1 <= ... <= g_dim */
    double c;                            /* lattice speed c* */
    double w_group[LBM_MAX_GROUPS];      /* weight of one velocity of each group */
} lbm_dvm_model_t;

/* All minimal DVMs of dimension dim and quadrature order Q whose stencil
 * energy is at most e_max (Section II.B, Eqs. dimker and Ssymbol; Table
 * tab:dvmSummary). A stencil is a set of distinct velocity groups (orbits of
 * integer generators under signed permutations) with one weight per group
 * (Eq. wdach); it is a minimal DVM at c* when the moment conditions to degree
 * Q have exactly one solution there (the orbit moment matrix has full column
 * rank) and none for c near c*, with all weights positive. Stencils of at
 * most max_groups groups are searched (0: one less than the number of moment
 * conditions, the most a minimal DVM can have); c* in [0.02, 50]. flags:
 * LBM_ENUM_SCATTERING keeps only scattering stencils (no velocity with a zero
 * component, so none parallel to a wall; Section IV.C). Models are
 * sorted by V, then E, then c; integer multiples of a stencil appear as
 * separate models (with c* divided by the factor). out[cap] (host) receives the
 * first cap models and *n_out the total count; LBM_E_NO_MEMORY when the total
 * exceeds cap (query with cap = 0). Host only. */
#define LBM_ENUM_SCATTERING 1
int lbm_dvm_enumerate(int dim, int Q, int e_max, int max_groups, int flags, lbm_dvm_model_t *out,
                      int cap, int *n_out);

/* Expand the groups into a velocity set with weights w_group (host arrays) and
 * lattice speed c, and check that it integrates every monomial of degree <= Q
 * exactly (relative tolerance 1e-12 against the Gaussian moment); otherwise
 * LBM_E_QUADRATURE. The library orders the velocities as rest velocities first,
 * then pairs (e, -e). */
int lbm_dvm_create(int dim, int n_groups, const int32_t *gen, const double *w_group,
                   double c, int Q, lbm_dvm_t **out);
int lbm_dvm_destroy(lbm_dvm_t *dvm);

/* Velocity count, integer velocities vel[V * dim] (xi = c * vel), weights w[V]
 * and lattice speed; vel, w and c may be NULL (size query). Host arrays. */
int lbm_dvm_info(const lbm_dvm_t *dvm, int *V, int32_t *vel, double *w, double *c);

/* ---- wall-moment diagnostics (Section IV.B-C) ----------------------------- */

/* Summary of how well a DVM reproduces the diffuse Maxwell wall. */
typedef struct {
    int n_components;       /* L: non-trivial wall moments of rank <= Q (Eq. nontriv) */
    int lambda_order;       /* wall accuracy order (Eq. defLambda); -1 if W itself is inexact */
    uint64_t lambda_index;  /* wall accuracy index (Eq. defbin): bit k set when the
                               (k+1)-th non-trivial moment is exact */
    double sigma_sigma;     /* e^-n weighted mean of |sigma| over the L moments (Eq. sigmaSigma) */
} lbm_wall_report_t;

/* Equilibrium wall moments of a DVM (Eqs. defW, Wscalar) against their
 * quadrature over the velocities leaving the wall into the fluid (Eq. wallQuad),
 * for the wall whose inward normal is +e along velocity component normal_axis
 * (0 <= normal_axis < dim; the other components are the tangential x and y in
 * increasing order). The L non-trivial moments are listed in the order of Eqs.
 * defT / defb: exps[3k..3k+2] = (m_x, m_y, m_z), the exact moment w_exact[k],
 * its quadrature w_dvm[k] and sigma[k] = (w_dvm - w_exact) / w_exact (the sign
 * of the paper's tables). A moment counts as exact to a relative 1e-10. The
 * arrays (host, `cap` entries, any may be NULL) need cap >= L, else
 * LBM_E_NO_MEMORY; query L with all arrays NULL. LBM_E_UNSUPPORTED if L > 64.
 * Host only. */
int lbm_dvm_wall_errors(const lbm_dvm_t *dvm, int normal_axis, int cap, int32_t *exps,
                        double *w_exact, double *w_dvm, double *sigma, lbm_wall_report_t *report);

/* ---- channel profile analysis (Section VI) -------------------------------- */

typedef struct {
    double u_center;  /* u at the channel centre: the middle node (odd ny) or the
                         cubic through the four middle nodes (even ny) */
    double u_wall;    /* u on the walls: quadratic through the three nodes next to
                         each wall, averaged over both walls */
    double slip;      /* u_s = u_wall / u_center (Eq. defSlip) */
    double mean;      /* node average of u (the integral of Eq. pf.1) */
} lbm_profile_stats_t;

/* Slip velocity and Knudsen-layer content of a plane-channel profile u[ny]
 * (host array; the streamwise velocity at the nodes y_j = (j + 1/2)/ny, e.g.
 * an x-average of lbm_observe's u). u_ns[ny] receives the parabola with the
 * same centre value and node-averaged mass flow (Eq. uNS; the continuum factor
 * 3/(l0/2)^2 is the inverse node average of z^2, z = y - 1/2, so the discrete
 * mass flow is kept exactly), u_neq[ny] = u - u_ns (Eq. uNEQ). stats, u_ns and
 * u_neq may be NULL. LBM_E_INVALID unless ny >= 3 (>= 4 when even). Host
 * only. */
int lbm_profile_analysis(const double *u, int ny, lbm_profile_stats_t *stats, double *u_ns,
                         double *u_neq);

/* ---- solver --------------------------------------------------------------- */

/* Derived scalars for a problem (pure host). */
int lbm_params(const lbm_dvm_t *dvm, const lbm_problem_t *prob, lbm_params_t *out);

/* Bytes the caller must provide: the population buffer (*pop_bytes: one copy of
 * the populations when stepped in place, two copies for ping-pong; see
 * enum lbm_layout) and the scratch buffer (*scratch_bytes). LBM_E_INVALID for
 * an unknown layout. */
int lbm_state_bytes(const lbm_dvm_t *dvm, const lbm_problem_t *prob, size_t *pop_bytes,
                    size_t *scratch_bytes);

/* Create a solver over caller device buffers pop_a (populations, >= pop_bytes)
 * and scratch (>= scratch_bytes), both aligned to 256 bytes, on the HIP stream
 * `stream` (hipStream_t; NULL = default stream). In place (prob->layout, by
 * default up to 512 MiB of populations) the update runs in one array (each
 * step reads and writes the same locations per node, alternating two
 * layouts); otherwise pop_a holds two copies, stepped ping-pong. pop_b is not
 * used and may be NULL.
 * Validation (LBM_E_INVALID): ny (and nz in 3D) >= the largest |e_n|;
 * 2 <= N <= (Q+1)/2; kn > 0; g.n = 0; sizes positive; 0 <= accommodation
 * <= 1. accommodation < 1 for a duct gives LBM_E_UNSUPPORTED, as do N > 5 and
 * a velocity set without a compiled kernel (N = 5 is compiled for the sets of
 * quadrature order 9). */
int lbm_solver_create(const lbm_dvm_t *dvm, const lbm_problem_t *prob, void *pop_a,
                      void *pop_b, void *scratch, size_t scratch_bytes, void *stream,
                      lbm_solver_t **out);
int lbm_solver_destroy(lbm_solver_t *s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not allocate, harnesses that forbid
 * hipMalloc): lbm_solver_create without a scratch argument. The scratch lives
 * in a static device array of the library (16 MiB; each device the library
 * runs on holds its own copy until the process ends), and the solver never
 * replays captured graphs (lbm_solver_set_graph_steps then returns
 * LBM_E_UNSUPPORTED), so neither this call nor any later call on the solver
 * allocates device or pinned memory; the handle itself is an ordinary host
 * object. The caller still provides pop_a (lbm_state_bytes) and the stream.
 * LBM_E_NO_MEMORY if the problem needs more than 16 MiB of scratch (its
 * *scratch_bytes from lbm_state_bytes). Every static solver on one device
 * shares that device's array, and creation clears it: at most one static
 * solver per device may be in use at a time; solvers that overlap on one
 * device race. */
int lbm_solver_create_static(const lbm_dvm_t *dvm, const lbm_problem_t *prob, void *pop_a,
                             void *stream, lbm_solver_t **out);

/* Set the post-collision state to the equilibrium f^(0)(rho, u) of Eq.
 * equi.hermite at every node. rho_dev[nodes] and u_dev[nodes * 3] are device
 * FP64 arrays in node order ((k * ny + j) * nx + i); NULL means rho0 and rest. */
int lbm_init_equilibrium(lbm_solver_t *s, const double *rho_dev, const double *u_dev);

/* Enqueue nsteps fused stream + wall + collide steps (Eq. nm.8); asynchronous.
 * For small problems (see lbm_solver_set_graph_steps) runs of two or more
 * steps are replayed from HIP graphs of up to 256 captured steps each, which
 * the library instantiates and caches per solver (at most 8); the results are
 * bit for bit those of one launch per step. */
int lbm_run(lbm_solver_t *s, int64_t nsteps);

/* Most steps lbm_run runs in one launch of one workgroup that loops over the
 * steps (a workgroup barrier between them), for 2D problems of at most 256
 * nodes stepped in place (0: off; at most 2^20). It removes the device-side
 * latency between dependent launches, which dominates such problems; the
 * arithmetic and results are those of one launch per step, FP16 stochastic
 * rounding included. Default 4096 where allowed, else 0; LBM_E_UNSUPPORTED
 * for a non-zero value elsewhere. Takes precedence over graph replay. */
int lbm_solver_set_resident_steps(lbm_solver_t *s, int max_steps);

/* Two time steps per launch for 2D problems stepped ping-pong (temporal
 * blocking): each workgroup computes step t for its tile widened by the
 * stencil's reach and keeps it in LDS, then step t + 1 of the tile, so a node
 * is read and written in HBM once per two lattice updates. The arithmetic and
 * results are bit for bit those of one launch per step. on = 0 switches it
 * off; band_rows is the height of each workgroup's band of rows (0: chosen
 * for the device). on = 1 alternates the two steps in all waves of a
 * workgroup; on = 2 gives them to producer and consumer waves that overlap;
 * on = 3 splits the producers into two groups that take alternate chunks of
 * rows, so that one group's HBM reads are in flight while the other
 * computes. Compiled for the 2D sets reaching at most 4 nodes. Default 3
 * (2 where mode 3's chunks of rows are more than one row shorter than mode
 * 2's, as for D2V17 in FP32) for ping-pong problems that are not
 * graph-replayed, in FP64 and FP32 storage; 0 otherwise (FP16 deviations:
 * their single step is bound by its arithmetic). LBM_E_UNSUPPORTED for
 * on != 0 where not compiled. lbm_run takes two-step launches while two or
 * more steps remain. */
int lbm_solver_set_pair_steps(lbm_solver_t *s, int on, int band_rows);

/* Longest step sequence lbm_run replays from one captured HIP graph
 * (0: one launch per step; at most 4096). The default is 256 for population
 * copies up to 16 MiB, where launch latency dominates the step, and 0 above.
 * LBM_E_UNSUPPORTED for a non-zero value in FP16-deviation storage, whose
 * stochastic rounding keys on the step counter (a replay repeats its launch
 * arguments). Graphs are captured on a private stream and launched on the
 * solver's stream; they use runtime-managed kernel-argument memory, no
 * caller buffer. */
int lbm_solver_set_graph_steps(lbm_solver_t *s, int max_steps);

/* Run until |mdot_k - mdot_{k-1}| / |mdot_k| < tol, where mdot is evaluated
 * every check_every steps; blocking (synchronises the stream at each check).
 * *steps = steps done, *mdot = last mass flow. LBM_E_NOT_CONVERGED if
 * max_steps is reached first. */
int lbm_run_to_tol(lbm_solver_t *s, double tol, int check_every, int64_t max_steps,
                   int64_t *steps, double *mdot);

/* Moments of the current state after streaming (the pre-collision state of the
 * next step, Eq. nm.10): rho_dev[nodes], u_dev[nodes * 3] (device FP64, may be
 * NULL); *mdot_host = normalised mass flow (Eq. pf.1), *mass_host = total mass
 * (host, may be NULL). Blocking when a host output is requested. */
int lbm_observe(lbm_solver_t *s, double *rho_dev, double *u_dev, double *mdot_host,
                double *mass_host);

/* Post-collision populations as FP64 [alpha][z][y][x] (device array of
 * V * nodes doubles, alpha in lbm_dvm_info order). */
int lbm_export_populations(lbm_solver_t *s, double *out_dev);

/* Replace the state by FP64 [alpha][z][y][x] populations (checkpoint resume);
 * rounds to the storage type (to nearest: an exported state re-imports
 * bit-exactly) and rebuilds the wall-flux balance. The step counter, which keys
 * stochastic rounding, is kept, so export, import and run continue a run
 * bit-exactly. */
int lbm_import_populations(lbm_solver_t *s, const double *in_dev);

/* Steps taken since the last init/import. */
int lbm_solver_steps(const lbm_solver_t *s, int64_t *steps);

/* ---- batched and served channel solves -------------------------------------
 * Many independent channels (2D, nx = 1: the streamwise-invariant plane
 * Poiseuille problem of Section VI) run together, each to a steady-state
 * tolerance on the mass flow. One workgroup owns one channel at a time and keeps
 * its populations in LDS while it steps; between launches a channel's state
 * lives in HBM, in the caller's pool. Every channel performs exactly the
 * per-node arithmetic of lbm_run, and its convergence test is that of
 * lbm_run_to_tol, so a result does not depend on which other channels share a
 * launch (tested bit for bit).
 *
 * Pool: a caller-owned device buffer. The batch keeps its slot table, velocity
 * tables and work counter at the start of the pool and carves per-channel state
 * (V * ny stored populations) from the rest; a request is admitted when a slot
 * and enough pool bytes are free ("admission by memory"). */

typedef struct {
    uint64_t req_id;   /* the caller's identifier */
    int status;        /* LBM_OK converged, LBM_E_NOT_CONVERGED step cap reached,
                          LBM_E_DEVICE mass flow not finite */
    int ny;
    int64_t steps;     /* steps taken */
    double mdot;       /* last mass flow evaluated (Eq. pf.1) */
    double kn;
} lbm_result_t;

typedef struct {
    int active;        /* channels resident on the device */
    int queued;        /* submitted, not yet admitted */
    int done;          /* finished, not yet returned by poll */
    int threads;       /* workgroup size in use */
    int quantum;       /* steps per launch in the served mode */
    int slots_per_cu;  /* persistent mode: resident workgroups per CU (LDS permitting) */
    int order;         /* persistent mode: work-queue order (LBM_BATCH_*) */
    int64_t graph_replays; /* persistent runs that replayed a captured graph */
    int64_t launches;  /* kernel launches so far */
    size_t pool_used;  /* state bytes allocated */
    size_t pool_free;
} lbm_batch_stats_t;

/* Create a batch with up to max_slots resident channels, all with the given
 * storage (LBM_F32, LBM_F16DEV or LBM_F32RAW), over the caller's device pool
 * (256-byte aligned) and HIP stream. LBM_E_NO_MEMORY if the pool cannot hold
 * the slot table. */
int lbm_batch_create(int max_slots, int storage, void *pool, size_t pool_bytes, void *stream,
                     lbm_batch_t **out);
int lbm_batch_destroy(lbm_batch_t *b);

/* Queue one channel solve: prob->dim = 2, prob->nx = 1, prob->storage equal
 * to the batch's, Hermite order N <= 4 and accommodation 1 (else
 * LBM_E_UNSUPPORTED); the DVM must be D2V17 or D2V37. It runs from the rest
 * state rho0 w until |mdot_k - mdot_{k-1}| < tol |mdot_k| with mdot evaluated
 * every check_every steps, or until max_steps. LBM_E_NO_MEMORY if it can
 * never fit the pool or the LDS of one workgroup. */
int lbm_batch_submit(lbm_batch_t *b, const lbm_dvm_t *dvm, const lbm_problem_t *prob, double tol,
                     int check_every, int64_t max_steps, uint64_t req_id);

/* Served mode, non-blocking: if the launch in flight has finished, harvest
 * finished channels and free their slots and pool bytes; admit queued requests
 * while slots and bytes allow; launch the next quantum over the resident
 * channels. Finished results (up to cap) go to out, their count to *n_out. */
int lbm_batch_poll(lbm_batch_t *b, lbm_result_t *out, int cap, int *n_out);

/* Blocking: poll until every submitted request has finished. */
int lbm_batch_drain(lbm_batch_t *b, lbm_result_t *out, int cap, int *n_out);

/* Batch mode, blocking: admit every queued request (they must all fit), then
 * run them in ONE persistent launch: workgroups take channels from a device
 * work queue (longest estimated first) and step each to its tolerance. The
 * launch is captured in a HIP graph the first time a launch shape (channel
 * count, grid, workgroup size, LDS) occurs and replayed from then on (at most
 * 8 graphs per batch, released by lbm_batch_destroy). */
int lbm_batch_run_persistent(lbm_batch_t *b, lbm_result_t *out, int cap, int *n_out);

/* Work-queue orders of persistent launches. */
#define LBM_BATCH_LONGEST_FIRST 1  /* largest estimated work ny^2 c / tau first (default) */
#define LBM_BATCH_SUBMIT_ORDER 2   /* order of submission */

/* Workgroup size (64..1024, multiple of 64; a channel of ny rows takes
 * ceil(ny / threads) <= 2 rows per thread), steps per served launch,
 * resident workgroups per CU of persistent launches (1..16) and their
 * work-queue order (LBM_BATCH_*); 0 keeps the current slots_per_cu / order.
 * LBM_E_INVALID if a queued or resident channel has more than twice
 * `threads` rows. */
int lbm_batch_tune(lbm_batch_t *b, int threads, int quantum, int slots_per_cu, int order);

typedef struct {
    int threads;       /* chosen workgroup size */
    int slots_per_cu;  /* chosen resident workgroups per CU */
    int order;         /* chosen work-queue order */
    int trials;        /* trial launches timed */
    float trial_ms;    /* the chosen trial's time */
} lbm_batch_tuning_t;

/* Time short persistent trials of the queued requests (each capped at
 * trial_steps steps) for every workgroup size in {256, 384, 512, 768, 1024}
 * that holds the tallest channel, times 1..4 resident workgroups per CU (LDS
 * permitting, at most 2048 threads per CU), times both work-queue orders, and
 * keep the fastest (results are identical for every choice). The queued
 * requests stay queued. `out` may be NULL. */
int lbm_batch_autotune(lbm_batch_t *b, int trial_steps, lbm_batch_tuning_t *out);

int lbm_batch_stats(const lbm_batch_t *b, lbm_batch_stats_t *out);

/* ---- measurement aid (not part of the method) ------------------------------ */

/* Plain streaming copy of `bytes` from src to dst (device buffers, 16-byte
 * aligned, not overlapping; bytes a multiple of 16), asynchronous on `stream`
 * (a hipStream_t; NULL = the default stream): each byte read once and written
 * once, one 16-byte vector per thread, non-temporal stores. Its bandwidth is
 * the practical ceiling the HBM-bound step kernels are compared with, next to
 * the part's peak.
 * LBM_E_INVALID on a bad argument, LBM_E_DEVICE if the launch fails. */
int lbm_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Duration of individual step launches: n times lbm_run(s, steps_per_launch),
 * each bracketed by HIP events recorded on `stream`, which must be the
 * solver's stream (the one it was created with), blocking until all have run; ms_out[k] (host, n floats) receives the
 * k-th run's event-to-event time. system_scope = 1 records the events with a
 * system-scope release (the GPU's caches are written back at each event, as
 * a per-dispatch kernel trace does), 0 with the default device scope.
 * steps_per_launch must match the solver's launch (1 for single steps, 2 for
 * two steps per launch). LBM_E_INVALID on a bad argument, LBM_E_DEVICE on a
 * runtime error. */
int lbm_time_launches(lbm_solver_t *s, void *stream, int n, int steps_per_launch,
                      int system_scope, float *ms_out);

#ifdef __cplusplus
}
#endif
#endif /* LBMDVM_H */
