/*
 * swsph.h -- C ABI of the MI355X (gfx950) SPH neighbour-loop library.
 *
 * The library computes, for particles in periodic cubic boxes, the three
 * neighbour loops that SWIFT offloads to GPUs in "Task-parallelism in SWIFT
 * for heterogeneous compute architectures" (Nasar et al.), Section 2.1:
 *
 *   density   number density n_i = sum_j W(r_ij, h_i) and dn_i/dh
 *             (Sec. 2.1.2, Eq. 5-6), mass density rho_i = sum_j m_j W_ij
 *             (Eq. 2) and drho_i/dh, the smoothing length h_i solved by
 *             Newton iteration on h^3 n(h) = eta^3 (Sec. 2.1.2), div v and
 *             curl v (Eq. 3-4), the grad-h factor f_i (Eq. 8, applied as
 *             1/Omega) and the neighbour count;
 *   gradient  the signal velocity max_j v_sig,ij (Eq. 10-11) and the
 *             Laplacian of u -- the per-particle inputs of the dissipation
 *             switches of Sec. 2.1.3 (Eq. 13, Eq. 21);
 *   force     acceleration and du/dt (Sec. 2.1.4, Eq. 17-18) with the
 *             pairwise artificial viscosity of Eq. 7 and Eq. 9-11;
 *
 * plus the adjoint of density -> force (gradients of a scalar loss on a and
 * du/dt with respect to positions, velocities, internal energies, masses).
 *
 * Kernel: M4 cubic spline with support H = eps*h (Sec. 2.1.1, eps = 2 as in
 * the paper's tests, Sec. 3.1).  Cells and tasks: the paper splits the box
 * into cubic cells and runs "self" (one cell) and "pair" (two neighbouring
 * cells) tasks (Sec. 2.2.2); here particles are binned on the GPU into a
 * hierarchy of cubic cells (Morton order, counting sort); every coarsest
 * cell holding at most `tile` particles is an i-tile, and each tile's task
 * is the list of cells -- its own (self) and neighbouring ones (pairs) --
 * found by a recursive cell search, in the spirit of the paper's sub-task
 * recursion down to cells of width ~H.
 *
 * ---------------------------------------------------------------------------
 * Conventions for every entry point
 *   - Return value: 0 (SWSPH_OK) or a negative swsph_status.  On failure
 *     swsph_last_error() returns a thread-local message.  No C++ exception
 *     crosses this boundary.
 *   - Arrays named "device" are device pointers owned by the caller, one
 *     element per particle, contiguous, in the caller's (original) particle
 *     order, of the plan's dtype (float or double) unless stated otherwise.
 *   - The workspace `ws` is caller-owned device memory of at least
 *     swsph_workspace_bytes() bytes, 256-byte aligned; it carries the binned
 *     particles between calls.  The library never allocates device memory
 *     in these calls and never synchronises the stream, except where stated.
 *   - Every call enqueues its work on `stream` (a hipStream_t passed as
 *     void*; NULL = the default stream) and is capturable into a HIP graph.
 *   - Arguments are validated on the host before any HIP call: a bad
 *     argument returns SWSPH_E_ARG without touching the device.
 *   - Conditions only the device can detect (a particle outside its box, a
 *     support radius reaching half the box, Newton not converging, a
 *     workspace too small) are latched into a status word in the workspace
 *     and reported by swsph_read_stats().
 *   - Calls on one workspace must not overlap (same stream, or ordered).
 */
#ifndef SWSPH_H
#define SWSPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWSPH_VERSION 1

typedef enum swsph_status {
    SWSPH_OK = 0,
    SWSPH_E_ARG = -1,       /* invalid argument (host-side check) */
    SWSPH_E_HIP = -2,       /* a HIP runtime call failed */
    SWSPH_E_STATE = -3,     /* loop called before swsph_bin / on a mismatched bin */
    SWSPH_E_CAPACITY = -4,  /* workspace or internal table too small (device) */
    SWSPH_E_REACH = -5,     /* some support radius reaches half a box (device) */
    SWSPH_E_NEWTON = -6,    /* some h did not converge (device) */
    SWSPH_E_DOMAIN = -7     /* a particle lies outside [0, L) (device) */
} swsph_status;

/* device status bits (swsph_stats.status) */
#define SWSPH_ST_CAPACITY 0x1u
#define SWSPH_ST_REACH    0x2u
#define SWSPH_ST_NEWTON   0x4u
#define SWSPH_ST_DOMAIN   0x8u
#define SWSPH_ST_LOOPCAP  0x10u  /* a device loop hit its iteration cap and stopped */

typedef enum swsph_dtype { SWSPH_F32 = 0, SWSPH_F64 = 1 } swsph_dtype;

/* swsph_config.flags */
#define SWSPH_FIXED_H          0x1u  /* density: use the given h, no Newton */
#define SWSPH_NO_VISC          0x2u  /* force: viscosity off */
#define SWSPH_PER_TASK_LAUNCH  0x4u  /* one kernel launch per tile task */
#define SWSPH_FLAT_LAUNCH      0x8u  /* one launch, one wavefront per task, no queue */
#define SWSPH_TIMING           0x10u /* record HIP events around every loop-kernel launch */
/* swsph_step only: the density, gradient and force loops of every box in one
 * persistent launch.  Its task queue holds every density tile, then every
 * gradient/force tile box by box; a gradient/force tile starts once all
 * density tiles of its box are done (a per-box phase counter), with task
 * lists built once beforehand, before h is known, at the density margin
 * over the guessed supports (a superset of what the force loop needs
 * wherever no h ends beyond that margin over its guess).  Boxes where some
 * h did (and tiles whose support outgrew their list) are finished after the
 * launch by the separate-launch path: density fix-up passes, lists at the
 * final h, the gradient/force loop.  Results agree with the default path
 * to rounding (sums in another order), neighbour counts exactly.  Meant for
 * many independent boxes with usable h guesses (Sec. 4 fine-graining). */
#define SWSPH_SINGLE_LAUNCH    0x20u

/* Scheme constants and execution options.  swsph_config_default() fills
 * eta = 1.2348, eps = 2, gamma = 5/3, alpha = 1, beta = 3, h_tol = 2e-6,
 * h_max_iter = 40, dtype = F32, flags = 0, tile and LDS sizes chosen by the
 * library (0). */
typedef struct swsph_config {
    double eta;          /* resolution: h^3 n(h) = eta^3 */
    double eps;          /* support radius H = eps * h */
    double gamma;        /* adiabatic index, P = (gamma-1) rho u */
    double alpha;        /* viscosity coefficient (constant, Eq. 16 with B = 1) */
    double beta;         /* signal-velocity coefficient (Eq. 10) */
    double h_tol;        /* Newton stop: |h^3 n - eta^3| <= h_tol * eta^3 */
    int32_t h_max_iter;  /* Newton sweeps before SWSPH_ST_NEWTON is latched */
    int32_t dtype;       /* swsph_dtype of every particle array */
    uint32_t flags;      /* SWSPH_* flags above */
    int32_t tile;        /* most i-particles per gradient/force task: 8, 16, 32, 64 (0: 64) */
    int32_t lds_cap;     /* staged j-particles per wavefront: 128, 256, 512 (0: 128) */
    int32_t order;       /* task order: 0 cost-descending, 1 Morton cut into one
                            segment per XCD (default) */
    int32_t leaf_max;    /* cell search: refine cells with more particles (0: 64;
                            the density task builds use 8x this, at most 4096) */
    int32_t tile_dens;   /* most i-particles per density task: 8, 16, 32, 64 (0: 16) */
    int32_t lds_cap_dens; /* staged j-particles per wavefront, density loop first pass
                             (0: 512; its fix-up passes stage up to 1024) */
    int32_t reserved[3];
} swsph_config;

/* Particle set.  Positions must lie in [0, box_size[b]) of their box b.
 * box_id (device int32, nullable when n_box == 1) gives each particle's box;
 * box_size and box_count are HOST arrays of n_box entries (box_count may be
 * NULL when n_box == 1: then box_count[0] = n).  h (device, nullable) is the
 * smoothing-length guess for swsph_bin (NULL: estimated from the local
 * particle density) and, with SWSPH_FIXED_H, the fixed smoothing lengths. */
typedef struct swsph_particles {
    int64_t n;
    const void *x, *y, *z;       /* positions (device) */
    const void *vx, *vy, *vz;    /* velocities (device) */
    const void *u;               /* internal energy per unit mass (device) */
    const void *m;               /* masses (device) */
    const int32_t* box_id;       /* device, nullable */
    int32_t n_box;
    const double* box_size;      /* host [n_box] */
    const int64_t* box_count;    /* host [n_box], nullable if n_box == 1 */
    const void* h;               /* device, nullable: guess (or fixed h) */
} swsph_particles;

/* Density results (device, original order).  swsph_density writes every
 * non-null pointer; h, rho and f are required.  The gradient, force and
 * backward calls read h, rho and f from here. */
typedef struct swsph_density_out {
    void *h, *rho, *rho_dh, *wcount, *wcount_dh;
    void *div_v, *curl_x, *curl_y, *curl_z;
    void *f;                     /* grad-h factor 1/Omega */
    int32_t* nngb;               /* #{j != i : r_ij^2 < H_i^2} (binary32 predicate) */
    int32_t* iters;              /* Newton sweeps used (negative: not converged) */
} swsph_density_out;

typedef struct swsph_gradient_out {
    void *v_sig;                 /* max(2 c_i, max_j c_i + c_j - beta mu_ij) */
    void *lap_u;                 /* 2 sum_j (m_j/rho_j)(u_i-u_j) (1/r) dW/dr(r,h_i) */
} swsph_gradient_out;

typedef struct swsph_force_out {
    void *ax, *ay, *az, *dudt;
    int32_t* nint;               /* nullable: #{j != i : r^2 < max(H_i^2, H_j^2)} */
} swsph_force_out;

/* Loss gradients on the force outputs (device, original order). */
typedef struct swsph_force_grad {
    const void *gax, *gay, *gaz; /* dL/da */
    const void *gdudt;           /* dL/d(du/dt) */
} swsph_force_grad;

/* Gradients with respect to the inputs (device, original order, written). */
typedef struct swsph_input_grad {
    void *gx, *gy, *gz, *gvx, *gvy, *gvz, *gu, *gm;
} swsph_input_grad;

typedef struct swsph_stats {
    uint32_t status;             /* SWSPH_ST_* bits latched since the last bin */
    uint32_t n_tiles;            /* gradient/force tile tasks of the last bin */
    uint64_t pairs_tested[4];    /* candidate pairs tested: density (all sweeps), gradient, force
                                    (the joint kernel: the same tests), backward */
    uint64_t pairs_inside[4];    /* pairs inside the support (useful pairs) */
    uint64_t newton_sweeps;      /* sum over density tiles of their sweeps */
    uint32_t newton_max;         /* largest sweep count of a tile */
    uint32_t newton_failed;      /* particles whose h did not converge */
    uint64_t listed;             /* candidate entries written by the task builds */
    uint64_t restages;           /* density tiles that widened their search */
    uint64_t n_tiles_dens;       /* density tile tasks of the last bin */
    uint64_t dens_listed;        /* density tile passes that swept per-particle neighbour
                                    lists (the others re-test the staged set every sweep) */
    uint64_t single_redo;        /* SWSPH_SINGLE_LAUNCH step: gradient/force tiles left to
                                    the separate-launch path */
    uint64_t reserved[3];
} swsph_stats;

typedef struct swsph_plan swsph_plan;

/* Library version (SWSPH_VERSION) and the last error message of this thread. */
int swsph_version(void);
const char* swsph_last_error(void);

/* Defaults listed at swsph_config. */
void swsph_config_default(swsph_config* cfg);

/* Create / destroy a host-side plan: a copy of the configuration, the
 * geometry of the last bin, and cached graphs.  Fails with SWSPH_E_ARG on
 * out-of-range constants (eta, eps, gamma > 1, alpha >= 0, beta >= 0,
 * h_tol > 0, tile/lds_cap values).  Destroying frees host memory only. */
int swsph_plan_create(swsph_plan** out, const swsph_config* cfg);
int swsph_plan_destroy(swsph_plan* plan);

/* Workspace size in bytes for n particles in n_box boxes with the given
 * per-box counts (host, may be NULL for one box) and sizes (host).  Pure
 * host computation. */
int swsph_workspace_bytes(const swsph_plan* plan, int64_t n, int32_t n_box,
                          const int64_t* box_count, const double* box_size,
                          uint64_t* bytes);

/* Bin the particles: per-box Morton key on a 2^k grid of cubic cells, a
 * device counting sort on that key (stable: equal keys keep input order),
 * sorted copies of the particle data in the workspace, the cell table and
 * the i-tiles (cells of at most tile / tile_dens particles).  Section 2.2
 * (cells, self and pair tasks).  The task lists are built by the loop calls.
 * Clears the device status word. */
int swsph_bin(swsph_plan* plan, const swsph_particles* p, void* ws, void* stream);

/* Density loop with Newton iteration on h (Sec. 2.1.2; SWSPH_FIXED_H: at
 * the given h).  Needs swsph_bin on the same particles first. */
int swsph_density(swsph_plan* plan, const swsph_particles* p, swsph_density_out* o,
                  void* ws, void* stream);

/* Gradient loop (Sec. 2.1.3) at the density results d.  The gradient and
 * force loops run in one kernel (one task build, one staging, one pass of
 * distance tests): this call and swsph_force each run it and copy out their
 * own outputs; swsph_gradient_force and swsph_step run it once for both;
 * all give the same bits. */
int swsph_gradient(swsph_plan* plan, const swsph_particles* p,
                   const swsph_density_out* d, swsph_gradient_out* o, void* ws,
                   void* stream);

/* Force loop (Sec. 2.1.4, Eq. 17-18 with the viscosity of Eq. 7, 9-11) at
 * the density results d. */
int swsph_force(swsph_plan* plan, const swsph_particles* p, const swsph_density_out* d,
                swsph_force_out* o, void* ws, void* stream);

/* The gradient (Sec. 2.1.3) and force (Sec. 2.1.4) loops together, at the
 * density results d: one task build and one pass of the joint kernel write
 * both outputs (the same bits as swsph_gradient and swsph_force, at the cost
 * of one of them).  go and fo are both required (SWSPH_E_ARG otherwise). */
int swsph_gradient_force(swsph_plan* plan, const swsph_particles* p,
                         const swsph_density_out* d, swsph_gradient_out* go,
                         swsph_force_out* fo, void* ws, void* stream);

/* Adjoint of density -> force: given dL/da and dL/d(du/dt), overwrite gi
 * with dL/dx, dL/dv, dL/du, dL/dm, differentiating through rho, f and h
 * (h by the implicit function theorem on h^3 n(h) = eta^3).  d must hold
 * the density results of the same particles (Newton converged); pair
 * geometry is recomputed, nothing per pair is stored. */
int swsph_force_backward(swsph_plan* plan, const swsph_particles* p,
                         const swsph_density_out* d, const swsph_force_grad* g,
                         swsph_input_grad* gi, void* ws, void* stream);

/* Time-dependent dissipation switches (Sec. 2.1.3 Eq. 12-16, Sec. 2.1.4
 * Eq. 19-24), the readings of the printed equations: alpha_loc =
 * alpha_V,max S / (v_sig^2 + S) with S = H^2 max(0, -(div v - div v_prev)/dt)
 * (Eq. 13-15, v_sig of the previous gradient loop); alpha_V jumps up to
 * alpha_loc or relaxes towards it as exp(-l c dt / H) (Eq. 12), floored at
 * alpha_V,min; the Balsara factor B = |div v| / (|div v| + |curl v| +
 * bal_eps c / H) (Eq. 16's B); alpha_ij = (alpha_V,i + alpha_V,j)/2
 * (B_i + B_j)/2 replaces the constant alpha of Eq. 9; alpha_c takes one
 * explicit step of d alpha_c/dt = beta_c H lap u / sqrt(u) - (alpha_c -
 * alpha_c,min) v_sig / H (Eq. 21) and is clamped to [alpha_c,min,
 * alpha_c,max (1 - alpha_V,ngb / alpha_V,max)] (Eq. 23-24, alpha_V,ngb the
 * largest alpha_V over the particle's support); the force loop adds the
 * conduction sum_j alpha_c,ij v_c,ij m_j (u_i - u_j) (f_i dW/dr(h_i) +
 * f_j dW/dr(h_j)) / (rho_i + rho_j) to du/dt (Eq. 19), with alpha_c,ij =
 * (P_i alpha_c,i + P_j alpha_c,j) / (P_i + P_j) (Eq. 20) and v_c,ij =
 * |v_ij . r_hat| + sqrt(2 |P_i - P_j| / (rho_i + rho_j)) (Eq. 22). */
typedef struct swsph_switch_params {
    double dt;           /* time step of the switch update (> 0) */
    double av_max;       /* alpha_V,max (> 0) */
    double av_min;       /* alpha_V,min (>= 0) */
    double ell;          /* decay length l of Eq. 12 (>= 0; the paper uses 0.05) */
    double beta_c;       /* beta_c of Eq. 21 (>= 0) */
    double ac_min;       /* alpha_c,min (>= 0) */
    double ac_max;       /* alpha_c,max (>= alpha_c,min) */
    double bal_eps;      /* Balsara softening in units of c / H (>= 0) */
} swsph_switch_params;

/* Per-particle switch state (device arrays of the plan's dtype, caller's
 * order).  alpha_v and alpha_c are read (time t) and overwritten (t + dt);
 * div_v_prev and v_sig_prev are the previous step's density and gradient
 * outputs; balsara and alpha_v_ngb, when not NULL, receive B and the
 * largest alpha_V over each support. */
typedef struct swsph_switch_state {
    void* alpha_v;
    void* alpha_c;
    const void* div_v_prev;
    const void* v_sig_prev;
    void* balsara;
    void* alpha_v_ngb;
} swsph_switch_state;

/* Gradient and force loops with the switches at the density results d
 * (which must include div_v and curl_x/y/z): the viscosity switch, the
 * gradient loop (v_sig, lap u and alpha_V,ngb), the conduction switch, then
 * the force loop with alpha_ij and conduction.  Needs swsph_bin and
 * swsph_density on the same particles; go and fo are written like
 * swsph_gradient / swsph_force (nint optional).  Arguments are checked on
 * the host (SWSPH_E_ARG). */
int swsph_gradient_force_sw(swsph_plan* plan, const swsph_particles* p,
                            const swsph_density_out* d, const swsph_switch_params* sp,
                            swsph_switch_state* st, swsph_gradient_out* go,
                            swsph_force_out* fo, void* ws, void* stream);

/* Leapfrog time integration between force evaluations (kick-drift-kick;
 * the paper's correctness test integrates the Gresho-Chan vortex in time
 * with SWIFT, Sec. 3.1, Fig. 6): v += a dt_kick and u += du/dt dt_kick
 * (skipped when dt_kick == 0; then a and dudt may be NULL), then
 * x += v dt_drift with the kicked v, wrapped into [0, box_size[b]) of the
 * particle's box b (skipped when dt_drift == 0).  All arrays are device
 * arrays of n elements of the plan's dtype in the caller's order, updated
 * in place; box_id (device, nullable when n_box == 1) and box_size (host,
 * n_box <= 64 entries) as in swsph_particles.  No binning needed; the next
 * swsph_bin takes the moved particles.  Argument errors: SWSPH_E_ARG. */
int swsph_kick_drift(const swsph_plan* plan, int64_t n, void* x, void* y, void* z, void* vx,
                     void* vy, void* vz, void* u, const void* ax, const void* ay,
                     const void* az, const void* dudt, double dt_kick, double dt_drift,
                     const int32_t* box_id, int32_t n_box, const double* box_size,
                     void* stream);

/* One whole step: bin, density, gradient and force (go / fo may be NULL to
 * skip that loop).  The step is captured once into a HIP graph (on a
 * stream the plan creates) and replayed on `stream` while the particle,
 * output and workspace pointers, the sizes, the box data and the options
 * stay the same; a change re-captures.  The box table is uploaded on
 * `stream` at each capture.  Each loop is one persistent launch over the
 * tiles of every box (the fine-graining answer of Sec. 4.4.3).  With
 * SWSPH_PER_TASK_LAUNCH or SWSPH_TIMING the calls run eagerly instead.
 * Same errors as the four calls it makes. */
int swsph_step(swsph_plan* plan, const swsph_particles* p, swsph_density_out* d,
               swsph_gradient_out* go, swsph_force_out* fo, void* ws, void* stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * step as swsph_step (bin, density, gradient, force; go / fo may be NULL),
 * run eagerly, with no workspace argument.  The library's scratch is a
 * file-scope device array of SWSPH_STATIC_SCRATCH_BYTES (64 MiB), one copy
 * on each GPU the library runs on, held until the process ends; its address
 * is looked up once per device.  This call allocates nothing (no hipMalloc,
 * no hipFree, no allocating library routine); the caller passes inputs and
 * outputs as for swsph_step.  A particle set whose workspace would exceed
 * the scratch (about 53,000 particles in float32, 43,000 in float64 in one
 * box; fewer with many boxes) is rejected with SWSPH_E_ARG before any HIP
 * call.  Every call on one GPU shares that GPU's scratch and binds the plan
 * to it, so calls that overlap on one GPU (other streams, other threads,
 * other plans) race: order them.  The scratch keeps the last call's contents; each call
 * clears what it counts from.  Device conditions are read afterwards with
 * swsph_read_stats(plan, NULL, ...). */
#define SWSPH_STATIC_SCRATCH_BYTES (64ull << 20)
int swsph_step_static(swsph_plan* plan, const swsph_particles* p, swsph_density_out* d,
                      swsph_gradient_out* go, swsph_force_out* fo, void* stream);

/* Copy the device statistics to the host (synchronises the stream).  The
 * return value is SWSPH_OK, or the first latched device condition as a
 * negative status (the stats are filled in either case).  ws NULL: the
 * workspace of the plan's last bin. */
int swsph_read_stats(swsph_plan* plan, const void* ws, swsph_stats* out, void* stream);

/* Time the candidate tile sizes, LDS capacities, task orders and task-search
 * leaf sizes on these particles (coordinate descent; runs bin + step several
 * times, synchronises) and store the fastest in the plan.  cache_path (nullable) names a text file used to
 * reuse the choice across processes (key: device, n, n_box, dtype). */
int swsph_autotune(swsph_plan* plan, const swsph_particles* p, void* ws, void* stream,
                   const char* cache_path);

/* Per-launch duration of the loop kernels, from HIP events the library
 * records on the call's stream around each loop-kernel launch when the plan
 * has SWSPH_TIMING (index 0 density, 1 the gradient loop with switches, 2 the
 * force loop (the joint gradient and force loop, or the force loop with
 * switches), 3 backward pair passes).  ms[k] = mean milliseconds per launch, launches[k] = launches
 * timed since the last reset.  Synchronises the stream.  Without
 * SWSPH_TIMING every entry is 0. */
int swsph_kernel_times(swsph_plan* plan, double ms[4], uint64_t launches[4], void* stream);

/* Forget the recorded kernel timings. */
int swsph_reset_timers(swsph_plan* plan);

/* The execution options in effect (after defaults or swsph_autotune). */
typedef struct swsph_tuning {
    int32_t tile, tile_dens, lds_cap, lds_cap_dens, order, leaf_max;
} swsph_tuning;
int swsph_plan_get_tuning(const swsph_plan* plan, swsph_tuning* out);

#ifdef __cplusplus
}
#endif

#endif /* SWSPH_H */
