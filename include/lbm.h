/*
 * lbm.h -- C ABI of the MI355X (gfx950) particle-resolved thermal lattice
 * Boltzmann library: the per-step hot path of Xu & Li, "Particle-resolved
 * thermal lattice Boltzmann simulation using OpenACC on multi-GPUs"
 * (arXiv 2308.16597).
 *
 * One step (Sec. 2 and Sec. 3 of the paper) is:
 *   1. collect the fluid-particle links into an index array, each
 *      particle's links packed at the front of its own segment of
 *      12 N - 12 entries (the paper's extended indirect addressing, Sec. 3);
 *   2. at every link: interpolated moving-wall bounce-back (Sec. 2.3,
 *      Eqs. (9)-(10)), the thermal curved-wall condition (Eqs. (11)-(12)) and
 *      the momentum-exchange force and torque (Sec. 2.4, Eqs. (13)-(14));
 *   3. per particle: FP64 reduction, spring repulsion (Eq. (15)), net weight
 *      and the Newton-Euler update (Sec. 2.2, Eqs. (7)-(8));
 *   4. the solid/fluid map at the new positions;
 *   5. the fused pull-stream + collide of the D2Q9 flow and D2Q5 heat MRT
 *      models with Boussinesq buoyancy (Sec. 2.1, Eqs. (5)-(6)) over the
 *      whole lattice, flat walls included;
 *   6. refilling (and collision) of newly uncovered fluid nodes (Sec. 2.5,
 *      Eqs. (16)-(17)).
 *
 * Geometry: node (i, j) is at (x, y) = (i, j), 0 <= i < nx, 0 <= j < ny; x is
 * periodic, or (periodic_x = 0, the closed cavity) bounded by static side
 * walls at x = -1/2 and x = nx - 1/2; the flat walls are halfway between
 * nodes, at y = -1/2 and y = ny - 1/2.  Gravity points along -y.  D2Q9 velocities e0..e8 are
 * (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1); D2Q5 uses the
 * first five.
 *
 * Conventions for every function:
 *   - The return value is a status (LBM_OK or a negative LBM_E* code);
 *     lbm_last_error gives a message for the handle (or, for a failed
 *     create, for the calling thread).
 *   - Host arrays belong to the caller and are never retained.  Field arrays
 *     hold nx*ny values, row-major (index j*nx + i).  Any output pointer may
 *     be NULL to skip that output.
 *   - Work is enqueued on the handle's HIP stream.  lbm_step returns without
 *     waiting; the lbm_read_* functions, lbm_sync and lbm_destroy wait for the
 *     stream.  Errors detected on the device (non-finite populations, a
 *     particle moving more than half a lattice spacing in one step, link
 *     array overflow) are reported by the next waiting call as
 *     LBM_EUNSTABLE.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Particle neighbours are searched on a cell grid of cells at least
 *     max_diameter + rep_range wide holding at most 7 particles each; a fuller
 *     cell is reported as LBM_EUNSTABLE.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 4

typedef struct lbm_sim* lbm_handle;

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument or parameter (checked on the host) */
    LBM_ENOMEM = -2,     /* device allocation failed */
    LBM_EDEVICE = -3,    /* HIP runtime error */
    LBM_ESEED = -4,      /* particle seeding could not place every particle */
    LBM_EUNSTABLE = -5,  /* the run became non-finite or a particle moved too fast */
    LBM_ESTATE = -6,     /* call not allowed in the handle's current state */
    LBM_EBUDGET = -7,    /* the caller's arena (device budget) is smaller than the run needs */
};

/* Population storage.  F64 computes in FP64; the others compute in FP32.
 * The SHIFT_ modes store deviations f_i - w_i rho0 and g_k - w_k T_shift. */
enum {
    LBM_STORE_F64 = 0,
    LBM_STORE_F32 = 1,
    LBM_STORE_SHIFT_F32 = 2,
    LBM_STORE_SHIFT_F16 = 3,
    LBM_STORE_SHIFT_BF16 = 4,
};

/* Population layout.  TWO_SETS streams from one set of 14 arrays into the
 * other (pull); IN_PLACE keeps one set and alternates the AA pattern's two
 * kernels (half the population memory, the same bytes per lattice update,
 * the same results bit for bit). */
enum {
    LBM_STREAM_TWO_SETS = 0,
    LBM_STREAM_IN_PLACE = 1,
};

/* Simulation parameters, all in lattice units.  Fill with lbm_params_default
 * and override.  Relaxation rates <= 0 select the defaults:
 *   s_nu = 1/(3 nu + 1/2); s_e = s_eps = s_nu; s_q from
 *   (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16; s_alpha = 1/(alpha/cs_T^2 + 1/2) with
 *   cs_T^2 = (4 + a_T)/10; sT_e = sT_p from (1/s_alpha - 1/2)(1/s_T - 1/2) = 1/4. */
typedef struct {
    int32_t abi_version;   /* must be LBM_ABI_VERSION */
    int32_t nx, ny;        /* 8 <= nx, ny <= 65535 */
    int32_t periodic_x;    /* 1: periodic; 0: static side walls (no-slip, Dirichlet side_T) */
    int32_t periodic_y;    /* 0: flat walls at y (required with particles); 1: periodic */
    int32_t storage;       /* LBM_STORE_* */
    double rho0;           /* reference density (> 0) */
    double nu, alpha;      /* kinematic viscosity, thermal diffusivity (> 0) */
    double gravity;        /* |g|, along -y */
    double beta;           /* thermal expansion coefficient */
    double T_ref;          /* T0 of the buoyancy force rho g beta (T - T0) y^ */
    double body_fx;        /* uniform extra force density along +x */
    double s_e, s_eps, s_q;/* D2Q9 free rates */
    double a_T;            /* D2Q5 equilibrium constant (n_e^eq = a_T T), -4 < a_T <= 1 */
    double sT_e, sT_p;     /* D2Q5 free rates */
    double wall_T[2];      /* Dirichlet temperature of the [bottom, top] wall */
    double wall_ux[2];     /* tangential velocity of the [bottom, top] wall */
    double T_fluid0;       /* initial fluid temperature */
    double particle_T;     /* particle surface temperature T_w */
    double rho_ratio;      /* particle/fluid density ratio */
    int32_t repulsion;     /* 1: spring repulsion between particles and with walls */
    double rep_eps;        /* stiffness epsilon_w */
    double rep_range;      /* threshold distance s */
    double T_shift;        /* SHIFT_ storage: g is stored as g_k - w_k T_shift */
    int32_t max_particles; /* capacity for particles (>= 0) */
    double max_diameter;   /* largest particle diameter the buffers are sized for */
    double side_T[2];      /* periodic_x = 0: Dirichlet temperature of the [left, right] wall */
    int32_t streaming;     /* LBM_STREAM_* */
} lbm_params;

/* Phases reported by lbm_time_phases, in the order of a sequential step.
 * The links a step uses are collected at the end of the step before it (and
 * by lbm_set_particles for the first). */
enum {
    LBM_PHASE_LINKS = 0,     /* bounce-back, thermal wall, momentum exchange per link */
    LBM_PHASE_PARTICLES = 1, /* per-particle sums, repulsion, net weight, Newton-Euler */
    LBM_PHASE_MASK = 2,      /* solid map at the new positions (in place: and the refill's values) */
    LBM_PHASE_LATTICE = 3,   /* fused stream + collide over the lattice */
    LBM_PHASE_REFILL = 4,    /* refilling of newborn nodes (in place: their store) */
    LBM_PHASE_COLLECT = 5,   /* link collection of the next step into the index array */
    LBM_NPHASES = 6
};

/* Library ABI version (LBM_ABI_VERSION). */
int32_t lbm_abi_version(void);

/* Defaults: 64 x 64 periodic-x channel, rho0 = 1, nu = alpha = 0.1, no
 * gravity, a_T = -2, FP64 storage, repulsion on with eps = 0.001 and s = 3
 * (Sec. 2.4), particle_T = 1, rho_ratio = 1.5, no particles. */
void lbm_params_default(lbm_params* p);

/* Device bytes a handle with these parameters needs (0 if invalid); the
 * size lbm_create_in_arena requires, and what a server admitting runs into a
 * fixed device budget compares against it.  The largest parts: two sets of
 * 9 + 5 population arrays over the padded lattice (Sec. 2.1; one set in
 * place), two owner maps, and max_particles link segments of 12 N - 12
 * entries (Sec. 3). */
size_t lbm_bytes_required(const lbm_params* p);

/* Admission of a run into a device budget: LBM_OK if a handle with these
 * parameters fits budget_bytes (lbm_bytes_required), LBM_EBUDGET if not,
 * LBM_EINVAL for invalid parameters (message: lbm_last_error(NULL)).  Host
 * only. */
int lbm_check_budget(const lbm_params* p, size_t budget_bytes);

/* Dynamic LDS bytes one block of the link collection (Sec. 3) requests for
 * these parameters, the largest over 1..max_particles particles (0 if
 * invalid or without particles).  The library keeps it within 64 KiB: where
 * four particles' windows would not fit one block, each particle takes a
 * whole block.  Host only. */
size_t lbm_collect_lds_bytes(const lbm_params* p);

/* Create a handle for one run of the method of Secs. 2-3: validate on the
 * host (relaxation times above 1/2 follow from nu, alpha > 0, Eqs. (5)-(6);
 * lattice of at least 8 x 8; particle windows of Sec. 3 no wider than the
 * lattice; a known storage mode), allocate device memory with hipMalloc, and
 * initialise the fluid at rest (rho0, T_fluid0) with no particles.
 * hip_stream is a hipStream_t (NULL: the handle creates its own stream).
 * On failure *out is NULL and lbm_last_error(NULL) explains: LBM_EINVAL for
 * invalid parameters, LBM_ENOMEM when hipMalloc runs out of device memory,
 * LBM_EDEVICE for any other HIP error (no GPU, for one). */
int lbm_create(const lbm_params* p, void* hip_stream, lbm_handle* out);

/* Same, carving every device buffer out of the caller's allocation
 * [dev_ptr, dev_ptr + bytes), which must be 256-byte aligned (else
 * LBM_EINVAL), hold lbm_bytes_required(p) bytes (else LBM_EBUDGET) and
 * outlive the handle.  Allocates no device memory. */
int lbm_create_in_arena(const lbm_params* p, void* dev_ptr, size_t bytes, void* hip_stream,
                        lbm_handle* out);

/* Wait for the stream and release the handle (and the memory it
 * allocated); the graphs and batch tables that refer to it are dropped. */
void lbm_destroy(lbm_handle h);

/* Message of the last error on h; with h == NULL, of the last failed
 * lbm_create* on the calling thread.  Valid until the next call on h. */
const char* lbm_last_error(lbm_handle h);

/* Host-only: random sequential addition of n disks of the given diameter in
 * an nx x ny channel, written to rows7 (n rows of x, y, r, ux, uy, theta,
 * omega; at rest).  Candidates come from SplitMix64 (x then y, each the top
 * 53 bits of an output times 2^-53, x scaled by nx, y into
 * [min_gap - 1/2 + r, ny - 1/2 - min_gap - r]); a candidate is accepted when
 * its surface gap to every accepted disk (minimum image along x) is
 * >= min_gap.  Fails with LBM_ESEED after 1000 n attempts. */
int lbm_rsa_seed(int32_t nx, int32_t ny, int32_t n, double diameter, double min_gap,
                 uint64_t seed, double* rows7);

/* lbm_rsa_seed with the handle's lattice, then lbm_set_particles.  Periodic
 * channels only (LBM_EINVAL for the closed cavity, whose particles are
 * placed with lbm_set_particles). */
int lbm_seed_particles(lbm_handle h, int32_t n, double diameter, double min_gap, uint64_t seed);

/* Replace the particles (n rows of x, y, r, ux, uy, theta, omega; host
 * memory) and re-initialise the run: fluid at rest at rho0 and T_fluid0,
 * step counter 0.  Requires n <= max_particles, 1 < r <= max_diameter/2,
 * finite values, walls in y, -1/2 <= y <= ny - 1/2 and, in the closed
 * cavity, -1/2 <= x <= nx - 1/2 (a periodic x is wrapped into [0, nx)). */
int lbm_set_particles(lbm_handle h, int32_t n, const double* rows7);

/* The same for elliptical particles (Sec. 2.6.2): n rows of (x, y, a, b,
 * ux, uy, theta, omega), a the semi-axis along the body axis at angle theta
 * from +x, b the semi-axis across it, 1 < b <= a <= max_diameter/2 (b == a
 * is a circle).  The solid test, link fractions, refill normal, repulsion
 * gaps (along the centre line for pairs, to the supporting line for walls),
 * mass pi a b rho_p and inertia M (a^2 + b^2)/4 follow the ellipse; theta
 * evolves with omega.  lbm_read_particles reports a in the r column. */
int lbm_set_particles_ellipse(lbm_handle h, int32_t n, const double* rows8);

/* Re-initialise fluid nodes to the equilibria f^eq(rho, u) and g^eq(T, u)
 * of the given fields (host arrays of nx*ny); particles are kept; step
 * counter 0. */
int lbm_set_equilibrium(lbm_handle h, const double* rho, const double* ux, const double* uy,
                        const double* T);

/* Link addressing of the link pass (Sec. 3 compares the two).
 * LBM_LINKS_INDIRECT (default): the links are collected into each
 * particle's segment of the index array and the pass runs over them.
 * LBM_LINKS_DIRECT: no collection; the pass runs one thread per lattice
 * node, each fluid node looking for particle neighbours, with FP64 atomic
 * force sums (their order, and so the last bits, vary between runs).  Kept
 * as the ablation; lbm_step_many rejects runs in this mode.  Waits; returns
 * LBM_EINVAL for an unknown mode. */
enum { LBM_LINKS_INDIRECT = 0, LBM_LINKS_DIRECT = 1 };
int lbm_set_addressing(lbm_handle h, int32_t mode);

/* Enqueue nsteps steps of the method (one step: the link pass of Secs.
 * 2.3-2.4 and 3, the particle update of Sec. 2.2, the solid map, the
 * stream-collide of Sec. 2.1 and the refilling of Sec. 2.5) on the handle's
 * stream and return.  Within a step, the particle update, the owner map of
 * t_n+1 and the link collection of t_n+1 run on a second stream of the
 * library's, concurrently with the lattice update; each step ends joined on
 * the handle's stream.  Whole 6-step cycles replay a HIP graph captured once
 * per step state (the state repeats every 6 steps) and kept until the
 * particles change.  LBM_EINVAL for nsteps < 0. */
int lbm_step(lbm_handle h, int32_t nsteps);

/* Advance count runs together, run i by nsteps[i] steps, for serving many
 * independent simulations on one GPU (the method of Secs. 2-3 applied to
 * each run; nothing couples the runs).  Every step kernel is launched once
 * per step as one grid over all runs that still have steps left (a run
 * table in device memory), and whole 6-step cycles of an unchanged set of
 * runs are replayed from a captured HIP graph.  A run computes the same bits
 * as with lbm_step.
 *   hs       count distinct handles of one storage mode
 *   nsteps   count step counts >= 0
 *   stream   HIP stream for the batched work, or NULL for hs[0]'s stream;
 *            it is ordered after, and each handle's stream before, the
 *            work already enqueued on the other.
 * Returns without waiting.  The library keeps device run tables and
 * graphs for the last 16 sets of runs; they are freed when a member handle
 * is destroyed or gets new particles.  Errors are reported on hs[0]
 * (LBM_EINVAL for a null or repeated handle, a negative count or mixed
 * storage modes, LBM_EDEVICE for a failed launch or capture); device errors
 * of a run surface at its next waiting call. */
int lbm_step_many(lbm_handle* hs, int32_t count, const int32_t* nsteps, void* stream);

/* lbm_step_many for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same batched kernels and the same bits, launched one by
 * one (no graph), from run tables and block maps written into a fixed
 * device array of 8 MiB that the library holds, one per GPU, until the
 * process ends.  No hipMalloc, hipFree or graph instantiation is made;
 * the first call on a GPU looks the array up and creates two events.
 *   hs, nsteps, stream  as for lbm_step_many; at most 64 runs per call.
 * The tables of the runs with steps must fit the array (3.8 KiB per run,
 * plus 8 bytes per block of each kernel: a block per 256 lattice nodes of
 * the padded rows, per particle, and per 1 to 4 particles, e.g. 64 runs of
 * 1024 x 2048 with 400 particles each take 4.5 MiB): a call that needs more
 * fails with LBM_EINVAL before enqueuing anything.  Every call on one GPU rewrites that GPU's array:
 * calls that overlap on one GPU (two host threads, or the same call
 * enqueued on two streams that run concurrently) race on it; calls in
 * sequence, on one stream or on streams ordered one after the other, are
 * safe.  The host waits, before rewriting its copy of the tables, until the
 * previous upload from it has completed. */
int lbm_step_many_noalloc(lbm_handle* hs, int32_t count, const int32_t* nsteps, void* stream);

/* Wait for the stream; report deferred device errors (LBM_EUNSTABLE: a
 * non-finite population, a particle faster than half a lattice spacing per
 * step, a link segment or neighbour cell overflowing). */
int lbm_sync(lbm_handle h);

/* Pre-collision macroscopics at the current time (Sec. 2.1): rho, u with
 * the half force, T (NaN inside particles), and the owner map (-1 for
 * fluid, else the particle index). */
int lbm_read_fields(lbm_handle h, double* rho, double* ux, double* uy, double* T, int32_t* owner);

/* Particle state (Sec. 2.2): n rows of x, y, r, ux, uy, theta, omega, Fx,
 * Fy, Tz, where (Fx, Fy, Tz) is the momentum-exchange force and torque of
 * the last step (Sec. 2.4, Eqs. (13)-(14)).  rows10 may be NULL to query *n
 * only.  Waits. */
int lbm_read_particles(lbm_handle h, double* rows10, int32_t* n);

/* The fluid-particle links of the current state (Sec. 3), as the library
 * collected them for the next step, copied out: node index j*nx + i of the fluid node, direction 1..8, particle,
 * and the link fraction q of Sec. 2.3.  The order of the links is
 * unspecified.  With every output NULL only *n_out is set; otherwise cap
 * must be >= the number of links. */
int lbm_read_links(lbm_handle h, int32_t* node, int32_t* dir, int32_t* particle, double* q,
                   int64_t cap, int64_t* n_out);

/* Timing: run nsteps steps with the phases one after another and HIP
 * events around each, then nsteps steps as lbm_step runs them (particle
 * phases concurrent with the lattice phase) with events around the lattice
 * kernel.  ms_out[LBM_NPHASES + 3] receives the mean device time per step
 * of each phase in sequence (ms_out[0 .. LBM_NPHASES-1]), of a sequential
 * step (ms_out[LBM_NPHASES]), of the lattice kernel within overlapped steps
 * (ms_out[LBM_NPHASES+1]) and of an overlapped step (ms_out[LBM_NPHASES+2]).
 * Advances the run by 2 nsteps steps.  Waits. */
int lbm_time_phases(lbm_handle h, int32_t nsteps, double* ms_out);

/* Bandwidth ceiling of the lattice update (Sec. 2.1): enqueue one untimed
 * and reps timed plain copies of the run's 9 + 5 population arrays (the
 * bytes one stream-collide moves, no arithmetic; the rows padded to a
 * multiple of 64 nodes; 8-byte values, whose arrays lie in tiles of 64
 * nodes, copied as one block), with 8-byte and again with 16-byte lanes and
 * non-temporal loads and stores, into the set the next step writes whole
 * (in place: onto itself); *ms_out receives the mean device milliseconds
 * per copy of the faster width.  The state is unchanged.  Waits. */
int lbm_time_copy(lbm_handle h, int32_t reps, double* ms_out);

/* Counters, out[LBM_NSTATS]: steps done; links of the current state (those
 * the next step uses, Sec. 3); newborn nodes refilled (Sec. 2.5) in the last
 * step; device milliseconds per step of the last lbm_step
 * call (0 before one); the HBM rate that implies for the lattice update's
 * algorithmic bytes (28 population values read and written per node,
 * GB/s); particles; lattice nodes; device bytes held.  Waits. */
enum {
    LBM_STAT_STEPS = 0,
    LBM_STAT_LINKS = 1,
    LBM_STAT_NEWBORN = 2,
    LBM_STAT_MS_PER_STEP = 3,
    LBM_STAT_GBPS = 4,
    LBM_STAT_PARTICLES = 5,
    LBM_STAT_NODES = 6,
    LBM_STAT_DEVICE_BYTES = 7,
    LBM_NSTATS = 8
};
int lbm_stats(lbm_handle h, double* out);

#ifdef __cplusplus
}
#endif
#endif
