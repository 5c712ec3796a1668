/*
 * duwp.h -- C ABI of the MI355X (gfx950) DUWP particle pipeline.
 *
 * One call to duwp_step advances every case of a context by one time step of
 * the direct unified wave-particle method (Cao, Liu, Yang, Zhong, arXiv
 * 2305.12071, Sec. 3.4 "Algorithm of DUWP", Steps 1-4): particle moments
 * (Eq. gkt_moment0), classification of particles for absorption into the
 * wave part by the fraction P of Eq. p, resampling of 1-P of the wave part
 * as Maxwellian particles (Eq. maxsample), DSMC no-time-counter collisions
 * with the VHS model (Appendix A), free transport and boundaries (Step 3),
 * a stable counting sort of particles into cells, and the finite-volume
 * update of the wave part with a Navier-Stokes flux (Eq. r1, Sec. 3.3).
 *
 * Conventions
 *  - Every call returns a duwp_status (0 = OK).  No exception crosses the ABI.
 *  - The context owns all device memory: it allocates every buffer at
 *    duwp_init, through the caller's allocator when duwp_opts gives one (the
 *    Python binding passes torch's caching allocator) and with hipMalloc
 *    otherwise, and frees them in duwp_destroy.  No other call allocates device
 *    memory.  Host buffers passed to accessors are owned by the caller and must
 *    hold the documented number of elements.
 *  - Work is queued on the stream given in duwp_opts (NULL: the null stream).
 *    duwp_step returns after the queued steps finish and the device error
 *    word has been read; the error is then reported as a status.
 *  - Cells of all cases are numbered case by case; particle arrays are
 *    structure-of-arrays sorted by cell, with cell offsets.
 *  - Not thread-safe: one host thread per context.
 */
#ifndef DUWP_H
#define DUWP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DUWP_OK = 0,
    DUWP_EINVAL = -1,     /* bad argument or case description */
    DUWP_ENOMEM = -2,     /* device allocation failed */
    DUWP_EDEVICE = -3,    /* a HIP call failed */
    DUWP_ECAPACITY = -4,  /* particle, staging or injection capacity exceeded during a step, or 2^28
                             (FP32; 2^27 FP64) particles or more in one cell or 33 consecutive cells */
    DUWP_ESTATE = -5,     /* non-finite cell state detected */
    DUWP_ERANGE = -6      /* a particle moved more than DUWP_SORT_WINDOW cells in one step */
} duwp_status;

/* Largest number of cells a particle may cross in one step (dt too large otherwise). */
#define DUWP_SORT_WINDOW 16

enum { DUWP_BC_RESERVOIR = 0, DUWP_BC_SPECULAR = 1 };
enum { DUWP_P_RATIONAL = 0,   /* P = max(0, 1 - tau/dt), Eq. p */
       DUWP_P_EXP = 1 };      /* P = 1 - exp(-dt/tau), the QMC probability of Sec. 3.2 */
enum { DUWP_EPS1 = 0, DUWP_EPS12 = 1, DUWP_EPS0 = 2, DUWP_EPS_FULL = 3 }; /* Eq. vp1, eps_12, eps_0, Eq. vp */
enum { DUWP_FP64 = 0,         /* particles and cells in FP64 */
       DUWP_MIXED = 1 };      /* particles in FP32 (position relative to its cell), cells in FP64 */

/* One independent 1D case.  Dimensional (SI) or nondimensional units. */
typedef struct {
    int32_t kind;                 /* informational: 0 shock, 1 Sod, 2 box */
    int32_t ncells;               /* > 0 */
    double x_lo, x_hi, x_split;   /* domain and position of the initial step */
    double rho_L, u_L, T_L;       /* initial state left of x_split; left reservoir state */
    double rho_R, u_R, T_R;       /* initial state right of x_split; right reservoir state */
    double R, omega, T_ref;       /* gas constant, viscosity index (mu ~ T^omega), reference T */
    double m_mol, d_ref;          /* VHS molecule mass and reference diameter (dimensional gas) */
    double lambda_ref, rho_ref;   /* or: reference mean free path at density rho_ref (if > 0) */
    double m_particle;            /* mass per simulated particle per unit area (> 0) */
    double dt;                    /* time step (> 0) */
    int32_t bc_lo, bc_hi;         /* DUWP_BC_* */
    int32_t classify_law;         /* DUWP_P_* */
    int32_t eps_law;              /* DUWP_EPS_* */
    int32_t dsmc_full_dt;         /* 0: collide over (1-P) dt (default); 1: over dt */
    int32_t flux_order;           /* 2: the wave flux's inviscid part takes MUSCL face states
                                     (minmod slopes of (rho,U,V,W,T)); else first order */
    int32_t absorb_stream;        /* 1: an absorbed particle first streams for its sampled free
                                     time t_f < dt (tau/(1-u), or -tau ln(1-u) under the
                                     exponential law) and joins the wave part of the cell it
                                     reaches (leaving through a reservoir, it leaves the domain);
                                     0 (default): it joins the wave part of its own cell at
                                     step start, as the paper's Step 2 states */
    int32_t reserved_case;        /* 0 */
    int64_t capacity;             /* particle capacity of this case; 0 = derived from the mass */
} duwp_case;

/* Tile shapes and thresholds of the step's kernels (the autotuner's knobs).  A
 * zero selects the default.  None of them changes an integer result (the sort
 * is stable and the collisions keep their sequential order whatever the
 * tiling), and only scatter_items (like block_cells) changes a floating one: it
 * sets the order in which the scatter sums each cell's particle moments, so
 * those agree to rounding. */
typedef struct {
    int32_t scatter_items;        /* particles per thread and chunk of multi-wave scatter blocks: 2 or 4 (0: 4) */
    int32_t big_block;            /* threads (candidates per chunk) of the block-per-cell collide:
                                     256, 512 or 1024 (0: 512 with FP32 particles, 256 with FP64) */
    int32_t big_blocks_per_cu;    /* blocks of that kernel per compute unit, 1..8 (0: 2, or 1 for
                                     1024 threads); more than the compute unit's LDS holds at once
                                     run one after another */
    int32_t big_min_particles;    /* a cell collides in that kernel when it holds at least this many
                                     particles ... (0: 4096; at least 64) */
    int32_t big_min_candidates;   /* ... and draws at least this many candidates (0: 4096; at least 64;
                                     2147483647: no cell does, and that kernel is not launched) */
    int32_t collide_by_cell_max;  /* up to this many cells in all a wave per cell runs the other cells'
                                     collisions, beyond it work items cut from the candidate list (0: 8192) */
    int32_t count_dests;          /* destination cells per block of the sort's count-and-base kernel
                                     on large grids, a multiple of 4 in 4..256 (0: 256) */
    int32_t collide_blocks_per_cu; /* 256-thread blocks per compute unit of the wave collide when it
                                     takes work items from the candidate list, 1..256 (0: 16) */
} duwp_tune;

typedef struct {
    uint64_t seed;                /* Philox key: (low 32 bits, high 32 bits + case index) */
    int32_t precision;            /* DUWP_FP64 or DUWP_MIXED */
    int32_t use_graph;            /* 1: replay each step as a captured HIP graph */
    void *stream;                 /* hipStream_t, or NULL */
    double headroom;              /* capacity = headroom * mass / m_particle when capacity = 0 (<= 0: 1.5) */
    int32_t block_cells;          /* threads per block of the per-cell kernels, 64..512 (0: 256) */
    int32_t reserved;             /* 0 */
    /* Device memory provider.  alloc = NULL: hipMalloc and hipFree.  Otherwise
     * duwp_init takes every device buffer from alloc(bytes, alloc_ctx) (device
     * memory of the current device, at least 256-byte aligned, NULL on failure,
     * usable from any stream), and duwp_destroy returns each through
     * free(ptr, alloc_ctx) after the context's streams have finished.  free must
     * be given with alloc. */
    void *(*alloc)(size_t bytes, void *alloc_ctx);
    void (*free)(void *ptr, void *alloc_ctx);
    void *alloc_ctx;
    duwp_tune tune;
} duwp_opts;

typedef struct duwp_ctx duwp_ctx;

/* Host copy of one case's state (FP64 whatever the precision; x absolute).
 * x,u,v,w: [n_particles]; off: [ncells+1]; psi_w: [ncells*5] = (rho, rho U, rho V,
 * rho W, rho E) of the wave part; cr_max: [ncells].  psi_p: [ncells*5], the
 * particle part (Eq. gkt_moment0 over the cell's particles, per unit area), or
 * NULL.  The step sums it in its own order while it sorts; a restore that
 * brings it back resumes bit for bit, one without it sums it afresh from the
 * particles (equal up to rounding order).  avg_sum: [ncells*5], the running
 * sum of Psi_t behind the time average (DUWP_M_AVG_*), or NULL; avg_count: the
 * number of steps in it, which the context shares among its cases. */
typedef struct {
    int64_t n_particles;
    int32_t ncells;
    uint32_t step;
    double *x, *u, *v, *w;
    int64_t *off;
    double *psi_w;
    double *cr_max;
    double *psi_p;
    double *avg_sum;
    int64_t avg_count;
} duwp_state;

/* What duwp_moments returns, each [ncells*5] doubles */
enum {
    DUWP_M_PRIM = 0,      /* (rho, U, V, W, T) of Psi_t = Psi_w + Psi_p, current state */
    DUWP_M_PSI_T = 1,     /* conserved total */
    DUWP_M_PSI_W = 2,     /* conserved wave part */
    DUWP_M_PSI_P = 3,     /* conserved particle part */
    DUWP_M_AVG_PRIM = 4,  /* (rho, U, V, W, T) of the time-averaged Psi_t */
    DUWP_M_AVG_SUM = 5,   /* running sum of Psi_t (divide by duwp_avg_count) */
    /* (Pi, Q, Pi_p, Q_p, rho_w/rho_t) of the current state: the normal stress and
     * heat flux of Eq. gkt_moment1 (xx entry of S, x component of Q), totals and
     * particle parts, and the wave part's share of the mass (Fig. 5f).  The
     * particle part is taken about the cell's total mean velocity; the wave part
     * adds the NS closure its flux carries (Sec. 3.3), -P (4/3) eps mu dU/dx and
     * -P (15/4) R eps mu dT/dx with central differences.  Computed on demand by a
     * kernel over the case's particles. */
    DUWP_M_STRESS_HEAT = 6
};

/* Create a context holding ncases independent cases; all cases step together.
 * Fails with DUWP_EINVAL on an invalid case (ncells <= 0, x_hi <= x_lo, m_particle
 * or dt <= 0, no gas constants, a mode field out of its range, reserved_case not 0)
 * or options (precision, block_cells not a multiple of 64 up to 512, a tuning
 * field out of its range, alloc without free), checked before any device call;
 * DUWP_ENOMEM when buffers do not fit (everything allocated so far is returned).
 * The initial state puts all mass in the wave part (no particles), the first
 * step samples them. */
duwp_status duwp_init(duwp_ctx **out, const duwp_case *cases, int32_t ncases, const duwp_opts *opts);

/* Advance all cases by nsteps >= 0 steps (Sec. 3.4, Steps 2-3, then Eq. r1).
 * Returns the first device error seen (DUWP_ECAPACITY, DUWP_ERANGE, DUWP_ESTATE);
 * after an error the state is undefined but the context may be destroyed or reset
 * with duwp_set_state. */
duwp_status duwp_step(duwp_ctx *ctx, int32_t nsteps);

/* Cell moments of one case into out[len], len >= ncells*5 (see DUWP_M_*).
 * out is host memory, or device memory when out_on_device = 1. */
duwp_status duwp_moments(duwp_ctx *ctx, int32_t case_id, int32_t what, double *out, int64_t len,
                         int32_t out_on_device);

/* For callers that cannot allocate (code under HIP graph capture, serving loops
 * that forbid allocation): duwp_moments into a device buffer out[len], len >=
 * ncells*5, that allocates nothing (device or host), copies nothing to or from
 * the host and does not synchronize.  Its kernels are queued on the context's
 * stream and the call returns; out holds the result once that stream reaches
 * them.  DUWP_M_STRESS_HEAT stages each cell's primitive state in a device array
 * of the library, one per GPU, of DUWP_NOALLOC_MAX_CELLS + 2 rows, held until
 * the process ends: a case with more cells gets DUWP_EINVAL.  Every call on one
 * GPU, from any context, uses that one array, so calls that overlap on a GPU
 * race: queue them on one stream or order them.  Launch failures give
 * DUWP_EDEVICE; the device error word is not read (duwp_sync reads it). */
#define DUWP_NOALLOC_MAX_CELLS 65536
duwp_status duwp_moments_noalloc(duwp_ctx *ctx, int32_t case_id, int32_t what, double *out, int64_t len);
int64_t duwp_avg_count(duwp_ctx *ctx);
duwp_status duwp_reset_average(duwp_ctx *ctx);

/* Particle-steps (particles alive at the start of each step, summed over steps and
 * cases) since duwp_init or the last reset; reset = 1 clears the counter after reading. */
duwp_status duwp_particle_steps(duwp_ctx *ctx, int64_t *psteps, int32_t reset);

/* Particle count, step index and cell count of one case. */
duwp_status duwp_counts(duwp_ctx *ctx, int32_t case_id, int64_t *n_particles, int32_t *ncells,
                        uint32_t *step);

/* Per-cell integers of the last step of one case (each [ncells]): particles absorbed,
 * particles resampled, NTC candidates, accepted collisions; and per case the
 * injected entrants per side [2] and particles leaving through reservoirs. */
duwp_status duwp_diag(duwp_ctx *ctx, int32_t case_id, int32_t *n_abs, int32_t *n_new,
                      int32_t *n_cand, int32_t *n_coll, int64_t *n_inj, int64_t *n_out);

/* Copy one case's state to host buffers sized from duwp_counts (checkpoint, parity).
 * A NULL array is skipped; avg_count is always written. */
duwp_status duwp_get_state(duwp_ctx *ctx, int32_t case_id, duwp_state *st);

/* Replace one case's state (and the context's step index) from host buffers.  The
 * particle moments of the case's cells are loaded from psi_p, or recomputed from
 * the particles when psi_p is NULL (a state whose particles were changed, or one
 * saved by a context of the other precision, whose particles the load rounds, must
 * not bring the old psi_p); other cases keep theirs.  With avg_sum the case's
 * running sums are loaded and the context's step count of the average becomes
 * avg_count (restore every case of a checkpoint with the same count); without,
 * both stay as they are.  The case keeps its place among the others.
 * Host work and transfers are in proportion to the case: its records are uploaded,
 * and when its particle count changes the later cases' records move on the
 * device.  The call clears the context's device error word first, so a context
 * can be reset after DUWP_ECAPACITY, DUWP_ERANGE or DUWP_ESTATE.
 * DUWP_EINVAL if offsets are not monotone, DUWP_ECAPACITY if it does not fit,
 * DUWP_ESTATE if a loaded cell total is not finite. */
duwp_status duwp_set_state(duwp_ctx *ctx, int32_t case_id, const duwp_state *st);

/* Average device duration in ms of each kernel of the step over nsteps eager steps
 * (HIP events on the context stream).  names/ms hold up to cap entries; returns the
 * number of kernels in *count. */
duwp_status duwp_profile(duwp_ctx *ctx, int32_t nsteps, const char **names, double *ms,
                         int32_t cap, int32_t *count);

duwp_status duwp_sync(duwp_ctx *ctx);
void duwp_destroy(duwp_ctx *ctx);
const char *duwp_strerror(duwp_status s);

#ifdef __cplusplus
}
#endif
#endif
