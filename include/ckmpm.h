/*
 * ckmpm.h - C ABI of the MI355X compact-kernel MPM step.
 *
 * One explicit MLS-MPM / APIC time step of CK-MPM (Liu, Wang, Li: "CK-MPM: A
 * Compact-Kernel Material Point Method", arXiv 2412.10399):
 *   - the C^2 compact kernel K1(x) = 1 - |x| + sin(2 pi |x|)/(2 pi) of section 4.1,
 *     applied as a tensor product on two staggered grids G- and G+ placed a quarter
 *     cell either side of the (unstored) grid G0 (section 4.2);
 *   - particle-to-grid transfer of mass and APIC affine momentum with the MLS stress
 *     force (sections 4.3-4.5): each particle touches the 2x2x2 nodes of its cell on
 *     each grid, 16 nodes in all;
 *   - grid velocity update with gravity and sticky walls (section 3.2, section 4.3);
 *   - grid-to-particle gather of velocity and the affine matrix B, update of the
 *     deformation gradient, plasticity return mapping and advection (section 3.2,
 *     sections 4.3-4.5).
 *
 * Every entry point is plain C: integers, doubles and pointers.  Particle arrays
 * and stream handles belong to the caller; device memory for the sparse grid, the
 * page table, sort scratch and the status word belongs to the library and is
 * allocated once in mpm_create.  Steps never allocate.  No entry point aborts or
 * prints; failures are reported through mpm_status.
 *
 * Conventions
 *   - world position of node i (integer triple, 0..n_cells per axis) of grid G_k,
 *     k = -1 (G-) or +1 (G+):   origin + (i + k/4) * dx;
 *   - a particle is valid while (x - origin)/dx lies in [1/4, n_cells - 1/4) on every
 *     axis (all 16 nodes of its stencil then exist);
 *   - particle state is structure-of-arrays FP32: one allocation of 27 planes of
 *     `stride` floats each, plane order x0 x1 x2 | v0 v1 v2 | B00 B01 B02 B10 .. B22 |
 *     H00 H01 .. H22 | r0 r1 r2 (matrices row-major), element p of plane q at
 *     base[q*stride + p].  The deformation gradient is stored as H = F - I: an FP32 F
 *     near the identity resolves strains only to about 6e-8, H keeps them to FP32
 *     relative precision.  The position is the unevaluated sum x + r: x is the
 *     position rounded to FP32 and r the FP32 remainder (|r| <= ulp(x)/2; zero is
 *     always a valid r).  An FP32 position alone cannot move by less than half its
 *     ulp in a step -- at x = 0.5 a particle slower than 1.5e-3 m/s would not move at
 *     dt = 2e-5 -- so every step advances the pair;
 *   - streams are hipStream_t values passed as void* (NULL = the null stream).
 */
#ifndef CKMPM_H
#define CKMPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CKMPM_ABI_VERSION 3
#define MPM_STATE_PLANES 27

typedef struct mpm_ctx mpm_ctx; /* opaque, owned by the library */

typedef enum {
    MPM_OK = 0,
    MPM_E_INVALID = 1,   /* bad argument or configuration (detected on the host)          */
    MPM_E_OOM = 2,       /* device allocation failed in mpm_create                          */
    MPM_E_DOMAIN = 3,    /* a particle left the valid domain (device-detected)               */
    MPM_E_CAPACITY = 4,  /* block pool or per-block particle capacity exceeded (device)      */
    MPM_E_NONFINITE = 5, /* a NaN/Inf appeared in v, B or F (device-detected)                */
    MPM_E_HIP = 6,       /* a HIP runtime call failed                                        */
    MPM_E_STALE = 7,     /* positions changed after the library computed their cell keys      */
    MPM_E_CFL = 8,       /* in mpm_step, a particle moved more than three cells in one step    */
    MPM_E_SCRATCH = 9    /* mpm_step_noalloc: the buffers do not fit its static scratch          */
} mpm_status;

enum { MPM_FIXED_COROTATED = 0, MPM_DRUCKER_PRAGER = 1 };
enum { MPM_BC_NONE = 0, MPM_BC_STICKY = 1 };
/* mpm_config.transfer: MLS-MPM (section 4.5, the hot path); APIC with the exact
 * kernel gradient for the force and the velocity gradient (section 4.4); PIC
 * (section 4.3: momentum m v only, exact gradients, particles carry no B — their B
 * output is zero).  The exact-gradient transfers run only as phase kernels on the
 * compact kernel (flags 0). */
enum { MPM_TRANSFER_MLS = 0, MPM_TRANSFER_APIC = 1, MPM_TRANSFER_PIC = 2 };
/* mpm_config.flags:
 * MPM_FLAG_FUSED_G2P2G: mpm_step runs each step's G2P and the next step's P2G as one
 *   kernel (section 3.2's fused transfer); same results up to summation order.
 * MPM_FLAG_QUADRATIC: the single-grid quadratic B-spline kernel (27 nodes; node i at
 *   origin + i dx) instead of the compact kernel on the two staggered grids, the
 *   baseline of the paper's comparison (section 6); the same MLS transfers, models
 *   and walls.  mpm_grid_read then fills only the first grid's half.  Positions must
 *   stay in (x - origin)/dx in [1/2, n - 1/2) (MPM_E_DOMAIN).  Not with the fused
 *   step. */
enum { MPM_FLAG_FUSED_G2P2G = 1, MPM_FLAG_QUADRATIC = 2 };

typedef struct {
    int32_t n_cells[3];    /* cells per axis; nodes per axis and grid = n_cells + 1                */
    double dx;             /* cell size; must be a power of two (exact cell keys)                   */
    double origin[3];      /* world position of G0 node (0,0,0)                                     */
    double gravity[3];     /* acceleration added in the grid update                                 */
    int32_t bc;            /* MPM_BC_NONE or MPM_BC_STICKY                                          */
    int32_t bc_band;       /* sticky: zero v~ at nodes closer than bc_band cells to a box face      */
    int64_t max_particles; /* capacity of every per-particle scratch array                          */
    int64_t max_blocks;    /* capacity of the grid block pool (blocks of 4x4x4 nodes, both grids);
                              device memory is about 16 KiB per block (two 2 KiB grids, 12 KiB
                              of sort buckets of up to 2048 particles and their sub-cell codes) */
    int32_t transfer;      /* MPM_TRANSFER_MLS, _APIC or _PIC                                       */
    int32_t flags;         /* 0, MPM_FLAG_FUSED_G2P2G or MPM_FLAG_QUADRATIC                          */
    int32_t deterministic; /* 0 or 1: bitwise reproducible steps (see below)                        */
} mpm_config;

/* mpm_config.deterministic = 1: every result is a function of the inputs alone, so
 * equal inputs give bitwise equal outputs from run to run, alone or beside other
 * work, and a run resumed from a copy of its particle state continues bitwise as
 * the uninterrupted run would.  The only order-dependent sums of the step are the
 * P2G's cross-block additions into the grid (sections 4.3-4.5; per block the
 * fixed-point tile sums are exact).  In this mode each particle block leaves its
 * tile in a staging area (4 x 341 floats per block of max_blocks, allocated in
 * mpm_create) and a gather adds the tiles of the blocks around every node in a fixed
 * order in FP64; the Kirchhoff stress is recomputed from F by every P2G instead of
 * being carried from the previous G2P.  Requires the compact kernel with the MLS
 * transfer and flags 0 (else MPM_E_INVALID). */

typedef struct {
    int32_t model;         /* MPM_FIXED_COROTATED or MPM_DRUCKER_PRAGER                             */
    float E, nu, rho;      /* Young's modulus, Poisson ratio (0 <= nu < 0.5), density               */
    float vol0;            /* initial particle volume V_p^0 (particle mass = rho * vol0)             */
    float friction_deg;    /* Drucker-Prager friction angle in degrees                              */
} mpm_material;

typedef struct {
    int64_t n;             /* live particles                                                         */
    int64_t stride;        /* elements per state plane, n <= stride                                  */
    float *state[2];       /* ping-pong buffers (device), MPM_STATE_PLANES planes each, see above    */
    uint32_t *id[2];       /* optional particle ids (device), permuted with the state; may be NULL   */
    uint8_t *mat[2];       /* optional material index per particle (device), permuted with the state;
                              NULL means material 0 for every particle                               */
    int32_t current;       /* 0 or 1: buffer holding the current state; the library flips it in
                              mpm_g2p and mpm_step, at enqueue time                                   */
    int32_t reserved;
} mpm_particles;

typedef struct {
    int64_t n_particle_blocks; /* 4x4x4-cell blocks holding particles in the last p2g              */
    int64_t n_grid_blocks;     /* grid blocks touched (both grids) in the last p2g                 */
    int64_t max_block_particles;
    uint32_t status_bits;      /* raw device status word (not cleared)                             */
    uint32_t reserved;
} mpm_stats;

/* Create a context.  Validates the configuration on the host (n_cells >= 4, dx a power
 * of two, capacities > 0, 0 < n_mat <= 8, materials with E > 0, 0 <= nu < 0.5, rho > 0,
 * vol0 > 0) and returns MPM_E_INVALID before touching the GPU if any check fails.
 * Allocates every device buffer on the current HIP device; MPM_E_OOM if that fails. */
mpm_status mpm_create(const mpm_config *cfg, const mpm_material *mats, int32_t n_mat, mpm_ctx **out);

/* Free every buffer of the context (synchronises the device first).  NULL is accepted. */
mpm_status mpm_destroy(mpm_ctx *ctx);

/* Sort + activation + P2G (sections 4.3-4.5): computes the particles' cell keys (unless
 * the previous mpm_g2p produced them for this buffer), orders the particles by 4^3-cell
 * block and, inside a block, in layers of one particle per (half-cell octant, cell) bin
 * -- the octant being the half of its G- cell a particle lies in along each axis; layer
 * q takes the q-th particle by index of every bin, in (octant, cell) order, or the
 * whole block runs in (octant, cell, index) order when a bin holds more than 16 --,
 * activates the grid blocks the 16-node
 * stencils touch, clears them and scatters mass and momentum
 * m v + (m B - dt V0 tau) D^-1 (x_i - x_p) to both grids.  Reads the current buffer
 * only.  Enqueued on `stream`; asynchronous. */
mpm_status mpm_p2g(mpm_ctx *ctx, const mpm_particles *p, double dt, void *stream);

/* Grid update (section 4.3): v~ = p/m + dt g on nodes with m > 0, zero elsewhere and
 * on sticky wall nodes.  Overwrites the momentum channels of the pool with v~. */
mpm_status mpm_grid_update(mpm_ctx *ctx, double dt, void *stream);

/* G2P (sections 4.3-4.5): v_p = 1/2 sum w v~, B_p = 1/2 sum w v~ (x_i - x_p)^T,
 * F <- (I + dt B_p D_p^-1) F (applied to H = F - I), Drucker-Prager return mapping,
 * x <- x + dt v_p.  Writes the new state into the other buffer in the order of the
 * preceding mpm_p2g (ids and materials permuted alongside), computes the next cell
 * keys, and flips p->current. */
mpm_status mpm_g2p(mpm_ctx *ctx, mpm_particles *p, double dt, void *stream);

/* nsteps x (p2g, grid_update, g2p), enqueued back to back without host syncs.  Inside
 * the sequence (compact kernel, MLS transfer, not deterministic) every G2P but the last
 * stores, in place of B, the matrix Q = (m B - dt V0 tau) D^-1 / dx that the next P2G
 * scatters, and no stress, so that the next P2G reads neither; the last step stores
 * the whole state.  The other ping-pong buffer's contents afterwards are unspecified.
 * With
 * MPM_FLAG_FUSED_G2P2G, each step's G2P and the next step's P2G run as one kernel
 * from the second step on (the same arithmetic; the grid each fused P2G writes is the
 * 3x3x3 block neighbourhood of the particle blocks, so a particle may move at most
 * three cells per step, else MPM_E_CFL).  Either way the state, the grid left for
 * mpm_grid_read and the carried keys and stress afterwards are those of the phase
 * calls, up to summation order. */
mpm_status mpm_step(mpm_ctx *ctx, mpm_particles *p, double dt, int32_t nsteps, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops that must not call hipMalloc, harnesses that forbid it): mpm_step
 * without a context.  The call validates cfg, mats and p as mpm_create and mpm_step
 * do, then runs nsteps steps exactly as mpm_step on a context created from the same
 * configuration would (same kernels, same results), with every library buffer carved
 * from one static device array of MPM_NOALLOC_SCRATCH_BYTES per GPU, held from the
 * first call on that GPU until the process ends.  It calls no hipMalloc, hipFree or
 * other allocating routine; the caller still owns the particle buffers.
 *   - The buffers needed are those mpm_create would allocate for cfg (a function of
 *     n_cells, max_particles, max_blocks and deterministic; mpm_footprint(cfg, 0)
 *     counts them); beyond MPM_NOALLOC_SCRATCH_BYTES the call returns MPM_E_SCRATCH
 *     before any GPU work.  A 32^3-cell grid with 32,768 particles and max_blocks 729
 *     needs about 14 MB.
 *   - Every call starts from a cleared state (keys, stress and page tables are
 *     recomputed from the particles) by fill kernels on `stream`; nothing carries over
 *     from the previous call, whose contents stay in the array.
 *   - Calls that overlap on one GPU share the array and race: serialise them (one
 *     stream, or events).
 *   - Device-detected errors: when `status` (device memory, one int32) is not NULL, a
 *     kernel enqueued after the steps writes the mpm_status code mpm_sync would have
 *     returned (MPM_OK when none); the call itself returns host-detected errors only.
 * Asynchronous on `stream`; p->current flips as in mpm_step. */
#define MPM_NOALLOC_SCRATCH_BYTES (32 * 1024 * 1024)
mpm_status mpm_step_noalloc(const mpm_config *cfg, const mpm_material *mats, int32_t n_mat, mpm_particles *p,
                            double dt, int32_t nsteps, int32_t *status, void *stream);

/* Wait for `stream`, then return (and clear) the device status word as a status code:
 * NONFINITE before DOMAIN before CAPACITY before STALE before CFL. */
mpm_status mpm_sync(mpm_ctx *ctx, void *stream);

/* Export grid `grid` as dense arrays (device pointers): -1 for G-, +1 for G+, each as
 * m[nz+1][ny+1][nx+1] and vec[nz+1][ny+1][nx+1][3]; 0 for both, as m[2][..] and
 * vec[2][..][3] with index 0 = G-, 1 = G+.  After mpm_p2g vec holds momentum, after
 * mpm_grid_update it holds v~.  Nodes outside active blocks are written as 0.
 * Either pointer may be NULL; any other `grid` is MPM_E_INVALID.  For tests and
 * diagnostics. */
mpm_status mpm_grid_read(mpm_ctx *ctx, int32_t grid, float *m, float *vec, void *stream);

/* Which ping-pong buffer (0 or 1) the last mpm_g2p or mpm_step of this context wrote
 * the particle state into -- the value it left in mpm_particles.current -- or -1
 * before the first one (or for a NULL context). */
int32_t mpm_current_buffer(const mpm_ctx *ctx);

/* Cell keys of the current buffer (computed from positions) and the stable sorting
 * permutation by key: keys[p] = block * 64 + cell (block = 4^3-cell block of the G- cell
 * c = floor((x - origin)/dx + 1/4)), perm[j] = index of the j-th particle in key order
 * (ties in index order).  Device output arrays of n.  Invalidates a pending mpm_g2p. */
mpm_status mpm_sort_keys(mpm_ctx *ctx, const mpm_particles *p, uint32_t *keys, uint32_t *perm, void *stream);

/* Forget cached cell keys: call after changing particle positions in place. */
mpm_status mpm_invalidate(mpm_ctx *ctx);

/* Synchronous statistics of the last p2g (blocks, largest block). */
mpm_status mpm_get_stats(mpm_ctx *ctx, mpm_stats *out, void *stream);

/* Per-phase timing with HIP events on the launch stream: enable, read totals (ms) and
 * interval counts of the phases {sort+activate, p2g, grid update, g2p, fused g2p+p2g}
 * since enabling (n_phases <= 5 are filled).  In mpm_step the steps after the first
 * time the fused kernel as phase 4 and have no separate g2p; the last step's sort and
 * G2P together count as g2p. */
mpm_status mpm_profile_enable(mpm_ctx *ctx, int32_t enable);
mpm_status mpm_profile_read(mpm_ctx *ctx, double *total_ms, int64_t *count, int32_t n_phases);

const char *mpm_status_string(mpm_status s);
int32_t mpm_abi_version(void);

/* Device memory (bytes) a context with this configuration and particle capacity
 * holds, plus two ping-pong particle buffers of n particles with ids and material
 * indices, each buffer counted as the library's allocators pad it (256 bytes of
 * slack, rounded up to 256).  This is exactly what a served job occupies. */
int64_t mpm_footprint(const mpm_config *cfg, int64_t n);

/* ------------------------------------------------------------------ serving
 * A server runs many independent simulation jobs on one GPU with continuous
 * batching.  It reserves its device memory once (an arena of memory_budget bytes)
 * and never allocates after that.  A submitted job waits until a resident slot and
 * enough arena memory (mpm_footprint of the job) are free; it is then admitted: its
 * context and particle buffers are carved from the arena, its initial state is
 * copied in, and from then on it stays resident in HBM and advances
 * steps_per_launch steps at a time on one of the server's streams, interleaved with
 * the other resident jobs.  After the first launch, a job's launches replay one
 * HIP graph captured from that job's step sequence.  Finished jobs keep their final
 * state until released.  All calls are non-blocking except mpm_server_drain,
 * mpm_server_job_read and mpm_server_destroy.  Calls on one server must not overlap
 * (one thread at a time). */
typedef struct mpm_server mpm_server;

typedef struct {
    int64_t memory_budget;     /* arena bytes for resident jobs (allocated in mpm_server_create)      */
    int32_t max_jobs;          /* resident (admitted, unreleased) jobs at most, >= 1                   */
    int32_t n_streams;         /* HIP streams the jobs are spread over, 1..64                          */
    int32_t steps_per_launch;  /* steps per launch, even (the ping-pong buffer returns to its start)  */
    int32_t flags;             /* 0 or MPM_SERVER_GROUPED                                              */
} mpm_server_config;

/* mpm_server_config.flags: jobs are sorted into size-class lanes (particle counts
 * eight-fold apart from 2^10 up, min(n_streams, 4) lanes, the last taking every larger
 * job); every phase of a step runs as one launch for all active jobs of a lane
 * (workgroup row y of each launch works on job y), steps_per_launch steps per round,
 * instead of each job launching its own kernels on its own stream.  Each lane runs its
 * rounds on its own stream, a round replaying a captured HIP graph while the lane's
 * job set is unchanged.  Jobs must use the compact kernel with the MLS transfer and
 * no config flags (else mpm_server_submit returns MPM_E_INVALID). */
enum { MPM_SERVER_GROUPED = 1 };

typedef struct {
    mpm_config cfg;            /* grid, walls and capacities of the job (max_particles >= n)           */
    const mpm_material *mats;  /* copied at submission                                                 */
    int32_t n_mat;
    int32_t nsteps;            /* steps to run, >= 0                                                   */
    int64_t n;                 /* particles, >= 1                                                      */
    const float *state;        /* initial state (device), 27 planes of stride n, H = F - I; copied at
                                  admission, so it must stay valid while the job is pending           */
    const uint8_t *mat;        /* optional per-particle material index (device, n), or NULL           */
    double dt;
    void *stream;              /* hipStream_t on which state and mat were produced (NULL = the null
                                  stream): the admission copy waits for the work queued there before
                                  mpm_server_submit (an event recorded at submission)               */
} mpm_job_desc;

enum { MPM_JOB_PENDING = 0, MPM_JOB_ACTIVE = 1, MPM_JOB_DONE = 2, MPM_JOB_FAILED = 3 };

typedef struct {
    int32_t state;             /* MPM_JOB_*                                                            */
    int32_t steps_done;
    int64_t n;
    int64_t footprint;         /* arena bytes while resident                                           */
    double t_submit, t_admit, t_done;   /* seconds on the server's clock (0 until reached)           */
    mpm_status status;         /* outcome: MPM_OK when done, the device status when failed             */
    int32_t reserved;
} mpm_job_info;

/* Allocates the arena and the streams (default priority). */
mpm_status mpm_server_create(const mpm_server_config *cfg, mpm_server **out);
/* Waits for every stream, then frees everything, including unreleased jobs. */
mpm_status mpm_server_destroy(mpm_server *srv);
/* Queues a job (validated on the host; MPM_E_CAPACITY if its footprint exceeds the
 * whole budget).  Job ids start at 0 and increase by one per submission. */
mpm_status mpm_server_submit(mpm_server *srv, const mpm_job_desc *job, int64_t *job_id);
/* Retires finished launches, admits waiting jobs in submission order and enqueues
 * the next launch of every resident job that has none in flight.  Returns at once;
 * the counts are optional. */
mpm_status mpm_server_poll(mpm_server *srv, int32_t *n_pending, int32_t *n_active, int32_t *n_done);
/* Polls until no job is pending or active (blocking on in-flight launches). */
mpm_status mpm_server_drain(mpm_server *srv);
mpm_status mpm_server_job_info(mpm_server *srv, int64_t job_id, mpm_job_info *info);
/* Copies a finished job's state (27 planes of stride n) and particle ids (the
 * initial index of each particle; the state is in the library's particle order)
 * into device buffers; either pointer may be NULL.  Synchronous. */
mpm_status mpm_server_job_read(mpm_server *srv, int64_t job_id, float *state, uint32_t *ids);
/* Returns a finished job's memory to the arena. */
mpm_status mpm_server_job_release(mpm_server *srv, int64_t job_id);
/* Per-step latencies (seconds, GPU event time between the ends of consecutive
 * launches of a job divided by the launch's steps; the first launch of a job is
 * timed from its admission).  Writes up to cap values in completion order and the
 * total count to *count. */
mpm_status mpm_server_step_latencies(mpm_server *srv, double *out, int64_t cap, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* CKMPM_H */
