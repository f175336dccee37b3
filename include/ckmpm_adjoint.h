/* Differentiable compact-kernel MPM step (reverse mode), MI355X / gfx950.
 *
 * The forward step is the one of ckmpm.h (sections 4.3-4.5 of arXiv 2412.10399:
 * MLS P2G of mass, affine momentum and stress impulse on the two staggered grids,
 * grid update with gravity and sticky walls, G2P with the F update and advection)
 * for one fixed-corotated material whose Young's modulus is given per particle as
 * exp(logE).  The paper does not treat derivatives; the backward call is the exact
 * vector-Jacobian product of that forward step, every phase reversed in turn:
 * the G2P gather becomes a scatter of particle cotangents to the grid velocities,
 * the grid update's division by the mass is differentiated node by node, the P2G
 * scatter becomes a gather, and the stress is differentiated through the polar
 * factor of F (the (s_i + s_j) denominators of the rotation's derivative).  The
 * positions enter through the kernel weights, through x_i - x_p and through the
 * moment matrix D_p(x_p); the compact kernel is C2, so all of them are
 * differentiable across cell faces.
 *
 * Particles keep their order (no sort).  mpm_ad_create allocates the grids once;
 * the calls allocate nothing.  When max_blocks covers every block of 4x4x4 nodes
 * of the (n+1)^3 node lattice, both staggered grids are dense (about 112 B per
 * node).  Otherwise they are block-sparse: a pool of max_blocks blocks per grid
 * (about 7 KiB per block, plus 10 B per block of the whole lattice for the page
 * tables); each call marks the blocks that its particles' stencils reach on each
 * grid, gives them pool slots and sweeps those slots only.  A call whose particles
 * reach more than max_blocks blocks on a grid reports MPM_E_CAPACITY (its results
 * are then meaningless); later calls are unaffected.
 *
 * State and cotangent layout: 27 planes of `stride` floats, the layout of
 * mpm_particles (x[3] v[3] B[9] H[9] r[3], H = F - I, row-major 3x3, position
 * x + r); a cotangent array has the same planes, its H planes holding dL/dF and its
 * x planes dL/d(position).  The backward call reads the position cotangent from
 * the x planes only and writes dL/d(position) to both the x and the r planes of
 * cot_in (the position depends on x and r alike).  All pointers are device
 * memory owned by the caller; calls are stream-ordered on `stream` (a hipStream_t,
 * NULL for the default stream) and return before the work completes.  The calls
 * of one context share its grids: they must not overlap (issue them on one stream,
 * or order the streams).
 */
#ifndef CKMPM_ADJOINT_H
#define CKMPM_ADJOINT_H
#include "ckmpm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpm_ad_ctx mpm_ad_ctx; /* opaque, owned by the library */

/* Context for the differentiable step.  cfg: grid, cell size, origin, gravity and
 * walls as in mpm_create (max_particles bounds n; max_blocks, the pool capacity of
 * each grid, and flags must be as mpm_create accepts; the transfer is MLS).
 * mat: one material, which must be MPM_FIXED_COROTATED; its E is only a default
 * (every call takes logE).
 * Errors: MPM_E_INVALID for a bad configuration or material, MPM_E_OOM. */
mpm_status mpm_ad_create(const mpm_config *cfg, const mpm_material *mat, mpm_ad_ctx **out);
mpm_status mpm_ad_destroy(mpm_ad_ctx *ctx);

/* One forward step: state_out = step(state_in), logE: n floats.  state_in and
 * state_out must not overlap.  Device-detected errors (a particle outside
 * (x - origin)/dx in [1/4, n - 1/4) on some axis, a non-finite result) set the
 * context's status word, read by mpm_ad_sync; such a particle adds nothing to
 * the grid.  A pool overflow sets it too (MPM_E_CAPACITY). */
mpm_status mpm_ad_forward(mpm_ad_ctx *ctx, int64_t n, int64_t stride, const float *state_in, const float *logE,
                          float *state_out, double dt, void *stream);

/* Reverse mode of the same step: given dL/d state_out (cot_out, 27 planes), writes
 * dL/d state_in into cot_in (27 planes) and adds this step's dL/dlogE to
 * logE_cot (n floats, accumulated so that a rollout sums over its steps).  The
 * step's grid is recomputed from state_in.  cot_in must not overlap cot_out or
 * state_in. */
mpm_status mpm_ad_backward(mpm_ad_ctx *ctx, int64_t n, int64_t stride, const float *state_in, const float *logE,
                           const float *cot_out, float *cot_in, float *logE_cot, double dt, void *stream);

/* Wait for `stream`, then return (and clear) the status word: NONFINITE before
 * DOMAIN before CAPACITY. */
mpm_status mpm_ad_sync(mpm_ad_ctx *ctx, void *stream);

#ifdef __cplusplus
}
#endif
#endif
