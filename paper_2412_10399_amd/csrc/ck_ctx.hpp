// Library-internal access to contexts for other parts of the library (the job
// server): creation on a given allocator and stream, destruction, status word.
#pragma once

#include "../../include/ckmpm.h"
#include "ck_common.hpp"

namespace ck {

// Creates a context whose device buffers come from `alloc`; the initial clears run
// on `init_stream`, which is then synchronised (the whole device when device_sync).
mpm_status ctx_create(const mpm_config *cfg, const mpm_material *mats, int32_t n_mat, const Allocator *alloc,
                      hipStream_t init_stream, bool device_sync, mpm_ctx **out);
// Returns every buffer to the context's allocator (after a device-wide
// synchronisation when device_sync; otherwise the caller guarantees that no work
// on the context is pending).
void ctx_destroy(mpm_ctx *ctx, bool device_sync);
// Device address of the context's status word (sticky error bits of the steps).
unsigned int *ctx_status_word(mpm_ctx *ctx);
mpm_status status_from_bits(unsigned int bits);
// Device bytes of every buffer a context with this configuration allocates.
int64_t ctx_device_bytes(const mpm_config &c);
// Host-side validation of a configuration and its materials, the device geometry
// (origin, cell size, wall bounds) and the device form of a material.
mpm_status check_config(const mpm_config *c, const mpm_material *m, int32_t n_mat);
void geometry_of(const mpm_config &c, Geometry &g);
DevMaterial device_material(const mpm_material &m);
// Steps of many jobs in shared launches: whether a context can take part (compact
// kernel, MLS transfer, no flags), and the table entry of its next step — the host
// bookkeeping of one unfused step (page table, buffers, key readiness) is done here,
// the launch itself by launch_step_multi.
bool group_capable(const mpm_ctx *ctx);
mpm_status group_step(mpm_ctx *ctx, mpm_particles *p, double dt, JobStep &out);

}  // namespace ck
