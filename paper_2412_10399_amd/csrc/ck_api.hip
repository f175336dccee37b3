// C ABI of the compact-kernel MPM library (declared in include/ckmpm.h): context
// creation and validation, launch sequencing of the step's kernels, status
// reporting and per-phase event timing.  No allocation happens after mpm_create.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ck_ctx.hpp"

using namespace ck;

namespace {

constexpr int kPhases = 5;          // sort+activate, p2g, grid update, g2p, fused g2p+p2g
constexpr int kSlotEvents = 5;      // boundaries of one step: sort | p2g | update | g2p |
constexpr int kEventRing = 512;     // steps recorded before the ring is folded into the totals

}  // namespace

// Device memory of mpm_step_noalloc: every buffer of its work (sort scratch, page
// tables, grid pools, stress, status word) is carved from this array.  Each GPU the
// library runs on holds its own copy until the process ends.  In host code the
// array's name is no device address: the address comes from hipGetSymbolAddress
// with the device current (noalloc_scratch below).
static_assert(MPM_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) unsigned char scratch[MPM_NOALLOC_SCRATCH_BYTES];

struct mpm_ctx {
    mpm_config cfg;
    std::vector<mpm_material> mats;
    DevCtx d;
    int device = 0;
    const float *next_ready = nullptr;   // buffer whose keys and next-epoch stamps are in place
    long long next_n = -1;
    const float *p2g_done = nullptr;     // buffer the last p2g ran on
    const float *carried = nullptr;      // buffer holding the carried state (an mpm_step G2P with carry wrote it)
    bool g2p_carried = false;            // the state the last P2G read (the next G2P's input) was carried
    int grid_pool = 0, grid_table = 0;   // the grid the last p2g (or fused step) wrote: pool and page table
    int next_table = 0;                  // page table the next sort builds
    int written = -1;                    // buffer the last g2p wrote (mpm_current_buffer)
    unsigned int *host_counters = nullptr;
    // profiling
    bool prof = false;
    std::vector<hipEvent_t> ev;          // kEventRing x kSlotEvents
    std::vector<char> ev_fused;          // per slot: its p2g interval is the fused kernel, no g2p
    int ev_used = 0;
    hipStream_t ev_stream = nullptr;
    double totals[kPhases] = {0, 0, 0, 0, 0};
    long long counts[kPhases] = {0, 0, 0, 0, 0};
    std::vector<void *> allocs;
    ck::Allocator alloc;                 // where the device buffers came from
    bool host_counters_pinned = false;
};

namespace {

bool is_pow2(double v) {
    if (!(v > 0.0) || !std::isfinite(v)) return false;
    int e;
    return std::frexp(v, &e) == 0.5;
}

mpm_status hip_ok(hipError_t e) { return e == hipSuccess ? MPM_OK : MPM_E_HIP; }

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

mpm_status validate_config(const mpm_config *c, const mpm_material *m, int32_t n_mat) {
    if (!c || !m) return MPM_E_INVALID;
    if (n_mat < 1 || n_mat > kMaxMaterials) return MPM_E_INVALID;
    long long nbv = 1;
    for (int a = 0; a < 3; ++a) {
        if (c->n_cells[a] < 4 || c->n_cells[a] > (1 << 16)) return MPM_E_INVALID;
        nbv *= (c->n_cells[a] / 4 + 1);
        if (!std::isfinite(c->origin[a]) || !std::isfinite(c->gravity[a])) return MPM_E_INVALID;
    }
    if (nbv >= (1ll << 26)) return MPM_E_INVALID;               // key = block * 64 + cell fits in 32 bits
    if (!is_pow2(c->dx)) return MPM_E_INVALID;
    if (c->max_particles < 1 || c->max_particles >= (1ll << kIndexBits)) return MPM_E_INVALID;
    if (c->max_blocks < 1 || c->max_blocks >= (1ll << 26)) return MPM_E_INVALID;
    if (c->bc != MPM_BC_NONE && c->bc != MPM_BC_STICKY) return MPM_E_INVALID;
    if (c->bc_band < 0) return MPM_E_INVALID;
    if (c->transfer != MPM_TRANSFER_MLS && c->transfer != MPM_TRANSFER_APIC && c->transfer != MPM_TRANSFER_PIC)
        return MPM_E_INVALID;
    if ((c->flags & ~(MPM_FLAG_FUSED_G2P2G | MPM_FLAG_QUADRATIC)) != 0) return MPM_E_INVALID;
    if ((c->flags & MPM_FLAG_FUSED_G2P2G) && (c->flags & MPM_FLAG_QUADRATIC)) return MPM_E_INVALID;
    if (c->flags != 0 && c->transfer != MPM_TRANSFER_MLS) return MPM_E_INVALID;
    if (c->deterministic != 0 && c->deterministic != 1) return MPM_E_INVALID;
    if (c->deterministic && (c->flags != 0 || c->transfer != MPM_TRANSFER_MLS)) return MPM_E_INVALID;
    for (int i = 0; i < n_mat; ++i) {
        const mpm_material &q = m[i];
        if (q.model != MPM_FIXED_COROTATED && q.model != MPM_DRUCKER_PRAGER) return MPM_E_INVALID;
        if (!(q.E > 0) || !(q.nu >= 0 && q.nu < 0.5f) || !(q.rho > 0) || !(q.vol0 > 0)) return MPM_E_INVALID;
        if (!std::isfinite(q.E) || !std::isfinite(q.rho) || !std::isfinite(q.vol0)) return MPM_E_INVALID;
        if (q.model == MPM_DRUCKER_PRAGER && !(q.friction_deg >= 0 && q.friction_deg < 90)) return MPM_E_INVALID;
    }
    return MPM_OK;
}

mpm_status validate_particles(const mpm_ctx *ctx, const mpm_particles *p) {
    if (!ctx || !p) return MPM_E_INVALID;
    if (p->n < 0 || p->n > ctx->cfg.max_particles || p->n > p->stride) return MPM_E_INVALID;
    if (p->current != 0 && p->current != 1) return MPM_E_INVALID;
    if (p->n > 0 && !p->state[p->current]) return MPM_E_INVALID;
    if ((reinterpret_cast<uintptr_t>(p->state[p->current]) & 3u) != 0) return MPM_E_INVALID;
    return MPM_OK;
}

void fill_geometry(const mpm_config &c, Geometry &g) {
    for (int a = 0; a < 3; ++a) {
        g.origin[a] = c.origin[a];
        g.n[a] = c.n_cells[a];
        g.NB[a] = c.n_cells[a] / 4 + 1;
    }
    g.inv_dx = 1.0 / c.dx;
    g.dx = (float)c.dx;
    g.inv_dx_f = (float)(1.0 / c.dx);
    // packed remainder unit: 2^-9 of the FP32 ulp of the axis's largest coordinate
    for (int a = 0; a < 3; ++a) {
        const double m = std::max(std::fabs(c.origin[a]), std::fabs(c.origin[a] + c.n_cells[a] * c.dx));
        const int e = m > 0.0 ? std::max(std::ilogb((float)m), -90) : -90;
        g.r_unit[a] = std::ldexp(1.0f, e - 23 - 9);
        g.inv_r_unit[a] = std::ldexp(1.0f, 23 + 9 - e);
    }
    // a node i of grid G_k (k = -1, +1) sits at (i + k/4) cells (the quadratic
    // comparison kernel's single grid, stored as G-, at i cells); it is inside the
    // sticky walls when band <= its position <= n - band on every axis
    const bool quad = (c.flags & MPM_FLAG_QUADRATIC) != 0;
    for (int gi = 0; gi < 2; ++gi) {
        const double k = quad ? 0.0 : (gi == 0 ? -0.25 : 0.25);
        if (c.bc == MPM_BC_STICKY && c.bc_band > 0) {
            g.stick_lo[gi] = (int)std::ceil(c.bc_band - k);
            for (int a = 0; a < 3; ++a) g.stick_hi[gi][a] = (int)std::floor(c.n_cells[a] - c.bc_band - k);
        } else {
            g.stick_lo[gi] = -(1 << 30);
            for (int a = 0; a < 3; ++a) g.stick_hi[gi][a] = 1 << 30;
        }
    }
}

DevMaterial dev_material(const mpm_material &m) {
    DevMaterial r;
    r.model = m.model;
    r.mass = m.rho * m.vol0;
    r.vol0 = m.vol0;
    const double E = m.E, nu = m.nu;
    const double mu = E / (2.0 * (1.0 + nu)), lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    r.mu = (float)mu;
    r.lambda = (float)lam;
    const double sphi = std::sin(m.friction_deg * 3.14159265358979323846 / 180.0);
    const double alpha = std::sqrt(2.0 / 3.0) * 2.0 * sphi / (3.0 - sphi);
    r.dp_coef = (float)((3.0 * lam + 2.0 * mu) / (2.0 * mu) * alpha);
    return r;
}

void *hip_alloc(void *, size_t bytes) {
    void *p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}
void hip_free(void *, void *p) { (void)hipFree(p); }

// Bytes of every device buffer a context allocates: carve_buffers asks for 256 bytes
// of slack per buffer, and allocators hand out multiples of 256 bytes.
int64_t device_bytes_of(const mpm_config &c) {
    long long nbv = 1;
    for (int a = 0; a < 3; ++a) nbv *= (c.n_cells[a] / 4 + 1);
    const long long np = c.max_particles, nb = c.max_blocks;
    const long long nchunks = (nbv + kCompactChunk - 1) / kCompactChunk;
    auto r = [](long long bytes) { return (bytes + 256 + 255) / 256 * 256; };
    // the buffers of ctx_create, in its order
    return r(4 * np) + r(2 * np) + r(4 * np) + r(4 * nb * (long long)kMaxBlockParticles) +
           r(2 * nb * (long long)kMaxBlockParticles) + 2 * r(8 * stamp_stride(nbv)) + 2 * r(4 * nbv) + 2 * r(4 * nbv) +
           3 * r(4 * nb) + r(4 * (nb + 1)) + r(4 * nb) + 2 * r(4 * nb) + r(4 * nchunks) + r(4 * nchunks) +
           2 * r(4 * nb * (long long)kBlockFloats) + r(24 * np) + r(4 * (long long)C_COUNT) + r(4 * (long long)kBoundWords) +
           r(4 * 27 * nb) + (c.deterministic ? r(4 * nb * (long long)kStageFloats) : 0);
}

PartArgs part_args(const mpm_particles *p, bool with_out) {
    PartArgs a;
    const int cur = p->current;
    a.in = p->state[cur];
    a.out = with_out ? p->state[cur ^ 1] : nullptr;
    a.stride = p->stride;
    a.n = (int)p->n;
    a.id_in = (p->id[0] && p->id[1]) ? p->id[cur] : nullptr;
    a.id_out = (with_out && p->id[0] && p->id[1]) ? p->id[cur ^ 1] : nullptr;
    a.mat_in = (p->mat[0] && p->mat[1]) ? p->mat[cur] : nullptr;
    a.mat_out = (with_out && p->mat[0] && p->mat[1]) ? p->mat[cur ^ 1] : nullptr;
    return a;
}

mpm_status last_error() { return hipGetLastError() == hipSuccess ? MPM_OK : MPM_E_HIP; }

void fold_events(mpm_ctx *ctx) {
    if (ctx->ev_used == 0) return;
    (void)hipStreamSynchronize(ctx->ev_stream);
    for (int s = 0; s < ctx->ev_used; ++s) {
        const bool fused = ctx->ev_fused[s] != 0;
        for (int ph = 0; ph < kSlotEvents - 1; ++ph) {
            if (ctx->ev_fused[s] == 1 && ph == 3) continue;
            const int to = (fused && ph == 1) ? 4 : ph;
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ctx->ev[s * kSlotEvents + ph], ctx->ev[s * kSlotEvents + ph + 1]) == hipSuccess) {
                ctx->totals[to] += ms;
                ctx->counts[to] += 1;
            }
        }
    }
    ctx->ev_used = 0;
}

hipEvent_t *event_slot(mpm_ctx *ctx, hipStream_t s) {
    if (!ctx->prof) return nullptr;
    if (ctx->ev_used == kEventRing || (ctx->ev_used > 0 && s != ctx->ev_stream)) fold_events(ctx);
    ctx->ev_stream = s;
    ctx->ev_fused[ctx->ev_used] = 0;
    return &ctx->ev[ctx->ev_used * kSlotEvents];
}

// sort + activation + P2G; ev (optional) receives phase boundaries 0, 1, 2
mpm_status enqueue_p2g(mpm_ctx *ctx, const mpm_particles *p, double dt, hipStream_t s, hipEvent_t *ev, bool physics) {
    const PartArgs pa = part_args(p, false);
    // keys, next-step block stamps and the stress of every particle are in place
    // when the previous mpm_g2p wrote this very buffer
    const bool ready = ctx->next_ready == pa.in && ctx->next_n == pa.n;
    const bool carried_in = ready && ctx->carried == pa.in;
    // the compact-kernel MLS G2P records the blocks it changes, so the next P2G may keep
    // the order of the others (the quadratic and exact-gradient kernels do not; the fused
    // step orders the first sort's blocks again from their buckets)
    const bool keep_orders = physics && ready && !ctx->d.quadratic && ctx->d.transfer == MPM_TRANSFER_MLS &&
                             !(ctx->cfg.flags & MPM_FLAG_FUSED_G2P2G);
    if (ev) (void)hipEventRecord(ev[0], s);
    if (!ready) launch_flag_keys(ctx->d, pa, 1, s);
    // deterministic mode recomputes the stress from F every step, so that a run
    // resumed from its particle state sees the same stress as the uninterrupted run;
    // the stress pass also adds the state's contribution bound, which the bucket scan
    // below hands to the P2G
    if (physics && (!ready || ctx->d.det)) launch_stress(ctx->d, pa, s);
    const int t = ctx->next_table;
    launch_compact(ctx->d, t, s);
    launch_bucket(ctx->d, pa.n, t, t, s, keep_orders);
    ctx->next_table = t ^ 1;
    if (ev) (void)hipEventRecord(ev[1], s);
    if (!physics) {
        launch_block_sort(ctx->d, s);
    } else {
        launch_p2g(ctx->d, pa, (float)dt, t, t, s, carried_in, keep_orders);
        if (ctx->d.det) launch_det_gather(ctx->d, t, t, s);
        ctx->grid_pool = t;
        ctx->grid_table = t;
    }
    if (ev) (void)hipEventRecord(ev[2], s);
    ctx->next_ready = nullptr;
    ctx->p2g_done = pa.in;
    ctx->g2p_carried = physics && carried_in;
    ctx->carried = nullptr;
    return last_error();
}

mpm_status enqueue_update(mpm_ctx *ctx, double dt, hipStream_t s) {
    float g[3] = {(float)ctx->cfg.gravity[0], (float)ctx->cfg.gravity[1], (float)ctx->cfg.gravity[2]};
    launch_grid_update(ctx->d, (float)dt, g, ctx->grid_pool, ctx->grid_table, s);
    return last_error();
}

// carry (inside mpm_step, for every step but the last): the new state's B planes take
// Q = (m B - dt V0 tau) D^-1 / dx for the next step's P2G, which then reads neither B nor
// the carried stress (24 B less written and read per particle); the plain compact-kernel
// MLS path only, and not in deterministic mode.
bool can_carry(const mpm_ctx *ctx) { return !ctx->d.det && !ctx->d.quadratic && ctx->d.transfer == MPM_TRANSFER_MLS; }

mpm_status enqueue_g2p(mpm_ctx *ctx, mpm_particles *p, double dt, hipStream_t s, bool carry = false) {
    if (ctx->p2g_done != p->state[p->current]) return MPM_E_INVALID;
    if (!p->state[p->current ^ 1]) return MPM_E_INVALID;
    if ((p->id[0] == nullptr) != (p->id[1] == nullptr)) return MPM_E_INVALID;
    if ((p->mat[0] == nullptr) != (p->mat[1] == nullptr)) return MPM_E_INVALID;
    const PartArgs pa = part_args(p, true);
    carry = carry && can_carry(ctx);
    launch_g2p(ctx->d, pa, (float)dt, ctx->grid_pool, ctx->grid_table, s, carry, ctx->g2p_carried);
    ctx->g2p_carried = false;
    ctx->carried = carry ? pa.out : nullptr;
    p->current ^= 1;
    ctx->written = p->current;
    ctx->next_ready = pa.out;
    ctx->next_n = pa.n;
    ctx->p2g_done = nullptr;
    return last_error();
}

// Device-context fields of a validated configuration (everything but the buffers).
void fill_devctx(DevCtx &d, const mpm_config &cfg, const mpm_material *mats, int32_t n_mat) {
    std::memset(&d, 0, sizeof d);
    fill_geometry(cfg, d.geo);
    d.quadratic = (cfg.flags & MPM_FLAG_QUADRATIC) ? 1 : 0;
    d.transfer = cfg.transfer;
    for (int i = 0; i < n_mat; ++i) d.mats[i] = dev_material(mats[i]);
    d.n_mat = n_mat;
    d.max_blocks = (int)cfg.max_blocks;
    d.nbv = (long long)d.geo.NB[0] * d.geo.NB[1] * d.geo.NB[2];
    d.tau_stride = (long long)cfg.max_particles;
    d.det = cfg.deterministic ? 1 : 0;
}

template <typename T, typename Take>
bool take_buffer(Take &take, T **ptr, size_t count) {
    // 256 bytes of slack per buffer, as device_bytes_of counts them
    *ptr = static_cast<T *>(take(count * sizeof(T) + 256));
    return *ptr != nullptr;
}

// Every device buffer of a context, in the order device_bytes_of counts them, from
// `take(bytes)` (nullptr when it cannot): MPM_E_OOM when one is refused.
template <typename Take>
mpm_status carve_buffers(DevCtx &d, const mpm_config &cfg, Take take) {
    const size_t np = (size_t)cfg.max_particles, nb = (size_t)cfg.max_blocks, nv = (size_t)d.nbv;
    const size_t nchunks = (nv + kCompactChunk - 1) / kCompactChunk;
    const bool ok = take_buffer(take, &d.key, np) && take_buffer(take, &d.sub, np) && take_buffer(take, &d.perm, np) &&
                    take_buffer(take, &d.bucket, nb * (size_t)kMaxBlockParticles) &&
                    take_buffer(take, &d.bsub, nb * (size_t)kMaxBlockParticles) &&
                    take_buffer(take, &d.pflag, 2 * (size_t)stamp_stride(d.nbv)) &&
                    take_buffer(take, &d.gflag, 2 * (size_t)stamp_stride(d.nbv)) &&
                    take_buffer(take, &d.page[0], nv) && take_buffer(take, &d.page[1], nv) &&
                    take_buffer(take, &d.prank, nv) && take_buffer(take, &d.bchg, nv) &&
                    take_buffer(take, &d.plist, nb) && take_buffer(take, &d.blo, nb) && take_buffer(take, &d.bhi, nb) &&
                    take_buffer(take, &d.pstart, nb + 1) && take_buffer(take, &d.bcount, nb) &&
                    take_buffer(take, &d.glist[0], nb) && take_buffer(take, &d.glist[1], nb) &&
                    take_buffer(take, &d.chunk_p, nchunks) && take_buffer(take, &d.chunk_g, nchunks) &&
                    take_buffer(take, &d.pool[0], nb * kBlockFloats) && take_buffer(take, &d.pool[1], nb * kBlockFloats) &&
                    take_buffer(take, &d.tau, 6 * np) && take_buffer(take, &d.counters, (size_t)C_COUNT) &&
                    take_buffer(take, &d.bslots, (size_t)kBoundWords) &&
                    take_buffer(take, &d.nbrs, 27 * nb) &&
                    (!d.det || take_buffer(take, &d.stage, nb * (size_t)kStageFloats));
    return ok ? MPM_OK : MPM_E_OOM;
}

}  // namespace

namespace ck {

mpm_status ctx_create(const mpm_config *cfg, const mpm_material *mats, int32_t n_mat, const Allocator *alloc,
                      hipStream_t init_stream, bool device_sync, mpm_ctx **out) {
    if (!out) return MPM_E_INVALID;
    *out = nullptr;
    const mpm_status v = validate_config(cfg, mats, n_mat);
    if (v != MPM_OK) return v;
    mpm_ctx *ctx = new (std::nothrow) mpm_ctx();
    if (!ctx) return MPM_E_OOM;
    ctx->cfg = *cfg;
    ctx->mats.assign(mats, mats + n_mat);
    ctx->alloc = *alloc;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return MPM_E_HIP;
    }
    DevCtx &d = ctx->d;
    fill_devctx(d, *cfg, mats, n_mat);
    mpm_status st = carve_buffers(d, *cfg, [ctx](size_t bytes) -> void * {
        void *p = ctx->alloc.alloc(ctx->alloc.self, bytes);
        if (p) ctx->allocs.push_back(p);
        return p;
    });
    const size_t nb = (size_t)cfg->max_blocks, nv = (size_t)d.nbv;
    if (st == MPM_OK) {
        if (hipHostMalloc((void **)&ctx->host_counters, C_COUNT * sizeof(unsigned int), hipHostMallocDefault) == hipSuccess)
            ctx->host_counters_pinned = true;
        else
            st = MPM_E_OOM;
    }
    if (st == MPM_OK) {
        bool ok = hipMemsetAsync(d.pflag, 0, 2 * stamp_stride(d.nbv) * sizeof(int), init_stream) == hipSuccess &&
                  hipMemsetAsync(d.gflag, 0, 2 * stamp_stride(d.nbv) * sizeof(int), init_stream) == hipSuccess &&
                  hipMemsetAsync(d.page[0], 0xff, nv * sizeof(int), init_stream) == hipSuccess &&
                  hipMemsetAsync(d.page[1], 0xff, nv * sizeof(int), init_stream) == hipSuccess &&
                  hipMemsetAsync(d.prank, 0xff, nv * sizeof(int), init_stream) == hipSuccess &&
                  hipMemsetAsync(d.bchg, 0xff, nv * sizeof(int), init_stream) == hipSuccess &&
                  hipMemsetAsync(d.pstart, 0, (nb + 1) * sizeof(int), init_stream) == hipSuccess &&
                  hipMemsetAsync(d.counters, 0, C_COUNT * sizeof(unsigned int), init_stream) == hipSuccess &&
                  hipMemsetAsync(d.bslots, 0, kBoundWords * sizeof(unsigned int), init_stream) == hipSuccess;
        ok = ok && (device_sync ? hipDeviceSynchronize() : hipStreamSynchronize(init_stream)) == hipSuccess;
        if (!ok) st = MPM_E_HIP;
    }
    if (st != MPM_OK) {
        ctx_destroy(ctx, device_sync);
        return st;
    }
    *out = ctx;
    return MPM_OK;
}

void ctx_destroy(mpm_ctx *ctx, bool device_sync) {
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    if (device_sync) (void)hipDeviceSynchronize();
    for (void *p : ctx->allocs) ctx->alloc.free(ctx->alloc.self, p);
    for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
    if (ctx->host_counters_pinned) (void)hipHostFree(ctx->host_counters);
    delete ctx;
}

unsigned int *ctx_status_word(mpm_ctx *ctx) { return ctx->d.counters + C_STATUS; }

int64_t ctx_device_bytes(const mpm_config &c) { return device_bytes_of(c); }

mpm_status status_from_bits(unsigned int bits) {
    if (bits & ST_NONFINITE) return MPM_E_NONFINITE;
    if (bits & ST_DOMAIN) return MPM_E_DOMAIN;
    if (bits & ST_CAPACITY) return MPM_E_CAPACITY;
    if (bits & ST_STALE) return MPM_E_STALE;
    if (bits & ST_CFL) return MPM_E_CFL;
    return MPM_OK;
}

bool group_capable(const mpm_ctx *ctx) { return ctx->cfg.flags == 0 && ctx->cfg.transfer == MPM_TRANSFER_MLS; }

mpm_status group_step(mpm_ctx *ctx, mpm_particles *p, double dt, JobStep &out) {
    const mpm_status v = validate_particles(ctx, p);
    if (v != MPM_OK) return v;
    if (!std::isfinite(dt) || dt < 0 || !p->state[p->current ^ 1]) return MPM_E_INVALID;
    if ((p->id[0] == nullptr) != (p->id[1] == nullptr)) return MPM_E_INVALID;
    if ((p->mat[0] == nullptr) != (p->mat[1] == nullptr)) return MPM_E_INVALID;
    // the bookkeeping of one unfused step of mpm_step: sort into the next page table,
    // P2G, update and G2P on it, G2P writing the other buffer and the next keys
    const PartArgs pa = part_args(p, true);
    const bool ready = ctx->next_ready == pa.in && ctx->next_n == pa.n;
    const int t = ctx->next_table;
    ctx->next_table = t ^ 1;
    ctx->grid_pool = t;
    ctx->grid_table = t;
    out.d = ctx->d;
    out.pa = pa;
    out.dt = (float)dt;
    for (int a = 0; a < 3; ++a) out.g[a] = (float)ctx->cfg.gravity[a];
    out.table = t;
    out.first = ready ? 0 : 1;
    p->current ^= 1;
    ctx->written = p->current;
    ctx->next_ready = pa.out;
    ctx->next_n = pa.n;
    ctx->p2g_done = nullptr;
    return MPM_OK;
}

mpm_status check_config(const mpm_config *c, const mpm_material *m, int32_t n_mat) {
    return validate_config(c, m, n_mat);
}
void geometry_of(const mpm_config &c, Geometry &g) { fill_geometry(c, g); }
DevMaterial device_material(const mpm_material &m) { return dev_material(m); }

}  // namespace ck

extern "C" {

int32_t mpm_abi_version(void) { return CKMPM_ABI_VERSION; }

const char *mpm_status_string(mpm_status s) {
    switch (s) {
        case MPM_OK: return "ok";
        case MPM_E_INVALID: return "invalid argument or configuration";
        case MPM_E_OOM: return "device allocation failed";
        case MPM_E_DOMAIN: return "particle outside the valid domain";
        case MPM_E_CAPACITY: return "grid block pool or per-block particle capacity exceeded";
        case MPM_E_NONFINITE: return "non-finite particle state";
        case MPM_E_HIP: return "HIP runtime error";
        case MPM_E_STALE: return "particle positions changed after their cell keys were computed";
        case MPM_E_CFL: return "a particle moved more than three cells in one fused step";
        case MPM_E_SCRATCH: return "buffers exceed the static scratch of mpm_step_noalloc";
    }
    return "unknown status";
}

mpm_status mpm_create(const mpm_config *cfg, const mpm_material *mats, int32_t n_mat, mpm_ctx **out) {
    ck::Allocator a{hip_alloc, hip_free, nullptr};
    return ck::ctx_create(cfg, mats, n_mat, &a, nullptr, true, out);
}

mpm_status mpm_destroy(mpm_ctx *ctx) {
    ck::ctx_destroy(ctx, true);
    return MPM_OK;
}

int64_t mpm_footprint(const mpm_config *cfg, int64_t n) {
    if (!cfg) return 0;
    auto r = [](long long bytes) { return (bytes + 256 + 255) / 256 * 256; };
    return device_bytes_of(*cfg) + 2 * (r((int64_t)MPM_STATE_PLANES * 4 * n) + r(4 * n) + r(n));
}

mpm_status mpm_p2g(mpm_ctx *ctx, const mpm_particles *p, double dt, void *stream) {
    const mpm_status v = validate_particles(ctx, p);
    if (v != MPM_OK) return v;
    if (!std::isfinite(dt) || dt < 0) return MPM_E_INVALID;
    DeviceGuard g(ctx->device);
    return enqueue_p2g(ctx, p, dt, (hipStream_t)stream, nullptr, true);
}

mpm_status mpm_grid_update(mpm_ctx *ctx, double dt, void *stream) {
    if (!ctx || !std::isfinite(dt) || dt < 0) return MPM_E_INVALID;
    DeviceGuard g(ctx->device);
    return enqueue_update(ctx, dt, (hipStream_t)stream);
}

mpm_status mpm_g2p(mpm_ctx *ctx, mpm_particles *p, double dt, void *stream) {
    const mpm_status v = validate_particles(ctx, p);
    if (v != MPM_OK) return v;
    if (!std::isfinite(dt) || dt < 0) return MPM_E_INVALID;
    DeviceGuard g(ctx->device);
    return enqueue_g2p(ctx, p, dt, (hipStream_t)stream);
}

}  // extern "C"

namespace {

// Host-side checks of mpm_step's arguments.
mpm_status validate_step(const mpm_ctx *ctx, const mpm_particles *p, double dt, int32_t nsteps) {
    const mpm_status v = validate_particles(ctx, p);
    if (v != MPM_OK) return v;
    if (!std::isfinite(dt) || dt < 0 || nsteps < 0) return MPM_E_INVALID;
    if (!p->state[p->current ^ 1]) return MPM_E_INVALID;
    if ((p->id[0] == nullptr) != (p->id[1] == nullptr)) return MPM_E_INVALID;
    if ((p->mat[0] == nullptr) != (p->mat[1] == nullptr)) return MPM_E_INVALID;
    return MPM_OK;
}

// The launch sequence of nsteps steps (mpm_step), on the context's buffers.
mpm_status step_sequence(mpm_ctx *ctx, mpm_particles *p, double dt, int32_t nsteps, hipStream_t s) {
    if (nsteps == 0) return MPM_OK;
    if (!(ctx->cfg.flags & MPM_FLAG_FUSED_G2P2G)) {
        for (int k = 0; k < nsteps; ++k) {
            hipEvent_t *ev = event_slot(ctx, s);
            mpm_status st = enqueue_p2g(ctx, p, dt, s, ev, true);
            if (st == MPM_OK) st = enqueue_update(ctx, dt, s);
            if (st == MPM_OK && ev) (void)hipEventRecord(ev[3], s);
            if (st == MPM_OK) st = enqueue_g2p(ctx, p, dt, s, k + 1 < nsteps);
            if (st == MPM_OK && ev) {
                (void)hipEventRecord(ev[4], s);
                ctx->ev_used += 1;
            }
            if (st != MPM_OK) return st;
        }
        return MPM_OK;
    }
    // first step: sort, P2G, grid update
    hipEvent_t *ev = event_slot(ctx, s);
    mpm_status st = enqueue_p2g(ctx, p, dt, s, ev, true);
    if (st == MPM_OK) st = enqueue_update(ctx, dt, s);
    if (st != MPM_OK) return st;
    if (ev) (void)hipEventRecord(ev[3], s);
    // steps 1 .. nsteps-1: G2P of the previous step fused with this step's P2G
    for (int k = 1; k < nsteps; ++k) {
        if (ev) {
            (void)hipEventRecord(ev[4], s);   // previous step: no separate G2P
            ctx->ev_used += 1;
            ev = event_slot(ctx, s);
            if (ev) {
                (void)hipEventRecord(ev[0], s);
                ctx->ev_fused[ctx->ev_used] = 1;
            }
        }
        const int gin = ctx->grid_pool, tin = ctx->grid_table;
        const int gout = gin ^ 1;
        int tout;
        if (k == 1) {
            // the first sort's block set (neighbourhood of the particle blocks) serves
            // the second grid as well
            tout = tin;
            launch_zero_pool(ctx->d, gout, tout, s);
        } else {
            tout = ctx->next_table;
            const PartArgs pa = part_args(p, false);
            launch_compact(ctx->d, tout, s);
            launch_bucket(ctx->d, pa.n, gout, tout, s);
            ctx->next_table = tout ^ 1;
        }
        if (ev) (void)hipEventRecord(ev[1], s);
        const PartArgs pa = part_args(p, true);
        launch_g2p2g(ctx->d, pa, (float)dt, gin, tin, gout, tout, s);
        p->current ^= 1;
        ctx->written = p->current;
        ctx->grid_pool = gout;
        ctx->grid_table = tout;
        if (ev) (void)hipEventRecord(ev[2], s);
        st = enqueue_update(ctx, dt, s);
        if (st != MPM_OK) return st;
        if (ev) (void)hipEventRecord(ev[3], s);
    }
    if (nsteps > 1) {
        // the last step's G2P needs the blocks of the state the fused kernel wrote
        const PartArgs pa = part_args(p, false);
        const int t = ctx->next_table;
        launch_compact(ctx->d, t, s);
        launch_bucket(ctx->d, pa.n, ctx->grid_pool ^ 1, t, s);
        ctx->next_table = t ^ 1;
        launch_block_order(ctx->d, s);
        ctx->p2g_done = pa.in;
    }
    st = enqueue_g2p(ctx, p, dt, s);
    if (st == MPM_OK && ev) {
        (void)hipEventRecord(ev[4], s);
        if (ctx->ev_fused[ctx->ev_used]) ctx->ev_fused[ctx->ev_used] = 2;   // keeps its g2p interval
        ctx->ev_used += 1;
    }
    return st;
}

}  // namespace

extern "C" {

mpm_status mpm_step(mpm_ctx *ctx, mpm_particles *p, double dt, int32_t nsteps, void *stream) {
    const mpm_status v = validate_step(ctx, p, dt, nsteps);
    if (v != MPM_OK) return v;
    DeviceGuard g(ctx->device);
    return step_sequence(ctx, p, dt, nsteps, (hipStream_t)stream);
}

mpm_status mpm_sync(mpm_ctx *ctx, void *stream) {
    if (!ctx) return MPM_E_INVALID;
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    if (hipStreamSynchronize(s) != hipSuccess) return MPM_E_HIP;
    unsigned int bits = 0;
    if (hipMemcpy(&bits, ctx->d.counters + C_STATUS, sizeof bits, hipMemcpyDeviceToHost) != hipSuccess) return MPM_E_HIP;
    const unsigned int zero = 0;
    if (hipMemcpy(ctx->d.counters + C_STATUS, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess) return MPM_E_HIP;
    return status_from_bits(bits);
}

mpm_status mpm_grid_read(mpm_ctx *ctx, int32_t grid, float *m, float *vec, void *stream) {
    if (!ctx || (grid != -1 && grid != 0 && grid != 1)) return MPM_E_INVALID;
    DeviceGuard g(ctx->device);
    const int g0 = grid == 1 ? 1 : 0, ng = grid == 0 ? 2 : 1;
    launch_grid_export(ctx->d, m, vec, ctx->grid_pool, ctx->grid_table, g0, ng, (hipStream_t)stream);
    return last_error();
}

int32_t mpm_current_buffer(const mpm_ctx *ctx) { return ctx ? ctx->written : -1; }

mpm_status mpm_sort_keys(mpm_ctx *ctx, const mpm_particles *p, uint32_t *keys, uint32_t *perm, void *stream) {
    const mpm_status v = validate_particles(ctx, p);
    if (v != MPM_OK) return v;
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    ctx->next_ready = nullptr;   // always recompute the keys from the positions
    mpm_status st = enqueue_p2g(ctx, p, 0.0, s, nullptr, false);
    if (st != MPM_OK) return st;
    launch_copy_keys(ctx->d, keys, perm, (int)p->n, s);
    ctx->p2g_done = nullptr;
    return last_error();
}

mpm_status mpm_invalidate(mpm_ctx *ctx) {
    if (!ctx) return MPM_E_INVALID;
    ctx->next_ready = nullptr;
    ctx->p2g_done = nullptr;
    return MPM_OK;
}

mpm_status mpm_get_stats(mpm_ctx *ctx, mpm_stats *out, void *stream) {
    if (!ctx || !out) return MPM_E_INVALID;
    DeviceGuard g(ctx->device);
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return MPM_E_HIP;
    if (hipMemcpy(ctx->host_counters, ctx->d.counters, C_COUNT * sizeof(unsigned int), hipMemcpyDeviceToHost) != hipSuccess)
        return MPM_E_HIP;
    out->n_particle_blocks = ctx->host_counters[C_NPB];
    out->n_grid_blocks = ctx->host_counters[ngb_slot(ctx->grid_table)];
    out->max_block_particles = ctx->host_counters[C_MAXPB];
    out->status_bits = ctx->host_counters[C_STATUS];
    out->reserved = 0;
    return MPM_OK;
}

mpm_status mpm_profile_enable(mpm_ctx *ctx, int32_t enable) {
    if (!ctx) return MPM_E_INVALID;
    DeviceGuard g(ctx->device);
    if (enable && ctx->ev.empty()) {
        ctx->ev.resize((size_t)kEventRing * kSlotEvents);
        ctx->ev_fused.assign(kEventRing, 0);
        for (auto &e : ctx->ev)
            if (hipEventCreate(&e) != hipSuccess) return MPM_E_HIP;
    }
    if (!enable) fold_events(ctx);
    ctx->prof = enable != 0;
    for (int i = 0; i < kPhases; ++i) {
        ctx->totals[i] = 0;
        ctx->counts[i] = 0;
    }
    ctx->ev_used = 0;
    return MPM_OK;
}

}  // extern "C"

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_addr[kMaxDevices];   // per device: the address of `scratch` there

// Address of the current device's scratch array, looked up once per device.
mpm_status noalloc_scratch(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kMaxDevices) return MPM_E_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MPM_E_HIP;
        g_scratch_addr[dev] = ptr;
    }
    *out = static_cast<unsigned char *>(g_scratch_addr[dev]);
    return MPM_OK;
}

__global__ void k_fill_words(uint32_t *p, uint32_t value, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = value;
}

void fill_words(void *p, uint32_t value, long long n, hipStream_t s) {
    const long long blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_words, dim3((unsigned)(blocks < 1024 ? (blocks > 0 ? blocks : 1) : 1024)), dim3(256), 0, s,
                       static_cast<uint32_t *>(p), value, n);
}

// mpm_status code of the status bits, in mpm_sync's order.
__global__ void k_status_code(const unsigned int *counters, int32_t *out) {
    const unsigned int b = counters[C_STATUS];
    *out = (b & ST_NONFINITE) ? MPM_E_NONFINITE
         : (b & ST_DOMAIN)    ? MPM_E_DOMAIN
         : (b & ST_CAPACITY)  ? MPM_E_CAPACITY
         : (b & ST_STALE)     ? MPM_E_STALE
         : (b & ST_CFL)       ? MPM_E_CFL
                              : MPM_OK;
}

}  // namespace

extern "C" {

mpm_status mpm_step_noalloc(const mpm_config *cfg, const mpm_material *mats, int32_t n_mat, mpm_particles *p,
                            double dt, int32_t nsteps, int32_t *status, void *stream) {
    const mpm_status vc = validate_config(cfg, mats, n_mat);
    if (vc != MPM_OK) return vc;
    if (device_bytes_of(*cfg) > (int64_t)MPM_NOALLOC_SCRATCH_BYTES) return MPM_E_SCRATCH;
    // a context on the stack: its buffers come from the scratch array; nothing in it
    // allocates (the vectors stay empty, profiling stays off)
    mpm_ctx ctx;
    ctx.cfg = *cfg;
    const mpm_status v = validate_step(&ctx, p, dt, nsteps);
    if (v != MPM_OK) return v;
    if (hipGetDevice(&ctx.device) != hipSuccess) return MPM_E_HIP;
    unsigned char *base = nullptr;
    const mpm_status sa = noalloc_scratch(ctx.device, &base);
    if (sa != MPM_OK) return sa;
    DevCtx &d = ctx.d;
    fill_devctx(d, *cfg, mats, n_mat);
    size_t used = 0;
    const mpm_status sc = carve_buffers(d, *cfg, [&](size_t bytes) -> void * {
        const size_t at = (used + 255) / 256 * 256;
        if (at + bytes > (size_t)MPM_NOALLOC_SCRATCH_BYTES) return nullptr;
        used = at + bytes;
        return base + at;
    });
    if (sc != MPM_OK) return MPM_E_SCRATCH;
    // the previous call's contents stay in the array: reset what a new context starts
    // from (epoch stamps, page tables, block ranks, block starts, counters), with fill
    // kernels on the caller's stream
    hipStream_t s = (hipStream_t)stream;
    const long long nv = d.nbv, nb = cfg->max_blocks;
    fill_words(d.pflag, 0u, 2 * stamp_stride(nv), s);
    fill_words(d.gflag, 0u, 2 * stamp_stride(nv), s);
    fill_words(d.page[0], 0xffffffffu, nv, s);
    fill_words(d.page[1], 0xffffffffu, nv, s);
    fill_words(d.prank, 0xffffffffu, nv, s);
    fill_words(d.bchg, 0xffffffffu, nv, s);
    fill_words(d.pstart, 0u, nb + 1, s);
    fill_words(d.counters, 0u, C_COUNT, s);
    fill_words(d.bslots, 0u, kBoundWords, s);
    mpm_status st = last_error();
    if (st == MPM_OK) st = step_sequence(&ctx, p, dt, nsteps, s);
    if (st == MPM_OK && status) {
        hipLaunchKernelGGL(k_status_code, dim3(1), dim3(1), 0, s, d.counters, status);
        st = last_error();
    }
    return st;
}

mpm_status mpm_profile_read(mpm_ctx *ctx, double *total_ms, int64_t *count, int32_t n_phases) {
    if (!ctx || n_phases < 0) return MPM_E_INVALID;
    DeviceGuard g(ctx->device);
    fold_events(ctx);
    for (int i = 0; i < n_phases && i < kPhases; ++i) {
        if (total_ms) total_ms[i] = ctx->totals[i];
        if (count) count[i] = ctx->counts[i];
    }
    return MPM_OK;
}

}  // extern "C"
