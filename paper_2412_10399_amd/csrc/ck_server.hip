// Job server (declared in include/ckmpm.h): many independent simulation jobs on
// one GPU with continuous batching.  The server owns one device arena, carved
// first-fit into the contexts and particle buffers of resident jobs, and a set of
// non-blocking streams; every resident job advances a fixed number of steps per
// launch on its stream, and all launches after a job's first replay one HIP graph
// captured from that job's step sequence.  In grouped mode a round runs every phase
// of every active job as shared launches; the round's launch sequence is captured in
// a HIP graph and replayed while the set of jobs and their step counts stay the
// same, and captured again when they change.  Nothing here allocates device memory
// after mpm_server_create, and no call synchronises the whole device.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "ck_ctx.hpp"

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over one device allocation; free ranges are coalesced.
class Arena {
public:
    bool init(size_t bytes) {
        size_ = round_up(bytes);
        if (hipMalloc(&base_, size_) != hipSuccess) {
            base_ = nullptr;
            return false;
        }
        free_[0] = size_;
        return true;
    }
    void release() {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
        free_.clear();
        used_.clear();
    }
    void *alloc(size_t bytes) {
        bytes = round_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rem = it->second - bytes;
            free_.erase(it);
            if (rem) free_[off + bytes] = rem;
            used_[off] = bytes;
            return base_ + off;
        }
        return nullptr;
    }
    void free(void *p) {
        if (!p) return;
        const size_t off = static_cast<size_t>(static_cast<char *>(p) - base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t start = off, len = u->second;
        used_.erase(u);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }
    size_t size() const { return size_; }
    static void *alloc_cb(void *self, size_t bytes) { return static_cast<Arena *>(self)->alloc(bytes); }
    static void free_cb(void *self, void *p) { static_cast<Arena *>(self)->free(p); }

private:
    char *base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    std::map<size_t, size_t> used_;
};

__global__ void k_iota(uint32_t *ids, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        ids[i] = (uint32_t)i;
}

struct Job {
    int64_t id = 0;
    mpm_job_desc desc{};
    std::vector<mpm_material> mats;
    mpm_job_info info{};
    mpm_ctx *ctx = nullptr;
    mpm_particles parts{};
    std::vector<void *> bufs;           // arena buffers of the particle state
    int slot = -1;                      // resident slot: events and pinned status word
    int stream = 0;
    int lane = 0;                       // grouped mode: size-class lane
    bool in_flight = false;
    int chunk = 0;                      // steps of the launch in flight
    int ev_cur = 0;                     // event the launch in flight records
    hipGraphExec_t graph = nullptr;
    hipEvent_t ready = nullptr;         // recorded on the submitter's stream: the input is complete
    ~Job() {
        if (ready) (void)hipEventDestroy(ready);
    }
};

struct Slot {
    hipEvent_t ev[2] = {nullptr, nullptr};   // end of the previous / current launch
    bool used = false;
};

// Grouped mode: the jobs of one size class share one launch per phase (their lane's
// round), and the lanes run on their own streams, each round as soon as that lane's
// previous one has finished, so a large job's step does not wait for the small jobs'
// launches, nor small jobs for the large one.
struct Lane {
    ck::JobStep *table_host = nullptr;         // pinned, max_jobs x steps_per_launch entries
    ck::JobStep *table_dev = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};    // start and end of the round in flight
    bool in_flight = false;
    std::vector<std::pair<int64_t, int>> round;   // (job, steps) of the round in flight
    hipGraphExec_t graph = nullptr;               // the last round's captured launch sequence
    std::vector<int64_t> sig;                     // what it was captured for (see poll_grouped)
    hipStream_t stream = nullptr;
};

// Lane of a job of n particles: classes eight-fold apart in particle count from 2^10 up,
// the last lane taking every larger job.
int lane_of(int64_t n, int lanes) {
    int lg = 0;
    while (lg < 62 && (int64_t(1) << (lg + 1)) <= n) ++lg;
    const int c = (lg - 10) / 3;
    return c < 0 ? 0 : (c >= lanes ? lanes - 1 : c);
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct mpm_server {
    mpm_server_config cfg{};
    int device = 0;
    // grouped mode: one launch per phase for all active jobs of a size-class lane
    bool grouped = false;
    std::vector<Lane> lanes;
    int64_t graph_captures = 0, graph_replays = 0;
    Arena arena;
    std::vector<hipStream_t> streams;
    hipStream_t init_stream = nullptr;
    std::vector<Slot> slots;
    unsigned int *status_host = nullptr;   // pinned, one word per slot
    std::map<int64_t, std::unique_ptr<Job>> jobs;
    std::deque<int64_t> pending;
    int64_t next_id = 0;
    int resident = 0;
    int active = 0;
    int next_stream = 0;
    std::vector<double> step_lat;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
};

namespace {

void free_particles(mpm_server *srv, Job &j) {
    for (void *p : j.bufs) srv->arena.free(p);
    j.bufs.clear();
}

void evict(mpm_server *srv, Job &j) {
    if (j.graph) (void)hipGraphExecDestroy(j.graph);
    j.graph = nullptr;
    if (j.ctx) ck::ctx_destroy(j.ctx, false);
    j.ctx = nullptr;
    free_particles(srv, j);
    if (j.slot >= 0) srv->slots[j.slot].used = false;
    j.slot = -1;
    srv->resident -= 1;
}

void fail(mpm_server *srv, Job &j, mpm_status st) {
    j.info.state = MPM_JOB_FAILED;
    j.info.status = st;
    j.info.t_done = seconds_since(srv->t0);
    j.in_flight = false;
    srv->active -= 1;
}

// Carves the job's context and particle buffers from the arena and enqueues the copy
// of its initial state.  Returns false (and takes nothing) when the arena cannot
// hold it right now.
bool admit(mpm_server *srv, Job &j) {
    int slot = -1;
    for (int i = 0; i < (int)srv->slots.size(); ++i)
        if (!srv->slots[i].used) {
            slot = i;
            break;
        }
    if (slot < 0) return false;
    const int64_t n = j.desc.n;
    const size_t state_bytes = (size_t)MPM_STATE_PLANES * 4 * (size_t)n;
    const bool with_mat = j.desc.mat != nullptr;
    auto take = [&](size_t bytes) -> void * {
        void *p = srv->arena.alloc(bytes + kAlign);
        if (p) j.bufs.push_back(p);
        return p;
    };
    float *st0 = static_cast<float *>(take(state_bytes));
    float *st1 = static_cast<float *>(take(state_bytes));
    uint32_t *id0 = static_cast<uint32_t *>(take(4 * (size_t)n));
    uint32_t *id1 = static_cast<uint32_t *>(take(4 * (size_t)n));
    uint8_t *m0 = static_cast<uint8_t *>(take((size_t)n));
    uint8_t *m1 = static_cast<uint8_t *>(take((size_t)n));
    if (!st0 || !st1 || !id0 || !id1 || !m0 || !m1) {
        free_particles(srv, j);
        return false;
    }
    ck::Allocator a{Arena::alloc_cb, Arena::free_cb, &srv->arena};
    mpm_ctx *ctx = nullptr;
    const mpm_status cs = ck::ctx_create(&j.desc.cfg, j.mats.data(), j.desc.n_mat, &a, srv->init_stream, false, &ctx);
    if (cs == MPM_E_OOM) {
        free_particles(srv, j);
        return false;
    }
    srv->resident += 1;
    srv->active += 1;
    j.slot = slot;
    srv->slots[slot].used = true;
    j.info.state = MPM_JOB_ACTIVE;
    j.info.t_admit = seconds_since(srv->t0);
    if (cs != MPM_OK) {
        fail(srv, j, cs);
        return true;
    }
    j.ctx = ctx;
    // grouped: the job's lane runs its rounds on stream `lane`, after this copy-in
    if (srv->grouped) j.lane = lane_of(n, (int)srv->lanes.size());
    j.stream = srv->grouped ? j.lane : srv->next_stream;
    if (!srv->grouped) srv->next_stream = (srv->next_stream + 1) % (int)srv->streams.size();
    hipStream_t s = srv->streams[j.stream];
    j.parts = mpm_particles{};
    j.parts.n = n;
    j.parts.stride = n;
    j.parts.state[0] = st0;
    j.parts.state[1] = st1;
    j.parts.id[0] = id0;
    j.parts.id[1] = id1;
    j.parts.mat[0] = with_mat ? m0 : nullptr;
    j.parts.mat[1] = with_mat ? m1 : nullptr;
    j.parts.current = 0;
    // the copy-in waits for the work the submitter queued before submitting
    bool ok = !j.ready || hipStreamWaitEvent(s, j.ready, 0) == hipSuccess;
    ok = ok && hipMemcpyAsync(st0, j.desc.state, state_bytes, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (with_mat) ok = ok && hipMemcpyAsync(m0, j.desc.mat, (size_t)n, hipMemcpyDeviceToDevice, s) == hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_iota, dim3(blocks), dim3(256), 0, s, id0, (long long)n);
    ok = ok && hipGetLastError() == hipSuccess;
    // launch timing starts at the end of the copy-in
    ok = ok && hipEventRecord(srv->slots[slot].ev[0], s) == hipSuccess;
    j.ev_cur = 1;
    if (!ok) fail(srv, j, MPM_E_HIP);
    return true;
}

mpm_status launch(mpm_server *srv, Job &j) {
    const int spl = srv->cfg.steps_per_launch;
    const int remaining = j.desc.nsteps - j.info.steps_done;
    const int chunk = std::min(spl, remaining);
    hipStream_t s = srv->streams[j.stream];
    mpm_status st = MPM_OK;
    if (chunk == spl && j.info.steps_done > 0) {
        if (!j.graph) {
            // steady state: keys, stamps and stress come from the previous G2P, and an
            // even number of steps returns the ping-pong buffers to where they are
            hipGraph_t g = nullptr;
            if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) return MPM_E_HIP;
            st = mpm_step(j.ctx, &j.parts, j.desc.dt, chunk, s);
            const hipError_t ce = hipStreamEndCapture(s, &g);
            if (st != MPM_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (ce != hipSuccess) return MPM_E_HIP;
            const hipError_t ie = hipGraphInstantiate(&j.graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) {
                j.graph = nullptr;
                return MPM_E_HIP;
            }
        }
        if (hipGraphLaunch(j.graph, s) != hipSuccess) return MPM_E_HIP;
    } else if (chunk > 0) {
        st = mpm_step(j.ctx, &j.parts, j.desc.dt, chunk, s);
        if (st != MPM_OK) return st;
    }
    if (hipMemcpyAsync(&srv->status_host[j.slot], ck::ctx_status_word(j.ctx), sizeof(unsigned int),
                       hipMemcpyDeviceToHost, s) != hipSuccess)
        return MPM_E_HIP;
    if (hipEventRecord(srv->slots[j.slot].ev[j.ev_cur], s) != hipSuccess) return MPM_E_HIP;
    j.chunk = chunk;
    j.in_flight = true;
    return MPM_OK;
}

// Grouped mode: retire the rounds in flight, admit, then run the next round of every
// idle lane (steps_per_launch steps of each of its active jobs, fewer for jobs that
// need fewer).
void retire_round(mpm_server *srv, Lane &ln, hipError_t q) {
    ln.in_flight = false;
    float ms = 0.0f;
    const bool timed = q == hipSuccess && hipEventElapsedTime(&ms, ln.gev[0], ln.gev[1]) == hipSuccess;
    int longest = 1;
    for (const auto &js : ln.round) longest = std::max(longest, js.second);
    for (const auto &js : ln.round) {
        Job &j = *srv->jobs[js.first];
        j.in_flight = false;
        if (q != hipSuccess) {
            fail(srv, j, MPM_E_HIP);
            continue;
        }
        if (timed)
            for (int k = 0; k < js.second; ++k) srv->step_lat.push_back(ms * 1e-3 / longest);
        j.info.steps_done += js.second;
        const unsigned int bits = srv->status_host[j.slot];
        if (bits != 0) {
            fail(srv, j, ck::status_from_bits(bits));
        } else if (j.info.steps_done >= j.desc.nsteps) {
            j.info.state = MPM_JOB_DONE;
            j.info.status = MPM_OK;
            j.info.t_done = seconds_since(srv->t0);
            srv->active -= 1;
        }
    }
    ln.round.clear();
}

// Builds and enqueues lane ln's next round over `run` (its idle active jobs, largest
// first).  The round's launches depend only on which job takes which table entry and
// whether that entry is the job's first step; the table's contents are uploaded by the
// graph's own copy from pinned memory on every replay, so the captured graph is
// replayed while that signature holds.
void start_round(mpm_server *srv, Lane &ln, std::vector<Job *> &run) {
    hipStream_t s = ln.stream;
    const int spl = srv->cfg.steps_per_launch;
    std::vector<int> steps(run.size()), count(spl, 0);
    size_t used = 0;
    bool ok = hipEventRecord(ln.gev[0], s) == hipSuccess;
    // step k of the round: entries of every job with more than k steps left
    for (int k = 0; k < spl && ok; ++k) {
        for (size_t r = 0; r < run.size(); ++r) {
            Job &j = *run[r];
            if (j.desc.nsteps - j.info.steps_done <= k) continue;
            const mpm_status st = ck::group_step(j.ctx, &j.parts, j.desc.dt, ln.table_host[used]);
            if (st != MPM_OK) {
                ok = false;
                break;
            }
            ++used;
            ++count[k];
            steps[r] += 1;
        }
    }
    std::vector<int64_t> sig;
    sig.reserve(used + (size_t)spl + 1);
    sig.push_back((int64_t)used);
    for (int k = 0; k < spl; ++k) sig.push_back(count[k]);
    {
        size_t e = 0;
        for (int k = 0; k < spl; ++k)
            for (size_t r = 0; r < run.size(); ++r) {
                Job &j = *run[r];
                if (j.desc.nsteps - j.info.steps_done <= k) continue;
                sig.push_back(j.id * 2 + ln.table_host[e].first);
                ++e;
            }
    }
    if (ok && (!ln.graph || sig != ln.sig)) {
        if (ln.graph) (void)hipGraphExecDestroy(ln.graph);
        ln.graph = nullptr;
        ln.sig.clear();
        hipGraph_t g = nullptr;
        ok = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) == hipSuccess;
        if (ok) {
            bool cap = hipMemcpyAsync(ln.table_dev, ln.table_host, used * sizeof(ck::JobStep), hipMemcpyHostToDevice,
                                      s) == hipSuccess;
            size_t off = 0;
            for (int k = 0; k < spl && cap; ++k) {
                if (count[k] == 0) break;
                ck::launch_step_multi(ln.table_dev + off, ln.table_host + off, count[k], s);
                off += (size_t)count[k];
            }
            cap = cap && hipGetLastError() == hipSuccess;
            for (size_t r = 0; r < run.size() && cap; ++r)
                cap = hipMemcpyAsync(&srv->status_host[run[r]->slot], ck::ctx_status_word(run[r]->ctx),
                                     sizeof(unsigned int), hipMemcpyDeviceToHost, s) == hipSuccess;
            const hipError_t ce = hipStreamEndCapture(s, &g);
            ok = cap && ce == hipSuccess && g && hipGraphInstantiate(&ln.graph, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
            if (!ok) ln.graph = nullptr;
        }
        if (ok) {
            ln.sig.swap(sig);
            srv->graph_captures += 1;
        }
    } else if (ok) {
        srv->graph_replays += 1;
    }
    ok = ok && hipGraphLaunch(ln.graph, s) == hipSuccess;
    ok = ok && hipEventRecord(ln.gev[1], s) == hipSuccess;
    if (!ok) {
        for (Job *j : run) fail(srv, *j, MPM_E_HIP);
        return;
    }
    for (size_t r = 0; r < run.size(); ++r) {
        run[r]->in_flight = true;
        ln.round.emplace_back(run[r]->id, steps[r]);
    }
    ln.in_flight = true;
}

mpm_status poll_grouped(mpm_server *srv, bool *progressed) {
    bool moved = false;
    for (Lane &ln : srv->lanes) {
        if (!ln.in_flight) continue;
        const hipError_t q = hipEventQuery(ln.gev[1]);
        if (q == hipErrorNotReady) continue;
        moved = true;
        retire_round(srv, ln, q);
    }
    while (!srv->pending.empty() && srv->resident < srv->cfg.max_jobs) {
        Job &j = *srv->jobs[srv->pending.front()];
        if (!admit(srv, j)) break;
        srv->pending.pop_front();
        moved = true;
    }
    // jobs with no steps to run finish at once; the others go to their lane's next round
    std::vector<std::vector<Job *>> run(srv->lanes.size());
    for (auto &kv : srv->jobs) {
        Job &j = *kv.second;
        if (j.info.state != MPM_JOB_ACTIVE || j.in_flight) continue;
        if (j.info.steps_done >= j.desc.nsteps) {
            j.info.state = MPM_JOB_DONE;
            j.info.status = MPM_OK;
            j.info.t_done = seconds_since(srv->t0);
            srv->active -= 1;
            moved = true;
            continue;
        }
        if (!srv->lanes[j.lane].in_flight) run[j.lane].push_back(&j);
    }
    for (size_t l = 0; l < srv->lanes.size(); ++l) {
        if (run[l].empty()) continue;
        // largest jobs first: each step's entries then fall into contiguous size classes
        std::stable_sort(run[l].begin(), run[l].end(), [](const Job *a, const Job *b) { return a->desc.n > b->desc.n; });
        start_round(srv, srv->lanes[l], run[l]);
        moved = true;
    }
    if (progressed) *progressed = moved;
    return MPM_OK;
}

mpm_status poll_once(mpm_server *srv, bool *progressed) {
    if (srv->grouped) return poll_grouped(srv, progressed);
    bool moved = false;
    // retire finished launches
    for (auto &kv : srv->jobs) {
        Job &j = *kv.second;
        if (j.info.state != MPM_JOB_ACTIVE || !j.in_flight) continue;
        Slot &sl = srv->slots[j.slot];
        const hipError_t q = hipEventQuery(sl.ev[j.ev_cur]);
        if (q == hipErrorNotReady) continue;
        moved = true;
        if (q != hipSuccess) {
            fail(srv, j, MPM_E_HIP);
            continue;
        }
        j.in_flight = false;
        float ms = 0.0f;
        if (j.chunk > 0 && hipEventElapsedTime(&ms, sl.ev[j.ev_cur ^ 1], sl.ev[j.ev_cur]) == hipSuccess)
            for (int k = 0; k < j.chunk; ++k) srv->step_lat.push_back(ms * 1e-3 / j.chunk);
        j.info.steps_done += j.chunk;
        j.ev_cur ^= 1;
        const unsigned int bits = srv->status_host[j.slot];
        if (bits != 0) {
            fail(srv, j, ck::status_from_bits(bits));
        } else if (j.info.steps_done >= j.desc.nsteps) {
            j.info.state = MPM_JOB_DONE;
            j.info.status = MPM_OK;
            j.info.t_done = seconds_since(srv->t0);
            srv->active -= 1;
        }
    }
    // admit waiting jobs in submission order
    while (!srv->pending.empty() && srv->resident < srv->cfg.max_jobs) {
        Job &j = *srv->jobs[srv->pending.front()];
        if (!admit(srv, j)) break;
        srv->pending.pop_front();
        moved = true;
    }
    // next launch of every resident job that is idle
    for (auto &kv : srv->jobs) {
        Job &j = *kv.second;
        if (j.info.state != MPM_JOB_ACTIVE || j.in_flight) continue;
        const mpm_status st = launch(srv, j);
        if (st != MPM_OK) fail(srv, j, st);
        moved = true;
    }
    if (progressed) *progressed = moved;
    return MPM_OK;
}

Job *find(mpm_server *srv, int64_t id) {
    auto it = srv->jobs.find(id);
    return it == srv->jobs.end() ? nullptr : it->second.get();
}

}  // namespace

extern "C" {

mpm_status mpm_server_create(const mpm_server_config *cfg, mpm_server **out) {
    if (!cfg || !out) return MPM_E_INVALID;
    *out = nullptr;
    if (cfg->memory_budget <= 0 || cfg->max_jobs < 1 || cfg->n_streams < 1 || cfg->n_streams > 64 ||
        cfg->steps_per_launch < 2 || (cfg->steps_per_launch & 1) || (cfg->flags & ~MPM_SERVER_GROUPED) != 0)
        return MPM_E_INVALID;
    mpm_server *srv = new (std::nothrow) mpm_server();
    if (!srv) return MPM_E_OOM;
    srv->cfg = *cfg;
    bool ok = hipGetDevice(&srv->device) == hipSuccess;
    if (ok && !srv->arena.init((size_t)cfg->memory_budget)) {
        delete srv;
        return MPM_E_OOM;
    }
    for (int i = 0; ok && i < cfg->n_streams; ++i) {
        hipStream_t s = nullptr;
        ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
        if (ok) srv->streams.push_back(s);
    }
    ok = ok && hipStreamCreateWithFlags(&srv->init_stream, hipStreamNonBlocking) == hipSuccess;
    srv->slots.resize((size_t)cfg->max_jobs);
    for (Slot &sl : srv->slots)
        for (int k = 0; ok && k < 2; ++k) ok = hipEventCreate(&sl.ev[k]) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&srv->status_host, sizeof(unsigned int) * (size_t)cfg->max_jobs,
                             hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        (void)mpm_server_destroy(srv);
        return MPM_E_HIP;
    }
    std::memset(srv->status_host, 0, sizeof(unsigned int) * (size_t)cfg->max_jobs);
    srv->grouped = (cfg->flags & MPM_SERVER_GROUPED) != 0;
    if (srv->grouped) {
        const size_t entries = (size_t)cfg->max_jobs * (size_t)cfg->steps_per_launch;
        srv->lanes.resize((size_t)std::min(cfg->n_streams, 4));
        for (size_t l = 0; ok && l < srv->lanes.size(); ++l) {
            Lane &ln = srv->lanes[l];
            ln.stream = srv->streams[l];
            ok = hipHostMalloc((void **)&ln.table_host, entries * sizeof(ck::JobStep), hipHostMallocDefault) == hipSuccess;
            ok = ok && hipMalloc((void **)&ln.table_dev, entries * sizeof(ck::JobStep)) == hipSuccess;
            for (int k = 0; ok && k < 2; ++k) ok = hipEventCreate(&ln.gev[k]) == hipSuccess;
        }
        if (!ok) {
            (void)mpm_server_destroy(srv);
            return MPM_E_HIP;
        }
    }
    *out = srv;
    return MPM_OK;
}

mpm_status mpm_server_destroy(mpm_server *srv) {
    if (!srv) return MPM_OK;
    for (hipStream_t s : srv->streams) (void)hipStreamSynchronize(s);
    if (srv->init_stream) (void)hipStreamSynchronize(srv->init_stream);
    for (auto &kv : srv->jobs) {
        Job &j = *kv.second;
        if (j.slot >= 0) evict(srv, j);
    }
    srv->jobs.clear();
    for (Slot &sl : srv->slots)
        for (hipEvent_t e : sl.ev)
            if (e) (void)hipEventDestroy(e);
    for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
    if (srv->init_stream) (void)hipStreamDestroy(srv->init_stream);
    if (srv->status_host) (void)hipHostFree(srv->status_host);
    for (Lane &ln : srv->lanes) {
        if (ln.table_host) (void)hipHostFree(ln.table_host);
        if (ln.table_dev) (void)hipFree(ln.table_dev);
        for (hipEvent_t e : ln.gev)
            if (e) (void)hipEventDestroy(e);
        if (ln.graph) (void)hipGraphExecDestroy(ln.graph);
    }
    srv->arena.release();
    delete srv;
    return MPM_OK;
}

mpm_status mpm_server_submit(mpm_server *srv, const mpm_job_desc *job, int64_t *job_id) {
    if (!srv || !job || !job->mats) return MPM_E_INVALID;
    if (job->n < 1 || job->nsteps < 0 || job->n > job->cfg.max_particles || !job->state) return MPM_E_INVALID;
    if (!(job->dt >= 0.0) || !(job->dt < 1e30)) return MPM_E_INVALID;
    if ((reinterpret_cast<uintptr_t>(job->state) & 3u) != 0) return MPM_E_INVALID;
    if (job->n_mat < 1 || job->n_mat > ck::kMaxMaterials) return MPM_E_INVALID;
    if (srv->grouped && (job->cfg.flags != 0 || job->cfg.transfer != MPM_TRANSFER_MLS)) return MPM_E_INVALID;
    const int64_t fp = mpm_footprint(&job->cfg, job->n);
    if (fp <= 0) return MPM_E_INVALID;
    if ((size_t)fp > srv->arena.size()) return MPM_E_CAPACITY;
    std::unique_ptr<Job> j(new (std::nothrow) Job());
    if (!j) return MPM_E_OOM;
    // order the admission's copy of state and mat after the submitter's work (the
    // server's streams do not synchronise with any other stream, the null stream
    // included)
    if (hipEventCreateWithFlags(&j->ready, hipEventDisableTiming) != hipSuccess) {
        j->ready = nullptr;
        return MPM_E_HIP;
    }
    if (hipEventRecord(j->ready, (hipStream_t)job->stream) != hipSuccess) return MPM_E_HIP;
    j->id = srv->next_id++;
    j->desc = *job;
    j->mats.assign(job->mats, job->mats + job->n_mat);
    j->desc.mats = nullptr;
    j->info.state = MPM_JOB_PENDING;
    j->info.n = job->n;
    j->info.footprint = fp;
    j->info.t_submit = seconds_since(srv->t0);
    j->info.status = MPM_OK;
    if (job_id) *job_id = j->id;
    srv->pending.push_back(j->id);
    srv->jobs[j->id] = std::move(j);
    return MPM_OK;
}

mpm_status mpm_server_poll(mpm_server *srv, int32_t *n_pending, int32_t *n_active, int32_t *n_done) {
    if (!srv) return MPM_E_INVALID;
    const mpm_status st = poll_once(srv, nullptr);
    if (n_pending) *n_pending = (int32_t)srv->pending.size();
    if (n_active) *n_active = srv->active;
    if (n_done) *n_done = (int32_t)srv->jobs.size() - (int32_t)srv->pending.size() - srv->active;
    return st;
}

mpm_status mpm_server_drain(mpm_server *srv) {
    if (!srv) return MPM_E_INVALID;
    while (!srv->pending.empty() || srv->active > 0) {
        bool moved = false;
        const mpm_status st = poll_once(srv, &moved);
        if (st != MPM_OK) return st;
        if (moved) continue;
        // nothing to do until a launch ends: block on the oldest one in flight
        if (srv->grouped)
            for (Lane &ln : srv->lanes)
                if (ln.in_flight) {
                    (void)hipEventSynchronize(ln.gev[1]);
                    break;
                }
        for (auto &kv : srv->jobs) {
            if (srv->grouped) break;
            Job &j = *kv.second;
            if (j.info.state == MPM_JOB_ACTIVE && j.in_flight) {
                (void)hipEventSynchronize(srv->slots[j.slot].ev[j.ev_cur]);
                break;
            }
        }
        if (srv->active == 0 && !srv->pending.empty()) {
            // the oldest pending job does not fit even with every finished job's
            // memory in use: it waits for releases that this call cannot make
            return MPM_E_CAPACITY;
        }
    }
    return MPM_OK;
}

mpm_status mpm_server_job_info(mpm_server *srv, int64_t job_id, mpm_job_info *info) {
    if (!srv || !info) return MPM_E_INVALID;
    Job *j = find(srv, job_id);
    if (!j) return MPM_E_INVALID;
    *info = j->info;
    return MPM_OK;
}

mpm_status mpm_server_job_read(mpm_server *srv, int64_t job_id, float *state, uint32_t *ids) {
    if (!srv) return MPM_E_INVALID;
    Job *j = find(srv, job_id);
    if (!j || (j->info.state != MPM_JOB_DONE && j->info.state != MPM_JOB_FAILED) || !j->ctx) return MPM_E_INVALID;
    hipStream_t s = srv->streams[j->stream];
    const int cur = j->parts.current;
    const size_t n = (size_t)j->desc.n;
    bool ok = true;
    if (state)
        ok = ok && hipMemcpyAsync(state, j->parts.state[cur], (size_t)MPM_STATE_PLANES * 4 * n, hipMemcpyDeviceToDevice,
                                  s) == hipSuccess;
    if (ids) ok = ok && hipMemcpyAsync(ids, j->parts.id[cur], 4 * n, hipMemcpyDeviceToDevice, s) == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    return ok ? MPM_OK : MPM_E_HIP;
}

mpm_status mpm_server_job_release(mpm_server *srv, int64_t job_id) {
    if (!srv) return MPM_E_INVALID;
    Job *j = find(srv, job_id);
    if (!j) return MPM_E_INVALID;
    if (j->info.state == MPM_JOB_PENDING) {
        srv->pending.erase(std::remove(srv->pending.begin(), srv->pending.end(), job_id), srv->pending.end());
    } else if (j->info.state == MPM_JOB_ACTIVE) {
        return MPM_E_INVALID;
    } else if (j->slot >= 0) {
        if (hipStreamSynchronize(srv->streams[j->stream]) != hipSuccess) return MPM_E_HIP;
        evict(srv, *j);
    }
    srv->jobs.erase(job_id);
    return MPM_OK;
}

mpm_status mpm_server_step_latencies(mpm_server *srv, double *out, int64_t cap, int64_t *count) {
    if (!srv || cap < 0 || (cap > 0 && !out)) return MPM_E_INVALID;
    const int64_t n = (int64_t)srv->step_lat.size();
    for (int64_t i = 0; i < std::min(n, cap); ++i) out[i] = srv->step_lat[(size_t)i];
    if (count) *count = n;
    return MPM_OK;
}

}  // extern "C"
