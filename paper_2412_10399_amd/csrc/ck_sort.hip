// Cell keys, grid-block activation and the bucketing half of the particle sort.
//
// The particles are sorted stably by key = (4^3-cell block) * 64 + (cell in block),
// the G- cell being floor((x - origin)/dx + 1/4) per axis.  A stable sort by key is
// the same as a sort by (key, index), which we build in two exact stages:
//   1. bucket by block: blocks holding particles are enumerated in increasing
//      virtual id (compaction of per-block epoch stamps), every particle takes a slot
//      in its block's fixed-size bucket with one wave-aggregated atomic, and a scan
//      of the bucket sizes gives each block its range of sorted positions;
//   2. inside each block (in the P2G workgroup, in LDS): order by (cell, index).
// Atomics only decide where a particle waits inside its bucket, never its final
// position, so the resulting permutation is deterministic and exact.
#include "ck_common.hpp"

#include <algorithm>

namespace ck {

namespace {

__device__ __forceinline__ int wave_lane() { return __lane_id(); }

// Stamp the virtual blocks a particle needs: its own block (it holds particles) and,
// as grid blocks, the 3 x 3 x 3 blocks around it.  That neighbourhood holds the
// particle's 16-node stencil, and also the stencil after a move of up to three
// cells, which lets one sort serve the grid that the next step's fused transfer
// writes.
__device__ __forceinline__ void stamp_blocks(const DevCtx &d, int bx, int by, int bz, int epoch) {
    const Geometry &g = d.geo;
    int *pf = stamps(d.pflag, d.nbv, epoch);
    int *gf = stamps(d.gflag, d.nbv, epoch);
    pf[vblock_id(g, bx, by, bz)] = epoch;
    for (int z = max(bz - 1, 0); z <= min(bz + 1, g.NB[2] - 1); ++z)
        for (int y = max(by - 1, 0); y <= min(by + 1, g.NB[1] - 1); ++y)
            for (int x = max(bx - 1, 0); x <= min(bx + 1, g.NB[0] - 1); ++x) gf[vblock_id(g, x, y, z)] = epoch;
}

__device__ __forceinline__ void b_flag_keys(const DevCtx &d, const PartArgs &pa, int epoch_offset) {
    const int i = blockIdx.x * kThreads + threadIdx.x;

    const int epoch = (int)d.counters[C_EPOCH] + epoch_offset;
    bool ok = i < pa.n;
    CellCoord cc;
    if (ok) {
        const float x[3] = {pa.in[i], pa.in[pa.stride + i], pa.in[2 * pa.stride + i]};
        const float xr[3] = {pa.in[kPlaneR * pa.stride + i], pa.in[(kPlaneR + 1) * pa.stride + i],
                             pa.in[(kPlaneR + 2) * pa.stride + i]};
        ok = cell_coord(d.geo, x, xr, cc);
        if (!ok) {
            d.key[i] = 0xffffffffu;
            set_status(d.counters, ST_DOMAIN);
        }
    }
    // every lane takes part in the neighbour comparison below
    const int vb = ok ? vblock_id(d.geo, cc.c[0] >> 2, cc.c[1] >> 2, cc.c[2] >> 2) : -1;
    const int prev = __shfl_up(vb, 1);
    if (!ok) return;
    d.key[i] = cell_key(d.geo, cc);
    d.sub[i] = (uint16_t)sub_code(cc);
    // one stamping lane per run of equal blocks (particles mostly arrive sorted)
    if ((threadIdx.x & 63) == 0 || prev != vb) stamp_blocks(d, cc.c[0] >> 2, cc.c[1] >> 2, cc.c[2] >> 2, epoch);
}

__global__ void __launch_bounds__(kThreads) k_flag_keys(DevCtx d, PartArgs pa, int epoch_offset) { b_flag_keys(d, pa, epoch_offset); }

// one launch for many jobs: workgroup row y runs job y
__global__ void __launch_bounds__(kThreads) k_flag_keys_multi(const JobStep *__restrict__ jobs) {
    const JobStep &J = jobs[blockIdx.y];
    if (!J.first) return;
    b_flag_keys(J.d, J.pa, 1);
}

__global__ void k_clear_flags(DevCtx d) {
    const long long nst = 2 * stamp_stride(d.nbv);
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < nst; v += (long long)gridDim.x * blockDim.x) {
        d.pflag[v] = 0;
        d.gflag[v] = 0;
    }
}

// Workgroup-wide sum of two counters (256 threads).
__device__ __forceinline__ void wg_sum2(int &a, int &b, int *sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off);
        b += __shfl_down(b, off);
    }
    const int w = threadIdx.x >> 6;
    if (wave_lane() == 0) {
        sh[2 * w] = a;
        sh[2 * w + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int sa = 0, sb = 0;
        for (int k = 0; k < kThreads / 64; ++k) {
            sa += sh[2 * k];
            sb += sh[2 * k + 1];
        }
        sh[2 * (kThreads / 64)] = sa;
        sh[2 * (kThreads / 64) + 1] = sb;
    }
    __syncthreads();
    a = sh[2 * (kThreads / 64)];
    b = sh[2 * (kThreads / 64) + 1];
}

constexpr int kPerThread = kCompactChunk / kThreads;   // 4 virtual blocks per thread
// up to this many chunks (a 1,024-block chunk each; 1,024 chunks is a 1,024^3-cell
// grid) the emitting workgroups form their own chunk offsets
constexpr int kPrefixChunks = 1024;

// Flags (stamp == E) of the kPerThread consecutive virtual blocks from `base`, both
// stamp arrays in one 16-byte load each (every epoch's stamps are 256-byte aligned);
// element loads where the range ends inside them.
__device__ __forceinline__ void load_flags(const DevCtx &d, const int *pf, const int *gf, long long base, int E,
                                           int (&fp)[kPerThread], int (&fg)[kPerThread]) {
    static_assert(kPerThread == 4, "one int4 per array");
    if (base + kPerThread <= d.nbv) {
        const int4 a = *reinterpret_cast<const int4 *>(pf + base);
        const int4 b = *reinterpret_cast<const int4 *>(gf + base);
        fp[0] = a.x == E;
        fp[1] = a.y == E;
        fp[2] = a.z == E;
        fp[3] = a.w == E;
        fg[0] = b.x == E;
        fg[1] = b.y == E;
        fg[2] = b.z == E;
        fg[3] = b.w == E;
    } else {
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
            const long long v = base + k;
            fp[k] = (v < d.nbv) && (pf[v] == E);
            fg[k] = (v < d.nbv) && (gf[v] == E);
        }
    }
}

__device__ __forceinline__ void b_compact_count(const DevCtx &d) {
    __shared__ int sh[16];
    const int E = (int)d.counters[C_EPOCH] + 1;
    const int *pf = stamps(d.pflag, d.nbv, E);
    const int *gf = stamps(d.gflag, d.nbv, E);
    const long long base = (long long)blockIdx.x * kCompactChunk + threadIdx.x * kPerThread;
    int fp[kPerThread], fg[kPerThread];
    load_flags(d, pf, gf, base, E, fp, fg);
    int cp = 0, cg = 0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        cp += fp[k];
        cg += fg[k];
    }
    wg_sum2(cp, cg, sh);
    if (threadIdx.x == 0) {
        d.chunk_p[blockIdx.x] = cp;
        d.chunk_g[blockIdx.x] = cg;
    }
}

__global__ void __launch_bounds__(kThreads) k_compact_count(DevCtx d) { b_compact_count(d); }

// one launch for many jobs: workgroup row y runs job y
__global__ void __launch_bounds__(kThreads) k_compact_count_multi(const JobStep *__restrict__ jobs) {
    const JobStep &J = jobs[blockIdx.y];
    if ((long long)blockIdx.x * kCompactChunk >= J.d.nbv) return;
    b_compact_count(J.d);
}

// Exclusive scans of two arrays of `n` ints in place by one workgroup of T threads,
// side by side (every load of both in flight together); returns the two totals.
template <int T>
__device__ void wg_scan2_inplace(int *da, int *db, int n, int *sh, int &ta, int &tb) {
    const int per = (n + T - 1) / T;
    const int beg = min(n, threadIdx.x * per), end = min(n, beg + per);
    int la = 0, lb = 0;
    for (int i = beg; i < end; ++i) {
        la += da[i];
        lb += db[i];
    }
    // inclusive scans of the per-thread sums across the workgroup
    int va = la, vb = lb;
    const int lane = wave_lane();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(va, off), u = __shfl_up(vb, off);
        if (lane >= off) {
            va += t;
            vb += u;
        }
    }
    const int w = threadIdx.x >> 6;
    constexpr int W = T / 64;
    if (lane == 63) {
        sh[w] = va;
        sh[W + 1 + w] = vb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int aa = 0, ab = 0;
        for (int k = 0; k < W; ++k) {
            const int t = sh[k], u = sh[W + 1 + k];
            sh[k] = aa;
            sh[W + 1 + k] = ab;
            aa += t;
            ab += u;
        }
        sh[W] = aa;
        sh[2 * W + 1] = ab;
    }
    __syncthreads();
    int ra = sh[w] + va - la, rb = sh[W + 1 + w] + vb - lb;
    for (int i = beg; i < end; ++i) {
        const int t = da[i], u = db[i];
        da[i] = ra;
        db[i] = rb;
        ra += t;
        rb += u;
    }
    ta = sh[W];
    tb = sh[2 * W + 1];
    __syncthreads();
}

__device__ __forceinline__ void b_compact_scan(const DevCtx &d, int nchunks, int table) {
    __shared__ int sh[2 * (1024 / 64) + 2];
    int np, ng;
    wg_scan2_inplace<1024>(d.chunk_p, d.chunk_g, nchunks, sh, np, ng);
    if (threadIdx.x == 0) {
        if (ng > d.max_blocks || np > d.max_blocks) set_status(d.counters, ST_CAPACITY);
        d.counters[C_NPB] = (unsigned)min(np, d.max_blocks);
        d.counters[ngb_slot(table)] = (unsigned)min(ng, d.max_blocks);
        d.counters[C_MAXPB] = 0u;
        d.counters[C_TOTAL] = 0u;
    }
}

__global__ void __launch_bounds__(1024) k_compact_scan(DevCtx d, int nchunks, int table) { b_compact_scan(d, nchunks, table); }

// one launch for many jobs: workgroup row y runs job y
__global__ void __launch_bounds__(1024) k_compact_scan_multi(const JobStep *__restrict__ jobs) {
    const JobStep &J = jobs[blockIdx.y];
    b_compact_scan(J.d, (int)((J.d.nbv + kCompactChunk - 1) / kCompactChunk), J.table);
}

// Workgroup exclusive scan of one int per thread (256 threads); returns the total.
__device__ __forceinline__ int wg_excl_scan(int x, int &excl, int *sh) {
    int v = x;
    const int lane = wave_lane();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    const int w = threadIdx.x >> 6;
    if (lane == 63) sh[w] = v;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kThreads / 64; ++k) {
        const int t = sh[k];
        pre += (k < w) ? t : 0;
        tot += t;
    }
    excl = pre + v - x;
    __syncthreads();
    return tot;
}

// prefix: the chunks' exclusive offsets come from the chunk scan (false), or each
// workgroup sums the counts of the chunks before its own (true; the last one then
// writes the totals), which saves the scan's launch when there are few chunks.
template <bool kPrefix = false>
__device__ __forceinline__ void b_compact_emit(const DevCtx &d, int table, int nchunks = 0) {
    __shared__ int sh[8];
    __shared__ int pre[2 * (kThreads / 64)];
    const int E = (int)d.counters[C_EPOCH] + 1;
    const int *pf = stamps(d.pflag, d.nbv, E);
    const int *gf = stamps(d.gflag, d.nbv, E);
    const long long base = (long long)blockIdx.x * kCompactChunk + threadIdx.x * kPerThread;
    int fp[kPerThread], fg[kPerThread];
    load_flags(d, pf, gf, base, E, fp, fg);
    int cbp = 0, cbg = 0;   // counts of the chunks before this one
    if (kPrefix) {
        for (int c = threadIdx.x; c < (int)blockIdx.x; c += kThreads) {
            cbp += d.chunk_p[c];
            cbg += d.chunk_g[c];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            cbp += __shfl_xor(cbp, off);
            cbg += __shfl_xor(cbg, off);
        }
    }
    int cp = 0, cg = 0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        cp += fp[k];
        cg += fg[k];
    }
    if (kPrefix) {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            pre[w] = cbp;
            pre[kThreads / 64 + w] = cbg;
        }
    }
    int ep, eg;
    wg_excl_scan(cp, ep, sh);
    const int gtot = wg_excl_scan(cg, eg, sh);   // (the scans' barriers publish pre)
    int offp, offg;
    if (kPrefix) {
        int bp = 0, bg = 0;
#pragma unroll
        for (int k = 0; k < kThreads / 64; ++k) {
            bp += pre[k];
            bg += pre[kThreads / 64 + k];
        }
        offp = bp + ep;
        offg = bg + eg;
        if ((int)blockIdx.x == nchunks - 1 && threadIdx.x == kThreads - 1) {
            const int np = bp + ep + cp, ng = bg + eg + cg;
            if (ng > d.max_blocks || np > d.max_blocks) set_status(d.counters, ST_CAPACITY);
            d.counters[C_NPB] = (unsigned)min(np, d.max_blocks);
            d.counters[ngb_slot(table)] = (unsigned)min(ng, d.max_blocks);
            d.counters[C_MAXPB] = 0u;
            d.counters[C_TOTAL] = 0u;
        }
    } else {
        offp = d.chunk_p[blockIdx.x] + ep;
        offg = d.chunk_g[blockIdx.x] + eg;
    }
    int rp = offp, rg = offg;
    int ph[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int v = (int)(base + k);
        if (fp[k]) {
            if (rp < d.max_blocks) {
                d.plist[rp] = v;
                d.prank[v] = rp;
                d.bcount[rp] = 0;
                d.blo[rp] = 0xffffffffu;
                d.bhi[rp] = 0u;
            } else {
                d.prank[v] = -1;
            }
            ++rp;
        }
        ph[k] = -1;
        if (fg[k]) {
            if (rg < d.max_blocks) {
                glist_of(d, table)[rg] = v;
                ph[k] = rg;
            }
            ++rg;
        }
    }
    // every virtual block gets its page entry, so the table is valid without stamps
    if (base + kPerThread <= d.nbv) {
        *reinterpret_cast<int4 *>(page_of(d, table) + base) = make_int4(ph[0], ph[1], ph[2], ph[3]);
    } else {
#pragma unroll
        for (int k = 0; k < kPerThread; ++k)
            if (base + k < d.nbv) page_of(d, table)[base + k] = ph[k];
    }
    (void)gtot;
}

__global__ void __launch_bounds__(kThreads) k_compact_emit(DevCtx d, int table, int nchunks) {
    b_compact_emit<true>(d, table, nchunks);
}

__global__ void __launch_bounds__(kThreads) k_compact_emit_scanned(DevCtx d, int table) { b_compact_emit(d, table); }

// one launch for many jobs: workgroup row y runs job y
__global__ void __launch_bounds__(kThreads) k_compact_emit_multi(const JobStep *__restrict__ jobs) {
    const JobStep &J = jobs[blockIdx.y];
    if ((long long)blockIdx.x * kCompactChunk >= J.d.nbv) return;
    b_compact_emit(J.d, J.table);
}

// Each particle takes a slot in its block's bucket and writes its index there.
// Particles arrive nearly sorted (the previous G2P wrote them in block order), so
// a workgroup's 1024 consecutive particles span few blocks: slots are ranked
// inside the workgroup (a run of equal blocks gets consecutive slots) and each run
// costs one global atomic.  Slots past the bucket capacity are not written; the
// scan below reports the overflow.  The same launch zeroes this step's grid blocks.
constexpr int kCountPer = 4;                       // consecutive particles per thread
constexpr int kCountTile = kThreads * kCountPer;   // particles per workgroup

// reuse: the state is the one the context's previous G2P wrote; a block that G2P
// left unchanged keeps its order in the P2G (its particles sit at consecutive
// positions), so its bucket is not filled: the run's first and last positions go to
// the block's position range instead.
__device__ __forceinline__ void b_bucket_count(const DevCtx &d, int n, int zero_pool, int zero_table, bool reuse) {
    __shared__ int rblk[kCountTile];   // particle block rank of each particle of the tile (-1: skipped)
    __shared__ int base_of[kCountTile];
    __shared__ unsigned char kept_of[kCountTile];   // per run start: the block's order is kept
    __shared__ int wmax[kThreads / 64];
    const int tid = threadIdx.x, lane = wave_lane(), w = tid >> 6;
    const int E = (int)d.counters[C_EPOCH] + 1;   // the epoch of this sort (the bucket scan ends it)
    const int *pf = stamps(d.pflag, d.nbv, E);
    const int base = blockIdx.x * kCountTile;
    // zero a share of the pool blocks handed out this step
    {
        const long long nfl = (long long)d.counters[ngb_slot(zero_table)] * (kBlockFloats / 4);
        float4 *pool4 = reinterpret_cast<float4 *>(pool_of(d, zero_pool));
        for (long long t = (long long)blockIdx.x * kThreads + tid; t < nfl; t += (long long)gridDim.x * kThreads)
            pool4[t] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    int r[kCountPer];
    uint16_t sb[kCountPer];
    uint32_t kv[kCountPer];
    {
        // the thread's 4 keys and sub-cell codes in one 16-byte and one 8-byte load
        // (the library's buffers are 256-byte aligned), element loads at the tail
        const int i0 = base + tid * kCountPer;
        if (i0 + kCountPer <= n) {
            const uint4 k4 = *reinterpret_cast<const uint4 *>(d.key + i0);
            const uint2 s4 = *reinterpret_cast<const uint2 *>(d.sub + i0);
            kv[0] = k4.x;
            kv[1] = k4.y;
            kv[2] = k4.z;
            kv[3] = k4.w;
            sb[0] = (uint16_t)(s4.x & 0xffffu);
            sb[1] = (uint16_t)(s4.x >> 16);
            sb[2] = (uint16_t)(s4.y & 0xffffu);
            sb[3] = (uint16_t)(s4.y >> 16);
        } else {
#pragma unroll
            for (int k = 0; k < kCountPer; ++k) {
                kv[k] = i0 + k < n ? d.key[i0 + k] : 0xffffffffu;
                sb[k] = i0 + k < n ? d.sub[i0 + k] : (uint16_t)0;
            }
        }
    }
    static_assert(kCountPer == 4, "vector loads take 4 keys");
#pragma unroll
    for (int k = 0; k < kCountPer; ++k) {
        const int i = base + tid * kCountPer + k;
        r[k] = -1;
        if (i < n) {
            const uint32_t key = kv[k];
            if (key != 0xffffffffu) {
                // a key whose block was not stamped this step cannot be placed; the
                // stamp and the rank are loaded together (one memory round trip)
                const int f = pf[key >> 6];
                const int pr = d.prank[key >> 6];
                if (f == E) r[k] = pr;
                else set_status(d.counters, ST_STALE);
            }
        }
        rblk[tid * kCountPer + k] = r[k];
    }
    __syncthreads();
    // start of the run of equal blocks each element belongs to: inclusive max-scan
    // of (element starts a run ? position : 0)
    int st[kCountPer];
    int m = 0;
#pragma unroll
    for (int k = 0; k < kCountPer; ++k) {
        const int j = tid * kCountPer + k;
        const bool starts = (j == 0) || (rblk[j - 1] != r[k]);
        m = starts ? j : m;
        st[k] = m;
    }
    int v = m;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off);
        if (lane >= off) v = max(v, t);
    }
    if (lane == 63) wmax[w] = v;
    __syncthreads();
    int carry = 0;
    for (int k = 0; k < w; ++k) carry = max(carry, wmax[k]);
    const int up = __shfl_up(v, 1);                       // every lane takes part in the shuffle
    const int prev_thread = lane > 0 ? max(carry, up) : carry;   // max over all earlier threads
#pragma unroll
    for (int k = 0; k < kCountPer; ++k) st[k] = max(st[k], prev_thread);
    // the last element of each run takes the run's slots with one atomic
#pragma unroll
    for (int k = 0; k < kCountPer; ++k) {
        const int j = tid * kCountPer + k;
        if (r[k] < 0) continue;
        const bool last = (j == kCountTile - 1) || (rblk[j + 1] != r[k]);
        if (last) {
            base_of[st[k]] = atomicAdd(&d.bcount[r[k]], j - st[k] + 1);
            const bool keep = reuse && d.bchg[kv[k] >> 6] != E;
            kept_of[st[k]] = keep ? 1 : 0;
            if (keep) {
                atomicMin(&d.blo[r[k]], (uint32_t)(base + st[k]));
                atomicMax(&d.bhi[r[k]], (uint32_t)(base + j));
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCountPer; ++k) {
        const int j = tid * kCountPer + k;
        if (r[k] < 0 || kept_of[st[k]]) continue;
        const int slot = base_of[st[k]] + (j - st[k]);
        if (slot < kMaxBlockParticles) {
            d.bucket[(size_t)r[k] * kMaxBlockParticles + slot] = (uint32_t)(base + j);
            d.bsub[(size_t)r[k] * kMaxBlockParticles + slot] = sb[k];
        }
    }
}

__global__ void __launch_bounds__(kThreads) k_bucket_count(DevCtx d, int n, int zero_pool, int zero_table, int reuse) {
    b_bucket_count(d, n, zero_pool, zero_table, reuse != 0);
}

// one launch for many jobs: workgroup row y runs job y
__global__ void __launch_bounds__(kThreads) k_bucket_count_multi(const JobStep *__restrict__ jobs) {
    const JobStep &J = jobs[blockIdx.y];
    // a job's steps after its first read the state its own G2P wrote
    b_bucket_count(J.d, J.pa.n, J.table, J.table, !J.first);
}

// Exclusive scan of the bucket sizes into the first sorted position of every
// particle block (one workgroup of 1024 threads).  In a pass, element
// base + 1024 u + t (row u) belongs to thread t: the 16 loads of a thread are
// coalesced across the workgroup and all in flight together.  Each row is scanned
// across the workgroup (wave scans, then the wave totals through LDS), and the rows
// follow each other.
__device__ __forceinline__ void b_bucket_scan(const DevCtx &d) {
    constexpr int kRows = 16, kPass = kRows * 1024;
    __shared__ int wtot[kRows][16];   // per row: wave totals, then their exclusive scan
    __shared__ int rtot[kRows];       // per row: total
    __shared__ int wmx[16];
    const int np = (int)d.counters[C_NPB];
    const int tid = threadIdx.x, lane = wave_lane(), w = tid >> 6;
    int mx = 0, carry = 0;
    for (int base = 0; base < np; base += kPass) {
        int c[kRows], incl[kRows];
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
            const int k = base + u * 1024 + tid;
            c[u] = k < np ? d.bcount[k] : 0;
        }
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
            int v = c[u];
            mx = max(mx, v);
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(v, off);
                if (lane >= off) v += t;
            }
            incl[u] = v;
            if (lane == 63) wtot[u][w] = v;
        }
        __syncthreads();
        if (tid < kRows) {
            int run = 0;
            for (int k = 0; k < 16; ++k) {
                const int t = wtot[tid][k];
                wtot[tid][k] = run;
                run += t;
            }
            rtot[tid] = run;
        }
        __syncthreads();
        int run = carry;
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
            const int k = base + u * 1024 + tid;
            if (k < np) d.pstart[k] = run + wtot[u][w] + incl[u] - c[u];
            run += rtot[u];
        }
        carry = run;
        __syncthreads();   // wtot and rtot are rewritten by the next pass
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_down(mx, off));
    if (lane == 0) wmx[w] = mx;
    __syncthreads();
    if (tid == 0) {
        int m = 0;
        for (int k = 0; k < 16; ++k) m = max(m, wmx[k]);
        d.pstart[np] = carry;
        d.counters[C_MAXPB] = (unsigned)m;
        d.counters[C_TOTAL] = (unsigned)carry;
        // the sort's epoch becomes the current one (every kernel of the sort read the
        // previous value)
        d.counters[C_EPOCH] += 1u;
        if (m > kMaxBlockParticles) set_status(d.counters, ST_CAPACITY);
    }
    // the contribution bound for the P2G about to run: maxima of the slots the previous
    // P2G (or the stress pass) filled, which are cleared for the next.  Empty slots (a
    // sequence of fused steps, which form no bound) leave the last bound in place.
    static_assert(kBoundSlots == 64, "one wave reduces the slots");
    if (tid < kBoundSlots) {
        unsigned int *sx = d.bslots + tid * 32, *sy = d.bslots + (kBoundSlots + tid) * 32;
        unsigned int bxv = *sx, byv = *sy;
        *sx = 0u;
        *sy = 0u;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            bxv = max(bxv, (unsigned int)__shfl_xor((int)bxv, off));
            byv = max(byv, (unsigned int)__shfl_xor((int)byv, off));
        }
        if (tid == 0 && (bxv | byv) != 0u) {
            d.counters[C_BOUND_X] = bxv;
            d.counters[C_BOUND_Y] = byv;
        }
    }
}

__global__ void __launch_bounds__(1024) k_bucket_scan(DevCtx d) { b_bucket_scan(d); }

// one launch for many jobs: workgroup row y runs job y
__global__ void __launch_bounds__(1024) k_bucket_scan_multi(const JobStep *__restrict__ jobs) {
    const JobStep &J = jobs[blockIdx.y];
    b_bucket_scan(J.d);
}

}  // namespace

void launch_flag_keys(const DevCtx &d, const PartArgs &pa, int epoch_offset, hipStream_t s) {
    if (pa.n <= 0) return;
    hipLaunchKernelGGL(k_flag_keys, dim3((pa.n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, d, pa, epoch_offset);
}

void launch_clear_flags(const DevCtx &d, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flags, dim3(1024), dim3(256), 0, s, d);
}

void launch_compact(const DevCtx &d, int table, hipStream_t s) {
    const int nchunks = (int)((d.nbv + kCompactChunk - 1) / kCompactChunk);
    hipLaunchKernelGGL(k_compact_count, dim3(nchunks), dim3(kThreads), 0, s, d);
    if (nchunks <= kPrefixChunks) {
        // each emitting workgroup sums the chunk counts before its own
        hipLaunchKernelGGL(k_compact_emit, dim3(nchunks), dim3(kThreads), 0, s, d, table, nchunks);
    } else {
        hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, d, nchunks, table);
        hipLaunchKernelGGL(k_compact_emit_scanned, dim3(nchunks), dim3(kThreads), 0, s, d, table);
    }
}

void launch_sort_multi(const JobStep *dev, const JobStep *host, int njobs, hipStream_t s) {
    int flag_grid = 0, chunks = 1, tiles = 1024;
    for (int j = 0; j < njobs; ++j) {
        const JobStep &J = host[j];
        if (J.first) flag_grid = std::max(flag_grid, (J.pa.n + kThreads - 1) / kThreads);
        chunks = std::max(chunks, (int)((J.d.nbv + kCompactChunk - 1) / kCompactChunk));
        tiles = std::max(tiles, (J.pa.n + kCountTile - 1) / kCountTile);
    }
    if (flag_grid > 0) hipLaunchKernelGGL(k_flag_keys_multi, dim3(flag_grid, njobs), dim3(kThreads), 0, s, dev);
    hipLaunchKernelGGL(k_compact_count_multi, dim3(chunks, njobs), dim3(kThreads), 0, s, dev);
    hipLaunchKernelGGL(k_compact_scan_multi, dim3(1, njobs), dim3(1024), 0, s, dev);
    hipLaunchKernelGGL(k_compact_emit_multi, dim3(chunks, njobs), dim3(kThreads), 0, s, dev);
    hipLaunchKernelGGL(k_bucket_count_multi, dim3(tiles, njobs), dim3(kThreads), 0, s, dev);
    hipLaunchKernelGGL(k_bucket_scan_multi, dim3(1, njobs), dim3(1024), 0, s, dev);
}

void launch_bucket(const DevCtx &d, int n, int zero_pool, int zero_table, hipStream_t s, bool reuse) {
    // at least a few hundred workgroups, so that the pool clearing is spread wide
    const int tiles = (n + kCountTile - 1) / kCountTile;
    hipLaunchKernelGGL(k_bucket_count, dim3(tiles > 1024 ? tiles : 1024), dim3(kThreads), 0, s, d, n, zero_pool,
                       zero_table, reuse ? 1 : 0);
    hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(1024), 0, s, d);
}

}  // namespace ck
