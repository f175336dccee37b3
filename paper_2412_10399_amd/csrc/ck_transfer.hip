// Particle-to-grid transfer, grid update and grid-to-particle transfer of the
// compact-kernel MPM step on the two staggered grids (sections 4.2-4.5 of the
// paper; pipeline order of section 3.2).
//
// Work decomposition: one workgroup per 4^3-cell particle block.  A block's
// particles touch G- nodes [4B, 4B+4] and G+ nodes [4B-1, 4B+4] on each axis
// (5^3 + 6^3 = 341 nodes), so that tile is staged in LDS: P2G sums into it and
// flushes each nonzero node once to the grid pool with a global float atomic; G2P
// reads the updated velocities of the same tile from LDS.
// Grid storage is a pool of 2 KiB blocks, [grid][channel m, p0, p1, p2][64 nodes],
// reached through a page table indexed by virtual block id.
#include "ck_common.hpp"

namespace ck {

namespace {

__device__ __forceinline__ void block_coords(const Geometry &g, int vb, int &bx, int &by, int &bz) {
    bx = vb % g.NB[0];
    by = (vb / g.NB[0]) % g.NB[1];
    bz = vb / (g.NB[0] * g.NB[1]);
}

// Physical pool block of the 27 neighbours of block (bx,by,bz), -1 when inactive.
__device__ __forceinline__ void load_neighbours(const DevCtx &d, int bx, int by, int bz, int E, int *nbr) {
    const int t = threadIdx.x;
    if (t < 27) {
        const int x = bx + t % 3 - 1, y = by + (t / 3) % 3 - 1, z = bz + t / 9 - 1;
        int ph = -1;
        if (x >= 0 && y >= 0 && z >= 0 && x < d.geo.NB[0] && y < d.geo.NB[1] && z < d.geo.NB[2]) {
            const int v = vblock_id(d.geo, x, y, z);
            if (stamps(d.gflag, d.nbv, E)[v] == E) ph = d.page[v];
        }
        nbr[t] = ph;
    }
}

// Map tile node `ni` (0..340) of block (bx,by,bz) to its grid (0 = G-, 1 = G+) and
// global node coordinates.
__device__ __forceinline__ void tile_node(int ni, int bx, int by, int bz, int &g, int &ix, int &iy, int &iz) {
    if (ni < kTileMinus) {
        g = 0;
        ix = 4 * bx + ni % 5;
        iy = 4 * by + (ni / 5) % 5;
        iz = 4 * bz + ni / 25;
    } else {
        const int k = ni - kTileMinus;
        g = 1;
        ix = 4 * bx - 1 + k % 6;
        iy = 4 * by - 1 + (k / 6) % 6;
        iz = 4 * bz - 1 + k / 36;
    }
}

// Pool address of channel `ch` of node (ix,iy,iz) on grid g, or -1.
__device__ __forceinline__ long long pool_index(const DevCtx &d, const int *nbr, int bx, int by, int bz, int g, int ix,
                                                int iy, int iz, int ch) {
    if (ix < 0 || iy < 0 || iz < 0 || ix > d.geo.n[0] || iy > d.geo.n[1] || iz > d.geo.n[2]) return -1;
    const int nb = ((iz >> 2) - bz + 1) * 9 + ((iy >> 2) - by + 1) * 3 + ((ix >> 2) - bx + 1);
    const int ph = nbr[nb];
    if (ph < 0) return -1;
    return (long long)ph * kBlockFloats + g * 256 + ch * 64 + ((iz & 3) * 16 + (iy & 3) * 4 + (ix & 3));
}

// Particle block of this workgroup in the round of blocks [base, base + G) (G
// workgroups).  Workgroups are dealt to the 8 XCDs round-robin by index; each XCD
// gets a contiguous, equal share of the round, so the halo nodes that neighbouring
// blocks share are reused from the same L2 and every XCD has the same work.
// Returns -1 when the workgroup has no block in this round.  Grids that are not a
// multiple of 8 keep the identity mapping.
__device__ __forceinline__ int round_block(int base, int np) {
    const int G = gridDim.x;
    const int m = min(G, np - base);
    if (G & 7) return (int)blockIdx.x < m ? base + (int)blockIdx.x : -1;
    const int per = (m + 7) >> 3;
    const int x = blockIdx.x & 7, y = blockIdx.x >> 3;
    const int i = x * per + y;
    return (y < per && i < m) ? base + i : -1;
}

struct Particle {
    float x[3], v[3], B[9], H[9];   // H = F - I
};

__device__ __forceinline__ void load_particle(const PartArgs &pa, int p, Particle &q, bool full) {
    const long long S = pa.stride;
#pragma unroll
    for (int a = 0; a < 3; ++a) q.x[a] = pa.in[a * S + p];
    if (full) {
#pragma unroll
        for (int a = 0; a < 3; ++a) q.v[a] = pa.in[(3 + a) * S + p];
#pragma unroll
        for (int a = 0; a < 9; ++a) q.B[a] = pa.in[(6 + a) * S + p];
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) q.H[a] = pa.in[(15 + a) * S + p];
}

// ---------------------------------------------------------------- block sort
// Exact stable order of one block's particles by (cell, particle index): counting
// sort by cell in LDS, then each particle's rank among the equal-cell particles by
// index.  Used where the sorting permutation itself is asked for.
constexpr int kSlots = kMaxBlockParticles / kThreads;   // bucket entries per thread
constexpr uint32_t kIndexMask = (1u << kIndexBits) - 1u;

__global__ void __launch_bounds__(kThreads) k_block_sort(DevCtx d) {
    __shared__ uint32_t lbuf[kMaxBlockParticles];
    __shared__ int ccount[64];
    __shared__ int cstart[65];
    const int np = (int)d.counters[C_NPB];
    const int tid = threadIdx.x;
    for (int base = 0; base < np; base += gridDim.x) {
        const int r = round_block(base, np);
        if (r < 0) continue;
        const int s = d.pstart[r];
        const int cnt = d.pstart[r + 1] - s;
        if (cnt > kMaxBlockParticles) continue;   // reported by the bucket scan
        if (tid < 64) ccount[tid] = 0;
        __syncthreads();
        uint32_t pk[kSlots];
        int ps[kSlots];
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int j = tid + k * kThreads;
            if (j < cnt) {
                const uint32_t idx = d.bucket[(size_t)r * kMaxBlockParticles + j];
                const uint32_t cell = d.key[idx] & 63u;
                pk[k] = (cell << kIndexBits) | idx;
                ps[k] = atomicAdd(&ccount[cell], 1);
            }
        }
        __syncthreads();
        if (tid < 64) {
            const int c = ccount[tid];
            int v = c;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(v, off);
                if (tid >= off) v += t;
            }
            cstart[tid] = v - c;
            if (tid == 63) cstart[64] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int j = tid + k * kThreads;
            if (j < cnt) lbuf[cstart[pk[k] >> kIndexBits] + ps[k]] = pk[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int j = tid + k * kThreads;
            if (j < cnt) {
                const uint32_t v = lbuf[j];
                const int c = (int)(v >> kIndexBits);
                const int lo = cstart[c], hi = cstart[c + 1];
                int rank = lo;
                for (int q = lo; q < hi; ++q) rank += (lbuf[q] < v) ? 1 : 0;
                d.perm[s + rank] = v & kIndexMask;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- stress
// Kirchhoff stress of every particle of the current buffer, for a P2G that does not
// follow a G2P of this context (first step, or positions changed by the caller).
__global__ void __launch_bounds__(kThreads) k_stress(DevCtx d, PartArgs pa) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= pa.n) return;
    const long long S = pa.stride;
    float H[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) H[a] = pa.in[(15 + a) * S + p];
    const int mi = pa.mat_in ? (int)pa.mat_in[p] : 0;
    const DevMaterial M = d.mats[mi < d.n_mat ? mi : 0];
    float tau[6];
    kirchhoff(M, H, tau);
#pragma unroll
    for (int i = 0; i < 6; ++i) d.tau[i * d.tau_stride + p] = tau[i];
}

// ---------------------------------------------------------------- P2G
// Particle contributions (section 4.4 APIC transfer plus the MLS stress impulse of
// section 4.5): mass w m_p and momentum w (m_p v_p + Q (x_i - x_p)) with
//   Q = (m_p B_p - dt V_p^0 tau_p) D_p^-1,
// where grad Phi_i = w D^-1 (x_i - x_p) and f_i = -V^0 tau grad Phi_i.  In cell units,
// with xi the particle's fractional position in its G- cell c, G- node c + o
// (o in {0,1}^3) sits at x_i - x_p = dx (o - xi) and G+ node c + r at
// dx (r + 1/2 - xi), G+ being shifted half a cell from G-.  With base = m_p v_p - Q xi
// the momenta are base + Q o and base + Q (r + 1/2).
//
// One wave per block, lane c owning G- cell c of the block, and no atomics inside
// the block (LDS float atomics run about a hundred times slower than plain LDS
// traffic on gfx950).  A particle in the upper or lower half of its cell along an
// axis reaches G+ nodes c, c + 1 or c - 1, c on that axis, so the half-cell octant
// fixes which 8 of the 27 G+ nodes around c it touches.  The block's particles are
// therefore ordered by (octant, cell, index); for each octant in turn, the wave
// stages that octant's particles as compact records in LDS (lane = particle,
// coalesced reads: the previous G2P wrote the state in this order), and lane c sums
// the records of cell c into registers: 8 G- nodes and, at indices known at compile
// time for the octant, 8 of its 27 G+ nodes.  The register sums are then added into
// the LDS tile in conflict-free phases (every lane targets a different node in a
// phase) and each nonzero tile node is flushed to the pool with one global atomic.
constexpr int kP2GThreads = 64;
constexpr int kBins = 512;                 // (octant, cell) bins of a block: octant * 64 + cell
constexpr int kRecVec = 5;                 // float4 per staged record
constexpr int kHold = 8;                   // bucket entries per lane kept in registers
constexpr uint32_t kNoRecord = 0xffffu;

// Record: xi[3] s+[3] m_p base[3] Q[9] (row-major), sub code.
__device__ __forceinline__ void stage_particle(const DevCtx &d, const PartArgs &pa, int p, int bx, int by, int bz,
                                               float dt, float4 *rec) {
    float out[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) out[i] = 0.0f;
    uint32_t code = kNoRecord;
    const long long S = pa.stride;
    float x[3], v[3], B[9], tau[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = pa.in[a * S + p];
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = pa.in[(3 + a) * S + p];
#pragma unroll
    for (int a = 0; a < 9; ++a) B[a] = pa.in[(6 + a) * S + p];
#pragma unroll
    for (int i = 0; i < 6; ++i) tau[i] = d.tau[i * d.tau_stride + p];
    const int mi = pa.mat_in ? (int)pa.mat_in[p] : 0;
    const DevMaterial M = d.mats[mi < d.n_mat ? mi : 0];
    CellCoord cc;
    if (!cell_coord(d.geo, x, cc)) {
        set_status(d.counters, ST_DOMAIN);
    } else if ((cc.c[0] >> 2) != bx || (cc.c[1] >> 2) != by || (cc.c[2] >> 2) != bz) {
        set_status(d.counters, ST_STALE);
    } else {
        code = sub_code(cc);
        Weights w;
        axis_weights(cc, w);
        float Di[9];
        moment_inverse(cc, w, Di);
        const float T[9] = {tau[0], tau[3], tau[4], tau[3], tau[1], tau[5], tau[4], tau[5], tau[2]};
        const float k = dt * M.vol0;
        float A[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) A[i] = M.mass * B[i] - k * T[i];
        const float sc = d.geo.inv_dx_f;
        float Q[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                Q[3 * i + j] = sc * (A[3 * i] * Di[j] + A[3 * i + 1] * Di[3 + j] + A[3 * i + 2] * Di[6 + j]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            out[a] = cc.xm[a];
            out[3 + a] = w.sp[a];
            out[7 + a] = M.mass * v[a] - (Q[3 * a] * cc.xm[0] + Q[3 * a + 1] * cc.xm[1] + Q[3 * a + 2] * cc.xm[2]);
        }
        out[6] = M.mass;
#pragma unroll
        for (int i = 0; i < 9; ++i) out[10 + i] = Q[i];
    }
    rec[0] = make_float4(out[0], out[1], out[2], out[3]);
    rec[1] = make_float4(out[4], out[5], out[6], out[7]);
    rec[2] = make_float4(out[8], out[9], out[10], out[11]);
    rec[3] = make_float4(out[12], out[13], out[14], out[15]);
    rec[4] = make_float4(out[16], out[17], out[18], __uint_as_float(code));
}

struct Rec {
    float xm[3], sp[3], mass, base[3], Q[9];
    uint32_t code;
};

__device__ __forceinline__ void read_rec(const float4 *r, Rec &q) {
    const float4 a = r[0], b = r[1], c = r[2], e = r[3], f = r[4];
    q.xm[0] = a.x; q.xm[1] = a.y; q.xm[2] = a.z; q.sp[0] = a.w;
    q.sp[1] = b.x; q.sp[2] = b.y; q.mass = b.z; q.base[0] = b.w;
    q.base[1] = c.x; q.base[2] = c.y; q.Q[0] = c.z; q.Q[1] = c.w;
    q.Q[2] = e.x; q.Q[3] = e.y; q.Q[4] = e.z; q.Q[5] = e.w;
    q.Q[6] = f.x; q.Q[7] = f.y; q.Q[8] = f.z; q.code = __float_as_uint(f.w);
}

// Adds w (m, m0 + Q o) for the 8 nodes o in {0,1}^3 of one grid, weights w[a][o_a],
// into acc[4 n(o) + channel], n(o) given by the node map of the grid.
template <typename NodeMap>
__device__ __forceinline__ void add_corners(const float (&w)[3][2], float mass, const float (&m0)[3], const float (&Q)[9],
                                            float *acc, NodeMap node) {
    float wxy[4];
#pragma unroll
    for (int oy = 0; oy < 2; ++oy)
#pragma unroll
        for (int ox = 0; ox < 2; ++ox) wxy[2 * oy + ox] = w[0][ox] * w[1][oy];
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy)
#pragma unroll
            for (int ox = 0; ox < 2; ++ox) {
                const float wt = wxy[2 * oy + ox] * w[2][oz];
                const int n = node(ox, oy, oz);
                acc[4 * n] += wt * mass;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float mom = m0[a] + (ox ? Q[3 * a] : 0.0f) + (oy ? Q[3 * a + 1] : 0.0f) + (oz ? Q[3 * a + 2] : 0.0f);
                    acc[4 * n + 1 + a] += wt * mom;
                }
            }
}

// One record of octant K into the cell sums: 8 G- nodes (am[4 o + ch],
// o = ox + 2 oy + 4 oz) and 8 of the 27 G+ nodes c + r, r in {-1,0,1}^3
// (ap[4 ((rz+1) 9 + (ry+1) 3 + rx+1) + ch]); along axis a the G+ nodes are
// r = o - 1 + bit_a(K).
template <int K>
__device__ __forceinline__ void accumulate_octant(const Rec &q, float (&am)[32], float (&ap)[108]) {
    constexpr int ux = K & 1, uy = (K >> 1) & 1, uz = (K >> 2) & 1;
    float wm[3][2], wp[3][2];
    constexpr int up[3] = {ux, uy, uz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        wm[a][0] = 1.0f - q.xm[a] - q.sp[a];
        wm[a][1] = q.xm[a] + q.sp[a];
        const float xp = up[a] ? q.xm[a] - 0.5f : q.xm[a] + 0.5f;
        wp[a][0] = 1.0f - xp + q.sp[a];
        wp[a][1] = xp - q.sp[a];
    }
    add_corners(wm, q.mass, q.base, q.Q, am, [](int ox, int oy, int oz) { return ox + 2 * oy + 4 * oz; });
    // G+ momentum at the first node r0 = up - 1: base + Q (r0 + 1/2)
    float m0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        m0[a] = q.base[a] + (ux - 0.5f) * q.Q[3 * a] + (uy - 0.5f) * q.Q[3 * a + 1] + (uz - 0.5f) * q.Q[3 * a + 2];
    add_corners(wp, q.mass, m0, q.Q, ap,
                [](int ox, int oy, int oz) { return (oz + uz) * 9 + (oy + uy) * 3 + (ox + ux); });
}

// All records of octant K: staged by the wave in chunks of 64, summed by their cell's lane.
template <int K>
__device__ __forceinline__ void octant_pass(const DevCtx &d, const PartArgs &pa, float dt, int s, int bx, int by,
                                            int bz, const int *bstart, float4 *rec, int lane, float (&am)[32],
                                            float (&ap)[108]) {
    const uint32_t want = ((uint32_t)lane << 3) | (uint32_t)K;
    const int olo = bstart[K * 64], ohi = bstart[K * 64 + 64];
    const int clo = bstart[K * 64 + lane], chi = bstart[K * 64 + lane + 1];
    for (int t0 = olo; t0 < ohi; t0 += kP2GThreads) {
        if (t0 + lane < ohi) stage_particle(d, pa, (int)d.perm[s + t0 + lane], bx, by, bz, dt, &rec[lane * kRecVec]);
        __syncthreads();
        const int lo = max(clo, t0), hi = min(chi, t0 + kP2GThreads);
        for (int i = lo; i < hi; ++i) {
            Rec q;
            read_rec(&rec[(i - t0) * kRecVec], q);
            if (q.code != want) {
                if (q.code != kNoRecord) set_status(d.counters, ST_STALE);
                continue;
            }
            accumulate_octant<K>(q, am, ap);
        }
        __syncthreads();
    }
}

// Adds the register sums of G+ node c + r, N = (rz+1) 9 + (ry+1) 3 + rx+1, into the
// tile; every lane targets a different node.
template <int N>
__device__ __forceinline__ void flush_plus(float *tile_p, int cx, int cy, int cz, const float (&ap)[108]) {
    constexpr int rx = N % 3, ry = (N / 3) % 3, rz = N / 9;
    const int node = (cz + rz) * 36 + (cy + ry) * 6 + cx + rx;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) tile_p[ch * kTilePlus + node] += ap[4 * N + ch];
    __syncthreads();
}

template <int... N>
__device__ __forceinline__ void flush_plus_list(float *tile_p, int cx, int cy, int cz, const float (&ap)[108]) {
    (flush_plus<N>(tile_p, cx, cy, cz, ap), ...);
}

__device__ __forceinline__ int bin_of(uint32_t sub) { return (int)((sub & 7u) * 64u + (sub >> 3)); }

__global__ void __launch_bounds__(kP2GThreads, 2) k_p2g(DevCtx d, PartArgs pa, float dt) {
    __shared__ int bcnt[kBins];                 // counts, then placement cursors
    __shared__ int bstart[kBins + 1];
    __shared__ int nbr[27];
    // ordering buffer, later the staged records and the tile
    constexpr int kTileFloats = 4 * (kTileMinus + kTilePlus);
    constexpr int kUnionFloats = kMaxBlockParticles > kP2GThreads * 4 * kRecVec + kTileFloats
                                     ? kMaxBlockParticles
                                     : kP2GThreads * 4 * kRecVec + kTileFloats;
    __shared__ float4 area4[kUnionFloats / 4];
    float *area = reinterpret_cast<float *>(area4);
    uint32_t *lbuf = reinterpret_cast<uint32_t *>(area4);
    float4 *rec = area4;
    float *tile_m = area + kP2GThreads * 4 * kRecVec;   // [4][125]
    float *tile_p = tile_m + 4 * kTileMinus;              // [4][216]
    const int np = (int)d.counters[C_NPB];
    const int E = (int)d.counters[C_EPOCH];
    const int lane = threadIdx.x;
    const int cx = lane & 3, cy = (lane >> 2) & 3, cz = lane >> 4;
    for (int base = 0; base < np; base += gridDim.x) {
        const int r = round_block(base, np);
        if (r < 0) continue;
        const int vb = d.plist[r];
        int bx, by, bz;
        block_coords(d.geo, vb, bx, by, bz);
        const int s = d.pstart[r];
        const int cnt = d.pstart[r + 1] - s;
        if (cnt > kMaxBlockParticles) continue;   // reported by the bucket scan
        const uint32_t *bkt = d.bucket + (size_t)r * kMaxBlockParticles;

        // ---- order the block's particles by (octant, cell, index)
        for (int b = lane; b < kBins; b += kP2GThreads) bcnt[b] = 0;
        __syncthreads();
        uint32_t hidx[kHold];
        int hbin[kHold];
#pragma unroll
        for (int k = 0; k < kMaxBlockParticles / kP2GThreads; ++k) {
            const int j = lane + k * kP2GThreads;
            if (j >= cnt) break;
            const uint32_t idx = bkt[j];
            const int bin = bin_of(d.sub[idx]);
            if (k < kHold) {
                hidx[k] = idx;
                hbin[k] = bin;
            }
            atomicAdd(&bcnt[bin], 1);
        }
        __syncthreads();
        {
            // exclusive scan of the 512 bins, 8 per lane
            int loc[kBins / kP2GThreads];
            int sum = 0;
#pragma unroll
            for (int k = 0; k < kBins / kP2GThreads; ++k) {
                loc[k] = bcnt[lane * (kBins / kP2GThreads) + k];
                sum += loc[k];
            }
            int v = sum;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(v, off);
                if (lane >= off) v += t;
            }
            int run = v - sum;
#pragma unroll
            for (int k = 0; k < kBins / kP2GThreads; ++k) {
                bstart[lane * (kBins / kP2GThreads) + k] = run;
                bcnt[lane * (kBins / kP2GThreads) + k] = run;
                run += loc[k];
            }
            if (lane == 63) bstart[kBins] = run;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kMaxBlockParticles / kP2GThreads; ++k) {
            const int j = lane + k * kP2GThreads;
            if (j >= cnt) break;
            uint32_t idx;
            int bin;
            if (k < kHold) {
                idx = hidx[k];
                bin = hbin[k];
            } else {
                idx = bkt[j];
                bin = bin_of(d.sub[idx]);
            }
            lbuf[atomicAdd(&bcnt[bin], 1)] = idx;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kMaxBlockParticles / kP2GThreads; ++k) {
            const int j = lane + k * kP2GThreads;
            if (j >= cnt) break;
            uint32_t idx;
            int bin;
            if (k < kHold) {
                idx = hidx[k];
                bin = hbin[k];
            } else {
                idx = bkt[j];
                bin = bin_of(d.sub[idx]);
            }
            const int lo = bstart[bin], hi = bstart[bin + 1];
            int rank = lo;
            for (int q = lo; q < hi; ++q) rank += (lbuf[q] < idx) ? 1 : 0;
            d.perm[s + rank] = idx;
        }
        __threadfence_block();   // the order is read back below by other lanes
        __syncthreads();

        // ---- per-cell register sums, one octant at a time
        load_neighbours(d, bx, by, bz, E, nbr);
        for (int q = lane; q < kTileFloats; q += kP2GThreads) tile_m[q] = 0.0f;
        float am[32], ap[108];
#pragma unroll
        for (int i = 0; i < 32; ++i) am[i] = 0.0f;
#pragma unroll
        for (int i = 0; i < 108; ++i) ap[i] = 0.0f;
        // Octants in order; a G+ node is added to the tile as soon as no later octant
        // reaches it, which keeps at most 15 of the 27 node sums live at a time.
        octant_pass<0>(d, pa, dt, s, bx, by, bz, bstart, rec, lane, am, ap);
        octant_pass<1>(d, pa, dt, s, bx, by, bz, bstart, rec, lane, am, ap);
        flush_plus_list<0, 1, 2>(tile_p, cx, cy, cz, ap);                      // ry = rz = -1
        octant_pass<2>(d, pa, dt, s, bx, by, bz, bstart, rec, lane, am, ap);
        octant_pass<3>(d, pa, dt, s, bx, by, bz, bstart, rec, lane, am, ap);
        flush_plus_list<3, 4, 5, 6, 7, 8>(tile_p, cx, cy, cz, ap);             // rz = -1
        octant_pass<4>(d, pa, dt, s, bx, by, bz, bstart, rec, lane, am, ap);
        octant_pass<5>(d, pa, dt, s, bx, by, bz, bstart, rec, lane, am, ap);
        flush_plus_list<9, 10, 11, 18, 19, 20>(tile_p, cx, cy, cz, ap);        // ry = -1
        octant_pass<6>(d, pa, dt, s, bx, by, bz, bstart, rec, lane, am, ap);
        octant_pass<7>(d, pa, dt, s, bx, by, bz, bstart, rec, lane, am, ap);
        flush_plus_list<12, 13, 14, 15, 16, 17, 21, 22, 23, 24, 25, 26>(tile_p, cx, cy, cz, ap);
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int node = (cz + (o >> 2)) * 25 + (cy + ((o >> 1) & 1)) * 5 + cx + (o & 1);
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) tile_m[ch * kTileMinus + node] += am[4 * o + ch];
            __syncthreads();
        }
        // ---- flush every nonzero tile node to the pool
        for (int ni = lane; ni < kTileNodes; ni += kP2GThreads) {
            int g, ix, iy, iz;
            tile_node(ni, bx, by, bz, g, ix, iy, iz);
            const long long a = pool_index(d, nbr, bx, by, bz, g, ix, iy, iz, 0);
            float val[4];
#pragma unroll
            for (int ch = 0; ch < 4; ++ch)
                val[ch] = ni < kTileMinus ? tile_m[ch * kTileMinus + ni] : tile_p[ch * kTilePlus + ni - kTileMinus];
            const bool any = val[0] != 0.0f || val[1] != 0.0f || val[2] != 0.0f || val[3] != 0.0f;
            if (!any) continue;
            if (a < 0) {
                set_status(d.counters, ST_CAPACITY);
                continue;
            }
#pragma unroll
            for (int ch = 0; ch < 4; ++ch)
                if (val[ch] != 0.0f) atomicAdd(&d.pool[a + ch * 64], val[ch]);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- grid update
// Section 4.3 grid update on each grid: m v~ = m v + dt f (the stress impulse is
// already in the momentum), plus gravity; v~ = 0 where m = 0 and on wall nodes.
__global__ void __launch_bounds__(128) k_grid_update(DevCtx d, float dt, float g0, float g1, float g2) {
    const int ng = (int)d.counters[C_NGB];
    const int t = threadIdx.x;
    const int g = t >> 6, l = t & 63;
    const int lx = l & 3, ly = (l >> 2) & 3, lz = l >> 4;
    for (int b = blockIdx.x; b < ng; b += gridDim.x) {
        int bx, by, bz;
        block_coords(d.geo, d.glist[b], bx, by, bz);
        const int ix = 4 * bx + lx, iy = 4 * by + ly, iz = 4 * bz + lz;
        const bool inside = ix >= d.geo.stick_lo[g] && iy >= d.geo.stick_lo[g] && iz >= d.geo.stick_lo[g] &&
                            ix <= d.geo.stick_hi[g][0] && iy <= d.geo.stick_hi[g][1] && iz <= d.geo.stick_hi[g][2];
        float *blk = d.pool + (size_t)b * kBlockFloats + g * 256;
        const float m = blk[l];
        float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f;
        if (m > 0.0f && inside) {
            const float im = fast_rcp(m);
            v0 = blk[64 + l] * im + dt * g0;
            v1 = blk[128 + l] * im + dt * g1;
            v2 = blk[192 + l] * im + dt * g2;
        }
        blk[64 + l] = v0;
        blk[128 + l] = v1;
        blk[192 + l] = v2;
    }
}

// ---------------------------------------------------------------- G2P
// v_p = 1/2 sum_k sum_i w v~_i,   B_p = 1/2 sum_k sum_i w v~_i (x_i - x_p)^T,
// C_p = B_p D_p^-1,   F <- (I + dt C_p) F,   plasticity,   x <- x + dt v_p.
// The new state is written at the particle's sorted position in the other buffer,
// together with its next cell key and the activation stamps of the next step.
__global__ void __launch_bounds__(kThreads) k_g2p(DevCtx d, PartArgs pa, float dt) {
    __shared__ float vt[3 * kTileNodes];
    __shared__ int nbr[27];
    const int np = (int)d.counters[C_NPB];
    const int E = (int)d.counters[C_EPOCH];
    const int tid = threadIdx.x;
    const long long S = pa.stride;
    for (int base = 0; base < np; base += gridDim.x) {
        const int r = round_block(base, np);
        if (r < 0) continue;
        const int vb = d.plist[r];
        int bx, by, bz;
        block_coords(d.geo, vb, bx, by, bz);
        const int s = d.pstart[r];
        const int cnt = d.pstart[r + 1] - s;
        if (cnt > kMaxBlockParticles) continue;
        load_neighbours(d, bx, by, bz, E, nbr);
        __syncthreads();
        for (int t = tid; t < 3 * kTileNodes; t += kThreads) {
            const int ch = t / kTileNodes;
            const int ni = t - ch * kTileNodes;
            int g, ix, iy, iz;
            tile_node(ni, bx, by, bz, g, ix, iy, iz);
            const long long a = pool_index(d, nbr, bx, by, bz, g, ix, iy, iz, ch + 1);
            vt[t] = a >= 0 ? d.pool[a] : 0.0f;
        }
        __syncthreads();
        for (int j = tid; j < cnt; j += kThreads) {
            const int p = (int)d.perm[s + j];
            const int out = s + j;
            Particle q;
            load_particle(pa, p, q, false);
            CellCoord cc;
            bool ok = cell_coord(d.geo, q.x, cc);
            ok = ok && (cc.c[0] >> 2) == bx && (cc.c[1] >> 2) == by && (cc.c[2] >> 2) == bz;
            if (!ok) {
                set_status(d.counters, ST_STALE);
                d.key[out] = 0xffffffffu;
                continue;
            }
            const int mi = pa.mat_in ? (int)pa.mat_in[p] : 0;
            const DevMaterial M = d.mats[mi < d.n_mat ? mi : 0];
            Weights w;
            axis_weights(cc, w);
            float Di[9];
            moment_inverse(cc, w, Di);
            // Gather.  The affine matrix sums w v~ (x_i - x_p)^T, whose weights have a zero
            // dual-grid first moment; subtracting one stencil node's velocity c first keeps
            // the FP32 sums at the size of the velocity differences, and c drops out:
            //   1/2 sum w (v~ - c)(x_i - x_p)^T = 1/2 sum w v~ (x_i - x_p)^T,
            //   v_p = c + 1/2 sum w (v~ - c)   (the weights of each grid sum to one).
            const int tm0 = ((cc.c[2] - 4 * bz) * 5 + (cc.c[1] - 4 * by)) * 5 + (cc.c[0] - 4 * bx);
            const int tp0 = kTileMinus + ((cc.bp[2] - 4 * bz + 1) * 6 + (cc.bp[1] - 4 * by + 1)) * 6 + (cc.bp[0] - 4 * bx + 1);
            const float cref[3] = {vt[tm0], vt[kTileNodes + tm0], vt[2 * kTileNodes + tm0]};
            float vs[3] = {0.0f, 0.0f, 0.0f};
            float Bh[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) Bh[i] = 0.0f;
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const float *xi = g == 0 ? cc.xm : cc.xp;
                const int t0 = g == 0 ? tm0 : tp0;
                const int sy = g == 0 ? 5 : 6, sz = g == 0 ? 25 : 36;
                const float(*wa)[2] = g == 0 ? w.wm : w.wp;
                float S3[3] = {0.0f, 0.0f, 0.0f};
                float T[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) T[i] = 0.0f;
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
                    const float wt = wa[0][ox] * wa[1][oy] * wa[2][oz];
                    const int t = t0 + ox + oy * sy + oz * sz;
                    const float wv[3] = {wt * (vt[t] - cref[0]), wt * (vt[kTileNodes + t] - cref[1]),
                                         wt * (vt[2 * kTileNodes + t] - cref[2])};
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        S3[a] += wv[a];
                        if (ox) T[3 * a] += wv[a];
                        if (oy) T[3 * a + 1] += wv[a];
                        if (oz) T[3 * a + 2] += wv[a];
                    }
                }
                // sum_o w v (o - xi)^T = T - S xi^T
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    vs[a] += S3[a];
#pragma unroll
                    for (int b = 0; b < 3; ++b) Bh[3 * a + b] += T[3 * a + b] - S3[a] * xi[b];
                }
            }
            float vn[3], Bn[9], C[9];
#pragma unroll
            for (int a = 0; a < 3; ++a) vn[a] = cref[a] + 0.5f * vs[a];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                Bh[i] *= 0.5f;
                Bn[i] = Bh[i] * d.geo.dx;
            }
            // C = B D^-1 = (dx Bh)(dx^2 Dhat)^-1 = Bh Dhat^-1 / dx
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    C[3 * i + j] = d.geo.inv_dx_f * (Bh[3 * i] * Di[j] + Bh[3 * i + 1] * Di[3 + j] + Bh[3 * i + 2] * Di[6 + j]);
            // F' = (I + dt C) F  ->  H' = H + dt (C + C H)
            float Fn[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Fn[3 * i + j] = q.H[3 * i + j] +
                                    dt * (C[3 * i + j] + C[3 * i] * q.H[j] + C[3 * i + 1] * q.H[3 + j] + C[3 * i + 2] * q.H[6 + j]);
            // stress of the new state for the next step's P2G
            float tau[6];
            if (M.model == 1) dp_return_map(M, Fn, tau);
            else kirchhoff(M, Fn, tau);
            float xn[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) xn[a] = q.x[a] + dt * vn[a];
            bool finite = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) finite = finite && isfinite(vn[a]) && isfinite(xn[a]);
#pragma unroll
            for (int i = 0; i < 9; ++i) finite = finite && isfinite(Fn[i]) && isfinite(Bn[i]);
            if (!finite) set_status(d.counters, ST_NONFINITE);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                pa.out[a * S + out] = xn[a];
                pa.out[(3 + a) * S + out] = vn[a];
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                pa.out[(6 + i) * S + out] = Bn[i];
                pa.out[(15 + i) * S + out] = Fn[i];
            }
#pragma unroll
            for (int i = 0; i < 6; ++i) d.tau[i * d.tau_stride + out] = tau[i];
            if (pa.id_out) pa.id_out[out] = pa.id_in[p];
            if (pa.mat_out) pa.mat_out[out] = pa.mat_in[p];
            // next cell key and activation stamps for the following step
            CellCoord cn;
            if (finite && cell_coord(d.geo, xn, cn)) {
                d.key[out] = cell_key(d.geo, cn);
                d.sub[out] = (uint16_t)sub_code(cn);
                const Geometry &g = d.geo;
                int *pf = stamps(d.pflag, d.nbv, E + 1);
                int *gf = stamps(d.gflag, d.nbv, E + 1);
                pf[vblock_id(g, cn.c[0] >> 2, cn.c[1] >> 2, cn.c[2] >> 2)] = E + 1;
                int lo[3], hi[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    lo[a] = min(cn.c[a], cn.bp[a]) >> 2;
                    hi[a] = (cn.c[a] + 1) >> 2;
                }
                for (int zz = lo[2]; zz <= hi[2]; ++zz)
                    for (int yy = lo[1]; yy <= hi[1]; ++yy)
                        for (int xx = lo[0]; xx <= hi[0]; ++xx) gf[vblock_id(g, xx, yy, zz)] = E + 1;
            } else {
                d.key[out] = 0xffffffffu;
                set_status(d.counters, ST_DOMAIN);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- exports
__global__ void k_grid_export(DevCtx d, float *m, float *vec) {
    const long long nx = d.geo.n[0] + 1, ny = d.geo.n[1] + 1, nz = d.geo.n[2] + 1;
    const long long nodes = nx * ny * nz;
    const int E = (int)d.counters[C_EPOCH];
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < 2 * nodes; t += (long long)gridDim.x * blockDim.x) {
        const int g = (int)(t / nodes);
        const long long r = t - g * nodes;
        const int ix = (int)(r % nx), iy = (int)((r / nx) % ny), iz = (int)(r / (nx * ny));
        const int v = vblock_id(d.geo, ix >> 2, iy >> 2, iz >> 2);
        float mm = 0.0f, a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
        if (stamps(d.gflag, d.nbv, E)[v] == E) {
            const int ph = d.page[v];
            if (ph >= 0) {
                const float *blk = d.pool + (size_t)ph * kBlockFloats + g * 256;
                const int l = (iz & 3) * 16 + (iy & 3) * 4 + (ix & 3);
                mm = blk[l];
                a0 = blk[64 + l];
                a1 = blk[128 + l];
                a2 = blk[192 + l];
            }
        }
        if (m) m[t] = mm;
        if (vec) {
            vec[3 * t] = a0;
            vec[3 * t + 1] = a1;
            vec[3 * t + 2] = a2;
        }
    }
}

__global__ void k_copy_keys(DevCtx d, uint32_t *keys, uint32_t *perm, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (keys) keys[i] = d.key[i];
        if (perm) perm[i] = d.perm[i];
    }
}

int particle_grid(const DevCtx &d) {
    const int g = d.max_blocks < 8192 ? d.max_blocks : 8192;
    return g >= 8 ? (g & ~7) : g;
}

}  // namespace

void launch_block_sort(const DevCtx &d, hipStream_t s) {
    hipLaunchKernelGGL(k_block_sort, dim3(particle_grid(d)), dim3(kThreads), 0, s, d);
}

void launch_stress(const DevCtx &d, const PartArgs &pa, hipStream_t s) {
    if (pa.n > 0) hipLaunchKernelGGL(k_stress, dim3((pa.n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, d, pa);
}

void launch_p2g(const DevCtx &d, const PartArgs &pa, float dt, hipStream_t s) {
    hipLaunchKernelGGL(k_p2g, dim3(particle_grid(d)), dim3(kP2GThreads), 0, s, d, pa, dt);
}

void launch_grid_update(const DevCtx &d, float dt, const float gravity[3], hipStream_t s) {
    hipLaunchKernelGGL(k_grid_update, dim3(d.max_blocks < 16384 ? d.max_blocks : 16384), dim3(128), 0, s, d, dt,
                       gravity[0], gravity[1], gravity[2]);
}

void launch_g2p(const DevCtx &d, const PartArgs &pa, float dt, hipStream_t s) {
    hipLaunchKernelGGL(k_g2p, dim3(particle_grid(d)), dim3(kThreads), 0, s, d, pa, dt);
}

void launch_grid_export(const DevCtx &d, float *m, float *vec, hipStream_t s) {
    hipLaunchKernelGGL(k_grid_export, dim3(4096), dim3(256), 0, s, d, m, vec);
}

void launch_copy_keys(const DevCtx &d, uint32_t *keys, uint32_t *perm, int n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_copy_keys, dim3(1024), dim3(256), 0, s, d, keys, perm, n);
}

}  // namespace ck
