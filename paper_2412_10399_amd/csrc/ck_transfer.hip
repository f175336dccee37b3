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

#include <algorithm>

namespace ck {

namespace {

__device__ __forceinline__ void block_coords(const Geometry &g, int vb, int &bx, int &by, int &bz) {
    bx = vb % g.NB[0];
    by = (vb / g.NB[0]) % g.NB[1];
    bz = vb / (g.NB[0] * g.NB[1]);
}

// Physical pool block of the 27 neighbours of block (bx,by,bz) in page table
// `table`, -1 when inactive; also copied to `keep` when given.
__device__ __forceinline__ void load_neighbours(const DevCtx &d, int table, int bx, int by, int bz, int *nbr,
                                                int first_thread = 0, int *keep = nullptr) {
    const int t = (int)threadIdx.x - first_thread;
    if (t < 0) return;
    if (t < 27) {
        const int x = bx + t % 3 - 1, y = by + (t / 3) % 3 - 1, z = bz + t / 9 - 1;
        int ph = -1;
        if (x >= 0 && y >= 0 && z >= 0 && x < d.geo.NB[0] && y < d.geo.NB[1] && z < d.geo.NB[2])
            ph = page_of(d, table)[vblock_id(d.geo, x, y, z)];
        nbr[t] = ph;
        if (keep) keep[t] = ph;
    }
}

// Stamps, for the next sort (epoch E), every distinct block among the lanes of a
// wave (vb < 0: none) as holding particles and its 3 x 3 x 3 neighbourhood as grid
// blocks, lanes 0..26 writing one neighbour each.  Called by every lane of the wave;
// particles in block order mostly share a few blocks per wave.
__device__ __forceinline__ void wave_stamp(const DevCtx &d, int vb, int E) {
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(vb, 1);
    unsigned long long lead = __ballot(vb >= 0 && (lane == 0 || prev != vb));
    const Geometry &g = d.geo;
    int *pf = stamps(d.pflag, d.nbv, E);
    int *gf = stamps(d.gflag, d.nbv, E);
    while (lead) {
        const int l = __ffsll((long long)lead) - 1;
        lead &= lead - 1;
        const int v = __shfl(vb, l);
        const int bx = v % g.NB[0], by = (v / g.NB[0]) % g.NB[1], bz = v / (g.NB[0] * g.NB[1]);
        if (lane < 27) {
            const int x = bx + lane % 3 - 1, y = by + (lane / 3) % 3 - 1, z = bz + lane / 9 - 1;
            if (x >= 0 && y >= 0 && z >= 0 && x < g.NB[0] && y < g.NB[1] && z < g.NB[2]) gf[vblock_id(g, x, y, z)] = E;
        } else if (lane == 27) {
            pf[v] = E;
        }
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

// Element i of an array whose base is uniform across the wave: 32-bit byte offset
// on a scalar base (one instruction, no 64-bit address arithmetic per access).
template <typename T>
__device__ __forceinline__ T ld_at(const T *base, uint32_t i) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (size_t)(i * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st_at(T *base, uint32_t i, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (size_t)(i * (uint32_t)sizeof(T))) = v;
}

// Element i of N consecutive planes of `stride` elements from plane `first`: one
// per-lane address advanced by the stride, instead of one wave-uniform base per
// plane (a kernel storing some thirty planes otherwise keeps thirty 64-bit bases in
// scalar registers, and the ones that do not fit cost two lane reads per access).
typedef __attribute__((address_space(1))) float global_float;
template <int N>
__device__ __forceinline__ void st_planes(float *base, long long stride, int first, uint32_t i, const float (&v)[N]) {
    uint64_t a = reinterpret_cast<uint64_t>(base + (long long)first * stride + i);
    const uint64_t step = (uint64_t)stride * sizeof(float);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        *reinterpret_cast<global_float *>(a) = v[k];
        a += step;
        asm volatile("" : "+v"(a));   // keep the address per lane
    }
}
typedef const __attribute__((address_space(1))) float global_cfloat;
template <int N>
__device__ __forceinline__ void ld_planes(const float *base, long long stride, int first, uint32_t i, float (&v)[N]) {
    uint64_t a = reinterpret_cast<uint64_t>(base + (long long)first * stride + i);
    const uint64_t step = (uint64_t)stride * sizeof(float);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        v[k] = *reinterpret_cast<global_cfloat *>(a);
        a += step;
        asm volatile("" : "+v"(a));
    }
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
// Also adds the P2G contribution bound of the state to the bound slots.
__device__ __forceinline__ void b_stress(const DevCtx &d, const PartArgs &pa) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    float X = 0.0f, Y = 0.0f;
    if (p < pa.n) {
        const long long S = pa.stride;
        float H[9], v[3], B[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) H[a] = pa.in[(kPlaneH + a) * S + p];
#pragma unroll
        for (int a = 0; a < 3; ++a) v[a] = pa.in[(kPlaneV + a) * S + p];
#pragma unroll
        for (int a = 0; a < 9; ++a) B[a] = pa.in[(kPlaneB + a) * S + p];
        const int mi = pa.mat_in ? (int)pa.mat_in[p] : 0;
        const DevMaterial M = material_of(d, mi);
        float tau[6];
        kirchhoff(M, H, tau);
#pragma unroll
        for (int i = 0; i < 6; ++i) d.tau[i * d.tau_stride + p] = tau[i];
        contribution_bound_xy(M.mass, M.vol0, d.geo.inv_dx_f, v, B, tau, X, Y);
    }
    wave_bound(d.bslots, (int)blockIdx.x, X, Y);
}

__global__ void __launch_bounds__(kThreads) k_stress(DevCtx d, PartArgs pa) { b_stress(d, pa); }

// one launch for many jobs: workgroup row y runs job y
__global__ void __launch_bounds__(kThreads) k_stress_multi(const JobStep *__restrict__ jobs) {
    const JobStep &J = jobs[blockIdx.y];
    if (!J.first && !J.d.det) return;
    b_stress(J.d, J.pa);
}

// ---------------------------------------------------------------- P2G
// Particle contributions (section 4.4 APIC transfer plus the MLS stress impulse of
// section 4.5): mass w m_p and momentum w (m_p v_p + Q (x_i - x_p)) with
//   Q = (m_p B_p - dt V_p^0 tau_p) D_p^-1,
// where grad Phi_i = w D^-1 (x_i - x_p) and f_i = -V^0 tau grad Phi_i.  In cell units,
// with xi the particle's fractional position in its G- cell c, G- node c + o
// (o in {0,1}^3) sits at x_i - x_p = dx (o - xi) and G+ node bp + o at
// dx (o + bp - c + 1/2 - xi), G+ being shifted half a cell from G-.  With
// base = m_p v_p - Q xi the momenta are base + Q o and base + Q (o + bp - c + 1/2).
//
// One workgroup per block, one thread per particle, and the block's 341-node tile
// in LDS as 64-bit fixed-point integers: LDS float atomics run about 26 times slower
// than 64-bit integer atomics on gfx950, and integer sums are exact, so the tile is
// independent of the order of the additions.  A block is scattered in passes of at
// most kChunk particles, each pass into a cleared tile with its own unit: 2^-39 of
// the pass's largest contribution bound, so every contribution is below 2^40 units
// and a node, which takes at most one contribution per particle, sums fewer than
// kChunk * 2^40 = 2^49 units in a pass -- below 2^51, where the magic-number
// conversion through FP64 stays exact.  Particles are ordered in layers: layer q holds the q-th particle
// (by index) of every nonempty (half-cell octant, cell) bin, and each layer runs in
// (octant, cell) order.  Within an octant distinct cells have distinct nodes on both
// grids, and spreading each bin's particles over the layers keeps most lanes of one
// atomic instruction off each other's nodes.  The tile is then converted back and
// each nonzero node is added to the pool with one global float atomic.
constexpr int kP2GThreads = 256;
constexpr int kBins = 512;                 // (octant, cell) bins of a block: octant * 64 + cell
constexpr int kPerThread = kMaxBlockParticles / kP2GThreads;   // bucket entries per thread
constexpr int kHold = 2;                   // of which kept in registers
constexpr int kChunk = 2 * kP2GThreads;    // particles scattered per pass (two per thread)
// a pass's node sums (< kChunk * 2^40 units) must stay below 2^51 for to_fixed and the
// conversion back through FP64 to be exact
static_assert((double)kChunk * 1099511627776.0 < 2251799813685248.0, "fixed-point tile sums would overflow 2^51");
// the step-global unit scatters a whole block in one pass: its node sums stay below
// kMaxBlockParticles * 2^40 units, which must not exceed 2^51 either
static_assert((double)kMaxBlockParticles * 1099511627776.0 <= 2251799813685248.0,
              "fixed-point tile sums with the step-global unit would overflow 2^51");
// Padded tile layout (64-bit words): node (x, y, z) of a grid at x + kTY y + kTZ z.
// For any node offset, the 4 x 4 x 4 cells of a block then map x + kTY y + kTZ z
// onto every residue modulo 32 exactly twice (and modulo 16 exactly four times), so
// the 64 lanes of one atomic whose particles lie in distinct cells spread evenly over
// the LDS banks; among the strides with that property these give the smallest tile
// (189 and 236 words per channel for the 125 and 216 nodes).
constexpr int kTY = 6, kTZ = 40;
constexpr int kTileMStride = 4 * kTZ + 5 * kTY;   // words per channel, G- ([0,4]^3)
constexpr int kTilePStride = 5 * kTZ + 6 * kTY;   // words per channel, G+ ([0,5]^3)
constexpr double kMagic = 6755399441055744.0;                  // 1.5 * 2^52
constexpr long long kMagicBits = 0x4338000000000000LL;

__device__ __forceinline__ int bin_of(uint32_t sub) { return (int)((sub & 7u) * 64u + (sub >> 3)); }

// v * S rounded to an integer, |v S| < 2^51: in the binade [2^52, 2^53) FP64 numbers
// are the integers, so the bit pattern of magic + v S is that of magic plus v S.
__device__ __forceinline__ unsigned long long to_fixed(float v, double S) {
    const double d = fma((double)v, S, kMagic);
    return (unsigned long long)(__double_as_longlong(d) - kMagicBits);
}

struct Staged {
    float xm[3], sp[3], mass, base[3], Q[9];
    int c[3];       // G- cell
    int oct;        // half-cell octant
    bool on;        // takes part in the scatter
};

// P2G record of a particle at cell coordinates cc with velocity v, affine matrix B
// and Kirchhoff stress tau (6 values).
__device__ __forceinline__ void stage_compute(const DevCtx &d, const DevMaterial &M, const CellCoord &cc,
                                              const float (&v)[3], const float (&B)[9], const float (&tau)[6], float dt,
                                              Staged &r) {
    const uint32_t code = sub_code(cc);
    r.oct = (int)(code & 7u);
#pragma unroll
    for (int a = 0; a < 3; ++a) r.c[a] = cc.c[a];
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
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r.Q[3 * i + j] = sc * (A[3 * i] * Di[j] + A[3 * i + 1] * Di[3 + j] + A[3 * i + 2] * Di[6 + j]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.xm[a] = cc.xm[a];
        r.sp[a] = w.sp[a];
        r.base[a] = M.mass * v[a] - (r.Q[3 * a] * cc.xm[0] + r.Q[3 * a + 1] * cc.xm[1] + r.Q[3 * a + 2] * cc.xm[2]);
    }
    r.mass = M.mass;
    r.on = true;
}

// P2G record of a particle whose B planes carry Q itself (the state an mpm_step G2P
// left for the next step): only the weights and base = m v - Q xi remain to form.
__device__ __forceinline__ void stage_compute_q(const DevMaterial &M, const CellCoord &cc, const float (&v)[3],
                                                const float (&Q)[9], Staged &r) {
    const uint32_t code = sub_code(cc);
    r.oct = (int)(code & 7u);
    Weights w;
    axis_weights(cc, w);
#pragma unroll
    for (int a = 0; a < 3; ++a) r.c[a] = cc.c[a];
#pragma unroll
    for (int i = 0; i < 9; ++i) r.Q[i] = Q[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.xm[a] = cc.xm[a];
        r.sp[a] = w.sp[a];
        r.base[a] = M.mass * v[a] - (Q[3 * a] * cc.xm[0] + Q[3 * a + 1] * cc.xm[1] + Q[3 * a + 2] * cc.xm[2]);
    }
    r.mass = M.mass;
    r.on = true;
}

// kCarried: the B planes of the input hold Q (and there is no carried stress), and
// the first remainder plane the packed remainder.
template <bool kCarried = false>
__device__ __forceinline__ void stage_particle(const DevCtx &d, const PartArgs &pa, int p, int bx, int by, int bz,
                                               float dt, Staged &r) {
    r.on = false;
    const long long S = pa.stride;
    const uint32_t up = (uint32_t)p;
    float x[3], xr[3], v[3], B[9], tau[6];
    ld_planes(pa.in, S, kPlaneX, up, x);
    if (kCarried) unpack_remainder(d.geo, ld_at(reinterpret_cast<const uint32_t *>(pa.in + kPlaneR * S), up), xr);
    else ld_planes(pa.in, S, kPlaneR, up, xr);
    ld_planes(pa.in, S, kPlaneV, up, v);
    ld_planes(pa.in, S, kPlaneB, up, B);
    if (!kCarried) ld_planes(d.tau, d.tau_stride, 0, up, tau);
    const int mi = pa.mat_in ? (int)ld_at(pa.mat_in, up) : 0;
    const DevMaterial M = material_of(d, mi);
    CellCoord cc;
    if (!cell_coord(d.geo, x, xr, cc)) {
        set_status(d.counters, ST_DOMAIN);
        return;
    }
    if ((cc.c[0] >> 2) != bx || (cc.c[1] >> 2) != by || (cc.c[2] >> 2) != bz) {
        set_status(d.counters, ST_STALE);
        return;
    }
    if (kCarried) stage_compute_q(M, cc, v, B, r);
    else stage_compute(d, M, cc, v, B, tau, dt, r);
}

// Upper bound of |w m| and |w (base + Q t)| over the particle's 16 nodes (w <= 1,
// every component of t in [-1/2, 3/2]).
__device__ __forceinline__ float contribution_bound(const Staged &r) {
    if (!r.on) return 0.0f;
    float b = r.mass;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        b = fmaxf(b, fabsf(r.base[a]) + 1.5f * (fabsf(r.Q[3 * a]) + fabsf(r.Q[3 * a + 1]) + fabsf(r.Q[3 * a + 2])));
    return b;
}

// Adds the particle's 8 contributions on one grid: nodes t0 + o (tile index steps
// sy, sz), weights w[a][o_a], momentum m0 + Q o.
__device__ __forceinline__ void scatter_grid(unsigned long long *tile, int ntile, int t0, int sy, int sz,
                                             const float (&w)[3][2], float mass, const float (&m0)[3],
                                             const float (&Q)[9], double S) {
    float mo[2][2][2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mo[0][0][0][a] = m0[a];
        mo[0][0][1][a] = m0[a] + Q[3 * a];
        mo[0][1][0][a] = m0[a] + Q[3 * a + 1];
        mo[0][1][1][a] = mo[0][0][1][a] + Q[3 * a + 1];
#pragma unroll
        for (int oy = 0; oy < 2; ++oy)
#pragma unroll
            for (int ox = 0; ox < 2; ++ox) mo[1][oy][ox][a] = mo[0][oy][ox][a] + Q[3 * a + 2];
    }
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy) {
            const float wyz = w[1][oy] * w[2][oz];
#pragma unroll
            for (int ox = 0; ox < 2; ++ox) {
                const float wt = w[0][ox] * wyz;
                const int t = t0 + ox + oy * sy + oz * sz;
                atomicAdd(&tile[t], to_fixed(wt * mass, S));
#pragma unroll
                for (int a = 0; a < 3; ++a) atomicAdd(&tile[(1 + a) * ntile + t], to_fixed(wt * mo[oz][oy][ox][a], S));
            }
        }
}

// Per-axis weights of a staged particle on both grids, the G+ base offset up (the
// G+ base node is c + up - 1) and the G+ momentum at that base node.
__device__ __forceinline__ void staged_weights(const Staged &r, float (&wm)[3][2], float (&wp)[3][2], int (&up)[3],
                                               float (&mp)[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        up[a] = (r.oct >> a) & 1;
        wm[a][0] = 1.0f - r.xm[a] - r.sp[a];
        wm[a][1] = r.xm[a] + r.sp[a];
        const float xp = up[a] ? r.xm[a] - 0.5f : r.xm[a] + 0.5f;
        wp[a][0] = 1.0f - xp + r.sp[a];
        wp[a][1] = xp - r.sp[a];
    }
    // base + Q (up - 1/2)
#pragma unroll
    for (int a = 0; a < 3; ++a)
        mp[a] = r.base[a] + ((float)up[0] - 0.5f) * r.Q[3 * a] + ((float)up[1] - 0.5f) * r.Q[3 * a + 1] +
                ((float)up[2] - 0.5f) * r.Q[3 * a + 2];
}

// Scatter into a fixed-point tile whose G- nodes start one node below the G+ origin
// offset: G- cell c at tile coordinates l, G+ base node at l + up.
template <int TY, int TZ, int SM, int SP>
__device__ __forceinline__ void scatter_particle(const Staged &r, int lx, int ly, int lz, unsigned long long *tile_m,
                                                 unsigned long long *tile_p, double S) {
    float wm[3][2], wp[3][2], mp[3];
    int up[3];
    staged_weights(r, wm, wp, up, mp);
    scatter_grid(tile_m, SM, lz * TZ + ly * TY + lx, TY, TZ, wm, r.mass, r.base, r.Q, S);
    scatter_grid(tile_p, SP, (lz + up[2]) * TZ + (ly + up[1]) * TY + (lx + up[0]), TY, TZ, wp, r.mass, mp, r.Q, S);
}

// FP64 form of scatter_grid: each contribution is the exact FP64 product of the
// FP32 weight and the FP32 mass or momentum term, added with an FP64 LDS atomic
// (as fast as the 64-bit integer add on gfx950, with no conversion to fixed point).
__device__ __forceinline__ void scatter_grid_f64(double *tile, int ntile, int t0, int sy, int sz,
                                                 const float (&w)[3][2], double mass, const float (&m0)[3],
                                                 const float (&Q)[9]) {
    float mo[2][2][2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mo[0][0][0][a] = m0[a];
        mo[0][0][1][a] = m0[a] + Q[3 * a];
        mo[0][1][0][a] = m0[a] + Q[3 * a + 1];
        mo[0][1][1][a] = mo[0][0][1][a] + Q[3 * a + 1];
#pragma unroll
        for (int oy = 0; oy < 2; ++oy)
#pragma unroll
            for (int ox = 0; ox < 2; ++ox) mo[1][oy][ox][a] = mo[0][oy][ox][a] + Q[3 * a + 2];
    }
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy) {
            const float wyz = w[1][oy] * w[2][oz];
#pragma unroll
            for (int ox = 0; ox < 2; ++ox) {
                const double wt = (double)(w[0][ox] * wyz);
                const int t = t0 + ox + oy * sy + oz * sz;
                atomicAdd(&tile[t], wt * mass);
#pragma unroll
                for (int a = 0; a < 3; ++a) atomicAdd(&tile[(1 + a) * ntile + t], wt * (double)mo[oz][oy][ox][a]);
            }
        }
}

// scatter_grid with FP64 products: each contribution is the exact FP64 product of the
// FP32 weight and the FP32 mass or momentum term, rounded once to the fixed-point unit
// 1/S (|product| S < 2^51) and added as a 64-bit integer.
__device__ __forceinline__ void scatter_grid_unit(unsigned long long *tile, int ntile, int t0, int sy, int sz,
                                                  const float (&w)[3][2], double mS, const float (&m0)[3],
                                                  const float (&Q)[9], double S) {
    float mo[2][2][2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mo[0][0][0][a] = m0[a];
        mo[0][0][1][a] = m0[a] + Q[3 * a];
        mo[0][1][0][a] = m0[a] + Q[3 * a + 1];
        mo[0][1][1][a] = mo[0][0][1][a] + Q[3 * a + 1];
#pragma unroll
        for (int oy = 0; oy < 2; ++oy)
#pragma unroll
            for (int ox = 0; ox < 2; ++ox) mo[1][oy][ox][a] = mo[0][oy][ox][a] + Q[3 * a + 2];
    }
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy) {
            const float wyz = w[1][oy] * w[2][oz];
#pragma unroll
            for (int ox = 0; ox < 2; ++ox) {
                const double wt = (double)(w[0][ox] * wyz);
                const double wS = wt * S;
                const int t = t0 + ox + oy * sy + oz * sz;
                atomicAdd(&tile[t], (unsigned long long)(__double_as_longlong(fma(wt, mS, kMagic)) - kMagicBits));
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    atomicAdd(&tile[(1 + a) * ntile + t],
                              (unsigned long long)(__double_as_longlong(fma((double)mo[oz][oy][ox][a], wS, kMagic)) -
                                                   kMagicBits));
            }
        }
}

template <int TY, int TZ, int SM, int SP>
__device__ __forceinline__ void scatter_particle_unit(const Staged &r, int lx, int ly, int lz, unsigned long long *tile_m,
                                                      unsigned long long *tile_p, double S) {
    float wm[3][2], wp[3][2], mp[3];
    int up[3];
    staged_weights(r, wm, wp, up, mp);
    const double mS = (double)r.mass * S;
    scatter_grid_unit(tile_m, SM, lz * TZ + ly * TY + lx, TY, TZ, wm, mS, r.base, r.Q, S);
    scatter_grid_unit(tile_p, SP, (lz + up[2]) * TZ + (ly + up[1]) * TY + (lx + up[0]), TY, TZ, wp, mS, mp, r.Q, S);
}

template <int TY, int TZ, int SM, int SP>
__device__ __forceinline__ void scatter_particle_f64(const Staged &r, int lx, int ly, int lz, double *tile_m,
                                                     double *tile_p) {
    float wm[3][2], wp[3][2], mp[3];
    int up[3];
    staged_weights(r, wm, wp, up, mp);
    const double mass = (double)r.mass;
    scatter_grid_f64(tile_m, SM, lz * TZ + ly * TY + lx, TY, TZ, wm, mass, r.base, r.Q);
    scatter_grid_f64(tile_p, SP, (lz + up[2]) * TZ + (ly + up[1]) * TY + (lx + up[0]), TY, TZ, wp, mass, mp, r.Q);
}

// Direct float atomics into the pool for a particle outside the workgroup's tile
// (moved more than one cell in a fused step); nbr holds the pool blocks around
// block (bx,by,bz).
__device__ __forceinline__ void scatter_pool(const DevCtx &d, float *pool, const int *nbr, int bx, int by, int bz,
                                             const Staged &r) {
    float wm[3][2], wp[3][2], mp[3];
    int up[3];
    staged_weights(r, wm, wp, up, mp);
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const float(*w)[2] = g == 0 ? wm : wp;
        const float *m0 = g == 0 ? r.base : mp;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
            const int ix = r.c[0] + (g ? up[0] - 1 : 0) + ox, iy = r.c[1] + (g ? up[1] - 1 : 0) + oy,
                      iz = r.c[2] + (g ? up[2] - 1 : 0) + oz;
            // nbr covers blocks bx-1 .. bx+1: a node outside them is out of reach
            const bool near = (unsigned)((ix >> 2) - bx + 1) <= 2u && (unsigned)((iy >> 2) - by + 1) <= 2u &&
                              (unsigned)((iz >> 2) - bz + 1) <= 2u;
            const long long a = near ? pool_index(d, nbr, bx, by, bz, g, ix, iy, iz, 0) : -1;
            if (a < 0) {
                set_status(d.counters, ST_CFL);
                continue;
            }
            const float wt = w[0][ox] * w[1][oy] * w[2][oz];
            atomicAdd(&pool[a], wt * r.mass);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                atomicAdd(&pool[a + (1 + c) * 64], wt * (m0[c] + ox * r.Q[3 * c] + oy * r.Q[3 * c + 1] + oz * r.Q[3 * c + 2]));
        }
    }
}

// Layered block order: the q-th particles (by index) of all nonempty (octant, cell)
// bins form layer q, and the block is ordered by (layer, octant, cell).  The 64 lanes
// of a wave then mostly hold particles of distinct bins, where the (octant, cell,
// index) order puts every particle of a bin into the same wave, so one scatter
// instruction hits fewer equal LDS addresses.  Bins of more than kLayers particles
// (dense blocks) keep the (octant, cell, index) order.
constexpr int kLayers = 16;
constexpr int kLayWords = 2 * kLayers * (kP2GThreads / 64) + kP2GThreads / 64;   // LDS ints of the layer tables
// per (layer, wave range): the ballots of its bins holding more than q particles,
// even and odd bins (64-bit words)
constexpr int kLayMaskWords = 2 * kLayers * (kP2GThreads / 64);
// 64-bit words of the ordering buffer, which shares a kernel's LDS area with its
// fixed-point tile
constexpr int kOrderWords = kMaxBlockParticles * 4 / 8;

// Orders the particles of block r (count cnt, first sorted position s) by (half-cell
// octant, cell, index), or in the layered order when `layered`: ord[j] = particle
// index at position j of the block, also written to the global permutation.  Uses
// bcnt, bstart, wsum and lbuf (LDS); the layered order also uses lay (kLayWords ints)
// and lmask (kLayMaskWords 64-bit words).
template <bool layered = false>
__device__ __forceinline__ void order_block(const DevCtx &d, int r, int s, int cnt, int *bcnt, int *bstart, int *wsum,
                                            uint32_t *lbuf, uint32_t *ord, int *lay = nullptr,
                                            unsigned long long *lmask = nullptr) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const uint32_t *bkt = d.bucket + (size_t)r * kMaxBlockParticles;
    const uint16_t *bsb = d.bsub + (size_t)r * kMaxBlockParticles;
    for (int b = tid; b < kBins; b += kP2GThreads) bcnt[b] = 0;
    lds_barrier();
    uint32_t hidx[kHold];
    int hbin[kHold];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int j = tid + k * kP2GThreads;
        if (j >= cnt) break;
        const uint32_t idx = bkt[j];
        const int bin = bin_of(bsb[j]);
        if (k < kHold) {
            hidx[k] = idx;
            hbin[k] = bin;
        }
        atomicAdd(&bcnt[bin], 1);
    }
    lds_barrier();
    {
        // exclusive scan of the 512 bins, two per thread
        const int c0 = bcnt[2 * tid], c1 = bcnt[2 * tid + 1];
        int v = c0 + c1;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(v, off);
            if (lane >= off) v += t;
        }
        if (lane == 63) wsum[w] = v;
        int mx = 0;
        if (layered) {
            mx = max(c0, c1);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off));
            if (lane == 0) lay[2 * kLayers * 4 + w] = mx;
        }
        lds_barrier();
        int pre = 0;
        for (int k = 0; k < w; ++k) pre += wsum[k];
        const int ex = pre + v - c0 - c1;
        bstart[2 * tid] = ex;
        bstart[2 * tid + 1] = ex + c0;
        bcnt[2 * tid] = ex;
        bcnt[2 * tid + 1] = ex + c0;
        if (tid == kP2GThreads - 1) bstart[kBins] = ex + c0 + c1;
        if (layered) {
            // largest bin of the block; layer tables when every bin fits kLayers layers:
            // the ballots of the wave's even and odd bins holding more than q particles
            // (lane l holds bins 2l and 2l + 1 of the wave's 128), and lay[q * 4 + w] =
            // the number of such bins in wave w's range
            mx = max(max(lay[2 * kLayers * 4], lay[2 * kLayers * 4 + 1]),
                     max(lay[2 * kLayers * 4 + 2], lay[2 * kLayers * 4 + 3]));
            if (mx <= kLayers) {
                for (int q = 0; q < mx; ++q) {
                    const unsigned long long m0 = __ballot(c0 > q), m1 = __ballot(c1 > q);
                    if (lane == 0) {
                        lmask[2 * (q * 4 + w)] = m0;
                        lmask[2 * (q * 4 + w) + 1] = m1;
                        lay[q * 4 + w] = __popcll(m0) + __popcll(m1);
                    }
                }
            }
        }
    }
    lds_barrier();
    bool lay_on = false;
    if (layered) {
        const int mx = max(max(lay[2 * kLayers * 4], lay[2 * kLayers * 4 + 1]),
                           max(lay[2 * kLayers * 4 + 2], lay[2 * kLayers * 4 + 3]));
        lay_on = mx <= kLayers;
        // first position of (layer q, wave range w): exclusive scan over (q, w) in order
        if (lay_on && tid < 64) {
            const int e = tid < mx * 4 ? lay[tid] : 0;
            int v = e;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(v, off);
                if (lane >= off) v += t;
            }
            lay[kLayers * 4 + tid] = v - e;
        }
    }
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int j = tid + k * kP2GThreads;
        if (j >= cnt) break;
        uint32_t idx;
        int bin;
        if (k < kHold) {
            idx = hidx[k];
            bin = hbin[k];
        } else {
            idx = bkt[j];
            bin = bin_of(bsb[j]);
        }
        lbuf[atomicAdd(&bcnt[bin], 1)] = idx;
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int j = tid + k * kP2GThreads;
        if (j >= cnt) break;
        uint32_t idx;
        int bin;
        if (k < kHold) {
            idx = hidx[k];
            bin = hbin[k];
        } else {
            idx = bkt[j];
            bin = bin_of(bsb[j]);
        }
        const int lo = bstart[bin], hi = bstart[bin + 1];
        int rank = lo;
        for (int q = lo; q < hi; ++q) rank += (lbuf[q] < idx) ? 1 : 0;
        if (lay_on) {
            // within layer q and the bin's wave range: the bins before it holding more
            // than q particles
            const int q = rank - lo, wr = bin >> 7, l = (bin & 127) >> 1;
            const unsigned long long m0 = lmask[2 * (q * 4 + wr)], m1 = lmask[2 * (q * 4 + wr) + 1];
            const unsigned long long lt = (1ull << l) - 1ull;
            int pq = __popcll(m0 & lt) + __popcll(m1 & lt);
            if (bin & 1) pq += (int)((m0 >> l) & 1ull);
            rank = lay[kLayers * 4 + q * 4 + wr] + pq;
        }
        ord[rank] = idx;
        st_at(d.perm, (uint32_t)(s + rank), idx);
    }
}

// The block's order kept from the previous step: when the previous G2P changed neither
// the set nor the (octant, cell) bins of the block's particles, they sit at consecutive
// positions in the layered order of the same bins, which this step's order would
// reproduce exactly (ranks within a bin follow the positions).  The sort then records
// the block's smallest and largest position instead of filling its bucket; when they
// span exactly cnt positions the block order is that range (ord and the global
// permutation are written).  Otherwise -- which a correct change record excludes --
// the status reports a stale state and false is returned: the block's bucket is empty.
__device__ __forceinline__ bool kept_block_order(const DevCtx &d, int r, int s, int cnt, uint32_t *ord) {
    const uint32_t lo = d.blo[r], hi = d.bhi[r];
    if (cnt <= 0 || hi < lo || hi - lo + 1u != (uint32_t)cnt) {
        set_status(d.counters, ST_STALE);
        return false;
    }
    for (int j = threadIdx.x; j < cnt; j += kP2GThreads) {
        ord[j] = lo + (uint32_t)j;
        st_at(d.perm, (uint32_t)(s + j), lo + (uint32_t)j);
    }
    return true;
}

// Reduces a per-thread contribution bound over the workgroup (bmax in LDS, reset by
// the caller before the preceding barrier) and returns the fixed-point scale.
__device__ __forceinline__ double block_scale(float bnd, unsigned int *bmax) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) bnd = fmaxf(bnd, __shfl_xor(bnd, off));
    if ((threadIdx.x & 63) == 0) atomicMax(bmax, __float_as_uint(bnd));
    lds_barrier();
    const float m = __uint_as_float(*bmax);
    return m > 0.0f ? ldexp(1.0, 39 - ilogbf(m)) : 1.0;
}

// P2G of the particle blocks.  kFixed (deterministic mode): the fixed-point tile,
// whose sums are exact and so independent of the order of the atomics; each pass
// stages two particles per thread, takes the block's unit from their bounds, then
// scatters them.  Otherwise an FP64 tile: every thread stages and scatters one
// particle at a time (no unit to agree on first), and the block takes a single pass.
// reuse: the input is the state the context's previous G2P wrote, so that the order
// of a block that G2P left unchanged is kept (kept_block_order).
template <bool kFixed, bool kCarried = false>
__device__ __forceinline__ void b_p2g(const DevCtx &d, const PartArgs &pa, float dt, int gp, int gt, bool reuse) {
    __shared__ int bcnt[kBins];                 // counts, then placement cursors
    __shared__ int bstart[kBins + 1];
    __shared__ int wsum[kP2GThreads / 64];
    __shared__ unsigned int bmax;
    __shared__ int nbr[27];
    __shared__ uint32_t ord[kMaxBlockParticles];   // particle index at each position of the block order
    // ordering buffer, then the fixed-point tile [4][G-] and [4][G+]
    constexpr int kTileWords = 4 * (kTileMStride + kTilePStride);
    constexpr int kAreaWords = kTileWords > kOrderWords ? kTileWords : kOrderWords;
    __shared__ unsigned long long area[kAreaWords];
    __shared__ int lay[kLayWords];
    __shared__ unsigned long long lmask[kLayMaskWords];
    uint32_t *lbuf = reinterpret_cast<uint32_t *>(area);
    unsigned long long *tile_m = area;
    unsigned long long *tile_p = area + 4 * kTileMStride;
    const int np = (int)d.counters[C_NPB];
    const int E = (int)d.counters[C_EPOCH];
    const int tid = threadIdx.x;
    // step-global fixed-point unit (plain mode): 2^(e-39) for the contribution bound in
    // [2^e, 2^(e+1)), so that every contribution is below 2^40 units and a node's sum
    // over the at most kMaxBlockParticles particles of a block below 2^51
    const float bound = __uint_as_float(d.counters[C_BOUND_X]) + dt * __uint_as_float(d.counters[C_BOUND_Y]);
    const double S = (bound > 0.0f && bound <= 3.0e38f) ? ldexp(1.0, 39 - ilogbf(bound)) : 1.0;
    const double inv_unit = 1.0 / S;
    float seen = 0.0f;   // largest contribution bound of this thread's particles
    for (int base = 0; base < np; base += gridDim.x) {
        const int r = round_block(base, np);
        if (r < 0) continue;
        const int vb = d.plist[r];
        int bx, by, bz;
        block_coords(d.geo, vb, bx, by, bz);
        // the neighbourhood loads while the block is ordered (the ordering's barriers
        // publish it; the previous block's last reader passed the barrier that ends
        // its iteration), and is kept for this step's G2P, for every block G2P visits
        load_neighbours(d, gt, bx, by, bz, nbr, 0, d.nbrs + 27 * (size_t)r);
        const int s = d.pstart[r];
        const int cnt = d.pstart[r + 1] - s;
        if (cnt > kMaxBlockParticles) continue;   // reported by the bucket scan
        if (reuse && d.bchg[vb] != E) {
            if (!kept_block_order(d, r, s, cnt, ord)) continue;
        } else {
            order_block<true>(d, r, s, cnt, bcnt, bstart, wsum, lbuf, ord, lay, lmask);
        }
        lds_barrier();

        if (!kFixed) {
            // ---- fixed-point tile with the step-global unit: the bound the preceding G2P
            // (or stress pass) formed over every particle of the state, so that every
            // thread stages and scatters one particle at a time (the first one loads while
            // the tile is cleared).  A particle above the bound (a state changed in place
            // without mpm_invalidate) adds to the pool with float atomics instead.
            Staged st;
            st.on = false;
            if (tid < cnt) stage_particle<kCarried>(d, pa, (int)ord[tid], bx, by, bz, dt, st);
            for (int q = tid; q < kTileWords; q += kP2GThreads) area[q] = 0ull;
            lds_barrier();
            for (int j = tid; j < cnt; j += kP2GThreads) {
                if (j > tid) stage_particle<kCarried>(d, pa, (int)ord[j], bx, by, bz, dt, st);
                if (!st.on) continue;
                const float cb = contribution_bound(st);
                seen = fmaxf(seen, cb);
                if (cb <= bound)
                    scatter_particle_unit<kTY, kTZ, kTileMStride, kTilePStride>(
                        st, st.c[0] - 4 * bx, st.c[1] - 4 * by, st.c[2] - 4 * bz, tile_m, tile_p, S);
                else
                    scatter_pool(d, pool_of(d, gp), nbr, bx, by, bz, st);
            }
            lds_barrier();
            for (int ni = tid; ni < kTileNodes; ni += kP2GThreads) {
                int g, ix, iy, iz;
                tile_node(ni, bx, by, bz, g, ix, iy, iz);
                const int lx = ix - 4 * bx + g, ly = iy - 4 * by + g, lz = iz - 4 * bz + g;   // tile-local
                const unsigned long long *tb = g == 0 ? tile_m : tile_p;
                const int cs = g == 0 ? kTileMStride : kTilePStride;
                const int t = lx + ly * kTY + lz * kTZ;
                float val[4];
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) val[ch] = (float)((double)(long long)tb[ch * cs + t] * inv_unit);
                if (val[0] == 0.0f && val[1] == 0.0f && val[2] == 0.0f && val[3] == 0.0f) continue;
                const long long a = pool_index(d, nbr, bx, by, bz, g, ix, iy, iz, 0);
                if (a < 0) {
                    set_status(d.counters, ST_CAPACITY);
                    continue;
                }
#pragma unroll
                for (int ch = 0; ch < 4; ++ch)
                    if (val[ch] != 0.0f) atomicAdd(&pool_of(d, gp)[a + ch * 64], val[ch]);
            }
            lds_barrier();
            continue;
        }

        // ---- fixed-point tile, kChunk particles per pass (one pass unless the block is dense)
        // (in deterministic mode a block without valid particles still writes a zero tile)
        const int cend = (d.det && cnt == 0) ? 1 : cnt;
        for (int c0 = 0; c0 < cend; c0 += kChunk) {
            for (int q = tid; q < kTileWords; q += kP2GThreads) area[q] = 0ull;
            if (tid == 0) bmax = 0u;
            Staged st[2];
            float bnd = 0.0f;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                st[k].on = false;
                const int j = c0 + tid + k * kP2GThreads;
                if (j < cnt) stage_particle(d, pa, (int)ord[j], bx, by, bz, dt, st[k]);
                bnd = fmaxf(bnd, contribution_bound(st[k]));
            }
            lds_barrier();   // tile cleared, bmax reset
            const double S = block_scale(bnd, &bmax);
#pragma unroll
            for (int k = 0; k < 2; ++k)
                if (st[k].on)
                    scatter_particle<kTY, kTZ, kTileMStride, kTilePStride>(st[k], st[k].c[0] - 4 * bx, st[k].c[1] - 4 * by,
                                                                           st[k].c[2] - 4 * bz, tile_m, tile_p, S);
            lds_barrier();
            // ---- flush every nonzero tile node to the pool
            const double inv = 1.0 / S;
            for (int ni = tid; ni < kTileNodes; ni += kP2GThreads) {
                int g, ix, iy, iz;
                tile_node(ni, bx, by, bz, g, ix, iy, iz);
                const int lx = ix - 4 * bx + g, ly = iy - 4 * by + g, lz = iz - 4 * bz + g;   // tile-local
                const unsigned long long *tb = g == 0 ? tile_m : tile_p;
                const int cs = g == 0 ? kTileMStride : kTilePStride;
                const int t = lx + ly * kTY + lz * kTZ;
                float val[4];
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) val[ch] = (float)((double)(long long)tb[ch * cs + t] * inv);
                if (d.det) {
                    // deterministic mode: the block's tile (the same thread owns node ni in
                    // every pass, so later passes add to what it wrote before)
                    float *sg = d.stage + (size_t)r * kStageFloats + ni;
#pragma unroll
                    for (int ch = 0; ch < 4; ++ch)
                        sg[ch * kTileNodes] = c0 == 0 ? val[ch] : sg[ch * kTileNodes] + val[ch];
                    continue;
                }
                if (val[0] == 0.0f && val[1] == 0.0f && val[2] == 0.0f && val[3] == 0.0f) continue;
                const long long a = pool_index(d, nbr, bx, by, bz, g, ix, iy, iz, 0);
                if (a < 0) {
                    set_status(d.counters, ST_CAPACITY);
                    continue;
                }
#pragma unroll
                for (int ch = 0; ch < 4; ++ch)
                    if (val[ch] != 0.0f) atomicAdd(&pool_of(d, gp)[a + ch * 64], val[ch]);
            }
            lds_barrier();
        }
    }
    // the next step's unit: kBoundHeadroom times the largest contribution bound of this
    // step (contributions change little from one step to the next; a particle beyond
    // the headroom takes the float-atomic path)
    if (!kFixed) wave_bound(d.bslots, (int)blockIdx.x, kBoundHeadroom * seen, 0.0f);
}

// Four waves per SIMD (128 VGPRs, none spilled; 40 KiB of LDS, four workgroups per
// CU): 0.263 ms on the sand column against 0.303 ms at three.
__global__ void __launch_bounds__(kP2GThreads, 4) k_p2g(DevCtx d, PartArgs pa, float dt, int gp, int gt, int reuse) {
    b_p2g<false>(d, pa, dt, gp, gt, reuse != 0);
}
// the same on a state whose B planes carry Q (the intermediate states of mpm_step)
__global__ void __launch_bounds__(kP2GThreads, 4) k_p2g_carried(DevCtx d, PartArgs pa, float dt, int gp, int gt,
                                                                 int reuse) {
    b_p2g<false, true>(d, pa, dt, gp, gt, reuse != 0);
}
__global__ void __launch_bounds__(kP2GThreads, 3) k_p2g_det(DevCtx d, PartArgs pa, float dt, int gp, int gt, int reuse) {
    b_p2g<true>(d, pa, dt, gp, gt, reuse != 0);
}

// one launch for many jobs: workgroup row y runs job y (rows of deterministic-mode
// jobs return at once; k_p2g_det_multi runs those)
__global__ void __launch_bounds__(kP2GThreads, 4) k_p2g_multi(const JobStep *__restrict__ jobs) {
    const JobStep &J = jobs[blockIdx.y];
    if (J.d.det) return;
    b_p2g<false>(J.d, J.pa, J.dt, J.table, J.table, !J.first);
}
__global__ void __launch_bounds__(kP2GThreads, 3) k_p2g_det_multi(const JobStep *__restrict__ jobs) {
    const JobStep &J = jobs[blockIdx.y];
    if (!J.d.det) return;
    b_p2g<true>(J.d, J.pa, J.dt, J.table, J.table, !J.first);
}

// ---------------------------------------------------------------- deterministic P2G sums
// Deterministic mode: each particle block's P2G left its whole tile (exact fixed-point
// sums converted to FP32) in the staging area instead of adding it to the pool with
// float atomics.  Here every node of every active grid block sums the tiles of the
// particle blocks that cover it -- per axis the block itself, the one below at a
// block's first node, and on G+ also the one above at its last node -- in a fixed
// order (z, then y, then x offset) in FP64, and stores the result.  No step of the
// pool sums depends on scheduling, so equal inputs give bitwise equal grids.
__device__ __forceinline__ void b_det_gather(const DevCtx &d, int gp, int gt) {
    const int ng = (int)d.counters[ngb_slot(gt)];
    const int E = (int)d.counters[C_EPOCH];
    const int *pf = stamps(d.pflag, d.nbv, E);
    const int t = threadIdx.x;
    const int g = t >> 6, l = t & 63;
    const int lc[3] = {l & 3, (l >> 2) & 3, l >> 4};
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = lc[a] == 0 ? -1 : 0;
        hi[a] = (g == 1 && lc[a] == 3) ? 1 : 0;
    }
    for (int b = blockIdx.x; b < ng; b += gridDim.x) {
        int bc[3];
        block_coords(d.geo, glist_of(d, gt)[b], bc[0], bc[1], bc[2]);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int oz = lo[2]; oz <= hi[2]; ++oz)
            for (int oy = lo[1]; oy <= hi[1]; ++oy)
                for (int ox = lo[0]; ox <= hi[0]; ++ox) {
                    const int P[3] = {bc[0] + ox, bc[1] + oy, bc[2] + oz};
                    if (P[0] < 0 || P[1] < 0 || P[2] < 0 || P[0] >= d.geo.NB[0] || P[1] >= d.geo.NB[1] ||
                        P[2] >= d.geo.NB[2])
                        continue;
                    const int v = vblock_id(d.geo, P[0], P[1], P[2]);
                    if (pf[v] != E) continue;   // no particles in that block this step
                    const int r = d.prank[v];
                    if (r < 0) continue;
                    // the node in block P's tile: G- [4P, 4P+4], G+ [4P-1, 4P+4] per axis
                    int tl[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) tl[a] = 4 * (bc[a] - P[a]) + lc[a] + g;
                    const int ni = g == 0 ? tl[0] + 5 * tl[1] + 25 * tl[2] : kTileMinus + tl[0] + 6 * tl[1] + 36 * tl[2];
                    const float *sg = d.stage + (size_t)r * kStageFloats + ni;
#pragma unroll
                    for (int ch = 0; ch < 4; ++ch) acc[ch] += (double)sg[ch * kTileNodes];
                }
        float *blk = pool_of(d, gp) + (size_t)b * kBlockFloats + g * 256;
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) blk[ch * 64 + l] = (float)acc[ch];
    }
}

__global__ void __launch_bounds__(128) k_det_gather(DevCtx d, int gp, int gt) { b_det_gather(d, gp, gt); }

// one launch for many jobs: workgroup row y runs job y
__global__ void __launch_bounds__(128) k_det_gather_multi(const JobStep *__restrict__ jobs) {
    const JobStep &J = jobs[blockIdx.y];
    if (!J.d.det) return;
    b_det_gather(J.d, J.table, J.table);
}

// ---------------------------------------------------------------- grid update
// Section 4.3 grid update on each grid: m v~ = m v + dt f (the stress impulse is
// already in the momentum), plus gravity; v~ = 0 where m = 0 and on wall nodes.
constexpr int kGridPer = 4;   // grid blocks per workgroup and pass of the update
constexpr int kGridWGs = 3072;

__device__ __forceinline__ void b_grid_update(const DevCtx &d, float dt, float g0, float g1, float g2, int gp, int gt) {
    const int ng = (int)d.counters[ngb_slot(gt)];
    const int t = threadIdx.x;
    const int g = t >> 6, l = t & 63;
    const int lx = l & 3, ly = (l >> 2) & 3, lz = l >> 4;
    // kGridPer blocks per workgroup and pass, every load of all of them (block ids and
    // the four channels) in one memory round trip
    for (int b0 = blockIdx.x; b0 < ng; b0 += kGridPer * gridDim.x) {
        float m[kGridPer], p0[kGridPer], p1[kGridPer], p2[kGridPer];
        int vb[kGridPer];
#pragma unroll
        for (int k = 0; k < kGridPer; ++k) {
            const int b = b0 + k * gridDim.x;
            if (b < ng) {
                const float *blk = pool_of(d, gp) + (size_t)b * kBlockFloats + g * 256;
                vb[k] = glist_of(d, gt)[b];
                m[k] = blk[l];
                p0[k] = blk[64 + l];
                p1[k] = blk[128 + l];
                p2[k] = blk[192 + l];
            }
        }
#pragma unroll
        for (int k = 0; k < kGridPer; ++k) {
            const int b = b0 + k * gridDim.x;
            if (b >= ng) break;
            int bx, by, bz;
            block_coords(d.geo, vb[k], bx, by, bz);
            const int ix = 4 * bx + lx, iy = 4 * by + ly, iz = 4 * bz + lz;
            const bool inside = ix >= d.geo.stick_lo[g] && iy >= d.geo.stick_lo[g] && iz >= d.geo.stick_lo[g] &&
                                ix <= d.geo.stick_hi[g][0] && iy <= d.geo.stick_hi[g][1] && iz <= d.geo.stick_hi[g][2];
            float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f;
            if (m[k] > 0.0f && inside) {
                const float im = fast_rcp(m[k]);
                v0 = p0[k] * im + dt * g0;
                v1 = p1[k] * im + dt * g1;
                v2 = p2[k] * im + dt * g2;
            }
            float *blk = pool_of(d, gp) + (size_t)b * kBlockFloats + g * 256;
            blk[64 + l] = v0;
            blk[128 + l] = v1;
            blk[192 + l] = v2;
        }
    }
}

__global__ void __launch_bounds__(128) k_grid_update(DevCtx d, float dt, float g0, float g1, float g2, int gp, int gt) { b_grid_update(d, dt, g0, g1, g2, gp, gt); }

// one launch for many jobs: workgroup row y runs job y
__global__ void __launch_bounds__(128) k_grid_update_multi(const JobStep *__restrict__ jobs) {
    const JobStep &J = jobs[blockIdx.y];
    b_grid_update(J.d, J.dt, J.g[0], J.g[1], J.g[2], J.table, J.table);
}

// ---------------------------------------------------------------- G2P
// v_p = 1/2 sum_k sum_i w v~_i,   B_p = 1/2 sum_k sum_i w v~_i (x_i - x_p)^T,
// C_p = B_p D_p^-1,   F <- (I + dt C_p) F,   plasticity,   x <- x + dt v_p.
// The new state is written at the particle's sorted position in the other buffer,
// together with its next cell key and the activation stamps of the next step.
struct G2PIn {
    uint32_t p;
    float x[3], xr[3], H[9];
    uint32_t rp;    // packed remainder of a carried input (unpacked into xr where it is used)
    int mat;
    uint32_t id;
};

// carried: the input is the carried state of an mpm_step sequence (packed remainder,
// left in rp so that loading a particle ahead of its use does not wait for the load)
__device__ __forceinline__ void g2p_load_index(const PartArgs &pa, uint32_t p, G2PIn &q, bool carried = false) {
    q.p = p;
    const long long S = pa.stride;
    // the optional arrays first: the unconditional loads issued last let a later use of
    // an earlier particle wait for fewer of the loads in flight
    q.mat = pa.mat_in ? (int)ld_at(pa.mat_in, p) : 0;
    q.id = pa.id_in ? ld_at(pa.id_in, p) : 0u;
    ld_planes(pa.in, S, kPlaneX, p, q.x);
    if (carried) q.rp = ld_at(reinterpret_cast<const uint32_t *>(pa.in + kPlaneR * S), p);
    else ld_planes(pa.in, S, kPlaneR, p, q.xr);
    ld_planes(pa.in, S, kPlaneH, p, q.H);
}

__device__ __forceinline__ void g2p_load(const DevCtx &d, const PartArgs &pa, uint32_t pos, G2PIn &q) {
    g2p_load_index(pa, ld_at(d.perm, pos), q);
}

// G2P of one particle (section 4.3 gather, section 4.5 affine matrix, F update,
// return mapping, advection) on the velocity tile vt of block (bx,by,bz): writes the
// new state at position `out` of the output buffer (and its stress when write_tau),
// the particle's next cell key and sub code, and returns its new block for the
// activation stamps (-1 when it is not placed).  On return `placed` tells whether
// the new state is finite and inside the domain; then ns and cn hold it.
struct NewState {
    float x[3], v[3], B[9], tau[6];
};

__device__ __forceinline__ int g2p_finish(const DevCtx &d, const PartArgs &pa, float dt, const G2PIn &q,
                                          const DevMaterial &M, const float (&vn)[3], const float (&Bh)[9],
                                          const float (&Di)[9], uint32_t out, bool write_tau, NewState &ns,
                                          CellCoord &cn, bool &placed, bool write_vB = true, bool carry = false);

__device__ __forceinline__ int g2p_particle(const DevCtx &d, const PartArgs &pa, float dt, const G2PIn &q,
                                            const CellCoord &cc, int bx, int by, int bz, const float *vt, uint32_t out,
                                            bool write_tau, NewState &ns, CellCoord &cn, bool &placed,
                                            bool write_vB = true, bool carry = false) {
    const DevMaterial M = material_of(d, q.mat);
    Weights w;
    axis_weights(cc, w);
    float Di[9];
    moment_inverse(cc, w, Di);
    // Gather.  The affine matrix sums w v~ (x_i - x_p)^T, whose weights have a
    // zero dual-grid first moment; subtracting one stencil node's velocity c
    // first keeps the FP32 sums at the size of the velocity differences, and c
    // drops out:
    //   1/2 sum w (v~ - c)(x_i - x_p)^T = 1/2 sum w v~ (x_i - x_p)^T,
    //   v_p = c + 1/2 sum w (v~ - c)   (the weights of each grid sum to one).
    const int tm0 = ((cc.c[2] - 4 * bz) * 5 + (cc.c[1] - 4 * by)) * 5 + (cc.c[0] - 4 * bx);
    const int tp0 = kTileMinus + ((cc.bp[2] - 4 * bz + 1) * 6 + (cc.bp[1] - 4 * by + 1)) * 6 +
                    (cc.bp[0] - 4 * bx + 1);
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
        // separable sums over the 2x2x2 nodes: S = sum w v, M_b = sum w v o_b
        float S3[3], Mx[3], My[3], Mz[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float A[2][2], X[2][2];   // [oz][oy]: x-reduced sum and x-moment
#pragma unroll
            for (int oz = 0; oz < 2; ++oz)
#pragma unroll
                for (int oy = 0; oy < 2; ++oy) {
                    const int t = a * kTileNodes + t0 + oy * sy + oz * sz;
                    const float v0 = vt[t] - cref[a], v1 = vt[t + 1] - cref[a];
                    X[oz][oy] = wa[0][1] * v1;
                    A[oz][oy] = wa[0][0] * v0 + X[oz][oy];
                }
            float Bz[2], BXz[2], BYz[2];
#pragma unroll
            for (int oz = 0; oz < 2; ++oz) {
                BYz[oz] = wa[1][1] * A[oz][1];
                Bz[oz] = wa[1][0] * A[oz][0] + BYz[oz];
                BXz[oz] = wa[1][0] * X[oz][0] + wa[1][1] * X[oz][1];
            }
            Mz[a] = wa[2][1] * Bz[1];
            S3[a] = wa[2][0] * Bz[0] + Mz[a];
            Mx[a] = wa[2][0] * BXz[0] + wa[2][1] * BXz[1];
            My[a] = wa[2][0] * BYz[0] + wa[2][1] * BYz[1];
        }
        // sum_o w v (o - xi)^T = M - S xi^T
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            vs[a] += S3[a];
            Bh[3 * a] += Mx[a] - S3[a] * xi[0];
            Bh[3 * a + 1] += My[a] - S3[a] * xi[1];
            Bh[3 * a + 2] += Mz[a] - S3[a] * xi[2];
        }
    }
    float vn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) vn[a] = cref[a] + 0.5f * vs[a];
#pragma unroll
    for (int i = 0; i < 9; ++i) Bh[i] *= 0.5f;
    return g2p_finish(d, pa, dt, q, M, vn, Bh, Di, out, write_tau, ns, cn, placed, write_vB, carry);
}

// The rest of G2P from the gathered velocity vn and Bh = B / dx (the affine sum in
// cell units), with Di = dx^2 D^-1: C = B D^-1, F update, constitutive update and
// return mapping, advection, stores of the new state, next cell key and sub code.
// As g2p_finish, with the velocity gradient given directly: C = Cc / dx.
__device__ __forceinline__ int g2p_finish_c(const DevCtx &d, const PartArgs &pa, float dt, const G2PIn &q,
                                            const DevMaterial &M, const float (&vn)[3], const float (&Bh)[9],
                                            const float (&Cc)[9], uint32_t out, bool write_tau, NewState &ns,
                                            CellCoord &cn, bool &placed, bool write_vB = true, bool carry = false) {
    const long long S = pa.stride;
    int sig = -1;
    placed = false;
    float Bn[9], C[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        Bn[i] = Bh[i] * d.geo.dx;
        C[i] = d.geo.inv_dx_f * Cc[i];
    }
    // F' = (I + dt C) F  ->  H' = H + dt (C + C H)
    float Fn[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j2 = 0; j2 < 3; ++j2)
            Fn[3 * i + j2] = q.H[3 * i + j2] + dt * (C[3 * i + j2] + C[3 * i] * q.H[j2] +
                                                     C[3 * i + 1] * q.H[3 + j2] + C[3 * i + 2] * q.H[6 + j2]);
    // stress of the new state for the next step's P2G
    float tau[6];
    if (M.model == 1) dp_return_map(M, Fn, tau);
    else kirchhoff(M, Fn, tau);
    float xn[3], xrn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) advance_position(q.x[a], q.xr[a], dt * vn[a], xn[a], xrn[a]);
    // the carried state keeps the packed remainder, and the new cell is that of the
    // packed position, which the next P2G and G2P read
    const uint32_t rpack = carry ? pack_remainder(d.geo, xrn) : 0u;
    if (carry) unpack_remainder(d.geo, rpack, xrn);
    // x * 0 is NaN exactly when x is infinite or NaN
    float probe = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) probe += vn[a] * 0.0f + xn[a] * 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i) probe += Fn[i] * 0.0f + Bn[i] * 0.0f;
    const bool finite = probe == 0.0f;
    if (!finite) set_status(d.counters, ST_NONFINITE);
    const bool inside = finite && cell_coord(d.geo, xn, xrn, cn);
    if (carry) {
        // carried form for the next P2G of the same step sequence: Q = (m B - dt V0 tau)
        // D^-1 / dx at the new position in place of B, and no stress (the same
        // arithmetic that P2G applies to a stored B and stress)
        Weights w2;
        axis_weights(cn, w2);
        float Di2[9];
        moment_inverse(cn, w2, Di2);
        const float T[9] = {tau[0], tau[3], tau[4], tau[3], tau[1], tau[5], tau[4], tau[5], tau[2]};
        const float k = dt * M.vol0;
        float A[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) A[i] = M.mass * Bn[i] - k * T[i];
        const float sc = d.geo.inv_dx_f;
        float st[24];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            st[a] = xn[a];
            st[3 + a] = vn[a];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j2 = 0; j2 < 3; ++j2)
                st[6 + 3 * i + j2] = sc * (A[3 * i] * Di2[j2] + A[3 * i + 1] * Di2[3 + j2] + A[3 * i + 2] * Di2[6 + j2]);
#pragma unroll
        for (int i = 0; i < 9; ++i) st[15 + i] = Fn[i];
        st_planes(pa.out, S, kPlaneX, out, st);
        st_at(reinterpret_cast<uint32_t *>(pa.out + kPlaneR * S), out, rpack);
    } else if (write_vB) {
        float st[24];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            st[a] = xn[a];
            st[3 + a] = vn[a];
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            st[6 + i] = Bn[i];
            st[15 + i] = Fn[i];
        }
        st_planes(pa.out, S, kPlaneX, out, st);
    } else {
        // the fused step: v and B go straight into the next P2G, only x and H are read
        // again (by the next step's G2P)
        st_planes(pa.out, S, kPlaneX, out, xn);
        st_planes(pa.out, S, kPlaneH, out, Fn);
    }
    if (!carry) st_planes(pa.out, S, kPlaneR, out, xrn);
    if (write_tau && !carry) st_planes(d.tau, d.tau_stride, 0, out, tau);
    if (pa.id_out) st_at(pa.id_out, out, q.id);
    if (pa.mat_out) st_at(pa.mat_out, out, (uint8_t)q.mat);
    // next cell key for the following step
    if (inside) {
        const uint32_t key = cell_key(d.geo, cn);
        st_at(d.key, out, key);
        st_at(d.sub, out, (uint16_t)sub_code(cn));
        sig = (int)(key >> 6);
        placed = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ns.x[a] = xn[a];
            ns.v[a] = vn[a];
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) ns.B[i] = Bn[i];
#pragma unroll
        for (int i = 0; i < 6; ++i) ns.tau[i] = tau[i];
    } else {
        st_at(d.key, out, 0xffffffffu);
        set_status(d.counters, ST_DOMAIN);
    }
    return sig;
}

// C = B D^-1 = (dx Bh)(dx^2 Dhat)^-1 = Bh Dhat^-1 / dx
__device__ __forceinline__ int g2p_finish(const DevCtx &d, const PartArgs &pa, float dt, const G2PIn &q,
                                          const DevMaterial &M, const float (&vn)[3], const float (&Bh)[9],
                                          const float (&Di)[9], uint32_t out, bool write_tau, NewState &ns,
                                          CellCoord &cn, bool &placed, bool write_vB, bool carry) {
    float Cc[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j2 = 0; j2 < 3; ++j2)
            Cc[3 * i + j2] = Bh[3 * i] * Di[j2] + Bh[3 * i + 1] * Di[3 + j2] + Bh[3 * i + 2] * Di[6 + j2];
    return g2p_finish_c(d, pa, dt, q, M, vn, Bh, Cc, out, write_tau, ns, cn, placed, write_vB, carry);
}

// G2P workgroups of 128 threads (all G2P kernels): the block's tile gather at the
// start of every block is latency-bound, and six such workgroups per CU (against
// three of 256 threads at the same three waves per SIMD) overlap more of those
// gathers with other blocks' particle work (G2P 0.251 -> 0.238 ms on the sand
// column; the quadratic and gradient G2P gain 9 %).
constexpr int kG2PThreads = 128;

// One pass of the G2P particle loop over particles j0 + thread of a block: `cur` holds
// the particle's inputs (loaded a pass before); `nxt` loads those of the next pass from
// the index pnext (loaded a pass before), and pnext the index after that.  Lanes past
// the end load the block's last particle again: loads on every path let the first
// use of a particle's inputs wait for that particle's loads alone.
template <bool kCarry, bool kCarried>
__device__ __forceinline__ void g2p_pass(const DevCtx &d, const PartArgs &pa, float dt, const float *vt, int bx,
                                         int by, int bz, int s, int cnt, uint32_t last, int j0, int E, G2PIn &cur,
                                         G2PIn &nxt, uint32_t &pnext) {
    const int j = j0 + (int)threadIdx.x;
    const bool act = j < cnt;
    if (kCarried) unpack_remainder(d.geo, cur.rp, cur.xr);
    const uint32_t pn = pnext;   // the index first, then the next particle's inputs
    pnext = ld_at(d.perm, min((uint32_t)(s + j + 2 * kG2PThreads), last));
    g2p_load_index(pa, pn, nxt, kCarried);
    const uint32_t out = (uint32_t)(s + j);
    CellCoord cc;
    bool ok = act && cell_coord(d.geo, cur.x, cur.xr, cc);
    ok = ok && (cc.c[0] >> 2) == bx && (cc.c[1] >> 2) == by && (cc.c[2] >> 2) == bz;
    // activation stamps of the next step (-1: none), deduplicated across the wave
    int sig = -1;
    // blocks whose particle set or bins change: this one when a particle leaves it or
    // its (octant, cell) bin, and the one it enters
    bool changed = false;
    if (act && !ok) {
        set_status(d.counters, ST_STALE);
        st_at(d.key, out, 0xffffffffu);
        changed = true;
    } else if (ok) {
        NewState ns;
        CellCoord cn;
        bool placed;
        sig = g2p_particle(d, pa, dt, cur, cc, bx, by, bz, vt, out, true, ns, cn, placed, true, kCarry);
        if (!placed) {
            changed = true;
        } else if (sig != vblock_id(d.geo, bx, by, bz) || sub_code(cn) != sub_code(cc)) {
            changed = true;
            d.bchg[sig] = E + 1;
        }
    }
    if (__any(changed)) {
        if (changed) d.bchg[vblock_id(d.geo, bx, by, bz)] = E + 1;
    }
    wave_stamp(d, sig, E + 1);
}

// kCarry: the output is the carried state for the next P2G of the same step sequence
// (Q in the B planes, the packed remainder); kCarried: so is the input.  The particle
// loop runs two passes per trip, each reading the inputs the other loaded: the two
// sets of registers then take turns, where one set copied into the other at the end
// of every pass would wait for every store of the pass.  kKept: the step's P2G was
// b_p2g, which kept every block's neighbourhood (one load, not a page lookup that
// waits for the block's id).
template <bool kCarry = false, bool kCarried = false, bool kKept = false>
__device__ __forceinline__ void b_g2p(const DevCtx &d, const PartArgs &pa, float dt, int gp, int gt) {
    __shared__ float vt[3 * kTileNodes];
    __shared__ int nbr[27];
    const int np = (int)d.counters[C_NPB];
    const int E = (int)d.counters[C_EPOCH];
    const int tid = threadIdx.x;
    for (int base = 0; base < np; base += gridDim.x) {
        const int r = round_block(base, np);
        if (r < 0) continue;
        const int vb = d.plist[r];
        int bx, by, bz;
        block_coords(d.geo, vb, bx, by, bz);
        const int s = d.pstart[r];
        const int cnt = d.pstart[r + 1] - s;
        if (cnt <= 0 || cnt > kMaxBlockParticles) continue;
        // the first particle's inputs load while the tile is gathered, and the index of
        // the one after
        const uint32_t last = (uint32_t)(s + cnt - 1);
        G2PIn qa, qb;
        g2p_load_index(pa, ld_at(d.perm, min((uint32_t)(s + tid), last)), qa, kCarried);
        uint32_t pnext = ld_at(d.perm, min((uint32_t)(s + tid + kG2PThreads), last));
        if (kKept) {
            if (tid < 27) nbr[tid] = d.nbrs[27 * (size_t)r + tid];
        } else {
            load_neighbours(d, gt, bx, by, bz, nbr);
        }
        lds_barrier();
        for (int ni = tid; ni < kTileNodes; ni += kG2PThreads) {
            int g, ix, iy, iz;
            tile_node(ni, bx, by, bz, g, ix, iy, iz);
            const long long a = pool_index(d, nbr, bx, by, bz, g, ix, iy, iz, 1);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) vt[ch * kTileNodes + ni] = a >= 0 ? pool_of(d, gp)[a + ch * 64] : 0.0f;
        }
        lds_barrier();
        for (int j0 = 0; j0 < cnt; j0 += 2 * kG2PThreads) {   // the same trip count for every lane
            g2p_pass<kCarry, kCarried>(d, pa, dt, vt, bx, by, bz, s, cnt, last, j0, E, qa, qb, pnext);
            if (j0 + kG2PThreads < cnt)
                g2p_pass<kCarry, kCarried>(d, pa, dt, vt, bx, by, bz, s, cnt, last, j0 + kG2PThreads, E, qb, qa, pnext);
        }
        lds_barrier();
    }
}

__global__ void __launch_bounds__(kG2PThreads) k_g2p(DevCtx d, PartArgs pa, float dt, int gp, int gt) { b_g2p(d, pa, dt, gp, gt); }
// The forms inside an mpm_step sequence, whose P2G (k_p2g or k_p2g_carried) kept every
// block's neighbourhood.
__global__ void __launch_bounds__(kG2PThreads) k_g2p_carry(DevCtx d, PartArgs pa, float dt, int gp, int gt) {
    b_g2p<true, false, true>(d, pa, dt, gp, gt);
}
__global__ void __launch_bounds__(kG2PThreads) k_g2p_cc(DevCtx d, PartArgs pa, float dt, int gp, int gt) {
    b_g2p<true, true, true>(d, pa, dt, gp, gt);
}
__global__ void __launch_bounds__(kG2PThreads) k_g2p_cf(DevCtx d, PartArgs pa, float dt, int gp, int gt) {
    b_g2p<false, true, true>(d, pa, dt, gp, gt);
}

// one launch for many jobs: workgroup row y runs job y (every job's P2G of the round,
// plain or deterministic, was b_p2g, which kept the neighbourhoods)
__global__ void __launch_bounds__(kG2PThreads) k_g2p_multi(const JobStep *__restrict__ jobs) {
    const JobStep &J = jobs[blockIdx.y];
    b_g2p<false, false, true>(J.d, J.pa, J.dt, J.table, J.table);
}

// ---------------------------------------------------------------- exact-gradient transfers
// APIC (section 4.4) and PIC (section 4.3) on the two staggered grids: the stress
// force uses the exact kernel gradient, f_i = -sum_p V0 tau grad w_ip, and G2P takes
// the velocity gradient as 1/2 sum_k sum_i v~_i grad w^T; APIC keeps the affine
// momentum m B D^-1 (x_i - x_p) and carries B, PIC transfers m v alone and carries no
// B.  Per axis on grid k with fraction xi the two weights 1 - xi + s, xi - s have
// x_p-derivatives (cos(2 pi xi) - 1)/dx and (1 - cos(2 pi xi))/dx, and the G- cosine
// is minus the G+ one (the fractions differ by half a cell).
struct GStaged {
    float xm[3], sp[3], cp[3];   // G- fraction, G+ sine and cosine per axis
    float mass, base[3], Q[9];   // affine part as in the MLS staging (Q = 0 for PIC)
    float T[9];                  // -dt V0 tau / dx: force per unit weight gradient (cell units)
    int c[3], oct;
    bool on;
};

__device__ __forceinline__ void grad_stage(const DevCtx &d, const PartArgs &pa, int p, int bx, int by, int bz,
                                           float dt, bool pic, GStaged &r) {
    r.on = false;
    const long long S = pa.stride;
    const uint32_t up = (uint32_t)p;
    float x[3], xr[3], v[3], B[9], tau[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = ld_at(pa.in + a * S, up);
#pragma unroll
    for (int a = 0; a < 3; ++a) xr[a] = ld_at(pa.in + (kPlaneR + a) * S, up);
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = ld_at(pa.in + (3 + a) * S, up);
#pragma unroll
    for (int a = 0; a < 9; ++a) B[a] = pic ? 0.0f : ld_at(pa.in + (6 + a) * S, up);
#pragma unroll
    for (int i = 0; i < 6; ++i) tau[i] = ld_at(d.tau + i * d.tau_stride, up);
    const int mi = pa.mat_in ? (int)ld_at(pa.mat_in, up) : 0;
    const DevMaterial M = material_of(d, mi);
    CellCoord cc;
    if (!cell_coord(d.geo, x, xr, cc)) {
        set_status(d.counters, ST_DOMAIN);
        return;
    }
    if ((cc.c[0] >> 2) != bx || (cc.c[1] >> 2) != by || (cc.c[2] >> 2) != bz) {
        set_status(d.counters, ST_STALE);
        return;
    }
    r.oct = (int)(sub_code(cc) & 7u);
    Weights w;
    axis_weights(cc, w);
    float Di[9];
    moment_inverse(cc, w, Di);
    const float sc = d.geo.inv_dx_f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r.Q[3 * i + j] = sc * M.mass * (B[3 * i] * Di[j] + B[3 * i + 1] * Di[3 + j] + B[3 * i + 2] * Di[6 + j]);
    const float Tf[9] = {tau[0], tau[3], tau[4], tau[3], tau[1], tau[5], tau[4], tau[5], tau[2]};
    const float k = -dt * M.vol0 * sc;
#pragma unroll
    for (int i = 0; i < 9; ++i) r.T[i] = k * Tf[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.c[a] = cc.c[a];
        r.xm[a] = cc.xm[a];
        r.sp[a] = w.sp[a];
        r.cp[a] = __builtin_amdgcn_cosf(cc.xp[a]);
        r.base[a] = M.mass * v[a] - (r.Q[3 * a] * cc.xm[0] + r.Q[3 * a + 1] * cc.xm[1] + r.Q[3 * a + 2] * cc.xm[2]);
    }
    r.mass = M.mass;
    r.on = true;
}

__device__ __forceinline__ float grad_bound(const GStaged &r) {
    if (!r.on) return 0.0f;
    float b = r.mass;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        b = fmaxf(b, fabsf(r.base[a]) + 1.5f * (fabsf(r.Q[3 * a]) + fabsf(r.Q[3 * a + 1]) + fabsf(r.Q[3 * a + 2])) +
                         2.0f * (fabsf(r.T[3 * a]) + fabsf(r.T[3 * a + 1]) + fabsf(r.T[3 * a + 2])));
    return b;
}

// Per-axis weights and x_p-derivatives (cell units) of both grids, the G+ base offset
// and the affine momentum at each grid's base node.
__device__ __forceinline__ void grad_axes(const GStaged &r, float (&w)[2][3][2], float (&dw)[2][3][2], int (&up)[3],
                                          float (&m0)[2][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        up[a] = (r.oct >> a) & 1;
        const float xp = up[a] ? r.xm[a] - 0.5f : r.xm[a] + 0.5f;
        w[0][a][0] = 1.0f - r.xm[a] - r.sp[a];
        w[0][a][1] = r.xm[a] + r.sp[a];
        w[1][a][0] = 1.0f - xp + r.sp[a];
        w[1][a][1] = xp - r.sp[a];
        dw[1][a][0] = r.cp[a] - 1.0f;
        dw[1][a][1] = 1.0f - r.cp[a];
        dw[0][a][0] = -r.cp[a] - 1.0f;
        dw[0][a][1] = 1.0f + r.cp[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        m0[0][a] = r.base[a];
        m0[1][a] = r.base[a] + ((float)up[0] - 0.5f) * r.Q[3 * a] + ((float)up[1] - 0.5f) * r.Q[3 * a + 1] +
                   ((float)up[2] - 0.5f) * r.Q[3 * a + 2];
    }
}

// Adds the particle's 16 contributions to the fixed-point tile (layout of k_p2g's).
__device__ __forceinline__ void grad_scatter(const GStaged &r, int lx, int ly, int lz, unsigned long long *tile_m,
                                             unsigned long long *tile_p, double S) {
    float w[2][3][2], dw[2][3][2], m0[2][3];
    int up[3];
    grad_axes(r, w, dw, up, m0);
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        unsigned long long *tile = g == 0 ? tile_m : tile_p;
        const int ntile = g == 0 ? kTileMStride : kTilePStride;
        const int t0 = g == 0 ? lz * kTZ + ly * kTY + lx : (lz + up[2]) * kTZ + (ly + up[1]) * kTY + (lx + up[0]);
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
            const float wx = w[g][0][ox], wy = w[g][1][oy], wz = w[g][2][oz];
            const float wt = wx * wy * wz;
            const float gx = dw[g][0][ox] * wy * wz, gy = wx * dw[g][1][oy] * wz, gz = wx * wy * dw[g][2][oz];
            const int t = t0 + ox + oy * kTY + oz * kTZ;
            atomicAdd(&tile[t], to_fixed(wt * r.mass, S));
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float mom = wt * (m0[g][a] + ox * r.Q[3 * a] + oy * r.Q[3 * a + 1] + oz * r.Q[3 * a + 2]) +
                                  r.T[3 * a] * gx + r.T[3 * a + 1] * gy + r.T[3 * a + 2] * gz;
                atomicAdd(&tile[(1 + a) * ntile + t], to_fixed(mom, S));
            }
        }
    }
}

__global__ void __launch_bounds__(kP2GThreads) k_p2g_grad(DevCtx d, PartArgs pa, float dt, int gp, int gt) {
    __shared__ int bcnt[kBins];
    __shared__ int bstart[kBins + 1];
    __shared__ int wsum[kP2GThreads / 64];
    __shared__ unsigned int bmax;
    __shared__ int nbr[27];
    __shared__ uint32_t ord[kMaxBlockParticles];
    constexpr int kTileWords = 4 * (kTileMStride + kTilePStride);
    constexpr int kAreaWords = kTileWords > kOrderWords ? kTileWords : kOrderWords;
    __shared__ unsigned long long area[kAreaWords];
    __shared__ int lay[kLayWords];
    __shared__ unsigned long long lmask[kLayMaskWords];
    uint32_t *lbuf = reinterpret_cast<uint32_t *>(area);
    unsigned long long *tile_m = area;
    unsigned long long *tile_p = area + 4 * kTileMStride;
    const bool pic = d.transfer == 2;
    const int np = (int)d.counters[C_NPB];
    const int tid = threadIdx.x;
    for (int base = 0; base < np; base += gridDim.x) {
        const int r = round_block(base, np);
        if (r < 0) continue;
        const int vb = d.plist[r];
        int bx, by, bz;
        block_coords(d.geo, vb, bx, by, bz);
        const int s = d.pstart[r];
        const int cnt = d.pstart[r + 1] - s;
        if (cnt > kMaxBlockParticles) continue;
        order_block<true>(d, r, s, cnt, bcnt, bstart, wsum, lbuf, ord, lay, lmask);
        load_neighbours(d, gt, bx, by, bz, nbr);
        lds_barrier();
        for (int c0 = 0; c0 < cnt; c0 += kChunk) {
            for (int q = tid; q < kTileWords; q += kP2GThreads) area[q] = 0ull;
            if (tid == 0) bmax = 0u;
            GStaged st[2];
            float bnd = 0.0f;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                st[k].on = false;
                const int j = c0 + tid + k * kP2GThreads;
                if (j < cnt) grad_stage(d, pa, (int)ord[j], bx, by, bz, dt, pic, st[k]);
                bnd = fmaxf(bnd, grad_bound(st[k]));
            }
            lds_barrier();
            const double S = block_scale(bnd, &bmax);
#pragma unroll
            for (int k = 0; k < 2; ++k)
                if (st[k].on)
                    grad_scatter(st[k], st[k].c[0] - 4 * bx, st[k].c[1] - 4 * by, st[k].c[2] - 4 * bz, tile_m, tile_p, S);
            lds_barrier();
            const double inv = 1.0 / S;
            for (int ni = tid; ni < kTileNodes; ni += kP2GThreads) {
                int g, ix, iy, iz;
                tile_node(ni, bx, by, bz, g, ix, iy, iz);
                const int lx = ix - 4 * bx + g, ly = iy - 4 * by + g, lz = iz - 4 * bz + g;
                const unsigned long long *tb = g == 0 ? tile_m : tile_p;
                const int cs = g == 0 ? kTileMStride : kTilePStride;
                const int t = lx + ly * kTY + lz * kTZ;
                float val[4];
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) val[ch] = (float)((double)(long long)tb[ch * cs + t] * inv);
                if (val[0] == 0.0f && val[1] == 0.0f && val[2] == 0.0f && val[3] == 0.0f) continue;
                const long long a = pool_index(d, nbr, bx, by, bz, g, ix, iy, iz, 0);
                if (a < 0) {
                    set_status(d.counters, ST_CAPACITY);
                    continue;
                }
#pragma unroll
                for (int ch = 0; ch < 4; ++ch)
                    if (val[ch] != 0.0f) atomicAdd(&pool_of(d, gp)[a + ch * 64], val[ch]);
            }
            lds_barrier();
        }
    }
}

// G2P with the exact velocity gradient: v = 1/2 sum w v~, B = 1/2 sum w v~ d^T (APIC;
// zero for PIC), C = 1/2 sum v~ grad w^T, all relative to the velocity of one stencil
// node (the weights of a grid sum to one, their gradients to zero).
__global__ void __launch_bounds__(kG2PThreads) k_g2p_grad(DevCtx d, PartArgs pa, float dt, int gp, int gt) {
    __shared__ float vt[3 * kTileNodes];
    __shared__ int nbr[27];
    const bool pic = d.transfer == 2;
    const int np = (int)d.counters[C_NPB];
    const int E = (int)d.counters[C_EPOCH];
    const int tid = threadIdx.x;
    for (int base = 0; base < np; base += gridDim.x) {
        const int r = round_block(base, np);
        if (r < 0) continue;
        const int vb = d.plist[r];
        int bx, by, bz;
        block_coords(d.geo, vb, bx, by, bz);
        const int s = d.pstart[r];
        const int cnt = d.pstart[r + 1] - s;
        if (cnt > kMaxBlockParticles) continue;
        G2PIn nxt;
        if (tid < cnt) g2p_load(d, pa, (uint32_t)(s + tid), nxt);
        load_neighbours(d, gt, bx, by, bz, nbr);
        lds_barrier();
        for (int ni = tid; ni < kTileNodes; ni += kG2PThreads) {
            int g, ix, iy, iz;
            tile_node(ni, bx, by, bz, g, ix, iy, iz);
            const long long a = pool_index(d, nbr, bx, by, bz, g, ix, iy, iz, 1);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) vt[ch * kTileNodes + ni] = a >= 0 ? pool_of(d, gp)[a + ch * 64] : 0.0f;
        }
        lds_barrier();
        for (int j0 = 0; j0 < cnt; j0 += kG2PThreads) {
            const int j = j0 + tid;
            const bool act = j < cnt;
            const G2PIn q = nxt;
            if (j + kG2PThreads < cnt) g2p_load(d, pa, (uint32_t)(s + j + kG2PThreads), nxt);
            const uint32_t out = (uint32_t)(s + j);
            CellCoord cc;
            bool ok = act && cell_coord(d.geo, q.x, q.xr, cc);
            ok = ok && (cc.c[0] >> 2) == bx && (cc.c[1] >> 2) == by && (cc.c[2] >> 2) == bz;
            int sig = -1;
            if (act && !ok) {
                set_status(d.counters, ST_STALE);
                st_at(d.key, out, 0xffffffffu);
            } else if (ok) {
                Weights wt;
                axis_weights(cc, wt);
                float cp[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) cp[a] = __builtin_amdgcn_cosf(cc.xp[a]);
                const int tm0 = ((cc.c[2] - 4 * bz) * 5 + (cc.c[1] - 4 * by)) * 5 + (cc.c[0] - 4 * bx);
                const int tp0 = kTileMinus + ((cc.bp[2] - 4 * bz + 1) * 6 + (cc.bp[1] - 4 * by + 1)) * 6 +
                                (cc.bp[0] - 4 * bx + 1);
                const float cref[3] = {vt[tm0], vt[kTileNodes + tm0], vt[2 * kTileNodes + tm0]};
                float vs[3] = {0.0f, 0.0f, 0.0f}, Bh[9], Cc[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    Bh[i] = 0.0f;
                    Cc[i] = 0.0f;
                }
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    const float *xi = g == 0 ? cc.xm : cc.xp;
                    const int t0 = g == 0 ? tm0 : tp0;
                    const int sy = g == 0 ? 5 : 6, sz = g == 0 ? 25 : 36;
                    const float(*wa)[2] = g == 0 ? wt.wm : wt.wp;
#pragma unroll
                    for (int o = 0; o < 8; ++o) {
                        const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
                        const int off[3] = {ox, oy, oz};
                        float wv = 1.0f, gd[3];
                        float wa3[3], dwa3[3];
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            wa3[a] = wa[a][off[a]];
                            const float c = g == 0 ? -cp[a] : cp[a];
                            dwa3[a] = off[a] ? 1.0f - c : c - 1.0f;
                            wv *= wa3[a];
                        }
                        gd[0] = dwa3[0] * wa3[1] * wa3[2];
                        gd[1] = wa3[0] * dwa3[1] * wa3[2];
                        gd[2] = wa3[0] * wa3[1] * dwa3[2];
                        const int t = t0 + ox + oy * sy + oz * sz;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            const float dv = vt[a * kTileNodes + t] - cref[a];
                            vs[a] += wv * dv;
#pragma unroll
                            for (int b = 0; b < 3; ++b) {
                                Bh[3 * a + b] += wv * dv * ((float)off[b] - xi[b]);
                                Cc[3 * a + b] += dv * gd[b];
                            }
                        }
                    }
                }
                float vn[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) vn[a] = cref[a] + 0.5f * vs[a];
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    Bh[i] = pic ? 0.0f : 0.5f * Bh[i];
                    Cc[i] *= 0.5f;
                }
                const DevMaterial M = material_of(d, q.mat);
                NewState ns;
                CellCoord cn;
                bool placed;
                sig = g2p_finish_c(d, pa, dt, q, M, vn, Bh, Cc, out, true, ns, cn, placed);
            }
            wave_stamp(d, sig, E + 1);
        }
        lds_barrier();
    }
}

// ---------------------------------------------------------------- quadratic B-spline
// The single-grid quadratic B-spline kernel the paper measures the compact kernel
// against (section 6).  Node i sits at origin + i dx; a particle at X (cells) reaches
// the 27 nodes base + o, base = floor(X - 1/2), o in {0,1,2}^3, with per-axis weights
//   1/2 (3/2 - xi)^2,  3/4 - (1 - xi)^2,  1/2 (xi - 1/2)^2,   xi = X - base in [1/2, 3/2),
// whose second moment is 1/4 on every axis: D = dx^2/4 I, so the momentum a particle
// gives node base + o is m v + Qc (o - xi) with Qc = (m B - dt V0 tau) 4/dx.
// The particles of block B reach nodes [4B-1, 4B+5]^3 (7^3 = 343), staged as one
// fixed-point tile in P2G and one velocity tile in G2P; the grid lives in the G-
// half of each pool block (the G+ half stays empty).
struct QStaged {
    float xi[3];
    int lb[3];      // base node relative to 4B - 1
    float mass, mom0[3], Qc[9];
    bool on;
};

// Quadratic base node and fraction from the G- cell coordinates (X = c + xm - 1/4):
// false when some node would fall off the grid.
__device__ __forceinline__ bool quad_coords(const Geometry &g, const CellCoord &cc, int bx, int by, int bz,
                                            float (&xi)[3], int (&lb)[3]) {
    const int b4[3] = {4 * bx - 1, 4 * by - 1, 4 * bz - 1};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool up = cc.xm[a] >= 0.75f;
        const int base = up ? cc.c[a] : cc.c[a] - 1;
        xi[a] = up ? cc.xm[a] - 0.25f : cc.xm[a] + 0.75f;
        ok = ok && base >= 0 && base + 2 <= g.n[a];
        lb[a] = base - b4[a];
    }
    return ok;
}

__device__ __forceinline__ void quad_weights(const float (&xi)[3], float (&w)[3][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = 1.5f - xi[a], c = 1.0f - xi[a], l = xi[a] - 0.5f;
        w[a][0] = 0.5f * u * u;
        w[a][1] = 0.75f - c * c;
        w[a][2] = 0.5f * l * l;
    }
}

__device__ __forceinline__ void quad_stage(const DevCtx &d, const PartArgs &pa, int p, int bx, int by, int bz,
                                           float dt, QStaged &r) {
    r.on = false;
    const long long S = pa.stride;
    const uint32_t up = (uint32_t)p;
    float x[3], xr[3], v[3], B[9], tau[6];
    ld_planes(pa.in, S, kPlaneX, up, x);
    ld_planes(pa.in, S, kPlaneR, up, xr);
    ld_planes(pa.in, S, kPlaneV, up, v);
    ld_planes(pa.in, S, kPlaneB, up, B);
    ld_planes(d.tau, d.tau_stride, 0, up, tau);
    const int mi = pa.mat_in ? (int)ld_at(pa.mat_in, up) : 0;
    const DevMaterial M = material_of(d, mi);
    CellCoord cc;
    if (!cell_coord(d.geo, x, xr, cc)) {
        set_status(d.counters, ST_DOMAIN);
        return;
    }
    if ((cc.c[0] >> 2) != bx || (cc.c[1] >> 2) != by || (cc.c[2] >> 2) != bz) {
        set_status(d.counters, ST_STALE);
        return;
    }
    if (!quad_coords(d.geo, cc, bx, by, bz, r.xi, r.lb)) {
        set_status(d.counters, ST_DOMAIN);
        return;
    }
    const float T[9] = {tau[0], tau[3], tau[4], tau[3], tau[1], tau[5], tau[4], tau[5], tau[2]};
    const float k = dt * M.vol0, sc = 4.0f * d.geo.inv_dx_f;
#pragma unroll
    for (int i = 0; i < 9; ++i) r.Qc[i] = sc * (M.mass * B[i] - k * T[i]);
#pragma unroll
    for (int a = 0; a < 3; ++a)
        r.mom0[a] = M.mass * v[a] - (r.Qc[3 * a] * r.xi[0] + r.Qc[3 * a + 1] * r.xi[1] + r.Qc[3 * a + 2] * r.xi[2]);
    r.mass = M.mass;
    r.on = true;
}

__device__ __forceinline__ float quad_bound(const QStaged &r) {
    if (!r.on) return 0.0f;
    float b = r.mass;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        b = fmaxf(b, fabsf(r.mom0[a]) + 2.0f * (fabsf(r.Qc[3 * a]) + fabsf(r.Qc[3 * a + 1]) + fabsf(r.Qc[3 * a + 2])));
    return b;
}

constexpr int kQTY = 8, kQTZ = 66;                    // padded strides of the 7^3 tile
constexpr int kQStride = 6 * kQTZ + 6 * kQTY + 7;     // words per channel
constexpr int kQNodes = 343;

__device__ __forceinline__ void quad_scatter(const QStaged &r, unsigned long long *tile, double S) {
    float w[3][3];
    quad_weights(r.xi, w);
#pragma unroll
    for (int oz = 0; oz < 3; ++oz)
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
            const float wyz = w[1][oy] * w[2][oz];
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
                const float wt = w[0][ox] * wyz;
                const int t = (r.lb[0] + ox) + (r.lb[1] + oy) * kQTY + (r.lb[2] + oz) * kQTZ;
                atomicAdd(&tile[t], to_fixed(wt * r.mass, S));
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    atomicAdd(&tile[(1 + a) * kQStride + t],
                              to_fixed(wt * (r.mom0[a] + r.Qc[3 * a] * ox + r.Qc[3 * a + 1] * oy + r.Qc[3 * a + 2] * oz), S));
            }
        }
}

__global__ void __launch_bounds__(kP2GThreads, 4) k_p2g_quad(DevCtx d, PartArgs pa, float dt, int gp, int gt) {
    __shared__ int bcnt[kBins];
    __shared__ int bstart[kBins + 1];
    __shared__ int wsum[kP2GThreads / 64];
    __shared__ unsigned int bmax;
    __shared__ int nbr[27];
    __shared__ uint32_t ord[kMaxBlockParticles];
    constexpr int kTileWords = 4 * kQStride;
    constexpr int kAreaWords = kTileWords > kOrderWords ? kTileWords : kOrderWords;
    __shared__ unsigned long long area[kAreaWords];
    __shared__ int lay[kLayWords];
    __shared__ unsigned long long lmask[kLayMaskWords];
    uint32_t *lbuf = reinterpret_cast<uint32_t *>(area);
    unsigned long long *tile = area;
    const int np = (int)d.counters[C_NPB];
    const int tid = threadIdx.x;
    for (int base = 0; base < np; base += gridDim.x) {
        const int r = round_block(base, np);
        if (r < 0) continue;
        const int vb = d.plist[r];
        int bx, by, bz;
        block_coords(d.geo, vb, bx, by, bz);
        const int s = d.pstart[r];
        const int cnt = d.pstart[r + 1] - s;
        if (cnt > kMaxBlockParticles) continue;   // reported by the bucket scan
        order_block<true>(d, r, s, cnt, bcnt, bstart, wsum, lbuf, ord, lay, lmask);
        load_neighbours(d, gt, bx, by, bz, nbr);
        lds_barrier();
        for (int c0 = 0; c0 < cnt; c0 += kChunk) {
            for (int q = tid; q < kTileWords; q += kP2GThreads) area[q] = 0ull;
            if (tid == 0) bmax = 0u;
            QStaged st[2];
            float bnd = 0.0f;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                st[k].on = false;
                const int j = c0 + tid + k * kP2GThreads;
                if (j < cnt) quad_stage(d, pa, (int)ord[j], bx, by, bz, dt, st[k]);
                bnd = fmaxf(bnd, quad_bound(st[k]));
            }
            lds_barrier();   // tile cleared, bmax reset
            const double S = block_scale(bnd, &bmax);
#pragma unroll
            for (int k = 0; k < 2; ++k)
                if (st[k].on) quad_scatter(st[k], tile, S);
            lds_barrier();
            const double inv = 1.0 / S;
            for (int ni = tid; ni < kQNodes; ni += kP2GThreads) {
                const int lx = ni % 7, ly = (ni / 7) % 7, lz = ni / 49;
                const int t = lx + ly * kQTY + lz * kQTZ;
                float val[4];
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) val[ch] = (float)((double)(long long)tile[ch * kQStride + t] * inv);
                if (val[0] == 0.0f && val[1] == 0.0f && val[2] == 0.0f && val[3] == 0.0f) continue;
                const int ix = 4 * bx - 1 + lx, iy = 4 * by - 1 + ly, iz = 4 * bz - 1 + lz;
                const long long a = pool_index(d, nbr, bx, by, bz, 0, ix, iy, iz, 0);
                if (a < 0) {
                    set_status(d.counters, ST_CAPACITY);
                    continue;
                }
#pragma unroll
                for (int ch = 0; ch < 4; ++ch)
                    if (val[ch] != 0.0f) atomicAdd(&pool_of(d, gp)[a + ch * 64], val[ch]);
            }
            lds_barrier();
        }
    }
}

__global__ void __launch_bounds__(kG2PThreads) k_g2p_quad(DevCtx d, PartArgs pa, float dt, int gp, int gt) {
    __shared__ float vt[3 * kQNodes];
    __shared__ int nbr[27];
    const int np = (int)d.counters[C_NPB];
    const int E = (int)d.counters[C_EPOCH];
    const int tid = threadIdx.x;
    for (int base = 0; base < np; base += gridDim.x) {
        const int r = round_block(base, np);
        if (r < 0) continue;
        const int vb = d.plist[r];
        int bx, by, bz;
        block_coords(d.geo, vb, bx, by, bz);
        const int s = d.pstart[r];
        const int cnt = d.pstart[r + 1] - s;
        if (cnt > kMaxBlockParticles) continue;
        G2PIn nxt;
        if (tid < cnt) g2p_load(d, pa, (uint32_t)(s + tid), nxt);
        load_neighbours(d, gt, bx, by, bz, nbr);
        lds_barrier();
        for (int ni = tid; ni < kQNodes; ni += kG2PThreads) {
            const int ix = 4 * bx - 1 + ni % 7, iy = 4 * by - 1 + (ni / 7) % 7, iz = 4 * bz - 1 + ni / 49;
            const long long a = pool_index(d, nbr, bx, by, bz, 0, ix, iy, iz, 1);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) vt[ch * kQNodes + ni] = a >= 0 ? pool_of(d, gp)[a + ch * 64] : 0.0f;
        }
        lds_barrier();
        for (int j0 = 0; j0 < cnt; j0 += kG2PThreads) {
            const int j = j0 + tid;
            const bool act = j < cnt;
            const G2PIn q = nxt;
            if (j + kG2PThreads < cnt) g2p_load(d, pa, (uint32_t)(s + j + kG2PThreads), nxt);
            const uint32_t out = (uint32_t)(s + j);
            CellCoord cc;
            bool ok = act && cell_coord(d.geo, q.x, q.xr, cc);
            ok = ok && (cc.c[0] >> 2) == bx && (cc.c[1] >> 2) == by && (cc.c[2] >> 2) == bz;
            float xi[3];
            int lb[3];
            const bool inside = ok && quad_coords(d.geo, cc, bx, by, bz, xi, lb);
            int sig = -1;
            if (act && !ok) {
                set_status(d.counters, ST_STALE);
                st_at(d.key, out, 0xffffffffu);
            } else if (ok && !inside) {
                set_status(d.counters, ST_DOMAIN);
                st_at(d.key, out, 0xffffffffu);
            } else if (ok) {
                // v = sum w v~, Bh = sum w v~ (o - xi)^T, relative to the velocity c of
                // the middle node (the weights sum to one and have zero first moment)
                float w[3][3];
                quad_weights(xi, w);
                const int t1 = (lb[0] + 1) + (lb[1] + 1) * 7 + (lb[2] + 1) * 49;
                const float cref[3] = {vt[t1], vt[kQNodes + t1], vt[2 * kQNodes + t1]};
                float vs[3] = {0.0f, 0.0f, 0.0f}, Bh[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) Bh[i] = 0.0f;
#pragma unroll
                for (int oz = 0; oz < 3; ++oz)
#pragma unroll
                    for (int oy = 0; oy < 3; ++oy)
#pragma unroll
                        for (int ox = 0; ox < 3; ++ox) {
                            const float wt = w[0][ox] * w[1][oy] * w[2][oz];
                            const int t = (lb[0] + ox) + (lb[1] + oy) * 7 + (lb[2] + oz) * 49;
                            const float dxo = (float)ox - xi[0], dyo = (float)oy - xi[1], dzo = (float)oz - xi[2];
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                const float dv = wt * (vt[a * kQNodes + t] - cref[a]);
                                vs[a] += dv;
                                Bh[3 * a] += dv * dxo;
                                Bh[3 * a + 1] += dv * dyo;
                                Bh[3 * a + 2] += dv * dzo;
                            }
                        }
                float vn[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) vn[a] = cref[a] + vs[a];
                const float Di[9] = {4.0f, 0.0f, 0.0f, 0.0f, 4.0f, 0.0f, 0.0f, 0.0f, 4.0f};
                const DevMaterial M = material_of(d, q.mat);
                NewState ns;
                CellCoord cn;
                bool placed;
                sig = g2p_finish(d, pa, dt, q, M, vn, Bh, Di, out, true, ns, cn, placed);
            }
            wave_stamp(d, sig, E + 1);
        }
        lds_barrier();
    }
}

// ---------------------------------------------------------------- exports
// Order of a block's particles alone (for a G2P that follows a sort without P2G).
__global__ void __launch_bounds__(kP2GThreads) k_block_order(DevCtx d) {
    __shared__ int bcnt[kBins];
    __shared__ int bstart[kBins + 1];
    __shared__ int wsum[kP2GThreads / 64];
    __shared__ uint32_t lbuf[kMaxBlockParticles];
    __shared__ uint32_t ord[kMaxBlockParticles];
    __shared__ int lay[kLayWords];
    __shared__ unsigned long long lmask[kLayMaskWords];
    const int np = (int)d.counters[C_NPB];
    for (int base = 0; base < np; base += gridDim.x) {
        const int r = round_block(base, np);
        if (r < 0) continue;
        const int s = d.pstart[r];
        const int cnt = d.pstart[r + 1] - s;
        if (cnt > kMaxBlockParticles) continue;
        order_block<true>(d, r, s, cnt, bcnt, bstart, wsum, lbuf, ord, lay, lmask);
        lds_barrier();
    }
}

// ---------------------------------------------------------------- fused G2P + P2G
// G2P of step n fused with P2G of step n+1 (the paper's G2P2G kernel structure):
// each workgroup gathers its block's particles from grid n, updates them, writes
// the new positions and deformation gradients (the new v and B go straight into the
// scatter and are never stored; the last step of a sequence runs the plain G2P, which
// stores the whole state), and scatters every particle into grid n+1 as soon as it is
// updated, through an FP64 tile covering every node the block's particles reach after
// moving at most one cell: G- nodes [4B-1, 4B+5]^3 and G+ nodes [4B-2, 4B+5]^3
// (7^3 + 8^3 = 855 nodes).  Particles that moved further add to the pool with float atomics (up to
// three cells; beyond that the step reports MPM_E_CFL).  Grid n+1 is the 3 x 3 x 3
// block neighbourhood of the particle blocks of step n, prepared by the same sort.
constexpr int kFTY = 8, kFTZ = 66;                   // for every node offset the 64 cells of a block
                                                     // fall on 16 distinct residues modulo 16
constexpr int kFMStride = 6 * kFTZ + 6 * kFTY + 7;   // words per channel, G- (tile-local [0,6]^3)
constexpr int kFPStride = 7 * kFTZ + 7 * kFTY + 8;   // G+ ([0,7]^3)
constexpr int kFNodesM = 343, kFNodesP = 512;

__global__ void __launch_bounds__(kP2GThreads, 2) k_g2p2g(DevCtx d, PartArgs pa, float dt, int gp_in, int gt_in,
                                                       int gp_out, int gt_out) {
    __shared__ int bcnt[kBins];
    __shared__ int bstart[kBins + 1];
    __shared__ int wsum[kP2GThreads / 64];
    __shared__ int nbr_in[27], nbr_out[27];
    __shared__ uint32_t ord[kMaxBlockParticles];
    __shared__ float vt[3 * kTileNodes];
    constexpr int kTileWords = 4 * (kFMStride + kFPStride);
    constexpr int kAreaWords = kTileWords > kOrderWords ? kTileWords : kOrderWords;
    __shared__ unsigned long long area[kAreaWords];
    __shared__ int lay[kLayWords];
    __shared__ unsigned long long lmask[kLayMaskWords];
    uint32_t *lbuf = reinterpret_cast<uint32_t *>(area);
    double *tile_m = reinterpret_cast<double *>(area);
    double *tile_p = tile_m + 4 * kFMStride;
    const int np = (int)d.counters[C_NPB];
    const int E = (int)d.counters[C_EPOCH];
    const int tid = threadIdx.x;
    for (int base = 0; base < np; base += gridDim.x) {
        const int r = round_block(base, np);
        if (r < 0) continue;
        const int vb = d.plist[r];
        int bx, by, bz;
        block_coords(d.geo, vb, bx, by, bz);
        const int s = d.pstart[r];
        const int cnt = d.pstart[r + 1] - s;
        if (cnt > kMaxBlockParticles) continue;   // reported by the bucket scan
        order_block<true>(d, r, s, cnt, bcnt, bstart, wsum, lbuf, ord, lay, lmask);
        load_neighbours(d, gt_in, bx, by, bz, nbr_in);
        load_neighbours(d, gt_out, bx, by, bz, nbr_out, 64);
        lds_barrier();
        // grid n's velocity tile, the first particle's inputs and the cleared FP64 tile
        // of grid n+1 (which reuses the ordering buffers) in one round
        G2PIn nxt;
        if (tid < cnt) g2p_load_index(pa, ord[tid], nxt);
        for (int ni = tid; ni < kTileNodes; ni += kP2GThreads) {
            int g, ix, iy, iz;
            tile_node(ni, bx, by, bz, g, ix, iy, iz);
            const long long a = pool_index(d, nbr_in, bx, by, bz, g, ix, iy, iz, 1);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) vt[ch * kTileNodes + ni] = a >= 0 ? pool_of(d, gp_in)[a + ch * 64] : 0.0f;
        }
        for (int q = tid; q < kTileWords; q += kP2GThreads) area[q] = 0ull;
        lds_barrier();
        // each particle: G2P from grid n, then at once its P2G into grid n+1 (no block
        // unit to agree on with an FP64 tile, so nothing is held between particles)
        for (int j0 = 0; j0 < cnt; j0 += kP2GThreads) {   // the same trip count for every lane
            const int j = j0 + tid;
            const bool act = j < cnt;
            const G2PIn q = nxt;
            if (j + kP2GThreads < cnt) g2p_load_index(pa, ord[j + kP2GThreads], nxt);
            const uint32_t out = (uint32_t)(s + j);
            CellCoord cc;
            bool ok = act && cell_coord(d.geo, q.x, q.xr, cc);
            ok = ok && (cc.c[0] >> 2) == bx && (cc.c[1] >> 2) == by && (cc.c[2] >> 2) == bz;
            int sig = -1;
            Staged st;
            st.on = false;
            if (act && !ok) {
                set_status(d.counters, ST_STALE);
                st_at(d.key, out, 0xffffffffu);
            } else if (ok) {
                NewState ns;
                CellCoord cn;
                bool placed;
                sig = g2p_particle(d, pa, dt, q, cc, bx, by, bz, vt, out, false, ns, cn, placed, false);
                if (placed) {
                    const DevMaterial M = material_of(d, q.mat);
                    stage_compute(d, M, cn, ns.v, ns.B, ns.tau, dt, st);
                }
            }
            wave_stamp(d, sig, E + 1);
            if (st.on) {
                const int lx = st.c[0] - 4 * bx + 1, ly = st.c[1] - 4 * by + 1, lz = st.c[2] - 4 * bz + 1;
                if (lx >= 0 && ly >= 0 && lz >= 0 && lx <= 5 && ly <= 5 && lz <= 5)
                    scatter_particle_f64<kFTY, kFTZ, kFMStride, kFPStride>(st, lx, ly, lz, tile_m, tile_p);
                else
                    scatter_pool(d, pool_of(d, gp_out), nbr_out, bx, by, bz, st);
            }
        }
        lds_barrier();
        // ---- flush every nonzero tile node to grid n+1
        for (int ni = tid; ni < kFNodesM + kFNodesP; ni += kP2GThreads) {
            const int g = ni < kFNodesM ? 0 : 1;
            int lx, ly, lz;
            if (g == 0) {
                lx = ni % 7;
                ly = (ni / 7) % 7;
                lz = ni / 49;
            } else {
                const int k = ni - kFNodesM;
                lx = k & 7;
                ly = (k >> 3) & 7;
                lz = k >> 6;
            }
            const double *tb = g == 0 ? tile_m : tile_p;
            const int cs = g == 0 ? kFMStride : kFPStride;
            const int t = lx + ly * kFTY + lz * kFTZ;
            float val[4];
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) val[ch] = (float)tb[ch * cs + t];
            if (val[0] == 0.0f && val[1] == 0.0f && val[2] == 0.0f && val[3] == 0.0f) continue;
            const int ix = 4 * bx - 1 - g + lx, iy = 4 * by - 1 - g + ly, iz = 4 * bz - 1 - g + lz;
            const long long a = pool_index(d, nbr_out, bx, by, bz, g, ix, iy, iz, 0);
            if (a < 0) {
                set_status(d.counters, ST_CFL);
                continue;
            }
#pragma unroll
            for (int ch = 0; ch < 4; ++ch)
                if (val[ch] != 0.0f) atomicAdd(&pool_of(d, gp_out)[a + ch * 64], val[ch]);
        }
        lds_barrier();
    }
}

__global__ void k_zero_pool(DevCtx d, int gp, int gt) {
    const long long nfl = (long long)d.counters[ngb_slot(gt)] * (kBlockFloats / 4);
    float4 *pool4 = reinterpret_cast<float4 *>(pool_of(d, gp));
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nfl; t += (long long)gridDim.x * blockDim.x)
        pool4[t] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Dense export of grids g0 .. g0 + ng - 1 (ng = 1 or 2).
__global__ void k_grid_export(DevCtx d, float *m, float *vec, int gp, int gt, int g0, int ng) {
    const long long nx = d.geo.n[0] + 1, ny = d.geo.n[1] + 1, nz = d.geo.n[2] + 1;
    const long long nodes = nx * ny * nz;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < ng * nodes; t += (long long)gridDim.x * blockDim.x) {
        const int g = g0 + (int)(t / nodes);
        const long long r = t - (g - g0) * nodes;
        const int ix = (int)(r % nx), iy = (int)((r / nx) % ny), iz = (int)(r / (nx * ny));
        const int v = vblock_id(d.geo, ix >> 2, iy >> 2, iz >> 2);
        float mm = 0.0f, a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
        const int ph = page_of(d, gt)[v];
        if (ph >= 0) {
            const float *blk = pool_of(d, gp) + (size_t)ph * kBlockFloats + g * 256;
            const int l = (iz & 3) * 16 + (iy & 3) * 4 + (ix & 3);
            mm = blk[l];
            a0 = blk[64 + l];
            a1 = blk[128 + l];
            a2 = blk[192 + l];
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

void launch_p2g(const DevCtx &d, const PartArgs &pa, float dt, int gp, int gt, hipStream_t s, bool carried,
                bool reuse) {
    const int ru = reuse ? 1 : 0;
    if (d.quadratic)
        hipLaunchKernelGGL(k_p2g_quad, dim3(particle_grid(d)), dim3(kP2GThreads), 0, s, d, pa, dt, gp, gt);
    else if (d.transfer != 0)
        hipLaunchKernelGGL(k_p2g_grad, dim3(particle_grid(d)), dim3(kP2GThreads), 0, s, d, pa, dt, gp, gt);
    else if (d.det)
        hipLaunchKernelGGL(k_p2g_det, dim3(particle_grid(d)), dim3(kP2GThreads), 0, s, d, pa, dt, gp, gt, ru);
    else if (carried)
        hipLaunchKernelGGL(k_p2g_carried, dim3(particle_grid(d)), dim3(kP2GThreads), 0, s, d, pa, dt, gp, gt, ru);
    else
        hipLaunchKernelGGL(k_p2g, dim3(particle_grid(d)), dim3(kP2GThreads), 0, s, d, pa, dt, gp, gt, ru);
}

void launch_det_gather(const DevCtx &d, int gp, int gt, hipStream_t s) {
    hipLaunchKernelGGL(k_det_gather, dim3(d.max_blocks < kGridWGs ? d.max_blocks : kGridWGs), dim3(128), 0, s, d, gp, gt);
}

void launch_grid_update(const DevCtx &d, float dt, const float gravity[3], int gp, int gt, hipStream_t s) {
    hipLaunchKernelGGL(k_grid_update, dim3(d.max_blocks < kGridWGs ? d.max_blocks : kGridWGs), dim3(128), 0, s, d, dt,
                       gravity[0], gravity[1], gravity[2], gp, gt);
}

void launch_g2p(const DevCtx &d, const PartArgs &pa, float dt, int gp, int gt, hipStream_t s, bool carry,
                bool carried) {
    if (d.quadratic)
        hipLaunchKernelGGL(k_g2p_quad, dim3(particle_grid(d)), dim3(kG2PThreads), 0, s, d, pa, dt, gp, gt);
    else if (d.transfer != 0)
        hipLaunchKernelGGL(k_g2p_grad, dim3(particle_grid(d)), dim3(kG2PThreads), 0, s, d, pa, dt, gp, gt);
    else if (carry && carried)
        hipLaunchKernelGGL(k_g2p_cc, dim3(particle_grid(d)), dim3(kG2PThreads), 0, s, d, pa, dt, gp, gt);
    else if (carry)
        hipLaunchKernelGGL(k_g2p_carry, dim3(particle_grid(d)), dim3(kG2PThreads), 0, s, d, pa, dt, gp, gt);
    else if (carried)
        hipLaunchKernelGGL(k_g2p_cf, dim3(particle_grid(d)), dim3(kG2PThreads), 0, s, d, pa, dt, gp, gt);
    else
        hipLaunchKernelGGL(k_g2p, dim3(particle_grid(d)), dim3(kG2PThreads), 0, s, d, pa, dt, gp, gt);
}

void launch_block_order(const DevCtx &d, hipStream_t s) {
    hipLaunchKernelGGL(k_block_order, dim3(particle_grid(d)), dim3(kP2GThreads), 0, s, d);
}

void launch_g2p2g(const DevCtx &d, const PartArgs &pa, float dt, int gp_in, int gt_in, int gp_out, int gt_out,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_g2p2g, dim3(particle_grid(d)), dim3(kP2GThreads), 0, s, d, pa, dt, gp_in, gt_in, gp_out,
                       gt_out);
}

void launch_zero_pool(const DevCtx &d, int gp, int gt, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_pool, dim3(2048), dim3(256), 0, s, d, gp, gt);
}

void launch_grid_export(const DevCtx &d, float *m, float *vec, int gp, int gt, int g0, int ng, hipStream_t s) {
    hipLaunchKernelGGL(k_grid_export, dim3(4096), dim3(256), 0, s, d, m, vec, gp, gt, g0, ng);
}

void launch_sort_multi(const JobStep *dev, const JobStep *host, int njobs, hipStream_t s);

namespace {

// Launches for the jobs of one size class (every grid sized for the largest of them).
void launch_step_run(const JobStep *dev, const JobStep *host, int njobs, hipStream_t s) {
    int stress_grid = 0, pgrid = 8, ugrid = 1;
    for (int j = 0; j < njobs; ++j)
        if (host[j].first || host[j].d.det)
            stress_grid = std::max(stress_grid, (host[j].pa.n + kThreads - 1) / kThreads);
    // the stress pass adds the contribution bound that the sort's bucket scan hands to P2G
    if (stress_grid > 0) hipLaunchKernelGGL(k_stress_multi, dim3(stress_grid, njobs), dim3(kThreads), 0, s, dev);
    launch_sort_multi(dev, host, njobs, s);
    bool any_det = false, any_plain = false;
    for (int j = 0; j < njobs; ++j) {
        const JobStep &J = host[j];
        pgrid = std::max(pgrid, particle_grid(J.d));
        ugrid = std::max(ugrid, J.d.max_blocks < kGridWGs ? J.d.max_blocks : kGridWGs);
        any_det = any_det || J.d.det;
        any_plain = any_plain || !J.d.det;
    }
    if (any_plain) hipLaunchKernelGGL(k_p2g_multi, dim3(pgrid, njobs), dim3(kP2GThreads), 0, s, dev);
    if (any_det) hipLaunchKernelGGL(k_p2g_det_multi, dim3(pgrid, njobs), dim3(kP2GThreads), 0, s, dev);
    if (any_det) hipLaunchKernelGGL(k_det_gather_multi, dim3(ugrid, njobs), dim3(128), 0, s, dev);
    hipLaunchKernelGGL(k_grid_update_multi, dim3(ugrid, njobs), dim3(128), 0, s, dev);
    hipLaunchKernelGGL(k_g2p_multi, dim3(pgrid, njobs), dim3(kG2PThreads), 0, s, dev);
}

int size_class(const JobStep &J) {
    const int w = std::max(particle_grid(J.d), (J.pa.n + kThreads - 1) / kThreads);
    int c = 0;
    while ((1 << c) < w) ++c;
    return c / 2;   // classes four-fold apart: at most 3/4 of a launch's rows are idle
}

}  // namespace

void launch_step_multi(const JobStep *dev, const JobStep *host, int njobs, hipStream_t s) {
    // consecutive entries of one size class share launches, so that small jobs do not
    // run empty workgroups sized for the largest job of the round
    int i0 = 0;
    while (i0 < njobs) {
        int i1 = i0 + 1;
        const int c = size_class(host[i0]);
        while (i1 < njobs && size_class(host[i1]) == c) ++i1;
        launch_step_run(dev + i0, host + i0, i1 - i0, s);
        i0 = i1;
    }
}

void launch_copy_keys(const DevCtx &d, uint32_t *keys, uint32_t *perm, int n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_copy_keys, dim3(1024), dim3(256), 0, s, d, keys, perm, n);
}

}  // namespace ck
