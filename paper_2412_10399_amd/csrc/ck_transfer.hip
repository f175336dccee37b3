// Particle-to-grid transfer, grid update and grid-to-particle transfer of the
// compact-kernel MPM step on the two staggered grids (sections 4.2-4.5 of the
// paper; pipeline order of section 3.2).
//
// Work decomposition: one workgroup per 4^3-cell particle block.  A block's
// particles touch G- nodes [4B, 4B+4] and G+ nodes [4B-1, 4B+4] on each axis
// (5^3 + 6^3 = 341 nodes), so that tile is staged in LDS: P2G accumulates into it
// with LDS float atomics and flushes each nonzero node once to the grid pool with a
// global float atomic; G2P reads the updated velocities of the same tile from LDS.
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

// ---------------------------------------------------------------- P2G
// One particle's contributions to the LDS tile.  Mass w m_p and momentum
//   w (m_p v_p + Q (x_i - x_p)),  Q = (m_p B_p - dt V_p^0 tau_p) D_p^-1,
// which is the APIC affine transfer of section 4.4 plus the MLS stress impulse
// (section 4.5: grad Phi_i = w D^-1 (x_i - x_p), f_i = -V^0 tau grad Phi_i).  In cell
// units x_i - x_p = dx (o - xi) for node offset o on the particle's cell of that grid.
//
// Sorted particles put the ~8 particles of a cell in neighbouring lanes, and all of
// them add to the same 16 nodes.  LDS atomics to one address from several lanes of
// an instruction serialise, so each particle walks its 8 nodes per grid starting at
// an offset given by its rank inside the cell: in any one instruction the lanes of a
// cell hit 8 different nodes.
__device__ __forceinline__ void p2g_particle(const DevCtx &d, const PartArgs &pa, int p, int rank_in_cell_base,
                                             const int *cstart, int bx, int by, int bz, float dt, float *tile,
                                             bool carried_tau) {
    Particle q;
    load_particle(pa, p, q, true);
    CellCoord cc;
    const bool ok = cell_coord(d.geo, q.x, cc);
    if (!ok) {
        set_status(d.counters, ST_DOMAIN);
        return;
    }
    if ((cc.c[0] >> 2) != bx || (cc.c[1] >> 2) != by || (cc.c[2] >> 2) != bz) {
        set_status(d.counters, ST_STALE);
        return;
    }
    const int mi = pa.mat_in ? (int)pa.mat_in[p] : 0;
    const DevMaterial M = d.mats[mi < d.n_mat ? mi : 0];
    Weights w;
    axis_weights(cc, w);
    float Di[9];
    moment_inverse(cc, w, Di);
    float tau[6];
    if (carried_tau) {
#pragma unroll
        for (int i = 0; i < 6; ++i) tau[i] = d.tau[i * d.tau_stride + p];
    } else {
        kirchhoff(M, q.H, tau);
    }
    const float T[9] = {tau[0], tau[3], tau[4], tau[3], tau[1], tau[5], tau[4], tau[5], tau[2]};
    const float k = dt * M.vol0;
    float A[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) A[i] = M.mass * q.B[i] - k * T[i];
    float Q[9];
    const float s = d.geo.inv_dx_f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Q[3 * i + j] = s * (A[3 * i] * Di[j] + A[3 * i + 1] * Di[3 + j] + A[3 * i + 2] * Di[6 + j]);
    const float mv[3] = {M.mass * q.v[0], M.mass * q.v[1], M.mass * q.v[2]};
    const int lcell = ((cc.c[2] & 3) * 4 + (cc.c[1] & 3)) * 4 + (cc.c[0] & 3);
    const int rot = (rank_in_cell_base - cstart[lcell]) & 7;

#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const float *xi = g == 0 ? cc.xm : cc.xp;
        float base[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) base[a] = mv[a] - (Q[3 * a] * xi[0] + Q[3 * a + 1] * xi[1] + Q[3 * a + 2] * xi[2]);
        int t0;
        if (g == 0) {
            t0 = ((cc.c[2] - 4 * bz) * 5 + (cc.c[1] - 4 * by)) * 5 + (cc.c[0] - 4 * bx);
        } else {
            t0 = kTileMinus + ((cc.bp[2] - 4 * bz + 1) * 6 + (cc.bp[1] - 4 * by + 1)) * 6 + (cc.bp[0] - 4 * bx + 1);
        }
        const int sy = g == 0 ? 5 : 6, sz = g == 0 ? 25 : 36;
        // per-axis weights as scalars: lane-dependent choices stay register selects
        const float wx0 = g == 0 ? w.wm[0][0] : w.wp[0][0], wx1 = g == 0 ? w.wm[0][1] : w.wp[0][1];
        const float wy0 = g == 0 ? w.wm[1][0] : w.wp[1][0], wy1 = g == 0 ? w.wm[1][1] : w.wp[1][1];
        const float wz0 = g == 0 ? w.wm[2][0] : w.wp[2][0], wz1 = g == 0 ? w.wm[2][1] : w.wp[2][1];
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int o = (it + rot) & 7;
            const bool ox = o & 1, oy = (o >> 1) & 1, oz = (o >> 2) & 1;
            const float wt = (ox ? wx1 : wx0) * (oy ? wy1 : wy0) * (oz ? wz1 : wz0);
            float m3[3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                m3[a] = base[a] + (ox ? Q[3 * a] : 0.0f) + (oy ? Q[3 * a + 1] : 0.0f) + (oz ? Q[3 * a + 2] : 0.0f);
            const int t = t0 + (ox ? 1 : 0) + (oy ? sy : 0) + (oz ? sz : 0);
            atomicAdd(&tile[t], wt * M.mass);
            atomicAdd(&tile[kTileNodes + t], wt * m3[0]);
            atomicAdd(&tile[2 * kTileNodes + t], wt * m3[1]);
            atomicAdd(&tile[3 * kTileNodes + t], wt * m3[2]);
        }
    }
}

constexpr int kSlots = kMaxBlockParticles / kThreads;   // bucket entries per thread
constexpr uint32_t kIndexMask = (1u << kIndexBits) - 1u;

template <bool PHYSICS, bool CARRIED_TAU>
__global__ void __launch_bounds__(kThreads, 3) k_p2g(DevCtx d, PartArgs pa, float dt) {
    __shared__ float tile[4 * kTileNodes];
    __shared__ uint32_t lbuf[kMaxBlockParticles];
    __shared__ uint32_t ord[kMaxBlockParticles];
    __shared__ int ccount[64];
    __shared__ int cstart[65];
    __shared__ int nbr[27];
    const int np = (int)d.counters[C_NPB];
    const int E = (int)d.counters[C_EPOCH];
    const int tid = threadIdx.x;
    for (int r = blockIdx.x; r < np; r += gridDim.x) {
        const int vb = d.plist[r];
        int bx, by, bz;
        block_coords(d.geo, vb, bx, by, bz);
        const int s = d.pstart[r];
        const int cnt = d.pstart[r + 1] - s;
        if (cnt > kMaxBlockParticles) continue;   // reported by the bucket scan
        // ---- exact order inside the block: by (cell, particle index)
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
            // exclusive scan of the 64 cell counts within one wave
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
                ord[rank] = v & kIndexMask;
                d.perm[s + rank] = v & kIndexMask;
            }
        }
        __syncthreads();
        if (PHYSICS) {
            // ---- scatter into the LDS tile
            load_neighbours(d, bx, by, bz, E, nbr);
            for (int t = tid; t < 4 * kTileNodes; t += kThreads) tile[t] = 0.0f;
            __syncthreads();
            for (int j = tid; j < cnt; j += kThreads)
                p2g_particle(d, pa, (int)ord[j], j, cstart, bx, by, bz, dt, tile, CARRIED_TAU);
            __syncthreads();
            // ---- flush nonzero tile entries to the pool
            for (int t = tid; t < 4 * kTileNodes; t += kThreads) {
                const float val = tile[t];
                if (val == 0.0f) continue;
                const int ch = t / kTileNodes;
                const int ni = t - ch * kTileNodes;
                int g, ix, iy, iz;
                tile_node(ni, bx, by, bz, g, ix, iy, iz);
                const long long a = pool_index(d, nbr, bx, by, bz, g, ix, iy, iz, ch);
                if (a < 0) {
                    set_status(d.counters, ST_CAPACITY);
                    continue;
                }
                atomicAdd(&d.pool[a], val);
            }
            __syncthreads();
        }
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
    for (int r = blockIdx.x; r < np; r += gridDim.x) {
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

int particle_grid(const DevCtx &d) { return d.max_blocks < 8192 ? d.max_blocks : 8192; }

}  // namespace

void launch_p2g(const DevCtx &d, const PartArgs &pa, float dt, bool physics, bool carried_tau, hipStream_t s) {
    if (!physics)
        hipLaunchKernelGGL((k_p2g<false, false>), dim3(particle_grid(d)), dim3(kThreads), 0, s, d, pa, dt);
    else if (carried_tau)
        hipLaunchKernelGGL((k_p2g<true, true>), dim3(particle_grid(d)), dim3(kThreads), 0, s, d, pa, dt);
    else
        hipLaunchKernelGGL((k_p2g<true, false>), dim3(particle_grid(d)), dim3(kThreads), 0, s, d, pa, dt);
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
