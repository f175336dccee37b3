// Shared definitions of the HIP implementation of the compact-kernel MPM step:
// device-side context, particle arguments, and the per-particle FP32 math
// (compact-kernel stencil, moment matrix, constitutive models).  Product code;
// it has no relation to the CPU checker and includes nothing from it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ck {

constexpr int kThreads = 256;           // threads per workgroup of the particle kernels
constexpr int kBlockFloats = 512;       // one pool block: [grid 2][channel 4][64 nodes] floats
constexpr int kMaxMaterials = 8;
constexpr int kMaxBlockParticles = 2048;  // particles one 4^3-cell block may hold (32 per cell on average)
constexpr int kTileMinus = 125;         // G- nodes [4B, 4B+4]^3 touched by the particles of block B
constexpr int kTilePlus = 216;          // G+ nodes [4B-1, 4B+4]^3
constexpr int kTileNodes = kTileMinus + kTilePlus;
constexpr int kCompactChunk = 1024;     // virtual blocks per workgroup in the block compaction
constexpr int kIndexBits = 26;          // particle index bits in the packed (cell, index) sort word

enum StatusBits : uint32_t {
    ST_DOMAIN = 1u,
    ST_CAPACITY = 2u,
    ST_NONFINITE = 4u,
    ST_STALE = 8u,
    ST_CFL = 16u,
};

enum Counter : int {
    C_NPB = 0,      // particle blocks this step
    C_NGB = 1,      // grid blocks of page table 0 (table 1: C_NGB1)
    C_STATUS = 2,   // status bits
    C_EPOCH = 3,    // current activation epoch
    C_MAXPB = 4,    // largest particle count of a block
    C_TOTAL = 5,    // particles placed by the sort
    C_NGB1 = 6,
    C_BOUND_X = 7,  // P2G contribution bound, as X + dt Y (FP32 bit patterns, maxima from bslots):
    C_BOUND_Y = 8,  //   the stress pass's exact form, or headroom times the previous P2G's largest
    C_COUNT = 10
};

__host__ __device__ constexpr int ngb_slot(int table) { return table ? C_NGB1 : C_NGB; }

struct DevMaterial {
    int model;      // 0 fixed corotated, 1 Drucker-Prager
    float mass;     // rho * vol0
    float vol0;
    float mu, lambda;
    float dp_coef;  // (3 lambda + 2 mu) / (2 mu) * alpha,  alpha = sqrt(2/3) 2 sin(phi) / (3 - sin(phi))
};

struct Geometry {
    double origin[3];
    double inv_dx;
    float dx, inv_dx_f;
    int n[3];              // cells per axis
    int NB[3];             // virtual blocks per axis (n/4 + 1)
    int stick_lo[2];       // per grid: a node is inside the walls when lo <= i <= hi on every axis
    int stick_hi[2][3];
    float r_unit[3];       // unit of the packed position remainder (a power of two), see pack_remainder
    float inv_r_unit[3];
};

struct DevCtx {
    Geometry geo;
    int quadratic;         // single-grid quadratic B-spline comparison kernel instead of the compact kernel
    int transfer;          // 0 MLS, 1 APIC with exact kernel gradients, 2 PIC
    DevMaterial mats[kMaxMaterials];
    int n_mat;
    int max_blocks;
    long long nbv;         // number of virtual blocks
    uint32_t *key;         // per particle: block * 64 + cell of the current buffer
    uint16_t *sub;         // per particle: (cell in block) << 3 | half-cell octant, see sub_code
    uint16_t *bsub;        // [max_blocks][kMaxBlockParticles]: sub code of each bucket entry
    uint32_t *bucket;      // [max_blocks][kMaxBlockParticles]: particle indices of each particle
                           // block, in arrival order
    uint32_t *perm;        // exact stable sort order
    int *pflag, *gflag;    // [2][stamp_stride(nbv)] epoch stamps ("holds particles" / "within one block of a
                           // block holding particles"), double-buffered by epoch parity so that
                           // stamping the next step never disturbs readers of the current one
    int *page[2];          // two page tables: per virtual block the physical pool block, or -1
    int *prank;            // per virtual block: rank among the particle blocks
    int *bchg;             // per virtual block: epoch of the last step whose G2P changed the set or the
                           // (octant, cell) bins of its particles (-1: never)
    uint32_t *blo, *bhi;   // per particle block whose order is kept: smallest and largest position of
                           // its particles (the bucket is not filled for such a block)
    int *plist;            // particle blocks in increasing virtual id
    int *nbrs;             // per particle block: pool blocks of its 3 x 3 x 3 neighbourhood in the
                           // step's page table (-1: none), written by P2G and read by G2P
    int *pstart;           // first sorted position of each particle block (+1 sentinel)
    int *bcount;           // particles per particle block
    int *glist[2];         // per page table: virtual id of each physical pool block
    int *chunk_p, *chunk_g;
    float *pool[2];        // two grids of max_blocks * 512 floats (the fused step reads one and
                           // writes the other)
    float *tau;            // [6][max_particles] Kirchhoff stress of the state G2P wrote, at its sorted position
    long long tau_stride;
    unsigned int *counters;
    int det;               // deterministic P2G: block tiles go to `stage`, then a fixed-order gather
    float *stage;          // [max_blocks][4 channels][kTileNodes] per particle block (deterministic mode)
    unsigned int *bslots;  // [2][kBoundSlots][32]: partial maxima of the contribution bound (X, then Y),
                           // one 128-byte line per slot, reduced into the counters by the bucket scan
};

// One of the context's two pools, page tables or block lists: a selection between two
// kernel-argument pointers by a uniform index, which the compiler keeps in scalar
// registers, where an indexed access to the argument would load the pointer from
// memory at every use (a vector load that waits for every load and store before it).
__device__ __forceinline__ float *pool_of(const DevCtx &d, int i) { return i ? d.pool[1] : d.pool[0]; }
__device__ __forceinline__ int *page_of(const DevCtx &d, int i) { return i ? d.page[1] : d.page[0]; }
__device__ __forceinline__ int *glist_of(const DevCtx &d, int i) { return i ? d.glist[1] : d.glist[0]; }

// The material of a particle: a per-lane selection among the context's materials,
// which are read with scalar loads (a uniform address), so that no vector memory
// load -- which would wait for every load issued before it -- stands in a
// particle's arithmetic.  Out-of-range indices take material 0.
__device__ __forceinline__ DevMaterial material_of(const DevCtx &d, int mi) {
    DevMaterial M = d.mats[0];
    for (int i = 1; i < d.n_mat; ++i) {
        const DevMaterial C = d.mats[i];
        const bool take = mi == i;
        M.model = take ? C.model : M.model;
        M.mass = take ? C.mass : M.mass;
        M.vol0 = take ? C.vol0 : M.vol0;
        M.mu = take ? C.mu : M.mu;
        M.lambda = take ? C.lambda : M.lambda;
        M.dp_coef = take ? C.dp_coef : M.dp_coef;
    }
    return M;
}

constexpr int kStageFloats = 4 * kTileNodes;   // one particle block's tile in the deterministic staging area
constexpr int kBoundSlots = 64;                // slots the contribution-bound maxima are spread over
constexpr float kBoundHeadroom = 4.0f;         // next step's bound over this step's largest contribution bound
constexpr int kBoundWords = 2 * kBoundSlots * 32;

// First plane of each field in a particle state buffer (MPM_STATE_PLANES planes):
// position x, velocity v, affine matrix B, H = F - I, position remainder r.
constexpr int kPlaneX = 0, kPlaneV = 3, kPlaneB = 6, kPlaneH = 15, kPlaneR = 24;

struct PartArgs {
    const float *in;       // MPM_STATE_PLANES planes
    float *out;            // MPM_STATE_PLANES planes
    long long stride;
    int n;
    const uint32_t *id_in;
    uint32_t *id_out;
    const uint8_t *mat_in;
    uint8_t *mat_out;
};

// One job's share of a step run for many jobs at once (one launch per phase, row y
// of every grid working on job y): the job's device context and particles, its time
// step and gravity, the page table and pool its sort builds and its P2G, update and
// G2P use, and whether its keys, stamps and stress still have to be formed (first
// step).
struct JobStep {
    DevCtx d;
    PartArgs pa;           // in: this step's state, out: the other buffer
    float dt;
    float g[3];
    int table;
    int first;
};

// ------------------------------------------------------------------ helpers
// Workgroup barrier that orders LDS accesses only: outstanding global stores and
// atomics of the workgroup are not waited for.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Hardware reciprocal and square root (about 1 ulp).  Used where a correctly
// rounded result buys nothing: rotation angles, inverses of well-conditioned
// quantities, normalisations.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ __forceinline__ void set_status(unsigned int *counters, uint32_t bits) {
    atomicOr(&counters[C_STATUS], bits);
}

// Bound, for any time step dt, on every P2G contribution of a particle of mass m and
// initial volume V0 with velocity v, affine matrix B and Kirchhoff stress tau, in the
// form X + dt Y.  The contributions are w m (w <= 1) and w (base + Q t) with t in
// [-1/2, 3/2] per axis, base = m v - Q xi (xi in [0, 1)), Q = (m B - dt V0 tau) D^-1 / dx
// (D in cell units, whose eigenvalues are at least 3/16 - 1/(4 pi) - 1/(4 pi^2) =
// 0.08259, so |D^-1| <= 12.108): per component |base + Q t| <= m |v| + 2.5 sum_b |Q_ab|
// <= m |v| + 2.5 sqrt(3) 12.108 |row a of (m B - dt V0 tau)| / dx.  1% of slack covers
// the FP32 rounding of Q.
__device__ __forceinline__ void contribution_bound_xy(float m, float vol0, float inv_dx, const float v[3],
                                                      const float B[9], const float tau[6], float &X, float &Y) {
    constexpr float kQ = 2.5f * 1.7320508f * 12.108f * 1.01f;
    float vmax = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fabsf(v[2]));
    float b2 = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i) b2 += B[i] * B[i];
    const float t2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2] +
                     2.0f * (tau[3] * tau[3] + tau[4] * tau[4] + tau[5] * tau[5]);
    X = fmaxf(m, m * vmax + kQ * inv_dx * m * __builtin_sqrtf(b2));
    Y = kQ * inv_dx * vol0 * __builtin_sqrtf(t2);
}

// Wave-wide maxima of X and Y into bound slot `slot` (called by every lane; lanes
// without a particle pass zeros).  The maxima of a whole launch would meet at one
// address; spread over kBoundSlots lines they do not queue behind each other.
// Non-finite values are left out (the status word reports them).
__device__ __forceinline__ void wave_bound(unsigned int *bslots, int slot, float X, float Y) {
    X = (X == X && X <= 3.0e38f) ? X : 0.0f;
    Y = (Y == Y && Y <= 3.0e38f) ? Y : 0.0f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        X = fmaxf(X, __shfl_xor(X, off));
        Y = fmaxf(Y, __shfl_xor(Y, off));
    }
    if ((threadIdx.x & 63) == 0) {
        const int k = slot & (kBoundSlots - 1);
        if (X > 0.0f) atomicMax(&bslots[k * 32], __float_as_uint(X));
        if (Y > 0.0f) atomicMax(&bslots[(kBoundSlots + k) * 32], __float_as_uint(Y));
    }
}

__device__ __forceinline__ int vblock_id(const Geometry &g, int bx, int by, int bz) {
    return (bz * g.NB[1] + by) * g.NB[0] + bx;
}

// Stamp array of a given epoch (double buffer indexed by the epoch's parity).
// Each epoch's stamps start at a multiple of 64 entries, so that both halves are
// 256-byte aligned for vector loads.
__host__ __device__ constexpr long long stamp_stride(long long nbv) { return (nbv + 63) / 64 * 64; }
__device__ __forceinline__ int *stamps(int *base, long long nbv, int epoch) {
    return base + (epoch & 1) * stamp_stride(nbv);
}

// Cell of a position on grid G- (particle keys) and the fractional coordinates on
// both grids.  A position is the unevaluated sum x + r of two FP32 numbers (x the
// position rounded to FP32, r the remainder, |r| <= ulp(x)/2).  The integer part is
// taken in FP64 from the FP64 sum x + r, so that it is identical to any FP64
// evaluation of floor((x + r - origin)/dx + 1/4) from that sum.
struct CellCoord {
    int c[3];       // G- cell: nodes c, c+1 of G- carry the particle
    int bp[3];      // G+ base node: nodes bp, bp+1 of G+ carry the particle (bp = c or c-1)
    float xm[3];    // fractional position inside the G- cell, in [0, 1)
    float xp[3];    // fractional position inside the G+ cell, in [0, 1)
};

__device__ __forceinline__ bool cell_coord(const Geometry &g, const float x[3], const float r[3], CellCoord &cc) {
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double X = ((double)x[a] + (double)r[a] - g.origin[a]) * g.inv_dx;
        ok = ok && (X >= 0.25) && (X < (double)g.n[a] - 0.25);
        const double Xm = X + 0.25;
        const double fl = floor(Xm);
        cc.c[a] = (int)fl;
        const double fm = Xm - fl;
        cc.xm[a] = (float)fm;
        if (fm >= 0.5) {
            cc.bp[a] = cc.c[a];
            cc.xp[a] = (float)(fm - 0.5);
        } else {
            cc.bp[a] = cc.c[a] - 1;
            cc.xp[a] = (float)(fm + 0.5);
        }
    }
    return ok;
}

// Advection x + r <- x + r + dt v: the sum is formed in FP64 and split again into
// its FP32 rounding and the FP32 remainder.  An FP32 position alone cannot move by
// less than half its ulp per step (3e-8 at x = 0.5: a particle slower than 1.5e-3
// m/s at dt = 2e-5 would not move at all); the pair resolves the displacement to
// FP32 relative precision.
__device__ __forceinline__ void advance_position(float x, float r, float d, float &xn, float &rn) {
    const double s = ((double)x + (double)r) + (double)d;
    xn = (float)s;
    rn = (float)(s - (double)xn);
}

// The position remainder of the carried state inside an mpm_step sequence: each
// FP32 remainder rounded to a multiple of its axis's unit, 2^-9 of the FP32 ulp of
// the largest coordinate of the domain on that axis, so that |r| <= ulp(x)/2 is at
// most 256 units, and the three stored as 10-bit signed integers in one 32-bit word
// (bits 0-9, 10-19, 20-29).  The position x + r then keeps 2^-10 of the domain's
// largest ulp (about 1e-10 for a unit domain) in 4 bytes instead of 12.  Every
// reader of the word (the next P2G and G2P) takes the same FP64 sum x + r, and the
// G2P that packs it takes the cell key from the packed value too.
__device__ __forceinline__ uint32_t pack_remainder(const Geometry &g, const float r[3]) {
    uint32_t w = 0u;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int q = min(max((int)rintf(r[a] * g.inv_r_unit[a]), -511), 511);
        w |= ((uint32_t)q & 1023u) << (10 * a);
    }
    return w;
}

__device__ __forceinline__ void unpack_remainder(const Geometry &g, uint32_t w, float r[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) r[a] = (float)((int)(w << (22 - 10 * a)) >> 22) * g.r_unit[a];
}

// Position of a particle inside its block: the G- cell (6 bits) and the half of the
// cell it lies in along each axis (bit a set when the G+ base node is c, i.e. the
// upper half; then the particle's G+ nodes are c and c + 1, else c - 1 and c).
__device__ __forceinline__ uint32_t sub_code(const CellCoord &cc) {
    const uint32_t cell = (uint32_t)((cc.c[2] & 3) * 16 + (cc.c[1] & 3) * 4 + (cc.c[0] & 3));
    const uint32_t oct = (uint32_t)(cc.bp[0] == cc.c[0]) | ((uint32_t)(cc.bp[1] == cc.c[1]) << 1) |
                         ((uint32_t)(cc.bp[2] == cc.c[2]) << 2);
    return (cell << 3) | oct;
}

__device__ __forceinline__ uint32_t cell_key(const Geometry &g, const CellCoord &cc) {
    const int vb = vblock_id(g, cc.c[0] >> 2, cc.c[1] >> 2, cc.c[2] >> 2);
    return ((uint32_t)vb << 6) | (uint32_t)((cc.c[2] & 3) * 16 + (cc.c[1] & 3) * 4 + (cc.c[0] & 3));
}

// Per-axis compact-kernel weights (section 4.1 kernel on the two staggered grids).
// On a grid whose cell holds the particle at fractional coordinate xi, the two nodes
// sit at distances xi and 1 - xi (cell units), so their weights are
//   K1(xi) = 1 - xi + s   and   K1(1 - xi) = xi - s,   s = sin(2 pi xi)/(2 pi).
// The G- coordinate is the G+ one shifted by half a cell, so its sine is the
// negative of the G+ sine; one sine per axis serves both grids, and the dual-grid
// cancellations (zero first moment of the pair) then hold exactly in FP32
// whatever the accuracy of the sine.
struct Weights {
    float wm[3][2], wp[3][2];   // G-, G+ weights per axis and node offset
    float sp[3];                // s on G+ (s on G- is -sp)
};

// The sine is the hardware instruction (its argument is in revolutions, so it
// returns sin(2 pi xi) directly); over every FP32 xi in [0, 1) it is within 1.3e-7
// of sin(2 pi xi), i.e. 2e-8 in s, below the FP32 rounding of the weights.
__device__ __forceinline__ void axis_weights(const CellCoord &cc, Weights &w) {
    constexpr float kInv2Pi = 0.15915494309189535f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float s = __builtin_amdgcn_sinf(cc.xp[a]) * kInv2Pi;
        w.sp[a] = s;
        w.wp[a][0] = 1.0f - cc.xp[a] + s;
        w.wp[a][1] = cc.xp[a] - s;
        w.wm[a][0] = 1.0f - cc.xm[a] - s;
        w.wm[a][1] = cc.xm[a] + s;
    }
}

// Moment matrix D_p / dx^2 of section 4.4 and its inverse.  Per axis the two
// weights of grid k have first moment -s_k and second moment
// xi_k (1 - xi_k) - s_k (1 - 2 xi_k) (cell units); the tensor-product kernel makes
// D separable: D_aa = 1/2 sum_k m2_k,a and D_ab = 1/2 sum_k s_k,a s_k,b = sp_a sp_b.
__device__ __forceinline__ void moment_inverse(const CellCoord &cc, const Weights &w, float Di[9]) {
    float d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float s = w.sp[a];
        const float m2p = cc.xp[a] * (1.0f - cc.xp[a]) - s * (1.0f - 2.0f * cc.xp[a]);
        const float m2m = cc.xm[a] * (1.0f - cc.xm[a]) + s * (1.0f - 2.0f * cc.xm[a]);
        d[a] = 0.5f * (m2p + m2m);
    }
    const float o01 = w.sp[0] * w.sp[1], o02 = w.sp[0] * w.sp[2], o12 = w.sp[1] * w.sp[2];
    // symmetric inverse by cofactors (D is SPD with condition number below 2)
    const float c00 = d[1] * d[2] - o12 * o12;
    const float c01 = o02 * o12 - o01 * d[2];
    const float c02 = o01 * o12 - o02 * d[1];
    const float c11 = d[0] * d[2] - o02 * o02;
    const float c12 = o01 * o02 - d[0] * o12;
    const float c22 = d[0] * d[1] - o01 * o01;
    const float inv_det = fast_rcp(d[0] * c00 + o01 * c01 + o02 * c02);
    Di[0] = c00 * inv_det; Di[1] = c01 * inv_det; Di[2] = c02 * inv_det;
    Di[3] = c01 * inv_det; Di[4] = c11 * inv_det; Di[5] = c12 * inv_det;
    Di[6] = c02 * inv_det; Di[7] = c12 * inv_det; Di[8] = c22 * inv_det;
}

// ------------------------------------------------------ constitutive models
// Particle state stores the deformation gradient as H = F - I.  Solids stay close
// to the identity, and an FP32 F near I resolves strains only to about 6e-8
// absolute; H keeps them to FP32 relative precision, and every quantity below is
// formed from H without subtracting numbers close to one.
//
// Both models are isotropic, so everything follows from the eigen-decomposition
// F^T F = V diag(sigma^2) V^T, taken of the small symmetric matrix
//   E = F^T F - I = H + H^T + H^T H  =  V diag(e) V^T,
// so that sigma_i^2 = 1 + e_i, sigma_i - 1 = e_i / (1 + sqrt(1 + e_i)) and
// log sigma_i = log1p(e_i)/2 are all resolved relative to the strain itself.  With
// W = F V = V + H V (columns w_i = F v_i, |w_i| = sigma_i) no explicit U is needed:
//   F = sum_i w_i v_i^T,  U = W diag(1/sigma),  R = W diag(1/sigma) V^T.
// det F < 0 is handled as in the rotation-variant SVD: the smallest singular value
// takes the sign.

struct Eig3 {
    float e[3];     // eigenvalues of F^T F - I, decreasing
    float V[9];     // eigenvectors (columns), row-major storage V[3*row + col]
};

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix (Golub & Van Loan,
// symmetric Schur rotations), fixed number of sweeps (convergence is quadratic:
// four sweeps reach FP32 rounding for 3x3 matrices).
__device__ __forceinline__ void jacobi_rotate(float A[3][3], float V[9], int p, int q) {
    const float apq = A[p][q];
    const float d = A[q][q] - A[p][p];
    // any t gives an exact rotation (c^2 + s^2 = 1 to rounding), so the angle may be
    // computed with hardware reciprocal and square root
    const float den = fabsf(d) + fast_sqrt(d * d + 4.0f * apq * apq);
    const float t = (den > 0.0f) ? (2.0f * apq * (d >= 0.0f ? 1.0f : -1.0f)) * fast_rcp(den) : 0.0f;
    const float c = rsqrtf(1.0f + t * t);
    const float s = t * c;
    A[p][p] -= t * apq;
    A[q][q] += t * apq;
    A[p][q] = A[q][p] = 0.0f;
    const int r = 3 - p - q;
    const float arp = A[r][p], arq = A[r][q];
    A[r][p] = A[p][r] = c * arp - s * arq;
    A[r][q] = A[q][r] = s * arp + c * arq;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float vp = V[3 * i + p], vq = V[3 * i + q];
        V[3 * i + p] = c * vp - s * vq;
        V[3 * i + q] = s * vp + c * vq;
    }
}

__device__ __forceinline__ void strain_eig(const float H[9], Eig3 &r) {
    float A[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            float v = H[3 * i + j] + H[3 * j + i];
#pragma unroll
            for (int k = 0; k < 3; ++k) v += H[3 * k + i] * H[3 * k + j];
            A[i][j] = A[j][i] = v;
        }
#pragma unroll
    for (int i = 0; i < 9; ++i) r.V[i] = (i % 4 == 0) ? 1.0f : 0.0f;
#pragma unroll
    for (int sweep = 0; sweep < 4; ++sweep) {
        jacobi_rotate(A, r.V, 0, 1);
        jacobi_rotate(A, r.V, 0, 2);
        jacobi_rotate(A, r.V, 1, 2);
    }
    float e0 = A[0][0], e1 = A[1][1], e2 = A[2][2];
    // sort decreasing, swapping eigenvector columns alongside
    auto swapcol = [&](int i, int j) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float t = r.V[3 * k + i];
            r.V[3 * k + i] = r.V[3 * k + j];
            r.V[3 * k + j] = t;
        }
    };
    if (e0 < e1) { const float t = e0; e0 = e1; e1 = t; swapcol(0, 1); }
    if (e1 < e2) { const float t = e1; e1 = e2; e2 = t; swapcol(1, 2); }
    if (e0 < e1) { const float t = e0; e0 = e1; e1 = t; swapcol(0, 1); }
    r.e[0] = e0; r.e[1] = e1; r.e[2] = e2;
}

// det F - 1 = det(I + H) - 1 = tr H + ((tr H)^2 - tr(H^2))/2 + det H.
__device__ __forceinline__ float det_minus_one(const float H[9]) {
    const float tr = H[0] + H[4] + H[8];
    const float trH2 = H[0] * H[0] + H[4] * H[4] + H[8] * H[8] + 2.0f * (H[1] * H[3] + H[2] * H[6] + H[5] * H[7]);
    const float detH = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) + H[2] * (H[3] * H[7] - H[4] * H[6]);
    return tr + 0.5f * (tr * tr - trH2) + detH;
}

// W = F V = V + H V
__device__ __forceinline__ void mat_W(const float H[9], const float V[9], float W[9]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            W[3 * i + j] = V[3 * i + j] + (H[3 * i] * V[j] + H[3 * i + 1] * V[3 + j] + H[3 * i + 2] * V[6 + j]);
}

constexpr float kSigmaFloor2 = 1e-8f;   // Drucker-Prager: singular values clamped at 1e-4 before logs

// Kirchhoff stress tau = P F^T (symmetric, stored as 6 values: 00 11 22 01 02 12).
// Fixed corotated (Stomakhin et al. 2012):  tau = 2 mu (F - R) F^T + lambda (J - 1) J I
//   with (F - R) F^T = W diag((sigma - 1)/sigma) W^T.
// Drucker-Prager elastic part (Hencky St. Venant-Kirchhoff, Klar et al. 2016):
//   tau = U diag(2 mu eps + lambda tr eps) U^T = W diag((2 mu eps + lambda tr eps)/sigma^2) W^T.
__device__ __forceinline__ void kirchhoff_eig(const DevMaterial &m, const float H[9], float tau[6]) {
    Eig3 ev;
    strain_eig(H, ev);
    float W[9];
    mat_W(H, ev.V, W);
    const float jm1 = det_minus_one(H);
    const bool inverted = (1.0f + jm1) < 0.0f;
    float coef[3];
    float iso = 0.0f;
    if (m.model == 0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float s2 = fmaxf(1.0f + ev.e[i], 0.0f);
            const float s = fast_sqrt(s2);
            float sm1 = ev.e[i] * fast_rcp(1.0f + s);   // sigma - 1
            float sig = s;
            if (i == 2 && inverted) {
                sig = -s;
                sm1 = -s - 1.0f;
            }
            const float sg = (fabsf(sig) < 1e-12f) ? (sig < 0.0f ? -1e-12f : 1e-12f) : sig;
            coef[i] = 2.0f * m.mu * sm1 * fast_rcp(sg);
        }
        iso = m.lambda * jm1 * (1.0f + jm1);
    } else {
        float eps[3];
        float tr = 0.0f;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float e = (i == 2 && inverted) ? (kSigmaFloor2 - 1.0f) : fmaxf(ev.e[i], kSigmaFloor2 - 1.0f);
            eps[i] = 0.5f * log1pf(e);
            tr += eps[i];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float s2 = fmaxf(1.0f + ev.e[i], 1e-30f);
            coef[i] = (2.0f * m.mu * eps[i] + m.lambda * tr) * fast_rcp(s2);
        }
    }
    // tau = sum_i coef_i w_i w_i^T + iso I
    float t00 = iso, t11 = iso, t22 = iso, t01 = 0.0f, t02 = 0.0f, t12 = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float a = W[i], b = W[3 + i], c = W[6 + i];
        t00 += coef[i] * a * a;
        t11 += coef[i] * b * b;
        t22 += coef[i] * c * c;
        t01 += coef[i] * a * b;
        t02 += coef[i] * a * c;
        t12 += coef[i] * b * c;
    }
    tau[0] = t00; tau[1] = t11; tau[2] = t22; tau[3] = t01; tau[4] = t02; tau[5] = t12;
}

// Drucker-Prager return mapping (Klar et al. 2016) on the trial elastic F = I + H,
// in place on H, returning also the Kirchhoff stress of the result (the next
// step's P2G then needs no decomposition of its own).  eps = log sigma,
// eps_hat = eps - tr(eps)/3:
//   tr eps > 0 or |eps_hat| = 0      -> sigma' = 1 (cone tip: stress free)
//   dgamma = |eps_hat| + c tr(eps) <= 0 -> unchanged (inside the cone)
//   otherwise                          -> eps' = eps - dgamma eps_hat / |eps_hat|
// and F' = sum_i (sigma'_i / sigma_i) w_i v_i^T, i.e.
//   H' = H + sum_i expm1(eps'_i - log sigma_i) w_i v_i^T.
// The left singular vectors u_i = w_i / sigma_i are unchanged by the projection, so
//   tau(F') = sum_i (2 mu eps'_i + lambda tr eps') / sigma_i^2 w_i w_i^T.
__device__ __forceinline__ void dp_return_map_eig(const DevMaterial &m, float H[9], float tau[6]) {
    Eig3 ev;
    strain_eig(H, ev);
    const float jm1 = det_minus_one(H);
    const bool inverted = (1.0f + jm1) < 0.0f;
    // log sigma_i = log1p(e_i)/2; the clamp sigma >= 1e-4 commutes with the monotone log
    constexpr float kLogSigmaFloor = -9.210340371976184f;   // log(1e-4)
    float eps[3], lns[3];
    float tr = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        lns[i] = 0.5f * log1pf(fmaxf(ev.e[i], -1.0f + 1e-30f));
        eps[i] = (i == 2 && inverted) ? kLogSigmaFloor : fmaxf(lns[i], kLogSigmaFloor);
        tr += eps[i];
    }
    float dev[3];
    float dn2 = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        dev[i] = eps[i] - tr * (1.0f / 3.0f);
        dn2 += dev[i] * dev[i];
    }
    const float dn = fast_sqrt(dn2);
    float target[3];
    bool changed = true;
    if (tr > 0.0f || dn == 0.0f) {
        target[0] = target[1] = target[2] = 0.0f;
    } else {
        const float dgamma = dn + m.dp_coef * tr;
        if (dgamma <= 0.0f) {
            changed = false;
#pragma unroll
            for (int i = 0; i < 3; ++i) target[i] = eps[i];
        } else {
            const float k = dgamma * fast_rcp(dn);
#pragma unroll
            for (int i = 0; i < 3; ++i) target[i] = eps[i] - k * dev[i];
        }
    }
    float W[9];
    mat_W(H, ev.V, W);
    // stress of the projected state
    const float trt = target[0] + target[1] + target[2];
    float t00 = 0.0f, t11 = 0.0f, t22 = 0.0f, t01 = 0.0f, t02 = 0.0f, t12 = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float c = (2.0f * m.mu * target[i] + m.lambda * trt) * fast_rcp(fmaxf(1.0f + ev.e[i], 1e-30f));
        const float a = W[i], b = W[3 + i], cc = W[6 + i];
        t00 += c * a * a;
        t11 += c * b * b;
        t22 += c * cc * cc;
        t01 += c * a * b;
        t02 += c * a * cc;
        t12 += c * b * cc;
    }
    tau[0] = t00; tau[1] = t11; tau[2] = t22; tau[3] = t01; tau[4] = t02; tau[5] = t12;
    if (!changed) return;
    float r[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) r[i] = expm1f(target[i] - lns[i]);
    if (inverted) {
        // sigma_3 carries the sign: sigma'_3 / sigma_3 = -exp(target_3) / |sigma_3|
        r[2] = -expf(target[2] - lns[2]) - 1.0f;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            H[3 * i + j] += r[0] * W[3 * i] * ev.V[3 * j] + r[1] * W[3 * i + 1] * ev.V[3 * j + 1] +
                            r[2] * W[3 * i + 2] * ev.V[3 * j + 2];
}

// ------------------------------------------ small-strain series evaluation
// For the strains of solids near rest the eigen-decomposition can be avoided.  With
// the left Cauchy-Green tensor b = F F^T = I + E, E = H + H^T + H H^T, both models
// are functions of E alone, evaluated as matrix power series (all terms are
// polynomials in E, so they commute and stay symmetric):
//   Hencky strain (left frame)   eps = 1/2 log(I + E) = 1/2 (E - E^2/2 + E^3/3 - ...),
//   Drucker-Prager elastic       tau = 2 mu eps + lambda tr(eps) I,
//   fixed corotated              (F - R) F^T = b - b^(1/2) = E/2 + E^2/8 - E^3/16 + 5E^4/128 - ...,
//   return mapping               F' = exp(eps' - eps) F (eps and eps' share eigenvectors),
//                                 tip: F' = exp(-eps) F = R.
// The number of terms is chosen per wave from the largest Frobenius norm r among its
// lanes (a bound on the spectral norm), so that the first omitted term stays below
// FP32 rounding relative to the sum: for the logarithm (and the square-root series,
// whose coefficients are smaller) degree K suffices while r^K / (K+1) <= 6e-8, for
// the exponential while r^K / (K+1)! <= 6e-8.  Strains with r > 0.05 (and inverted
// elements) take the eigen-decomposition path above.
struct Sym3 {
    float xx, yy, zz, xy, xz, yz;
};

// product of two commuting symmetric matrices (the result is symmetric)
__device__ __forceinline__ Sym3 sym_mul(const Sym3 &a, const Sym3 &b) {
    Sym3 r;
    r.xx = a.xx * b.xx + a.xy * b.xy + a.xz * b.xz;
    r.yy = a.xy * b.xy + a.yy * b.yy + a.yz * b.yz;
    r.zz = a.xz * b.xz + a.yz * b.yz + a.zz * b.zz;
    r.xy = a.xx * b.xy + a.xy * b.yy + a.xz * b.yz;
    r.xz = a.xx * b.xz + a.xy * b.yz + a.xz * b.zz;
    r.yz = a.xy * b.xz + a.yy * b.yz + a.yz * b.zz;
    return r;
}

// c0 I + E * acc
__device__ __forceinline__ Sym3 horner_step(float c0, const Sym3 &E, const Sym3 &acc) {
    Sym3 r = sym_mul(E, acc);
    r.xx += c0;
    r.yy += c0;
    r.zz += c0;
    return r;
}

__device__ __forceinline__ Sym3 scaled_identity(float c) { return Sym3{c, c, c, 0.0f, 0.0f, 0.0f}; }

// sum_{k=1..K} c[k] E^k by Horner's rule (K >= 1, the same on every lane of the wave)
__device__ __forceinline__ Sym3 power_series(const Sym3 &E, const float *c, int K) {
    Sym3 acc = scaled_identity(c[K]);
    for (int k = K - 1; k >= 1; --k) acc = horner_step(c[k], E, acc);
    return sym_mul(E, acc);
}

constexpr float kSeriesMax2 = 0.0025f;   // |E|_F^2 <= 0.05^2

// Largest degree needed on the wave: K = kmin + number of thresholds some lane's r^2 exceeds.
__device__ __forceinline__ int wave_terms(float r2, const float *thr2, int n, int kmin) {
    int K = kmin;
    for (int i = 0; i < n; ++i) K += __any(r2 > thr2[i]) ? 1 : 0;
    return K;
}

// r^2 thresholds for degrees 2..6 of the logarithm and 2..5 of the exponential
__device__ __constant__ const float kLogThr2[4] = {1.7e-7f, 3.8e-5f, 5.4e-4f, 1.6e-3f};
__device__ __constant__ const float kExpThr2[3] = {3.6e-7f, 1.28e-4f, 2.7e-3f};
// coefficients, index = degree
__device__ __constant__ const float kLogHalf[7] = {0.0f, 0.5f, -0.25f, 1.0f / 6.0f, -0.125f, 0.1f, -1.0f / 12.0f};
__device__ __constant__ const float kExpm1[6] = {0.0f, 1.0f, 0.5f, 1.0f / 6.0f, 1.0f / 24.0f, 1.0f / 120.0f};
__device__ __constant__ const float kSqrtDiff[7] = {0.0f,           0.5f,           0.125f,        -1.0f / 16.0f,
                                                    5.0f / 128.0f, -7.0f / 256.0f, 21.0f / 1024.0f};

__device__ __forceinline__ Sym3 left_cauchy_green_minus_I(const float H[9]) {
    Sym3 E;
    E.xx = 2.0f * H[0] + H[0] * H[0] + H[1] * H[1] + H[2] * H[2];
    E.yy = 2.0f * H[4] + H[3] * H[3] + H[4] * H[4] + H[5] * H[5];
    E.zz = 2.0f * H[8] + H[6] * H[6] + H[7] * H[7] + H[8] * H[8];
    E.xy = H[1] + H[3] + H[0] * H[3] + H[1] * H[4] + H[2] * H[5];
    E.xz = H[2] + H[6] + H[0] * H[6] + H[1] * H[7] + H[2] * H[8];
    E.yz = H[5] + H[7] + H[3] * H[6] + H[4] * H[7] + H[5] * H[8];
    return E;
}

__device__ __forceinline__ float frob2(const Sym3 &a) {
    return a.xx * a.xx + a.yy * a.yy + a.zz * a.zz + 2.0f * (a.xy * a.xy + a.xz * a.xz + a.yz * a.yz);
}

// 1/2 log(I + E)
__device__ __forceinline__ Sym3 hencky_series(const Sym3 &E, float r2) {
    return power_series(E, kLogHalf, wave_terms(r2, kLogThr2, 4, 2));
}

// exp(X) - I
__device__ __forceinline__ Sym3 expm1_series(const Sym3 &X) {
    return power_series(X, kExpm1, wave_terms(frob2(X), kExpThr2, 3, 2));
}

// H <- H + G (I + H), i.e. F <- (I + G) F
__device__ __forceinline__ void apply_left(const Sym3 &G, float H[9]) {
    const float g[9] = {G.xx, G.xy, G.xz, G.xy, G.yy, G.yz, G.xz, G.yz, G.zz};
    float r[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r[3 * i + j] = H[3 * i + j] + g[3 * i + j] + g[3 * i] * H[j] + g[3 * i + 1] * H[3 + j] + g[3 * i + 2] * H[6 + j];
#pragma unroll
    for (int i = 0; i < 9; ++i) H[i] = r[i];
}

__device__ __forceinline__ void store_tau(const Sym3 &t, float tau[6]) {
    tau[0] = t.xx; tau[1] = t.yy; tau[2] = t.zz; tau[3] = t.xy; tau[4] = t.xz; tau[5] = t.yz;
}

// The path is chosen per wave: if any active lane needs the decomposition, the
// whole wave takes it (both forms agree to FP32 rounding), so no wave runs both.
__device__ __forceinline__ bool wave_needs_eig(float r2, float jm1) {
    return __any(r2 > kSeriesMax2 || 1.0f + jm1 <= 0.0f);
}

__device__ __forceinline__ void kirchhoff(const DevMaterial &m, const float H[9], float tau[6]) {
    const Sym3 E = left_cauchy_green_minus_I(H);
    const float jm1 = det_minus_one(H);
    const float r2 = frob2(E);
    if (wave_needs_eig(r2, jm1)) {
        kirchhoff_eig(m, H, tau);
        return;
    }
    Sym3 t;
    if (m.model == 0) {
        const Sym3 D = power_series(E, kSqrtDiff, wave_terms(r2, kLogThr2, 4, 2));
        const float iso = m.lambda * jm1 * (1.0f + jm1);
        const float k = 2.0f * m.mu;
        t = Sym3{k * D.xx + iso, k * D.yy + iso, k * D.zz + iso, k * D.xy, k * D.xz, k * D.yz};
    } else {
        const Sym3 e = hencky_series(E, r2);
        const float iso = m.lambda * (e.xx + e.yy + e.zz);
        const float k = 2.0f * m.mu;
        t = Sym3{k * e.xx + iso, k * e.yy + iso, k * e.zz + iso, k * e.xy, k * e.xz, k * e.yz};
    }
    store_tau(t, tau);
}

// Series form of the return mapping above.  The three cases differ only in the
// strain correction X (tip: -eps, projection: -k eps_hat, inside the cone: 0), so
// one exponential serves the whole wave: exp(0) - I = 0 leaves H unchanged.
__device__ __forceinline__ void dp_return_map(const DevMaterial &m, float H[9], float tau[6]) {
    const Sym3 E = left_cauchy_green_minus_I(H);
    const float jm1 = det_minus_one(H);
    const float r2 = frob2(E);
    if (wave_needs_eig(r2, jm1)) {
        dp_return_map_eig(m, H, tau);
        return;
    }
    const Sym3 e = hencky_series(E, r2);
    const float tr = e.xx + e.yy + e.zz;
    const float t3 = tr * (1.0f / 3.0f);
    const Sym3 dev{e.xx - t3, e.yy - t3, e.zz - t3, e.xy, e.xz, e.yz};
    const float dn = fast_sqrt(frob2(dev));
    const bool tip = tr > 0.0f || dn == 0.0f;
    const float dgamma = dn + m.dp_coef * tr;
    const bool proj = !tip && dgamma > 0.0f;
    // eps' = eps - k eps_hat: F' = exp(-k eps_hat) F, tau from eps' (same trace)
    const float k = proj ? dgamma * fast_rcp(dn) : 0.0f;
    const Sym3 X = tip ? Sym3{-e.xx, -e.yy, -e.zz, -e.xy, -e.xz, -e.yz}
                       : Sym3{-k * dev.xx, -k * dev.yy, -k * dev.zz, -k * dev.xy, -k * dev.xz, -k * dev.yz};
    if (__any(tip || proj)) apply_left(expm1_series(X), H);
    const float k2 = tip ? 0.0f : 2.0f * m.mu;
    const float iso = tip ? 0.0f : m.lambda * tr;
    store_tau(Sym3{k2 * (e.xx + X.xx) + iso, k2 * (e.yy + X.yy) + iso, k2 * (e.zz + X.zz) + iso, k2 * (e.xy + X.xy),
                   k2 * (e.xz + X.xz), k2 * (e.yz + X.yz)},
              tau);
}

// ------------------------------------------------------------ launchers
}  // namespace ck

struct mpm_ctx;  // host context (ck_api.hip)

namespace ck {

// Device memory source of a context: hipMalloc for stand-alone contexts, the
// server's arena for served jobs.
struct Allocator {
    void *(*alloc)(void *self, size_t bytes);
    void (*free)(void *self, void *p);
    void *self;
};

void launch_flag_keys(const DevCtx &d, const PartArgs &pa, int epoch_offset, hipStream_t s);
void launch_clear_flags(const DevCtx &d, hipStream_t s);
void launch_compact(const DevCtx &d, int table, hipStream_t s);
// reuse: as for launch_p2g (blocks whose order the P2G keeps get their position range
// instead of a filled bucket)
void launch_bucket(const DevCtx &d, int n, int zero_pool, int zero_table, hipStream_t s, bool reuse = false);
void launch_block_sort(const DevCtx &d, hipStream_t s);
void launch_stress(const DevCtx &d, const PartArgs &pa, hipStream_t s);
// carried: the B planes of pa.in hold Q, the first remainder plane the packed remainder,
// and there is no carried stress (the state an mpm_step G2P with carry left for the
// next step)
// reuse: the input is the state the context's previous G2P wrote, whose blocks' orders
// the P2G may keep where that G2P changed nothing (see DevCtx::bchg)
void launch_p2g(const DevCtx &d, const PartArgs &pa, float dt, int gp, int gt, hipStream_t s, bool carried = false,
                bool reuse = false);
void launch_grid_update(const DevCtx &d, float dt, const float gravity[3], int gp, int gt, hipStream_t s);
void launch_det_gather(const DevCtx &d, int gp, int gt, hipStream_t s);
// carry: write the carried state (Q = (m B - dt V0 tau) D^-1 / dx in the B planes and no
// stress, the packed remainder) for a P2G with `carried` that follows in the same step
// sequence; carried: the input is such a state
void launch_g2p(const DevCtx &d, const PartArgs &pa, float dt, int gp, int gt, hipStream_t s, bool carry = false,
                bool carried = false);
void launch_grid_export(const DevCtx &d, float *m, float *vec, int gp, int gt, int g0, int ng, hipStream_t s);
void launch_block_order(const DevCtx &d, hipStream_t s);
void launch_g2p2g(const DevCtx &d, const PartArgs &pa, float dt, int gp_in, int gt_in, int gp_out, int gt_out,
                  hipStream_t s);
void launch_zero_pool(const DevCtx &d, int gp, int gt, hipStream_t s);
void launch_copy_keys(const DevCtx &d, uint32_t *keys, uint32_t *perm, int n, hipStream_t s);
// Every phase of one step for `njobs` jobs (host copy `host`, the same table already
// enqueued to `dev`), compact-kernel MLS jobs only: one launch per phase for each run
// of consecutive entries of one size class, sized for the largest job of the run.
void launch_step_multi(const JobStep *dev, const JobStep *host, int njobs, hipStream_t s);

}  // namespace ck
