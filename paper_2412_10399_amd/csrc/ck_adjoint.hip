// Differentiable compact-kernel MPM step: forward step on dense or block-sparse grids
// and its exact reverse mode (vector-Jacobian product), one thread per particle or node.
//
// Forward, for particle p at X = (x - origin)/dx (cell units), on grid G_k
// (k = -1 for G-, +1 for G+, node i at i + k/4 cells), per axis a:
//   xi = X_a - k/4 - floor(X_a - k/4), weights of the two nodes
//   w0 = K1(xi) = 1 - xi + s,  w1 = K1(1 - xi) = xi - s,  s = sin(2 pi xi)/(2 pi),
//   dw0/dX = cos(2 pi xi) - 1,  dw1/dX = 1 - cos(2 pi xi)        (section 4.1 kernel);
// w_i is the product over the axes, d_i = x_i - x_p;
//   D = 1/2 sum_k sum_i w d d^T  (section 4.4; per axis the first moment on grid k
//       is -s dx and the second (xi (1 - xi) - s (1 - 2 xi)) dx^2),
//   P2G: m_i += w m,  p_i += w (m v + Q d),  Q = (m B - dt V0 tau) D^-1    (4.3, 4.5),
//   grid: v~ = p/m + dt g where m > 0 and the node is inside the walls, else 0,
//   G2P: v' = 1/2 sum w v~,  B' = 1/2 sum w v~ d^T,  F' = (I + dt B' D^-1) F,
//        x' = x + dt v',
//   tau = 2 mu (F - R) F^T + lambda (J - 1) J I  (fixed corotated), mu and lambda
//   proportional to E = exp(logE).
// Reverse: the three phases in the opposite order, each product rule written out
// next to the line that applies it.
#include "../../include/ckmpm_adjoint.h"
#include "ck_common.hpp"
#include "ck_ctx.hpp"

#include <algorithm>
#include <cmath>
#include <new>

#include <climits>

using namespace ck;

struct mpm_ad_ctx {
    int device = 0;
    Geometry geo;
    float gravity[3];
    float nu, rho, vol0;
    int64_t max_particles = 0;
    int cap = 0;              // pool slots per grid (blocks of 4x4x4 nodes)
    int nb[3] = {0, 0, 0};    // blocks per axis covering the (n+1)^3 node lattice
    long long nbv = 0;        // nb[0] nb[1] nb[2]
    long long nodes = 0;      // nodes of one grid: (n+1)^3 when direct, else (cap + 1) * 64
                              // (pool slots, the last a spill slot)
    float *grid = nullptr;    // 14 planes of 2 * nodes floats, see below
    int *page = nullptr;      // [grid][nbv]: pool slot of a block in this call, -1 if untouched
    int *blist = nullptr;     // [grid][cap]: block of a slot
    bool direct = false;      // max_blocks covers the lattice: dense grids, no marking
    unsigned char *flag = nullptr;   // [grid][nbv]: touched by a particle's stencil
    unsigned int *cnt = nullptr;     // [2]: slots taken per grid
    unsigned int *status = nullptr;
};

namespace {

// Grids.  When max_blocks covers every 4x4x4-node block of the lattice (`direct`),
// the grids are dense, node (ix, iy, iz) at (iz ny + iy) nx + ix, and the sweeps run
// over all nodes.  Otherwise they are block-sparse: each call marks the blocks that
// its particles' stencils touch (k_ad_mark) and gives them pool slots (k_ad_alloc);
// the node lives at page[g][block] * 64 + ((iz & 3) * 4 + (iy & 3)) * 4 + (ix & 3),
// and the sweeps run over the taken slots only.  Past the pool's capacity a block
// gets the spill slot `cap` (never swept, its values meaningless) and the call
// reports ST_CAPACITY.
// Planes of the pool buffer (each 2 * nodes floats: G- then G+):
enum GridPlane { GM = 0, GP = 1, GV = 4, GVB = 7, GMB = 10, GPB = 11, kGridPlanes = 14 };

struct AdArgs {
    Geometry geo;
    float g[3];
    float mass, vol0, nu_mu, nu_lambda;   // mu = nu_mu E, lambda = nu_lambda E
    int nx, ny;   // lattice nodes per axis (direct)
    int nbx, nby, cap;
    long long nbv, nodes;
    float *grid;
    int *page, *blist;
    int direct;
    unsigned char *flag;
    unsigned int *cnt;
    unsigned int *status;
    int n;
    long long stride;
    float dt;
};

__device__ __forceinline__ float *plane(const AdArgs &a, int k) { return a.grid + (long long)k * 2 * a.nodes; }

// Sets status bits in the context's one status word (read by mpm_ad_sync).
__device__ __forceinline__ void ad_status(const AdArgs &a, unsigned int bits) { atomicOr(a.status, bits); }

// Index of node (ix, iy, iz) of grid g in the grid planes: dense, or in the pool
// (kSparse; the node's block was marked by this call).
template <bool kSparse>
__device__ __forceinline__ long long ad_index(const AdArgs &a, int g, int ix, int iy, int iz) {
    if (!kSparse) return g * a.nodes + ((long long)iz * a.ny + iy) * a.nx + ix;
    const long long b = ((long long)(iz >> 2) * a.nby + (iy >> 2)) * a.nbx + (ix >> 2);
    const int slot = a.page[g * a.nbv + b];
    return g * a.nodes + (long long)slot * 64 + (((iz & 3) * 4 + (iy & 3)) * 4 + (ix & 3));
}

// Node coordinates of local node l of pool slot `slot` of grid g (block-sparse).
__device__ __forceinline__ void ad_coords(const AdArgs &a, int g, int slot, int l, int &ix, int &iy, int &iz) {
    const int b = a.blist[(long long)g * a.cap + slot];
    const int bxy = a.nbx * a.nby;
    iz = 4 * (b / bxy) + (l >> 4);
    iy = 4 * ((b % bxy) / a.nbx) + ((l >> 2) & 3);
    ix = 4 * (b % a.nbx) + (l & 3);
}

// ------------------------------------------------------------ particle stencil
struct AdStencil {
    int base[2][3];     // node base + o (o = 0, 1) on grid g, axis a
    float w[2][3][2];   // per-axis weights
    float dw[2][3][2];  // their derivatives with respect to X_a (cell units)
    float s[2][3], c[2][3], xi[2][3];
    float Dinv[9];      // D^-1 in world units
};

// X = (x + r - origin) / dx (the position is x + r, FP32 rounding and remainder,
// summed in FP64); false when the particle is outside the valid domain.
__device__ __forceinline__ bool ad_position(const AdArgs &a, const float x[3], const float r[3], float X[3]) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        X[ax] = (float)(((double)x[ax] + (double)r[ax] - a.geo.origin[ax]) * a.geo.inv_dx);
        if (!(X[ax] >= 0.25f && X[ax] < (float)a.geo.n[ax] - 0.25f)) return false;
    }
    return true;
}

// False (and nothing filled in) when the particle is outside the valid domain.
__device__ __forceinline__ bool ad_stencil(const AdArgs &a, const float x[3], const float r[3], AdStencil &st) {
    constexpr float kInv2Pi = 0.15915494309189535f;
    float X[3];
    if (!ad_position(a, x, r, X)) return false;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const float k = g == 0 ? -0.25f : 0.25f;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const float Xk = X[ax] - k;
            const float b = floorf(Xk);
            const float xi = Xk - b;
            st.base[g][ax] = (int)b;
            const float s = __builtin_amdgcn_sinf(xi) * kInv2Pi;   // argument in revolutions
            const float c = __builtin_amdgcn_cosf(xi);
            st.xi[g][ax] = xi;
            st.s[g][ax] = s;
            st.c[g][ax] = c;
            st.w[g][ax][0] = 1.0f - xi + s;
            st.w[g][ax][1] = xi - s;
            st.dw[g][ax][0] = c - 1.0f;
            st.dw[g][ax][1] = 1.0f - c;
        }
    }
    // D / dx^2: diagonal 1/2 sum_k (xi (1 - xi) - s (1 - 2 xi)), off-diagonal
    // 1/2 sum_k s_a s_b (the first moments are -s on each grid)
    float Dh[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float v = 0.0f;
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                if (i == j) {
                    const float xi = st.xi[g][i];
                    v += 0.5f * (xi * (1.0f - xi) - st.s[g][i] * (1.0f - 2.0f * xi));
                } else {
                    v += 0.5f * st.s[g][i] * st.s[g][j];
                }
            }
            Dh[3 * i + j] = v;
        }
    // inverse by cofactors (D is symmetric positive definite, condition number < 2)
    const float c00 = Dh[4] * Dh[8] - Dh[5] * Dh[7], c01 = Dh[5] * Dh[6] - Dh[3] * Dh[8],
                c02 = Dh[3] * Dh[7] - Dh[4] * Dh[6];
    const float c11 = Dh[0] * Dh[8] - Dh[2] * Dh[6], c12 = Dh[2] * Dh[3] - Dh[0] * Dh[5];
    const float c22 = Dh[0] * Dh[4] - Dh[1] * Dh[3];
    const float det = Dh[0] * c00 + Dh[1] * c01 + Dh[2] * c02;
    const float sc = a.geo.inv_dx_f * a.geo.inv_dx_f / det;
    st.Dinv[0] = c00 * sc; st.Dinv[1] = c01 * sc; st.Dinv[2] = c02 * sc;
    st.Dinv[3] = c01 * sc; st.Dinv[4] = c11 * sc; st.Dinv[5] = c12 * sc;
    st.Dinv[6] = c02 * sc; st.Dinv[7] = c12 * sc; st.Dinv[8] = c22 * sc;
    return true;
}

// Node o (bits x, y, z) of grid g: weight, d = x_i - x_p (world) and the gradient
// of the weight with respect to x_p (world).
__device__ __forceinline__ void ad_weights(const AdArgs &a, const AdStencil &st, int g, int o, float &w, float d[3],
                                           float gw[3]) {
    const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
    const int off[3] = {ox, oy, oz};
    float wa[3], dwa[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        wa[ax] = st.w[g][ax][off[ax]];
        dwa[ax] = st.dw[g][ax][off[ax]] * a.geo.inv_dx_f;
        d[ax] = ((float)off[ax] - st.xi[g][ax]) * a.geo.dx;
    }
    w = wa[0] * wa[1] * wa[2];
    gw[0] = dwa[0] * wa[1] * wa[2];
    gw[1] = wa[0] * dwa[1] * wa[2];
    gw[2] = wa[0] * wa[1] * dwa[2];
}

// The same and the node's pool index.
template <bool kSparse>
__device__ __forceinline__ long long ad_node(const AdArgs &a, const AdStencil &st, int g, int o, float &w, float d[3],
                                             float gw[3]) {
    ad_weights(a, st, g, o, w, d, gw);
    return ad_index<kSparse>(a, g, st.base[g][0] + (o & 1), st.base[g][1] + ((o >> 1) & 1), st.base[g][2] + (o >> 2));
}

// Adds to xb the adjoint of D(x_p) for Db = dL/dD (world units):
//   dD/dx_a = dx dD^/dX_a,  dD^_aa/dX_a = 1/2 sum_k ((1 - 2 xi)(1 - c) + 2 s),
//   dD^_ab/dX_a = 1/2 sum_k c_a s_b  (b != a);  other entries do not depend on X_a.
__device__ __forceinline__ void ad_moment_vjp(const AdArgs &a, const AdStencil &st, const float Db[9], float xb[3]) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        float acc = 0.0f;
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const float xi = st.xi[g][ax], c = st.c[g][ax], s = st.s[g][ax];
            acc += Db[4 * ax] * 0.5f * ((1.0f - 2.0f * xi) * (1.0f - c) + 2.0f * s);
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (b != ax) acc += (Db[3 * ax + b] + Db[3 * b + ax]) * 0.5f * c * st.s[g][b];
        }
        xb[ax] += a.geo.dx * acc;
    }
}

// dL/dD from dL/dD^-1: d(D^-1) = -D^-1 dD D^-1, so Db = -D^-T Dib D^-T (D^-1 symmetric).
__device__ __forceinline__ void ad_inverse_vjp(const float Di[9], const float Dib[9], float Db[9]) {
    float t[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) t[3 * i + j] = Dib[3 * i] * Di[j] + Dib[3 * i + 1] * Di[3 + j] + Dib[3 * i + 2] * Di[6 + j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Db[3 * i + j] = -(Di[3 * i] * t[j] + Di[3 * i + 1] * t[3 + j] + Di[3 * i + 2] * t[6 + j]);
}

// ------------------------------------------------------------ fixed corotated
// Polar pieces of F = I + H from the eigen-decomposition of F^T F - I (Jacobi):
// V, signed singular values (the smallest negative for an inverted element),
// U = F V diag(1/s), R = U V^T.
struct Polar {
    float U[9], V[9], R[9], s[3];
    float J;
};

__device__ __forceinline__ void ad_polar(const float H[9], Polar &P) {
    Eig3 ev;
    strain_eig(H, ev);
    float W[9];
    mat_W(H, ev.V, W);
    const float J = 1.0f + det_minus_one(H);
    P.J = J;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float s = fast_sqrt(fmaxf(1.0f + ev.e[i], 1e-30f));
        if (i == 2 && J < 0.0f) s = -s;
        P.s[i] = s;
        const float inv = 1.0f / s;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            P.U[3 * r + i] = W[3 * r + i] * inv;
            P.V[3 * r + i] = ev.V[3 * r + i];
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            P.R[3 * i + j] = P.U[3 * i] * P.V[3 * j] + P.U[3 * i + 1] * P.V[3 * j + 1] + P.U[3 * i + 2] * P.V[3 * j + 2];
}

// tau = 2 mu (F - R) F^T + lambda (J - 1) J I with (F - R) F^T = W diag((s - 1)/s) W^T,
// W = F V, s - 1 formed from e = s^2 - 1 without cancellation.
__device__ __forceinline__ void ad_tau(const float H[9], const Polar &P, float mu, float lam, float tau[9]) {
    float coef[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float s = P.s[i];
        const float e = s * s - 1.0f;
        const float sm1 = s > 0.0f ? e / (1.0f + s) : s - 1.0f;
        coef[i] = 2.0f * mu * sm1 / s;
    }
    const float iso = lam * (P.J - 1.0f) * P.J;
    // W_i = s_i U_i
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float v = (r == c) ? iso : 0.0f;
#pragma unroll
            for (int i = 0; i < 3; ++i) v += coef[i] * P.s[i] * P.s[i] * P.U[3 * r + i] * P.U[3 * c + i];
            tau[3 * r + c] = v;
        }
    (void)H;
}

// Fb += dL/dF for tb = dL/dtau:
//   dtau = 2 mu (dF F^T + F dF^T - dR F^T - R dF^T) + lambda (2J - 1) dJ I,
//   so Fb = 2 mu (tb F + tb^T F - tb^T R) + lambda (2J - 1) tr(tb) cof F, and
//   Rb = -2 mu tb F enters through dR = U M V^T, M_ij = (A_ij - A_ji)/(s_i + s_j),
//   A = U^T dF V:  Fb += U Z V^T,  Z_ij = (Y_ij - Y_ji)/(s_i + s_j),  Y = U^T Rb V.
__device__ __forceinline__ void ad_tau_vjp(const float H[9], const Polar &P, float mu, float lam, const float tb[9],
                                           float Fb[9]) {
    float F[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) F[i] = H[i] + ((i % 4 == 0) ? 1.0f : 0.0f);
    float tF[9], tTF[9], tTR[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float a = 0.0f, b = 0.0f, c = 0.0f;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                a += tb[3 * i + k] * F[3 * k + j];
                b += tb[3 * k + i] * F[3 * k + j];
                c += tb[3 * k + i] * P.R[3 * k + j];
            }
            tF[3 * i + j] = a;
            tTF[3 * i + j] = b;
            tTR[3 * i + j] = c;
        }
    // Y = U^T Rb V with Rb = -2 mu tb F
    float RbV[9], Y[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            RbV[3 * i + j] = -2.0f * mu * (tF[3 * i] * P.V[j] + tF[3 * i + 1] * P.V[3 + j] + tF[3 * i + 2] * P.V[6 + j]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Y[3 * i + j] = P.U[i] * RbV[j] + P.U[3 + i] * RbV[3 + j] + P.U[6 + i] * RbV[6 + j];
    float Z[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Z[3 * i + j] = (i == j) ? 0.0f : (Y[3 * i + j] - Y[3 * j + i]) / (P.s[i] + P.s[j]);
    // cofactor matrix of F
    float cof[9];
    cof[0] = F[4] * F[8] - F[5] * F[7];
    cof[1] = F[5] * F[6] - F[3] * F[8];
    cof[2] = F[3] * F[7] - F[4] * F[6];
    cof[3] = F[2] * F[7] - F[1] * F[8];
    cof[4] = F[0] * F[8] - F[2] * F[6];
    cof[5] = F[1] * F[6] - F[0] * F[7];
    cof[6] = F[1] * F[5] - F[2] * F[4];
    cof[7] = F[2] * F[3] - F[0] * F[5];
    cof[8] = F[0] * F[4] - F[1] * F[3];
    const float jc = lam * (2.0f * P.J - 1.0f) * (tb[0] + tb[4] + tb[8]);
    // U Z V^T
    float ZV[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) ZV[3 * i + j] = Z[3 * i] * P.V[3 * j] + Z[3 * i + 1] * P.V[3 * j + 1] + Z[3 * i + 2] * P.V[3 * j + 2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float uzv = P.U[3 * i] * ZV[j] + P.U[3 * i + 1] * ZV[3 + j] + P.U[3 * i + 2] * ZV[6 + j];
            Fb[3 * i + j] += 2.0f * mu * (tF[3 * i + j] + tTF[3 * i + j] - tTR[3 * i + j]) + uzv + jc * cof[3 * i + j];
        }
}

__device__ __forceinline__ void load_planes(const float *base, long long stride, int p, int first, int count, float *out) {
    for (int i = 0; i < count; ++i) out[i] = base[(first + i) * stride + p];
}

// ------------------------------------------------------------ workgroup node tiles
// The two scattering kernels accumulate into a 64-bit fixed-point LDS tile over the
// node box of their workgroup's 256 particles (both grids), then add every nonzero
// node to the grid with one float atomic per channel.  Particles keep their
// creation order, cell by cell, so consecutive particles sit in neighbouring cells
// and the box is small (a row of about 34 x 3 x 3 nodes for the box workload); a
// workgroup whose box does not fit adds its contributions to the grid directly.
// Integer sums are exact; the unit is 2^-39 of the largest contribution bound of
// the workgroup, so a node's sum of at most 256 contributions stays below 2^48.
constexpr int kAdTileWords = 5120;   // 40 KiB

struct AdTile {
    unsigned long long *w;   // [channel][grid][T]
    int lo[3], L[3], T;
    bool on;
    double S;
};

// round(v S) as a two's-complement 64-bit integer (|v S| < 2^51): in [2^52, 2^53) the
// FP64 numbers are the integers, so magic + v S carries it in its low bits.
__device__ __forceinline__ unsigned long long ad_fixed(float v, double S) {
    constexpr double kMagic = 6755399441055744.0;   // 1.5 * 2^52
    return (unsigned long long)(__double_as_longlong(fma((double)v, S, kMagic)) - 0x4338000000000000LL);
}

// Called by every thread of the workgroup: node box of the valid particles'
// stencils on both grids, scale from the largest bound `bnd`, tile of `nch`
// channels cleared when it fits.  sh: 7 ints of LDS.
__device__ void ad_tile_begin(bool valid, const AdStencil &st, float bnd, int nch, unsigned long long *words, int *sh,
                              AdTile &t) {
    const int tid = threadIdx.x;
    if (tid < 3) sh[tid] = INT_MAX;
    else if (tid < 6) sh[tid] = INT_MIN;
    else if (tid == 6) sh[6] = 0;
    __syncthreads();
    if (valid) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            atomicMin(&sh[ax], min(st.base[0][ax], st.base[1][ax]));
            atomicMax(&sh[3 + ax], max(st.base[0][ax], st.base[1][ax]) + 1);
        }
    }
    float b = valid ? bnd : 0.0f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) b = fmaxf(b, __shfl_xor(b, off));
    if ((tid & 63) == 0) atomicMax(reinterpret_cast<unsigned int *>(&sh[6]), __float_as_uint(b));
    __syncthreads();
    t.w = words;
    long long T = 1;
    bool on = sh[0] <= sh[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        t.lo[ax] = sh[ax];
        t.L[ax] = on ? sh[3 + ax] - sh[ax] + 1 : 0;
        T *= t.L[ax];
    }
    on = on && 2 * T * nch <= kAdTileWords;
    t.on = on;
    t.T = on ? (int)T : 0;
    const float m = __uint_as_float((unsigned int)sh[6]);
    t.S = m > 0.0f ? ldexp(1.0, 39 - ilogbf(m)) : 1.0;
    if (on)
        for (int q = tid; q < 2 * t.T * nch; q += blockDim.x) words[q] = 0ull;
    __syncthreads();
}

// Adds v to channel ch of node (ix, iy, iz) of grid g (pool index id): into the tile,
// or straight into plane plane0 + ch of the grid when the tile is off.
__device__ __forceinline__ void ad_tile_add(const AdArgs &a, const AdTile &t, int plane0, int ch, int g, int ix, int iy,
                                            int iz, long long id, float v) {
    if (t.on) {
        const int r = ((iz - t.lo[2]) * t.L[1] + (iy - t.lo[1])) * t.L[0] + (ix - t.lo[0]);
        atomicAdd(&t.w[(ch * 2 + g) * t.T + r], ad_fixed(v, t.S));
    } else {
        atomicAdd(&plane(a, plane0 + ch)[id], v);
    }
}

// Called by every thread after its adds: every nonzero tile node to the grid.
template <bool kSparse>
__device__ void ad_tile_flush(const AdArgs &a, const AdTile &t, int plane0, int nch) {
    __syncthreads();
    if (!t.on) return;
    const double inv = 1.0 / t.S;
    const int LxLy = t.L[0] * t.L[1];
    for (int q = threadIdx.x; q < 2 * t.T; q += blockDim.x) {
        const int g = q >= t.T ? 1 : 0, r = q - g * t.T;
        const int ix = t.lo[0] + r % t.L[0], iy = t.lo[1] + (r / t.L[0]) % t.L[1], iz = t.lo[2] + r / LxLy;
        long long id = -1;   // looked up for a touched node only (its block is marked)
        for (int ch = 0; ch < nch; ++ch) {
            const long long v = (long long)t.w[(ch * 2 + g) * t.T + r];
            if (v == 0) continue;
            if (id < 0) id = ad_index<kSparse>(a, g, ix, iy, iz);
            atomicAdd(&plane(a, plane0 + ch)[id], (float)((double)v * inv));
        }
    }
}

// ------------------------------------------------------------ kernels
// P2G through the workgroup's node tile (direct float atomics when it does not fit).
template <bool kSparse>
__global__ void __launch_bounds__(256) k_ad_p2g(AdArgs a, const float *state, const float *logE) {
    __shared__ unsigned long long tw[kAdTileWords];
    __shared__ int sh[8];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    float x[3], v[3], Q[9];
    AdStencil st;
    bool valid = false;
    if (p < a.n) {
        float B[9], H[9], xr[3];
        load_planes(state, a.stride, p, 0, 3, x);
        load_planes(state, a.stride, p, 3, 3, v);
        load_planes(state, a.stride, p, 6, 9, B);
        load_planes(state, a.stride, p, 15, 9, H);
        load_planes(state, a.stride, p, kPlaneR, 3, xr);
        valid = ad_stencil(a, x, xr, st);
        if (!valid) {
            ad_status(a, ST_DOMAIN);
        } else {
            const float E = expf(logE[p]);
            Polar P;
            ad_polar(H, P);
            float tau[9];
            ad_tau(H, P, a.nu_mu * E, a.nu_lambda * E, tau);
            float A[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) A[i] = a.mass * B[i] - a.dt * a.vol0 * tau[i];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Q[3 * i + j] = A[3 * i] * st.Dinv[j] + A[3 * i + 1] * st.Dinv[3 + j] + A[3 * i + 2] * st.Dinv[6 + j];
        }
    }
    // |w m| <= m and |w (m v + Q d)| <= |m v| + dx sum |Q| (w <= 1, |d_b| <= dx)
    float bnd = 0.0f;
    if (valid) {
        bnd = a.mass;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax)
            bnd = fmaxf(bnd, fabsf(a.mass * v[ax]) +
                                 a.geo.dx * (fabsf(Q[3 * ax]) + fabsf(Q[3 * ax + 1]) + fabsf(Q[3 * ax + 2])));
    }
    AdTile t;
    ad_tile_begin(valid, st, bnd, 4, tw, sh, t);
    if (valid) {
        for (int g = 0; g < 2; ++g)
            for (int o = 0; o < 8; ++o) {
                float w, d[3], gw[3];
                ad_weights(a, st, g, o, w, d, gw);
                const int ix = st.base[g][0] + (o & 1), iy = st.base[g][1] + ((o >> 1) & 1), iz = st.base[g][2] + (o >> 2);
                const long long id = t.on ? 0 : ad_index<kSparse>(a, g, ix, iy, iz);   // the tile's flush looks it up
                ad_tile_add(a, t, GM, 0, g, ix, iy, iz, id, w * a.mass);
#pragma unroll
                for (int ax = 0; ax < 3; ++ax)
                    ad_tile_add(a, t, GM, 1 + ax, g, ix, iy, iz, id,
                                w * (a.mass * v[ax] + Q[3 * ax] * d[0] + Q[3 * ax + 1] * d[1] + Q[3 * ax + 2] * d[2]));
            }
    }
    ad_tile_flush<kSparse>(a, t, GM, 4);
}

// Marks the blocks of the nodes a valid particle's stencil reaches on both grids
// (nodes base and base + 1 per axis, base = floor(X - k/4) as in ad_stencil).
// Also zeroes the slot counters that k_ad_alloc then counts up.
__global__ void __launch_bounds__(256) k_ad_mark(AdArgs a, const float *state) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) {
        a.cnt[0] = 0u;
        a.cnt[1] = 0u;
    }
    if (p >= a.n) return;
    float x[3], xr[3], X[3];
    load_planes(state, a.stride, p, 0, 3, x);
    load_planes(state, a.stride, p, kPlaneR, 3, xr);
    if (!ad_position(a, x, xr, X)) return;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const float k = g == 0 ? -0.25f : 0.25f;
        int lo[3], hi[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const float Xk = X[ax] - k;
            const int b = (int)floorf(Xk);
            lo[ax] = b >> 2;
            hi[ax] = (b + 1) >> 2;
        }
        for (int bz = lo[2]; bz <= hi[2]; ++bz)
            for (int by = lo[1]; by <= hi[1]; ++by)
                for (int bx = lo[0]; bx <= hi[0]; ++bx)
                    a.flag[g * a.nbv + ((long long)bz * a.nby + by) * a.nbx + bx] = 1;
    }
}

// One thread per block of grid blockIdx.y: a marked block takes the grid's next pool
// slot (one counter update per wave) and is recorded in blist; its flag is cleared.
// Every block's page entry is rewritten (-1 for an untouched one).
__global__ void __launch_bounds__(256) k_ad_alloc(AdArgs a) {
    const int g = blockIdx.y;
    const long long b = blockIdx.x * 256LL + threadIdx.x;
    const bool in = b < a.nbv;
    const bool f = in && a.flag[g * a.nbv + b] != 0;
    const unsigned long long m = __ballot(f);
    if (m == 0ull) {
        if (in) a.page[g * a.nbv + b] = -1;
        return;
    }
    const int lane = threadIdx.x & 63, leader = __builtin_ctzll(m);
    unsigned int base = 0u;
    if (lane == leader) base = atomicAdd(&a.cnt[g], (unsigned int)__popcll(m));
    base = __shfl(base, leader);
    if (!in) return;
    int slot = -1;
    if (f) {
        const unsigned int s = base + (unsigned int)__popcll(m & ((1ull << lane) - 1ull));
        if (s < (unsigned int)a.cap) {
            slot = (int)s;
            a.blist[(long long)g * a.cap + s] = (int)b;
        } else {
            slot = a.cap;
            ad_status(a, ST_CAPACITY);
        }
        a.flag[g * a.nbv + b] = 0;
    }
    a.page[g * a.nbv + b] = slot;
}

// Nodes the sweeps visit, both grids: [0, n0) on G-, then G+ (every node when
// dense, else the nodes of the slots taken in this call).
template <bool kSparse>
__device__ __forceinline__ long long taken_nodes(const AdArgs &a, long long &n0) {
    if (!kSparse) {
        n0 = a.nodes;
        return 2 * a.nodes;
    }
    const unsigned int cap = (unsigned int)a.cap;
    const unsigned int c0 = min(a.cnt[0], cap), c1 = min(a.cnt[1], cap);
    n0 = 64ll * c0;
    return 64ll * (c0 + c1);
}

// Coordinates of node r of grid g in the order of taken_nodes (r < 2^32 when dense:
// at most 2^26 blocks of 64 nodes).
template <bool kSparse>
__device__ __forceinline__ void taken_coords(const AdArgs &a, int g, long long r, int &ix, int &iy, int &iz) {
    if (kSparse) {
        ad_coords(a, g, (int)(r >> 6), (int)(r & 63), ix, iy, iz);
    } else {
        const unsigned int q = (unsigned int)r, nx = (unsigned int)a.nx, ny = (unsigned int)a.ny;
        ix = (int)(q % nx);
        iy = (int)((q / nx) % ny);
        iz = (int)(q / (nx * ny));
    }
}

__device__ __forceinline__ bool node_free(const AdArgs &a, int g, int ix, int iy, int iz) {
    return ix >= a.geo.stick_lo[g] && iy >= a.geo.stick_lo[g] && iz >= a.geo.stick_lo[g] &&
           ix <= a.geo.stick_hi[g][0] && iy <= a.geo.stick_hi[g][1] && iz <= a.geo.stick_hi[g][2];
}

// Grid update on the taken blocks.  With zero_mp (a forward call: m and p have no
// later reader) m and p are zeroed after the read, ready for the next P2G.
template <bool kSparse>
__global__ void k_ad_grid(AdArgs a, int zero_mp) {
    float *gm = plane(a, GM);
    long long n0;
    const long long total = taken_nodes<kSparse>(a, n0);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int g = i >= n0 ? 1 : 0;
        const long long r = g ? i - n0 : i, id = g * a.nodes + r;
        const float m = gm[id];
        bool live = false;
        if (m > 0.0f) {
            int ix, iy, iz;
            taken_coords<kSparse>(a, g, r, ix, iy, iz);
            live = node_free(a, g, ix, iy, iz);
        }
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            float *pp = plane(a, GP + ax) + id;
            plane(a, GV + ax)[id] = live ? *pp / m + a.dt * a.g[ax] : 0.0f;
            if (zero_mp) *pp = 0.0f;
        }
        if (zero_mp) gm[id] = 0.0f;
    }
}

template <bool kSparse>
__global__ void __launch_bounds__(256) k_ad_g2p(AdArgs a, const float *state, float *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    float x[3], xr[3], H[9];
    load_planes(state, a.stride, p, 0, 3, x);
    load_planes(state, a.stride, p, kPlaneR, 3, xr);
    load_planes(state, a.stride, p, 15, 9, H);
    AdStencil st;
    if (!ad_stencil(a, x, xr, st)) {
        ad_status(a, ST_DOMAIN);
        for (int i = 0; i < MPM_STATE_PLANES; ++i) out[i * a.stride + p] = state[i * a.stride + p];
        return;
    }
    float vp[3] = {0.0f, 0.0f, 0.0f}, Bn[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Bn[i] = 0.0f;
    for (int g = 0; g < 2; ++g)
        for (int o = 0; o < 8; ++o) {
            float w, d[3], gw[3];
            const long long id = ad_node<kSparse>(a, st, g, o, w, d, gw);
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const float vi = plane(a, GV + ax)[id];
                vp[ax] += 0.5f * w * vi;
#pragma unroll
                for (int b = 0; b < 3; ++b) Bn[3 * ax + b] += 0.5f * w * vi * d[b];
            }
        }
    float C[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = Bn[3 * i] * st.Dinv[j] + Bn[3 * i + 1] * st.Dinv[3 + j] + Bn[3 * i + 2] * st.Dinv[6 + j];
    // F' = (I + dt C) F  ->  H' = H + dt C (I + H)
    float Hn[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Hn[3 * i + j] = H[3 * i + j] + a.dt * (C[3 * i + j] + C[3 * i] * H[j] + C[3 * i + 1] * H[3 + j] + C[3 * i + 2] * H[6 + j]);
    float probe = 0.0f;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        float xn, xrn;
        advance_position(x[ax], xr[ax], a.dt * vp[ax], xn, xrn);
        out[ax * a.stride + p] = xn;
        out[(kPlaneR + ax) * a.stride + p] = xrn;
        out[(3 + ax) * a.stride + p] = vp[ax];
        probe += vp[ax] * 0.0f;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        out[(6 + i) * a.stride + p] = Bn[i];
        out[(15 + i) * a.stride + p] = Hn[i];
        probe += Bn[i] * 0.0f + Hn[i] * 0.0f;
    }
    if (!(probe == 0.0f)) ad_status(a, ST_NONFINITE);
}

// G2P reversed: scatters dL/dv~ to the grid, writes the G2P part of dL/dx and dL/dF.
template <bool kSparse>
__global__ void __launch_bounds__(256) k_ad_g2p_vjp(AdArgs a, const float *state, const float *cot_out,
                                                    float *cot_in) {
    __shared__ unsigned long long tw[kAdTileWords];
    __shared__ int sh[8];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    float x[3], xr[3], H[9];
    float xbo[3], vbo[3], Bbo[9], Fbo[9];
    AdStencil st;
    bool valid = false;
    if (p < a.n) {
        load_planes(state, a.stride, p, 0, 3, x);
        load_planes(state, a.stride, p, kPlaneR, 3, xr);
        load_planes(state, a.stride, p, 15, 9, H);
        load_planes(cot_out, a.stride, p, 0, 3, xbo);
        load_planes(cot_out, a.stride, p, 3, 3, vbo);
        load_planes(cot_out, a.stride, p, 6, 9, Bbo);
        load_planes(cot_out, a.stride, p, 15, 9, Fbo);
        valid = ad_stencil(a, x, xr, st);
        if (!valid) {
            // the forward step left this particle unchanged; the position cotangent
            // is that of the x planes, written to the r planes as well
            ad_status(a, ST_DOMAIN);
            for (int i = 0; i < MPM_STATE_PLANES; ++i) cot_in[i * a.stride + p] = cot_out[i * a.stride + p];
            for (int i = 0; i < 3; ++i) cot_in[(kPlaneR + i) * a.stride + p] = xbo[i];
        }
    }
    // Every thread reaches the tile's set-up and flush (they hold workgroup barriers)
    // at the same two points, whatever its particle; invalid lanes add nothing.
    float Bn[9], C[9], xb[3], vbt[3], Fb[9], Bbt[9], Dib[9];
    float bnd = 0.0f;
    if (valid) {
        // forward quantities: B' and C = B' D^-1
#pragma unroll
        for (int i = 0; i < 9; ++i) Bn[i] = 0.0f;
        for (int g = 0; g < 2; ++g)
            for (int o = 0; o < 8; ++o) {
                float w, d[3], gw[3];
                const long long id = ad_node<kSparse>(a, st, g, o, w, d, gw);
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    const float vi = plane(a, GV + ax)[id];
#pragma unroll
                    for (int b = 0; b < 3; ++b) Bn[3 * ax + b] += 0.5f * w * vi * d[b];
                }
            }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                C[3 * i + j] =
                    Bn[3 * i] * st.Dinv[j] + Bn[3 * i + 1] * st.Dinv[3 + j] + Bn[3 * i + 2] * st.Dinv[6 + j];
        // x' = x + dt v'  ->  xb = xb',  v'b = vb' + dt xb'
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            xb[ax] = xbo[ax];
            vbt[ax] = vbo[ax] + a.dt * xbo[ax];
        }
        // F' = (I + dt C) F  ->  Cb = dt Fb' F^T,  Fb = (I + dt C)^T Fb'
        float Cb[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                float cb = 0.0f, fb = Fbo[3 * i + j];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    cb += Fbo[3 * i + k] * (H[3 * j + k] + (j == k ? 1.0f : 0.0f));
                    fb += a.dt * C[3 * k + i] * Fbo[3 * k + j];
                }
                Cb[3 * i + j] = a.dt * cb;
                Fb[3 * i + j] = fb;
            }
        // C = B' D^-1  ->  B'b += Cb D^-T,  (D^-1)b = B'^T Cb
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                Bbt[3 * i + j] = Bbo[3 * i + j] + Cb[3 * i] * st.Dinv[3 * j] + Cb[3 * i + 1] * st.Dinv[3 * j + 1] +
                                 Cb[3 * i + 2] * st.Dinv[3 * j + 2];
                Dib[3 * i + j] = Bn[i] * Cb[j] + Bn[3 + i] * Cb[3 + j] + Bn[6 + i] * Cb[6 + j];
            }
        // |1/2 w (v'b + B'b d)| <= 1/2 (|v'b| + dx sum |B'b|)
#pragma unroll
        for (int ax = 0; ax < 3; ++ax)
            bnd = fmaxf(bnd, 0.5f * (fabsf(vbt[ax]) + a.geo.dx * (fabsf(Bbt[3 * ax]) + fabsf(Bbt[3 * ax + 1]) +
                                                                  fabsf(Bbt[3 * ax + 2]))));
    }
    AdTile t;
    ad_tile_begin(valid, st, bnd, 3, tw, sh, t);
    if (valid) {
        // v' = 1/2 sum w v~,  B' = 1/2 sum w v~ d^T:
        //   v~b_i += 1/2 w (v'b + B'b d),  wb = 1/2 v~ . (v'b + B'b d),  db = 1/2 w B'b^T v~,
        //   and d = x_i - x_p moves against x_p
        for (int g = 0; g < 2; ++g)
            for (int o = 0; o < 8; ++o) {
                float w, d[3], gw[3];
                const long long id = ad_node<kSparse>(a, st, g, o, w, d, gw);
                const int ix = st.base[g][0] + (o & 1), iy = st.base[g][1] + ((o >> 1) & 1),
                          iz = st.base[g][2] + (o >> 2);
                float vi[3], gv[3];
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    vi[ax] = plane(a, GV + ax)[id];
                    gv[ax] = vbt[ax] + Bbt[3 * ax] * d[0] + Bbt[3 * ax + 1] * d[1] + Bbt[3 * ax + 2] * d[2];
                }
                float wb = 0.0f;
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    ad_tile_add(a, t, GVB, ax, g, ix, iy, iz, id, 0.5f * w * gv[ax]);
                    wb += 0.5f * vi[ax] * gv[ax];
                }
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const float db = 0.5f * w * (Bbt[b] * vi[0] + Bbt[3 + b] * vi[1] + Bbt[6 + b] * vi[2]);
                    xb[b] += wb * gw[b] - db;
                }
            }
        float Db[9];
        ad_inverse_vjp(st.Dinv, Dib, Db);
        ad_moment_vjp(a, st, Db, xb);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) cot_in[ax * a.stride + p] = xb[ax];
#pragma unroll
        for (int i = 0; i < 9; ++i) cot_in[(15 + i) * a.stride + p] = Fb[i];
    }
    ad_tile_flush<kSparse>(a, t, GVB, 3);
}

// Grid update reversed: pb = v~b / m,  mb = -(v~b . p) / m^2 on live nodes.
// As the last reader of m, p and v~b in a backward call, it also zeroes them for the
// next call's scatters.
template <bool kSparse>
__global__ void k_ad_grid_vjp(AdArgs a) {
    float *gm = plane(a, GM);
    long long n0;
    const long long total = taken_nodes<kSparse>(a, n0);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int g = i >= n0 ? 1 : 0;
        const long long r = g ? i - n0 : i, id = g * a.nodes + r;
        const float m = gm[id];
        bool live = false;
        if (m > 0.0f) {
            int ix, iy, iz;
            taken_coords<kSparse>(a, g, r, ix, iy, iz);
            live = node_free(a, g, ix, iy, iz);
        }
        float dot = 0.0f;
        const float im = live ? 1.0f / m : 0.0f;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            float *vbp = plane(a, GVB + ax) + id;
            float *pp = plane(a, GP + ax) + id;
            const float vb = *vbp;
            plane(a, GPB + ax)[id] = vb * im;
            dot += vb * *pp;
            *vbp = 0.0f;
            *pp = 0.0f;
        }
        plane(a, GMB)[id] = live ? -dot * im * im : 0.0f;
        gm[id] = 0.0f;
    }
}

// P2G reversed (a gather): completes dL/dx and dL/dF, writes dL/dv, dL/dB, adds dL/dlogE.
template <bool kSparse>
__global__ void __launch_bounds__(256) k_ad_p2g_vjp(AdArgs a, const float *state, const float *logE, float *cot_in,
                                                    float *logE_cot) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    float x[3], xr[3], v[3], B[9], H[9];
    load_planes(state, a.stride, p, 0, 3, x);
    load_planes(state, a.stride, p, kPlaneR, 3, xr);
    load_planes(state, a.stride, p, 3, 3, v);
    load_planes(state, a.stride, p, 6, 9, B);
    load_planes(state, a.stride, p, 15, 9, H);
    AdStencil st;
    if (!ad_stencil(a, x, xr, st)) return;   // cotangent already passed through by the G2P adjoint
    const float E = expf(logE[p]);
    const float mu = a.nu_mu * E, lam = a.nu_lambda * E;
    Polar P;
    ad_polar(H, P);
    float tau[9];
    ad_tau(H, P, mu, lam, tau);
    float A[9], Q[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) A[i] = a.mass * B[i] - a.dt * a.vol0 * tau[i];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Q[3 * i + j] = A[3 * i] * st.Dinv[j] + A[3 * i + 1] * st.Dinv[3 + j] + A[3 * i + 2] * st.Dinv[6 + j];
    float xb[3], vb[3] = {0.0f, 0.0f, 0.0f}, Qb[9];
    load_planes(cot_in, a.stride, p, 0, 3, xb);
#pragma unroll
    for (int i = 0; i < 9; ++i) Qb[i] = 0.0f;
    // m_i += w m,  p_i += w (m v + Q d):
    //   wb = m mb_i + pb_i . (m v + Q d),  vb += w m pb_i,  Qb += w pb_i d^T,  db = w Q^T pb_i
    for (int g = 0; g < 2; ++g)
        for (int o = 0; o < 8; ++o) {
            float w, d[3], gw[3];
            const long long id = ad_node<kSparse>(a, st, g, o, w, d, gw);
            float pb[3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) pb[ax] = plane(a, GPB + ax)[id];
            float wb = a.mass * plane(a, GMB)[id];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const float pi = a.mass * v[ax] + Q[3 * ax] * d[0] + Q[3 * ax + 1] * d[1] + Q[3 * ax + 2] * d[2];
                wb += pb[ax] * pi;
                vb[ax] += w * a.mass * pb[ax];
#pragma unroll
                for (int b = 0; b < 3; ++b) Qb[3 * ax + b] += w * pb[ax] * d[b];
            }
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const float db = w * (Q[b] * pb[0] + Q[3 + b] * pb[1] + Q[6 + b] * pb[2]);
                xb[b] += wb * gw[b] - db;
            }
        }
    // Q = A D^-1  ->  Ab = Qb D^-T,  (D^-1)b = A^T Qb
    float Ab[9], Dib[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Ab[3 * i + j] = Qb[3 * i] * st.Dinv[3 * j] + Qb[3 * i + 1] * st.Dinv[3 * j + 1] + Qb[3 * i + 2] * st.Dinv[3 * j + 2];
            Dib[3 * i + j] = A[i] * Qb[j] + A[3 + i] * Qb[3 + j] + A[6 + i] * Qb[6 + j];
        }
    float Db[9];
    ad_inverse_vjp(st.Dinv, Dib, Db);
    ad_moment_vjp(a, st, Db, xb);
    // A = m B - dt V0 tau  ->  Bb = m Ab,  taub = -dt V0 Ab
    float tb[9], Fb[9];
    float lb = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        tb[i] = -a.dt * a.vol0 * Ab[i];
        lb += tb[i] * tau[i];   // tau is proportional to E = exp(logE)
    }
    load_planes(cot_in, a.stride, p, 15, 9, Fb);
    ad_tau_vjp(H, P, mu, lam, tb, Fb);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        cot_in[ax * a.stride + p] = xb[ax];
        cot_in[(kPlaneR + ax) * a.stride + p] = xb[ax];   // the position is x + r
        cot_in[(3 + ax) * a.stride + p] = vb[ax];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        cot_in[(6 + i) * a.stride + p] = a.mass * Ab[i];
        cot_in[(15 + i) * a.stride + p] = Fb[i];
    }
    logE_cot[p] += lb;
}

AdArgs make_args(const mpm_ad_ctx *c, int64_t n, int64_t stride, double dt) {
    AdArgs a;
    a.geo = c->geo;
    for (int i = 0; i < 3; ++i) a.g[i] = c->gravity[i];
    a.mass = c->rho * c->vol0;
    a.vol0 = c->vol0;
    a.nu_mu = (float)(1.0 / (2.0 * (1.0 + c->nu)));
    a.nu_lambda = (float)(c->nu / ((1.0 + c->nu) * (1.0 - 2.0 * c->nu)));
    a.nbx = c->nb[0];
    a.nby = c->nb[1];
    a.cap = c->cap;
    a.nbv = c->nbv;
    a.nodes = c->nodes;
    a.nx = c->geo.n[0] + 1;
    a.ny = c->geo.n[1] + 1;
    a.grid = c->grid;
    a.page = c->page;
    a.blist = c->blist;
    a.direct = c->direct ? 1 : 0;
    a.flag = c->flag;
    a.cnt = c->cnt;
    a.status = c->status;
    a.n = (int)n;
    a.stride = stride;
    a.dt = (float)dt;
    return a;
}

int grid_blocks(long long work) {
    const long long b = (work + 255) / 256;
    return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

// Launch size of the sweeps (all nodes, or at most the pool's 2 * cap * 64).
int sweep_blocks(const AdArgs &a) { return grid_blocks(a.direct ? 2 * a.nodes : 2ll * a.cap * 64); }

// Blocks marked and given slots (unless direct), P2G into the (zero) m and p planes,
// the grid update;
// zero_mp for a forward call.
void enqueue_forward_grid(const AdArgs &a, const float *state, const float *logE, int zero_mp, hipStream_t s) {
    if (!a.direct) {
        hipLaunchKernelGGL(k_ad_mark, dim3(a.n > 0 ? (a.n + 255) / 256 : 1), dim3(256), 0, s, a, state);
        hipLaunchKernelGGL(k_ad_alloc, dim3((unsigned int)((a.nbv + 255) / 256), 2), dim3(256), 0, s, a);
    }
    const dim3 pg((a.n + 255) / 256), sg(sweep_blocks(a)), wg(256);
    if (a.direct) {
        if (a.n > 0) hipLaunchKernelGGL(k_ad_p2g<false>, pg, wg, 0, s, a, state, logE);
        hipLaunchKernelGGL(k_ad_grid<false>, sg, wg, 0, s, a, zero_mp);
    } else {
        if (a.n > 0) hipLaunchKernelGGL(k_ad_p2g<true>, pg, wg, 0, s, a, state, logE);
        hipLaunchKernelGGL(k_ad_grid<true>, sg, wg, 0, s, a, zero_mp);
    }
}

void free_buffers(mpm_ad_ctx *c) {
    void *bufs[] = {c->grid, c->page, c->blist, c->flag, c->cnt, c->status};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
}

void launch_backward_scatter(const AdArgs &a, const float *state, const float *cot_out, float *cot_in, hipStream_t s) {
    const dim3 pg((a.n + 255) / 256), wg(256);
    if (a.direct) hipLaunchKernelGGL(k_ad_g2p_vjp<false>, pg, wg, 0, s, a, state, cot_out, cot_in);
    else hipLaunchKernelGGL(k_ad_g2p_vjp<true>, pg, wg, 0, s, a, state, cot_out, cot_in);
}

void launch_backward_gather(const AdArgs &a, const float *state, const float *logE, float *cot_in, float *logE_cot,
                            hipStream_t s) {
    const dim3 pg((a.n + 255) / 256), wg(256);
    if (a.direct) hipLaunchKernelGGL(k_ad_p2g_vjp<false>, pg, wg, 0, s, a, state, logE, cot_in, logE_cot);
    else hipLaunchKernelGGL(k_ad_p2g_vjp<true>, pg, wg, 0, s, a, state, logE, cot_in, logE_cot);
}

mpm_status check_call(const mpm_ad_ctx *c, int64_t n, int64_t stride, const float *state, double dt) {
    if (!c || n < 0 || n > c->max_particles || stride < n) return MPM_E_INVALID;
    if (n > 0 && !state) return MPM_E_INVALID;
    if (!std::isfinite(dt) || dt < 0) return MPM_E_INVALID;
    return MPM_OK;
}

}  // namespace

extern "C" {

mpm_status mpm_ad_create(const mpm_config *cfg, const mpm_material *mat, mpm_ad_ctx **out) {
    if (!out) return MPM_E_INVALID;
    *out = nullptr;
    if (check_config(cfg, mat, 1) != MPM_OK || mat->model != MPM_FIXED_COROTATED) return MPM_E_INVALID;
    mpm_ad_ctx *c = new (std::nothrow) mpm_ad_ctx();
    if (!c) return MPM_E_OOM;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return MPM_E_HIP;
    }
    geometry_of(*cfg, c->geo);
    for (int i = 0; i < 3; ++i) c->gravity[i] = (float)cfg->gravity[i];
    c->nu = mat->nu;
    c->rho = mat->rho;
    c->vol0 = mat->vol0;
    c->max_particles = cfg->max_particles;
    c->nbv = 1;
    for (int i = 0; i < 3; ++i) {
        c->nb[i] = cfg->n_cells[i] / 4 + 1;
        c->nbv *= c->nb[i];
    }
    c->cap = (int)std::min<long long>(cfg->max_blocks, c->nbv);
    c->direct = c->cap == c->nbv;
    c->nodes = c->direct ? (long long)(cfg->n_cells[0] + 1) * (cfg->n_cells[1] + 1) * (cfg->n_cells[2] + 1)
                         : (long long)(c->cap + 1) * 64;
    const size_t bytes = (size_t)kGridPlanes * 2 * c->nodes * sizeof(float);
    const size_t nbv2 = 2 * (size_t)c->nbv;
    bool ok = hipMalloc(&c->grid, bytes) == hipSuccess && hipMalloc(&c->cnt, 2 * sizeof(unsigned int)) == hipSuccess &&
              hipMalloc(&c->status, sizeof(unsigned int)) == hipSuccess;
    if (!c->direct)   // page tables, slot list and marks of the block-sparse pool
        ok = ok && hipMalloc(&c->page, nbv2 * sizeof(int)) == hipSuccess &&
             hipMalloc(&c->blist, 2 * (size_t)c->cap * sizeof(int)) == hipSuccess &&
             hipMalloc(&c->flag, nbv2) == hipSuccess && hipMemset(c->flag, 0, nbv2) == hipSuccess;
    // the scatter targets (m, p, v~b) start at zero and every call leaves the nodes it
    // swept at zero; no block is marked between calls
    ok = ok && hipMemset(c->grid, 0, bytes) == hipSuccess &&
         hipMemset(c->cnt, 0, 2 * sizeof(unsigned int)) == hipSuccess &&
         hipMemset(c->status, 0, sizeof(unsigned int)) == hipSuccess;
    if (!ok) {
        free_buffers(c);
        delete c;
        return MPM_E_OOM;
    }
    *out = c;
    return MPM_OK;
}

mpm_status mpm_ad_destroy(mpm_ad_ctx *c) {
    if (!c) return MPM_E_INVALID;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    free_buffers(c);
    delete c;
    return MPM_OK;
}

mpm_status mpm_ad_forward(mpm_ad_ctx *c, int64_t n, int64_t stride, const float *state_in, const float *logE,
                          float *state_out, double dt, void *stream) {
    const mpm_status v = check_call(c, n, stride, state_in, dt);
    if (v != MPM_OK) return v;
    if (n > 0 && (!logE || !state_out)) return MPM_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return MPM_E_HIP;
    hipStream_t s = (hipStream_t)stream;
    const AdArgs a = make_args(c, n, stride, dt);
    enqueue_forward_grid(a, state_in, logE, 1, s);
    if (n > 0) {
        if (a.direct) hipLaunchKernelGGL(k_ad_g2p<false>, dim3((n + 255) / 256), dim3(256), 0, s, a, state_in, state_out);
        else hipLaunchKernelGGL(k_ad_g2p<true>, dim3((n + 255) / 256), dim3(256), 0, s, a, state_in, state_out);
    }
    return hipGetLastError() == hipSuccess ? MPM_OK : MPM_E_HIP;
}

mpm_status mpm_ad_backward(mpm_ad_ctx *c, int64_t n, int64_t stride, const float *state_in, const float *logE,
                           const float *cot_out, float *cot_in, float *logE_cot, double dt, void *stream) {
    const mpm_status v = check_call(c, n, stride, state_in, dt);
    if (v != MPM_OK) return v;
    if (n > 0 && (!logE || !cot_out || !cot_in || !logE_cot)) return MPM_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return MPM_E_HIP;
    hipStream_t s = (hipStream_t)stream;
    const AdArgs a = make_args(c, n, stride, dt);
    enqueue_forward_grid(a, state_in, logE, 0, s);
    if (n > 0)
        launch_backward_scatter(a, state_in, cot_out, cot_in, s);
    if (a.direct) hipLaunchKernelGGL(k_ad_grid_vjp<false>, dim3(sweep_blocks(a)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_ad_grid_vjp<true>, dim3(sweep_blocks(a)), dim3(256), 0, s, a);
    if (n > 0)
        launch_backward_gather(a, state_in, logE, cot_in, logE_cot, s);
    return hipGetLastError() == hipSuccess ? MPM_OK : MPM_E_HIP;
}

mpm_status mpm_ad_sync(mpm_ad_ctx *c, void *stream) {
    if (!c) return MPM_E_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return MPM_E_HIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return MPM_E_HIP;
    unsigned int bits = 0;
    if (hipMemcpy(&bits, c->status, sizeof bits, hipMemcpyDeviceToHost) != hipSuccess) return MPM_E_HIP;
    const unsigned int zero = 0;
    if (hipMemcpy(c->status, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess) return MPM_E_HIP;
    return status_from_bits(bits);
}

}  // extern "C"
