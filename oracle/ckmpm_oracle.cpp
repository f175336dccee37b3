// FP64 CPU oracle for one compact-kernel MPM step (CK-MPM, arXiv 2412.10399).
//
// TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's
// CPU-baseline leg use it to check the HIP path.  The product path never links
// or calls it, and it shares no code, header, table or helper with the HIP path.
//
// Every routine is a plain transcription of a definition or an algorithm step
// from the paper (cited per function), written for readability: no blocking,
// no fusion, FP64 throughout.  Parallel loops (OpenMP) only run over
// independent particles or nodes; the particle-to-grid scatter is serial so its
// summation order is fixed.
//
// Readings of the paper that this file relies on (the paper is silent or
// inconsistent on them):
//  * node i of grid G_k sits at origin + (i + k/4) dx (section 4.2 places the two
//    grids a quarter cell either side of the unstored grid G_0; only their
//    half-cell relative offset enters the identities);
//  * the grid-to-particle velocity is the plain average 1/2 sum_k sum_i w v~
//    (the printed PIC formula carries an extra m_i/m_p factor that breaks affine
//    reproduction; the APIC section and the supplement's G2P step use the plain
//    form);
//  * the stress force is f_i = -sum_p V_p^0 tau_p grad(Phi_i) (minus sign and
//    reference volume as in the background section and the supplement);
//  * the F update multiplies the old F (the supplement's form);
//  * B (not C = B D^-1) is carried between steps and D is recomputed at the
//    current position in both transfers;
//  * sticky walls zero v~ on nodes closer than bc_band cells to the box faces;
//  * Drucker-Prager return mapping after Klar et al. 2016 without hardening or
//    cohesion, singular values clamped at 1e-4 before taking logs.
#include "ckmpm_oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- 3x3 helpers
struct M3 {
    double a[3][3];
};

M3 zero3() {
    M3 r;
    std::memset(r.a, 0, sizeof r.a);
    return r;
}
M3 eye3() {
    M3 r = zero3();
    r.a[0][0] = r.a[1][1] = r.a[2][2] = 1.0;
    return r;
}
M3 load3(const double *p) {
    M3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = p[3 * i + j];
    return r;
}
void store3(const M3 &m, double *p) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) p[3 * i + j] = m.a[i][j];
}
M3 mul(const M3 &x, const M3 &y) {
    M3 r = zero3();
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) r.a[i][j] += x.a[i][k] * y.a[k][j];
    return r;
}
M3 transpose(const M3 &x) {
    M3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = x.a[j][i];
    return r;
}
double det(const M3 &m) {
    const auto &a = m.a;
    return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
           a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
}
// Inverse by Gauss-Jordan elimination with partial pivoting.
M3 inverse(const M3 &m) {
    double w[3][6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            w[i][j] = m.a[i][j];
            w[i][j + 3] = (i == j) ? 1.0 : 0.0;
        }
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (std::fabs(w[r][c]) > std::fabs(w[piv][c])) piv = r;
        if (piv != c)
            for (int j = 0; j < 6; ++j) std::swap(w[c][j], w[piv][j]);
        const double d = w[c][c];
        for (int j = 0; j < 6; ++j) w[c][j] /= d;
        for (int r = 0; r < 3; ++r) {
            if (r == c) continue;
            const double f = w[r][c];
            for (int j = 0; j < 6; ++j) w[r][j] -= f * w[c][j];
        }
    }
    M3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = w[i][j + 3];
    return r;
}

struct Lame {
    double mu, lambda;
};
Lame lame(const ora_material *m, double logE) {
    const double E = std::isnan(logE) ? m->E : std::exp(logE);
    return {E / (2.0 * (1.0 + m->nu)), E * m->nu / ((1.0 + m->nu) * (1.0 - 2.0 * m->nu))};
}

// ------------------------------------------------------------ SVD (FP64)
// One-sided Jacobi (Hestenes) SVD: plane rotations applied on the right make the
// columns of A mutually orthogonal; then A V = U diag(s).  Returned in the
// rotation-variant convention: det U = det V = +1, singular values sorted in
// decreasing magnitude, the sign (if any) carried by the last one.
void svd_jacobi(const M3 &F, M3 &U, double s[3], M3 &V) {
    M3 A = F;
    V = eye3();
    for (int sweep = 0; sweep < 80; ++sweep) {
        bool rotated = false;
        static const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (const auto &pq : pairs) {
            const int p = pq[0], q = pq[1];
            double alpha = 0, beta = 0, gamma = 0;
            for (int r = 0; r < 3; ++r) {
                alpha += A.a[r][p] * A.a[r][p];
                beta += A.a[r][q] * A.a[r][q];
                gamma += A.a[r][p] * A.a[r][q];
            }
            if (gamma == 0.0 || std::fabs(gamma) <= 1e-17 * std::sqrt(alpha * beta)) continue;
            rotated = true;
            const double zeta = (beta - alpha) / (2.0 * gamma);
            const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
            for (int r = 0; r < 3; ++r) {
                const double ap = A.a[r][p], aq = A.a[r][q];
                A.a[r][p] = c * ap - sn * aq;
                A.a[r][q] = sn * ap + c * aq;
                const double vp = V.a[r][p], vq = V.a[r][q];
                V.a[r][p] = c * vp - sn * vq;
                V.a[r][q] = sn * vp + c * vq;
            }
        }
        if (!rotated) break;
    }
    double nrm[3];
    for (int j = 0; j < 3; ++j) nrm[j] = std::sqrt(A.a[0][j] * A.a[0][j] + A.a[1][j] * A.a[1][j] + A.a[2][j] * A.a[2][j]);
    int order[3] = {0, 1, 2};
    std::sort(order, order + 3, [&](int i, int j) { return nrm[i] > nrm[j]; });
    M3 As = A, Vs = V;
    for (int j = 0; j < 3; ++j)
        for (int r = 0; r < 3; ++r) {
            As.a[r][j] = A.a[r][order[j]];
            Vs.a[r][j] = V.a[r][order[j]];
        }
    for (int j = 0; j < 3; ++j) s[j] = nrm[order[j]];
    const double tiny = 1e-300;
    U = zero3();
    // first column
    if (s[0] > tiny) {
        for (int r = 0; r < 3; ++r) U.a[r][0] = As.a[r][0] / s[0];
    } else {
        U.a[0][0] = 1.0;
    }
    // second column: normalised A column, or any unit vector orthogonal to the first
    if (s[1] > 1e-12 * std::max(s[0], tiny)) {
        for (int r = 0; r < 3; ++r) U.a[r][1] = As.a[r][1] / s[1];
    } else {
        double e[3] = {0, 0, 0};
        int k = 0;
        for (int r = 1; r < 3; ++r)
            if (std::fabs(U.a[r][0]) < std::fabs(U.a[k][0])) k = r;
        e[k] = 1.0;
        double d = e[0] * U.a[0][0] + e[1] * U.a[1][0] + e[2] * U.a[2][0];
        double u[3], un = 0;
        for (int r = 0; r < 3; ++r) {
            u[r] = e[r] - d * U.a[r][0];
            un += u[r] * u[r];
        }
        un = std::sqrt(un);
        for (int r = 0; r < 3; ++r) U.a[r][1] = u[r] / un;
    }
    // third column: normalised A column, or the cross product of the first two
    if (s[2] > 1e-12 * std::max(s[0], tiny)) {
        for (int r = 0; r < 3; ++r) U.a[r][2] = As.a[r][2] / s[2];
    } else {
        U.a[0][2] = U.a[1][0] * U.a[2][1] - U.a[2][0] * U.a[1][1];
        U.a[1][2] = U.a[2][0] * U.a[0][1] - U.a[0][0] * U.a[2][1];
        U.a[2][2] = U.a[0][0] * U.a[1][1] - U.a[1][0] * U.a[0][1];
    }
    V = Vs;
    if (det(V) < 0) {  // flip the last column of both factors: U S V^T unchanged
        for (int r = 0; r < 3; ++r) {
            V.a[r][2] = -V.a[r][2];
            U.a[r][2] = -U.a[r][2];
        }
    }
    if (det(U) < 0) {  // move the reflection into the last singular value
        for (int r = 0; r < 3; ++r) U.a[r][2] = -U.a[r][2];
        s[2] = -s[2];
    }
}

// ------------------------------------------------------ constitutive models
// Fixed corotated (Stomakhin et al. 2012, cited in section 6.1):
//   psi = mu |F - R|^2 + lambda/2 (J-1)^2,  P = 2 mu (F - R) + lambda (J-1) J F^-T,
//   Kirchhoff tau = P F^T = 2 mu (F - R) F^T + lambda (J-1) J I.
// Drucker-Prager (Klar et al. 2016, cited in sections 3.2 and 6.2) with the
// Hencky (log-strain) St. Venant-Kirchhoff energy:
//   psi = mu tr(eps^2) + lambda/2 tr(eps)^2,  tau = U (2 mu eps + lambda tr(eps) I) U^T.
constexpr double kSigmaFloor = 1e-4;

M3 kirchhoff(const ora_material *m, double logE, const M3 &F) {
    const Lame L = lame(m, logE);
    M3 U, V;
    double s[3];
    svd_jacobi(F, U, s, V);
    M3 tau = zero3();
    if (m->model == 0) {
        const M3 R = mul(U, transpose(V));
        const double J = det(F);
        M3 FmR;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) FmR.a[i][j] = F.a[i][j] - R.a[i][j];
        tau = mul(FmR, transpose(F));
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) tau.a[i][j] *= 2.0 * L.mu;
        for (int i = 0; i < 3; ++i) tau.a[i][i] += L.lambda * (J - 1.0) * J;
    } else {
        double eps[3], tr = 0;
        for (int i = 0; i < 3; ++i) {
            eps[i] = std::log(std::max(s[i], kSigmaFloor));
            tr += eps[i];
        }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k) tau.a[i][j] += U.a[i][k] * (2.0 * L.mu * eps[k] + L.lambda * tr) * U.a[j][k];
    }
    return tau;
}

double energy_density(const ora_material *m, double logE, const M3 &F) {
    const Lame L = lame(m, logE);
    M3 U, V;
    double s[3];
    svd_jacobi(F, U, s, V);
    if (m->model == 0) {
        const M3 R = mul(U, transpose(V));
        double fr = 0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) fr += (F.a[i][j] - R.a[i][j]) * (F.a[i][j] - R.a[i][j]);
        const double J = det(F);
        return L.mu * fr + 0.5 * L.lambda * (J - 1.0) * (J - 1.0);
    }
    double e2 = 0, tr = 0;
    for (int i = 0; i < 3; ++i) {
        const double e = std::log(std::max(s[i], kSigmaFloor));
        e2 += e * e;
        tr += e;
    }
    return L.mu * e2 + 0.5 * L.lambda * tr * tr;
}

// Vector-Jacobian product of the fixed-corotated Kirchhoff stress above, the
// differentiable step's constitutive adjoint: given tb = dL/dtau (a full 3x3
// matrix; tau is symmetric for every F), returns dL/dF and dL/dlogE.
//   dtau = 2 mu (dF F^T + F dF^T - dR F^T - R dF^T) + lambda (2J - 1) dJ I,
//   dJ = <cof F, dF>,  and tau is linear in E = exp(logE).
// The rotation R = U V^T of F = U S V^T moves as dR = U M V^T with
// M_ij = (A_ij - A_ji) / (s_i + s_j), A = U^T dF V (the derivative of the polar
// factor), so its adjoint adds U Z V^T, Z_ij = (Y_ij - Y_ji) / (s_i + s_j),
// Y = U^T Rbar V.
void kirchhoff_fc_vjp(const ora_material *m, double logE, const M3 &F, const M3 &tb, M3 &Fb, double &logEb) {
    const Lame L = lame(m, logE);
    M3 U, V;
    double s[3];
    svd_jacobi(F, U, s, V);
    const M3 R = mul(U, transpose(V));
    const double J = det(F);
    const M3 tbT = transpose(tb);
    const M3 t1 = mul(tb, F), t2 = mul(tbT, F), t3 = mul(tbT, R);
    Fb = zero3();
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Fb.a[i][j] = 2.0 * L.mu * (t1.a[i][j] + t2.a[i][j] - t3.a[i][j]);
    M3 Rb;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Rb.a[i][j] = -2.0 * L.mu * t1.a[i][j];
    const M3 Y = mul(transpose(U), mul(Rb, V));
    M3 Z = zero3();
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (i != j) Z.a[i][j] = (Y.a[i][j] - Y.a[j][i]) / (s[i] + s[j]);
    const M3 dFR = mul(U, mul(Z, transpose(V)));
    // cofactor matrix cof(F) = J F^-T
    M3 cof;
    const auto &f = F.a;
    cof.a[0][0] = f[1][1] * f[2][2] - f[1][2] * f[2][1];
    cof.a[0][1] = f[1][2] * f[2][0] - f[1][0] * f[2][2];
    cof.a[0][2] = f[1][0] * f[2][1] - f[1][1] * f[2][0];
    cof.a[1][0] = f[0][2] * f[2][1] - f[0][1] * f[2][2];
    cof.a[1][1] = f[0][0] * f[2][2] - f[0][2] * f[2][0];
    cof.a[1][2] = f[0][1] * f[2][0] - f[0][0] * f[2][1];
    cof.a[2][0] = f[0][1] * f[1][2] - f[0][2] * f[1][1];
    cof.a[2][1] = f[0][2] * f[1][0] - f[0][0] * f[1][2];
    cof.a[2][2] = f[0][0] * f[1][1] - f[0][1] * f[1][0];
    const double trtb = tb.a[0][0] + tb.a[1][1] + tb.a[2][2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Fb.a[i][j] += dFR.a[i][j] + L.lambda * (2.0 * J - 1.0) * trtb * cof.a[i][j];
    const M3 tau = kirchhoff(m, logE, F);
    logEb = 0.0;
    if (!std::isnan(logE))
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) logEb += tb.a[i][j] * tau.a[i][j];
}

// Drucker-Prager return mapping (Klar et al. 2016, projection onto the cone in
// log-strain space), applied to the trial elastic F after the F update.
void dp_return_map(const ora_material *m, double logE, M3 &F) {
    const Lame L = lame(m, logE);
    M3 U, V;
    double s[3];
    svd_jacobi(F, U, s, V);
    const double sphi = std::sin(m->friction_deg * kPi / 180.0);
    const double alpha = std::sqrt(2.0 / 3.0) * 2.0 * sphi / (3.0 - sphi);
    double eps[3], tr = 0;
    for (int i = 0; i < 3; ++i) {
        eps[i] = std::log(std::max(s[i], kSigmaFloor));
        tr += eps[i];
    }
    double dev[3], devn = 0;
    for (int i = 0; i < 3; ++i) {
        dev[i] = eps[i] - tr / 3.0;
        devn += dev[i] * dev[i];
    }
    devn = std::sqrt(devn);
    double snew[3];
    if (tr > 0.0 || devn == 0.0) {
        snew[0] = snew[1] = snew[2] = 1.0;  // tension or pure dilation: project to the cone tip
    } else {
        const double dgamma = devn + (3.0 * L.lambda + 2.0 * L.mu) / (2.0 * L.mu) * tr * alpha;
        if (dgamma <= 0.0) {
            // inside the cone: elastic, F unchanged
            return;
        }
        for (int i = 0; i < 3; ++i) snew[i] = std::exp(eps[i] - dgamma * dev[i] / devn);
    }
    M3 r = zero3();
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) r.a[i][j] += U.a[i][k] * snew[k] * V.a[j][k];
    F = r;
}

// --------------------------------------------------------- compact kernel
// Section 4.1: K1(x) = 1 - |x| + sin(2 pi |x|) / (2 pi) for |x| < 1, else 0.
double K1(double x) {
    const double a = std::fabs(x);
    if (a >= 1.0) return 0.0;
    return 1.0 - a + std::sin(2.0 * kPi * a) / (2.0 * kPi);
}
double dK1(double x) {
    const double a = std::fabs(x);
    if (a >= 1.0) return 0.0;
    const double sg = (x > 0) ? 1.0 : (x < 0 ? -1.0 : 0.0);
    return sg * (-1.0 + std::cos(2.0 * kPi * a));
}
double d2K1(double x) {
    const double a = std::fabs(x);
    if (a >= 1.0) return 0.0;
    return -2.0 * kPi * std::sin(2.0 * kPi * a);
}

// Quadratic B-spline N(r) = 3/4 - r^2 for |r| < 1/2, (3/2 - |r|)^2 / 2 for 1/2 <= |r| < 3/2,
// the single-grid kernel the paper compares the compact kernel against (27 nodes).
double Nq(double r) {
    const double a = std::fabs(r);
    if (a < 0.5) return 0.75 - a * a;
    if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
}
double dNq(double r) {
    const double a = std::fabs(r);
    const double sg = (r > 0) ? 1.0 : (r < 0 ? -1.0 : 0.0);
    if (a < 0.5) return -2.0 * r;
    if (a < 1.5) return -sg * (1.5 - a);
    return 0.0;
}

struct Stencil {
    int64_t node[2][8];     // dense node index per grid, -1 when off the grid
    int32_t ijk[2][8][3];
    double w[2][8];
    double d[2][8][3];      // x_i - x_p (world units)
    double gw[2][8][3];     // gradient of w with respect to the particle position
};

int64_t node_index(const ora_config *c, const int32_t ijk[3]) {
    for (int a = 0; a < 3; ++a)
        if (ijk[a] < 0 || ijk[a] > c->n_cells[a]) return -1;
    const int64_t nx = c->n_cells[0] + 1, ny = c->n_cells[1] + 1;
    return ((int64_t)ijk[2] * ny + ijk[1]) * nx + ijk[0];
}

// Section 4.2-4.3: the particle interacts with the 2x2x2 nodes of the cell it
// occupies on each staggered grid; w_ipk = K((x_{i,G_k} - x_p)/dx) with the
// tensor-product kernel K(x) = prod_beta K1(x^beta).
void stencil(const ora_config *c, const double xp[3], Stencil &st) {
    for (int g = 0; g < 2; ++g) {
        const double k = (g == 0) ? -1.0 : 1.0;
        int32_t base[3];
        for (int a = 0; a < 3; ++a) base[a] = (int32_t)std::floor((xp[a] - c->origin[a]) / c->dx - k / 4.0);
        for (int o = 0; o < 8; ++o) {
            const int off[3] = {o & 1, (o >> 1) & 1, (o >> 2) & 1};
            double r[3], wa[3], dwa[3];
            for (int a = 0; a < 3; ++a) {
                st.ijk[g][o][a] = base[a] + off[a];
                const double xi = c->origin[a] + (st.ijk[g][o][a] + k / 4.0) * c->dx;
                st.d[g][o][a] = xi - xp[a];
                r[a] = st.d[g][o][a] / c->dx;
                wa[a] = K1(r[a]);
                dwa[a] = -dK1(r[a]) / c->dx;  // d/dx_p of K1((x_i - x_p)/dx)
            }
            st.w[g][o] = wa[0] * wa[1] * wa[2];
            st.gw[g][o][0] = dwa[0] * wa[1] * wa[2];
            st.gw[g][o][1] = wa[0] * dwa[1] * wa[2];
            st.gw[g][o][2] = wa[0] * wa[1] * dwa[2];
            st.node[g][o] = node_index(c, st.ijk[g][o]);
        }
    }
}

// Section 4.4: D_p = 1/2 sum_k sum_i w (x_i - x_p)(x_i - x_p)^T.
M3 moment_matrix(const Stencil &st) {
    M3 D = zero3();
    for (int g = 0; g < 2; ++g)
        for (int o = 0; o < 8; ++o)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) D.a[a][b] += 0.5 * st.w[g][o] * st.d[g][o][a] * st.d[g][o][b];
    return D;
}

// Adjoint of D_p = 1/2 sum_k sum_i w (x_i - x_p)(x_i - x_p)^T with respect to the
// particle position, term by term: given Db = dL/dD, adds to xb
//   1/2 sum [ grad w (d^T Db d) - w (Db d + Db^T d) ],   d = x_i - x_p.
void moment_matrix_vjp(const Stencil &st, const M3 &Db, double xb[3]) {
    for (int g = 0; g < 2; ++g)
        for (int o = 0; o < 8; ++o) {
            const double *d = st.d[g][o];
            double Dd[3] = {0, 0, 0}, DTd[3] = {0, 0, 0}, q = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    Dd[a] += Db.a[a][b] * d[b];
                    DTd[a] += Db.a[b][a] * d[b];
                    q += d[a] * Db.a[a][b] * d[b];
                }
            for (int a = 0; a < 3; ++a) xb[a] += 0.5 * (st.gw[g][o][a] * q - st.w[g][o] * (Dd[a] + DTd[a]));
        }
}

// d(D^-1) = -D^-1 dD D^-1, so the adjoint of the inverse is Db = -D^-T Dib D^-T.
M3 inverse_vjp(const M3 &Di, const M3 &Dib) {
    const M3 DiT = transpose(Di);
    M3 r = mul(DiT, mul(Dib, DiT));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = -r.a[i][j];
    return r;
}

bool in_domain(const ora_config *c, const double xp[3]) {
    for (int a = 0; a < 3; ++a) {
        const double X = (xp[a] - c->origin[a]) / c->dx;
        if (!(X >= 0.25 && X < c->n_cells[a] - 0.25)) return false;
    }
    return true;
}

bool sticky(const ora_config *c, const int32_t ijk[3], double k) {
    if (c->bc_band <= 0) return false;
    for (int a = 0; a < 3; ++a) {
        const double pos = ijk[a] + k / 4.0;  // node coordinate in cells from the origin
        if (pos < c->bc_band || pos > c->n_cells[a] - c->bc_band) return true;
    }
    return false;
}

void cross(const double a[3], const double b[3], double out[3]) {
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

}  // namespace

extern "C" {

double ora_K1(double x) { return K1(x); }
double ora_dK1(double x) { return dK1(x); }
double ora_d2K1(double x) { return d2K1(x); }

int ora_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

// Threads of the following parallel loops (timing only; results do not depend on it).
void ora_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void ora_stencil(const ora_config *cfg, const double xp[3], int32_t nodes[2][8][3], double w[2][8], double dpos[2][8][3]) {
    Stencil st;
    stencil(cfg, xp, st);
    for (int g = 0; g < 2; ++g)
        for (int o = 0; o < 8; ++o) {
            w[g][o] = st.w[g][o];
            for (int a = 0; a < 3; ++a) {
                nodes[g][o][a] = st.ijk[g][o][a];
                dpos[g][o][a] = st.d[g][o][a];
            }
        }
}

void ora_moment_matrix(const ora_config *cfg, const double xp[3], double D[9]) {
    Stencil st;
    stencil(cfg, xp, st);
    store3(moment_matrix(st), D);
}

int ora_svd3(const double F[9], double U[9], double S[3], double V[9]) {
    M3 u, v;
    svd_jacobi(load3(F), u, S, v);
    store3(u, U);
    store3(v, V);
    return 0;
}

void ora_kirchhoff(const ora_material *m, double logE, const double F[9], double tau[9]) {
    store3(kirchhoff(m, logE, load3(F)), tau);
}

double ora_energy_density(const ora_material *m, double logE, const double F[9]) {
    return energy_density(m, logE, load3(F));
}

void ora_kirchhoff_vjp(const ora_material *m, double logE, const double F[9], const double tb[9], double Fb[9],
                       double *logEb) {
    M3 fb;
    double lb = 0.0;
    kirchhoff_fc_vjp(m, logE, load3(F), load3(tb), fb, lb);
    store3(fb, Fb);
    if (logEb) *logEb = lb;
}

void ora_dp_return_map(const ora_material *m, double logE, double F[9]) {
    M3 f = load3(F);
    dp_return_map(m, logE, f);
    store3(f, F);
}

// Cell keys for the particle sort: the particle's G- cell c = floor((x - origin)/dx + 1/4)
// per axis, grouped by its 4x4x4-cell block: key = (block id) * 64 + (cell within block),
// block id = (bz * NBy + by) * NBx + bx with NB_a = n_cells[a]/4 + 1, cell within block
// = (cz mod 4) * 16 + (cy mod 4) * 4 + (cx mod 4).  Positions are the FP32 values the GPU
// sees, promoted exactly to FP64.  `bad` counts particles outside the valid domain.
void ora_cell_keys(const ora_config *cfg, int64_t n, const float *x_soa, int64_t stride, uint32_t *keys, int32_t *bad) {
    const int64_t NB[3] = {cfg->n_cells[0] / 4 + 1, cfg->n_cells[1] / 4 + 1, cfg->n_cells[2] / 4 + 1};
    int32_t nbad = 0;
    for (int64_t p = 0; p < n; ++p) {
        double xp[3];
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            xp[a] = (double)x_soa[a * stride + p];
            c[a] = (int64_t)std::floor((xp[a] - cfg->origin[a]) / cfg->dx + 0.25);
        }
        if (!in_domain(cfg, xp)) {
            ++nbad;
            keys[p] = 0xffffffffu;
            continue;
        }
        const int64_t vb = ((c[2] >> 2) * NB[1] + (c[1] >> 2)) * NB[0] + (c[0] >> 2);
        keys[p] = (uint32_t)((vb << 6) | ((c[2] & 3) * 16 + (c[1] & 3) * 4 + (c[0] & 3)));
    }
    if (bad) *bad = nbad;
}

void ora_stable_sort(int64_t n, const uint32_t *keys, uint32_t *perm) {
    std::vector<uint32_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0u);
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return keys[a] < keys[b]; });
    std::copy(idx.begin(), idx.end(), perm);
}

// One explicit step, in the pipeline order of section 3.2 with the dual-grid
// transfers of sections 4.3-4.5:
//   P2G (mass, APIC/MLS momentum) -> stress force -> grid update (gravity, walls)
//   -> G2P (velocity, affine matrix B) -> F update -> plasticity -> advection.
// Returns 0 on success, 3 if a particle lies outside the valid domain
// (some node of its stencil would be off the grid).
//
// diag (32 doubles):
//   [0] particle mass, [1..3] particle momentum, [4..6] particle angular momentum (with the B term),
//   [7] grid mass 1/2 sum m, [8..10] grid momentum 1/2 sum m v after the transfer,
//   [11..13] grid angular momentum 1/2 sum x_i x m v, [14..16] total force 1/2 sum f,
//   [17..19] total torque 1/2 sum x_i x f, [20..22] grid momentum after the update 1/2 sum m v~,
//   [23..25] grid angular momentum after the update about the moved nodes x_i + dt v~,
//   [26..28] particle momentum after G2P, [29..31] particle angular momentum after G2P.
int ora_step(const ora_config *cfg, const ora_material *mats, int32_t n_mat, int64_t n, double *x, double *v, double *B,
             double *F, const uint8_t *mat, const double *logE, double dt, ora_outputs *out) {
    for (int64_t p = 0; p < n; ++p)
        if (!in_domain(cfg, x + 3 * p)) return 3;
    for (int64_t p = 0; p < n; ++p)
        if (mat && mat[p] >= n_mat) return 1;

    const int64_t nx = cfg->n_cells[0] + 1, ny = cfg->n_cells[1] + 1, nz = cfg->n_cells[2] + 1;
    const int64_t nodes = nx * ny * nz;
    const bool mls = (cfg->transfer == 0);
    const bool pic = (cfg->transfer == 2);   // section 4.3: no affine term, particles carry no B
    std::vector<double> gm(2 * nodes, 0.0), gmv(6 * nodes, 0.0), gf(6 * nodes, 0.0), gv(6 * nodes, 0.0);
    double diag[32] = {0};

    auto material = [&](int64_t p) -> const ora_material * { return &mats[mat ? mat[p] : 0]; };
    auto mass = [&](int64_t p) { return material(p)->rho * material(p)->vol0; };
    auto logEp = [&](int64_t p) { return logE ? logE[p] : std::nan(""); };

    // particle totals before the step (supplement eqs. 1 and 3)
    for (int64_t p = 0; p < n; ++p) {
        const double m = mass(p);
        diag[0] += m;
        double mv[3], L[3];
        for (int a = 0; a < 3; ++a) mv[a] = m * v[3 * p + a];
        cross(x + 3 * p, mv, L);
        const double *b = B + 9 * p;
        L[0] += m * (b[2 * 3 + 1] - b[1 * 3 + 2]);
        L[1] += m * (b[0 * 3 + 2] - b[2 * 3 + 0]);
        L[2] += m * (b[1 * 3 + 0] - b[0 * 3 + 1]);
        for (int a = 0; a < 3; ++a) {
            diag[1 + a] += mv[a];
            diag[4 + a] += L[a];
        }
    }

    // per-particle D^-1 and Kirchhoff stress (independent per particle)
    std::vector<double> Dinv(9 * n), tau(9 * n);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        Stencil st;
        stencil(cfg, x + 3 * p, st);
        store3(inverse(moment_matrix(st)), &Dinv[9 * p]);
        store3(kirchhoff(material(p), logEp(p), load3(F + 9 * p)), &tau[9 * p]);
    }

    // P2G (serial scatter, fixed order).  Mass and APIC momentum, section 4.4:
    //   m_ik += w m_p;  (m v)_ik += w m_p (v_p + B_p D_p^-1 (x_i - x_p)).
    // Force, section 4.3 with the MLS gradient of section 4.5 (or the exact kernel
    // gradient for the APIC variant):
    //   f_ik -= V_p^0 tau_p grad Phi_ik,  grad Phi_ik = w D_p^-1 (x_i - x_p)  (MLS).
    for (int64_t p = 0; p < n; ++p) {
        Stencil st;
        stencil(cfg, x + 3 * p, st);
        const double m = mass(p), V0 = material(p)->vol0;
        const M3 Di = load3(&Dinv[9 * p]), T = load3(&tau[9 * p]), Bp = load3(B + 9 * p);
        const M3 BD = mul(Bp, Di);
        for (int g = 0; g < 2; ++g)
            for (int o = 0; o < 8; ++o) {
                const int64_t id = st.node[g][o];
                const double w = st.w[g][o];
                double grad[3];
                if (mls) {
                    for (int a = 0; a < 3; ++a) {
                        grad[a] = 0;
                        for (int b = 0; b < 3; ++b) grad[a] += w * Di.a[a][b] * st.d[g][o][b];
                    }
                } else {
                    for (int a = 0; a < 3; ++a) grad[a] = st.gw[g][o][a];
                }
                gm[g * nodes + id] += w * m;
                for (int a = 0; a < 3; ++a) {
                    double aff = 0, fa = 0;
                    for (int b = 0; b < 3; ++b) {
                        if (!pic) aff += BD.a[a][b] * st.d[g][o][b];
                        fa += T.a[a][b] * grad[b];
                    }
                    gmv[(g * nodes + id) * 3 + a] += w * m * (v[3 * p + a] + aff);
                    gf[(g * nodes + id) * 3 + a] -= V0 * fa;
                }
            }
    }

    // Grid update, section 4.3: m v~ = m v + dt f, plus gravity; walls; v~ = 0 where m = 0.
#pragma omp parallel for schedule(static)
    for (int64_t id = 0; id < 2 * nodes; ++id) {
        const int g = (int)(id / nodes);
        const int64_t r = id % nodes;
        const int32_t ijk[3] = {(int32_t)(r % nx), (int32_t)((r / nx) % ny), (int32_t)(r / (nx * ny))};
        const double mm = gm[id];
        for (int a = 0; a < 3; ++a) gv[id * 3 + a] = 0.0;
        if (mm > 0.0 && !sticky(cfg, ijk, g == 0 ? -1.0 : 1.0))
            for (int a = 0; a < 3; ++a) gv[id * 3 + a] = (gmv[id * 3 + a] + dt * gf[id * 3 + a]) / mm + dt * cfg->gravity[a];
    }
    (void)nz;

    // grid totals (supplement eqs. 1, 2; angular momentum after the update about moved nodes)
    for (int64_t id = 0; id < 2 * nodes; ++id) {
        const double mm = gm[id];
        if (mm == 0.0) continue;
        const int g = (int)(id / nodes);
        const int64_t r = id % nodes;
        const int32_t ijk[3] = {(int32_t)(r % nx), (int32_t)((r / nx) % ny), (int32_t)(r / (nx * ny))};
        double xi[3], xm[3], L[3], T[3], Lm[3], mvt[3];
        for (int a = 0; a < 3; ++a) {
            xi[a] = cfg->origin[a] + (ijk[a] + (g == 0 ? -0.25 : 0.25)) * cfg->dx;
            xm[a] = xi[a] + dt * gv[id * 3 + a];
            mvt[a] = mm * gv[id * 3 + a];
        }
        cross(xi, &gmv[id * 3], L);
        cross(xi, &gf[id * 3], T);
        cross(xm, mvt, Lm);
        diag[7] += 0.5 * mm;
        for (int a = 0; a < 3; ++a) {
            diag[8 + a] += 0.5 * gmv[id * 3 + a];
            diag[11 + a] += 0.5 * L[a];
            diag[14 + a] += 0.5 * gf[id * 3 + a];
            diag[17 + a] += 0.5 * T[a];
            diag[20 + a] += 0.5 * mvt[a];
            diag[23 + a] += 0.5 * Lm[a];
        }
    }

    // G2P, sections 4.3-4.5 and the supplement:
    //   v_p = 1/2 sum_k sum_i w v~_i,  B_p = 1/2 sum sum w v~_i (x_i - x_p)^T,
    //   grad v = B_p D_p^-1 (MLS) or 1/2 sum sum v~_i grad w^T (APIC),
    //   F <- (I + dt grad v) F, return mapping, x <- x + dt v_p.
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        Stencil st;
        stencil(cfg, x + 3 * p, st);
        double vp[3] = {0, 0, 0};
        M3 Bn = zero3(), G = zero3();
        for (int g = 0; g < 2; ++g)
            for (int o = 0; o < 8; ++o) {
                const double *vi = &gv[(g * nodes + st.node[g][o]) * 3];
                const double w = st.w[g][o];
                for (int a = 0; a < 3; ++a) {
                    vp[a] += 0.5 * w * vi[a];
                    for (int b = 0; b < 3; ++b) {
                        Bn.a[a][b] += 0.5 * w * vi[a] * st.d[g][o][b];
                        G.a[a][b] += 0.5 * vi[a] * st.gw[g][o][b];
                    }
                }
            }
        const M3 C = mls ? mul(Bn, load3(&Dinv[9 * p])) : G;
        M3 A = eye3();
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A.a[a][b] += dt * C.a[a][b];
        M3 Fn = mul(A, load3(F + 9 * p));
        if (material(p)->model == 1) dp_return_map(material(p), logEp(p), Fn);
        store3(Fn, F + 9 * p);
        store3(pic ? zero3() : Bn, B + 9 * p);
        for (int a = 0; a < 3; ++a) {
            v[3 * p + a] = vp[a];
            x[3 * p + a] += dt * vp[a];
        }
    }

    for (int64_t p = 0; p < n; ++p) {
        const double m = mass(p);
        double mv[3], L[3];
        for (int a = 0; a < 3; ++a) mv[a] = m * v[3 * p + a];
        cross(x + 3 * p, mv, L);
        const double *b = B + 9 * p;
        L[0] += m * (b[2 * 3 + 1] - b[1 * 3 + 2]);
        L[1] += m * (b[0 * 3 + 2] - b[2 * 3 + 0]);
        L[2] += m * (b[1 * 3 + 0] - b[0 * 3 + 1]);
        for (int a = 0; a < 3; ++a) {
            diag[26 + a] += mv[a];
            diag[29 + a] += L[a];
        }
    }

    if (out) {
        if (out->grid_m) std::copy(gm.begin(), gm.end(), out->grid_m);
        if (out->grid_p)
            for (int64_t i = 0; i < 6 * nodes; ++i) out->grid_p[i] = gmv[i] + dt * gf[i];
        if (out->grid_v) std::copy(gv.begin(), gv.end(), out->grid_v);
        if (out->diag) std::copy(diag, diag + 32, out->diag);
    }
    return 0;
}

// One explicit step with the quadratic B-spline kernel on a single grid (node i at
// origin + i dx, the 27 nodes of the 3x3x3 neighbourhood), the baseline of the
// paper's comparison (section 6): the same MLS transfers, constitutive models,
// grid update and return mapping as ora_step, with the sums over one grid only:
//   m_i = sum_p w m_p,  p_i = sum_p w (m_p v_p + (m_p B_p - dt V0 tau_p) D_p^-1 d),
//   D_p = sum_i w d d^T  (= dx^2/4 I for this kernel),
//   v_p = sum_i w v~_i,  B_p = sum_i w v~_i d^T,  F <- (I + dt B_p D_p^-1) F.
// Valid positions: (x - origin)/dx in [1/2, n - 1/2) on every axis (all 27 nodes on
// the grid).  grid_m / grid_p / grid_v hold the single grid ([nodes] / [nodes][3]);
// diag as for ora_step with the grid totals taken over the one grid.
int ora_step_quadratic(const ora_config *cfg, const ora_material *mats, int32_t n_mat, int64_t n, double *x,
                       double *v, double *B, double *F, const uint8_t *mat, const double *logE, double dt,
                       ora_outputs *out) {
    for (int64_t p = 0; p < n; ++p) {
        for (int a = 0; a < 3; ++a) {
            const double X = (x[3 * p + a] - cfg->origin[a]) / cfg->dx;
            if (!(X >= 0.5 && X < cfg->n_cells[a] - 0.5)) return 3;
        }
        if (mat && mat[p] >= n_mat) return 1;
    }
    const int64_t nx = cfg->n_cells[0] + 1, ny = cfg->n_cells[1] + 1, nz = cfg->n_cells[2] + 1;
    const int64_t nodes = nx * ny * nz;
    std::vector<double> gm(nodes, 0.0), gp(3 * nodes, 0.0), gv(3 * nodes, 0.0);
    double diag[32] = {0};
    auto material = [&](int64_t p) -> const ora_material * { return &mats[mat ? mat[p] : 0]; };
    auto mass = [&](int64_t p) { return material(p)->rho * material(p)->vol0; };
    auto logEp = [&](int64_t p) { return logE ? logE[p] : std::nan(""); };
    // the 27 nodes of a particle: index, weight, d = x_i - x_p
    struct Q27 {
        int64_t id[27];
        double w[27], d[27][3];
    };
    auto stencil27 = [&](const double *xp, Q27 &q) {
        int32_t base[3];
        for (int a = 0; a < 3; ++a) base[a] = (int32_t)std::floor((xp[a] - cfg->origin[a]) / cfg->dx - 0.5);
        for (int o = 0; o < 27; ++o) {
            const int off[3] = {o % 3, (o / 3) % 3, o / 9};
            int32_t ijk[3];
            double w = 1.0;
            for (int a = 0; a < 3; ++a) {
                ijk[a] = base[a] + off[a];
                q.d[o][a] = cfg->origin[a] + ijk[a] * cfg->dx - xp[a];
                w *= Nq(q.d[o][a] / cfg->dx);
            }
            q.w[o] = w;
            q.id[o] = node_index(cfg, ijk);
        }
    };
    for (int64_t p = 0; p < n; ++p) {
        const double m = mass(p);
        diag[0] += m;
        for (int a = 0; a < 3; ++a) diag[1 + a] += m * v[3 * p + a];
    }
    // P2G (serial scatter)
    for (int64_t p = 0; p < n; ++p) {
        Q27 q;
        stencil27(x + 3 * p, q);
        M3 D = zero3();
        for (int o = 0; o < 27; ++o)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) D.a[a][b] += q.w[o] * q.d[o][a] * q.d[o][b];
        const M3 Di = inverse(D);
        const M3 T = kirchhoff(material(p), logEp(p), load3(F + 9 * p));
        const double m = mass(p), V0 = material(p)->vol0;
        M3 A;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) A.a[i][j] = m * B[9 * p + 3 * i + j] - dt * V0 * T.a[i][j];
        const M3 Qm = mul(A, Di);
        for (int o = 0; o < 27; ++o) {
            gm[q.id[o]] += q.w[o] * m;
            for (int a = 0; a < 3; ++a) {
                double qd = 0;
                for (int b = 0; b < 3; ++b) qd += Qm.a[a][b] * q.d[o][b];
                gp[3 * q.id[o] + a] += q.w[o] * (m * v[3 * p + a] + qd);
            }
        }
    }
    // grid update
    for (int64_t id = 0; id < nodes; ++id) {
        const int32_t ijk[3] = {(int32_t)(id % nx), (int32_t)((id / nx) % ny), (int32_t)(id / (nx * ny))};
        if (gm[id] > 0.0 && !sticky(cfg, ijk, 0.0))
            for (int a = 0; a < 3; ++a) gv[3 * id + a] = gp[3 * id + a] / gm[id] + dt * cfg->gravity[a];
        if (gm[id] > 0.0) {
            diag[7] += gm[id];
            for (int a = 0; a < 3; ++a) {
                diag[8 + a] += gp[3 * id + a];
                diag[20 + a] += gm[id] * gv[3 * id + a];
            }
        }
    }
    (void)nz;
    // G2P
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        Q27 q;
        stencil27(x + 3 * p, q);
        M3 D = zero3(), Bn = zero3();
        double vp[3] = {0, 0, 0};
        for (int o = 0; o < 27; ++o) {
            const double *vi = &gv[3 * q.id[o]];
            for (int a = 0; a < 3; ++a) {
                vp[a] += q.w[o] * vi[a];
                for (int b = 0; b < 3; ++b) {
                    Bn.a[a][b] += q.w[o] * vi[a] * q.d[o][b];
                    D.a[a][b] += q.w[o] * q.d[o][a] * q.d[o][b];
                }
            }
        }
        const M3 C = mul(Bn, inverse(D));
        M3 Ip = eye3();
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Ip.a[a][b] += dt * C.a[a][b];
        M3 Fn = mul(Ip, load3(F + 9 * p));
        if (material(p)->model == 1) dp_return_map(material(p), logEp(p), Fn);
        store3(Fn, F + 9 * p);
        store3(Bn, B + 9 * p);
        for (int a = 0; a < 3; ++a) {
            v[3 * p + a] = vp[a];
            x[3 * p + a] += dt * vp[a];
        }
    }
    for (int64_t p = 0; p < n; ++p)
        for (int a = 0; a < 3; ++a) diag[26 + a] += mass(p) * v[3 * p + a];
    if (out) {
        if (out->grid_m) std::copy(gm.begin(), gm.end(), out->grid_m);
        if (out->grid_p) std::copy(gp.begin(), gp.end(), out->grid_p);
        if (out->grid_v) std::copy(gv.begin(), gv.end(), out->grid_v);
        if (out->diag) std::copy(diag, diag + 32, out->diag);
    }
    return 0;
}

double ora_Nq(double r) { return Nq(r); }
double ora_dNq(double r) { return dNq(r); }

// Reverse-mode derivative (vector-Jacobian product) of one MLS step with the
// fixed-corotated model, for the differentiable rollout: given the state entering
// the step (x, v, B, F, logE) and the cotangents of the state it produces
// (xb_out .. Fb_out), returns the cotangents of the entering state and of logE.
// The forward step is recomputed here; then its three phases are reversed in
// turn, every product rule written out:
//   G2P:  x' = x + dt v',  v' = 1/2 sum w v~,  B' = 1/2 sum w v~ d^T,
//         F' = (I + dt B' D^-1) F,  with w, d = x_i - x and D depending on x;
//   grid: v~ = p / m + dt g where m > 0 and the node is free, else 0;
//   P2G:  m_i = sum w m_p,  p_i = sum w (m_p v + (m_p B - dt V0 tau) D^-1 d).
// Returns 0 on success, 1 for a bad material index, 2 for a configuration it does
// not differentiate (Drucker-Prager or the exact-gradient transfer), 3 for a
// particle outside the valid domain.
int ora_step_vjp(const ora_config *cfg, const ora_material *mats, int32_t n_mat, int64_t n, const double *x,
                 const double *v, const double *B, const double *F, const uint8_t *mat, const double *logE, double dt,
                 const double *xb_out, const double *vb_out, const double *Bb_out, const double *Fb_out, double *xb,
                 double *vb, double *Bb, double *Fb, double *logEb) {
    if (cfg->transfer != 0) return 2;
    for (int64_t p = 0; p < n; ++p) {
        if (mat && mat[p] >= n_mat) return 1;
        if (mats[mat ? mat[p] : 0].model != 0) return 2;
        if (!in_domain(cfg, x + 3 * p)) return 3;
    }
    const int64_t nx = cfg->n_cells[0] + 1, ny = cfg->n_cells[1] + 1, nz = cfg->n_cells[2] + 1;
    const int64_t nodes = nx * ny * nz;
    auto material = [&](int64_t p) -> const ora_material * { return &mats[mat ? mat[p] : 0]; };
    auto logEp = [&](int64_t p) { return logE ? logE[p] : std::nan(""); };

    // ---- forward recomputation: D^-1, tau, grid mass and momentum, grid velocity
    std::vector<double> Dinv(9 * n), tau(9 * n), gm(2 * nodes, 0.0), gp(6 * nodes, 0.0), gv(6 * nodes, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        Stencil st;
        stencil(cfg, x + 3 * p, st);
        store3(inverse(moment_matrix(st)), &Dinv[9 * p]);
        store3(kirchhoff(material(p), logEp(p), load3(F + 9 * p)), &tau[9 * p]);
    }
    for (int64_t p = 0; p < n; ++p) {
        Stencil st;
        stencil(cfg, x + 3 * p, st);
        const double m = material(p)->rho * material(p)->vol0, V0 = material(p)->vol0;
        const M3 Di = load3(&Dinv[9 * p]), T = load3(&tau[9 * p]), Bp = load3(B + 9 * p);
        M3 A;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) A.a[i][j] = m * Bp.a[i][j] - dt * V0 * T.a[i][j];
        const M3 Q = mul(A, Di);
        for (int g = 0; g < 2; ++g)
            for (int o = 0; o < 8; ++o) {
                const int64_t id = g * nodes + st.node[g][o];
                const double w = st.w[g][o];
                gm[id] += w * m;
                for (int a = 0; a < 3; ++a) {
                    double qd = 0;
                    for (int b = 0; b < 3; ++b) qd += Q.a[a][b] * st.d[g][o][b];
                    gp[id * 3 + a] += w * (m * v[3 * p + a] + qd);
                }
            }
    }
    std::vector<char> live(2 * nodes, 0);
    for (int64_t id = 0; id < 2 * nodes; ++id) {
        const int g = (int)(id / nodes);
        const int64_t r = id % nodes;
        const int32_t ijk[3] = {(int32_t)(r % nx), (int32_t)((r / nx) % ny), (int32_t)(r / (nx * ny))};
        if (gm[id] > 0.0 && !sticky(cfg, ijk, g == 0 ? -1.0 : 1.0)) {
            live[id] = 1;
            for (int a = 0; a < 3; ++a) gv[id * 3 + a] = gp[id * 3 + a] / gm[id] + dt * cfg->gravity[a];
        }
    }
    (void)nz;

    // ---- G2P reversed (per particle; the grid cotangent is summed serially)
    std::vector<double> gvb(6 * nodes, 0.0);
    for (int64_t p = 0; p < n; ++p) {
        Stencil st;
        stencil(cfg, x + 3 * p, st);
        const M3 Di = load3(&Dinv[9 * p]), Fp = load3(F + 9 * p), Fbo = load3(Fb_out + 9 * p);
        M3 Bn = zero3();
        for (int g = 0; g < 2; ++g)
            for (int o = 0; o < 8; ++o) {
                const double *vi = &gv[(g * nodes + st.node[g][o]) * 3];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) Bn.a[a][b] += 0.5 * st.w[g][o] * vi[a] * st.d[g][o][b];
            }
        const M3 C = mul(Bn, Di);
        double xbar[3], vbt[3];
        for (int a = 0; a < 3; ++a) {
            xbar[a] = xb_out[3 * p + a];
            vbt[a] = vb_out[3 * p + a] + dt * xb_out[3 * p + a];
        }
        M3 Cb = mul(Fbo, transpose(Fp));
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Cb.a[i][j] *= dt;
        M3 IC = eye3();
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) IC.a[i][j] += dt * C.a[i][j];
        store3(mul(transpose(IC), Fbo), Fb + 9 * p);
        M3 Bbt = mul(Cb, transpose(Di));
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Bbt.a[i][j] += Bb_out[9 * p + 3 * i + j];
        const M3 Dib = mul(transpose(Bn), Cb);
        for (int g = 0; g < 2; ++g)
            for (int o = 0; o < 8; ++o) {
                const int64_t id = g * nodes + st.node[g][o];
                const double *vi = &gv[id * 3];
                const double w = st.w[g][o];
                double gvec[3], wb = 0;
                for (int a = 0; a < 3; ++a) {
                    gvec[a] = vbt[a];
                    for (int b = 0; b < 3; ++b) gvec[a] += Bbt.a[a][b] * st.d[g][o][b];
                }
                for (int a = 0; a < 3; ++a) {
                    gvb[id * 3 + a] += 0.5 * w * gvec[a];
                    wb += 0.5 * vi[a] * gvec[a];
                }
                for (int b = 0; b < 3; ++b) {
                    double db = 0;   // dL/d(d_b) = 1/2 w (Bbt^T v~)_b ; d = x_i - x
                    for (int a = 0; a < 3; ++a) db += 0.5 * w * Bbt.a[a][b] * vi[a];
                    xbar[b] += wb * st.gw[g][o][b] - db;
                }
            }
        moment_matrix_vjp(st, inverse_vjp(Di, Dib), xbar);
        for (int a = 0; a < 3; ++a) xb[3 * p + a] = xbar[a];
    }

    // ---- grid update reversed: p-bar = v~-bar / m, m-bar = -(v~-bar . p) / m^2
    std::vector<double> gmb(2 * nodes, 0.0), gpb(6 * nodes, 0.0);
    for (int64_t id = 0; id < 2 * nodes; ++id) {
        if (!live[id]) continue;
        double dot = 0;
        for (int a = 0; a < 3; ++a) {
            gpb[id * 3 + a] = gvb[id * 3 + a] / gm[id];
            dot += gvb[id * 3 + a] * gp[id * 3 + a];
        }
        gmb[id] = -dot / (gm[id] * gm[id]);
    }

    // ---- P2G reversed (a gather per particle)
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        Stencil st;
        stencil(cfg, x + 3 * p, st);
        const double m = material(p)->rho * material(p)->vol0, V0 = material(p)->vol0;
        const M3 Di = load3(&Dinv[9 * p]), T = load3(&tau[9 * p]), Bp = load3(B + 9 * p);
        M3 A;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) A.a[i][j] = m * Bp.a[i][j] - dt * V0 * T.a[i][j];
        const M3 Q = mul(A, Di);
        double xbar[3] = {xb[3 * p], xb[3 * p + 1], xb[3 * p + 2]}, vbar[3] = {0, 0, 0};
        M3 Qb = zero3();
        for (int g = 0; g < 2; ++g)
            for (int o = 0; o < 8; ++o) {
                const int64_t id = g * nodes + st.node[g][o];
                const double w = st.w[g][o];
                const double *pb = &gpb[id * 3];
                double wb = m * gmb[id];
                for (int a = 0; a < 3; ++a) {
                    double pi = m * v[3 * p + a];
                    for (int b = 0; b < 3; ++b) pi += Q.a[a][b] * st.d[g][o][b];
                    wb += pb[a] * pi;
                    vbar[a] += w * m * pb[a];
                    for (int b = 0; b < 3; ++b) Qb.a[a][b] += w * pb[a] * st.d[g][o][b];
                }
                for (int b = 0; b < 3; ++b) {
                    double db = 0;   // dL/d(d_b) = w (Q^T p-bar)_b
                    for (int a = 0; a < 3; ++a) db += w * Q.a[a][b] * pb[a];
                    xbar[b] += wb * st.gw[g][o][b] - db;
                }
            }
        const M3 Ab = mul(Qb, transpose(Di));
        moment_matrix_vjp(st, inverse_vjp(Di, mul(transpose(A), Qb)), xbar);
        M3 tb;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                Bb[9 * p + 3 * i + j] = m * Ab.a[i][j];
                tb.a[i][j] = -dt * V0 * Ab.a[i][j];
            }
        M3 Ftb;
        double lb;
        kirchhoff_fc_vjp(material(p), logEp(p), load3(F + 9 * p), tb, Ftb, lb);
        for (int i = 0; i < 9; ++i) Fb[9 * p + i] += Ftb.a[i / 3][i % 3];
        if (logEb) logEb[p] = lb;
        for (int a = 0; a < 3; ++a) {
            xb[3 * p + a] = xbar[a];
            vb[3 * p + a] = vbar[a];
        }
    }
    return 0;
}

}  // extern "C"
