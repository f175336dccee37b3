/* FP64 CPU oracle for one compact-kernel MPM step (CK-MPM, arXiv 2412.10399).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke check
 * and the benchmark's CPU-baseline leg can check the HIP path against a plain,
 * slow, obviously correct implementation of the paper's method.  Nothing in the
 * product path may link, load or call it.  It shares no code with the HIP path.
 *
 * Conventions (all FP64):
 *  - grid G_k (k = -1, +1) node i (integer triple) sits at world position
 *    origin + (i + k/4) dx; node indices run 0..n_cells[a] on each axis;
 *  - particle arrays are array-of-structures: x[p*3+a], F[p*9 + 3*row + col];
 *  - dense grid arrays are indexed [g][node] with g = 0 for G-, 1 for G+ and
 *    node = (iz*(ny+1) + iy)*(nx+1) + ix; vector channels are [g][node][3].
 */
#ifndef CKMPM_ORACLE_H
#define CKMPM_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_cells[3];
    double dx;
    double origin[3];
    double gravity[3];
    int32_t bc_band;     /* sticky wall band width in cells (0 = no walls) */
    int32_t transfer;    /* 0 = MLS-MPM (section 4.5), 1 = APIC with exact kernel gradients (section 4.4),
                            2 = PIC (section 4.3: momentum m v only, exact kernel gradients, no B carried) */
} ora_config;

typedef struct {
    int32_t model;       /* 0 = fixed corotated, 1 = Drucker-Prager */
    double E, nu, rho, vol0, friction_deg;
} ora_material;

/* outputs of one step; any pointer may be NULL */
typedef struct {
    double *grid_m;      /* [2][nodes]    mass after P2G                       */
    double *grid_p;      /* [2][nodes][3] momentum after P2G                   */
    double *grid_v;      /* [2][nodes][3] velocity after the grid update       */
    double *diag;        /* 32 doubles, see ora_step                           */
} ora_outputs;

double ora_K1(double x);
double ora_dK1(double x);
double ora_d2K1(double x);
void   ora_stencil(const ora_config *cfg, const double xp[3], int32_t nodes[2][8][3], double w[2][8],
                   double dpos[2][8][3]);
void   ora_moment_matrix(const ora_config *cfg, const double xp[3], double D[9]);
int    ora_svd3(const double F[9], double U[9], double S[3], double V[9]);
void   ora_kirchhoff(const ora_material *m, double logE_or_nan, const double F[9], double tau[9]);
double ora_energy_density(const ora_material *m, double logE_or_nan, const double F[9]);
/* adjoint of the fixed-corotated stress: tb = dL/dtau -> dL/dF, dL/dlogE */
void   ora_kirchhoff_vjp(const ora_material *m, double logE, const double F[9], const double tb[9], double Fb[9],
                         double *logEb);
void   ora_dp_return_map(const ora_material *m, double logE_or_nan, double F[9]);
void   ora_cell_keys(const ora_config *cfg, int64_t n, const float *x_soa, int64_t stride, uint32_t *keys,
                     int32_t *bad);
void   ora_stable_sort(int64_t n, const uint32_t *keys, uint32_t *perm);
int    ora_step(const ora_config *cfg, const ora_material *mats, int32_t n_mat, int64_t n,
                double *x, double *v, double *B, double *F, const uint8_t *mat, const double *logE,
                double dt, ora_outputs *out);
/* Reverse-mode derivative of ora_step (fixed corotated, MLS transfer): cotangents of
 * the entering state (and of the per-particle log Young's modulus, when logE is
 * given) from those of the produced state; AoS layouts as above. */
int    ora_step_vjp(const ora_config *cfg, const ora_material *mats, int32_t n_mat, int64_t n, const double *x,
                    const double *v, const double *B, const double *F, const uint8_t *mat, const double *logE,
                    double dt, const double *xb_out, const double *vb_out, const double *Bb_out,
                    const double *Fb_out, double *xb, double *vb, double *Bb, double *Fb, double *logEb);
/* One step with the single-grid quadratic B-spline kernel (27 nodes), the
 * comparison baseline; grids in the outputs are the one grid ([nodes], [nodes][3]). */
int    ora_step_quadratic(const ora_config *cfg, const ora_material *mats, int32_t n_mat, int64_t n, double *x,
                          double *v, double *B, double *F, const uint8_t *mat, const double *logE, double dt,
                          ora_outputs *out);
double ora_Nq(double r);
double ora_dNq(double r);
int    ora_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
