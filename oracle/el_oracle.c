/*
 * FP64 CPU oracle for the elastic forward operator H and its adjoint H^T.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  It shares no code
 * with the GPU path (no headers, no helpers, no tables).
 *
 * What it computes (Mitsuhashi et al., "A forward-adjoint operator pair based
 * on the elastic wave equation for use in transcranial PACT"):
 *
 *   H  = M' T'_{M-1} ... T'_1 T'_0          (Appendix, Discrete formulation, eq. HPML)
 *   H^T = T'_0^T T'_1^T ... T'_{M-1}^T M'^T  (eq. adjHPML)
 *
 * applied to vectors.  The state is the paper's 27N vector
 *   v'_m = [ phi (9N) ; u (3N) ; psi (9N) ; sigma (6N) ]
 * with phi/psi ordered 11,12,13,21,22,23,31,32,33 (eq. auxPML) and sigma in
 * Voigt order 11,22,33,23,13,12 (Sec. 2.2).  Memory variables are stored on
 * the whole grid, exactly as in the paper's matrices; they stay zero where
 * the PML coefficient a vanishes.
 *
 * One forward step W' is the four sub-updates of the Appendix discrete
 * formulation (phi, then u, then psi, then sigma).  The adjoint step W'^T is
 * written as the transposes of those four linear maps in reverse order; each
 * transposed difference is evaluated in gather form, i.e. by visiting the
 * same (output point, input point, weight) triples as the forward difference
 * from the input side.  No step of it is derived from the GPU kernels.
 *
 * Readings taken where the paper is silent or garbled (all documented in the
 * design notes):
 *  - staggered positions: normal stresses, lambda, mu, p0 at (i,j,k);
 *    u^1 at (i+1/2,j,k), u^2 at (i,j+1/2,k), u^3 at (i,j,k+1/2);
 *    sigma12 at (i+1/2,j+1/2,k), sigma13 at (i+1/2,j,k+1/2),
 *    sigma23 at (i,j+1/2,k+1/2); every array has N entries and values
 *    outside the grid are zero;
 *  - 4th-order staggered difference (Sec. 2.2, eq. derivative), forward
 *    type  D+f[i] = (9/8 (f[i+1]-f[i]) - 1/24 (f[i+2]-f[i-1])) / dx  and
 *    backward type  D-f[i] = (9/8 (f[i]-f[i-1]) - 1/24 (f[i+1]-f[i-2])) / dx;
 *  - rho and alpha at velocity points: arithmetic mean of the two adjacent
 *    cells (Sec. 6 methods), the upper neighbour replicated at the last index;
 *    mu at shear points: harmonic mean of the four adjacent cells, 0 if any
 *    of them is 0; lambda, mu at normal points: the cell value;
 *  - injection tau' = -1/3 on sigma11, sigma22, sigma33 (Sec. 3, eq. Ini and
 *    eq. initialp0; the Appendix's -I conflicts with eq. p0);
 *  - measurement row  -R_l (sigma11+sigma22+sigma33), trilinear R_l on the
 *    normal-stress grid, base index clamped to n-2; a receiver must lie in
 *    [0, n-1] cells on each axis (1e-9 cells of rounding allowed, clamped);
 *  - nsteps = M samples including m = 0, hence M-1 applications of W';
 *  - adjoint recursion v_{m-1} = Theta^T p_{m-1} + W^T v_m (Sec. 4, eq. Adjup);
 *  - memory variable phi^{ij} lives at the u^i point, psi^{ij} at the
 *    sigma^{ij} point; its a, b, chi use axis j at that point's coordinate;
 *  - C-PML profile (kappa = 1, Appendix A.2): d = d0 xi^n,
 *    d0 = -(n+1) c_max ln(R) / (2 P dx), beta = pi f0 (1 - xi),
 *    xi = depth into the layer / P clamped to [0,1], measured from the inner
 *    planes P and n-1-P; b = exp(-(d+beta) dt), a = d/(d+beta) (b-1).
 *
 * Frequency-dependent absorption (the extension the conclusion, Sec. 8, asks
 * for, of the velocity damping alpha u of Sec. 2.1 eq. subeq1): optional
 * relaxation mechanisms add sum_l beta_l (u - zeta_l) to the damping, with
 * d/dt zeta_l = omega_l (u - zeta_l), i.e. a damping rate
 *   a(omega) = alpha + sum_l beta_l i omega / (omega_l + i omega)
 * that grows with frequency.  Discretely, a pointwise sub-update R follows the
 * velocity update (2) of every step (relax_matrix); the adjoint step applies
 * R^T, the transpose of the same matrix, at the mirrored place.  The memory
 * variables zeta_l extend the state after the paper's 27N entries.
 *
 * Parity unpinned: the C-PML constants (d0, R, beta, f0) are a convention
 * that no value of the paper fixes; the tests hold the oracle to their stated
 * form only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny, nz;
    double dx, dt;
    int32_t nsteps, npml;
    double pml_R, pml_npower, pml_f0;
} eo_grid;

typedef struct {
    eo_grid g;
    int64_t N;
    int n[3];                 /* nx, ny, nz                                    */
    int64_t stride[3];        /* 1, nx, nx*ny                                  */
    double *rho_u[3];         /* rho at u^i points                            */
    double *alpha_u[3];       /* alpha at u^i points                          */
    double *lam, *mu;         /* at normal-stress points                      */
    double *mu_s[3];          /* mu at sigma23, sigma13, sigma12 points       */
    /* 1-D PML profiles: [axis][0 = integer position, 1 = half position][n] */
    double *pa[3][2], *pb[3][2], *pchi[3][2];
    double cmax;
    int32_t nrec;
    int64_t *rbase;           /* [L][8] cell indices of the 8 trilinear corners */
    double *rw;               /* [L][8] weights                                */
    int32_t *coord[3];        /* x, y, z index of every grid point             */
    /* frequency-dependent absorption (relaxation mechanisms l = 0..nmech-1):
       damping alpha u + sum_l beta_l (u - zeta_l), d/dt zeta_l = omega_l (u - zeta_l),
       beta_l = w_l * beta_u; zeta_l stored after the 27N state, 3 arrays per mechanism */
    int nmech;
    double mech_w[4], mech_c[4];   /* weights w_l and c_l = exp(-omega_l dt)        */
    double *beta_u[3];        /* relaxation strength at u^i points (NULL if nmech = 0) */
} eo_model;

/* Length of the state vector: the 27N of the Appendix plus 3N per relaxation mechanism. */
static int64_t state_len(const eo_model *m) { return (int64_t)(27 + 3 * m->nmech) * m->N; }

/* ---------------------------------------------------------------- helpers */

/* Taps of the two difference types along one axis: out[p] = sum w_t f[p+o_t]. */
static const int OFF_P[4] = {1, 0, 2, -1};     /* D+ (value at +1/2 from integer samples) */
static const double WGT_P[4] = {9.0 / 8.0, -9.0 / 8.0, -1.0 / 24.0, 1.0 / 24.0};
static const int OFF_M[4] = {0, -1, 1, -2};    /* D- (value at integer from +1/2 samples) */
static const double WGT_M[4] = {9.0 / 8.0, -9.0 / 8.0, -1.0 / 24.0, 1.0 / 24.0};

enum { DPLUS = 0, DMINUS = 1 };


/* out[p] += coef[p] * scale * (D_axis f)[p]   (coef may be NULL = 1) */
static void diff_fwd(const eo_model *m, int axis, int kind, const double *coef, double scale,
                     const double *f, double *out) {
    const int *off = kind == DPLUS ? OFF_P : OFF_M;
    const double *w = kind == DPLUS ? WGT_P : WGT_M;
    const double inv = scale / m->g.dx;
    const int n = m->n[axis];
    const int64_t st = m->stride[axis];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < m->n[2]; ++k) {
        for (int j = 0; j < m->n[1]; ++j) {
            for (int i = 0; i < m->n[0]; ++i) {
                int64_t p = i + (int64_t)m->n[0] * (j + (int64_t)m->n[1] * k);
                int c = axis == 0 ? i : (axis == 1 ? j : k);
                double s = 0.0;
                for (int t = 0; t < 4; ++t) {
                    int q = c + off[t];
                    if (q >= 0 && q < n) s += w[t] * f[p + (int64_t)off[t] * st];
                }
                out[p] += (coef ? coef[p] : 1.0) * inv * s;
            }
        }
    }
}

/* Transpose of diff_fwd:  ft[n] += sum_p D[p][n] coef[p] scale outt[p], in gather form. */
static void diff_tr(const eo_model *m, int axis, int kind, const double *coef, double scale,
                    const double *outt, double *ft) {
    const int *off = kind == DPLUS ? OFF_P : OFF_M;
    const double *w = kind == DPLUS ? WGT_P : WGT_M;
    const double inv = scale / m->g.dx;
    const int n = m->n[axis];
    const int64_t st = m->stride[axis];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < m->n[2]; ++k) {
        for (int j = 0; j < m->n[1]; ++j) {
            for (int i = 0; i < m->n[0]; ++i) {
                int64_t q = i + (int64_t)m->n[0] * (j + (int64_t)m->n[1] * k);
                int c = axis == 0 ? i : (axis == 1 ? j : k);
                double s = 0.0;
                for (int t = 0; t < 4; ++t) {
                    int pc = c - off[t];          /* output point p with p + off = q */
                    if (pc >= 0 && pc < n) {
                        int64_t p = q - (int64_t)off[t] * st;
                        s += w[t] * (coef ? coef[p] : 1.0) * outt[p];
                    }
                }
                ft[q] += inv * s;
            }
        }
    }
}

/* 1-D profile value of the axis at the grid point p (coordinate looked up per point). */
static inline double prof(const eo_model *m, double *const tab[3][2], int axis, int half, int64_t p) {
    return tab[axis][half][m->coord[axis][p]];
}

/* ---------------------------------------------------------- state layout */
/* Voigt index of sigma^{ij} (0-based i, j). */
static int voigt(int i, int j) {
    if (i == j) return i;
    int s = i + j;            /* (1,2)->3 -> sigma23 ; (0,2)->2 -> sigma13 ; (0,1)->1 -> sigma12 */
    return s == 3 ? 3 : (s == 2 ? 4 : 5);
}
/* Shear-modulus array index for sigma^{ij}, i != j: 0 = 23, 1 = 13, 2 = 12. */
static int shear_id(int i, int j) { return voigt(i, j) - 3; }

typedef struct {
    double *phi[3][3];
    double *u[3];
    double *psi[3][3];
    double *sig[6];
    double *zeta[4][3];       /* relaxation memory variables [mechanism][component] */
} eo_view;

static eo_view view(const eo_model *m, double *v) {
    eo_view s;
    int64_t N = m->N;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s.phi[i][j] = v + (3 * i + j) * N;
    for (int i = 0; i < 3; ++i) s.u[i] = v + (9 + i) * N;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s.psi[i][j] = v + (12 + 3 * i + j) * N;
    for (int a = 0; a < 6; ++a) s.sig[a] = v + (21 + a) * N;
    for (int l = 0; l < 4; ++l)
        for (int i = 0; i < 3; ++i) s.zeta[l][i] = l < m->nmech ? v + (27 + 3 * l + i) * N : NULL;
    return s;
}

/* The relaxation sub-update R at one point of component i, as its (1+L) x (1+L) matrix on
   x = [u; zeta_0 .. zeta_{L-1}]:
     u'      = (u + dt sum_l beta_l zeta_l) / (1 + dt sum_l beta_l)
     zeta_l' = c_l zeta_l + (1 - c_l) u'
   (the damping term beta_l (u - zeta_l) taken at the new velocity, the memory variable
   advanced exactly for a velocity held at u' over the step). */
static void relax_matrix(const eo_model *m, int i, int64_t p, double R[5][5]) {
    const int L = m->nmech;
    const double dt = m->g.dt;
    double beta[4], B = 0.0;
    for (int l = 0; l < L; ++l) {
        beta[l] = m->mech_w[l] * m->beta_u[i][p];
        B += beta[l];
    }
    const double a = 1.0 / (1.0 + dt * B);
    R[0][0] = a;
    for (int l = 0; l < L; ++l) R[0][1 + l] = dt * beta[l] * a;
    for (int l = 0; l < L; ++l) {
        R[1 + l][0] = (1.0 - m->mech_c[l]) * R[0][0];
        for (int k = 0; k < L; ++k) R[1 + l][1 + k] = (1.0 - m->mech_c[l]) * R[0][1 + k] + (l == k ? m->mech_c[l] : 0.0);
    }
}

/* x <- R x (transpose = 0) or x <- R^T x (transpose = 1) at every point and component. */
static void relax(const eo_model *m, eo_view *s, int transpose) {
    const int L = m->nmech;
    for (int i = 0; i < 3; ++i) {
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < m->N; ++p) {
            double R[5][5], x[5], y[5] = {0.0};
            relax_matrix(m, i, p, R);
            x[0] = s->u[i][p];
            for (int l = 0; l < L; ++l) x[1 + l] = s->zeta[l][i][p];
            for (int r = 0; r <= L; ++r) {
                y[r] = 0.0;
                for (int c = 0; c <= L; ++c) y[r] += (transpose ? R[c][r] : R[r][c]) * x[c];
            }
            s->u[i][p] = y[0];
            for (int l = 0; l < L; ++l) s->zeta[l][i][p] = y[1 + l];
        }
    }
}

/* Derivative type of the velocity update along axis j for u^i (Sec. 2.2):
   D+ on sigma^{ii} along i, D- on sigma^{ij} along j != i.
   The stress update uses the opposite type: D- for d_i u^i, D+ for d_j u^i, j != i. */
static int vel_kind(int i, int j) { return i == j ? DPLUS : DMINUS; }
static int str_kind(int i, int j) { return i == j ? DMINUS : DPLUS; }
/* Position along axis j of the point where phi^{ij} (u^i point) lives: half if i == j.
   psi^{ij} lives at the sigma^{ij} point: half along j if i != j. */
static int phi_half(int i, int j) { return i == j; }
static int psi_half(int i, int j) { return i != j; }

/* ------------------------------------------------------------- one step */

/* v <- W' v  (Appendix, Discrete formulation: the four sub-updates). */
static void step_fwd(const eo_model *m, double *v, double *tmp) {
    const int64_t N = m->N;
    const double dt = m->g.dt;
    eo_view s = view(m, v);
    /* (1) phi^{ij}_{m+1/2} = b_j phi^{ij}_{m-1/2} + a_j D_j sigma^{ij}_m */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            memset(tmp, 0, sizeof(double) * N);
            diff_fwd(m, j, vel_kind(i, j), NULL, 1.0, s.sig[voigt(i, j)], tmp);
            int h = phi_half(i, j);
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < N; ++p)
                s.phi[i][j][p] = prof(m, m->pb, j, h, p) * s.phi[i][j][p] + prof(m, m->pa, j, h, p) * tmp[p];
        }
    /* (2) u^i_{m+1/2} = (1 - dt alpha_i) u^i + dt/rho_i sum_j (D_j sigma^{ij} + chi_j phi^{ij}) */
    for (int i = 0; i < 3; ++i) {
        memset(tmp, 0, sizeof(double) * N);
        for (int j = 0; j < 3; ++j) diff_fwd(m, j, vel_kind(i, j), NULL, 1.0, s.sig[voigt(i, j)], tmp);
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < N; ++p) {
            double acc = tmp[p];
            for (int j = 0; j < 3; ++j) acc += prof(m, m->pchi, j, phi_half(i, j), p) * s.phi[i][j][p];
            s.u[i][p] = (1.0 - dt * m->alpha_u[i][p]) * s.u[i][p] + dt / m->rho_u[i][p] * acc;
        }
    }
    /* (2b) frequency-dependent absorption: the relaxation sub-update R on (u, zeta) */
    if (m->nmech > 0) relax(m, &s, 0);
    /* (3) psi^{ij}_{m+1} = b_j psi^{ij}_m + a_j D_j u^i_{m+1/2} */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            memset(tmp, 0, sizeof(double) * N);
            diff_fwd(m, j, str_kind(i, j), NULL, 1.0, s.u[i], tmp);
            int h = psi_half(i, j);
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < N; ++p)
                s.psi[i][j][p] = prof(m, m->pb, j, h, p) * s.psi[i][j][p] + prof(m, m->pa, j, h, p) * tmp[p];
        }
    /* (4) sigma_{m+1} = sigma_m + Psi u_{m+1/2} + Delta psi_{m+1}  (Sec. 2.2 operator Psi,
           Appendix operator Delta).  Normal rows: dt [lambda sum_k (D_k u^k + psi^{kk})
           + 2 mu (D_i u^i + chi_i psi^{ii})]; the indicator multiplies only the mu part,
           as in the paper's Delta. */
    double *ekk = tmp;                     /* sum_k (D_k u^k + psi^{kk}) */
    double *dii = tmp + N;                 /* D_i u^i, one array per i   */
    memset(ekk, 0, sizeof(double) * 4 * N);
    for (int k = 0; k < 3; ++k) {
        diff_fwd(m, k, str_kind(k, k), NULL, 1.0, s.u[k], dii + k * N);
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < N; ++p) ekk[p] += dii[k * N + p] + s.psi[k][k][p];
    }
    for (int i = 0; i < 3; ++i) {
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < N; ++p)
            s.sig[i][p] += dt * (m->lam[p] * ekk[p]
                                 + 2.0 * m->mu[p] * (dii[i * N + p] + prof(m, m->pchi, i, 0, p) * s.psi[i][i][p]));
    }
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j) {
            double *g = tmp;           /* gamma_ij = D_j u^i + chi_j psi^{ij} + D_i u^j + chi_i psi^{ji} */
            memset(g, 0, sizeof(double) * N);
            diff_fwd(m, j, str_kind(i, j), NULL, 1.0, s.u[i], g);
            diff_fwd(m, i, str_kind(j, i), NULL, 1.0, s.u[j], g);
            const double *mus = m->mu_s[shear_id(i, j)];
            double *sg = s.sig[voigt(i, j)];
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < N; ++p) {
                double gg = g[p] + prof(m, m->pchi, j, psi_half(i, j), p) * s.psi[i][j][p]
                                 + prof(m, m->pchi, i, psi_half(j, i), p) * s.psi[j][i][p];
                sg[p] += dt * mus[p] * gg;
            }
        }
}

/* v <- W'^T v : transposes of sub-updates (4), (3), (2), (1) in that order. */
static void step_tr(const eo_model *m, double *v, double *tmp) {
    const int64_t N = m->N;
    const double dt = m->g.dt;
    eo_view s = view(m, v);
    /* (4)^T: sigma' = sigma + Psi u + Delta psi.  Adjoint: u~ += Psi^T s~, psi~ += Delta^T s~. */
    for (int i = 0; i < 3; ++i) {
        /* rows sigma_ii: dt*lambda*(D_k u^k + psi^{kk}) for every k, dt*2mu*(D_i u^i + chi_i psi^{ii}) */
        double *w = tmp;
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < N; ++p) w[p] = dt * m->lam[p] * s.sig[i][p];
        for (int k = 0; k < 3; ++k) {
            diff_tr(m, k, str_kind(k, k), NULL, 1.0, w, s.u[k]);
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < N; ++p) s.psi[k][k][p] += w[p];
        }
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < N; ++p) w[p] = dt * 2.0 * m->mu[p] * s.sig[i][p];
        diff_tr(m, i, str_kind(i, i), NULL, 1.0, w, s.u[i]);
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < N; ++p) s.psi[i][i][p] += prof(m, m->pchi, i, 0, p) * w[p];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j) {
            double *w = tmp;
            const double *mus = m->mu_s[shear_id(i, j)];
            const double *sg = s.sig[voigt(i, j)];
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < N; ++p) w[p] = dt * mus[p] * sg[p];
            diff_tr(m, j, str_kind(i, j), NULL, 1.0, w, s.u[i]);
            diff_tr(m, i, str_kind(j, i), NULL, 1.0, w, s.u[j]);
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < N; ++p) {
                s.psi[i][j][p] += prof(m, m->pchi, j, psi_half(i, j), p) * w[p];
                s.psi[j][i][p] += prof(m, m->pchi, i, psi_half(j, i), p) * w[p];
            }
        }
    /* (3)^T: psi' = B~ psi + A~ D u.  Adjoint: u~^i += D_j^T (a_j psi~^{ij}); psi~ <- b psi~. */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            int h = psi_half(i, j);
            double *w = tmp;
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < N; ++p) w[p] = prof(m, m->pa, j, h, p) * s.psi[i][j][p];
            diff_tr(m, j, str_kind(i, j), NULL, 1.0, w, s.u[i]);
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < N; ++p) s.psi[i][j][p] *= prof(m, m->pb, j, h, p);
        }
    /* (2b)^T: the transposed relaxation matrix on (u~, zeta~) */
    if (m->nmech > 0) relax(m, &s, 1);
    /* (2)^T: u' = J u + Phi sigma + Gamma phi.
       Adjoint: sigma~ += Phi^T u~, phi~ += Gamma^T u~ (with the incoming u~), then u~ <- J u~. */
    for (int i = 0; i < 3; ++i) {
        double *w = tmp;
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < N; ++p) w[p] = dt / m->rho_u[i][p] * s.u[i][p];
        for (int j = 0; j < 3; ++j) {
            diff_tr(m, j, vel_kind(i, j), NULL, 1.0, w, s.sig[voigt(i, j)]);
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < N; ++p) s.phi[i][j][p] += prof(m, m->pchi, j, phi_half(i, j), p) * w[p];
        }
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < N; ++p) s.u[i][p] *= (1.0 - dt * m->alpha_u[i][p]);
    }
    /* (1)^T: phi' = B phi + A D sigma.  Adjoint: sigma~ += D_j^T (a_j phi~^{ij}); phi~ <- b phi~. */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            int h = phi_half(i, j);
            double *w = tmp;
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < N; ++p) w[p] = prof(m, m->pa, j, h, p) * s.phi[i][j][p];
            diff_tr(m, j, vel_kind(i, j), NULL, 1.0, w, s.sig[voigt(i, j)]);
#pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < N; ++p) s.phi[i][j][p] *= prof(m, m->pb, j, h, p);
        }
}

/* --------------------------------------------- injection and measurement */

/* v'_0 = tau' p0 : sigma_kk = -p0/3, everything else zero (Sec. 3, eq. initialp0). */
static void inject(const eo_model *m, const double *p0, double *v) {
    memset(v, 0, sizeof(double) * state_len(m));
    eo_view s = view(m, v);
    for (int64_t p = 0; p < m->N; ++p)
        for (int k = 0; k < 3; ++k) s.sig[k][p] = -p0[p] / 3.0;
}

/* p_adj = tau'^T v : -(sigma11 + sigma22 + sigma33)/3 */
static void extract(const eo_model *m, double *v, double *p) {
    eo_view s = view(m, v);
    for (int64_t q = 0; q < m->N; ++q) p[q] = -(s.sig[0][q] + s.sig[1][q] + s.sig[2][q]) / 3.0;
}

/* p_l = Theta' v = -sum_c w_lc (sigma11 + sigma22 + sigma33)[c]  (Sec. 3, eq. interpgrid) */
static void measure(const eo_model *m, double *v, double *out) {
    eo_view s = view(m, v);
    for (int l = 0; l < m->nrec; ++l) {
        double acc = 0.0;
        for (int c = 0; c < 8; ++c) {
            int64_t q = m->rbase[8 * l + c];
            acc += m->rw[8 * l + c] * (s.sig[0][q] + s.sig[1][q] + s.sig[2][q]);
        }
        out[l] = -acc;
    }
}

/* v += Theta'^T y */
static void measure_tr(const eo_model *m, const double *y, double *v) {
    eo_view s = view(m, v);
    for (int l = 0; l < m->nrec; ++l)
        for (int c = 0; c < 8; ++c) {
            int64_t q = m->rbase[8 * l + c];
            double t = -m->rw[8 * l + c] * y[l];
            for (int k = 0; k < 3; ++k) s.sig[k][q] += t;
        }
}

/* ---------------------------------------------------------- model build */

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static void pml_profile(const eo_model *m, int axis, double d0, double f0) {
    const int n = m->n[axis];
    const int P = m->g.npml;
    const double dt = m->g.dt;
    const double npow = m->g.pml_npower;
    for (int half = 0; half < 2; ++half)
        for (int i = 0; i < n; ++i) {
            double x = i + 0.5 * half;
            double a = 0.0, b = 1.0, chi = 0.0;
            if (P > 0) {
                double depth = 0.0;
                if (x < P) depth = P - x;
                if (x > (n - 1 - P)) depth = x - (n - 1 - P);
                double xi = depth / P;
                if (xi > 1.0) xi = 1.0;
                if (xi > 0.0) {
                    double d = d0 * pow(xi, npow);
                    double beta = M_PI * f0 * (1.0 - xi);
                    b = exp(-(d + beta) * dt);
                    a = d / (d + beta) * (b - 1.0);
                    chi = 1.0;
                } else {
                    b = exp(-(M_PI * f0) * dt);
                }
            }
            m->pa[axis][half][i] = a;
            m->pb[axis][half][i] = b;
            m->pchi[axis][half][i] = chi;
        }
}

void eo_model_free(eo_model *m);

/* Build the oracle model.  Returns NULL on invalid input. */
eo_model *eo_model_create(const eo_grid *g, const float *lam, const float *mu, const float *rho,
                          const float *alpha, const double *rec, int32_t nrec) {
    if (g->nx < 4 || g->ny < 4 || g->nz < 4 || g->dx <= 0 || g->dt <= 0 || g->nsteps < 1 || g->npml < 0)
        return NULL;
    eo_model *m = (eo_model *)calloc(1, sizeof(eo_model));
    m->g = *g;
    if (m->g.pml_R <= 0) m->g.pml_R = 1e-3;
    if (m->g.pml_npower <= 0) m->g.pml_npower = 2.0;
    if (m->g.pml_f0 <= 0) m->g.pml_f0 = 1500.0 / (8.0 * g->dx);
    m->n[0] = g->nx; m->n[1] = g->ny; m->n[2] = g->nz;
    m->stride[0] = 1; m->stride[1] = g->nx; m->stride[2] = (int64_t)g->nx * g->ny;
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    m->N = N;
    for (int i = 0; i < 3; ++i) {
        m->rho_u[i] = (double *)malloc(sizeof(double) * N);
        m->alpha_u[i] = (double *)malloc(sizeof(double) * N);
        m->mu_s[i] = (double *)malloc(sizeof(double) * N);
    }
    for (int a = 0; a < 3; ++a) m->coord[a] = (int32_t *)malloc(sizeof(int32_t) * N);
    for (int64_t p = 0; p < N; ++p) {
        m->coord[0][p] = (int32_t)(p % g->nx);
        m->coord[1][p] = (int32_t)((p / g->nx) % g->ny);
        m->coord[2][p] = (int32_t)(p / ((int64_t)g->nx * g->ny));
    }
    m->lam = (double *)malloc(sizeof(double) * N);
    m->mu = (double *)malloc(sizeof(double) * N);
    double cmax = 0.0;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                int c[3] = {i, j, k};
                int64_t p = i + (int64_t)g->nx * (j + (int64_t)g->ny * k);
                m->lam[p] = lam[p];
                m->mu[p] = mu[p];
                double cp = sqrt(((double)lam[p] + 2.0 * (double)mu[p]) / (double)rho[p]);
                if (cp > cmax) cmax = cp;
                for (int a = 0; a < 3; ++a) {
                    int cc[3] = {c[0], c[1], c[2]};
                    cc[a] = clampi(c[a] + 1, 0, m->n[a] - 1);
                    int64_t q = cc[0] + (int64_t)g->nx * (cc[1] + (int64_t)g->ny * cc[2]);
                    m->rho_u[a][p] = 0.5 * ((double)rho[p] + (double)rho[q]);
                    m->alpha_u[a][p] = 0.5 * ((double)alpha[p] + (double)alpha[q]);
                }
                /* shear points: id 0 = (y,z) sigma23, 1 = (x,z) sigma13, 2 = (x,y) sigma12 */
                static const int ax[3][2] = {{1, 2}, {0, 2}, {0, 1}};
                for (int sidx = 0; sidx < 3; ++sidx) {
                    int a0 = ax[sidx][0], a1 = ax[sidx][1];
                    double inv = 0.0;
                    int zero = 0;
                    for (int da = 0; da < 2; ++da)
                        for (int db = 0; db < 2; ++db) {
                            int cc[3] = {c[0], c[1], c[2]};
                            cc[a0] = clampi(c[a0] + da, 0, m->n[a0] - 1);
                            cc[a1] = clampi(c[a1] + db, 0, m->n[a1] - 1);
                            double v = mu[cc[0] + (int64_t)g->nx * (cc[1] + (int64_t)g->ny * cc[2])];
                            if (v == 0.0) zero = 1; else inv += 1.0 / v;
                        }
                    m->mu_s[sidx][p] = zero ? 0.0 : 4.0 / inv;
                }
            }
    m->cmax = cmax;
    double d0 = 0.0;
    if (g->npml > 0) d0 = -(m->g.pml_npower + 1.0) * cmax * log(m->g.pml_R) / (2.0 * g->npml * g->dx);
    for (int a = 0; a < 3; ++a) {
        for (int h = 0; h < 2; ++h) {
            m->pa[a][h] = (double *)malloc(sizeof(double) * m->n[a]);
            m->pb[a][h] = (double *)malloc(sizeof(double) * m->n[a]);
            m->pchi[a][h] = (double *)malloc(sizeof(double) * m->n[a]);
        }
        pml_profile(m, a, d0, m->g.pml_f0);
    }
    m->nrec = nrec;
    m->rbase = (int64_t *)malloc(sizeof(int64_t) * 8 * (nrec > 0 ? nrec : 1));
    m->rw = (double *)malloc(sizeof(double) * 8 * (nrec > 0 ? nrec : 1));
    for (int l = 0; l < nrec; ++l) {
        int b[3];
        double f[3];
        for (int a = 0; a < 3; ++a) {
            double x = rec[3 * l + a] / g->dx;
            /* inside [0, n-1] up to 1e-9 cells of rounding, then clamped onto the box */
            if (!(x >= -1e-9 && x <= (double)(m->n[a] - 1) + 1e-9)) { eo_model_free(m); return NULL; }
            if (x < 0.0) x = 0.0;
            if (x > (double)(m->n[a] - 1)) x = (double)(m->n[a] - 1);
            int bb = (int)floor(x);
            if (bb > m->n[a] - 2) bb = m->n[a] - 2;
            b[a] = bb;
            f[a] = x - bb;
        }
        for (int c = 0; c < 8; ++c) {
            int dx_ = c & 1, dy_ = (c >> 1) & 1, dz_ = (c >> 2) & 1;
            m->rbase[8 * l + c] = (b[0] + dx_) + (int64_t)g->nx * ((b[1] + dy_) + (int64_t)g->ny * (b[2] + dz_));
            m->rw[8 * l + c] = (dx_ ? f[0] : 1 - f[0]) * (dy_ ? f[1] : 1 - f[1]) * (dz_ ? f[2] : 1 - f[2]);
        }
    }
    return m;
}

void eo_model_free(eo_model *m) {
    if (!m) return;
    for (int i = 0; i < 3; ++i) { free(m->rho_u[i]); free(m->alpha_u[i]); free(m->mu_s[i]); free(m->beta_u[i]); }
    free(m->lam); free(m->mu);
    for (int a = 0; a < 3; ++a)
        for (int h = 0; h < 2; ++h) { free(m->pa[a][h]); free(m->pb[a][h]); free(m->pchi[a][h]); }
    free(m->rbase); free(m->rw);
    for (int a = 0; a < 3; ++a) free(m->coord[a]);
    free(m);
}

/* ------------------------------------------------------------ public API */

int64_t eo_ncells(const eo_model *m) { return m->N; }
double eo_cmax(const eo_model *m) { return m->cmax; }

/* Copy staggered coefficients: rho_u[3N], alpha_u[3N], lam[N], mu[N], mu_s[3N] (23,13,12). */
void eo_coefficients(const eo_model *m, double *rho_u, double *alpha_u, double *lam, double *mu, double *mu_s) {
    const int64_t N = m->N;
    for (int i = 0; i < 3; ++i) {
        memcpy(rho_u + i * N, m->rho_u[i], sizeof(double) * N);
        memcpy(alpha_u + i * N, m->alpha_u[i], sizeof(double) * N);
        memcpy(mu_s + i * N, m->mu_s[i], sizeof(double) * N);
    }
    memcpy(lam, m->lam, sizeof(double) * N);
    memcpy(mu, m->mu, sizeof(double) * N);
}

/* 1-D PML tables of one axis: a, b, chi at integer (half=0) or half (half=1) positions. */
void eo_pml_table(const eo_model *m, int axis, int half, double *a, double *b, double *chi) {
    memcpy(a, m->pa[axis][half], sizeof(double) * m->n[axis]);
    memcpy(b, m->pb[axis][half], sizeof(double) * m->n[axis]);
    memcpy(chi, m->pchi[axis][half], sizeof(double) * m->n[axis]);
}

/* Receiver tables: base[L][8] cell indices and w[L][8] weights. */
void eo_receivers(const eo_model *m, int64_t *base, double *w) {
    memcpy(base, m->rbase, sizeof(int64_t) * 8 * m->nrec);
    memcpy(w, m->rw, sizeof(double) * 8 * m->nrec);
}

/* Frequency-dependent absorption: nmech (1..4) relaxation mechanisms with angular frequencies
   omega_l > 0 and weights w_l >= 0, and the cell map alpha_r >= 0 (1/s) of their strength; at a
   u^i point beta_u is the mean of the two adjacent cells (as alpha, the upper neighbour
   replicated at the last index) and beta_l = w_l beta_u.  nmech = 0 removes them.  The state
   grows to (27 + 3 nmech) N (eo_state_len).  Returns 0, or -1 for invalid arguments. */
int eo_set_relaxation(eo_model *m, int32_t nmech, const double *omega, const double *weight, const float *alpha_r) {
    if (nmech < 0 || nmech > 4) return -1;
    for (int i = 0; i < 3; ++i) { free(m->beta_u[i]); m->beta_u[i] = NULL; }
    m->nmech = 0;
    if (nmech == 0) return 0;
    for (int l = 0; l < nmech; ++l)
        if (!(omega[l] > 0.0) || !(weight[l] >= 0.0) || !isfinite(omega[l]) || !isfinite(weight[l])) return -1;
    const int64_t N = m->N;
    for (int64_t p = 0; p < N; ++p)
        if (!(alpha_r[p] >= 0.0f) || !isfinite(alpha_r[p])) return -1;
    for (int i = 0; i < 3; ++i) m->beta_u[i] = (double *)malloc(sizeof(double) * N);
    for (int k = 0; k < m->n[2]; ++k)
        for (int j = 0; j < m->n[1]; ++j)
            for (int i = 0; i < m->n[0]; ++i) {
                const int c[3] = {i, j, k};
                const int64_t p = i + (int64_t)m->n[0] * (j + (int64_t)m->n[1] * k);
                for (int a = 0; a < 3; ++a) {
                    int cc[3] = {c[0], c[1], c[2]};
                    cc[a] = clampi(c[a] + 1, 0, m->n[a] - 1);
                    const int64_t q = cc[0] + (int64_t)m->n[0] * (cc[1] + (int64_t)m->n[1] * cc[2]);
                    m->beta_u[a][p] = 0.5 * ((double)alpha_r[p] + (double)alpha_r[q]);
                }
            }
    for (int l = 0; l < nmech; ++l) {
        m->mech_w[l] = weight[l];
        m->mech_c[l] = exp(-omega[l] * m->g.dt);
    }
    m->nmech = nmech;
    return 0;
}

int64_t eo_state_len(const eo_model *m) { return state_len(m); }

/* In-place v <- W' v or v <- W'^T v on a state of eo_state_len() doubles. */
void eo_step(const eo_model *m, double *v, int transpose) {
    double *tmp = (double *)malloc(sizeof(double) * 4 * m->N);
    if (transpose) step_tr(m, v, tmp); else step_fwd(m, v, tmp);
    free(tmp);
}

void eo_inject(const eo_model *m, const double *p0, double *v) { inject(m, p0, v); }
void eo_extract(const eo_model *m, double *v, double *p) { extract(m, v, p); }
void eo_measure(const eo_model *m, double *v, double *out) { measure(m, v, out); }
void eo_measure_tr(const eo_model *m, const double *y, double *v) { measure_tr(m, y, v); }

/* traces[M][L] = H p0  (eq. STforHPML), nsteps_override > 0 replaces M. */
int eo_forward(const eo_model *m, const double *p0, double *traces, int32_t nsteps_override) {
    const int M = nsteps_override > 0 ? nsteps_override : m->g.nsteps;
    double *v = (double *)malloc(sizeof(double) * state_len(m));
    double *tmp = (double *)malloc(sizeof(double) * 4 * m->N);
    if (!v || !tmp) { free(v); free(tmp); return -4; }
    inject(m, p0, v);
    measure(m, v, traces);
    for (int t = 1; t < M; ++t) {
        step_fwd(m, v, tmp);
        measure(m, v, traces + (int64_t)t * m->nrec);
    }
    free(v); free(tmp);
    return 0;
}

/* p_adj = H^T y  via  v_{M-1} = Theta^T y_{M-1};  v_{m-1} = Theta^T y_{m-1} + W'^T v_m;
   p_adj = tau'^T v_0   (Sec. 4, eq. Adjup; Appendix eq. AdjupPML with the index read as m-1). */
int eo_adjoint(const eo_model *m, const double *y, double *p_adj, int32_t nsteps_override) {
    const int M = nsteps_override > 0 ? nsteps_override : m->g.nsteps;
    double *v = (double *)calloc((size_t)state_len(m), sizeof(double));
    double *tmp = (double *)malloc(sizeof(double) * 4 * m->N);
    if (!v || !tmp) { free(v); free(tmp); return -4; }
    measure_tr(m, y + (int64_t)(M - 1) * m->nrec, v);
    for (int t = M - 1; t >= 1; --t) {
        step_tr(m, v, tmp);
        measure_tr(m, y + (int64_t)(t - 1) * m->nrec, v);
    }
    extract(m, v, p_adj);
    free(v); free(tmp);
    return 0;
}

/* Run the forward recursion for `steps` updates from v (eo_state_len() doubles, in/out). */
void eo_run(const eo_model *m, double *v, int32_t steps) {
    double *tmp = (double *)malloc(sizeof(double) * 4 * m->N);
    for (int t = 0; t < steps; ++t) step_fwd(m, v, tmp);
    free(tmp);
}

int eo_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
