/*
 * couple_oracle.c -- plain, slow, FP64 CPU oracle of the dual-grid coupling exchange.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no source, header, table or helper with the GPU path.
 *
 * Every function writes out the plain definition of one stage of the per-step
 * exchange between Lagrangian particles, the coarse ("bulk") grid and the fine
 * grid of the dual-grid multiscale CFD-DEM coupling (Sec. 2.1, Fig. 1):
 *
 *   bin          particle -> containing bulk cell, canonical (cell, id) order;
 *                the connectivity that must be rebuilt every coupling step (Sec. 2.2)
 *   deposit      volume-averaged solid fraction and momentum source on the bulk
 *                grid (Sec. 1 unresolved coupling; porosity in Table 1 and Sec. 2.4;
 *                momentum source F_fpi of Eq. UFP, Sec. 2.5)
 *   restrict     fine -> bulk "fluid solution" transfer (Fig. 1, Sec. 2.1, 2.3)
 *   interp       fluid value at a particle ("cell values or locally interpolated
 *                values", Sec. 1)
 *   drag         F = beta (u_f - u_p), Eq. DragLaw (Sec. 2.4), beta by the
 *                Di Felice voidage correlation; optionally with the two-fluid
 *                (VOF) density and viscosity at the particle (Sec. 2.5)
 *   semi         deposited drag coefficient and beta-weighted particle velocity,
 *                the semi-implicit form of the momentum source (Sec. 2.5)
 *   prolong      bulk -> fine "particle related fields" transfer (Fig. 1)
 *   remap        volume-weighted transfer between two grids that need not be
 *                nested (the sender -> receiver interpolation of Sec. 2.3)
 *   advect       explicit Euler update of Eq. DEM_EQUATIONS with drag only
 *
 * All arithmetic is FP64, except where a floating-point comparison decides an
 * integer (the containing-cell index): there the caller chooses the precision
 * the kernel uses (prec32 = 1 evaluates the index in IEEE binary32).
 *
 * Layout: particle vectors are [n][3] (x,y,z); grid fields are [nz][ny][nx] with x
 * fastest; vector grid fields are three such arrays back to back ([3][nz][ny][nx]).
 *
 * Threads: loops whose iterations are independent (one particle, one cell or one
 * point each, no shared sum) may run on several OpenMP threads (orc_set_threads;
 * one thread unless asked).  Every sum whose order is the canonical one (the
 * depositions in (cell, id) order, the sort) stays serial, so the results do not
 * depend on the number of threads.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* Threads of the independent-iteration loops (see the header comment). */
void orc_set_threads(int k) { omp_set_num_threads(k > 0 ? k : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }

static int64_t lin3(int64_t i, int64_t j, int64_t k, const int n[3])
{
    return i + (int64_t)n[0] * (j + (int64_t)n[1] * k);
}

static int clampi(int64_t v, int n)
{
    if (v < 0) return 0;
    if (v > n - 1) return n - 1;
    return (int)v;
}

/* Position clamped into the closed box [0, L]; a NaN coordinate becomes 0
 * (fmax returns the non-NaN operand).  Returns 1 if the input was outside. */
static int clamp_pos(const double *p, const double box[3], double out[3])
{
    int outside = 0;
    for (int a = 0; a < 3; ++a) {
        double x = p[a];
        if (!(x >= 0.0 && x <= box[a])) outside = 1;
        out[a] = fmin(fmax(x, 0.0), box[a]);
    }
    return outside;
}

/* Same clamp in binary32 arithmetic (the box length rounded to float). */
static int clamp_pos32(const double *p, const double box[3], double out[3])
{
    int outside = 0;
    for (int a = 0; a < 3; ++a) {
        float x = (float)p[a];
        float L = (float)box[a];
        if (!(x >= 0.0f && x <= L)) outside = 1;
        out[a] = (double)fminf(fmaxf(x, 0.0f), L);
    }
    return outside;
}

/* ------------------------------------------------------------------------- */
/* Bin: containing bulk cell of each particle (connectivity, Sec. 2.2).        */
/* i_a = floor(x_a * n_a / L_a), clamped to [0, n_a-1]; x = L falls in n-1.   */
/* Linear key k = i_x + n_x (i_y + n_y i_z).  Returns the number of particles  */
/* whose position was outside the box (or not finite).                        */
/* ------------------------------------------------------------------------- */
int64_t orc_bin(int64_t n, const double *pos, const double box[3], const int nb[3],
                int prec32, int32_t *cell)
{
    int64_t outside = 0;
#pragma omp parallel for schedule(static) reduction(+ : outside)
    for (int64_t p = 0; p < n; ++p) {
        double x[3];
        int idx[3];
        if (prec32) {
            outside += clamp_pos32(pos + 3 * p, box, x);
            for (int a = 0; a < 3; ++a) {
                float s = (float)((double)nb[a] / box[a]);
                float c = (float)x[a] * s;
                idx[a] = clampi((int64_t)floorf(c), nb[a]);
            }
        } else {
            outside += clamp_pos(pos + 3 * p, box, x);
            for (int a = 0; a < 3; ++a) {
                double s = (double)nb[a] / box[a];
                idx[a] = clampi((int64_t)floor(x[a] * s), nb[a]);
            }
        }
        cell[p] = (int32_t)lin3(idx[0], idx[1], idx[2], nb);
    }
    return outside;
}

/* Stable order of particle ids by cell (ties by ascending id), per-cell counts
 * and the exclusive prefix sum of the counts ("start", length ncell+1).
 * Written as a counting sort: count, scan, then place ids in ascending order. */
void orc_sort(int64_t n, const int32_t *cell, int64_t ncell,
              int32_t *perm, int32_t *count, int32_t *start)
{
    memset(count, 0, sizeof(int32_t) * (size_t)ncell);
    for (int64_t p = 0; p < n; ++p) count[cell[p]] += 1;
    start[0] = 0;
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] = start[c] + count[c];
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncell > 0 ? ncell : 1));
    for (int64_t c = 0; c < ncell; ++c) next[c] = start[c];
    for (int64_t p = 0; p < n; ++p) perm[next[cell[p]]++] = (int32_t)p;
    free(next);
}

/* ------------------------------------------------------------------------- */
/* Particle -> bulk-cell weights.                                             */
/*   NGP: weight 1 on the containing cell.                                    */
/*   CIC: trilinear weights to the 8 bulk cell centres around the particle;   */
/*        g = x n / L - 1/2, j = floor(g), t = g - j; corner delta in {0,1}^3 */
/*        has weight prod_a (delta_a ? t_a : 1 - t_a) on cell clamp(j+delta). */
/*        Corners folded onto the same cell by the clamp have their weights   */
/*        added, so the weights always sum to one.                            */
/* Returns the number of distinct cells written to cells[]/w[].               */
/* ------------------------------------------------------------------------- */
static int weights(const double x[3], const double box[3], const int nb[3], int cic,
                   int prec32, int64_t cells[8], double w[8])
{
    if (!cic) {
        int idx[3];
        for (int a = 0; a < 3; ++a) {
            if (prec32) {
                float s = (float)((double)nb[a] / box[a]);
                idx[a] = clampi((int64_t)floorf((float)x[a] * s), nb[a]);
            } else {
                idx[a] = clampi((int64_t)floor(x[a] * ((double)nb[a] / box[a])), nb[a]);
            }
        }
        cells[0] = lin3(idx[0], idx[1], idx[2], nb);
        w[0] = 1.0;
        return 1;
    }
    int64_t j[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        double g = x[a] * ((double)nb[a] / box[a]) - 0.5;
        j[a] = (int64_t)floor(g);
        t[a] = g - (double)j[a];
    }
    int m = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                int d[3] = {dx, dy, dz};
                double wt = 1.0;
                int idx[3];
                for (int a = 0; a < 3; ++a) {
                    wt *= d[a] ? t[a] : 1.0 - t[a];
                    idx[a] = clampi(j[a] + d[a], nb[a]);
                }
                int64_t c = lin3(idx[0], idx[1], idx[2], nb);
                int found = -1;
                for (int q = 0; q < m; ++q)
                    if (cells[q] == c) found = q;
                if (found >= 0) {
                    w[found] += wt;
                } else {
                    cells[m] = c;
                    w[m] = wt;
                    ++m;
                }
            }
    return m;
}

/* Exported for tests: the (cell, weight) list of one particle. */
int orc_weights(const double *pos, const double box[3], const int nb[3], int cic,
                int prec32, int64_t *cells, double *w)
{
    double x[3];
    if (prec32) clamp_pos32(pos, box, x); else clamp_pos(pos, box, x);
    return weights(x, box, nb, cic, prec32, cells, w);
}

static double particle_volume(double d) { return ORC_PI * d * d * d / 6.0; }

/* ------------------------------------------------------------------------- */
/* Solid volume fraction of each bulk cell (porosity eps = 1 - phi):          */
/*   phi_c = sum_p w_pc V_p / V_b,  V_p = pi d^3 / 6, V_b = hx hy hz,          */
/* accumulated particle by particle in the canonical (cell, id) order.       */
/* ------------------------------------------------------------------------- */
void orc_deposit_volume(int64_t n, const double *pos, const double *diam, const int32_t *perm,
                        const double box[3], const int nb[3], int cic, int prec32, double *phi)
{
    int64_t nc = (int64_t)nb[0] * nb[1] * nb[2];
    double vb = (box[0] / nb[0]) * (box[1] / nb[1]) * (box[2] / nb[2]);
    for (int64_t c = 0; c < nc; ++c) phi[c] = 0.0;
    for (int64_t q = 0; q < n; ++q) {
        int64_t p = perm[q];
        double x[3];
        if (prec32) clamp_pos32(pos + 3 * p, box, x); else clamp_pos(pos + 3 * p, box, x);
        int64_t cells[8];
        double w[8];
        int m = weights(x, box, nb, cic, prec32, cells, w);
        double vp = particle_volume(diam[p]);
        for (int k = 0; k < m; ++k) phi[cells[k]] += w[k] * vp / vb;
    }
}

/* Momentum source on the bulk grid, equal and opposite to the particle drag:
 *   F_fpi,c = -(1/V_b) sum_p w_pc F_p   (three components, [3][ncell]). */
void orc_deposit_force(int64_t n, const double *pos, const double *force, const int32_t *perm,
                       const double box[3], const int nb[3], int cic, int prec32, double *fc)
{
    int64_t nc = (int64_t)nb[0] * nb[1] * nb[2];
    double vb = (box[0] / nb[0]) * (box[1] / nb[1]) * (box[2] / nb[2]);
    for (int64_t c = 0; c < 3 * nc; ++c) fc[c] = 0.0;
    for (int64_t q = 0; q < n; ++q) {
        int64_t p = perm[q];
        double x[3];
        if (prec32) clamp_pos32(pos + 3 * p, box, x); else clamp_pos(pos + 3 * p, box, x);
        int64_t cells[8];
        double w[8];
        int m = weights(x, box, nb, cic, prec32, cells, w);
        for (int k = 0; k < m; ++k)
            for (int a = 0; a < 3; ++a) fc[a * nc + cells[k]] -= w[k] * force[3 * p + a] / vb;
    }
}

/* Semi-implicit split of the momentum source (the drag counterpart of Eq. UFP
 * is treated semi-implicitly in the fluid solve, Sec. 2.5).  With
 * F_p = beta_p (u_f - u_p) the source is -K_c u_f + KU_c wherever the fluid
 * velocity is uniform over the deposition stencil, where
 *   K_c  = (1/V_b) sum_p w_pc beta_p          (implicit coefficient, [ncell])
 *   KU_c = (1/V_b) sum_p w_pc beta_p u_p      (explicit part, [3][ncell]).
 * Same weights and canonical (cell, id) order as the other depositions. */
void orc_deposit_semi(int64_t n, const double *pos, const double *beta, const double *vel, const int32_t *perm,
                      const double box[3], const int nb[3], int cic, int prec32, double *K, double *KU)
{
    int64_t nc = (int64_t)nb[0] * nb[1] * nb[2];
    double vb = (box[0] / nb[0]) * (box[1] / nb[1]) * (box[2] / nb[2]);
    for (int64_t c = 0; c < nc; ++c) K[c] = 0.0;
    for (int64_t c = 0; c < 3 * nc; ++c) KU[c] = 0.0;
    for (int64_t q = 0; q < n; ++q) {
        int64_t p = perm[q];
        double x[3];
        if (prec32) clamp_pos32(pos + 3 * p, box, x); else clamp_pos(pos + 3 * p, box, x);
        int64_t cells[8];
        double w[8];
        int m = weights(x, box, nb, cic, prec32, cells, w);
        for (int k = 0; k < m; ++k) {
            K[cells[k]] += w[k] * beta[p] / vb;
            for (int a = 0; a < 3; ++a) KU[a * nc + cells[k]] += w[k] * beta[p] * vel[3 * p + a] / vb;
        }
    }
}

/* Void fraction seen by each particle: eps_p = sum_c w_pc (1 - phi_c), with the
 * same weights as the deposition (the transpose of the deposition operator). */
void orc_gather_eps(int64_t n, const double *pos, const double *phi, const double box[3],
                    const int nb[3], int cic, int prec32, double *eps_p)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        double x[3];
        if (prec32) clamp_pos32(pos + 3 * p, box, x); else clamp_pos(pos + 3 * p, box, x);
        int64_t cells[8];
        double w[8];
        int m = weights(x, box, nb, cic, prec32, cells, w);
        double e = 0.0;
        for (int k = 0; k < m; ++k) e += w[k] * (1.0 - phi[cells[k]]);
        eps_p[p] = e;
    }
}

/* ------------------------------------------------------------------------- */
/* Restriction fine -> bulk: average of the r^3 fine children of each bulk    */
/* cell (conservative volume average), children visited in raster order.     */
/* ------------------------------------------------------------------------- */
void orc_restrict(const double *qf, const int nb[3], int r, double *qb)
{
    int nf[3] = {nb[0] * r, nb[1] * r, nb[2] * r};
    double inv = 1.0 / ((double)r * r * r);
#pragma omp parallel for schedule(static) collapse(2)
    for (int k = 0; k < nb[2]; ++k)
        for (int j = 0; j < nb[1]; ++j)
            for (int i = 0; i < nb[0]; ++i) {
                double s = 0.0;
                for (int c = 0; c < r; ++c)
                    for (int b = 0; b < r; ++b)
                        for (int a = 0; a < r; ++a)
                            s += qf[lin3(i * r + a, j * r + b, k * r + c, nf)];
                qb[lin3(i, j, k, nb)] = s * inv;
            }
}

/* Pressure gradient on the bulk grid: central differences
 * (P[c+e] - P[c-e]) / (2h), one-sided (P[c+e]-P[c])/h or (P[c]-P[c-e])/h at the
 * two walls, zero along an axis with a single cell. Output [3][ncell]. */
void orc_gradient(const double *P, const int nb[3], const double box[3], double *G)
{
    int64_t nc = (int64_t)nb[0] * nb[1] * nb[2];
#pragma omp parallel for schedule(static) collapse(2)
    for (int k = 0; k < nb[2]; ++k)
        for (int j = 0; j < nb[1]; ++j)
            for (int i = 0; i < nb[0]; ++i) {
                int idx[3] = {i, j, k};
                int64_t c = lin3(i, j, k, nb);
                for (int a = 0; a < 3; ++a) {
                    double h = box[a] / nb[a];
                    int lo[3] = {i, j, k}, hi[3] = {i, j, k};
                    double g;
                    if (nb[a] == 1) {
                        g = 0.0;
                    } else if (idx[a] == 0) {
                        hi[a] = 1;
                        g = (P[lin3(hi[0], hi[1], hi[2], nb)] - P[c]) / h;
                    } else if (idx[a] == nb[a] - 1) {
                        lo[a] = nb[a] - 2;
                        g = (P[c] - P[lin3(lo[0], lo[1], lo[2], nb)]) / h;
                    } else {
                        lo[a] = idx[a] - 1;
                        hi[a] = idx[a] + 1;
                        g = (P[lin3(hi[0], hi[1], hi[2], nb)] - P[lin3(lo[0], lo[1], lo[2], nb)]) / (2.0 * h);
                    }
                    G[a * nc + c] = g;
                }
            }
}

/* ------------------------------------------------------------------------- */
/* Trilinear interpolation of a cell-centred field q ([n2][n1][n0] over the   */
/* box) at points; node indices outside the grid are clamped (zero gradient   */
/* at the walls).  Used for the fine-grid lookup and for the bulk-grid lookup. */
/* ------------------------------------------------------------------------- */
static double trilinear(const double *q, const int n[3], const double box[3], const double x[3])
{
    int64_t j[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        double g = x[a] * ((double)n[a] / box[a]) - 0.5;
        j[a] = (int64_t)floor(g);
        t[a] = g - (double)j[a];
    }
    double s = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                int d[3] = {dx, dy, dz};
                double wt = 1.0;
                int idx[3];
                for (int a = 0; a < 3; ++a) {
                    wt *= d[a] ? t[a] : 1.0 - t[a];
                    idx[a] = clampi(j[a] + d[a], n[a]);
                }
                s += wt * q[lin3(idx[0], idx[1], idx[2], n)];
            }
    return s;
}

void orc_interp(const double *q, const int n[3], const double box[3], int64_t npts,
                const double *pos, int prec32, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npts; ++p) {
        double x[3];
        if (prec32) clamp_pos32(pos + 3 * p, box, x); else clamp_pos(pos + 3 * p, box, x);
        out[p] = trilinear(q, n, box, x);
    }
}

/* ------------------------------------------------------------------------- */
/* Drag, Eq. DragLaw: F = beta (u_f - u_p).  beta after Di Felice:            */
/*   u_r = u_f - u_p, eps* = max(eps_p, eps_min),                             */
/*   Re = rho_f eps* d |u_r| / mu_f,  C_D = (0.63 + 4.8 / sqrt(Re))^2,         */
/*   chi = 3.7 - 0.65 exp(-(1.5 - log10 Re)^2 / 2),                           */
/*   beta = 1/2 C_D rho_f (pi d^2 / 4) eps*^(2 - chi) |u_r|.                  */
/* At |u_r| = 0 the force is zero and beta takes its limit                    */
/*   beta_0 = 1/2 rho_f (pi d^2/4) eps*^(2-3.7) * 4.8^2 mu_f / (rho_f eps* d). */
/* Returns the number of particles whose void fraction was raised to eps_min.  */
/* ------------------------------------------------------------------------- */
/* beta of one particle (Di Felice, as above) for relative speed |u_r| = mag,
 * void fraction e (already raised to eps_min), diameter d and the fluid's
 * density and viscosity at the particle. */
static double drag_beta(double mag, double e, double d, double rho_f, double mu_f)
{
    double area = ORC_PI * d * d / 4.0;
    if (mag > 0.0) {
        double re = rho_f * e * d * mag / mu_f;
        double cd = 0.63 + 4.8 / sqrt(re);
        cd = cd * cd;
        double l = 1.5 - log10(re);
        double chi = 3.7 - 0.65 * exp(-l * l / 2.0);
        return 0.5 * cd * rho_f * area * pow(e, 2.0 - chi) * mag;
    }
    return 0.5 * rho_f * area * pow(e, 2.0 - 3.7) * 4.8 * 4.8 * mu_f / (rho_f * e * d);
}

/* Drag of particles p in [0, n) with the fluid density and viscosity rho_f[p],
 * mu_f[p] at each particle; returns the number of clamped void fractions. */
static int64_t drag_var(int64_t n, const double *uf, const double *up, const double *diam,
                        const double *eps_p, const double *rho_f, const double *mu_f, double eps_min,
                        double *force, double *beta)
{
    int64_t clamped = 0;
#pragma omp parallel for schedule(static) reduction(+ : clamped)
    for (int64_t p = 0; p < n; ++p) {
        double ur[3], mag2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            ur[a] = uf[3 * p + a] - up[3 * p + a];
            mag2 += ur[a] * ur[a];
        }
        double e = eps_p[p];
        if (e < eps_min) { e = eps_min; ++clamped; }
        double b = drag_beta(sqrt(mag2), e, diam[p], rho_f[p], mu_f[p]);
        if (beta) beta[p] = b;
        for (int a = 0; a < 3; ++a) force[3 * p + a] = b * ur[a];
    }
    return clamped;
}

int64_t orc_drag(int64_t n, const double *uf, const double *up, const double *diam,
                 const double *eps_p, double rho_f, double mu_f, double eps_min,
                 double *force, double *beta)
{
    double *rv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *mv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t p = 0; p < n; ++p) { rv[p] = rho_f; mv[p] = mu_f; }
    int64_t c = drag_var(n, uf, up, diam, eps_p, rv, mv, eps_min, force, beta);
    free(rv);
    free(mv);
    return c;
}

/* Two-fluid (VOF) drag: the fluid density and viscosity at the particle follow
 * the liquid volume fraction alpha_p there (the local-property mixture of the
 * VOF fluid, Sec. 2.5):
 *   rho_f = rho_1 alpha + rho_2 (1 - alpha),   mu_f = mu_1 alpha + mu_2 (1 - alpha). */
int64_t orc_drag_vof(int64_t n, const double *uf, const double *up, const double *diam,
                     const double *eps_p, const double *alpha_p, double rho1, double mu1, double rho2,
                     double mu2, double eps_min, double *force, double *beta)
{
    double *rv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *mv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t p = 0; p < n; ++p) {
        rv[p] = rho1 * alpha_p[p] + rho2 * (1.0 - alpha_p[p]);
        mv[p] = mu1 * alpha_p[p] + mu2 * (1.0 - alpha_p[p]);
    }
    int64_t c = drag_var(n, uf, up, diam, eps_p, rv, mv, eps_min, force, beta);
    free(rv);
    free(mv);
    return c;
}

/* ------------------------------------------------------------------------- */
/* Prolongation bulk -> fine (conservative trilinear).                        */
/*   T_f = trilinear interpolation of the bulk field B at the fine centre x_f  */
/*         (bulk cell-centred nodes, clamped);                                 */
/*   D_c = B_c - (1/r^3) sum_{f in c} T_f  (defect of the parent cell c);       */
/*   P(B)_f = T_f + D_c.                                                        */
/* Restricting P(B) gives back B exactly, and sum_f P(B)_f V_f = sum_c B_c V_b. */
/* ------------------------------------------------------------------------- */
static double fine_trilinear(const double *B, const int nb[3], int r, int64_t fi, int64_t fj, int64_t fk)
{
    /* fine centre in bulk-index coordinates: g = (f + 1/2)/r - 1/2 */
    int64_t f[3] = {fi, fj, fk};
    double box1[3] = {(double)nb[0], (double)nb[1], (double)nb[2]};
    double x[3];
    for (int a = 0; a < 3; ++a) x[a] = ((double)f[a] + 0.5) / (double)r;
    return trilinear(B, nb, box1, x);
}

static double defect(const double *B, const int nb[3], int r, int i, int j, int k)
{
    double s = 0.0;
    for (int c = 0; c < r; ++c)
        for (int b = 0; b < r; ++b)
            for (int a = 0; a < r; ++a)
                s += fine_trilinear(B, nb, r, (int64_t)i * r + a, (int64_t)j * r + b, (int64_t)k * r + c);
    return B[lin3(i, j, k, nb)] - s / ((double)r * r * r);
}

void orc_prolong(const double *B, const int nb[3], int r, int conservative, double *out)
{
    int nf[3] = {nb[0] * r, nb[1] * r, nb[2] * r};
#pragma omp parallel for schedule(static) collapse(2)
    for (int k = 0; k < nb[2]; ++k)
        for (int j = 0; j < nb[1]; ++j)
            for (int i = 0; i < nb[0]; ++i) {
                double dc = conservative ? defect(B, nb, r, i, j, k) : 0.0;
                for (int c = 0; c < r; ++c)
                    for (int b = 0; b < r; ++b)
                        for (int a = 0; a < r; ++a) {
                            int64_t fi = (int64_t)i * r + a, fj = (int64_t)j * r + b, fk = (int64_t)k * r + c;
                            out[lin3(fi, fj, fk, nf)] = fine_trilinear(B, nb, r, fi, fj, fk) + dc;
                        }
            }
}

/* Prolongation at selected flat fine indices only (for sampled comparisons). */
void orc_prolong_at(const double *B, const int nb[3], int r, int conservative,
                    int64_t m, const int64_t *fidx, double *out)
{
    int nf[3] = {nb[0] * r, nb[1] * r, nb[2] * r};
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < m; ++q) {
        int64_t f = fidx[q];
        int64_t fi = f % nf[0];
        int64_t fj = (f / nf[0]) % nf[1];
        int64_t fk = f / ((int64_t)nf[0] * nf[1]);
        double dc = conservative ? defect(B, nb, r, (int)(fi / r), (int)(fj / r), (int)(fk / r)) : 0.0;
        out[q] = fine_trilinear(B, nb, r, fi, fj, fk) + dc;
    }
}

/* ------------------------------------------------------------------------- */
/* Explicit Euler step of Eq. DEM_EQUATIONS with the drag as the only force:   */
/*   x <- x + dt u,  u <- u + dt F / m,  m = rho_p pi d^3 / 6,                */
/* from the clamped old position; a coordinate that leaves [0, L] is          */
/* mirrored back (x -> -x, or x -> 2L - x) and that velocity component flips.  */
/* The new position and velocity are computed in FP64 in both modes.          */
/* Whether a wall was crossed is a discrete decision taken on floating-point  */
/* values: with prec32 it is taken in binary32, the precision of the state    */
/* the FP32 modes advance, on the candidate position x + dt u rounded once to */
/* binary32 (fmaf: the exact product and sum, one rounding; x, u, dt and L    */
/* being binary32 values there).  Without prec32 the FP64 candidate decides.  */
/* ------------------------------------------------------------------------- */
void orc_advect(int64_t n, double *pos, double *vel, const double *diam, const double *force,
                double rho_p, double dt, const double box[3], int prec32)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        double x[3];
        if (prec32) clamp_pos32(pos + 3 * p, box, x); else clamp_pos(pos + 3 * p, box, x);
        double m = rho_p * particle_volume(diam[p]);
        for (int a = 0; a < 3; ++a) {
            double u = vel[3 * p + a];
            double L = box[a];
            double xn = x[a] + dt * u;
            double un = u + dt * force[3 * p + a] / m;
            int below, above;
            if (prec32) {
                float c = fmaf((float)dt, (float)u, (float)x[a]);
                below = c < 0.0f;
                above = c > (float)L;
            } else {
                below = xn < 0.0;
                above = xn > L;
            }
            if (below) { xn = -xn; un = -un; }
            else if (above) { xn = 2.0 * L - xn; un = -un; }
            xn = fmin(fmax(xn, 0.0), L);
            pos[3 * p + a] = xn;
            vel[3 * p + a] = un;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Grid-to-grid interpolation between two grids that need not be nested      */
/* (the sender -> receiver map of Sec. 2.3, static for non-deforming grids).  */
/* Both grids are rectilinear and cell-centred over the same box; axis a of a */
/* grid has n[a] cells between nodes x_a[0] < ... < x_a[n[a]]; the nodes of  */
/* the three axes are stored one after the other.  The receiver value is the  */
/* volume-weighted average of the sender cells it overlaps:                   */
/*   dst_c = (sum_f |f intersect c| src_f) / |c|.                             */
/* ------------------------------------------------------------------------- */
static double overlap1(double a0, double a1, double b0, double b1)
{
    double lo = a0 > b0 ? a0 : b0, hi = a1 < b1 ? a1 : b1;
    return hi > lo ? hi - lo : 0.0;
}

void orc_remap(const int ns[3], const double *src_nodes, const int nd[3], const double *dst_nodes,
               const double *src, double *dst)
{
    const double *xs[3], *xd[3];
    xs[0] = src_nodes; xs[1] = xs[0] + ns[0] + 1; xs[2] = xs[1] + ns[1] + 1;
    xd[0] = dst_nodes; xd[1] = xd[0] + nd[0] + 1; xd[2] = xd[1] + nd[1] + 1;
#pragma omp parallel for schedule(static) collapse(2)
    for (int k = 0; k < nd[2]; ++k)
        for (int j = 0; j < nd[1]; ++j)
            for (int i = 0; i < nd[0]; ++i) {
                double acc = 0.0;
                for (int fk = 0; fk < ns[2]; ++fk) {
                    double oz = overlap1(xd[2][k], xd[2][k + 1], xs[2][fk], xs[2][fk + 1]);
                    if (oz == 0.0) continue;
                    for (int fj = 0; fj < ns[1]; ++fj) {
                        double oy = overlap1(xd[1][j], xd[1][j + 1], xs[1][fj], xs[1][fj + 1]);
                        if (oy == 0.0) continue;
                        for (int fi = 0; fi < ns[0]; ++fi) {
                            double ox = overlap1(xd[0][i], xd[0][i + 1], xs[0][fi], xs[0][fi + 1]);
                            if (ox == 0.0) continue;
                            acc += ox * oy * oz * src[lin3(fi, fj, fk, ns)];
                        }
                    }
                }
                double vol = (xd[0][i + 1] - xd[0][i]) * (xd[1][j + 1] - xd[1][j]) * (xd[2][k + 1] - xd[2][k]);
                dst[lin3(i, j, k, nd)] = acc / vol;
            }
}

/* ------------------------------------------------------------------------- */
/* Grid-to-grid transfer between two grids made of arbitrary axis-aligned    */
/* cells (boxes), e.g. locally refined grids that are not nested in each      */
/* other (Sec. 2.1: the fine grid may be non-uniform and locally refined;    */
/* Sec. 2.3: a static sender -> receiver map).  Cell c of a grid is the box   */
/* [b[6c], b[6c+1]] x [b[6c+2], b[6c+3]] x [b[6c+4], b[6c+5]].  The receiver */
/* value is the volume-weighted average of the sender cells it overlaps,     */
/*   dst_r = (sum_s |r intersect s| src_s) / |r|,                            */
/* computed here by brute force over every (receiver, sender) pair.          */
/* ------------------------------------------------------------------------- */
void orc_box_remap(int64_t ns, const double *sbox, int64_t nr, const double *rbox, const double *src,
                   double *dst)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nr; ++r) {
        const double *R = rbox + 6 * r;
        double acc = 0.0;
        for (int64_t c = 0; c < ns; ++c) {
            const double *S = sbox + 6 * c;
            double ox = overlap1(R[0], R[1], S[0], S[1]);
            if (ox == 0.0) continue;
            double oy = overlap1(R[2], R[3], S[2], S[3]);
            if (oy == 0.0) continue;
            double oz = overlap1(R[4], R[5], S[4], S[5]);
            if (oz == 0.0) continue;
            acc += ox * oy * oz * src[c];
        }
        double vol = (R[1] - R[0]) * (R[3] - R[2]) * (R[5] - R[4]);
        dst[r] = acc / vol;
    }
}

/* Particle volumes V_p = pi d^3 / 6 (for the conservation diagnostics). */
void orc_particle_volumes(int64_t n, const double *diam, double *vp)
{
    for (int64_t p = 0; p < n; ++p) vp[p] = particle_volume(diam[p]);
}
