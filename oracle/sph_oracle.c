/*
 * CPU oracle for the converted-view SPH step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant with the HIP library.
 *
 * Everything is scalar IEEE double, compiled with -ffp-contract=off and no
 * fast-math, so every product and sum is rounded on its own.
 *
 * What the paper fixes and what is read from the literature it cites:
 *  - The step structure (density with an iterated smoothing length, force,
 *    kick / drift / kick) is the paper's SPH blueprint (Sec. 2.1).
 *  - Pairs are (local i, active j), j != i, filtered by a radius predicate;
 *    out-of-range pairs contribute the neutral element (Sec. 2.3, Sec. 5.6).
 *  - The paper names the formulas only by citation.  Two kernels, both with
 *    support 2h: the cubic M4 spline of Monaghan & Lattanzio (kernel 0) and the
 *    quartic M5 spline the paper employs (Sec. 2.1, kernel 1); density / grad-h terms
 *    follow Springel & Hernquist 2002 and Price 2012; the artificial viscosity
 *    is the signal-velocity form of Monaghan 1997 as used by Springel 2005.
 *
 * Pins (tests/test_oracle_*.py): kernel normalisation by quadrature, finite-
 * difference derivatives, textbook spline values, the quartic against scipy's
 * degree-4 B-spline (Cox-de Boor), lattice neighbour counts and
 * lattice sums, brute force == cell list, momentum / energy conservation,
 * adiabatic du/dt == (P/rho^2) drho/dt by finite differences, the pressure
 * force == -grad of the thermal energy by finite differences.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------ kernel */

/* Cubic M4 spline shape w(q), support q < 2 (Monaghan & Lattanzio 1985). */
double orc_w(double q)
{
    if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    if (q < 2.0) { double t = 2.0 - q; return 0.25 * t * t * t; }
    return 0.0;
}

/* dw/dq of the same spline. */
double orc_dw(double q)
{
    if (q < 1.0) return -3.0 * q + 2.25 * q * q;
    if (q < 2.0) { double t = 2.0 - q; return -0.75 * t * t; }
    return 0.0;
}

/*
 * Quartic M5 spline (Monaghan 1985), the kernel the paper employs (Sec. 2.1).
 * In its own variable s, with support s < 2.5, its shape is
 *   f(s) = (2.5-s)^4 - 5 (1.5-s)^4 + 10 (0.5-s)^4   for 0   <= s < 0.5,
 *   f(s) = (2.5-s)^4 - 5 (1.5-s)^4                  for 0.5 <= s < 1.5,
 *   f(s) = (2.5-s)^4                                for 1.5 <= s < 2.5,
 * and f(r/h')/(20 pi h'^3) integrates to one in three dimensions.  Reading:
 * it is scaled to the same support 2h as the cubic (h' = 0.8 h, s = 1.25 q),
 * so cells, reach and the pair predicate do not depend on the kernel; then
 * W = w(q)/(pi h^3) with w(q) = f(1.25 q) / 10.24, since 20 * 0.8^3 = 10.24.
 */
double orc_w5(double q)
{
    double s = 1.25 * q;
    if (s >= 2.5) return 0.0;
    double a = 2.5 - s;
    double f = a * a * a * a;
    if (s < 1.5) { double b = 1.5 - s; f -= 5.0 * b * b * b * b; }
    if (s < 0.5) { double c = 0.5 - s; f += 10.0 * c * c * c * c; }
    return f / 10.24;
}

/* dw/dq of the M5 spline: 1.25 f'(s) / 10.24. */
double orc_dw5(double q)
{
    double s = 1.25 * q;
    if (s >= 2.5) return 0.0;
    double a = 2.5 - s;
    double fp = -4.0 * a * a * a;
    if (s < 1.5) { double b = 1.5 - s; fp += 20.0 * b * b * b; }
    if (s < 0.5) { double c = 0.5 - s; fp -= 40.0 * c * c * c; }
    return 1.25 * fp / 10.24;
}

/* kernel 0: cubic M4, kernel 1: quartic M5 */
static double kw(int32_t kernel, double q) { return kernel == 1 ? orc_w5(q) : orc_w(q); }
static double kdw(int32_t kernel, double q) { return kernel == 1 ? orc_dw5(q) : orc_dw(q); }
static int kernel_ok(int32_t kernel) { return kernel == 0 || kernel == 1; }

/* W(r,h) = w(r/h) / (pi h^3) */
double orc_W(int32_t kernel, double r, double h) { return kw(kernel, r / h) / (ORC_PI * h * h * h); }
/* dW/dr */
double orc_dWdr(int32_t kernel, double r, double h) { return kdw(kernel, r / h) / (ORC_PI * h * h * h * h); }
/* dW/dh = -(3 w + q w') / (pi h^4) */
double orc_dWdh(int32_t kernel, double r, double h)
{
    double q = r / h;
    return -(3.0 * kw(kernel, q) + q * kdw(kernel, q)) / (ORC_PI * h * h * h * h);
}

/* -------------------------------------------------------------- geometry */

typedef struct {
    double lo[3];
    double len[3];
    int32_t periodic[3];
} orc_box;

/* minimum-image difference a - b along one axis */
static double mi(double a, double b, const orc_box* bx, int d)
{
    double dx = a - b;
    if (bx->periodic[d]) {
        double half = 0.5 * bx->len[d];
        if (dx > half) dx = dx - bx->len[d];
        else if (dx < -half) dx = dx + bx->len[d];
    }
    return dx;
}

/* Oracle-private uniform grid used only to enumerate candidate neighbours. */
typedef struct {
    int64_t np;
    int n[3];
    double cs[3];
    int64_t* start;  /* ncell + 1 */
    int64_t* idx;    /* np */
    double* hmax;    /* per cell max h, may be NULL */
    const orc_box* bx;
    const double *x, *y, *z;
} ogrid;

static int cell_of(double v, const orc_box* bx, const ogrid* g, int d)
{
    double t = floor((v - bx->lo[d]) / g->cs[d]);
    if (t < 0.0) t = 0.0;
    if (t > (double)(g->n[d] - 1)) t = (double)(g->n[d] - 1);
    return (int)t;
}

static int grid_build(ogrid* g, int64_t np, const double* x, const double* y, const double* z,
                      const double* h, const orc_box* bx, double cell_hint)
{
    memset(g, 0, sizeof(*g));
    g->np = np; g->bx = bx; g->x = x; g->y = y; g->z = z;
    for (int d = 0; d < 3; ++d) {
        int n = (int)floor(bx->len[d] / cell_hint);
        if (n < 1) n = 1;
        if (n > 256) n = 256;
        g->n[d] = n;
        g->cs[d] = bx->len[d] / (double)n;
    }
    int64_t nc = (int64_t)g->n[0] * g->n[1] * g->n[2];
    g->start = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
    g->idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
    int64_t* key = (int64_t*)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
    if (h) g->hmax = (double*)calloc((size_t)nc, sizeof(double));
    if (!g->start || !g->idx || !key || (h && !g->hmax)) { free(key); return -1; }
    const double* c[3] = {x, y, z};
    for (int64_t i = 0; i < np; ++i) {
        int k0 = cell_of(c[0][i], bx, g, 0), k1 = cell_of(c[1][i], bx, g, 1), k2 = cell_of(c[2][i], bx, g, 2);
        key[i] = ((int64_t)k2 * g->n[1] + k1) * g->n[0] + k0;
        g->start[key[i] + 1] += 1;
        if (h && h[i] > g->hmax[key[i]]) g->hmax[key[i]] = h[i];
    }
    for (int64_t k = 0; k < nc; ++k) g->start[k + 1] += g->start[k];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)nc);
    if (!fill) { free(key); return -1; }
    memcpy(fill, g->start, sizeof(int64_t) * (size_t)nc);
    for (int64_t i = 0; i < np; ++i) g->idx[fill[key[i]]++] = i;
    free(fill);
    free(key);
    return 0;
}

static void grid_free(ogrid* g)
{
    free(g->start); free(g->idx); free(g->hmax);
    memset(g, 0, sizeof(*g));
}

/* Cell window [k0, k1] along axis d around value v with radius R.  For a
 * periodic axis whose window would cover the grid, every cell once. */
static void window(const ogrid* g, double v, double R, int d, int* k0, int* k1)
{
    const orc_box* bx = g->bx;
    double a = floor((v - R - bx->lo[d]) / g->cs[d]);
    double b = floor((v + R - bx->lo[d]) / g->cs[d]);
    if (bx->periodic[d]) {
        if (b - a + 1.0 >= (double)g->n[d]) { *k0 = 0; *k1 = g->n[d] - 1; return; }
        *k0 = (int)a; *k1 = (int)b;
    } else {
        if (a < 0.0) a = 0.0;
        if (b > (double)(g->n[d] - 1)) b = (double)(g->n[d] - 1);
        *k0 = (int)a; *k1 = (int)b;
    }
}

static int wrapk(int k, int n) { k %= n; return k < 0 ? k + n : k; }

/* Lower bound of the distance from point v to any particle of cell k along
 * axis d (open-axis boundary cells are unbounded outward: particles that left
 * the box are clamped into them). */
static double gap_iv(double v, double clo, double chi)
{
    if (v < clo) return clo - v;
    if (v > chi) return v - chi;
    return 0.0;
}

static double gap1(const ogrid* g, double v, int kw, int d)
{
    const orc_box* bx = g->bx;
    int k = wrapk(kw, g->n[d]);
    double clo = bx->lo[d] + (double)k * g->cs[d];
    double chi = clo + g->cs[d];
    if (bx->periodic[d]) {
        /* nearest of the cell's periodic images (a lower bound in any case) */
        double best = INFINITY;
        for (int s = -1; s <= 1; ++s) {
            double sh = (double)s * bx->len[d];
            double gg = gap_iv(v, clo + sh, chi + sh);
            if (gg < best) best = gg;
        }
        return best;
    }
    if (k == 0) clo = -INFINITY;
    if (k == g->n[d] - 1) chi = INFINITY;
    return gap_iv(v, clo, chi);
}

/* ------------------------------------------------------------- density */

typedef struct {
    double rho, drho, nsum, sdrho;
    int64_t count;   /* pairs j != i inside the support */
} dacc;

static void dens_pair(dacc* a, int32_t kernel, double r2, double h, double mj, int self)
{
    double H = 2.0 * h;
    if (!(r2 < H * H)) return;
    double r = sqrt(r2);
    double q = r / h;
    double w = kw(kernel, q), dw = kdw(kernel, q);
    double norm = 1.0 / (ORC_PI * h * h * h);
    double Wv = w * norm;
    double dWh = -(3.0 * w + q * dw) * norm / h;
    a->rho += mj * Wv;
    a->drho += mj * dWh;
    a->sdrho += fabs(mj * dWh);
    a->nsum += Wv;
    if (!self) a->count += 1;
}

typedef struct {
    int64_t n;
    const double *x, *y, *z, *m;
    const orc_box* bx;
    int32_t kernel;
} pset;

static void dens_sums(const pset* P, const ogrid* g, int64_t i, double h, dacc* a)
{
    memset(a, 0, sizeof(*a));
    const double xi = P->x[i], yi = P->y[i], zi = P->z[i];
    if (!g) {
        for (int64_t j = 0; j < P->n; ++j) {
            double dx = mi(xi, P->x[j], P->bx, 0);
            double dy = mi(yi, P->y[j], P->bx, 1);
            double dz = mi(zi, P->z[j], P->bx, 2);
            double r2 = dx * dx + dy * dy + dz * dz;
            dens_pair(a, P->kernel, r2, h, P->m[j], j == i);
        }
        return;
    }
    double H = 2.0 * h;
    int lo[3], hi[3];
    window(g, xi, H, 0, &lo[0], &hi[0]);
    window(g, yi, H, 1, &lo[1], &hi[1]);
    window(g, zi, H, 2, &lo[2], &hi[2]);
    for (int kz = lo[2]; kz <= hi[2]; ++kz) {
        double gz = gap1(g, zi, kz, 2);
        for (int ky = lo[1]; ky <= hi[1]; ++ky) {
            double gy = gap1(g, yi, ky, 1);
            for (int kx = lo[0]; kx <= hi[0]; ++kx) {
                double gx = gap1(g, xi, kx, 0);
                if (gx * gx + gy * gy + gz * gz >= H * H) continue;
                int64_t c = ((int64_t)wrapk(kz, g->n[2]) * g->n[1] + wrapk(ky, g->n[1])) * g->n[0]
                            + wrapk(kx, g->n[0]);
                for (int64_t t = g->start[c]; t < g->start[c + 1]; ++t) {
                    int64_t j = g->idx[t];
                    double dx = mi(xi, P->x[j], P->bx, 0);
                    double dy = mi(yi, P->y[j], P->bx, 1);
                    double dz = mi(zi, P->z[j], P->bx, 2);
                    double r2 = dx * dx + dy * dy + dz * dz;
                    dens_pair(a, P->kernel, r2, h, P->m[j], j == i);
                }
            }
        }
    }
}

/*
 * Density sums at a given smoothing length, no iteration: rho_i, drho_i/dh,
 * n_i = sum_j W(r_ij, h_i) (self included) and the number of pairs j != i.
 */
int orc_density_at(int64_t n, const double* x, const double* y, const double* z, const double* m,
                   const orc_box* bx, int32_t brute, double cell_hint,
                   int64_t nt, const int64_t* targets, const double* h_eval,
                   double* rho, double* drho, double* nsum, int64_t* count, int32_t nthreads,
                   int32_t kernel)
{
    if (!kernel_ok(kernel)) return -2;
    pset P = {n, x, y, z, m, bx, kernel};
    ogrid G, *g = NULL;
    if (!brute) { if (grid_build(&G, n, x, y, z, NULL, bx, cell_hint)) return -1; g = &G; }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t t = 0; t < nt; ++t) {
        dacc a;
        dens_sums(&P, g, targets[t], h_eval[t], &a);
        rho[t] = a.rho; drho[t] = a.drho; nsum[t] = a.nsum; count[t] = a.count;
    }
    (void)nthreads;
    if (g) grid_free(g);
    return 0;
}

/*
 * Density with the smoothing-length iteration (paper Sec. 2.1, step 1:
 * h and rho are updated until each particle meets its termination criterion).
 *
 * Root condition (reading): rho_i(h) h^3 = m_i eta^3, i.e. f(h) = rho_i(h) - m_i eta^3 / h^3.
 * Newton: h+ = h - f/f', f' = drho/dh + 3 m_i eta^3 / h^4, clamped to [h/2, 2h];
 * if f' <= 0 or h+ is not finite, the fixed point h+ = eta (m_i/rho_i)^(1/3).
 * Stop: the current h (whose sums were just evaluated) is accepted when
 * |h+ - h| <= tol h; after max_iter evaluations the last one is returned and
 * the particle is flagged not converged.
 * Outputs at the accepted h: rho, Omega = 1 + h/(3 rho) drho/dh,
 * wcount = (4 pi/3)(2h)^3 n_i, drho/dh, sum |m_j dW/dh|, pair count,
 * number of evaluations, converged flag.
 */
int orc_density(int64_t n, const double* x, const double* y, const double* z, const double* m,
                const double* h0, const orc_box* bx, double eta, double tol, int32_t max_iter,
                int32_t brute, double cell_hint, int64_t nt, const int64_t* targets,
                double* out_h, double* out_rho, double* out_omega, double* out_wcount,
                double* out_drho, double* out_sdrho, int64_t* out_count, int32_t* out_iters,
                int32_t* out_conv, int32_t nthreads, int32_t kernel)
{
    if (!kernel_ok(kernel)) return -2;
    pset P = {n, x, y, z, m, bx, kernel};
    ogrid G, *g = NULL;
    if (!brute) { if (grid_build(&G, n, x, y, z, NULL, bx, cell_hint)) return -1; g = &G; }
    const double eta3 = eta * eta * eta;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targets[t];
        double h = h0[i];
        dacc a;
        int it = 0, conv = 0;
        for (;;) {
            dens_sums(&P, g, i, h, &a);
            ++it;
            double mq = m[i] * eta3;
            double f = a.rho - mq / (h * h * h);
            double fp = a.drho + 3.0 * mq / (h * h * h * h);
            double hn;
            if (fp > 0.0) {
                hn = h - f / fp;
                if (hn < 0.5 * h) hn = 0.5 * h;
                if (hn > 2.0 * h) hn = 2.0 * h;
            } else {
                hn = eta * cbrt(m[i] / a.rho);
            }
            if (!isfinite(hn)) hn = eta * cbrt(m[i] / a.rho);
            if (fabs(hn - h) <= tol * h) { conv = 1; break; }
            if (it >= max_iter) break;
            h = hn;
        }
        out_h[t] = h;
        out_rho[t] = a.rho;
        out_omega[t] = 1.0 + h / (3.0 * a.rho) * a.drho;
        out_wcount[t] = (4.0 * ORC_PI / 3.0) * (8.0 * h * h * h) * a.nsum;
        out_drho[t] = a.drho;
        out_sdrho[t] = a.sdrho;
        out_count[t] = a.count;
        out_iters[t] = it;
        out_conv[t] = conv;
    }
    (void)nthreads;
    if (g) grid_free(g);
    return 0;
}

/* --------------------------------------------------------------- force */

typedef struct {
    int64_t n;
    const double *x, *y, *z, *vx, *vy, *vz, *m, *h, *rho, *omega, *u, *alpha;
    const orc_box* bx;
    double gamma;
    int32_t kernel;
} fset;

typedef struct {
    double ax, ay, az, udot, vsig, sa, su;
    int64_t count;
} facc;

static void force_pair(const fset* F, int64_t i, int64_t j, facc* a)
{
    if (j == i) return;
    double dx = mi(F->x[i], F->x[j], F->bx, 0);
    double dy = mi(F->y[i], F->y[j], F->bx, 1);
    double dz = mi(F->z[i], F->z[j], F->bx, 2);
    double r2 = dx * dx + dy * dy + dz * dz;
    double hi = F->h[i], hj = F->h[j];
    double H = 2.0 * (hi > hj ? hi : hj);
    if (!(r2 < H * H)) return;
    a->count += 1;
    if (r2 == 0.0) return;                       /* coincident: no direction, no force */
    const double gm = F->gamma;
    double Pi_ = (gm - 1.0) * F->rho[i] * F->u[i];
    double Pj_ = (gm - 1.0) * F->rho[j] * F->u[j];
    double ci = sqrt(gm * (gm - 1.0) * F->u[i]);
    double cj = sqrt(gm * (gm - 1.0) * F->u[j]);
    double Ai = Pi_ / (F->omega[i] * F->rho[i] * F->rho[i]);
    double Aj = Pj_ / (F->omega[j] * F->rho[j] * F->rho[j]);
    double r = sqrt(r2);
    double gi = orc_dWdr(F->kernel, r, hi);       /* 0 outside 2 h_i */
    double gj = orc_dWdr(F->kernel, r, hj);
    double gbar = 0.5 * (gi + gj);
    double ex = dx / r, ey = dy / r, ez = dz / r;
    double dvx = F->vx[i] - F->vx[j], dvy = F->vy[i] - F->vy[j], dvz = F->vz[i] - F->vz[j];
    double wdot = dvx * ex + dvy * ey + dvz * ez;
    double mu = wdot < 0.0 ? wdot : 0.0;
    double vs = ci + cj - 3.0 * mu;
    double visc = -0.5 * (0.5 * (F->alpha[i] + F->alpha[j])) * vs * mu / (0.5 * (F->rho[i] + F->rho[j]));
    double mj = F->m[j];
    double coef = mj * (Ai * gi + Aj * gj + visc * gbar);
    a->ax -= coef * ex;
    a->ay -= coef * ey;
    a->az -= coef * ez;
    double du = mj * (Ai * gi + 0.5 * visc * gbar) * wdot;
    a->udot += du;
    a->sa += fabs(coef);
    a->su += fabs(du);
    if (vs > a->vsig) a->vsig = vs;
}

/*
 * Force (paper Sec. 2.1, step 2: the sum of the forces between a particle and
 * its neighbours).  Pair set: j != i with r_ij < 2 max(h_i, h_j).
 *   P = (gamma-1) rho u, c = sqrt(gamma (gamma-1) u), A = P / (Omega rho^2)
 *   a_i  -= m_j (A_i g_i + A_j g_j + Pi_ij gbar) r_hat
 *   du_i += m_j (A_i g_i + Pi_ij gbar / 2) (v_ij . r_hat)
 *   g = dW/dr(r, h) per side, gbar = (g_i + g_j)/2, mu = min(v_ij.r_hat, 0),
 *   v_sig,ij = c_i + c_j - 3 mu, Pi_ij = -(alpha_bar/2) v_sig,ij mu / rho_bar,
 *   v_sig,i = max(2 c_i, max_j v_sig,ij).
 * Also returns sum_j |coef| and sum_j |du| (scales for the error metric).
 */
int orc_force(int64_t n, const double* x, const double* y, const double* z,
              const double* vx, const double* vy, const double* vz, const double* m,
              const double* h, const double* rho, const double* omega, const double* u,
              const double* alpha, const orc_box* bx, double gamma, int32_t brute,
              double cell_hint, int64_t nt, const int64_t* targets,
              double* out_ax, double* out_ay, double* out_az, double* out_udot,
              double* out_vsig, double* out_sa, double* out_su, int64_t* out_count,
              int32_t nthreads, int32_t kernel)
{
    if (!kernel_ok(kernel)) return -2;
    fset F = {n, x, y, z, vx, vy, vz, m, h, rho, omega, u, alpha, bx, gamma, kernel};
    ogrid G, *g = NULL;
    double hglob = 0.0;
    for (int64_t i = 0; i < n; ++i) if (h[i] > hglob) hglob = h[i];
    if (!brute) { if (grid_build(&G, n, x, y, z, h, bx, cell_hint)) return -1; g = &G; }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targets[t];
        facc a;
        memset(&a, 0, sizeof(a));
        a.vsig = 2.0 * sqrt(gamma * (gamma - 1.0) * u[i]);
        if (!g) {
            for (int64_t j = 0; j < n; ++j) force_pair(&F, i, j, &a);
        } else {
            double xi[3] = {x[i], y[i], z[i]};
            double R = 2.0 * (h[i] > hglob ? h[i] : hglob);
            int lo[3], hi[3];
            for (int d = 0; d < 3; ++d) window(g, xi[d], R, d, &lo[d], &hi[d]);
            for (int kz = lo[2]; kz <= hi[2]; ++kz) {
                double gz = gap1(g, xi[2], kz, 2);
                for (int ky = lo[1]; ky <= hi[1]; ++ky) {
                    double gy = gap1(g, xi[1], ky, 1);
                    for (int kx = lo[0]; kx <= hi[0]; ++kx) {
                        double gx = gap1(g, xi[0], kx, 0);
                        int64_t c = ((int64_t)wrapk(kz, g->n[2]) * g->n[1] + wrapk(ky, g->n[1])) * g->n[0]
                                    + wrapk(kx, g->n[0]);
                        double hc = g->hmax[c] > h[i] ? g->hmax[c] : h[i];
                        if (gx * gx + gy * gy + gz * gz >= 4.0 * hc * hc) continue;
                        for (int64_t s = g->start[c]; s < g->start[c + 1]; ++s)
                            force_pair(&F, i, g->idx[s], &a);
                    }
                }
            }
        }
        out_ax[t] = a.ax; out_ay[t] = a.ay; out_az[t] = a.az;
        out_udot[t] = a.udot; out_vsig[t] = a.vsig;
        out_sa[t] = a.sa; out_su[t] = a.su; out_count[t] = a.count;
    }
    (void)nthreads;
    if (g) grid_free(g);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
