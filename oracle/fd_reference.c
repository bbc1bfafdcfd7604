/*
 * fd_reference.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Finite-difference reference solution of the relaxed Winslow system
 * (Sect. 2, eq. (3)):
 *
 *     u_t = Lu,   L = Laplacian + b . grad,   b = -grad w / w   (eq. (6)),
 *
 * for u in {xi, eta} on the unit square with Dirichlet boundary data and
 * initial data (Sect. 3), used as the ground truth that the Monte-Carlo
 * estimates are measured against.  It approximates the PDE solution itself,
 * not the Euler-Maruyama chain.
 *
 * Scheme (a textbook one, chosen to be easy to check rather than fast):
 * second-order central differences on a uniform (n+1)^2 nodal grid and the
 * Peaceman-Rachford alternating-direction implicit splitting in time,
 *
 *     (I - D/2 A_x) u*      = (I + D/2 A_y) u^m
 *     (I - D/2 A_y) u^{m+1} = (I + D/2 A_x) u*,
 *
 * with A_x = d_xx + b_x d_x, A_y = d_yy + b_y d_y and the coefficients taken
 * at the half step.  Each implicit half step is a set of tridiagonal solves
 * (Thomas algorithm).  The boundary data are static in every case used here,
 * so the intermediate u* takes the boundary data too.
 *
 * Grids are row-major [j][i] with x = i/n, y = j/n.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FD_PI 3.14159265358979323846

/* Density and drift, FP64, for the finite-difference coefficients.  Written
 * again here (not shared with the Monte-Carlo oracle file) so that a slip in
 * one of the two would show up as a disagreement between them. */
static void fd_drift(int kind, const double *par, double tau, double x, double y,
                     double *bx, double *by)
{
    const double A = par[0], s2 = par[1], cx = par[2], cy = par[3];
    const double R = par[4], om = par[5];
    double gx = 0.0, gy = 0.0, w = 1.0; /* grad w and w */
    if (kind == 1 || kind == 2) {
        double ccx = cx, ccy = cy;
        if (kind == 2) { ccx += R * cos(om * tau); ccy += R * sin(om * tau); }
        double e = exp(-((x - ccx) * (x - ccx) + (y - ccy) * (y - ccy)) / s2);
        w = 1.0 + A * e;
        gx = -2.0 * A * e * (x - ccx) / s2;
        gy = -2.0 * A * e * (y - ccy) / s2;
    } else if (kind == 3) {
        double c = R * cos(om * tau), s = R * sin(om * tau);
        double ax = cx + c, bxx = cx - c, ay = cy + s;
        double e1 = exp(-((x - ax) * (x - ax) + (y - ay) * (y - ay)) / s2);
        double e2 = exp(-((x - bxx) * (x - bxx) + (y - ay) * (y - ay)) / s2);
        w = 1.0 + A * (e1 + e2);
        gx = -2.0 * A * (e1 * (x - ax) + e2 * (x - bxx)) / s2;
        gy = -2.0 * A * (e1 + e2) * (y - ay) / s2;
    } else if (kind == 4) {
        double ccx = cx + R * cos(om * tau), ccy = cy + R * sin(om * tau);
        double q = (x - ccx) * (x - ccx) + (y - ccy) * (y - ccy) - 0.01;
        double e = exp(s2 * fabs(q));
        double rho = 1.0 + A * e;
        double sg = q > 0 ? 1.0 : (q < 0 ? -1.0 : 0.0);
        /* w = 1/rho: -grad w / w = grad rho / rho */
        *bx = A * e * s2 * sg * 2.0 * (x - ccx) / rho;
        *by = A * e * s2 * sg * 2.0 * (y - ccy) / rho;
        return;
    } else if (kind == 5) {
        double e = exp(-(x - cx) * (x - cx) / s2);
        w = 1.0 + A * e;
        gx = -2.0 * A * e * (x - cx) / s2;
        gy = 0.0;
    }
    *bx = -gx / w;
    *by = -gy / w;
}

static double fd_sin_mode(double x, double y) { return sin(FD_PI * x) * sin(FD_PI * y); }

/* Tridiagonal solve a_i u_{i-1} + d_i u_i + c_i u_{i+1} = r_i, i = 0..m-1
 * (a_0 and c_{m-1} unused); overwrites r with the solution. */
static void thomas(int m, const double *a, const double *d, const double *c, double *r, double *work)
{
    double *cp = work;
    double beta = d[0];
    r[0] /= beta;
    for (int i = 1; i < m; ++i) {
        cp[i - 1] = c[i - 1] / beta;
        beta = d[i] - a[i] * cp[i - 1];
        r[i] = (r[i] - a[i] * r[i - 1]) / beta;
    }
    for (int i = m - 2; i >= 0; --i) r[i] -= cp[i] * r[i + 1];
}

/*
 * Solve from PDE time t_init over a duration t with about t/dtau steps.
 *   init_kind: 0 identity, 1 sine mode, 3 grid (grid_xi0/grid_eta0, (n+1)^2)
 *   bdry_kind: 0 identity, 1 sine mode (zero on the boundary), 2 zero
 *   xi, eta:   (n+1)^2 outputs
 * Returns 0, or -1 on bad arguments.
 */
int or_fd_solve(int kind, int time_mode, const double *par, int init_kind, int bdry_kind,
                double t_init, double t, int n, double dtau,
                const double *grid_xi0, const double *grid_eta0, int n_threads,
                double *xi, double *eta)
{
    if (n < 2 || !(dtau > 0.0) || t < 0.0) return -1;
    const int N1 = n + 1;
    const double h = 1.0 / n;
    const int64_t NN = (int64_t)N1 * N1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    /* initial data */
    for (int j = 0; j < N1; ++j)
        for (int i = 0; i < N1; ++i) {
            double x = i * h, y = j * h;
            int64_t id = (int64_t)j * N1 + i;
            if (init_kind == 0) { xi[id] = x; eta[id] = y; }
            else if (init_kind == 1) { xi[id] = eta[id] = fd_sin_mode(x, y); }
            else if (init_kind == 3) { xi[id] = grid_xi0[id]; eta[id] = grid_eta0[id]; }
            else { xi[id] = eta[id] = 0.0; }
        }
    /* static boundary data */
    for (int j = 0; j < N1; ++j)
        for (int i = 0; i < N1; ++i) {
            if (i != 0 && i != n && j != 0 && j != n) continue;
            double x = i * h, y = j * h;
            int64_t id = (int64_t)j * N1 + i;
            if (bdry_kind == 0) { xi[id] = x; eta[id] = y; }
            else { xi[id] = eta[id] = 0.0; } /* sine mode vanishes on the boundary */
        }
    if (t == 0.0) return 0;

    int64_t nst = (int64_t)ceil(t / dtau - 1e-9);
    double D = t / (double)nst;
    double *bx = (double *)malloc(sizeof(double) * NN);
    double *by = (double *)malloc(sizeof(double) * NN);
    double *sx = (double *)malloc(sizeof(double) * NN);
    double *se = (double *)malloc(sizeof(double) * NN);
    if (!bx || !by || !sx || !se) { free(bx); free(by); free(sx); free(se); return -1; }
    memcpy(sx, xi, sizeof(double) * NN);
    memcpy(se, eta, sizeof(double) * NN);
    const double ih2 = 1.0 / (h * h), i2h = 1.0 / (2.0 * h);

    for (int64_t m = 0; m < nst; ++m) {
        double tau = (time_mode == 0) ? t_init + (m + 0.5) * D : par[6];
        if (m == 0 || time_mode == 0) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
            for (int j = 0; j < N1; ++j)
                for (int i = 0; i < N1; ++i)
                    fd_drift(kind, par, tau, i * h, j * h, &bx[(int64_t)j * N1 + i], &by[(int64_t)j * N1 + i]);
        }
        /* half step 1: implicit in x along each interior row j */
#ifdef _OPENMP
#pragma omp parallel
#endif
        {
            double *a = (double *)malloc(sizeof(double) * N1 * 6);
            double *d = a + N1, *c = d + N1, *r1 = c + N1, *r2 = r1 + N1, *wk = r2 + N1;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int j = 1; j < n; ++j) {
                int mm = n - 1;
                for (int i = 1; i < n; ++i) {
                    int64_t id = (int64_t)j * N1 + i;
                    double bxv = bx[id], byv = by[id];
                    a[i - 1] = -0.5 * D * (ih2 - bxv * i2h);
                    d[i - 1] = 1.0 + D * ih2;
                    c[i - 1] = -0.5 * D * (ih2 + bxv * i2h);
                    const double *u = xi, *v = eta;
                    double ay_u = (u[id + N1] - 2 * u[id] + u[id - N1]) * ih2 + byv * (u[id + N1] - u[id - N1]) * i2h;
                    double ay_v = (v[id + N1] - 2 * v[id] + v[id - N1]) * ih2 + byv * (v[id + N1] - v[id - N1]) * i2h;
                    r1[i - 1] = u[id] + 0.5 * D * ay_u;
                    r2[i - 1] = v[id] + 0.5 * D * ay_v;
                }
                /* Dirichlet ends (u* = boundary data) */
                int64_t row = (int64_t)j * N1;
                r1[0] -= a[0] * sx[row];
                r2[0] -= a[0] * se[row];
                r1[mm - 1] -= c[mm - 1] * sx[row + n];
                r2[mm - 1] -= c[mm - 1] * se[row + n];
                thomas(mm, a, d, c, r1, wk);
                thomas(mm, a, d, c, r2, wk);
                for (int i = 1; i < n; ++i) {
                    sx[row + i] = r1[i - 1];
                    se[row + i] = r2[i - 1];
                }
            }
            free(a);
        }
        /* half step 2: implicit in y along each interior column i */
#ifdef _OPENMP
#pragma omp parallel
#endif
        {
            double *a = (double *)malloc(sizeof(double) * N1 * 6);
            double *d = a + N1, *c = d + N1, *r1 = c + N1, *r2 = r1 + N1, *wk = r2 + N1;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int i = 1; i < n; ++i) {
                int mm = n - 1;
                for (int j = 1; j < n; ++j) {
                    int64_t id = (int64_t)j * N1 + i;
                    double bxv = bx[id], byv = by[id];
                    a[j - 1] = -0.5 * D * (ih2 - byv * i2h);
                    d[j - 1] = 1.0 + D * ih2;
                    c[j - 1] = -0.5 * D * (ih2 + byv * i2h);
                    double ax_u = (sx[id + 1] - 2 * sx[id] + sx[id - 1]) * ih2 + bxv * (sx[id + 1] - sx[id - 1]) * i2h;
                    double ax_v = (se[id + 1] - 2 * se[id] + se[id - 1]) * ih2 + bxv * (se[id + 1] - se[id - 1]) * i2h;
                    r1[j - 1] = sx[id] + 0.5 * D * ax_u;
                    r2[j - 1] = se[id] + 0.5 * D * ax_v;
                }
                r1[0] -= a[0] * xi[i];
                r2[0] -= a[0] * eta[i];
                r1[mm - 1] -= c[mm - 1] * xi[(int64_t)n * N1 + i];
                r2[mm - 1] -= c[mm - 1] * eta[(int64_t)n * N1 + i];
                thomas(mm, a, d, c, r1, wk);
                thomas(mm, a, d, c, r2, wk);
                for (int j = 1; j < n; ++j) {
                    xi[(int64_t)j * N1 + i] = r1[j - 1];
                    eta[(int64_t)j * N1 + i] = r2[j - 1];
                }
            }
            free(a);
        }
    }
    free(bx); free(by); free(sx); free(se);
    return 0;
}
