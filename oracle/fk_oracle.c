/*
 * fk_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Plain, slow, FP64 CPU oracle of the Monte-Carlo evaluation of the
 * Feynman-Kac representation of the relaxed Winslow mesh equations
 * (Bihlo & Haynes, "A stochastic domain decomposition method for time
 * dependent mesh generation", Sect. 3, eqs. (5)-(7); Sect. 4).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * load this file's library.  It shares no source with the GPU path: the
 * counter-based generator, the normal transform, the densities, the
 * Euler-Maruyama step, the exit test, the scoring and the statistics are all
 * written out here a second time, in FP64, one path at a time.
 *
 * What is computed, for an interface node P and component c in {xi, eta}:
 *
 *   U_c(P) = mean over paths of  g_c(t - s_kappa, X_kappa)  if the path left
 *            the closed unit square at step kappa <= K, else u0_c(X_K),
 *
 * where X_0 = P and X_{k+1} = X_k + b(tau_k, X_k) D_k + sqrt(2 D_k) z_k is the
 * Euler-Maruyama chain of dX = -(grad w / w) ds + sqrt(2) dW (eq. (7a);
 * Sect. 4 integrates it with the Euler-Maruyama scheme and Brownian
 * increments sqrt(D) times a standard normal).  The drift is the
 * Winslow choice a = I, b = -grad w / w (eq. (6)).  The estimator is the
 * arithmetic mean of eq. (7b) (Sect. 4), with a sample standard error.
 *
 * Readings where the paper is silent (each one is also listed in the design
 * notes):
 *  - time argument of w along a path: BACKWARD uses the PDE time
 *    t_init + t - s reached by running the path backward from the evaluation
 *    time; FROZEN holds w at t_freeze over the whole solve (Sect. 4 freezes w
 *    over one mesh step).
 *  - the exit test runs after every step, the last included; points on the
 *    boundary count as inside (eq. (5) uses strict inequalities).
 *  - a path that exits scores the boundary data at its first outside point,
 *    unclamped, with the data extended off the square (identity data extends
 *    as xi = x, eta = y); a PROJECT mode clamps the point first; a BRIDGE
 *    mode adds the Brownian-bridge crossing test within each step (see
 *    bridge_exit) and scores every exit at the point projected onto the
 *    square.
 *  - the normal generator: Philox4x32-10 (Salmon, Moraes, Dror & Shaw,
 *    SC'11), key = (seed low word, seed high word), counter = (k/2, path,
 *    node, (level << 4) | stream); one call serves two steps (words 0,1 for
 *    even steps, 2,3 for odd); Box-Muller on the words' low 23 bits
 *    m: u1 = 1 - m 2^-23 in (0,1], u2 = m 2^-23 in [0,1).
 *  - step sizes: K = ceil(t/dt), every step dt except the last, which is
 *    t - (K-1) dt.
 *  - exponential time-stepping (score mode 4; Sect. 4 names it as the
 *    alternative to the fixed steps, after Jansons & Lythe 2003): see
 *    run_path_expo.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ---------------------------------------------------------------------------
 * Philox4x32-10, written from its published definition (Salmon et al. 2011):
 * a 4-word counter goes through 10 rounds; each round multiplies words 0 and 2
 * by two fixed odd constants into 64-bit products, and the new state is
 *   (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0)).
 * Between rounds the 2-word key is advanced by the Weyl constants
 * (golden ratio and sqrt(3)-1 in 32-bit fixed point).
 * ------------------------------------------------------------------------- */
static const uint32_t PHILOX_MULT_A = 0xD2511F53u;
static const uint32_t PHILOX_MULT_B = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL_A = 0x9E3779B9u;
static const uint32_t PHILOX_WEYL_B = 0xBB67AE85u;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL_A;
            k1 += PHILOX_WEYL_B;
        }
        uint64_t pa = (uint64_t)PHILOX_MULT_A * (uint64_t)x0;
        uint64_t pb = (uint64_t)PHILOX_MULT_B * (uint64_t)x2;
        uint32_t n0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
        uint32_t n1 = (uint32_t)pb;
        uint32_t n2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
        uint32_t n3 = (uint32_t)pa;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void or_philox_batch(const uint32_t *ctr, const uint32_t *key, int64_t n, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i)
        or_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* Box-Muller on the two 23-bit uniforms taken from a pair of Philox words
 * (their low 23 bits). */
static void box_muller(uint32_t ra, uint32_t rb, double *z0, double *z1)
{
    double u1 = 1.0 - (double)(ra & 0x7fffffu) * 0x1p-23;   /* (0, 1] */
    double u2 = (double)(rb & 0x7fffffu) * 0x1p-23;         /* [0, 1) */
    double r = sqrt(-2.0 * log(u1));
    *z0 = r * cos(2.0 * OR_PI * u2);
    *z1 = r * sin(2.0 * OR_PI * u2);
}

void or_normals_batch(const uint32_t *ra, const uint32_t *rb, int64_t n, double *z)
{
    for (int64_t i = 0; i < n; ++i)
        box_muller(ra[i], rb[i], &z[2 * i], &z[2 * i + 1]);
}

/* ---------------------------------------------------------------------------
 * Densities w(tau, x, y) and the Winslow drift b = -grad w / w (eq. (6)).
 * par = {amp, width2, cx, cy, orbit_r, omega, t_freeze}.
 * ------------------------------------------------------------------------- */
enum { K_CONST = 0, K_BUMP = 1, K_MOVING = 2, K_TWO = 3, K_RING = 4, K_RIDGE = 5, K_GRID = 6 };

/* A density: its kind and parameters, and for K_GRID its nodal samples. */
typedef struct {
    int kind;
    const double *par;
    const double *wg;  /* K_GRID: w at the nodes of an n-cell grid, [(n+1)^2] row-major [j][i], x = i/n */
    int wn;
} or_dens;


/* w and its gradient, analytically. */
static void density(int kind, const double *par, double tau, double x, double y,
                    double *w, double *wx, double *wy)
{
    const double A = par[0], s2 = par[1], cx = par[2], cy = par[3];
    const double R = par[4], om = par[5];
    switch (kind) {
    case K_BUMP: {
        double dx = x - cx, dy = y - cy;
        double e = exp(-(dx * dx + dy * dy) / s2);
        *w = 1.0 + A * e;
        *wx = A * e * (-2.0 * dx / s2);
        *wy = A * e * (-2.0 * dy / s2);
        return;
    }
    case K_MOVING: {
        double ccx = cx + R * cos(om * tau), ccy = cy + R * sin(om * tau);
        double dx = x - ccx, dy = y - ccy;
        double e = exp(-(dx * dx + dy * dy) / s2);
        *w = 1.0 + A * e;
        *wx = A * e * (-2.0 * dx / s2);
        *wy = A * e * (-2.0 * dy / s2);
        return;
    }
    case K_TWO: {
        double c = R * cos(om * tau), s = R * sin(om * tau);
        double d1x = x - (cx + c), d1y = y - (cy + s);
        double d2x = x - (cx - c), d2y = y - (cy + s);
        double e1 = exp(-(d1x * d1x + d1y * d1y) / s2);
        double e2 = exp(-(d2x * d2x + d2y * d2y) / s2);
        *w = 1.0 + A * (e1 + e2);
        *wx = A * (e1 * (-2.0 * d1x / s2) + e2 * (-2.0 * d2x / s2));
        *wy = A * (e1 * (-2.0 * d1y / s2) + e2 * (-2.0 * d2y / s2));
        return;
    }
    case K_RING: {
        /* w = 1/rho, rho = 1 + alpha exp(beta |r^2 - 1/100|)  (Sect. 5);
           amp = alpha, width2 = beta. */
        double ccx = cx + R * cos(om * tau), ccy = cy + R * sin(om * tau);
        double dx = x - ccx, dy = y - ccy;
        double q = dx * dx + dy * dy - 0.01;
        double e = exp(s2 * fabs(q));
        double rho = 1.0 + A * e;
        double sg = (q > 0.0) ? 1.0 : ((q < 0.0) ? -1.0 : 0.0);
        double rx = A * e * s2 * sg * 2.0 * dx, ry = A * e * s2 * sg * 2.0 * dy;
        *w = 1.0 / rho;
        *wx = -rx / (rho * rho);
        *wy = -ry / (rho * rho);
        return;
    }
    case K_RIDGE: {
        double dx = x - cx;
        double e = exp(-dx * dx / s2);
        *w = 1.0 + A * e;
        *wx = A * e * (-2.0 * dx / s2);
        *wy = 0.0;
        return;
    }
    default:
        *w = 1.0; *wx = 0.0; *wy = 0.0;
        return;
    }
}

/* ---------------------------------------------------------------------------
 * The paper's data path for w (Sect. 4): w is known only at the nodes of a
 * grid; the derivatives in grad w are finite differences there and b is
 * interpolated bilinearly between the nodes.  Readings: central differences
 * at interior nodes, the second-order one-sided formula on the edges
 * (f'(0) ~ (-3 f0 + 4 f1 - f2) / 2h), b = -grad w / w at each node, and the
 * bilinear interpolant of those nodal drifts inside each cell.
 * ------------------------------------------------------------------------- */

/* Derivative at index i of the n+1 values v[0], v[step], ..., v[n step]
   spaced h = 1/n apart. */
static double fd_derivative(const double *v, int n, int i, int64_t step)
{
    const double h = 1.0 / n;
    if (i == 0) return (-3.0 * v[0] + 4.0 * v[step] - v[2 * step]) / (2.0 * h);
    if (i == n) return (3.0 * v[n * step] - 4.0 * v[(n - 1) * step] + v[(n - 2) * step]) / (2.0 * h);
    return (v[(i + 1) * step] - v[(i - 1) * step]) / (2.0 * h);
}

/* b = -grad w / w at grid node (i, j). */
static void grid_node_drift(const double *wg, int n, int i, int j, double *bx, double *by)
{
    const double *row = wg + (int64_t)j * (n + 1);  /* w(., y_j) */
    const double *col = wg + i;                    /* w(x_i, .) */
    const double w = row[i];
    *bx = -fd_derivative(row, n, i, 1) / w;
    *by = -fd_derivative(col, n, j, n + 1) / w;
}

/* The cell of point (x, y) in an n-cell grid (the edge cells continued
   outside) and the local coordinates in it. */
static void grid_cell(int n, double x, double y, int *i, int *j, double *ax, double *ay)
{
    double fx = x * n, fy = y * n;
    int ci = (int)floor(fx), cj = (int)floor(fy);
    if (ci < 0) ci = 0;
    if (ci > n - 1) ci = n - 1;
    if (cj < 0) cj = 0;
    if (cj > n - 1) cj = n - 1;
    *i = ci;
    *j = cj;
    *ax = fx - ci;
    *ay = fy - cj;
}

static void grid_drift(const double *wg, int n, double x, double y, double *bx, double *by)
{
    int i, j;
    double ax, ay, b[2][2][2];
    grid_cell(n, x, y, &i, &j, &ax, &ay);
    for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) grid_node_drift(wg, n, i + di, j + dj, &b[dj][di][0], &b[dj][di][1]);
    double out[2];
    for (int c = 0; c < 2; ++c)
        out[c] = (1 - ay) * ((1 - ax) * b[0][0][c] + ax * b[0][1][c]) + ay * ((1 - ax) * b[1][0][c] + ax * b[1][1][c]);
    *bx = out[0];
    *by = out[1];
}

/* w itself between the nodes of a grid density: bilinear. */
static double grid_w(const double *wg, int n, double x, double y)
{
    int i, j;
    double ax, ay;
    grid_cell(n, x, y, &i, &j, &ax, &ay);
    const double *r0 = wg + (int64_t)j * (n + 1), *r1 = r0 + (n + 1);
    return (1 - ay) * ((1 - ax) * r0[i] + ax * r0[i + 1]) + ay * ((1 - ax) * r1[i] + ax * r1[i + 1]);
}

static void drift(const or_dens *d, double tau, double x, double y, double *bx, double *by)
{
    if (d->kind == K_GRID) {
        grid_drift(d->wg, d->wn, x, y, bx, by);
        return;
    }
    double w, wx, wy;
    density(d->kind, d->par, tau, x, y, &w, &wx, &wy);
    *bx = -wx / w;
    *by = -wy / w;
}

static int dens_bind(or_dens *d, int kind, const double *par, const double *wg, int wn)
{
    d->kind = kind;
    d->par = par;
    d->wg = wg;
    d->wn = wn;
    if (kind < K_CONST || kind > K_GRID) return -1;
    if (kind == K_GRID && (!wg || wn < 2)) return -1;
    return 0;
}

/* w and b at n points; w_grid / w_n are read for kind 6 only. */
int or_density_batch(int kind, const double *par, const double *w_grid, int w_n, double tau,
                     const double *pts, int64_t n, double *w, double *b)
{
    or_dens d;
    if (dens_bind(&d, kind, par, w_grid, w_n) != 0) return -1;
    for (int64_t i = 0; i < n; ++i) {
        const double x = pts[2 * i], y = pts[2 * i + 1];
        if (kind == K_GRID) {
            w[i] = grid_w(w_grid, w_n, x, y);
        } else {
            double wx, wy;
            density(kind, par, tau, x, y, &w[i], &wx, &wy);
        }
        drift(&d, tau, x, y, &b[2 * i], &b[2 * i + 1]);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Initial data u0 and boundary data g (Sect. 3: xi0 = x, eta0 = y; boundary
 * data of the uniform mesh).  Test modes: the decaying sine mode and zero.
 * ------------------------------------------------------------------------- */
enum { D_IDENTITY = 0, D_SIN = 1, D_ZERO = 2, D_GRID = 3 };

static double sin_mode(double x, double y) { return sin(OR_PI * x) * sin(OR_PI * y); }

static double bilinear(const double *g, int n, double x, double y)
{
    double fx = x * n, fy = y * n;
    int i = (int)floor(fx), j = (int)floor(fy);
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    if (j < 0) j = 0;
    if (j > n - 1) j = n - 1;
    double ax = fx - i, ay = fy - j;
    const double *r0 = g + (int64_t)j * (n + 1), *r1 = r0 + (n + 1);
    return (1 - ay) * ((1 - ax) * r0[i] + ax * r0[i + 1]) + ay * ((1 - ax) * r1[i] + ax * r1[i + 1]);
}

typedef struct {
    int init_kind, bdry_kind, score_mode;
    const double *grid_xi, *grid_eta;
    int grid_n;
} or_data;

static void initial_value(const or_data *d, double x, double y, double *xi, double *eta)
{
    switch (d->init_kind) {
    case D_IDENTITY: *xi = x; *eta = y; return;
    case D_SIN: *xi = *eta = sin_mode(x, y); return;
    case D_GRID:
        *xi = bilinear(d->grid_xi, d->grid_n, x, y);
        *eta = bilinear(d->grid_eta, d->grid_n, x, y);
        return;
    default: *xi = *eta = 0.0; return;
    }
}

/* Boundary data at elapsed time since the initial data, at an exit point. */
static void boundary_value(const or_data *d, double elapsed, double x, double y,
                           double *xi, double *eta)
{
    if (d->score_mode == 2) {
        /* the grid initial data continued bilinearly from its edge cells: the
           boundary data (the grid's edge nodes) extended by the grid's slope */
        *xi = bilinear(d->grid_xi, d->grid_n, x, y);
        *eta = bilinear(d->grid_eta, d->grid_n, x, y);
        return;
    }
    if (d->score_mode == 1 || d->score_mode == 3 || d->score_mode == 4) {
        x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
        y = y < 0.0 ? 0.0 : (y > 1.0 ? 1.0 : y);
    }

    switch (d->bdry_kind) {
    case D_IDENTITY: *xi = x; *eta = y; return;
    case D_SIN: *xi = *eta = exp(-2.0 * OR_PI * OR_PI * elapsed) * sin_mode(x, y); return;
    case D_GRID:
        /* the grid initial data on the square's edge (its edge nodes hold the
           boundary data), at the projected exit point */
        *xi = bilinear(d->grid_xi, d->grid_n, x, y);
        *eta = bilinear(d->grid_eta, d->grid_n, x, y);
        return;
    default: *xi = *eta = 0.0; return;
    }
}

/* ---------------------------------------------------------------------------
 * One Euler-Maruyama path from P; returns its exit step (k+1) or -1.
 * ------------------------------------------------------------------------- */
typedef struct {
    int kind, time_mode;
    const double *par;
    or_dens dens;
    or_data data;
    double t_init, t, dt;
    int64_t K;
    uint32_t key[2];
    uint32_t ctr3;
} or_problem;

/* ---------------------------------------------------------------------------
 * Brownian-bridge exit test (score mode 3).  Between two inside points X_k
 * and X_{k+1} of a step of length D, the diffusion sqrt(2) dW, pinned at both
 * ends, crosses a straight side at distances d0 and d1 with probability
 * exp(-2 d0 d1 / (2 D)) = exp(-d0 d1 / D); the four sides of the square are
 * taken as independent, p = 1 - prod (1 - p_side).  Reading: a side's
 * probability is taken as 0 where d0 d1 / D > 17 (below the resolution
 * 2^-24 of the uniforms); the uniform of step k is word (k & 1) of
 * Philox(k/2, path, node, ctr3 | 4), u = ((r >> 8) + 1) 2^-24 in (0, 1]; the
 * path exits within the step if u < p, at the end point projected onto the
 * side with the largest crossing probability.  Returns 1 on an exit and
 * moves (x, y) there.
 * ------------------------------------------------------------------------- */
static int bridge_exit(const or_problem *pb, int64_t k, uint32_t path, uint32_t node, double D,
                       double x0, double y0, double *x, double *y)
{
    const double d0[4] = {x0, 1.0 - x0, y0, 1.0 - y0};
    const double d1[4] = {*x, 1.0 - *x, *y, 1.0 - *y};
    double surv = 1.0, pmax = 0.0;
    int side = -1;
    for (int i = 0; i < 4; ++i) {
        const double e = d0[i] * d1[i] / D;
        if (!(e <= 17.0)) continue;   /* also a zero-length step on a side: 0/0 */
        const double ps = exp(-e);
        surv *= 1.0 - ps;
        if (ps > pmax) { pmax = ps; side = i; }
    }
    if (side < 0) return 0;
    uint32_t ctr[4] = {(uint32_t)(k >> 1), path, node, pb->ctr3 | 4u}, r[4];
    or_philox4x32_10(ctr, pb->key, r);
    const double u = ((double)(r[k & 1] >> 8) + 1.0) * 0x1p-24;
    if (!(u < 1.0 - surv)) return 0;
    if (side == 0) *x = 0.0;
    else if (side == 1) *x = 1.0;
    else if (side == 2) *y = 0.0;
    else *y = 1.0;
    return 1;
}

static int64_t run_path(const or_problem *pb, double px, double py, uint32_t path, uint32_t node,
                        double *score_xi, double *score_eta)
{
    double x = px, y = py, s = 0.0;
    uint32_t r[4] = {0, 0, 0, 0};
    for (int64_t k = 0; k < pb->K; ++k) {
        if ((k & 1) == 0) {
            uint32_t ctr[4] = {(uint32_t)(k >> 1), path, node, pb->ctr3};
            or_philox4x32_10(ctr, pb->key, r);
        }
        double z0, z1;
        if ((k & 1) == 0) box_muller(r[0], r[1], &z0, &z1);
        else box_muller(r[2], r[3], &z0, &z1);
        double D = (k == pb->K - 1) ? pb->t - (double)(pb->K - 1) * pb->dt : pb->dt;
        double tau = (pb->time_mode == 0) ? pb->t_init + pb->t - s : pb->par[6];
        double bx, by;
        drift(&pb->dens, tau, x, y, &bx, &by);
        double sd = sqrt(2.0 * D);
        const double x0 = x, y0 = y;
        x = x + bx * D + sd * z0;
        y = y + by * D + sd * z1;
        s = s + D;
        if (x < 0.0 || x > 1.0 || y < 0.0 || y > 1.0 ||
            (pb->data.score_mode == 3 && bridge_exit(pb, k, path, node, D, x0, y0, &x, &y))) {
            boundary_value(&pb->data, pb->t - s, x, y, score_xi, score_eta);
            return k + 1;
        }
    }
    initial_value(&pb->data, x, y, score_xi, score_eta);
    return -1;
}

/* ---------------------------------------------------------------------------
 * Exponential time-stepping (score mode 4).  Reading of the method of
 * Jansons & Lythe (2003) for this problem: the steps have independent
 * exponentially distributed lengths D_k with mean dt, and the step that
 * would pass the horizon t is cut at it (so a path that never exits takes
 * 1 + Poisson(t / dt) steps).  Given D_k, the step is the Euler-Maruyama
 * step of that length with the drift frozen at its start, and the exit test
 * within the step is the Brownian-bridge test of mode 3 for a step of
 * length D_k.  For Brownian motion with constant drift this gives the end
 * point and the crossing event of a step over an exponential time exactly
 * (the Gaussian-bridge test given D_k averages to the exponential law of
 * the running maximum given the end point); it leaves the drift's variation
 * within a step as the only time-step error.  Exits are scored at the end
 * point projected onto the square.  Random numbers of step k: the normals
 * of the fixed-step scheme (stream word 3 = ctr3), and from
 * Philox(k/2, path, node, ctr3 | 4) word (k & 1) the bridge uniform (as in
 * mode 3) and word 2 + (k & 1), u = ((r >> 8) + 1) 2^-24 in (0, 1], the
 * step length D_k = -dt ln u.  *steps receives the number of steps taken.
 * ------------------------------------------------------------------------- */
static int64_t run_path_expo(const or_problem *pb, double px, double py, uint32_t path, uint32_t node,
                             double *score_xi, double *score_eta, int64_t *steps)
{
    double x = px, y = py, s = 0.0;
    *steps = 0;
    if (!(pb->t > 0.0)) {
        initial_value(&pb->data, x, y, score_xi, score_eta);
        return -1;
    }
    for (int64_t k = 0;; ++k) {
        uint32_t ctr[4] = {(uint32_t)(k >> 1), path, node, pb->ctr3}, r[4];
        or_philox4x32_10(ctr, pb->key, r);
        uint32_t ctr_u[4] = {(uint32_t)(k >> 1), path, node, pb->ctr3 | 4u}, q[4];
        or_philox4x32_10(ctr_u, pb->key, q);
        double z0, z1;
        if ((k & 1) == 0) box_muller(r[0], r[1], &z0, &z1);
        else box_muller(r[2], r[3], &z0, &z1);
        const double u = ((double)(q[2 + (k & 1)] >> 8) + 1.0) * 0x1p-24;
        double D = -pb->dt * log(u);
        const int last = s + D >= pb->t;
        if (last) D = pb->t - s;
        const double tau = (pb->time_mode == 0) ? pb->t_init + pb->t - s : pb->par[6];
        double bx, by;
        drift(&pb->dens, tau, x, y, &bx, &by);
        const double sd = sqrt(2.0 * D);
        const double x0 = x, y0 = y;
        x = x + bx * D + sd * z0;
        y = y + by * D + sd * z1;
        s = last ? pb->t : s + D;
        *steps = k + 1;
        if (x < 0.0 || x > 1.0 || y < 0.0 || y > 1.0 || bridge_exit(pb, k, path, node, D, x0, y0, &x, &y)) {
            boundary_value(&pb->data, pb->t - s, x, y, score_xi, score_eta);
            return k + 1;
        }
        if (last) break;
    }
    initial_value(&pb->data, x, y, score_xi, score_eta);
    return -1;
}

/* One path of the problem's scheme; *steps receives the steps it took. */
static int64_t run_path_any(const or_problem *pb, double px, double py, uint32_t path, uint32_t node,
                            double *score_xi, double *score_eta, int64_t *steps)
{
    if (pb->data.score_mode == 4) return run_path_expo(pb, px, py, path, node, score_xi, score_eta, steps);
    const int64_t e = run_path(pb, px, py, path, node, score_xi, score_eta);
    *steps = e < 0 ? pb->K : e;
    return e;
}

static int64_t n_steps(double t, double dt)
{
    if (t <= 0.0) return 0;
    return (int64_t)ceil(t / dt - 1e-9);
}

int64_t or_n_steps(double t, double dt) { return n_steps(t, dt); }

/*
 * Plain Monte-Carlo solve at n_nodes points.
 *   pts        [n_nodes][2]           node coordinates
 *   node_ids   [n_nodes] or NULL      counter word 2 (NULL: the index)
 *   mean, se   [n_nodes][2]           (xi, eta) estimate and standard error
 *   exit_step  [n_nodes][n_paths] or NULL
 *   scores     [n_nodes][n_paths][2] or NULL
 *   steps      [n_nodes] or NULL      Euler-Maruyama steps taken in total
 * Returns 0, or -1 on bad arguments.
 */
int or_fk_solve(int kind, int time_mode, const double *par, const double *w_grid, int w_n,
                int init_kind, int bdry_kind, int score_mode, double t_init,
                const double *grid_xi, const double *grid_eta, int grid_n,
                const double *pts, const int64_t *node_ids, int64_t n_nodes,
                double t, double dt, int64_t n_paths, uint64_t seed, uint32_t level_id,
                uint32_t stream, int n_threads,
                double *mean, double *se, int32_t *exit_step, double *scores, int64_t *steps)
{
    if (n_nodes < 0 || n_paths < 2 || !(dt > 0.0) || !(t >= 0.0)) return -1;
    or_problem pb;
    pb.kind = kind;
    pb.time_mode = time_mode;
    pb.par = par;
    if (dens_bind(&pb.dens, kind, par, w_grid, w_n) != 0) return -1;
    pb.data.init_kind = init_kind;
    pb.data.bdry_kind = bdry_kind;
    pb.data.score_mode = score_mode;
    if (score_mode < 0 || score_mode > 4 || (score_mode == 2 && (init_kind != D_GRID || !grid_xi || !grid_eta)) ||
        (bdry_kind == D_GRID && (init_kind != D_GRID || (score_mode != 1 && score_mode != 3 && score_mode != 4))))
        return -1;
    pb.data.grid_xi = grid_xi;
    pb.data.grid_eta = grid_eta;
    pb.data.grid_n = grid_n;
    pb.t_init = t_init;
    pb.t = t;
    pb.dt = dt;
    pb.K = n_steps(t, dt);
    pb.key[0] = (uint32_t)seed;
    pb.key[1] = (uint32_t)(seed >> 32);
    pb.ctr3 = (level_id << 4) | (stream & 15u);

    double *sc = scores;
    if (!sc) {
        sc = (double *)malloc(sizeof(double) * 2 * (size_t)(n_nodes * n_paths));
        if (!sc) return -1;
    }
    int64_t *st = (int64_t *)calloc((size_t)(n_nodes * n_paths > 0 ? n_nodes * n_paths : 1), sizeof(int64_t));
    const int64_t total = n_nodes * n_paths;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t g = 0; g < total; ++g) {
        int64_t i = g / n_paths, p = g % n_paths;
        uint32_t nid = (uint32_t)(node_ids ? node_ids[i] : i);
        double a, b;
        int64_t ns;
        int64_t e = run_path_any(&pb, pts[2 * i], pts[2 * i + 1], (uint32_t)p, nid, &a, &b, &ns);
        sc[2 * g] = a;
        sc[2 * g + 1] = b;
        st[g] = ns;
        if (exit_step) exit_step[g] = (int32_t)e;
    }
    /* Two-pass sample mean and variance per node and component. */
    for (int64_t i = 0; i < n_nodes; ++i) {
        for (int c = 0; c < 2; ++c) {
            double sum = 0.0;
            for (int64_t p = 0; p < n_paths; ++p) sum += sc[2 * (i * n_paths + p) + c];
            double m = sum / (double)n_paths;
            double ss = 0.0;
            for (int64_t p = 0; p < n_paths; ++p) {
                double d = sc[2 * (i * n_paths + p) + c] - m;
                ss += d * d;
            }
            double var = ss / (double)(n_paths - 1);
            mean[2 * i + c] = m;
            se[2 * i + c] = sqrt(var / (double)n_paths);
        }
        if (steps) {
            int64_t tot = 0;
            for (int64_t p = 0; p < n_paths; ++p) tot += st[i * n_paths + p];
            steps[i] = tot;
        }
    }
    free(st);
    if (!scores) free(sc);
    return 0;
}

/*
 * Individual paths, for sampled checks at sizes where a full oracle solve is
 * out of reach: path path_ids[j] of the node at pts[j] with counter word 2
 * node_ids[j].  Outputs the scores [m][2] and exit steps [m] (-1 = survived).
 */
int or_fk_paths(int kind, int time_mode, const double *par, const double *w_grid, int w_n,
                int init_kind, int bdry_kind, int score_mode, double t_init,
                const double *grid_xi, const double *grid_eta, int grid_n,
                const double *pts, const int64_t *node_ids, const int64_t *path_ids, int64_t m,
                double t, double dt, uint64_t seed, uint32_t level_id, uint32_t stream, int n_threads,
                double *scores, int32_t *exit_step)
{
    if (m < 0 || !(dt > 0.0) || !(t >= 0.0)) return -1;
    or_problem pb;
    pb.kind = kind;
    pb.time_mode = time_mode;
    pb.par = par;
    if (dens_bind(&pb.dens, kind, par, w_grid, w_n) != 0) return -1;
    pb.data.init_kind = init_kind;
    pb.data.bdry_kind = bdry_kind;
    pb.data.score_mode = score_mode;
    if (score_mode < 0 || score_mode > 4 || (score_mode == 2 && (init_kind != D_GRID || !grid_xi || !grid_eta)) ||
        (bdry_kind == D_GRID && (init_kind != D_GRID || (score_mode != 1 && score_mode != 3 && score_mode != 4))))
        return -1;
    pb.data.grid_xi = grid_xi;
    pb.data.grid_eta = grid_eta;
    pb.data.grid_n = grid_n;
    pb.t_init = t_init;
    pb.t = t;
    pb.dt = dt;
    pb.K = n_steps(t, dt);
    pb.key[0] = (uint32_t)seed;
    pb.key[1] = (uint32_t)(seed >> 32);
    pb.ctr3 = (level_id << 4) | (stream & 15u);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t j = 0; j < m; ++j) {
        double a, b;
        int64_t ns;
        int64_t e = run_path_any(&pb, pts[2 * j], pts[2 * j + 1], (uint32_t)path_ids[j], (uint32_t)node_ids[j], &a, &b,
                                 &ns);
        scores[2 * j] = a;
        scores[2 * j + 1] = b;
        exit_step[j] = (int32_t)e;
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Control-variate (Dynkin-form) estimator.  For a smooth function
 * u_hat(tau, X) of PDE time and position, V(s, X) = u_hat(t_init + t - s, X)
 * satisfies, along the diffusion, E[V(end)] = V(0, P) + E[integral of
 * (L u_hat - d_tau u_hat) ds], L = Laplacian + b . grad.  So
 *
 *   u(P) = u_hat(t_init + t, P) + E[ score - u_hat(tau_end, X_end)
 *                                    + sum_j r(tau_j, X_j) (s_{j+1} - s_j) ],
 *
 * with r = Laplacian u_hat + b . grad u_hat - d_tau u_hat evaluated at the
 * pre-step state of every stride-th Euler-Maruyama step and at the path's
 * end, the time integral taken by the trapezoidal rule between consecutive
 * evaluation points (the left-point rule biases the estimate by
 * O(stride dt); the trapezoidal rule by O((stride dt)^2)).  This is the
 * reading of the exact control-variate estimator this build uses; the same
 * paths also give the plain estimate.
 *
 * u_hat kinds: 0 the tanh MLP 3-64-64-64-2 (flat FP64 parameters, input
 * z = (2 tau / T - 1, 2x - 1, 2y - 1)); 1 the linear maps (x, y); 2 the
 * decaying sine mode exp(-2 pi^2 (tau - t_init)) sin(pi x) sin(pi y) for
 * both components; 3 zero; 4 the grid initial data (martingale form); 5 the
 * MLP plus the identity map (the network as the deviation from it).
 * ------------------------------------------------------------------------- */
typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
    double t_scale;
} or_mlp;

static void mlp_bind(or_mlp *m, const double *flat, double t_scale)
{
    m->W1 = flat;
    m->b1 = m->W1 + 64 * 3;
    m->W2 = m->b1 + 64;
    m->b2 = m->W2 + 64 * 64;
    m->W3 = m->b2 + 64;
    m->b3 = m->W3 + 64 * 64;
    m->W4 = m->b3 + 64;
    m->b4 = m->W4 + 2 * 64;
    m->t_scale = t_scale;
}

/* out[c][0..4] = value, d/dx, d/dy, d/dtau, Laplacian of output c. */
static void mlp_forward_mode(const or_mlp *m, double tau, double x, double y, double out[2][5])
{
    double z0 = 2.0 * tau / m->t_scale - 1.0, z1 = 2.0 * x - 1.0, z2 = 2.0 * y - 1.0;
    /* channels: 0 value, 1 d/dx, 2 d/dy, 3 d/dtau, 4 Laplacian */
    double h[5][64], a[5][64];
    for (int j = 0; j < 64; ++j) {
        const double *w = m->W1 + 3 * j;
        a[0][j] = w[0] * z0 + w[1] * z1 + w[2] * z2 + m->b1[j];
        a[1][j] = 2.0 * w[1];
        a[2][j] = 2.0 * w[2];
        a[3][j] = 2.0 / m->t_scale * w[0];
        a[4][j] = 0.0;
    }
    const double *Ws[2] = {m->W2, m->W3}, *bs[2] = {m->b2, m->b3};
    for (int layer = 0; layer < 3; ++layer) {
        if (layer > 0) {
            const double *W = Ws[layer - 1], *b = bs[layer - 1];
            for (int j = 0; j < 64; ++j) {
                double acc[5] = {b[j], 0.0, 0.0, 0.0, 0.0};
                for (int k = 0; k < 64; ++k)
                    for (int c = 0; c < 5; ++c) acc[c] += W[64 * j + k] * h[c][k];
                for (int c = 0; c < 5; ++c) a[c][j] = acc[c];
            }
        }
        for (int j = 0; j < 64; ++j) {
            double v = tanh(a[0][j]), s = 1.0 - v * v;
            h[0][j] = v;
            h[1][j] = s * a[1][j];
            h[2][j] = s * a[2][j];
            h[3][j] = s * a[3][j];
            h[4][j] = -2.0 * v * s * (a[1][j] * a[1][j] + a[2][j] * a[2][j]) + s * a[4][j];
        }
    }
    for (int o = 0; o < 2; ++o)
        for (int c = 0; c < 5; ++c) {
            double acc = (c == 0) ? m->b4[o] : 0.0;
            for (int k = 0; k < 64; ++k) acc += m->W4[64 * o + k] * h[c][k];
            out[o][c] = acc;
        }
}

int or_mlp_eval(const double *flat, double t_scale, const double *txy, int64_t n, double *out)
{
    or_mlp m;
    mlp_bind(&m, flat, t_scale);
    for (int64_t i = 0; i < n; ++i) {
        double o[2][5];
        mlp_forward_mode(&m, txy[3 * i], txy[3 * i + 1], txy[3 * i + 2], o);
        for (int c = 0; c < 2; ++c)
            for (int k = 0; k < 5; ++k) out[10 * i + 5 * c + k] = o[c][k];
    }
    return 0;
}

typedef struct {
    int kind;
    or_mlp mlp;
    double t_init;
    const double *grid_xi, *grid_eta;   /* kind 4: the grid initial data */
    int grid_n;
} or_uhat;

/* Partial derivatives of the bilinear interpolant of a nodal grid at (x, y),
   in the cell bilinear() uses. */
static void bilinear_grad(const double *g, int n, double x, double y, double *gx, double *gy)
{
    double fx = x * n, fy = y * n;
    int i = (int)floor(fx), j = (int)floor(fy);
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    if (j < 0) j = 0;
    if (j > n - 1) j = n - 1;
    double ax = fx - i, ay = fy - j;
    const double *r0 = g + (int64_t)j * (n + 1), *r1 = r0 + (n + 1);
    *gx = n * ((1 - ay) * (r0[i + 1] - r0[i]) + ay * (r1[i + 1] - r1[i]));
    *gy = n * ((1 - ax) * (r1[i] - r0[i]) + ax * (r1[i + 1] - r0[i + 1]));
}

static void uhat_eval(const or_uhat *u, double tau, double x, double y, double out[2][5])
{
    if (u->kind == 7) {
        /* the network as the deviation from the grid initial data (the mesh
           at the step's start): u_hat = bilinear(grid) + MLP; the martingale
           form uses only the gradient */
        const double *g[2] = {u->grid_xi, u->grid_eta};
        mlp_forward_mode(&u->mlp, tau, x, y, out);
        for (int c = 0; c < 2; ++c) {
            double gx, gy;
            bilinear_grad(g[c], u->grid_n, x, y, &gx, &gy);
            out[c][0] += bilinear(g[c], u->grid_n, x, y);
            out[c][1] += gx;
            out[c][2] += gy;
        }
        return;
    }
    if (u->kind == 4) {
        /* the grid initial data, bilinear: value and gradient (the martingale
           form uses only the gradient) */
        const double *g[2] = {u->grid_xi, u->grid_eta};
        for (int c = 0; c < 2; ++c) {
            out[c][0] = bilinear(g[c], u->grid_n, x, y);
            bilinear_grad(g[c], u->grid_n, x, y, &out[c][1], &out[c][2]);
            out[c][3] = 0.0;
            out[c][4] = 0.0;
        }
        return;
    }
    switch (u->kind) {
    case 0: mlp_forward_mode(&u->mlp, tau, x, y, out); return;
    case 5:
        /* the network fits the deviation from the identity map:
           u_hat = (x, y) + MLP */
        mlp_forward_mode(&u->mlp, tau, x, y, out);
        out[0][0] += x;
        out[1][0] += y;
        out[0][1] += 1.0;
        out[1][2] += 1.0;
        return;
    case 1:
        out[0][0] = x; out[0][1] = 1.0; out[0][2] = 0.0; out[0][3] = 0.0; out[0][4] = 0.0;
        out[1][0] = y; out[1][1] = 0.0; out[1][2] = 1.0; out[1][3] = 0.0; out[1][4] = 0.0;
        return;
    case 6:
        /* test function u_hat = (tau x^2, tau y^2): under w = 1 the Dynkin
           integrand 2 tau - x^2 has a mean linear in the path time, which the
           trapezoidal rule integrates exactly and the left-point rule not */
        out[0][0] = tau * x * x; out[0][1] = 2.0 * tau * x; out[0][2] = 0.0; out[0][3] = x * x; out[0][4] = 2.0 * tau;
        out[1][0] = tau * y * y; out[1][1] = 0.0; out[1][2] = 2.0 * tau * y; out[1][3] = y * y; out[1][4] = 2.0 * tau;
        return;
    case 2: {
        double e = exp(-2.0 * OR_PI * OR_PI * (tau - u->t_init));
        double sx = sin(OR_PI * x), sy = sin(OR_PI * y), cx = cos(OR_PI * x), cy = cos(OR_PI * y);
        for (int c = 0; c < 2; ++c) {
            out[c][0] = e * sx * sy;
            out[c][1] = e * OR_PI * cx * sy;
            out[c][2] = e * OR_PI * sx * cy;
            out[c][3] = -2.0 * OR_PI * OR_PI * e * sx * sy;
            out[c][4] = -2.0 * OR_PI * OR_PI * e * sx * sy;
        }
        return;
    }
    default:
        for (int c = 0; c < 2; ++c)
            for (int k = 0; k < 5; ++k) out[c][k] = 0.0;
        return;
    }
}

/* One path with the control variate; returns the exit step (-1 survived). */
static int64_t run_path_cv(const or_problem *pb, const or_uhat *u, int stride, double px, double py,
                           uint32_t path, uint32_t node, double plain[2], double cv[2])
{
    double x = px, y = py, s = 0.0;
    uint32_t r[4] = {0, 0, 0, 0};
    double integ[2] = {0.0, 0.0}, rlast[2] = {0.0, 0.0}, s_last = 0.0;
    int64_t exit_k = -1;
    for (int64_t k = 0; k < pb->K; ++k) {
        if ((k & 1) == 0) {
            uint32_t ctr[4] = {(uint32_t)(k >> 1), path, node, pb->ctr3};
            or_philox4x32_10(ctr, pb->key, r);
        }
        double z0, z1;
        if ((k & 1) == 0) box_muller(r[0], r[1], &z0, &z1);
        else box_muller(r[2], r[3], &z0, &z1);
        double D = (k == pb->K - 1) ? pb->t - (double)(pb->K - 1) * pb->dt : pb->dt;
        double tau = (pb->time_mode == 0) ? pb->t_init + pb->t - s : pb->par[6];
        double bx, by;
        drift(&pb->dens, tau, x, y, &bx, &by);
        if (k % stride == 0) {
            /* close the previous interval (trapezoidal rule), open a new one */
            double e[2][5];
            uhat_eval(u, pb->t_init + pb->t - s, x, y, e);
            for (int c = 0; c < 2; ++c) {
                double rn = e[c][4] + bx * e[c][1] + by * e[c][2] - e[c][3];
                integ[c] += 0.5 * (rlast[c] + rn) * (s - s_last);
                rlast[c] = rn;
            }
            s_last = s;
        }
        double sd = sqrt(2.0 * D);
        x = x + bx * D + sd * z0;
        y = y + by * D + sd * z1;
        s = s + D;
        if (x < 0.0 || x > 1.0 || y < 0.0 || y > 1.0) {
            boundary_value(&pb->data, pb->t - s, x, y, &plain[0], &plain[1]);
            exit_k = k + 1;
            break;
        }
    }
    if (exit_k < 0) initial_value(&pb->data, x, y, &plain[0], &plain[1]);
    /* end point: u_hat there, and the integrand closing the last interval */
    double e[2][5];
    const double tau_end = pb->t_init + pb->t - s;
    uhat_eval(u, tau_end, x, y, e);
    double bx, by;
    drift(&pb->dens, (pb->time_mode == 0) ? tau_end : pb->par[6], x, y, &bx, &by);
    for (int c = 0; c < 2; ++c) {
        double rn = e[c][4] + bx * e[c][1] + by * e[c][2] - e[c][3];
        integ[c] += 0.5 * (rlast[c] + rn) * (s - s_last);
    }
    cv[0] = plain[0] - e[0][0] + integ[0];
    cv[1] = plain[1] - e[1][0] + integ[1];
    return exit_k;
}

/*
 * One path with the control variate in martingale form (Ito's formula
 * applied to u_hat along the path): the score is g - sum_j G_j . dB_j, where
 * dB_j is the Brownian part (the sum of the sqrt(2 D_k) z_k) of the path's
 * steps in block j and G_j = grad u_hat at the block's first state, blocks
 * starting every `stride` steps from the path's start and the last one
 * closed at the path's end.  Each G_j is fixed before the increments it
 * multiplies, so the sum has mean zero for the discrete chain itself.  With
 * the grid base (u_hat kind 7) blocks start every 2 steps, with G_j the
 * mesh's gradient there plus the network's gradient taken every `stride`
 * steps (stride even) and held.
 */
static int64_t run_path_mg(const or_problem *pb, const or_uhat *u, int stride, double px, double py,
                           uint32_t path, uint32_t node, double plain[2], double cv[2])
{
    double x = px, y = py, s = 0.0;
    uint32_t r[4] = {0, 0, 0, 0};
    double G[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, dB[2] = {0.0, 0.0}, M[2] = {0.0, 0.0};
    double Gn[2][2] = {{0.0, 0.0}, {0.0, 0.0}};   /* grid base: the network's part of G */
    int64_t exit_k = -1;
    for (int64_t k = 0; k < pb->K; ++k) {
        if ((k & 1) == 0) {
            uint32_t ctr[4] = {(uint32_t)(k >> 1), path, node, pb->ctr3};
            or_philox4x32_10(ctr, pb->key, r);
        }
        double z0, z1;
        if ((k & 1) == 0) box_muller(r[0], r[1], &z0, &z1);
        else box_muller(r[2], r[3], &z0, &z1);
        double D = (k == pb->K - 1) ? pb->t - (double)(pb->K - 1) * pb->dt : pb->dt;
        double tau = (pb->time_mode == 0) ? pb->t_init + pb->t - s : pb->par[6];
        double bx, by;
        drift(&pb->dens, tau, x, y, &bx, &by);
        if (u->kind == 7) {
            /* grid base: blocks every 2 steps with the mesh's gradient there,
               plus the network's gradient taken every `stride` steps and held */
            if (k % 2 == 0) {
                for (int c = 0; c < 2; ++c) M[c] += G[c][0] * dB[0] + G[c][1] * dB[1];
                dB[0] = dB[1] = 0.0;
                if (k % stride == 0) {
                    double e[2][5];
                    mlp_forward_mode(&u->mlp, pb->t_init + pb->t - s, x, y, e);
                    for (int c = 0; c < 2; ++c) {
                        Gn[c][0] = e[c][1];
                        Gn[c][1] = e[c][2];
                    }
                }
                const double *g[2] = {u->grid_xi, u->grid_eta};
                for (int c = 0; c < 2; ++c) {
                    bilinear_grad(g[c], u->grid_n, x, y, &G[c][0], &G[c][1]);
                    G[c][0] += Gn[c][0];
                    G[c][1] += Gn[c][1];
                }
            }
        } else if (k % stride == 0) {
            double e[2][5];
            for (int c = 0; c < 2; ++c) M[c] += G[c][0] * dB[0] + G[c][1] * dB[1];
            dB[0] = dB[1] = 0.0;
            uhat_eval(u, pb->t_init + pb->t - s, x, y, e);
            for (int c = 0; c < 2; ++c) {
                G[c][0] = e[c][1];
                G[c][1] = e[c][2];
            }
        }
        double sd = sqrt(2.0 * D);
        double w0 = sd * z0, w1 = sd * z1;
        const double x0 = x, y0 = y;
        x = x + bx * D + w0;
        y = y + by * D + w1;
        s = s + D;
        dB[0] += w0;
        dB[1] += w1;
        /* score mode 3: the bridge test of the step too (the last block then
           ends with this step; the stopping rule sees only this step's
           increments and its own uniform, so the sum keeps mean zero) */
        if (x < 0.0 || x > 1.0 || y < 0.0 || y > 1.0 ||
            (pb->data.score_mode == 3 && bridge_exit(pb, k, path, node, D, x0, y0, &x, &y))) {
            boundary_value(&pb->data, pb->t - s, x, y, &plain[0], &plain[1]);
            exit_k = k + 1;
            break;
        }
    }
    if (exit_k < 0) initial_value(&pb->data, x, y, &plain[0], &plain[1]);
    for (int c = 0; c < 2; ++c) {
        M[c] += G[c][0] * dB[0] + G[c][1] * dB[1];
        cv[c] = plain[c] - M[c];
    }
    return exit_k;
}

static void two_pass(const double *sc, int64_t i, int64_t n_paths, double *mean, double *se)
{
    for (int c = 0; c < 2; ++c) {
        double sum = 0.0;
        for (int64_t p = 0; p < n_paths; ++p) sum += sc[2 * (i * n_paths + p) + c];
        double m = sum / (double)n_paths, ss = 0.0;
        for (int64_t p = 0; p < n_paths; ++p) {
            double d = sc[2 * (i * n_paths + p) + c] - m;
            ss += d * d;
        }
        mean[2 * i + c] = m;
        se[2 * i + c] = sqrt(ss / (double)(n_paths - 1) / (double)n_paths);
    }
}

/*
 * Control-variate solve.  form 0 (Dynkin): mean/se are the CV estimate
 * u_hat(t_init + t, P) + mean(cv score) and its standard error; form 1
 * (martingale): mean(cv score).  plain_mean/plain_se: the plain estimate from
 * the same paths.  cv_scores [n][N][2] and exit_step [n][N] optional.
 */
int or_fk_solve_cv(int kind, int time_mode, const double *par, const double *w_grid, int w_n,
                   int init_kind, int bdry_kind, int score_mode, double t_init,
                   const double *grid_xi, const double *grid_eta, int grid_n,
                   const double *pts, const int64_t *node_ids, int64_t n_nodes,
                   double t, double dt, int64_t n_paths, uint64_t seed, uint32_t level_id,
                   uint32_t stream, int n_threads,
                   int uhat_kind, const double *flat, double t_scale, int stride, int form,
                   double *mean, double *se, double *plain_mean, double *plain_se,
                   double *cv_scores, int32_t *exit_step)
{
    if (n_nodes < 0 || n_paths < 2 || !(dt > 0.0) || !(t >= 0.0) || stride < 1) return -1;
    if (form != 0 && form != 1) return -1;
    if ((uhat_kind == 0 || uhat_kind == 5 || uhat_kind == 7) && !flat) return -1;
    or_problem pb;
    pb.kind = kind;
    pb.time_mode = time_mode;
    pb.par = par;
    if (dens_bind(&pb.dens, kind, par, w_grid, w_n) != 0) return -1;
    pb.data.init_kind = init_kind;
    pb.data.bdry_kind = bdry_kind;
    pb.data.score_mode = score_mode;
    /* the bridge test (mode 3) in the martingale form only */
    if (score_mode < 0 || score_mode > 3 || (score_mode == 3 && form != 1) ||
        (score_mode == 2 && (init_kind != D_GRID || !grid_xi || !grid_eta)))
        return -1;
    pb.data.grid_xi = grid_xi;
    pb.data.grid_eta = grid_eta;
    pb.data.grid_n = grid_n;
    pb.t_init = t_init;
    pb.t = t;
    pb.dt = dt;
    pb.K = n_steps(t, dt);
    pb.key[0] = (uint32_t)seed;
    pb.key[1] = (uint32_t)(seed >> 32);
    pb.ctr3 = (level_id << 4) | (stream & 15u);
    or_uhat u;
    u.kind = uhat_kind;
    u.t_init = t_init;
    u.grid_xi = grid_xi;
    u.grid_eta = grid_eta;
    u.grid_n = grid_n;
    if (uhat_kind == 0 || uhat_kind == 5 || uhat_kind == 7) mlp_bind(&u.mlp, flat, t_scale);
    /* the grid's bilinear interpolant has no Laplacian: martingale form only */
    if ((uhat_kind == 4 || uhat_kind == 7) && (form != 1 || init_kind != D_GRID || !grid_xi || !grid_eta))
        return -1;
    const int64_t total = n_nodes * n_paths;
    double *pl = (double *)malloc(sizeof(double) * 2 * (size_t)(total > 0 ? total : 1));
    double *cs = cv_scores ? cv_scores : (double *)malloc(sizeof(double) * 2 * (size_t)(total > 0 ? total : 1));
    if (!pl || !cs) { free(pl); if (!cv_scores) free(cs); return -1; }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t g = 0; g < total; ++g) {
        int64_t i = g / n_paths, p = g % n_paths;
        uint32_t nid = (uint32_t)(node_ids ? node_ids[i] : i);
        int64_t e = form == 0
                        ? run_path_cv(&pb, &u, stride, pts[2 * i], pts[2 * i + 1], (uint32_t)p, nid, &pl[2 * g], &cs[2 * g])
                        : run_path_mg(&pb, &u, stride, pts[2 * i], pts[2 * i + 1], (uint32_t)p, nid, &pl[2 * g], &cs[2 * g]);
        if (exit_step) exit_step[g] = (int32_t)e;
    }
    for (int64_t i = 0; i < n_nodes; ++i) {
        two_pass(pl, i, n_paths, plain_mean, plain_se);
        two_pass(cs, i, n_paths, mean, se);
        if (form == 1) continue;
        double e[2][5];
        uhat_eval(&u, t_init + t, pts[2 * i], pts[2 * i + 1], e);
        mean[2 * i] += e[0][0];
        mean[2 * i + 1] += e[1][0];
    }
    free(pl);
    if (!cv_scores) free(cs);
    return 0;
}
