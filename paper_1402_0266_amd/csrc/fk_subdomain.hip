// fk_subdomain.hip -- deterministic sub-domain solves (Sect. 4): with the
// interface values from the stochastic solver as Dirichlet data, each
// sub-domain takes one backward-Euler step of the relaxed Winslow system
// (Sect. 2, eq. (3)) discretised by central differences,
//
//   (1 + 4c) u_P - (c + cx) u_E - (c - cx) u_W - (c + cy) u_N - (c - cy) u_S = u^n_P,
//   c = D/h^2,  cx = D b_x / (2h),  cy = D b_y / (2h),  b = -grad w / w (eq. (6)),
//
// and the system is solved by LU factorisation without pivoting (strictly
// diagonally dominant while |b| h / 2 < 1).  Plus the mesh-quality reduction.
//
// MI355X mapping: the unit square's N x N grid is split into px x py
// sub-domains of mx x my cells.  A sub-domain's interior unknowns are
// numbered along the shorter side first (the fast index), so its matrix is
// banded with half-bandwidth q = the number of unknowns on that side, and
// the fill of the LU stays in the band.  Large sub-domains are eliminated
// from both ends at once (twisted: two workgroups meet at a separator line,
// whose dense system one workgroup then solves).  The elimination window
// lives in registers: one wavefront, a column per lane, for q < 32
// (subdomain_lu_wave_kernel); otherwise 256 lanes as a 16 x 16 grid of
// register tiles (subdomain_lu_tile_kernel).  Finished U rows go to the
// workspace, and one wavefront per end back-substitutes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "fk.h"
#include "fk_internal.hpp"

namespace fk {

struct SubArgs {
    const double *xi_n, *eta_n;  // previous mesh, (N+1)^2
    double *xi_out, *eta_out;    // Dirichlet data pre-filled; interior written
    double *ubuf;                // per sub-domain: n rows of ustride doubles (U row k: entries k .. k+q)
    int ustride;                 // U row stride: q + 1 (one-wavefront kernels), or the tile kernel's window
    double *ybuf;                // per sub-domain: 2 n doubles
    double *cbuf;                // per sub-domain: 4 n doubles, (E, W, N, S) coefficients of each row
    double *rbuf;                // per sub-domain: 2 n doubles, right-hand sides (xi, eta) of each row
    int N;                       // grid cells a side
    int px, py, mx, my;          // px x py sub-domains of mx x my cells
    int qf, qs;                  // interior unknowns along the fast / slow index of the ordering
    int xfast;                   // 1: x is the fast index (row-major), 0: y is
    double c, half_d_over_h;     // D/h^2 and D/(2h); steady: 1/h^2 and 1/(2h)
    double diag0;                // 1 (backward Euler), 0 (steady: the rows divided by D, D -> inf)
    int steady;                  // no previous values in the right-hand side
    int kind;
    double amp, width2, cx, cy, orbit_r, omega, t_w;
    const double *wg;            // FK_DENSITY_GRID: samples of w on this grid, (N+1)^2
    int twisted;                 // two workgroups per sub-domain, eliminating from both ends
    int sep;                     // twisted: the separator's first row (its grid row times q)
    double *sbuf;                // twisted, per sub-domain: both ends' separator blocks and rhs, then x_S
};

// Twisted elimination (two workgroups per sub-domain): the top workgroup
// eliminates rows 0 .. sep-1 in the natural order, the bottom one rows
// n-1 .. sep+q in reverse (the same kernel on the reversed system, in which
// east/west and north/south swap).  Both stop at the separator, the grid row
// of rows sep .. sep+q-1, which no other row couples across, and write its
// block of their trailing window: A_SS minus their side's contribution.
// The separator system is then A_SS - (top part) - (bottom part) = S_top +
// S_bot - A_SS (a dense q x q solve), and each side back-substitutes from it.
__host__ __device__ inline size_t sep_stride(int q) { return (size_t)2 * ((size_t)q * q + 2 * q) + 2 * q; }

// Lower-left grid node (i0, j0) of sub-domain sd (row-major over the layout).
__device__ __forceinline__ void sub_origin(const SubArgs &a, int sd, int &i0, int &j0) {
    i0 = (sd % a.px) * a.mx;
    j0 = (sd / a.px) * a.my;
}

// Grid index of interior unknown r (natural order) of the sub-domain at (i0, j0).
__device__ __forceinline__ int64_t unknown_node(const SubArgs &a, int r, int i0, int j0) {
    const int f = r % a.qf, s = r / a.qf;
    const int gi = i0 + 1 + (a.xfast ? f : s), gj = j0 + 1 + (a.xfast ? s : f);
    return (int64_t)gj * (a.N + 1) + gi;
}

// ---------------------------------------------------------------------------
// Grid densities (Sect. 4: w known at the grid points only; the derivatives
// in grad w by finite differences).  h = 1/n; central differences at interior
// nodes, second-order one-sided differences on the edges.
// ---------------------------------------------------------------------------
// d/ds of the samples v[0], v[stride], ..., v[n stride] at index i.
__device__ double grid_fd(const double *v, int n, int i, int stride) {
    const double inv2h = 0.5 * n;
    if (i == 0) return (4.0 * v[stride] - 3.0 * v[0] - v[2 * stride]) * inv2h;
    if (i == n) return (3.0 * v[n * stride] - 4.0 * v[(n - 1) * stride] + v[(n - 2) * stride]) * inv2h;
    return (v[(i + 1) * stride] - v[(i - 1) * stride]) * inv2h;
}

// b = -grad w / w at node (i, j) of the n-cell grid of samples wg.
__device__ void grid_node_drift_f64(const double *wg, int n, int i, int j, double &bx, double &by) {
    const double *row = wg + (int64_t)j * (n + 1);
    const double inv_w = 1.0 / row[i];
    bx = -grid_fd(row, n, i, 1) * inv_w;
    by = -grid_fd(wg + i, n, j, n + 1) * inv_w;
}

// Nodal drift table of a grid density, FP32 pairs.
__global__ void grid_drift_kernel(const double *wg, int n, float2 *b) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n1 = n + 1;
    if (t >= n1 * n1) return;
    double bx, by;
    grid_node_drift_f64(wg, n, (int)(t % n1), (int)(t / n1), bx, by);
    b[t] = make_float2((float)bx, (float)by);
}

// -grad w / w in FP64 at (x, y), density frozen at t_w.
__device__ void drift_f64(const SubArgs &a, double x, double y, double &bx, double &by) {
    const double A = a.amp, s2 = a.width2;
    if (a.kind == FK_DENSITY_CONST) {
        bx = 0.0;
        by = 0.0;
        return;
    }
    double ccx = a.cx, ccy = a.cy, ox = 0.0, oy = 0.0;
    if (a.kind == FK_DENSITY_MOVING_BUMP || a.kind == FK_DENSITY_TWO_BUMPS || a.kind == FK_DENSITY_RING) {
        ox = a.orbit_r * cos(a.omega * a.t_w);
        oy = a.orbit_r * sin(a.omega * a.t_w);
    }
    if (a.kind == FK_DENSITY_RING) {
        // w = 1/rho, rho = 1 + A exp(beta |q|): b = grad rho / rho (beta = width2)
        const double dx = x - (ccx + ox), dy = y - (ccy + oy);
        const double q = dx * dx + dy * dy - 0.01;
        const double e = exp(s2 * fabs(q));
        const double sg = q > 0.0 ? 1.0 : (q < 0.0 ? -1.0 : 0.0);
        const double f = 2.0 * A * s2 * sg * e / (1.0 + A * e);
        bx = f * dx;
        by = f * dy;
        return;
    }
    if (a.kind == FK_DENSITY_TWO_BUMPS) {
        const double dy = y - (ccy + oy);
        const double d1 = x - (ccx + ox), d2 = x - (ccx - ox);
        const double e1 = exp(-(d1 * d1 + dy * dy) / s2), e2 = exp(-(d2 * d2 + dy * dy) / s2);
        const double f = 2.0 * A / s2 / (1.0 + A * (e1 + e2));
        bx = f * (e1 * d1 + e2 * d2);
        by = f * (e1 + e2) * dy;
        return;
    }
    const double dx = x - (ccx + ox);
    const double dy = (a.kind == FK_DENSITY_RIDGE) ? 0.0 : y - (ccy + oy);
    const double e = exp(-(dx * dx + dy * dy) / s2);
    const double f = 2.0 * A / s2 * e / (1.0 + A * e);
    bx = f * dx;
    by = f * dy;
}

// Drift at grid node (gi, gj) of the mesh: the finite-difference drift of a
// grid density, else the analytic drift at (gi/N, gj/N).
__device__ void node_drift_f64(const SubArgs &a, int gi, int gj, double &bx, double &by) {
    if (a.kind == FK_DENSITY_GRID) {
        grid_node_drift_f64(a.wg, a.N, gi, gj, bx, by);
        return;
    }
    drift_f64(a, (double)gi / a.N, (double)gj / a.N, bx, by);  // i/N exactly, as the grid is defined
}

constexpr int kMaxP1 = 128;  // window side limit: q <= 127 interior nodes per side

// The orbit offset of a moving centre at t_w (zero for static densities).
__device__ void orbit_f64(const SubArgs &a, double &ox, double &oy) {
    ox = oy = 0.0;
    if (a.kind == FK_DENSITY_MOVING_BUMP || a.kind == FK_DENSITY_TWO_BUMPS || a.kind == FK_DENSITY_RING) {
        ox = a.orbit_r * cos(a.omega * a.t_w);
        oy = a.orbit_r * sin(a.omega * a.t_w);
    }
}

// The density w in FP64 at (x, y), frozen at t_w, given the orbit offset.
__device__ double density_f64(const SubArgs &a, double ox, double oy, double x, double y) {
    const double A = a.amp, s2 = a.width2;
    if (a.kind == FK_DENSITY_CONST) return 1.0;
    if (a.kind == FK_DENSITY_RING) {
        const double dx = x - (a.cx + ox), dy = y - (a.cy + oy);
        return 1.0 / (1.0 + A * exp(s2 * fabs(dx * dx + dy * dy - 0.01)));
    }
    if (a.kind == FK_DENSITY_TWO_BUMPS) {
        const double dy = y - (a.cy + oy), d1 = x - (a.cx + ox), d2 = x - (a.cx - ox);
        return 1.0 + A * (exp(-(d1 * d1 + dy * dy) / s2) + exp(-(d2 * d2 + dy * dy) / s2));
    }
    const double dx = x - (a.cx + ox), dy = (a.kind == FK_DENSITY_RIDGE) ? 0.0 : y - (a.cy + oy);
    return 1.0 + A * exp(-(dx * dx + dy * dy) / s2);
}

// Integrals of w over the grid cells along the four edges (composite
// Simpson, 256 panels per cell): edge 0 y = 0, 1 y = 1 (over x), 2 x = 0,
// 3 x = 1 (over y).  cells[e * N + c] is the integral over cell c.  One
// wavefront per cell: each lane sums every 64th Simpson node, then a
// butterfly (fixed order) adds the lanes.  Launch: 4 N wavefronts.
__global__ void edge_cells_kernel(const SubArgs a, double *cells) {
    constexpr int M = 256;
    const int N = a.N;
    const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= 4 * N) return;                      // the whole wavefront
    const int e = t / N, c = t % N;
    const bool horizontal = e < 2;
    const double fixed = (e == 1 || e == 3) ? 1.0 : 0.0;
    if (a.kind == FK_DENSITY_GRID) {
        // samples along the edge; w is linear between them: trapezoid, exact
        const int64_t N1 = N + 1;
        const int64_t at = horizontal ? (e == 1 ? (int64_t)N * N1 : 0) + c : (int64_t)c * N1 + (e == 3 ? N : 0);
        const int64_t next = horizontal ? 1 : N1;
        if (lane == 0) cells[t] = 0.5 * (a.wg[at] + a.wg[at + next]) / N;
        return;
    }
    double ox, oy;
    orbit_f64(a, ox, oy);
    const double u0 = (double)c / N, hq = 1.0 / ((double)N * M);
    double acc = 0.0;
    for (int i = lane; i <= M; i += 64) {
        const double u = u0 + i * hq;
        const double w = horizontal ? density_f64(a, ox, oy, u, fixed) : density_f64(a, ox, oy, fixed, u);
        acc += w * ((i == 0 || i == M) ? 1.0 : ((i & 1) ? 4.0 : 2.0));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) cells[t] = acc * hq / 3.0;
}

// w(t_w, i/n, j/n) at the nodes of an n-cell grid.
__global__ void density_sample_kernel(const SubArgs a, int n, double *out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n1 = n + 1;
    if (t >= n1 * n1) return;
    double ox, oy;
    orbit_f64(a, ox, oy);
    out[t] = density_f64(a, ox, oy, (double)(t % n1) / n, (double)(t / n1) / n);
}

// int_0^{i/N} w / int_0^1 w along edge e, from the cell integrals (summed in
// a fixed order).
__device__ double edge_fraction(const double *cells, int N, int e, int i) {
    double part = 0.0, total = 0.0;
    for (int c = 0; c < N; ++c) {
        const double v = cells[e * N + c];
        if (c < i) part += v;
        total += v;
    }
    return part / total;
}

// Lane `l` of a wave-uniform index: its FP64 value, in scalar registers.
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// A DPP move of an FP64 value (both halves by the same lane pattern; a lane
// whose source is outside the pattern's range gets an unspecified value).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over lanes 0 .. 31, wave-uniform: within each row of 16 lanes by DPP
// (quad swaps 1 and 2, then the 8- and 16-lane mirrors), then the two rows.
__device__ __forceinline__ double sum32_f64(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    return readlane_f64(v, 0) + readlane_f64(v, 16);
}


// Back substitution by one wavefront, kD rows at a time: x_k = (y_k -
// sum_j U[k][k+j] x_{k+j}) / U[k][k] for k = n-1 .. 0.  Lane l holds
// x_{top+l+1} and x_{top+l+65} (the ring; zero beyond n).  For the block of
// rows k_j = top - j (j < kD) every lane forms its share of the sums over the
// columns already solved (beyond top) for all kD rows and both components,
// and one butterfly reduces all 2 kD of them; the kD x kD triangle inside
// the block is then solved in registers (its U entries are wave-uniform
// loads), and the ring shifts by kD.  The next block's U entries and y
// values are loaded while the current one is reduced.
// top0: the last row to solve; xs (or nullptr): the separator's values, the
// q unknowns after top0 (xi then eta; in reverse for the reversed system);
// rev: rows are those of the reversed system (natural row n - 1 - k).
template <int P1>
__device__ __forceinline__ void back_substitute_blocked(const SubArgs &a, const double *U, const double *Y, int n,
                                                        int top0, int i0, int j0, const double *xs, bool rev) {
    constexpr int p = P1 - 1, q = P1 - 1, kD = 8;
    const int lane = threadIdx.x & 63;
    // the ring: x_{top+lane+1}, x_{top+lane+65}; eta likewise
    auto sep_val = [&](int t, int comp) -> double {
        if (!xs || t >= q) return 0.0;
        return xs[comp * q + (rev ? q - 1 - t : t)];
    };
    double xr0 = sep_val(lane, 0), xr1 = sep_val(lane + 64, 0);
    double yr0 = sep_val(lane, 1), yr1 = sep_val(lane + 64, 1);
    double c0[kD], c1[kD], cd[kD], cyx[kD], cyy[kD];
    double n0[kD], n1[kD], nd[kD], nyx[kD], nyy[kD];
    // rows top - j: the entries multiplying the ring, the diagonal and y
    auto load = [&](int top, double *u0, double *u1, double *ud, double *yx, double *yy) {
#pragma unroll
        for (int j = 0; j < kD; ++j) {
            const int k = top - j;
            const bool ok = k >= 0;
            const double *row = U + (int64_t)(ok ? k : 0) * P1;
            const int o0 = j + 1 + lane, o1 = j + 65 + lane;
            u0[j] = (ok && o0 <= p) ? row[o0] : 0.0;
            u1[j] = (ok && o1 <= p) ? row[o1] : 0.0;
            ud[j] = ok ? row[0] : 1.0;
            yx[j] = ok ? Y[k] : 0.0;
            yy[j] = ok ? Y[n + k] : 0.0;
        }
    };
    load(top0, c0, c1, cd, cyx, cyy);
    for (int top = top0; top >= 0; top -= kD) {
        load(top - kD, n0, n1, nd, nyx, nyy);
        // 2 kD partial sums per lane, reduced across the wave by a butterfly
        // that halves the values each lane keeps (offsets 32, 16, 8, 4: lane
        // l ends with value l >> 2 summed over the 16 lanes that share its
        // low two bits), then offsets 2 and 1 complete the sums.
        double v[2 * kD];
#pragma unroll
        for (int j = 0; j < kD; ++j) {
            v[j] = fma(c0[j], xr0, c1[j] * xr1);
            v[kD + j] = fma(c0[j], yr0, c1[j] * yr1);
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int off = 32 >> st, half = kD >> st;   // values held: 2 half
            const bool up = (lane & off) != 0;
#pragma unroll
            for (int t = 0; t < half; ++t) {
                const double keep = up ? v[half + t] : v[t];
                const double give = up ? v[t] : v[half + t];
                v[t] = keep + __shfl_xor(give, off, 64);
            }
        }
        double tot = v[0];
        tot += __shfl_xor(tot, 2, 64);
        tot += __shfl_xor(tot, 1, 64);
        double sx[kD], sy[kD];
#pragma unroll
        for (int j = 0; j < kD; ++j) {
            sx[j] = __shfl(tot, 4 * j, 64);
            sy[j] = __shfl(tot, 4 * (kD + j), 64);
        }
        // the triangle inside the block
        double xb[kD], yb[kD];
#pragma unroll
        for (int j = 0; j < kD; ++j) {
            const int k = top - j;
            double tx = cyx[j] - sx[j], ty = cyy[j] - sy[j];
            if (k >= 0) {
                const double *row = U + (int64_t)k * P1;
#pragma unroll
                for (int i = 0; i < j; ++i) {
                    const double u = row[j - i];   // U[k][k + (j - i)] multiplies x_{k_i}
                    tx = fma(-u, xb[i], tx);
                    ty = fma(-u, yb[i], ty);
                }
            }
            xb[j] = tx / cd[j];
            yb[j] = ty / cd[j];
        }
#pragma unroll
        for (int j = 0; j < kD; ++j) {
            const int k = top - j;
            if (lane == j && k >= 0) {
                const int64_t g = unknown_node(a, rev ? n - 1 - k : k, i0, j0);
                a.xi_out[g] = xb[j];
                a.eta_out[g] = yb[j];
            }
        }
        // shift the ring by kD: lane l now holds x_{top-kD+1+l}
        const int src = (lane + 64 - kD) & 63;
        const double sx0 = __shfl(xr0, src, 64), sx1 = __shfl(xr1, src, 64);
        const double sy0 = __shfl(yr0, src, 64), sy1 = __shfl(yr1, src, 64);
        double bx = 0.0, by = 0.0;
#pragma unroll
        for (int j = 0; j < kD; ++j) {
            bx = (lane == kD - 1 - j) ? xb[j] : bx;
            by = (lane == kD - 1 - j) ? yb[j] : by;
        }
        const bool head = lane < kD;
        xr1 = head ? sx0 : sx1;
        yr1 = head ? sy0 : sy1;
        xr0 = head ? bx : sx0;
        yr0 = head ? by : sy0;
#pragma unroll
        for (int j = 0; j < kD; ++j) {
            c0[j] = n0[j];
            c1[j] = n1[j];
            cd[j] = nd[j];
            cyx[j] = nyx[j];
            cyy[j] = nyy[j];
        }
    }
}

// Every row's coefficients of a sub-domain system (Dirichlet neighbours
// moved to the right-hand side), in the natural or the reversed order (row
// n-1-r, fast+ <-> fast-, slow+ <-> slow-), by the threads of the
// workgroup.  cf[r] = (fast+, fast-, slow+, slow-) neighbour coefficients:
// (east, west, north, south) when x is the fast index, (north, south, east,
// west) when y is.
__device__ void assemble_rows(const SubArgs &a, int n, int i0, int j0, bool rev, double4 *cf, double2 *rh) {
    const int N1 = a.N + 1, qf = a.qf, qs = a.qs;
    const int64_t of = a.xfast ? 1 : N1, os = a.xfast ? N1 : 1;   // grid offsets of the fast / slow neighbours
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const int f = r % qf, s = r / qf;
        const int gi = i0 + 1 + (a.xfast ? f : s), gj = j0 + 1 + (a.xfast ? s : f);
        double bx, by;
        node_drift_f64(a, gi, gj, bx, by);
        const double cxr = a.half_d_over_h * bx, cyr = a.half_d_over_h * by;
        const double cE = -a.c - cxr, cW = -a.c + cxr, cN = -a.c - cyr, cS = -a.c + cyr;
        const double cFp = a.xfast ? cE : cN, cFm = a.xfast ? cW : cS;
        const double cSp = a.xfast ? cN : cE, cSm = a.xfast ? cS : cW;
        const int64_t g = (int64_t)gj * N1 + gi;
        double fx = a.steady ? 0.0 : a.xi_n[g], fy = a.steady ? 0.0 : a.eta_n[g];
        if (f == qf - 1) { fx -= cFp * a.xi_out[g + of]; fy -= cFp * a.eta_out[g + of]; }
        if (f == 0) { fx -= cFm * a.xi_out[g - of]; fy -= cFm * a.eta_out[g - of]; }
        if (s == qs - 1) { fx -= cSp * a.xi_out[g + os]; fy -= cSp * a.eta_out[g + os]; }
        if (s == 0) { fx -= cSm * a.xi_out[g - os]; fy -= cSm * a.eta_out[g - os]; }
        const double e = f < qf - 1 ? cFp : 0.0, w = f > 0 ? cFm : 0.0;
        const double nn = s < qs - 1 ? cSp : 0.0, ss = s > 0 ? cSm : 0.0;
        cf[rev ? n - 1 - r : r] = rev ? make_double4(w, e, ss, nn) : make_double4(e, w, nn, ss);
        rh[rev ? n - 1 - r : r] = make_double2(fx, fy);
    }
}

// Original matrix entry (r, c) of an assembled system with band width q;
// identity beyond n.  (With q = 1 the fast and slow neighbours are the same
// column: their coefficients add.)
__device__ __forceinline__ double band_entry(const double4 *cf, int n, int q, double diag, int r, int c) {
    if (r >= n || c >= n) return r == c ? 1.0 : 0.0;
    const int d = c - r;
    if (d == 0) return diag;
    if (d != 1 && d != -1 && d != q && d != -q) return 0.0;
    const double4 f = cf[r];
    if (q == 1) return d == 1 ? f.x + f.z : f.y + f.w;
    return d == 1 ? f.x : d == -1 ? f.y : d == q ? f.z : f.w;
}

// 1 / x for the pivots of the elimination (positive, diagonally dominant):
// the hardware reciprocal refined by two Newton steps y <- y + y (1 - x y),
// each of which squares the relative error; the result is within an ulp or
// two of the correctly rounded quotient, in 5 instructions instead of the
// division's scaled sequence.
__device__ __forceinline__ double pivot_rcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// Banded LU with the window spread over a 16 x 16 grid of lanes.  The
// window of elimination step k is rows and columns k .. k + W - 1, W = 16 T
// >= q + 16 (rows and columns past the band of row k are zero where they
// meet column / row k and are left unchanged), kept circularly: global
// index g sits at physical index g mod W.  Lane (rg, cg) holds the T x T
// entries of the rows rg + (16-blocks) and columns cg + (16-blocks), and the
// lanes with cg < 2 the right-hand side cg (xi, eta) of their rows.
// Register slot 0 always holds the 16-block of the current pivots; after 16
// steps the slots rotate by one, so every register index is a compile-time
// constant.  Step k:
//  * the lanes holding the pivot column write it to LDS, the lanes holding
//    the pivot row write it and its right-hand sides to LDS and out as U row
//    k and y_k; one barrier;
//  * every lane reads its T pivot-column and T pivot-row entries and updates
//    its entries: T^2 FMAs (plus T for the right-hand sides).
// The freed row and column of the pivot are refilled only after the block's
// 16 steps, all at once: the 16 rows and columns k0 + W .. k0 + W + 15 that
// enter are not touched by an elimination step before step k0 + W - q >=
// k0 + 16 (their first entries in the band), so until then the freed slots
// may hold anything -- they only ever meet each other.  Entering rows and
// columns carry their original entries (west / south and east / north
// neighbours, loaded a block ahead).  Twisted elimination stops at the
// separator and writes its block of the trailing window; the U rows are
// solved by back_block_kernel.
template <int T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
subdomain_lu_tile_kernel(const SubArgs a) {
    constexpr int W = 16 * T;
    // [buffer][pivot 0 / 1] the pivot column by row and the pivot row by
    // column, indexed by register slot and lane (16 t + lane: slot 0 holds the
    // pivots' block), then the row's two right-hand sides
    __shared__ double colb[2][2][W];
    __shared__ double rowb[2][2][W + 2];
    const int qf = a.qf, P1 = qf + 1, n = qf * a.qs;
    const int sd = a.twisted ? blockIdx.x >> 1 : blockIdx.x;
    const bool rev = a.twisted && (blockIdx.x & 1);
    int i0, j0;
    sub_origin(a, sd, i0, j0);
    const int steps = !a.twisted ? n : (rev ? n - a.sep - qf : a.sep);
    const int off = rev ? a.sep : 0;
    const int us = a.ustride;                    // = W: every window column has a slot in U's rows
    double *U = a.ubuf + (int64_t)sd * n * us + (int64_t)off * us;
    double *Y = a.ybuf + (int64_t)sd * 2 * n + off;
    const int64_t cix = a.twisted ? 2 * (int64_t)sd + (rev ? 1 : 0) : sd;
    double4 *cf = reinterpret_cast<double4 *>(a.cbuf + cix * 4 * n);
    double2 *rh = reinterpret_cast<double2 *>(a.rbuf + cix * 2 * n);
    const int tid = threadIdx.x;

    assemble_rows(a, n, i0, j0, rev, cf, rh);
    __threadfence_block();
    __syncthreads();

    const double diag = a.diag0 + 4.0 * a.c;
    const int rg = tid >> 4, cg = tid & 15;
    const bool rhs = cg < 2;
    double A[T][T], B[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
        for (int u = 0; u < T; ++u) A[t][u] = band_entry(cf, n, qf, diag, rg + 16 * t, cg + 16 * u);
        const int r = rg + 16 * t;
        B[t] = (rhs && r < n) ? (cg == 0 ? rh[r].x : rh[r].y) : 0.0;
    }
    // Wait for the window's loads here, once: the waits the compiler places
    // for registers loaded before the step loop would otherwise sit inside
    // it (vmcnt 0 on every step, behind the U-row stores of the step).
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt and lgkmcnt unconstrained
    // what the block of steps k0 .. k0 + 15 lets in: this lane's row
    // k0 + W + rg (coefficients and right-hand side) and, for its column
    // c = k0 + W + cg, the fast+ coefficient of row c - 1 and the slow+ one
    // of row c - q; zero past the last row
    double4 crow;
    double2 rrow;
    double fcol, scol;
    auto load_enter = [&](int k0) {
        const int Rr = k0 + W + rg, Rc = k0 + W + cg;
        crow = Rr < n ? cf[Rr] : make_double4(0.0, 0.0, 0.0, 0.0);
        rrow = (rhs && Rr < n) ? rh[Rr] : make_double2(0.0, 0.0);
        fcol = Rc - 1 < n ? cf[Rc - 1].x : 0.0;
        scol = Rc - qf < n ? cf[Rc - qf].z : 0.0;
    };

    int base = 0, k = 0;
    double rnext = pivot_rcp(A[0][0]);  // reciprocal of the next pivot (meaningful in its lane)
    int po[T];                     // physical offset of slot t: 16 ((t + base) mod T)
    auto set_offsets = [&]() {
#pragma unroll
        for (int t = 0; t < T; ++t) po[t] = 16 * ((t + base) % T);
    };
    set_offsets();
    // U row k (global) from this lane's entries v of the row whose pivot is
    // lane column gg of slot 0: the window column at band offset d goes to
    // slot d of the row (d in 0 .. W-1; the slots past q receive columns
    // outside the band and are never read), so the stores need no test.  The
    // band offset of slot u is cg - gg + 16 u modulo W whatever the rotation
    // (slot u sits 16 u physical columns after slot 0, circularly), which is
    // cg - gg + 16 u itself for u >= 1.
    auto put_u = [&](int kk, int gg, const double (&v)[T]) {
        const int64_t rb = (int64_t)kk * us + (cg - gg);
        U[rb + (cg < gg ? W : 0)] = v[0];
#pragma unroll
        for (int u = 1; u < T; ++u) U[rb + 16 * u] = v[u];
    };
    // Steps k and k + 1 (block-relative pivots g and g + 1) behind one
    // barrier, with LDS buffer BUF (the buffers alternate from barrier to
    // barrier; a block's 16 steps are 8 pairs, so its first pair takes buffer
    // 0 and the buffer index is a compile-time constant).
    auto pair = [&](int g, auto bufc) {
        constexpr int buf = decltype(bufc)::value;
        // ---- steps k and k + 1 behind one barrier -------------------
        // The lanes of columns g and g + 1 publish them (the pivot's
        // reciprocal, formed at the end of the previous step, at the
        // pivot), the lanes of rows g and g + 1 theirs and their
        // right-hand sides, all as they stand before step k.
        if (cg == g) {
#pragma unroll
            for (int t = 0; t < T; ++t) colb[buf][0][16 * t + rg] = (t == 0 && rg == g) ? rnext : A[t][0];
        } else if (cg == g + 1) {
#pragma unroll
            for (int t = 0; t < T; ++t) colb[buf][1][16 * t + rg] = A[t][0];
        }
        if (rg == g || rg == g + 1) {
            const int h = rg - g;
            double v[T];
#pragma unroll
            for (int u = 0; u < T; ++u) {
                v[u] = A[0][u];
                rowb[buf][h][16 * u + cg] = v[u];
            }
            if (rhs) rowb[buf][h][W + cg] = B[0];
            if (h == 0) {
                put_u(k, g, v);
                if (rhs) Y[(int64_t)cg * n + k] = B[0];
            }
        }
        __syncthreads();
        double l0[T], c1[T], r0[T], r1[T];
        const double inv0 = colb[buf][0][g];
        const double a1k = colb[buf][0][g + 1], ak1 = rowb[buf][0][g + 1], a11 = rowb[buf][1][g + 1];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            l0[t] = colb[buf][0][16 * t + rg];
            c1[t] = colb[buf][1][16 * t + rg];
        }
#pragma unroll
        for (int u = 0; u < T; ++u) {
            r0[u] = rowb[buf][0][16 * u + cg];
            r1[u] = rowb[buf][1][16 * u + cg];
        }
        const double b0 = rowb[buf][0][W + cg], b1 = rowb[buf][1][W + cg];
        // step k's multipliers; row k + 1, its right-hand side and its
        // pivot as step k leaves them (the operations step k would
        // apply to them, in the same order)
        const double l01 = a1k * inv0;
        const double inv1 = pivot_rcp(fma(-l01, ak1, a11));
#pragma unroll
        for (int t = 0; t < T; ++t) l0[t] *= inv0;
#pragma unroll
        for (int u = 0; u < T; ++u) r1[u] = fma(-l01, r0[u], r1[u]);
        const double b1p = fma(-l01, b0, b1);
        if (rg == g + 1) {
            put_u(k + 1, g + 1, r1);
            if (rhs) Y[(int64_t)cg * n + k + 1] = b1p;
        }
        // step k on every entry (the reciprocal's latency hides behind it)
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int u = 0; u < T; ++u) A[t][u] = fma(-l0[t], r0[u], A[t][u]);
        if (rhs) {
#pragma unroll
            for (int t = 0; t < T; ++t) B[t] = fma(-l0[t], b0, B[t]);
        }
        // step k + 1: column k + 1 as step k leaves it, its multipliers
        double l1[T];
#pragma unroll
        for (int t = 0; t < T; ++t) l1[t] = fma(-l0[t], ak1, c1[t]) * inv1;
        // the entry that is the next pivot first, and its reciprocal
        double np;
        if (T > 1 && g == 14) {
            A[1][1] = fma(-l1[1], r1[1], A[1][1]);
            np = A[1][1];
        } else {
            A[0][0] = fma(-l1[0], r1[0], A[0][0]);
            np = A[0][0];
        }
        rnext = pivot_rcp(np);
#pragma unroll
        for (int t = 0; t < T; ++t) {
#pragma unroll
            for (int u = 0; u < T; ++u) {
                if (t == 0 && u == 0 && !(T > 1 && g == 14)) continue;
                if (T > 1 && t == 1 && u == 1 && g == 14) continue;
                A[t][u] = fma(-l1[t], r1[u], A[t][u]);
            }
        }
        if (rhs) {
#pragma unroll
            for (int t = 0; t < T; ++t) B[t] = fma(-l1[t], b1p, B[t]);
        }
    };
    int k0 = 0, npair = 0;
    while (k < steps) {
        k0 = k;
        load_enter(k0);
        npair = 0;
        for (int g = 0; g < 16 && k + 1 < steps;) {
            pair(g, std::integral_constant<int, 0>{});
            g += 2;
            k += 2;
            ++npair;
            if (g >= 16 || k + 1 >= steps) break;
            pair(g, std::integral_constant<int, 1>{});
            g += 2;
            k += 2;
            ++npair;
        }
        if (k - k0 < 16 || k >= steps) break;
        // the block is done: its rows and columns k0 + W + (0 .. 15) enter
        // slot 0.  The window now starts at k0 + 16, at physical 16 (base + 1).
        const int ws = k0 + 16, wp = 16 * (base + 1 == T ? 0 : base + 1);
        const int Rr = k0 + W + rg, Rc = k0 + W + cg;
        const double dR = Rr < n ? diag : 1.0;
        // row Rr over every column of the window
#pragma unroll
        for (int u = 0; u < T; ++u) {
            int rel = cg + po[u] - wp;
            rel += rel < 0 ? W : 0;
            const int d = ws + rel - Rr;             // column minus row
            double v = d == 0 ? dR : 0.0;
            v += d == 1 ? crow.x : 0.0;
            v += d == -1 ? crow.y : 0.0;
            v += d == qf ? crow.z : 0.0;
            v += d == -qf ? crow.w : 0.0;
            A[0][u] = v;
        }
        if (rhs) B[0] = cg == 0 ? rrow.x : rrow.y;
        // column Rc in the rows that were already there (slots 1 .. T-1)
#pragma unroll
        for (int t = 1; t < T; ++t) {
            int rel = rg + po[t] - wp;
            rel += rel < 0 ? W : 0;
            const int d = Rc - (ws + rel);            // column minus row, > 0
            double v = d == 1 ? fcol : 0.0;
            v += d == qf ? scol : 0.0;
            A[t][0] = v;
        }
        // rotate the slots by one: slot 0 (the rows and columns that just
        // entered, the last of the window) goes last
        {
            double a0[T], b0 = B[0];
#pragma unroll
            for (int u = 0; u < T; ++u) a0[u] = A[0][u];
#pragma unroll
            for (int t = 0; t + 1 < T; ++t) {
                const double c0 = A[t + 1][0];
#pragma unroll
                for (int u = 0; u + 1 < T; ++u) A[t][u] = A[t + 1][u + 1];
                A[t][T - 1] = c0;
                B[t] = B[t + 1];
            }
#pragma unroll
            for (int u = 0; u + 1 < T; ++u) A[T - 1][u] = a0[u + 1];
            A[T - 1][T - 1] = a0[0];
            B[T - 1] = b0;
        }
        base = base + 1 == T ? 0 : base + 1;
        set_offsets();
    }
    if (k < steps) {
        // ---- the last step of an odd count, alone --------------------------
        const int g = k - k0, buf = npair & 1;
        if (cg == g) {
            // the pivot column; at the pivot its reciprocal, formed at the
            // end of the previous step
#pragma unroll
            for (int t = 0; t < T; ++t) colb[buf][0][16 * t + rg] = (t == 0 && rg == g) ? rnext : A[t][0];
        }
        if (rg == g) {
            double v[T];
#pragma unroll
            for (int u = 0; u < T; ++u) {
                v[u] = A[0][u];
                rowb[buf][0][16 * u + cg] = v[u];
            }
            put_u(k, g, v);
            if (rhs) {
                rowb[buf][0][W + cg] = B[0];
                Y[(int64_t)cg * n + k] = B[0];
            }
        }
        __syncthreads();
        // every LDS read of the step at once, then the update
        double l[T], r[T];
        const double inv = colb[buf][0][g];
#pragma unroll
        for (int t = 0; t < T; ++t) l[t] = colb[buf][0][16 * t + rg];
#pragma unroll
        for (int u = 0; u < T; ++u) r[u] = rowb[buf][0][16 * u + cg];
        const double bp = rowb[buf][0][W + cg];
#pragma unroll
        for (int t = 0; t < T; ++t) l[t] *= inv;
        // the entry that is the next pivot first (slot 0's diagonal, or
        // slot 1's after the last step of the block), and its reciprocal,
        // whose latency the rest of the update hides
        double np;
        if (T > 1 && g == 15) {
            A[1][1] = fma(-l[1], r[1], A[1][1]);
            np = A[1][1];
        } else {
            A[0][0] = fma(-l[0], r[0], A[0][0]);
            np = A[0][0];
        }
        rnext = pivot_rcp(np);
#pragma unroll
        for (int t = 0; t < T; ++t) {
#pragma unroll
            for (int u = 0; u < T; ++u) {
                if (t == 0 && u == 0 && !(T > 1 && g == 15)) continue;
                if (T > 1 && t == 1 && u == 1 && g == 15) continue;
                A[t][u] = fma(-l[t], r[u], A[t][u]);
            }
        }
        if (rhs) {
#pragma unroll
            for (int t = 0; t < T; ++t) B[t] = fma(-l[t], bp, B[t]);
        }
        ++k;
    }
    if (a.twisted) {
        // the separator block of the trailing window (its first q rows and
        // columns, global steps .. steps + q - 1) and its right-hand sides;
        // the rows and columns freed in the last block are past it
        double *S = a.sbuf + (int64_t)sd * sep_stride(qf) + (rev ? (size_t)qf * qf + 2 * qf : 0);
        const int kp0 = steps % W;
#pragma unroll
        for (int t = 0; t < T; ++t) {
            int dr = rg + po[t] - kp0;
            dr += dr < 0 ? W : 0;
            if (dr >= qf) continue;
#pragma unroll
            for (int u = 0; u < T; ++u) {
                int dc = cg + po[u] - kp0;
                dc += dc < 0 ? W : 0;
                if (dc < qf) S[(size_t)dr * qf + dc] = A[t][u];
            }
            if (rhs) S[(size_t)qf * qf + (size_t)cg * qf + dr] = B[t];
        }
    }
}

// Back substitution after the tile kernel, one workgroup per elimination
// (per end when twisted): x_k = (y_k - sum_d U[k][k+d] x_{k+d}) / U[k][k],
// rows from the last one up, 64 at a time.  Wavefront 0 solves a block
// while wavefronts 1-3 copy the next block's U rows and right-hand sides to
// the other of two LDS buffers (coalesced, 16 loads in flight per lane), so
// the copy's latency hides behind the solve; one barrier per block.  The
// solve: lane l takes row top - l and first sums its terms with the columns
// already solved (beyond the block, from an LDS ring of solutions), all
// lanes at once; the triangle inside the block is then swept row by row: the
// value of each row is broadcast from its lane (readlane) and every lane
// below adds its term; then every lane stores its own row's solution.  The
// ring starts with the separator's values (twisted) or zeros (past the last
// row).
constexpr int kBackRows = 64;
__host__ __device__ inline int back_stride(int P1) { return (P1 + 2) & ~1; }

__global__ void __launch_bounds__(256) back_block_kernel(const SubArgs a) {
    // 2 x kBackRows rows of stride S, the ring, the y blocks.  S is even:
    // lane l reads its row nb-1-l at column l + d, a stride of 1 - S (odd)
    // doubles from lane to lane, which spreads a wavefront's reads over the
    // banks (an odd S put every lane on one bank)
    extern __shared__ double Ub[];
    const int qf = a.qf, P1 = qf + 1, n = qf * a.qs, S = back_stride(P1);
    double *xr = Ub + (size_t)2 * kBackRows * S; // [2][256]: solutions by row & 255
    double *yb = xr + 512;                       // [2 buffers][2 components][kBackRows]
    const int sd = a.twisted ? blockIdx.x >> 1 : blockIdx.x;
    const bool rev = a.twisted && (blockIdx.x & 1);
    int i0, j0;
    sub_origin(a, sd, i0, j0);
    const int steps = !a.twisted ? n : (rev ? n - a.sep - qf : a.sep);
    const int off = rev ? a.sep : 0;
    const int us = a.ustride;
    const double *U = a.ubuf + (int64_t)sd * n * us + (int64_t)off * us;
    const double *Y = a.ybuf + (int64_t)sd * 2 * n + off;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int t = tid; t < 512; t += 256) xr[t] = 0.0;
    __syncthreads();
    if (a.twisted) {
        const double *xs = a.sbuf + (int64_t)sd * sep_stride(qf) + 2 * ((size_t)qf * qf + 2 * qf);
        for (int t = tid; t < qf; t += 256) {
            const int row = (steps + t) & 255, src = rev ? qf - 1 - t : t;
            xr[row] = xs[src];
            xr[256 + row] = xs[qf + src];
        }
    }
    // the U rows and y values of the block ending at row `top` into buffer
    // `buf`, by threads t of nt
    auto load_block = [&](int top, int buf, int t, int nt) {
        const int nb = min(kBackRows, top + 1), base = top - nb + 1;
        const double *src = U + (int64_t)base * us;
        double *dst = Ub + (size_t)buf * kBackRows * S;
        const int tot = nb * P1;                 // the first P1 slots of each row
        if (t < nb) {
            yb[(2 * buf) * kBackRows + t] = Y[base + t];
            yb[(2 * buf + 1) * kBackRows + t] = Y[n + base + t];
        }
        for (int e0 = 0; e0 < tot; e0 += 16 * nt) {
            double v[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int e = e0 + i * nt + t, rr = e / P1;
                v[i] = e < tot ? src[(int64_t)rr * us + (e - rr * P1)] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int e = e0 + i * nt + t;
                if (e < tot) {
                    const int rr = e / P1;
                    dst[rr * S + (e - rr * P1)] = v[i];
                }
            }
        }
    };
    if (steps > 0) load_block(steps - 1, 0, tid, 256);
    __syncthreads();
    int buf = 0;
    for (int top = steps - 1; top >= 0; top -= kBackRows, buf ^= 1) {
        if (wave != 0) {
            if (top >= kBackRows) load_block(top - kBackRows, buf ^ 1, tid - 64, 192);
        } else {
            const int nb = min(kBackRows, top + 1);
            const bool has = lane < nb;
            const int r = top - lane, lr = nb - 1 - lane;   // this lane's row and its place in the block
            const double *ur = Ub + (size_t)buf * kBackRows * S + (has ? lr : 0) * S;
            double sx = 0.0, sy = 0.0, yx = 0.0, yy = 0.0, d0 = 1.0;
            if (has) {
                d0 = ur[0];
                yx = yb[(2 * buf) * kBackRows + lr];
                yy = yb[(2 * buf + 1) * kBackRows + lr];
                // four terms per pass, so the LDS reads of a pass are in flight together
                int d = lane + 1;
                for (; d + 3 <= qf; d += 4) {
                    double u4[4], x4[4], y4[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int c = (r + d + i) & 255;
                        u4[i] = ur[d + i];
                        x4[i] = xr[c];
                        y4[i] = xr[256 + c];
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        sx = fma(u4[i], x4[i], sx);
                        sy = fma(u4[i], y4[i], sy);
                    }
                }
                for (; d <= qf; ++d) {
                    const int c = (r + d) & 255;
                    sx = fma(ur[d], xr[c], sx);
                    sy = fma(ur[d], xr[256 + c], sy);
                }
            }
            const double inv = 1.0 / d0;
            double ucur = (has && lane >= 1 && lane <= qf) ? ur[lane] : 0.0;   // term of row top at step 0
            double mx = 0.0, my = 0.0;                   // this lane's own row's solution
            for (int s = 0; s < nb; ++s) {
                const int dn = lane - s - 1;
                const double unext = (has && dn >= 1 && dn <= qf) ? ur[dn] : 0.0;
                const double ox = (yx - sx) * inv, oy = (yy - sy) * inv;
                const double xv = readlane_f64(ox, s), yv = readlane_f64(oy, s);
                if (lane == s) {
                    mx = ox;
                    my = oy;
                }
                sx = fma(ucur, xv, sx);
                sy = fma(ucur, yv, sy);
                ucur = unext;
            }
            if (has) {
                xr[r & 255] = mx;
                xr[256 + (r & 255)] = my;
                const int64_t gn = unknown_node(a, rev ? n - 1 - r : r, i0, j0);
                a.xi_out[gn] = mx;
                a.eta_out[gn] = my;
            }
        }
        __syncthreads();
    }
}

// Banded LU of a small window (P1 <= 32) in one wavefront, one lane per
// window column: lane t < P1 holds the columns c = t (mod P1) with all P1
// window rows in v[0 .. P1-1], lanes P1 and P1 + 1 the two right-hand sides.
// Step k reads the pivot column from its lane into scalar registers
// (readlane: the lane is wave-uniform), and every lane updates and shifts
// its column in one pass, v[i] = v[i + 1] - pivotcol[i + 1] * (v[0] / pivot).
// The pivot column becomes exactly zero and its lane takes the entering
// column k + P1 (rows k + 1, k + q and k + P1: north neighbour, east
// neighbour, diagonal); the row k + P1 enters at the bottom with its
// original entries (west and south neighbours), staged in LDS a batch ahead.
// No barrier per step, no LDS traffic for the window.  The outputs are those
// of subdomain_lu_kernel: U rows, y values, and in twisted mode the
// separator block of the trailing window.
template <int P1, bool TW>
__global__ void __launch_bounds__(64) subdomain_lu_wave_kernel(const SubArgs a) {
    constexpr int q = P1 - 1;
    constexpr int kW = 64;   // steps per staging batch: one entering row per lane
    static_assert(P1 + 2 <= 64, "one lane per window column and right-hand side");
    __shared__ double4 Cst[2][kW];   // coefficients of the entering rows R = k + P1
    __shared__ double2 Rst[2][kW];   // their right-hand sides
    __shared__ double Nst[2][kW];    // slow+ coefficients of the rows k + 1
    const int n = q * a.qs;
    const int sd = TW ? blockIdx.x >> 1 : blockIdx.x;
    const bool rev = TW && (blockIdx.x & 1);
    int i0, j0;
    sub_origin(a, sd, i0, j0);
    const int steps = !TW ? n : (rev ? n - a.sep - q : a.sep);
    const int off = rev ? a.sep : 0;
    double *U = a.ubuf + (int64_t)sd * n * P1 + (int64_t)off * P1;
    double *Y = a.ybuf + (int64_t)sd * 2 * n + off;
    const int64_t cix = TW ? 2 * (int64_t)sd + (rev ? 1 : 0) : sd;
    double4 *cf = reinterpret_cast<double4 *>(a.cbuf + cix * 4 * n);
    double2 *rh = reinterpret_cast<double2 *>(a.rbuf + cix * 2 * n);
    const int lane = threadIdx.x;

    assemble_rows(a, n, i0, j0, rev, cf, rh);
    __threadfence_block();
    __syncthreads();

    const double diag = a.diag0 + 4.0 * a.c;
    const bool is_col = lane < P1;
    const bool is_rhs = lane == P1 || lane == P1 + 1;
    const int rhs_c = lane - P1;                 // 0: xi, 1: eta (right-hand-side lanes)
    int col = lane;                              // the column a column lane holds
    double v[P1];
#pragma unroll
    for (int i = 0; i < P1; ++i) {
        double e = 0.0;
        if (is_col) e = band_entry(cf, n, q, diag, i, col);
        else if (is_rhs && i < n) e = rhs_c == 0 ? rh[i].x : rh[i].y;
        v[i] = e;
    }
    // lane j loads the entering coefficients of step bt kW + j
    auto load_batch = [&](int bt, double4 &c4, double2 &r2, double &cn) {
        const int kk = bt * kW + lane, R = kk + P1;
        c4 = (kk < steps && R < n) ? cf[R] : make_double4(0.0, 0.0, 0.0, 0.0);
        r2 = (kk < steps && R < n) ? rh[R] : make_double2(0.0, 0.0);
        cn = (kk < steps && kk + 1 < n) ? cf[kk + 1].z : 0.0;
    };
    double4 pc4;
    double2 pr2;
    double pcn;
    load_batch(0, pc4, pr2, pcn);
    double cE_Rm1 = (P1 - 1 < n) ? cf[P1 - 1].x : 0.0;   // east coefficient of row R - 1

    int owner = 0;
    for (int k = 0; k < steps; ++k) {
        const int j = k % kW, bb = (k / kW) & 1;
        if (j == 0) {
            Cst[bb][lane] = pc4;
            Rst[bb][lane] = pr2;
            Nst[bb][lane] = pcn;
            load_batch(k / kW + 1, pc4, pr2, pcn);
            __syncthreads();
        }
        // the pivot column, wave-uniform
        double pc[P1];
#pragma unroll
        for (int i = 0; i < P1; ++i) pc[i] = readlane_f64(v[i], owner);
        const double u = v[0];                   // row k of this lane's column
        // U row k (band offset col - k) and the y values
        if (is_col) U[(int64_t)k * P1 + (col - k)] = u;
        else if (is_rhs) Y[rhs_c * n + k] = u;
        const bool own = lane == owner;
        // the pivot column itself: scale exactly 1, so it becomes exactly zero
        const double sc = own ? 1.0 : u * (1.0 / pc[0]);
#pragma unroll
        for (int i = 0; i < P1 - 1; ++i) v[i] = fma(-pc[i + 1], sc, v[i + 1]);
        const int R = k + P1;
        const bool live = R < n;
        const double4 cR = Cst[bb][j];
        double last;
        if (is_col) last = (live && col < n) ? (col == R - 1 ? cR.y : (col == R - q ? cR.w : 0.0)) : 0.0;
        else last = rhs_c == 0 ? Rst[bb][j].x : Rst[bb][j].y;
        if (own) {
            // the entering column R: rows k + 1 (north of k + 1), R - 1 (east of R - 1), R
            col = R;
            v[0] = live ? Nst[bb][j] : 0.0;
            v[P1 - 2] = live ? cE_Rm1 : 0.0;
            last = live ? diag : 1.0;
        }
        v[P1 - 1] = last;
        cE_Rm1 = cR.x;
        owner = (owner + 1 == P1) ? 0 : owner + 1;
    }
    if constexpr (TW) {
        // the separator block of the trailing window and its right-hand sides
        double *S = a.sbuf + (int64_t)sd * sep_stride(q) + (rev ? (size_t)q * q + 2 * q : 0);
        const int c = col - steps;
#pragma unroll
        for (int i = 0; i < q; ++i) {
            if (is_col && c < q) S[i * q + c] = v[i];
            else if (is_rhs) S[(size_t)q * q + rhs_c * q + i] = v[i];
        }
    } else {
        __threadfence_block();
        __syncthreads();
        back_substitute_blocked<P1>(a, U, Y, n, n - 1, i0, j0, nullptr, false);
    }
}

// The separator system of a twisted elimination, one workgroup per
// sub-domain: S_top + S_bot - A_SS and its right-hand sides assembled in
// LDS, LU without pivoting (the Schur complement of a diagonally dominant
// matrix is diagonally dominant), then x_S into the workspace and the grid.
__global__ void __launch_bounds__(256) separator_kernel(const SubArgs a) {
    extern __shared__ double M[];   // [q][q] then the two right-hand sides [2][q]
    const int q = a.qf, n = q * a.qs, sd = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    int i0, j0;
    sub_origin(a, sd, i0, j0);
    double *S = a.sbuf + (int64_t)sd * sep_stride(q);
    const double *St = S, *Sb = S + (size_t)q * q + 2 * q;
    double *xs = S + 2 * ((size_t)q * q + 2 * q);
    const double4 *cf = reinterpret_cast<const double4 *>(a.cbuf + (int64_t)(2 * sd) * 4 * n);   // natural order
    const double2 *rh = reinterpret_cast<const double2 *>(a.rbuf + (int64_t)(2 * sd) * 2 * n);
    const double diag = a.diag0 + 4.0 * a.c;
    double *b = M + (size_t)q * q;
    for (int e = tid; e < q * q; e += nt) {
        const int r = e / q, c = e % q;
        const double4 f = cf[a.sep + r];
        const double A = c == r ? diag : (c == r + 1 ? f.x : (c == r - 1 ? f.y : 0.0));
        M[e] = St[e] + Sb[(q - 1 - r) * q + (q - 1 - c)] - A;
    }
    for (int e = tid; e < 2 * q; e += nt) {
        const int comp = e / q, r = e % q;
        const double2 f = rh[a.sep + r];
        b[e] = St[(size_t)q * q + e] + Sb[(size_t)q * q + comp * q + (q - 1 - r)] - (comp ? f.y : f.x);
    }
    __syncthreads();
    // rows by groups of 32 lanes, columns by the lanes of a group (no index
    // division per entry)
    const int tj = tid & 31, ti = tid >> 5, ng = nt >> 5;
    for (int k = 0; k < q; ++k) {
        const double inv = 1.0 / M[k * q + k];
        const int w = q - 1 - k + 2;   // columns k+1 .. q-1, then the two right-hand sides
        for (int i = k + 1 + ti; i < q; i += ng) {
            const double l = M[i * q + k] * inv;
            for (int jj = tj; jj < w; jj += 32) {
                if (jj < q - 1 - k) {
                    const int j = k + 1 + jj;
                    M[i * q + j] = fma(-l, M[k * q + j], M[i * q + j]);
                } else {
                    const int comp = jj - (q - 1 - k);
                    b[comp * q + i] = fma(-l, b[comp * q + k], b[comp * q + i]);
                }
            }
        }
        __syncthreads();
    }
    for (int k = q - 1; k >= 0; --k) {
        if (tid < 2) b[tid * q + k] = b[tid * q + k] / M[k * q + k];
        __syncthreads();
        for (int e = tid; e < 2 * k; e += nt) {
            const int comp = e >= k ? 1 : 0, i = e - comp * k;
            b[comp * q + i] = fma(-M[i * q + k], b[comp * q + k], b[comp * q + i]);
        }
        __syncthreads();
    }
    for (int e = tid; e < 2 * q; e += nt) {
        const int comp = e / q, r = e % q;
        xs[e] = b[e];
        const int64_t g = unknown_node(a, a.sep + r, i0, j0);
        (comp ? a.eta_out : a.xi_out)[g] = b[e];
    }
}

// The same for windows up to 32, a row at a time: lane l < q holds
// x_{k+l+1} (both components), each row's sum over them is a DPP reduction
// within the first 32 lanes, and the window shifts up by one lane (DPP wave
// shift).  U rows and y values are loaded kR rows ahead.
template <int P1>
__global__ void __launch_bounds__(64) twisted_back_wave_kernel(const SubArgs a) {
    constexpr int q = P1 - 1, kR = 8;
    static_assert(q <= 32, "the window fits the first 32 lanes");
    const int n = q * a.qs;
    const int sd = blockIdx.x >> 1;
    const bool rev = (blockIdx.x & 1) != 0;
    const int steps = rev ? n - a.sep - q : a.sep, off = rev ? a.sep : 0;
    int i0, j0;
    sub_origin(a, sd, i0, j0);
    const double *U = a.ubuf + (int64_t)sd * n * P1 + (int64_t)off * P1;
    const double *Y = a.ybuf + (int64_t)sd * 2 * n + off;
    const double *xs = a.sbuf + (int64_t)sd * sep_stride(q) + 2 * ((size_t)q * q + 2 * q);
    const int lane = threadIdx.x;
    // the window starts with the separator's values, the q unknowns after the last row
    double xw = 0.0, yw = 0.0;
    if (lane < q) {
        xw = xs[rev ? q - 1 - lane : lane];
        yw = xs[q + (rev ? q - 1 - lane : lane)];
    }
    double ur[kR], ud[kR], fx[kR], fy[kR];
    auto load = [&](int k, double &u, double &d, double &yx, double &yy) {
        const bool ok = k >= 0;
        const double *row = U + (int64_t)(ok ? k : 0) * P1;
        u = (ok && lane < q) ? row[lane + 1] : 0.0;
        d = ok ? row[0] : 1.0;
        yx = ok ? Y[k] : 0.0;
        yy = ok ? Y[n + k] : 0.0;
    };
#pragma unroll
    for (int r = 0; r < kR; ++r) load(steps - 1 - r, ur[r], ud[r], fx[r], fy[r]);
    for (int k0 = steps - 1; k0 >= 0; k0 -= kR) {
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int k = k0 - r;
            const double sx = sum32_f64(ur[r] * xw), sy = sum32_f64(ur[r] * yw);
            const double x = (fx[r] - sx) / ud[r], y = (fy[r] - sy) / ud[r];
            if (lane == 0 && k >= 0) {
                const int64_t g = unknown_node(a, rev ? n - 1 - k : k, i0, j0);
                a.xi_out[g] = x;
                a.eta_out[g] = y;
            }
            const double ux = dpp_f64<0x138>(xw), uy = dpp_f64<0x138>(yw);   // wave_shr:1
            xw = lane == 0 ? x : ux;
            yw = lane == 0 ? y : uy;
            load(k - kR, ur[r], ud[r], fx[r], fy[r]);
        }
    }
}

// Dirichlet data of the output grids: outer boundary and interface nodes.
__global__ void dirichlet_kernel(const SubArgs a, const double *iface_xi, const double *iface_eta, int64_t n_iface,
                                 int bdry_kind, const double *edge_cells, double *xi_out, double *eta_out) {
    const int N = a.N, px = a.px, mx = a.mx, my = a.my;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int N1 = N + 1;
    const int64_t n_bd = 4 * (int64_t)N;
    if (t < n_bd) {
        // boundary nodes walked as four edges of N nodes each
        const int side = (int)(t / N), o = (int)(t % N);
        int i, j;
        if (side == 0) { i = o; j = 0; }
        else if (side == 1) { i = N; j = o; }
        else if (side == 2) { i = N - o; j = N; }
        else { i = 0; j = N - o; }
        const int64_t g = (int64_t)j * N1 + i;
        double xv = 0.0, ev = 0.0;
        if (bdry_kind == FK_DATA_IDENTITY) {
            xv = (double)i / N;
            ev = (double)j / N;
        } else if (bdry_kind == FK_DATA_EQUIDISTRIBUTED) {
            // xi = 0 / 1 on the left / right edges, eta = 0 / 1 on the bottom /
            // top edges; on the others the 1-D equidistribution of w
            if (i == 0) xv = 0.0;
            else if (i == N) xv = 1.0;
            else xv = edge_fraction(edge_cells, N, j == 0 ? 0 : 1, i);
            if (j == 0) ev = 0.0;
            else if (j == N) ev = 1.0;
            else ev = edge_fraction(edge_cells, N, i == 0 ? 2 : 3, j);
        }
        xi_out[g] = xv;
        eta_out[g] = ev;
        return;
    }
    const int64_t f = t - n_bd;
    if (f >= n_iface) return;
    // canonical order: vertical lines x = a/px (nodes y = j/N), then
    // horizontal lines y = c/py without the crossings
    const int64_t nv = (int64_t)(px - 1) * (N - 1);
    int i, j;
    if (f < nv) {
        i = (int)(f / (N - 1) + 1) * mx;
        j = (int)(f % (N - 1)) + 1;
    } else {
        const int64_t h = f - nv;
        const int per = N - px;  // non-crossing nodes per horizontal line
        const int c = (int)(h / per) + 1;
        const int r = (int)(h % per);
        i = r + 1 + r / (mx - 1);
        j = c * my;
    }
    const int64_t g = (int64_t)j * N1 + i;
    xi_out[g] = iface_xi[f];
    eta_out[g] = iface_eta[f];
}

// min Jacobian and max skewness over all cells (cell-centred differences),
// in three launches on the caller's stream: out's two words set to the
// order keys of +inf and 0, every block's extremes folded in with 64-bit
// integer atomics on the keys, the keys turned back into doubles.  The key
// of a double orders like the double (non-NaN); min and max are exact, so
// the result does not depend on the order of the blocks.
__device__ __forceinline__ unsigned long long order_key(double d) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double key_value(unsigned long long k) {
    return __longlong_as_double((long long)((k >> 63) ? (k & 0x7fffffffffffffffull) : ~k));
}

__global__ void quality_init_kernel(unsigned long long *keys) {
    if (threadIdx.x == 0) {
        keys[0] = order_key(INFINITY);
        keys[1] = order_key(0.0);
    }
}

constexpr int kQualityBlock = 256;

__global__ void __launch_bounds__(kQualityBlock) quality_kernel(const double *xi, const double *eta, int n,
                                                                unsigned long long *keys) {
    const int64_t N1 = n + 1;
    const double inv2h = 0.5 * n;
    // fmin / fmax pass over NaN values (a degenerate cell's skewness 0/0),
    // so a block's extremes, and their keys, are never NaN
    double jmin = INFINITY, smax = 0.0;
    const int64_t cells = (int64_t)n * n;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = c / n, i = c - j * n;
        const int64_t g = j * N1 + i;
        const double a0 = xi[g], a1 = xi[g + 1], a2 = xi[g + N1], a3 = xi[g + N1 + 1];
        const double b0 = eta[g], b1 = eta[g + 1], b2 = eta[g + N1], b3 = eta[g + N1 + 1];
        const double xx = ((a1 - a0) + (a3 - a2)) * inv2h, xy = ((a2 - a0) + (a3 - a1)) * inv2h;
        const double ex = ((b1 - b0) + (b3 - b2)) * inv2h, ey = ((b2 - b0) + (b3 - b1)) * inv2h;
        const double J = xx * ey - xy * ex;
        const double sk = fabs(xx * ex + xy * ey) / (sqrt(xx * xx + xy * xy) * sqrt(ex * ex + ey * ey));
        jmin = fmin(jmin, J);
        smax = fmax(smax, sk);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        jmin = fmin(jmin, __shfl_xor(jmin, off, 64));
        smax = fmax(smax, __shfl_xor(smax, off, 64));
    }
    __shared__ double pj[kQualityBlock / 64], ps[kQualityBlock / 64];
    if ((threadIdx.x & 63) == 0) {
        pj[threadIdx.x >> 6] = jmin;
        ps[threadIdx.x >> 6] = smax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kQualityBlock / 64; ++w) {
            jmin = fmin(jmin, pj[w]);
            smax = fmax(smax, ps[w]);
        }
        atomicMin(&keys[0], order_key(jmin));
        atomicMax(&keys[1], order_key(smax));
    }
}

__global__ void quality_final_kernel(unsigned long long *keys) {
    if (threadIdx.x == 0) {
        const double jmin = key_value(keys[0]), smax = key_value(keys[1]);
        double *out = reinterpret_cast<double *>(keys);
        out[0] = jmin;
        out[1] = smax;
    }
}

// Layout of a px x py split of an N-cell grid: sub-domain sizes, the
// ordering (the shorter side is the fast index) and the band.
struct SubGeom {
    int px, py, mx, my, qf, qs, xfast;
    int64_t n;       // unknowns per sub-domain
    int64_t n_iface;
};
static SubGeom sub_geom(int px, int py, int N) {
    SubGeom g{};
    g.px = px;
    g.py = py;
    g.mx = N / px;
    g.my = N / py;
    g.xfast = g.mx <= g.my ? 1 : 0;
    g.qf = (g.xfast ? g.mx : g.my) - 1;
    g.qs = (g.xfast ? g.my : g.mx) - 1;
    g.n = (int64_t)g.qf * g.qs;
    g.n_iface = (int64_t)(px - 1) * (N - 1) + (int64_t)(py - 1) * (N - px);
    return g;
}

// U row stride of a band of q = qf unknowns: q + 1 for the one-wavefront
// kernels (the bands they take), otherwise the tile kernel's window 16 T.
static int u_stride(int qf) {
    const int P1 = qf + 1;
    if (P1 == 8 || P1 == 12 || P1 == 16 || P1 == 20 || P1 == 24 || P1 == 32) return P1;
    return 16 * ((qf + 16 + 15) / 16);
}

// Workspace: U rows, y values, row coefficients and right-hand sides (two
// copies per sub-domain: natural and reversed order), the separator blocks,
// and the edge integrals.
static size_t sub_ws_bytes(const SubGeom &g, int N) {
    const size_t n = (size_t)g.n, us = (size_t)u_stride(g.qf);
    const size_t blocks = (size_t)g.px * g.py;
    return align256(blocks * n * us * sizeof(double)) + align256(blocks * 2 * n * sizeof(double)) +
           align256(2 * blocks * 4 * n * sizeof(double)) + align256(2 * blocks * 2 * n * sizeof(double)) +
           align256(blocks * sep_stride(g.qf) * sizeof(double)) + align256(4 * (size_t)N * sizeof(double));
}

// Twisted elimination (two workgroups per sub-domain) from this many
// unknowns: below, one workgroup's sequential steps are cheap and the extra
// launches would cost more than they save.
constexpr int64_t kTwistedMinN = 225;

// The dynamic LDS limits of the separator and back-substitution kernels,
// raised once per device to what the largest band needs (not at every
// launch: launches may be recorded into a graph).
static hipError_t lds_limits_once() {
    static std::mutex mu;
    static bool done[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    if (dev >= 0 && dev < 64 && done[dev]) return hipSuccess;
    const int qmax = kMaxP1 - 1;
    const size_t sep = ((size_t)qmax * qmax + 2 * qmax) * sizeof(double);
    const size_t back = ((size_t)2 * kBackRows * back_stride(kMaxP1) + 512 + 4 * kBackRows) * sizeof(double);
    if ((e = hipFuncSetAttribute((const void *)separator_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)sep)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)back_block_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)back)) != hipSuccess)
        return e;
    if (dev >= 0 && dev < 64) done[dev] = true;
    return hipSuccess;
}

// Elimination, separator and back substitution of every sub-domain.
static hipError_t launch_elimination(const SubArgs &a, int blocks, hipStream_t s) {
    const int P1 = a.qf + 1;
    const unsigned nwg = (unsigned)(a.twisted ? 2 * blocks : blocks);
    hipError_t e = lds_limits_once();
    if (e != hipSuccess) return e;
    auto separator = [&]() -> hipError_t {
        const size_t lds = ((size_t)a.qf * a.qf + 2 * a.qf) * sizeof(double);
        hipLaunchKernelGGL(separator_kernel, dim3((unsigned)blocks), dim3(256), lds, s, a);
        return hipGetLastError();
    };
    // windows up to 32: one wavefront per elimination, the back
    // substitution in the kernel or one wavefront per end
    auto wave = [&](auto lu, auto back) -> hipError_t {
        hipLaunchKernelGGL(lu, dim3(nwg), dim3(64), 0, s, a);
        hipError_t r = hipGetLastError();
        if (r != hipSuccess || !a.twisted) return r;
        if ((r = separator()) != hipSuccess) return r;
        hipLaunchKernelGGL(back, dim3(nwg), dim3(64), 0, s, a);
        return hipGetLastError();
    };
#define FK_WAVE(P)                                                                                    \
    case P:                                                                                           \
        return a.twisted ? wave(subdomain_lu_wave_kernel<P, true>, twisted_back_wave_kernel<P>)       \
                         : wave(subdomain_lu_wave_kernel<P, false>, twisted_back_wave_kernel<P>);
    switch (P1) {
        FK_WAVE(8)
        FK_WAVE(12)
        FK_WAVE(16)
        FK_WAVE(20)
        FK_WAVE(24)
        FK_WAVE(32)
    default: break;
    }
#undef FK_WAVE
    // any other band: the tile kernel, its window at least q + 16 wide
    const int T = (a.qf + 16 + 15) / 16;
    switch (T) {
    case 2: hipLaunchKernelGGL(subdomain_lu_tile_kernel<2>, dim3(nwg), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(subdomain_lu_tile_kernel<3>, dim3(nwg), dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL(subdomain_lu_tile_kernel<4>, dim3(nwg), dim3(256), 0, s, a); break;
    case 5: hipLaunchKernelGGL(subdomain_lu_tile_kernel<5>, dim3(nwg), dim3(256), 0, s, a); break;
    case 6: hipLaunchKernelGGL(subdomain_lu_tile_kernel<6>, dim3(nwg), dim3(256), 0, s, a); break;
    case 7: hipLaunchKernelGGL(subdomain_lu_tile_kernel<7>, dim3(nwg), dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL(subdomain_lu_tile_kernel<8>, dim3(nwg), dim3(256), 0, s, a); break;
    case 9: hipLaunchKernelGGL(subdomain_lu_tile_kernel<9>, dim3(nwg), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.twisted && (e = separator()) != hipSuccess) return e;
    const size_t lds = ((size_t)2 * kBackRows * back_stride(P1) + 512 + 4 * kBackRows) * sizeof(double);
    hipLaunchKernelGGL(back_block_kernel, dim3(nwg), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace fk

using namespace fk;

extern "C" {

size_t subdomain_workspace_bytes_rect(int32_t px, int32_t py, int32_t n_cells) {
    if (px < 1 || py < 1 || n_cells < 2 || n_cells > 65535 || n_cells % px || n_cells % py) return 0;
    const SubGeom g = sub_geom(px, py, n_cells);
    if (g.mx < 2 || g.my < 2 || g.qf >= kMaxP1) return 0;
    return sub_ws_bytes(g, n_cells);
}

size_t subdomain_workspace_bytes(int32_t px, int32_t m) {
    if (px < 1 || m < 2 || (int64_t)px * m > 65535) return 0;
    return subdomain_workspace_bytes_rect(px, px, px * m);
}

int subdomain_solve_rect(const fk_density *w, double t_w, double dt_mesh, int32_t px, int32_t py, int32_t n_cells,
                         int32_t bdry_kind, const double *xi_n, const double *eta_n, const double *iface_xi,
                         const double *iface_eta, double *xi_out, double *eta_out, void *workspace,
                         size_t workspace_bytes, hipStream_t stream) {
    g_last_error.clear();
    int rc;
    if ((rc = validate_density(w)) != FK_OK) return rc;
    if (px < 1 || py < 1 || n_cells < 2 || n_cells > 65535)
        return fail(FK_E_INVAL, "need px >= 1, py >= 1 and 2 <= n_cells <= 65535");
    if (n_cells % px || n_cells % py) return fail(FK_E_INVAL, "px and py must divide n_cells");
    const SubGeom geo = sub_geom(px, py, n_cells);
    if (geo.mx < 2 || geo.my < 2) return fail(FK_E_INVAL, "sub-domains need at least 2 cells a side");
    if (geo.qf >= kMaxP1)
        return fail(FK_E_UNSUPPORTED, "the shorter sub-domain side must be <= %d cells", kMaxP1);
    const bool steady = std::isinf(dt_mesh) && dt_mesh > 0.0;
    if (!std::isfinite(t_w) || std::isnan(dt_mesh) || !(dt_mesh > 0.0))
        return fail(FK_E_INVAL, "t_w must be finite and dt_mesh > 0 (or +inf: the steady solve)");
    if (bdry_kind != FK_DATA_IDENTITY && bdry_kind != FK_DATA_ZERO && bdry_kind != FK_DATA_EQUIDISTRIBUTED)
        return fail(FK_E_INVAL, "outer boundary data must be FK_DATA_IDENTITY, _ZERO or _EQUIDISTRIBUTED");
    const int N = n_cells;
    const int64_t n_iface = geo.n_iface;
    if ((!steady && (!xi_n || !eta_n)) || !xi_out || !eta_out || (n_iface > 0 && (!iface_xi || !iface_eta)))
        return fail(FK_E_INVAL, "NULL array");
    const size_t need = sub_ws_bytes(geo, N);
    if (!workspace || workspace_bytes < need) return fail(FK_E_NOMEM, "workspace too small: need %zu bytes", need);
    if (((uintptr_t)workspace & 255u) != 0) return fail(FK_E_INVAL, "workspace must be 256-byte aligned");
    const double h = 1.0 / N;
    if (w->kind == FK_DENSITY_GRID && w->grid_n != N)
        return fail(FK_E_INVAL, "a grid density must be sampled on the mesh grid (grid_n %d != N %d)", w->grid_n, N);
    // Diagonal dominance (LU without pivoting) needs |b| h / 2 < 1.  For one
    // bump |b| = (2A/s2) r e / (1 + A e), e = exp(-r^2/s2), maximised over r
    // on a fine sample; two bumps are bounded by twice that.  For the ring
    // |b| = 2 A |beta| r e / (1 + A e), e = exp(beta |r^2 - 1/100|), over r
    // up to the square's diagonal.
    if (w->kind == FK_DENSITY_RING) {
        double bmax = 0.0;
        const double A = w->amp, be = w->width2;
        for (int i = 1; i <= 20000; ++i) {
            const double r = 1.5 * i / 20000.0, e = std::exp(be * std::fabs(r * r - 0.01));
            bmax = std::max(bmax, 2.0 * A * std::fabs(be) * r * e / (1.0 + A * e));
        }
        if (bmax * h / 2.0 >= 1.0) return fail(FK_E_UNSUPPORTED, "grid too coarse for the drift (|b| h / 2 >= 1)");
    } else if (w->kind != FK_DENSITY_CONST && w->kind != FK_DENSITY_GRID) {
        double bmax = 0.0;
        const double A = std::fabs(w->amp), s2 = w->width2, rs = 4.0 * std::sqrt(s2);
        for (int i = 1; i <= 4000; ++i) {
            const double r = rs * i / 4000.0, e = std::exp(-r * r / s2);
            bmax = std::max(bmax, 2.0 * A / s2 * r * e / (1.0 - (w->amp < 0 ? A : -A) * e));
        }
        if (w->kind == FK_DENSITY_TWO_BUMPS) bmax *= 2.0;
        if (bmax * h / 2.0 >= 1.0) return fail(FK_E_UNSUPPORTED, "grid too coarse for the drift (|b| h / 2 >= 1)");
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(FK_E_NODEVICE, "no HIP device: %s", hipGetErrorString(e));

    SubArgs a{};
    a.xi_n = xi_n;
    a.eta_n = eta_n;
    a.xi_out = xi_out;
    a.eta_out = eta_out;
    const size_t n = (size_t)geo.n;
    const size_t blocks = (size_t)px * py;
    char *ws = (char *)workspace;
    a.ustride = u_stride(geo.qf);
    a.ubuf = (double *)ws;
    ws += align256(blocks * n * (size_t)a.ustride * sizeof(double));
    a.ybuf = (double *)ws;
    ws += align256(blocks * 2 * n * sizeof(double));
    a.cbuf = (double *)ws;
    ws += align256(2 * blocks * 4 * n * sizeof(double));
    a.rbuf = (double *)ws;
    ws += align256(2 * blocks * 2 * n * sizeof(double));
    a.sbuf = (double *)ws;
    ws += align256(blocks * sep_stride(geo.qf) * sizeof(double));
    double *edge_cells = (double *)ws;
    a.N = N;
    a.px = px;
    a.py = py;
    a.mx = geo.mx;
    a.my = geo.my;
    a.qf = geo.qf;
    a.qs = geo.qs;
    a.xfast = geo.xfast;
    // steady: the rows divided by D (D -> inf) -- no identity term, no
    // previous values -- and scaled by h^2
    a.steady = steady ? 1 : 0;
    a.diag0 = steady ? 0.0 : 1.0;
    a.c = steady ? 1.0 : dt_mesh / (h * h);
    a.half_d_over_h = steady ? 0.5 * h : dt_mesh / (2.0 * h);
    a.kind = w->kind;
    a.amp = w->amp;
    a.width2 = w->width2;
    a.cx = w->cx;
    a.cy = w->cy;
    a.orbit_r = w->orbit_r;
    a.omega = w->omega;
    a.t_w = t_w;
    a.wg = w->kind == FK_DENSITY_GRID ? w->grid_w : nullptr;
    if (bdry_kind == FK_DATA_EQUIDISTRIBUTED) {
        hipLaunchKernelGGL(edge_cells_kernel, dim3((unsigned)((4 * N + 3) / 4)), dim3(256), 0, stream, a,
                           edge_cells);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "edge integral kernel launch");
    }
    const int64_t nthr = 4 * (int64_t)N + n_iface;
    hipLaunchKernelGGL(dirichlet_kernel, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, stream, a, iface_xi,
                       iface_eta, n_iface, (int)bdry_kind, (const double *)edge_cells, xi_out, eta_out);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "dirichlet kernel launch");
    // two workgroups per sub-domain, meeting at the slow line qs/2
    a.twisted = (geo.n >= kTwistedMinN && geo.qs >= 3) ? 1 : 0;
    a.sep = (geo.qs / 2) * geo.qf;
    if ((e = launch_elimination(a, (int)blocks, stream)) != hipSuccess) return hip_fail(e, "sub-domain kernel launch");
    return FK_OK;
}

int subdomain_solve(const fk_density *w, double t_w, double dt_mesh, int32_t px, int32_t m, int32_t bdry_kind,
                    const double *xi_n, const double *eta_n, const double *iface_xi, const double *iface_eta,
                    double *xi_out, double *eta_out, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (px < 1 || m < 2) return fail(FK_E_INVAL, "need px >= 1 and m >= 2");
    if ((int64_t)px * m > 65535) return fail(FK_E_INVAL, "grid too large (px m > 65535)");
    return subdomain_solve_rect(w, t_w, dt_mesh, px, px, px * m, bdry_kind, xi_n, eta_n, iface_xi, iface_eta, xi_out,
                                eta_out, workspace, workspace_bytes, stream);
}

size_t fk_boundary_workspace_bytes(int32_t n) {
    if (n < 2 || n > 65535) return 0;
    return align256((size_t)4 * n * sizeof(double));
}

int fk_boundary_data(const fk_density *w, double t_w, int32_t n, int32_t bdry_kind, double *xi_out, double *eta_out,
                     void *workspace, size_t workspace_bytes, hipStream_t stream) {
    g_last_error.clear();
    int rc;
    if ((rc = validate_density(w)) != FK_OK) return rc;
    if (n < 2 || n > 65535) return fail(FK_E_INVAL, "need 2 <= n <= 65535");
    if (!std::isfinite(t_w)) return fail(FK_E_INVAL, "t_w is not finite");
    if (bdry_kind != FK_DATA_IDENTITY && bdry_kind != FK_DATA_ZERO && bdry_kind != FK_DATA_EQUIDISTRIBUTED)
        return fail(FK_E_INVAL, "outer boundary data must be FK_DATA_IDENTITY, _ZERO or _EQUIDISTRIBUTED");
    if (w->kind == FK_DENSITY_GRID && w->grid_n != n)
        return fail(FK_E_INVAL, "a grid density must be sampled on this grid (grid_n %d != n %d)", w->grid_n, n);
    if (!xi_out || !eta_out) return fail(FK_E_INVAL, "NULL array");
    const size_t need = fk_boundary_workspace_bytes(n);
    if (bdry_kind == FK_DATA_EQUIDISTRIBUTED) {
        if (!workspace || workspace_bytes < need) return fail(FK_E_NOMEM, "workspace too small: need %zu bytes", need);
        if (((uintptr_t)workspace & 255u) != 0) return fail(FK_E_INVAL, "workspace must be 256-byte aligned");
    }
    SubArgs a{};
    a.xi_out = xi_out;
    a.eta_out = eta_out;
    a.N = n;
    a.px = a.py = 1;
    a.mx = a.my = n;
    a.kind = w->kind;
    a.amp = w->amp;
    a.width2 = w->width2;
    a.cx = w->cx;
    a.cy = w->cy;
    a.orbit_r = w->orbit_r;
    a.omega = w->omega;
    a.t_w = t_w;
    a.wg = w->kind == FK_DENSITY_GRID ? w->grid_w : nullptr;
    double *edge_cells = (double *)workspace;
    hipError_t e;
    if (bdry_kind == FK_DATA_EQUIDISTRIBUTED) {
        hipLaunchKernelGGL(edge_cells_kernel, dim3((unsigned)((4 * n + 3) / 4)), dim3(256), 0, stream, a,
                           edge_cells);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "edge integral kernel launch");
    }
    hipLaunchKernelGGL(dirichlet_kernel, dim3((unsigned)((4 * n + 255) / 256)), dim3(256), 0, stream, a,
                       (const double *)nullptr, (const double *)nullptr, (int64_t)0, (int)bdry_kind,
                       (const double *)edge_cells, xi_out, eta_out);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "boundary kernel launch");
    return FK_OK;
}

int fk_density_sample(const fk_density *w, double tau, int32_t n, double *w_out, hipStream_t stream) {
    g_last_error.clear();
    int rc;
    if ((rc = validate_density(w)) != FK_OK) return rc;
    if (w->kind == FK_DENSITY_GRID) return fail(FK_E_INVAL, "fk_density_sample takes an analytic density");
    if (n < 1 || n > 65535 || !w_out) return fail(FK_E_INVAL, "need 1 <= n <= 65535 and a non-NULL output");
    if (!std::isfinite(tau)) return fail(FK_E_INVAL, "tau is not finite");
    SubArgs a{};
    a.kind = w->kind;
    a.amp = w->amp;
    a.width2 = w->width2;
    a.cx = w->cx;
    a.cy = w->cy;
    a.orbit_r = w->orbit_r;
    a.omega = w->omega;
    a.t_w = tau;
    const int64_t total = (int64_t)(n + 1) * (n + 1);
    hipLaunchKernelGGL(density_sample_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, a, (int)n,
                       w_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FK_OK : hip_fail(e, "density sample kernel launch");
}

int fk_density_grid_drift(const double *grid_w, int32_t n, float *grid_b, hipStream_t stream) {
    g_last_error.clear();
    if (n < 2 || n > 65535 || !grid_w || !grid_b) return fail(FK_E_INVAL, "need 2 <= n <= 65535 and non-NULL arrays");
    if (((uintptr_t)grid_b & 7u) != 0) return fail(FK_E_INVAL, "grid_b must be 8-byte aligned");
    const int64_t total = (int64_t)(n + 1) * (n + 1);
    hipLaunchKernelGGL(grid_drift_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, grid_w,
                       (int)n, (float2 *)grid_b);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FK_OK : hip_fail(e, "grid drift kernel launch");
}

int fk_mesh_quality(const double *xi, const double *eta, int32_t n, double *out, hipStream_t stream) {
    g_last_error.clear();
    if (n < 1 || !xi || !eta || !out) return fail(FK_E_INVAL, "need n >= 1 and non-NULL arrays");
    if (((uintptr_t)out & 7u) != 0) return fail(FK_E_INVAL, "out must be 8-byte aligned");
    unsigned long long *keys = reinterpret_cast<unsigned long long *>(out);
    const int64_t cells = (int64_t)n * n;
    const int blocks = (int)std::min<int64_t>((cells + kQualityBlock - 1) / kQualityBlock, 2048);
    hipLaunchKernelGGL(quality_init_kernel, dim3(1), dim3(64), 0, stream, keys);
    hipLaunchKernelGGL(quality_kernel, dim3(blocks), dim3(kQualityBlock), 0, stream, xi, eta, n, keys);
    hipLaunchKernelGGL(quality_final_kernel, dim3(1), dim3(64), 0, stream, keys);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FK_OK : hip_fail(e, "quality kernel launch");
}

}  // extern "C"
