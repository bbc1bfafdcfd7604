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
// MI355X mapping: one workgroup per sub-domain.  With the q x q interior
// unknowns in row-major order the matrix is banded with half-bandwidth
// p = q, and the fill of the LU stays in the band; elimination step k only
// touches rows and columns k..k+p, and the new row and column that enter
// the (p+1)^2 window carry their original stencil values (at most five
// non-zeros).  Both right-hand sides (xi and eta) are eliminated with the
// same multipliers.  For the sub-domain sizes it is built for, the window
// lives in registers, one column per thread (subdomain_lu_kernel); other
// sizes keep it in LDS, indexed circularly (subdomain_be_kernel).  Finished U
// rows go to the workspace; one wavefront then back-substitutes, prefetching
// the next U row while it reduces the current one.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "fk.h"
#include "fk_internal.hpp"

namespace fk {

struct SubArgs {
    const double *xi_n, *eta_n;  // previous mesh, (N+1)^2
    double *xi_out, *eta_out;    // Dirichlet data pre-filled; interior written
    double *ubuf;                // per sub-domain: n * (p+1) doubles
    double *ybuf;                // per sub-domain: 2 n doubles
    double *cbuf;                // per sub-domain: 4 n doubles, (E, W, N, S) coefficients of each row
    double *rbuf;                // per sub-domain: 2 n doubles, right-hand sides (xi, eta) of each row
    int N, m, px;
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

constexpr int kB = 32;   // steps per staging batch of the register-window kernel

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
    const int N1 = a.N + 1;
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
                const int r = rev ? n - 1 - k : k;
                const int ii = r % q, jj = r / q;
                const int64_t g = (int64_t)(j0 + 1 + jj) * N1 + (i0 + 1 + ii);
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
// n-1-r, east <-> west, north <-> south), by the threads of the workgroup.
__device__ void assemble_rows(const SubArgs &a, int n, int q, int i0, int j0, bool rev, double4 *cf, double2 *rh) {
    const int N1 = a.N + 1;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const int ii = r % q, jj = r / q;
        const int gi = i0 + 1 + ii, gj = j0 + 1 + jj;
        double bx, by;
        node_drift_f64(a, gi, gj, bx, by);
        const double cxr = a.half_d_over_h * bx, cyr = a.half_d_over_h * by;
        const double cE = -a.c - cxr, cW = -a.c + cxr, cN = -a.c - cyr, cS = -a.c + cyr;
        const int64_t g = (int64_t)gj * N1 + gi;
        double fx = a.steady ? 0.0 : a.xi_n[g], fy = a.steady ? 0.0 : a.eta_n[g];
        if (ii == q - 1) { fx -= cE * a.xi_out[g + 1]; fy -= cE * a.eta_out[g + 1]; }
        if (ii == 0) { fx -= cW * a.xi_out[g - 1]; fy -= cW * a.eta_out[g - 1]; }
        if (jj == q - 1) { fx -= cN * a.xi_out[g + N1]; fy -= cN * a.eta_out[g + N1]; }
        if (jj == 0) { fx -= cS * a.xi_out[g - N1]; fy -= cS * a.eta_out[g - N1]; }
        const double e = ii < q - 1 ? cE : 0.0, w = ii > 0 ? cW : 0.0;
        const double nn = jj < q - 1 ? cN : 0.0, ss = jj > 0 ? cS : 0.0;
        cf[rev ? n - 1 - r : r] = rev ? make_double4(w, e, ss, nn) : make_double4(e, w, nn, ss);
        rh[rev ? n - 1 - r : r] = make_double2(fx, fy);
    }
}

// Original matrix entry (r, c) of an assembled system; identity beyond n.
__device__ __forceinline__ double band_entry(const double4 *cf, int n, int q, double diag, int r, int c) {
    if (r >= n || c >= n) return r == c ? 1.0 : 0.0;
    const int d = c - r;
    if (d == 0) return diag;
    if (d != 1 && d != -1 && d != q && d != -q) return 0.0;
    const double4 f = cf[r];
    return d == 1 ? f.x : d == -1 ? f.y : d == q ? f.z : f.w;
}

// Banded LU with the window in registers.  For P1 = q + 1 the window of
// elimination step k is rows and columns k .. k + q.  Column slot t < P1
// holds the columns c = t (mod P1), split over two lanes: the upper lane
// keeps window rows 0 .. H-1 (H = P1/2) in v[0 .. H-1], the lower lane rows
// H .. P1-1; four more lanes hold the two right-hand sides the same way.
// Step k: the two lanes of the pivot column's slot write it to LDS (1/pivot
// in place of the pivot), every upper lane publishes its row-k entry u and
// every lower lane its first row, then one barrier; each lane updates and
// shifts its rows in one pass,
//   v[i] = v[i + 1] - pivotcol[i + 1] * (u / pivot),
// the upper lane's last row taking the lower lane's first, the lower lane's
// last row taking the original entry of the row k + P1 that enters.  The
// pivot column becomes exactly zero and its slot takes the entering column
// k + P1: non-zero only in rows k + 1 (north neighbour), k + q (east
// neighbour) and k + P1 (diagonal).  LDS buffers alternate between steps, so
// one barrier per step suffices; every register index is a compile-time
// constant.  Rows and columns beyond n are identity padding.
template <int P1>
__global__ void __launch_bounds__(256) subdomain_lu_kernel(const SubArgs a) {
    constexpr int q = P1 - 1, H = P1 / 2;
    static_assert(P1 % 2 == 0 && H >= 2, "even window of at least 4");
    __shared__ __align__(16) double Vs[2][P1];   // pivot column, 1/pivot first
    __shared__ double Us[2][P1 + 2];    // row-k entry of every column and rhs
    __shared__ double Ls[2][P1 + 2];    // first lower row of every column and rhs
    __shared__ double Ust[2][kB][P1];   // U rows of a batch
    __shared__ double2 Yst[2][kB];      // y values (xi, eta) of a batch
    __shared__ double4 Cst[2][kB];      // coefficients of the entering rows R
    __shared__ double2 Rst[2][kB];      // right-hand sides of the entering rows R
    __shared__ double Nst[2][kB];       // north coefficients of the rows k + 1
    const int n = q * q;
    const int sd = a.twisted ? blockIdx.x >> 1 : blockIdx.x;   // sub-domain
    const bool rev = a.twisted && (blockIdx.x & 1);           // the reversed (bottom) end
    const int si = sd % a.px, sj = sd / a.px;
    const int i0 = si * a.m, j0 = sj * a.m;
    const int N1 = a.N + 1;
    // rows eliminated here, and where this end's U rows and y values go
    const int steps = !a.twisted ? n : (rev ? n - a.sep - q : a.sep);
    const int off = rev ? a.sep : 0;
    double *U = a.ubuf + (int64_t)sd * n * P1 + (int64_t)off * P1;
    double *Y = a.ybuf + (int64_t)sd * 2 * n + off;
    const int64_t cix = a.twisted ? 2 * (int64_t)sd + (rev ? 1 : 0) : sd;
    double4 *cf = reinterpret_cast<double4 *>(a.cbuf + cix * 4 * n);
    double2 *rh = reinterpret_cast<double2 *>(a.rbuf + cix * 2 * n);
    const int tid = threadIdx.x;

    // ---- every row's coefficients (Dirichlet neighbours moved to the rhs) --
    for (int r = tid; r < n; r += blockDim.x) {
        const int ii = r % q, jj = r / q;
        const int gi = i0 + 1 + ii, gj = j0 + 1 + jj;
        double bx, by;
        node_drift_f64(a, gi, gj, bx, by);
        const double cxr = a.half_d_over_h * bx, cyr = a.half_d_over_h * by;
        const double cE = -a.c - cxr, cW = -a.c + cxr, cN = -a.c - cyr, cS = -a.c + cyr;
        const int64_t g = (int64_t)gj * N1 + gi;
        double fx = a.steady ? 0.0 : a.xi_n[g], fy = a.steady ? 0.0 : a.eta_n[g];
        if (ii == q - 1) { fx -= cE * a.xi_out[g + 1]; fy -= cE * a.eta_out[g + 1]; }
        if (ii == 0) { fx -= cW * a.xi_out[g - 1]; fy -= cW * a.eta_out[g - 1]; }
        if (jj == q - 1) { fx -= cN * a.xi_out[g + N1]; fy -= cN * a.eta_out[g + N1]; }
        if (jj == 0) { fx -= cS * a.xi_out[g - N1]; fy -= cS * a.eta_out[g - N1]; }
        const double e = ii < q - 1 ? cE : 0.0, w = ii > 0 ? cW : 0.0;
        const double nn = jj < q - 1 ? cN : 0.0, ss = jj > 0 ? cS : 0.0;
        // the reversed system: row n-1-r, east <-> west, north <-> south
        cf[rev ? n - 1 - r : r] = rev ? make_double4(w, e, ss, nn) : make_double4(e, w, nn, ss);
        rh[rev ? n - 1 - r : r] = make_double2(fx, fy);
    }
    __threadfence_block();
    __syncthreads();

    const double diag = a.diag0 + 4.0 * a.c;
    // original matrix entry (r, c); identity beyond n
    auto entry = [&](int r, int c) -> double {
        if (r >= n || c >= n) return r == c ? 1.0 : 0.0;
        const int d = c - r;
        if (d == 0) return diag;
        if (d != 1 && d != -1 && d != q && d != -q) return 0.0;
        const double4 f = cf[r];
        return d == 1 ? f.x : d == -1 ? f.y : d == q ? f.z : f.w;
    };
    // roles: column slot / right-hand side, and which half of the rows
    const bool is_col = tid < 2 * P1;
    const bool is_rhs = !is_col && tid < 2 * P1 + 4;
    const int slot = is_col ? tid % P1 : 0;
    const int rhs_c = is_rhs ? (tid - 2 * P1) & 1 : 0;            // 0: xi, 1: eta
    const bool lower = is_col ? tid >= P1 : (is_rhs && tid - 2 * P1 >= 2);
    const int pub = is_col ? slot : P1 + rhs_c;                    // index in Us / Ls
    const int r0 = lower ? H : 0;                                  // first window row held
    int col = slot;
    double v[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        double e = 0.0;
        if (is_col) e = entry(r0 + i, col);
        else if (is_rhs && r0 + i < n) e = rhs_c == 0 ? rh[r0 + i].x : rh[r0 + i].y;
        v[i] = e;
    }

    // Per-step memory traffic goes through LDS in batches of kB steps, so no
    // step waits on global memory: the coefficients of the rows that enter
    // (row R = k + P1: west, south, east and rhs; row k + 1: north) are
    // loaded a batch ahead by the first kB lanes and staged in LDS; the U rows
    // and y values a batch produces are staged in LDS and written out by the
    // whole workgroup, coalesced, at the next batch boundary.
    const int nb = (n + kB - 1) / kB;
    auto load_batch = [&](int bt, double4 &c4, double2 &r2, double &cn) {
        const int j = tid, kk = bt * kB + j, R = kk + P1;
        const bool ok = tid < kB && bt < nb;
        c4 = (ok && R < n) ? cf[R] : make_double4(0.0, 0.0, 0.0, 0.0);
        r2 = (ok && R < n) ? rh[R] : make_double2(0.0, 0.0);
        cn = (ok && kk + 1 < n) ? cf[kk + 1].z : 0.0;
    };
    double4 pc4;
    double2 pr2;
    double pcn;
    load_batch(0, pc4, pr2, pcn);
    const double cE_first = (P1 - 1 < n) ? cf[P1 - 1].x : 0.0;   // east coefficient of row P1 - 1

    int owner = 0;
    for (int k = 0; k < steps; ++k) {
        const int b = k & 1;
        const int R = k + P1;
        const int j = k % kB, bt = k / kB, bb = bt & 1;
        if (j == 0) {
            // batch boundary: stage this batch's coefficients, fetch the next
            if (tid < kB) {
                Cst[bb][tid] = pc4;
                Rst[bb][tid] = pr2;
                Nst[bb][tid] = pcn;
            }
            load_batch(bt + 1, pc4, pr2, pcn);
        }
        if (is_col || is_rhs) {
            if (lower) Ls[b][pub] = v[0];
            else Us[b][pub] = v[0];
        }
        if (is_col && slot == owner) {
            double2 *dst = reinterpret_cast<double2 *>(&Vs[b][r0]);
            dst[0] = make_double2(lower ? v[0] : 1.0 / v[0], v[1]);
#pragma unroll
            for (int i = 2; i < H; i += 2) dst[i / 2] = make_double2(v[i], (i + 1 < H) ? v[i + 1] : 0.0);
        }
        __syncthreads();
        if (j == 0 && bt > 0) {
            // write out the previous batch's U rows and y values
            const int kp = (bt - 1) * kB;
            const double *src = &Ust[bb ^ 1][0][0];
            double *dstU = U + (int64_t)kp * P1;
            for (int e = tid; e < kB * P1; e += blockDim.x) dstU[e] = src[e];
            if (tid < kB) {
                Y[kp + tid] = Yst[bb ^ 1][tid].x;
                Y[n + kp + tid] = Yst[bb ^ 1][tid].y;
            }
        }
        if (is_col || is_rhs) {
            const double u = lower ? Us[b][pub] : v[0];
            if (!lower) {
                if (is_col) Ust[bb][j][col - k] = u;
                else if (rhs_c == 0) Yst[bb][j].x = u;
                else Yst[bb][j].y = u;
            }
            // the pivot column itself: scale exactly 1, so it becomes exactly zero
            const double sc = (is_col && slot == owner) ? 1.0 : u * Vs[b][0];
            const double nxt = lower ? 0.0 : Ls[b][pub];        // the row below the upper half
#pragma unroll
            for (int i = 0; i < H - 1; ++i) {
                if (i % 16 == 0) asm volatile("" ::: "memory");
                v[i] = fma(-Vs[b][r0 + i + 1], sc, v[i + 1]);
            }
            const bool live = R < n;
            if (!lower) {
                v[H - 1] = fma(-Vs[b][H], sc, nxt);
                if (is_col && slot == owner) {
                    v[0] = live ? Nst[bb][j] : 0.0;                        // entering column, row k + 1
                    col = R;
                }
            } else if (is_col) {
                if (slot == owner) {
                    col = R;
                    // row R - 1: the east coefficient of the row that entered
                    // one step earlier (staged in the previous step's slot)
                    const int kp = k - 1;
                    const double cE = k == 0 ? cE_first : Cst[(kp / kB) & 1][kp % kB].x;
                    v[H - 2] = live ? cE : 0.0;
                    v[H - 1] = live ? diag : 1.0;                          // row R
                } else {
                    const double4 cR = Cst[bb][j];
                    v[H - 1] = (live && col < n) ? (col == R - 1 ? cR.y : (col == R - q ? cR.w : 0.0)) : 0.0;
                }
            } else {
                v[H - 1] = rhs_c == 0 ? Rst[bb][j].x : Rst[bb][j].y;
            }
        }
        owner = (owner + 1 == P1) ? 0 : owner + 1;
    }
    __syncthreads();
    {
        // the last batch
        const int bt = (steps - 1) / kB, bb = bt & 1, kp = bt * kB, cnt = steps - kp;
        const double *src = &Ust[bb][0][0];
        double *dstU = U + (int64_t)kp * P1;
        for (int e = tid; e < cnt * P1; e += blockDim.x) dstU[e] = src[e];
        if (tid < cnt) {
            Y[kp + tid] = Yst[bb][tid].x;
            Y[n + kp + tid] = Yst[bb][tid].y;
        }
    }
    if (a.twisted) {
        // the separator block of the trailing window (window rows and columns
        // 0 .. q-1 are this end's separator rows) and its right-hand sides
        double *S = a.sbuf + (int64_t)sd * sep_stride(q) + (rev ? (size_t)q * q + 2 * q : 0);
        if (is_col) {
            const int c = col - steps;
#pragma unroll
            for (int i = 0; i < H; ++i)
                if (r0 + i < q && c < q) S[(r0 + i) * q + c] = v[i];
        } else if (is_rhs) {
#pragma unroll
            for (int i = 0; i < H; ++i)
                if (r0 + i < q) S[(size_t)q * q + rhs_c * q + r0 + i] = v[i];
        }
        return;
    }
    __threadfence_block();
    __syncthreads();
    if (tid < 64) back_substitute_blocked<P1>(a, U, Y, n, n - 1, i0, j0, nullptr, false);
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
    __shared__ double Nst[2][kW];    // north coefficients of the rows k + 1
    const int n = q * q;
    const int sd = TW ? blockIdx.x >> 1 : blockIdx.x;
    const bool rev = TW && (blockIdx.x & 1);
    const int si = sd % a.px, sj = sd / a.px;
    const int i0 = si * a.m, j0 = sj * a.m;
    const int steps = !TW ? n : (rev ? n - a.sep - q : a.sep);
    const int off = rev ? a.sep : 0;
    double *U = a.ubuf + (int64_t)sd * n * P1 + (int64_t)off * P1;
    double *Y = a.ybuf + (int64_t)sd * 2 * n + off;
    const int64_t cix = TW ? 2 * (int64_t)sd + (rev ? 1 : 0) : sd;
    double4 *cf = reinterpret_cast<double4 *>(a.cbuf + cix * 4 * n);
    double2 *rh = reinterpret_cast<double2 *>(a.rbuf + cix * 2 * n);
    const int lane = threadIdx.x;

    assemble_rows(a, n, q, i0, j0, rev, cf, rh);
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
    const int q = a.m - 1, n = q * q, sd = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int si = sd % a.px, sj = sd / a.px;
    const int i0 = si * a.m, j0 = sj * a.m, N1 = a.N + 1;
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
    for (int k = 0; k < q; ++k) {
        const double inv = 1.0 / M[k * q + k];
        const int w = q - 1 - k + 2;   // columns k+1 .. q-1, then the two right-hand sides
        for (int e = tid; e < (q - 1 - k) * w; e += nt) {
            const int i = k + 1 + e / w, jj = e % w;
            const double l = M[i * q + k] * inv;
            if (jj < q - 1 - k) {
                const int j = k + 1 + jj;
                M[i * q + j] = fma(-l, M[k * q + j], M[i * q + j]);
            } else {
                const int comp = jj - (q - 1 - k);
                b[comp * q + i] = fma(-l, b[comp * q + k], b[comp * q + i]);
            }
        }
        __syncthreads();
    }
    for (int k = q - 1; k >= 0; --k) {
        if (tid < 2) b[tid * q + k] = b[tid * q + k] / M[k * q + k];
        __syncthreads();
        for (int e = tid; e < 2 * k; e += nt) {
            const int comp = e / k, i = e % k;
            b[comp * q + i] = fma(-M[i * q + k], b[comp * q + k], b[comp * q + i]);
        }
        __syncthreads();
    }
    const int jj = a.sep / q;
    for (int e = tid; e < 2 * q; e += nt) {
        const int comp = e / q, r = e % q;
        xs[e] = b[e];
        const int64_t g = (int64_t)(j0 + 1 + jj) * N1 + (i0 + 1 + r);
        (comp ? a.eta_out : a.xi_out)[g] = b[e];
    }
}

// Back substitution of each end of a twisted elimination, from the
// separator's values: one wavefront per (sub-domain, end).
template <int P1>
__global__ void __launch_bounds__(64) twisted_back_kernel(const SubArgs a) {
    constexpr int q = P1 - 1;
    const int n = q * q;
    const int sd = blockIdx.x >> 1;
    const bool rev = (blockIdx.x & 1) != 0;
    const int steps = rev ? n - a.sep - q : a.sep, off = rev ? a.sep : 0;
    const int si = sd % a.px, sj = sd / a.px;
    const double *U = a.ubuf + (int64_t)sd * n * P1 + (int64_t)off * P1;
    const double *Y = a.ybuf + (int64_t)sd * 2 * n + off;
    const double *xs = a.sbuf + (int64_t)sd * sep_stride(q) + 2 * ((size_t)q * q + 2 * q);
    back_substitute_blocked<P1>(a, U, Y, n, steps - 1, si * a.m, sj * a.m, xs, rev);
}


// The same for windows up to 32, a row at a time: lane l < q holds
// x_{k+l+1} (both components), each row's sum over them is a DPP reduction
// within the first 32 lanes, and the window shifts up by one lane (DPP wave
// shift).  U rows and y values are loaded kR rows ahead.
template <int P1>
__global__ void __launch_bounds__(64) twisted_back_wave_kernel(const SubArgs a) {
    constexpr int q = P1 - 1, kR = 8;
    static_assert(q <= 32, "the window fits the first 32 lanes");
    const int n = q * q;
    const int sd = blockIdx.x >> 1;
    const bool rev = (blockIdx.x & 1) != 0;
    const int steps = rev ? n - a.sep - q : a.sep, off = rev ? a.sep : 0;
    const int si = sd % a.px, sj = sd / a.px;
    const int i0 = si * a.m, j0 = sj * a.m, N1 = a.N + 1;
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
                const int rr = rev ? n - 1 - k : k;
                const int64_t g = (int64_t)(j0 + 1 + rr / q) * N1 + (i0 + 1 + rr % q);
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

__global__ void __launch_bounds__(256) subdomain_be_kernel(const SubArgs a) {
    extern __shared__ double lds[];
    const int q = a.m - 1, p = q, P1 = p + 1, n = q * q;
    const int si = blockIdx.x % a.px, sj = blockIdx.x / a.px;
    const int i0 = si * a.m, j0 = sj * a.m;
    const int N1 = a.N + 1;
    double *W = lds;                     // P1 x P1 window
    double *rx = W + P1 * P1;            // rhs ring, xi
    double *ry = rx + P1;                // rhs ring, eta
    double *kx = ry + P1;                // cx of the rows in the window
    double *ky = kx + P1;                // cy of the rows in the window
    double *U = a.ubuf + (int64_t)blockIdx.x * n * P1;
    double *Y = a.ybuf + (int64_t)blockIdx.x * 2 * n;
    const int tid = threadIdx.x, nth = blockDim.x;

    // Row r enters the window: its drift coefficients, its right-hand side
    // with the Dirichlet neighbours moved over, and its lower entries (W, S)
    // in window column coordinates relative to step k.
    auto row_enter = [&](int r, int k) {
        const int ii = r % q, jj = r / q;
        const int gi = i0 + 1 + ii, gj = j0 + 1 + jj;
        double bx, by;
        node_drift_f64(a, gi, gj, bx, by);
        const double cxr = a.half_d_over_h * bx, cyr = a.half_d_over_h * by;
        const int s = r % P1;
        kx[s] = cxr;
        ky[s] = cyr;
        const int64_t g = (int64_t)gj * N1 + gi;
        double fx = a.steady ? 0.0 : a.xi_n[g], fy = a.steady ? 0.0 : a.eta_n[g];
        const double cE = -a.c - cxr, cW = -a.c + cxr, cN = -a.c - cyr, cS = -a.c + cyr;
        if (ii == q - 1) { fx -= cE * a.xi_out[g + 1]; fy -= cE * a.eta_out[g + 1]; }
        if (ii == 0) { fx -= cW * a.xi_out[g - 1]; fy -= cW * a.eta_out[g - 1]; }
        if (jj == q - 1) { fx -= cN * a.xi_out[g + N1]; fy -= cN * a.eta_out[g + N1]; }
        if (jj == 0) { fx -= cS * a.xi_out[g - N1]; fy -= cS * a.eta_out[g - N1]; }
        rx[s] = fx;
        ry[s] = fy;
        double *row = W + s * P1;
        row[r % P1] = a.diag0 + 4.0 * a.c;
        if (ii > 0 && r - 1 >= k) row[(r - 1) % P1] = cW;
        if (jj > 0 && r - q >= k) row[(r - q) % P1] = cS;
    };

    // ---- initial window: rows and columns 0..p ------------------------------
    for (int e = tid; e < P1 * P1; e += nth) W[e] = 0.0;
    __syncthreads();
    for (int r = tid; r < P1 && r < n; r += nth) row_enter(r, 0);
    __syncthreads();
    // upper entries (E, N) of rows 0..p that fall inside the window
    for (int r = tid; r < P1 && r < n; r += nth) {
        const int ii = r % q, jj = r / q;
        double *row = W + (r % P1) * P1;
        if (ii < q - 1 && r + 1 <= p) row[(r + 1) % P1] = -a.c - kx[r % P1];
        if (jj < q - 1 && r + q <= p) row[(r + q) % P1] = -a.c - ky[r % P1];
    }
    __syncthreads();

    // ---- forward elimination ------------------------------------------------
    for (int k = 0; k < n; ++k) {
        const int s0 = k % P1;
        const double *prow = W + s0 * P1;
        const double inv = 1.0 / prow[s0];
        const int span = min(p, n - 1 - k);  // rows/cols below and right of the pivot
        // save the U row and the eliminated right-hand side of step k
        for (int c = tid; c <= p; c += nth) U[(int64_t)k * P1 + c] = (c <= span) ? prow[(k + c) % P1] : 0.0;
        if (tid == 0) {
            Y[k] = rx[s0];
            Y[n + k] = ry[s0];
        }
        // rank-1 update of the window, and the right-hand sides
        const int tot = span * span;
        for (int e = tid; e < tot; e += nth) {
            const int r = 1 + e / span, c = 1 + e % span;
            double *row = W + ((k + r) % P1) * P1;
            const double l = row[s0] * inv;
            row[(k + c) % P1] -= l * prow[(k + c) % P1];
        }
        for (int r = 1 + tid; r <= span; r += nth) {
            const int s = (k + r) % P1;
            const double l = W[s * P1 + s0] * inv;
            rx[s] -= l * rx[s0];
            ry[s] -= l * ry[s0];
        }
        __syncthreads();
        // slide: slot s0 becomes row / column k + P1
        const int R = k + P1;
        if (R < n) {
            for (int e = tid; e < P1; e += nth) {
                W[s0 * P1 + e] = 0.0;   // the new row
                W[e * P1 + s0] = 0.0;   // the new column
            }
            __syncthreads();
            if (tid == 0) row_enter(R, k + 1);
            if (tid == 1) {
                // new column entries: E of row R-1, N of row R-q
                const int r1 = R - 1, rq = R - q;
                if (r1 % q < q - 1) W[(r1 % P1) * P1 + s0] = -a.c - kx[r1 % P1];
                if (rq >= k + 1 && (rq / q) < q - 1) W[(rq % P1) * P1 + s0] = -a.c - ky[rq % P1];
            }
        }
        __syncthreads();
    }

    // ---- back substitution (one wavefront) ----------------------------------
    if (tid < 64) {
        double *xw = W;            // x ring (xi), reuse of the window storage
        double *yw = W + P1;       // x ring (eta)
        const int lane = tid;
        double u0 = 0.0, u1 = 0.0, ud = 1.0;
        int k = n - 1;
        // prefetch row n-1
        if (k >= 0) {
            u0 = (lane + 1 <= p) ? U[(int64_t)k * P1 + lane + 1] : 0.0;
            u1 = (lane + 65 <= p) ? U[(int64_t)k * P1 + lane + 65] : 0.0;
            ud = U[(int64_t)k * P1];
        }
        for (; k >= 0; --k) {
            double n0 = 0.0, n1 = 0.0, nd = 1.0;
            if (k > 0) {
                n0 = (lane + 1 <= p) ? U[(int64_t)(k - 1) * P1 + lane + 1] : 0.0;
                n1 = (lane + 65 <= p) ? U[(int64_t)(k - 1) * P1 + lane + 65] : 0.0;
                nd = U[(int64_t)(k - 1) * P1];
            }
            double sx = 0.0, sy = 0.0;
            if (lane + 1 <= p && k + lane + 1 < n) {
                sx += u0 * xw[(k + lane + 1) % P1];
                sy += u0 * yw[(k + lane + 1) % P1];
            }
            if (lane + 65 <= p && k + lane + 65 < n) {
                sx += u1 * xw[(k + lane + 65) % P1];
                sy += u1 * yw[(k + lane + 65) % P1];
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                sx += __shfl_xor(sx, off, 64);
                sy += __shfl_xor(sy, off, 64);
            }
            const double xk = (Y[k] - sx) / ud, yk = (Y[n + k] - sy) / ud;
            if (lane == 0) {
                xw[k % P1] = xk;
                yw[k % P1] = yk;
                const int ii = k % q, jj = k / q;
                const int64_t g = (int64_t)(j0 + 1 + jj) * N1 + (i0 + 1 + ii);
                a.xi_out[g] = xk;
                a.eta_out[g] = yk;
            }
            __builtin_amdgcn_wave_barrier();
            u0 = n0;
            u1 = n1;
            ud = nd;
        }
    }
}

// Dirichlet data of the output grids: outer boundary and interface nodes.
__global__ void dirichlet_kernel(const SubArgs a, const double *iface_xi, const double *iface_eta, int64_t n_iface,
                                 int bdry_kind, const double *edge_cells, double *xi_out, double *eta_out) {
    const int N = a.N, m = a.m, px = a.px;
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
    // horizontal lines y = c/px without the crossings
    const int64_t nv = (int64_t)(px - 1) * (N - 1);
    int i, j;
    if (f < nv) {
        i = (int)(f / (N - 1) + 1) * m;
        j = (int)(f % (N - 1)) + 1;
    } else {
        const int64_t h = f - nv;
        const int per = N - px;  // non-crossing nodes per horizontal line
        const int c = (int)(h / per) + 1;
        const int r = (int)(h % per);
        i = r + 1 + r / (m - 1);
        j = c * m;
    }
    const int64_t g = (int64_t)j * N1 + i;
    xi_out[g] = iface_xi[f];
    eta_out[g] = iface_eta[f];
}

// min Jacobian and max skewness over all cells (cell-centred differences).
__global__ void __launch_bounds__(1024) quality_kernel(const double *xi, const double *eta, int n, double *out) {
    const int N1 = n + 1;
    const double inv2h = 0.5 * n;
    double jmin = INFINITY, smax = 0.0;
    const int64_t cells = (int64_t)n * n;
    for (int64_t c = threadIdx.x; c < cells; c += blockDim.x) {
        const int i = (int)(c % n), j = (int)(c / n);
        const int64_t g = (int64_t)j * N1 + i;
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
    __shared__ double pj[16], ps[16];
    if ((threadIdx.x & 63) == 0) {
        pj[threadIdx.x >> 6] = jmin;
        ps[threadIdx.x >> 6] = smax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            jmin = fmin(jmin, pj[w]);
            smax = fmax(smax, ps[w]);
        }
        out[0] = jmin;
        out[1] = smax;
    }
}

// Workspace: U rows, y values, row coefficients and right-hand sides (two
// copies per sub-domain: natural and reversed order), the separator blocks,
// and the edge integrals.
static size_t sub_ws_bytes(int px, int m) {
    const size_t q = (size_t)m - 1, n = q * q, P1 = q + 1;
    const size_t blocks = (size_t)px * px, N = (size_t)px * m;
    return align256(blocks * n * P1 * sizeof(double)) + align256(blocks * 2 * n * sizeof(double)) +
           align256(2 * blocks * 4 * n * sizeof(double)) + align256(2 * blocks * 2 * n * sizeof(double)) +
           align256(blocks * sep_stride((int)q) * sizeof(double)) + align256(4 * N * sizeof(double));
}

// Sides from which the twisted elimination (two workgroups per sub-domain)
// is used: below, one workgroup's sequential steps are cheap and three
// launches would cost more than they save.
constexpr int kTwistedMinM = 16;

// Launch of the register-window kernel for the window widths it is built
// for; false if m is not one of them.
static bool launch_lu(const SubArgs &a, int blocks, hipStream_t s, hipError_t *err) {
    auto go = [&](auto kern, int P1) {
        const int threads = ((2 * P1 + 4 + 63) / 64) * 64;
        hipLaunchKernelGGL(kern, dim3((unsigned)(a.twisted ? 2 * blocks : blocks)), dim3(threads), 0, s, a);
        *err = hipGetLastError();
        return true;
    };
    auto wave = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((unsigned)(a.twisted ? 2 * blocks : blocks)), dim3(64), 0, s, a);
        *err = hipGetLastError();
        return true;
    };
    // windows up to 32: one wavefront per elimination (both ends when twisted)
    if (a.twisted) {
        switch (a.m) {
        case 16: return wave(subdomain_lu_wave_kernel<16, true>);
        case 20: return wave(subdomain_lu_wave_kernel<20, true>);
        case 24: return wave(subdomain_lu_wave_kernel<24, true>);
        case 32: return wave(subdomain_lu_wave_kernel<32, true>);
        default: break;
        }
    } else {
        switch (a.m) {
        case 8: return wave(subdomain_lu_wave_kernel<8, false>);
        case 12: return wave(subdomain_lu_wave_kernel<12, false>);
        default: break;
        }
    }
    switch (a.m) {
    case 8: return go(subdomain_lu_kernel<8>, 8);
    case 12: return go(subdomain_lu_kernel<12>, 12);
    case 16: return go(subdomain_lu_kernel<16>, 16);
    case 20: return go(subdomain_lu_kernel<20>, 20);
    case 24: return go(subdomain_lu_kernel<24>, 24);
    case 32: return go(subdomain_lu_kernel<32>, 32);
    case 40: return go(subdomain_lu_kernel<40>, 40);
    case 48: return go(subdomain_lu_kernel<48>, 48);
    case 64: return go(subdomain_lu_kernel<64>, 64);
    case 96: return go(subdomain_lu_kernel<96>, 96);
    default: return false;
    }
}

// The separator solves and the back substitutions of a twisted elimination.
static hipError_t launch_twisted_rest(const SubArgs &a, int blocks, hipStream_t s) {
    const int q = a.m - 1;
    const size_t lds = ((size_t)q * q + 2 * q) * sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void *)separator_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(separator_kernel, dim3((unsigned)blocks), dim3(256), lds, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    auto back = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((unsigned)(2 * blocks)), dim3(64), 0, s, a);
        return hipGetLastError();
    };
    switch (a.m) {
    case 16: return back(twisted_back_wave_kernel<16>);
    case 20: return back(twisted_back_wave_kernel<20>);
    case 24: return back(twisted_back_wave_kernel<24>);
    case 32: return back(twisted_back_wave_kernel<32>);
    case 40: return back(twisted_back_kernel<40>);
    case 48: return back(twisted_back_kernel<48>);
    case 64: return back(twisted_back_kernel<64>);
    case 96: return back(twisted_back_kernel<96>);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fk

using namespace fk;

extern "C" {

size_t subdomain_workspace_bytes(int32_t px, int32_t m) {
    if (px < 1 || m < 2 || m - 1 >= kMaxP1) return 0;
    return sub_ws_bytes(px, m);
}

int subdomain_solve(const fk_density *w, double t_w, double dt_mesh, int32_t px, int32_t m, int32_t bdry_kind,
                    const double *xi_n, const double *eta_n, const double *iface_xi, const double *iface_eta,
                    double *xi_out, double *eta_out, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    g_last_error.clear();
    int rc;
    if ((rc = validate_density(w)) != FK_OK) return rc;
    if (px < 1 || m < 2) return fail(FK_E_INVAL, "need px >= 1 and m >= 2");
    if (m - 1 >= kMaxP1) return fail(FK_E_UNSUPPORTED, "sub-domain side m must be <= %d", kMaxP1);
    const bool steady = std::isinf(dt_mesh) && dt_mesh > 0.0;
    if (!std::isfinite(t_w) || std::isnan(dt_mesh) || !(dt_mesh > 0.0))
        return fail(FK_E_INVAL, "t_w must be finite and dt_mesh > 0 (or +inf: the steady solve)");
    if (bdry_kind != FK_DATA_IDENTITY && bdry_kind != FK_DATA_ZERO && bdry_kind != FK_DATA_EQUIDISTRIBUTED)
        return fail(FK_E_INVAL, "outer boundary data must be FK_DATA_IDENTITY, _ZERO or _EQUIDISTRIBUTED");
    const int N = px * m;
    const int64_t n_iface = 2 * (int64_t)(px - 1) * (N - 1) - (int64_t)(px - 1) * (px - 1);
    if ((!steady && (!xi_n || !eta_n)) || !xi_out || !eta_out || (n_iface > 0 && (!iface_xi || !iface_eta)))
        return fail(FK_E_INVAL, "NULL array");
    const size_t need = sub_ws_bytes(px, m);
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
    const size_t q = (size_t)m - 1, n = q * q, P1 = q + 1;
    const size_t blocks = (size_t)px * px;
    char *ws = (char *)workspace;
    a.ubuf = (double *)ws;
    ws += align256(blocks * n * P1 * sizeof(double));
    a.ybuf = (double *)ws;
    ws += align256(blocks * 2 * n * sizeof(double));
    a.cbuf = (double *)ws;
    ws += align256(2 * blocks * 4 * n * sizeof(double));
    a.rbuf = (double *)ws;
    ws += align256(2 * blocks * 2 * n * sizeof(double));
    a.sbuf = (double *)ws;
    ws += align256(blocks * sep_stride((int)q) * sizeof(double));
    double *edge_cells = (double *)ws;
    a.N = N;
    a.m = m;
    a.px = px;
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
    // two workgroups per sub-domain from the separator grid row q/2
    a.twisted = (m >= kTwistedMinM) ? 1 : 0;
    a.sep = (int)((q / 2) * q);
    if (launch_lu(a, px * px, stream, &e)) {
        if (e != hipSuccess) return hip_fail(e, "sub-domain kernel launch");
        if (a.twisted && (e = launch_twisted_rest(a, px * px, stream)) != hipSuccess)
            return hip_fail(e, "separator / back substitution launch");
        return FK_OK;
    }
    a.twisted = 0;
    // other sub-domain sizes: the window in LDS
    const size_t lds = (P1 * P1 + 4 * P1) * sizeof(double);
    if ((e = hipFuncSetAttribute((const void *)subdomain_be_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds)) != hipSuccess)
        return hip_fail(e, "hipFuncSetAttribute (LDS)");
    hipLaunchKernelGGL(subdomain_be_kernel, dim3((unsigned)(px * px)), dim3(256), lds, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "sub-domain kernel launch");
    return FK_OK;
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
    a.m = n;
    a.px = 1;
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
    hipLaunchKernelGGL(quality_kernel, dim3(1), dim3(1024), 0, stream, xi, eta, n, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FK_OK : hip_fail(e, "quality kernel launch");
}

}  // extern "C"
