// fk_keys.hip -- key points on the sub-domain interfaces and the piecewise
// cubic Hermite interpolation of the other interface nodes (Sect. 4, further
// speed-up; the paper's run in Sect. 5 uses both).
//
// Interface lines of px x px sub-domains on the N = px m grid: vertical
// lines x = a/px (a = 1 .. px-1) and horizontal lines y = c/px; a line's
// nodes are its positions k = 0 .. N, the two ends on the outer boundary.
// Interface nodes are numbered in the canonical order of the sub-domain
// solve: vertical lines (positions 1 .. N-1), then horizontal lines without
// their crossings.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "fk.h"
#include "fk_internal.hpp"

namespace fk {

// Canonical index of position k (1 .. N-1) on line `line` (vertical lines
// 0 .. px-2, then horizontal lines); a horizontal line's crossing at k = a m
// is the vertical line a's node at position c m.
__device__ __forceinline__ int64_t line_node(int px, int m, int line, int k) {
    const int N = px * m;
    if (line < px - 1) return (int64_t)line * (N - 1) + (k - 1);
    const int c = line - (px - 1) + 1;
    if (k % m == 0) return (int64_t)(k / m - 1) * (N - 1) + (c * m - 1);
    const int64_t nv = (int64_t)(px - 1) * (N - 1);
    return nv + (int64_t)(c - 1) * (N - px) + (k - 1 - k / m);
}

// Line and position of canonical interface node f.
__device__ __forceinline__ void node_line(int px, int m, int64_t f, int &line, int &k) {
    const int N = px * m;
    const int64_t nv = (int64_t)(px - 1) * (N - 1);
    if (f < nv) {
        line = (int)(f / (N - 1));
        k = (int)(f % (N - 1)) + 1;
        return;
    }
    const int64_t g = f - nv;
    line = (px - 1) + (int)(g / (N - px));
    const int r = (int)(g % (N - px));  // r-th non-crossing position
    k = r + 1 + r / (m - 1);
}

// Grid offset j (N+1) + i of position k on a line.
__device__ __forceinline__ int64_t line_grid(int px, int m, int line, int k) {
    const int N = px * m;
    if (line < px - 1) return (int64_t)k * (N + 1) + (line + 1) * m;
    return (int64_t)((line - (px - 1) + 1) * m) * (N + 1) + k;
}

// ---------------------------------------------------------------------------
// Key points.  rho = 1/w along the line; its derivatives up to the constant
// factors 1/2h and 1/h^2 at the interior positions,
//   f1_k = rho_{k+1} - rho_{k-1},  f2_k = (rho_{k+1} + rho_{k-1}) - (rho_k + rho_k)
// (sums and differences only, so every rounding is fixed).  A key point is a
// position 2 <= k <= N-2 where f1 or f2 has a discrete extremum (greater than
// the left neighbour and not less than the right one, or the reverse) of
// size at least tol times the line's largest |f|; crossings are key points;
// gaps between consecutive knots (keys and the two ends) longer than max_gap
// positions get ceil(g / max_gap) - 1 evenly spaced keys.
// ---------------------------------------------------------------------------
struct KeyArgs {
    const double *w;
    int px, m;
    double tol;
    int max_gap;
    uint8_t *mask;
};

__device__ __forceinline__ double line_rho(const KeyArgs &a, int line, int k) {
    return 1.0 / a.w[line_grid(a.px, a.m, line, k)];
}

__device__ __forceinline__ void line_f(const KeyArgs &a, int line, int k, double &f1, double &f2) {
    const double rl = line_rho(a, line, k - 1), rc = line_rho(a, line, k), rr = line_rho(a, line, k + 1);
    f1 = rr - rl;
    f2 = (rr + rl) - (rc + rc);
}

__device__ __forceinline__ bool extremum(double fl, double fk, double fr, double thr) {
    return fabs(fk) >= thr && ((fk > fl && fk >= fr) || (fk < fl && fk <= fr));
}

// One workgroup per line: the line's largest |f1|, |f2| by a block
// reduction, the extremum flags of its positions in LDS, then one lane
// walks the flags for the gap filling and the workgroup writes the mask.
constexpr int kKeyThreads = 256;
constexpr int kKeyMaxN = 8192;  // LDS flags: positions 0 .. N

__device__ __forceinline__ double block_max(double v, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < kKeyThreads / 64; ++w) r = fmax(r, red[w]);
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kKeyThreads) key_points_kernel(const KeyArgs a) {
    __shared__ uint8_t flag[kKeyMaxN + 1];
    __shared__ double red[kKeyThreads / 64];
    const int line = blockIdx.x;
    const int N = a.px * a.m;
    const bool vertical = line < a.px - 1;
    double m1 = 0.0, m2 = 0.0;
    for (int k = 1 + threadIdx.x; k < N; k += blockDim.x) {
        double f1, f2;
        line_f(a, line, k, f1, f2);
        m1 = fmax(m1, fabs(f1));
        m2 = fmax(m2, fabs(f2));
    }
    const double t1 = a.tol * block_max(m1, red), t2 = a.tol * block_max(m2, red);
    // extrema and crossings
    for (int k = threadIdx.x; k <= N; k += blockDim.x) {
        bool key = (k == 0) || (k == N) || (k % a.m == 0);  // knots: the ends and the crossings
        if (k >= 2 && k <= N - 2) {
            double p1, p2, c1, c2, n1, n2;
            line_f(a, line, k - 1, p1, p2);
            line_f(a, line, k, c1, c2);
            line_f(a, line, k + 1, n1, n2);
            key = key || (t1 > 0.0 && extremum(p1, c1, n1, t1)) || (t2 > 0.0 && extremum(p2, c2, n2, t2));
        }
        flag[k] = key ? 1 : 0;
    }
    __syncthreads();
    // gap filling between consecutive knots
    if (threadIdx.x == 0) {
        int prev = 0;
        for (int k = 1; k <= N; ++k) {
            if (!flag[k]) continue;
            const int g = k - prev;
            if (g > a.max_gap) {
                const int q = (g + a.max_gap - 1) / a.max_gap;
                for (int r = 1; r < q; ++r) flag[prev + (r * g) / q] = 1;
            }
            prev = k;
        }
    }
    __syncthreads();
    // every position this line owns, written once (a crossing belongs to its vertical line)
    for (int k = 1 + threadIdx.x; k < N; k += blockDim.x)
        if (vertical || k % a.m != 0) a.mask[line_node(a.px, a.m, line, k)] = flag[k];
}

// ---------------------------------------------------------------------------
// Interpolation: the monotone piecewise cubic Hermite interpolant (Fritsch &
// Carlson 1980, slopes of Fritsch & Butland 1984) through the line's two
// boundary ends and its key points, in the node coordinate k/N.  One thread
// per interface node: a key point copies its value; any other node finds the
// two knots around it and their outer neighbours by walking its line.
// ---------------------------------------------------------------------------
struct InterpArgs {
    int px, m;
    const int32_t *slot;  // [n_iface]: index into key_xi / key_eta, or -1 (slot form)
    const uint8_t *mask;  // [n_iface]: key point where nonzero (mask form: values in out_xi / out_eta)
    int64_t n_keys;
    const double *key_xi, *key_eta;
    const double *edge_xi, *edge_eta;  // grids whose edge nodes hold the boundary data
    double *out_xi, *out_eta;
    int64_t n_iface;
};

__device__ __forceinline__ bool is_knot(const InterpArgs &a, int line, int k) {
    const int N = a.px * a.m;
    if (k == 0 || k == N) return true;
    const int64_t f = line_node(a.px, a.m, line, k);
    return a.mask ? a.mask[f] != 0 : a.slot[f] >= 0;
}

// Value of component c at knot position k (a boundary end or a key point).
__device__ __forceinline__ double knot_value(const InterpArgs &a, int line, int k, int c) {
    const int N = a.px * a.m;
    if (k == 0 || k == N) return (c == 0 ? a.edge_xi : a.edge_eta)[line_grid(a.px, a.m, line, k)];
    if (a.mask) return (c == 0 ? a.out_xi : a.out_eta)[line_node(a.px, a.m, line, k)];
    const int32_t s = a.slot[line_node(a.px, a.m, line, k)];
    if (s >= a.n_keys) return NAN;
    return (c == 0 ? a.key_xi : a.key_eta)[s];
}

// Interior knot slope from the secants on its left (hl, dl) and right (hr, dr).
__device__ __forceinline__ double inner_slope(double hl, double dl, double hr, double dr) {
    if (!(dl * dr > 0.0)) return 0.0;
    const double w1 = 2.0 * hr + hl, w2 = hr + 2.0 * hl;
    return (w1 + w2) / (w1 / dl + w2 / dr);
}

// End slope from the end secant (h0, d0) and the next one (h1, d1).
__device__ __forceinline__ double end_slope(double h0, double d0, double h1, double d1) {
    const double v = ((2.0 * h0 + h1) * d0 - h0 * d1) / (h0 + h1);
    const auto sgn = [](double x) { return (x > 0.0) - (x < 0.0); };
    if (sgn(v) != sgn(d0)) return 0.0;
    if (sgn(d0) != sgn(d1) && fabs(v) > fabs(3.0 * d0)) return 3.0 * d0;
    return v;
}

__global__ void interpolate_kernel(const InterpArgs a) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= a.n_iface) return;
    if (a.mask) {
        // in place: a key point keeps its value (and is only read by others)
        if (a.mask[f] != 0) return;
    } else if (const int32_t s = a.slot[f]; s >= 0) {
        const bool ok = s < a.n_keys;
        a.out_xi[f] = ok ? a.key_xi[s] : NAN;
        a.out_eta[f] = ok ? a.key_eta[s] : NAN;
        return;
    }
    const int N = a.px * a.m;
    int line, k;
    node_line(a.px, a.m, f, line, k);
    // knots L1 < k < R1 and their outer neighbours L0 (or -1) and R2 (or N+1)
    int L1 = k - 1;
    while (!is_knot(a, line, L1)) --L1;
    int R1 = k + 1;
    while (!is_knot(a, line, R1)) ++R1;
    int L0 = -1;
    for (int q = L1 - 1; q >= 0; --q)
        if (is_knot(a, line, q)) { L0 = q; break; }
    int R2 = N + 1;
    for (int q = R1 + 1; q <= N; ++q)
        if (is_knot(a, line, q)) { R2 = q; break; }
    // knot coordinates k/N, rounded as the nodes are defined
    const double xL1 = (double)L1 / N, xR1 = (double)R1 / N;
    const double h = xR1 - xL1, t = ((double)k / N - xL1) / h;
    const double h00 = (1.0 + 2.0 * t) * (1.0 - t) * (1.0 - t), h10 = t * (1.0 - t) * (1.0 - t);
    const double h01 = t * t * (3.0 - 2.0 * t), h11 = t * t * (t - 1.0);
    for (int c = 0; c < 2; ++c) {
        const double yL1 = knot_value(a, line, L1, c), yR1 = knot_value(a, line, R1, c);
        const double d = (yR1 - yL1) / h;
        double sL, sR;
        if (L0 < 0 && R2 > N) {
            sL = sR = d;  // two knots: the straight line
        } else {
            double hl = 0.0, dl = 0.0, hr = 0.0, dr = 0.0;
            if (L0 >= 0) {
                hl = xL1 - (double)L0 / N;
                dl = (yL1 - knot_value(a, line, L0, c)) / hl;
            }
            if (R2 <= N) {
                hr = (double)R2 / N - xR1;
                dr = (knot_value(a, line, R2, c) - yR1) / hr;
            }
            sL = L0 >= 0 ? inner_slope(hl, dl, h, d) : end_slope(h, d, hr, dr);
            sR = R2 <= N ? inner_slope(h, d, hr, dr) : end_slope(h, d, hl, dl);
        }
        const double v = h00 * yL1 + h10 * h * sL + h01 * yR1 + h11 * h * sR;
        (c == 0 ? a.out_xi : a.out_eta)[f] = v;
    }
}

}  // namespace fk

using namespace fk;

extern "C" {

int fk_key_points(const double *grid_w, int32_t px, int32_t m, double tol, int32_t max_gap, uint8_t *mask,
                  hipStream_t stream) {
    g_last_error.clear();
    if (px < 2 || m < 2) return fail(FK_E_INVAL, "need px >= 2 and m >= 2");
    if ((int64_t)px * m > kKeyMaxN) return fail(FK_E_INVAL, "grid too large (px m > %d)", kKeyMaxN);
    if (!std::isfinite(tol) || tol < 0.0) return fail(FK_E_INVAL, "tol must be finite and >= 0");
    if (max_gap < 1) return fail(FK_E_INVAL, "max_gap must be >= 1");
    if (!grid_w || !mask) return fail(FK_E_INVAL, "NULL array");
    KeyArgs a{grid_w, (int)px, (int)m, tol, (int)max_gap, mask};
    hipLaunchKernelGGL(key_points_kernel, dim3((unsigned)(2 * (px - 1))), dim3(kKeyThreads), 0, stream, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FK_OK : hip_fail(e, "key point kernel launch");
}

int fk_interface_interpolate(int32_t px, int32_t m, const int32_t *slot, int64_t n_keys, const double *key_xi,
                             const double *key_eta, const double *edge_xi, const double *edge_eta, double *iface_xi,
                             double *iface_eta, hipStream_t stream) {
    g_last_error.clear();
    if (px < 2 || m < 2) return fail(FK_E_INVAL, "need px >= 2 and m >= 2");
    if ((int64_t)px * m > 65535) return fail(FK_E_INVAL, "grid too large (px m > 65535)");
    if (n_keys < 0) return fail(FK_E_INVAL, "n_keys must be >= 0");
    if (!slot || !edge_xi || !edge_eta || !iface_xi || !iface_eta || (n_keys > 0 && (!key_xi || !key_eta)))
        return fail(FK_E_INVAL, "NULL array");
    const int64_t N = (int64_t)px * m;
    InterpArgs a{};
    a.px = px;
    a.m = m;
    a.slot = slot;
    a.n_keys = n_keys;
    a.key_xi = key_xi;
    a.key_eta = key_eta;
    a.edge_xi = edge_xi;
    a.edge_eta = edge_eta;
    a.out_xi = iface_xi;
    a.out_eta = iface_eta;
    a.n_iface = 2 * (px - 1) * (N - 1) - (int64_t)(px - 1) * (px - 1);
    hipLaunchKernelGGL(interpolate_kernel, dim3((unsigned)((a.n_iface + 255) / 256)), dim3(256), 0, stream, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FK_OK : hip_fail(e, "interface interpolation kernel launch");
}

int fk_interface_interpolate_mask(int32_t px, int32_t m, const uint8_t *mask, const double *edge_xi,
                                  const double *edge_eta, double *iface_xi, double *iface_eta, hipStream_t stream) {
    g_last_error.clear();
    if (px < 2 || m < 2) return fail(FK_E_INVAL, "need px >= 2 and m >= 2");
    if ((int64_t)px * m > 65535) return fail(FK_E_INVAL, "grid too large (px m > 65535)");
    if (!mask || !edge_xi || !edge_eta || !iface_xi || !iface_eta) return fail(FK_E_INVAL, "NULL array");
    const int64_t N = (int64_t)px * m;
    InterpArgs a{};
    a.px = px;
    a.m = m;
    a.mask = mask;
    a.edge_xi = edge_xi;
    a.edge_eta = edge_eta;
    a.out_xi = iface_xi;
    a.out_eta = iface_eta;
    a.n_iface = 2 * (px - 1) * (N - 1) - (int64_t)(px - 1) * (px - 1);
    hipLaunchKernelGGL(interpolate_kernel, dim3((unsigned)((a.n_iface + 255) / 256)), dim3(256), 0, stream, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FK_OK : hip_fail(e, "interface interpolation kernel launch");
}

}  // extern "C"
