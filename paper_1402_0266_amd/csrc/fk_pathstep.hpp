// fk_pathstep.hpp -- per-lane Euler-Maruyama path state and step, shared
// by the plain and the control-variate path kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fk.h"
#include "fk_accum.hpp"
#include "fk_device.hpp"
#include "fk_internal.hpp"

namespace fk {

// Lane path state.
struct Lane {
    float xh, xl, yh, yl;  // position as hi + lo pairs
    int32_t k;             // steps taken
    int32_t K;             // steps allowed
    uint32_t path, nid, ctr3;
    uint32_t out;          // output row of the path's node
    float px, py;          // start point (score shift for identity data)
    float horizon, dt, dt_last, cbm, cbm_last;
    float ox, oy;          // frozen / static centre offset
    float rev0, drev, cos_d, sin_d;  // orbit angle at path start, step, rotation
    float s_hi, s_lo;      // exponential time-stepping: elapsed time as a hi + lo pair
    DensityRegs dens;
};

// Index of the lane's path in the optional per-path outputs [n_out][n_paths].
__device__ __forceinline__ uint64_t path_rec(const Lane &L, uint32_t n_paths) {
    return (uint64_t)L.out * n_paths + L.path;
}

// Adds an increment to a (hi, lo) pair and renormalises so that hi is the
// FP32 rounding of hi + lo.
__device__ __forceinline__ void comp_add(float &hi, float &lo, float inc) {
    const float t = lo + inc;
    const float s = hi + t;
    lo = (hi - s) + t;
    hi = s;
}

// One Euler-Maruyama step with centre offset (ox, oy); returns true if the
// new point is outside the closed unit square, and the step's Brownian part
// sqrt(2 D) z in (dwx, dwy).  UNIFORM: every step has length dt (t/dt
// integral), so the last-step selection is compiled out.
template <int KIND, bool UNIFORM>
__device__ __forceinline__ bool em_step_w(Lane &L, uint32_t ra, uint32_t rb, float ox, float oy, float &dwx,
                                          float &dwy) {
    float D = L.dt, cb = L.cbm;
    if constexpr (!UNIFORM) {
        const bool last = (L.k == L.K - 1);
        D = last ? L.dt_last : D;
        cb = last ? L.cbm_last : cb;
    }
    brownian_increment(ra, rb, cb, dwx, dwy);
    float bx, by;
    drift<KIND>(L.dens, ox, oy, L.xh, L.yh, bx, by);
    comp_add(L.xh, L.xl, fmaf(bx, D, dwx));
    comp_add(L.yh, L.yl, fmaf(by, D, dwy));
    L.k += 1;
    // Outside the closed square: -x > 0, -y > 0, x - 1 > 0 or y - 1 > 0, as
    // one maximum and one compare.  hi is the rounded position; (hi - 1) is
    // exact near 1, so the tests against 1 see the lo part too.
    const float m = fmaxf(fmaxf(-L.xh, -L.yh), fmaxf((L.xh - 1.f) + L.xl, (L.yh - 1.f) + L.yl));
    return m > 0.f;
}

template <int KIND, bool UNIFORM>
__device__ __forceinline__ bool em_step(Lane &L, uint32_t ra, uint32_t rb, float ox, float oy) {
    float dwx, dwy;
    return em_step_w<KIND, UNIFORM>(L, ra, rb, ox, oy, dwx, dwy);
}

// Brownian-bridge exit test of the step just taken (from (x0h + x0l,
// y0h + y0l) to the lane's position, both inside), for a step of length D
// (iD = 1/D).  The diffusion sqrt(2) W pinned at both ends crosses a side at
// distances d0, d1 with probability exp(-d0 d1 / D); the four sides combine
// as independent events.  A side whose exponent d0 d1 / D exceeds 17 counts
// as 0 (below the uniforms' resolution 2^-24; a zero-length step on a side,
// 0/0, too).  Returns the crossing probability and the side most likely
// crossed (-1: none within reach, and the caller needs no uniform).
__device__ __forceinline__ float bridge_prob(const Lane &L, float x0h, float x0l, float y0h, float y0l, float iD,
                                             int &side) {
    const float d0[4] = {x0h + x0l, (1.f - x0h) - x0l, y0h + y0l, (1.f - y0h) - y0l};
    const float d1[4] = {L.xh + L.xl, (1.f - L.xh) - L.xl, L.yh + L.yl, (1.f - L.yh) - L.yl};
    float p = 0.f, pmax = 0.f;
    side = -1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float e = d0[i] * d1[i] * iD;
        if (e <= 17.f) {
            const float ps = hw_exp2(-1.44269504f * e);
            p = (p + ps) - p * ps;  // 1 - (1 - p)(1 - ps)
            if (ps > pmax) {
                pmax = ps;
                side = i;
            }
        }
    }
    return p;
}

// The lane's end point projected onto side 0 (x = 0), 1 (x = 1), 2 (y = 0) or 3 (y = 1).
__device__ __forceinline__ void move_to_side(Lane &L, int side) {
    if (side == 0) { L.xh = 0.f; L.xl = 0.f; }
    else if (side == 1) { L.xh = 1.f; L.xl = 0.f; }
    else if (side == 2) { L.yh = 0.f; L.yl = 0.f; }
    else { L.yh = 1.f; L.yl = 0.f; }
}

// The bridge test of fixed step k (FK_SCORE_BRIDGE).  The uniform of step k
// is word (k & 1) of Philox(k/2, path, node, ctr3 | 4), u = ((r >> 8) + 1)
// 2^-24; on u < p the path has left within the step and is moved onto the
// side it most likely crossed (its end point projected).
template <bool UNIFORM>
__device__ __forceinline__ bool bridge_exit(Lane &L, float x0h, float x0l, float y0h, float y0l, uint32_t key0,
                                            uint32_t key1) {
    const int32_t k = L.k - 1;
    float D = L.dt;
    if constexpr (!UNIFORM) D = (k == L.K - 1) ? L.dt_last : D;
    int side;
    const float p = bridge_prob(L, x0h, x0l, y0h, y0l, 1.f / D, side);
    if (side < 0) return false;
    const PhiloxOut r = philox4x32_10((uint32_t)k >> 1, L.path, L.nid, L.ctr3 | 4u, key0, key1);
    const uint32_t word = (k & 1) ? r.r1 : r.r0;
    const float u = fmaf((float)(word >> 8), 0x1p-24f, 0x1p-24f);
    if (!(u < p)) return false;
    move_to_side(L, side);
    return true;
}

// Bilinear interpolation in a nodal grid; off the grid, the nearest cell's
// bilinear function continued (linear extrapolation).
__device__ __forceinline__ float grid_bilinear(const double *g, int n, float x, float y) {
    const float fx = x * (float)n, fy = y * (float)n;
    int i = (int)floorf(fx), j = (int)floorf(fy);
    i = min(max(i, 0), n - 1);
    j = min(max(j, 0), n - 1);
    const float ax = fx - (float)i, ay = fy - (float)j;
    const double *r0 = g + (int64_t)j * (n + 1);
    const double *r1 = r0 + (n + 1);
    const float v00 = (float)r0[i], v01 = (float)r0[i + 1];
    const float v10 = (float)r1[i], v11 = (float)r1[i + 1];
    return (1.f - ay) * ((1.f - ax) * v00 + ax * v01) + ay * ((1.f - ax) * v10 + ax * v11);
}


// Work chunks of a wavefront in the control-variate kernels (wave-uniform).
// A wavefront's first chunk is its own index in the grid, so a launch starts
// without every wavefront contending for the one counter at once; later
// chunks come from the counter, past the first grid-full.  Which wavefront
// runs which chunk does not change any result: paths draw their numbers by
// their own counters.  (The plain path kernel keeps its first grab on the
// counter: the same change there costs ~3% in its hot loop's code.)
__device__ __forceinline__ uint32_t first_chunk() { return blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); }
__device__ __forceinline__ uint32_t next_chunk(const PathArgs &a) {
    uint32_t c = 0;
    if ((threadIdx.x & 63u) == 0) c = atomicAdd(a.queue, 1u);
    return __builtin_amdgcn_readfirstlane(c) + gridDim.x * (blockDim.x >> 6);
}
// The launch's work-chunk count (set by the node-table kernels or the host).
__device__ __forceinline__ uint32_t launch_chunks(const PathArgs &a) {
    return __builtin_amdgcn_readfirstlane(a.queue[kCtrTotal]);
}

// Node slot and path chunk of work chunk c (c < total).  Node by node, or
// (tile_shift > 0) with the chunks of 2^tile_shift consecutive slots
// interleaved; a last, partial tile runs node by node.  Only the division by
// cpn of the node-by-node order is needed: the tile is a power of two, so the
// rest is masks and shifts.  The order only changes the schedule: every path
// draws from its own counters and every sum is exact.
__device__ __forceinline__ void chunk_slot(const PathArgs &a, uint32_t total, uint32_t c, uint32_t &slot,
                                           uint32_t &pc) {
    const uint32_t q = c / a.cpn;
    slot = q;
    pc = c - q * a.cpn;
    const uint32_t sh = a.tile_shift;
    if (sh == 0u) return;
    const uint32_t m = (1u << sh) - 1u;
    if ((uint64_t)((q | m) + 1u) * a.cpn > total) return;   // in the partial last tile
    const uint32_t r = (q & m) * a.cpn + pc;                 // rank of the chunk within its tile
    slot = (q & ~m) | (r & m);
    pc = r >> sh;
}

// The cursor (node slot, path range) of chunk c; false past the last chunk.
__device__ __forceinline__ bool chunk_cursor(const PathArgs &a, uint32_t total, uint32_t c, uint32_t &slot,
                                             uint32_t &next, uint32_t &end) {
    if (c >= total) return false;
    uint32_t pc;
    chunk_slot(a, total, c, slot, pc);
    next = pc * a.chunk;
    end = min(next + a.chunk, a.n_paths);
    return true;
}

// chunk_cursor, and on success the chunk's accumulation slot: its tag
// (wave-uniform; every lane calls this).
template <int NV>
__device__ __forceinline__ bool grab_chunk(const PathArgs &a, uint32_t total, uint32_t c, uint32_t &slot,
                                           uint32_t &next, uint32_t &end, AccSlot<NV> *slots, NodeAcc *const *accs,
                                           uint32_t &tag, uint32_t &grabs, uint32_t lane) {
    if (!chunk_cursor(a, total, c, slot, next, end)) return false;
    tag = slot_open<NV>(slots, accs, grabs++, (uint32_t)a.nodes[slot].out, end - next, lane);
    return true;
}

// The level constants of a lane (horizon, step sizes, density parameters,
// Philox counter word 3), loaded with every path: a wavefront may hold paths
// of several levels in a batched launch.  (Held once per launch in scalar
// registers instead, they cost the hot loop more than they save: a VALU
// instruction reads one scalar operand, and the extra scalar pressure
// spills.)
template <int KIND, int TMODE>
__device__ __forceinline__ void lane_level(Lane &L, const LevelDev &lv) {
    L.K = lv.K;
    L.ctr3 = lv.ctr3;
    L.horizon = lv.horizon;
    L.dt = lv.dt;
    L.dt_last = lv.dt_last;
    L.cbm = lv.cbm;
    L.cbm_last = lv.cbm_last;
    L.rev0 = lv.rev0;
    L.drev = lv.drev;
    L.cos_d = lv.cos_d;
    L.sin_d = lv.sin_d;
    L.dens.amp = lv.amp;
    L.dens.nscale = lv.nscale;
    L.dens.a2s = lv.a2s;
    L.dens.cx = lv.cx;
    L.dens.cy = lv.cy;
    L.dens.orbit_r = lv.orbit_r;
    L.dens.omega_rev = lv.omega_rev;
    if constexpr (KIND == KIND_GRID) {
        L.dens.gb = lv.gb;
        L.dens.gn = lv.gn;
        L.dens.fn = lv.fn;
    }
    L.ox = 0.f;
    L.oy = 0.f;
    if constexpr (moving_kind(KIND) && TMODE == TIME_FROZEN) {
        orbit(L.dens, lv.t_freeze, L.ox, L.oy);
    }
}

// Loads path `path` of node `nd` into a lane, with its level's constants.
template <int KIND, int TMODE>
__device__ __forceinline__ void lane_start(Lane &L, const NodeDev &nd, const LevelDev *levels, uint32_t path) {
    L.path = path;
    L.xh = nd.x;
    L.yh = nd.y;
    L.xl = nd.xlo;
    L.yl = nd.ylo;
    L.px = nd.x;
    L.py = nd.y;
    L.k = 0;
    L.nid = nd.nid;
    L.out = (uint32_t)nd.out;
    lane_level<KIND, TMODE>(L, levels[nd.level]);
}

// Score of a finished path (eq. (7b)): boundary data at the exit point if
// it left the square (out), else the initial data at its end point.  With
// a.shift the identity scores are stored relative to the start point.
// FK_SCORE_EXTEND scores an exit with the grid initial data extrapolated
// bilinearly to the exit point (grid_bilinear extrapolates off the grid);
// FK_SCORE_PROJECT, FK_SCORE_BRIDGE and FK_SCORE_EXPONENTIAL score it at
// the point clamped onto the square (boundary data FK_DATA_GRID: the grid's
// edge there).
__device__ __forceinline__ void score_path(const PathArgs &a, const Lane &L, bool out, float &sx, float &sy) {
    const int kind = out ? (a.score_mode == FK_SCORE_EXTEND ? FK_DATA_GRID : a.bdry_kind) : a.init_kind;
    float x = L.xh, y = L.yh;
    float lx = L.xl, ly = L.yl;
    if (out && (a.score_mode == FK_SCORE_PROJECT || a.score_mode == FK_SCORE_BRIDGE ||
                a.score_mode == FK_SCORE_EXPONENTIAL)) {
        if (x < 0.f || x > 1.f) { x = fminf(fmaxf(x, 0.f), 1.f); lx = 0.f; }
        if (y < 0.f || y > 1.f) { y = fminf(fmaxf(y, 0.f), 1.f); ly = 0.f; }
    }
    if (kind == FK_DATA_IDENTITY) {
        const float bx0 = a.shift ? L.px : 0.f, by0 = a.shift ? L.py : 0.f;
        sx = (x - bx0) + lx;
        sy = (y - by0) + ly;
    } else if (kind == FK_DATA_SIN) {
        float v = sin_mode(x, y);
        if (out) {
            // elapsed time since the initial data: t - s_kappa
            float s = (L.k >= L.K) ? L.horizon : (float)L.k * L.dt;
            if (a.score_mode == FK_SCORE_EXPONENTIAL) s = L.s_hi + L.s_lo;
            v *= hw_exp2(-2.f * 9.8696044f * 1.44269504f * (L.horizon - s));
        }
        sx = v;
        sy = v;
    } else if (kind == FK_DATA_GRID) {
        sx = grid_bilinear(a.grid_xi, a.grid_n, x, y);
        // one grid at a time: keeps the scoring's registers below the path
        // loop's (this runs once per path)
        __builtin_amdgcn_sched_barrier(0);
        sy = grid_bilinear(a.grid_eta, a.grid_n, x, y);
    } else {
        sx = 0.f;
        sy = 0.f;
    }
}

}  // namespace fk
