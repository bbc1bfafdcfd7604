// fk_paths.hip -- the Monte-Carlo hot path: a persistent path kernel (one
// path per lane, lanes refilled from a device work queue as their paths
// end) and the FP64 estimator reduction.
//
// Method (Sect. 3, eqs. (5)-(7); Sect. 4): for an interface node P, a path
// X_0 = P, X_{k+1} = X_k + b(tau_k, X_k) D_k + sqrt(2 D_k) z_k takes
// Euler-Maruyama steps of dX = -(grad w / w) ds + sqrt(2) dW with a boundary
// test after every step.  A path that leaves the square scores the boundary
// data at its exit point; a path alive after K steps scores the initial data.
// The node value is the mean of the scores over its paths.
//
// MI355X mapping:
//  * The path loop is ALU-bound (Philox integer multiplies, 6-8 hardware
//    transcendentals, ~40 FP32 ops per step) and touches no memory, so every
//    lane keeps its whole path state in registers.
//  * Exit times vary by two orders of magnitude between nodes and
//    geometrically within a node; lanes therefore refill individually: a
//    wavefront grabs `chunk` consecutive paths of one node from a global
//    atomic queue and hands them to whichever lanes are idle, so a lane never
//    waits for the rest of its wavefront.  Nodes are queued in decreasing
//    expected cost so the launch ends on short paths.
//  * Each finished path adds its score to its node's sums inside the kernel
//    (fixed-point integer sums: per wavefront in LDS per work chunk, then
//    per node in HBM), so results do not depend on the launch schedule and
//    no per-path record is written unless the caller asks for the scores;
//    a small kernel turns the sums into means and standard errors.
//  * Positions are FP32 pairs (hi, lo): each increment is added to lo and the
//    pair renormalised, which keeps the position to ~2^-48 over 10^4 steps
//    (plain FP32 accumulation drifts by ~1e-6 and flips exit decisions).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <utility>

#include "fk_accum.hpp"
#include "fk_device.hpp"
#include "fk_internal.hpp"
#include "fk_pathstep.hpp"

namespace fk {

__global__ void zero_u32_kernel(uint32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_zero_u32(uint32_t *p, int n_words, hipStream_t s) {
    const int blocks = (n_words + 255) / 256;
    hipLaunchKernelGGL(zero_u32_kernel, dim3(blocks), dim3(256), 0, s, p, n_words);
    return hipGetLastError();
}

__global__ void counters_init_kernel(uint32_t *c, uint32_t total_chunks) {
    const int i = threadIdx.x;
    if (i < 64) c[i] = (i == kCtrTotal) ? total_chunks : 0u;
}

hipError_t launch_counters_init(uint32_t *counters, uint32_t total_chunks, hipStream_t s) {
    hipLaunchKernelGGL(counters_init_kernel, dim3(1), dim3(64), 0, s, counters, total_chunks);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Node tables from device coordinates.  Nodes are queued in decreasing
// expected cost -- a proxy of the mean exit time, capped by the horizon --
// bucketed into kCostBuckets classes (the order within a class is that of
// the atomics: it only changes the schedule, never a result, since every
// path draws its numbers by its own counters).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool node_wanted(const TableArgs &t, int64_t i, double &x, double &y, bool &ok) {
    x = t.pts[2 * i];
    y = t.pts[2 * i + 1];
    ok = (x >= 0.0 && x <= 1.0 && y >= 0.0 && y <= 1.0);   // false for NaN
    return !t.mask || t.mask[i];
}

__device__ __forceinline__ int cost_bucket(const TableArgs &t, double x, double y) {
    if (!t.sort) return 0;
    const double ax = x * (1.0 - x), ay = y * (1.0 - y);
    double c = 0.0;
    if (ax > 0.0 && ay > 0.0) c = fmin((double)t.horizon, 1.0 / (2.0 / ax + 2.0 / ay));
    const double f = t.horizon > 0.f ? c / (double)t.horizon : 0.0;     // in [0, 1]
    return min(kCostBuckets - 1, max(0, (int)((1.0 - f) * kCostBuckets)));
}

// Adds, for every lane with `take`, one to hist[b] -- one atomic per
// distinct b in the wavefront (a mesh step's nodes mostly share a bucket,
// and one atomic per node on one address serialises) -- and returns the
// lane's slot: the old count plus its rank among the wavefront's lanes with
// the same b.  Every lane of the wavefront calls it.
__device__ __forceinline__ uint32_t wave_bucket_add(uint32_t *hist, bool take, int b) {
    const int lane = (int)(threadIdx.x & 63u);
    uint64_t left = __ballot(take);
    uint32_t slot = 0;
    while (left != 0ull) {
        const int leader = __builtin_ctzll(left);
        const int lb = __shfl(b, leader, 64);
        const bool mine = take && b == lb;
        const uint64_t grp = __ballot(mine);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&hist[lb], (uint32_t)__popcll(grp));
        base = (uint32_t)__shfl((int)base, leader, 64);
        if (mine) slot = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(grp >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)grp, 0u));
        left &= ~grp;
    }
    return slot;
}

__global__ void table_count_kernel(const TableArgs t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *t.levels_out = t.level;
    bool take = false;
    int bucket = 0;
    if (i < t.n) {
        double x, y;
        bool ok;
        const bool want = node_wanted(t, i, x, y, ok);
        OutDev o{};
        o.shift_x = t.shift ? (double)(float)x : 0.0;
        o.shift_y = t.shift ? (double)(float)y : 0.0;
        o.K = t.level.K;
        t.outs_out[i] = o;
        if (t.outs_zero_out) {
            o.shift_x = o.shift_y = 0.0;
            t.outs_zero_out[i] = o;
        }
        if (want && !ok) {
            // not a node of the square: no paths, NaN results
            t.acc[i].bad = 1u;
            if (t.acc2) t.acc2[i].bad = 1u;
        }
        take = want && ok;
        if (take) bucket = cost_bucket(t, x, y);
    }
    wave_bucket_add(t.counters + kCtrHist, take, bucket);
}

__global__ void table_scan_kernel(uint32_t *c, uint32_t cpn) {
    if (threadIdx.x != 0) return;
    uint32_t run = 0;
    for (int b = 0; b < kCostBuckets; ++b) {
        const uint32_t k = c[kCtrHist + b];
        c[kCtrHist + b] = run;
        run += k;
    }
    c[kCtrActive] = run;
    c[kCtrTotal] = run * cpn;
}

__global__ void table_scatter_kernel(const TableArgs t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double x = 0.0, y = 0.0;
    bool ok = false, take = false;
    int bucket = 0;
    if (i < t.n) {
        take = node_wanted(t, i, x, y, ok) && ok;
        if (take) bucket = cost_bucket(t, x, y);
    }
    const uint32_t slot = wave_bucket_add(t.counters + kCtrHist, take, bucket);
    if (!take) return;
    NodeDev nd{};
    // the start point as an FP32 (hi, lo) pair holding the FP64 node to ~2^-48
    nd.x = (float)x;
    nd.y = (float)y;
    nd.xlo = (float)(x - (double)nd.x);
    nd.ylo = (float)(y - (double)nd.y);
    nd.nid = (uint32_t)i;
    nd.level = 0;
    nd.out = (uint64_t)i;
    t.nodes_out[slot] = nd;
}

hipError_t launch_tables(const TableArgs &t, hipStream_t s) {
    const unsigned blocks = (unsigned)std::max<int64_t>(1, (t.n + 255) / 256);
    hipLaunchKernelGGL(table_count_kernel, dim3(blocks), dim3(256), 0, s, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(table_scan_kernel, dim3(1), dim3(64), 0, s, t.counters, t.cpn);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(table_scatter_kernel, dim3(blocks), dim3(256), 0, s, t);
    return hipGetLastError();
}


// BRIDGE: the Brownian-bridge crossing test after every step that stays
// inside (score mode FK_SCORE_BRIDGE).  FIRST_BY_INDEX (short horizons): a
// wavefront's first chunk is its index in the grid, later ones come from the
// counter past the first grid-full, so a launch of short paths does not open
// with every wavefront contending for the counter.  Long horizons keep the
// counter for every grab (the other form costs their hot loop ~3% in code).
template <int KIND, int TMODE, bool UNIFORM, bool BRIDGE, bool FIRST_BY_INDEX = false>
__global__ void __launch_bounds__(256) fk_path_kernel(const PathArgs a) {
    constexpr bool kMovingBackward = moving_kind(KIND) && TMODE == TIME_BACKWARD;
    const uint32_t lane = threadIdx.x & 63u;
    __shared__ AccSlot<2> slot_tab[4][kAccSlots];
    AccSlot<2> *slots = slot_tab[threadIdx.x >> 6];
    NodeAcc *const accs[1] = {a.acc};
    slots_init<2>(slots, lane);
    // Wavefront-uniform queue cursor: current node slot and path range, and
    // the grab number of the chunk (its accumulation slot).
    uint32_t q_slot = 0, q_next = 0, q_end = 0, q_tag = 0, grabs = 0;
    bool q_done = false;
    const uint32_t total_chunks = launch_chunks(a);
    if constexpr (FIRST_BY_INDEX) {
        q_done = !chunk_cursor(a, total_chunks, first_chunk(), q_slot, q_next, q_end);
        if (!q_done) {
            q_tag = slot_open<2>(slots, accs, grabs++, (uint32_t)a.nodes[q_slot].out, q_end - q_next, lane);
        }
    }
    const uint32_t key0 = a.key0, key1 = a.key1;

    Lane L;
    PhiloxPath pp{};          // the lane's path's fixed Philox products
    bool active = false;
    uint32_t my_tag = 0;      // accumulation tag of the lane's path's chunk
    uint32_t my_steps = 0;

    bool closed = false;      // the lane's last path closed its chunk's slot
    for (;;) {
        // ---- flush closed chunks, refill idle lanes ---------------------
        if (__ballot(closed) != 0ull) {
            slots_collect<2>(slots, accs, lane);
            closed = false;
        }
        uint64_t need = __ballot(!active);
        while (need != 0ull && !q_done) {
            if (q_next >= q_end) {
                if constexpr (FIRST_BY_INDEX) {
                    // a grid no larger than the chunk count hands out no more
                    // chunks: finish without touching the counter
                    if (gridDim.x * (blockDim.x >> 6) >= total_chunks) {
                        q_done = true;
                        break;
                    }
                }
                uint32_t c = 0;
                if (lane == 0) c = atomicAdd(a.queue, 1u);
                c = __builtin_amdgcn_readfirstlane(c);
                if constexpr (FIRST_BY_INDEX) c += gridDim.x * (blockDim.x >> 6);
                if (c >= total_chunks) {
                    q_done = true;
                    break;
                }
                uint32_t pc;
                chunk_slot(a, total_chunks, c, q_slot, pc);
                q_next = pc * a.chunk;
                q_end = min(q_next + a.chunk, a.n_paths);
                q_tag = slot_open<2>(slots, accs, grabs++, (uint32_t)a.nodes[q_slot].out, q_end - q_next, lane);
                continue;
            }
            const uint32_t avail = q_end - q_next;
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            if (!active && rank < avail) {
                lane_start<KIND, TMODE>(L, a.nodes[q_slot], a.levels, q_next + rank);
                pp = philox_path(L.path, L.nid, key0);
                my_tag = q_tag;
                active = true;
            }
            const uint32_t n_need = (uint32_t)__popcll(need);
            q_next += min(n_need, avail);
            need = __ballot(!active);
        }
        if (__ballot(active) == 0ull) break;

        // ---- two Euler-Maruyama steps from one Philox call ----------------
        if (active) {
            bool out = false;
            if (L.k < L.K) {
                const PhiloxOut r = philox4x32_10_path((uint32_t)L.k >> 1, L.ctr3, pp, key0, key1);
                float ox = L.ox, oy = L.oy, cr = 0.f, sr = 0.f;
                if constexpr (kMovingBackward) {
                    // Orbit angle at PDE time t_init + t - k dt, in revolutions.
                    const float rev = fmaf(-(float)L.k, L.drev, L.rev0);
                    cr = hw_cos_rev(rev);
                    sr = hw_sin_rev(rev);
                    ox = L.dens.orbit_r * cr;
                    oy = L.dens.orbit_r * sr;
                }
                float x0h = 0.f, x0l = 0.f, y0h = 0.f, y0l = 0.f;
                if constexpr (BRIDGE) {
                    x0h = L.xh; x0l = L.xl; y0h = L.yh; y0l = L.yl;
                }
                out = em_step<KIND, UNIFORM>(L, r.r0, r.r1, ox, oy);
                if constexpr (BRIDGE) {
                    if (!out) out = bridge_exit<UNIFORM>(L, x0h, x0l, y0h, y0l, key0, key1);
                }
                if (!out && L.k < L.K) {
                    if constexpr (kMovingBackward) {
                        // One step later the angle is smaller by omega dt:
                        // rotate (cos, sin) instead of re-evaluating them.
                        const float c2 = fmaf(cr, L.cos_d, sr * L.sin_d);
                        const float s2 = fmaf(sr, L.cos_d, -cr * L.sin_d);
                        ox = L.dens.orbit_r * c2;
                        oy = L.dens.orbit_r * s2;
                    }
                    if constexpr (BRIDGE) {
                        x0h = L.xh; x0l = L.xl; y0h = L.yh; y0l = L.yl;
                    }
                    out = em_step<KIND, UNIFORM>(L, r.r2, r.r3, ox, oy);
                    if constexpr (BRIDGE) {
                        if (!out) out = bridge_exit<UNIFORM>(L, x0h, x0l, y0h, y0l, key0, key1);
                    }
                }
            }
            if (out || L.k >= L.K) {
                // ---- score (eq. (7b)) and its node's sums ------------------
                float v[2];
                score_path(a, L, out, v[0], v[1]);
                closed = acc_path<2>(slots, accs, my_tag, L.out, v, (uint32_t)L.k);
                my_steps += (uint32_t)L.k;      // the path's steps, counted once at its end
                if (a.scores) a.scores[path_rec(L, a.n_paths)] = make_float2(v[0], v[1]);
                if (a.exit_step) a.exit_step[path_rec(L, a.n_paths)] = out ? L.k : -1;
                active = false;
            }
        }
    }

    // ---- the last closed chunks' sums ----------------------------------------
    slots_collect<2>(slots, accs, lane);
    // ---- step count: wavefront sum, one atomic per wavefront --------------
    unsigned long long st = my_steps;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) st += __shfl_xor(st, off, 64);
    // a null count: the caller did not ask for it (every kernel skips it)
    if (lane == 0 && st != 0ull && a.total_steps) atomicAdd(a.total_steps, st);
}

// Exponential time-stepping (FK_SCORE_EXPONENTIAL): the same persistent
// queue and in-kernel estimator as fk_path_kernel; each step has its own
// length D = -dt ln u (u from word 2 + (k & 1) of Philox(k/2, path, node,
// ctr3 | 4)), cut at the horizon, then the Euler-Maruyama step of length D
// and the bridge test for D with that Philox call's word k & 1.  The elapsed
// time is kept as a hi + lo pair; the orbit angle of a moving density at
// PDE time t_init + t - s follows it.  A path ends when it exits or when
// the cut step has been taken (L.K is set to the step count then).
template <int KIND, int TMODE>
__global__ void __launch_bounds__(256) fk_expo_path_kernel(const PathArgs a) {
    constexpr bool kMovingBackward = moving_kind(KIND) && TMODE == TIME_BACKWARD;
    const uint32_t lane = threadIdx.x & 63u;
    __shared__ AccSlot<2> slot_tab[4][kAccSlots];
    AccSlot<2> *slots = slot_tab[threadIdx.x >> 6];
    NodeAcc *const accs[1] = {a.acc};
    slots_init<2>(slots, lane);
    uint32_t q_slot = 0, q_next = 0, q_end = 0, q_tag = 0, grabs = 0;
    bool q_done = false;
    const uint32_t total_chunks = launch_chunks(a);
    const uint32_t key0 = a.key0, key1 = a.key1;
    Lane L;
    bool active = false;
    uint32_t my_tag = 0, my_steps = 0;
    bool closed = false;
    for (;;) {
        if (__ballot(closed) != 0ull) {
            slots_collect<2>(slots, accs, lane);
            closed = false;
        }
        uint64_t need = __ballot(!active);
        while (need != 0ull && !q_done) {
            if (q_next >= q_end) {
                uint32_t c = 0;
                if (lane == 0) c = atomicAdd(a.queue, 1u);
                c = __builtin_amdgcn_readfirstlane(c);
                if (!grab_chunk<2>(a, total_chunks, c, q_slot, q_next, q_end, slots, accs, q_tag, grabs, lane)) {
                    q_done = true;
                    break;
                }
                continue;
            }
            const uint32_t avail = q_end - q_next;
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            if (!active && rank < avail) {
                lane_start<KIND, TMODE>(L, a.nodes[q_slot], a.levels, q_next + rank);
                L.K = L.K > 0 ? 0x7fffffff : 0;      // open-ended; 0 for a zero horizon
                L.s_hi = 0.f;
                L.s_lo = 0.f;
                my_tag = q_tag;
                active = true;
            }
            q_next += min((uint32_t)__popcll(need), avail);
            need = __ballot(!active);
        }
        if (__ballot(active) == 0ull) break;

        if (active) {
            bool out = false;
            if (L.k < L.K) {
                const PhiloxOut r = philox4x32_10((uint32_t)L.k >> 1, L.path, L.nid, L.ctr3, key0, key1);
                const PhiloxOut q = philox4x32_10((uint32_t)L.k >> 1, L.path, L.nid, L.ctr3 | 4u, key0, key1);
                const bool odd = (L.k & 1) != 0;
                const float u = fmaf((float)((odd ? q.r3 : q.r2) >> 8), 0x1p-24f, 0x1p-24f);
                float D = -0.69314718f * L.dt * hw_log2(u);
                const float rem = (L.horizon - L.s_hi) - L.s_lo;
                const bool last = D >= rem;
                D = last ? rem : D;
                float ox = L.ox, oy = L.oy;
                if constexpr (kMovingBackward) {
                    const float rev = fmaf(-L.s_hi, L.dens.omega_rev, L.rev0);
                    ox = L.dens.orbit_r * hw_cos_rev(rev);
                    oy = L.dens.orbit_r * hw_sin_rev(rev);
                }
                float dwx, dwy;
                brownian_increment(odd ? r.r2 : r.r0, odd ? r.r3 : r.r1, -2.77258872f * D, dwx, dwy);
                float bx, by;
                drift<KIND>(L.dens, ox, oy, L.xh, L.yh, bx, by);
                const float x0h = L.xh, x0l = L.xl, y0h = L.yh, y0l = L.yl;
                comp_add(L.xh, L.xl, fmaf(bx, D, dwx));
                comp_add(L.yh, L.yl, fmaf(by, D, dwy));
                if (last) {
                    L.s_hi = L.horizon;
                    L.s_lo = 0.f;
                } else {
                    comp_add(L.s_hi, L.s_lo, D);
                }
                L.k += 1;
                my_steps += 1;
                const float lo = fminf(L.xh, L.yh);
                const float hi = fmaxf((L.xh - 1.f) + L.xl, (L.yh - 1.f) + L.yl);
                out = (lo < 0.f) | (hi > 0.f);
                if (!out) {
                    int side;
                    const float p = bridge_prob(L, x0h, x0l, y0h, y0l, 1.f / D, side);
                    if (side >= 0) {
                        const float ub = fmaf((float)((odd ? q.r1 : q.r0) >> 8), 0x1p-24f, 0x1p-24f);
                        if (ub < p) {
                            move_to_side(L, side);
                            out = true;
                        }
                    }
                }
                if (last) L.K = L.k;
            }
            if (out || L.k >= L.K) {
                float v[2];
                score_path(a, L, out, v[0], v[1]);
                closed = acc_path<2>(slots, accs, my_tag, L.out, v, (uint32_t)L.k);
                if (a.scores) a.scores[path_rec(L, a.n_paths)] = make_float2(v[0], v[1]);
                if (a.exit_step) a.exit_step[path_rec(L, a.n_paths)] = out ? L.k : -1;
                active = false;
            }
        }
    }
    slots_collect<2>(slots, accs, lane);
    unsigned long long st = my_steps;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) st += __shfl_xor(st, off, 64);
    if (lane == 0 && st != 0ull && a.total_steps) atomicAdd(a.total_steps, st);
}

namespace {
template <int KIND, int TMODE, bool UNIFORM, bool BRIDGE, bool FIRST>
hipError_t launch_one(const PathArgs &a, int grid, int block, hipStream_t s) {
    hipLaunchKernelGGL((fk_path_kernel<KIND, TMODE, UNIFORM, BRIDGE, FIRST>), dim3(grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

template <int KIND, int TMODE, bool UNIFORM, bool BRIDGE, bool FIRST>
int max_blocks(int block) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fk_path_kernel<KIND, TMODE, UNIFORM, BRIDGE, FIRST>, block,
                                                     0) != hipSuccess)
        return 0;
    return nb;
}

// Calls F<KIND, TMODE, UNIFORM, BRIDGE, FIRST>::run(args...) for the runtime
// values; the first-chunk-by-index form only for uniform steps without the
// bridge test (a mesh step's sub-steps).
template <template <int, int, bool, bool, bool> class F, typename... Args>
auto dispatch(int kind, int time_mode, bool uniform, bool bridge, bool first_by_index, Args &&...args) {
    const bool frozen = (time_mode == TIME_FROZEN);
#define FK_CASE(K, T)                                                                          \
    if (bridge)                                                                                \
        return uniform ? F<K, T, true, true, false>::run(std::forward<Args>(args)...)         \
                       : F<K, T, false, true, false>::run(std::forward<Args>(args)...);       \
    if (uniform && first_by_index) return F<K, T, true, false, true>::run(std::forward<Args>(args)...); \
    return uniform ? F<K, T, true, false, false>::run(std::forward<Args>(args)...)            \
                   : F<K, T, false, false, false>::run(std::forward<Args>(args)...)
    switch (kind) {
    case KIND_CONST: FK_CASE(KIND_CONST, TIME_BACKWARD);
    case KIND_BUMP: FK_CASE(KIND_BUMP, TIME_BACKWARD);
    case KIND_RIDGE: FK_CASE(KIND_RIDGE, TIME_BACKWARD);
    case KIND_GRID: FK_CASE(KIND_GRID, TIME_BACKWARD);
    case KIND_MOVING:
        if (frozen) { FK_CASE(KIND_MOVING, TIME_FROZEN); }
        FK_CASE(KIND_MOVING, TIME_BACKWARD);
    case KIND_RING:
        if (frozen) { FK_CASE(KIND_RING, TIME_FROZEN); }
        FK_CASE(KIND_RING, TIME_BACKWARD);
    default:
        if (frozen) { FK_CASE(KIND_TWO, TIME_FROZEN); }
        FK_CASE(KIND_TWO, TIME_BACKWARD);
    }
#undef FK_CASE
}

template <int K, int T, bool U, bool B, bool F>
struct LaunchF {
    static hipError_t run(const PathArgs &a, int grid, int block, hipStream_t s) {
        return launch_one<K, T, U, B, F>(a, grid, block, s);
    }
};
template <int K, int T, bool U, bool B, bool F>
struct OccF {
    static int run(int block) { return max_blocks<K, T, U, B, F>(block); }
};

bool kind_known(int kind) {
    return kind == KIND_CONST || kind == KIND_BUMP || kind == KIND_RIDGE || kind == KIND_MOVING || kind == KIND_TWO ||
           kind == KIND_RING || kind == KIND_GRID;
}
}  // namespace

hipError_t launch_paths(int kind, int time_mode, bool uniform, bool first_by_index, const PathArgs &a, int grid,
                        int block, hipStream_t s) {
    if (!kind_known(kind)) return hipErrorInvalidValue;
    return dispatch<LaunchF>(kind, time_mode, uniform, a.score_mode == FK_SCORE_BRIDGE, first_by_index, a, grid,
                             block, s);
}

int path_kernel_max_blocks_per_cu(int kind, int time_mode, bool uniform, bool bridge, bool first_by_index,
                                  int block) {
    if (!kind_known(kind)) return 0;
    return dispatch<OccF>(kind, time_mode, uniform, bridge, first_by_index, block);
}

namespace {
template <int K, int T, bool U, bool B, bool F>
struct ExpoLaunchF {
    static hipError_t run(const PathArgs &a, int grid, int block, hipStream_t s) {
        hipLaunchKernelGGL((fk_expo_path_kernel<K, T>), dim3(grid), dim3(block), 0, s, a);
        return hipGetLastError();
    }
};
template <int K, int T, bool U, bool B, bool F>
struct ExpoOccF {
    static int run(int block) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fk_expo_path_kernel<K, T>, block, 0) != hipSuccess)
            return 0;
        return nb;
    }
};
}  // namespace

// The kind / time-mode dispatch of the fixed-step kernels, with one
// instantiation per pair (uniform, bridge and first-chunk flags unused).
hipError_t launch_expo_paths(int kind, int time_mode, const PathArgs &a, int grid, int block, hipStream_t s) {
    if (!kind_known(kind)) return hipErrorInvalidValue;
    return dispatch<ExpoLaunchF>(kind, time_mode, false, false, false, a, grid, block, s);
}

int expo_kernel_max_blocks_per_cu(int kind, int time_mode, int block) {
    if (!kind_known(kind)) return 0;
    return dispatch<ExpoOccF>(kind, time_mode, false, false, false, block);
}

// ---------------------------------------------------------------------------
// Estimator (Sect. 4: expectations replaced by arithmetic means): the node
// sums of the path kernel -> mean, sample variance (N - 1), standard error,
// in FP64; one thread per output node.
// ---------------------------------------------------------------------------
size_t acc_bytes(int64_t n_out) { return sizeof(NodeAcc) * (size_t)(n_out > 0 ? n_out : 0); }

__global__ void __launch_bounds__(256) fk_finalize_kernel(const FinalArgs f) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= f.n_out) return;
    if (f.mask && !f.mask[o]) return;
    const NodeAcc &A = f.acc[o];
    const double N = (double)f.n_paths;
    double mean[2], se[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double s1 = split_to_double(A.sum[2 * c]) * (1.0 / kQ1);
        const double s2 = split_to_double(A.sum[2 * c + 1]) * (1.0 / kQ2);
        const double m = s1 / N;
        const double var = fmax((s2 - s1 * m) / (N - 1.0), 0.0);
        mean[c] = m;
        se[c] = sqrt(var / N);
    }
    const bool bad = A.bad != 0u;
    const double nan = __builtin_nan("");
    f.xi[o] = bad ? nan : f.outs[o].shift_x + mean[0];
    f.eta[o] = bad ? nan : f.outs[o].shift_y + mean[1];
    f.se_xi[o] = bad ? nan : se[0];
    f.se_eta[o] = bad ? nan : se[1];
    if (f.steps) f.steps[o] = (int64_t)A.steps;
}

hipError_t launch_finalize(const FinalArgs &f, hipStream_t s) {
    if (f.n_out == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((f.n_out + 255) / 256);
    hipLaunchKernelGGL(fk_finalize_kernel, dim3(blocks), dim3(256), 0, s, f);
    return hipGetLastError();
}

}  // namespace fk
