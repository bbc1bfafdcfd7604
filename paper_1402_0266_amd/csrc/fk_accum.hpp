// fk_accum.hpp -- in-kernel accumulation of the Monte-Carlo estimator
// (Sect. 4: expectations replaced by arithmetic means over the paths).
//
// Each finished path adds its score s and s^2 to its node's sums.  The sums
// are kept in fixed point: q1 = round(s 2^48) and q2 = round(s^2 2^45) as
// integers, so every partial sum is an exact integer and any grouping or
// order of the additions gives bitwise the same totals -- the results do not
// depend on the launch plan or on which lane ran which path.  A score is
// rounded by at most 2^-49 (s^2 by 2^-46) before it is summed.
//
// Two levels:
//  * per wavefront, an LDS table of kAccSlots open work chunks: a path adds
//    q1, q2 and (with the chunk's count of unfinished paths, in one word) its
//    step count to its chunk's slot with 64-bit LDS atomics;
//    a slot whose paths have all finished is flushed to its node's
//    accumulator in HBM by the whole wavefront at the top of its next
//    iteration (and at its end).  A chunk grabbed while every slot still has paths running
//    gets no slot, and its paths add to HBM directly.
//  * per output node, a NodeAcc in HBM: each sum as two 64-bit integer sums
//    of the terms' high and low parts (plain atomic adds, exact, no carries),
//    the step count and a count of rejected paths; a finalize kernel turns
//    them into the mean, the sample variance (N - 1) and the standard error
//    in FP64.
// A slot's sums stay below 2^62 for chunks of at most kMaxChunk paths with
// |s| < kLdsBound; scores with kLdsBound <= |s| < kGlobalBound go to HBM
// directly; a non-finite score or one beyond kGlobalBound is rejected and
// the node's results become NaN.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fk {

constexpr int kAccSlots = 8;                   // open chunks per wavefront (power of two)
constexpr uint32_t kMaxChunk = 2048;           // paths per chunk the LDS slots can hold
constexpr double kQ1 = 0x1p48;                 // fixed-point scale of a score
constexpr double kQ2 = 0x1p45;                 // ... of a squared score
constexpr float kLdsBound = 8.f;               // |s| < 8: q1 < 2^51, q2 < 2^51
constexpr float kGlobalBound = 512.f;          // |s| < 512: q1 < 2^57, q2 < 2^63

// Per output node, zeroed before the path kernel.  Each sum S (an exact
// integer) is kept as two 64-bit integer sums, S = hi 2^24 + lo, of the
// parts hi = S_i >> 24 (arithmetic) and lo = S_i & (2^24 - 1) of the terms
// S_i added to it (a closed chunk's sum, or one path's q): plain 64-bit
// atomic adds, no carries, and neither part can overflow for up to 2^24
// terms per node.  v = 0: q1 of xi, 1: q2 of xi, 2: q1 of eta, 3: q2 of eta.
struct alignas(16) NodeAcc {
    unsigned long long sum[4][2];   // [v][0] = sum of hi parts, [v][1] = sum of lo parts
    unsigned long long steps;
    uint32_t bad;
    uint32_t pad;
};

// Adds one term (signed, |x| < 2^63) to a split sum; no return values.
__device__ __forceinline__ void add_split(unsigned long long *p, long long x) {
    atomicAdd(p, (unsigned long long)(x >> 24));
    atomicAdd(p + 1, (unsigned long long)(x & 0xffffffll));
}

// One open chunk of a wavefront.  NV values per path: 2 (xi, eta) or 4
// (plain xi, eta and control-variate xi, eta).
template <int NV>
struct AccSlot {
    uint32_t tag;        // (grab number << 3) | slot index of the chunk held, or kSlotFree
    uint32_t out;        // output row of the chunk's node
    unsigned long long cnt;            // (paths not finished) << 48 | steps of the finished ones
    unsigned long long m[2 * NV];      // per value: q1 sum, q2 sum
};
constexpr unsigned long long kCntOne = 1ull << 48;   // one unfinished path in AccSlot::cnt
constexpr unsigned long long kStepMask = kCntOne - 1;
constexpr uint32_t kSlotFree = 0xffffffffu;
constexpr uint32_t kNoSlot = 0xfffffffeu;   // a chunk that found no free slot: its paths add to HBM

// Orders this wavefront's LDS accesses (the compiler must not move them
// across; the hardware keeps one wavefront's LDS operations in order).
__device__ __forceinline__ void lds_order() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup"); }
// Wave-uniform: flushes every closed slot of the wavefront to the node sums
// (lane 2 v + k adds moment k of value v, lane 2 NV the step count) and
// frees it.
template <int NV>
__device__ __forceinline__ void slots_collect(AccSlot<NV> *slots, NodeAcc *const *acc, uint32_t lane) {
    lds_order();
    bool closed = false;
    if (lane < (uint32_t)kAccSlots) closed = slots[lane].tag != kSlotFree && slots[lane].cnt < kCntOne;
    uint64_t cm = __ballot(closed);
    while (cm != 0ull) {
        const int j = __builtin_ctzll(cm);
        cm &= cm - 1ull;
        const AccSlot<NV> &S = slots[j];
        if (lane < (uint32_t)(2 * NV)) {
            // lane 2 v + k: moment k of value v
            const uint32_t v = lane >> 1, k = lane & 1u;
            add_split(acc[v >> 1][S.out].sum[2 * (v & 1u) + k], (long long)S.m[lane]);
        } else if (lane == (uint32_t)(2 * NV)) {
            if (S.cnt != 0ull) atomicAdd(&acc[0][S.out].steps, S.cnt);
        }
        lds_order();
        if (lane == 0) slots[j].tag = kSlotFree;
    }
    lds_order();
}

// Wave-uniform: the wavefront has grabbed a chunk of `n` paths for output row
// `out` as its grab number `seq`.  Returns the chunk's tag: a free slot
// reset for it, or kNoSlot when no slot is free.  Every lane of the
// wavefront calls this.
template <int NV>
__device__ __forceinline__ uint32_t slot_open(AccSlot<NV> *slots, NodeAcc *const *acc, uint32_t seq, uint32_t out,
                                              uint32_t n, uint32_t lane) {
    // free slots (closed ones wait for slots_collect)
    lds_order();
    const uint32_t fm = (uint32_t)__ballot(lane < (uint32_t)kAccSlots && slots[lane & (kAccSlots - 1)].tag == kSlotFree);
    if (fm == 0u) return kNoSlot;
    const uint32_t j = (uint32_t)__builtin_ctz(fm);
    const uint32_t tag = (seq << 3) | j;
    AccSlot<NV> &S = slots[j];
    if (lane < (uint32_t)(2 * NV)) S.m[lane] = 0ull;
    if (lane == 0) {
        S.tag = tag;
        S.out = out;
        S.cnt = (unsigned long long)n * kCntOne;
    }
    lds_order();
    return tag;
}

// Wave start: every slot free.
template <int NV>
__device__ __forceinline__ void slots_init(AccSlot<NV> *slots, uint32_t lane) {
    if (lane < (uint32_t)kAccSlots) slots[lane].tag = kSlotFree;
    lds_order();
}

// q1 = round(s 2^48) and q2 = round(s^2 2^45) for |s| < kLdsBound, as the
// FP64 expressions round them (to nearest, ties to even), by adding a
// constant that puts the integer part in the low mantissa bits: 1.5 2^52
// keeps s 2^48 (|.| < 2^51) inside [2^52, 2^53), where the double's bit
// pattern counts units; the same with 2^52 for s^2 2^45 (< 2^51, and s^2 is
// exact in FP64).
__device__ __forceinline__ long long q1_small(float s) {
    const double t = fma((double)s, 0x1p48, 0x1.8p52);
    return __double_as_longlong(t) - 0x4338000000000000ll;   // bits of 1.5 2^52
}
__device__ __forceinline__ long long q2_small(float s) {
    const double d = (double)s;
    const double t = fma(d * d, 0x1p45, 0x1p52);
    return __double_as_longlong(t) - 0x4330000000000000ll;   // bits of 2^52
}

// A finished path (divergent: only finishing lanes call it).  v[NV]: its
// values relative to the node's shift; tag: its chunk's tag; out: its
// output row; steps: the Euler-Maruyama steps it took.  The path that
// finishes a chunk leaves its slot closed and returns true; the wavefront
// then calls slots_collect.
template <int NV>
__device__ __forceinline__ bool acc_path(AccSlot<NV> *slots, NodeAcc *const *acc, uint32_t tag, uint32_t out,
                                         const float (&v)[NV], uint32_t steps) {
    float amax = 0.f;
#pragma unroll
    for (int i = 0; i < NV; ++i) amax = fmaxf(amax, fabsf(v[i]));
    const bool finite = amax < kGlobalBound;      // false for NaN and infinities too
    AccSlot<NV> &S = slots[tag & (uint32_t)(kAccSlots - 1)];
    lds_order();
    const bool mine = tag != kNoSlot && S.tag == tag;
    const bool in_lds = mine && amax < kLdsBound;
    if (in_lds) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            atomicAdd(&S.m[2 * i], (unsigned long long)q1_small(v[i]));
            atomicAdd(&S.m[2 * i + 1], (unsigned long long)q2_small(v[i]));
        }
    } else if (finite) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const double d = (double)v[i];
            NodeAcc &A = acc[i >> 1][out];
            const int c = i & 1;
            add_split(A.sum[2 * c], __double2ll_rn(d * kQ1));
            add_split(A.sum[2 * c + 1], (long long)__double2ull_rn(d * d * kQ2));   // s^2 is exact in FP64
        }
    } else {
#pragma unroll
        for (int i = 0; i < NV; i += 2) atomicAdd(&acc[i >> 1][out].bad, 1u);
    }
    bool closed = false;
    if (mine) {
        lds_order();
        // one path fewer to wait for, and its steps, in one atomic
        closed = (atomicAdd(&S.cnt, (unsigned long long)steps - kCntOne) >> 48) == 1ull;
        lds_order();
    } else {
        atomicAdd(&acc[0][out].steps, (unsigned long long)steps);
    }
    return closed;
}

// The paths that finished in this iteration of the wavefront, from
// converged code (every lane calls this; fin marks the lanes whose path
// finished, with its values v, chunk tag, output row and step count); closed
// slots are flushed at once.
template <int NV>
__device__ __forceinline__ void acc_wave(AccSlot<NV> *slots, NodeAcc *const *acc, bool fin, uint32_t tag,
                                         uint32_t out, const float (&v)[NV], uint32_t steps, uint32_t lane) {
    if (__ballot(fin) == 0ull) return;
    bool cl = false;
    if (fin) cl = acc_path<NV>(slots, acc, tag, out, v, steps);
    if (__ballot(cl) != 0ull) slots_collect<NV>(slots, acc, lane);
}

// A split sum as FP64: hi 2^24 + lo, both exact in FP64 while |hi| < 2^53,
// one rounding in the addition.
__device__ __forceinline__ double split_to_double(const unsigned long long (&p)[2]) {
    return (double)(long long)p[0] * 0x1p24 + (double)(long long)p[1];
}

}  // namespace fk
