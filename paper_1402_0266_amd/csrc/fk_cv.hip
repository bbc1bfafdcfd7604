// fk_cv.hip -- the learned control variate: a tanh MLP u_hat(t, x, y) ->
// (xi_hat, eta_hat), 3 -> 64 -> 64 -> 64 -> 2 on z = (2t/T - 1, 2x - 1, 2y - 1),
// with BF16 weights.
//
//  * Training: mean-squared error on (t, x, y) -> Monte-Carlo interface
//    estimates, Adam (FP32 master weights and moments).  Forward and
//    backward run on BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulate)
//    over LDS-resident 64-sample tiles; the per-tile weight gradients are
//    summed in a fixed order by the Adam kernel.
//  * Evaluation: forward-mode value, d/dx, d/dy, d/dt and Laplacian of both
//    outputs, wavefront-wide: 16 points per round, the derivative channels
//    as MFMA column blocks.  A 16x16x32 product's output (lane = point
//    column, 4 consecutive units per lane group) of two adjacent 16-unit
//    tiles is the B operand of one 32-unit K block of the next layer, once
//    the K order inside the block is permuted alike in the weights, so
//    layers chain in registers.  Activations are split into BF16 hi + lo
//    parts (two MFMAs per product) so that the evaluation carries ~16
//    mantissa bits: the Dynkin-form estimator is only unbiased if value and
//    derivative channels describe one function consistently.  The martingale
//    form's gradient may instead round activations to BF16 once (one MFMA
//    per product): its estimator stays unbiased for any gradient fixed
//    before the block's increments.
//  * The control-variate path kernel: plain Euler-Maruyama paths (same
//    counters as fk_interface_solve) plus, every `stride` steps and at the
//    path's end, the integrand r = Laplacian u_hat + b . grad u_hat - d_t u_hat
//    (trapezoidal rule in between); the score is g - u_hat(end) + sum r ds.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "fk.h"
#include "fk_accum.hpp"
#include "fk_device.hpp"
#include "fk_internal.hpp"
#include "fk_pathstep.hpp"

typedef __bf16 fk_b8 __attribute__((ext_vector_type(8)));
typedef float fk_f4 __attribute__((ext_vector_type(4)));

namespace fk {

constexpr int kNP = 8706;
constexpr int OW1 = 0, OB1 = 192, OW2 = 256, OB2 = 4352, OW3 = 4416, OB3 = 8512, OW4 = 8576, OB4 = 8704;
constexpr int kWS = 72;  // padded LDS row stride (bf16 elements) of W2 / W3: rows on 16-byte boundaries

struct TrainDesc;

// A captured training loop: `steps` iterations of (gradient, Adam) for a
// minibatch of `batch` samples, replayed by fk_cv_train.
struct TrainGraph {
    int steps = 0;
    int64_t batch = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct CvState {
    TrainDesc *desc = nullptr; // per-call values of fk_cv_train (device)
    float *master = nullptr;   // [kNP] FP32
    float *m = nullptr;        // Adam first moment
    float *v = nullptr;        // Adam second moment
    uint16_t *bf = nullptr;    // [kNP] BF16 bits: the network every kernel uses
    float *partial = nullptr;  // [cap_tiles][kNP + 1] per-tile gradients (+ loss)
    int cap_tiles = 0;
};

}  // namespace fk

struct fk_cv {
    int device = 0;
    hipStream_t capture_stream = nullptr;     // where training loops are captured (never run on)
    std::vector<fk::TrainGraph> graphs;       // captured training loops
    float t_scale = 0.1f;
    float base = 0.f;    // 1: u_hat = (x, y) + network (the identity base)
    int grid_base = 0;   // 1: u_hat = bilinear(grid initial data) + network (martingale solves)
    int grad_bf16 = 0;   // 1: the martingale forms take the network's gradient with BF16-rounded
                         // activations (FK_CV_GRAD_BF16), else with hi + lo operands
    int64_t steps_done = 0;
    fk::CvState s;
};

namespace fk {

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// ---------------------------------------------------------------------------
// The network in LDS.
// ---------------------------------------------------------------------------
// 2 log2(e): tanh(a) = 1 - 2 / (1 + 2^(a K2)).
constexpr float K2 = 2.8853900817779268f;

struct NetLds {
    float w1[64 * 3];
    float b1[64], b2[64], b3[64];
    float w4[128];
    float b4[2];
    uint16_t w2[64 * kWS];
    uint16_t w3[64 * kWS];
    // for the gradient evaluation: per unit u (K2 w0, K2 w1, K2 w2, K2 b1);
    // per group of four units 4 q .. 4 q + 3 (the four a lane takes from one
    // 16x16 output tile) K2 b2, K2 b3, W4[0] and W4[1]
    float4 g1[64];
    float4 q2[16], q3[16], q40[16], q41[16];
};

// Column position of unit k of a W2 / W3 row in LDS: inside each 32-unit
// block, the units lane group g takes as MFMA operand elements 0-7 (ku: 4 g
// .. 4 g + 3 and 16 + 4 g .. 16 + 4 g + 3) sit next to each other at 8 g, so
// an operand is one 16-byte read.
__device__ __forceinline__ int wcol(int k) {
    const int b = k & 31;
    return (k & ~31) | (8 * ((b & 15) >> 2) + 4 * (b >> 4) + (b & 3));
}

__device__ void load_net(NetLds &N, const uint16_t *bf) {
    for (int i = threadIdx.x; i < 192; i += blockDim.x) N.w1[i] = bf2f(bf[OW1 + i]);
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
        N.b1[i] = bf2f(bf[OB1 + i]);
        N.b2[i] = bf2f(bf[OB2 + i]);
        N.b3[i] = bf2f(bf[OB3 + i]);
    }
    for (int i = threadIdx.x; i < 128; i += blockDim.x) N.w4[i] = bf2f(bf[OW4 + i]);
    if (threadIdx.x < 2) N.b4[threadIdx.x] = bf2f(bf[OB4 + threadIdx.x]);
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) {
        const int r = i >> 6, c = i & 63;
        N.w2[r * kWS + wcol(c)] = bf[OW2 + i];
        N.w3[r * kWS + wcol(c)] = bf[OW3 + i];
    }
    for (int u = threadIdx.x; u < 64; u += blockDim.x) {
        const float w0 = bf2f(bf[OW1 + 3 * u]), w1 = bf2f(bf[OW1 + 3 * u + 1]), w2 = bf2f(bf[OW1 + 3 * u + 2]);
        N.g1[u] = make_float4(K2 * w0, K2 * w1, K2 * w2, K2 * bf2f(bf[OB1 + u]));
        reinterpret_cast<float *>(N.q2)[u] = K2 * bf2f(bf[OB2 + u]);
        reinterpret_cast<float *>(N.q3)[u] = K2 * bf2f(bf[OB3 + u]);
        reinterpret_cast<float *>(N.q40)[u] = bf2f(bf[OW4 + u]);
        reinterpret_cast<float *>(N.q41)[u] = bf2f(bf[OW4 + 64 + u]);
    }
}

// tanh and its forward-mode channels: h = tanh(a), s = 1 - h^2 = 4 e / (1+e)^2
// with e = exp(2a); dh = s da; Laplacian h = s (Laplacian a - 2 h |grad a|^2).
__device__ __forceinline__ void act5(float a, float ax, float ay, float at, float al, float &h, float &hx,
                                     float &hy, float &ht, float &hl) {
    const float ac = fminf(fmaxf(a, -15.f), 15.f);
    const float e = hw_exp2(ac * K2);
    const float r = hw_rcp(1.f + e);
    h = fmaf(-2.f, r, 1.f);
    const float s = 4.f * e * r * r;
    hx = s * ax;
    hy = s * ay;
    ht = s * at;
    hl = s * fmaf(-2.f * h, fmaf(ax, ax, ay * ay), al);
}

// The identity base (base = 1): u_hat = (x, y) + network, so the value of
// xi gains x and that of eta gains y, and their gradients the identity; the
// d/dtau and Laplacian channels are unchanged.
__device__ __forceinline__ void add_base(float base, float x, float y, float o[2][5]) {
    o[0][0] = fmaf(base, x, o[0][0]);
    o[1][0] = fmaf(base, y, o[1][0]);
    o[0][1] += base;
    o[1][2] += base;
}
__device__ __forceinline__ void add_base_grad(float base, float o[2][2]) {
    o[0][0] += base;
    o[1][1] += base;
}

__device__ __forceinline__ fk_f4 mfma32(fk_b8 a, fk_b8 b, fk_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// K order of the 32-unit block kb inside a product: lane group g's operand
// element j is unit ku(kb, g, j) = 32 kb + 16 (j / 4) + 4 g + j % 4, i.e.
// elements 0-3 are the 16x16 output rows 4 g .. 4 g + 3 of tile 2 kb and
// elements 4-7 those of tile 2 kb + 1.  A and B use the same order, so the
// product sums every unit of the block once.
__device__ __forceinline__ int ku(int kb, int g, int j) { return 32 * kb + 16 * (j >> 2) + 4 * g + (j & 3); }

// A operand of a padded BF16 weight matrix: lane (g, n) holds
// W[16 mt + n][ku(kb, g, 0..7)], 16 bytes at column 32 kb + 8 g (wcol).
__device__ __forceinline__ fk_b8 load_a(const uint16_t *W, int mt, int kb, int n, int g) {
    return __builtin_bit_cast(fk_b8, *reinterpret_cast<const uint4 *>(W + (16 * mt + n) * kWS + 32 * kb + 8 * g));
}

// BF16 hi (+ lo with SPLIT) operand element of an FP32 value.
template <bool SPLIT>
__device__ __forceinline__ void put_bf16(float v, fk_b8 &hi, fk_b8 &lo, int j) {
    const __bf16 h = (__bf16)v;
    hi[j] = h;
    if constexpr (SPLIT) lo[j] = (__bf16)(v - (float)h);
}

// Wavefront-wide forward-mode evaluation.  Every lane of the wavefront must
// call it.  Lane l's point is (tau, x, y); on return out[o][c] holds, for
// output o, channel c = value, d/dx, d/dy, d/dtau, Laplacian (x, y).
// Activations enter the products as BF16 hi + lo pairs.
//
// Register budget: per round (16 points) at most the layer-2 accumulators
// (4 output tiles x 5 channels x 4) plus one operand block are live; layer 1
// is computed per K block as it is consumed, and layer 3 per output tile from
// the hi/lo operands of both K blocks.
__device__ void net_eval_wave(const NetLds &N, float tscale2, float tau, float x, float y, float out[2][5]) {
    const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
#pragma unroll 1
    for (int r = 0; r < 4; ++r) {
        // an index offset the compiler cannot see through: keeps the weight
        // reads inside the loop instead of hoisting them into registers
        int lz = 0;
        asm volatile("" : "+s"(lz));
        const NetLds &M = *reinterpret_cast<const NetLds *>(reinterpret_cast<const char *>(&N) + lz);
        const int src = 16 * r + n;
        const float z0 = __shfl(tau, src, 64) * tscale2 - 1.f;
        const float z1 = 2.f * __shfl(x, src, 64) - 1.f;
        const float z2 = 2.f * __shfl(y, src, 64) - 1.f;
        // ---- layer 2 pre-activations, K block by K block ---------------------
        fk_f4 acc[4][5];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int c = 0; c < 5; ++c) acc[mt][c] = fk_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            // layer 1 (VALU) for units ku(kb, g, j) of point n
            fk_b8 Bh[5], Bl[5];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int u = ku(kb, g, j);
                const float w0 = M.w1[3 * u], w1 = M.w1[3 * u + 1], w2 = M.w1[3 * u + 2];
                const float a = fmaf(w0, z0, fmaf(w1, z1, fmaf(w2, z2, M.b1[u])));
                float ch[5];
                act5(a, 2.f * w1, 2.f * w2, tscale2 * w0, 0.f, ch[0], ch[1], ch[2], ch[3], ch[4]);
#pragma unroll
                for (int c = 0; c < 5; ++c) put_bf16<true>(ch[c], Bh[c], Bl[c], j);
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const fk_b8 A = load_a(M.w2, mt, kb, n, g);
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    acc[mt][c] = mfma32(A, Bh[c], acc[mt][c]);
                    acc[mt][c] = mfma32(A, Bl[c], acc[mt][c]);
                }
            }
        }
        // ---- layer 2 activations -> layer 3 operands -------------------------
        fk_b8 Ch[2][5], Cl[2][5];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int mt = 2 * kb + (j >> 2), i = j & 3, u = ku(kb, g, j);
                float ch[5];
                act5(acc[mt][0][i] + M.b2[u], acc[mt][1][i], acc[mt][2][i], acc[mt][3][i], acc[mt][4][i], ch[0], ch[1],
                     ch[2], ch[3], ch[4]);
#pragma unroll
                for (int c = 0; c < 5; ++c) put_bf16<true>(ch[c], Ch[kb][c], Cl[kb][c], j);
            }
        // ---- layer 3, one output tile at a time, into the output layer -------
        float po[2][5];
#pragma unroll
        for (int o = 0; o < 2; ++o)
#pragma unroll
            for (int c = 0; c < 5; ++c) po[o][c] = 0.f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            fk_f4 a3[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) a3[c] = fk_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const fk_b8 A = load_a(M.w3, mt, kb, n, g);
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    a3[c] = mfma32(A, Ch[kb][c], a3[c]);
                    a3[c] = mfma32(A, Cl[kb][c], a3[c]);
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = 16 * mt + 4 * g + i;
                float ch[5];
                act5(a3[0][i] + M.b3[u], a3[1][i], a3[2][i], a3[3][i], a3[4][i], ch[0], ch[1], ch[2], ch[3], ch[4]);
#pragma unroll
                for (int o = 0; o < 2; ++o) {
                    const float w = M.w4[64 * o + u];
#pragma unroll
                    for (int c = 0; c < 5; ++c) po[o][c] = fmaf(w, ch[c], po[o][c]);
                }
            }
        }
        // ---- output layer: sum over the four lane groups of point n ---------
#pragma unroll
        for (int o = 0; o < 2; ++o)
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                float v = po[o][c];
                v += __shfl_xor(v, 16, 64);
                v += __shfl_xor(v, 32, 64);
                if (c == 0) v += M.b4[o];
                if (g == r) out[o][c] = v;
            }
    }
}

// tanh with its first derivatives from the pre-activation scaled by K2
// (as = K2 a): h = tanh(a) = 1 - 2 / (1 + 2^as), s = 1 - h^2, dh = s da.
// Saturated units need no clamp: 2^as = inf gives h = 1, s = 0, and 2^as = 0
// gives h = -1, s = 0.  s is formed as 1 - h^2 (one FMA; its absolute error
// ~1e-7 is far below the operands' BF16 rounding).
__device__ __forceinline__ void act3(float as, float ax, float ay, float &h, float &hx, float &hy) {
    const float r = hw_rcp(1.f + hw_exp2(as));
    h = fmaf(-2.f, r, 1.f);
    const float s = fmaf(-h, h, 1.f);
    hx = s * ax;
    hy = s * ay;
}

// A 16-byte LDS value at a compile-time field address plus a per-lane byte
// offset (one ds_read_b128 with the field address as its immediate offset;
// every read of the gradient evaluation is such a full 16-byte read, so none
// is merged into a two-address read, whose 8-bit offsets could not hold it).
template <typename T>
__device__ __forceinline__ T lds_at(const T *field, int byte_off) {
    static_assert(sizeof(T) == 16, "16-byte reads only");
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(field) + byte_off);
}

// A operand of W2 / W3 (as load_a) from the lane's byte offset 2 (n kWS + 8 g).
__device__ __forceinline__ fk_b8 load_a_at(const uint16_t *W, int mt, int kb, int off_w) {
    return __builtin_bit_cast(fk_b8, lds_at(reinterpret_cast<const uint4 *>(W + 16 * mt * kWS + 32 * kb), off_w));
}

// Wavefront-wide gradient of both outputs in (x, y) at lane l's point, for
// the martingale form: out[o] = (d/dx, d/dy) of output o.  Three channels
// (value, d/dx, d/dy).  SPLIT: the operands are BF16 hi + lo pairs as in
// net_eval_wave, and the gradient matches the FP64 evaluation of the network
// to ~1e-5 relative; otherwise activations are rounded to BF16 once (half
// the products and operand conversions; ~1e-2 relative).
//
// Every LDS read is a field address known at compile time plus one of four
// per-lane byte offsets (lane group g's units sit 4 g on, lane n's weight
// row n kWS on).  The offsets pass through an empty asm each round, so the
// reads stay inside the round (the weights are not hoisted into registers)
// and fold into the reads' immediate offsets.
template <bool SPLIT>
__device__ void net_grad_wave(const NetLds &N, float tscale2, float tau, float x, float y, float out[2][2]) {
    const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
#pragma unroll 1
    for (int r = 0; r < 4; ++r) {
        int off_g = 64 * g, off_q = 16 * g, off_w = 2 * (n * kWS + 8 * g);
        asm volatile("" : "+v"(off_g), "+v"(off_q), "+v"(off_w));
        const int src = 16 * r + n;
        const float z0 = __shfl(tau, src, 64) * tscale2 - 1.f;
        const float z1 = 2.f * __shfl(x, src, 64) - 1.f;
        const float z2 = 2.f * __shfl(y, src, 64) - 1.f;
        // Layer 1 (VALU) for units ku(kb, g, j) of point n.  The derivative
        // channels start from K2 w (not 2 w): they are linear through the
        // network, so the outputs are scaled back by 2 / K2 at the end.
        auto layer1 = [&](int kb, fk_b8 (&Bh)[3], fk_b8 (&Bl)[3]) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float4 gw = lds_at(N.g1 + ku(kb, 0, j), off_g);   // lane group g's unit is 4 g on
                const float as = fmaf(gw.x, z0, fmaf(gw.y, z1, fmaf(gw.z, z2, gw.w)));
                float ch[3];
                act3(as, gw.y, gw.z, ch[0], ch[1], ch[2]);
#pragma unroll
                for (int c = 0; c < 3; ++c) put_bf16<SPLIT>(ch[c], Bh[c], Bl[c], j);
            }
        };
        // Layer-2 tile mt's activations into the layer-3 operands: tile mt is
        // elements 4 (mt % 2) .. + 3 of K block mt / 2.
        fk_b8 Ch[2][3], Cl[2][3];
        auto act2 = [&](int mt, const fk_f4 (&a2)[3]) {
            const float4 b2 = lds_at(N.q2 + 4 * mt, off_q);   // units 16 mt + 4 g + 0..3
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float ch[3];
                act3(fmaf(a2[0][i], K2, b2[i]), a2[1][i], a2[2][i], ch[0], ch[1], ch[2]);
#pragma unroll
                for (int c = 0; c < 3; ++c) put_bf16<SPLIT>(ch[c], Ch[mt >> 1][c], Cl[mt >> 1][c], 4 * (mt & 1) + i);
            }
        };
        if constexpr (SPLIT) {
            // K block by K block: one block's hi + lo operands and all four
            // tiles' accumulators live
            fk_f4 acc[4][3];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[mt][c] = fk_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                fk_b8 Bh[3], Bl[3];
                layer1(kb, Bh, Bl);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    const fk_b8 A = load_a_at(N.w2, mt, kb, off_w);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        acc[mt][c] = mfma32(A, Bh[c], acc[mt][c]);
                        acc[mt][c] = mfma32(A, Bl[c], acc[mt][c]);
                    }
                }
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) act2(mt, acc[mt]);
        } else {
            // both K blocks' operands (half the registers of a hi + lo pair),
            // then tile by tile: one tile's accumulators live
            fk_b8 B[2][3], unused[3];
            layer1(0, B[0], unused);
            layer1(1, B[1], unused);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                fk_f4 a2[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) a2[c] = fk_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    const fk_b8 A = load_a_at(N.w2, mt, kb, off_w);
#pragma unroll
                    for (int c = 0; c < 3; ++c) a2[c] = mfma32(A, B[kb][c], a2[c]);
                }
                act2(mt, a2);
            }
        }
        // ---- layer 3, one output tile at a time, into the output layer -------
        float po[2][2] = {{0.f, 0.f}, {0.f, 0.f}};
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            fk_f4 a3[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) a3[c] = fk_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const fk_b8 A = load_a_at(N.w3, mt, kb, off_w);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    a3[c] = mfma32(A, Ch[kb][c], a3[c]);
                    if constexpr (SPLIT) a3[c] = mfma32(A, Cl[kb][c], a3[c]);
                }
            }
            const float4 b3 = lds_at(N.q3 + 4 * mt, off_q), v0 = lds_at(N.q40 + 4 * mt, off_q),
                         v1 = lds_at(N.q41 + 4 * mt, off_q);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float h, hx, hy;
                act3(fmaf(a3[0][i], K2, b3[i]), a3[1][i], a3[2][i], h, hx, hy);
                po[0][0] = fmaf(v0[i], hx, po[0][0]);
                po[0][1] = fmaf(v0[i], hy, po[0][1]);
                po[1][0] = fmaf(v1[i], hx, po[1][0]);
                po[1][1] = fmaf(v1[i], hy, po[1][1]);
            }
        }
#pragma unroll
        for (int o = 0; o < 2; ++o)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                float v = po[o][c];
                v += __shfl_xor(v, 16, 64);
                v += __shfl_xor(v, 32, 64);
                if (g == r) out[o][c] = v * (2.f / K2);
            }
    }
}

// ---------------------------------------------------------------------------
// Evaluation at given points (also the parity hook of the path evaluation).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) cv_eval_kernel(const uint16_t *bf, float tscale2, float base, const float *txy,
                                                      int64_t n, float *out) {
    __shared__ NetLds N;
    load_net(N, bf);
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = i < n;
    const float t = ok ? txy[3 * i] : 0.f, x = ok ? txy[3 * i + 1] : 0.5f, y = ok ? txy[3 * i + 2] : 0.5f;
    float o[2][5];
    net_eval_wave(N, tscale2, t, x, y, o);
    add_base(base, x, y, o);
    if (ok)
        for (int c = 0; c < 2; ++c)
            for (int k = 0; k < 5; ++k) out[10 * i + 5 * c + k] = o[c][k];
}

// The network's (x, y) gradient at given points, as the martingale path
// kernels take it (the parity hook of their evaluation).
template <bool SPLIT>
__global__ void __launch_bounds__(256) cv_eval_grad_kernel(const uint16_t *bf, float tscale2, float base,
                                                           const float *txy, int64_t n, float *out) {
    __shared__ NetLds N;
    load_net(N, bf);
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = i < n;
    const float t = ok ? txy[3 * i] : 0.f, x = ok ? txy[3 * i + 1] : 0.5f, y = ok ? txy[3 * i + 2] : 0.5f;
    float o[2][2];
    net_grad_wave<SPLIT>(N, tscale2, t, x, y, o);
    add_base_grad(base, o);
    if (ok)
        for (int c = 0; c < 2; ++c)
            for (int k = 0; k < 2; ++k) out[4 * i + 2 * c + k] = o[c][k];
}

// ---------------------------------------------------------------------------
// Control-variate path kernel.
// ---------------------------------------------------------------------------
struct CvArgs {
    const uint16_t *bf;
    float tscale2;               // 2 / T
    uint32_t stride_iters;       // network evaluations every stride_iters iterations (2 steps each)
    float base;                  // identity base (0 or 1)
    const float2 *r0;            // [n_out] integrand at the start point of each node
    NodeAcc *acc_cv;             // [n_out] sums of the CV scores
    float2 *cv_scores;           // [n_out * n_paths] or nullptr
};

template <int KIND, int TMODE, bool UNIFORM>
__device__ __forceinline__ void drift_at(const Lane &L, float &bx, float &by) {
    float ox = L.ox, oy = L.oy;
    if constexpr (moving_kind(KIND) && TMODE == TIME_BACKWARD) {
        const float rev = fmaf(-(float)L.k, L.drev, L.rev0);
        ox = L.dens.orbit_r * hw_cos_rev(rev);
        oy = L.dens.orbit_r * hw_sin_rev(rev);
    }
    drift<KIND>(L.dens, ox, oy, L.xh, L.yh, bx, by);
}

// Drift at the lane's position and PDE time tau (end states).
template <int KIND, int TMODE>
__device__ __forceinline__ void drift_at_tau(const Lane &L, float tau, float &bx, float &by) {
    float ox = L.ox, oy = L.oy;
    if constexpr (moving_kind(KIND) && TMODE == TIME_BACKWARD) {
        const float rev = tau * L.dens.omega_rev;
        ox = L.dens.orbit_r * hw_cos_rev(rev);
        oy = L.dens.orbit_r * hw_sin_rev(rev);
    }
    drift<KIND>(L.dens, ox, oy, L.xh, L.yh, bx, by);
}

template <int KIND, int TMODE, bool UNIFORM>
__global__ void __launch_bounds__(256, 2) fk_cv_path_kernel(const PathArgs a, const CvArgs c) {
    constexpr bool kMovingBackward = moving_kind(KIND) && TMODE == TIME_BACKWARD;
    __shared__ NetLds N;
    load_net(N, c.bf);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    __shared__ AccSlot<2> slot_tab[4][kAccSlots];
    AccSlot<2> *slots = slot_tab[threadIdx.x >> 6];
    NodeAcc *const accs[1] = {c.acc_cv};
    slots_init<2>(slots, lane);
    uint32_t q_slot = 0, q_next = 0, q_end = 0, q_tag = 0, grabs = 0;
    const uint32_t total_chunks = launch_chunks(a);
    bool q_done = !grab_chunk<2>(a, total_chunks, first_chunk(), q_slot, q_next, q_end, slots, accs, q_tag, grabs, lane);
    const uint32_t key0 = a.key0, key1 = a.key1;
    Lane L;
    bool active = false, parked = false, out = false;
    float plx = 0.f, ply = 0.f;              // plain score of a parked path
    float Ix = 0.f, Iy = 0.f;                // sum of r ds
    float rx = 0.f, ry = 0.f;                // integrand at the last evaluation
    int32_t k_last = 0;
    const float tend = a.levels[0].tend;     // PDE time at path start
    uint32_t my_tag = 0;                     // accumulation tag of the path's chunk
    uint32_t my_steps = 0;
    uint32_t until_eval = 0;                 // iterations to the next evaluation point

    for (;; --until_eval) {
        if (until_eval == 0) {
            until_eval = c.stride_iters;
            // ---- evaluation point: integrand of running paths, end value of
            //      parked ones (every lane of the wavefront joins) ------------
            if (__ballot(active || parked) != 0ull) {
                const bool ev = active || parked;
                const float sk = (parked && L.k >= L.K) ? L.horizon : (float)L.k * L.dt;
                const float tau = ev ? tend - sk : 0.f;
                float o[2][5];
                net_eval_wave(N, c.tscale2, tau, ev ? L.xh : 0.5f, ev ? L.yh : 0.5f, o);
                add_base(c.base, L.xh, L.yh, o);
                // integrand at this state; for a parked path its end state,
                // with the drift at the end time
                float bx = 0.f, by = 0.f;
                if (active) drift_at<KIND, TMODE, UNIFORM>(L, bx, by);
                if (parked) drift_at_tau<KIND, TMODE>(L, tau, bx, by);
                const float rnx = o[0][4] + fmaf(bx, o[0][1], by * o[0][2]) - o[0][3];
                const float rny = o[1][4] + fmaf(bx, o[1][1], by * o[1][2]) - o[1][3];
                if (ev) {
                    // trapezoidal rule over the interval since the last evaluation
                    const float ds = sk - (float)k_last * L.dt;
                    Ix = fmaf(0.5f * (rx + rnx), ds, Ix);
                    Iy = fmaf(0.5f * (ry + rny), ds, Iy);
                    rx = rnx;
                    ry = rny;
                    k_last = L.k;
                }
                // plain scores may be relative to the start point; the CV
                // score is g - u_hat(end) + sum r ds, absolute
                const float sx0 = a.shift ? L.px : 0.f, sy0 = a.shift ? L.py : 0.f;
                const float v[2] = {(plx - (o[0][0] - sx0)) + Ix, (ply - (o[1][0] - sy0)) + Iy};
                if (parked) {
                    const uint64_t rec = path_rec(L, a.n_paths);
                    if (a.scores) a.scores[rec] = make_float2(plx, ply);
                    if (c.cv_scores) c.cv_scores[rec] = make_float2(v[0], v[1]);
                    if (a.exit_step) a.exit_step[rec] = out ? L.k : -1;
                }
                acc_wave<2>(slots, accs, parked, my_tag, L.out, v, (uint32_t)L.k, lane);
                parked = false;
            }
            // ---- refill idle lanes (paths start only at evaluation points) ----
            uint64_t need = __ballot(!active && !parked);
            while (need != 0ull && !q_done) {
                if (q_next >= q_end) {
                    if (!grab_chunk<2>(a, total_chunks, next_chunk(a), q_slot, q_next, q_end, slots, accs, q_tag, grabs, lane)) {
                        q_done = true;
                        break;
                    }
                    continue;
                }
                const uint32_t avail = q_end - q_next;
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
                if (!active && !parked && rank < avail) {
                    const NodeDev nd = a.nodes[q_slot];
                    lane_start<KIND, TMODE>(L, nd, a.levels, q_next + rank);
                    my_tag = q_tag;
                    const float2 r0 = c.r0[nd.out];
                    rx = r0.x;
                    ry = r0.y;
                    Ix = 0.f;
                    Iy = 0.f;
                    k_last = 0;
                    active = true;
                }
                q_next += min((uint32_t)__popcll(need), avail);
                need = __ballot(!active && !parked);
            }
        }
        if (__ballot(active || parked) == 0ull && q_done) break;

        if (active) {
            out = false;
            if (L.k < L.K) {
                const PhiloxOut r = philox4x32_10((uint32_t)L.k >> 1, L.path, L.nid, L.ctr3, key0, key1);
                float ox = L.ox, oy = L.oy, cr = 0.f, sr = 0.f;
                if constexpr (kMovingBackward) {
                    const float rev = fmaf(-(float)L.k, L.drev, L.rev0);
                    cr = hw_cos_rev(rev);
                    sr = hw_sin_rev(rev);
                    ox = L.dens.orbit_r * cr;
                    oy = L.dens.orbit_r * sr;
                }
                out = em_step<KIND, UNIFORM>(L, r.r0, r.r1, ox, oy);
                my_steps += 1;
                if (!out && L.k < L.K) {
                    if constexpr (kMovingBackward) {
                        const float c2 = fmaf(cr, L.cos_d, sr * L.sin_d);
                        const float s2 = fmaf(sr, L.cos_d, -cr * L.sin_d);
                        ox = L.dens.orbit_r * c2;
                        oy = L.dens.orbit_r * s2;
                    }
                    out = em_step<KIND, UNIFORM>(L, r.r2, r.r3, ox, oy);
                    my_steps += 1;
                }
            }
            if (out || L.k >= L.K) {
                // the last interval is closed at the next evaluation point,
                // where u_hat and the integrand at the end state are known
                score_path(a, L, out, plx, ply);
                active = false;
                parked = true;
            }
        }
    }
    slots_collect<2>(slots, accs, lane);
    unsigned long long st = my_steps;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) st += __shfl_xor(st, off, 64);
    if (lane == 0 && st != 0ull && a.total_steps) atomicAdd(a.total_steps, st);
}

// Gradient of the bilinear interpolant of a nodal grid at (x, y) (the cell
// grid_bilinear uses); differences taken in FP64.
__device__ __forceinline__ void grid_gradient(const double *g, int n, float x, float y, float &gx, float &gy) {
    const float fx = x * (float)n, fy = y * (float)n;
    int i = (int)floorf(fx), j = (int)floorf(fy);
    i = min(max(i, 0), n - 1);
    j = min(max(j, 0), n - 1);
    const float ax = fx - (float)i, ay = fy - (float)j;
    const double *r0 = g + (int64_t)j * (n + 1);
    const double *r1 = r0 + (n + 1);
    const float d0x = (float)(r0[i + 1] - r0[i]), d1x = (float)(r1[i + 1] - r1[i]);
    const float d0y = (float)(r1[i] - r0[i]), d1y = (float)(r1[i + 1] - r0[i + 1]);
    gx = (float)n * fmaf(ay, d1x - d0x, d0x);
    gy = (float)n * fmaf(ax, d1y - d0y, d0y);
}

// Per cell (i, j) of the grid initial data, the FP32 terms grid_gradient
// forms from the four corner values: (d0x, d1x - d0x, d0y, d1y - d0y) for
// xi at tab[2 c] and for eta at tab[2 c + 1], c = j n + i.  The gradient
// taken from the table is bitwise the one taken from the grids, at one
// 16-byte load per component instead of four FP64 loads.
__global__ void grad_table_kernel(const double *gxi, const double *geta, int n, float4 *tab) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)n * n) return;
    const int i = (int)(c % n), j = (int)(c / n);
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        const double *r0 = (comp ? geta : gxi) + (int64_t)j * (n + 1);
        const double *r1 = r0 + (n + 1);
        const float d0x = (float)(r0[i + 1] - r0[i]), d1x = (float)(r1[i + 1] - r1[i]);
        const float d0y = (float)(r1[i] - r0[i]), d1y = (float)(r1[i + 1] - r0[i + 1]);
        tab[2 * c + comp] = make_float4(d0x, d1x - d0x, d0y, d1y - d0y);
    }
}

__device__ __forceinline__ void table_gradient(const float4 *tab, int n, int comp, float x, float y, float &gx,
                                               float &gy) {
    const float fx = x * (float)n, fy = y * (float)n;
    int i = (int)floorf(fx), j = (int)floorf(fy);
    i = min(max(i, 0), n - 1);
    j = min(max(j, 0), n - 1);
    const float ax = fx - (float)i, ay = fy - (float)j;
    const float4 t = tab[2 * ((int64_t)j * n + i) + comp];
    gx = (float)n * fmaf(ay, t.y, t.x);
    gy = (float)n * fmaf(ax, t.w, t.z);
}

// One Euler-Maruyama step with its Brownian part (wx, wy); with BRIDGE the
// Brownian-bridge exit test of the step follows (FK_SCORE_BRIDGE), on the
// same counters as in the plain kernel.  The step's Brownian part counts in
// full toward the block it ends: the test sees only this step.
template <int KIND, bool UNIFORM, bool BRIDGE>
__device__ __forceinline__ bool cv_step(Lane &L, uint32_t ra, uint32_t rb, float ox, float oy, float &wx, float &wy,
                                        uint32_t key0, uint32_t key1) {
    float x0h = 0.f, x0l = 0.f, y0h = 0.f, y0l = 0.f;
    if constexpr (BRIDGE) {
        x0h = L.xh;
        x0l = L.xl;
        y0h = L.yh;
        y0l = L.yl;
    }
    bool out = em_step_w<KIND, UNIFORM>(L, ra, rb, ox, oy, wx, wy);
    if constexpr (BRIDGE) {
        if (!out) out = bridge_exit<UNIFORM>(L, x0h, x0l, y0h, y0l, key0, key1);
    }
    return out;
}

// Martingale-form path kernel.  The score is g - sum_j G_j . dB_j: dB_j is the
// Brownian part of the path's steps in block j, G_j the gradient of u_hat at
// the block's first state.  Blocks start at the path's start (G_0 from the
// node table) and every stride steps after it, and the last one closes at
// the path's end, so a finished path is scored at once.  Paths start only at
// evaluation points, which keeps every path's blocks at fixed step offsets
// and the result independent of the schedule.
struct MgArgs {
    const uint16_t *bf;
    float tscale2;
    uint32_t stride_iters;
    float base;                  // identity base (0 or 1)
    const float4 *g0;            // [n_out] (dxi/dx, dxi/dy, deta/dx, deta/dy) at the start point
    int32_t grid_base;           // 1: u_hat = bilinear(grid initial data) + network: blocks every
                                 // iteration (2 steps) with the mesh's gradient there, plus the
                                 // network's taken at the evaluation points and held
    const float4 *gtab;          // grid base: per-cell gradient table, or NULL (read the grids)
    NodeAcc *acc_cv;             // [n_out] sums of the CV scores
    float2 *cv_scores;           // [n_out * n_paths], absolute, or nullptr
    int32_t split;               // host side: the network's gradient with BF16 hi + lo operands (1) or
                                 // BF16-rounded activations (0); selects the instantiation
};

// Four waves per SIMD (128 VGPRs) with the BF16 gradient, three (168) with
// the hi + lo split: the few values the compiler moves to scratch are
// touched at block boundaries, and the path loop between them gains the
// latency hiding of the extra waves (four waves were about 14% faster per
// path than two on the moving bump; at four the split form spills ~57
// registers around each evaluation and runs 5% slower at stride 20 than at
// three).  The Dynkin kernel, whose evaluation points are ten times as
// frequent, stays at two.
template <int KIND, int TMODE, bool UNIFORM, bool BRIDGE, bool SPLIT>
__global__ void __launch_bounds__(256, SPLIT ? 3 : 4) fk_mg_path_kernel(const PathArgs a, const MgArgs c) {
    constexpr bool kMovingBackward = moving_kind(KIND) && TMODE == TIME_BACKWARD;
    __shared__ NetLds N;
    load_net(N, c.bf);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    __shared__ AccSlot<2> slot_tab[4][kAccSlots];
    AccSlot<2> *slots = slot_tab[threadIdx.x >> 6];
    NodeAcc *const accs[1] = {c.acc_cv};
    slots_init<2>(slots, lane);
    uint32_t q_slot = 0, q_next = 0, q_end = 0, q_tag = 0, grabs = 0;
    const uint32_t total_chunks = launch_chunks(a);
    bool q_done = !grab_chunk<2>(a, total_chunks, first_chunk(), q_slot, q_next, q_end, slots, accs, q_tag, grabs, lane);
    const uint32_t key0 = a.key0, key1 = a.key1;
    Lane L;
    bool active = false;
    float gxx = 0.f, gxy = 0.f, gyx = 0.f, gyy = 0.f;   // gradient of (xi_hat, eta_hat) held over the block
    float dbx = 0.f, dby = 0.f;                         // Brownian part of the block so far
    float mx = 0.f, my = 0.f;                           // the martingale sum of the closed blocks
    float nxx = 0.f, nxy = 0.f, nyx = 0.f, nyy = 0.f;   // grid base: the network's part of the gradient
    const float tend = a.levels[0].tend;                // PDE time at path start
    uint32_t my_tag = 0;                                // accumulation tag of the path's chunk
    uint32_t my_steps = 0;

    bool closed = false;                                // the lane's last path closed its chunk's slot
    for (uint32_t until_eval = 0;; --until_eval) {     // iterations to the next block boundary
        if (__ballot(closed) != 0ull) {
            slots_collect<2>(slots, accs, lane);
            closed = false;
        }
        if (until_eval == 0) {
            until_eval = c.stride_iters;
            // ---- block boundary of running paths (every lane joins) ---------
            if (__ballot(active) != 0ull) {
                const float tau = active ? tend - (float)L.k * L.dt : 0.f;
                float o[2][2];
                net_grad_wave<SPLIT>(N, c.tscale2, tau, active ? L.xh : 0.5f, active ? L.yh : 0.5f, o);
                add_base_grad(c.base, o);
                if (c.grid_base) {
                    // grid base: the network's part, held until the next
                    // evaluation point; the blocks close every iteration
                    nxx = o[0][0];
                    nxy = o[0][1];
                    nyx = o[1][0];
                    nyy = o[1][1];
                } else if (active) {
                    mx = fmaf(gxx, dbx, fmaf(gxy, dby, mx));
                    my = fmaf(gyx, dbx, fmaf(gyy, dby, my));
                    dbx = dby = 0.f;
                    gxx = o[0][0];
                    gxy = o[0][1];
                    gyx = o[1][0];
                    gyy = o[1][1];
                }
            }
            // ---- refill idle lanes ------------------------------------------
            uint64_t need = __ballot(!active);
            while (need != 0ull && !q_done) {
                if (q_next >= q_end) {
                    if (!grab_chunk<2>(a, total_chunks, next_chunk(a), q_slot, q_next, q_end, slots, accs, q_tag, grabs, lane)) {
                        q_done = true;
                        break;
                    }
                    continue;
                }
                const uint32_t avail = q_end - q_next;
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
                if (!active && rank < avail) {
                    const NodeDev nd = a.nodes[q_slot];
                    lane_start<KIND, TMODE>(L, nd, a.levels, q_next + rank);
                    my_tag = q_tag;
                    const float4 g0 = c.g0[nd.out];
                    gxx = g0.x;
                    gxy = g0.y;
                    gyx = g0.z;
                    gyy = g0.w;
                    nxx = g0.x;
                    nxy = g0.y;
                    nyx = g0.z;
                    nyy = g0.w;
                    dbx = dby = mx = my = 0.f;
                    active = true;
                }
                q_next += min((uint32_t)__popcll(need), avail);
                need = __ballot(!active);
            }
        }
        if (__ballot(active) == 0ull && q_done) break;

        if (active) {
            bool out = false;
            if (L.k < L.K) {
                if (c.grid_base) {
                    // close the block (every 2 steps): G = the mesh's gradient
                    // here + the network's part
                    mx = fmaf(gxx, dbx, fmaf(gxy, dby, mx));
                    my = fmaf(gyx, dbx, fmaf(gyy, dby, my));
                    dbx = dby = 0.f;
                    if (c.gtab) {
                        table_gradient(c.gtab, a.grid_n, 0, L.xh, L.yh, gxx, gxy);
                        table_gradient(c.gtab, a.grid_n, 1, L.xh, L.yh, gyx, gyy);
                    } else {
                        grid_gradient(a.grid_xi, a.grid_n, L.xh, L.yh, gxx, gxy);
                        grid_gradient(a.grid_eta, a.grid_n, L.xh, L.yh, gyx, gyy);
                    }
                    gxx += nxx;
                    gxy += nxy;
                    gyx += nyx;
                    gyy += nyy;
                }
                const PhiloxOut r = philox4x32_10((uint32_t)L.k >> 1, L.path, L.nid, L.ctr3, key0, key1);
                float ox = L.ox, oy = L.oy, cr = 0.f, sr = 0.f;
                if constexpr (kMovingBackward) {
                    const float rev = fmaf(-(float)L.k, L.drev, L.rev0);
                    cr = hw_cos_rev(rev);
                    sr = hw_sin_rev(rev);
                    ox = L.dens.orbit_r * cr;
                    oy = L.dens.orbit_r * sr;
                }
                float wx, wy;
                out = cv_step<KIND, UNIFORM, BRIDGE>(L, r.r0, r.r1, ox, oy, wx, wy, key0, key1);
                dbx += wx;
                dby += wy;
                my_steps += 1;
                if (!out && L.k < L.K) {
                    if constexpr (kMovingBackward) {
                        const float c2 = fmaf(cr, L.cos_d, sr * L.sin_d);
                        const float s2 = fmaf(sr, L.cos_d, -cr * L.sin_d);
                        ox = L.dens.orbit_r * c2;
                        oy = L.dens.orbit_r * s2;
                    }
                    out = cv_step<KIND, UNIFORM, BRIDGE>(L, r.r2, r.r3, ox, oy, wx, wy, key0, key1);
                    dbx += wx;
                    dby += wy;
                    my_steps += 1;
                }
            }
            if (out || L.k >= L.K) {
                float plx, ply;
                score_path(a, L, out, plx, ply);
                mx = fmaf(gxx, dbx, fmaf(gxy, dby, mx));
                my = fmaf(gyx, dbx, fmaf(gyy, dby, my));
                const float sx0 = a.shift ? L.px : 0.f, sy0 = a.shift ? L.py : 0.f;
                const float v[2] = {(plx + sx0) - mx, (ply + sy0) - my};
                closed = acc_path<2>(slots, accs, my_tag, L.out, v, (uint32_t)L.k);
                const uint64_t rec = path_rec(L, a.n_paths);
                if (a.scores) a.scores[rec] = make_float2(plx, ply);
                if (c.cv_scores) c.cv_scores[rec] = make_float2(v[0], v[1]);
                if (a.exit_step) a.exit_step[rec] = out ? L.k : -1;
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

// Martingale form with the grid initial data as the control: every `stride`
// steps of a path (from its start) the lane takes G = the gradient of the
// bilinear interpolant of (grid_xi, grid_eta) at its position, and the score
// is g - sum_j G_j . dB_j.  No network: lanes need no common evaluation
// points, so they start new paths at once, and each path's blocks sit at
// fixed offsets from its start (schedule-independent results).
struct MggArgs {
    uint32_t stride_iters;       // the stride in iterations (2 steps each)
    NodeAcc *acc_cv;             // [n_out] sums of the CV scores
    float2 *cv_scores;           // [n_out * n_paths], absolute, or nullptr
    const float4 *gtab;          // per-cell gradient table (grad_table_kernel), or NULL: read the grids
    const float4 *gofs;          // [n_out] a gradient added to the mesh's at every block of the node's
                                 // paths (the network's at the node: the grid base with the network
                                 // taken only at the path's start), or NULL
};

template <int KIND, int TMODE, bool UNIFORM, bool BRIDGE>
__global__ void __launch_bounds__(256) fk_mgg_path_kernel(const PathArgs a, const MggArgs c) {
    constexpr bool kMovingBackward = moving_kind(KIND) && TMODE == TIME_BACKWARD;
    const uint32_t lane = threadIdx.x & 63u;
    __shared__ AccSlot<2> slot_tab[4][kAccSlots];
    AccSlot<2> *slots = slot_tab[threadIdx.x >> 6];
    NodeAcc *const accs[1] = {c.acc_cv};
    slots_init<2>(slots, lane);
    uint32_t q_slot = 0, q_next = 0, q_end = 0, q_tag = 0, grabs = 0;
    const uint32_t total_chunks = launch_chunks(a);
    bool q_done = !grab_chunk<2>(a, total_chunks, first_chunk(), q_slot, q_next, q_end, slots, accs, q_tag, grabs, lane);
    const uint32_t key0 = a.key0, key1 = a.key1;
    Lane L;
    bool active = false;
    float gxx = 0.f, gxy = 0.f, gyx = 0.f, gyy = 0.f;
    float dbx = 0.f, dby = 0.f, mx = 0.f, my = 0.f;
    uint32_t blk_left = 0;       // iterations (2 steps each) to the path's next block boundary
    uint32_t my_tag = 0;         // accumulation tag of the path's chunk
    uint32_t my_steps = 0;

    bool closed = false;         // the lane's last path closed its chunk's slot
    for (;;) {
        if (__ballot(closed) != 0ull) {
            slots_collect<2>(slots, accs, lane);
            closed = false;
        }
        uint64_t need = __ballot(!active);
        while (need != 0ull && !q_done) {
            if (q_next >= q_end) {
                if (!grab_chunk<2>(a, total_chunks, next_chunk(a), q_slot, q_next, q_end, slots, accs, q_tag, grabs, lane)) {
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
                my_tag = q_tag;
                dbx = dby = mx = my = 0.f;
                blk_left = 0;
                active = true;
            }
            q_next += min((uint32_t)__popcll(need), avail);
            need = __ballot(!active);
        }
        if (__ballot(active) == 0ull) break;

        if (active) {
            bool out = false;
            if (L.k < L.K) {
                if (blk_left == 0) {
                    // block boundary (L.k a multiple of the stride): close the
                    // block, take the gradient here
                    blk_left = c.stride_iters;
                    mx = fmaf(gxx, dbx, fmaf(gxy, dby, mx));
                    my = fmaf(gyx, dbx, fmaf(gyy, dby, my));
                    dbx = dby = 0.f;
                    if (c.gtab) {
                        table_gradient(c.gtab, a.grid_n, 0, L.xh, L.yh, gxx, gxy);
                        table_gradient(c.gtab, a.grid_n, 1, L.xh, L.yh, gyx, gyy);
                    } else {
                        grid_gradient(a.grid_xi, a.grid_n, L.xh, L.yh, gxx, gxy);
                        grid_gradient(a.grid_eta, a.grid_n, L.xh, L.yh, gyx, gyy);
                    }
                    if (c.gofs) {
                        const float4 o = c.gofs[L.out];   // L2-resident, 16 B per node
                        gxx += o.x;
                        gxy += o.y;
                        gyx += o.z;
                        gyy += o.w;
                    }
                }
                --blk_left;
                const PhiloxOut r = philox4x32_10((uint32_t)L.k >> 1, L.path, L.nid, L.ctr3, key0, key1);
                float ox = L.ox, oy = L.oy, cr = 0.f, sr = 0.f;
                if constexpr (kMovingBackward) {
                    const float rev = fmaf(-(float)L.k, L.drev, L.rev0);
                    cr = hw_cos_rev(rev);
                    sr = hw_sin_rev(rev);
                    ox = L.dens.orbit_r * cr;
                    oy = L.dens.orbit_r * sr;
                }
                float wx, wy;
                out = cv_step<KIND, UNIFORM, BRIDGE>(L, r.r0, r.r1, ox, oy, wx, wy, key0, key1);
                dbx += wx;
                dby += wy;
                my_steps += 1;
                if (!out && L.k < L.K) {
                    if constexpr (kMovingBackward) {
                        const float c2 = fmaf(cr, L.cos_d, sr * L.sin_d);
                        const float s2 = fmaf(sr, L.cos_d, -cr * L.sin_d);
                        ox = L.dens.orbit_r * c2;
                        oy = L.dens.orbit_r * s2;
                    }
                    out = cv_step<KIND, UNIFORM, BRIDGE>(L, r.r2, r.r3, ox, oy, wx, wy, key0, key1);
                    dbx += wx;
                    dby += wy;
                    my_steps += 1;
                }
            }
            if (out || L.k >= L.K) {
                float plx, ply;
                score_path(a, L, out, plx, ply);
                mx = fmaf(gxx, dbx, fmaf(gxy, dby, mx));
                my = fmaf(gyx, dbx, fmaf(gyy, dby, my));
                const float sx0 = a.shift ? L.px : 0.f, sy0 = a.shift ? L.py : 0.f;
                const float v[2] = {(plx + sx0) - mx, (ply + sy0) - my};
                closed = acc_path<2>(slots, accs, my_tag, L.out, v, (uint32_t)L.k);
                const uint64_t rec = path_rec(L, a.n_paths);
                if (a.scores) a.scores[rec] = make_float2(plx, ply);
                if (c.cv_scores) c.cv_scores[rec] = make_float2(v[0], v[1]);
                if (a.exit_step) a.exit_step[rec] = out ? L.k : -1;
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

// Per node: u_hat at the start (the shift of the CV estimate) and the
// integrand r0 there.
struct CvNodeArgs {
    const NodeDev *nodes;
    const LevelDev *levels;
    int64_t n_nodes;               // bound on the slots
    const uint32_t *active;        // the slots in use (set by the node-table kernels)
    OutDev *outs_cv;   // shift_x/shift_y <- u_hat(t_init + t, P), or NULL
    float2 *r0;        // integrand at P, or NULL
    float4 *g0;        // gradient of both outputs at P, or NULL
    int kind, time_mode;
    float base;        // identity base (0 or 1)
};

template <int KIND, int TMODE>
__global__ void __launch_bounds__(256) cv_node_kernel(const CvNodeArgs na, const uint16_t *bf, float tscale2) {
    __shared__ NetLds N;
    load_net(N, bf);
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = s < na.n_nodes && s < (int64_t)*na.active;
    Lane L;
    float tend = 0.f;
    if (ok) {
        const NodeDev nd = na.nodes[s];
        lane_start<KIND, TMODE>(L, nd, na.levels, 0);
        tend = na.levels[nd.level].tend;
    } else {
        L.xh = 0.5f;
        L.yh = 0.5f;
        L.xl = 0.f;
        L.yl = 0.f;
    }
    float o[2][5];
    net_eval_wave(N, tscale2, tend, L.xh, L.yh, o);
    // the value's base in FP64 from the node's hi + lo coordinates
    const double vx = (double)o[0][0] + na.base * ((double)L.xh + (double)L.xl);
    const double vy = (double)o[1][0] + na.base * ((double)L.yh + (double)L.yl);
    add_base(na.base, L.xh, L.yh, o);
    if (ok) {
        const NodeDev nd = na.nodes[s];
        float bx, by;
        drift_at<KIND, TMODE, true>(L, bx, by);
        if (na.outs_cv) {
            na.outs_cv[nd.out].shift_x = vx;
            na.outs_cv[nd.out].shift_y = vy;
        }
        if (na.r0)
            na.r0[nd.out] = make_float2(o[0][4] + fmaf(bx, o[0][1], by * o[0][2]) - o[0][3],
                                        o[1][4] + fmaf(bx, o[1][1], by * o[1][2]) - o[1][3]);
        if (na.g0) na.g0[nd.out] = make_float4(o[0][1], o[0][2], o[1][1], o[1][2]);
    }
}

// ---------------------------------------------------------------------------
// Training: per-tile forward + backward on MFMA, then Adam.
// ---------------------------------------------------------------------------
constexpr int kTS = 65;  // LDS row stride (floats) of the 64 x 64 activation tiles

struct TrainLds {
    NetLds net;
    float z[3][64];
    float y[2][64];
    float dout[2][64];
    float H1[64 * kTS], H2[64 * kTS], H3[64 * kTS];
    float D[64 * kTS], E[64 * kTS];
    float red[256];
};

// Per-call values of fk_cv_train, read by the kernels from device memory so
// that one captured graph of `steps` iterations serves every call with the
// same step count and minibatch size.
struct TrainDesc {
    const float *txy;      // [n][3]
    const float *target;   // [n][2]
    int64_t n;
    int64_t step0;         // Adam steps taken before the call
    uint32_t key0, key1;   // minibatch Philox key
    float lr;
    float loss_scale;      // 1 / (2 batch)
    float *loss_out;       // [steps] or nullptr
    float tscale2, base;
    int64_t pad;
};

struct TrainArgs {
    const TrainDesc *desc; // iteration `iter` of fk_cv_train (the fields below from desc), or nullptr
    uint32_t iter;
    const uint16_t *bf;
    const float *txy;      // [n][3]
    const float *target;   // [n][2]
    int64_t n;
    int64_t batch;         // samples in this step (loss normalisation)
    int full;              // 1: tile b takes samples 64 b .. 64 b + 63; 0: Philox minibatch
    uint32_t step, key0, key1;
    float tscale2;
    float base;            // identity base: the network fits target - (x, y)
    float *partial;        // [tiles][kNP + 1]
};

// C[M = 64][N = 64] = A[64 x K] B[K x 64] with K = 64, A and B given by
// element accessors, on MFMA (two 32-deep K blocks); each wavefront computes
// four 16 x 16 tiles and hands each result fragment to `sink(row, col, value)`.
template <typename FA, typename FB, typename FS>
__device__ __forceinline__ void wave_gemm64(FA A, FB B, FS sink) {
    const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15, w = threadIdx.x >> 6;
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
        const int tile = 4 * w + t, mt = tile >> 2, nt = tile & 3;
        fk_f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            fk_b8 a, b;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = ku(kb, g, j);
                a[j] = (__bf16)A(16 * mt + n, k);
                b[j] = (__bf16)B(k, 16 * nt + n);
            }
            acc = mfma32(a, b, acc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) sink(16 * mt + 4 * g + i, 16 * nt + n, acc[i]);
    }
}

__global__ void __launch_bounds__(256) cv_grad_kernel(TrainArgs ta) {
    if (ta.desc) {
        const TrainDesc &d = *ta.desc;
        ta.txy = d.txy;
        ta.target = d.target;
        ta.n = d.n;
        ta.step = (uint32_t)(d.step0 + ta.iter + 1);
        ta.key0 = d.key0;
        ta.key1 = d.key1;
        ta.tscale2 = d.tscale2;
        ta.base = d.base;
    }
    extern __shared__ char smem[];
    TrainLds &S = *reinterpret_cast<TrainLds *>(smem);
    const int tid = threadIdx.x;
    load_net(S.net, ta.bf);
    float *P = ta.partial + (int64_t)blockIdx.x * (kNP + 1);
    // ---- the tile's samples ----------------------------------------------------
    if (tid < 64) {
        int64_t idx;
        bool valid = true;
        if (ta.full) {
            idx = (int64_t)blockIdx.x * 64 + tid;
            valid = idx < ta.n;
            if (!valid) idx = 0;
        } else {
            const int64_t j = (int64_t)blockIdx.x * 64 + tid;
            const PhiloxOut r = philox4x32_10((uint32_t)j, ta.step, 0u, 2u, ta.key0, ta.key1);
            idx = (int64_t)(r.r0 % (uint32_t)ta.n);
            valid = j < ta.batch;
        }
        S.z[0][tid] = ta.txy[3 * idx] * ta.tscale2 - 1.f;
        S.z[1][tid] = 2.f * ta.txy[3 * idx + 1] - 1.f;
        S.z[2][tid] = 2.f * ta.txy[3 * idx + 2] - 1.f;
        S.y[0][tid] = fmaf(-ta.base, ta.txy[3 * idx + 1], ta.target[2 * idx]);
        S.y[1][tid] = fmaf(-ta.base, ta.txy[3 * idx + 2], ta.target[2 * idx + 1]);
        S.dout[0][tid] = valid ? 1.f : 0.f;  // validity mask until the residual is known
    }
    __syncthreads();
    // ---- forward ------------------------------------------------------------------
    for (int e = tid; e < 4096; e += 256) {
        const int u = e >> 6, s = e & 63;
        const float a = fmaf(S.net.w1[3 * u], S.z[0][s],
                             fmaf(S.net.w1[3 * u + 1], S.z[1][s], fmaf(S.net.w1[3 * u + 2], S.z[2][s], S.net.b1[u])));
        S.H1[u * kTS + s] = tanhf(a);
    }
    __syncthreads();
    wave_gemm64([&](int m, int k) { return bf2f(S.net.w2[m * kWS + wcol(k)]); }, [&](int k, int n) { return S.H1[k * kTS + n]; },
                [&](int m, int n, float v) { S.H2[m * kTS + n] = tanhf(v + S.net.b2[m]); });
    __syncthreads();
    wave_gemm64([&](int m, int k) { return bf2f(S.net.w3[m * kWS + wcol(k)]); }, [&](int k, int n) { return S.H2[k * kTS + n]; },
                [&](int m, int n, float v) { S.H3[m * kTS + n] = tanhf(v + S.net.b3[m]); });
    __syncthreads();
    // outputs, residuals and d loss / d out (mean over batch and both outputs)
    float lsum = 0.f;
    if (tid < 128) {
        const int o = tid >> 6, s = tid & 63;
        float acc = S.net.b4[o];
        for (int u = 0; u < 64; ++u) acc = fmaf(S.net.w4[64 * o + u], S.H3[u * kTS + s], acc);
        const float valid = S.dout[0][s];
        const float res = (acc - S.y[o][s]) * valid;
        lsum = res * res;
        S.red[tid] = 2.f * res / (2.f * (float)ta.batch);
    }
    __syncthreads();
    if (tid < 128) S.dout[tid >> 6][tid & 63] = S.red[tid];
    // loss of the tile
    {
        float v = lsum;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        __syncthreads();
        if ((tid & 63) == 0) S.red[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) P[kNP] = S.red[0] + S.red[1] + S.red[2] + S.red[3];
    }
    __syncthreads();
    // ---- backward -----------------------------------------------------------------
    // W4, b4
    if (tid < 128) {
        const int o = tid >> 6, u = tid & 63;
        float acc = 0.f;
        for (int s = 0; s < 64; ++s) acc = fmaf(S.dout[o][s], S.H3[u * kTS + s], acc);
        P[OW4 + 64 * o + u] = acc;
    } else if (tid < 130) {
        const int o = tid - 128;
        float acc = 0.f;
        for (int s = 0; s < 64; ++s) acc += S.dout[o][s];
        P[OB4 + o] = acc;
    }
    // dA3 = (W4^T dout) (1 - H3^2)
    for (int e = tid; e < 4096; e += 256) {
        const int u = e >> 6, s = e & 63;
        const float h = S.H3[u * kTS + s];
        S.D[u * kTS + s] = fmaf(S.net.w4[u], S.dout[0][s], S.net.w4[64 + u] * S.dout[1][s]) * (1.f - h * h);
    }
    __syncthreads();
    // dW3 = dA3 H2^T, db3
    wave_gemm64([&](int m, int k) { return S.D[m * kTS + k]; }, [&](int k, int n) { return S.H2[n * kTS + k]; },
                [&](int m, int n, float v) { P[OW3 + 64 * m + n] = v; });
    if (tid < 64) {
        float acc = 0.f;
        for (int s = 0; s < 64; ++s) acc += S.D[tid * kTS + s];
        P[OB3 + tid] = acc;
    }
    // dA2 = (W3^T dA3) (1 - H2^2)
    wave_gemm64([&](int m, int k) { return bf2f(S.net.w3[k * kWS + wcol(m)]); }, [&](int k, int n) { return S.D[k * kTS + n]; },
                [&](int m, int n, float v) {
                    const float h = S.H2[m * kTS + n];
                    S.E[m * kTS + n] = v * (1.f - h * h);
                });
    __syncthreads();
    // dW2 = dA2 H1^T, db2
    wave_gemm64([&](int m, int k) { return S.E[m * kTS + k]; }, [&](int k, int n) { return S.H1[n * kTS + k]; },
                [&](int m, int n, float v) { P[OW2 + 64 * m + n] = v; });
    if (tid < 64) {
        float acc = 0.f;
        for (int s = 0; s < 64; ++s) acc += S.E[tid * kTS + s];
        P[OB2 + tid] = acc;
    }
    // dA1 = (W2^T dA2) (1 - H1^2)
    wave_gemm64([&](int m, int k) { return bf2f(S.net.w2[k * kWS + wcol(m)]); }, [&](int k, int n) { return S.E[k * kTS + n]; },
                [&](int m, int n, float v) {
                    const float h = S.H1[m * kTS + n];
                    S.D[m * kTS + n] = v * (1.f - h * h);
                });
    __syncthreads();
    // dW1 = dA1 Z^T, db1
    if (tid < 192) {
        const int u = tid / 3, j = tid % 3;
        float acc = 0.f;
        for (int s = 0; s < 64; ++s) acc = fmaf(S.D[u * kTS + s], S.z[j][s], acc);
        P[OW1 + tid] = acc;
    } else {
        for (int u = tid - 192; u < 64; u += 64) {
            float acc = 0.f;
            for (int s = 0; s < 64; ++s) acc += S.D[u * kTS + s];
            P[OB1 + u] = acc;
        }
    }
}

// Sum of the tiles' gradients in a fixed order: grad[i] (and the loss).
__global__ void cv_sum_kernel(const float *partial, int tiles, float *grad, float *loss, float loss_scale) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > kNP) return;
    float acc = 0.f;
    for (int t = 0; t < tiles; ++t) acc += partial[(int64_t)t * (kNP + 1) + i];
    if (i < kNP) {
        if (grad) grad[i] = acc;
    } else if (loss) {
        *loss = acc * loss_scale;
    }
}

struct AdamArgs {
    const TrainDesc *desc;  // iteration `iter` of fk_cv_train (lr, c1, c2, loss_out from desc), or nullptr
    uint32_t iter;
    float *master, *m, *v;
    uint16_t *bf;
    const float *partial;   // per-tile gradients, or nullptr with `grad`
    const float *grad;
    int tiles;
    float lr, c1, c2;       // c1 = 1 - beta1^step, c2 = 1 - beta2^step
    float *loss_out;        // or nullptr
    float loss_scale;
};

// Bias corrections of Adam step `step` (>= 1), in FP64 then rounded.
__device__ __forceinline__ void adam_corrections(int64_t step, float &c1, float &c2) {
    c1 = (float)(1.0 - pow(0.9, (double)step));
    c2 = (float)(1.0 - pow(0.999, (double)step));
}

__global__ void cv_adam_kernel(AdamArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > kNP) return;
    if (A.desc) {
        const TrainDesc &d = *A.desc;
        adam_corrections(d.step0 + A.iter + 1, A.c1, A.c2);
        A.lr = d.lr;
        A.loss_out = d.loss_out ? d.loss_out + A.iter : nullptr;
        A.loss_scale = d.loss_scale;
    }
    float g = 0.f;
    if (A.partial) {
        for (int t = 0; t < A.tiles; ++t) g += A.partial[(int64_t)t * (kNP + 1) + i];
    } else if (i < kNP) {
        g = A.grad[i];
    }
    if (i == kNP) {
        if (A.loss_out) *A.loss_out = g * A.loss_scale;
        return;
    }
    const float m = 0.9f * A.m[i] + 0.1f * g;
    const float v = 0.999f * A.v[i] + 0.001f * g * g;
    A.m[i] = m;
    A.v[i] = v;
    const float p = A.master[i] - A.lr * (m / A.c1) / (sqrtf(v / A.c2) + 1e-8f);
    A.master[i] = p;
    A.bf[i] = f2bf(p);
}

__global__ void cv_to_bf16_kernel(const float *master, uint16_t *bf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kNP) bf[i] = f2bf(master[i]);
}

static void drop_graphs(fk_cv *cv) {
    for (TrainGraph &g : cv->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    cv->graphs.clear();
}

static int ensure_partial(fk_cv *cv, int tiles) {
    if (tiles <= cv->s.cap_tiles) return FK_OK;
    drop_graphs(cv);   // they hold the old buffer's address
    if (cv->s.partial) (void)hipFree(cv->s.partial);
    cv->s.partial = nullptr;
    cv->s.cap_tiles = 0;
    hipError_t e = hipMalloc(&cv->s.partial, sizeof(float) * (size_t)tiles * (kNP + 1));
    if (e != hipSuccess) return fail(FK_E_NOMEM, "hipMalloc of gradient partials: %s", hipGetErrorString(e));
    cv->s.cap_tiles = tiles;
    return FK_OK;
}

// The gradient kernel's LDS (~105 KB) is above the default dynamic limit:
// raised once per device, when a network is created there.
static std::mutex g_attr_mu;
static bool g_attr_done[64] = {};

static hipError_t grad_kernel_attribute(int dev) {
    std::lock_guard<std::mutex> lk(g_attr_mu);
    if (dev >= 0 && dev < 64 && g_attr_done[dev]) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute((const void *)cv_grad_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(TrainLds));
    if (e == hipSuccess && dev >= 0 && dev < 64) g_attr_done[dev] = true;
    return e;
}

static hipError_t launch_grad(const TrainArgs &ta, int tiles, hipStream_t s) {
    hipLaunchKernelGGL(cv_grad_kernel, dim3(tiles), dim3(256), sizeof(TrainLds), s, ta);
    return hipGetLastError();
}

__global__ void train_desc_kernel(const TrainDesc d, TrainDesc *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = d;
}

// Captures `steps` training iterations for minibatches of `batch` samples
// (on the handle's own stream; nothing runs during capture).
static int capture_training(fk_cv *cv, int steps, int64_t batch, TrainGraph &g) {
    const int tiles = (int)((batch + 63) / 64);
    hipError_t e = hipStreamBeginCapture(cv->capture_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    for (int j = 0; j < steps && le == hipSuccess; ++j) {
        TrainArgs ta{};
        ta.desc = cv->s.desc;
        ta.iter = (uint32_t)j;
        ta.bf = cv->s.bf;
        ta.batch = batch;
        ta.full = 0;
        ta.partial = cv->s.partial;
        le = launch_grad(ta, tiles, cv->capture_stream);
        if (le != hipSuccess) break;
        AdamArgs A{};
        A.desc = cv->s.desc;
        A.iter = (uint32_t)j;
        A.master = cv->s.master;
        A.m = cv->s.m;
        A.v = cv->s.v;
        A.bf = cv->s.bf;
        A.partial = cv->s.partial;
        A.tiles = tiles;
        hipLaunchKernelGGL(cv_adam_kernel, dim3((kNP + 256) / 256), dim3(256), 0, cv->capture_stream, A);
        le = hipGetLastError();
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cv->capture_stream, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le != hipSuccess ? le : e, "capture of the training loop");
    }
    hipGraphExec_t exec = nullptr;
    if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate of the training loop");
    }
    g.steps = steps;
    g.batch = batch;
    g.graph = graph;
    g.exec = exec;
    return FK_OK;
}

// Launches of the control-variate path kernel.
template <int K, int T, bool U>
struct CvLaunchF {
    static hipError_t run(const PathArgs &a, const CvArgs &c, int grid, hipStream_t s) {
        hipLaunchKernelGGL((fk_cv_path_kernel<K, T, U>), dim3(grid), dim3(256), 0, s, a, c);
        return hipGetLastError();
    }
};
template <int K, int T, bool U>
struct CvOccF {
    static int run() {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fk_cv_path_kernel<K, T, U>, 256, 0) != hipSuccess)
            return 0;
        return nb;
    }
};
// The martingale kernels with and without the bridge test (a.score_mode).
template <int K, int T, bool U>
struct MgLaunchF {
    template <bool B, bool S>
    static hipError_t go(const PathArgs &a, const MgArgs &c, int grid, hipStream_t s) {
        hipLaunchKernelGGL((fk_mg_path_kernel<K, T, U, B, S>), dim3(grid), dim3(256), 0, s, a, c);
        return hipGetLastError();
    }
    static hipError_t run(const PathArgs &a, const MgArgs &c, int grid, hipStream_t s) {
        const bool b = a.score_mode == FK_SCORE_BRIDGE;
        if (c.split) return b ? go<true, true>(a, c, grid, s) : go<false, true>(a, c, grid, s);
        return b ? go<true, false>(a, c, grid, s) : go<false, false>(a, c, grid, s);
    }
};
template <int K, int T, bool U>
struct MgOccF {
    template <bool B, bool S>
    static int occ() {
        int nb = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fk_mg_path_kernel<K, T, U, B, S>, 256, 0) ==
                       hipSuccess
                   ? nb
                   : 0;
    }
    static int run(bool bridge, bool split) {
        if (split) return bridge ? occ<true, true>() : occ<false, true>();
        return bridge ? occ<true, false>() : occ<false, false>();
    }
};
template <int K, int T, bool U>
struct MggLaunchF {
    static hipError_t run(const PathArgs &a, const MggArgs &c, int grid, hipStream_t s) {
        if (a.score_mode == FK_SCORE_BRIDGE)
            hipLaunchKernelGGL((fk_mgg_path_kernel<K, T, U, true>), dim3(grid), dim3(256), 0, s, a, c);
        else
            hipLaunchKernelGGL((fk_mgg_path_kernel<K, T, U, false>), dim3(grid), dim3(256), 0, s, a, c);
        return hipGetLastError();
    }
};
template <int K, int T, bool U>
struct MggOccF {
    static int run(bool bridge) {
        int nb = 0;
        const hipError_t e =
            bridge ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fk_mgg_path_kernel<K, T, U, true>, 256, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fk_mgg_path_kernel<K, T, U, false>, 256, 0);
        return e == hipSuccess ? nb : 0;
    }
};
template <int K, int T, bool U>
struct CvNodeF {
    static hipError_t run(const CvNodeArgs &na, const uint16_t *bf, float ts2, hipStream_t s) {
        const int blocks = (int)((na.n_nodes + 255) / 256);
        hipLaunchKernelGGL((cv_node_kernel<K, T>), dim3(blocks), dim3(256), 0, s, na, bf, ts2);
        return hipGetLastError();
    }
};

template <template <int, int, bool> class F, typename... Args>
auto cv_dispatch(int kind, int time_mode, bool uniform, Args &&...args) {
    const bool frozen = (time_mode == TIME_FROZEN);
#define FK_CV_CASE(K, T)                                                       \
    return uniform ? F<K, T, true>::run(std::forward<Args>(args)...)          \
                   : F<K, T, false>::run(std::forward<Args>(args)...)
    switch (kind) {
    case KIND_CONST: FK_CV_CASE(KIND_CONST, TIME_BACKWARD);
    case KIND_BUMP: FK_CV_CASE(KIND_BUMP, TIME_BACKWARD);
    case KIND_RIDGE: FK_CV_CASE(KIND_RIDGE, TIME_BACKWARD);
    case KIND_GRID: FK_CV_CASE(KIND_GRID, TIME_BACKWARD);
    case KIND_MOVING:
        if (frozen) FK_CV_CASE(KIND_MOVING, TIME_FROZEN);
        FK_CV_CASE(KIND_MOVING, TIME_BACKWARD);
    case KIND_RING:
        if (frozen) FK_CV_CASE(KIND_RING, TIME_FROZEN);
        FK_CV_CASE(KIND_RING, TIME_BACKWARD);
    default:
        if (frozen) FK_CV_CASE(KIND_TWO, TIME_FROZEN);
        FK_CV_CASE(KIND_TWO, TIME_BACKWARD);
    }
#undef FK_CV_CASE
}

// Workspace of one control-variate solve: counters, tables, the per-node
// start values of the control and the estimator sums (plain and CV).
struct CvWs {
    size_t counters, levels, nodes, outs, outs_cv, r0, g0, acc, acc_cv, total;
};

static CvWs cv_ws_layout(int64_t n_nodes) {
    CvWs L{};
    size_t off = 0;
    L.counters = off;
    off += 256;
    L.levels = off;
    off += align256(sizeof(LevelDev));
    L.nodes = off;
    off += align256(sizeof(NodeDev) * (size_t)n_nodes);
    L.outs = off;
    off += align256(sizeof(OutDev) * (size_t)n_nodes);
    L.outs_cv = off;
    off += align256(sizeof(OutDev) * (size_t)n_nodes);
    L.r0 = off;
    off += align256(sizeof(float2) * (size_t)n_nodes);
    L.g0 = off;
    off += align256(sizeof(float4) * (size_t)n_nodes);
    L.acc = off;
    off += align256(acc_bytes(n_nodes));
    L.acc_cv = off;
    off += align256(acc_bytes(n_nodes));
    L.total = off;
    return L;
}

// The per-cell gradient table of the grid initial data, built on the stream
// in the workspace past `used` bytes when it has room (NULL otherwise: the
// kernels then read the grids).
static const float4 *grid_table(const fk_data *d, void *workspace, size_t workspace_bytes, size_t used,
                                hipStream_t stream, hipError_t *err) {
    *err = hipSuccess;
    const size_t tab_off = align256(used), tab_bytes = (size_t)d->grid_n * d->grid_n * 2 * sizeof(float4);
    if (workspace_bytes < tab_off + tab_bytes) return nullptr;
    float4 *tab = (float4 *)((char *)workspace + tab_off);
    const int64_t cells = (int64_t)d->grid_n * d->grid_n;
    hipLaunchKernelGGL(grad_table_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, stream, d->grid_xi,
                       d->grid_eta, d->grid_n, tab);
    *err = hipGetLastError();
    return tab;
}

}  // namespace fk

using namespace fk;

extern "C" {

int fk_cv_create(const float *params, double t_scale, fk_cv_t *out) {
    g_last_error.clear();
    if (!out || !params) return fail(FK_E_INVAL, "NULL argument");
    *out = nullptr;
    if (!(t_scale > 0.0) || !std::isfinite(t_scale)) return fail(FK_E_INVAL, "t_scale must be > 0");
    for (int i = 0; i < kNP; ++i)
        if (!std::isfinite(params[i])) return fail(FK_E_INVAL, "parameter %d is not finite", i);
    fk_cv *cv = new fk_cv();
    hipError_t e = hipGetDevice(&cv->device);
    if (e != hipSuccess) {
        delete cv;
        return fail(FK_E_NODEVICE, "no HIP device: %s", hipGetErrorString(e));
    }
    cv->t_scale = (float)t_scale;
    if ((e = grad_kernel_attribute(cv->device)) != hipSuccess) {
        delete cv;
        return hip_fail(e, "LDS limit of the gradient kernel");
    }
    if ((e = hipStreamCreateWithFlags(&cv->capture_stream, hipStreamNonBlocking)) != hipSuccess) {
        delete cv;
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    float *buf = nullptr;
    const size_t state = align256(sizeof(float) * 3 * kNP + sizeof(uint16_t) * kNP);
    if ((e = hipMalloc(&buf, state + align256(sizeof(TrainDesc)))) != hipSuccess) {
        (void)hipStreamDestroy(cv->capture_stream);
        delete cv;
        return fail(FK_E_NOMEM, "hipMalloc of network state: %s", hipGetErrorString(e));
    }
    cv->s.master = buf;
    cv->s.m = buf + kNP;
    cv->s.v = buf + 2 * kNP;
    cv->s.bf = (uint16_t *)(buf + 3 * kNP);
    cv->s.desc = (TrainDesc *)((char *)buf + state);
    std::vector<float> zeros(2 * kNP, 0.f);
    if ((e = hipMemcpy(cv->s.master, params, sizeof(float) * kNP, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(cv->s.m, zeros.data(), sizeof(float) * 2 * kNP, hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(buf);
        (void)hipStreamDestroy(cv->capture_stream);
        delete cv;
        return hip_fail(e, "upload network");
    }
    hipLaunchKernelGGL(cv_to_bf16_kernel, dim3((kNP + 255) / 256), dim3(256), 0, 0, cv->s.master, cv->s.bf);
    if ((e = hipDeviceSynchronize()) != hipSuccess) {
        (void)hipFree(buf);
        (void)hipStreamDestroy(cv->capture_stream);
        delete cv;
        return hip_fail(e, "convert network");
    }
    *out = cv;
    return FK_OK;
}

int fk_cv_set_identity_base(fk_cv_t cv, int32_t on) {
    g_last_error.clear();
    if (!cv) return fail(FK_E_INVAL, "network is NULL");
    if (on != 0 && on != 1) return fail(FK_E_INVAL, "on must be 0 or 1");
    cv->base = (float)on;
    cv->grid_base = 0;
    return FK_OK;
}

int fk_cv_set_base(fk_cv_t cv, int32_t base) {
    g_last_error.clear();
    if (!cv) return fail(FK_E_INVAL, "network is NULL");
    if (base != FK_CV_BASE_NONE && base != FK_CV_BASE_IDENTITY && base != FK_CV_BASE_GRID)
        return fail(FK_E_INVAL, "unknown base %d", base);
    cv->base = base == FK_CV_BASE_IDENTITY ? 1.f : 0.f;
    cv->grid_base = base == FK_CV_BASE_GRID ? 1 : 0;
    return FK_OK;
}

void fk_cv_destroy(fk_cv_t cv) {
    if (!cv) return;
    (void)hipDeviceSynchronize();   // queued training or solves may still use the handle's memory
    drop_graphs(cv);
    if (cv->capture_stream) (void)hipStreamDestroy(cv->capture_stream);
    if (cv->s.master) hipFree(cv->s.master);
    if (cv->s.partial) hipFree(cv->s.partial);
    delete cv;
}

int fk_cv_get_params(fk_cv_t cv, float *params, uint16_t *bf16_params) {
    g_last_error.clear();
    if (!cv) return fail(FK_E_INVAL, "network is NULL");
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "synchronise");
    if (params && (e = hipMemcpy(params, cv->s.master, sizeof(float) * kNP, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "download master weights");
    if (bf16_params && (e = hipMemcpy(bf16_params, cv->s.bf, sizeof(uint16_t) * kNP, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "download BF16 weights");
    return FK_OK;
}

int fk_cv_set_params(fk_cv_t cv, const float *params) {
    g_last_error.clear();
    if (!cv || !params) return fail(FK_E_INVAL, "NULL argument");
    hipError_t e = hipMemcpy(cv->s.master, params, sizeof(float) * kNP, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload weights");
    hipLaunchKernelGGL(cv_to_bf16_kernel, dim3((kNP + 255) / 256), dim3(256), 0, 0, cv->s.master, cv->s.bf);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "convert network");
    return FK_OK;
}

int fk_cv_eval(fk_cv_t cv, const float *txy, int64_t n, float *out, hipStream_t stream) {
    g_last_error.clear();
    if (!cv) return fail(FK_E_INVAL, "network is NULL");
    if (n < 0) return fail(FK_E_INVAL, "n < 0");
    if (n == 0) return FK_OK;
    if (!txy || !out) return fail(FK_E_INVAL, "NULL array");
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(cv_eval_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, cv->s.bf, 2.f / cv->t_scale,
                       cv->base, txy, n, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FK_OK : hip_fail(e, "eval kernel launch");
}

int fk_cv_set_grad_precision(fk_cv_t cv, int32_t mode) {
    g_last_error.clear();
    if (!cv) return fail(FK_E_INVAL, "network is NULL");
    if (mode != FK_CV_GRAD_SPLIT && mode != FK_CV_GRAD_BF16) return fail(FK_E_INVAL, "unknown gradient precision %d", mode);
    cv->grad_bf16 = mode == FK_CV_GRAD_BF16 ? 1 : 0;
    return FK_OK;
}

int fk_cv_eval_grad(fk_cv_t cv, const float *txy, int64_t n, float *out, hipStream_t stream) {
    g_last_error.clear();
    if (!cv) return fail(FK_E_INVAL, "network is NULL");
    if (n < 0) return fail(FK_E_INVAL, "n < 0");
    if (n == 0) return FK_OK;
    if (!txy || !out) return fail(FK_E_INVAL, "NULL array");
    const int64_t blocks = (n + 255) / 256;
    if (cv->grad_bf16)
        hipLaunchKernelGGL(cv_eval_grad_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, stream, cv->s.bf,
                           2.f / cv->t_scale, cv->base, txy, n, out);
    else
        hipLaunchKernelGGL(cv_eval_grad_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, stream, cv->s.bf,
                           2.f / cv->t_scale, cv->base, txy, n, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FK_OK : hip_fail(e, "gradient eval kernel launch");
}

int fk_cv_grad(fk_cv_t cv, const float *txy, const float *target, int64_t n, float *grad, float *loss,
               hipStream_t stream) {
    g_last_error.clear();
    if (!cv) return fail(FK_E_INVAL, "network is NULL");
    if (n < 1 || n > (int64_t)1 << 31) return fail(FK_E_INVAL, "n out of range");
    if (!txy || !target || !grad) return fail(FK_E_INVAL, "NULL array");
    const int tiles = (int)((n + 63) / 64);
    int rc;
    if ((rc = ensure_partial(cv, tiles)) != FK_OK) return rc;
    TrainArgs ta{};
    ta.bf = cv->s.bf;
    ta.txy = txy;
    ta.target = target;
    ta.n = n;
    ta.batch = n;
    ta.full = 1;
    ta.tscale2 = 2.f / cv->t_scale;
    ta.base = cv->base;
    ta.partial = cv->s.partial;
    hipError_t e = launch_grad(ta, tiles, stream);
    if (e != hipSuccess) return hip_fail(e, "gradient kernel launch");
    // the tiles' loss entries are sums of squared residuals: report the mean
    hipLaunchKernelGGL(cv_sum_kernel, dim3((kNP + 256) / 256), dim3(256), 0, stream, cv->s.partial, tiles, grad,
                       loss, 1.f / (2.f * (float)n));
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "sum kernel launch");
    return FK_OK;
}

int fk_cv_adam_apply(fk_cv_t cv, const float *grad, float lr, hipStream_t stream) {
    g_last_error.clear();
    if (!cv || !grad) return fail(FK_E_INVAL, "NULL argument");
    const int64_t step = ++cv->steps_done;
    AdamArgs A{};
    A.master = cv->s.master;
    A.m = cv->s.m;
    A.v = cv->s.v;
    A.bf = cv->s.bf;
    A.grad = grad;
    A.lr = lr;
    A.c1 = (float)(1.0 - std::pow(0.9, (double)step));
    A.c2 = (float)(1.0 - std::pow(0.999, (double)step));
    hipLaunchKernelGGL(cv_adam_kernel, dim3((kNP + 256) / 256), dim3(256), 0, stream, A);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FK_OK : hip_fail(e, "adam kernel launch");
}

int fk_cv_train(fk_cv_t cv, const float *txy, const float *target, int64_t n, int32_t steps, int32_t batch, float lr,
                uint64_t seed, float *loss_out, hipStream_t stream) {
    g_last_error.clear();
    if (!cv) return fail(FK_E_INVAL, "network is NULL");
    if (n < 1 || n > 0xffffffffLL) return fail(FK_E_INVAL, "n out of range");
    if (steps < 0 || batch < 1 || batch > (1 << 24)) return fail(FK_E_INVAL, "steps >= 0 and batch in [1, 2^24]");
    if (!(lr > 0.f)) return fail(FK_E_INVAL, "lr must be > 0");
    if (!txy || !target) return fail(FK_E_INVAL, "NULL array");
    if (steps == 0) return FK_OK;
    const int tiles = (batch + 63) / 64;
    int rc;
    if ((rc = ensure_partial(cv, tiles)) != FK_OK) return rc;
    // this call's values for the kernels, in stream order
    TrainDesc d{};
    d.txy = txy;
    d.target = target;
    d.n = n;
    d.step0 = cv->steps_done;
    d.key0 = (uint32_t)seed;
    d.key1 = (uint32_t)(seed >> 32);
    d.lr = lr;
    d.loss_scale = 1.f / (2.f * (float)batch);
    d.loss_out = loss_out;
    d.tscale2 = 2.f / cv->t_scale;
    d.base = cv->base;
    hipLaunchKernelGGL(train_desc_kernel, dim3(1), dim3(64), 0, stream, d, cv->s.desc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "training descriptor kernel launch");
    TrainGraph *g = nullptr;
    for (TrainGraph &c : cv->graphs)
        if (c.steps == steps && c.batch == batch) g = &c;
    if (!g) {
        TrainGraph ng;
        if ((rc = capture_training(cv, steps, batch, ng)) != FK_OK) return rc;
        cv->graphs.push_back(ng);
        g = &cv->graphs.back();
    }
    if ((e = hipGraphLaunch(g->exec, stream)) != hipSuccess) return hip_fail(e, "hipGraphLaunch of the training loop");
    cv->steps_done += steps;
    return FK_OK;
}

size_t fk_interface_cv_workspace_bytes(int64_t n_nodes, int64_t n_paths) {
    if (n_nodes < 0 || n_paths < 2) return 0;
    return cv_ws_layout(n_nodes).total;
}

size_t fk_interface_cv_grid_workspace_bytes(int64_t n_nodes, int64_t n_paths, int32_t grid_n) {
    if (n_nodes < 0 || n_paths < 2 || grid_n < 1 || grid_n > 65535) return 0;
    return align256(cv_ws_layout(n_nodes).total) + (size_t)grid_n * grid_n * 2 * sizeof(float4);
}

int fk_interface_solve_cv(const fk_density *w, const fk_data *d, const double *pts, const uint8_t *mask,
                          int64_t n_nodes, double t, double dt, int64_t n_paths, uint64_t seed, uint32_t level_id,
                          fk_cv_t cv, int32_t stride,
                          int32_t form, double *xi, double *eta, double *se_xi, double *se_eta, double *plain_xi,
                          double *plain_eta, double *plain_se_xi, double *plain_se_eta, int32_t *exit_step,
                          float *cv_scores, uint64_t *total_steps, const fk_plan *plan, void *workspace,
                          size_t workspace_bytes, hipStream_t stream) {
    g_last_error.clear();
    int rc;
    const bool grid_ctl = (form == FK_CV_MARTINGALE_GRID);
    if (!cv && !grid_ctl) return fail(FK_E_INVAL, "network is NULL");
    if ((rc = validate_density(w)) != FK_OK) return rc;
    if ((rc = validate_data(d)) != FK_OK) return rc;
    if (d->score_mode == FK_SCORE_BRIDGE && form == FK_CV_DYNKIN)
        return fail(FK_E_UNSUPPORTED, "the Brownian-bridge exit test is for the plain and martingale forms only");
    if (d->score_mode == FK_SCORE_EXPONENTIAL)
        return fail(FK_E_UNSUPPORTED, "exponential time-stepping is for single plain solves only");
    if ((rc = validate_common(n_paths, dt)) != FK_OK) return rc;
    if ((rc = validate_horizon(t, d->t_init, dt, level_id)) != FK_OK) return rc;
    if ((rc = validate_device_points(pts, n_nodes)) != FK_OK) return rc;
    if (stride < 2 || stride % 2 != 0 || stride > (1 << 20)) return fail(FK_E_INVAL, "stride must be even and >= 2");
    if (form != FK_CV_DYNKIN && form != FK_CV_MARTINGALE && form != FK_CV_MARTINGALE_GRID)
        return fail(FK_E_INVAL, "unknown control-variate form");
    if (grid_ctl && d->init_kind != FK_DATA_GRID)
        return fail(FK_E_INVAL, "the grid control needs grid initial data");
    const bool grid_base = !grid_ctl && cv->grid_base;
    if (grid_base && form != FK_CV_MARTINGALE)
        return fail(FK_E_UNSUPPORTED, "the grid base needs the martingale form (its interpolant has no Laplacian)");
    if (grid_base && d->init_kind != FK_DATA_GRID) return fail(FK_E_INVAL, "the grid base needs grid initial data");
    if (n_nodes > 0 && (!xi || !eta || !se_xi || !se_eta)) return fail(FK_E_INVAL, "an output pointer is NULL");
    fk_plan pl;
    if ((rc = resolve_plan(plan, &pl)) != FK_OK) return rc;
    pl.block = 256;
    if ((rc = check_chunks(n_nodes, n_paths, pl)) != FK_OK) return rc;
    const CvWs lay = cv_ws_layout(n_nodes);
    if (!workspace || workspace_bytes < lay.total)
        return fail(FK_E_NOMEM, "workspace too small: need %zu bytes", lay.total);
    if (((uintptr_t)workspace & 255u) != 0) return fail(FK_E_INVAL, "workspace must be 256-byte aligned");
    if (n_nodes == 0) return FK_OK;
    int n_cu = 0;
    if ((rc = device_cus(&n_cu)) != FK_OK) return rc;

    char *ws = (char *)workspace;
    const LevelDev level = make_level(w, d->t_init, t, dt, level_id, 0u);
    const bool shift = (d->init_kind == FK_DATA_IDENTITY && d->bdry_kind == FK_DATA_IDENTITY);
    const bool uniform = (level.dt_last == level.dt && level.cbm_last == level.cbm);
    const bool mg = (form != FK_CV_DYNKIN);
    // network forms on short paths (a mesh step's sub-steps): 256 per grab
    // by default (the network-control mesh step went from 29.9 to 22.6 ms on
    // the 768-cell run against 128); the grid control keeps 128.  Larger
    // grabs, which the plain kernel prefers there, cost these kernels 5%.
    // Longer horizons: 32 to 128 by the path count, so that a solve with a
    // few hundred paths per node still spreads over every wavefront (the
    // Dynkin solve at 163 paths per node: 9.7 ms with 32, 11.7 with 128).
    if ((!plan || plan->chunk == 0) && !grid_ctl && level.K <= 64) pl.chunk = 256;
    else if ((!plan || plan->chunk == 0) && level.K > 64) pl.chunk = few_paths_chunk(n_nodes, n_paths, n_cu);
    const int64_t cpn = (n_paths + pl.chunk - 1) / pl.chunk;
    hipError_t e;
    uint32_t *counters = (uint32_t *)(ws + lay.counters);
    if ((e = launch_zero_u32(counters, 64, stream)) != hipSuccess) return hip_fail(e, "zero counters");
    // the plain and the CV sums lie back to back
    if ((e = launch_zero_u32((uint32_t *)(ws + lay.acc), (int)((lay.total - lay.acc) / 4), stream)) != hipSuccess)
        return hip_fail(e, "zero estimator sums");
    if (total_steps && (e = launch_zero_u32((uint32_t *)total_steps, 2, stream)) != hipSuccess)
        return hip_fail(e, "zero total_steps");
    // node tables from the device coordinates; the CV estimates have zero
    // shift (the Dynkin form's, u_hat at the node, is written by the node kernel)
    TableArgs tab{};
    tab.pts = pts;
    tab.mask = mask;
    tab.n = n_nodes;
    tab.level = level;
    tab.levels_out = (LevelDev *)(ws + lay.levels);
    tab.nodes_out = (NodeDev *)(ws + lay.nodes);
    tab.outs_out = (OutDev *)(ws + lay.outs);
    tab.outs_zero_out = (OutDev *)(ws + lay.outs_cv);
    tab.acc = (NodeAcc *)(ws + lay.acc);
    tab.acc2 = (NodeAcc *)(ws + lay.acc_cv);
    tab.counters = counters;
    tab.cpn = (uint32_t)cpn;
    tab.shift = shift ? 1 : 0;
    tab.sort = level.K > 64 ? 1 : 0;
    tab.horizon = (float)t;
    if ((e = launch_tables(tab, stream)) != hipSuccess) return hip_fail(e, "node table kernels");

    // per-node u_hat and integrand at the start
    CvNodeArgs na{};
    na.nodes = (const NodeDev *)(ws + lay.nodes);
    na.levels = (const LevelDev *)(ws + lay.levels);
    na.n_nodes = n_nodes;
    na.active = counters + kCtrActive;
    na.outs_cv = mg ? nullptr : (OutDev *)(ws + lay.outs_cv);
    na.r0 = mg ? nullptr : (float2 *)(ws + lay.r0);
    na.g0 = mg ? (float4 *)(ws + lay.g0) : nullptr;
    na.base = grid_ctl ? 0.f : cv->base;

    const float ts2 = grid_ctl ? 0.f : 2.f / cv->t_scale;
    if ((e = timing_record(0, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if (!grid_ctl &&
        (e = cv_dispatch<CvNodeF>(w->kind, w->time_mode, true, na, (const uint16_t *)cv->s.bf, ts2, stream)) !=
            hipSuccess)
        return hip_fail(e, "node kernel launch");
    // The grid base with a stride of at least the horizon takes the network
    // only at each path's start: that is the node kernel's gradient, and the
    // grid-control kernel adds it to the mesh's at every block (bitwise the
    // same arithmetic as the network kernel, without its evaluation points).
    const bool base_at_start = grid_base && (int64_t)stride >= (int64_t)level.K;

    PathArgs a{};
    SolveLaunch S{};
    S.args = a;
    fill_common_args(S, d, shift, seed);
    a = S.args;
    a.levels = (const LevelDev *)(ws + lay.levels);
    a.nodes = (const NodeDev *)(ws + lay.nodes);
    a.acc = (NodeAcc *)(ws + lay.acc);
    a.scores = nullptr;
    a.exit_step = exit_step;
    a.queue = counters;
    a.total_steps = total_steps ? (unsigned long long *)total_steps : (unsigned long long *)(counters + 2);
    a.n_paths = (uint32_t)n_paths;
    a.chunk = (uint32_t)pl.chunk;
    a.cpn = (uint32_t)cpn;
    a.total_chunks = (uint32_t)(n_nodes * cpn);
    float2 *cv_rec = (float2 *)cv_scores;
    NodeAcc *acc_cv = (NodeAcc *)(ws + lay.acc_cv);
    int bpc = pl.blocks_per_cu;
    if (!mg) {
        CvArgs c{};
        c.bf = cv->s.bf;
        c.tscale2 = ts2;
        c.stride_iters = (uint32_t)(stride / 2);
        c.base = cv->base;
        c.r0 = (const float2 *)(ws + lay.r0);
        c.cv_scores = cv_rec;
        c.acc_cv = acc_cv;
        const int occ = cv_dispatch<CvOccF>(w->kind, w->time_mode, uniform);
        if (bpc == 0 || (occ > 0 && bpc > occ)) bpc = occ > 0 ? occ : 1;
        if ((e = cv_dispatch<CvLaunchF>(w->kind, w->time_mode, uniform, a, c, cap_grid(n_cu * bpc, a.total_chunks, 256), stream)) != hipSuccess)
            return hip_fail(e, "control-variate path kernel launch");
    } else if (grid_ctl || base_at_start) {
        MggArgs c{};
        c.stride_iters = base_at_start ? 1u : (uint32_t)(stride / 2);
        c.gofs = base_at_start ? (const float4 *)(ws + lay.g0) : nullptr;
        c.cv_scores = cv_rec;
        c.acc_cv = acc_cv;
        c.gtab = grid_table(d, workspace, workspace_bytes, lay.total, stream, &e);
        if (e != hipSuccess) return hip_fail(e, "gradient table kernel launch");
        const int occ = cv_dispatch<MggOccF>(w->kind, w->time_mode, uniform, d->score_mode == FK_SCORE_BRIDGE);
        if (bpc == 0 || (occ > 0 && bpc > occ)) bpc = occ > 0 ? occ : 1;
        if ((e = cv_dispatch<MggLaunchF>(w->kind, w->time_mode, uniform, a, c, cap_grid(n_cu * bpc, a.total_chunks, 256), stream)) != hipSuccess)
            return hip_fail(e, "control-variate path kernel launch");
    } else {
        MgArgs c{};
        c.bf = cv->s.bf;
        c.tscale2 = ts2;
        c.stride_iters = (uint32_t)(stride / 2);
        c.base = grid_ctl ? 0.f : cv->base;
        c.g0 = (const float4 *)(ws + lay.g0);
        c.grid_base = grid_base ? 1 : 0;
        if (grid_base) c.gtab = grid_table(d, workspace, workspace_bytes, lay.total, stream, &e);
        if (e != hipSuccess) return hip_fail(e, "gradient table kernel launch");
        c.cv_scores = cv_rec;
        c.acc_cv = acc_cv;
        c.split = cv->grad_bf16 ? 0 : 1;
        const int occ = cv_dispatch<MgOccF>(w->kind, w->time_mode, uniform, d->score_mode == FK_SCORE_BRIDGE,
                                            c.split != 0);
        if (bpc == 0 || (occ > 0 && bpc > occ)) bpc = occ > 0 ? occ : 1;
        if ((e = cv_dispatch<MgLaunchF>(w->kind, w->time_mode, uniform, a, c, cap_grid(n_cu * bpc, a.total_chunks, 256), stream)) != hipSuccess)
            return hip_fail(e, "control-variate path kernel launch");
    }
    if ((e = timing_record(1, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");

    FinalArgs f{};
    f.acc = acc_cv;
    f.outs = (const OutDev *)(ws + lay.outs_cv);
    f.n_out = n_nodes;
    f.n_paths = n_paths;
    f.xi = xi;
    f.eta = eta;
    f.se_xi = se_xi;
    f.se_eta = se_eta;
    f.mask = mask;
    if ((e = launch_finalize(f, stream)) != hipSuccess) return hip_fail(e, "finalize kernel launch");
    if ((e = timing_record(2, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if (plain_xi && plain_eta && plain_se_xi && plain_se_eta) {
        // the plain estimate from the same paths: the plain path kernel on the
        // same tables and counters (bitwise the scores the CV kernel saw)
        SolveLaunch P{};
        P.args = a;
        P.args.acc = (NodeAcc *)(ws + lay.acc);
        P.args.scores = nullptr;
        P.args.exit_step = nullptr;
        P.kind = w->kind;
        P.time_mode = w->time_mode;
        P.uniform = uniform;
        P.first_by_index = level.K <= 64;
        if ((rc = resolve_plan(nullptr, &P.plan)) != FK_OK) return rc;
        if (P.first_by_index) P.plan.chunk = short_chunk(n_nodes, n_paths, n_cu, mask != nullptr);
        P.n_nodes = n_nodes;
        P.n_paths = n_paths;
        P.counters = counters;
        P.total_steps = nullptr;
        P.fin.outs = (const OutDev *)(ws + lay.outs);
        P.fin.xi = plain_xi;
        P.fin.eta = plain_eta;
        P.fin.se_xi = plain_se_xi;
        P.fin.se_eta = plain_se_eta;
        P.fin.mask = mask;
        TableArgs tp = tab;
        tp.outs_zero_out = nullptr;
        tp.acc2 = nullptr;
        tp.sort = P.first_by_index ? 0 : 1;
        P.tables = &tp;
        if ((rc = enqueue_solve(P, stream, false)) != FK_OK) return rc;
    }
    return FK_OK;
}

}  // extern "C"
