// fk_device.hpp -- per-lane device math of the path kernels: counter-based
// normals, the Winslow drift of the analytic densities, and the data
// functions.  Everything here runs in registers in FP32 (integer for the
// generator); nothing touches memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fk {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Ten rounds of two
// 32x32->64-bit products (one v_mad_u64_u32 each on CDNA) and XORs; the key
// schedule is wave-uniform and lives in scalar registers.
// ---------------------------------------------------------------------------
struct PhiloxOut {
    uint32_t r0, r1, r2, r3;
};

// a ^ b ^ k in one VALU instruction (gfx950 three-input bit operation with
// truth table 0x96 = XOR of the three inputs); k is wave-uniform (a key word).
__device__ __forceinline__ uint32_t xor3_uniform(uint32_t a, uint32_t b, uint32_t k) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

__device__ __forceinline__ PhiloxOut philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                   uint32_t k0, uint32_t k1) {
    // The round keys are re-derived per call (two scalar adds a round, off
    // the VALU) instead of being hoisted out of the path loop, where twenty
    // live key words would push loop values out of the scalar file.
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3_uniform((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3_uniform((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return PhiloxOut{c0, c1, c2, c3};
}

// A path's counter words 1 and 2 (path, node) stay fixed over its calls, so
// round 1's second product (M1 times the node word) and round 2's first
// product (M0 times round 1's first output, which combines that product with
// the path word and key word 0) are the same in every call: formed once per
// path, they save two of the twenty products of each call.
struct PhiloxPath {
    uint32_t b;        // round 1's second output: low half of M1 * node
    uint32_t h0, l0;   // round 2's product M0 * (round 1's first output)
};

__device__ __forceinline__ PhiloxPath philox_path(uint32_t c1, uint32_t c2, uint32_t k0) {
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t a = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint64_t q0 = (uint64_t)0xD2511F53u * a;
    return PhiloxPath{(uint32_t)p1, (uint32_t)(q0 >> 32), (uint32_t)q0};
}

// philox4x32_10(c0, c1, c2, c3, k0, k1) with P = philox_path(c1, c2, k0):
// bitwise the same four words.
__device__ __forceinline__ PhiloxOut philox4x32_10_path(uint32_t c0, uint32_t c3, const PhiloxPath &P, uint32_t k0,
                                                        uint32_t k1) {
    asm volatile("" : "+s"(k0), "+s"(k1));
    // round 1: words 0 and 1 of the result are fixed (their product is in P)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint32_t x2 = xor3_uniform((uint32_t)(p0 >> 32), c3, k1);
    const uint32_t x3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    // round 2: M0 times the fixed word 0 is P.h0, P.l0
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
    c0 = xor3_uniform((uint32_t)(p1 >> 32), P.b, k0);
    uint32_t c1 = (uint32_t)p1;
    uint32_t c2 = xor3_uniform(P.h0, x3, k1);
    c3 = P.l0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
#pragma unroll
    for (int r = 2; r < 10; ++r) {
        const uint64_t q0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t q1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3_uniform((uint32_t)(q1 >> 32), c1, k0);
        const uint32_t n2 = xor3_uniform((uint32_t)(q0 >> 32), c3, k1);
        c1 = (uint32_t)q1;
        c3 = (uint32_t)q0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return PhiloxOut{c0, c1, c2, c3};
}

// Hardware transcendentals.  v_sin/v_cos take their argument in revolutions
// (sin(2 pi x)), v_log is log2 and v_exp is exp2.
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_sin_rev(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float hw_cos_rev(float x) { return __builtin_amdgcn_cosf(x); }

// Box-Muller increments on the low 23 bits of each word: with
// ma = ra mod 2^23 and mb = rb mod 2^23, u1 = 1 - ma 2^-23 in (0,1] and
// u2 = mb 2^-23 in [0,1), returns sqrt(2 D) (z0, z1) where
// z0 = sqrt(-2 ln u1) cos(2 pi u2), z1 = sqrt(-2 ln u1) sin(2 pi u2).
// cbm = -4 ln2 D folds sqrt(2 D) and the change of logarithm base.  The
// bits m under the exponent of 1.0 make the float 1 + m 2^-23 in one
// instruction: u1 is 2 minus that (exact), and the angle is that float
// itself, as sin and cos in revolutions have period 1.
__device__ __forceinline__ void brownian_increment(uint32_t ra, uint32_t rb, float cbm,
                                                   float &dwx, float &dwy) {
    const float u1 = 2.f - __uint_as_float((ra & 0x7fffffu) | 0x3f800000u);
    const float a2 = __uint_as_float((rb & 0x7fffffu) | 0x3f800000u);   // 1 + u2
    const float rad = hw_sqrt(cbm * hw_log2(u1));
    dwx = rad * hw_cos_rev(a2);
    dwy = rad * hw_sin_rev(a2);
}

// ---------------------------------------------------------------------------
// Densities and the Winslow drift b = -grad w / w (eq. (6)).  For a Gaussian
// bump w = 1 + A e, e = exp(-|X - c|^2 / s2):  b = (2 A / s2) e / w * (X - c).
// ---------------------------------------------------------------------------
enum : int { KIND_CONST = 0, KIND_BUMP = 1, KIND_MOVING = 2, KIND_TWO = 3, KIND_RING = 4, KIND_RIDGE = 5, KIND_GRID = 6 };

// Kinds whose centre moves on the orbit (R cos(omega tau), R sin(omega tau)).
constexpr bool moving_kind(int k) { return k == KIND_MOVING || k == KIND_TWO || k == KIND_RING; }
enum : int { TIME_BACKWARD = 0, TIME_FROZEN = 1 };

struct DensityRegs {
    float amp, nscale, a2s;
    float cx, cy;        // centre (static) / orbit centre
    float orbit_r, omega_rev;
    const float2 *gb;    // grid density: nodal drift table, row-major [j][i]
    int gn;              // grid density: cells per side
    float fn;            // (float) gn
};

// Bump centre offset (R cos(omega tau), R sin(omega tau)).
__device__ __forceinline__ void orbit(const DensityRegs &d, float tau, float &ox, float &oy) {
    const float rev = tau * d.omega_rev;
    ox = d.orbit_r * hw_cos_rev(rev);
    oy = d.orbit_r * hw_sin_rev(rev);
}

// Drift at (x, y); (ox, oy) is the centre offset (zero for static kinds).
template <int KIND>
__device__ __forceinline__ void drift(const DensityRegs &d, float ox, float oy, float x, float y,
                                      float &bx, float &by) {
    if constexpr (KIND == KIND_CONST) {
        bx = 0.f;
        by = 0.f;
    } else if constexpr (KIND == KIND_BUMP || KIND == KIND_MOVING) {
        const float dx = x - (d.cx + ox);
        const float dy = y - (d.cy + oy);
        const float r2 = fmaf(dx, dx, dy * dy);
        const float e = hw_exp2(r2 * d.nscale);
        const float f = e * d.a2s * hw_rcp(fmaf(d.amp, e, 1.f));
        bx = f * dx;
        by = f * dy;
    } else if constexpr (KIND == KIND_TWO) {
        const float dy = y - (d.cy + oy);
        const float d1x = x - (d.cx + ox);
        const float d2x = x - (d.cx - ox);
        const float dy2 = dy * dy;
        const float e1 = hw_exp2(fmaf(d1x, d1x, dy2) * d.nscale);
        const float e2 = hw_exp2(fmaf(d2x, d2x, dy2) * d.nscale);
        const float f = d.a2s * hw_rcp(fmaf(d.amp, e1 + e2, 1.f));
        bx = f * fmaf(e1, d1x, e2 * d2x);
        by = f * (e1 + e2) * dy;
    } else if constexpr (KIND == KIND_RING) {
        // w = 1/rho, rho = 1 + A e, e = exp(beta |q|), q = |X - c|^2 - 1/100:
        // b = -grad w / w = grad rho / rho = 2 A beta sgn(q) e (X - c) / rho
        // (nscale = beta log2(e), a2s = 2 A beta).
        const float dx = x - (d.cx + ox);
        const float dy = y - (d.cy + oy);
        const float q = fmaf(dx, dx, fmaf(dy, dy, -0.01f));
        const float e = hw_exp2(fabsf(q) * d.nscale);
        const float sg = q > 0.f ? 1.f : (q < 0.f ? -1.f : 0.f);
        const float f = sg * e * d.a2s * hw_rcp(fmaf(d.amp, e, 1.f));
        bx = f * dx;
        by = f * dy;
    } else if constexpr (KIND == KIND_GRID) {
        // w known at grid nodes only (Sect. 4): the nodal drifts of the
        // finite-difference table, bilinear in the cell.  The cell index is
        // clamped, so a point outside the square (a Dynkin-form end point)
        // takes the edge cell's bilinear function continued.
        const float fx = x * d.fn, fy = y * d.fn;
        const int i = min(max((int)floorf(fx), 0), d.gn - 1);
        const int j = min(max((int)floorf(fy), 0), d.gn - 1);
        const float ax = fx - (float)i, ay = fy - (float)j;
        const float2 *r0 = d.gb + (j * (d.gn + 1) + i);
        const float2 b00 = r0[0], b01 = r0[1], b10 = r0[d.gn + 1], b11 = r0[d.gn + 2];
        const float lx0 = fmaf(ax, b01.x - b00.x, b00.x), lx1 = fmaf(ax, b11.x - b10.x, b10.x);
        const float ly0 = fmaf(ax, b01.y - b00.y, b00.y), ly1 = fmaf(ax, b11.y - b10.y, b10.y);
        bx = fmaf(ay, lx1 - lx0, lx0);
        by = fmaf(ay, ly1 - ly0, ly0);
    } else {  // KIND_RIDGE: depends on x only
        const float dx = x - d.cx;
        const float e = hw_exp2(dx * dx * d.nscale);
        bx = e * d.a2s * hw_rcp(fmaf(d.amp, e, 1.f)) * dx;
        by = 0.f;
    }
}

// sin(pi x) sin(pi y) via the revolution-argument sine.
__device__ __forceinline__ float sin_mode(float x, float y) {
    return hw_sin_rev(0.5f * x) * hw_sin_rev(0.5f * y);
}

}  // namespace fk
