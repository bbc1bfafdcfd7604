// fk_rng.hip -- the path kernels' counter-based generator and normal
// transform, exposed on their own so that they can be checked bitwise.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fk.h"
#include "fk_device.hpp"
#include "fk_internal.hpp"

namespace fk {

__global__ void philox_words_kernel(const uint4 *ctr, int64_t n, uint32_t k0, uint32_t k1, uint4 *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 c = ctr[i];
    const PhiloxOut r = philox4x32_10(c.x, c.y, c.z, c.w, k0, k1);
    out[i] = make_uint4(r.r0, r.r1, r.r2, r.r3);
}

__global__ void normals_kernel(const uint32_t *ra, const uint32_t *rb, int64_t n, float cbm, float2 *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x, y;
    brownian_increment(ra[i], rb[i], cbm, x, y);
    out[i] = make_float2(x, y);
}
}  // namespace fk

using namespace fk;

extern "C" {

int fk_philox_words(const uint32_t *ctr, int64_t n, uint64_t seed, uint32_t *out, hipStream_t stream) {
    if (n < 0) return fail(FK_E_INVAL, "n < 0");
    if (n == 0) return FK_OK;
    if (!ctr || !out) return fail(FK_E_INVAL, "NULL array");
    if (n > ((int64_t)1 << 40)) return fail(FK_E_INVAL, "n too large");
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(philox_words_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, (const uint4 *)ctr, n,
                       (uint32_t)seed, (uint32_t)(seed >> 32), (uint4 *)out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FK_OK : hip_fail(e, "philox kernel launch");
}

int fk_normals(const uint32_t *ra, const uint32_t *rb, int64_t n, double D, float *out, hipStream_t stream) {
    if (n < 0 || !(D > 0.0)) return fail(FK_E_INVAL, "n < 0 or D <= 0");
    if (n == 0) return FK_OK;
    if (!ra || !rb || !out) return fail(FK_E_INVAL, "NULL array");
    if (n > ((int64_t)1 << 40)) return fail(FK_E_INVAL, "n too large");
    const int64_t blocks = (n + 255) / 256;
    const float cbm = (float)(-4.0 * 0.69314718055994530942 * D);
    hipLaunchKernelGGL(normals_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, ra, rb, n, cbm, (float2 *)out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FK_OK : hip_fail(e, "normals kernel launch");
}

}  // extern "C"
