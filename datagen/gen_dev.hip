// gen_dev.hip -- device side of the seeded column generator (see gen_core.h).
//
// gg_fill_device writes rows [row0, row0 + n) of one column into device memory
// with exactly the arithmetic of gg_fill_host, so tables of hundreds of GB can
// be made resident without a host round trip.  For a Zipf column, c->cdf must
// be a device pointer to the table built by gg_zipf_cdf.
#include <hip/hip_runtime.h>

#define GG_FN __device__ static inline
#include "gen_core.h"

__global__ void __launch_bounds__(256) gg_fill_kernel(gg_col c, uint64_t row0, uint64_t n, void* out) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int64_t v = gg_value(&c, row0 + i);
        if (c.dtype == GG_I32) ((int32_t*)out)[i] = (int32_t)v;
        else if (c.dtype == GG_I64) ((int64_t*)out)[i] = v;
        else ((uint32_t*)out)[i] = (uint32_t)v;
    }
}

extern "C" int gg_fill_device(const gg_col* c, uint64_t row0, uint64_t n, void* out, void* stream) {
    if (!c || (!out && n)) return -1;
    if (c->kind == GG_ZIPF && (!c->cdf || c->ncdf == 0)) return -1;
    if (c->kind == GG_UNIFORM && c->span == 0) return -1;
    if (n == 0) return 0;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(gg_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, *c, row0, n, out);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
