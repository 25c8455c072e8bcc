// Probes (declared in include/fdbb_probe.h).  The streaming probes are
// grid-stride loops of 16-byte accesses, 256 threads per workgroup; grid <= 0
// launches 8 workgroups per compute unit; their stores are the streaming
// stores of the fused kernel (nt + sc1, fdbb::put<kStoreNTSc1>).  The power
// probe evaluates the building blocks' shared power elementwise.
#include "../../include/fdbb.h"
#include "../../include/fdbb_probe.h"

#include <hip/hip_runtime.h>

#include "euler_tiles.hpp"

namespace {

using u64x2 = unsigned long long __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_copy(const u64x2 *__restrict__ src, u64x2 *__restrict__ dst,
                                              int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        fdbb::put<fdbb::kStoreNTSc1, u64x2>(dst + i, src[i]);
}

__global__ __launch_bounds__(256) void k_write(u64x2 *__restrict__ dst, int64_t n, unsigned long long pat)
{
    u64x2 v;
    v.x = pat;
    v.y = pat;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        fdbb::put<fdbb::kStoreNTSc1, u64x2>(dst + i, v);
}

__global__ __launch_bounds__(256) void k_read(const u64x2 *__restrict__ src, int64_t n,
                                              unsigned long long *__restrict__ sink)
{
    __shared__ unsigned long long part[256];
    unsigned long long acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const u64x2 v = src[i];
        acc ^= v.x ^ v.y;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] ^= part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = part[0];
}

// The fused 3D pass's store pattern with constant values: 256 points per
// wave, two waves per workgroup; F and R chunk by chunk (two chunks of 128
// points, 16 bytes per lane), then each direction's 256 blocks as 50
// lane-contiguous 1 KB stores.
__global__ __launch_bounds__(128) void k_fused_stores(double *__restrict__ F, double *__restrict__ R,
                                                      double *__restrict__ A, int64_t n)
{
    using d2 = double __attribute__((ext_vector_type(2)));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t wave0 = (int64_t)blockIdx.x * 512 + wave * 256;
    const d2 v = {1.0, 2.0};
    for (int c = 0; c < 2; ++c)
        for (int f = 0; f < 22; ++f) {
            double *base = f < 15 ? F + (int64_t)f * n : R + (int64_t)(f - 15) * n;
            fdbb::put<fdbb::kStoreNTSc1, d2>(reinterpret_cast<d2 *>(base + wave0 + c * 128 + lane * 2), v);
        }
    for (int d = 0; d < 3; ++d) {
        d2 *base = reinterpret_cast<d2 *>(A + ((int64_t)d * n + wave0) * 25);
        for (int k = 0; k < 50; ++k) fdbb::put<fdbb::kStoreNTSc1, d2>(base + k * 64 + lane, v);
    }
}

// x^y = exp(y log x) for each element, by the library's exp and log
// (FP32 false, the FP64-storage kernels) or by the base-2 form of the
// FP32-storage kernels (FP32 true): the same device functions the building
// blocks call.  One element per thread, grid-stride; regular stores.
template <bool FP32>
__global__ __launch_bounds__(256) void k_pow(const double *__restrict__ x, const double *__restrict__ y,
                                            double *__restrict__ out, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
        out[i] = fdbb::pos_pow_t<FP32>(x[i], y[i]);
}

int grid_for(int grid)
{
    if (grid > 0) return grid;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
    return 8 * cus;
}

bool aligned(const void *p) { return p && ((uintptr_t)p % 16) == 0; }

bool aligned8(const void *p) { return p && ((uintptr_t)p % 8) == 0; }

}  // namespace

extern "C" {

int fdbb_probe_copy(const void *src, void *dst, int64_t bytes, int grid, void *stream)
{
    if (!aligned(src) || !aligned(dst) || bytes < 0 || bytes % 16) return FDBB_EINVAL;
    if (bytes == 0) return FDBB_OK;
    const int g = grid_for(grid);
    if (g <= 0) return FDBB_EHIP;
    hipLaunchKernelGGL(k_copy, dim3(g), dim3(256), 0, (hipStream_t)stream, (const u64x2 *)src, (u64x2 *)dst,
                       bytes / 16);
    return hipGetLastError() == hipSuccess ? FDBB_OK : FDBB_EHIP;
}

int fdbb_probe_write(void *dst, int64_t bytes, uint64_t pattern, int grid, void *stream)
{
    if (!aligned(dst) || bytes < 0 || bytes % 16) return FDBB_EINVAL;
    if (bytes == 0) return FDBB_OK;
    const int g = grid_for(grid);
    if (g <= 0) return FDBB_EHIP;
    hipLaunchKernelGGL(k_write, dim3(g), dim3(256), 0, (hipStream_t)stream, (u64x2 *)dst, bytes / 16,
                       (unsigned long long)pattern);
    return hipGetLastError() == hipSuccess ? FDBB_OK : FDBB_EHIP;
}

int fdbb_probe_read(const void *src, int64_t bytes, uint64_t *sink, int grid, void *stream)
{
    if (!aligned(src) || !sink || bytes < 0 || bytes % 16) return FDBB_EINVAL;
    if (bytes == 0) return FDBB_OK;
    const int g = grid_for(grid);
    if (g <= 0) return FDBB_EHIP;
    hipLaunchKernelGGL(k_read, dim3(g), dim3(256), 0, (hipStream_t)stream, (const u64x2 *)src, bytes / 16,
                       (unsigned long long *)sink);
    return hipGetLastError() == hipSuccess ? FDBB_OK : FDBB_EHIP;
}

int fdbb_probe_fused_stores(double *F, double *R, double *A, int64_t n, void *stream)
{
    if (!aligned(F) || !aligned(R) || !aligned(A) || n <= 0 || n % 512) return FDBB_EINVAL;
    hipLaunchKernelGGL(k_fused_stores, dim3((unsigned)(n / 512)), dim3(128), 0, (hipStream_t)stream, F, R, A, n);
    return hipGetLastError() == hipSuccess ? FDBB_OK : FDBB_EHIP;
}

int fdbb_probe_pow(const double *x, const double *y, double *out, int64_t n, int fp32_form, void *stream)
{
    if (!aligned8(x) || !aligned8(y) || !aligned8(out) || n < 0) return FDBB_EINVAL;
    if (n == 0) return FDBB_OK;
    const int cap = grid_for(0);
    if (cap <= 0) return FDBB_EHIP;
    const int64_t want = (n + 255) / 256;
    const unsigned g = (unsigned)(want < cap ? want : cap);
    if (fp32_form)
        hipLaunchKernelGGL(k_pow<true>, dim3(g), dim3(256), 0, (hipStream_t)stream, x, y, out, n);
    else
        hipLaunchKernelGGL(k_pow<false>, dim3(g), dim3(256), 0, (hipStream_t)stream, x, y, out, n);
    return hipGetLastError() == hipSuccess ? FDBB_OK : FDBB_EHIP;
}

}  // extern "C"
