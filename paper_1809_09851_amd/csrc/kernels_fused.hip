// Fused pass kernel: flux tensor, flux Jacobian blocks (staged through LDS)
// and Riemann invariants of the same state in one pass.  The flux-Jacobian
// entry point runs this kernel with the flux and invariant outputs NULL.
#include "fdbb_internal.hpp"

namespace fdbb {

template <int D, typename T, int P, int NT>
__global__ __launch_bounds__(kMaxBlockStaged) void k_fused(Args a, int64_t ntiles)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    T *lds = reinterpret_cast<T *>(smem);
    const int64_t tile_pts = (int64_t)blockDim.x * P;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x)
        tile_fused<D, T, P, NT>(a, t * tile_pts, lds);
}

template <int D, typename T, int NT>
static const void *pick_p(int ppt)
{
    switch (ppt) {
    case 1: return (const void *)&k_fused<D, T, 1, NT>;
    case 2: return (const void *)&k_fused<D, T, 2, NT>;
    case 4: return (const void *)&k_fused<D, T, 4, NT>;
    default: return nullptr;
    }
}

template <int D, typename T>
static const void *pick_p(int ppt, bool nt)
{
    return nt ? pick_p<D, T, kStoreNTSc1>(ppt) : pick_p<D, T, kStoreRegular>(ppt);
}

const void *kernel_fused(int dim, int dtype, int ppt, bool nt)
{
    if (dtype == 0) {
        if (dim == 1) return pick_p<1, double>(ppt, nt);
        if (dim == 2) return pick_p<2, double>(ppt, nt);
        if (dim == 3) return pick_p<3, double>(ppt, nt);
    } else {
        if (dim == 1) return pick_p<1, float>(ppt, nt);
        if (dim == 2) return pick_p<2, float>(ppt, nt);
        if (dim == 3) return pick_p<3, float>(ppt, nt);
    }
    return nullptr;
}

}  // namespace fdbb
