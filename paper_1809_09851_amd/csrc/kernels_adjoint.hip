// Adjoint kernel: Ubar = sum_d A_d(U)^T Fbar_d (or one direction) without
// forming A_d.
#include "fdbb_internal.hpp"

namespace fdbb {

template <int D, typename T, int P, int NT>
__global__ __launch_bounds__(1024) void k_adjoint(Args a, int64_t ntiles)
{
    const int64_t tile_pts = (int64_t)blockDim.x * P;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) tile_adjoint<D, T, P, NT>(a, t * tile_pts);
}

template <int D, typename T, int NT>
static const void *pick_p(int ppt)
{
    switch (ppt) {
    case 1: return (const void *)&k_adjoint<D, T, 1, NT>;
    case 2: return (const void *)&k_adjoint<D, T, 2, NT>;
    case 4: return (const void *)&k_adjoint<D, T, 4, NT>;
    default: return nullptr;
    }
}

template <int D, typename T>
static const void *pick_p(int ppt, bool nt)
{
    return nt ? pick_p<D, T, kStoreNT>(ppt) : pick_p<D, T, kStoreRegular>(ppt);
}

const void *kernel_adjoint(int dim, int dtype, int ppt, bool nt)
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
