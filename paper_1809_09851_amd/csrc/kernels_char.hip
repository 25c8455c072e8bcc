// Single-operation kernels for the characteristic transforms of one
// direction (W <-> U).
#include "fdbb_internal.hpp"

namespace fdbb {

template <int FAM, int D, typename T, int P, int NT>
__global__ __launch_bounds__(1024) void k_char(Args a, int64_t ntiles)
{
    const int64_t tile_pts = (int64_t)blockDim.x * P;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t tile0 = t * tile_pts;
        if constexpr (FAM == kFamCons2Char) tile_cons2char<D, T, P, NT>(a, tile0);
        else tile_char2cons<D, T, P, NT>(a, tile0);
    }
}

template <int FAM, int D, typename T, int NT>
static const void *pick_p(int ppt)
{
    switch (ppt) {
    case 1: return (const void *)&k_char<FAM, D, T, 1, NT>;
    case 2: return (const void *)&k_char<FAM, D, T, 2, NT>;
    case 4: return (const void *)&k_char<FAM, D, T, 4, NT>;
    default: return nullptr;
    }
}

template <int FAM, int D, typename T>
static const void *pick_p(int ppt, bool nt)
{
    return nt ? pick_p<FAM, D, T, kStoreNT>(ppt) : pick_p<FAM, D, T, kStoreRegular>(ppt);
}

template <int FAM>
static const void *pick(int dim, int dtype, int ppt, bool nt)
{
    if (dtype == 0) {
        if (dim == 1) return pick_p<FAM, 1, double>(ppt, nt);
        if (dim == 2) return pick_p<FAM, 2, double>(ppt, nt);
        if (dim == 3) return pick_p<FAM, 3, double>(ppt, nt);
    } else {
        if (dim == 1) return pick_p<FAM, 1, float>(ppt, nt);
        if (dim == 2) return pick_p<FAM, 2, float>(ppt, nt);
        if (dim == 3) return pick_p<FAM, 3, float>(ppt, nt);
    }
    return nullptr;
}

const void *kernel_char(int family, int dim, int dtype, int ppt, bool nt)
{
    if (family == kFamCons2Char) return pick<kFamCons2Char>(dim, dtype, ppt, nt);
    if (family == kFamChar2Cons) return pick<kFamChar2Cons>(dim, dtype, ppt, nt);
    return nullptr;
}

}  // namespace fdbb
