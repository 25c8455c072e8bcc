// Single-operation kernels for the characteristic transforms of one
// direction (W <-> U).
#include "fdbb_internal.hpp"

namespace fdbb {

template <int FAM, int D, typename T, int P>
__global__ __launch_bounds__(1024) void k_char(Args a, int64_t ntiles)
{
    const int64_t tile_pts = (int64_t)blockDim.x * P;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t tile0 = t * tile_pts;
        if constexpr (FAM == kFamCons2Char) tile_cons2char<D, T, P>(a, tile0);
        else tile_char2cons<D, T, P>(a, tile0);
    }
}

template <int FAM, int D, typename T>
static const void *pick_p(int ppt)
{
    switch (ppt) {
    case 1: return (const void *)&k_char<FAM, D, T, 1>;
    case 2: return (const void *)&k_char<FAM, D, T, 2>;
    case 4: return (const void *)&k_char<FAM, D, T, 4>;
    default: return nullptr;
    }
}

template <int FAM>
static const void *pick(int dim, int dtype, int ppt)
{
    if (dtype == 0) {
        if (dim == 1) return pick_p<FAM, 1, double>(ppt);
        if (dim == 2) return pick_p<FAM, 2, double>(ppt);
        if (dim == 3) return pick_p<FAM, 3, double>(ppt);
    } else {
        if (dim == 1) return pick_p<FAM, 1, float>(ppt);
        if (dim == 2) return pick_p<FAM, 2, float>(ppt);
        if (dim == 3) return pick_p<FAM, 3, float>(ppt);
    }
    return nullptr;
}

const void *kernel_char(int family, int dim, int dtype, int ppt)
{
    if (family == kFamCons2Char) return pick<kFamCons2Char>(dim, dtype, ppt);
    if (family == kFamChar2Cons) return pick<kFamChar2Cons>(dim, dtype, ppt);
    return nullptr;
}

}  // namespace fdbb
