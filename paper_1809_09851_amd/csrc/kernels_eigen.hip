// Characteristic decomposition kernels: eigenvector blocks of every
// direction (staged through LDS like the Jacobian) and products with L or R
// of one direction.
#include "fdbb_internal.hpp"

namespace fdbb {

template <int D, typename T, int P, int NT>
__global__ __launch_bounds__(kMaxBlockStaged) void k_eigen(Args a, int64_t ntiles)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    T *lds = reinterpret_cast<T *>(smem);
    const int64_t tile_pts = (int64_t)blockDim.x * P;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) tile_eigen<D, T, P, NT>(a, t * tile_pts, lds);
}

template <int D, typename T, int P, int NT>
__global__ __launch_bounds__(1024) void k_char_apply(Args a, int64_t ntiles)
{
    const int64_t tile_pts = (int64_t)blockDim.x * P;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) tile_char_apply<D, T, P, NT>(a, t * tile_pts);
}

template <int FAM, int D, typename T, int NT>
static const void *pick_p(int ppt)
{
    if constexpr (FAM == kFamEigen) {
        switch (ppt) {
        case 1: return (const void *)&k_eigen<D, T, 1, NT>;
        case 2: return (const void *)&k_eigen<D, T, 2, NT>;
        case 4: return (const void *)&k_eigen<D, T, 4, NT>;
        default: return nullptr;
        }
    } else {
        switch (ppt) {
        case 1: return (const void *)&k_char_apply<D, T, 1, NT>;
        case 2: return (const void *)&k_char_apply<D, T, 2, NT>;
        case 4: return (const void *)&k_char_apply<D, T, 4, NT>;
        default: return nullptr;
        }
    }
}

template <int FAM, int D, typename T>
static const void *pick_p(int ppt, bool nt)
{
    // eigenvector blocks stream with nt + sc1, the products with nt
    constexpr int streaming = FAM == kFamEigen ? kStoreNTSc1 : kStoreNT;
    return nt ? pick_p<FAM, D, T, streaming>(ppt) : pick_p<FAM, D, T, kStoreRegular>(ppt);
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

const void *kernel_eigen(int family, int dim, int dtype, int ppt, bool nt)
{
    if (family == kFamEigen) return pick<kFamEigen>(dim, dtype, ppt, nt);
    if (family == kFamCharApply) return pick<kFamCharApply>(dim, dtype, ppt, nt);
    return nullptr;
}

}  // namespace fdbb
