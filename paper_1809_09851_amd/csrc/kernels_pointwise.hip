// Single-operation kernels for the pointwise building blocks: cons2prim,
// prim2cons, EOS (perfect gas, and the general entry with temperature),
// inviscid and viscous flux tensors, Riemann invariants, |v|^2 and the
// Roe-averaged state.  Each workgroup loops
// over tiles of blockDim.x * P points (grid-stride when the grid is capped).
#include "fdbb_internal.hpp"

namespace fdbb {

template <int FAM, int D, typename T, int P, int NT>
__global__ __launch_bounds__(1024) void k_pointwise(Args a, int64_t ntiles)
{
    const int64_t tile_pts = (int64_t)blockDim.x * P;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t tile0 = t * tile_pts;
        if constexpr (FAM == kFamCons2Prim) tile_cons2prim<D, T, P, NT>(a, tile0);
        else if constexpr (FAM == kFamPrim2Cons) tile_prim2cons<D, T, P, NT>(a, tile0);
        else if constexpr (FAM == kFamEos) tile_eos<D, T, P, NT>(a, tile0);
        else if constexpr (FAM == kFamFlux) tile_flux<D, T, P, NT>(a, tile0);
        else if constexpr (FAM == kFamRiemann) tile_riemann<D, T, P, NT>(a, tile0);
        else if constexpr (FAM == kFamVmag2) tile_vmag2<D, T, P, NT>(a, tile0);
        else if constexpr (FAM == kFamRoe) tile_roe<D, T, P, NT>(a, tile0);
        else if constexpr (FAM == kFamEosPvt) tile_eos_pvt<D, T, P, NT>(a, tile0);
        else if constexpr (FAM == kFamViscous) tile_viscous<D, T, P, NT>(a, tile0);
    }
}

template <int FAM, int D, typename T, int NT>
static const void *pick_p(int ppt)
{
    switch (ppt) {
    case 1: return (const void *)&k_pointwise<FAM, D, T, 1, NT>;
    case 2: return (const void *)&k_pointwise<FAM, D, T, 2, NT>;
    case 4: return (const void *)&k_pointwise<FAM, D, T, 4, NT>;
    default: return nullptr;
    }
}

// Streaming store flavour per family and storage type: nt + sc1 where it
// measured faster than nt alone, timed alternately in one process on the
// same buffers (3D, a 2 GB working set: cons2prim and prim2cons FP64 by
// 3.8 and 2.3 %, flux 2.0 / 4.2 %, Riemann invariants 2.0 / 7.6 %, |v|^2
// FP32 3.8 %), nt elsewhere (the viscous flux FP64 ran 7 % slower with sc1,
// cons2prim and prim2cons FP32 2-3 %).
template <int FAM, typename T>
constexpr int streaming_mode()
{
    constexpr bool f64 = sizeof(T) == 8;
    if constexpr (FAM == kFamFlux || FAM == kFamRiemann) return kStoreNTSc1;
    else if constexpr ((FAM == kFamCons2Prim || FAM == kFamPrim2Cons) && f64) return kStoreNTSc1;
    else if constexpr (FAM == kFamVmag2 && !f64) return kStoreNTSc1;
    else return kStoreNT;
}

template <int FAM, int D, typename T>
static const void *pick_p(int ppt, bool nt)
{
    return nt ? pick_p<FAM, D, T, streaming_mode<FAM, T>()>(ppt) : pick_p<FAM, D, T, kStoreRegular>(ppt);
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

const void *kernel_pointwise(int family, int dim, int dtype, int ppt, bool nt)
{
    switch (family) {
    case kFamCons2Prim: return pick<kFamCons2Prim>(dim, dtype, ppt, nt);
    case kFamPrim2Cons: return pick<kFamPrim2Cons>(dim, dtype, ppt, nt);
    case kFamEos: return pick<kFamEos>(dim, dtype, ppt, nt);
    case kFamFlux: return pick<kFamFlux>(dim, dtype, ppt, nt);
    case kFamRiemann: return pick<kFamRiemann>(dim, dtype, ppt, nt);
    case kFamVmag2: return pick<kFamVmag2>(dim, dtype, ppt, nt);
    case kFamRoe: return pick<kFamRoe>(dim, dtype, ppt, nt);
    case kFamEosPvt: return pick<kFamEosPvt>(dim, dtype, ppt, nt);
    case kFamViscous: return pick<kFamViscous>(dim, dtype, ppt, nt);
    default: return nullptr;
    }
}

}  // namespace fdbb
