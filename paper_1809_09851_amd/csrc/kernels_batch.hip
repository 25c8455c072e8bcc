// Batch kernel: a grid of workgroups walks the tiles of many independent
// tasks of uneven size.  Tiles are dealt round-robin (tile t to workgroup
// t mod gridDim.x); the owning task of a tile is found in the tile prefix
// sums by a galloping search from the workgroup's previous task (tiles
// only move forward).  Every tile costs about the same, so the static
// deal balances without a shared counter.  The grid is part of the launch
// configuration: a few workgroups per compute unit make the launch
// persistent, a grid near the tile count leaves the order of tiles to the
// hardware dispatcher (the tuned FP32 shape).
#include "fdbb_internal.hpp"

#include <atomic>

namespace fdbb {

template <int D, typename T, int P, int NT>
__device__ __forceinline__ void run_tile(int op, const Args &a, int64_t tile0, unsigned char *smem)
{
    switch (op) {
    case 0: tile_cons2prim<D, T, P, NT>(a, tile0); break;
    case 1: tile_prim2cons<D, T, P, NT>(a, tile0); break;
    case 2: tile_eos<D, T, P, NT>(a, tile0); break;
    case 3:
    case 16: tile_flux<D, T, P, NT>(a, tile0); break;
    case 4:
    case 8: tile_fused<D, T, P, NT>(a, tile0, reinterpret_cast<T *>(smem)); break;
    case 5: tile_riemann<D, T, P, NT>(a, tile0); break;
    case 6: tile_cons2char<D, T, P, NT>(a, tile0); break;
    case 7: tile_char2cons<D, T, P, NT>(a, tile0); break;
    case 9: tile_adjoint<D, T, P, NT>(a, tile0); break;
    case 10: tile_vmag2<D, T, P, NT>(a, tile0); break;
    case 13: tile_roe<D, T, P, NT>(a, tile0); break;
    default: break;
    }
}

template <int P, int NT>
__global__ __launch_bounds__(kMaxBlockStaged) void k_batch(const TaskDev *__restrict__ tasks,
                                                const int64_t *__restrict__ prefix,
                                                const int64_t *__restrict__ header)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int ntasks = (int)header[0];
    const int64_t ntiles = header[1];
    const int64_t tile_pts = (int64_t)blockDim.x * P;
    int lo = 0;  // owning task of the previous tile: tiles only move forward
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        // last task whose first tile is <= t: gallop forward from the
        // previous owner, then bisect the bracket (one load when the tile
        // stays in the same task)
        int step = 1;
        while (lo + step < ntasks && prefix[lo + step] <= t) {
            lo += step;
            step <<= 1;
        }
        int hi = (lo + step < ntasks ? lo + step : ntasks) - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const TaskDev &td = tasks[lo];
        const int64_t tile0 = (t - prefix[lo]) * tile_pts;
        if (td.dtype == 0) {
            if (td.dim == 1) run_tile<1, double, P, NT>(td.op, td.a, tile0, smem);
            else if (td.dim == 2) run_tile<2, double, P, NT>(td.op, td.a, tile0, smem);
            else run_tile<3, double, P, NT>(td.op, td.a, tile0, smem);
        } else {
            if (td.dim == 1) run_tile<1, float, P, NT>(td.op, td.a, tile0, smem);
            else if (td.dim == 2) run_tile<2, float, P, NT>(td.op, td.a, tile0, smem);
            else run_tile<3, float, P, NT>(td.op, td.a, tile0, smem);
        }
    }
}

// Task table of the allocation-free batch entry point: one fixed array per
// device, holding the table layout of a plan of capacity kNoAllocMaxTasks.
// Host code never passes `scratch` itself (in host code the name is a
// host-side stand-in, not a device address): batch_scratch looks up the
// device address once per device and every caller uses that.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

int batch_scratch(void **ptr)
{
    static std::atomic<uintptr_t> addr[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= 64) return (int)hipErrorInvalidDevice;
    uintptr_t a = addr[dev].load(std::memory_order_acquire);
    if (a == 0) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (p == nullptr) return (int)hipErrorInvalidSymbol;
        a = (uintptr_t)p;
        addr[dev].store(a, std::memory_order_release);
    }
    *ptr = (void *)a;
    return 0;
}

template <int NT>
static const void *pick_batch(int ppt)
{
    switch (ppt) {
    case 1: return (const void *)&k_batch<1, NT>;
    case 2: return (const void *)&k_batch<2, NT>;
    case 4: return (const void *)&k_batch<4, NT>;
    case 8: return (const void *)&k_batch<8, NT>;
    default: return nullptr;
    }
}

// store_mode: 0 regular, 1 nt, 2 nt + sc1 (a batch plan's `nontemporal`).
const void *kernel_batch(int ppt, int store_mode)
{
    switch (store_mode) {
    case 0: return pick_batch<kStoreRegular>(ppt);
    case 1: return pick_batch<kStoreNT>(ppt);
    case 2: return pick_batch<kStoreNTSc1>(ppt);
    default: return nullptr;
    }
}

}  // namespace fdbb
