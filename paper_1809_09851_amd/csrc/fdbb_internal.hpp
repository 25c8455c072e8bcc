// Host-side glue between the C ABI (fdbb_api.hip) and the kernel
// translation units.  Each kernel unit returns the address of the template
// instance for (dim, dtype, points per thread).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "euler_tiles.hpp"

namespace fdbb {

// Device image of one batch task: the operation's arguments plus what the
// persistent kernel needs to pick the tile function.
struct TaskDev {
    Args a;
    int32_t op;
    int32_t dim;
    int32_t dtype;
    int32_t pad;
};

// Largest workgroup of the kernels that stage Jacobian blocks (the fused
// kernel and the batch kernel).  Bounding them at 256 threads lets the
// compiler give each thread up to 256 registers, so the staged blocks never
// spill; their occupancy is set by LDS anyway.
constexpr int kMaxBlockStaged = 256;

// Kernel families (a family covers one or more public ops).
enum Family : int {
    kFamCons2Prim = 0,
    kFamPrim2Cons,
    kFamEos,
    kFamFlux,
    kFamRiemann,
    kFamCons2Char,
    kFamChar2Cons,
    kFamFused,  // fused pass and flux Jacobian (F and R NULL)
    kFamAdjoint,
    kFamVmag2,
    kFamEigen,      // eigenvector blocks (staged like the Jacobian)
    kFamCharApply,  // products with L or R of one direction
    kFamRoe,        // Roe-averaged state of two states
    kFamEosPvt,     // p, c and T of the general EOS entry
    kFamViscous,    // viscous flux tensor
    kNumFamilies
};

// Single-operation kernels: void k(Args a, int64_t ntiles).  nt selects
// non-temporal output stores.
const void *kernel_pointwise(int family, int dim, int dtype, int ppt, bool nt);
const void *kernel_char(int family, int dim, int dtype, int ppt, bool nt);
const void *kernel_fused(int dim, int dtype, int ppt, bool nt);
const void *kernel_adjoint(int dim, int dtype, int ppt, bool nt);
const void *kernel_eigen(int family, int dim, int dtype, int ppt, bool nt);

// Persistent batch kernel: void k(const TaskDev*, const int64_t* prefix,
// const int64_t* header).  header = {ntasks, ntiles}; prefix has ntasks + 1
// entries, prefix[b] = first tile of task b.  ppt 1, 2, 4 or 8; store_mode
// 0 regular, 1 nt, 2 nt + sc1.
const void *kernel_batch(int ppt, int store_mode);

// The allocation-free batch entry point's fixed task table: room for
// kNoAllocMaxTasks tasks in the layout of a plan's table (header, tile
// prefix sums, task images).
constexpr int kNoAllocMaxTasks = 1024;
constexpr size_t kNoAllocBytes =
    (((2 + (size_t)kNoAllocMaxTasks + 1) * sizeof(int64_t) + 63) & ~(size_t)63) + (size_t)kNoAllocMaxTasks * sizeof(TaskDev);

// Device address of that table on the current device (looked up with
// hipGetSymbolAddress on a device's first call, then cached); 0 or a
// hipError_t.
int batch_scratch(void **ptr);

}  // namespace fdbb
