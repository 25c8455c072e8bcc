// C ABI of the library (declared in include/fdbb.h): host-side validation,
// launch configuration, kernel launches on the caller's stream, and the
// persistent batch plans with their HIP graphs.
#include "../../include/fdbb.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fdbb_internal.hpp"

using namespace fdbb;

namespace {

thread_local std::string g_last_error;

int fail(int status, const std::string &msg)
{
    g_last_error = msg;
    return status;
}

int fail_hip(hipError_t e, const char *what)
{
    return fail(FDBB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t elem_size(int dtype) { return dtype == FDBB_F64 ? 8 : 4; }

// ------------------------------------------------------------ device facts

struct DeviceInfo {
    int id = 0;
    int cus = 0;
    size_t lds_max = 0;
};

// Per-device facts, read once and then served without a lock: the first
// callers on a device may query concurrently, and all store the same values.
constexpr int kMaxDevices = 64;
std::atomic<int> g_dev_cus[kMaxDevices];
std::atomic<int64_t> g_dev_lds[kMaxDevices];

int device_info(DeviceInfo *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(FDBB_EHIP, "device index out of range");
    int cus = g_dev_cus[dev].load(std::memory_order_acquire);
    if (cus == 0) {
        int lds = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return fail_hip(e, "hipDeviceGetAttribute");
        e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) return fail_hip(e, "hipDeviceGetAttribute");
        g_dev_lds[dev].store(lds, std::memory_order_relaxed);
        g_dev_cus[dev].store(cus, std::memory_order_release);
    }
    out->id = dev;
    out->cus = cus;
    out->lds_max = (size_t)g_dev_lds[dev].load(std::memory_order_relaxed);
    return FDBB_OK;
}

// ------------------------------------------------------------ launch table

struct Config {
    int block;
    int ppt;
    int grid_cap;
    int nt;
};

std::atomic<uint64_t> g_cfg[FDBB_NUM_OPS][3][2];
std::once_flag g_cfg_once;

uint64_t pack(const Config &c)
{
    return (uint64_t)(uint16_t)c.block | ((uint64_t)(uint8_t)c.ppt << 16) | ((uint64_t)(c.nt ? 1 : 0) << 24) |
           ((uint64_t)(uint32_t)c.grid_cap << 32);
}

Config unpack(uint64_t v)
{
    Config c;
    c.block = (int)(v & 0xffff);
    c.ppt = (int)((v >> 16) & 0xff);
    c.nt = (int)((v >> 24) & 1);
    c.grid_cap = (int)(uint32_t)(v >> 32);
    return c;
}

void init_configs()
{
    for (int op = 0; op < FDBB_NUM_OPS; ++op)
        for (int d = 0; d < 3; ++d)
            for (int t = 0; t < 2; ++t) {
                Config c;
                // one point per thread where a point holds many registers
                // (staged Jacobian blocks; the viscous flux's K + D*D + D
                // input and K*D output fields)
                const bool wide = (op == FDBB_OP_FLUX_JACOBIAN || op == FDBB_OP_FUSED || op == FDBB_OP_VISCOUS_FLUX);
                c.block = 256;
                c.ppt = wide ? 1 : (t == FDBB_F64 ? 2 : 4);
                c.grid_cap = 0;
                c.nt = 1;
                g_cfg[op][d][t].store(pack(c));
            }
}

Config get_config(int op, int dim, int dtype)
{
    std::call_once(g_cfg_once, init_configs);
    return unpack(g_cfg[op][dim - 1][dtype].load(std::memory_order_relaxed));
}

// The small-launch entries: calls of n <= g_small_max points take
// g_small_cfg (no entry while g_small_max is 0).  The setter stores the
// configuration before the bound and the remover clears the bound first, so
// a launch that sees a non-zero bound also sees a configuration that was
// valid for this (op, dim, dtype).
std::atomic<uint64_t> g_small_cfg[FDBB_NUM_OPS][3][2];
std::atomic<int64_t> g_small_max[FDBB_NUM_OPS][3][2];

Config get_config(int op, int dim, int dtype, int64_t n)
{
    const int64_t max_n = g_small_max[op][dim - 1][dtype].load(std::memory_order_acquire);
    if (max_n > 0 && n <= max_n) return unpack(g_small_cfg[op][dim - 1][dtype].load(std::memory_order_relaxed));
    return get_config(op, dim, dtype);
}

// Launch configuration of the persistent batch kernel, per storage type:
// what plans created with block == 0 (and the request server's plans) use.
// grid_per_cu 0 sizes the grid to 2048 / block workgroups per compute unit.
struct BatchConfig {
    int block;
    int ppt;
    int grid_per_cu;
    int nt;  // 0 regular, 1 nt, 2 nt + sc1
};

// [0] FP64, [1] FP32, [2] the request server's batched launches
std::atomic<uint64_t> g_batch_cfg[3] = {{0}, {0}, {0}};

uint64_t pack_batch(const BatchConfig &c)
{
    return (uint64_t)(uint16_t)c.block | ((uint64_t)(uint8_t)c.ppt << 16) | ((uint64_t)(uint8_t)c.nt << 24) |
           ((uint64_t)(uint32_t)c.grid_per_cu << 32);
}

// dtype FDBB_F64 or FDBB_F32, or 2 for the server's entry
BatchConfig get_batch_config(int dtype)
{
    const uint64_t v = g_batch_cfg[dtype == FDBB_F32 ? 1 : (dtype == 2 ? 2 : 0)].load(std::memory_order_relaxed);
    if (v == 0) return BatchConfig{256, 1, 0, 1};
    BatchConfig c;
    c.block = (int)(v & 0xffff);
    c.ppt = (int)((v >> 16) & 0xff);
    c.nt = (int)((v >> 24) & 0xff);
    c.grid_per_cu = (int)(uint32_t)(v >> 32);
    return c;
}

bool batch_config_ok(int block, int ppt, int nt)
{
    return block >= 64 && block <= kMaxBlockStaged && block % 64 == 0 &&
           (ppt == 1 || ppt == 2 || ppt == 4 || ppt == 8) && nt >= 0 && nt <= 2;
}

bool config_ok(int block, int ppt, int grid_cap, int nt)
{
    return block >= 64 && block <= 1024 && block % 64 == 0 && (ppt == 1 || ppt == 2 || ppt == 4) &&
           grid_cap >= 0 && (nt == 0 || nt == 1);
}

// ------------------------------------------------------------ validation

// Byte range of a field set: `fields` rows of stride ld, the last one n long,
// each element `unit` elements of T wide (K*K for Jacobian blocks).
struct Range {
    uintptr_t lo, hi;
    bool input;
    const void *base;
    int64_t ld;
    int task;
};

Range field_range(const void *base, int64_t ld, int64_t fields, int64_t n, int64_t unit, size_t es,
                  bool input, int task = 0)
{
    Range r;
    r.lo = (uintptr_t)base;
    r.hi = r.lo + (uintptr_t)(((fields - 1) * ld + n) * unit) * es;
    r.input = input;
    r.base = base;
    r.ld = ld;
    r.task = task;
    return r;
}

bool overlap(const Range &a, const Range &b) { return a.lo < b.hi && b.lo < a.hi; }

int check_common(int dim, double gamma, int dtype, int64_t n)
{
    if (dim < 1 || dim > 3) return fail(FDBB_EINVAL, "dim must be 1, 2 or 3");
    if (!std::isfinite(gamma) || !(gamma > 1.0)) return fail(FDBB_EINVAL, "gamma must be finite and > 1");
    if (dtype != FDBB_F64 && dtype != FDBB_F32) return fail(FDBB_EINVAL, "unknown dtype");
    if (n < 0) return fail(FDBB_EINVAL, "n must be >= 0");
    if (n >= FDBB_MAX_POINTS) return fail(FDBB_EINVAL, "n must be below 2^31 points per call");
    return FDBB_OK;
}

Gas make_gas(double gamma)
{
    Gas g;
    g.gamma = gamma;
    g.g1 = gamma - 1.0;
    g.half_g1 = 0.5 * (gamma - 1.0);
    g.inv_g1 = 1.0 / (gamma - 1.0);
    g.two_inv_g1 = 2.0 / (gamma - 1.0);
    g.quarter_g1 = 0.25 * (gamma - 1.0);
    g.inv_gamma = 1.0 / gamma;
    g.p_inf = 0.0;
    g.inv_cv = 0.0;
    g.mu = 0.0;
    g.kappa = 0.0;
    return g;
}

// Everything one launch needs, built and validated on the host.
struct Call {
    int op = 0, dim = 0, dtype = 0;
    Args a{};
    Range ranges[8];            // field sets of the call, for alias checks
    int nranges = 0;
    bool inplace_ok = false;    // K -> K transform
    size_t unit_out0 = 1;       // elements per point of out0 (K*K for blocks)
    size_t unit_out1 = 1;       // elements per point of out1 (K*K for blocks)
};

// Register one field set: checks NULL, ld and alignment.
int add_fields(Call &c, const void *base, int64_t ld, int64_t fields, int64_t unit, bool input,
               bool required, const char *name)
{
    const int64_t n = c.a.n;
    const size_t es = elem_size(c.dtype);
    if (base == nullptr) {
        if (required && n > 0) return fail(FDBB_EINVAL, std::string(name) + " must not be NULL");
        return FDBB_OK;
    }
    if (fields > 1 && ld < n) return fail(FDBB_EINVAL, std::string("ld of ") + name + " must be >= n");
    if ((uintptr_t)base % es != 0)
        return fail(FDBB_EALIGN, std::string(name) + " is not aligned to its element size");
    if (n > 0) {
        if (c.nranges >= 8) return fail(FDBB_EINVAL, "too many field sets in one call");
        c.ranges[c.nranges++] = field_range(base, fields > 1 ? ld : 0, fields, n, unit, es, input);
    }
    return FDBB_OK;
}

int check_alias(const Call &c)
{
    const Range *R = c.ranges;
    for (int i = 0; i < c.nranges; ++i)
        for (int j = i + 1; j < c.nranges; ++j) {
            if (R[i].input && R[j].input) continue;
            if (!overlap(R[i], R[j])) continue;
            const bool exact = R[i].base == R[j].base && R[i].ld == R[j].ld && R[i].input != R[j].input;
            if (exact && c.inplace_ok) continue;
            return fail(FDBB_EALIAS, "input and output field sets overlap");
        }
    return FDBB_OK;
}

// 16-byte access is allowed when every base is 16-byte aligned and every row
// stride is a multiple of 16 bytes.
bool vector_ok(const Call &c)
{
    const size_t es = elem_size(c.dtype);
    const void *bases[6] = {c.a.in0, c.a.in1, c.a.in2, c.a.out0, c.a.out1, c.a.out2};
    const int64_t lds[6] = {c.a.ld_in0, c.a.ld_in1, c.a.ld_in2, c.a.ld_out0, c.a.ld_out1, c.a.ld_out2};
    const size_t units[6] = {1, 1, 1, c.unit_out0, c.unit_out1, 1};
    for (int k = 0; k < 6; ++k) {
        if (!bases[k]) continue;
        if ((uintptr_t)bases[k] % 16 != 0) return false;
        if (((size_t)lds[k] * units[k] * es) % 16 != 0) return false;
    }
    return true;
}

int family_of(int op)
{
    switch (op) {
    case FDBB_OP_CONS2PRIM: return kFamCons2Prim;
    case FDBB_OP_PRIM2CONS: return kFamPrim2Cons;
    case FDBB_OP_EOS: return kFamEos;
    case FDBB_OP_FLUX:
    case FDBB_OP_FLUX_DIR: return kFamFlux;
    case FDBB_OP_RIEMANN: return kFamRiemann;
    case FDBB_OP_CONS2CHAR: return kFamCons2Char;
    case FDBB_OP_CHAR2CONS: return kFamChar2Cons;
    case FDBB_OP_FLUX_JACOBIAN:
    case FDBB_OP_FUSED: return kFamFused;
    case FDBB_OP_ADJOINT: return kFamAdjoint;
    case FDBB_OP_V_MAG2: return kFamVmag2;
    case FDBB_OP_EIGENVECTORS: return kFamEigen;
    case FDBB_OP_CHAR_APPLY: return kFamCharApply;
    case FDBB_OP_ROE_AVERAGE: return kFamRoe;
    case FDBB_OP_EOS_PVT: return kFamEosPvt;
    case FDBB_OP_VISCOUS_FLUX: return kFamViscous;
    default: return -1;
    }
}

const void *kernel_for(int op, int dim, int dtype, int ppt, bool nt)
{
    const int fam = family_of(op);
    switch (fam) {
    case kFamCons2Prim:
    case kFamPrim2Cons:
    case kFamEos:
    case kFamFlux:
    case kFamRiemann:
    case kFamVmag2:
    case kFamRoe:
    case kFamEosPvt:
    case kFamViscous: return kernel_pointwise(fam, dim, dtype, ppt, nt);
    case kFamCons2Char:
    case kFamChar2Cons: return kernel_char(fam, dim, dtype, ppt, nt);
    case kFamFused: return kernel_fused(dim, dtype, ppt, nt);
    case kFamAdjoint: return kernel_adjoint(dim, dtype, ppt, nt);
    case kFamEigen:
    case kFamCharApply: return kernel_eigen(fam, dim, dtype, ppt, nt);
    default: return nullptr;
    }
}

bool stages_blocks(int op) { return family_of(op) == kFamFused || family_of(op) == kFamEigen; }

size_t lds_bytes(int op, int dim, int dtype, int block, int ppt)
{
    if (!stages_blocks(op)) return 0;
    // Jacobian blocks only need staging when they are written.
    const size_t K = (size_t)dim + 2;
    return (size_t)block * ppt * K * K * elem_size(dtype);
}

// Kernels whose dynamic-LDS limit has been raised on a device, as an
// open-addressed set of (kernel address | device << 56) keys.  The limit is
// raised once, to the device maximum, the first time a kernel needs more
// than the default 64 KB; later launches only look the key up (no lock, no
// runtime call).  Two threads may both raise it for the same kernel the
// first time; the call is idempotent.
constexpr int kAttrSlots = 4096;
std::atomic<uintptr_t> g_attr_done[kAttrSlots];

int set_lds_attr(const void *fn, size_t lds, const DeviceInfo &dev)
{
    if (lds <= 65536) return FDBB_OK;
    if (lds > dev.lds_max) return fail(FDBB_EINVAL, "launch configuration needs more LDS than a workgroup may use");
    const uintptr_t key = (uintptr_t)fn | ((uintptr_t)(dev.id + 1) << 56);
    size_t h = (size_t)((key >> 4) * 0x9E3779B97F4A7C15ull) % kAttrSlots;
    for (int probe = 0; probe < kAttrSlots; ++probe, h = (h + 1) % kAttrSlots) {
        uintptr_t v = g_attr_done[h].load(std::memory_order_acquire);
        if (v == key) return FDBB_OK;
        if (v != 0) continue;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dev.lds_max);
        if (e != hipSuccess) return fail_hip(e, "hipFuncSetAttribute");
        uintptr_t expected = 0;
        if (g_attr_done[h].compare_exchange_strong(expected, key, std::memory_order_acq_rel)) return FDBB_OK;
        if (expected == key) return FDBB_OK;
        // another kernel took this slot meanwhile: keep probing
    }
    return FDBB_OK;  // table full (more kernels than exist): the limit is raised anyway
}

int launch(Call &c, void *stream)
{
    if (c.a.n == 0) return FDBB_OK;
    int rc = check_alias(c);
    if (rc) return rc;
    if (vector_ok(c)) c.a.flags |= kFlagVector;

    const Config cfg = get_config(c.op, c.dim, c.dtype, c.a.n);
    const void *fn = kernel_for(c.op, c.dim, c.dtype, cfg.ppt, cfg.nt != 0);
    if (!fn) return fail(FDBB_EINVAL, "no kernel for this configuration");
    DeviceInfo dev;
    rc = device_info(&dev);
    if (rc) return rc;
    const bool needs_lds = (c.op == FDBB_OP_FLUX_JACOBIAN) || (c.op == FDBB_OP_FUSED && c.a.out1) ||
                           (c.op == FDBB_OP_EIGENVECTORS);
    const size_t lds = needs_lds ? lds_bytes(c.op, c.dim, c.dtype, cfg.block, cfg.ppt) : 0;
    rc = set_lds_attr(fn, lds, dev);
    if (rc) return rc;

    const int64_t tile_pts = (int64_t)cfg.block * cfg.ppt;
    int64_t ntiles = (c.a.n + tile_pts - 1) / tile_pts;
    int64_t grid = ntiles;
    if (cfg.grid_cap > 0 && grid > cfg.grid_cap) grid = cfg.grid_cap;
    // keep a dispatch below 2^31 work-items (the grid-dimension bound HIP
    // reports on this device); the kernels loop over tiles, so a capped grid
    // still covers every point
    const int64_t max_grid = 0x7fffffffLL / cfg.block;
    if (grid > max_grid) grid = max_grid;
    void *args[] = {&c.a, &ntiles};
    hipError_t e = hipLaunchKernel(fn, dim3((unsigned)grid), dim3((unsigned)cfg.block), args, lds,
                                   (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return FDBB_OK;
}

int begin(Call &c, int op, int dim, double gamma, int dtype, int64_t n)
{
    int rc = check_common(dim, gamma, dtype, n);
    if (rc) return rc;
    c.op = op;
    c.dim = dim;
    c.dtype = dtype;
    c.a.n = n;
    c.a.gas = make_gas(gamma);
    g_last_error.clear();
    return FDBB_OK;
}

// Fills c for any op from the task-style argument list; shared by the
// single-call entry points and the batch plans.  `mode` selects R (1) or L
// (0) for the characteristic products.
int build_call(Call &c, const fdbb_task &t, int mode = 0)
{
    int rc = begin(c, t.op, t.dim, t.gamma, t.dtype, t.n);
    if (rc) return rc;
    const int D = t.dim, K = D + 2;
    Args &a = c.a;
    a.dir = 0;
    switch (t.op) {
    case FDBB_OP_CONS2PRIM:
    case FDBB_OP_PRIM2CONS:
    case FDBB_OP_CONS2CHAR:
    case FDBB_OP_CHAR2CONS: {
        if (t.op == FDBB_OP_CONS2CHAR || t.op == FDBB_OP_CHAR2CONS) {
            if (t.dir < 0 || t.dir >= D) return fail(FDBB_EINVAL, "dir out of range");
            a.dir = t.dir;
        }
        c.inplace_ok = true;
        a.in0 = t.in0, a.ld_in0 = t.ld_in0, a.out0 = t.out0, a.ld_out0 = t.ld_out0;
        if ((rc = add_fields(c, t.in0, t.ld_in0, K, 1, true, true, "input"))) return rc;
        if ((rc = add_fields(c, t.out0, t.ld_out0, K, 1, false, true, "output"))) return rc;
        if (t.in0 == t.out0 && t.ld_in0 == t.ld_out0 &&
            (t.op == FDBB_OP_CONS2PRIM || t.op == FDBB_OP_PRIM2CONS))
            a.flags |= kFlagInPlace;
        break;
    }
    case FDBB_OP_EOS:
        if (!t.out0 && !t.out1 && t.n > 0) return fail(FDBB_EINVAL, "p and c must not both be NULL");
        a.in0 = t.in0, a.ld_in0 = t.ld_in0, a.out0 = t.out0, a.out1 = t.out1;
        if ((rc = add_fields(c, t.in0, t.ld_in0, K, 1, true, true, "U"))) return rc;
        if ((rc = add_fields(c, t.out0, 0, 1, 1, false, false, "p"))) return rc;
        if ((rc = add_fields(c, t.out1, 0, 1, 1, false, false, "c"))) return rc;
        break;
    case FDBB_OP_FLUX:
        a.in0 = t.in0, a.ld_in0 = t.ld_in0, a.out0 = t.out0, a.ld_out0 = t.ld_out0;
        if ((rc = add_fields(c, t.in0, t.ld_in0, K, 1, true, true, "U"))) return rc;
        if ((rc = add_fields(c, t.out0, t.ld_out0, (int64_t)K * D, 1, false, true, "F"))) return rc;
        break;
    case FDBB_OP_FLUX_DIR:
        if (t.dir < 0 || t.dir >= D) return fail(FDBB_EINVAL, "dir out of range");
        a.dir = t.dir;
        a.flags |= kFlagOneDir;
        a.in0 = t.in0, a.ld_in0 = t.ld_in0, a.out0 = t.out0, a.ld_out0 = t.ld_out0;
        if ((rc = add_fields(c, t.in0, t.ld_in0, K, 1, true, true, "U"))) return rc;
        if ((rc = add_fields(c, t.out0, t.ld_out0, K, 1, false, true, "F_dir"))) return rc;
        break;
    case FDBB_OP_EIGENVECTORS:
        if (!t.out0 && !t.out1 && t.n > 0) return fail(FDBB_EINVAL, "L and R must not both be NULL");
        c.unit_out0 = c.unit_out1 = (size_t)K * K;
        a.in0 = t.in0, a.ld_in0 = t.ld_in0;
        a.out0 = t.out0, a.ld_out0 = t.ld_out0, a.out1 = t.out1, a.ld_out1 = t.ld_out1;
        if ((rc = add_fields(c, t.in0, t.ld_in0, K, 1, true, true, "U"))) return rc;
        if ((rc = add_fields(c, t.out0, t.ld_out0, D, (int64_t)K * K, false, false, "L"))) return rc;
        if ((rc = add_fields(c, t.out1, t.ld_out1, D, (int64_t)K * K, false, false, "R"))) return rc;
        break;
    case FDBB_OP_CHAR_APPLY:
        if (t.dir < 0 || t.dir >= D) return fail(FDBB_EINVAL, "dir out of range");
        if (mode != 0 && mode != 1) return fail(FDBB_EINVAL, "mode must be 0 (L) or 1 (R)");
        a.dir = t.dir;
        if (mode == 1) a.flags |= kFlagRight;
        c.inplace_ok = true;
        a.in0 = t.in0, a.ld_in0 = t.ld_in0, a.in1 = t.in1, a.ld_in1 = t.ld_in1;
        a.out0 = t.out0, a.ld_out0 = t.ld_out0;
        if ((rc = add_fields(c, t.in0, t.ld_in0, K, 1, true, true, "U"))) return rc;
        if ((rc = add_fields(c, t.in1, t.ld_in1, K, 1, true, true, "X"))) return rc;
        if ((rc = add_fields(c, t.out0, t.ld_out0, K, 1, false, true, "Y"))) return rc;
        break;
    case FDBB_OP_EOS_PVT:
        if (!t.out0 && !t.out1 && !t.out2 && t.n > 0) return fail(FDBB_EINVAL, "p, c and T must not all be NULL");
        a.in0 = t.in0, a.ld_in0 = t.ld_in0, a.out0 = t.out0, a.out1 = t.out1, a.out2 = t.out2;
        if ((rc = add_fields(c, t.in0, t.ld_in0, K, 1, true, true, "U"))) return rc;
        if ((rc = add_fields(c, t.out0, 0, 1, 1, false, false, "p"))) return rc;
        if ((rc = add_fields(c, t.out1, 0, 1, 1, false, false, "c"))) return rc;
        if ((rc = add_fields(c, t.out2, 0, 1, 1, false, false, "T"))) return rc;
        break;
    case FDBB_OP_ROE_AVERAGE:
        c.inplace_ok = true;
        a.in0 = t.in0, a.ld_in0 = t.ld_in0, a.in1 = t.in1, a.ld_in1 = t.ld_in1;
        a.out0 = t.out0, a.ld_out0 = t.ld_out0;
        if ((rc = add_fields(c, t.in0, t.ld_in0, K, 1, true, true, "UL"))) return rc;
        if ((rc = add_fields(c, t.in1, t.ld_in1, K, 1, true, true, "UR"))) return rc;
        if ((rc = add_fields(c, t.out0, t.ld_out0, K, 1, false, true, "Uh"))) return rc;
        break;
    case FDBB_OP_V_MAG2:
        a.in0 = t.in0, a.ld_in0 = t.ld_in0, a.out0 = t.out0;
        if ((rc = add_fields(c, t.in0, t.ld_in0, D + 1, 1, true, true, "U"))) return rc;
        if ((rc = add_fields(c, t.out0, 0, 1, 1, false, true, "y"))) return rc;
        break;
    case FDBB_OP_RIEMANN:
        a.in0 = t.in0, a.ld_in0 = t.ld_in0, a.out0 = t.out0, a.ld_out0 = t.ld_out0;
        if ((rc = add_fields(c, t.in0, t.ld_in0, K, 1, true, true, "U"))) return rc;
        if ((rc = add_fields(c, t.out0, t.ld_out0, 2 * D + 1, 1, false, true, "R"))) return rc;
        break;
    case FDBB_OP_FLUX_JACOBIAN:
        // The Jacobian blocks travel in out1 of the fused kernel.
        c.unit_out1 = (size_t)K * K;
        a.in0 = t.in0, a.ld_in0 = t.ld_in0, a.out1 = t.out0, a.ld_out1 = t.ld_out0;
        if ((rc = add_fields(c, t.in0, t.ld_in0, K, 1, true, true, "U"))) return rc;
        if ((rc = add_fields(c, t.out0, t.ld_out0, D, (int64_t)K * K, false, true, "A"))) return rc;
        break;
    case FDBB_OP_FUSED:
        if (!t.out0 && !t.out1 && !t.out2 && t.n > 0) return fail(FDBB_EINVAL, "F, A and R must not all be NULL");
        c.unit_out1 = (size_t)K * K;
        a.in0 = t.in0, a.ld_in0 = t.ld_in0;
        a.out0 = t.out0, a.ld_out0 = t.ld_out0;
        a.out1 = t.out1, a.ld_out1 = t.ld_out1;
        a.out2 = t.out2, a.ld_out2 = t.ld_out2;
        if ((rc = add_fields(c, t.in0, t.ld_in0, K, 1, true, true, "U"))) return rc;
        if ((rc = add_fields(c, t.out0, t.ld_out0, (int64_t)K * D, 1, false, false, "F"))) return rc;
        if ((rc = add_fields(c, t.out1, t.ld_out1, D, (int64_t)K * K, false, false, "A"))) return rc;
        if ((rc = add_fields(c, t.out2, t.ld_out2, 2 * D + 1, 1, false, false, "R"))) return rc;
        break;
    case FDBB_OP_ADJOINT:
        if (t.dir < -1 || t.dir >= D) return fail(FDBB_EINVAL, "dir out of range");
        a.dir = t.dir;
        a.in0 = t.in0, a.ld_in0 = t.ld_in0, a.in1 = t.in1, a.ld_in1 = t.ld_in1;
        a.out0 = t.out0, a.ld_out0 = t.ld_out0;
        if ((rc = add_fields(c, t.in0, t.ld_in0, K, 1, true, true, "U"))) return rc;
        if ((rc = add_fields(c, t.in1, t.ld_in1, t.dir < 0 ? (int64_t)K * D : K, 1, true, true, "Fbar")))
            return rc;
        if ((rc = add_fields(c, t.out0, t.ld_out0, K, 1, false, true, "Ubar"))) return rc;
        break;
    case FDBB_OP_VISCOUS_FLUX:
        return fail(FDBB_EINVAL, "the viscous flux needs its gradients and coefficients: call fdbb_viscous_flux");
    default: return fail(FDBB_EINVAL, "unknown op");
    }
    return FDBB_OK;
}

// Ops a batch plan can run: everything the persistent kernel dispatches.
// The eigenvector blocks and characteristic products have kernels of their
// own, and the general EOS needs parameters a task does not carry.
bool batchable(int op)
{
    return op >= 0 && op < FDBB_NUM_OPS && op != FDBB_OP_EIGENVECTORS && op != FDBB_OP_CHAR_APPLY &&
           op != FDBB_OP_EOS_PVT && op != FDBB_OP_VISCOUS_FLUX;
}

fdbb_task make_task(int op, int dim, int dir, double gamma, int dtype, int64_t n)
{
    fdbb_task t;
    std::memset(&t, 0, sizeof(t));
    t.op = op;
    t.dim = dim;
    t.dir = dir;
    t.gamma = gamma;
    t.dtype = dtype;
    t.n = n;
    return t;
}

int run(const fdbb_task &t, void *stream, int mode = 0)
{
    Call c;
    int rc = build_call(c, t, mode);
    if (rc) return rc;
    return launch(c, stream);
}

}  // namespace

// ================================================================ C ABI

extern "C" {

int fdbb_cons2prim(int dim, double gamma, int dtype, const void *U, int64_t ldU, void *V, int64_t ldV,
                   int64_t n, void *stream)
{
    fdbb_task t = make_task(FDBB_OP_CONS2PRIM, dim, 0, gamma, dtype, n);
    t.in0 = U, t.ld_in0 = ldU, t.out0 = V, t.ld_out0 = ldV;
    return run(t, stream);
}

int fdbb_prim2cons(int dim, double gamma, int dtype, const void *V, int64_t ldV, void *U, int64_t ldU,
                   int64_t n, void *stream)
{
    fdbb_task t = make_task(FDBB_OP_PRIM2CONS, dim, 0, gamma, dtype, n);
    t.in0 = V, t.ld_in0 = ldV, t.out0 = U, t.ld_out0 = ldU;
    return run(t, stream);
}

int fdbb_velocity_magnitude2(int dim, int dtype, const void *U, int64_t ldU, void *y, int64_t n, void *stream)
{
    // gamma does not enter |v|^2; any valid value passes validation
    fdbb_task t = make_task(FDBB_OP_V_MAG2, dim, 0, 1.4, dtype, n);
    t.in0 = U, t.ld_in0 = ldU, t.out0 = y;
    return run(t, stream);
}

int fdbb_eos(int dim, double gamma, int dtype, const void *U, int64_t ldU, void *p, void *c, int64_t n,
             void *stream)
{
    fdbb_task t = make_task(FDBB_OP_EOS, dim, 0, gamma, dtype, n);
    t.in0 = U, t.ld_in0 = ldU, t.out0 = p, t.out1 = c;
    return run(t, stream);
}

int fdbb_flux(int dim, double gamma, int dtype, const void *U, int64_t ldU, void *F, int64_t ldF, int64_t n,
              void *stream)
{
    fdbb_task t = make_task(FDBB_OP_FLUX, dim, 0, gamma, dtype, n);
    t.in0 = U, t.ld_in0 = ldU, t.out0 = F, t.ld_out0 = ldF;
    return run(t, stream);
}

int fdbb_flux_direction(int dim, int dir, double gamma, int dtype, const void *U, int64_t ldU, void *Fd,
                        int64_t ldFd, int64_t n, void *stream)
{
    fdbb_task t = make_task(FDBB_OP_FLUX_DIR, dim, dir, gamma, dtype, n);
    t.in0 = U, t.ld_in0 = ldU, t.out0 = Fd, t.ld_out0 = ldFd;
    return run(t, stream);
}

int fdbb_flux_jacobian(int dim, double gamma, int dtype, const void *U, int64_t ldU, void *A, int64_t ldA,
                       int64_t n, void *stream)
{
    fdbb_task t = make_task(FDBB_OP_FLUX_JACOBIAN, dim, 0, gamma, dtype, n);
    t.in0 = U, t.ld_in0 = ldU, t.out0 = A, t.ld_out0 = ldA;
    return run(t, stream);
}

int fdbb_riemann_invariants(int dim, double gamma, int dtype, const void *U, int64_t ldU, void *R,
                            int64_t ldR, int64_t n, void *stream)
{
    fdbb_task t = make_task(FDBB_OP_RIEMANN, dim, 0, gamma, dtype, n);
    t.in0 = U, t.ld_in0 = ldU, t.out0 = R, t.ld_out0 = ldR;
    return run(t, stream);
}

int fdbb_cons2char(int dim, int dir, double gamma, int dtype, const void *U, int64_t ldU, void *W,
                   int64_t ldW, int64_t n, void *stream)
{
    fdbb_task t = make_task(FDBB_OP_CONS2CHAR, dim, dir, gamma, dtype, n);
    t.in0 = U, t.ld_in0 = ldU, t.out0 = W, t.ld_out0 = ldW;
    return run(t, stream);
}

int fdbb_char2cons(int dim, int dir, double gamma, int dtype, const void *W, int64_t ldW, void *U,
                   int64_t ldU, int64_t n, void *stream)
{
    fdbb_task t = make_task(FDBB_OP_CHAR2CONS, dim, dir, gamma, dtype, n);
    t.in0 = W, t.ld_in0 = ldW, t.out0 = U, t.ld_out0 = ldU;
    return run(t, stream);
}

int fdbb_euler_fused(int dim, double gamma, int dtype, const void *U, int64_t ldU, void *F, int64_t ldF,
                     void *A, int64_t ldA, void *R, int64_t ldR, int64_t n, void *stream)
{
    fdbb_task t = make_task(FDBB_OP_FUSED, dim, 0, gamma, dtype, n);
    t.in0 = U, t.ld_in0 = ldU;
    t.out0 = F, t.ld_out0 = ldF;
    t.out1 = A, t.ld_out1 = ldA;
    t.out2 = R, t.ld_out2 = ldR;
    return run(t, stream);
}

int fdbb_flux_adjoint(int dim, int dir, double gamma, int dtype, const void *U, int64_t ldU,
                      const void *Fbar, int64_t ldFbar, void *Ubar, int64_t ldUbar, int64_t n, void *stream)
{
    fdbb_task t = make_task(FDBB_OP_ADJOINT, dim, dir, gamma, dtype, n);
    t.in0 = U, t.ld_in0 = ldU, t.in1 = Fbar, t.ld_in1 = ldFbar, t.out0 = Ubar, t.ld_out0 = ldUbar;
    return run(t, stream);
}

int fdbb_eigenvectors(int dim, double gamma, int dtype, const void *U, int64_t ldU, void *L, int64_t ldL,
                      void *R, int64_t ldR, int64_t n, void *stream)
{
    fdbb_task t = make_task(FDBB_OP_EIGENVECTORS, dim, 0, gamma, dtype, n);
    t.in0 = U, t.ld_in0 = ldU, t.out0 = L, t.ld_out0 = ldL, t.out1 = R, t.ld_out1 = ldR;
    return run(t, stream);
}

int fdbb_char_apply(int dim, int dir, int mode, double gamma, int dtype, const void *U, int64_t ldU,
                    const void *X, int64_t ldX, void *Y, int64_t ldY, int64_t n, void *stream)
{
    fdbb_task t = make_task(FDBB_OP_CHAR_APPLY, dim, dir, gamma, dtype, n);
    t.in0 = U, t.ld_in0 = ldU, t.in1 = X, t.ld_in1 = ldX, t.out0 = Y, t.ld_out0 = ldY;
    return run(t, stream, mode);
}

int fdbb_roe_average(int dim, double gamma, int dtype, const void *UL, int64_t ldUL, const void *UR,
                     int64_t ldUR, void *Uh, int64_t ldUh, int64_t n, void *stream)
{
    fdbb_task t = make_task(FDBB_OP_ROE_AVERAGE, dim, 0, gamma, dtype, n);
    t.in0 = UL, t.ld_in0 = ldUL, t.in1 = UR, t.ld_in1 = ldUR, t.out0 = Uh, t.ld_out0 = ldUh;
    return run(t, stream);
}

int fdbb_eos_pvt(int dim, int eos, const double *params, int dtype, const void *U, int64_t ldU, void *p,
                 void *c, void *T, int64_t n, void *stream)
{
    g_last_error.clear();
    if (!params) return fail(FDBB_EINVAL, "params must not be NULL");
    double gamma = 0.0, p_inf = 0.0, cv = 0.0;
    if (eos == FDBB_EOS_PERFECT_GAS) {
        const double cp = params[0];
        cv = params[1];
        if (!std::isfinite(cp) || !std::isfinite(cv) || !(cv > 0.0) || !(cp > cv))
            return fail(FDBB_EINVAL, "perfect gas needs c_p > c_v > 0");
        gamma = cp / cv;
    } else if (eos == FDBB_EOS_STIFFENED_GAS) {
        gamma = params[0];
        p_inf = params[1];
        cv = params[2];
        if (!std::isfinite(p_inf) || !(p_inf >= 0.0) || !std::isfinite(cv) || !(cv > 0.0))
            return fail(FDBB_EINVAL, "stiffened gas needs p_inf >= 0 and c_v > 0");
    } else {
        return fail(FDBB_EINVAL, "unknown EOS id");
    }
    fdbb_task t = make_task(FDBB_OP_EOS_PVT, dim, 0, gamma, dtype, n);
    t.in0 = U, t.ld_in0 = ldU, t.out0 = p, t.out1 = c, t.out2 = T;
    Call call;
    int rc = build_call(call, t);
    if (rc) return rc;
    call.a.gas.p_inf = p_inf;
    call.a.gas.inv_cv = 1.0 / cv;
    return launch(call, stream);
}

int fdbb_viscous_flux(int dim, double mu, double kappa, int dtype, const void *U, int64_t ldU, const void *G,
                      int64_t ldG, const void *gradT, int64_t ldGT, void *Fv, int64_t ldFv, int64_t n,
                      void *stream)
{
    Call c;
    // gamma does not enter the viscous flux; any valid value passes the checks
    int rc = begin(c, FDBB_OP_VISCOUS_FLUX, dim, 2.0, dtype, n);
    if (rc) return rc;
    if (!std::isfinite(mu) || !(mu >= 0.0) || !std::isfinite(kappa) || !(kappa >= 0.0))
        return fail(FDBB_EINVAL, "mu and kappa must be finite and >= 0");
    const int64_t D = dim, K = D + 2;
    Args &a = c.a;
    a.in0 = U, a.ld_in0 = ldU, a.in1 = G, a.ld_in1 = ldG, a.in2 = gradT, a.ld_in2 = ldGT;
    a.out0 = Fv, a.ld_out0 = ldFv;
    a.gas.mu = mu;
    a.gas.kappa = kappa;
    if ((rc = add_fields(c, U, ldU, K, 1, true, true, "U"))) return rc;
    if ((rc = add_fields(c, G, ldG, D * D, 1, true, true, "G"))) return rc;
    if ((rc = add_fields(c, gradT, ldGT, D, 1, true, true, "gradT"))) return rc;
    if ((rc = add_fields(c, Fv, ldFv, K * D, 1, false, true, "Fv"))) return rc;
    return launch(c, stream);
}

int fdbb_task_check(const fdbb_task *task)
{
    if (!task) return fail(FDBB_EINVAL, "task must not be NULL");
    if (task->op == FDBB_OP_EOS_PVT) return fail(FDBB_EINVAL, "the general EOS needs its parameters: call fdbb_eos_pvt");
    Call c;
    int rc = build_call(c, *task);
    if (!rc) rc = check_alias(c);
    return rc;
}

int fdbb_task_run(const fdbb_task *task, void *stream)
{
    if (!task) return fail(FDBB_EINVAL, "task must not be NULL");
    if (task->op == FDBB_OP_EOS_PVT) return fail(FDBB_EINVAL, "the general EOS needs its parameters: call fdbb_eos_pvt");
    return run(*task, stream);
}

int fdbb_set_launch_config(int op, int dim, int dtype, int block, int ppt, int grid_cap, int nontemporal)
{
    if (op < 0 || op >= FDBB_NUM_OPS || dim < 1 || dim > 3 || (dtype != FDBB_F64 && dtype != FDBB_F32))
        return fail(FDBB_EINVAL, "unknown op, dim or dtype");
    if (!config_ok(block, ppt, grid_cap, nontemporal)) return fail(FDBB_EINVAL, "invalid launch configuration");
    if (stages_blocks(op) && block > kMaxBlockStaged)
        return fail(FDBB_EINVAL, "kernels that stage K x K blocks take at most 256 threads per workgroup");
    std::call_once(g_cfg_once, init_configs);
    Config c{block, ppt, grid_cap, nontemporal};
    g_cfg[op][dim - 1][dtype].store(pack(c));
    return FDBB_OK;
}

int fdbb_get_launch_config(int op, int dim, int dtype, int *block, int *ppt, int *grid_cap, int *nontemporal)
{
    if (op < 0 || op >= FDBB_NUM_OPS || dim < 1 || dim > 3 || (dtype != FDBB_F64 && dtype != FDBB_F32))
        return fail(FDBB_EINVAL, "unknown op, dim or dtype");
    const Config c = get_config(op, dim, dtype);
    if (block) *block = c.block;
    if (ppt) *ppt = c.ppt;
    if (grid_cap) *grid_cap = c.grid_cap;
    if (nontemporal) *nontemporal = c.nt;
    return FDBB_OK;
}

int fdbb_set_small_launch_config(int op, int dim, int dtype, int64_t max_n, int block, int ppt, int grid_cap,
                                 int nontemporal)
{
    if (op < 0 || op >= FDBB_NUM_OPS || dim < 1 || dim > 3 || (dtype != FDBB_F64 && dtype != FDBB_F32))
        return fail(FDBB_EINVAL, "unknown op, dim or dtype");
    if (max_n < 0) return fail(FDBB_EINVAL, "max_n must not be negative");
    if (max_n == 0) {
        g_small_max[op][dim - 1][dtype].store(0, std::memory_order_release);
        return FDBB_OK;
    }
    if (!config_ok(block, ppt, grid_cap, nontemporal)) return fail(FDBB_EINVAL, "invalid launch configuration");
    if (stages_blocks(op) && block > kMaxBlockStaged)
        return fail(FDBB_EINVAL, "kernels that stage K x K blocks take at most 256 threads per workgroup");
    // clear the bound while the configuration changes, then publish both
    g_small_max[op][dim - 1][dtype].store(0, std::memory_order_release);
    g_small_cfg[op][dim - 1][dtype].store(pack(Config{block, ppt, grid_cap, nontemporal}), std::memory_order_relaxed);
    g_small_max[op][dim - 1][dtype].store(max_n, std::memory_order_release);
    return FDBB_OK;
}

int fdbb_get_small_launch_config(int op, int dim, int dtype, int64_t *max_n, int *block, int *ppt, int *grid_cap,
                                 int *nontemporal)
{
    if (op < 0 || op >= FDBB_NUM_OPS || dim < 1 || dim > 3 || (dtype != FDBB_F64 && dtype != FDBB_F32))
        return fail(FDBB_EINVAL, "unknown op, dim or dtype");
    const int64_t m = g_small_max[op][dim - 1][dtype].load(std::memory_order_acquire);
    const Config c = m > 0 ? unpack(g_small_cfg[op][dim - 1][dtype].load(std::memory_order_relaxed))
                           : get_config(op, dim, dtype);
    if (max_n) *max_n = m;
    if (block) *block = c.block;
    if (ppt) *ppt = c.ppt;
    if (grid_cap) *grid_cap = c.grid_cap;
    if (nontemporal) *nontemporal = c.nt;
    return FDBB_OK;
}

int fdbb_launch_config_for(int op, int dim, int dtype, int64_t n, int *block, int *ppt, int *grid_cap,
                           int *nontemporal)
{
    if (op < 0 || op >= FDBB_NUM_OPS || dim < 1 || dim > 3 || (dtype != FDBB_F64 && dtype != FDBB_F32))
        return fail(FDBB_EINVAL, "unknown op, dim or dtype");
    if (n < 0) return fail(FDBB_EINVAL, "n must not be negative");
    const Config c = get_config(op, dim, dtype, n);
    if (block) *block = c.block;
    if (ppt) *ppt = c.ppt;
    if (grid_cap) *grid_cap = c.grid_cap;
    if (nontemporal) *nontemporal = c.nt;
    return FDBB_OK;
}

int fdbb_kernel_info(int op, int dim, int dtype, int ppt, int nontemporal, int *vgprs, int *scratch_bytes)
{
    if (op < 0 || op >= FDBB_NUM_OPS || dim < 1 || dim > 3 || (dtype != FDBB_F64 && dtype != FDBB_F32) ||
        !(ppt == 1 || ppt == 2 || ppt == 4) || (nontemporal != 0 && nontemporal != 1))
        return fail(FDBB_EINVAL, "unknown op, dim, dtype, ppt or store mode");
    const void *fn = kernel_for(op, dim, dtype, ppt, nontemporal != 0);
    if (!fn) return fail(FDBB_EINVAL, "no kernel for this configuration");
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, fn);
    if (e != hipSuccess) return fail_hip(e, "hipFuncGetAttributes");
    if (vgprs) *vgprs = attr.numRegs;
    if (scratch_bytes) *scratch_bytes = (int)attr.localSizeBytes;
    return FDBB_OK;
}

const char *fdbb_status_string(int status)
{
    switch (status) {
    case FDBB_OK: return "ok";
    case FDBB_EINVAL: return "invalid argument";
    case FDBB_EALIGN: return "misaligned pointer";
    case FDBB_EALIAS: return "input and output overlap";
    case FDBB_EHIP: return "HIP runtime error";
    case FDBB_ENOMEM: return "out of memory";
    default: return "unknown status";
    }
}

const char *fdbb_last_error(void) { return g_last_error.c_str(); }

int fdbb_version(void) { return 400; }

}  // extern "C"

// ================================================================ batches

// Layout of a task table, on the device and in its host staging copy:
// [header: ntasks, ntiles (int64)][tile prefix sums, cap + 1 int64][pad to
// 64 B][cap TaskDev].
static size_t table_task_offset(int cap) { return ((2 + (size_t)cap + 1) * sizeof(int64_t) + 63) & ~(size_t)63; }
static size_t table_bytes(int cap) { return table_task_offset(cap) + (size_t)cap * sizeof(TaskDev); }
static int64_t *table_header(unsigned char *base) { return reinterpret_cast<int64_t *>(base); }
static int64_t *table_prefix(unsigned char *base) { return reinterpret_cast<int64_t *>(base) + 2; }
static TaskDev *table_tasks(unsigned char *base, int cap) { return reinterpret_cast<TaskDev *>(base + table_task_offset(cap)); }

struct fdbb_batch_plan {
    int device = 0;
    int capacity = 0;
    int ntasks = 0;
    int block = 256;
    int ppt = 1;
    int grid = 0;
    int nt = 1;
    size_t lds = 0;      // reserved at creation: what the captured graph launches with
    size_t cur_lds = 0;  // what the current task list needs: direct launches use it
    int64_t points = 0;
    int64_t tiles = 0;
    const void *kernel = nullptr;
    unsigned char *dev = nullptr;   // task table (layout above), capacity `capacity`
    unsigned char *host = nullptr;  // pinned staging copy of the same layout
    size_t bytes = 0;
    hipEvent_t uploaded = nullptr;  // the last upload has left the staging copy
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    int64_t *header(unsigned char *base) const { return table_header(base); }
    int64_t *prefix(unsigned char *base) const { return table_prefix(base); }
    TaskDev *tasks(unsigned char *base) const { return table_tasks(base, capacity); }
};

namespace {

// What filling a task table found.
struct TableInfo {
    size_t lds = 0;      // dynamic LDS the tasks' Jacobian staging needs
    int64_t tiles = 0;
    int64_t points = 0;
};

// Validate `tasks` (each as its single-call entry point would, then every
// pair of tasks for overlapping outputs) and write the table for tiles of
// block * ppt points into `host` (layout above, capacity `cap`).  `all`
// must have room for 8 * ntasks ranges.  Uses no heap memory of its own.
int fill_table(const fdbb_task *tasks, int ntasks, int cap, int block, int ppt, unsigned char *host, Range *all,
               TableInfo *info)
{
    if (ntasks > 0 && !tasks) return fail(FDBB_EINVAL, "tasks must not be NULL");
    int64_t *hdr = table_header(host);
    int64_t *pre = table_prefix(host);
    TaskDev *td = table_tasks(host, cap);
    const int64_t tile_pts = (int64_t)block * ppt;
    size_t nall = 0;
    TableInfo r;
    for (int b = 0; b < ntasks; ++b) {
        if (!batchable(tasks[b].op))
            return fail(FDBB_EINVAL, "task " + std::to_string(b) + ": op not available in batches");
        Call c;
        int rc = build_call(c, tasks[b]);
        if (rc) return fail(rc, "task " + std::to_string(b) + ": " + g_last_error);
        rc = check_alias(c);
        if (rc) return fail(rc, "task " + std::to_string(b) + ": " + g_last_error);
        if (vector_ok(c)) c.a.flags |= kFlagVector;
        const bool jac = tasks[b].op == FDBB_OP_FLUX_JACOBIAN || (tasks[b].op == FDBB_OP_FUSED && tasks[b].out1);
        if (jac) r.lds = std::max(r.lds, lds_bytes(tasks[b].op, tasks[b].dim, tasks[b].dtype, block, ppt));
        for (int k = 0; k < c.nranges; ++k) {
            all[nall] = c.ranges[k];
            all[nall].task = b;
            ++nall;
        }
        pre[b] = r.tiles;
        r.tiles += (tasks[b].n + tile_pts - 1) / tile_pts;
        r.points += tasks[b].n;
        td[b].a = c.a;
        td[b].op = tasks[b].op;
        td[b].dim = tasks[b].dim;
        td[b].dtype = tasks[b].dtype;
        td[b].pad = 0;
    }
    // Across tasks: no output may overlap another task's input or output.
    std::sort(all, all + nall, [](const Range &x, const Range &y) { return x.lo < y.lo; });
    for (size_t i = 0; i < nall; ++i) {
        for (size_t j = i + 1; j < nall && all[j].lo < all[i].hi; ++j) {
            if (all[i].task == all[j].task) continue;
            if (all[i].input && all[j].input) continue;
            return fail(FDBB_EALIAS, "tasks " + std::to_string(all[i].task) + " and " +
                                         std::to_string(all[j].task) + " overlap");
        }
    }
    pre[ntasks] = r.tiles;
    hdr[0] = ntasks;
    hdr[1] = r.tiles;
    *info = r;
    return FDBB_OK;
}

// Validate tasks and fill the plan's pinned staging copy.
int stage_tasks(fdbb_batch_plan *p, const fdbb_task *tasks, int ntasks)
{
    if (ntasks < 0 || ntasks > p->capacity) return fail(FDBB_EINVAL, "ntasks exceeds the plan capacity");
    if (ntasks > 0 && !tasks) return fail(FDBB_EINVAL, "tasks must not be NULL");
    // Fill a private copy first, so that a rejected list neither waits for
    // nor disturbs an upload still reading the staging copy.
    std::vector<unsigned char> tmp(p->bytes);
    std::vector<Range> all((size_t)ntasks * 8);
    TableInfo info;
    int rc = fill_table(tasks, ntasks, p->capacity, p->block, p->ppt, tmp.data(), all.data(), &info);
    if (rc) return rc;
    if (info.lds > p->lds) return fail(FDBB_EINVAL, "tasks need more LDS than the plan was created with");
    // The previous upload must have consumed the staging copy.
    if (p->uploaded) {
        hipError_t e = hipEventSynchronize(p->uploaded);
        if (e != hipSuccess) return fail_hip(e, "hipEventSynchronize");
    }
    const size_t used = table_task_offset(p->capacity) + (size_t)ntasks * sizeof(TaskDev);
    std::memcpy(p->host, tmp.data(), used);
    p->ntasks = ntasks;
    p->tiles = info.tiles;
    p->points = info.points;
    p->cur_lds = info.lds;
    return FDBB_OK;
}

int upload(fdbb_batch_plan *p, hipStream_t s)
{
    // header, prefix sums and the tasks in use (not the whole capacity)
    const size_t used = (size_t)((unsigned char *)(p->tasks(p->host) + p->ntasks) - p->host);
    hipError_t e = hipMemcpyAsync(p->dev, p->host, used, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync");
    e = hipEventRecord(p->uploaded, s);
    if (e != hipSuccess) return fail_hip(e, "hipEventRecord");
    return FDBB_OK;
}

// The persistent launch of p's table with `lds` bytes of dynamic LDS (the
// reserve when captured into the graph, the current list's need when
// launched directly: a list without Jacobian staging then runs at full
// occupancy).
int launch_plan(fdbb_batch_plan *p, hipStream_t s, size_t lds)
{
    unsigned char *d = p->dev;
    const TaskDev *tasks = p->tasks(d);
    const int64_t *prefix = p->prefix(d);
    const int64_t *header = p->header(d);
    void *args[] = {&tasks, &prefix, &header};
    hipError_t e = hipLaunchKernel(p->kernel, dim3((unsigned)p->grid), dim3((unsigned)p->block), args, lds, s);
    if (e != hipSuccess) return fail_hip(e, "batch kernel launch");
    return FDBB_OK;
}

void free_plan(fdbb_batch_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->uploaded) (void)hipEventDestroy(p->uploaded);
    if (p->dev) (void)hipFree(p->dev);
    if (p->host) (void)hipHostFree(p->host);
    delete p;
}

}  // namespace

extern "C" {

int fdbb_batch_plan_create(const fdbb_task *tasks, int ntasks, int capacity, int block, int ppt, int grid,
                           int nontemporal, fdbb_batch_plan **plan)
{
    g_last_error.clear();
    if (!plan) return fail(FDBB_EINVAL, "plan must not be NULL");
    *plan = nullptr;
    if (capacity < 1 || capacity < ntasks) return fail(FDBB_EINVAL, "capacity must be >= max(1, ntasks)");
    if (ntasks > 0 && !tasks) return fail(FDBB_EINVAL, "tasks must not be NULL");
    int grid_per_cu = 0;
    if (block == 0) {
        // the installed configuration of the first task's storage type
        const BatchConfig bc = get_batch_config(ntasks > 0 ? tasks[0].dtype : FDBB_F64);
        block = bc.block, ppt = bc.ppt, nontemporal = bc.nt, grid_per_cu = bc.grid_per_cu, grid = 0;
    }
    if (!batch_config_ok(block, ppt, nontemporal) || grid < 0)
        return fail(FDBB_EINVAL, "invalid launch configuration (batches take 64..256 threads per workgroup in "
                                 "multiples of 64, 1, 2, 4 or 8 points per thread, store mode 0, 1 or 2)");
    // Argument checks of every task come before any HIP call.
    for (int b = 0; b < ntasks; ++b) {
        if (!batchable(tasks[b].op))
            return fail(FDBB_EINVAL, "task " + std::to_string(b) + ": op not available in batches");
        Call c;
        int rc = build_call(c, tasks[b]);
        if (!rc) rc = check_alias(c);
        if (rc) return fail(rc, "task " + std::to_string(b) + ": " + g_last_error);
    }
    DeviceInfo dev;
    int rc = device_info(&dev);
    if (rc) return rc;

    fdbb_batch_plan *p = new fdbb_batch_plan();
    p->capacity = capacity;
    p->block = block;
    p->ppt = ppt;
    p->kernel = kernel_batch(ppt, nontemporal);
    p->nt = nontemporal;
    (void)hipGetDevice(&p->device);
    // LDS for the largest Jacobian staging among the first task list; a plan
    // created empty reserves enough for any task (3D FP64 blocks).
    size_t lds = ntasks == 0 ? lds_bytes(FDBB_OP_FLUX_JACOBIAN, 3, FDBB_F64, block, ppt) : 0;
    for (int b = 0; b < ntasks && tasks; ++b) {
        const bool jac = tasks[b].op == FDBB_OP_FLUX_JACOBIAN || (tasks[b].op == FDBB_OP_FUSED && tasks[b].out1);
        if (jac && tasks[b].dim >= 1 && tasks[b].dim <= 3 && (tasks[b].dtype == 0 || tasks[b].dtype == 1))
            lds = std::max(lds, lds_bytes(tasks[b].op, tasks[b].dim, tasks[b].dtype, block, ppt));
    }
    p->lds = lds;
    if ((rc = set_lds_attr(p->kernel, lds, dev))) {
        free_plan(p);
        return rc;
    }
    p->grid = grid > 0 ? grid : dev.cus * (grid_per_cu > 0 ? grid_per_cu : std::max(1, 2048 / block));
    p->bytes = table_bytes(capacity);
    hipError_t e = hipMalloc((void **)&p->dev, p->bytes);
    if (e != hipSuccess) {
        free_plan(p);
        return fail_hip(e, "hipMalloc");
    }
    e = hipHostMalloc((void **)&p->host, p->bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        free_plan(p);
        return fail_hip(e, "hipHostMalloc");
    }
    std::memset(p->host, 0, p->bytes);
    e = hipEventCreateWithFlags(&p->uploaded, hipEventDisableTiming);
    if (e != hipSuccess) {
        free_plan(p);
        return fail_hip(e, "hipEventCreate");
    }
    if ((rc = stage_tasks(p, tasks, ntasks))) {
        const std::string msg = g_last_error;
        free_plan(p);
        return fail(rc, msg);
    }
    e = hipMemcpy(p->dev, p->host, p->bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_plan(p);
        return fail_hip(e, "hipMemcpy");
    }
    // Capture the persistent launch once; later task lists only change the
    // device table the kernel reads, so the graph is replayed unchanged.
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        free_plan(p);
        return fail_hip(e, "hipStreamCreate");
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = launch_plan(p, cs, p->lds);
        hipError_t e2 = hipStreamEndCapture(cs, &p->graph);
        if (rc == FDBB_OK && e2 != hipSuccess) rc = fail_hip(e2, "hipStreamEndCapture");
    } else {
        rc = fail_hip(e, "hipStreamBeginCapture");
    }
    (void)hipStreamDestroy(cs);
    if (rc == FDBB_OK) {
        e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = fail_hip(e, "hipGraphInstantiate");
    }
    if (rc) {
        const std::string msg = g_last_error;
        free_plan(p);
        return fail(rc, msg);
    }
    *plan = p;
    return FDBB_OK;
}

int fdbb_batch_plan_update(fdbb_batch_plan *plan, const fdbb_task *tasks, int ntasks, void *stream)
{
    g_last_error.clear();
    if (!plan) return fail(FDBB_EINVAL, "plan must not be NULL");
    int rc = stage_tasks(plan, tasks, ntasks);
    if (rc) return rc;
    return upload(plan, (hipStream_t)stream);
}

int fdbb_batch_exec(fdbb_batch_plan *plan, void *stream, int use_graph)
{
    g_last_error.clear();
    if (!plan) return fail(FDBB_EINVAL, "plan must not be NULL");
    if (plan->tiles == 0) return FDBB_OK;
    if (use_graph) {
        hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
        if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
        return FDBB_OK;
    }
    return launch_plan(plan, (hipStream_t)stream, plan->cur_lds);
}

int fdbb_set_batch_config(int dtype, int block, int ppt, int grid_per_cu, int nontemporal)
{
    g_last_error.clear();
    if (dtype != FDBB_F64 && dtype != FDBB_F32) return fail(FDBB_EINVAL, "unknown dtype");
    if (!batch_config_ok(block, ppt, nontemporal) || grid_per_cu < 0 || grid_per_cu > 1024)
        return fail(FDBB_EINVAL, "invalid batch configuration");
    // a plan of this configuration must be able to stage 3D Jacobian blocks
    if (lds_bytes(FDBB_OP_FLUX_JACOBIAN, 3, dtype, block, ppt) > 160 * 1024)
        return fail(FDBB_EINVAL, "batch configuration needs more LDS than a workgroup may use");
    g_batch_cfg[dtype == FDBB_F32 ? 1 : 0].store(pack_batch(BatchConfig{block, ppt, grid_per_cu, nontemporal}));
    return FDBB_OK;
}

int fdbb_set_server_batch_config(int block, int ppt, int grid_per_cu, int nontemporal)
{
    g_last_error.clear();
    if (block == 0) {
        g_batch_cfg[2].store(0);
        return FDBB_OK;
    }
    if (!batch_config_ok(block, ppt, nontemporal) || grid_per_cu < 0 || grid_per_cu > 1024)
        return fail(FDBB_EINVAL, "invalid batch configuration");
    if (lds_bytes(FDBB_OP_FLUX_JACOBIAN, 3, FDBB_F64, block, ppt) > 160 * 1024)
        return fail(FDBB_EINVAL, "batch configuration needs more LDS than a workgroup may use");
    g_batch_cfg[2].store(pack_batch(BatchConfig{block, ppt, grid_per_cu, nontemporal}));
    return FDBB_OK;
}

int fdbb_get_server_batch_config(int *block, int *ppt, int *grid_per_cu, int *nontemporal)
{
    const uint64_t v = g_batch_cfg[2].load(std::memory_order_relaxed);
    const BatchConfig c = v ? get_batch_config(2) : get_batch_config(FDBB_F64);
    if (block) *block = c.block;
    if (ppt) *ppt = c.ppt;
    if (grid_per_cu) *grid_per_cu = c.grid_per_cu;
    if (nontemporal) *nontemporal = c.nt;
    return FDBB_OK;
}

int fdbb_get_batch_config(int dtype, int *block, int *ppt, int *grid_per_cu, int *nontemporal)
{
    if (dtype != FDBB_F64 && dtype != FDBB_F32) return fail(FDBB_EINVAL, "unknown dtype");
    const BatchConfig c = get_batch_config(dtype);
    if (block) *block = c.block;
    if (ppt) *ppt = c.ppt;
    if (grid_per_cu) *grid_per_cu = c.grid_per_cu;
    if (nontemporal) *nontemporal = c.nt;
    return FDBB_OK;
}

int fdbb_batch_plan_config(const fdbb_batch_plan *plan, int *block, int *ppt, int *grid, int *nontemporal)
{
    if (!plan) return fail(FDBB_EINVAL, "plan must not be NULL");
    if (block) *block = plan->block;
    if (ppt) *ppt = plan->ppt;
    if (grid) *grid = plan->grid;
    if (nontemporal) *nontemporal = plan->nt;
    return FDBB_OK;
}

int fdbb_batch_plan_info(const fdbb_batch_plan *plan, int64_t *points, int64_t *tiles)
{
    if (!plan) return fail(FDBB_EINVAL, "plan must not be NULL");
    if (points) *points = plan->points;
    if (tiles) *tiles = plan->tiles;
    return FDBB_OK;
}

int fdbb_batch_plan_destroy(fdbb_batch_plan *plan)
{
    free_plan(plan);
    return FDBB_OK;
}

int fdbb_batch_run_noalloc(const fdbb_task *tasks, int ntasks, int block, int ppt, int grid, int nontemporal,
                           void *stream)
{
    g_last_error.clear();
    if (ntasks < 0 || ntasks > FDBB_NOALLOC_MAX_TASKS)
        return fail(FDBB_EINVAL, "the allocation-free batch takes 0 to " + std::to_string(FDBB_NOALLOC_MAX_TASKS) +
                                     " tasks, got " + std::to_string(ntasks));
    if (ntasks > 0 && !tasks) return fail(FDBB_EINVAL, "tasks must not be NULL");
    int grid_per_cu = 0;
    if (block == 0) {
        const BatchConfig bc = get_batch_config(ntasks > 0 ? tasks[0].dtype : FDBB_F64);
        block = bc.block, ppt = bc.ppt, nontemporal = bc.nt, grid_per_cu = bc.grid_per_cu, grid = 0;
    }
    if (!batch_config_ok(block, ppt, nontemporal) || grid < 0)
        return fail(FDBB_EINVAL, "invalid launch configuration (batches take 64..256 threads per workgroup in "
                                 "multiples of 64, 1, 2, 4 or 8 points per thread, store mode 0, 1 or 2)");
    DeviceInfo dev;
    int rc = device_info(&dev);
    if (rc) return rc;
    // Host staging of the table and the range list of the overlap check:
    // static, so this call uses no heap; the lock makes concurrent callers
    // take turns over them.
    static std::mutex staging_mutex;
    alignas(64) static unsigned char staging[kNoAllocBytes];
    static Range ranges[8 * (size_t)kNoAllocMaxTasks];
    std::lock_guard<std::mutex> lock(staging_mutex);
    TableInfo info;
    rc = fill_table(tasks, ntasks, kNoAllocMaxTasks, block, ppt, staging, ranges, &info);
    if (rc) return rc;
    if (info.tiles == 0) return FDBB_OK;
    void *table = nullptr;
    const int se = batch_scratch(&table);
    if (se) return fail_hip((hipError_t)se, "hipGetSymbolAddress of the batch task table");
    const void *kernel = kernel_batch(ppt, nontemporal);
    if (!kernel) return fail(FDBB_EINVAL, "no batch kernel for this configuration");
    if ((rc = set_lds_attr(kernel, info.lds, dev))) return rc;
    // From pageable host memory the copy completes before the call returns,
    // so the staging array is free again once it does; it is ordered on
    // `stream` before the launch that reads the table.
    const size_t used = table_task_offset(kNoAllocMaxTasks) + (size_t)ntasks * sizeof(TaskDev);
    hipError_t e = hipMemcpyAsync(table, staging, used, hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync");
    unsigned char *base = static_cast<unsigned char *>(table);
    const TaskDev *dtasks = table_tasks(base, kNoAllocMaxTasks);
    const int64_t *prefix = table_prefix(base);
    const int64_t *header = table_header(base);
    void *args[] = {&dtasks, &prefix, &header};
    const int g = grid > 0 ? grid : dev.cus * (grid_per_cu > 0 ? grid_per_cu : std::max(1, 2048 / block));
    e = hipLaunchKernel(kernel, dim3((unsigned)g), dim3((unsigned)block), args, info.lds, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "batch kernel launch");
    return FDBB_OK;
}

}  // extern "C"
