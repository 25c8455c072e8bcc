// Tile code: one workgroup evaluates one tile of blockDim.x * P consecutive
// points; each wave takes 64 * P of them and each thread P (see Lane), laid
// out so that every SoA field is read and written as whole contiguous runs
// (16-byte vector accesses per lane when the call's pointers allow it).  The
// flux Jacobian blocks, which are stored point-major (K*K contiguous values
// per point), are staged through a per-wave LDS region and written out as
// contiguous runs of 16-byte stores.
#pragma once

#include "euler_point.hpp"

namespace fdbb {

constexpr int kWave = 64;

enum : int32_t {
    kFlagInPlace = 1,  // K -> K transform with output == input: skip the rho store
    kFlagVector = 2,   // every base pointer and row stride allows 16-byte access
    kFlagRight = 4,    // characteristic product with R (else with L)
    kFlagOneDir = 8,   // flux of direction Args::dir only, as K fields
};

// One operation on one field-set group (the device image of fdbb_task).
struct Args {
    const void *in0;
    int64_t ld_in0;
    const void *in1;
    int64_t ld_in1;
    const void *in2;
    int64_t ld_in2;
    void *out0;
    int64_t ld_out0;
    void *out1;
    int64_t ld_out1;
    void *out2;
    int64_t ld_out2;
    int64_t n;
    int32_t dir;
    int32_t flags;
    Gas gas;
};

template <typename T, int N>
using vec_t = T __attribute__((ext_vector_type(N)));

// Points per chunk and chunks per thread.  A chunk is the unit of one
// vector access and of the FP64 per-point state held in registers at one
// time: up to 16 bytes, two FP64 or four FP32 values, when the thread has
// that many points (two points, 8 bytes, for FP32 at two points per
// thread).
template <typename T, int P>
struct Chunk {
    static constexpr int VW = 16 / (int)sizeof(T);
    static constexpr int W = P >= VW ? VW : (P >= 2 ? 2 : 1);
    static constexpr int N = P / W;
};

// One load, regular or non-temporal (NTL: the nt bit, no normal cache
// allocation).  The kernels that read two input field sets (adjoint, Roe
// average, products with L or R) load with nt: timed alternately in one
// process on the same buffers, that made them 5-8 % faster in 3D FP64,
// while the single-input kernels (flux, fused pass) were 2-3 % slower.
template <bool NTL, typename V>
__device__ __forceinline__ V get(const V *p)
{
    if constexpr (NTL) return __builtin_nontemporal_load(p);
    else return *p;
}

// Load the W consecutive values at p (cnt of them valid) widened to FP64.
template <typename T, int W, bool NTL = false>
__device__ __forceinline__ void load_chunk(const T *__restrict__ p, int cnt, bool vec, double *x)
{
    if (vec && cnt == W) {
        if constexpr (W == 1) {
            x[0] = (double)get<NTL, T>(p);
        } else {
            const vec_t<T, W> v = get<NTL, vec_t<T, W>>(reinterpret_cast<const vec_t<T, W> *>(p));
#pragma unroll
            for (int j = 0; j < W; ++j) x[j] = (double)v[j];
        }
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j) x[j] = (j < cnt) ? (double)get<NTL, T>(p + j) : 1.0;
    }
}

// Output store modes, a template parameter of every kernel:
//   kStoreRegular: plain stores, allocated in the caches as usual;
//   kStoreNT:      non-temporal stores (the nt bit: streamed past the
//                  caches' normal allocation);
//   kStoreNTSc1:   nt plus sc1 (the device-scope coherence bit).
// The launch configuration chooses between regular and streaming stores;
// each kernel family's picker fixes which streaming flavour it uses, from
// timings of both taken alternately in one process on the same buffers.
// The single-launch kernels that write K x K blocks (fused pass, flux
// Jacobian, eigenvector blocks) stream with nt + sc1, under which they ran
// 1.8-3.5 % faster on this device than with nt alone (a plain write
// stream: 7.0 against 6.7-6.8 TB/s).  The persistent batch kernel takes any
// of the three modes; its autotuned configuration picks one.
enum : int { kStoreRegular = 0, kStoreNT = 1, kStoreNTSc1 = 2 };

// No compiler builtin sets sc1 on a global store, hence the inline
// assembly (vector stores only).  The compiler does not count these stores
// in its vector-memory wait counter, which can only make its waits
// stricter: that counter completes in issue order, so an extra store issued
// after a load never lets a wait for the load pass early.  The statements
// declare no memory clobber, so the compiler keeps scheduling loads and
// arithmetic across them; that is safe because no kernel reads back what it
// stores except an in-place transform, where each address is read and
// written by one thread and the stored value depends on the loaded one.
// A store of more than 64 bits reads its data registers during the two
// wait states after it issues, and a VALU instruction that overwrites
// them inside that window corrupts the stored value.  The compiler pads
// its own wide stores for this, but it cannot see the store inside an asm
// statement and reuses the registers as soon as the statement ends, so
// the 16-byte form carries its own s_nop 1 (two wait states).
template <int NT, typename V>
__device__ __forceinline__ void put(V *p, V v)
{
    if constexpr (NT == kStoreNTSc1) {
        static_assert(sizeof(V) == 4 || sizeof(V) == 8 || sizeof(V) == 16, "4-, 8- or 16-byte stores");
        if constexpr (sizeof(V) == 16)
            asm volatile("global_store_dwordx4 %0, %1, off nt sc1\n\ts_nop 1" : : "v"(p), "v"(v));
        else if constexpr (sizeof(V) == 8)
            asm volatile("global_store_dwordx2 %0, %1, off nt sc1" : : "v"(p), "v"(v));
        else
            asm volatile("global_store_dword %0, %1, off nt sc1" : : "v"(p), "v"(v));
    } else if constexpr (NT == kStoreNT) {
        __builtin_nontemporal_store(v, p);
    } else {
        *p = v;
    }
}

// Store W consecutive FP64 values at p, rounded to T (cnt of them valid).
template <typename T, int W, int NT>
__device__ __forceinline__ void store_chunk(T *__restrict__ p, int cnt, bool vec, const double *x)
{
    if (vec && cnt == W) {
        if constexpr (W == 1) {
            put<NT, T>(p, (T)x[0]);
        } else {
            vec_t<T, W> v;
#pragma unroll
            for (int j = 0; j < W; ++j) v[j] = (T)x[j];
            put<NT, vec_t<T, W>>(reinterpret_cast<vec_t<T, W> *>(p), v);
        }
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j)
            if (j < cnt) put<NT, T>(p + j, (T)x[j]);
    }
}

// Per-thread view of one tile.  Wave w of the workgroup covers the 64 * P
// consecutive points starting at tile0 + w * 64 * P.  A thread owns P of
// them as P / W chunks of W consecutive points (W * sizeof(T) <= 16 bytes);
// chunk c of lane l starts at wave point c * 64 * W + l * W, so every load
// or store instruction of a wave covers one contiguous run of 64 * W
// points (whole cache lines), whatever P is.
template <typename T, int P, int NT>
struct Lane {
    static constexpr int W = Chunk<T, P>::W;
    static constexpr int NC = Chunk<T, P>::N;
    static constexpr int CS = kWave * W;  // points between a thread's chunks

    int64_t i;     // first point of this thread's first chunk
    int64_t left;  // points from i to the end of the range
    int lane;
    bool vec;

    __device__ __forceinline__ Lane(const Args &a, int64_t tile0)
    {
        lane = threadIdx.x & (kWave - 1);
        const int wave = threadIdx.x / kWave;
        i = tile0 + (int64_t)wave * kWave * P + (int64_t)lane * W;
        left = a.n - i;
        vec = (a.flags & kFlagVector) != 0;
    }

    __device__ __forceinline__ bool any() const { return left > 0; }

    // Valid points of chunk c.
    __device__ __forceinline__ int count(int c) const
    {
        const int64_t l = left - (int64_t)c * CS;
        return l <= 0 ? 0 : (l >= W ? W : (int)l);
    }

    // Position, inside the wave's 64 * P points, of the thread's point j.
    __device__ __forceinline__ int local(int j) const { return (j / W) * CS + lane * W + (j % W); }

    // Chunk c (W values) of field `field` of a field set with row stride ld
    // (NTL: non-temporal loads).
    template <bool NTL = false>
    __device__ __forceinline__ void load(const void *base, int64_t ld, int field, int c, double *x) const
    {
        const T *b = static_cast<const T *>(base) + i + (int64_t)field * ld + c * CS;
        load_chunk<T, W, NTL>(b, count(c), vec, x);
    }

    // Chunk c of `FIELDS` consecutive fields into x[field][W].
    template <int FIELDS, bool NTL = false>
    __device__ __forceinline__ void load_fields(const void *base, int64_t ld, int c,
                                                double (&x)[FIELDS][W]) const
    {
#pragma unroll
        for (int k = 0; k < FIELDS; ++k) load<NTL>(base, ld, k, c, x[k]);
    }

    __device__ __forceinline__ void store(void *base, int64_t ld, int field, int c, const double *x) const
    {
        T *b = static_cast<T *>(base) + i + (int64_t)field * ld + c * CS;
        store_chunk<T, W, NT>(b, count(c), vec, x);
    }
};


// ------------------------------------------------------------ pointwise ops
//
// Every op loads all of a thread's chunks first (so that the loads are in
// flight together) and then evaluates and stores chunk by chunk, holding the
// FP64 state of at most W points at a time.

template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_cons2prim(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
    double u[NC][K][W];
#pragma unroll
    for (int c = 0; c < NC; ++c) L.template load_fields<K>(a.in0, a.ld_in0, c, u[c]);
    const int first = (a.flags & kFlagInPlace) ? 1 : 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double out[K][W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double uj[K], vj[K];
#pragma unroll
            for (int k = 0; k < K; ++k) uj[k] = u[c][k][j];
            to_primitive<D>(make_state<D>(a.gas, uj), vj);
#pragma unroll
            for (int k = 0; k < K; ++k) out[k][j] = vj[k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k >= first) L.store(a.out0, a.ld_out0, k, c, out[k]);
    }
}

template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_prim2cons(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
    double w[NC][K][W];
#pragma unroll
    for (int c = 0; c < NC; ++c) L.template load_fields<K>(a.in0, a.ld_in0, c, w[c]);
    const int first = (a.flags & kFlagInPlace) ? 1 : 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double out[K][W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double vj[K], uj[K];
#pragma unroll
            for (int k = 0; k < K; ++k) vj[k] = w[c][k][j];
            from_primitive<D>(a.gas, vj, uj);
#pragma unroll
            for (int k = 0; k < K; ++k) out[k][j] = uj[k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (k >= first) L.store(a.out0, a.ld_out0, k, c, out[k]);
    }
}

// Roe-averaged state between the states in in0 (left) and in1 (right).
// Per chunk, the left states are folded into weighted sums before the right
// states are loaded, so that one side's raw state is live at a time.
template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_roe(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double sum[W][D + 1], wl[W], wr[W];
#pragma unroll
        for (int j = 0; j < W; ++j)
#pragma unroll
            for (int k = 0; k <= D; ++k) sum[j][k] = 0.0;
        {
            double u[K][W];
            L.template load_fields<K, true>(a.in0, a.ld_in0, c, u);
#pragma unroll
            for (int j = 0; j < W; ++j) {
                double uj[K];
#pragma unroll
                for (int k = 0; k < K; ++k) uj[k] = u[k][j];
                wl[j] = roe_accumulate<D>(a.gas, uj, sum[j]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        {
            double u[K][W];
            L.template load_fields<K, true>(a.in1, a.ld_in1, c, u);
#pragma unroll
            for (int j = 0; j < W; ++j) {
                double uj[K];
#pragma unroll
                for (int k = 0; k < K; ++k) uj[k] = u[k][j];
                wr[j] = roe_accumulate<D>(a.gas, uj, sum[j]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        double out[K][W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double hj[K];
            roe_finish<D>(a.gas, sum[j], wl[j], wr[j], hj);
#pragma unroll
            for (int k = 0; k < K; ++k) out[k][j] = hj[k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) L.store(a.out0, a.ld_out0, k, c, out[k]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_vmag2(const Args &a, int64_t tile0)
{
    constexpr int R = D + 1;  // rho and the momenta; E is not read
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
    double u[NC][R][W];
#pragma unroll
    for (int c = 0; c < NC; ++c) L.template load_fields<R>(a.in0, a.ld_in0, c, u[c]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double y[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double uj[R];
#pragma unroll
            for (int k = 0; k < R; ++k) uj[k] = u[c][k][j];
            y[j] = velocity_magnitude2<D>(uj);
        }
        L.store(a.out0, 0, 0, c, y);
    }
}

template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_eos(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
    double u[NC][K][W];
#pragma unroll
    for (int c = 0; c < NC; ++c) L.template load_fields<K>(a.in0, a.ld_in0, c, u[c]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double p[W], cs[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double uj[K];
#pragma unroll
            for (int k = 0; k < K; ++k) uj[k] = u[c][k][j];
            const State<D> s = make_state<D>(a.gas, uj);
            p[j] = s.p;
            cs[j] = sound_speed<D>(a.gas, s);
        }
        if (a.out0) L.store(a.out0, 0, 0, c, p);
        if (a.out1) L.store(a.out1, 0, 0, c, cs);
    }
}

// General EOS entry: pressure, speed of sound and temperature of the
// stiffened gas p = (gamma-1) rho e - gamma p_inf, T = (e - p_inf/rho)/c_v,
// c^2 = gamma (p + p_inf)/rho, which is the perfect gas when p_inf = 0.
// Outputs out0 (p), out1 (c), out2 (T), each optional.
template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_eos_pvt(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
    double u[NC][K][W];
#pragma unroll
    for (int c = 0; c < NC; ++c) L.template load_fields<K>(a.in0, a.ld_in0, c, u[c]);
    const Gas &g = a.gas;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double p[W], cs[W], t[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double uj[K];
#pragma unroll
            for (int k = 0; k < K; ++k) uj[k] = u[c][k][j];
            const State<D> s = make_state<D>(g, uj);
            // s.p is (gamma-1) rho e; e = E/rho - |v|^2/2
            const double e = s.E * s.rinv - 0.5 * s.q;
            p[j] = s.p - g.gamma * g.p_inf;
            cs[j] = sqrt(g.gamma * (p[j] + g.p_inf) * s.rinv);
            t[j] = (e - g.p_inf * s.rinv) * g.inv_cv;
        }
        if (a.out0) L.store(a.out0, 0, 0, c, p);
        if (a.out1) L.store(a.out1, 0, 0, c, cs);
        if (a.out2) L.store(a.out2, 0, 0, c, t);
    }
}

// Viscous flux tensor from the state (in0, K fields), the velocity gradient
// (in1, D*D fields, field i*D + j = dv_i/dx_j) and the temperature gradient
// (in2, D fields), in the flux tensor's layout (out0, field r*D + d):
// F^v_d = (0, tau_1d .. tau_Dd, sum_j v_j tau_jd + kappa dT/dx_d) with
// tau_ij = mu (dv_i/dx_j + dv_j/dx_i) - (2/3) mu delta_ij div v.  Loads go
// chunk by chunk (K + D*D + D input fields per point) and each stress
// entry is stored as soon as it is formed.
template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_viscous(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
    const double mu = a.gas.mu, kappa = a.gas.kappa;
    const double zero[W] = {};
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double gv[D * D][W], v[D][W], bulk[W];
        {
            double u[K][W];
            L.template load_fields<K>(a.in0, a.ld_in0, c, u);
            L.template load_fields<D * D>(a.in1, a.ld_in1, c, gv);
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const double rinv = 1.0 / u[0][j];
                double div = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    v[i][j] = u[1 + i][j] * rinv;
                    div += gv[i * D + i][j];
                }
                bulk[j] = (2.0 / 3.0) * mu * div;
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            L.store(a.out0, a.ld_out0, d, c, zero);
            double e[W];
            L.load(a.in2, a.ld_in2, d, c, e);
#pragma unroll
            for (int j = 0; j < W; ++j) e[j] *= kappa;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double t[W];
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    t[j] = mu * (gv[i * D + d][j] + gv[d * D + i][j]) - (i == d ? bulk[j] : 0.0);
                    e[j] += v[i][j] * t[j];
                }
                L.store(a.out0, a.ld_out0, (1 + i) * D + d, c, t);
            }
            L.store(a.out0, a.ld_out0, (D + 1) * D + d, c, e);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The K*D flux fields of W points.
template <int D, typename T, int P, int NT>
__device__ __forceinline__ void store_flux(const Lane<T, P, NT> &L, const State<D> *s, int c, void *F,
                                           int64_t ldF)
{
    constexpr int W = Lane<T, P, NT>::W;
#pragma unroll
    for (int r = 0; r < D + 2; ++r) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            double f[W];
#pragma unroll
            for (int j = 0; j < W; ++j) f[j] = flux_entry<D>(s[j], r, d);
            L.store(F, ldF, r * D + d, c, f);
        }
    }
}

// The K components of F_dir alone (field r = component r), of W points.
// dir is uniform over the launch, so the test below does not diverge.
template <int D, typename T, int P, int NT>
__device__ __forceinline__ void store_flux_dir(const Lane<T, P, NT> &L, const State<D> *s, int c, int dir,
                                               void *F, int64_t ldF)
{
    constexpr int W = Lane<T, P, NT>::W;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (d != dir) continue;
#pragma unroll
        for (int r = 0; r < D + 2; ++r) {
            double f[W];
#pragma unroll
            for (int j = 0; j < W; ++j) f[j] = flux_entry<D>(s[j], r, d);
            L.store(F, ldF, r, c, f);
        }
    }
}

// Riemann invariants of every direction and the entropy, of W points.
template <int D, typename T, int P, int NT>
__device__ __forceinline__ void store_riemann(const Args &a, const Lane<T, P, NT> &L, const State<D> *s, int c,
                                              void *R, int64_t ldR)
{
    constexpr int W = Lane<T, P, NT>::W;
    double t[W];
#pragma unroll
    for (int j = 0; j < W; ++j) t[j] = a.gas.two_inv_g1 * sound_speed<D>(a.gas, s[j]);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double wm[W], wp[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            wm[j] = s[j].v[d] - t[j];
            wp[j] = s[j].v[d] + t[j];
        }
        L.store(R, ldR, 2 * d, c, wm);
        L.store(R, ldR, 2 * d + 1, c, wp);
    }
    double en[W];
#pragma unroll
    for (int j = 0; j < W; ++j) en[j] = entropy<D, sizeof(T) == 4>(a.gas, s[j]);
    L.store(R, ldR, 2 * D, c, en);
}

template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_flux(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
    double u[NC][K][W];
#pragma unroll
    for (int c = 0; c < NC; ++c) L.template load_fields<K>(a.in0, a.ld_in0, c, u[c]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        State<D> s[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double uj[K];
#pragma unroll
            for (int k = 0; k < K; ++k) uj[k] = u[c][k][j];
            s[j] = make_state<D>(a.gas, uj);
        }
        if (a.flags & kFlagOneDir) store_flux_dir<D, T, P, NT>(L, s, c, a.dir, a.out0, a.ld_out0);
        else store_flux<D, T, P, NT>(L, s, c, a.out0, a.ld_out0);
    }
}

template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_riemann(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
    double u[NC][K][W];
#pragma unroll
    for (int c = 0; c < NC; ++c) L.template load_fields<K>(a.in0, a.ld_in0, c, u[c]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        State<D> s[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double uj[K];
#pragma unroll
            for (int k = 0; k < K; ++k) uj[k] = u[c][k][j];
            s[j] = make_state<D>(a.gas, uj);
        }
        store_riemann<D, T, P, NT>(a, L, s, c, a.out0, a.ld_out0);
    }
}

// W = (w-_dir, s, tangential v ascending, w+_dir).
template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_cons2char(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
    double u[NC][K][W];
#pragma unroll
    for (int c = 0; c < NC; ++c) L.template load_fields<K>(a.in0, a.ld_in0, c, u[c]);
    const int dir = a.dir;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double out[K][W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double uj[K];
#pragma unroll
            for (int k = 0; k < K; ++k) uj[k] = u[c][k][j];
            const State<D> s = make_state<D>(a.gas, uj);
            const double t = a.gas.two_inv_g1 * sound_speed<D>(a.gas, s);
            double vd = s.v[0];
#pragma unroll
            for (int k = 1; k < D; ++k)
                if (k == dir) vd = s.v[k];
            out[0][j] = vd - t;
            out[1][j] = entropy<D, sizeof(T) == 4>(a.gas, s);
            out[K - 1][j] = vd + t;
            // tangential components: slot 2 + (k < dir ? k : k - 1) for k != dir
#pragma unroll
            for (int slot = 0; slot < D - 1; ++slot) {
                double vt = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k)
                    if (k != dir && (k < dir ? k : k - 1) == slot) vt = s.v[k];
                out[2 + slot][j] = vt;
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) L.store(a.out0, a.ld_out0, k, c, out[k]);
    }
}

template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_char2cons(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
    double w[NC][K][W];
#pragma unroll
    for (int c = 0; c < NC; ++c) L.template load_fields<K>(a.in0, a.ld_in0, c, w[c]);
    const int dir = a.dir;
    const Gas &g = a.gas;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double out[K][W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const double wm = w[c][0][j], s = w[c][1][j], wp = w[c][K - 1][j];
            const double cs = g.quarter_g1 * (wp - wm);
            const double c2 = cs * cs;
            // rho = (c^2 / (gamma s))^(1/(gamma-1)),  p = rho c^2 / gamma
            const double rho = pos_pow_t<sizeof(T) == 4>(c2 * g.inv_gamma / s, g.inv_g1);
            const double p = rho * c2 * g.inv_gamma;
            double vp[K];
            vp[0] = rho;
            vp[K - 1] = p;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                // v_dir from the invariants; tangential k from slot 2 +
                // (k < dir ? k : k - 1), picked with fixed indices (a
                // runtime index would put w in scratch memory)
                double vk = 0.5 * (wp + wm);
#pragma unroll
                for (int slot = 0; slot < D - 1; ++slot)
                    if (k != dir && (k < dir ? k : k - 1) == slot) vk = w[c][2 + slot][j];
                vp[1 + k] = vk;
            }
            double uj[K];
            from_primitive<D>(g, vp, uj);
#pragma unroll
            for (int k = 0; k < K; ++k) out[k][j] = uj[k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) L.store(a.out0, a.ld_out0, k, c, out[k]);
    }
}

// Ubar = sum_d A_d^T Fbar_d (dir < 0) or A_dir^T Fbar (dir >= 0), chunk by
// chunk: the state, the cotangents and the accumulators of W points.
template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_adjoint(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
    double u[NC][K][W];
#pragma unroll
    for (int c = 0; c < NC; ++c) L.template load_fields<K, true>(a.in0, a.ld_in0, c, u[c]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        State<D> s[W];
        double phi[W], H[W], ub[K][W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double uj[K];
#pragma unroll
            for (int k = 0; k < K; ++k) uj[k] = u[c][k][j];
            s[j] = make_state<D>(a.gas, uj);
            phi[j] = a.gas.half_g1 * s[j].q;
            H[j] = (s[j].E + s[j].p) * s[j].rinv;
#pragma unroll
            for (int k = 0; k < K; ++k) ub[k][j] = 0.0;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (a.dir >= 0 && d != a.dir) continue;
            double f[K][W];
#pragma unroll
            for (int r = 0; r < K; ++r) L.template load<true>(a.in1, a.ld_in1, a.dir < 0 ? r * D + d : r, c, f[r]);
#pragma unroll
            for (int j = 0; j < W; ++j) {
                double fj[K], uj[K];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    fj[k] = f[k][j];
                    uj[k] = ub[k][j];
                }
                adjoint_accumulate<D>(a.gas, s[j], phi[j], H[j], d, fj, uj);
#pragma unroll
                for (int k = 0; k < K; ++k) ub[k][j] = uj[k];
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) L.store(a.out0, a.ld_out0, k, c, ub[k]);
    }
}

// ------------------------------------------------------------ Jacobian blocks

// Copy the wave's staged blocks (count elements of T, contiguous in LDS and
// in global memory) with lane-contiguous 16-byte stores when allowed.
template <typename T, int NT>
__device__ __forceinline__ void wave_copy_out(const T *lds, T *dst, int count, bool vec, int lane)
{
    if (vec) {
        constexpr int W = 16 / (int)sizeof(T);
        const int chunks = count / W;
        const vec_t<T, W> *src = reinterpret_cast<const vec_t<T, W> *>(lds);
        vec_t<T, W> *out = reinterpret_cast<vec_t<T, W> *>(dst);
        for (int c = lane; c < chunks; c += kWave) put<NT, vec_t<T, W>>(out + c, src[c]);
        for (int e = chunks * W + lane; e < count; e += kWave) put<NT, T>(dst + e, lds[e]);
    } else {
        for (int e = lane; e < count; e += kWave) put<NT, T>(dst + e, lds[e]);
    }
}

// Stage this wave's 64 * P blocks of one K x K matrix per point in LDS
// (entry(q, r, c) gives entry (r, c) of the thread's point q), then copy them
// to `dst`, the global address of the wave's first block, as one contiguous
// run.  Every thread of the workgroup must call this (it holds barriers).
template <int D, typename T, int P, int NT, class Entry>
__device__ __forceinline__ void stage_blocks(const Lane<T, P, NT> &L, T *region, T *dst, int wave_pts,
                                             Entry entry)
{
    constexpr int K = D + 2;
    constexpr int KK = K * K;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        T *blk = region + L.local(q) * KK;
#pragma unroll
        for (int r = 0; r < K; ++r)
#pragma unroll
            for (int c = 0; c < K; ++c) blk[r * K + c] = (T)entry(q, r, c);
        // one block at a time: keeps the scheduler from holding the entries
        // of several blocks in registers at once
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    if (wave_pts > 0) wave_copy_out<T, NT>(region, dst, wave_pts * KK, L.vec, L.lane);
    __syncthreads();
}

// Points of the range in this wave's part of the tile.
template <int P>
__device__ __forceinline__ int wave_points(int64_t n, int64_t wave0)
{
    const int64_t left = n - wave0;
    return left <= 0 ? 0 : (left >= kWave * P ? kWave * P : (int)left);
}

// The fused pass: flux tensor (out0, may be NULL), Jacobian blocks (out1,
// may be NULL) and Riemann invariants (out2, may be NULL) of the same state.
// Flux and invariants are stored chunk by chunk from the full state; the
// Jacobian keeps only v, H and phi of each point, and its blocks go through
// `lds`, this workgroup's staging area of blockDim.x * P * K * K values
// (each wave uses its own 64 * P blocks).  Every thread of the workgroup
// must call this (it holds barriers).
template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_fused(const Args &a, int64_t tile0, T *lds)
{
    constexpr int K = D + 2;
    constexpr int KK = K * K;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    const int wave = threadIdx.x / kWave;
    const int64_t wave0 = tile0 + (int64_t)wave * kWave * P;

    double u[NC][K][W];
#pragma unroll
    for (int c = 0; c < NC; ++c) L.template load_fields<K>(a.in0, a.ld_in0, c, u[c]);

    double jv[P][D], jH[P], jphi[P];  // what the Jacobian blocks need
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        State<D> s[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double uj[K];
#pragma unroll
            for (int k = 0; k < K; ++k) uj[k] = u[c][k][j];
            s[j] = make_state<D>(a.gas, uj);
            const int q = c * W + j;
#pragma unroll
            for (int k = 0; k < D; ++k) jv[q][k] = s[j].v[k];
            jH[q] = (s[j].E + s[j].p) * s[j].rinv;
            jphi[q] = a.gas.half_g1 * s[j].q;
        }
        if (L.any()) {
            if (a.out0) store_flux<D, T, P, NT>(L, s, c, a.out0, a.ld_out0);
            if (a.out2) store_riemann<D, T, P, NT>(a, L, s, c, a.out2, a.ld_out2);
        }
        __builtin_amdgcn_sched_barrier(0);  // one chunk's state at a time
    }

    if (a.out1) {
        T *region = lds + (size_t)wave * kWave * P * KK;
        const int wave_pts = wave_points<P>(a.n, wave0);
        T *A = static_cast<T *>(a.out1);
#pragma unroll
        for (int d = 0; d < D; ++d)
            stage_blocks<D, T, P, NT>(L, region, A + (d * a.ld_out1 + wave0) * KK, wave_pts,
                                      [&](int q, int r, int c) {
                                          return jacobian_entry<D>(a.gas, jv[q], jphi[q], jH[q], d, r, c);
                                      });
    }
}

// Characteristic decomposition of every direction: left eigenvector blocks
// L_d (out0, may be NULL) and right eigenvector blocks R_d (out1, may be
// NULL), point-major K x K blocks like the Jacobian, staged through LDS.
template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_eigen(const Args &a, int64_t tile0, T *lds)
{
    constexpr int K = D + 2;
    constexpr int KK = K * K;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    const int wave = threadIdx.x / kWave;
    const int64_t wave0 = tile0 + (int64_t)wave * kWave * P;

    double u[NC][K][W];
#pragma unroll
    for (int c = 0; c < NC; ++c) L.template load_fields<K>(a.in0, a.ld_in0, c, u[c]);
    double v[P][D];
    Waves w[P];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double uj[K];
#pragma unroll
            for (int k = 0; k < K; ++k) uj[k] = u[c][k][j];
            const State<D> s = make_state<D>(a.gas, uj);
            const int q = c * W + j;
#pragma unroll
            for (int k = 0; k < D; ++k) v[q][k] = s.v[k];
            w[q] = make_waves<D>(a.gas, s);
        }
    }
    T *region = lds + (size_t)wave * kWave * P * KK;
    const int wave_pts = wave_points<P>(a.n, wave0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (a.out0)
            stage_blocks<D, T, P, NT>(L, region, static_cast<T *>(a.out0) + (d * a.ld_out0 + wave0) * KK,
                                      wave_pts,
                                      [&](int q, int r, int c) { return left_entry<D>(v[q], w[q], d, r, c); });
        if (a.out1)
            stage_blocks<D, T, P, NT>(L, region, static_cast<T *>(a.out1) + (d * a.ld_out1 + wave0) * KK,
                                      wave_pts,
                                      [&](int q, int r, int c) { return right_entry<D>(v[q], w[q], d, r, c); });
    }
}

// Y = L_dir(U) X, or R_dir(U) X with kFlagRight: in0 = U, in1 = X, out0 = Y.
template <int D, typename T, int P, int NT>
__device__ __forceinline__ void tile_char_apply(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    using L_t = Lane<T, P, NT>;
    constexpr int W = L_t::W, NC = L_t::NC;
    const L_t L(a, tile0);
    if (!L.any()) return;
    const bool right = (a.flags & kFlagRight) != 0;
    const int dir = a.dir;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double u[K][W], x[K][W], y[K][W];
        L.template load_fields<K, true>(a.in0, a.ld_in0, c, u);
        L.template load_fields<K, true>(a.in1, a.ld_in1, c, x);
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double uj[K];
#pragma unroll
            for (int k = 0; k < K; ++k) uj[k] = u[k][j];
            const State<D> s = make_state<D>(a.gas, uj);
            const Waves wv = make_waves<D>(a.gas, s);
#pragma unroll
            for (int r = 0; r < K; ++r) {
                double acc = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    if (d != dir) continue;
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        acc += (right ? right_entry<D>(s.v, wv, d, r, k) : left_entry<D>(s.v, wv, d, r, k)) *
                               x[k][j];
                }
                y[r][j] = acc;
            }
        }
#pragma unroll
        for (int r = 0; r < K; ++r) L.store(a.out0, a.ld_out0, r, c, y[r]);
    }
}

}  // namespace fdbb
