// Tile code: one workgroup evaluates one tile of blockDim.x * P consecutive
// points.  Thread t of the workgroup owns the P consecutive points starting
// at tile0 + t * P, so every SoA field is read and written as one contiguous
// run of blockDim.x * P elements (16-byte vector accesses per lane when the
// call's pointers allow it).  The flux Jacobian blocks, which are stored
// point-major (K*K contiguous values per point), are staged through a
// per-wave LDS region and written out as contiguous runs of 16-byte stores.
#pragma once

#include "euler_point.hpp"

namespace fdbb {

constexpr int kWave = 64;

enum : int32_t {
    kFlagInPlace = 1,  // K -> K transform with output == input: skip the rho store
    kFlagVector = 2,   // every base pointer and row stride allows 16-byte access
};

// One operation on one field-set group (the device image of fdbb_task).
struct Args {
    const void *in0;
    int64_t ld_in0;
    const void *in1;
    int64_t ld_in1;
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

// Elements of T per 16-byte chunk, capped at P.
template <typename T, int P>
struct Chunk {
    static constexpr int W = (P * (int)sizeof(T) > 16) ? 16 / (int)sizeof(T) : P;
    static constexpr int N = P / W;
};

// Load the P consecutive values at p (cnt of them valid) widened to FP64.
template <typename T, int P>
__device__ __forceinline__ void load_run(const T *__restrict__ p, int cnt, bool vec, double *x)
{
    if (vec && cnt == P) {
        using C = Chunk<T, P>;
#pragma unroll
        for (int c = 0; c < C::N; ++c) {
            if constexpr (C::W == 1) {
                x[c] = (double)p[c];
            } else {
                const vec_t<T, C::W> v = *reinterpret_cast<const vec_t<T, C::W> *>(p + c * C::W);
#pragma unroll
                for (int j = 0; j < C::W; ++j) x[c * C::W + j] = (double)v[j];
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j) x[j] = (j < cnt) ? (double)p[j] : 1.0;
    }
}

// Output stores: non-temporal (NT, streamed past the caches' normal
// allocation policy) or regular; which one the HBM write path prefers is a
// launch-configuration choice.
template <bool NT, typename V>
__device__ __forceinline__ void put(V *p, V v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Store P consecutive FP64 values at p, rounded to T (cnt of them valid).
template <typename T, int P, bool NT>
__device__ __forceinline__ void store_run(T *__restrict__ p, int cnt, bool vec, const double *x)
{
    if (vec && cnt == P) {
        using C = Chunk<T, P>;
#pragma unroll
        for (int c = 0; c < C::N; ++c) {
            if constexpr (C::W == 1) {
                put<NT, T>(p + c, (T)x[c]);
            } else {
                vec_t<T, C::W> v;
#pragma unroll
                for (int j = 0; j < C::W; ++j) v[j] = (T)x[c * C::W + j];
                put<NT, vec_t<T, C::W>>(reinterpret_cast<vec_t<T, C::W> *>(p + c * C::W), v);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (j < cnt) put<NT, T>(p + j, (T)x[j]);
    }
}

// Per-thread view of one tile.
template <typename T, int P, bool NT>
struct Lane {
    int64_t i;  // first point of this thread
    int cnt;    // valid points of this thread, 0..P
    bool vec;

    __device__ __forceinline__ Lane(const Args &a, int64_t tile0)
    {
        i = tile0 + (int64_t)threadIdx.x * P;
        const int64_t left = a.n - i;
        cnt = left <= 0 ? 0 : (left >= P ? P : (int)left);
        vec = (a.flags & kFlagVector) != 0;
    }

    // Load `fields` consecutive fields of a field set into x[field][P].
    template <int FIELDS>
    __device__ __forceinline__ void load(const void *base, int64_t ld, double (&x)[FIELDS][P]) const
    {
        const T *b = static_cast<const T *>(base) + i;
#pragma unroll
        for (int k = 0; k < FIELDS; ++k) load_run<T, P>(b + k * ld, cnt, vec, x[k]);
    }

    __device__ __forceinline__ void store(void *base, int64_t ld, int field, const double *x) const
    {
        T *b = static_cast<T *>(base) + i + field * ld;
        store_run<T, P, NT>(b, cnt, vec, x);
    }
};

// ------------------------------------------------------------ pointwise ops

template <int D, typename T, int P, bool NT>
__device__ __forceinline__ void tile_cons2prim(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    Lane<T, P, NT> L(a, tile0);
    if (L.cnt == 0) return;
    double u[K][P];
    L.template load<K>(a.in0, a.ld_in0, u);
    double out[K][P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double uj[K], vj[K];
#pragma unroll
        for (int k = 0; k < K; ++k) uj[k] = u[k][j];
        const State<D> s = make_state<D>(a.gas, uj);
        to_primitive<D>(s, vj);
#pragma unroll
        for (int k = 0; k < K; ++k) out[k][j] = vj[k];
    }
    const int first = (a.flags & kFlagInPlace) ? 1 : 0;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (k >= first) L.store(a.out0, a.ld_out0, k, out[k]);
}

template <int D, typename T, int P, bool NT>
__device__ __forceinline__ void tile_prim2cons(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    Lane<T, P, NT> L(a, tile0);
    if (L.cnt == 0) return;
    double w[K][P];
    L.template load<K>(a.in0, a.ld_in0, w);
    double out[K][P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double vj[K], uj[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vj[k] = w[k][j];
        from_primitive<D>(a.gas, vj, uj);
#pragma unroll
        for (int k = 0; k < K; ++k) out[k][j] = uj[k];
    }
    const int first = (a.flags & kFlagInPlace) ? 1 : 0;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (k >= first) L.store(a.out0, a.ld_out0, k, out[k]);
}

template <int D, typename T, int P, bool NT>
__device__ __forceinline__ void tile_eos(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    Lane<T, P, NT> L(a, tile0);
    if (L.cnt == 0) return;
    double u[K][P];
    L.template load<K>(a.in0, a.ld_in0, u);
    double p[P], c[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double uj[K];
#pragma unroll
        for (int k = 0; k < K; ++k) uj[k] = u[k][j];
        const State<D> s = make_state<D>(a.gas, uj);
        p[j] = s.p;
        c[j] = sound_speed<D>(a.gas, s);
    }
    if (a.out0) L.store(a.out0, 0, 0, p);
    if (a.out1) L.store(a.out1, 0, 0, c);
}

template <int D, typename T, int P, bool NT>
__device__ __forceinline__ void tile_flux(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    Lane<T, P, NT> L(a, tile0);
    if (L.cnt == 0) return;
    double u[K][P];
    L.template load<K>(a.in0, a.ld_in0, u);
    State<D> s[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double uj[K];
#pragma unroll
        for (int k = 0; k < K; ++k) uj[k] = u[k][j];
        s[j] = make_state<D>(a.gas, uj);
    }
#pragma unroll
    for (int r = 0; r < K; ++r) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            double f[P];
#pragma unroll
            for (int j = 0; j < P; ++j) f[j] = flux_entry<D>(s[j], r, d);
            L.store(a.out0, a.ld_out0, r * D + d, f);
        }
    }
}

// Riemann invariants of every direction and the entropy, from a state.
template <int D, typename T, int P, bool NT>
__device__ __forceinline__ void store_riemann(const Args &a, const Lane<T, P, NT> &L, const State<D> (&s)[P],
                                              const double (&c)[P], void *R, int64_t ldR)
{
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double wm[P], wp[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const double t = a.gas.two_inv_g1 * c[j];
            wm[j] = s[j].v[d] - t;
            wp[j] = s[j].v[d] + t;
        }
        L.store(R, ldR, 2 * d, wm);
        L.store(R, ldR, 2 * d + 1, wp);
    }
    double en[P];
#pragma unroll
    for (int j = 0; j < P; ++j) en[j] = entropy<D>(a.gas, s[j]);
    L.store(R, ldR, 2 * D, en);
}

template <int D, typename T, int P, bool NT>
__device__ __forceinline__ void tile_riemann(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    Lane<T, P, NT> L(a, tile0);
    if (L.cnt == 0) return;
    double u[K][P];
    L.template load<K>(a.in0, a.ld_in0, u);
    State<D> s[P];
    double c[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double uj[K];
#pragma unroll
        for (int k = 0; k < K; ++k) uj[k] = u[k][j];
        s[j] = make_state<D>(a.gas, uj);
        c[j] = sound_speed<D>(a.gas, s[j]);
    }
    store_riemann<D, T, P, NT>(a, L, s, c, a.out0, a.ld_out0);
}

// W = (w-_dir, s, tangential v ascending, w+_dir).
template <int D, typename T, int P, bool NT>
__device__ __forceinline__ void tile_cons2char(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    Lane<T, P, NT> L(a, tile0);
    if (L.cnt == 0) return;
    double u[K][P];
    L.template load<K>(a.in0, a.ld_in0, u);
    double out[K][P];
    const int dir = a.dir;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double uj[K];
#pragma unroll
        for (int k = 0; k < K; ++k) uj[k] = u[k][j];
        const State<D> s = make_state<D>(a.gas, uj);
        const double t = a.gas.two_inv_g1 * sound_speed<D>(a.gas, s);
        double vd = s.v[0];
#pragma unroll
        for (int k = 1; k < D; ++k)
            if (k == dir) vd = s.v[k];
        out[0][j] = vd - t;
        out[1][j] = entropy<D>(a.gas, s);
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
    for (int k = 0; k < K; ++k) L.store(a.out0, a.ld_out0, k, out[k]);
}

template <int D, typename T, int P, bool NT>
__device__ __forceinline__ void tile_char2cons(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    Lane<T, P, NT> L(a, tile0);
    if (L.cnt == 0) return;
    double w[K][P];
    L.template load<K>(a.in0, a.ld_in0, w);
    double out[K][P];
    const int dir = a.dir;
    const Gas &g = a.gas;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const double wm = w[0][j], s = w[1][j], wp = w[K - 1][j];
        const double c = g.quarter_g1 * (wp - wm);
        const double c2 = c * c;
        // rho = (c^2 / (gamma s))^(1/(gamma-1)),  p = rho c^2 / gamma
        const double rho = pow(c2 * g.inv_gamma / s, g.inv_g1);
        const double p = rho * c2 * g.inv_gamma;
        double vp[K];
        vp[0] = rho;
        vp[K - 1] = p;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double vk = 0.5 * (wp + wm);
            if (k != dir) vk = w[2 + (k < dir ? k : k - 1)][j];
            vp[1 + k] = vk;
        }
        double uj[K];
        from_primitive<D>(g, vp, uj);
#pragma unroll
        for (int k = 0; k < K; ++k) out[k][j] = uj[k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) L.store(a.out0, a.ld_out0, k, out[k]);
}

// Ubar = sum_d A_d^T Fbar_d (dir < 0) or A_dir^T Fbar (dir >= 0).
template <int D, typename T, int P, bool NT>
__device__ __forceinline__ void tile_adjoint(const Args &a, int64_t tile0)
{
    constexpr int K = D + 2;
    Lane<T, P, NT> L(a, tile0);
    if (L.cnt == 0) return;
    double u[K][P];
    L.template load<K>(a.in0, a.ld_in0, u);
    State<D> s[P];
    double phi[P], H[P];
    double ub[K][P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double uj[K];
#pragma unroll
        for (int k = 0; k < K; ++k) uj[k] = u[k][j];
        s[j] = make_state<D>(a.gas, uj);
        phi[j] = a.gas.half_g1 * s[j].q;
        H[j] = (s[j].E + s[j].p) * s[j].rinv;
#pragma unroll
        for (int k = 0; k < K; ++k) ub[k][j] = 0.0;
    }
    const T *fb = static_cast<const T *>(a.in1);
    if (a.dir < 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            double f[K][P];
#pragma unroll
            for (int r = 0; r < K; ++r)
                load_run<T, P>(fb + L.i + (int64_t)(r * D + d) * a.ld_in1, L.cnt, L.vec, f[r]);
#pragma unroll
            for (int j = 0; j < P; ++j) {
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
    } else {
        double f[K][P];
#pragma unroll
        for (int r = 0; r < K; ++r)
            load_run<T, P>(fb + L.i + (int64_t)r * a.ld_in1, L.cnt, L.vec, f[r]);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (d != a.dir) continue;
#pragma unroll
            for (int j = 0; j < P; ++j) {
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
    }
#pragma unroll
    for (int k = 0; k < K; ++k) L.store(a.out0, a.ld_out0, k, ub[k]);
}

// ------------------------------------------------------------ Jacobian blocks

// LDS bytes the Jacobian staging needs per workgroup of `block` threads.
template <int D, typename T, int P>
constexpr size_t jacobian_lds_bytes(int block)
{
    return (size_t)block * P * (D + 2) * (D + 2) * sizeof(T);
}

// Copy the wave's staged blocks (count elements of T, contiguous in LDS and
// in global memory) with lane-contiguous 16-byte stores when allowed.
template <typename T, bool NT>
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

// The fused pass: flux tensor (out0, may be NULL), Jacobian blocks (out1,
// may be NULL) and Riemann invariants (out2, may be NULL) of the same state.
// `lds` is this workgroup's staging area of jacobian_lds_bytes(blockDim.x);
// every thread of the workgroup must call this (it holds barriers).
template <int D, typename T, int P, bool NT>
__device__ __forceinline__ void tile_fused(const Args &a, int64_t tile0, T *lds)
{
    constexpr int K = D + 2;
    constexpr int KK = K * K;
    Lane<T, P, NT> L(a, tile0);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int64_t wave0 = tile0 + (int64_t)wave * kWave * P;

    double u[K][P];
    L.template load<K>(a.in0, a.ld_in0, u);
    State<D> s[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double uj[K];
#pragma unroll
        for (int k = 0; k < K; ++k) uj[k] = u[k][j];
        s[j] = make_state<D>(a.gas, uj);
    }

    if (a.out0 && L.cnt > 0) {
#pragma unroll
        for (int r = 0; r < K; ++r) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                double f[P];
#pragma unroll
                for (int j = 0; j < P; ++j) f[j] = flux_entry<D>(s[j], r, d);
                L.store(a.out0, a.ld_out0, r * D + d, f);
            }
        }
    }
    if (a.out2 && L.cnt > 0) {
        double c[P];
#pragma unroll
        for (int j = 0; j < P; ++j) c[j] = sound_speed<D>(a.gas, s[j]);
        store_riemann<D, T, P, NT>(a, L, s, c, a.out2, a.ld_out2);
    }
    if (a.out1) {
        double phi[P], H[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            phi[j] = a.gas.half_g1 * s[j].q;
            H[j] = (s[j].E + s[j].p) * s[j].rinv;
        }
        T *region = lds + (size_t)wave * kWave * P * KK;
        const int64_t left = a.n - wave0;
        const int wave_pts = left <= 0 ? 0 : (left >= kWave * P ? kWave * P : (int)left);
        T *A = static_cast<T *>(a.out1);
#pragma unroll
        for (int d = 0; d < D; ++d) {
#pragma unroll
            for (int j = 0; j < P; ++j) {
                T *blk = region + (lane * P + j) * KK;
#pragma unroll
                for (int r = 0; r < K; ++r)
#pragma unroll
                    for (int c = 0; c < K; ++c)
                        blk[r * K + c] = (T)jacobian_entry<D>(a.gas, s[j], phi[j], H[j], d, r, c);
            }
            __syncthreads();
            if (wave_pts > 0)
                wave_copy_out<T, NT>(region, A + (d * a.ld_out1 + wave0) * KK, wave_pts * KK, L.vec, lane);
            __syncthreads();
        }
    }
}

}  // namespace fdbb
