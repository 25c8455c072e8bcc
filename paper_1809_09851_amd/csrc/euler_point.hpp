// Per-point algebra of the compressible-Euler building blocks, FP64 in
// registers.  Everything here is a __device__ inline function of one point;
// the tile code in euler_tiles.hpp feeds it from SoA loads and writes its
// results out.
//
// Conservative state U = (rho, m_1..m_D, E) with E the total energy per unit
// volume (Sec. 2.2, "Variables"); perfect gas with gamma = c_p / c_v.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdbb {

// Constants derived from gamma once per call, on the host, in FP64, so that
// no kernel divides by (gamma - 1).
struct Gas {
    double gamma;        // c_p / c_v
    double g1;           // gamma - 1
    double half_g1;      // (gamma - 1) / 2
    double inv_g1;       // 1 / (gamma - 1)
    double two_inv_g1;   // 2 / (gamma - 1)
    double quarter_g1;   // (gamma - 1) / 4
    double inv_gamma;    // 1 / gamma
    double p_inf;        // stiffening pressure of the general EOS entry (0: perfect gas)
    double inv_cv;       // 1 / c_v of the general EOS entry (0 elsewhere)
    double mu;           // dynamic viscosity of the viscous flux (0 elsewhere)
    double kappa;        // heat conductivity of the viscous flux (0 elsewhere)
};

// Shared sub-expressions of one conservative state, computed once and reused
// by every building block of the point.
template <int D>
struct State {
    double rho, rinv, E, p;
    double m[D];
    double v[D];
    double q;  // |v|^2
};

template <int D>
__device__ __forceinline__ State<D> make_state(const Gas &g, const double *u)
{
    State<D> s;
    s.rho = u[0];
    s.rinv = 1.0 / u[0];
    s.E = u[D + 1];
    double q = 0.0, mv = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        s.m[k] = u[1 + k];
        s.v[k] = s.m[k] * s.rinv;
        q += s.v[k] * s.v[k];
        mv += s.m[k] * s.v[k];  // rho |v|^2
    }
    s.q = q;
    // p = (gamma - 1)(E - rho |v|^2 / 2): the pressure of the perfect gas.
    s.p = g.g1 * (s.E - 0.5 * mv);
    return s;
}

template <int D>
__device__ __forceinline__ double sound_speed(const Gas &g, const State<D> &s)
{
    return sqrt(g.gamma * s.p * s.rinv);
}

// Primitive state V = (rho, v, p).
template <int D>
__device__ __forceinline__ void to_primitive(const State<D> &s, double *out)
{
    out[0] = s.rho;
#pragma unroll
    for (int k = 0; k < D; ++k) out[1 + k] = s.v[k];
    out[D + 1] = s.p;
}

// Conservative state from primitive V = (rho, v, p):
// m = rho v, E = p / (gamma - 1) + rho |v|^2 / 2.
template <int D>
__device__ __forceinline__ void from_primitive(const Gas &g, const double *vp, double *out)
{
    const double rho = vp[0];
    double q = 0.0;
    out[0] = rho;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        out[1 + k] = rho * vp[1 + k];
        q += vp[1 + k] * vp[1 + k];
    }
    out[D + 1] = vp[D + 1] * g.inv_g1 + 0.5 * rho * q;
}

// (m . m) / (rho rho), in the order the micro-benchmark expression writes it.
template <int D>
__device__ __forceinline__ double velocity_magnitude2(const double *u)
{
    double mm = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) mm += u[1 + k] * u[1 + k];
    return mm / (u[0] * u[0]);
}

// Component r of the inviscid flux in direction d: F_d = (m_d,
// m_i v_d + delta_id p, v_d (E + p)).
template <int D>
__device__ __forceinline__ double flux_entry(const State<D> &s, int r, int d)
{
    if (r == 0) return s.m[d];
    if (r == D + 1) return s.v[d] * (s.E + s.p);
    const int i = r - 1;
    const double mom = s.m[i] * s.v[d];
    return (i == d) ? mom + s.p : mom;
}

// Entry (r, c) of A_d = dF_d/dU, the derivative of the flux above through
// dp/drho = phi, dp/dm_j = -(gamma-1) v_j, dp/dE = gamma - 1, with
// phi = (gamma-1)|v|^2/2 and the total enthalpy H = (E + p)/rho:
//   row 0       : e_{1+d}
//   row 1+i     : [delta_id phi - v_i v_d,
//                  delta_ij v_d + delta_jd v_i - (gamma-1) delta_id v_j,
//                  (gamma-1) delta_id]
//   row D+1     : [v_d (phi - H), delta_jd H - (gamma-1) v_j v_d, gamma v_d]
// v is the velocity of the point.  r, c and d are compile-time constants
// after unrolling, so every branch folds away.
template <int D>
__device__ __forceinline__ double jacobian_entry(const Gas &g, const double *v, double phi, double H, int d,
                                                 int r, int c)
{
    constexpr int K = D + 2;
    if (r == 0) return (c == 1 + d) ? 1.0 : 0.0;
    if (r == K - 1) {
        if (c == 0) return v[d] * (phi - H);
        if (c == K - 1) return g.gamma * v[d];
        const int j = c - 1;
        const double t = -g.g1 * v[j] * v[d];
        return (j == d) ? t + H : t;
    }
    const int i = r - 1;
    if (c == 0) return (i == d) ? phi - v[i] * v[d] : -v[i] * v[d];
    if (c == K - 1) return (i == d) ? g.g1 : 0.0;
    const int j = c - 1;
    double t = 0.0;
    if (i == j) t += v[d];
    if (j == d) t += v[i];
    if (i == d) t -= g.g1 * v[j];
    return t;
}

// Characteristic decomposition A_d = R diag(v_d - c, v_d.., v_d + c) L in
// closed form.  Columns of R (rows of L) are ordered as the characteristic
// variables: the v_d - c wave, the entropy wave, the shear waves j != d in
// ascending j, the v_d + c wave.  With b = (gamma-1)/c^2:
//   r-  = (1, v - c e_d, H - c v_d)      l-  = (b q/2 + v_d/c, -b v - e_d/c, b) / 2
//   r0  = (1, v, q/2)                    l0  = (1 - b q/2, b v, -b)
//   r_j = (0, e_j, v_j)                  l_j = (-v_j, e_j, 0)
//   r+  = (1, v + c e_d, H + c v_d)      l+  = (b q/2 - v_d/c, -b v + e_d/c, b) / 2
// (q = |v|^2).  Each l is orthogonal to every r of another wave and has
// unit product with its own, which the reader can check row by column.
struct Waves {
    double c, inv_c, H, q, b;
};

template <int D>
__device__ __forceinline__ int shear_axis(int slot, int d)
{
    return slot < d ? slot : slot + 1;
}

template <int D>
__device__ __forceinline__ double right_entry(const double *v, const Waves &w, int d, int r, int col)
{
    constexpr int K = D + 2;
    if (col == 0 || col == K - 1) {
        const double sg = col == 0 ? -1.0 : 1.0;
        if (r == 0) return 1.0;
        if (r == K - 1) return w.H + sg * w.c * v[d];
        return (r - 1 == d) ? v[r - 1] + sg * w.c : v[r - 1];
    }
    if (col == 1) {
        if (r == 0) return 1.0;
        if (r == K - 1) return 0.5 * w.q;
        return v[r - 1];
    }
    const int j = shear_axis<D>(col - 2, d);
    if (r == 0) return 0.0;
    if (r == K - 1) return v[j];
    return (r - 1 == j) ? 1.0 : 0.0;
}

template <int D>
__device__ __forceinline__ double left_entry(const double *v, const Waves &w, int d, int row, int c)
{
    constexpr int K = D + 2;
    if (row == 0 || row == K - 1) {
        const double sg = row == 0 ? 1.0 : -1.0;
        if (c == 0) return 0.5 * (0.5 * w.b * w.q + sg * v[d] * w.inv_c);
        if (c == K - 1) return 0.5 * w.b;
        const double t = -w.b * v[c - 1];
        return 0.5 * ((c - 1 == d) ? t - sg * w.inv_c : t);
    }
    if (row == 1) {
        if (c == 0) return 1.0 - 0.5 * w.b * w.q;
        if (c == K - 1) return -w.b;
        return w.b * v[c - 1];
    }
    const int j = shear_axis<D>(row - 2, d);
    if (c == 0) return -v[j];
    if (c == K - 1) return 0.0;
    return (c - 1 == j) ? 1.0 : 0.0;
}

template <int D>
__device__ __forceinline__ Waves make_waves(const Gas &g, const State<D> &s)
{
    Waves w;
    w.c = sqrt(g.gamma * s.p * s.rinv);
    w.inv_c = 1.0 / w.c;
    w.H = (s.E + s.p) * s.rinv;
    w.q = s.q;
    w.b = g.g1 * w.inv_c * w.inv_c;
    return w;
}

// x^y for the positive bases of the entropy and of its inverse, as
// exp(y log x): the general pow also serves negative bases, integer
// exponents and a doubled-precision logarithm, which these uses do not need.
// The exponent y log x carries an absolute error of a few units in the last
// place of |y log x|, which is the relative error of the result (below
// 1e-14 for |y log x| < 40).  x <= 0 gives NaN or the limit at 0, as pow.
__device__ __forceinline__ double pos_pow(double x, double y) { return exp(y * log(x)); }

// The same power for outputs stored in FP32, where the library's FP64 exp
// and log would make the entropy-carrying transforms bound by the FP64
// instruction rate rather than by HBM.  Base-2 decomposition:
//   x = m 2^e (frexp, exact; m in [1/2, 1)),
//   z = y (e + log2 m),  z = k + f (k = floor z, f in [0, 1)),
//   x^y = 2^f 2^k,
// with log2 m and 2^f from the GPU's FP32 transcendental instructions
// (v_log_f32, v_exp_f32, each within about one unit in the last place),
// and the exponent split, the sum e + log2 m, the product with y and the
// scaling by 2^k in FP64.  Relative error: |y| ln 2 (2^-24 / ln 2 + 2^-24)
// from the FP32 rounding of m and the logarithm, plus 2^-24 ln 2 + 2^-23
// from f and the exponential, below 6e-7 for |y| <= 3; the building blocks
// take y = -gamma and y = 1/(gamma-1), and the FP32-storage contract is
// 1e-5.  Zero, negative and non-finite x give what exp(y log x) gives in
// IEEE arithmetic (selected, not branched, so no library code enters the
// kernels); results beyond the range of doubles saturate to inf or 0.
__device__ __forceinline__ double pos_pow_fp32(double x, double y)
{
    const bool ok = x > 0.0 && x < INFINITY;
    int e;
    const double m = frexp(ok ? x : 1.0, &e);
    const double l2 = (double)e + (double)__builtin_amdgcn_logf((float)m);
    // log2 0 = -inf, log2 inf = inf, NaN below zero and for NaN
    const double lg = ok ? l2 : (x == 0.0 ? -INFINITY : (x == INFINITY ? INFINITY : NAN));
    const double z = y * lg;
    const double zc = fmin(fmax(z, -1100.0), 1100.0);  // 2^k saturates beyond
    const double k = floor(zc);
    const double r = ldexp((double)__builtin_amdgcn_exp2f((float)(zc - k)), (int)k);
    return z != z ? z : r;
}

// x^y for x > 0: FP32-storage form when FP32 (outputs stored in FP32).
template <bool FP32>
__device__ __forceinline__ double pos_pow_t(double x, double y)
{
    if constexpr (FP32) return pos_pow_fp32(x, y);
    else return pos_pow(x, y);
}

// Entropy s = p / rho^gamma.
template <int D, bool FP32 = false>
__device__ __forceinline__ double entropy(const Gas &g, const State<D> &s)
{
    return s.p * pos_pow_t<FP32>(s.rho, -g.gamma);
}

// Adjoint contribution of direction d: ubar += A_d^T fb, where fb = (a,
// b_1..b_D, e) is the cotangent of F_d.  Written out from the transposed
// Jacobian above with bv = b . v:
//   ubar_0    += phi b_d - v_d bv + e v_d (phi - H)
//   ubar_1+j  += delta_jd (a + bv + e H) + b_j v_d - (gamma-1) v_j (b_d + e v_d)
//   ubar_D+1  += (gamma-1) b_d + gamma v_d e
template <int D>
__device__ __forceinline__ void adjoint_accumulate(const Gas &g, const State<D> &s, double phi,
                                                   double H, int d, const double *fb,
                                                   double *ubar)
{
    const double a = fb[0];
    const double e = fb[D + 1];
    double bv = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) bv += fb[1 + i] * s.v[i];
    const double bd = fb[1 + d];
    const double vd = s.v[d];
    ubar[0] += phi * bd - vd * bv + e * vd * (phi - H);
    const double w = g.g1 * (bd + e * vd);
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double t = fb[1 + j] * vd - w * s.v[j];
        if (j == d) t += a + bv + e * H;
        ubar[1 + j] += t;
    }
    ubar[D + 1] += g.g1 * bd + g.gamma * vd * e;
}

// Roe-averaged state between a left and a right state, as a conservative
// state: with a = sqrt(rho_L), b = sqrt(rho_R), rho^ = a b and the velocity
// and total enthalpy H = (E + p) / rho averaged with weights a and b; the
// pressure follows from H^ = gamma p^ / ((gamma - 1) rho^) + |v^|^2 / 2.
// The flux Jacobians at this state satisfy A(U^)(U_R - U_L) = F(U_R) - F(U_L).
// One side at a time is folded into weighted sums, so that only those sums
// and one raw state are live at once.

// Adds sqrt(rho) (v, H) of the conservative state u to sum[0..D] (v, then
// H); returns sqrt(rho).  With r = 1/sqrt(rho): sqrt(rho) v = m r,
// sqrt(rho) H = (E + p) r and rho |v|^2 = |m|^2 r^2, so one reciprocal
// square root replaces a square root and a division.
template <int D>
__device__ __forceinline__ double roe_accumulate(const Gas &g, const double *u, double *sum)
{
    const double r = rsqrt(u[0]);
    double mm = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        mm += u[1 + k] * u[1 + k];
        sum[k] += u[1 + k] * r;
    }
    const double p = g.g1 * (u[D + 1] - 0.5 * mm * (r * r));
    sum[D] += (u[D + 1] + p) * r;
    return u[0] * r;
}

// Completes the average from the weighted sums of both sides and the two
// weights a = sqrt(rho_L), b = sqrt(rho_R).
template <int D>
__device__ __forceinline__ void roe_finish(const Gas &g, const double *sum, double a, double b, double *out)
{
    const double w = 1.0 / (a + b);
    const double rho = a * b;
    const double H = sum[D] * w;
    double q = 0.0;
    out[0] = rho;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double v = sum[k] * w;
        q += v * v;
        out[1 + k] = rho * v;
    }
    const double p = g.g1 * g.inv_gamma * rho * (H - 0.5 * q);
    out[D + 1] = rho * H - p;
}

}  // namespace fdbb
