/*
 * Plain CPU oracle for the compressible-Euler building blocks of
 * "FDBB: Fluid Dynamics Building Blocks" (Moeller, Jaeschke).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the HIP library.
 *
 * Every function is a direct, single-threaded FP64 evaluation of the
 * per-point definition, one point at a time, with no blocking or fusion.
 * Build with -O2 -ffp-contract=off so that no multiply-add is contracted.
 *
 * Notation (Sec. 2.2, paragraph "Variables"): the conservative state in
 * D dimensions is U = (rho, m_1..m_D, E) with m = rho*v the momentum and E
 * the total energy per unit volume (the paper's "rho E").  K = D + 2.
 * Perfect gas with adiabatic index gamma = c_p/c_v (paper: 7/2 over 5/2).
 *
 * Array layout, shared by every function:
 *   a field set is one base pointer plus a leading dimension ld (elements);
 *   component k of point i lives at base[k*ld + i]                   (SoA);
 *   the flux tensor F is N_U x N_D row-major (Sec. 2.1, "Block Expressions",
 *   row-major default; Sec. 2.2, "Inviscid Fluxes", 5x3 block), so flux
 *   component (r, d) is field r*D + d;
 *   flux Jacobian blocks are stored point-major: entry (r, c) of
 *   A_d at point i is A[(d*ldA + i)*K*K + r*K + c].
 *
 * Return value: 0 on success, -1 for an unsupported dim or direction.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define ORACLE_MAXK 5

static int dim_ok(int dim) { return dim >= 1 && dim <= 3; }

/* Primitive quantities of one conservative state (Sec. 2.2, "Variables";
 * pressure of the perfect gas, p = (gamma-1) * rho * e, with e the specific
 * internal energy, as in the p_rhoe member of the EOS prototype). */
typedef struct {
    double rho;
    double v[3];
    double q;   /* |v|^2 */
    double E;
    double p;
} point_state;

static point_state load_cons(int dim, double gamma, const double *U,
                             int64_t ld, int64_t i)
{
    point_state s;
    int k;
    double kinetic, e;
    s.rho = U[0 * ld + i];
    s.q = 0.0;
    for (k = 0; k < 3; ++k)
        s.v[k] = 0.0;
    for (k = 0; k < dim; ++k) {
        s.v[k] = U[(1 + k) * ld + i] / s.rho;
        s.q = s.q + s.v[k] * s.v[k];
    }
    s.E = U[(dim + 1) * ld + i];
    /* specific internal energy e = E/rho - |v|^2/2, then p = (gamma-1) rho e */
    kinetic = 0.5 * s.q;
    e = s.E / s.rho - kinetic;
    s.p = (gamma - 1.0) * s.rho * e;
    return s;
}

/* Conservative -> primitive, V = (rho, v_1..v_D, p)
 * (Sec. 2.2, "Variables", the conversion figure). */
int oracle_cons2prim(int dim, double gamma, const double *U, int64_t ldU,
                     double *V, int64_t ldV, int64_t n)
{
    int64_t i;
    int k;
    if (!dim_ok(dim))
        return -1;
    for (i = 0; i < n; ++i) {
        point_state s = load_cons(dim, gamma, U, ldU, i);
        V[0 * ldV + i] = s.rho;
        for (k = 0; k < dim; ++k)
            V[(1 + k) * ldV + i] = s.v[k];
        V[(dim + 1) * ldV + i] = s.p;
    }
    return 0;
}

/* Primitive -> conservative: m = rho v, E = rho e + rho |v|^2 / 2 with
 * rho e = p / (gamma - 1) (Sec. 2.2, "Variables"). */
int oracle_prim2cons(int dim, double gamma, const double *V, int64_t ldV,
                     double *U, int64_t ldU, int64_t n)
{
    int64_t i;
    int k;
    if (!dim_ok(dim))
        return -1;
    for (i = 0; i < n; ++i) {
        double rho = V[0 * ldV + i];
        double p = V[(dim + 1) * ldV + i];
        double q = 0.0;
        double v[3];
        for (k = 0; k < dim; ++k) {
            v[k] = V[(1 + k) * ldV + i];
            q = q + v[k] * v[k];
        }
        U[0 * ldU + i] = rho;
        for (k = 0; k < dim; ++k)
            U[(1 + k) * ldU + i] = rho * v[k];
        U[(dim + 1) * ldU + i] = p / (gamma - 1.0) + 0.5 * rho * q;
    }
    return 0;
}

/* Squared velocity magnitude from the conservative state, the paper's
 * micro-benchmark expression (Sec. 3, Eq. 2): |v|^2 = (m . m) / (rho rho). */
int oracle_v_mag2(int dim, const double *U, int64_t ldU, double *y, int64_t n)
{
    int64_t i;
    int k;
    if (!dim_ok(dim))
        return -1;
    for (i = 0; i < n; ++i) {
        double rho = U[0 * ldU + i];
        double mm = 0.0;
        for (k = 0; k < dim; ++k) {
            double m = U[(1 + k) * ldU + i];
            mm = mm + m * m;
        }
        y[i] = mm / (rho * rho);
    }
    return 0;
}

/* Equation of state of the perfect gas (Sec. 2.2, "Equations of state"):
 * pressure p and speed of sound c = sqrt(gamma p / rho).  Either output
 * may be NULL. */
int oracle_eos(int dim, double gamma, const double *U, int64_t ldU,
               double *p, double *c, int64_t n)
{
    int64_t i;
    if (!dim_ok(dim))
        return -1;
    for (i = 0; i < n; ++i) {
        point_state s = load_cons(dim, gamma, U, ldU, i);
        if (p)
            p[i] = s.p;
        if (c)
            c[i] = sqrt(gamma * s.p / s.rho);
    }
    return 0;
}

/* Inviscid flux tensor (Sec. 2.2, "Inviscid Fluxes"):
 *   F(U) = [ rho v ; rho v (x) v + I p ; v (rho E + p) ],
 * an N_U x N_D block; column d is the flux F_d in direction d. */
int oracle_flux(int dim, double gamma, const double *U, int64_t ldU,
                double *F, int64_t ldF, int64_t n)
{
    int64_t i;
    int d, r;
    if (!dim_ok(dim))
        return -1;
    for (i = 0; i < n; ++i) {
        point_state s = load_cons(dim, gamma, U, ldU, i);
        for (d = 0; d < dim; ++d) {
            double col[ORACLE_MAXK];
            col[0] = s.rho * s.v[d];
            for (r = 0; r < dim; ++r)
                col[1 + r] = s.rho * s.v[r] * s.v[d] + (r == d ? s.p : 0.0);
            col[dim + 1] = s.v[d] * (s.E + s.p);
            for (r = 0; r < dim + 2; ++r)
                F[(r * dim + d) * ldF + i] = col[r];
        }
    }
    return 0;
}

/* Flux Jacobian A_d = dF_d/dU of one point, written out term by term from
 * the flux tensor and p = (gamma-1)(E - rho |v|^2 / 2).  The paper names
 * the flux Jacobians (Fig. 1) but leaves them unfinished (Sec. 2.2,
 * "Inviscid Fluxes"); this is the exact derivative.  With
 * phi = (gamma-1)|v|^2/2 and H = (E + p)/rho:
 *   dp/drho = phi, dp/dm_j = -(gamma-1) v_j, dp/dE = gamma-1. */
static void jacobian_point(int dim, double gamma, const point_state *s, int d,
                           double A[ORACLE_MAXK][ORACLE_MAXK])
{
    int K = dim + 2, r, c, i, j;
    double g1 = gamma - 1.0;
    double phi = 0.5 * g1 * s->q;
    double H = (s->E + s->p) / s->rho;
    double dp_drho = phi;
    double dp_dm[3];
    double dp_dE = g1;

    for (j = 0; j < dim; ++j)
        dp_dm[j] = -g1 * s->v[j];
    for (r = 0; r < K; ++r)
        for (c = 0; c < K; ++c)
            A[r][c] = 0.0;

    /* row 0: F_d[0] = m_d */
    A[0][1 + d] = 1.0;

    /* rows 1..D: F_d[1+i] = m_i m_d / rho + delta_id p */
    for (i = 0; i < dim; ++i) {
        A[1 + i][0] = -s->v[i] * s->v[d] + (i == d ? dp_drho : 0.0);
        for (j = 0; j < dim; ++j) {
            double t = 0.0;
            if (i == j)
                t = t + s->v[d];
            if (j == d)
                t = t + s->v[i];
            if (i == d)
                t = t + dp_dm[j];
            A[1 + i][1 + j] = t;
        }
        A[1 + i][K - 1] = (i == d ? dp_dE : 0.0);
    }

    /* row K-1: F_d[K-1] = m_d (E + p) / rho */
    A[K - 1][0] = s->v[d] * dp_drho - s->v[d] * H;
    for (j = 0; j < dim; ++j)
        A[K - 1][1 + j] = (j == d ? H : 0.0) + s->v[d] * dp_dm[j];
    A[K - 1][K - 1] = s->v[d] * (1.0 + dp_dE);
}

/* Flux Jacobians A_d for every direction d (Fig. 1, "flux-Jacobians"). */
int oracle_flux_jacobian(int dim, double gamma, const double *U, int64_t ldU,
                         double *A, int64_t ldA, int64_t n)
{
    int64_t i;
    int d, r, c, K = dim + 2;
    double blk[ORACLE_MAXK][ORACLE_MAXK];
    if (!dim_ok(dim))
        return -1;
    for (i = 0; i < n; ++i) {
        point_state s = load_cons(dim, gamma, U, ldU, i);
        for (d = 0; d < dim; ++d) {
            double *dst = A + (d * ldA + i) * (int64_t)(K * K);
            jacobian_point(dim, gamma, &s, d, blk);
            for (r = 0; r < K; ++r)
                for (c = 0; c < K; ++c)
                    dst[r * K + c] = blk[r][c];
        }
    }
    return 0;
}

/* Riemann invariants (Fig. 1, "Riemann invariants"): for each direction d
 * the pair w-_d = v_d - 2c/(gamma-1), w+_d = v_d + 2c/(gamma-1), followed
 * by the entropy s = p / rho^gamma.  Output fields, in order:
 * (w-_0, w+_0, ..., w-_{D-1}, w+_{D-1}, s). */
int oracle_riemann_invariants(int dim, double gamma, const double *U,
                              int64_t ldU, double *R, int64_t ldR, int64_t n)
{
    int64_t i;
    int d;
    if (!dim_ok(dim))
        return -1;
    for (i = 0; i < n; ++i) {
        point_state s = load_cons(dim, gamma, U, ldU, i);
        double c = sqrt(gamma * s.p / s.rho);
        double two_c_over_g1 = 2.0 * c / (gamma - 1.0);
        for (d = 0; d < dim; ++d) {
            R[(2 * d + 0) * ldR + i] = s.v[d] - two_c_over_g1;
            R[(2 * d + 1) * ldR + i] = s.v[d] + two_c_over_g1;
        }
        R[(2 * dim) * ldR + i] = s.p / pow(s.rho, gamma);
    }
    return 0;
}

/* Characteristic variables for direction dir (Fig. 1, "characteristic
 * variables"), taken pointwise as W = (w-_dir, s, v_j for j != dir in
 * ascending j, w+_dir): the invariants ordered by the eigenvalues
 * v_dir - c, v_dir (D times), v_dir + c of A_dir. */
int oracle_cons2char(int dim, int dir, double gamma, const double *U,
                     int64_t ldU, double *W, int64_t ldW, int64_t n)
{
    int64_t i;
    int j, slot;
    if (!dim_ok(dim) || dir < 0 || dir >= dim)
        return -1;
    for (i = 0; i < n; ++i) {
        point_state s = load_cons(dim, gamma, U, ldU, i);
        double c = sqrt(gamma * s.p / s.rho);
        double two_c_over_g1 = 2.0 * c / (gamma - 1.0);
        W[0 * ldW + i] = s.v[dir] - two_c_over_g1;
        W[1 * ldW + i] = s.p / pow(s.rho, gamma);
        slot = 2;
        for (j = 0; j < dim; ++j) {
            if (j == dir)
                continue;
            W[slot * ldW + i] = s.v[j];
            slot = slot + 1;
        }
        W[(dim + 1) * ldW + i] = s.v[dir] + two_c_over_g1;
    }
    return 0;
}

/* Inverse of oracle_cons2char: from w-, w+ recover v_dir and c, from c and
 * s = p/rho^gamma recover rho = (c^2 / (gamma s))^(1/(gamma-1)) and
 * p = rho c^2 / gamma, then build U from (rho, v, p). */
int oracle_char2cons(int dim, int dir, double gamma, const double *W,
                     int64_t ldW, double *U, int64_t ldU, int64_t n)
{
    int64_t i;
    int j, slot;
    double g1 = gamma - 1.0;
    if (!dim_ok(dim) || dir < 0 || dir >= dim)
        return -1;
    for (i = 0; i < n; ++i) {
        double wm = W[0 * ldW + i];
        double s = W[1 * ldW + i];
        double wp = W[(dim + 1) * ldW + i];
        double v[3];
        double c, rho, p, q;
        slot = 2;
        for (j = 0; j < dim; ++j) {
            if (j == dir)
                continue;
            v[j] = W[slot * ldW + i];
            slot = slot + 1;
        }
        v[dir] = 0.5 * (wp + wm);
        c = 0.25 * g1 * (wp - wm);
        rho = pow(c * c / (gamma * s), 1.0 / g1);
        p = rho * c * c / gamma;
        q = 0.0;
        for (j = 0; j < dim; ++j)
            q = q + v[j] * v[j];
        U[0 * ldU + i] = rho;
        for (j = 0; j < dim; ++j)
            U[(1 + j) * ldU + i] = rho * v[j];
        U[(dim + 1) * ldU + i] = p / g1 + 0.5 * rho * q;
    }
    return 0;
}

/* Adjoint of the flux map: Ubar = sum_d A_d(U)^T Fbar_d, with A_d built as
 * an explicit K x K matrix and multiplied in transposed form.
 * dir == -1: Fbar has the flux tensor's layout (field r*D + d), summed
 * over all d.  dir in [0, D): Fbar holds K fields, Fbar_dir only. */
int oracle_flux_adjoint(int dim, int dir, double gamma, const double *U,
                        int64_t ldU, const double *Fb, int64_t ldFb,
                        double *Ub, int64_t ldUb, int64_t n)
{
    int64_t i;
    int d, r, c, K = dim + 2;
    double blk[ORACLE_MAXK][ORACLE_MAXK];
    if (!dim_ok(dim) || dir < -1 || dir >= dim)
        return -1;
    for (i = 0; i < n; ++i) {
        point_state s = load_cons(dim, gamma, U, ldU, i);
        double acc[ORACLE_MAXK];
        for (c = 0; c < K; ++c)
            acc[c] = 0.0;
        for (d = 0; d < dim; ++d) {
            if (dir >= 0 && d != dir)
                continue;
            jacobian_point(dim, gamma, &s, d, blk);
            for (c = 0; c < K; ++c) {
                for (r = 0; r < K; ++r) {
                    int64_t field = (dir >= 0) ? r : (r * dim + d);
                    acc[c] = acc[c] + blk[r][c] * Fb[field * ldFb + i];
                }
            }
        }
        for (c = 0; c < K; ++c)
            Ub[c * ldUb + i] = acc[c];
    }
    return 0;
}

/* Right eigenvectors of A_dir as the columns of a K x K matrix, in the order
 * of the eigenvalues v_d - c, v_d (entropy, then the tangential directions
 * in ascending order), v_d + c (the order of the characteristic variables
 * above).  Normalised with a unit density component for the acoustic and
 * entropy waves and a unit tangential momentum for the shear waves:
 *   r- = (1, v - c e_d, H - c v_d),  r0 = (1, v, |v|^2/2),
 *   r_j = (0, e_j, v_j) for j != d,   r+ = (1, v + c e_d, H + c v_d). */
static void right_eigenvectors(int dim, double gamma, const point_state *s, int d,
                               double Rm[ORACLE_MAXK][ORACLE_MAXK])
{
    int K = dim + 2, r, c, j, col;
    double cs = sqrt(gamma * s->p / s->rho);
    double H = (s->E + s->p) / s->rho;
    for (r = 0; r < K; ++r)
        for (c = 0; c < K; ++c)
            Rm[r][c] = 0.0;
    /* r- */
    Rm[0][0] = 1.0;
    for (j = 0; j < dim; ++j)
        Rm[1 + j][0] = s->v[j] - (j == d ? cs : 0.0);
    Rm[K - 1][0] = H - cs * s->v[d];
    /* r0 */
    Rm[0][1] = 1.0;
    for (j = 0; j < dim; ++j)
        Rm[1 + j][1] = s->v[j];
    Rm[K - 1][1] = 0.5 * s->q;
    /* shear waves */
    col = 2;
    for (j = 0; j < dim; ++j) {
        if (j == d)
            continue;
        Rm[1 + j][col] = 1.0;
        Rm[K - 1][col] = s->v[j];
        col = col + 1;
    }
    /* r+ */
    Rm[0][K - 1] = 1.0;
    for (j = 0; j < dim; ++j)
        Rm[1 + j][K - 1] = s->v[j] + (j == d ? cs : 0.0);
    Rm[K - 1][K - 1] = H + cs * s->v[d];
}

/* Inverse of a K x K matrix by Gauss-Jordan elimination with partial
 * pivoting.  Returns 0, or -1 for a singular matrix. */
static int invert(int K, double M[ORACLE_MAXK][ORACLE_MAXK], double X[ORACLE_MAXK][ORACLE_MAXK])
{
    double a[ORACLE_MAXK][2 * ORACLE_MAXK];
    int r, c, k, piv;
    for (r = 0; r < K; ++r)
        for (c = 0; c < 2 * K; ++c)
            a[r][c] = (c < K) ? M[r][c] : (c - K == r ? 1.0 : 0.0);
    for (k = 0; k < K; ++k) {
        piv = k;
        for (r = k + 1; r < K; ++r)
            if (fabs(a[r][k]) > fabs(a[piv][k]))
                piv = r;
        if (a[piv][k] == 0.0)
            return -1;
        if (piv != k)
            for (c = 0; c < 2 * K; ++c) {
                double t = a[k][c];
                a[k][c] = a[piv][c];
                a[piv][c] = t;
            }
        {
            double inv = 1.0 / a[k][k];
            for (c = 0; c < 2 * K; ++c)
                a[k][c] = a[k][c] * inv;
        }
        for (r = 0; r < K; ++r) {
            double f;
            if (r == k)
                continue;
            f = a[r][k];
            for (c = 0; c < 2 * K; ++c)
                a[r][c] = a[r][c] - f * a[k][c];
        }
    }
    for (r = 0; r < K; ++r)
        for (c = 0; c < K; ++c)
            X[r][c] = a[r][K + c];
    return 0;
}

/* Characteristic decomposition A_d = R_d diag(lambda) L_d of every
 * direction: R_d as above and L_d = R_d^{-1}, both as point-major row-major
 * K x K blocks (the Jacobian layout).  Either output may be NULL.  Returns -2
 * if some R_d is singular (c = 0). */
int oracle_eigenvectors(int dim, double gamma, const double *U, int64_t ldU,
                        double *L, int64_t ldL, double *R, int64_t ldR, int64_t n)
{
    int64_t i;
    int d, r, c, K = dim + 2;
    double Rm[ORACLE_MAXK][ORACLE_MAXK], Lm[ORACLE_MAXK][ORACLE_MAXK];
    if (!dim_ok(dim))
        return -1;
    for (i = 0; i < n; ++i) {
        point_state s = load_cons(dim, gamma, U, ldU, i);
        for (d = 0; d < dim; ++d) {
            right_eigenvectors(dim, gamma, &s, d, Rm);
            if (R)
                for (r = 0; r < K; ++r)
                    for (c = 0; c < K; ++c)
                        R[(d * ldR + i) * (int64_t)(K * K) + r * K + c] = Rm[r][c];
            if (L) {
                if (invert(K, Rm, Lm) != 0)
                    return -2;
                for (r = 0; r < K; ++r)
                    for (c = 0; c < K; ++c)
                        L[(d * ldL + i) * (int64_t)(K * K) + r * K + c] = Lm[r][c];
            }
        }
    }
    return 0;
}

/* Y = L_dir(U) X (mode 0: state increments to characteristic increments)
 * or Y = R_dir(U) X (mode 1: back), with X and Y K-field sets. */
int oracle_char_apply(int dim, int dir, int mode, double gamma, const double *U, int64_t ldU,
                      const double *X, int64_t ldX, double *Y, int64_t ldY, int64_t n)
{
    int64_t i;
    int r, c, K = dim + 2;
    double Rm[ORACLE_MAXK][ORACLE_MAXK], Lm[ORACLE_MAXK][ORACLE_MAXK];
    if (!dim_ok(dim) || dir < 0 || dir >= dim || mode < 0 || mode > 1)
        return -1;
    for (i = 0; i < n; ++i) {
        point_state s = load_cons(dim, gamma, U, ldU, i);
        double (*M)[ORACLE_MAXK] = Rm;
        right_eigenvectors(dim, gamma, &s, dir, Rm);
        if (mode == 0) {
            if (invert(K, Rm, Lm) != 0)
                return -2;
            M = Lm;
        }
        for (r = 0; r < K; ++r) {
            double acc = 0.0;
            for (c = 0; c < K; ++c)
                acc = acc + M[r][c] * X[c * ldX + i];
            Y[r * ldY + i] = acc;
        }
    }
    return 0;
}

/* Roe-averaged state between a left and a right state (the linearisation
 * point of the characteristic decomposition between two states; Roe's
 * average for the perfect gas).  With weights a = sqrt(rho_L), b =
 * sqrt(rho_R):
 *   rho^ = a b,   v^ = (a v_L + b v_R) / (a + b),
 *   H^   = (a H_L + b H_R) / (a + b),  H = (E + p) / rho,
 * returned as the conservative state with that density, velocity and total
 * enthalpy: m^ = rho^ v^, and, since H = gamma p / ((gamma-1) rho) + |v|^2/2,
 *   p^ = (gamma-1)/gamma * rho^ (H^ - |v^|^2/2),   E^ = rho^ H^ - p^. */
int oracle_roe_average(int dim, double gamma, const double *UL, int64_t ldL,
                       const double *UR, int64_t ldR, double *Uh, int64_t ldH, int64_t n)
{
    int64_t i;
    int k;
    if (!dim_ok(dim))
        return -1;
    for (i = 0; i < n; ++i) {
        point_state l = load_cons(dim, gamma, UL, ldL, i);
        point_state r = load_cons(dim, gamma, UR, ldR, i);
        double a = sqrt(l.rho), b = sqrt(r.rho);
        double HL = (l.E + l.p) / l.rho, HR = (r.E + r.p) / r.rho;
        double rho = a * b;
        double H = (a * HL + b * HR) / (a + b);
        double q = 0.0, p;
        double v[3];
        for (k = 0; k < dim; ++k) {
            v[k] = (a * l.v[k] + b * r.v[k]) / (a + b);
            q = q + v[k] * v[k];
        }
        p = (gamma - 1.0) / gamma * rho * (H - 0.5 * q);
        Uh[0 * ldH + i] = rho;
        for (k = 0; k < dim; ++k)
            Uh[(1 + k) * ldH + i] = rho * v[k];
        Uh[(dim + 1) * ldH + i] = rho * H - p;
    }
    return 0;
}

/* Equations of state of the form f(p, V, T) = 0 behind a runtime id (Sec.
 * 2.2, "Equations of state": each EOS supplies p(rho, e) and T(rho, e),
 * with e the specific internal energy).  From the conservative state,
 * e = E/rho - |v|^2/2, then per point the pressure p, the speed of sound c
 * and the temperature T; any output may be NULL.
 *
 *   eos 0, perfect gas, params = (c_p, c_v):  gamma = c_p/c_v,
 *     p = (gamma-1) rho e,  T = e / c_v,  c^2 = gamma p / rho.
 *   eos 1, stiffened gas, params = (gamma, p_inf, c_v):
 *     p = (gamma-1) rho e - gamma p_inf,  T = (e - p_inf/rho) / c_v,
 *     c^2 = gamma (p + p_inf) / rho.
 * The speed of sound is the isentropic derivative (dp/drho)_s =
 * (dp/drho)_e + (p/rho^2) (dp/de)_rho of each p(rho, e).  Returns -1 for an
 * unknown id. */
int oracle_eos_pvt(int dim, int eos, const double *params, const double *U, int64_t ldU,
                   double *p, double *c, double *T, int64_t n)
{
    int64_t i;
    int k;
    if (!dim_ok(dim) || eos < 0 || eos > 1)
        return -1;
    for (i = 0; i < n; ++i) {
        double rho = U[0 * ldU + i];
        double q = 0.0, e, pi, ci, Ti;
        for (k = 0; k < dim; ++k) {
            double v = U[(1 + k) * ldU + i] / rho;
            q = q + v * v;
        }
        e = U[(dim + 1) * ldU + i] / rho - 0.5 * q;
        if (eos == 0) {
            double gamma = params[0] / params[1];
            pi = (gamma - 1.0) * rho * e;
            Ti = e / params[1];
            ci = sqrt(gamma * pi / rho);
        } else {
            double gamma = params[0], pinf = params[1];
            pi = (gamma - 1.0) * rho * e - gamma * pinf;
            Ti = (e - pinf / rho) / params[2];
            ci = sqrt(gamma * (pi + pinf) / rho);
        }
        if (p)
            p[i] = pi;
        if (c)
            c[i] = ci;
        if (T)
            T[i] = Ti;
    }
    return 0;
}

/* Viscous flux tensor (Fig. 1, "viscous fluxes"; the paper names it without
 * a definition, so this is the compressible Navier-Stokes one): Newtonian
 * stress with Stokes' hypothesis and Fourier heat conduction, constant
 * dynamic viscosity mu and conductivity kappa.
 *   tau_ij = mu (dv_i/dx_j + dv_j/dx_i) - (2/3) mu delta_ij div v,
 *   F^v_d  = (0, tau_1d, ..., tau_Dd, sum_j v_j tau_jd + kappa dT/dx_d).
 * Inputs per point: the conservative state U (v = m / rho), the velocity
 * gradient G with field i*D + j holding dv_i/dx_j, and the temperature
 * gradient gT (D fields).  Output in the flux tensor's layout (field
 * r*D + d). */
int oracle_viscous_flux(int dim, double mu, double kappa, const double *U, int64_t ldU,
                        const double *G, int64_t ldG, const double *gT, int64_t ldT,
                        double *Fv, int64_t ldF, int64_t n)
{
    int64_t i;
    int a, b, d;
    double tau[3][3], v[3];
    if (!dim_ok(dim))
        return -1;
    for (i = 0; i < n; ++i) {
        double rho = U[0 * ldU + i];
        double div = 0.0;
        for (a = 0; a < dim; ++a) {
            v[a] = U[(1 + a) * ldU + i] / rho;
            div = div + G[(a * dim + a) * ldG + i];
        }
        for (a = 0; a < dim; ++a)
            for (b = 0; b < dim; ++b) {
                double t = mu * (G[(a * dim + b) * ldG + i] + G[(b * dim + a) * ldG + i]);
                if (a == b)
                    t = t - 2.0 / 3.0 * mu * div;
                tau[a][b] = t;
            }
        for (d = 0; d < dim; ++d) {
            double work = 0.0;
            Fv[(0 * dim + d) * ldF + i] = 0.0;
            for (a = 0; a < dim; ++a) {
                Fv[((1 + a) * dim + d) * ldF + i] = tau[a][d];
                work = work + v[a] * tau[a][d];
            }
            Fv[((dim + 1) * dim + d) * ldF + i] = work + kappa * gT[d * ldT + i];
        }
    }
    return 0;
}
