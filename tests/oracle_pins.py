"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises on failure.
None of them re-types the oracle's formulas; they check it against
  * closed forms built on a different route (temperature, enthalpy),
  * textbook special cases (the 1D and 3D x-direction Jacobians),
  * invariants of the Euler equations (Galilean boosts, rotations, axis
    permutations, homogeneity F = A U, dimension embedding),
  * library routines (numpy eigenvalues) and brute force (finite
    differences of the oracle's own flux and invariants).
``tests/test_oracle_mutations.py`` plants mistakes in copies of the oracle
and checks that these pins catch every one of them.

Gas model used by the closed forms (Sec. 2.2, "Variables": perfect gas,
gamma = c_p/c_v): c_v = 1/(gamma-1), c_p = gamma/(gamma-1), so that the gas
constant R = c_p - c_v = 1, p = rho R T, e = c_v T, h = c_p T, c^2 = gamma R T.
"""
from __future__ import annotations

import numpy as np

GAMMAS = (1.4, 5.0 / 3.0, 1.1)


# ---------------------------------------------------------------- helpers
def thermal_state(dim, n, seed, gamma):
    """Conservative state built from (rho, v, T) without the oracle:
    E = rho (c_v T + |v|^2/2), the total energy per unit volume."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, n)
    v = rng.normal(0.0, 0.6, (dim, n))
    T = rng.uniform(0.3, 1.5, n)
    cv = 1.0 / (gamma - 1.0)
    q = (v * v).sum(axis=0)
    E = rho * (cv * T + 0.5 * q)
    U = np.vstack([rho[None], rho[None] * v, E[None]])
    return U, rho, v, T


def rel(a, b, scale=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(np.max(np.abs(b)), scale, 1e-300)
    return float(np.max(np.abs(a - b)) / den)


def close(a, b, tol, what, scale=0.0):
    """max |a - b| <= tol * max(max |b|, scale); NaN never passes."""
    e = rel(a, b, scale)
    if not (e <= tol):
        raise AssertionError(f"{what}: relative error {e:.3e} > {tol:.1e}")


def flux_columns(F, dim, i):
    """F_d (K-vector) of point i for every d, as a (K, D) matrix."""
    K = dim + 2
    return np.array([[F[r * dim + d, i] for d in range(dim)] for r in range(K)])


def fd_jacobian(o, dim, gamma, U, fun, h_rel=1e-3):
    """Brute-force d fun(U) / dU by central differences with one Richardson
    step.  fun maps U (K, n) to an (m, n) array; the result is (n, m, K)."""
    K = dim + 2
    n = U.shape[1]
    out = None
    for k in range(K):
        scale = np.maximum(np.abs(U[k]), 1.0)
        h = h_rel * scale

        def d(hh):
            Up = U.copy()
            Um = U.copy()
            Up[k] += hh
            Um[k] -= hh
            return (fun(Up) - fun(Um)) / (2.0 * hh)

        g = (4.0 * d(0.5 * h) - d(h)) / 3.0
        if out is None:
            out = np.zeros((n, g.shape[0], K))
        out[:, :, k] = g.T
    return out


# ---------------------------------------------------------------- pins
def pin_worked_state(o):
    """1D, gamma = 7/5, rho = 7/5, u = 1/2, p = 1 (T = 5/7, c_v = 5/2):
    E = rho c_v T + rho u^2/2 = 5/2 + 7/40 = 107/40; c = sqrt(gamma R T) = 1;
    H = c^2/(gamma-1) + u^2/2 = 21/8; F = (rho u, rho u^2 + p, rho u H)
    = (7/10, 27/20, 147/80); w = u -/+ 2c/(gamma-1) = (-9/2, 11/2)."""
    g = 1.4
    U = np.array([[1.4], [0.7], [107.0 / 40.0]])
    V = o.cons2prim(1, g, U)
    close(V[:, 0], [1.4, 0.5, 1.0], 1e-14, "worked state cons2prim")
    p, c = o.eos(1, g, U)
    close(p, [1.0], 1e-14, "worked state p")
    close(c, [1.0], 1e-14, "worked state c")
    F = o.flux(1, g, U)
    close(F[:, 0], [0.7, 27.0 / 20.0, 147.0 / 80.0], 1e-14, "worked state flux")
    R = o.riemann_invariants(1, g, U)
    close(R[:2, 0], [-4.5, 5.5], 1e-14, "worked state Riemann invariants")
    U2 = o.prim2cons(1, g, np.array([[1.4], [0.5], [1.0]]))
    close(U2[:, 0], U[:, 0], 1e-14, "worked state prim2cons")


def pin_temperature_route(o):
    """p = rho R T, c^2 = gamma R T, momentum flux rho v_i v_d + p delta_id,
    energy flux = mass flux times total enthalpy c_p T + |v|^2/2."""
    for dim in (1, 2, 3):
        for g in GAMMAS:
            U, rho, v, T = thermal_state(dim, 64, 10 + dim, g)
            cp = g / (g - 1.0)
            q = (v * v).sum(axis=0)
            V = o.cons2prim(dim, g, U)
            close(V[0], rho, 1e-15, "cons2prim rho")
            close(V[1:dim + 1], v, 1e-14, "cons2prim v")
            close(V[dim + 1], rho * T, 1e-13, "cons2prim p = rho R T")
            p, c = o.eos(dim, g, U)
            close(p, rho * T, 1e-13, "eos p = rho R T")
            close(c, np.sqrt(g * T), 1e-13, "eos c = sqrt(gamma R T)")
            F = o.flux(dim, g, U)
            for d in range(dim):
                close(F[0 * dim + d], rho * v[d], 1e-14, "mass flux")
                for i in range(dim):
                    ref = rho * v[i] * v[d] + (rho * T if i == d else 0.0)
                    close(F[(1 + i) * dim + d], ref, 1e-13, "momentum flux")
                close(F[(dim + 1) * dim + d], rho * v[d] * (cp * T + 0.5 * q), 1e-13,
                      "energy flux = mass flux * total enthalpy")


def pin_v_mag2(o):
    """|v|^2 of the temperature-route states (v known), a worked value, and
    frame indifference (rotation) and a Galilean boost."""
    for dim in (1, 2, 3):
        U, rho, v, T = thermal_state(dim, 64, 15 + dim, 1.4)
        close(o.v_mag2(dim, U), (v * v).sum(axis=0), 1e-14, "v_mag2 = |v|^2")
    U = np.array([[2.0], [2.0], [4.0], [4.0], [50.0]])
    close(o.v_mag2(3, U), [9.0], 1e-15, "v_mag2 worked value (4 + 16 + 16) / 4")
    rng = np.random.default_rng(17)
    U, rho, v, T = thermal_state(3, 32, 18, 1.4)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    UQ = U.copy()
    UQ[1:4] = Q @ U[1:4]
    close(o.v_mag2(3, UQ), o.v_mag2(3, U), 1e-14, "v_mag2 rotation")
    w = rng.normal(size=(3, 1))
    Ub = U.copy()
    Ub[1:4] = U[1:4] + rho * w
    close(o.v_mag2(3, Ub), ((v + w) ** 2).sum(axis=0), 1e-13, "v_mag2 boost")


def pin_roundtrip(o):
    for dim in (1, 2, 3):
        for g in GAMMAS:
            U, _, _, _ = thermal_state(dim, 64, 20 + dim, g)
            close(o.prim2cons(dim, g, o.cons2prim(dim, g, U)), U, 1e-14, "cons->prim->cons")
            V = o.cons2prim(dim, g, U)
            close(o.cons2prim(dim, g, o.prim2cons(dim, g, V)), V, 1e-14, "prim->cons->prim")


def pin_galilean(o):
    """A boost by w maps (rho, m, E) to (rho, m + rho w, E + m.w + rho|w|^2/2);
    pressure, sound speed and entropy are unchanged, velocity shifts by w,
    and F_d - v_d U = (0, p e_d, p v_d) in every frame."""
    rng = np.random.default_rng(5)
    for dim in (1, 2, 3):
        g = 1.4
        U, rho, v, T = thermal_state(dim, 64, 30 + dim, g)
        w = rng.normal(0.0, 1.0, (dim, 1))
        m = U[1:dim + 1]
        Ub = U.copy()
        Ub[1:dim + 1] = m + rho * w
        Ub[dim + 1] = U[dim + 1] + (m * w).sum(axis=0) + 0.5 * rho * (w * w).sum()
        p0, c0 = o.eos(dim, g, U)
        p1, c1 = o.eos(dim, g, Ub)
        close(p1, p0, 1e-13, "boosted p")
        close(c1, c0, 1e-13, "boosted c")
        close(o.cons2prim(dim, g, Ub)[1:dim + 1], v + w, 1e-13, "boosted v")
        R0 = o.riemann_invariants(dim, g, U)
        R1 = o.riemann_invariants(dim, g, Ub)
        close(R1[2 * dim], R0[2 * dim], 1e-13, "boosted entropy")
        for d in range(dim):
            close(R1[2 * d + 1] - R1[2 * d], R0[2 * d + 1] - R0[2 * d], 1e-13,
                  "boosted w+ - w-")
        F = o.flux(dim, g, Ub)
        vb = v + w
        for d in range(dim):
            for r in range(dim + 2):
                ref = np.zeros_like(rho)
                if 1 <= r <= dim and r - 1 == d:
                    ref = p0
                if r == dim + 1:
                    ref = p0 * vb[d]
                close(F[r * dim + d] - vb[d] * Ub[r], ref, 1e-12, "pressure part of flux",
                      scale=np.max(np.abs(F[r * dim + d])))


def pin_homogeneity(o):
    """The perfect-gas flux is homogeneous of degree one, so A_d(U) U = F_d(U)."""
    for dim in (1, 2, 3):
        for g in GAMMAS:
            U, _, _, _ = thermal_state(dim, 32, 40 + dim, g)
            F = o.flux(dim, g, U)
            A = o.flux_jacobian(dim, g, U)
            for d in range(dim):
                AU = np.einsum("nrc,cn->rn", A[d], U)
                Fd = np.array([F[r * dim + d] for r in range(dim + 2)])
                close(AU, Fd, 1e-13, "A U = F")


def pin_jacobian_fd(o):
    for dim in (1, 2, 3):
        g = 1.4
        U, _, _, _ = thermal_state(dim, 16, 50 + dim, g)
        J = fd_jacobian(o, dim, g, U, lambda X: o.flux(dim, g, X))
        A = o.flux_jacobian(dim, g, U)
        for d in range(dim):
            rows = [r * dim + d for r in range(dim + 2)]
            for i in range(U.shape[1]):
                close(A[d, i], J[i][rows], 1e-8, "Jacobian vs finite differences")


def pin_eigenvalues(o):
    """Eigenvalues of A_d are v_d - c, v_d (D times), v_d + c."""
    for dim in (1, 2, 3):
        for g in GAMMAS:
            U, rho, v, T = thermal_state(dim, 16, 60 + dim, g)
            c = np.sqrt(g * T)
            A = o.flux_jacobian(dim, g, U)
            for d in range(dim):
                for i in range(U.shape[1]):
                    ev = np.sort(np.linalg.eigvals(A[d, i]).real)
                    ref = np.sort([v[d, i] - c[i]] + [v[d, i]] * dim + [v[d, i] + c[i]])
                    close(ev, ref, 1e-7, "eigenvalues of A_d")


def pin_eigenvectors(o):
    """Textbook right eigenvectors: r(-/+) = (1, v -/+ c e_d, H -/+ v_d c),
    r_0 = (1, v, |v|^2/2) and r_j = (0, e_j, v_j) for j != d, with
    H = c_p T + |v|^2/2."""
    for dim in (1, 2, 3):
        g = 1.4
        U, rho, v, T = thermal_state(dim, 16, 70 + dim, g)
        c = np.sqrt(g * T)
        H = g / (g - 1.0) * T + 0.5 * (v * v).sum(axis=0)
        A = o.flux_jacobian(dim, g, U)
        K = dim + 2
        for d in range(dim):
            for i in range(U.shape[1]):
                vi = v[:, i]
                ed = np.eye(dim)[d]
                vecs = []
                for sgn in (-1.0, 1.0):
                    r = np.concatenate([[1.0], vi + sgn * c[i] * ed, [H[i] + sgn * vi[d] * c[i]]])
                    vecs.append((r, vi[d] + sgn * c[i]))
                vecs.append((np.concatenate([[1.0], vi, [0.5 * vi @ vi]]), vi[d]))
                for j in range(dim):
                    if j != d:
                        vecs.append((np.concatenate([[0.0], np.eye(dim)[j], [vi[j]]]), vi[d]))
                for r, lam in vecs:
                    close(A[d, i] @ r, lam * r, 1e-13, "A r = lambda r")
                assert len(vecs) == K


def pin_textbook_jacobian(o):
    """1D: [[0,1,0],[(g-3)u^2/2,(3-g)u,g-1],[u((g-1)u^2/2-H),H-(g-1)u^2,g u]];
    3D, x-direction, with phi = (g-1)|v|^2/2 (standard textbook form)."""
    g = 1.4
    U, rho, v, T = thermal_state(1, 8, 80, g)
    H = g / (g - 1.0) * T + 0.5 * v[0] ** 2
    A = o.flux_jacobian(1, g, U)
    for i in range(U.shape[1]):
        u = v[0, i]
        ref = np.array([[0.0, 1.0, 0.0],
                        [(g - 3.0) * u * u / 2.0, (3.0 - g) * u, g - 1.0],
                        [u * ((g - 1.0) * u * u / 2.0 - H[i]), H[i] - (g - 1.0) * u * u, g * u]])
        close(A[0, i], ref, 1e-13, "1D textbook Jacobian")
    U, rho, v, T = thermal_state(3, 8, 81, g)
    A = o.flux_jacobian(3, g, U)
    for i in range(U.shape[1]):
        u, vv, w = v[:, i]
        q = u * u + vv * vv + w * w
        phi = (g - 1.0) * q / 2.0
        H = g / (g - 1.0) * T[i] + q / 2.0
        g1 = g - 1.0
        ref = np.array([
            [0.0, 1.0, 0.0, 0.0, 0.0],
            [phi - u * u, (3.0 - g) * u, -g1 * vv, -g1 * w, g1],
            [-u * vv, vv, u, 0.0, 0.0],
            [-u * w, w, 0.0, u, 0.0],
            [u * (phi - H), H - g1 * u * u, -g1 * u * vv, -g1 * u * w, g * u]])
        close(A[0, i], ref, 1e-13, "3D textbook x-Jacobian")


def _perm_matrix(dim, a, b):
    K = dim + 2
    P = np.eye(K)
    P[[1 + a, 1 + b]] = P[[1 + b, 1 + a]]
    return P


def pin_axis_permutation(o):
    """Swapping axes a and b: F_b(U) = P F_a(P U), A_b(U) = P A_a(P U) P,
    and the Riemann invariants of b are those of a for P U."""
    g = 1.4
    for dim in (2, 3):
        U, _, _, _ = thermal_state(dim, 32, 90 + dim, g)
        for a in range(dim):
            for b in range(dim):
                if a == b:
                    continue
                P = _perm_matrix(dim, a, b)
                PU = P @ U
                F = o.flux(dim, g, U)
                FP = o.flux(dim, g, PU)
                Fb = np.array([F[r * dim + b] for r in range(dim + 2)])
                Fa = np.array([FP[r * dim + a] for r in range(dim + 2)])
                close(Fb, P @ Fa, 1e-14, "axis permutation of F")
                A = o.flux_jacobian(dim, g, U)
                AP = o.flux_jacobian(dim, g, PU)
                for i in range(U.shape[1]):
                    close(A[b, i], P @ AP[a, i] @ P, 1e-14, "axis permutation of A")
                R = o.riemann_invariants(dim, g, U)
                RP = o.riemann_invariants(dim, g, PU)
                close(R[2 * b:2 * b + 2], RP[2 * a:2 * a + 2], 1e-14, "axis permutation of w")


def pin_dimension_embedding(o):
    """A state with zero momentum in the last axis behaves as the
    lower-dimensional state: every output restricted to the remaining axes
    equals the lower-dimensional output."""
    g = 1.4
    for dim in (2, 3):
        lo = dim - 1
        Ulo, _, _, _ = thermal_state(lo, 32, 100 + dim, g)
        U = np.vstack([Ulo[:lo + 1], np.zeros((1, Ulo.shape[1])), Ulo[lo + 1:]])
        keep = list(range(lo + 1)) + [dim + 1]
        close(o.cons2prim(dim, g, U)[keep], o.cons2prim(lo, g, Ulo), 1e-15, "embed cons2prim")
        close(np.array(o.eos(dim, g, U)), np.array(o.eos(lo, g, Ulo)), 1e-15, "embed eos")
        F = o.flux(dim, g, U)
        Flo = o.flux(lo, g, Ulo)
        for d in range(lo):
            for ri, r in enumerate(keep):
                close(F[r * dim + d], Flo[ri * lo + d], 1e-15, "embed flux")
        A = o.flux_jacobian(dim, g, U)
        Alo = o.flux_jacobian(lo, g, Ulo)
        for d in range(lo):
            close(A[d][:, keep][:, :, keep], Alo[d], 1e-15, "embed Jacobian")
        R = o.riemann_invariants(dim, g, U)
        Rlo = o.riemann_invariants(lo, g, Ulo)
        close(R[:2 * lo], Rlo[:2 * lo], 1e-15, "embed w")
        close(R[2 * dim], Rlo[2 * lo], 1e-15, "embed s")


def _rotation(dim, rng):
    M = rng.normal(size=(dim, dim))
    Q, _ = np.linalg.qr(M)
    return Q


def pin_rotation(o):
    """Rotating the momentum by Q rotates the mass and energy flux vectors
    by Q and the momentum flux tensor by Q . Q^T (frame indifference)."""
    rng = np.random.default_rng(7)
    g = 1.4
    for dim in (2, 3):
        U, _, _, _ = thermal_state(dim, 16, 110 + dim, g)
        Q = _rotation(dim, rng)
        UQ = U.copy()
        UQ[1:dim + 1] = Q @ U[1:dim + 1]
        F = o.flux(dim, g, U)
        FQ = o.flux(dim, g, UQ)
        for i in range(U.shape[1]):
            M = flux_columns(F, dim, i)
            MQ = flux_columns(FQ, dim, i)
            close(MQ[0], Q @ M[0], 1e-13, "rotated mass flux")
            close(MQ[1:dim + 1], Q @ M[1:dim + 1] @ Q.T, 1e-13, "rotated momentum flux")
            close(MQ[dim + 1], Q @ M[dim + 1], 1e-13, "rotated energy flux")


def pin_at_rest(o):
    """At rest F_d = p e_{1+d} and A_d has eigenvalues -c, 0 (D times), +c."""
    g = 1.4
    for dim in (1, 2, 3):
        U, rho, v, T = thermal_state(dim, 8, 120 + dim, g)
        U[1:dim + 1] = 0.0
        U[dim + 1] = rho * T / (g - 1.0)
        F = o.flux(dim, g, U)
        for d in range(dim):
            for r in range(dim + 2):
                ref = rho * T if r == 1 + d else np.zeros_like(rho)
                close(F[r * dim + d], ref, 1e-14, "flux at rest")


def pin_riemann_isentrope(o):
    """States on one isentrope p = k rho^gamma share the entropy s = k."""
    for dim in (1, 2, 3):
        for g in GAMMAS:
            rng = np.random.default_rng(130 + dim)
            n = 32
            rho = rng.uniform(0.5, 2.0, n)
            k = 0.8
            T = k * rho ** g / rho  # p = rho T
            cv = 1.0 / (g - 1.0)
            v = rng.normal(0, 0.5, (dim, n))
            U = np.vstack([rho[None], rho[None] * v, (rho * (cv * T + 0.5 * (v * v).sum(0)))[None]])
            R = o.riemann_invariants(dim, g, U)
            close(R[2 * dim], np.full(n, k), 1e-13, "entropy on an isentrope")
            c = np.sqrt(g * T)
            for d in range(dim):
                close(R[2 * d], v[d] - 2 * c / (g - 1), 1e-13, "w- on an isentrope")
                close(R[2 * d + 1], v[d] + 2 * c / (g - 1), 1e-13, "w+ on an isentrope")


def pin_riemann_characteristic(o):
    """Brute-force gradients of the invariants are left eigenvectors of the
    Jacobian: grad s (A_d - v_d I) = 0, and grad w+-_d lies in the span of
    the left eigenvectors for v_d +- c and v_d, i.e.
    grad w+-_d (A_d - (v_d +- c) I)(A_d - v_d I) = 0."""
    g = 1.4
    for dim in (1, 2, 3):
        U, rho, v, T = thermal_state(dim, 8, 140 + dim, g)
        c = np.sqrt(g * T)
        G = fd_jacobian(o, dim, g, U, lambda X: o.riemann_invariants(dim, g, X))
        A = o.flux_jacobian(dim, g, U)
        K = dim + 2
        I = np.eye(K)
        for d in range(dim):
            for i in range(U.shape[1]):
                Ad = A[d, i]
                scale = np.linalg.norm(Ad, np.inf)
                gs = G[i][2 * dim]
                res = gs @ (Ad - v[d, i] * I)
                assert np.max(np.abs(res)) <= 1e-6 * np.max(np.abs(gs)) * scale, "grad s"
                for sgn, row in ((-1.0, 2 * d), (1.0, 2 * d + 1)):
                    gw = G[i][row]
                    res = gw @ (Ad - (v[d, i] + sgn * c[i]) * I) @ (Ad - v[d, i] * I)
                    assert np.max(np.abs(res)) <= 1e-6 * np.max(np.abs(gw)) * scale ** 2, "grad w"


def pin_characteristic_transform(o):
    """W_dir carries (w-_dir, s, tangential v ascending, w+_dir), and
    char2cons inverts cons2char."""
    for dim in (1, 2, 3):
        for g in GAMMAS:
            U, rho, v, T = thermal_state(dim, 32, 150 + dim, g)
            R = o.riemann_invariants(dim, g, U)
            for d in range(dim):
                W = o.cons2char(dim, d, g, U)
                close(W[0], R[2 * d], 1e-15, "W[0] = w-")
                close(W[dim + 1], R[2 * d + 1], 1e-15, "W[K-1] = w+")
                close(W[1], R[2 * dim], 1e-15, "W[1] = s")
                tang = [j for j in range(dim) if j != d]
                for slot, j in enumerate(tang):
                    close(W[2 + slot], v[j], 1e-14, "tangential velocity")
                close(o.char2cons(dim, d, g, W), U, 1e-12, "char2cons o cons2char")


def pin_adjoint_fd(o):
    """Ubar = d/dU sum(w . F(U)) by brute-force central differences, and the
    sum over directions equals the per-direction adjoints added up."""
    g = 1.4
    for dim in (1, 2, 3):
        U, _, _, _ = thermal_state(dim, 32, 160 + dim, g)
        rng = np.random.default_rng(161 + dim)
        w = rng.normal(size=((dim + 2) * dim, U.shape[1]))
        Ub = o.flux_adjoint(dim, -1, g, U, w)
        G = fd_jacobian(o, dim, g, U, lambda X: (w * o.flux(dim, g, X)).sum(axis=0, keepdims=True))
        close(Ub, G[:, 0, :].T, 1e-8, "adjoint vs finite differences")
        tot = np.zeros_like(U)
        for d in range(dim):
            wd = np.array([w[r * dim + d] for r in range(dim + 2)])
            tot += o.flux_adjoint(dim, d, g, U, wd)
        close(tot, Ub, 1e-13, "adjoint: all directions = sum of single directions")


def pin_characteristic_decomposition(o):
    """A_d R_d = R_d diag(v_d - c, v_d .., v_d + c) and L_d A_d = diag(..) L_d
    against the (separately pinned) Jacobian; L_d R_d = I; char_apply is
    the product with L_d or R_d."""
    for dim in (1, 2, 3):
        for g in GAMMAS:
            U, rho, v, T = thermal_state(dim, 16, 170 + dim, g)
            c = np.sqrt(g * T)
            A = o.flux_jacobian(dim, g, U)
            L, R = o.eigenvectors(dim, g, U)
            K = dim + 2
            for d in range(dim):
                for i in range(U.shape[1]):
                    lam = np.diag([v[d, i] - c[i]] + [v[d, i]] * dim + [v[d, i] + c[i]])
                    scale = np.linalg.norm(A[d, i], np.inf) * np.linalg.norm(R[d, i], np.inf)
                    close(A[d, i] @ R[d, i], R[d, i] @ lam, 1e-13, "A R = R Lambda", scale=scale)
                    close(L[d, i] @ A[d, i], lam @ L[d, i], 1e-12, "L A = Lambda L",
                          scale=np.linalg.norm(A[d, i], np.inf) * np.linalg.norm(L[d, i], np.inf))
                    close(L[d, i] @ R[d, i], np.eye(K), 1e-13, "L R = I")
                    # column order: r-, entropy, shear (ascending), r+
                    assert R[d, i][0, 0] == 1.0 and R[d, i][0, 1] == 1.0 and R[d, i][0, K - 1] == 1.0
            rng = np.random.default_rng(180 + dim)
            X = rng.normal(size=(K, U.shape[1]))
            for d in range(dim):
                YL = o.char_apply(dim, d, 0, g, U, X)
                YR = o.char_apply(dim, d, 1, g, U, X)
                close(YL, np.einsum("nrc,cn->rn", L[d], X), 1e-14, "char_apply L")
                close(YR, np.einsum("nrc,cn->rn", R[d], X), 1e-14, "char_apply R")
                close(o.char_apply(dim, d, 1, g, U, YL), X, 1e-12, "R L = I")


def _state_pairs(dim, n, seed, gamma):
    """Two independent thermal states per point, built without the oracle."""
    UL = thermal_state(dim, n, seed, gamma)[0]
    UR = thermal_state(dim, n, seed + 1000, gamma)[0]
    # a few pairs far apart: strong density and temperature jumps
    UR[:, : n // 4] *= np.linspace(0.05, 20.0, n // 4)[None]
    return UL, UR


def pin_roe_property(o):
    """Roe's defining property: the Jacobian at the averaged state maps the
    jump in state onto the jump in flux exactly, A_d(U^)(U_R - U_L) =
    F_d(U_R) - F_d(U_L), for every direction d.  This fixes the averaged
    velocity and total enthalpy."""
    for g in GAMMAS:
        for dim in (1, 2, 3):
            UL, UR = _state_pairs(dim, 64, 40 + dim, g)
            Uh = o.roe_average(dim, g, UL, UR)
            A = o.flux_jacobian(dim, g, Uh)
            dF = o.flux(dim, g, UR) - o.flux(dim, g, UL)
            dU = UR - UL
            for d in range(dim):
                lhs = np.einsum("nrc,cn->rn", A[d], dU)
                rhs = dF[[r * dim + d for r in range(dim + 2)]]
                for i in range(dU.shape[1]):
                    close(lhs[:, i], rhs[:, i], 1e-12, f"Roe property {dim}D d={d}",
                          scale=np.abs(A[d, i]).max() * np.abs(dU[:, i]).max())


def pin_roe_product_rule(o):
    """The averaged density makes the discrete product rule exact for the
    momentum: (rho v)_R - (rho v)_L = rho^ (v_R - v_L) + v^ (rho_R - rho_L)
    (v^ is pinned by the Roe property), which fixes rho^ = sqrt(rho_L rho_R)
    without restating it."""
    for g in GAMMAS:
        for dim in (1, 2, 3):
            UL, UR = _state_pairs(dim, 64, 50 + dim, g)
            Uh = o.roe_average(dim, g, UL, UR)
            rho = Uh[0]
            v = Uh[1:dim + 1] / rho
            vL = UL[1:dim + 1] / UL[0]
            vR = UR[1:dim + 1] / UR[0]
            for k in range(dim):
                lhs = UR[1 + k] - UL[1 + k]
                rhs = rho * (vR[k] - vL[k]) + v[k] * (UR[0] - UL[0])
                scale = np.abs(UR[1 + k]) + np.abs(UL[1 + k])
                close(lhs / scale, rhs / scale, 1e-12, f"product rule {dim}D k={k}", scale=1.0)


def pin_roe_consistency(o):
    """Between a state and itself the average is that state; the average
    does not depend on which state is called left; and in the sound speed
    of the averaged state, c^2 = (gamma-1)(H^ - |v^|^2/2), lies between the
    limits set by the two states' enthalpies (H^ is a convex combination)."""
    for g in GAMMAS:
        for dim in (1, 2, 3):
            UL, UR = _state_pairs(dim, 64, 60 + dim, g)
            close(o.roe_average(dim, g, UL, UL), UL, 1e-14, "average of equal states")
            close(o.roe_average(dim, g, UL, UR), o.roe_average(dim, g, UR, UL), 1e-15, "symmetry")
            Uh = o.roe_average(dim, g, UL, UR)
            p = o.eos(dim, g, Uh)[0]
            H = (Uh[-1] + p) / Uh[0]
            HL = (UL[-1] + o.eos(dim, g, UL)[0]) / UL[0]
            HR = (UR[-1] + o.eos(dim, g, UR)[0]) / UR[0]
            lo, hi = np.minimum(HL, HR), np.maximum(HL, HR)
            assert np.all(H >= lo * (1 - 1e-14)) and np.all(H <= hi * (1 + 1e-14)), "H^ outside [H_L, H_R]"


EOS_CASES = ((0, (3.5, 2.5)), (0, (1.0, 0.6)), (1, (4.4, 0.0, 1.0)), (1, (4.4, 3.0, 0.7)),
             (1, (1.9, 0.4, 2.5)))


def _eos_states(dim, n, seed, eos, params):
    """Admissible states for an EOS case: rho in [0.5, 2], v ~ N(0, 0.6^2),
    and an internal energy that keeps p + p_inf > 0."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, n)
    v = rng.normal(0.0, 0.6, (dim, n))
    pinf = params[1] if eos == 1 else 0.0
    e = pinf / rho + rng.uniform(0.5, 3.0, n)
    E = rho * (e + 0.5 * (v * v).sum(axis=0))
    return np.vstack([rho[None], rho[None] * v, E[None]]), rho, e


def _with_rho_e(U, dim, rho, e):
    """The state with density rho and specific internal energy e, keeping
    the velocity of U."""
    v = U[1:dim + 1] / U[0]
    E = rho * (e + 0.5 * (v * v).sum(axis=0))
    return np.vstack([rho[None], rho[None] * v, E[None]])


def pin_eos_perfect_gas_thermal(o):
    """Perfect gas with c_p, c_v (R = c_p - c_v need not be 1): states built
    from (rho, v, T) with e = c_v T must give back T, p = rho R T and
    c^2 = gamma R T; the same gas through the gamma-only EOS entry gives the
    same p and c."""
    for cp, cv in ((3.5, 2.5), (1.0, 0.6), (5.0, 3.0)):
        for dim in (1, 2, 3):
            rng = np.random.default_rng(70 + dim)
            n = 50
            rho = rng.uniform(0.5, 2.0, n)
            v = rng.normal(0.0, 0.6, (dim, n))
            T = rng.uniform(0.3, 1.5, n)
            U = np.vstack([rho[None], rho[None] * v, (rho * (cv * T + 0.5 * (v * v).sum(axis=0)))[None]])
            p, c, Tt = o.eos_pvt(dim, 0, (cp, cv), U)
            close(Tt, T, 1e-14, "T = e / c_v")
            close(p, rho * (cp - cv) * T, 1e-14, "p = rho R T")
            close(c * c, cp / cv * (cp - cv) * T, 1e-14, "c^2 = gamma R T")
            p2, c2 = o.eos(dim, cp / cv, U)
            close(p, p2, 1e-14, "same gas, gamma-only entry (p)")
            close(c, c2, 1e-14, "same gas, gamma-only entry (c)")


def pin_eos_stiffened_reduces(o):
    """With p_inf = 0 the stiffened gas is the perfect gas with c_p = gamma c_v."""
    for g, cv in ((1.4, 2.5), (4.4, 0.7)):
        for dim in (1, 2, 3):
            U = _eos_states(dim, 40, 80 + dim, 0, (g * cv, cv))[0]
            a = o.eos_pvt(dim, 1, (g, 0.0, cv), U)
            b = o.eos_pvt(dim, 0, (g * cv, cv), U)
            for x, y, what in zip(a, b, "pcT"):
                close(x, y, 1e-14, f"p_inf = 0 reduction ({what})")


def pin_eos_sound_speed_fd(o):
    """c^2 is the isentropic derivative (dp/drho)_e + (p/rho^2)(dp/de)_rho of
    each EOS's own p(rho, e), taken here by central differences."""
    for eos, prm in EOS_CASES:
        dim = 2
        U, rho, e = _eos_states(dim, 40, 90, eos, prm)
        p, c, _ = o.eos_pvt(dim, eos, prm, U)
        h = 1e-5
        pr = (o.eos_pvt(dim, eos, prm, _with_rho_e(U, dim, rho * (1 + h), e))[0]
              - o.eos_pvt(dim, eos, prm, _with_rho_e(U, dim, rho * (1 - h), e))[0]) / (2 * h * rho)
        pe = (o.eos_pvt(dim, eos, prm, _with_rho_e(U, dim, rho, e * (1 + h)))[0]
              - o.eos_pvt(dim, eos, prm, _with_rho_e(U, dim, rho, e * (1 - h)))[0]) / (2 * h * e)
        close(c * c, pr + p / rho ** 2 * pe, 1e-7, f"isentropic c^2, eos {eos} {prm}")


def pin_eos_thermodynamic_consistency(o):
    """p(rho, e) and T(rho, e) of one EOS must be consistent (they come from
    one free energy): rho^2 (dT/drho)_e = T (dp/de)_rho - p (dT/de)_rho.
    Checked by central differences; this ties T's density dependence to
    p's (for the stiffened gas, the p_inf terms of both)."""
    for eos, prm in EOS_CASES:
        dim = 1
        U, rho, e = _eos_states(dim, 40, 95, eos, prm)
        p, _, T = o.eos_pvt(dim, eos, prm, U)
        h = 1e-5

        def at(r, ee):
            return o.eos_pvt(dim, eos, prm, _with_rho_e(U, dim, r, ee))

        Tr = (at(rho * (1 + h), e)[2] - at(rho * (1 - h), e)[2]) / (2 * h * rho)
        Te = (at(rho, e * (1 + h))[2] - at(rho, e * (1 - h))[2]) / (2 * h * e)
        pe = (at(rho, e * (1 + h))[0] - at(rho, e * (1 - h))[0]) / (2 * h * e)
        lhs = rho ** 2 * Tr
        rhs = T * pe - p * Te
        scale = np.abs(T * pe) + np.abs(p * Te) + 1.0
        close(lhs / scale, rhs / scale, 1e-8, f"consistency, eos {eos} {prm}", scale=1.0)


def _visc_inputs(dim, n, seed):
    rng = np.random.default_rng(seed)
    U = thermal_state(dim, n, seed, 1.4)[0]
    return U, rng.normal(size=(dim * dim, n)), rng.normal(size=(dim, n))


def _visc_columns(Fv, dim, i):
    """(K, D) matrix of point i: column d is F^v_d."""
    return flux_columns(Fv, dim, i)


def pin_viscous_couette(o):
    """Plane Couette flow (textbook): velocity (u, 0, 0) with the only
    gradient dv_x/dy = s gives tau_xy = tau_yx = mu s, no normal stresses,
    and the energy flux u mu s across y; heat flux kappa dT/dx_d adds to the
    energy row."""
    mu, kappa = 0.7, 0.3
    for dim in (2, 3):
        rng = np.random.default_rng(dim)
        n = 8
        rho = rng.uniform(0.5, 2.0, n)
        u = rng.normal(size=n)
        s = rng.normal(size=n)
        U = np.zeros((dim + 2, n))
        U[0], U[1], U[-1] = rho, rho * u, 3.0
        G = np.zeros((dim * dim, n))
        G[0 * dim + 1] = s
        gT = rng.normal(size=(dim, n))
        Fv = o.viscous_flux(dim, mu, kappa, U, G, gT)
        for i in range(n):
            M = _visc_columns(Fv, dim, i)
            want = np.zeros((dim + 2, dim))
            want[1, 1] = want[2, 0] = mu * s[i]
            want[dim + 1, :] = kappa * gT[:, i]
            want[dim + 1, 1] += u[i] * mu * s[i]
            close(M, want, 1e-14, f"Couette {dim}D", scale=1.0)


def pin_viscous_rigid_rotation(o):
    """A rigid rotation (antisymmetric velocity gradient) does no viscous
    work and carries no stress: only the heat flux remains."""
    for dim in (2, 3):
        U, G, gT = _visc_inputs(dim, 20, 110 + dim)
        Gm = G.reshape(dim, dim, -1)
        G = (Gm - Gm.transpose(1, 0, 2)).reshape(dim * dim, -1)
        Fv = o.viscous_flux(dim, 0.9, 0.4, U, G, gT)
        want = np.zeros_like(Fv)
        for d in range(dim):
            want[(dim + 1) * dim + d] = 0.4 * gT[d]
        close(Fv, want, 1e-14, f"rigid rotation {dim}D", scale=1.0)


def pin_viscous_stokes(o):
    """Stokes' hypothesis: in 3D the stress is trace-free, so a pure
    expansion (gradient a I) carries no stress; the stress is symmetric for
    any gradient; F^v is linear in (mu, kappa)."""
    U, G, gT = _visc_inputs(3, 30, 120)
    Fv = o.viscous_flux(3, 0.8, 0.5, U, G, gT)
    for i in range(30):
        tau = _visc_columns(Fv, 3, i)[1:4]
        close(tau, tau.T, 1e-15, "stress symmetry", scale=np.abs(tau).max())
        close(np.trace(tau), 0.0, 1e-14, "trace-free stress", scale=np.abs(tau).max())
    a = np.random.default_rng(5).normal(size=30)
    Gi = np.zeros((9, 30))
    for k in range(3):
        Gi[k * 3 + k] = a
    Fi = o.viscous_flux(3, 0.8, 0.5, U, Gi, np.zeros((3, 30)))
    close(Fi, np.zeros_like(Fi), 1e-14, "pure expansion", scale=np.abs(a).max())
    close(o.viscous_flux(3, 1.6, 1.0, U, G, gT), 2.0 * Fv, 1e-15, "linear in (mu, kappa)")


def pin_viscous_rotation(o):
    """Frame rotation Q: with v' = Q v, G' = Q G Q^T, grad T' = Q grad T,
    the stress turns as tau' = Q tau Q^T and the energy flux as Q q."""
    rng = np.random.default_rng(130)
    for dim in (2, 3):
        U, G, gT = _visc_inputs(dim, 12, 131 + dim)
        Fv = o.viscous_flux(dim, 0.6, 0.2, U, G, gT)
        for i in range(12):
            Q = _rotation(dim, rng)
            v = U[1:dim + 1, i] / U[0, i]
            Up = U[:, i:i + 1].copy()
            Up[1:dim + 1, 0] = U[0, i] * (Q @ v)
            Gp = (Q @ G[:, i].reshape(dim, dim) @ Q.T).reshape(dim * dim, 1)
            gp = (Q @ gT[:, i]).reshape(dim, 1)
            Mp = _visc_columns(o.viscous_flux(dim, 0.6, 0.2, Up, Gp, gp), dim, 0)
            M = _visc_columns(Fv, dim, i)
            close(Mp[1:dim + 1], Q @ M[1:dim + 1] @ Q.T, 1e-13, f"stress rotation {dim}D")
            close(Mp[dim + 1], Q @ M[dim + 1], 1e-13, f"energy flux rotation {dim}D")


PINS = [
    pin_worked_state,
    pin_v_mag2,
    pin_temperature_route,
    pin_roundtrip,
    pin_galilean,
    pin_homogeneity,
    pin_jacobian_fd,
    pin_eigenvalues,
    pin_eigenvectors,
    pin_textbook_jacobian,
    pin_axis_permutation,
    pin_dimension_embedding,
    pin_rotation,
    pin_at_rest,
    pin_riemann_isentrope,
    pin_riemann_characteristic,
    pin_characteristic_transform,
    pin_adjoint_fd,
    pin_characteristic_decomposition,
    pin_roe_property,
    pin_roe_product_rule,
    pin_roe_consistency,
    pin_eos_perfect_gas_thermal,
    pin_eos_stiffened_reduces,
    pin_eos_sound_speed_fd,
    pin_eos_thermodynamic_consistency,
    pin_viscous_couette,
    pin_viscous_rigid_rotation,
    pin_viscous_stokes,
    pin_viscous_rotation,
]
