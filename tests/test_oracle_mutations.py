"""Plant one mistake at a time in a copy of the oracle's C source and check
that at least one pin catches it.  Mistakes are planted on the CPU only,
in a temporary copy; the committed oracle is never changed."""
import os

import pytest

import oracle
from oracle_pins import PINS

# (name, original text, planted text); each original must occur in the source.
MUTATIONS = [
    ("kinetic half dropped", "double kinetic, e;\n    s.rho", None),
    ("kinetic energy factor", "kinetic = 0.5 * s.q;", "kinetic = 1.0 * s.q;"),
    ("pressure uses gamma", "s.p = (gamma - 1.0) * s.rho * e;", "s.p = gamma * s.rho * e;"),
    ("velocity not divided", "s.v[k] = U[(1 + k) * ld + i] / s.rho;", "s.v[k] = U[(1 + k) * ld + i];"),
    ("cons2prim stores E", "V[(dim + 1) * ldV + i] = s.p;", "V[(dim + 1) * ldV + i] = s.E;"),
    ("prim2cons kinetic", "p / (gamma - 1.0) + 0.5 * rho * q;", "p / (gamma - 1.0) + rho * q;"),
    ("prim2cons internal", "p / (gamma - 1.0) + 0.5 * rho * q;", "p / gamma + 0.5 * rho * q;"),
    ("sound speed without gamma", "c[i] = sqrt(gamma * s.p / s.rho);", "c[i] = sqrt(s.p / s.rho);"),
    ("pressure on every momentum row", "(r == d ? s.p : 0.0)", "s.p"),
    ("energy flux without p", "col[dim + 1] = s.v[d] * (s.E + s.p);", "col[dim + 1] = s.v[d] * s.E;"),
    ("flux stored column-major", "F[(r * dim + d) * ldF + i] = col[r];",
     "F[(d * (dim + 2) + r) * ldF + i] = col[r];"),
    ("Jacobian row 0", "A[0][1 + d] = 1.0;", "A[0][1 + d] = s->v[d];"),
    ("Jacobian dp/drho sign", "double dp_drho = phi;", "double dp_drho = -phi;"),
    ("Jacobian index swap", "t = t + s->v[i];", "t = t + s->v[j];"),
    ("Jacobian energy row sign", "A[K - 1][0] = s->v[d] * dp_drho - s->v[d] * H;",
     "A[K - 1][0] = s->v[d] * dp_drho + s->v[d] * H;"),
    ("Jacobian corner", "A[K - 1][K - 1] = s->v[d] * (1.0 + dp_dE);", "A[K - 1][K - 1] = s->v[d] * dp_dE;"),
    ("Jacobian block transposed", "dst[r * K + c] = blk[r][c];", "dst[r * K + c] = blk[c][r];"),
    ("Jacobian dp/dE", "double dp_dE = g1;", "double dp_dE = gamma;"),
    ("Riemann factor 2", "double two_c_over_g1 = 2.0 * c / (gamma - 1.0);\n        for (d",
     "double two_c_over_g1 = c / (gamma - 1.0);\n        for (d"),
    ("Riemann sign", "R[(2 * d + 0) * ldR + i] = s.v[d] - two_c_over_g1;",
     "R[(2 * d + 0) * ldR + i] = s.v[d] + two_c_over_g1;"),
    ("entropy exponent", "R[(2 * dim) * ldR + i] = s.p / pow(s.rho, gamma);",
     "R[(2 * dim) * ldR + i] = s.p / pow(s.rho, gamma - 1.0);"),
    ("char2cons sound speed", "c = 0.25 * g1 * (wp - wm);", "c = 0.5 * g1 * (wp - wm);"),
    ("cons2char tangential", "W[slot * ldW + i] = s.v[j];", "W[slot * ldW + i] = s.v[dir];"),
    ("cons2char entropy", "W[1 * ldW + i] = s.p / pow(s.rho, gamma);", "W[1 * ldW + i] = s.p;"),
    ("v_mag2 divides by rho once", "y[i] = mm / (rho * rho);", "y[i] = mm / rho;"),
    ("v_mag2 drops a component", "for (k = 0; k < dim; ++k) {\n            double m", "for (k = 1; k < dim; ++k) {\n            double m"),
    ("eigenvector acoustic sign", "Rm[K - 1][0] = H - cs * s->v[d];", "Rm[K - 1][0] = H + cs * s->v[d];"),
    ("eigenvector entropy energy", "Rm[K - 1][1] = 0.5 * s->q;", "Rm[K - 1][1] = s->q;"),
    ("eigenvector shear energy", "Rm[K - 1][col] = s->v[j];", "Rm[K - 1][col] = s->v[d];"),
    ("char_apply uses R for L", "        if (mode == 0) {\n            if (invert", "        if (mode == 1) {\n            if (invert"),
    ("adjoint not transposed", "acc[c] = acc[c] + blk[r][c] * Fb[field * ldFb + i];",
     "acc[c] = acc[c] + blk[c][r] * Fb[field * ldFb + i];"),
    ("adjoint cotangent layout", "int64_t field = (dir >= 0) ? r : (r * dim + d);",
     "int64_t field = (dir >= 0) ? r : (d * (dim + 2) + r);"),
]
MUTATIONS += [
    ("Roe velocity plain mean", "v[k] = (a * l.v[k] + b * r.v[k]) / (a + b);",
     "v[k] = 0.5 * (l.v[k] + r.v[k]);"),
    ("Roe velocity weights swapped", "v[k] = (a * l.v[k] + b * r.v[k]) / (a + b);",
     "v[k] = (b * l.v[k] + a * r.v[k]) / (a + b);"),
    ("Roe density plain mean", "double rho = a * b;", "double rho = 0.5 * (l.rho + r.rho);"),
    ("Roe enthalpy from left only", "double H = (a * HL + b * HR) / (a + b);", "double H = HL;"),
    ("Roe enthalpy without pressure", "double HL = (l.E + l.p) / l.rho,", "double HL = l.E / l.rho,"),
    ("Roe pressure factor", "p = (gamma - 1.0) / gamma * rho * (H - 0.5 * q);",
     "p = (gamma - 1.0) * rho * (H - 0.5 * q);"),
    ("Roe energy sign", "Uh[(dim + 1) * ldH + i] = rho * H - p;", "Uh[(dim + 1) * ldH + i] = rho * H + p;"),
]
MUTATIONS += [
    ("EOS temperature uses c_p", "Ti = e / params[1];", "Ti = e / params[0];"),
    ("EOS perfect-gas gamma inverted", "double gamma = params[0] / params[1];", "double gamma = params[1] / params[0];"),
    ("EOS internal energy without kinetic half", "e = U[(dim + 1) * ldU + i] / rho - 0.5 * q;",
     "e = U[(dim + 1) * ldU + i] / rho - q;"),
    ("stiffened pressure p_inf factor", "pi = (gamma - 1.0) * rho * e - gamma * pinf;",
     "pi = (gamma - 1.0) * rho * e - pinf;"),
    ("stiffened temperature without p_inf", "Ti = (e - pinf / rho) / params[2];", "Ti = e / params[2];"),
    ("stiffened sound speed without p_inf", "ci = sqrt(gamma * (pi + pinf) / rho);", "ci = sqrt(gamma * pi / rho);"),
    ("stiffened temperature c_v slot", "Ti = (e - pinf / rho) / params[2];", "Ti = (e - pinf / rho) / params[1];"),
]
MUTATIONS += [
    ("viscous bulk factor", "t = t - 2.0 / 3.0 * mu * div;", "t = t - 1.0 / 3.0 * mu * div;"),
    ("viscous stress not symmetrised", "double t = mu * (G[(a * dim + b) * ldG + i] + G[(b * dim + a) * ldG + i]);",
     "double t = 2.0 * mu * G[(a * dim + b) * ldG + i];"),
    ("viscous heat flux dropped", "Fv[((dim + 1) * dim + d) * ldF + i] = work + kappa * gT[d * ldT + i];",
     "Fv[((dim + 1) * dim + d) * ldF + i] = work;"),
    ("viscous layout transposed", "Fv[((1 + a) * dim + d) * ldF + i] = tau[a][d];",
     "Fv[(d * (dim + 2) + 1 + a) * ldF + i] = tau[a][d];"),
    ("viscous work uses the flux direction velocity", "work = work + v[a] * tau[a][d];",
     "work = work + v[d] * tau[a][d];"),
    ("viscous velocity not divided", "v[a] = U[(1 + a) * ldU + i] / rho;", "v[a] = U[(1 + a) * ldU + i];"),
]
MUTATIONS = [m for m in MUTATIONS if m[2] is not None]


@pytest.fixture(scope="module")
def source():
    with open(oracle.SOURCE) as f:
        return f.read()


@pytest.mark.parametrize("name,orig,planted", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, source, name, orig, planted):
    assert source.count(orig) == 1, f"mutation anchor not unique: {name}"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(orig, planted))
    lib = oracle.compile_source(str(src), str(tmp_path / "libmutant.so"))
    o = oracle.Oracle(lib)
    caught = []
    for pin in PINS:
        try:
            pin(o)
        except Exception as exc:  # any failure counts as detection
            caught.append(f"{pin.__name__}: {exc}")
    assert caught, f"no pin caught the planted mistake '{name}'"
