"""Planted mistakes in copies of the oracle (on the CPU) must each fail a pin.

Each mutant is oracle.c with one plausible slip (dropped term, wrong sign,
wrong index, transposed quotient, off-by-one), compiled with gcc into a
temporary directory and run against the whole pin battery in a child
process.  A mutant that passes every pin would mean the pins cannot tell that
slip from the paper's definitions.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, text, replacement, scope): the mutation replaces every occurrence of
# the text inside the function whose definition starts with `scope` (the
# whole file when scope is None); the text must occur there.
MUTANTS = [
    ("spmv wrong gather index", "s += val[k] * x[col[k]];", "s += val[k] * x[i];", "void orc_spmv("),
    ("spmv dropped last term", "for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += val[k] * x[col[k]];",
     "for (int64_t k = row_ptr[i]; k < row_ptr[i + 1] - 1; ++k) s += val[k] * x[col[k]];", "void orc_spmv("),
    ("spmv_abs dropped abs", "s += fabs(val[k]) * fabs(x[col[k]]);", "s += fabs(val[k]) * x[col[k]];", None),
    ("residual sign", "r[i] = b[i] - r[i];", "r[i] = r[i] - b[i];", None),
    ("alpha transposed", "const double alpha = rho / pq;", "const double alpha = pq / rho;", "int orc_cg("),
    ("x update uses r", "x[i] = x[i] + alpha * p[i];", "x[i] = x[i] + alpha * r[i];", "int orc_cg("),
    ("r update sign", "r[i] = r[i] - alpha * q[i];", "r[i] = r[i] + alpha * q[i];", "int orc_cg("),
    ("beta transposed", "const double beta = rho_new / rho;", "const double beta = rho / rho_new;", "int orc_cg("),
    ("p update sign", "p[i] = r[i] + beta * p[i];", "p[i] = r[i] - beta * p[i];", "int orc_cg("),
    ("rho not carried", "rho = rho_new;\n", "\n", "int orc_cg("),
    ("criterion drops rhs norm", "if (resnorm <= tau * bnorm) { reason = ORC_CONVERGED; break; }",
     "if (resnorm <= tau) { reason = ORC_CONVERGED; break; }", "int orc_cg("),
    ("iteration cap off by one", "if (k >= max_iters) { reason = ORC_MAX_ITERS; break; }",
     "if (k > max_iters) { reason = ORC_MAX_ITERS; break; }", "int orc_cg("),
    ("no initial check", "else if (resnorm <= tau * bnorm) reason = ORC_CONVERGED;", "", "int orc_cg("),
    ("breakdown test inclusive dropped", "if (pq <= 0.0) { reason = ORC_BREAKDOWN; break; }",
     "if (pq < 0.0) { reason = ORC_BREAKDOWN; break; }", "int orc_cg("),
    ("zero rhs keeps guess", "for (int64_t i = 0; i < n; ++i) x[i] = 0.0;", ";", "int orc_cg("),
    ("validate strict monotone", "if (row_ptr[i + 1] < row_ptr[i]) return ORC_CSR_DECREASING;",
     "if (row_ptr[i + 1] <= row_ptr[i]) return ORC_CSR_DECREASING;", None),
    ("validate column bound", "if (col[k] < 0 || col[k] >= n_cols) return ORC_CSR_BAD_COLUMN;",
     "if (col[k] < 0 || col[k] > n_cols) return ORC_CSR_BAD_COLUMN;", "int orc_csr_validate("),
    ("validate check order", "if (row_ptr[0] != 0) return ORC_CSR_BAD_FIRST;\n", "\n", None),
    ("partition strict target", "while (i < n && row_ptr[i] < target) ++i;",
     "while (i < n && row_ptr[i] <= target) ++i;", None),
    ("gershgorin sign", "if (d - R < lo) lo = d - R;", "if (d + R < lo) lo = d + R;", None),
    ("history index", "if (hist) hist[k] = resnorm;", "if (hist) hist[k - 1] = resnorm;", "int orc_cg("),
    ("residual sumsq drops square", "acc += r * r;", "acc += r;", "double orc_residual_sumsq("),
    ("residual sumsq skips last row", "for (int64_t i = 0; i < n_rows; ++i) {\n        double s",
     "for (int64_t i = 0; i + 1 < n_rows; ++i) {\n        double s", "double orc_residual_sumsq("),
    ("residual sumsq gathers by row", "s += val[k] * x[col[k]];\n        const double r",
     "s += val[k] * x[i];\n        const double r", "double orc_residual_sumsq("),
    # COO
    ("coo no zero fill", "for (int64_t i = 0; i < n_rows; ++i) y[i] = 0.0;", ";", "void orc_coo_spmv("),
    ("coo gather by row", "y[row[k]] += val[k] * x[col[k]];", "y[row[k]] += val[k] * x[row[k]];",
     "void orc_coo_spmv("),
    ("coo last entry dropped", "for (int64_t k = 0; k < nnz; ++k) y[row[k]]", "for (int64_t k = 1; k < nnz; ++k) y[row[k]]",
     "void orc_coo_spmv("),
    ("coo row bound", "if (row[k] < 0 || row[k] >= n_rows) return ORC_CSR_BAD_FIRST;",
     "if (row[k] < 0 || row[k] > n_rows) return ORC_CSR_BAD_FIRST;", "int orc_coo_validate("),
    ("coo column bound", "if (col[k] < 0 || col[k] >= n_cols) return ORC_CSR_BAD_COLUMN;",
     "if (col[k] < 0 || col[k] > n_cols) return ORC_CSR_BAD_COLUMN;", "int orc_coo_validate("),
    ("coo sortedness strict", "if (row[k] < row[k - 1]) *row_sorted = 0;",
     "if (row[k] <= row[k - 1]) *row_sorted = 0;", "int orc_coo_validate("),
    ("coo check order", "if (row[k] < 0 || row[k] >= n_rows) return ORC_CSR_BAD_FIRST;\n    for",
     "if (row[k] < 0 || row[k] >= n_rows) return ORC_CSR_BAD_FIRST;\n    for (int64_t k = 0; k < 0; ++k)\n    for",
     "int orc_coo_validate("),
    # CGS
    ("cgs beta transposed", "const double beta = rho / rho_prev;", "const double beta = rho_prev / rho;",
     "static int cgs_core("),
    ("cgs u uses p", "u[i] = r[i] + beta * q[i];", "u[i] = r[i] + beta * p[i];", "static int cgs_core("),
    ("cgs p drops beta squared", "p[i] = u[i] + beta * (q[i] + beta * p[i]);", "p[i] = u[i] + beta * (q[i] + p[i]);",
     "static int cgs_core("),
    ("cgs q sign", "q[i] = u[i] - alpha * v[i];", "q[i] = u[i] + alpha * v[i];", "static int cgs_core("),
    ("cgs uh drops q", "uh[i] = u[i] + q[i];", "uh[i] = u[i];", "static int cgs_core("),
    ("cgs x update uses u", "x[i] = x[i] + alpha * uh[i];", "x[i] = x[i] + alpha * u[i];", "static int cgs_core("),
    ("cgs r update sign", "r[i] = r[i] - alpha * qh[i];", "r[i] = r[i] + alpha * qh[i];", "static int cgs_core("),
    ("cgs sigma uses r", "const double sigma = dot(n, rt, v);", "const double sigma = dot(n, r, v);",
     "static int cgs_core("),
    ("cgs rho uses r.r", "const double rho = dot(n, rt, r);", "const double rho = dot(n, r, r);", "static int cgs_core("),
    ("cgs rho_prev not carried", "rho_prev = rho;\n", "\n", "static int cgs_core("),
    ("cgs shadow is b", "rt[i] = r[i];", "rt[i] = b[i];", "static int cgs_core("),
    ("cgs sigma breakdown dropped", "if (sigma == 0.0) { reason = ORC_BREAKDOWN; break; }", "", "static int cgs_core("),
    ("cgs cap off by one", "if (k >= max_iters) { reason = ORC_MAX_ITERS; break; }",
     "if (k > max_iters) { reason = ORC_MAX_ITERS; break; }", "static int cgs_core("),
    ("cgs history index", "if (hist) hist[k] = resnorm;", "if (hist) hist[k - 1] = resnorm;", "static int cgs_core("),
    # GMRES
    ("gmres projection sign", "for (int64_t t = 0; t < n; ++t) w[t] = w[t] - h * vi[t];",
     "for (int64_t t = 0; t < n; ++t) w[t] = w[t] + h * vi[t];", "static int gmres_core("),
    ("gmres projection uses v_j", "const double h = dot(n, w, vi);", "const double h = dot(n, w, vj);",
     "static int gmres_core("),
    ("gmres old rotations skipped", "for (int64_t i = 0; i < j; ++i) {\n                const double a",
     "for (int64_t i = 0; i < 0; ++i) {\n                const double a", "static int gmres_core("),
    ("gmres rotation sign", "H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;", "H[(i + 1) * m + j] = sn[i] * a + cs[i] * c;",
     "static int gmres_core("),
    ("gmres g update sign", "g[j + 1] = -sn[j] * g[j];", "g[j + 1] = sn[j] * g[j];", "static int gmres_core("),
    ("gmres g not rotated", "g[j] = cs[j] * g[j];", ";", "static int gmres_core("),
    ("gmres back substitution index", "for (int64_t t = i + 1; t < used; ++t) s -= H[i * m + t] * y[t];",
     "for (int64_t t = i + 1; t < used; ++t) s -= H[t * m + i] * y[t];", "static int gmres_core("),
    ("gmres basis not normalised", "for (int64_t t = 0; t < n; ++t) vn[t] = w[t] / hnext;",
     "for (int64_t t = 0; t < n; ++t) vn[t] = w[t];", "static int gmres_core("),
    ("gmres x update drops last column", "for (int64_t i = 0; i < used; ++i) {\n                const double *vi",
     "for (int64_t i = 0; i + 1 < used; ++i) {\n                const double *vi", "static int gmres_core("),
    ("gmres restart keeps old residual", "orc_residual(n, row_ptr, col, val, b, x, V);\n        const double beta",
     "if (k == 0) orc_residual(n, row_ptr, col, val, b, x, V);\n        const double beta", "static int gmres_core("),
    ("gmres cap off by one", "if (k >= max_iters) { reason = ORC_MAX_ITERS; break; }\n            if (hnext",
     "if (k > max_iters) { reason = ORC_MAX_ITERS; break; }\n            if (hnext", "static int gmres_core("),
    # right-preconditioned (Jacobi) CGS and GMRES
    ("cgs jacobi p not scaled", "for (int64_t i = 0; i < n; ++i) qh[i] = p[i] / d[i];",
     "for (int64_t i = 0; i < n; ++i) qh[i] = p[i];", "static int cgs_core("),
    ("cgs jacobi uh scaled twice", "for (int64_t i = 0; i < n; ++i) uh[i] = uh[i] / d[i];",
     "for (int64_t i = 0; i < n; ++i) uh[i] = uh[i] / (d[i] * d[i]);", "static int cgs_core("),
    ("gmres jacobi v not scaled", "for (int64_t t = 0; t < n; ++t) y_n[t] = vj[t] / d[t];",
     "for (int64_t t = 0; t < n; ++t) y_n[t] = vj[t];", "static int gmres_core("),
    ("gmres jacobi x update unscaled", "for (int64_t t = 0; t < n; ++t) x[t] = x[t] + y_n[t] / d[t];",
     "for (int64_t t = 0; t < n; ++t) x[t] = x[t] + y_n[t];", "static int gmres_core("),
    ("jacobi zero diagonal accepted", "if (d[i] == 0.0 || !isfinite(d[i])) ok = -1;",
     "if (!isfinite(d[i])) ok = -1;", "static int jacobi_diag_ok("),
    # Jacobi PCG
    ("diagonal keeps last duplicate", "if (col[k] == i) s += val[k];", "if (col[k] == i) s = val[k];",
     "void orc_diagonal("),
    ("pcg z multiplies", "z[i] = r[i] / d[i];", "z[i] = r[i] * d[i];", "int orc_pcg_jacobi("),
    ("pcg rho uses r.r", "const double rho_new = dot(n, r, z);", "const double rho_new = dot(n, r, r);",
     "int orc_pcg_jacobi("),
    ("pcg p update uses r", "p[i] = z[i] + beta * p[i];", "p[i] = r[i] + beta * p[i];", "int orc_pcg_jacobi("),
    ("pcg initial direction r", "for (int64_t i = 0; i < n; ++i) p[i] = z[i];",
     "for (int64_t i = 0; i < n; ++i) p[i] = r[i];", "int orc_pcg_jacobi("),
    ("pcg stop on preconditioned norm", "resnorm = sqrt(dot(n, r, r));\n        if (hist) hist[k] = resnorm;",
     "resnorm = sqrt(rho_new);\n        if (hist) hist[k] = resnorm;", "int orc_pcg_jacobi("),
    ("pcg zero diagonal accepted", "if (d[i] == 0.0 || !isfinite(d[i])) {", "if (!isfinite(d[i])) {",
     "int orc_pcg_jacobi("),
    ("pcg alpha transposed", "const double alpha = rho / pq;", "const double alpha = pq / rho;",
     "int orc_pcg_jacobi("),
    ("pcg rho not carried", "rho = rho_new;\n", "\n", "int orc_pcg_jacobi("),
]

RUNNER = r"""
import sys
sys.path.insert(0, {root!r})
import oracle
from tests import pins
orc = oracle.Oracle(oracle.load({lib!r}))
failed = []
for pin in pins.ALL_PINS:
    try:
        pin(orc)
    except Exception as e:  # an assertion, or a numpy error caused by garbage
        failed.append(pin.__name__)
print("FAILED:" + ",".join(failed))
sys.exit(1 if failed else 0)
"""


def mutate(src, old, new, scope):
    """src with `old` replaced by `new` inside the function starting at `scope`."""
    if scope is None:
        assert src.count(old) == 1, "mutation site %r not unique/present" % old
        return src.replace(old, new)
    a = src.index(scope)
    b = src.index("\n}\n", a)
    body = src[a:b]
    assert old in body, "mutation site %r not in %s" % (old, scope)
    return src[:a] + body.replace(old, new) + src[b:]


@pytest.mark.parametrize("name,old,new,scope", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new, scope):
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    mpath = tmp_path / "mutant.c"
    mpath.write_text(mutate(src, old, new, scope))
    lib = oracle.build(force=True, src=str(mpath), out=str(tmp_path / "libmutant.so"))
    try:
        proc = subprocess.run([sys.executable, "-c", RUNNER.format(root=ROOT, lib=lib)],
                              capture_output=True, text=True, timeout=120)
        caught = proc.returncode != 0
    except subprocess.TimeoutExpired:
        caught = True
    assert caught, "mutant %r passed every pin" % name


def test_unmutated_copy_passes(tmp_path):
    """Control: the runner reports success for an unmodified copy."""
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    mpath = tmp_path / "same.c"
    mpath.write_text(src)
    lib = oracle.build(force=True, src=str(mpath), out=str(tmp_path / "libsame.so"))
    proc = subprocess.run([sys.executable, "-c", RUNNER.format(root=ROOT, lib=lib)],
                          capture_output=True, text=True, timeout=120)
    assert proc.returncode == 0, proc.stdout + proc.stderr
