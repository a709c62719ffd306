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

MUTANTS = [
    ("spmv wrong gather index", "s += val[k] * x[col[k]];", "s += val[k] * x[i];"),
    ("spmv dropped last term", "for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += val[k] * x[col[k]];",
     "for (int64_t k = row_ptr[i]; k < row_ptr[i + 1] - 1; ++k) s += val[k] * x[col[k]];"),
    ("spmv_abs dropped abs", "s += fabs(val[k]) * fabs(x[col[k]]);", "s += fabs(val[k]) * x[col[k]];"),
    ("residual sign", "r[i] = b[i] - r[i];", "r[i] = r[i] - b[i];"),
    ("alpha transposed", "const double alpha = rho / pq;", "const double alpha = pq / rho;"),
    ("x update uses r", "x[i] = x[i] + alpha * p[i];", "x[i] = x[i] + alpha * r[i];"),
    ("r update sign", "r[i] = r[i] - alpha * q[i];", "r[i] = r[i] + alpha * q[i];"),
    ("beta transposed", "const double beta = rho_new / rho;", "const double beta = rho / rho_new;"),
    ("p update sign", "p[i] = r[i] + beta * p[i];", "p[i] = r[i] - beta * p[i];"),
    ("rho not carried", "rho = rho_new;\n", "\n"),
    ("criterion drops rhs norm", "if (resnorm <= tau * bnorm) { reason = ORC_CONVERGED; break; }",
     "if (resnorm <= tau) { reason = ORC_CONVERGED; break; }"),
    ("iteration cap off by one", "if (k >= max_iters) { reason = ORC_MAX_ITERS; break; }",
     "if (k > max_iters) { reason = ORC_MAX_ITERS; break; }"),
    ("no initial check", "else if (resnorm <= tau * bnorm) reason = ORC_CONVERGED;", ""),
    ("breakdown test inclusive dropped", "if (pq <= 0.0) { reason = ORC_BREAKDOWN; break; }",
     "if (pq < 0.0) { reason = ORC_BREAKDOWN; break; }"),
    ("zero rhs keeps guess", "for (int64_t i = 0; i < n; ++i) x[i] = 0.0;", ";"),
    ("validate strict monotone", "if (row_ptr[i + 1] < row_ptr[i]) return ORC_CSR_DECREASING;",
     "if (row_ptr[i + 1] <= row_ptr[i]) return ORC_CSR_DECREASING;"),
    ("validate column bound", "if (col[k] < 0 || col[k] >= n_cols) return ORC_CSR_BAD_COLUMN;",
     "if (col[k] < 0 || col[k] > n_cols) return ORC_CSR_BAD_COLUMN;"),
    ("validate check order", "if (row_ptr[0] != 0) return ORC_CSR_BAD_FIRST;\n", "\n"),
    ("partition strict target", "while (i < n && row_ptr[i] < target) ++i;",
     "while (i < n && row_ptr[i] <= target) ++i;"),
    ("gershgorin sign", "if (d - R < lo) lo = d - R;", "if (d + R < lo) lo = d + R;"),
    ("history index", "if (hist) hist[k] = resnorm;", "if (hist) hist[k - 1] = resnorm;"),
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


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert src.count(old) == 1, "mutation site for %r not unique/present" % name
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
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
