"""The C ABI driven from plain C (tests/c_client/spk_c_client.c: HIP runtime
buffers, no Python or torch in the process): spk_csr_check, an SpMV plan and
a solve, compared with the FP64 oracle.

Tolerances as in the solver tests: SpMV within 2 gamma_m (|A||x|); solutions
within 1e-12 relative of the oracle's, iteration counts within +-1."""
import os
import subprocess

import numpy as np
import pytest

import inputs
import oracle
from tests.gpu_util import U64, gamma

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "spk_c_client")


def row_scaled_ns(N, seed):
    A = inputs.stencil7_ns(N, seed)
    s = np.array([2.0 ** (inputs.unif(seed, 29, i) * 3) for i in range(A.n_rows)])
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    return inputs.CSR(A.n_rows, A.n_cols, A.row_ptr.copy(), A.col.copy(), A.val * s[rows])


CASES = {
    "cg": (lambda: inputs.stencil7(24, 3), 0, 0, lambda A, b: oracle.cg(A, b, tau=1e-13)),
    "cg_jacobi": (lambda: inputs.stencil7(24, 3), 0, 1, lambda A, b: oracle.pcg_jacobi(A, b, tau=1e-13)),
    "cgs": (lambda: inputs.stencil7_ns(24, 4), 1, 0, lambda A, b: oracle.cgs(A, b, tau=1e-13)),
    "gmres_jacobi": (lambda: row_scaled_ns(24, 5), 2, 1,
                     lambda A, b: oracle.gmres(A, b, tau=1e-13, m=30, jacobi=True)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_c_client_matches_oracle(tmp_path, name):
    assert os.path.exists(EXE), "the C client is not built (run __graft_entry__.build())"
    make, solver, precond, ref = CASES[name]
    A = make()
    n = A.n_rows
    b = inputs.rhs(n, 6)
    xv = inputs.vec(n, 6, 5)
    (tmp_path / "meta.txt").write_text("%d %d\n" % (n, A.nnz))
    A.row_ptr.astype(np.int32).tofile(tmp_path / "row_ptr.i32")
    A.col.astype(np.int32).tofile(tmp_path / "col.i32")
    A.val.astype(np.float64).tofile(tmp_path / "val.f64")
    b.tofile(tmp_path / "b.f64")
    xv.tofile(tmp_path / "x.f64")
    out = subprocess.run([EXE, str(tmp_path), str(solver), str(precond), "1e-13", "1000"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    verdict, iters, stop, bnorm, true_res = out.stdout.split()
    assert int(verdict) == 0 and int(stop) == 1
    y = np.fromfile(tmp_path / "y.f64", np.float64)
    m = np.maximum(np.diff(A.row_ptr), 1)
    assert np.all(np.abs(y - oracle.spmv(A, xv)) <= 2 * gamma(m, U64) * oracle.spmv_abs(A, xv))
    x = np.fromfile(tmp_path / "sol.f64", np.float64)
    xo, ro, _ = ref(A, b)
    assert abs(int(iters) - ro.iterations) <= 1
    assert np.linalg.norm(x - xo) <= 1e-12 * np.linalg.norm(xo)
    assert abs(float(bnorm) - ro.rhs_norm) <= 1e-14 * ro.rhs_norm
    assert float(true_res) <= 10 * 1e-13 * float(bnorm)


def test_c_client_serving(tmp_path):
    """Three requests through the serving API from plain C: b, b/2 and -b on one
    matrix.  Scaling by a power of two and negation are exact in every operation,
    so the three solutions are exact scalings of one another (bitwise); request 0
    meets the FP64 criterion and is within 1e-10 of the oracle's FP64 CG solution
    (the mixed-precision tolerance)."""
    assert os.path.exists(EXE), "the C client is not built (run __graft_entry__.build())"
    A = inputs.stencil7(24, 3)
    n = A.n_rows
    b = inputs.rhs(n, 7)
    (tmp_path / "meta.txt").write_text("%d %d\n" % (n, A.nnz))
    A.row_ptr.astype(np.int32).tofile(tmp_path / "row_ptr.i32")
    A.col.astype(np.int32).tofile(tmp_path / "col.i32")
    A.val.astype(np.float64).tofile(tmp_path / "val.f64")
    b.tofile(tmp_path / "b.f64")
    inputs.vec(n, 7, 5).tofile(tmp_path / "x.f64")
    out = subprocess.run([EXE, str(tmp_path), "9", "0", "1e-12", "10000"], capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    verdict, iters, stop, bnorm, true_res = out.stdout.split()
    assert int(verdict) == 0 and int(stop) == 1 and int(iters) > 0
    x = np.fromfile(tmp_path / "sol.f64", np.float64)
    xh = np.fromfile(tmp_path / "sol_half.f64", np.float64)
    xn = np.fromfile(tmp_path / "sol_neg.f64", np.float64)
    assert np.array_equal(xh, 0.5 * x) and np.array_equal(xn, -x)
    assert np.linalg.norm(oracle.residual(A, b, x)) <= 1e-12 * np.linalg.norm(b) * 1.01
    xo, _, _ = oracle.cg(A, b, tau=1e-14)
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)
