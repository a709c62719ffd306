"""Pins of the FP64 oracle to things other than itself.

Every pin checks the oracle against mathematics or an independent library
routine (dense numpy algebra, scipy.sparse, scipy's CG, numpy's
searchsorted), never against a retyping of the oracle's own formula.  The
pins are chosen so that a plausible mistake anywhere in the oracle (a dropped
term, a wrong sign or index, a transposed quotient, an off-by-one in the
iteration count or in a validation check) fails at least one of them;
``test_oracle_mutants.py`` plants such mistakes in copies of the oracle and
checks that.

Each pin is a function ``pin_*(orc)`` that raises AssertionError on failure.
Sizes are small so the whole battery runs in a couple of seconds.
"""
from __future__ import annotations

import math

import numpy as np

import inputs

U64 = 2.0 ** -53


def gamma(m, u=U64):
    """gamma_m = m u / (1 - m u) (Higham, Accuracy and Stability, Sec. 3.1)."""
    mu = np.asarray(m, np.float64) * u
    return mu / (1.0 - mu)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ----------------------------------------------------------------- SpMV
def pin_spmv_dense_bruteforce(orc):
    """Random rectangular CSR (n <= 64) vs dense numpy A @ x, within 2*gamma_m*(|A||x|)."""
    for seed, (nr, nc) in enumerate([(17, 17), (40, 23), (64, 64), (5, 60)]):
        A = inputs.dyadic_random(nr, nc, 7, seed)
        A.val = A.val * np.array([inputs.unif(seed, 11, k) for k in range(A.val.size)])
        x = np.array([inputs.unif(seed, 12, j) for j in range(nc)])
        D = A.to_dense()
        y = orc.spmv(A, x)
        ref = D @ x
        m = np.diff(A.row_ptr)
        bound = 2 * gamma(np.maximum(m, 1)) * (np.abs(D) @ np.abs(x))
        assert np.all(np.abs(y - ref) <= bound), "SpMV differs from dense brute force"
        # the |A||x| helper is pinned too, against dense |A| @ |x|
        sa = orc.spmv_abs(A, x)
        assert np.all(np.abs(sa - np.abs(D) @ np.abs(x)) <= bound)


def pin_spmv_dyadic_exact(orc):
    """Dyadic values and small-integer x: every partial sum is exact, so bit-exact."""
    A = inputs.dyadic_random(50, 37, 9, 3)
    x = np.array([float((inputs.hash64(3, 13, j) % 17) - 8) for j in range(37)])
    y = orc.spmv(A, x)
    assert np.array_equal(y, A.to_dense() @ x)


def pin_spmv_identity_permutation(orc):
    x = np.array([inputs.unif(5, 14, j) for j in range(33)])
    assert np.array_equal(orc.spmv(inputs.diagonal(np.ones(33)), x), x)
    P = inputs.permutation(33, 2)
    assert np.array_equal(orc.spmv(P, x), x[P.col.astype(np.int64)])


def pin_spmv_duplicates_unsorted(orc):
    """Unsorted columns and duplicate entries: duplicates are summed."""
    A = inputs.CSR(3, 4, np.array([0, 3, 3, 6], np.int64), np.array([2, 0, 2, 3, 1, 0], np.int32),
                   np.array([1.5, -2.0, 0.25, 4.0, 8.0, -1.0]))
    x = np.array([1.0, 2.0, 4.0, -8.0])
    assert np.array_equal(orc.spmv(A, x), np.array([1.5 * 4 - 2 + 0.25 * 4, 0.0, -32 + 16 - 1]))


def pin_spmv_scipy_stencil(orc):
    """stencil7 N=12 vs scipy.sparse csr_matrix @ x (independent code) within the gamma bound."""
    import scipy.sparse as sp
    A = inputs.stencil7(12, 0)
    x = inputs.vec(A.n_rows, 0, 5)
    S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))
    ref = S @ x
    y = orc.spmv(A, x)
    bound = 2 * gamma(np.diff(A.row_ptr)) * (abs(S) @ np.abs(x))
    assert np.all(np.abs(y - ref) <= bound)


# ----------------------------------------------------------------- validation
def _coo_of(A):
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int64), np.diff(A.row_ptr))
    return rows, A.col.astype(np.int64), A.val.copy()


def pin_coo_spmv_scipy_and_dense(orc):
    """COO product vs scipy.sparse.coo_matrix (independent code) and dense numpy, entries
    shuffled and duplicated, within the gamma bound of the longest row."""
    import scipy.sparse as sp
    A = inputs.dyadic_random(60, 45, 6, 11)
    rows, cols, vals = _coo_of(A)
    vals = vals * np.array([inputs.unif(12, 23, k) for k in range(vals.size)])   # generic values
    perm = np.argsort(np.array([inputs.hash64(12, 24, k) for k in range(vals.size)], np.uint64), kind="stable")
    rows, cols, vals = (np.concatenate([rows[perm], rows[:7]]), np.concatenate([cols[perm], cols[:7]]),
                        np.concatenate([vals[perm], vals[:7]]))
    x = np.array([inputs.unif(12, 25, j) for j in range(45)])
    y = orc.coo_spmv(60, rows, cols, vals, x)
    ys = sp.coo_matrix((vals, (rows, cols)), shape=(60, 45)).tocsr() @ x
    D = np.zeros((60, 45))
    np.add.at(D, (rows, cols), vals)
    m = np.bincount(rows, minlength=60)
    absb = np.zeros(60)
    np.add.at(absb, rows, np.abs(vals) * np.abs(x[cols]))
    assert np.all(np.abs(y - ys) <= 2 * gamma(m) * absb)
    assert np.all(np.abs(y - D @ x) <= 2 * gamma(m) * absb)


def pin_coo_spmv_dyadic_exact_and_empty_rows(orc):
    A = inputs.dyadic_random(40, 30, 5, 13)
    rows, cols, vals = _coo_of(A)
    keep = rows % 3 != 1                      # every third row left empty
    rows, cols, vals = rows[keep], cols[keep], vals[keep]
    x = np.array([float((j * 7) % 11 - 5) for j in range(30)])
    y = orc.coo_spmv(40, rows, cols, vals, x)
    D = np.zeros((40, 30))
    np.add.at(D, (rows, cols), vals)
    assert np.array_equal(y, D @ x) and not y[1::3].any()


def pin_coo_validate(orc):
    r = np.array([0, 0, 2, 2, 3], np.int64)
    c = np.array([1, 0, 2, 3, 0], np.int64)
    assert orc.coo_validate(4, 4, r, c) == (0, True)
    assert orc.coo_validate(4, 4, r[::-1], c) == (0, False)
    assert orc.coo_validate(3, 4, r, c)[0] == 2          # row 3 out of range
    assert orc.coo_validate(4, 3, r, c)[0] == 5          # column 3 out of range
    assert orc.coo_validate(4, 4, np.array([0, -1], np.int64), np.array([0, 0], np.int64))[0] == 2
    assert orc.coo_validate(-1, 4, r, c)[0] == 1
    assert orc.coo_validate(4, 4, r[:0], c[:0]) == (0, True)
    # a bad column before a bad row: rows are checked first over all entries
    assert orc.coo_validate(3, 3, np.array([0, 1, 3], np.int64), np.array([5, 0, 0], np.int64))[0] == 2
    assert orc.coo_validate(4, 4, np.array([1, 1, 0, 2], np.int64), np.array([0, 1, 2, 3], np.int64)) == (0, False)


def pin_csr_validate(orc):
    rp = np.array([0, 2, 3, 5], np.int64)
    ci = np.array([0, 2, 1, 0, 2], np.int64)
    assert orc.csr_validate(3, 3, 5, rp, ci) == 0
    assert orc.csr_validate(-1, 3, 5, rp, ci) == 1
    assert orc.csr_validate(3, 3, -5, rp, ci) == 1
    assert orc.csr_validate(3, 3, 5, np.array([1, 2, 3, 5]), ci) == 2
    assert orc.csr_validate(3, 3, 5, np.array([0, 3, 2, 5]), ci) == 3
    assert orc.csr_validate(3, 3, 5, np.array([0, 2, 2, 5]), ci) == 0   # empty row is fine
    assert orc.csr_validate(3, 3, 5, np.array([0, 2, 3, 4]), ci) == 4
    assert orc.csr_validate(3, 3, 5, rp, np.array([0, 3, 1, 0, 2])) == 5  # col == n_cols
    assert orc.csr_validate(3, 3, 5, rp, np.array([0, 2, -1, 0, 2])) == 5
    assert orc.csr_validate(3, 3, 5, rp, np.array([0, 2, 1, 0, 2])) == 0
    assert orc.csr_validate(0, 0, 0, np.array([0]), np.array([], np.int64)) == 0
    # first failing check wins: decreasing AND bad column -> decreasing
    assert orc.csr_validate(3, 3, 5, np.array([0, 3, 2, 5]), np.array([9, 9, 9, 9, 9])) == 3


# ----------------------------------------------------------------- CG closed forms
def pin_cg_identity(orc):
    b = np.array([1.0, -2.0, 0.5, 3.0, -0.25])
    x, r, _ = orc.cg(inputs.diagonal(np.ones(5)), b, tau=1e-14)
    assert r.stop_reason == 1 and r.iterations == 1 and np.array_equal(x, b)


def pin_cg_scaled_identity(orc):
    b = np.array([inputs.unif(1, 15, i) for i in range(20)])
    x, r, _ = orc.cg(inputs.diagonal(np.full(20, 4.0)), b, tau=1e-14)
    assert r.iterations == 1 and r.stop_reason == 1 and np.array_equal(x, b / 4.0)
    assert r.implicit_resnorm == 0.0 and r.rhs_norm == np.linalg.norm(b)


def pin_cg_diag_distinct(orc):
    """m distinct eigenvalues: exact Krylov termination after m iterations, not before."""
    d = np.repeat(np.array([1.0, 2.0, 3.5, 5.0, 9.0]), 4)
    b = np.array([1.0 + (i % 3) for i in range(d.size)])
    _, r5, _ = orc.cg(inputs.diagonal(d), b, tau=0.0, max_iters=5)
    assert r5.true_resnorm <= 1e-12 * np.linalg.norm(b)
    _, r4, _ = orc.cg(inputs.diagonal(d), b, tau=0.0, max_iters=4)
    assert r4.iterations == 4 and r4.true_resnorm > 1e-6


def pin_cg_laplacian1d(orc):
    """tridiag(-1,2,-1) x = 1 has x_i = i(n+1-i)/2 (i = 1..n)."""
    n = 31
    i = np.arange(1, n + 1, dtype=np.float64)
    xs = i * (n + 1 - i) / 2
    x, r, _ = orc.cg(inputs.laplacian1d(n), np.ones(n), tau=1e-15, max_iters=n)
    assert r.stop_reason == 1 and r.iterations <= n
    assert _rel(x, xs) <= 1e-13


def pin_cg_dense_solve(orc):
    """Tiny random SPD systems vs dense numpy.linalg.solve, within kappa * 1e-14."""
    for seed in range(3):
        A = inputs.randsym(40, seed, delta=0.05)
        b = inputs.rhs(40, seed)
        D = A.to_dense()
        xs = np.linalg.solve(D, b)
        kappa = np.linalg.cond(D)
        x, r, _ = orc.cg(A, b, tau=1e-15, max_iters=400)
        assert r.stop_reason == 1
        assert _rel(x, xs) <= max(kappa, 1.0) * 1e-14


def pin_cg_krylov_minimiser(orc):
    """x_k (x0 = 0) minimises ||x - x*||_A over K_k(A, b): checks every iterate, not just the end."""
    A = inputs.randsym(24, 7, delta=0.3)
    D = A.to_dense()
    b = inputs.rhs(24, 7)
    K = np.empty((24, 6))
    v = b.copy()
    for k in range(6):
        K[:, k] = v
        v = D @ v
    for k in range(1, 7):
        Q, _ = np.linalg.qr(K[:, :k])
        y = np.linalg.solve(Q.T @ D @ Q, Q.T @ b)
        xk_ref = Q @ y
        xk, r, _ = orc.cg(A, b, tau=0.0, max_iters=k)
        assert r.iterations == k
        assert _rel(xk, xk_ref) <= 1e-10, "iterate %d off the Krylov minimiser" % k


def pin_cg_history_true_residual(orc):
    """Recorded ||r_k|| tracks ||b - A x_k|| (recomputed densely) at every early k."""
    A = inputs.randsym(30, 9, delta=0.5)
    D = A.to_dense()
    b = inputs.rhs(30, 9)
    _, _, hist = orc.cg(A, b, tau=0.0, max_iters=8, history=True)
    assert hist.size == 9 and hist[0] == np.linalg.norm(b)
    for k in range(1, 9):
        xk, _, _ = orc.cg(A, b, tau=0.0, max_iters=k)
        assert abs(hist[k] - np.linalg.norm(b - D @ xk)) <= 1e-12 * np.linalg.norm(b)


def pin_cg_scipy(orc):
    """scipy.sparse.linalg.cg (independent code, same ||r|| <= tau ||b|| criterion)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    for A in (inputs.stencil7(10, 0), inputs.randsym(2000, 3)):
        b = inputs.rhs(A.n_rows, 0)
        S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))
        count = [0]

        def cb(_xk):
            count[0] += 1
        tau = 1e-10
        xs, info = spla.cg(S, b, rtol=tau, atol=0.0, maxiter=2000, callback=cb)
        assert info == 0
        x, r, _ = orc.cg(A, b, tau=tau, max_iters=2000)
        kappa_g = orc.gershgorin_kappa(A)
        assert r.stop_reason == 1 and abs(r.iterations - count[0]) <= 2
        assert _rel(x, xs) <= 2 * kappa_g * tau


def pin_cg_energy_monotone_chebyshev(orc):
    """||x_k - x*||_A is non-increasing and within the Chebyshev bound with kappa_G."""
    A = inputs.randsym(60, 11, delta=0.5)
    D = A.to_dense()
    b = inputs.rhs(60, 11)
    xs = np.linalg.solve(D, b)
    kappa = orc.gershgorin_kappa(A)
    rate = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
    e0 = math.sqrt(xs @ D @ xs)
    prev = e0
    for k in range(1, 16):
        xk, _, _ = orc.cg(A, b, tau=0.0, max_iters=k)
        e = xk - xs
        ek = math.sqrt(max(e @ D @ e, 0.0))
        assert ek <= prev * (1 + 1e-9) + 1e-14 * e0
        assert ek <= 2 * rate ** k * e0 * (1 + 1e-9) + 1e-14 * e0
        prev = ek


# ----------------------------------------------------------------- stop semantics
def pin_cg_stop_semantics(orc):
    A = inputs.diagonal(np.array([2.0, 3.0, 5.0]))
    b = np.array([1.0, 1.0, 1.0])
    x0 = np.array([0.5, -1.0, 7.0])
    x, r, h = orc.cg(A, b, x0=x0, tau=1e-12, max_iters=0, history=True)
    assert r.stop_reason == 2 and r.iterations == 0 and np.array_equal(x, x0)
    assert h.size == 1 and h[0] == np.linalg.norm(b - A.to_dense() @ x0)
    # b = 0: x = 0, converged, no iteration (even with a nonzero guess)
    x, r, _ = orc.cg(A, np.zeros(3), x0=x0, tau=1e-12, max_iters=10)
    assert r.stop_reason == 1 and r.iterations == 0 and np.array_equal(x, np.zeros(3))
    # exact initial guess: converged before the first iteration
    xs = np.array([0.5, 1.0 / 3.0, 0.2])
    x, r, _ = orc.cg(A, b, x0=xs, tau=1e-12, max_iters=10)
    assert r.stop_reason == 1 and r.iterations == 0
    # iteration cap reached exactly
    x, r, _ = orc.cg(inputs.laplacian1d(20), np.ones(20), tau=1e-15, max_iters=3)
    assert r.stop_reason == 2 and r.iterations == 3
    # the relative criterion uses ||b||: scaling b scales nothing else
    _, r1, _ = orc.cg(inputs.laplacian1d(20), np.ones(20), tau=1e-6, max_iters=100)
    _, r2, _ = orc.cg(inputs.laplacian1d(20), 1024.0 * np.ones(20), tau=1e-6, max_iters=100)
    assert r1.iterations == r2.iterations and r1.stop_reason == 1
    # a loose tolerance stops early: the test compares against tau * ||b||, not tau
    R = inputs.randsym(200, 5, delta=0.2)
    bb = 1e6 * inputs.rhs(200, 5)
    _, r3, _ = orc.cg(R, bb, tau=1e-3, max_iters=500)
    _, r4, _ = orc.cg(R, bb, tau=1e-9, max_iters=500)
    assert r3.stop_reason == 1 and r4.stop_reason == 1 and r3.iterations < r4.iterations
    assert r3.implicit_resnorm <= 1e-3 * np.linalg.norm(bb) < r3.implicit_resnorm * 1e4


def pin_cg_breakdown_nonfinite(orc):
    # indefinite: p.q = 1 - 2 < 0 on the first step
    _, r, _ = orc.cg(inputs.diagonal(np.array([1.0, -2.0])), np.array([1.0, 1.0]), tau=1e-12)
    assert r.stop_reason == 3 and r.iterations == 0
    # p.q == 0 exactly
    _, r, _ = orc.cg(inputs.diagonal(np.array([1.0, -1.0])), np.array([1.0, 1.0]), tau=1e-12)
    assert r.stop_reason == 3
    b = np.ones(4)
    b[2] = np.nan
    _, r, _ = orc.cg(inputs.diagonal(np.ones(4)), b, tau=1e-12)
    assert r.stop_reason == 4
    A = inputs.diagonal(np.array([1.0, np.inf, 1.0]))
    _, r, _ = orc.cg(A, np.ones(3), tau=1e-12)
    assert r.stop_reason == 4


# ----------------------------------------------------------------- CGS
def _ns_dense(N, seed, delta=1.0):
    A = inputs.stencil7_ns(N, seed, delta)
    return A, A.to_dense()


def _bicg_poly_residual(D, r0, rt, k):
    """phi_k(A) r0 of BiCG from its Petrov-Galerkin definition: r0 - A K c with
    K = [r0, A r0, ..]_k and (L^T A K) c = L^T r0, L = [rt, A^T rt, ..]_k.
    Returns (c, apply) where apply(v) = phi_k(A) v for the same polynomial."""
    K = np.column_stack([np.linalg.matrix_power(D, j) @ r0 for j in range(k)])
    L = np.column_stack([np.linalg.matrix_power(D.T, j) @ rt for j in range(k)])
    c = np.linalg.solve(L.T @ D @ K, L.T @ r0)

    def apply(v):
        out = v.copy()
        Av = D @ v
        for j in range(k):
            out -= c[j] * Av
            Av = D @ Av
        return out
    return c, apply


def pin_cgs_first_step_closed_form(orc):
    """One CGS step from x0 (rt = r0): alpha = r0.r0 / r0.A r0, x1 = x0 + alpha (2 r0 - alpha A r0),
    r1 = (I - alpha A)^2 r0; nonsymmetric A and a nonzero guess."""
    A, D = _ns_dense(3, 2)
    n = A.n_rows
    b = inputs.rhs(n, 2)
    x0 = inputs.vec(n, 3, 20)
    r0 = b - D @ x0
    Ar = D @ r0
    alpha = (r0 @ r0) / (r0 @ Ar)
    x1 = x0 + alpha * (2 * r0 - alpha * Ar)
    r1 = r0 - 2 * alpha * Ar + alpha * alpha * (D @ Ar)
    x, r, h = orc.cgs(A, b, x0=x0, tau=0.0, max_iters=1, history=True)
    assert r.iterations == 1 and r.stop_reason == 2
    assert _rel(x, x1) <= 1e-13
    assert abs(h[1] - np.linalg.norm(r1)) <= 1e-12 * np.linalg.norm(r1)


def pin_cgs_squared_bicg_polynomial(orc):
    """The CGS residual after k steps is phi_k(A)^2 r0 with phi_k the BiCG residual
    polynomial (Sonneveld): checked for k = 2, 3 on a nonsymmetric and a symmetric A."""
    for A, D in (_ns_dense(3, 4), (inputs.randsym(20, 4, delta=0.5), None)):
        if D is None:
            D = A.to_dense()
        n = A.n_rows
        b = inputs.rhs(n, 5)
        xs = np.linalg.solve(D, b)
        for k in (2, 3):
            _, apply = _bicg_poly_residual(D, b, b, k)
            rk = apply(apply(b))
            xk_ref = xs - np.linalg.solve(D, rk)
            x, r, h = orc.cgs(A, b, tau=0.0, max_iters=k, history=True)
            assert r.iterations == k
            assert _rel(x, xk_ref) <= 1e-9, (k, _rel(x, xk_ref))
            assert abs(h[k] - np.linalg.norm(rk)) <= 1e-8 * np.linalg.norm(b)


def pin_cgs_diag_distinct(orc):
    """Diagonal A with m distinct eigenvalues: phi_m vanishes on the spectrum, so CGS
    converges at iteration m and not before."""
    d = np.repeat(np.array([1.0, 2.5, 4.0, 7.0]), 3)
    b = np.array([inputs.unif(6, 17, i) for i in range(d.size)])
    x, r, h = orc.cgs(inputs.diagonal(d), b, tau=1e-12, max_iters=50, history=True)
    assert r.stop_reason == 1 and r.iterations == 4
    assert np.all(h[:4] > 1e-12 * np.linalg.norm(b))
    assert _rel(x, b / d) <= 1e-12


def pin_cgs_dense_solve_and_scipy(orc):
    """Nonsymmetric diagonally dominant systems: converged x vs numpy.linalg.solve,
    iteration count vs scipy.sparse.linalg.cgs (independent code, same criterion)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    for seed in range(3):
        A, D = _ns_dense(4, seed, delta=0.5)
        b = inputs.rhs(A.n_rows, seed)
        tau = 1e-10
        x, r, _ = orc.cgs(A, b, tau=tau, max_iters=500)
        assert r.stop_reason == 1
        cond = np.linalg.cond(D)
        assert _rel(x, np.linalg.solve(D, b)) <= 10 * cond * tau
        assert r.true_resnorm <= 10 * tau * r.rhs_norm
        count = [0]

        def cb(_xk):
            count[0] += 1
        S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))
        _, info = spla.cgs(S, b, rtol=tau, atol=0.0, maxiter=500, callback=cb)
        assert info == 0 and abs(r.iterations - count[0]) <= 2


def pin_cgs_stop_semantics(orc):
    A = inputs.diagonal(np.array([2.0, 3.0, 5.0]))
    b = np.array([1.0, 1.0, 1.0])
    x0 = np.array([0.5, -1.0, 7.0])
    x, r, h = orc.cgs(A, b, x0=x0, tau=1e-12, max_iters=0, history=True)
    assert r.stop_reason == 2 and r.iterations == 0 and np.array_equal(x, x0)
    assert h[0] == np.linalg.norm(b - A.to_dense() @ x0)
    x, r, _ = orc.cgs(A, np.zeros(3), x0=x0, tau=1e-12, max_iters=10)
    assert r.stop_reason == 1 and r.iterations == 0 and np.array_equal(x, np.zeros(3))
    x, r, _ = orc.cgs(A, b, x0=np.array([0.5, 1.0 / 3.0, 0.2]), tau=1e-12, max_iters=10)
    assert r.stop_reason == 1 and r.iterations == 0
    x, r, _ = orc.cgs(inputs.laplacian1d(20), np.ones(20), tau=1e-15, max_iters=3)
    assert r.stop_reason == 2 and r.iterations == 3
    # skew-symmetric: rt . A r0 = 0 on the first step -> breakdown, x untouched
    S = inputs.from_dense(np.array([[0.0, 1.0], [-1.0, 0.0]]))
    x, r, _ = orc.cgs(S, np.array([1.0, 1.0]), tau=1e-12, max_iters=10)
    assert r.stop_reason == 3 and r.iterations == 0 and np.array_equal(x, np.zeros(2))
    bb = np.ones(4)
    bb[1] = np.inf
    _, r, _ = orc.cgs(inputs.diagonal(np.ones(4)), bb, tau=1e-12)
    assert r.stop_reason == 4


# ----------------------------------------------------------------- GMRES
def _lsq_step(D, x0, b, k):
    """x0 + argmin over K_k(A, r0) of ||b - A x||, from an orthonormal Krylov basis (dense QR)."""
    r0 = b - D @ x0
    K = np.column_stack([np.linalg.matrix_power(D, j) @ r0 for j in range(k)])
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(D @ Q, r0, rcond=None)
    return x0 + Q @ y


def pin_gmres_krylov_least_squares(orc):
    """Every iterate of the first cycle minimises ||b - A x|| over x0 + K_k(A, r0)
    (dense least squares), and the recorded estimate equals that minimum."""
    A, D = _ns_dense(3, 5)
    b = inputs.rhs(A.n_rows, 5)
    x0 = inputs.vec(A.n_rows, 5, 20)
    for k in range(1, 7):
        xr = _lsq_step(D, x0, b, k)
        x, r, h = orc.gmres(A, b, x0=x0, tau=0.0, max_iters=k, m=30, history=True)
        assert r.iterations == k and r.stop_reason == 2
        assert _rel(x, xr) <= 1e-9, (k, _rel(x, xr))
        assert abs(h[k] - np.linalg.norm(b - D @ xr)) <= 1e-9 * np.linalg.norm(b)


def pin_gmres_restart(orc):
    """GMRES(2): the third step restarts from x_2 and minimises over x_2 + K_1(A, r_2);
    a cap in the middle of a cycle still applies the columns built so far."""
    A, D = _ns_dense(3, 6)
    b = inputs.rhs(A.n_rows, 6)
    x0 = np.zeros(A.n_rows)
    x2 = _lsq_step(D, x0, b, 2)
    x3 = _lsq_step(D, x2, b, 1)
    x5 = _lsq_step(D, _lsq_step(D, x2, b, 2), b, 1)
    x, r, _ = orc.gmres(A, b, tau=0.0, max_iters=3, m=2)
    assert r.iterations == 3 and _rel(x, x3) <= 1e-9
    x, r, _ = orc.gmres(A, b, tau=0.0, max_iters=5, m=2)
    assert r.iterations == 5 and _rel(x, x5) <= 1e-9


def pin_gmres_diag_distinct_and_dense(orc):
    """Diagonal A with 5 distinct eigenvalues: converged at step 5, not before; nonsymmetric
    systems converge to numpy.linalg.solve within cond * tau."""
    d = np.repeat(np.array([1.0, 2.0, 3.5, 6.0, 9.0]), 3)
    b = np.array([inputs.unif(8, 28, i) for i in range(d.size)])
    x, r, h = orc.gmres(inputs.diagonal(d), b, tau=1e-12, max_iters=50, m=30, history=True)
    assert r.stop_reason == 1 and r.iterations == 5 and np.all(h[:5] > 1e-12 * np.linalg.norm(b))
    assert _rel(x, b / d) <= 1e-12
    for seed in range(2):
        A, D = _ns_dense(4, seed, delta=0.5)
        bb = inputs.rhs(A.n_rows, seed)
        for m in (30, 4):
            x, r, _ = orc.gmres(A, bb, tau=1e-10, max_iters=2000, m=m)
            assert r.stop_reason == 1 and r.true_resnorm <= 2e-10 * r.rhs_norm
            assert _rel(x, np.linalg.solve(D, bb)) <= 10 * np.linalg.cond(D) * 1e-10


def pin_gmres_scipy(orc):
    """scipy.sparse.linalg.gmres (independent code, restart m) reaches the same solution."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    A, D = _ns_dense(5, 3, delta=0.3)
    b = inputs.rhs(A.n_rows, 3)
    S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))
    xs, info = spla.gmres(S, b, rtol=1e-11, atol=0.0, restart=10, maxiter=500)
    x, r, _ = orc.gmres(A, b, tau=1e-11, max_iters=5000, m=10)
    assert info == 0 and r.stop_reason == 1
    assert _rel(x, xs) <= 10 * np.linalg.cond(D) * 1e-11


def pin_gmres_stop_semantics(orc):
    A, D = _ns_dense(2, 7)
    n = A.n_rows
    b = inputs.rhs(n, 7)
    x0 = inputs.vec(n, 7, 21)
    x, r, h = orc.gmres(A, b, x0=x0, tau=1e-12, max_iters=0, history=True)
    assert r.stop_reason == 2 and r.iterations == 0 and np.array_equal(x, x0)
    r0 = np.linalg.norm(b - D @ x0)
    assert abs(h[0] - r0) <= 1e-14 * r0
    x, r, _ = orc.gmres(A, np.zeros(n), x0=x0, tau=1e-12)
    assert r.stop_reason == 1 and r.iterations == 0 and not x.any()
    xs = np.linalg.solve(D, b)
    _, r, _ = orc.gmres(A, D @ xs, x0=xs, tau=1e-12)
    assert r.stop_reason == 1 and r.iterations == 0
    bb = b.copy()
    bb[0] = np.nan
    _, r, _ = orc.gmres(A, bb, tau=1e-12)
    assert r.stop_reason == 4


# ----------------------------------------------------------------- right-preconditioned CGS / GMRES
def _ns_scaled(N, seed):
    """Nonsymmetric stencil with rows scaled by positive factors 1..8: a varying diagonal."""
    A = inputs.stencil7_ns(N, seed)
    s = np.array([2.0 ** (inputs.unif(seed, 29, i) * 3) for i in range(A.n_rows)])
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    B = inputs.CSR(A.n_rows, A.n_cols, A.row_ptr.copy(), A.col.copy(), A.val * s[rows])
    return B, B.to_dense()


def pin_gmres_jacobi_least_squares(orc):
    """Right-preconditioned GMRES: x_k = x0 + D^{-1} z with z minimising ||r0 - A D^{-1} z|| over
    K_k(A D^{-1}, r0) (dense least squares); the estimate equals the true residual."""
    A, D = _ns_scaled(3, 8)
    b = inputs.rhs(A.n_rows, 8)
    x0 = inputs.vec(A.n_rows, 8, 20)
    dinv = 1.0 / np.diag(D)
    Ah = D * dinv[None, :]
    r0 = b - D @ x0
    for k in (1, 3, 6):
        K = np.column_stack([np.linalg.matrix_power(Ah, j) @ r0 for j in range(k)])
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(Ah @ Q, r0, rcond=None)
        xr = x0 + dinv * (Q @ y)
        x, r, h = orc.gmres(A, b, x0=x0, tau=0.0, max_iters=k, m=30, history=True, jacobi=True)
        assert r.iterations == k and _rel(x, xr) <= 1e-9, (k, _rel(x, xr))
        assert abs(h[k] - np.linalg.norm(b - D @ xr)) <= 1e-9 * np.linalg.norm(b)


def pin_cgs_jacobi_first_step(orc):
    """Right-preconditioned CGS, one step: with Ah = A D^{-1}, alpha = r0.r0 / r0.Ah r0,
    x1 = x0 + alpha D^{-1} (2 r0 - alpha Ah r0), r1 = (I - alpha Ah)^2 r0."""
    A, D = _ns_scaled(3, 9)
    b = inputs.rhs(A.n_rows, 9)
    x0 = inputs.vec(A.n_rows, 9, 20)
    dinv = 1.0 / np.diag(D)
    Ah = D * dinv[None, :]
    r0 = b - D @ x0
    Ar = Ah @ r0
    alpha = (r0 @ r0) / (r0 @ Ar)
    x1 = x0 + alpha * dinv * (2 * r0 - alpha * Ar)
    r1 = r0 - 2 * alpha * Ar + alpha * alpha * (Ah @ Ar)
    x, r, h = orc.cgs_jacobi(A, b, x0=x0, tau=0.0, max_iters=1, history=True)
    assert r.iterations == 1 and _rel(x, x1) <= 1e-13
    assert abs(h[1] - np.linalg.norm(r1)) <= 1e-12 * np.linalg.norm(r1)


def pin_right_jacobi_solves_and_breakdown(orc):
    A, D = _ns_scaled(4, 10)
    b = inputs.rhs(A.n_rows, 10)
    xs = np.linalg.solve(D, b)
    cond = np.linalg.cond(D)
    x, r, _ = orc.cgs_jacobi(A, b, tau=1e-11, max_iters=500)
    assert r.stop_reason == 1 and _rel(x, xs) <= 10 * cond * 1e-11 and r.true_resnorm <= 2e-11 * r.rhs_norm
    x, r, _ = orc.gmres(A, b, tau=1e-11, max_iters=500, m=10, jacobi=True)
    assert r.stop_reason == 1 and _rel(x, xs) <= 10 * cond * 1e-11 and r.true_resnorm <= 2e-11 * r.rhs_norm
    _, rc, _ = orc.gmres(A, b, tau=1e-11, max_iters=500, m=10)
    assert r.iterations < rc.iterations   # the row scaling is what Jacobi undoes
    Z = inputs.diagonal(np.array([1.0, 0.0, 2.0]))
    x0 = np.array([1.0, 2.0, 3.0])
    for f in (lambda **k: orc.cgs_jacobi(Z, np.ones(3), **k), lambda **k: orc.gmres(Z, np.ones(3), jacobi=True, **k)):
        x, r, _ = f(x0=x0, tau=1e-12)
        assert r.stop_reason == 3 and r.iterations == 0 and np.array_equal(x, x0)


# ----------------------------------------------------------------- Jacobi PCG
def _scaled_spd(n, seed):
    """S A S with S a positive diagonal: SPD with a strongly varying diagonal."""
    A = inputs.randsym(n, seed, delta=0.5)
    s = np.array([2.0 ** (inputs.unif(seed, 18, i) * 3) for i in range(n)])
    D = A.to_dense() * s[:, None] * s[None, :]
    return inputs.from_dense(D), D


def pin_diagonal_sums_duplicates(orc):
    A = inputs.CSR(3, 3, np.array([0, 3, 4, 6], np.int64), np.array([2, 0, 0, 1, 2, 2], np.int32),
                   np.array([5.0, 1.5, 2.25, -4.0, 0.5, 0.25]))
    assert np.array_equal(orc.diagonal(A), np.diag(A.to_dense()))
    assert np.array_equal(orc.diagonal(inputs.CSR(2, 2, np.array([0, 1, 1], np.int64),
                                                  np.array([1], np.int32), np.array([3.0]))), [0.0, 0.0])


def pin_pcg_diagonal_one_step(orc):
    """M = A for diagonal A: converged after exactly one iteration with x = b / d."""
    d = np.array([1.0, 3.0, 0.25, 8.0, 2.0, 5.5])
    b = np.array([inputs.unif(7, 19, i) for i in range(d.size)])
    x, r, _ = orc.pcg_jacobi(inputs.diagonal(d), b, tau=1e-14, max_iters=10)
    assert r.stop_reason == 1 and r.iterations == 1
    assert _rel(x, b / d) <= 1e-15


def pin_pcg_is_cg_on_scaled_system(orc):
    """x_k of Jacobi PCG = D^{-1/2} y_k, y_k the CG iterate of D^{-1/2} A D^{-1/2} y = D^{-1/2} b,
    taken from its Krylov-minimiser definition (dense), for k = 1..5."""
    A, D = _scaled_spd(24, 3)
    b = inputs.rhs(24, 3)
    dh = 1.0 / np.sqrt(np.diag(D))
    Ah = D * dh[:, None] * dh[None, :]
    bh = b * dh
    for k in range(1, 6):
        K = np.column_stack([np.linalg.matrix_power(Ah, j) @ bh for j in range(k)])
        y = K @ np.linalg.solve(K.T @ Ah @ K, K.T @ bh)
        x, r, h = orc.pcg_jacobi(A, b, tau=0.0, max_iters=k, history=True)
        assert r.iterations == k
        assert _rel(x, dh * y) <= 1e-10, (k, _rel(x, dh * y))
        assert abs(h[k] - np.linalg.norm(b - D @ x)) <= 1e-10 * np.linalg.norm(b)


def pin_pcg_dense_solve(orc):
    for seed in range(2):
        A, D = _scaled_spd(30, seed)
        b = inputs.rhs(30, seed)
        x, r, _ = orc.pcg_jacobi(A, b, tau=1e-12, max_iters=500)
        assert r.stop_reason == 1
        assert _rel(x, np.linalg.solve(D, b)) <= np.linalg.cond(D) * 1e-12 * 10
        _, rc, _ = orc.cg(A, b, tau=1e-12, max_iters=500)
        assert r.iterations < rc.iterations   # the scaling is what Jacobi undoes


def pin_pcg_stop_semantics(orc):
    A = inputs.laplacian1d(6)
    x0 = np.arange(6.0)
    # zero diagonal entry: no preconditioner, breakdown before the first iteration
    Z = inputs.diagonal(np.array([1.0, 0.0, 2.0]))
    x, r, _ = orc.pcg_jacobi(Z, np.ones(3), x0=np.array([1.0, 2.0, 3.0]), tau=1e-12)
    assert r.stop_reason == 3 and r.iterations == 0 and np.array_equal(x, [1.0, 2.0, 3.0])
    x, r, h = orc.pcg_jacobi(A, np.ones(6), x0=x0, tau=1e-12, max_iters=0, history=True)
    assert r.stop_reason == 2 and r.iterations == 0 and np.array_equal(x, x0)
    assert h[0] == np.linalg.norm(np.ones(6) - A.to_dense() @ x0)
    x, r, _ = orc.pcg_jacobi(A, np.zeros(6), x0=x0, tau=1e-12)
    assert r.stop_reason == 1 and r.iterations == 0 and np.array_equal(x, np.zeros(6))
    x, r, _ = orc.pcg_jacobi(inputs.laplacian1d(20), np.ones(20), tau=1e-15, max_iters=3)
    assert r.stop_reason == 2 and r.iterations == 3
    # indefinite with a positive diagonal: p.q < 0 on the first step
    _, r, _ = orc.pcg_jacobi(inputs.from_dense(np.array([[1.0, 2.0], [2.0, 1.0]])), np.array([1.0, -1.0]),
                             tau=1e-12)
    assert r.stop_reason == 3 and r.iterations == 0


# ----------------------------------------------------------------- partition, kappa
def pin_partition(orc):
    for rp in (inputs.stencil7(5, 0).row_ptr, inputs.randsym(300, 2).row_ptr,
               np.array([0, 0, 0, 5, 5, 9, 9, 9, 20, 20, 20], np.int64),
               np.array([0, 0, 0], np.int64)):
        n = rp.size - 1
        nnz = int(rp[-1])
        for P in (1, 2, 3, 7, 64, 1000):
            s = orc.partition(rp, P)
            targets = np.array([(j * nnz) // P for j in range(P)], np.int64)
            ref = np.searchsorted(rp, targets, side="left")
            assert np.array_equal(s[:P], ref) and s[P] == n


def pin_residual_norm_rows(orc):
    """The block-by-block residual norm (for matrices too large to assemble)
    equals ||b - A x||_2 of the assembled matrix by scipy.sparse for any split
    of the rows into blocks; x = 0 gives ||b||; closed forms on a dyadic
    diagonal system: 0 for the exact solution, 1 and 5 (a 3-4-5 triple) for
    solutions off by whole units in chosen rows."""
    import scipy.sparse as sp
    for N, f32x, seed in ((9, False, 3), (7, True, 4)):
        A = inputs.stencil7(N, seed, f32x=f32x)
        n = A.n_rows
        S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(n, n))
        b = inputs.rhs(n, seed)
        x = inputs.vec(n, seed, 5)
        ref = float(np.linalg.norm(b - S @ x))

        def mk(r0, r1):
            return inputs.stencil7_block(N, seed, r0, r1, f32x=f32x)

        for bs in (n, 1, 100, 97):
            blocks = [(r, min(r + bs, n)) for r in range(0, n, bs)]
            got = orc.residual_norm_rows(blocks, mk, b, x)
            assert abs(got - ref) <= 1e-13 * ref, (N, bs, got, ref)
        z = orc.residual_norm_rows([(0, n // 3), (n // 3, n)], mk, b, np.zeros(n))
        assert abs(z - np.linalg.norm(b)) <= 1e-14 * np.linalg.norm(b)
    d = np.array([2.0, 4.0, 0.5, 1.0, 8.0, 1.0])
    xs = np.array([1.0, -0.5, 3.0, 0.25, 2.0, -1.0])
    bd = d * xs                                   # exact in FP64

    def mkd(r0, r1):
        return np.arange(r1 - r0 + 1, dtype=np.int64), np.arange(r0, r1, dtype=np.int64), d[r0:r1]

    blocks = [(0, 2), (2, 5), (5, 6)]
    assert orc.residual_norm_rows(blocks, mkd, bd, xs) == 0.0
    x1 = xs.copy()
    x1[3] -= 1.0                                  # row 3: d = 1, residual 1
    assert orc.residual_norm_rows(blocks, mkd, bd, x1) == 1.0
    x2 = xs.copy()
    x2[3] -= 3.0                                  # residual 3 in row 3 ...
    x2[5] += 4.0                                  # ... and -4 in the last row: norm 5
    assert orc.residual_norm_rows(blocks, mkd, bd, x2) == 5.0


def pin_gershgorin(orc):
    d = np.array([2.0, 8.0, 0.5, 3.0])
    assert orc.gershgorin_kappa(inputs.diagonal(d)) == 16.0
    for seed in range(3):
        A = inputs.randsym(30, seed, delta=0.2)
        ev = np.linalg.eigvalsh(A.to_dense())
        kg = orc.gershgorin_kappa(A)
        assert ev[0] > 0 and ev[-1] / ev[0] <= kg * (1 + 1e-12)
    assert math.isinf(orc.gershgorin_kappa(inputs.laplacian1d(5)))   # only weakly dominant


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
