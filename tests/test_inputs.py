"""The seeded input generators: published RNG values, structure, determinism."""
import numpy as np

import inputs

M64 = (1 << 64) - 1
G = 0x9E3779B97F4A7C15


def _splitmix_next(state):
    """SplitMix64 (Steele, Lea & Flood 2014): returns (new_state, output)."""
    state = (state + G) & M64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return state, z ^ (z >> 31)


def test_splitmix_published_value():
    # first output of SplitMix64 seeded with 0 is 0xE220A8397B1DCDAF
    assert _splitmix_next(0)[1] == 0xE220A8397B1DCDAF


def test_counter_hash_is_splitmix_stream():
    for seed, stream in [(0, 0), (1, 2), (12345, 4)]:
        _, K = _splitmix_next(((seed * G) + stream - G) & M64)   # K = mix64(seed*G + stream)
        st = K
        for ctr in range(5):
            st, out = _splitmix_next(st)
            assert inputs.hash64(seed, stream, ctr) == out


def test_uniform_draws_exact():
    for ctr in range(50):
        h = inputs.hash64(3, 0, ctr)
        assert inputs.unif(3, 0, ctr) == 2.0 * ((h >> 11) * 2.0 ** -53) - 1.0
        v = inputs.unif_f32x(3, 0, ctr)
        assert v == (h >> 40) * 2.0 ** -23 - 1.0 and float(np.float32(v)) == v
        assert -1.0 <= v < 1.0


def _check_spd_structure(A, delta, f32x=False):
    n = A.n_rows
    assert A.row_ptr[0] == 0 and np.all(np.diff(A.row_ptr) >= 1)
    D = {}
    for i in range(n):
        cols = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0), "row %d not strictly ascending" % i
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[(i, int(A.col[k]))] = A.val[k]
    for (i, j), v in D.items():
        assert D[(j, i)] == v, "not bitwise symmetric"
    for i in range(n):
        r = 0.0
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            if A.col[k] != i:
                r += abs(A.val[k])
        d = D[(i, i)]
        if f32x:
            assert d >= r + delta and float(np.float32(d)) == d
        else:
            assert d == r + delta


def test_stencil7_structure():
    for N in (1, 2, 3, 6):
        A = inputs.stencil7(N, 5)
        assert A.nnz == 7 * N ** 3 - 6 * N ** 2 == inputs.stencil7_nnz(N)
        _check_spd_structure(A, 1.0)
    A = inputs.stencil7(5, 2, delta=0.01, f32x=True)
    _check_spd_structure(A, 0.01, f32x=True)
    assert np.array_equal(A.val.astype(np.float32).astype(np.float64), A.val)


def test_stencil7_neighbours():
    N = 4
    A = inputs.stencil7(N, 0)
    for i in range(N ** 3):
        x, y, z = i % N, (i // N) % N, i // (N * N)
        want = sorted([i] + [i + s for s, ok in ((1, x < N - 1), (-1, x > 0), (N, y < N - 1),
                                                  (-N, y > 0), (N * N, z < N - 1), (-N * N, z > 0)) if ok])
        assert list(A.col[A.row_ptr[i]:A.row_ptr[i + 1]]) == want


def test_randsym_structure_and_determinism():
    A = inputs.randsym(300, 9)
    _check_spd_structure(A, 1.0)
    B = inputs.randsym(300, 9)
    assert np.array_equal(A.row_ptr, B.row_ptr) and np.array_equal(A.col, B.col)
    assert np.array_equal(A.val.view(np.uint64), B.val.view(np.uint64))
    C = inputs.randsym(300, 10)
    assert not np.array_equal(A.col, C.col)
    one = inputs.randsym(1, 0)
    assert one.nnz == 1 and one.val[0] == 1.0


def test_randsym_degree_distribution():
    A = inputs.randsym(20000, 1)
    deg = np.diff(A.row_ptr)
    # 1 diagonal + 3 own draws + Poisson(3) incoming, minus rare duplicates
    assert abs(deg.mean() - 7.0) < 0.05 and deg.min() >= 2


def test_powerlaw_structure_and_hubs():
    """randsym plus hub rows: symmetric, strictly dominant (SPD), the hub rows
    hold their drawn partners (minus duplicates) and every other row stays
    randsym-like; the randsym part is the same pattern as randsym(n)."""
    n, seed = 20000, 3
    A = inputs.powerlaw(n, seed, hubs=8, lo=500, hi=4000)
    _check_spd_structure(A, 1.0)
    deg = np.diff(A.row_ptr)
    hubs = inputs.powerlaw_hubs(n, seed, hubs=8, lo=500, hi=4000)
    rows = {r for r, _ in hubs}
    for r, d in hubs:
        assert 500 <= d <= 4000
        assert deg[r] >= 0.9 * d          # duplicates among the draws are merged
    others = np.array([i for i in range(n) if i not in rows])
    assert deg[others].max() < 60 and abs(deg[others].mean() - 7.0) < 0.6
    # removing the hub draws leaves randsym: every randsym entry is present
    R = inputs.randsym(n, seed)
    for i in range(0, n, 997):
        assert set(R.col[R.row_ptr[i]:R.row_ptr[i + 1]]) <= set(A.col[A.row_ptr[i]:A.row_ptr[i + 1]])
    B = inputs.powerlaw(n, seed, hubs=8, lo=500, hi=4000)
    assert np.array_equal(A.col, B.col) and np.array_equal(A.val.view(np.uint64), B.val.view(np.uint64))


def test_rhs_and_instances():
    b = inputs.rhs(1000, 4)
    assert np.all((b >= -1) & (b < 1)) and abs(b.mean()) < 0.1
    assert np.array_equal(b, inputs.rhs(1000, 4))
    sizes, seeds = inputs.instances(256, 4)
    assert sizes.min() >= 1000 and sizes.max() <= 1_000_000
    lg = np.log(sizes)
    assert abs(lg.mean() - (np.log(1e3) + np.log(1e6)) / 2) < 0.4
    assert len(set(seeds.tolist())) == 256


def test_stencil7_block_equals_whole_matrix_rows():
    for N, f32x in ((6, False), (5, True)):
        A = inputs.stencil7(N, 3, delta=0.5, f32x=f32x)
        n = A.n_rows
        for r0, r1 in ((0, n), (0, 1), (7, 60), (n - 1, n), (40, 40)):
            rp, col, val = inputs.stencil7_block(N, 3, r0, r1, delta=0.5, f32x=f32x)
            s, e = A.row_ptr[r0], A.row_ptr[r1]
            assert np.array_equal(rp, A.row_ptr[r0:r1 + 1] - s)
            assert np.array_equal(col, A.col[s:e].astype(np.int64))
            assert np.array_equal(val.view(np.uint64), A.val[s:e].view(np.uint64))


def test_serving_mix_matches_instance_table():
    mats, rhs = inputs.serving_mix(12, 4, 1e3, 2e4, threads=4)
    sizes, seeds = inputs.instances(12, 4, 1e3, 2e4)
    for A, b, n, sd in zip(mats, rhs, sizes, seeds):
        B = inputs.randsym(int(n), int(sd) % (1 << 31))
        assert A.n_rows == int(n) and np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)
        assert np.array_equal(b, inputs.rhs(int(n), int(sd) % (1 << 31)))
