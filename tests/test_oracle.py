"""Pins for the FP64 oracle against things other than itself.

* brute-force enumeration of every legal path on all shapes up to 7x7
  (random costs, small-integer costs with exact ties, constant costs);
* worked closed forms derived from the step set and weights (Sec. V);
* the constant-cost property that every path has the same total weight
  (Sec. V: the weights equal the Manhattan length of each step);
* affine, transpose and self-alignment invariants;
* independent column-order and anti-diagonal-order sweeps, which is the
  paper's exactness claim for ParDTW (Sec. II-D, Sec. V);
* scipy's cosine distance for the cost (Sec. IV);
* central finite differences for the path gradient.
"""
import itertools

import numpy as np
import pytest

import oracle
from tests import brute, parity


def _rand_C(rng, n, m, kind):
    if kind == "rand":
        return rng.uniform(0.0, 1.0, size=(n, m))
    if kind == "int":
        return rng.integers(0, 2, size=(n, m)).astype(np.float64)
    return np.full((n, m), 0.5)


def _codes_from_path(path):
    out = []
    for a, b in zip(path[:-1], path[1:]):
        d = (int(b[0] - a[0]), int(b[1] - a[1]))
        out.append(brute.STEPS.index(d))
    return out


@pytest.mark.parametrize("kind", ["rand", "int", "const"])
def test_brute_force_all_shapes(kind):
    rng = np.random.default_rng({"rand": 11, "int": 12, "const": 13}[kind])
    for n, m in itertools.product(range(1, 8), range(1, 8)):
        for _ in range(3 if kind != "const" else 1):
            C = _rand_C(rng, n, m, kind)
            J, codes, nopt = brute.brute_dtw(C)
            total, BP, _ = oracle.dtw_matrix(C)
            assert oracle.feasible(n, m) == (codes is not None), (n, m)
            if codes is None:
                assert np.isinf(total) and total > 0
                assert oracle.backtrace(BP).shape == (0, 2) or BP[n - 1, m - 1] == oracle.CODE_NONE
                continue
            assert total == pytest.approx(J, rel=1e-12, abs=1e-12), (n, m, kind)
            path = oracle.backtrace(BP)
            assert _codes_from_path(path) == codes, (n, m, kind, nopt)


def test_brute_force_ties_exercised():
    # the integer-cost sweep above must actually contain multi-optimum cases
    rng = np.random.default_rng(12)
    multi = 0
    for n, m in itertools.product(range(3, 8), range(3, 8)):
        for _ in range(3):
            C = _rand_C(rng, n, m, "int")
            _, codes, nopt = brute.brute_dtw(C)
            multi += codes is not None and nopt > 1
    assert multi >= 10


def test_worked_closed_forms():
    rng = np.random.default_rng(3)
    C = rng.uniform(0.1, 1.0, size=(8, 8))
    J = lambda n, m: oracle.dtw_matrix(C[:n, :m])[0]
    assert J(1, 1) == C[0, 0]
    assert J(2, 2) == pytest.approx(C[0, 0] + 2 * C[1, 1])
    assert J(2, 3) == pytest.approx(C[0, 0] + 3 * C[1, 2])
    assert J(3, 2) == pytest.approx(C[0, 0] + 3 * C[2, 1])
    assert J(3, 3) == pytest.approx(C[0, 0] + 2 * C[1, 1] + 2 * C[2, 2])
    assert J(4, 4) == pytest.approx(min(C[0, 0] + 2 * (C[1, 1] + C[2, 2] + C[3, 3]),
                                        C[0, 0] + 3 * C[1, 2] + 3 * C[3, 3],
                                        C[0, 0] + 3 * C[2, 1] + 3 * C[3, 3]))
    for k in (2, 3, 5, 8):
        assert np.isinf(J(k, 1)) and np.isinf(J(1, k))
    # m-1 = 2(n-1): only the all-(1,2) path exists
    n = 4
    m = 2 * (n - 1) + 1
    C2 = rng.uniform(0.1, 1.0, size=(n, m))
    total, BP, _ = oracle.dtw_matrix(C2)
    assert total == pytest.approx(C2[0, 0] + 3 * sum(C2[l, 2 * l] for l in range(1, n)))
    assert _codes_from_path(oracle.backtrace(BP)) == [1] * (n - 1)


def _const_path(n, m):
    # tie rule (lowest code wins) under constant cost: for n <= m first
    # (m-n) steps of (1,2) then (2n-m-1) of (1,1); mirrored for n > m
    if n <= m:
        return [1] * (m - n) + [0] * (2 * n - m - 1)
    return [2] * (n - m) + [0] * (2 * m - n - 1)


@pytest.mark.parametrize("c", [0.5, 1.0, 0.37])
def test_constant_cost_closed_form(c):
    for n, m in [(1, 1), (5, 5), (5, 9), (9, 5), (17, 30), (40, 23), (64, 127), (100, 101)]:
        C = np.full((n, m), c)
        total, BP, _ = oracle.dtw_matrix(C)
        assert total == pytest.approx(c * (n + m - 1), rel=1e-14)
        if c in (0.5, 1.0):
            # sums of these are exact, so every candidate ties exactly and the
            # tie rule alone decides the path
            assert _codes_from_path(oracle.backtrace(BP)) == _const_path(n, m)
        # the constant-cost case in FP32 input form is exact as well
        total32, BP32, _ = oracle.dtw_matrix(C.astype(np.float32))
        if c in (0.5, 1.0):
            assert total32 == c * (n + m - 1)
            assert np.array_equal(BP32, BP)


def test_affine_invariance():
    rng = np.random.default_rng(5)
    for n, m in [(30, 40), (57, 33), (64, 64)]:
        C = rng.uniform(0, 1, (n, m))
        t0, BP0, _ = oracle.dtw_matrix(C)
        for a, b in [(2.0, 0.0), (0.5, 0.25), (3.0, -0.1)]:
            t1, BP1, _ = oracle.dtw_matrix(a * C + b)
            assert t1 == pytest.approx(a * t0 + b * (n + m - 1), rel=1e-12)
            assert np.array_equal(oracle.backtrace(BP1), oracle.backtrace(BP0))


def test_transpose_invariance():
    rng = np.random.default_rng(6)
    for n, m in [(30, 40), (57, 33)]:
        C = rng.uniform(0, 1, (n, m))
        t0, BP0, _ = oracle.dtw_matrix(C)
        t1, BP1, _ = oracle.dtw_matrix(C.T.copy())
        assert t1 == pytest.approx(t0, rel=1e-13)
        assert np.array_equal(oracle.backtrace(BP1)[:, ::-1], oracle.backtrace(BP0))


def _sweep_other_orders(C):
    """Independent re-implementation in column order and in anti-diagonal
    order (k = i + j): D_k needs only diagonals k-2 and k-3."""
    n, m = C.shape
    INF = np.inf

    def cell(D, i, j):
        if i == 0 and j == 0:
            return C[0, 0], 3
        cands = []
        for (di, dj), w in zip(brute.STEPS, brute.WEIGHTS):
            pi, pj = i - di, j - dj
            cands.append(D[pi, pj] + w * C[i, j] if pi >= 0 and pj >= 0 else INF)
        best, code = cands[0], 0
        for r in (1, 2):
            if cands[r] < best:
                best, code = cands[r], r
        return best, (3 if np.isinf(best) else code)

    out = []
    for order in ("col", "diag"):
        D = np.full((n, m), np.nan)
        B = np.full((n, m), -1, dtype=np.int8)
        if order == "col":
            cells = [(i, j) for j in range(m) for i in range(n)]
        else:
            cells = [(i, k - i) for k in range(n + m - 1) for i in range(n) if 0 <= k - i < m]
        for i, j in cells:
            D[i, j], B[i, j] = cell(D, i, j)
        out.append((D, B))
    return out


def test_sweep_order_independence():
    rng = np.random.default_rng(7)
    for n, m in [(13, 17), (20, 11), (25, 25)]:
        C = rng.uniform(0, 1, (n, m))
        _, BP, D = oracle.dtw_matrix(C, want_D=True)
        for D2, B2 in _sweep_other_orders(C):
            assert np.array_equal(B2, BP)
            assert np.array_equal(np.nan_to_num(D2, posinf=1e300), np.nan_to_num(D, posinf=1e300))


def test_cost_matches_scipy_and_properties():
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(8)
    X = rng.normal(size=(37, 12)).astype(np.float32)
    Y = rng.normal(size=(41, 12)).astype(np.float32)
    C = oracle.cost(X, Y)
    ref = cdist(X.astype(np.float64), Y.astype(np.float64), metric="cosine")
    assert np.allclose(C, ref, rtol=0, atol=1e-13)
    assert np.allclose(np.diag(oracle.cost(X, X)), 0.0, atol=1e-14)
    Cs = oracle.cost(X * np.float32(4.0), Y * np.float32(0.25))
    assert np.allclose(Cs, C, atol=1e-14)
    # zero frame reads as the zero vector: cost 1
    Z = X.copy()
    Z[3] = 0
    assert np.all(oracle.cost(Z, Y)[3] == 1.0)


def test_features_matches_matrix_path():
    from paper_2607_15478_amd import synth
    X, Y = synth.chroma_pair(21, 300, 360)
    C = oracle.cost(X, Y)
    t0, BP0, _ = oracle.dtw_matrix(C)
    t1, BP1 = oracle.dtw_features(X, Y)
    assert t0 == t1
    assert np.array_equal(BP0, BP1)


def test_path_properties_and_rescore():
    from paper_2607_15478_amd import synth
    for n, m, seed in [(200, 240, 1), (333, 250, 2), (150, 290, 3)]:
        X, Y = synth.chroma_pair(seed, n, m, lo=0.8 * (m - 1) / (n - 1), hi=1.25 * (m - 1) / (n - 1))
        total, path, BP = oracle.align(X, Y)
        assert tuple(path[0]) == (0, 0) and tuple(path[-1]) == (n - 1, m - 1)
        steps = np.diff(path, axis=0)
        assert all(tuple(s) in brute.STEPS for s in steps)
        L = len(path)
        assert -(-(n + m - 2) // 3) + 1 <= L <= min(n, m)
        assert oracle.path_cost(X, Y, path) == pytest.approx(total, rel=1e-12)


def test_self_alignment():
    from paper_2607_15478_amd import synth
    rng = np.random.default_rng(9)
    X = synth.chroma_like(rng, 400)
    total, path, _ = oracle.align(X, X)
    assert abs(total) <= 1e-12 * 400
    assert np.array_equal(path, np.stack([np.arange(400)] * 2, 1))


def test_probe_matches_full_D():
    rng = np.random.default_rng(10)
    C = rng.uniform(0, 1, (40, 50)).astype(np.float32)
    _, _, D = oracle.dtw_matrix(C, want_D=True)
    cells = np.array([[i, j] for i in range(0, 40, 3) for j in range(0, 50, 7)])
    cand, dval = oracle.probe(cells, C32=C)
    for (i, j), cd, dv in zip(cells, cand, dval):
        assert dv == D[i, j] or (np.isinf(dv) and np.isinf(D[i, j]))
        for r, ((di, dj), w) in enumerate(zip(brute.STEPS, brute.WEIGHTS)):
            if i - di >= 0 and j - dj >= 0:
                exp = D[i - di, j - dj] + w * float(C[i, j])
                assert cd[r] == exp or (np.isinf(cd[r]) and np.isinf(exp))
            else:
                assert np.isinf(cd[r])


def test_gradient_finite_differences():
    from paper_2607_15478_amd import synth
    X, Y = synth.gaussian_pair(5, 40, 46, d=8, lo=0.8 * 45 / 39, hi=1.25 * 45 / 39)
    total, path, _ = oracle.align(X, Y)
    dX, dY = oracle.path_grad(X, Y, path, 1.0)
    # scale invariance of the cosine: x_i . dX[i] = 0 and y_j . dY[j] = 0
    assert np.allclose(np.sum(dX * X, 1), 0, atol=1e-12)
    assert np.allclose(np.sum(dY * Y, 1), 0, atol=1e-12)
    on_rows = set(path[:, 0].tolist())
    on_cols = set(path[:, 1].tolist())
    for i in range(40):
        if i not in on_rows:
            assert np.all(dX[i] == 0)
    for j in range(46):
        if j not in on_cols:
            assert np.all(dY[j] == 0)
    rng = np.random.default_rng(0)
    eps = 1e-3
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)

    def J_of(Xa, Ya):
        C = 1.0 - (Xa / np.linalg.norm(Xa, axis=1, keepdims=True)) @ (Ya / np.linalg.norm(Ya, axis=1, keepdims=True)).T
        t, BP, _ = oracle.dtw_matrix(C)
        return t, oracle.backtrace(BP)

    checked = 0
    for _ in range(60):
        which = rng.integers(2)
        A = (X64 if which == 0 else Y64).copy()
        r = int(rng.integers(A.shape[0]))
        k = int(rng.integers(A.shape[1]))
        A[r, k] += eps
        tp, pp = J_of(A, Y64) if which == 0 else J_of(X64, A)
        A[r, k] -= 2 * eps
        tm, pm = J_of(A, Y64) if which == 0 else J_of(X64, A)
        if not (np.array_equal(pp, path) and np.array_equal(pm, path)):
            continue  # the optimal path moved: the derivative is one-sided there
        fd = (tp - tm) / (2 * eps)
        an = (dX if which == 0 else dY)[r, k]
        assert fd == pytest.approx(an, rel=1e-4, abs=1e-7)
        checked += 1
    assert checked >= 40


@pytest.mark.parametrize("n,m", [(1, 1), (2, 3), (3, 10), (7, 5), (5, 9), (13, 20), (20, 13), (30, 31), (17, 40)])
def test_band_mask_is_forward_and_backward_reachability(n, m):
    """The band helper used by the parity tests equals the set of cells reached
    from (0,0) by the three steps and reaching (n-1, m-1), found by search."""
    steps = [(1, 1), (1, 2), (2, 1)]
    fwd = np.zeros((n, m), dtype=bool)
    fwd[0, 0] = True
    for i in range(n):
        for j in range(m):
            if fwd[i, j]:
                for di, dj in steps:
                    if i + di < n and j + dj < m:
                        fwd[i + di, j + dj] = True
    bwd = np.zeros((n, m), dtype=bool)
    bwd[n - 1, m - 1] = True
    for i in range(n - 1, -1, -1):
        for j in range(m - 1, -1, -1):
            if bwd[i, j]:
                for di, dj in steps:
                    if i - di >= 0 and j - dj >= 0:
                        bwd[i - di, j - dj] = True
    assert np.array_equal(parity.band_mask(n, m), fwd & bwd)


def _probe_expected(C, D, cells):
    """Candidate totals of the DTW recursion rebuilt from a full D and C."""
    out = np.full((len(cells), 3), np.inf)
    for q, (i, j) in enumerate(cells):
        for r, ((di, dj), w) in enumerate(zip(brute.STEPS, brute.WEIGHTS)):
            if i - di >= 0 and j - dj >= 0:
                out[q, r] = D[i - di, j - dj] + w * float(C[i, j])
    return out


def _one_hot_features(rng, n, d=3):
    """Frames that are unit basis vectors: every cosine distance is exactly 0
    or 1, so candidate totals tie exactly all over the matrix."""
    X = np.zeros((n, d), dtype=np.float32)
    X[np.arange(n), rng.integers(0, d, n)] = 1.0
    return X


@pytest.mark.parametrize("kind", ["chroma", "one_hot"])
def test_probe_features_branch(kind):
    """The tie arbiter of every path audit: oracle.probe(cells, X=, Y=) gives
    the candidate totals and D of the DTW recursion over the cosine cost of
    the features. Expected values come from scipy's cosine distance and the
    brute-force-pinned matrix DP, with exact ties in the one-hot case."""
    from scipy.spatial.distance import cdist

    from paper_2607_15478_amd import synth
    rng = np.random.default_rng(21)
    n, m = 37, 45
    if kind == "chroma":
        X, Y = synth.chroma_pair(rng, n, m)
    else:
        X, Y = _one_hot_features(rng, n), _one_hot_features(rng, m)
    Cs = cdist(X.astype(np.float64), Y.astype(np.float64), "cosine")
    _, _, D = oracle.dtw_matrix(Cs, want_D=True)
    cells = np.array([[i, j] for i in range(n) for j in range(m) if (i * 7 + j * 3) % 5 == 0])
    cand, dval = oracle.probe(cells, X=X, Y=Y)
    exp = _probe_expected(Cs, D, cells)
    fin = np.isfinite(exp)
    assert np.array_equal(np.isfinite(cand), fin)
    np.testing.assert_allclose(cand[fin], exp[fin], rtol=1e-12, atol=1e-12)
    dexp = D[cells[:, 0], cells[:, 1]]
    assert np.array_equal(np.isfinite(dval), np.isfinite(dexp))
    np.testing.assert_allclose(dval[np.isfinite(dexp)], dexp[np.isfinite(dexp)], rtol=1e-12, atol=1e-12)
    if kind == "one_hot":
        # the winner's candidate equals D exactly, and exact ties really occur
        ties = sum(1 for c in cand if np.isfinite(c).sum() >= 2 and np.sort(c)[0] == np.sort(c)[1])
        assert ties > 0
        assert np.all(np.min(cand[np.isfinite(dval) & (cells[:, 0] + cells[:, 1] > 0)], 1)
                      == dval[np.isfinite(dval) & (cells[:, 0] + cells[:, 1] > 0)])


def test_probe_features_brute_force_prefixes():
    """On tiny features, the probe's D at (i, j) is the brute-force optimum of
    the prefix pair X[:i+1], Y[:j+1], and each candidate is the brute-force
    optimum at the step's source plus the weighted cost (no dynamic program
    on the expected side)."""
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(22)
    n, m, d = 6, 7, 4
    X = rng.uniform(0.0, 1.0, (n, d)).astype(np.float32)
    Y = rng.uniform(0.0, 1.0, (m, d)).astype(np.float32)
    Cs = cdist(X.astype(np.float64), Y.astype(np.float64), "cosine")

    def best(i, j):
        return brute.brute_dtw(Cs[:i + 1, :j + 1])[0]

    cells = np.array([[i, j] for i in range(n) for j in range(m)])
    cand, dval = oracle.probe(cells, X=X, Y=Y)
    for q, (i, j) in enumerate(cells):
        b = best(i, j)
        assert (np.isinf(dval[q]) and np.isinf(b)) or dval[q] == pytest.approx(b, rel=1e-12, abs=1e-12)
        for r, ((di, dj), w) in enumerate(zip(brute.STEPS, brute.WEIGHTS)):
            src = best(i - di, j - dj) if (i - di >= 0 and j - dj >= 0) else np.inf
            exp = src + w * Cs[i, j]
            assert (np.isinf(cand[q, r]) and np.isinf(exp)) or cand[q, r] == pytest.approx(exp, rel=1e-12)


@pytest.mark.parametrize("threads", [2, 3, 8])
def test_multithreaded_sweep_bit_identical(threads):
    """The all-core timing variant splits each row's columns over threads; a
    cell needs only rows above it, so codes and total equal the serial
    sweep's bit for bit (on shapes with fewer columns than blocks, too)."""
    from paper_2607_15478_amd import synth
    rng = np.random.default_rng(44)
    for n, m, seed in ((1, 1, 1), (5, 3, 2), (4, 30, 5), (300, 360, 3), (1001, 1203, 4)):
        if n >= 100:
            X, Y = synth.chroma_pair(seed, n, m)
        else:  # tiny and infeasible shapes
            X, Y = synth.chroma_like(rng, n), synth.chroma_like(rng, m)
        J1, B1 = oracle.dtw_features(X, Y)
        Jt, Bt = oracle.dtw_features(X, Y, threads=threads)
        assert (J1 == Jt) or (np.isinf(J1) and np.isinf(Jt))
        assert np.array_equal(B1, Bt)
