"""Pins for the subsequence-DTW and Segmental-DTW parts of the FP64 oracle.

* brute-force enumeration of every subsequence path (any start column on the
  first query row, steps (1,1), (1,2), (2,1) with weights 1, 1, 2; Sec. II-B)
  on all shapes up to 6x7, with random, small-integer (exact ties) and
  constant costs;
* the constant-cost property: the weights equal each step's query advance, so
  every subsequence path weighs exactly n;
* affine invariance of the scores and codes;
* the exactness of the overlapping reference chunks (Sec. III-A);
* brute-force enumeration of every ordered placement of fragment ends for the
  segment-level programs (Sec. II-C step 4; NSDTW's independent minima,
  Sec. II-B) and numpy's argmin for the one-fragment and NSDTW cases;
* self-alignment of a sequence with itself, which Segmental DTW must recover.
"""
import itertools

import numpy as np
import pytest

import oracle

STEPS = ((1, 1), (1, 2), (2, 1))
SUB_W = (1.0, 1.0, 2.0)


def _enumerate_subseq(n, m):
    """Every subsequence path as (start column, codes), by direct recursion."""
    out = []

    def rec(j0, i, j, codes):
        if i == n - 1:
            out.append((j0, list(codes)))
            return
        for c, (di, dj) in enumerate(STEPS):
            if i + di <= n - 1 and j + dj <= m - 1:
                codes.append(c)
                rec(j0, i + di, j + dj, codes)
                codes.pop()

    for j0 in range(m):
        rec(j0, 0, j0, [])
    return out


def _cells(j0, codes):
    cells = [(0, j0)]
    for c in codes:
        cells.append((cells[-1][0] + STEPS[c][0], cells[-1][1] + STEPS[c][1]))
    return cells


def _score(C, j0, codes):
    cells = _cells(j0, codes)
    total = float(C[cells[0]])
    for c, cell in zip(codes, cells[1:]):
        total += SUB_W[c] * float(C[cell])
    return total


def _brute_subseq(C):
    """Per end column: (best score, codes of the selected optimal path). The
    selected path is the optimal one whose codes read backward from the end
    are lexicographically smallest, which is what a backtrace that keeps the
    lowest-index optimal step at every cell recovers."""
    n, m = C.shape
    best = {}
    for j0, codes in _enumerate_subseq(n, m):
        end = _cells(j0, codes)[-1][1]
        s = _score(C, j0, codes)
        best.setdefault(end, []).append((s, j0, codes))
    out = {}
    for end, lst in best.items():
        b = min(s for s, _, _ in lst)
        opt = [(j0, codes) for s, j0, codes in lst if s == b]
        out[end] = (b, min(opt, key=lambda t: tuple(reversed(t[1]))))
    return out


def _codes_of(path):
    return [STEPS.index((int(b[0] - a[0]), int(b[1] - a[1]))) for a, b in zip(path[:-1], path[1:])]


@pytest.mark.parametrize("kind", ["rand", "int", "const"])
def test_subseq_brute_force_all_shapes(kind):
    rng = np.random.default_rng({"rand": 21, "int": 22, "const": 23}[kind])
    for n, m in itertools.product(range(1, 7), range(1, 8)):
        for _ in range(2 if kind != "const" else 1):
            if kind == "rand":
                C = rng.uniform(0.0, 1.0, size=(n, m))
            elif kind == "int":
                C = rng.integers(0, 2, size=(n, m)).astype(np.float64)
            else:
                C = np.full((n, m), 0.5)
            brute = _brute_subseq(C)
            S, BP, _ = oracle.subseq_matrix(C)
            for j in range(m):
                if j not in brute:
                    assert np.isinf(S[j]) and S[j] > 0, (n, m, j)
                    assert not oracle.subseq_reachable(n - 1, j)
                    assert oracle.subseq_backtrace(BP, j).shape == (0, 2)
                    continue
                assert oracle.subseq_reachable(n - 1, j)
                b, (j0, codes) = brute[j]
                assert S[j] == pytest.approx(b, rel=1e-12, abs=1e-12), (n, m, j, kind)
                path = oracle.subseq_backtrace(BP, j)
                assert tuple(path[0]) == (0, j0) and tuple(path[-1]) == (n - 1, j), (n, m, j, kind)
                assert _codes_of(path) == codes, (n, m, j, kind)
                assert oracle.subseq_path_score(C, path) == pytest.approx(b, rel=1e-12, abs=1e-12)


def test_subseq_ties_exercised():
    rng = np.random.default_rng(22)
    multi = 0
    for n, m in itertools.product(range(3, 7), range(3, 8)):
        C = rng.integers(0, 2, size=(n, m)).astype(np.float64)
        per_end = {}
        for j0, codes in _enumerate_subseq(n, m):
            end = _cells(j0, codes)[-1][1]
            per_end.setdefault(end, []).append(_score(C, j0, codes))
        multi += sum(1 for v in per_end.values() if v.count(min(v)) > 1)
    assert multi > 20


def test_subseq_constant_cost_weighs_query_length():
    # every path from the first to the last query row weighs n (Sec. II-B
    # weights 1, 1, 2 = each step's query advance), so S[j] = c n wherever the
    # end is reachable (2j >= n-1)
    for n, m in [(1, 5), (2, 3), (5, 5), (9, 4), (17, 30), (40, 25)]:
        S, BP, D = oracle.subseq_matrix(np.full((n, m), 0.75), want_D=True)
        for j in range(m):
            if 2 * j >= n - 1:
                assert S[j] == 0.75 * n, (n, m, j)
            else:
                assert np.isinf(S[j])
        assert np.all(BP[0] == oracle.CODE_NONE)
        for i in range(n):
            for j in range(m):
                assert np.isfinite(D[i, j]) == oracle.subseq_reachable(i, j)


def test_subseq_first_rows_closed_form():
    rng = np.random.default_rng(24)
    C = rng.uniform(size=(2, 11))
    S, _, _ = oracle.subseq_matrix(C[:1])
    assert np.array_equal(S, C[0])
    S, BP, _ = oracle.subseq_matrix(C)
    # two rows: one (1,1) or (1,2) step from anywhere on the first row
    for j in range(11):
        prev = [C[0, j - 1]] if j >= 1 else []
        prev += [C[0, j - 2]] if j >= 2 else []
        want = min(prev) + C[1, j] if prev else np.inf
        assert S[j] == want


@pytest.mark.parametrize("alpha,beta", [(2.0, 0.25), (0.5, -0.1), (3.0, 1.0)])
def test_subseq_affine_invariance(alpha, beta):
    rng = np.random.default_rng(25)
    for n, m in [(7, 12), (20, 31), (33, 40)]:
        C = rng.uniform(size=(n, m))
        S, BP, _ = oracle.subseq_matrix(C)
        S2, BP2, _ = oracle.subseq_matrix(alpha * C + beta)
        fin = np.isfinite(S)
        assert np.array_equal(np.isfinite(S2), fin)
        assert np.allclose(S2[fin], alpha * S[fin] + beta * n, rtol=1e-12, atol=1e-12)
        reach = np.array([[oracle.subseq_reachable(i, j) for j in range(m)] for i in range(n)])
        assert np.array_equal(BP[reach], BP2[reach])


@pytest.mark.parametrize("n,m", [(1, 9), (4, 30), (10, 64), (25, 200), (60, 333)])
def test_overlapping_chunks_are_exact(n, m):
    # Sec. III-A: a chunk of end columns needs only the 2(n-1) reference
    # columns before it, and the decomposition gives the same scores exactly
    rng = np.random.default_rng(26 + n)
    C = rng.uniform(size=(n, m))
    S, _, _ = oracle.subseq_matrix(C)
    for k in (1, 2, 3, 7, 16):
        S2 = oracle.subseq_chunked(C, k)
        assert np.array_equal(np.isinf(S), np.isinf(S2))
        assert np.array_equal(S[np.isfinite(S)], S2[np.isfinite(S2)]), k


def _brute_placements(S, hop):
    """All end tuples e_0 < ... with e_f - e_{f-1} >= hop and finite scores."""
    nf, m = S.shape
    out = []
    for ends in itertools.product(range(m), repeat=nf):
        if any(ends[f] - ends[f - 1] < hop for f in range(1, nf)):
            continue
        tot = sum(S[f, e] for f, e in enumerate(ends))
        if np.isfinite(tot):
            out.append((tot, ends))
    return out


@pytest.mark.parametrize("kind", ["rand", "int"])
def test_wsdtw_segment_dp_brute_force(kind):
    rng = np.random.default_rng({"rand": 31, "int": 32}[kind])
    for nf, m, hop in itertools.product(range(1, 4), range(1, 8), range(1, 4)):
        for _ in range(2):
            if kind == "rand":
                S = rng.uniform(size=(nf, m))
            else:
                S = rng.integers(0, 3, size=(nf, m)).astype(np.float64)
            # some unreachable ends, as at the start of short references
            S[:, : rng.integers(0, 2)] = np.inf
            total, ends = oracle.segment_ends(S, hop, oracle.WSDTW)
            pl = _brute_placements(S, hop)
            if not pl:
                assert np.isinf(total) and np.all(ends == -1), (nf, m, hop)
                continue
            best = min(t for t, _ in pl)
            assert total == pytest.approx(best, rel=1e-12, abs=1e-12), (nf, m, hop)
            # tie rule: the match replaces the skip only when strictly smaller,
            # so the backtrack keeps the earliest end of the last fragment, then
            # of the one before, ...
            opt = [e for t, e in pl if t == best]
            want = min(opt, key=lambda e: tuple(reversed(e)))
            assert tuple(int(e) for e in ends) == want, (nf, m, hop, kind)


def test_nsdtw_is_independent_argmin():
    rng = np.random.default_rng(33)
    S = rng.integers(0, 4, size=(6, 40)).astype(np.float64)
    S[:, :3] = np.inf
    total, ends = oracle.segment_ends(S, 5, oracle.NSDTW)
    assert np.array_equal(ends, np.argmin(S, axis=1))
    assert total == S.min(axis=1).sum()


def test_one_fragment_wsdtw_is_global_minimum():
    rng = np.random.default_rng(34)
    for m in (1, 5, 100):
        S = rng.uniform(size=(1, m))
        for variant in (oracle.NSDTW, oracle.WSDTW):
            total, ends = oracle.segment_ends(S, 3, variant)
            assert ends[0] == np.argmin(S[0]) and total == S[0].min()


def test_fragment_split_and_hop():
    starts = oracle.fragment_starts(10, 3)
    assert list(starts) == [0, 3, 6, 10]
    for la, nf in [(7, 7), (100, 3), (50000, 32), (1001, 10)]:
        s = oracle.fragment_starts(la, nf)
        lens = np.diff(s)
        assert s[0] == 0 and s[-1] == la and lens.min() >= 1 and lens.max() - lens.min() <= 1
    assert oracle.segment_hop(100, 5) == 10
    assert oracle.segment_hop(5, 4) == 1
    with pytest.raises(ValueError):
        oracle.fragment_starts(3, 4)


def _smooth_features(rng, n, d=12):
    X = rng.uniform(0.0, 1.0, size=(n, d))
    k = np.ones(5) / 5.0
    Xp = np.pad(X, ((2, 2), (0, 0)), mode="edge")
    X = np.stack([np.convolve(Xp[:, c], k, mode="valid") for c in range(d)], axis=1)
    return (X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("nfrag", [1, 2, 5])
def test_segmental_self_alignment(variant, nfrag):
    # aligning a sequence with itself: each fragment's zero-cost match is its
    # own position, so the fragments end where they end in A and the
    # concatenated path is the diagonal
    rng = np.random.default_rng(35)
    X = _smooth_features(rng, 60)
    r = oracle.segmental(X, X, nfrag, variant)
    starts = r["starts"]
    assert np.array_equal(r["ends"], starts[1:] - 1)
    assert np.array_equal(r["path"], np.stack([np.arange(60), np.arange(60)], axis=1))
    assert abs(r["total"]) < 1e-9


@pytest.mark.parametrize("variant", [0, 1])
def test_segmental_brute_force_end_to_end(variant):
    # the whole pipeline on tiny features against path and placement
    # enumeration: per-fragment scores by enumerating subsequence paths, then
    # the best ordered (or independent) placement
    rng = np.random.default_rng(36 + variant)
    for la, lb, nf in [(6, 7, 2), (7, 6, 3), (5, 9, 1), (8, 8, 4)]:
        X = rng.uniform(size=(la, 3)).astype(np.float32)
        Y = rng.uniform(size=(lb, 3)).astype(np.float32)
        r = oracle.segmental(X, Y, nf, variant)
        C = oracle.cost(X, Y)
        starts = oracle.fragment_starts(la, nf)
        S = np.full((nf, lb), np.inf)
        for f in range(nf):
            for end, (b, _) in _brute_subseq(C[starts[f]:starts[f + 1]]).items():
                S[f, end] = b
        assert np.allclose(r["S"][np.isfinite(S)], S[np.isfinite(S)], rtol=1e-12, atol=1e-12)
        assert np.array_equal(np.isfinite(r["S"]), np.isfinite(S))
        hop = oracle.segment_hop(la, nf)
        if variant == oracle.WSDTW:
            pl = _brute_placements(S, hop)
            want = min(t for t, _ in pl) if pl else np.inf
        else:
            want = S.min(axis=1).sum()
        assert r["total"] == pytest.approx(want, rel=1e-12, abs=1e-12)
        if np.isfinite(r["total"]):
            ends = r["ends"]
            if variant == oracle.WSDTW:
                assert np.all(np.diff(ends) >= hop)
            got = sum(S[f, e] for f, e in enumerate(ends))
            assert got == pytest.approx(r["total"], rel=1e-12, abs=1e-12)
            for f, p in enumerate(r["paths"]):
                assert p[0][0] == starts[f] and p[-1][0] == starts[f + 1] - 1 and p[-1][1] == ends[f]
                loc = p.astype(np.int64) - np.array([starts[f], 0])
                sc = oracle.subseq_path_score(C[starts[f]:starts[f + 1]], loc)
                assert sc == pytest.approx(S[f, ends[f]], rel=1e-12, abs=1e-12)


def test_wsdtw_ends_strictly_increase():
    # Sec. II-C: the segment-level path gives strictly increasing fragment ends
    rng = np.random.default_rng(37)
    X = _smooth_features(rng, 300)
    Y = _smooth_features(rng, 360)
    for nf in (2, 4, 8, 16):
        r = oracle.segmental(X, Y, nf, oracle.WSDTW)
        assert np.isfinite(r["total"])
        assert np.all(np.diff(r["ends"]) >= r["hop"]) and r["hop"] >= 1


def test_subseq_matrix_f32_equals_widened_f64():
    """The FP32 branch of subseq_matrix (used by every subsequence GPU test)
    widens each cost exactly and runs the same recursion: its scores, codes
    and D equal, bit for bit, those of the FP64 branch on the widened matrix,
    which the enumeration pins above cover."""
    rng = np.random.default_rng(31)
    for n, m in ((1, 5), (3, 2), (9, 40), (33, 70)):
        for C32 in (rng.uniform(-0.01, 1.0, (n, m)).astype(np.float32),
                    rng.integers(0, 3, (n, m)).astype(np.float32)):
            S1, BP1, D1 = oracle.subseq_matrix(C32, want_D=True)
            S2, BP2, D2 = oracle.subseq_matrix(C32.astype(np.float64), want_D=True)
            assert np.array_equal(S1, S2)
            assert np.array_equal(BP1, BP2)
            assert np.array_equal(D1, D2)


def _sub_candidates(C, D, cells):
    out = np.full((len(cells), 3), np.inf)
    for q, (i, j) in enumerate(cells):
        for r, ((di, dj), w) in enumerate(zip(STEPS, SUB_W)):
            if i - di >= 0 and j - dj >= 0:
                out[q, r] = D[i - di, j - dj] + w * float(C[i, j])
    return out


@pytest.mark.parametrize("src", ["C32", "features"])
def test_subseq_probe(src):
    """subseq_probe gives the subsequence recursion's candidate totals and D
    at chosen cells: rebuilt here from the enumeration-pinned matrix sweep
    (over scipy's cosine distance for the feature branch)."""
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(32)
    n, m = 23, 61
    if src == "C32":
        C = rng.uniform(0.0, 1.0, (n, m)).astype(np.float32)
        Cref = C.astype(np.float64)
    else:
        X = rng.uniform(0.0, 1.0, (n, 5)).astype(np.float32)
        Y = rng.uniform(0.0, 1.0, (m, 5)).astype(np.float32)
        Cref = cdist(X.astype(np.float64), Y.astype(np.float64), "cosine")
    _, _, D = oracle.subseq_matrix(Cref, want_D=True)
    cells = np.array([[i, j] for i in range(n) for j in range(m) if (3 * i + j) % 4 == 1])
    if src == "C32":
        cand, dval = oracle.subseq_probe(cells, C32=C)
    else:
        cand, dval = oracle.subseq_probe(cells, X=X, Y=Y)
    exp = _sub_candidates(Cref, D, cells)
    assert np.array_equal(np.isfinite(cand), np.isfinite(exp))
    fin = np.isfinite(exp)
    np.testing.assert_allclose(cand[fin], exp[fin], rtol=1e-12, atol=1e-12)
    dexp = D[cells[:, 0], cells[:, 1]]
    fd = np.isfinite(dexp)
    assert np.array_equal(np.isfinite(dval), fd)
    np.testing.assert_allclose(dval[fd], dexp[fd], rtol=1e-12, atol=1e-12)
    # row 0 is a free start: D = C there and no candidate is finite
    row0 = cells[:, 0] == 0
    assert np.all(np.isinf(cand[row0]))
