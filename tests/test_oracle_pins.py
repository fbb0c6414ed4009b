"""Pins for the CPU oracle: each check ties it to something other than itself
(a published generator vector, closed forms of the paper's equations,
invariants, brute force, an independent routine, statistics of Eq. 4)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle.oracle as orc
from workloads import make_items, make_queries

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


# ------------------------------------------------------------- generator
def test_splitmix64_published_vector():
    lines = _golden_lines("splitmix64_seed1234567.txt")
    seed = int(lines[0][1])
    expect = [int(x[0]) for x in lines[1:]]
    got = [orc.splitmix64_at(seed, k) for k in range(len(expect))]
    assert got == expect


def test_box_muller_special_points():
    # u1 = 1 gives g = 0 whatever u2 (sqrt(-2 ln 1) = 0).
    top = ((1 << 53) - 1) << 11
    assert orc.box_muller(top, 12345 << 11) == 0.0
    # u2 = 0 -> cos = 1 -> g = +sqrt(-2 ln u1) > 0;  u2 = 1/2 -> cos(pi) = -1.
    h1 = (1 << 52) << 11  # u1 = (2^52 + 1) / 2^53, just above 1/2
    u1 = ((1 << 52) + 1) / 2.0 ** 53
    r = math.sqrt(-2.0 * math.log(u1))
    assert orc.box_muller(h1, 0) == pytest.approx(r, rel=1e-15)
    assert orc.box_muller(h1, (1 << 52) << 11) == pytest.approx(-r, rel=1e-15)
    # u2 = 1/4 -> cos(pi/2) ~ 0.
    assert abs(orc.box_muller(h1, (1 << 51) << 11)) < 1e-15
    # smallest u1 = 2^-53 gives the largest radius sqrt(106 ln 2).
    assert orc.box_muller(0, 0) == pytest.approx(math.sqrt(106 * math.log(2)), rel=1e-15)


def test_projection_is_standard_normal():
    A = orc.projection(7, 64, 2047).astype(np.float64).ravel()  # 131072 entries
    assert A.size >= 1e5
    assert abs(A.mean()) < 5.0 / math.sqrt(A.size)
    assert abs(A.var() - 1.0) < 5.0 * math.sqrt(2.0 / A.size)
    assert stats.kstest(A, "norm").pvalue > 1e-3
    # no serial correlation between consecutive entries (independent draws)
    rho = np.corrcoef(A[:-1], A[1:])[0, 1]
    assert abs(rho) < 5.0 / math.sqrt(A.size)
    # symmetric: P(A > 0) = 1/2
    frac = (A > 0).mean()
    assert abs(frac - 0.5) < 5.0 * 0.5 / math.sqrt(A.size)


def test_projection_counter_layout():
    # Entry (r, c) uses counter r*(d+1)+c: rows do not depend on L, and row 0
    # depends only on c (so it is a prefix across d).
    A1 = orc.projection(99, 8, 10)
    A2 = orc.projection(99, 3, 10)
    assert np.array_equal(A1[:3], A2)
    B1 = orc.projection(99, 1, 5)
    B2 = orc.projection(99, 1, 20)
    assert np.array_equal(B1[0], B2[0, :6])
    assert not np.array_equal(orc.projection(1, 4, 4), orc.projection(2, 4, 4))
    # Counter-based generator: entry (r,c) equals the standalone draw.
    d = 10
    r, c = 5, 7
    t = r * (d + 1) + c
    g = orc.box_muller(orc.splitmix64_at(99, 2 * t), orc.splitmix64_at(99, 2 * t + 1))
    assert A1[r, c] == np.float32(g)


# ------------------------------------------------------------- keys / ranking
def test_keys_exact_on_integers():
    rng = np.random.default_rng(0)
    X = rng.integers(-1000, 1000, size=(50, 37)).astype(np.float32)
    k = orc.keys(X)
    exact = np.array([sum(int(v) * int(v) for v in row) for row in X.astype(np.int64)])
    assert np.array_equal(k, exact.astype(np.float64))


def test_keys_ascending_order():
    # Sequential ascending sum: 1 + 2^-54 + 2^-54 + 2^-54 + 2^-54 rounds to 1
    # at every step; the reverse order would reach 1 + 2^-52.
    e = 2.0 ** -27
    X = np.array([[1.0, e, e, e, e], [e, e, e, e, 1.0]], dtype=np.float32)
    k = orc.keys(X)
    assert k[0] == 1.0
    assert k[1] == 1.0 + 2.0 ** -52


def test_rank_brute_force_with_ties():
    rng = np.random.default_rng(1)
    base = rng.standard_normal((20, 6)).astype(np.float32)
    X = np.concatenate([base, base[::2], base[:5]])  # duplicates -> equal keys
    key = orc.keys(X)
    rank = orc.ranks(key)
    order = sorted(range(len(key)), key=lambda i: (key[i], i))
    expect = np.empty(len(key), dtype=np.int64)
    for pos, i in enumerate(order):
        expect[i] = pos
    assert np.array_equal(rank, expect)


@pytest.mark.parametrize("n,m", [(10, 3), (1000, 8), (1001, 7), (64, 64), (5, 1), (97, 13)])
def test_partition_invariants(n, m):
    X = make_items("lognormal", n, 9, seed=n + m, sigma=0.9)
    key = orc.keys(X)
    rank = orc.ranks(key)
    sid, keymax, U = orc.partition(key, rank, m)
    sizes = np.bincount(sid, minlength=m)
    assert set(sizes.tolist()) <= {n // m, -(-n // m)}
    assert sizes.sum() == n
    # every item of S_{j-1} has a key <= every item of S_j
    for j in range(1, m):
        assert key[sid == j - 1].max() <= key[sid == j].min()
        assert U[j - 1] <= U[j]
    for j in range(m):
        assert keymax[j] == key[sid == j].max()
    # U_m is the global max 2-norm (computed independently in FP64 via numpy)
    norms = np.linalg.norm(X.astype(np.float64), axis=1)
    assert U[-1] == pytest.approx(norms.max(), rel=1e-14)
    # subset j holds ranks [ceil(jn/m), ceil((j+1)n/m))
    for j in range(m):
        lo, hi = -(-j * n // m), -(-(j + 1) * n // m)
        assert np.array_equal(np.sort(rank[sid == j]), np.arange(lo, hi))


# ------------------------------------------------------------- uniform partition
def _integer_norm_items(norms):
    """Items whose 2-norms are the given integers: (3k, 4k) has norm 5k, so
    every key (a sum of integer squares) is exact."""
    X = np.zeros((len(norms), 2), np.float32)
    X[:, 0] = np.asarray(norms, np.float32)
    return X


def test_uniform_partition_hand_worked():
    """Section 5's alternative: the norm domain [1, 10] cut into 3 ranges of
    width 3 gives boundaries 4 and 7; an item exactly on a boundary belongs
    to the upper range.  Percentile partitioning of the same 10 items gives
    sizes 4, 3, 3 instead."""
    X = _integer_norm_items(range(1, 11))
    ix = orc.OracleIndex(X, 3, 8, 1, partition="uniform")
    assert ix.sid.tolist() == [0, 0, 0, 1, 1, 1, 2, 2, 2, 2]
    assert ix.keymax.tolist() == [9.0, 36.0, 100.0]
    assert ix.U.tolist() == [3.0, 6.0, 10.0]
    px = orc.OracleIndex(X, 3, 8, 1)
    assert np.bincount(px.sid).tolist() == [4, 3, 3]


def test_uniform_partition_empty_and_degenerate_ranges():
    # norms {1, 2, 9, 10} with m = 3: ranges [1,4) [4,7) [7,10] -> sizes 2, 0, 2
    ix = orc.OracleIndex(_integer_norm_items([1, 2, 9, 10]), 3, 8, 1, partition="uniform")
    assert ix.sid.tolist() == [0, 0, 2, 2]
    assert ix.keymax.tolist() == [4.0, 0.0, 100.0] and ix.U[1] == 0.0
    # all norms equal: zero width, every boundary equals the norm -> last range
    ix = orc.OracleIndex(_integer_norm_items([5] * 7), 4, 8, 1, partition="uniform")
    assert ix.sid.tolist() == [3] * 7
    # m = 1 is the whole dataset, as with percentiles
    X = make_items("lognormal", 300, 7, seed=5, sigma=0.8)
    a = orc.OracleIndex(X, 1, 16, 2, partition="uniform")
    b = orc.OracleIndex(X, 1, 16, 2)
    assert np.array_equal(a.sid, b.sid) and np.array_equal(a.codes, b.codes)


@pytest.mark.parametrize("m", [2, 7, 32])
def test_uniform_partition_ranges_have_equal_width(m):
    """Every item lies in its range [nmin + j w, nmin + (j+1) w] of the norm
    domain (checked on norms computed independently with numpy), ranges are
    ordered, and keymax_j is the largest key of range j."""
    X = make_items("lognormal", 2000, 11, seed=m, sigma=1.0)
    ix = orc.OracleIndex(X, m, 16, 3, partition="uniform")
    norms = np.linalg.norm(X.astype(np.float64), axis=1)
    nmin, nmax = norms.min(), norms.max()
    w = (nmax - nmin) / m
    tol = 1e-12 * nmax
    for j in range(m):
        sel = ix.sid == j
        if sel.any():
            assert norms[sel].min() >= nmin + j * w - tol
            assert norms[sel].max() <= nmin + (j + 1) * w + tol
            assert ix.keymax[j] == ix.key[sel].max()
        else:
            assert ix.keymax[j] == 0.0
    order = np.argsort(norms, kind="stable")
    assert np.all(np.diff(ix.sid[order]) >= 0)


# ------------------------------------------------------------- transform / hash
def test_transform_unit_norm_and_inner_product():
    n, d, m = 400, 33, 5
    X = make_items("lognormal", n, d, seed=3, sigma=1.0)
    q = make_queries(1, d, seed=4)[0]
    key = orc.keys(X)
    sid, keymax, U = orc.partition(key, orc.ranks(key), m)
    for i in range(n):
        s = sid[i]
        v = orc.transform(X[i], key[i], keymax[s], U[s])
        assert abs(float(np.dot(v, v)) - 1.0) <= 4 * 2.0 ** -52 * (d + 1) + 1e-15
        # P(q)^T P(x) * U_j = q^T x  (Eq. 8 with P(q) = [q; 0])
        lhs = float(np.dot(q.astype(np.float64), v[:d])) * U[s]
        rhs = float(np.dot(q.astype(np.float64), X[i].astype(np.float64)))
        assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-12)
    # the largest item of each subset has a zero last coordinate
    for j in range(m):
        i = int(np.flatnonzero((sid == j) & (key == keymax[j]))[0])
        assert orc.transform(X[i], key[i], keymax[j], U[j])[d] == 0.0


def test_transform_zero_subset():
    v = orc.transform(np.zeros(4, np.float32), 0.0, 0.0, 0.0)
    assert np.array_equal(v, [0, 0, 0, 0, 1.0])


def test_hash_basis_vectors():
    L, d = 40, 12
    A = orc.projection(5, L, d)
    for c in range(d + 1):
        e = np.zeros(d + 1)
        e[c] = 1.0
        code = orc.hash_vec(A, e)
        expect = sum(1 << r for r in range(L) if A[r, c] > 0)
        assert code == expect
        code_neg = orc.hash_vec(A, -e)
        assert code_neg == sum(1 << r for r in range(L) if A[r, c] < 0)


def test_sign_of_zero_is_bit_zero():
    """sign(0) maps to bit 0: a zero vector hashes to the all-zero code."""
    A = orc.projection(3, 64, 9)
    assert orc.hash_vec(A, np.zeros(10)) == 0
    assert orc.query_code(A, np.zeros(9, np.float32)) == 0
    # exact cancellation: v = e_a * A[r,b] - e_b * A[r,a] has A_r . v = 0 for row r
    r, a, b = 5, 2, 7
    v = np.zeros(10)
    v[a], v[b] = float(A[r, b]), -float(A[r, a])
    assert (orc.hash_vec(A, v) >> r) & 1 == 0
    assert (orc.hash_vec(A, -v) >> r) & 1 == 0


def test_query_code_symmetries():
    L, d = 64, 20
    A = orc.projection(11, L, d)
    Q = make_queries(50, d, seed=12)
    full = (1 << L) - 1
    for q in Q:
        c = orc.query_code(A, q)
        assert orc.query_code(A, -q) == (~c) & full  # sign flip complements bits
        assert orc.query_code(A, 2.0 * q) == c  # positive scaling invariant
    # basis query: bit r = [A_rt > 0] (the (d+1)-th coordinate of P(q) is 0)
    for t in range(d):
        e = np.zeros(d, np.float32)
        e[t] = 1.0
        assert orc.query_code(A, e) == sum(1 << r for r in range(L) if A[r, t] > 0)


def test_same_bits_brute_force():
    rng = np.random.default_rng(2)
    for L in (1, 7, 16, 31, 32, 33, 64):
        for _ in range(50):
            a = int(rng.integers(0, 1 << L, dtype=np.uint64)) if L < 64 else int(rng.integers(0, 2**63)) * 2 + 1
            b = int(rng.integers(0, 1 << L, dtype=np.uint64)) if L < 64 else int(rng.integers(0, 2**63))
            a &= (1 << L) - 1
            b &= (1 << L) - 1
            assert orc.same_bits(a, b, L) == L - bin(a ^ b).count("1")


def _angle_pair(dim, theta, rng):
    u = rng.standard_normal(dim)
    u /= np.linalg.norm(u)
    w = rng.standard_normal(dim)
    w -= np.dot(w, u) * u
    w /= np.linalg.norm(w)
    return u, math.cos(theta) * u + math.sin(theta) * w


@pytest.mark.parametrize("deg", [10, 45, 90, 135])
def test_srp_collision_rate(deg):
    """Eq. 4: P[h(x) = h(y)] = 1 - theta/pi, over fresh projections."""
    rng = np.random.default_rng(deg)
    theta = math.radians(deg)
    dim = 9  # hash_vec works on (d+1)-vectors; d = 8
    x, y = _angle_pair(dim, theta, rng)
    L, seeds = 64, 1600
    same = 0
    for s in range(seeds):
        A = orc.projection(1000 + s, L, dim - 1)
        same += orc.same_bits(orc.hash_vec(A, x), orc.hash_vec(A, y), L)
    B = L * seeds
    p = 1.0 - theta / math.pi
    assert abs(same - B * p) <= 5.0 * math.sqrt(B * p * (1 - p))


def test_item_query_collision_rate():
    """Section 3.3: an item x in S_j and the query collide on one bit with
    probability 1 - arccos(q.x / U_j) / pi."""
    rng = np.random.default_rng(77)
    d = 8
    q = rng.standard_normal(d)
    q /= np.linalg.norm(q)
    # item with ||x|| = 0.6 and angle 50 degrees to q; subset max norm U_j = 1.5
    w = rng.standard_normal(d)
    w -= np.dot(w, q) * q
    w /= np.linalg.norm(w)
    x = 0.6 * (math.cos(math.radians(50)) * q + math.sin(math.radians(50)) * w)
    x32, q32 = x.astype(np.float32), q.astype(np.float32)
    key = np.array([float(np.dot(x32.astype(np.float64), x32.astype(np.float64)))])
    Uj = 1.5
    L, seeds = 64, 1600
    same = 0
    for s in range(seeds):
        A = orc.projection(5000 + s, L, d)
        code = orc.item_codes(x32[None], A, key, np.zeros(1, np.int32), np.array([Uj * Uj]),
                              np.array([Uj]))[0]
        same += orc.same_bits(int(code), orc.query_code(A, q32), L)
    B = L * seeds
    ip = float(np.dot(q32.astype(np.float64), x32.astype(np.float64)))
    p = 1.0 - math.acos(ip / Uj) / math.pi
    assert abs(same - B * p) <= 5.0 * math.sqrt(B * p * (1 - p))


def test_equal_norms_reduce_to_single_subset():
    """All items with the same 2-norm: every U_j = U, so the codes equal the
    single-subset (SimpleLSH) codes (Section 3.2 remark)."""
    rng = np.random.default_rng(5)
    base = np.array([3, -1, 2, 0, 5, -4], dtype=np.float32)
    X = np.stack([rng.permutation(base) * rng.choice([-1, 1], size=6) for _ in range(60)])
    X = X.astype(np.float32)
    i1 = orc.OracleIndex(X, 1, 32, seed=9)
    i4 = orc.OracleIndex(X, 4, 32, seed=9)
    assert np.all(i1.key == i1.key[0])
    assert np.array_equal(i1.codes, i4.codes)


# ------------------------------------------------------------- rank table
def test_rank_table_hand_worked_golden():
    lines = _golden_lines("rank_table_U1_U2_L2.txt")
    U = np.array([float(v) for v in lines[0][1:]])
    L = int(lines[1][1])
    expect = np.array([[int(v) for v in row[1:]] for row in lines[2:]])
    R, shat = orc.rank_table(U, L)
    assert np.array_equal(R, expect)


@pytest.mark.parametrize("L", [1, 2, 15, 16, 31, 32, 64])
def test_rank_table_closed_forms(L):
    rng = np.random.default_rng(L)
    m = 9
    U = np.sort(rng.lognormal(0, 1, m))
    U[0] = 0.0  # an all-zero subset
    R, shat = orc.rank_table(U, L)
    assert sorted(R.ravel().tolist()) == list(range(m * (L + 1)))
    for j in range(m):
        assert shat[j, L] == U[j]  # cos(0) = 1
        assert shat[j, 0] == -U[j]  # cos(pi) = -1 by antisymmetry
        if L % 2 == 0:
            assert shat[j, L // 2] == 0.0
        for l in range(L + 1):
            assert shat[j, l] == -shat[j, L - l]
            assert shat[j, l] == pytest.approx(U[j] * math.cos(math.pi * (1 - l / L)), abs=1e-15 * max(1, U[j]))
        assert np.all(np.diff(R[j]) < 0)  # better l probes earlier
    # probing order is descending s_hat
    order = np.argsort(R.ravel())
    s_sorted = shat.ravel()[order]
    assert np.all(np.diff(s_sorted) <= 0)


def test_rank_table_single_subset_is_hamming():
    L = 16
    R, _ = orc.rank_table(np.array([2.5]), L)
    assert np.array_equal(R[0], L - np.arange(L + 1))


def test_rank_table_eps_zero_crossing():
    """Adjusted metric: cos[pi(1-eps)(1-l/L)] < 0 only when
    l < L [1/2 - eps / (2 (1 - eps))]  (Section 3.3)."""
    for L, eps in [(16, 0.25), (32, 0.1), (64, 0.05)]:
        bound = L * (0.5 - eps / (2 * (1 - eps)))
        for l in range(L + 1):
            c = orc.cos_level(l, L, eps)
            assert (c < 0) == (l < bound)


# ------------------------------------------------------------- candidates / top-k
def _hamming_ranking(codes, qcode, L, T):
    """Independent SimpleLSH Hamming ranking: items by (identical bits desc, index asc)."""
    same = np.array([L - bin(int(c) ^ qcode).count("1") for c in codes])
    order = np.lexsort((np.arange(len(codes)), -same))
    return order[:min(T, len(codes))]


def _bucket_walk(ix, q, T):
    """Probe by walking the sorted (U_j, l) structure best-first and listing
    each bucket's items in index order (the traversal of Section 3.3)."""
    qc = ix.query_code(q)
    same = np.array([ix.L - bin(int(c) ^ qc).count("1") for c in ix.codes])
    pairs = sorted(((ix.R[j, l], j, l) for j in range(ix.m) for l in range(ix.L + 1)))
    out = []
    for _, j, l in pairs:
        for i in np.flatnonzero((ix.sid == j) & (same == l)):
            if len(out) == min(T, ix.n):
                return out
            out.append(int(i))
    return out


def test_single_subset_candidates_equal_hamming_ranking():
    X = make_items("lognormal", 700, 16, seed=8, sigma=0.7)
    Q = make_queries(10, 16, seed=9)
    ix = orc.OracleIndex(X, 1, 16, seed=3)
    for q in Q:
        for T in (1, 17, 100, 699, 700, 5000):
            cand, _ = ix.candidates(q, T)
            assert np.array_equal(np.sort(cand), np.sort(_hamming_ranking(ix.codes, ix.query_code(q), 16, T)))


@pytest.mark.parametrize("m,L", [(4, 8), (7, 16), (16, 5)])
def test_candidates_equal_bucket_walk(m, L):
    X = make_items("lognormal", 300, 10, seed=m * L, sigma=1.0)
    Q = make_queries(6, 10, seed=m + L)
    ix = orc.OracleIndex(X, m, L, seed=21)
    for q in Q:
        for T in (1, 9, 50, 299, 300, 301):
            cand, _ = ix.candidates(q, T)
            assert sorted(cand.tolist()) == sorted(_bucket_walk(ix, q, T))


def test_candidates_nested_exhaustive_tiny():
    X = make_items("lognormal", 40, 5, seed=31, sigma=1.2)
    X[7] = X[3]  # duplicate row
    Q = make_queries(4, 5, seed=32)
    ix = orc.OracleIndex(X, 5, 6, seed=4)
    for q in Q:
        prev = set()
        for T in range(1, 45):
            cur = set(ix.candidates(q, T)[0].tolist())
            assert len(cur) == min(T, 40)
            assert prev <= cur
            prev = cur


def _exact_topk(X, q, k):
    """Exact rational inner products, order (ip desc, index asc)."""
    qf = [Fraction(float(v)) for v in q]
    ips = [sum(a * Fraction(float(b)) for a, b in zip(qf, row)) for row in X]
    order = sorted(range(len(X)), key=lambda i: (-ips[i], i))
    return order[:k]


def test_full_budget_is_exact_mips():
    X = make_items("lognormal", 120, 7, seed=41, sigma=0.8)
    Q = make_queries(8, 7, seed=42)
    X[50] = X[10] = 64.0 * Q[0]  # the two best items for Q[0] tie; index 10 wins
    X[90] = X[30] = -64.0 * Q[1]  # a tie at the bottom for Q[1]
    ix = orc.OracleIndex(X, 6, 16, seed=5)
    ids, ips = ix.query(Q, k=5, T=120)
    for qi, q in enumerate(Q):
        assert ids[qi].tolist() == _exact_topk(X, q, 5)
    assert ids[0, :2].tolist() == [10, 50]
    one, _ = ix.query(Q[:1], k=1, T=120)
    assert one[0, 0] == 10
    last, _ = ix.query(-Q[1:2], k=2, T=120)
    assert last[0].tolist() == [30, 90]
    # FP64 inner products within rounding of the exact value
    for qi, q in enumerate(Q):
        for r in range(5):
            exact = float(sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(q, X[ids[qi, r]])))
            assert ips[qi, r] == pytest.approx(exact, rel=1e-14, abs=1e-14)


def test_short_results_are_padded():
    X = make_items("lognormal", 6, 4, seed=51)
    Q = make_queries(2, 4, seed=52)
    ix = orc.OracleIndex(X, 2, 8, seed=6)
    ids, ips = ix.query(Q, k=10, T=3)
    assert np.all(ids[:, 3:] == -1)
    assert np.all(np.isneginf(ips[:, 3:]))
    assert np.all(ids[:, :3] >= 0)


def test_recall_invariant():
    """With an exact rerank, top-k(C_T) meets top-k(S) exactly in C_T."""
    X = make_items("lognormal", 2000, 16, seed=61, sigma=0.6)
    Q = make_queries(10, 16, seed=62)
    ix = orc.OracleIndex(X, 8, 16, seed=7)
    gt, _ = orc.bruteforce(X, Q, 10)
    for T in (50, 200, 2000):
        ids, _ = ix.query(Q, 10, T)
        for qi, q in enumerate(Q):
            cand = set(ix.candidates(q, T)[0].tolist())
            truth = set(gt[qi].tolist())
            assert len(set(ids[qi].tolist()) & truth) == len(cand & truth)
    ids, _ = ix.query(Q, 10, 2000)
    assert np.array_equal(ids, gt)


def test_build_drivers_consistent_and_thread_invariant():
    X = make_items("lognormal", 3000, 24, seed=71, sigma=0.9)
    Q = make_queries(12, 24, seed=72)
    a = orc.OracleIndex(X, 8, 32, seed=11, threads=1)
    b = orc.OracleIndex(X, 8, 32, seed=11, threads=5)
    for name in ("A", "key", "rank", "sid", "keymax", "U", "codes", "R"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name
    # pieces agree with the driver
    key = orc.keys(X)
    assert np.array_equal(key, a.key)
    sid, keymax, U = orc.partition(key, orc.ranks(key), 8)
    assert np.array_equal(sid, a.sid) and np.array_equal(U, a.U)
    assert np.array_equal(orc.projection(11, 32, 24), a.A)
    assert np.array_equal(orc.item_codes(X, a.A, key, sid, keymax, U), a.codes)
    R, _ = orc.rank_table(U, 32)
    assert np.array_equal(R, a.R)
    i1, p1 = a.query(Q, 10, 300, threads=1)
    i2, p2 = b.query(Q, 10, 300, threads=4)
    assert np.array_equal(i1, i2) and np.array_equal(p1, p2)
    # codes use only the low L bits
    assert np.all(a.codes < (1 << 32))


# ------------------------------------------- independent projections per subset
def _per_subset_case(n=500, d=10, m=5, L=12, seed=81):
    X = make_items("lognormal", n, d, seed=seed, sigma=1.0)
    Q = make_queries(8, d, seed=seed + 1)
    ix = orc.OracleIndex(X, m, L, seed=seed + 2, projections="per_subset")
    return X, Q, ix


def test_per_subset_projection_layout():
    """Sub-dataset j draws rows j L .. j L + L - 1 of one m L-row projection, so
    sub-dataset 0 sees the shared projection and every block is fresh."""
    X, Q, ix = _per_subset_case()
    m, L, d = ix.m, ix.L, ix.d
    assert ix.A.shape == (m * L, d + 1)
    assert np.array_equal(ix.A, orc.projection(ix.seed, m * L, d))
    assert np.array_equal(ix.A[:L], orc.projection(ix.seed, L, d))
    for j in range(1, m):
        assert not np.array_equal(ix.A[j * L:(j + 1) * L], ix.A[:L])


def test_per_subset_item_codes_use_own_rows():
    """An item of sub-dataset j hashes exactly as the shared-projection routine
    does with A_j; with m >= 2 these codes differ from the ones A_0 gives, so a
    dropped sub-dataset offset fails here."""
    X, Q, ix = _per_subset_case()
    m, L = ix.m, ix.L
    differs = 0
    for j in range(m):
        Aj = ix.A[j * L:(j + 1) * L]
        own = orc.item_codes(X, Aj, ix.key, ix.sid, ix.keymax, ix.U)
        sel = ix.sid == j
        assert np.array_equal(ix.codes[sel], own[sel]), j
        if j:
            base = orc.item_codes(X, ix.A[:L], ix.key, ix.sid, ix.keymax, ix.U)
            differs += int(np.count_nonzero(base[sel] != own[sel]))
    assert differs > 0
    assert np.array_equal(
        orc.item_codes(X, ix.A, ix.key, ix.sid, ix.keymax, ix.U, per_subset=True), ix.codes)


def test_per_subset_query_codes_basis():
    X, Q, ix = _per_subset_case()
    m, L, d = ix.m, ix.L, ix.d
    for q in Q:
        qc = ix.query_code(q)
        assert qc.shape == (m,)
        for j in range(m):
            assert int(qc[j]) == orc.query_code(ix.A[j * L:(j + 1) * L], q)
    for t in range(d):
        e = np.zeros(d, np.float32)
        e[t] = 1.0
        qc = ix.query_code(e)
        for j in range(m):
            rows = ix.A[j * L:(j + 1) * L, t]
            assert int(qc[j]) == sum(1 << r for r in range(L) if rows[r] > 0)


def test_per_subset_single_subset_equals_shared():
    X = make_items("pareto", 600, 12, seed=91, alpha=2.5)
    Q = make_queries(10, 12, seed=92)
    a = orc.OracleIndex(X, 1, 20, seed=93)
    b = orc.OracleIndex(X, 1, 20, seed=93, projections="per_subset")
    assert np.array_equal(a.A, b.A) and np.array_equal(a.codes, b.codes)
    for T in (1, 50, 600):
        ia, pa = a.query(Q, 10, T)
        ib, pb = b.query(Q, 10, T)
        assert np.array_equal(ia, ib) and np.array_equal(pa, pb)


def _bucket_walk_per_subset(ix, q, T):
    """Best-first walk over (U_j, l) where l counts agreement with the query
    code of the item's own sub-dataset."""
    qc = ix.query_code(q)
    same = np.array([ix.L - bin(int(c) ^ int(qc[s])).count("1") for c, s in zip(ix.codes, ix.sid)])
    pairs = sorted(((ix.R[j, l], j, l) for j in range(ix.m) for l in range(ix.L + 1)))
    out = []
    for _, j, l in pairs:
        for i in np.flatnonzero((ix.sid == j) & (same == l)):
            if len(out) == min(T, ix.n):
                return out
            out.append(int(i))
    return out


@pytest.mark.parametrize("m,L", [(4, 8), (9, 16)])
def test_per_subset_candidates_equal_bucket_walk(m, L):
    X = make_items("lognormal", 300, 10, seed=m * L + 1, sigma=1.0)
    Q = make_queries(6, 10, seed=m + L + 1)
    ix = orc.OracleIndex(X, m, L, seed=22, projections="per_subset")
    shared = orc.OracleIndex(X, m, L, seed=22)
    moved = 0
    for q in Q:
        for T in (1, 9, 50, 299, 300, 301):
            cand, ls = ix.candidates(q, T)
            assert sorted(cand.tolist()) == sorted(_bucket_walk_per_subset(ix, q, T))
            qc = ix.query_code(q)
            for c, l in zip(cand, ls):
                assert l == L - bin(int(ix.codes[c]) ^ int(qc[ix.sid[c]])).count("1")
            moved += set(cand.tolist()) != set(shared.candidates(q, T)[0].tolist())
    assert moved > 0


def test_per_subset_full_budget_is_exact_mips():
    X = make_items("lognormal", 150, 7, seed=95, sigma=0.8)
    Q = make_queries(6, 7, seed=96)
    ix = orc.OracleIndex(X, 6, 16, seed=97, projections="per_subset")
    ids, _ = ix.query(Q, k=5, T=150)
    for qi, q in enumerate(Q):
        assert ids[qi].tolist() == _exact_topk(X, q, 5)


# ---------------------------------------------------------------- multi-table single probe
def _np_query_codes(A, q, L):
    """Codes of P(q) = [q; 0] for each L-row block of A, by numpy (FP64 dot
    products of float32 entries): independent of the oracle's loops."""
    out = []
    for b in range(A.shape[0] // L):
        s = A[b * L:(b + 1) * L, :-1].astype(np.float64) @ q.astype(np.float64)
        out.append(sum(1 << r for r in range(L) if s[r] > 0.0))
    return out


def test_multi_table_layout_extends_single_table():
    """Table 0 of a multi-table index is the single-table index: the same
    projection rows (the counter rule continues into the later blocks) and the
    same item codes."""
    X = make_items("lognormal", 1500, 12, seed=31, sigma=0.9)
    for proj in ("shared", "per_subset"):
        one = orc.OracleIndex(X, 5, 10, 77, projections=proj)
        three = orc.OracleIndex(X, 5, 10, 77, projections=proj, tables=3)
        rows = one.A.shape[0]
        assert three.A.shape[0] == 3 * rows
        assert np.array_equal(three.A[:rows], one.A)
        assert np.array_equal(three.A, orc.projection(77, 3 * rows, 12))
        assert np.array_equal(three.codes_t[0], one.codes)
        assert not np.array_equal(three.codes_t[1], three.codes_t[0])


@pytest.mark.parametrize("proj", ["shared", "per_subset"])
def test_single_probe_candidates_by_independent_walk(proj):
    """The probed items equal an independent computation: the first table
    whose code for the item's sub-dataset equals the item's code, items
    ordered by (that table, sub-dataset descending, index), cut at T."""
    n, d, m, L, t = 3000, 10, 6, 6, 4
    X = make_items("lognormal", n, d, seed=41, sigma=0.8)
    Q = make_queries(6, d, seed=42)
    ix = orc.OracleIndex(X, m, L, 5, projections=proj, tables=t)
    P = m if proj == "per_subset" else 1
    for q in Q:
        qc = np.array(_np_query_codes(ix.A, q, L), dtype=np.uint64).reshape(t, P)
        assert np.array_equal(qc, ix.query_codes_all(q).reshape(t, P))
        f = np.full(n, -1)
        for tb in range(t - 1, -1, -1):
            hit = ix.codes_t[tb] == qc[tb, ix.sid if P > 1 else 0]
            f[hit] = tb
        members = np.nonzero(f >= 0)[0]
        order = sorted(members.tolist(), key=lambda i: (f[i], -ix.sid[i], i))
        for T in (1, 7, len(order) // 2 + 1, len(order), n):
            got = ix.candidates_single_probe(q, T)
            assert got.tolist() == order[:min(T, len(order))], T


def test_single_probe_membership_rate_closed_form():
    """Sign random projection (Eq. 4) with t independent tables: an item at
    angle theta from the query shares the query's L-bit bucket in one table
    with probability p^L, p = 1 - theta/pi, so it is probed with probability
    1 - (1 - p^L)^t.  One item (m = 1, U = its norm), many seeds."""
    d, L, t = 8, 3, 4
    rng = np.random.Generator(np.random.PCG64(5))
    q = rng.standard_normal(d)
    q /= np.linalg.norm(q)
    w = rng.standard_normal(d)
    w -= (w @ q) * q
    w /= np.linalg.norm(w)
    theta = math.radians(60.0)
    x = (math.cos(theta) * q + math.sin(theta) * w) * 3.0
    X = x.astype(np.float32)[None, :]
    Qf = q.astype(np.float32)
    trials = 3000
    hits = 0
    for seed in range(trials):
        ix = orc.OracleIndex(X, 1, L, 1000 + seed, tables=t)
        hits += len(ix.candidates_single_probe(Qf, 1)) == 1
        ix.close()
    p = 1.0 - theta / math.pi
    prob = 1.0 - (1.0 - p ** L) ** t
    sd = math.sqrt(trials * prob * (1 - prob))
    assert abs(hits - trials * prob) <= 5 * sd, (hits, trials * prob)
    # one table would give p^L: far outside the band
    assert abs(hits - trials * p ** L) > 10 * sd


def test_single_probe_topk_is_exact_over_candidates():
    n, d, m, L, t = 2500, 9, 4, 5, 3
    X = make_items("lognormal", n, d, seed=51, sigma=1.0)
    Q = make_queries(8, d, seed=52)
    ix = orc.OracleIndex(X, m, L, 9, tables=t)
    for T in (3, 40, n):
        ids, ips = ix.query_single_probe(Q, 6, T, threads=2)
        for qi, q in enumerate(Q):
            cand = ix.candidates_single_probe(q, T)
            exact = [sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(q, X[i])) for i in cand]
            order = sorted(range(len(cand)), key=lambda c: (-exact[c], cand[c]))[:6]
            want = [int(cand[c]) for c in order] + [-1] * (6 - len(order))
            assert ids[qi].tolist() == want, (T, qi)
            fin = ids[qi] >= 0
            assert np.all(np.isneginf(ips[qi][~fin]))
