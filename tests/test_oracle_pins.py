"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test compares the oracle with something other than itself: brute force
on the explicit join, an explicit Givens sequence (Claim 1), LAPACK through
numpy, closed forms (Helmert rows, the Gram matrix J^T J, the Frobenius
norm), invariants, and hand values.
"""
import numpy as np
import pytest

import oracle
from bruteforce import (frob2_closed_form, givens_compact_cartesian, gram_closed_form,
                        groups_bruteforce, join_matrix, lapack_r, relF, sign_rows)
from paper_2503_23385_amd import workloads as W


def inst_of(A, B, kA=None, kB=None):
    return W.Instance(np.asarray(A, dtype=np.float64), np.asarray(B, dtype=np.float64),
                      None if kA is None else np.asarray(kA, dtype=np.int32),
                      None if kB is None else np.asarray(kB, dtype=np.int32))


# ---------------------------------------------------------------- groups

KEY_CASES = [
    ([0, 0, 1, 2, 2, 2], [0, 2, 2, 3]),
    ([5, 5, 5], [5, 5]),
    ([1, 2, 3], [4, 5, 6]),                      # empty join
    ([-7, -7, 0, 3, 3, 9], [-7, 0, 0, 0, 9, 9, 9]),  # negative keys
    ([2147483647], [2147483647, 2147483647]),
    ([-2147483648, 0], [-2147483648]),
    ([0], [1]),
]


@pytest.mark.parametrize("kA,kB", KEY_CASES)
def test_groups_match_bruteforce(kA, kB):
    tab, counts = oracle.groups(np.array(kA), np.array(kB))
    bf = groups_bruteforce(np.array(kA), np.array(kB))
    assert tab.shape[0] == len(bf) == counts[0]
    r1 = r2 = 0
    J = 0
    for g, (key, oa, ma, ob, mb) in enumerate(bf):
        assert list(tab[g]) == [key, oa, ma, ob, mb, r1, r2]
        r1 += ma
        r2 += mb - 1
        J += ma * mb
    assert list(counts) == [len(bf), r1, r2, J]


def test_groups_random_bruteforce():
    rng = W.rng_for(100)
    for trial in range(20):
        m1, m2 = rng.integers(1, 300, size=2)
        nv = int(rng.integers(1, 50))
        kA = np.sort(rng.integers(-nv, nv, size=m1)).astype(np.int32)
        kB = np.sort(rng.integers(-nv, nv, size=m2)).astype(np.int32)
        tab, counts = oracle.groups(kA, kB)
        bf = groups_bruteforce(kA, kB)
        assert [tuple(t[:5]) for t in tab.tolist()] == bf
        assert counts[3] == join_matrix(inst_of(np.zeros((m1, 1)), np.zeros((m2, 1)), kA, kB)).shape[0]


def test_groups_unsorted_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.groups(np.array([0, 2, 1]), np.array([0, 1]))
    with pytest.raises(oracle.OracleError):
        oracle.groups(np.array([0, 1]), np.array([3, 1]))


def test_groups_cartesian():
    tab, counts = oracle.groups(None, None, 7, 5)
    assert list(tab[0]) == [0, 0, 7, 0, 5, 0, 0]
    assert list(counts) == [1, 7, 4, 35]


# ------------------------------------------------------ head / tail (H, T)

def head_tail_via_oracle(Bcol_matrix):
    """H(B), T(B) from the oracle with m1 = 1 (so the tails are not scaled)."""
    B = np.asarray(Bcol_matrix, dtype=np.float64)
    M, heads, tab, counts = oracle.compact(inst_of(np.zeros((1, 1)), B))
    return heads[0], M[1:, 1:]


def test_head_tail_hand_values_m2():
    a1, a2 = 0.3, -1.7
    H, T = head_tail_via_oracle([[a1], [a2]])
    assert np.isclose(H[0], (a1 + a2) / np.sqrt(2), rtol=0, atol=1e-15)
    assert np.isclose(T[0, 0], (a2 - a1) / np.sqrt(2), rtol=0, atol=1e-15)


def test_head_tail_hand_values_m3():
    a1, a2, a3 = 2.0, -0.5, 1.25
    H, T = head_tail_via_oracle([[a1], [a2], [a3]])
    assert np.isclose(H[0], (a1 + a2 + a3) / np.sqrt(3), atol=1e-15)
    assert np.isclose(T[0, 0], (a2 - a1) / np.sqrt(2), atol=1e-15)
    assert np.isclose(T[1, 0], (2 * a3 - a1 - a2) / np.sqrt(6), atol=1e-15)


def test_head_tail_constant_column():
    for m in (1, 2, 5, 64, 1000):
        H, T = head_tail_via_oracle(np.full((m, 1), 3.5))
        assert np.isclose(H[0], np.sqrt(m) * 3.5, rtol=1e-15)
        assert np.all(np.abs(T) <= 1e-14 * np.sqrt(m))


def helmert(m):
    """Textbook Helmert matrix: first row 1/sqrt(m); row k (k>=1) is the normalised contrast
    (row k+1 against the mean of rows 1..k)."""
    Hm = np.zeros((m, m))
    Hm[0, :] = 1.0 / np.sqrt(m)
    for k in range(1, m):
        Hm[k, :k] = -1.0
        Hm[k, k] = float(k)
        Hm[k] /= np.linalg.norm(Hm[k])
    return Hm


@pytest.mark.parametrize("m", [1, 2, 3, 7, 50])
def test_head_tail_is_helmert_transform(m):
    Hm = helmert(m)
    assert np.allclose(Hm @ Hm.T, np.eye(m), atol=1e-14)
    B = W.rng_for(101, m).standard_normal((m, 4))
    H, T = head_tail_via_oracle(B)
    ref = Hm @ B
    assert np.allclose(H, ref[0], atol=1e-13)
    assert np.allclose(T, ref[1:], atol=1e-13)


# --------------------------------------------------------- Claim 1 (M)

@pytest.mark.parametrize("m1,n1,m2,n2", [(1, 1, 1, 1), (2, 1, 3, 2), (3, 2, 4, 3), (5, 3, 6, 2), (1, 2, 5, 3), (4, 2, 1, 3)])
def test_compact_equals_explicit_givens(m1, n1, m2, n2):
    rng = W.rng_for(102, m1 * 100 + m2)
    A = rng.random((m1, n1))
    B = rng.random((m2, n2))
    heads, tails, rest = givens_compact_cartesian(A, B)
    M, hd, tab, counts = oracle.compact(inst_of(A, B))
    assert M.shape == (m1 + m2 - 1, n1 + n2)
    assert np.allclose(M[:m1], heads, atol=1e-13)
    assert np.allclose(M[m1:], tails, atol=1e-13)
    assert np.all(np.abs(rest) < 1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_compact_gram_equals_join_gram(seed):
    rng = W.rng_for(103, seed)
    m1, m2 = rng.integers(1, 40, size=2)
    n1, n2 = rng.integers(1, 5, size=2)
    inst = W.random_instance(rng, int(m1), int(n1), int(m2), int(n2), n_values=int(rng.integers(1, 8)))
    M, _, _, _ = oracle.compact(inst)
    J = join_matrix(inst)
    assert np.allclose(M.T @ M, J.T @ J, rtol=1e-12, atol=1e-11)
    assert np.allclose(M.T @ M, gram_closed_form(inst), rtol=1e-12, atol=1e-11)


def test_compact_special_cases():
    rng = W.rng_for(104)
    # m2_g = 1 for every group: no tails, M is J up to row order
    inst = W.random_instance(rng, 20, 3, 6, 2, n_values=None)
    kA = np.sort(rng.integers(0, 6, size=20)).astype(np.int32)
    kB = np.arange(6, dtype=np.int32)
    inst = W.Instance(inst.A, inst.B, kA, kB)
    M, _, _, counts = oracle.compact(inst)
    J = join_matrix(inst)
    assert counts[2] == 0
    assert np.allclose(M, J, atol=1e-15)
    # all singleton groups: M == J
    kA2 = np.arange(6, dtype=np.int32)
    inst2 = W.Instance(rng.random((6, 2)), inst.B, kA2, kB)
    M2, _, _, _ = oracle.compact(inst2)
    assert np.allclose(M2, join_matrix(inst2), atol=1e-15)


def test_compact_pin_detects_planted_mistakes():
    """Plausible mistakes in the compact matrix break the Gram pin."""
    rng = W.rng_for(105)
    inst = W.random_instance(rng, 30, 3, 25, 2, n_values=4)
    M, _, tab, counts = oracle.compact(inst)
    Gref = gram_closed_form(inst)
    R1 = int(counts[1])
    n1 = 3
    assert np.allclose(M.T @ M, Gref, rtol=1e-12, atol=1e-11)
    bad = []
    X = M.copy(); X[R1:] /= 1.7; bad.append(X)                       # wrong sqrt(m1) scaling
    X = M.copy(); X[:R1, :n1] /= 1.3; bad.append(X)                  # wrong sqrt(m2) scaling
    X = M.copy(); X[:R1, n1:] = 0; bad.append(X)                     # head block dropped
    X = M.copy(); X[R1 + 1:] = M[R1:-1]; bad.append(X)               # tail index shifted
    X = M.copy(); X[:R1, n1:] *= -1; bad.append(X)                   # head sign flipped
    for X in bad:
        assert not np.allclose(X.T @ X, Gref, rtol=1e-6, atol=1e-6)


# ----------------------------------------------------------- Householder R

@pytest.mark.parametrize("rows,N", [(10, 4), (64, 64), (100, 7), (3, 5), (1, 1), (257, 33)])
def test_householder_matches_lapack(rows, N):
    X = W.rng_for(106, rows * N).standard_normal((rows, N))
    R = oracle.householder_r(X)
    assert relF(R, lapack_r(X)) < 1e-13


def test_householder_zero_and_repeated_columns():
    X = W.rng_for(107).standard_normal((20, 5))
    X[:, 2] = 0.0
    R = oracle.householder_r(X)
    assert np.allclose(R.T @ R, X.T @ X, atol=1e-12)
    assert np.all(np.diag(R) >= 0)
    assert np.all(np.tril(R, -1) == 0)


def test_sign_normalise_rules():
    R = np.array([[-2.0, 1.0, -0.0], [0.0, 0.0, -3.0], [0.0, 0.0, 0.0]])
    S = oracle.sign_normalise(R)
    assert np.array_equal(S, np.array([[2.0, -1.0, 0.0], [0.0, 0.0, 3.0], [0.0, 0.0, 0.0]]))
    assert not np.any(np.signbit(S[S == 0.0]))  # no -0.0 left


@pytest.mark.parametrize("seed", range(8))
def test_r_matches_lapack_on_explicit_join(seed):
    rng = W.rng_for(108, seed)
    m1, m2 = (int(x) for x in rng.integers(2, 25, size=2))
    n1, n2 = (int(x) for x in rng.integers(1, 5, size=2))
    nv = None if seed % 3 == 0 else int(rng.integers(1, 6))
    inst = W.random_instance(rng, m1, n1, m2, n2, n_values=nv)
    J = join_matrix(inst)
    if J.shape[0] < n1 + n2:
        pytest.skip("rank deficient by construction: R not unique (parity unpinned)")
    assert relF(oracle.r(inst), lapack_r(J)) < 1e-12


def test_r_gram_cholesky_pin_medium():
    rng = W.rng_for(109)
    inst = W.random_instance(rng, 3000, 6, 2500, 5, n_values=40, key_skew=1.1)
    R = oracle.r(inst)
    L = np.linalg.cholesky(gram_closed_form(inst))
    assert relF(R, L.T) < 1e-12


def test_r_empty_join():
    inst = inst_of(np.ones((3, 2)), np.ones((2, 2)), [0, 1, 2], [5, 6])
    assert np.all(oracle.r(inst) == 0.0)


def test_r_rank_deficient_gram_only():
    """rows_M < N: R is not unique beyond the rank (parity unpinned); R^T R must still equal J^T J."""
    inst = inst_of(np.array([[1.0, 2.0, 3.0]]), np.array([[0.5, -1.0, 2.0]]))
    R = oracle.r(inst)
    J = join_matrix(inst)
    assert np.allclose(R.T @ R, J.T @ J, atol=1e-14)


def test_config1_claim1_preserves_r():
    """Config 1 (1000x4 each, 1e6-row join): R through Claim 1 equals R of the explicit join."""
    inst = W.config1()
    J = np.hstack([np.repeat(inst.A, 1000, axis=0), np.tile(inst.B, (1000, 1))])
    Rj = oracle.householder_r(J)
    Rc = oracle.r(inst)
    assert relF(Rc, Rj) < 1e-12
    L = np.linalg.cholesky(gram_closed_form(inst))
    assert relF(Rc, L.T) < 1e-12


@pytest.mark.parametrize("cfg", [2])
def test_config_gram_cholesky_pin(cfg):
    inst = W.CONFIGS[cfg]()
    R = oracle.r(inst)
    L = np.linalg.cholesky(gram_closed_form(inst))
    assert relF(R, L.T) < 1e-12


@pytest.mark.parametrize("maker", [lambda: W.config3(m=1 << 15), lambda: W.config5(m=1 << 13, n=64)])
def test_scaled_config_gram_cholesky_pin(maker):
    inst = maker()
    R = oracle.r(inst)
    L = np.linalg.cholesky(gram_closed_form(inst))
    # columnwise check too: configs with column scales spanning 1e-3..1
    assert relF(R, L.T) < 1e-12
    colerr = np.linalg.norm(R - L.T, axis=0) / np.linalg.norm(L.T, axis=0)
    assert colerr.max() < 1e-11


@pytest.mark.slow
@pytest.mark.parametrize("cfg", [3, 5])
def test_full_config_gram_cholesky_pin(cfg):
    inst = W.CONFIGS[cfg]()
    R = oracle.r(inst)
    L = np.linalg.cholesky(gram_closed_form(inst))
    assert relF(R, L.T) < 1e-12


# ------------------------------------------------------------------ sigma

@pytest.mark.parametrize("seed", range(6))
def test_sigma_matches_lapack_svd_of_join(seed):
    rng = W.rng_for(110, seed)
    inst = W.random_instance(rng, 12, 3, 9, 2, n_values=None if seed % 2 else 3)
    J = join_matrix(inst)
    s = oracle.sigma(oracle.r(inst))
    ref = np.linalg.svd(J, compute_uv=False)
    ref = np.concatenate([ref, np.zeros(s.size - ref.size)])
    assert np.linalg.norm(s - ref) / np.linalg.norm(ref) < 1e-13


def test_sigma_invariants():
    rng = W.rng_for(111)
    inst = W.random_instance(rng, 400, 5, 300, 6, n_values=20)
    R = oracle.r(inst)
    s = oracle.sigma(R)
    assert np.isclose(np.sum(s ** 2), frob2_closed_form(inst), rtol=1e-13)
    assert np.isclose(np.sum(np.log(s)), np.sum(np.log(np.abs(np.diag(R)))), rtol=1e-12)
    assert np.all(np.diff(s) <= 0)


def test_sigma_two_by_two_closed_form():
    rng = W.rng_for(112)
    inst = W.random_instance(rng, 50, 1, 40, 1, n_values=7)
    Gm = gram_closed_form(inst)
    a, b, c = Gm[0, 0], Gm[1, 1], Gm[0, 1]
    tr, det = a + b, a * b - c * c
    disc = np.sqrt((a - b) ** 2 + 4 * c * c)
    ev = np.array([(tr + disc) / 2, det / ((tr + disc) / 2)])
    s = oracle.sigma(oracle.r(inst))
    assert np.allclose(s, np.sqrt(ev), rtol=1e-12)


def test_sigma_known_spectrum():
    rng = W.rng_for(113)
    n = 40
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sv = np.sort(10.0 ** rng.uniform(-3, 0, size=n))[::-1]
    R = oracle.householder_r(U @ np.diag(sv) @ V.T)
    s, sweeps = oracle.sigma(R, return_sweeps=True)
    assert np.linalg.norm(s - sv) / np.linalg.norm(sv) < 1e-13
    assert np.max(np.abs(s - sv) / sv) < 1e-11
    assert 1 <= sweeps <= 20


def test_sigma_diagonal_and_zero():
    d = np.array([3.0, -1.0, 0.0, 2.0])
    assert np.array_equal(oracle.sigma(np.diag(d)), np.array([3.0, 2.0, 1.0, 0.0]))
    assert np.array_equal(oracle.sigma(np.zeros((3, 3))), np.zeros(3))


# ------------------------------------------------------------------ sort (unsorted inputs)

@pytest.mark.parametrize("seed", range(5))
def test_sort_table_matches_brute_force(seed):
    """oracle.sort_table against a brute-force stable sort: Python's sorted() on (key, row index)."""
    rng = W.rng_for(120, seed)
    m = int(rng.integers(0, 300))
    keys = rng.integers(-5, 6 if seed % 2 else 2 ** 31 - 1, size=m).astype(np.int32)
    if seed == 3:
        keys[:] = np.int32(-2 ** 31)
    X = rng.standard_normal((m, 3))
    Xs, ks = oracle.sort_table(X, keys)
    order = [i for _, i in sorted((int(k), i) for i, k in enumerate(keys))]
    assert np.array_equal(ks, keys[order])
    assert np.array_equal(Xs, X[order])
    assert np.all(np.diff(ks.astype(np.int64)) >= 0)


# ------------------------------------------------------------------ right singular vectors

def _sign_fix(V):
    """Each column's entry of largest magnitude made positive (the sign is free)."""
    idx = np.argmax(np.abs(V), axis=0)
    sg = np.sign(V[idx, np.arange(V.shape[1])])
    sg[sg == 0] = 1.0
    return V * sg[None, :]


@pytest.mark.parametrize("seed", range(4))
def test_svd_v_invariants_and_lapack(seed):
    """V orthogonal, R V with orthogonal columns of norms sigma, sigma equal to oracle_sigma's,
    and V equal (up to column signs) to LAPACK's right singular vectors of R."""
    rng = W.rng_for(121, seed)
    n = [5, 16, 33, 64][seed]
    R = np.triu(rng.standard_normal((n, n)))
    s, V = oracle.svd_v(R)
    assert np.allclose(s, oracle.sigma(R), rtol=1e-13, atol=0)
    assert np.abs(V.T @ V - np.eye(n)).max() < 1e-13
    RV = R @ V
    assert np.abs(RV.T @ RV - np.diag(s ** 2)).max() < 1e-12 * s[0] ** 2
    _, sl, Vt = np.linalg.svd(R)
    assert np.allclose(s, sl, rtol=1e-12)
    assert np.abs(_sign_fix(V) - _sign_fix(Vt.T)).max() < 1e-9


def test_svd_v_of_join_matches_lapack():
    """The right singular vectors of the join (through the oracle's R) against LAPACK on the
    explicit join."""
    rng = W.rng_for(122)
    inst = W.random_instance(rng, 40, 3, 30, 4, n_values=5)
    J = join_matrix(inst)
    s, V = oracle.svd_v(oracle.r(inst))
    _, sl, Vt = np.linalg.svd(J)
    assert np.allclose(s, sl, rtol=1e-12)
    assert np.abs(_sign_fix(V) - _sign_fix(Vt.T)).max() < 1e-9


def test_svd_v_diagonal():
    s, V = oracle.svd_v(np.diag([1.0, -3.0, 2.0]))
    assert np.array_equal(s, [3.0, 2.0, 1.0])
    assert np.array_equal(np.abs(V), np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], dtype=float))
