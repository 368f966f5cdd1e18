"""Brute-force references used to pin the oracle.  Test-only.

Nothing here shares code with the oracle or the GPU path: each helper
computes its quantity the long way (explicit join, explicit rotations,
LAPACK through numpy) so that a mistake in the oracle cannot hide behind
the same mistake here.
"""
from __future__ import annotations

import numpy as np


def groups_bruteforce(kA, kB, m1=None, m2=None):
    """Group table by dictionaries: {key: (first row, count)} per table, matched keys ascending."""
    if kA is None:
        if m1 and m2:
            return [(0, 0, m1, 0, m2)]
        return []
    def runs(k):
        d = {}
        for i, v in enumerate(np.asarray(k).tolist()):
            if v not in d:
                d[v] = [i, 0]
            d[v][1] += 1
        return d
    ra, rb = runs(kA), runs(kB)
    out = []
    for key in sorted(set(ra) & set(rb)):
        out.append((key, ra[key][0], ra[key][1], rb[key][0], rb[key][1]))
    return out


def join_matrix(inst):
    """Explicit join matrix J: rows [A_r | B_s] for every matching pair, A order major."""
    A = np.asarray(inst.A, dtype=np.float64)
    B = np.asarray(inst.B, dtype=np.float64)
    m1, m2 = A.shape[0], B.shape[0]
    rows = []
    if inst.keys_A is None:
        for r in range(m1):
            rows.append(np.hstack([np.repeat(A[r:r + 1], m2, axis=0), B]))
    else:
        kA, kB = np.asarray(inst.keys_A), np.asarray(inst.keys_B)
        for r in range(m1):
            sel = np.nonzero(kB == kA[r])[0]
            if len(sel):
                rows.append(np.hstack([np.repeat(A[r:r + 1], len(sel), axis=0), B[sel]]))
    if not rows:
        return np.zeros((0, A.shape[1] + B.shape[1]))
    return np.vstack(rows)


def gram_closed_form(inst):
    """J^T J without the join: per group [[m2 A^T A, a b^T], [b a^T, m1 B^T B]], a, b column sums."""
    A = np.asarray(inst.A, dtype=np.float64)
    B = np.asarray(inst.B, dtype=np.float64)
    n1, n2 = A.shape[1], B.shape[1]
    Gm = np.zeros((n1 + n2, n1 + n2))
    for (_, oa, ma, ob, mb) in groups_bruteforce(inst.keys_A, inst.keys_B, A.shape[0], B.shape[0]):
        Ag, Bg = A[oa:oa + ma], B[ob:ob + mb]
        a, b = Ag.sum(axis=0), Bg.sum(axis=0)
        Gm[:n1, :n1] += mb * (Ag.T @ Ag)
        Gm[n1:, n1:] += ma * (Bg.T @ Bg)
        Gm[:n1, n1:] += np.outer(a, b)
        Gm[n1:, :n1] += np.outer(b, a)
    return Gm


def frob2_closed_form(inst):
    A = np.asarray(inst.A, dtype=np.float64)
    B = np.asarray(inst.B, dtype=np.float64)
    tot = 0.0
    for (_, oa, ma, ob, mb) in groups_bruteforce(inst.keys_A, inst.keys_B, A.shape[0], B.shape[0]):
        tot += mb * np.sum(A[oa:oa + ma] ** 2) + ma * np.sum(B[ob:ob + mb] ** 2)
    return tot


def givens_compact_cartesian(A, B):
    """Apply Claim 1's rotation sequence to the explicit Cartesian product, rotation by rotation.

    Within each block C^(i) the running first row is rotated against the next row with
    c = sqrt(k/(k+1)), s = 1/sqrt(k+1); then, for each surviving row position, the m1 copies
    across blocks are rotated together the same way.  Returns the rotated matrix split as
    (head rows m1 x N, tail rows (m2-1) x N, rest) -- rest should be zero.
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    m1, n1 = A.shape
    m2, n2 = B.shape
    J = np.zeros((m1 * m2, n1 + n2))
    for i in range(m1):
        J[i * m2:(i + 1) * m2, :n1] = A[i]
        J[i * m2:(i + 1) * m2, n1:] = B

    def rot(X, p, q, c, s):
        xp, xq = X[p].copy(), X[q].copy()
        X[p] = c * xp + s * xq
        X[q] = -s * xp + c * xq

    # phase 1: inside each block, fold row k+1 into the running head row (row 0 of the block)
    for i in range(m1):
        base = i * m2
        for k in range(1, m2):
            c, s = np.sqrt(k / (k + 1.0)), 1.0 / np.sqrt(k + 1.0)
            rot(J, base, base + k, c, s)
    # phase 2: for each row position k >= 1 (tails), fold the copies of blocks 1.. into block 0
    for k in range(1, m2):
        for i in range(1, m1):
            c, s = np.sqrt(i / (i + 1.0)), 1.0 / np.sqrt(i + 1.0)
            rot(J, k, i * m2 + k, c, s)
    heads = np.vstack([J[i * m2] for i in range(m1)])
    tails = J[1:m2].copy()
    rest_idx = [i * m2 + k for i in range(1, m1) for k in range(1, m2)]
    rest = J[rest_idx] if rest_idx else np.zeros((0, n1 + n2))
    return heads, tails, rest


def sign_rows(R):
    """Make diag(R) >= 0 by negating rows (plain numpy, for LAPACK results)."""
    R = np.triu(np.array(R, dtype=np.float64))
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return R * d[:, None]


def lapack_r(J):
    n = J.shape[1]
    if J.shape[0] == 0:
        return np.zeros((n, n))
    R = np.linalg.qr(J, mode="r")
    if R.shape[0] < n:
        R = np.vstack([R, np.zeros((n - R.shape[0], n))])
    return sign_rows(R)


def relF(X, Y):
    nY = np.linalg.norm(Y)
    return np.linalg.norm(X - Y) / (nY if nY > 0 else 1.0)
