"""The stored full-size oracle references (``tests/golden/oracle_cfg*.npz``) pinned on the CPU.

The references are written by ``tests/golden/make_golden.py`` from the oracle
alone.  Here each is checked against what holds at any size without the
oracle: the seeded generator still reproduces the inputs it was made from; R is
upper triangular with a non-negative diagonal and equals the Cholesky factor
of the closed-form Gram matrix J^T J (Section 1: R is that factor; the Gram is
summed per key group without the join); sigma is descending and satisfies
sum sigma^2 = ||J||_F^2 in closed form and sum log sigma = sum log |R_ii|.
"""
import os
import sys

import numpy as np
import pytest

from bruteforce import frob2_closed_form, gram_closed_form, relF
from paper_2503_23385_amd import workloads as W

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_golden  # noqa: E402

SINGLE = ["cfg1", "cfg2", "cfg3", "cfg5"]


def check_pair(inst, R, S, tol_r=1e-12):
    N = inst.A.shape[1] + inst.B.shape[1]
    assert R.shape == (N, N) and S.shape == (N,)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    L = np.linalg.cholesky(gram_closed_form(inst))
    assert relF(R, L.T) < tol_r
    # column-wise as well: the wide workload's columns span 1e-3 .. 1
    colerr = np.linalg.norm(R - L.T, axis=0) / np.linalg.norm(L.T, axis=0)
    assert colerr.max() < 1e-11
    assert np.all(np.diff(S) <= 0)
    assert np.isclose(np.sum(S ** 2), frob2_closed_form(inst), rtol=1e-12)
    assert np.isclose(np.sum(np.log(S)), np.sum(np.log(np.diag(R))), rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("name", SINGLE)
def test_golden_single(name):
    refs, digest = make_golden.load(name)
    insts = make_golden.instances(name)
    assert make_golden.input_digest(insts) == digest, "generator no longer reproduces the stored inputs"
    (R, S), = refs
    check_pair(insts[0], R, S)


def test_golden_batch():
    refs, digest = make_golden.load("cfg4")
    insts = make_golden.instances("cfg4")
    assert len(refs) == len(insts) == 256
    assert make_golden.input_digest(insts) == digest
    for inst, (R, S) in zip(insts, refs):
        check_pair(inst, R, S)
