"""Right singular vectors: the device's Jacobi with accumulated rotations against the
oracle's (FP64), on special matrices, on the R of joins, and on the stored references."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2503_23385_amd import workloads as W
from test_gpu_parity import CASES, SPECIAL, dev, fg, say, to_dev

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_golden  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def sign_fix(V):
    idx = np.argmax(np.abs(V), axis=0)
    sg = np.sign(V[idx, np.arange(V.shape[1])])
    sg[sg == 0] = 1.0
    return V * sg[None, :]


def check(R, label):
    n = R.shape[0]
    S, V = fg().svd(torch.from_numpy(np.ascontiguousarray(R)).to(dev()))
    torch.cuda.synchronize()
    S, V = S.cpu().numpy(), V.cpu().numpy()
    So, Vo = oracle.svd_v(R)
    top = So[0] if So[0] > 0 else 1.0
    es = np.linalg.norm(S - So) / max(np.linalg.norm(So), 1e-300)
    # orthogonality and R V = U Sigma hold for every input
    assert np.abs(V.T @ V - np.eye(n)).max() < 1e-12
    RV = (R / top) @ V
    assert np.abs(RV.T @ RV - np.diag((S / top) ** 2)).max() < 1e-12
    # the vectors of well separated values are unique up to sign: compare them
    gap = np.full(n, np.inf)
    if n > 1:
        d = np.abs(np.diff(So)) / top
        gap[:-1] = np.minimum(gap[:-1], d)
        gap[1:] = np.minimum(gap[1:], d)
    sep = gap > 1e-6
    ev = np.abs(sign_fix(V)[:, sep] - sign_fix(Vo)[:, sep]).max() if sep.any() else 0.0
    # the error of a singular vector grows like (rounding) / (relative gap)
    tol = 1e-13 / np.min(gap[sep]) if sep.any() else 0.0
    say(f"[svd] {label} n={n} rel2(sigma)={es:.3e} max|dV| (separated)={ev:.3e} tol={tol:.1e}")
    assert es <= 1e-12
    assert ev <= max(tol, 1e-11)


@pytest.mark.parametrize("name", [k for k in SPECIAL if SPECIAL[k].shape[0] <= 128 and np.abs(SPECIAL[k]).max() < 2.0 ** 400
                                  and np.abs(SPECIAL[k]).max() > 2.0 ** -400])
def test_svd_special(name):
    check(SPECIAL[name], name)


@pytest.mark.parametrize("name", ["cart_ragged", "keyed_zipf_n64", "keyed_narrow", "cart_n125_ragged", "keyed_n128"])
def test_svd_of_join_r(name):
    inst = CASES[name]
    A, B, kA, kB = to_dev(inst)
    R, _ = fg().r(A, B, kA, kB, "fp64")
    check(R.cpu().numpy(), name)


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg3"])
def test_svd_of_stored_references(name):
    refs, _ = make_golden.load(name)
    check(refs[0][0], name)
