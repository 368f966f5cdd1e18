"""Full-size parity: the HIP path (through the C ABI) against the stored oracle references.

Every workload at its full size, every precision and both forms of the compact
matrix, compared element by element with the FP64 CPU oracle's R and sigma
(``tests/golden/``, written by ``make_golden.py`` from the oracle alone):

  - R: relative Frobenius error <= 1e-12 (FP64 form and FP32 + FP64 refinement
    sweep), <= 1e-5 (FP32 form), after both sides normalise row signs;
  - sigma: relative 2-norm error within the same bounds;
  - the key grouping of the natural joins: bit-exact against the oracle's table.

The Cholesky factor of the closed-form Gram matrix is checked as well, as an
extra property that holds at any size (its own error is about kappa^2 * 2^-53).
"""
import functools
import os
import sys

import numpy as np
import pytest

import oracle
from bruteforce import gram_closed_form, relF
from paper_2503_23385_amd import workloads as W

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_golden  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp32_refine": 1e-12}
GROUP_COLS = ("key", "offA", "m1", "offB", "m2", "r1", "r2")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def fg():
    import paper_2503_23385_amd as m
    return m


def to_dev(inst):
    d = dev()
    A = torch.from_numpy(np.ascontiguousarray(inst.A)).to(d)
    B = torch.from_numpy(np.ascontiguousarray(inst.B)).to(d)
    kA = None if inst.keys_A is None else torch.from_numpy(inst.keys_A).to(d)
    kB = None if inst.keys_B is None else torch.from_numpy(inst.keys_B).to(d)
    return A, B, kA, kB


@functools.lru_cache(maxsize=1)
def workload(name):
    """Inputs (host and device) and stored references of one workload, the inputs checked
    against the digest the references were made from."""
    refs, digest = make_golden.load(name)
    insts = make_golden.instances(name)
    assert make_golden.input_digest(insts) == digest, "stale reference: regenerate tests/golden"
    return insts, [to_dev(i) for i in insts], refs


def errors(R, S, Ro, So):
    Rg, Sg = R.cpu().numpy(), S.cpu().numpy()
    assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) >= 0)
    return relF(Rg, Ro), float(np.linalg.norm(Sg - So) / np.linalg.norm(So))


def run_single(name, prec, two_sided):
    insts, tens, refs = workload(name)
    A, B, kA, kB = tens[0]
    say(f"[full] {name} shape={insts[0].shape} {prec} two_sided={two_sided}")
    R, ws = fg().r(A, B, kA, kB, prec, two_sided=two_sided)
    S = fg().sigma(R)
    torch.cuda.synchronize()
    assert fg().status(ws) == 0
    (Ro, So), = refs
    er, es = errors(R, S, Ro, So)
    say(f"    relF(R)={er:.3e} rel2(sigma)={es:.3e}")
    assert er <= TOL[prec] and es <= TOL[prec]
    return R


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_refine"])
@pytest.mark.parametrize("two_sided", [False, True])
def test_cartesian_full(name, prec, two_sided):
    run_single(name, prec, two_sided)


def test_cfg3_groups_bit_exact():
    insts, tens, _ = workload("cfg3")
    A, B, kA, kB = tens[0]
    out = fg().compact(A, B, kA, kB, "fp64")
    tab, counts = oracle.groups(insts[0].keys_A, insts[0].keys_B)
    assert np.array_equal(out["counts"], counts)
    got = np.stack([out["groups"][k] for k in GROUP_COLS], axis=1)
    assert np.array_equal(got.astype(np.int64), tab)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_refine"])
@pytest.mark.parametrize("two_sided", [False, True])
def test_cfg3_full(prec, two_sided):
    """Natural join of two 2^20 x 64 tables on Zipf(1.1) keys over 1e4 values."""
    R = run_single("cfg3", prec, two_sided)
    L = np.linalg.cholesky(gram_closed_form(workload("cfg3")[0][0]))
    assert relF(R.cpu().numpy(), L.T) <= max(TOL[prec], 1e-12)


def test_cfg5_groups_bit_exact():
    insts, tens, _ = workload("cfg5")
    A, B, kA, kB = tens[0]
    out = fg().compact(A, B, kA, kB, "fp32", two_sided=True)
    tab, counts = oracle.groups(insts[0].keys_A, insts[0].keys_B)
    assert np.array_equal(out["counts"], counts)
    got = np.stack([out["groups"][k] for k in GROUP_COLS], axis=1)
    assert np.array_equal(got.astype(np.int64), tab)


@pytest.mark.parametrize("prec,two_sided", [("fp64", True), ("fp64", False), ("fp32", True),
                                            ("fp32_refine", True)])
def test_cfg5_full(prec, two_sided):
    """Wide natural join: 2^18 x 256 FP32 tables, scaled columns (kappa ~ 1e3), N = 512."""
    R = run_single("cfg5", prec, two_sided)
    L = np.linalg.cholesky(gram_closed_form(workload("cfg5")[0][0]))
    # the Gram reference carries about kappa^2 * 2^-53 of its own
    assert relF(R.cpu().numpy(), L.T) <= max(TOL[prec], 1e-9)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_refine"])
def test_cfg4_full_batch(prec):
    """All 256 instances of the batch (m1, m2 log-uniform in [1e3, 1e5], n in {8..64}) in one
    captured graph, every instance against its stored reference, on two replays."""
    insts, tens, refs = workload("cfg4")
    say(f"[full] cfg4 batch of {len(insts)} {prec}")
    d = dev()
    plan = fg().Plan(tens, prec, two_sided=True)
    ws = torch.empty(plan.ws_bytes, dtype=torch.uint8, device=d)
    R = torch.zeros(plan.r_total, dtype=torch.float64, device=d)
    S = torch.zeros(plan.s_total, dtype=torch.float64, device=d)
    for rep in range(2):
        R.zero_()
        S.zero_()
        plan.execute(ws, R, S)
        torch.cuda.synchronize()
        Rh, Sh = R.cpu().numpy(), S.cpu().numpy()
        worst = (0.0, 0.0)
        for i, inst in enumerate(insts):
            N = inst.A.shape[1] + inst.B.shape[1]
            Rg = Rh[plan.r_off[i]:plan.r_off[i] + N * N].reshape(N, N)
            Sg = Sh[plan.s_off[i]:plan.s_off[i] + N]
            Ro, So = refs[i]
            er = relF(Rg, Ro)
            es = float(np.linalg.norm(Sg - So) / np.linalg.norm(So))
            worst = (max(worst[0], er), max(worst[1], es))
            assert er <= TOL[prec] and es <= TOL[prec], (rep, i, inst.shape, er, es)
        say(f"    replay {rep}: max relF(R)={worst[0]:.3e} max rel2(sigma)={worst[1]:.3e}")


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg3"])
@pytest.mark.parametrize("method", ["jacobi", "bidiag", "dqds"])
def test_sigma_routes_on_oracle_r(name, method):
    """Both sigma routes (n <= 128) on the oracle's own R, against the oracle's sigma."""
    _, _, refs = workload(name)
    (Ro, So), = refs
    S = fg().sigma(torch.from_numpy(np.ascontiguousarray(Ro)).to(dev()), method=method).cpu().numpy()
    es = float(np.linalg.norm(S - So) / np.linalg.norm(So))
    say(f"[sigma] {name} {method} n={Ro.shape[0]} rel2={es:.3e}")
    assert es <= 1e-12


@pytest.mark.parametrize("method", ["jacobi", "bidiag", "dqds"])
def test_sigma_routes_on_batch_r(method):
    """Every width class of the batch (n = 16, 32, 64, 128), each sigma route against the oracle."""
    _, _, refs = workload("cfg4")
    seen = {}
    for Ro, So in refs:
        seen.setdefault(Ro.shape[0], (Ro, So))
    for n, (Ro, So) in sorted(seen.items()):
        S = fg().sigma(torch.from_numpy(np.ascontiguousarray(Ro)).to(dev()), method=method).cpu().numpy()
        es = float(np.linalg.norm(S - So) / np.linalg.norm(So))
        say(f"[sigma] cfg4 n={n} {method} rel2={es:.3e}")
        assert es <= 1e-12
