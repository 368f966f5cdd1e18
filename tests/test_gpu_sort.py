"""Unsorted inputs: the device's stable sort by key against the oracle's (bit-exact), the
whole path on tables sorted on the device, and the memory report against the oracle's counts."""
import numpy as np
import pytest

import oracle
from bruteforce import relF
from paper_2503_23385_amd import workloads as W
from test_gpu_parity import dev, fg, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def sort_cases():
    rng = lambda k: W.rng_for(730, k)  # noqa: E731
    c = {}
    c["dups_small_range"] = (rng(1).integers(-50, 51, size=10007).astype(np.int32), 5, np.float64)
    c["full_int32_range"] = (rng(2).integers(-2 ** 31, 2 ** 31 - 1, size=50000, dtype=np.int64).astype(np.int32), 3,
                             np.float32)
    c["all_equal"] = (np.full(4099, -7, dtype=np.int32), 4, np.float64)
    c["extremes"] = (np.array([2 ** 31 - 1, -2 ** 31, 0, -1, 1, -2 ** 31, 2 ** 31 - 1] * 300, dtype=np.int32), 2,
                     np.float64)
    c["sorted"] = (np.sort(rng(3).integers(0, 1000, size=3000)).astype(np.int32), 6, np.float32)
    c["reverse"] = (np.sort(rng(4).integers(0, 1000, size=3000))[::-1].astype(np.int32), 6, np.float64)
    c["one_row"] = (np.array([5], dtype=np.int32), 3, np.float64)
    c["ragged_block"] = (rng(5).integers(0, 7, size=2049).astype(np.int32), 1, np.float64)
    return c


CASES = sort_cases()


@pytest.mark.parametrize("name", list(CASES))
def test_sort_bit_exact(name):
    keys, n, dt = CASES[name]
    X = W.rng_for(731).standard_normal((keys.size, n)).astype(dt)
    say(f"[sort] {name} rows={keys.size} cols={n} {np.dtype(dt).name}")
    d = dev()
    Xs, ks = fg().sort_table(torch.from_numpy(X).to(d), torch.from_numpy(keys).to(d))
    torch.cuda.synchronize()
    Xo, ko = oracle.sort_table(X, keys)
    assert np.array_equal(ks.cpu().numpy(), ko)
    assert np.array_equal(Xs.cpu().numpy(), Xo)


def test_sort_strided_rows():
    keys = W.rng_for(732).integers(0, 40, size=5000).astype(np.int32)
    big = W.rng_for(733).standard_normal((5000, 9))
    d = dev()
    Xd = torch.from_numpy(big).to(d)[:, 2:7]
    Xs, ks = fg().sort_table(Xd, torch.from_numpy(keys).to(d))
    Xo, ko = oracle.sort_table(big[:, 2:7], keys)
    assert np.array_equal(ks.cpu().numpy(), ko) and np.array_equal(Xs.cpu().numpy(), Xo)


def unsorted(inst, seed):
    """The same tables with their rows shuffled (keys with them)."""
    rng = W.rng_for(734, seed)
    pa = rng.permutation(inst.A.shape[0])
    pb = rng.permutation(inst.B.shape[0])
    return W.Instance(inst.A[pa], inst.B[pb], inst.keys_A[pa], inst.keys_B[pb])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("two_sided", [False, True])
def test_unsorted_tables_end_to_end(prec, two_sided):
    """Shuffled tables, sorted on the device, then R and sigma against the oracle on the
    oracle-sorted tables; the group table bit-exact."""
    base = W.random_instance(W.rng_for(735), 20000, 12, 15000, 9, n_values=300, key_skew=1.1)
    inst = unsorted(base, 1)
    d = dev()
    A, kA = fg().sort_table(torch.from_numpy(inst.A).to(d), torch.from_numpy(inst.keys_A).to(d))
    B, kB = fg().sort_table(torch.from_numpy(inst.B).to(d), torch.from_numpy(inst.keys_B).to(d))
    R, ws = fg().r(A, B, kA, kB, prec, two_sided=two_sided)
    S = fg().sigma(R)
    torch.cuda.synchronize()
    assert fg().status(ws) == 0
    Ao, kAo = oracle.sort_table(inst.A, inst.keys_A)
    Bo, kBo = oracle.sort_table(inst.B, inst.keys_B)
    so = W.Instance(Ao, Bo, kAo, kBo)
    out = fg().compact(A, B, kA, kB, prec, two_sided=two_sided)
    tab, counts = oracle.groups(kAo, kBo)
    assert np.array_equal(out["counts"], counts)
    Ro = oracle.r(so)
    So = oracle.sigma(Ro)
    tol = 1e-12 if prec == "fp64" else 1e-5
    er = relF(R.cpu().numpy(), Ro)
    es = np.linalg.norm(S.cpu().numpy() - So) / np.linalg.norm(So)
    say(f"    relF(R)={er:.3e} rel2(sigma)={es:.3e}")
    assert er <= tol and es <= tol


def test_sort_full_size_keys():
    """The 2^20-row Zipf-keyed table, shuffled, sorted on the device: bit-exact."""
    inst = W.config3()
    rng = W.rng_for(736)
    p = rng.permutation(inst.A.shape[0])
    X, keys = inst.A[p], inst.keys_A[p]
    d = dev()
    Xs, ks = fg().sort_table(torch.from_numpy(X).to(d), torch.from_numpy(keys).to(d))
    Xo, ko = oracle.sort_table(X, keys)
    assert np.array_equal(ks.cpu().numpy(), ko) and np.array_equal(Xs.cpu().numpy(), Xo)


@pytest.mark.parametrize("two_sided", [False, True])
def test_memory_report(two_sided):
    inst = W.random_instance(W.rng_for(737), 3000, 7, 2500, 5, n_values=40)
    d = dev()
    A, B = torch.from_numpy(inst.A).to(d), torch.from_numpy(inst.B).to(d)
    kA, kB = torch.from_numpy(inst.keys_A).to(d), torch.from_numpy(inst.keys_B).to(d)
    R, ws = fg().r(A, B, kA, kB, "fp64", two_sided=two_sided)
    rep = fg().memory_report(A, B, kA, kB, ws, "fp64", two_sided=two_sided)
    tab, counts = oracle.groups(inst.keys_A, inst.keys_B)
    G, R1, R2, join = (int(c) for c in counts)
    assert rep["groups"] == G and rep["join_rows"] == join
    TA = int(tab[:, 2].sum()) - G
    rows = (G + TA + R2) if two_sided else (R1 + R2)
    assert rep["compact_rows"] == rows
    assert rep["join_bytes"] == 8.0 * join * 12
    assert rep["input_bytes"] == 8.0 * (3000 * 7 + 2500 * 5) + 4.0 * (3000 + 2500)
    width = (G * 12 + TA * 7 + R2 * 5) if two_sided else (R1 * 12 + R2 * 5)
    assert rep["compact_bytes"] == 8.0 * width
    assert rep["workspace_bytes"] >= rep["compact_bytes"]
