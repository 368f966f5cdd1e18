"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Gates:
  - group table, counts and offsets: bit-exact;
  - compact matrix (diagnostic): max |diff| <= 1e-13 * max |M|;
  - R: relative Frobenius error <= 1e-12 (plain FP64 form), <= 1e-5 (FP32 form);
  - sigma: relative 2-norm error <= 1e-12 (FP64 form) / 1e-5 (FP32 form), the GPU's sigma of its
    own R (bidiagonalisation + multisection up to n = 128, block Jacobi above) vs the oracle's.

Full sizes are in test_gpu_full_size.py.
"""
import sys

import numpy as np
import pytest

import oracle
from bruteforce import gram_closed_form, relF
from paper_2503_23385_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_R = {"fp64": 1e-12, "fp32": 1e-5, "fp32_refine": 1e-12}
TOL_S = {"fp64": 1e-12, "fp32": 1e-5}


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(inst, dtype=None):
    d = dev()
    A = torch.from_numpy(np.ascontiguousarray(inst.A if dtype is None else inst.A.astype(dtype))).to(d)
    B = torch.from_numpy(np.ascontiguousarray(inst.B if dtype is None else inst.B.astype(dtype))).to(d)
    kA = None if inst.keys_A is None else torch.from_numpy(inst.keys_A).to(d)
    kB = None if inst.keys_B is None else torch.from_numpy(inst.keys_B).to(d)
    return A, B, kA, kB


def fg():
    import paper_2503_23385_amd as m
    return m


def small_cases():
    rng = lambda k: W.rng_for(700, k)  # noqa: E731
    cases = {
        "cart_tiny": W.random_instance(rng(1), 3, 2, 5, 3),
        "cart_one_row_B": W.random_instance(rng(2), 50, 3, 1, 4),
        "cart_one_row_A": W.random_instance(rng(3), 1, 3, 70, 4),
        "cart_ragged": W.random_instance(rng(4), 4099, 13, 3001, 19),
        "cart_uniform_paper": W.cartesian_uniform(800, 16, seed_k=5),
        "keyed_zipf_n64": W.random_instance(rng(6), 20000, 32, 15000, 32, n_values=300, key_skew=1.1),
        "keyed_uniform_sparse": W.random_instance(rng(7), 5000, 7, 6000, 9, n_values=4000),
        "keyed_n128": W.random_instance(rng(8), 3000, 64, 3500, 64, n_values=40),
        "keyed_one_big_group": W.random_instance(rng(9), 40, 5, 50000, 8, n_values=1),
        "keyed_narrow": W.random_instance(rng(10), 1000, 1, 1200, 1, n_values=30),
        # A tail leaf with a single row: its rank-deficient residual columns shrink
        # geometrically (regression case for reflector scalars that must not underflow).
        "cart_tail_leaf": W.random_instance(rng(14), 4097, 5, 2000, 59),
        # a Cartesian root of padded width 128: the single head row merged by one wave
        "cart_n125_ragged": W.random_instance(rng(18), 2100, 64, 1700, 61),
        # wide rows: blocked panel TSQR (padded widths 256 and 512) and block Jacobi
        "cart_n192_ragged": W.random_instance(rng(15), 1500, 70, 900, 122),
        "keyed_n256": W.random_instance(rng(16), 3000, 128, 2600, 128, n_values=60),
        "keyed_n512": W.random_instance(rng(17), 2500, 256, 2200, 256, n_values=30),
    }
    # every group has one B row: no tails at all
    inst = W.random_instance(rng(11), 3000, 6, 1, 5)
    kB = np.arange(0, 600, dtype=np.int32)
    B = rng(12).standard_normal((600, 5))
    kA = np.sort(rng(13).integers(-50, 650, size=3000)).astype(np.int32)
    cases["keyed_singleton_B"] = W.Instance(inst.A, B, kA, kB)
    return cases


CASES = small_cases()


def oracle_results(inst):
    Ro = oracle.r(inst)
    return Ro, oracle.sigma(Ro)


@pytest.mark.parametrize("name", list(CASES))
def test_groups_bit_exact(name):
    inst = CASES[name]
    say(f"[groups] {name} shape={inst.shape}")
    A, B, kA, kB = to_dev(inst)
    out = fg().compact(A, B, kA, kB, "fp64")
    assert out["status"] == 0
    if inst.keys_A is None:
        tab, counts = oracle.groups(None, None, inst.A.shape[0], inst.B.shape[0])
    else:
        tab, counts = oracle.groups(inst.keys_A, inst.keys_B)
    assert np.array_equal(out["counts"], counts), (out["counts"], counts)
    G = int(counts[0])
    got = np.stack([out["groups"][k] for k in ("key", "offA", "m1", "offB", "m2", "r1", "r2")], axis=1)
    assert np.array_equal(got.astype(np.int64), tab[:G])


@pytest.mark.parametrize("name", list(CASES))
def test_compact_matrix_diagnostic(name):
    inst = CASES[name]
    say(f"[compact] {name}")
    A, B, kA, kB = to_dev(inst)
    out = fg().compact(A, B, kA, kB, "fp64")
    M, heads, tab, counts = oracle.compact(inst)
    R1, R2 = int(counts[1]), int(counts[2])
    n1 = inst.A.shape[1]
    scale = max(1.0, np.abs(M).max() if M.size else 1.0)
    assert out["M1"].shape == (R1, M.shape[1]) and out["M2"].shape == (R2, inst.B.shape[1])
    if R1:
        assert np.abs(out["M1"] - M[:R1]).max() <= 1e-13 * scale
    if R2:
        assert np.abs(out["M2"] - M[R1:, n1:]).max() <= 1e-13 * scale
    if heads.size:
        assert np.abs(out["heads"] - heads).max() <= 1e-13 * max(1.0, np.abs(heads).max())


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("form", ["claim1", "two_sided"])
def test_r_and_sigma_parity(name, prec, form):
    inst = CASES[name]
    say(f"[r+sigma] {name} {prec} {form}")
    A, B, kA, kB = to_dev(inst)
    R, ws = fg().r(A, B, kA, kB, prec, two_sided=(form == "two_sided"))
    S = fg().sigma(R)
    torch.cuda.synchronize()
    assert fg().status(ws) == 0
    Ro, So = oracle_results(inst)
    Rg, Sg = R.cpu().numpy(), S.cpu().numpy()
    assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) >= 0)
    d = np.abs(np.diag(Ro))
    if d.size and d.min() <= 1e-10 * max(d.max(), 1e-300):
        # rank deficient: R not unique beyond the rank (parity unpinned); check R^T R only
        Gm = gram_closed_form(inst)
        tol = 1e-10 if prec == "fp64" else 1e-5
        assert np.allclose(Rg.T @ Rg, Gm, rtol=tol, atol=tol * max(1, np.abs(Gm).max()))
        return
    er = relF(Rg, Ro)
    es = np.linalg.norm(Sg - So) / max(np.linalg.norm(So), 1e-300)
    say(f"    relF(R)={er:.3e} rel2(sigma)={es:.3e}")
    assert er <= TOL_R[prec]
    assert es <= TOL_S[prec]


@pytest.mark.parametrize("name", ["cart_ragged", "keyed_zipf_n64", "keyed_uniform_sparse", "keyed_singleton_B"])
def test_two_sided_intermediates(name):
    """Two-sided form: H(A_g) and the A tails against per-group sums and the Helmert rows."""
    inst = CASES[name]
    say(f"[two-sided compact] {name}")
    A, B, kA, kB = to_dev(inst)
    out = fg().compact(A, B, kA, kB, "fp64", two_sided=True)
    tab, counts = (oracle.groups(inst.keys_A, inst.keys_B) if inst.keys_A is not None
                   else oracle.groups(None, None, inst.A.shape[0], inst.B.shape[0]))
    assert np.array_equal(out["counts"], counts)
    Af = np.asarray(inst.A, dtype=np.float64)
    Bf = np.asarray(inst.B, dtype=np.float64)
    n1 = Af.shape[1]
    ta = out["tails_a"]
    hr = out["heads_rows"]
    for g, (key, oa, ma, ob, mb, r1, r2) in enumerate(tab.tolist()):
        Ag = Af[oa:oa + ma]
        hA = Ag.sum(axis=0) / np.sqrt(ma)
        assert np.allclose(out["heads_a"][g], hA, rtol=1e-13, atol=1e-13)
        hB = Bf[ob:ob + mb].sum(axis=0) / np.sqrt(mb)
        assert np.allclose(hr[g], np.concatenate([np.sqrt(mb) * hA, np.sqrt(ma) * hB]), rtol=1e-13, atol=1e-12)
        # tail i: (i * A_{i+1} - S_i) / sqrt(i (i+1)), scaled by sqrt(m2_g)
        if ma > 1:
            i = np.arange(1, ma)[:, None]
            S = np.cumsum(Ag, axis=0)[:-1]
            ref = np.sqrt(mb) * (i * Ag[1:] - S) / np.sqrt(i * (i + 1.0))
            got = ta[r1 - g:r1 - g + ma - 1]
            assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(ref).max()))


def test_fp32_inputs_widened_exactly():
    inst = CASES["keyed_zipf_n64"]
    i32 = W.Instance(inst.A.astype(np.float32), inst.B.astype(np.float32), inst.keys_A, inst.keys_B)
    A, B, kA, kB = to_dev(i32)
    R, ws = fg().r(A, B, kA, kB, "fp64")
    Ro = oracle.r(i32)
    assert relF(R.cpu().numpy(), Ro) <= 1e-12


def test_empty_join():
    inst = W.Instance(np.ones((10, 3)), np.ones((8, 2)), np.arange(10, dtype=np.int32),
                      np.arange(100, 108, dtype=np.int32))
    A, B, kA, kB = to_dev(inst)
    R, ws = fg().r(A, B, kA, kB, "fp64")
    S = fg().sigma(R)
    assert torch.count_nonzero(R).item() == 0 and torch.count_nonzero(S).item() == 0
    out = fg().compact(A, B, kA, kB, "fp64")
    assert list(out["counts"]) == [0, 0, 0, 0]


def test_unsorted_keys_reported():
    inst = W.random_instance(W.rng_for(701), 100, 3, 100, 3, n_values=10)
    kA = inst.keys_A.copy()
    kA[10], kA[90] = kA[90], kA[10]
    bad = W.Instance(inst.A, inst.B, kA, inst.keys_B)
    A, B, kA_d, kB_d = to_dev(bad)
    R, ws = fg().r(A, B, kA_d, kB_d, "fp64")
    assert fg().status(ws) == fg().FIGARO_EUNSORTED
    # no group is formed from unsorted keys: the join is taken as empty and R = 0
    assert torch.count_nonzero(R).item() == 0
    out = fg().compact(A, B, kA_d, kB_d, "fp64")
    assert out["status"] == fg().FIGARO_EUNSORTED and list(out["counts"]) == [0, 0, 0, 0]


@pytest.mark.parametrize("two_sided", [False, True])
def test_deterministic(two_sided):
    inst = CASES["keyed_zipf_n64"]
    A, B, kA, kB = to_dev(inst)
    R1, ws = fg().r(A, B, kA, kB, "fp64", two_sided=two_sided)
    R1 = R1.clone()
    S1 = fg().sigma(R1).clone()
    for _ in range(3):
        R2, _ = fg().r(A, B, kA, kB, "fp64", ws=ws, two_sided=two_sided)
        S2 = fg().sigma(R2)
        assert torch.equal(R1, R2) and torch.equal(S1, S2)


def test_strided_inputs():
    inst = W.random_instance(W.rng_for(702), 2000, 6, 2500, 10, n_values=50)
    A, B, kA, kB = to_dev(inst)
    Abig = torch.zeros((2000, 11), dtype=torch.float64, device=A.device)
    Abig[:, 2:8] = A
    Bbig = torch.zeros((2500, 17), dtype=torch.float64, device=A.device)
    Bbig[:, 5:15] = B
    R, ws = fg().r(Abig[:, 2:8], Bbig[:, 5:15], kA, kB, "fp64")
    assert relF(R.cpu().numpy(), oracle.r(inst)) <= 1e-12


# ------------------------------------------------------------------ the two sigma routes

def special_matrices():
    rng = np.random.default_rng(7)
    out = {
        "zero_8": np.zeros((8, 8)),
        "identity_16": np.eye(16),
        "diag_known_32": np.diag(np.linspace(1.0, 32.0, 32)[::-1].copy()),
        "repeated_64": np.triu(np.linalg.qr(rng.standard_normal((64, 64)))[1] * 0 + np.diag(np.r_[np.full(32, 3.0), np.full(32, 1e-3)])),
        "graded_48": np.triu(rng.standard_normal((48, 48))) * (10.0 ** -np.arange(48) / 4)[None, :],
        "huge_64": np.triu(rng.standard_normal((64, 64))) * 2.0 ** 600,
        "tiny_64": np.triu(rng.standard_normal((64, 64))) * 2.0 ** -600,
        "rank3_100": np.triu(rng.standard_normal((100, 3)) @ rng.standard_normal((3, 100))),
        "random_128": np.triu(rng.standard_normal((128, 128))),
        "random_5": rng.standard_normal((5, 5)),
    }
    return out


SPECIAL = special_matrices()


@pytest.mark.parametrize("name", list(SPECIAL))
@pytest.mark.parametrize("method", ["jacobi", "bidiag", "dqds"])
def test_sigma_routes_match_lapack(name, method):
    """Both sigma routes (one-sided Jacobi; bidiagonalisation + multisection) on special
    matrices against LAPACK's singular values (numpy.linalg.svd), normwise rel2 <= 1e-12."""
    M = SPECIAL[name]
    d = dev()
    R = torch.from_numpy(np.ascontiguousarray(M)).to(d)
    S = fg().sigma(R, method=method).cpu().numpy()
    ref = np.linalg.svd(M, compute_uv=False)
    top = ref[0] if ref.size and ref[0] > 0 else 1.0  # normalise first: norms of 2^600-sized values overflow
    err = np.linalg.norm((S - ref) / top) / max(np.linalg.norm(ref / top), 1e-300) if ref[0] > 0 else np.abs(S).max()
    say(f"[sigma] {name} {method} rel2={err:.3e}")
    assert np.all(np.diff(S) <= 0)
    assert err <= 1e-12
    # and against the oracle's one-sided Jacobi where its squared norms stay finite
    So = oracle.sigma(M) if np.abs(M).max() < 2.0 ** 400 else None
    if So is not None and So[0] > 0:
        eo = np.linalg.norm((S - So) / So[0]) / np.linalg.norm(So / So[0])
        say(f"    vs oracle rel2={eo:.3e}")
        assert eo <= 1e-12


# ------------------------------------------------------------------ refinement sweep

def refine_cases():
    c = {k: CASES[k] for k in ("cart_ragged", "keyed_zipf_n64", "keyed_uniform_sparse",
                               "keyed_singleton_B", "cart_tail_leaf", "keyed_n128", "keyed_n256")}
    # the wide workload's value recipe at a small size: columns scaled by 10^U(-3,0), kappa ~ 1e3
    c["keyed_scaled_small"] = W.config5(m=1 << 13, n=32, n_values=256)
    return c


REFINE_CASES = refine_cases()


@pytest.mark.parametrize("name", list(REFINE_CASES))
@pytest.mark.parametrize("form", ["claim1", "two_sided"])
def test_refine_sweep(name, form):
    """One FP64 sweep against the exact Gram matrix lifts the FP32 form's R to FP64 accuracy."""
    inst = REFINE_CASES[name]
    two = form == "two_sided"
    say(f"[refine] {name} {form} shape={inst.shape}")
    A, B, kA, kB = to_dev(inst)
    R32, _ = fg().r(A, B, kA, kB, "fp32", two_sided=two)
    Rr, ws = fg().r(A, B, kA, kB, "fp32_refine", two_sided=two)
    Sr = fg().sigma(Rr)
    torch.cuda.synchronize()
    assert fg().status(ws) == 0
    Ro, So = oracle_results(inst)
    e32 = relF(R32.cpu().numpy(), Ro)
    er = relF(Rr.cpu().numpy(), Ro)
    es = np.linalg.norm(Sr.cpu().numpy() - So) / np.linalg.norm(So)
    say(f"    relF(R) fp32={e32:.3e} refined={er:.3e} rel2(sigma)={es:.3e}")
    Rg = Rr.cpu().numpy()
    assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) > 0)
    assert er <= 1e-12 and es <= 1e-12
    assert er <= e32


def test_refine_rank_deficient_keeps_gram():
    """Rank-deficient join (one A row): R is not unique; R^T R must still equal J^T J."""
    inst = CASES["cart_one_row_A"]
    A, B, kA, kB = to_dev(inst)
    Rr, ws = fg().r(A, B, kA, kB, "fp32_refine")
    torch.cuda.synchronize()
    Rg = Rr.cpu().numpy()
    Gm = gram_closed_form(inst)
    assert np.all(np.isfinite(Rg))
    assert np.allclose(Rg.T @ Rg, Gm, rtol=1e-5, atol=1e-5 * np.abs(Gm).max())


def test_refine_empty_join():
    inst = W.Instance(np.ones((10, 3)), np.ones((8, 2)), np.arange(10, dtype=np.int32),
                      np.arange(100, 108, dtype=np.int32))
    A, B, kA, kB = to_dev(inst)
    R, ws = fg().r(A, B, kA, kB, "fp32_refine")
    assert torch.count_nonzero(R).item() == 0


# ------------------------------------------------------------------ batched plan (graph)

@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("fp32_refine", 1e-12)])
@pytest.mark.parametrize("two_sided", [False, True])
def test_plan_graph_replays_match_oracle(prec, tol, two_sided):
    """A batch of uneven instances in one captured graph; every replay checked against the oracle."""
    insts = W.config4(count=10, lo=2.0, hi=3.3)
    say(f"[plan] {prec} two_sided={two_sided} shapes={[i.shape for i in insts]}")
    tens = [to_dev(i) for i in insts]
    plan = fg().Plan(tens, prec, two_sided=two_sided)
    d = tens[0][0].device
    ws = torch.empty(plan.ws_bytes, dtype=torch.uint8, device=d)
    R = torch.zeros(plan.r_total, dtype=torch.float64, device=d)
    S = torch.zeros(plan.s_total, dtype=torch.float64, device=d)
    refs = []
    for inst in insts:
        Ro = oracle.r(inst)
        refs.append((Ro, oracle.sigma(Ro)))
    for rep in range(3):
        R.zero_()
        S.zero_()
        plan.execute(ws, R, S)
        torch.cuda.synchronize()
        # eager work between replays
        junk = torch.randn(1000, device=d).sum()
        torch.cuda.synchronize()
        Rh, Sh = R.cpu().numpy(), S.cpu().numpy()
        for i, inst in enumerate(insts):
            N = inst.A.shape[1] + inst.B.shape[1]
            Rg = Rh[plan.r_off[i]:plan.r_off[i] + N * N].reshape(N, N)
            Sg = Sh[plan.s_off[i]:plan.s_off[i] + N]
            Ro, So = refs[i]
            er = relF(Rg, Ro)
            es = np.linalg.norm(Sg - So) / np.linalg.norm(So)
            assert er <= tol and es <= tol, (rep, i, er, es)
        del junk


def mixed_plan_instances():
    """Instances of every kind a plan batches by stage or runs on its own: Cartesian and
    keyed, FP64 and FP32 inputs, padded widths 8 to 128, a ragged keyed join whose root
    is merged per instance, and an empty join."""
    rng = lambda k: W.rng_for(720, k)  # noqa: E731
    out = [
        W.random_instance(rng(1), 700, 4, 900, 4),
        W.random_instance(rng(2), 3000, 5, 2500, 7, n_values=40, key_skew=1.1),
        W.random_instance(rng(3), 1500, 64, 1300, 64, n_values=25),
        W.random_instance(rng(4), 5000, 32, 4000, 32, dtype=np.float32),
        W.random_instance(rng(5), 2200, 16, 1800, 48),
        W.Instance(np.ones((10, 3)), np.ones((8, 2)), np.arange(10, dtype=np.int32),
                   np.arange(100, 108, dtype=np.int32)),
        W.random_instance(rng(6), 1200, 60, 1100, 61),
    ]
    return out


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("fp32_refine", 1e-12)])
@pytest.mark.parametrize("two_sided", [False, True])
def test_plan_mixed_instances(prec, tol, two_sided):
    """A plan whose instances take every route of the stage-by-stage batch, each instance
    against the oracle, on two replays and on an eager run."""
    insts = mixed_plan_instances()
    say(f"[plan mixed] {prec} two_sided={two_sided} shapes={[i.shape for i in insts]}")
    tens = [to_dev(i) for i in insts]
    plan = fg().Plan(tens, prec, two_sided=two_sided)
    d = tens[0][0].device
    ws = torch.empty(plan.ws_bytes, dtype=torch.uint8, device=d)
    R = torch.zeros(plan.r_total, dtype=torch.float64, device=d)
    S = torch.zeros(plan.s_total, dtype=torch.float64, device=d)
    refs = []
    for inst in insts:
        Ro = oracle.r(inst)
        refs.append((Ro, oracle.sigma(Ro)))
    for rep in range(3):
        R.fill_(7.0)
        S.fill_(7.0)
        if rep < 2:
            plan.execute(ws, R, S)
        else:
            plan.execute_eager(ws, R, S)
        torch.cuda.synchronize()
        Rh, Sh = R.cpu().numpy(), S.cpu().numpy()
        for i, inst in enumerate(insts):
            N = inst.A.shape[1] + inst.B.shape[1]
            Rg = Rh[plan.r_off[i]:plan.r_off[i] + N * N].reshape(N, N)
            Sg = Sh[plan.s_off[i]:plan.s_off[i] + N]
            Ro, So = refs[i]
            if not np.any(Ro):
                assert not np.any(Rg) and not np.any(Sg), (rep, i)
                continue
            er = relF(Rg, Ro)
            es = np.linalg.norm(Sg - So) / np.linalg.norm(So)
            assert er <= tol and es <= tol, (rep, i, inst.shape, er, es)


def test_plan_destroyed_while_in_flight():
    """A plan destroyed right after its graph was launched, with no synchronisation in
    between: destruction waits for the launch, the results are whole, and a new plan on
    the same buffers runs normally (regression: plans used to destroy in-flight graphs)."""
    import gc
    insts = W.config4(count=6, lo=2.0, hi=3.3)
    say(f"[plan destroy] shapes={[i.shape for i in insts]}")
    tens = [to_dev(i) for i in insts]
    refs = [oracle.r(inst) for inst in insts]
    d = tens[0][0].device
    for rep in range(2):
        plan = fg().Plan(tens, "fp32", two_sided=True)
        r_off = list(plan.r_off)
        ws = torch.empty(plan.ws_bytes, dtype=torch.uint8, device=d)
        R = torch.full((plan.r_total,), 7.0, dtype=torch.float64, device=d)
        S = torch.zeros(plan.s_total, dtype=torch.float64, device=d)
        plan.execute(ws, R, S)
        del plan
        gc.collect()
        Rh = R.cpu().numpy()
        for i, inst in enumerate(insts):
            N = inst.A.shape[1] + inst.B.shape[1]
            Rg = Rh[r_off[i]:r_off[i] + N * N].reshape(N, N)
            assert relF(Rg, refs[i]) <= 1e-5, (rep, i)


# ------------------------------------------------------------------ the Givens route

@pytest.mark.parametrize("name", ["cart_tiny", "cart_ragged", "cart_uniform_paper", "keyed_zipf_n64",
                                  "keyed_uniform_sparse", "keyed_one_big_group", "keyed_narrow", "keyed_singleton_B",
                                  "cart_tail_leaf", "cart_n125_ragged"])
@pytest.mark.parametrize("form", ["claim1", "two_sided"])
def test_givens_route(name, form):
    """R by Givens rotations entry by entry after Claim 1 (Section 1) against the oracle's R."""
    inst = CASES[name]
    N = inst.A.shape[1] + inst.B.shape[1]
    two = form == "two_sided"
    if N > 64 and not (two and inst.keys_A is None):
        pytest.skip("the Givens route takes regions up to 64 columns")
    say(f"[givens] {name} {form}")
    A, B, kA, kB = to_dev(inst)
    R, ws = fg().r(A, B, kA, kB, "fp64", two_sided=two, givens=True)
    S = fg().sigma(R)
    torch.cuda.synchronize()
    assert fg().status(ws) == 0
    Ro, So = oracle_results(inst)
    Rg = R.cpu().numpy()
    assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) >= 0)
    d = np.abs(np.diag(Ro))
    if d.size and d.min() <= 1e-10 * max(d.max(), 1e-300):
        Gm = gram_closed_form(inst)
        assert np.allclose(Rg.T @ Rg, Gm, rtol=1e-10, atol=1e-10 * max(1, np.abs(Gm).max()))
        return
    er = relF(Rg, Ro)
    es = np.linalg.norm(S.cpu().numpy() - So) / np.linalg.norm(So)
    say(f"    relF(R)={er:.3e} rel2(sigma)={es:.3e}")
    assert er <= 1e-12 and es <= 1e-12


def test_givens_route_full_cfg2():
    inst = W.config2()
    A, B, kA, kB = to_dev(inst)
    R, ws = fg().r(A, B, kA, kB, "fp64", two_sided=True, givens=True)
    torch.cuda.synchronize()
    assert relF(R.cpu().numpy(), oracle.r(inst)) <= 1e-12
