"""C-ABI boundary checks that need no GPU: the library loads, exports every
declared symbol, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2503_23385_amd as fg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "figaro.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(figaro_[a-z_]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert declared_functions() == sorted(fg.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = fg.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def table(rows=4, cols=3, ld=None, dtype=fg.FIGARO_F64, data=1, keys=None):
    return fg.Table(ctypes.c_void_p(data) if data else None, rows, cols, ld if ld is not None else cols,
                    dtype, ctypes.c_void_p(keys) if keys else None)


def ws_size(A, B, prec=0):
    n = ctypes.c_size_t(0)
    rc = fg.lib().figaro_r_workspace_size(ctypes.byref(A), ctypes.byref(B), prec, ctypes.byref(n))
    return rc, n.value


def test_workspace_size_ok_and_monotone():
    rc, n1 = ws_size(table(100, 4), table(100, 4))
    assert rc == 0 and n1 > 0
    rc, n2 = ws_size(table(1000, 4), table(1000, 4))
    assert rc == 0 and n2 > n1
    rc, nk = ws_size(table(1000, 4, keys=8), table(1000, 4, keys=8))
    assert rc == 0 and nk > n2


@pytest.mark.parametrize("A,B,prec", [
    (table(4, 3, ld=2), table(), 0),                      # ld < cols
    (table(dtype=fg.FIGARO_F32), table(), 0),             # dtype mismatch
    (table(keys=8), table(), 0),                          # keys on one side only
    (table(cols=0), table(), 0),                          # empty width
    (table(data=0), table(), 0),                          # null data
    (table(dtype=7), table(dtype=7), 0),                  # bad dtype
    (table(), table(), 9),                                # bad precision
    (table(cols=300), table(cols=300), 1),                # N > 512
    (table(), table(), 0x400),                            # unknown flag
    (table(), table(), 0x201),                            # Givens route with FP32
    (table(cols=40), table(cols=30), 0x200),              # Givens route, region 1 wider than 64
    (table(cols=65), table(cols=3), 0x300),               # Givens route, a tail wider than 64
    (table(), table(), 0x101 | 0x400),                    # unknown flag beside a valid one
])
def test_invalid_arguments_rejected_on_host(A, B, prec):
    rc, _ = ws_size(A, B, prec)
    assert rc == fg.FIGARO_EINVAL
    msg = fg.lib().figaro_last_error().decode()
    assert msg


@pytest.mark.parametrize("prec", [0, 1, 2, 0x100, 0x102])
def test_wide_rows_accepted(prec):
    """Widths up to FIGARO_MAX_N in every precision and form (blocked panel kernel)."""
    for n1, n2 in ((100, 100), (256, 256), (1, 511)):
        rc, n = ws_size(table(1000, n1, keys=8), table(900, n2, keys=8), prec)
        assert rc == 0 and n > 0, (n1, n2, prec)


def test_two_sided_flag_accepted_and_sized():
    rc, n_c = ws_size(table(1000, 4, keys=8), table(1000, 4, keys=8), 0)
    rc2, n_t = ws_size(table(1000, 4, keys=8), table(1000, 4, keys=8), 0x100)
    assert rc == 0 and rc2 == 0 and n_t > 0


def test_refine_precision_adds_workspace():
    """The refinement sweep needs FP64 Gram and solve buffers beyond the FP32 form's."""
    A, B = table(5000, 64, keys=8), table(4000, 64, keys=8)
    rc1, n32 = ws_size(A, B, 1)
    rc2, nref = ws_size(A, B, 2)
    rc3, nref2 = ws_size(A, B, 2 | 0x100)
    assert rc1 == rc2 == rc3 == 0
    assert nref >= n32 + 3 * 128 * 128 * 8


def test_figaro_r_host_checks():
    L = fg.lib()
    A, B = table(), table()
    rc, n = ws_size(A, B)
    # null R
    assert L.figaro_r(ctypes.byref(A), ctypes.byref(B), 0, None, 6, ctypes.c_void_p(256), n, None) == fg.FIGARO_EINVAL
    # ldr < N
    assert L.figaro_r(ctypes.byref(A), ctypes.byref(B), 0, ctypes.c_void_p(256), 5, ctypes.c_void_p(256), n, None) == fg.FIGARO_EINVAL
    # workspace too small
    assert L.figaro_r(ctypes.byref(A), ctypes.byref(B), 0, ctypes.c_void_p(256), 6, ctypes.c_void_p(256), n - 1, None) == fg.FIGARO_EWORKSPACE
    # misaligned workspace
    assert L.figaro_r(ctypes.byref(A), ctypes.byref(B), 0, ctypes.c_void_p(256), 6, ctypes.c_void_p(264), n, None) == fg.FIGARO_EINVAL


def test_sigma_host_checks():
    L = fg.lib()
    n = ctypes.c_size_t(0)
    assert L.figaro_sigma_workspace_size(0, ctypes.byref(n)) == fg.FIGARO_EINVAL
    assert L.figaro_sigma_workspace_size(8, ctypes.byref(n)) == 0 and n.value > 0
    p = ctypes.c_void_p(256)
    for fn in (L.figaro_sigma, L.figaro_sigma_jacobi, L.figaro_sigma_bidiag):
        assert fn(None, 8, 8, p, p, n.value, None) == fg.FIGARO_EINVAL          # R is NULL
        assert fn(p, 8, 4, p, p, n.value, None) == fg.FIGARO_EINVAL             # ldr < n
        assert fn(p, 8, 8, p, ctypes.c_void_p(264), n.value, None) == fg.FIGARO_EINVAL  # misaligned
        assert fn(p, 8, 8, p, p, n.value - 1, None) == fg.FIGARO_EWORKSPACE    # workspace too small
        assert fn(p, 513, 513, p, p, 1 << 30, None) == fg.FIGARO_EINVAL         # n above 512


def test_sigma_workspace_covers_both_routes():
    """The workspace holds the multisection inputs of the bidiagonal route (2n + 2 doubles
    after the 256-byte control block) up to n = 128 and the block-Jacobi columns above."""
    L = fg.lib()
    for k, want in ((8, 256 + 8 * 18), (64, 256 + 8 * 130), (128, 256 + 8 * 258), (200, 256 + 8 * 256 * 256),
                    (512, 256 + 8 * 512 * 512)):
        n = ctypes.c_size_t(0)
        assert L.figaro_sigma_workspace_size(k, ctypes.byref(n)) == 0
        assert n.value == want, (k, n.value, want)


def test_sigma_bidiag_rejects_wide():
    L = fg.lib()
    n = ctypes.c_size_t(0)
    assert L.figaro_sigma_workspace_size(200, ctypes.byref(n)) == 0
    p = ctypes.c_void_p(256)
    assert L.figaro_sigma_bidiag(p, 200, 200, p, p, n.value, None) == fg.FIGARO_EINVAL


def test_plan_host_checks():
    L = fg.lib()
    arr = (fg.Instance * 2)()
    arr[0].A, arr[0].B = table(10, 3), table(12, 2)
    arr[1].A, arr[1].B = table(5, 4), table(7, 4)
    h = ctypes.c_void_p()
    assert L.figaro_plan_create(arr, 2, 0, ctypes.byref(h)) == 0
    import numpy as np
    ro, so = np.zeros(2, np.int64), np.zeros(2, np.int64)
    rt, st = ctypes.c_int64(), ctypes.c_int64()
    assert L.figaro_plan_offsets(h, ro.ctypes.data_as(ctypes.c_void_p), so.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(rt), ctypes.byref(st)) == 0
    assert list(ro) == [0, 25] and list(so) == [0, 5] and rt.value == 25 + 64 and st.value == 13
    L.figaro_plan_destroy(h)
    bad = (fg.Instance * 1)()
    bad[0].A, bad[0].B = table(10, 3, ld=1), table(12, 2)
    assert L.figaro_plan_create(bad, 1, 0, ctypes.byref(h)) == fg.FIGARO_EINVAL


def test_tuning_cache_plan_entries(tmp_path):
    """Plan-level tuning entries (host only): the chaining mode per accumulation type
    (acc_f64 3) and the width-128 tree choice load and save; out-of-range kinds are
    skipped; plan workspace sizes do not depend on them."""
    arr = (fg.Instance * 2)()
    arr[0].A, arr[0].B = table(3000, 64), table(2000, 64)
    arr[1].A, arr[1].B = table(500, 8), table(700, 8)
    h = ctypes.c_void_p()
    n0 = ctypes.c_size_t(0)
    assert fg.lib().figaro_plan_create(arr, 2, 0, ctypes.byref(h)) == 0
    assert fg.lib().figaro_plan_workspace_size(h, ctypes.byref(n0)) == 0
    fg.lib().figaro_plan_destroy(h)
    path = tmp_path / "plan.jsonl"
    lines = ['{"arch":"gfx950","acc_f64":3,"np":0,"batched":1,"rows_log2":0,"kind":1,"leaf_blocks":0,"arity":2,"ms":1}',
             '{"arch":"gfx950","acc_f64":0,"np":128,"batched":0,"rows_log2":20,"kind":1,"leaf_blocks":4,'
             '"arity":2,"ms":1}',
             '{"arch":"gfx950","acc_f64":4,"np":0,"batched":1,"rows_log2":0,"kind":1,"leaf_blocks":0,"arity":2}']
    path.write_text("\n".join(lines) + "\n")
    assert fg.lib().figaro_tune_load(os.fsencode(str(path))) == 0
    tab = fg.tune_table()
    assert any(e["acc_f64"] == 3 and e["np"] == 0 and e["kind"] == 1 for e in tab)
    assert any(e["acc_f64"] == 0 and e["np"] == 128 and e["kind"] == 1 and e["leaf_blocks"] == 4 for e in tab)
    assert not any(e["acc_f64"] == 4 for e in tab)
    n1 = ctypes.c_size_t(0)
    assert fg.lib().figaro_plan_create(arr, 2, 0, ctypes.byref(h)) == 0
    assert fg.lib().figaro_plan_workspace_size(h, ctypes.byref(n1)) == 0
    fg.lib().figaro_plan_destroy(h)
    assert n0.value == n1.value
    # back to the defaults: chains one after the other, the panel tree at width 128
    path.write_text('{"arch":"gfx950","acc_f64":3,"np":0,"batched":1,"rows_log2":0,"kind":0,"leaf_blocks":0,'
                    '"arity":2,"ms":0}\n'
                    '{"arch":"gfx950","acc_f64":0,"np":128,"batched":0,"rows_log2":20,"kind":0,"leaf_blocks":0,'
                    '"arity":2,"ms":0}\n')
    assert fg.lib().figaro_tune_load(os.fsencode(str(path))) == 0


def test_tuning_cache_round_trip(tmp_path):
    """The tuning cache (host only): entries load, malformed or foreign lines are skipped,
    the table saves and reloads, and workspace sizes do not depend on the table."""
    A, B = table(200000, 32), table(150000, 32)
    before = {p: ws_size(A, B, p)[1] for p in (0, 1, 0x100, 0x101)}
    path = tmp_path / "tune.jsonl"
    good = ('{"arch":"gfx950","acc_f64":0,"np":32,"batched":0,"rows_log2":18,"kind":1,'
            '"leaf_blocks":16,"arity":2,"ms":0.5}')
    lines = [good,
             '{"arch":"gfx942","acc_f64":0,"np":32,"batched":0,"rows_log2":18,"kind":1,"leaf_blocks":8,"arity":2}',
             '{"arch":"gfx950","acc_f64":0,"np":32,"batched":0,"rows_log2":17,"kind":5,"leaf_blocks":8,"arity":2}',
             'not json']
    path.write_text("\n".join(lines) + "\n")
    assert fg.lib().figaro_tune_load(os.fsencode(str(path))) == 0
    tab = fg.tune_table()
    mine = [e for e in tab if e["np"] == 32 and e["batched"] == 0 and e["acc_f64"] == 0]
    assert any(e["rows_log2"] == 18 and e["kind"] == 1 and e["leaf_blocks"] == 16 for e in mine)
    assert not any(e["rows_log2"] == 17 for e in mine)
    out = tmp_path / "saved.jsonl"
    assert fg.lib().figaro_tune_save(os.fsencode(str(out))) == 0
    saved = out.read_text().splitlines()
    assert any('"rows_log2":18' in line and '"leaf_blocks":16' in line for line in saved)
    assert fg.lib().figaro_tune_load(os.fsencode(str(out))) == 0
    assert fg.lib().figaro_tune_load(os.fsencode(str(tmp_path / "missing.jsonl"))) == fg.FIGARO_EINVAL
    after = {p: ws_size(A, B, p)[1] for p in (0, 1, 0x100, 0x101)}
    assert before == after
