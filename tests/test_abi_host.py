"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/dmpc.h declares, and its host-only validation and workspace
sizing behave as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2510_06179_amd import _lib, batch
from paper_2510_06179_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "dmpc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dmpc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTED)


def test_version_and_status_strings():
    lib = _lib.load()
    assert lib.dmpc_version() >= 100
    for code in range(5):
        assert lib.dmpc_status_string(code)
    assert lib.dmpc_status_string(0) == b"ok"


def _validate(pk, opts=None):
    lib = _lib.load()
    o = opts or _lib.make_opts()
    bad = ctypes.c_int32(-7)
    d = np.ascontiguousarray(pk.descs)
    rc = lib.dmpc_validate(d.ctypes.data_as(ctypes.c_void_p), len(d), pk.data_len, pk.sol_len,
                           ctypes.byref(o), ctypes.byref(bad))
    return rc, bad.value


def test_validate_accepts_benchmark_batches():
    for probs in (W.lq_batch(0), W.cartpole_batch(0, batch=4), W.bicycle_batch(0, batch=2),
                  W.ltv_uneven_batch(0, batch=16)):
        rc, bad = _validate(batch.pack(probs))
        assert rc == _lib.DMPC_OK and bad == -1


def test_validate_empty_batch():
    pk = batch.pack([])
    rc, _ = _validate(pk)
    assert rc == _lib.DMPC_OK


@pytest.mark.parametrize("field,value", [
    ("T", 0), ("nx", 0), ("nx", 17), ("nu", 0), ("dyn", 7), ("cost", 5), ("reserved", 1),
    ("dyn_off", -1), ("x0_off", 10 ** 9), ("sol_off", 10 ** 9), ("cost_phases", 2),
])
def test_validate_rejects_bad_descriptor(field, value):
    pk = batch.pack(W.lq_batch(0, batch=3))
    pk.descs[1][field] = value
    rc, bad = _validate(pk)
    assert rc == _lib.DMPC_ERR_INVALID_ARG
    assert bad == 1


def test_validate_model_shapes():
    pk = batch.pack(W.cartpole_batch(0, batch=2))
    pk.descs[0]["dyn"] = _lib.DYN_BICYCLE          # bicycle needs nx=8, nu=2
    rc, bad = _validate(pk)
    assert rc == _lib.DMPC_ERR_INVALID_ARG and bad == 0


def test_validate_unsupported_state_size():
    rng = np.random.default_rng(0)
    pk = batch.pack([W.ltv_problem(rng, 5, 5, 2)])  # nx=5 has no kernel
    rc, bad = _validate(pk)
    assert rc == _lib.DMPC_ERR_UNSUPPORTED and bad == 0


def test_validate_overlapping_solution_blocks():
    pk = batch.pack(W.lq_batch(0, batch=3))
    pk.descs[2]["sol_off"] = pk.descs[1]["sol_off"] + 1
    rc, bad = _validate(pk)
    assert rc == _lib.DMPC_ERR_INVALID_ARG


@pytest.mark.parametrize("kw", [
    dict(sqp_iters=0), dict(alphas=()), dict(alphas=(1.0, 1.0)), dict(alphas=(0.5, 0.7)),
    dict(alphas=(1.5,)), dict(ls_eta=1.0), dict(pcg_tol=-1.0), dict(init=3),
    dict(block_threads=100), dict(pcg_max_iter=-2),
])
def test_validate_rejects_bad_options(kw):
    pk = batch.pack(W.lq_batch(0, batch=2))
    if kw.get("alphas") == ():
        o = _lib.make_opts()
        o.n_alphas = 0
    else:
        o = _lib.make_opts(**kw)
    rc, _ = _validate(pk, o)
    assert rc == _lib.DMPC_ERR_INVALID_ARG


def test_workspace_size_is_additive():
    lib = _lib.load()
    o = _lib.make_opts()
    sizes = []
    pks = [batch.pack(W.lq_batch(0, batch=2)), batch.pack(W.cartpole_batch(0, batch=3))]
    for pk in pks:
        n = ctypes.c_size_t()
        d = np.ascontiguousarray(pk.descs)
        assert lib.dmpc_workspace_size(d.ctypes.data_as(ctypes.c_void_p), len(d), ctypes.byref(o),
                                       ctypes.byref(n)) == 0
        assert n.value > 0 and n.value % 256 == 0
        sizes.append(n.value)
    both = np.concatenate([pks[0].descs, pks[1].descs])
    n = ctypes.c_size_t()
    assert lib.dmpc_workspace_size(both.ctypes.data_as(ctypes.c_void_p), len(both), ctypes.byref(o),
                                   ctypes.byref(n)) == 0
    assert n.value == sum(sizes)


def test_default_options_follow_the_paper():
    o = _lib.make_opts()
    assert [round(o.alphas[i], 6) for i in range(o.n_alphas)] == [1.0, 0.7, 0.3, 0.1, 0.01]
    assert abs(o.ls_eta - 0.4) < 1e-7


def test_pack_roundtrip():
    probs = W.ltv_uneven_batch(3, batch=5)
    pk = batch.pack(probs)
    for k, p in enumerate(probs):
        x, u, lam = batch.split_sol(pk, pk.sol0, k)
        assert np.array_equal(x, p["xbar"].astype(np.float32))
        g = batch.split_grad(pk, pk.data, k)
        assert np.array_equal(g["A"], p["A"].astype(np.float32))
        assert np.array_equal(g["Rd"], p["Rd"].astype(np.float32))
        assert np.array_equal(g["x0"], p["x0"].astype(np.float32))


# ---------------------------------------------------------------------------
# kernel mapping: variants, cost model, tuning table (host only)
# ---------------------------------------------------------------------------
def _mapping(p, **opts):
    from paper_2510_06179_amd import batch as bt
    pk = bt.pack([p])
    d = pk.descs[0]
    desc = _lib.Problem(*[d[n].item() for n in _lib.PROBLEM_DTYPE.names])
    o = _lib.make_opts(**opts)
    out = np.zeros(4, np.int32)
    rc = _lib.load().dmpc_choose_mapping(ctypes.byref(desc), ctypes.byref(o), out.ctypes.data)
    return rc, tuple(int(v) for v in out)


def test_variants_cover_every_state_size():
    v = _lib.variants()
    assert {r[0] for r in v} == {2, 3, 4, 8, 12, 16, 32}
    for nx, slots, maxbt, reg in v:
        assert slots >= 1 and maxbt % 64 == 0 and 64 <= maxbt <= 1024 and reg in (0, 1, 2, 3, 4, 5)
        assert reg != 2 or (maxbt == 64 and slots % nx == 0)
        assert reg != 4 or (maxbt == 512 and slots >= 2)


def test_mapping_holds_the_rows_and_respects_forced_threads():
    saved = _saved_tuning()
    try:
        _lib.install_tuning([])
        rng = np.random.default_rng(0)
        for T in (16, 50, 128):
            for nx in (4, 8, 12, 16):
                rc, (slots, maxbt, reg, bt) = _mapping(W.ltv_problem(rng, T, nx, 2))
                assert rc == _lib.DMPC_OK
                assert slots * bt >= (T + 1) * nx and bt % 64 == 0 and bt <= maxbt
        rc, m = _mapping(W.cartpole_batch(0, batch=1)[0], block_threads=128)
        assert rc == _lib.DMPC_OK and m[3] == 128
    finally:
        _lib.install_tuning(saved)


def _saved_tuning():
    lib = _lib.load()
    n = lib.dmpc_get_tuning(None, 0)
    rows = np.zeros((max(n, 1), 7), np.int32)
    lib.dmpc_get_tuning(rows.ctypes.data, n)
    return [tuple(int(v) for v in r) for r in rows[:n]]


def test_tuning_table_overrides_the_cost_model():
    saved = _saved_tuning()
    try:
        p = W.cartpole_batch(0, batch=1)[0]          # nx=4, T=50: 204 rows
        _lib.install_tuning([(4, 40, 60, 1, 256, 1, 256)])
        assert _mapping(p)[1] == (1, 256, 1, 256)
        assert _saved_tuning() == [(4, 40, 60, 1, 256, 1, 256)]
        # a row that cannot hold the problem is skipped
        _lib.install_tuning([(4, 40, 60, 1, 128, 1, 128)])
        rc, m = _mapping(p)
        assert rc == _lib.DMPC_OK and m[0] * m[3] >= 204 and m != (1, 128, 1, 128)
        # outside the T range the cost model decides
        _lib.install_tuning([])
        model = _mapping(p)[1]
        _lib.install_tuning([(4, 1, 10, 1, 256, 1, 256)])
        assert _mapping(p)[1] == model
        # forcing the threads per workgroup bypasses the table
        _lib.install_tuning([(4, 40, 60, 1, 256, 1, 256)])
        assert _mapping(p, block_threads=64)[1][3] == 64
        # malformed rows are refused and leave the table as it was
        for bad in [(5, 1, 9, 1, 64, 1, 64), (4, 9, 1, 1, 64, 1, 64), (4, 1, 9, 1, 64, 4, 64), (4, 1, 9, 2, 64, 2, 64),
                    (4, 1, 9, 1, 64, 1, 96), (4, 1, 9, 1, 64, 1, 128), (16, 1, 9, 5, 512, 4, 448),
                    (16, 1, 9, 1, 512, 4, 512), (16, 1, 9, 5, 512, 6, 512)]:
            with pytest.raises(_lib.DmpcError):
                _lib.install_tuning([bad])
        assert _saved_tuning() == [(4, 40, 60, 1, 256, 1, 256)]
    finally:
        _lib.install_tuning(saved)


def test_lds_row_mapping_only_where_its_lds_fits():
    """Kernels with the last slot's Schur rows in LDS (register_rows = 4) hold
    T = 128, nx = 16 (2064 rows: four register slots of 512 threads and 16 LDS
    rows); one more stage no longer fits the LDS, and the table row is
    skipped."""
    saved = _saved_tuning()
    try:
        rng = np.random.default_rng(3)
        _lib.install_tuning([(16, 1, 1000, 5, 512, 4, 512)])
        assert _mapping(W.ltv_problem(rng, 128, 16, 4)) == (_lib.DMPC_OK, (5, 512, 4, 512))
        assert _mapping(W.ltv_problem(rng, 100, 16, 2)) == (_lib.DMPC_OK, (5, 512, 4, 512))
        rc, m = _mapping(W.ltv_problem(rng, 129, 16, 4))
        assert rc == _lib.DMPC_OK and m[2] != 4 and m[0] * m[3] >= 130 * 16
    finally:
        _lib.install_tuning(saved)
