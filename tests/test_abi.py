"""The C-ABI library loads and exports every declared symbol; host-side checks.

No GPU needed: only host code of the library runs here (validation and the
arena size computation).
"""
import ctypes as C
import os

import pytest

from paper_2111_11682_amd import lshmf


def test_library_exports_every_header_function():
    L = lshmf.lib()
    names = lshmf.header_functions()
    assert {"build_lsh_neighbours", "sgd_epoch", "predict", "online_update", "lshmf_ingest",
            "lshmf_rmse", "lshmf_loss", "lshmf_check"} <= set(names)
    for n in names:
        assert hasattr(L, n), n


def _create(**kw):
    base = dict(M=943, N=1682, F=32, K=10, G=8, p=1, q=8, rscale=1, psi_exp=2, n_strata=16,
                storage=0, hash_family=0, model=0, reserved=0, nnz=90000, M_cap=0, N_cap=0, nnz_cap=0, batch_cap=0)
    base.update(kw)
    d = lshmf.Dims(*[base[f] for f, _ in lshmf.Dims._fields_])
    h = C.c_void_p()
    st = lshmf.lib().lshmf_create(C.byref(d), C.byref(h))
    return st, h


@pytest.mark.parametrize("bad", [dict(K=-1), dict(K=1682), dict(K=129), dict(F=0), dict(F=257),
                                 dict(G=8, p=8, q=1), dict(G=8, p=1, q=1025), dict(G=8, p=7, q=512),
                                 dict(G=40, p=1, q=4, hash_family=2), dict(hash_family=3),
                                 dict(model=1), dict(model=2, K=0),
                                 dict(rscale=3),
                                 dict(psi_exp=0), dict(n_strata=0), dict(storage=3),
                                 dict(nnz=-1), dict(M=0), dict(N=1), dict(M_cap=900),
                                 dict(N_cap=1000), dict(nnz_cap=100), dict(batch_cap=-1)])
def test_create_rejects_bad_dims(bad):
    st, h = _create(**bad)
    assert st == -1
    assert lshmf.lib().lshmf_last_error()


def test_arena_size_and_bind_checks():
    st, h = _create()
    assert st == 0
    n = C.c_size_t()
    assert lshmf.lib().lshmf_arena_bytes(h, C.byref(n)) == 0
    assert n.value > 90000 * 20
    t = lshmf.Tables(*([0] * 16))
    assert lshmf.lib().lshmf_bind(h, C.byref(t), C.c_void_p(256), n.value) == -1   # NULL tables
    t = lshmf.Tables(*([4096] * 12 + [0] * 4))
    assert lshmf.lib().lshmf_bind(h, C.byref(t), C.c_void_p(4096 + 16), n.value) == -1  # unaligned
    assert lshmf.lib().lshmf_bind(h, C.byref(t), C.c_void_p(4096), n.value - 1) == -3  # too small
    # BF16 storage needs its four copies
    st, h2 = _create(storage=1)
    assert st == 0
    n2 = C.c_size_t()
    assert lshmf.lib().lshmf_arena_bytes(h2, C.byref(n2)) == 0
    assert lshmf.lib().lshmf_bind(h2, C.byref(t), C.c_void_p(4096), n2.value) == -1
    lshmf.lib().lshmf_destroy(h2)
    # calls out of order report ESTATE without touching the device
    assert lshmf.lib().sgd_epoch(h, None, 0, None, None) == -2
    assert lshmf.lib().lshmf_loss(h, None, None, None) == -2
    assert lshmf.lib().online_update(h, None, None, None, 0, 943, 1682, None, 0, None, 0, 1, 0,
                                     None) == -2
    lshmf.lib().lshmf_destroy(h)


def test_k0_binds_without_neighbour_tables():
    # K = 0 (no neighbour term): W, C, JK and their BF16 copies may be NULL;
    # with K > 0 they may not.  A one-byte-short arena then gives ECAPACITY.
    for storage in (0, 1):
        st, h = _create(K=0, storage=storage)
        assert st == 0
        n = C.c_size_t()
        assert lshmf.lib().lshmf_arena_bytes(h, C.byref(n)) == 0
        ptr = [4096] * 16
        for x in (4, 5, 6, 14, 15):   # W, C, JK, W16, C16
            ptr[x] = 0
        t = lshmf.Tables(*ptr)
        assert lshmf.lib().lshmf_bind(h, C.byref(t), C.c_void_p(4096), n.value - 1) == -3
        lshmf.lib().lshmf_destroy(h)
    st, h = _create(K=10)
    n = C.c_size_t()
    assert lshmf.lib().lshmf_arena_bytes(h, C.byref(n)) == 0
    assert lshmf.lib().lshmf_bind(h, C.byref(t), C.c_void_p(4096), n.value - 1) == -1
    lshmf.lib().lshmf_destroy(h)


def test_arena_grows_with_capacities():
    sizes = []
    for kw in (dict(), dict(M_cap=2000, N_cap=3000, nnz_cap=200000), dict(batch_cap=50000)):
        st, h = _create(**kw)
        assert st == 0
        n = C.c_size_t()
        assert lshmf.lib().lshmf_arena_bytes(h, C.byref(n)) == 0
        sizes.append(n.value)
        lshmf.lib().lshmf_destroy(h)
    assert sizes[1] > sizes[0] + 110000 * 20 and sizes[2] > sizes[0] + 3 * 50000 * 20


def test_binding_has_no_cpu_fallback(monkeypatch):
    monkeypatch.setattr(lshmf, "_lib", None)
    monkeypatch.setattr(lshmf, "LIB_PATH", os.path.join(os.path.dirname(lshmf.LIB_PATH), "missing.so"))
    with pytest.raises(ImportError):
        lshmf.lib()


def test_serve_entry_checks_on_host():
    st, h = _create(batch_cap=1000)
    assert st == 0
    n = C.c_size_t()
    assert lshmf.lib().lshmf_serve_stage_bytes(h, 4096, C.byref(n)) == 0
    assert n.value >= 1000 * 9 + 2 * 3 * 4096 * 4
    assert lshmf.lib().lshmf_serve_stage_bytes(h, 0, C.byref(n)) == -1
    io = lshmf.ServeIO()
    # before the neighbours exist the loop refuses to start, without touching the device
    assert lshmf.lib().lshmf_serve(h, C.byref(io), C.c_void_p(1), C.c_void_p(2)) == -2
    lshmf.lib().lshmf_destroy(h)


def test_request_record_layout():
    import numpy as np
    from paper_2111_11682_amd import synth

    class Req(C.Structure):
        _fields_ = [("kind", C.c_int32), ("M_new", C.c_int32), ("N_new", C.c_int32),
                    ("reserved", C.c_int32), ("offset", C.c_int64), ("n", C.c_int64),
                    ("arrival", C.c_double)]
    assert lshmf.REQUEST_DTYPE.itemsize == C.sizeof(Req) == 40
    assert np.dtype(synth.REQUEST_FIELDS, align=True) == lshmf.REQUEST_DTYPE
    for name, _ in Req._fields_:
        assert lshmf.REQUEST_DTYPE.fields[name][1] == getattr(Req, name).offset


@pytest.mark.parametrize("ok", [dict(G=8, p=3, q=100), dict(G=8, p=3, q=200), dict(G=8, p=2, q=16),
                                dict(G=8, p=7, q=128), dict(G=8, p=1, q=16, hash_family=1),
                                dict(G=8, p=3, q=16, hash_family=2)])
def test_create_accepts_the_papers_hash_shapes(ok):
    # Sec. 5.3 runs simLSH with G = 8, p = 3 and q = 100 or 200 (B = 2400, 4800)
    st, h = _create(**ok)
    assert st == 0, lshmf.lib().lshmf_last_error()
    lshmf.lib().lshmf_destroy(h)


def test_the_1b_rating_shape_fits_one_gpu():
    """2M users x 500k items with 999M training ratings, F = 128, K = 64,
    B = 256 and 4096 strata: accepted, with an arena that leaves room for the
    tables and the input triples in 288 GB of HBM."""
    from paper_2111_11682_amd import synth
    w = synth.WORKLOADS["large1b"]
    nnz = w.nnz - w.n_test
    st, h = _create(M=w.M, N=w.N, F=w.F, K=w.K, G=w.G, p=w.p, q=w.q, rscale=w.rscale,
                    n_strata=w.n_strata, nnz=nnz)
    assert st == 0, lshmf.lib().lshmf_last_error()
    n = C.c_size_t()
    assert lshmf.lib().lshmf_arena_bytes(h, C.byref(n)) == 0
    lshmf.lib().lshmf_destroy(h)
    tables = 4 * (w.M * w.F + w.N * w.F + 3 * w.N * w.K + w.N * w.B + 2 * (w.M + w.N))
    inputs = 9 * nnz + 4 * (w.M + w.N) * w.F
    assert nnz * 60 < n.value and n.value + tables + inputs < 200e9
    # the stream sort key (block, item rank, user rank) must fit 64 bits
    bits = lambda v: int(v - 1).bit_length()
    assert bits(w.n_strata ** 2) + bits(w.N) + bits(w.M) <= 64
