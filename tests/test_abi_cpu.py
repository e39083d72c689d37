"""Host-side checks of the C ABI that run without a GPU: every declared
symbol is exported, input validation and error codes, footprints, and the
library's sweep order equals the oracle's colouring."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2111_13628_amd import instances, nmc


def test_library_exports_every_header_symbol():
    L = nmc.lib()
    names = nmc.header_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert L.nmc_version() >= 100


def _load(n, cp, lits, cap=0):
    return nmc.Instance.ksat(n, cp, lits, cap)


@pytest.mark.parametrize("cp,lits,code", [
    ([0, 2], [1, 0], -1),              # literal 0
    ([0, 2], [1, 4], -1),              # variable out of range
    ([0, 2], [2, -2], -1),             # repeated variable
    ([0, 0, 2], [1, 2], -1),           # empty clause
    ([0, 4], [1, 2, 3, -1], -1),       # repeated variable in a 4-literal clause
    ([0, 1, 0], [1], -1),              # decreasing offsets
])
def test_ksat_validation_errors(cp, lits, code):
    with pytest.raises(nmc.NmcError) as e:
        _load(3, np.array(cp), np.array(lits))
    assert e.value.code == code


def test_ksat_offsets_checked_before_literals():
    # clause 0 claims four literals but only three exist: the offsets are
    # rejected (clause 1 decreases) before any literal is read through them
    lits = np.array([1, 2, 3], dtype=np.int32)
    with pytest.raises(nmc.NmcError) as e:
        _load(3, np.array([0, 4, 3]), lits)
    assert e.value.code == -1
    assert "clause 1 is empty or offsets decrease" in str(e.value)
    with pytest.raises(nmc.NmcError) as e:
        _load(6, np.array([0, 5, 3]), lits)
    assert e.value.code == -6 and "clause 0 has 5 literals" in str(e.value)


def test_ksat_unsupported():
    with pytest.raises(nmc.NmcError) as e:
        _load(6, np.array([0, 5]), np.array([1, 2, 3, 4, 5]))
    assert e.value.code == -6
    with pytest.raises(nmc.NmcError) as e:
        _load((1 << 24) - 1, np.array([0, 1]), np.array([1]))
    assert e.value.code == -6
    # a variable in 128 clauses exceeds the per-variable accumulator range
    cp = np.arange(0, 129 * 2, 2)
    lits = np.array([[1, v + 2] for v in range(128)]).ravel()
    with pytest.raises(nmc.NmcError) as e:
        _load(200, cp, lits)
    assert e.value.code == -6


def test_qap_validation_errors():
    F, D = instances.gen_qap(6, 1)
    bad = F.copy()
    bad[0, 1] += 1
    with pytest.raises(nmc.NmcError) as e:
        nmc.Instance.qap(bad, D)
    assert e.value.code == -1
    bad = D.copy()
    bad[2, 2] = 3
    with pytest.raises(nmc.NmcError) as e:
        nmc.Instance.qap(F, bad)
    assert e.value.code == -1
    big = F.copy()
    big[0, 1] = big[1, 0] = 300
    with pytest.raises(nmc.NmcError) as e:
        nmc.Instance.qap(big, D)
    assert e.value.code == -6
    with pytest.raises(nmc.NmcError):
        nmc.Instance.qap(np.zeros((1, 1)), np.zeros((1, 1)))


@pytest.mark.parametrize("n,alpha,k,cap", [(200, "9.6", 4, 0), (300, "4.15", 3, 0), (1000, "9.8", 4, 64),
                                           (5000, "9.9", 4, 1024), (5000, "9.9", 4, 0)])
def test_order_equals_oracle_colouring(n, alpha, k, cap):
    cp, lits = instances.gen_ksat(n, alpha, k, 20211126)
    inst = _load(n, cp, lits, cap)
    order, cptr = inst.order()
    _, o_order, o_cptr = oracle.KSat(n, cp, lits).color(cap)
    assert (order == o_order).all()
    assert (cptr == o_cptr).all()
    assert inst.info.n_colors == len(o_cptr) - 1
    assert inst.info.max_degree == np.bincount(np.abs(lits) - 1, minlength=n).max()


def test_footprints_scale():
    cp, lits = instances.gen_ksat(1000, "9.6", 4, 1)
    inst = _load(1000, cp, lits)
    ib, r64 = inst.footprint(64)
    _, r128 = inst.footprint(128)
    assert ib > 1000 * 38 * 8   # chunk records dominate
    assert r128 > r64 >= 2 * 16 * 1000
    with pytest.raises(nmc.NmcError):
        inst.footprint(0)


def test_unbound_instance_rejects_replicas():
    cp, lits = instances.gen_ksat(50, "9.6", 4, 1)
    inst = _load(50, cp, lits)
    h = ctypes.c_void_p()
    rc = nmc.lib().nmc_replicas_create(inst._h, 4, 1, ctypes.c_void_p(256), 1 << 20, None, ctypes.byref(h))
    assert rc == -4


def test_server_validation_without_gpu():
    """Config and request checks happen on the calling thread, before any GPU
    work; a server whose worker finds no GPU reports it on submit or wait."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("the no-GPU error path needs a machine without a GPU")
    L = nmc.lib()
    h = ctypes.c_void_p()
    bad = nmc.ServerConfig(0, 10, 0, 1, 0, 11, 10, 1)
    assert L.nmc_server_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    bad = nmc.ServerConfig(0, 10, 0, 1, 100, 0, 0, 1)
    assert L.nmc_server_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    cfg = nmc.ServerConfig(0, 10, 0, 1, 0, 0, 0, 1)
    assert L.nmc_server_create(ctypes.byref(cfg), ctypes.byref(h)) == 0
    try:
        cp, lits = instances.gen_ksat(100, "4.2", 3, 1)
        r = nmc.Request(kind=nmc.KIND_KSAT, n_vars=100, n_clauses=cp.size - 1, clause_ptr=cp.ctypes.data,
                        lits=lits.ctypes.data, n_replicas=8, seed=1, beta0=0.1, beta1=3.0, beta_hot=1.0,
                        anneal_sweeps=15, rounds=0, reanneal_sweeps=0)
        rid = ctypes.c_uint64()
        assert L.nmc_server_submit(h, ctypes.byref(r), ctypes.byref(rid)) == -1  # not a multiple of 10
        r.anneal_sweeps, r.kind = 20, 7
        assert L.nmc_server_submit(h, ctypes.byref(r), ctypes.byref(rid)) == -1
        r.kind, r.n_replicas = nmc.KIND_KSAT, 0
        assert L.nmc_server_submit(h, ctypes.byref(r), ctypes.byref(rid)) == -1
        q = nmc.Request(kind=nmc.KIND_QAP, n=300, n_replicas=8, anneal_sweeps=10)
        assert L.nmc_server_submit(h, ctypes.byref(q), ctypes.byref(rid)) == -1
        r.n_replicas = 8
        rc = L.nmc_server_submit(h, ctypes.byref(r), ctypes.byref(rid))
        assert rc in (0, -3)
        assert L.nmc_server_wait_idle(h, 5.0) == -3
        assert b"GPU" in L.nmc_last_error()
        res = nmc.Result()
        assert L.nmc_server_poll(h, 12345, ctypes.byref(res)) == -1
    finally:
        L.nmc_server_free(h)


def test_ksat_wide_layout_chosen_by_size(monkeypatch):
    """Above 65534 variables the instance takes the wide layout (spins in
    device memory); NMC_KSAT_WIDE=1 takes it for any size.  Its replica
    footprint holds the variable-major spin, complement and best tables."""
    cp, lits = instances.gen_ksat(70000, "4.2", 3, 5)
    big = nmc.Instance.ksat(70000, cp, lits)
    assert big.info.wide == 1 and big.info.n_items == 70000
    cp, lits = instances.gen_ksat(300, "9.6", 4, 5)
    small = nmc.Instance.ksat(300, cp, lits)
    assert small.info.wide == 0
    monkeypatch.setenv("NMC_KSAT_WIDE", "1")
    forced = nmc.Instance.ksat(300, cp, lits)
    assert forced.info.wide == 1
    # same colouring and sweep order either way
    assert (forced.order()[0] == small.order()[0]).all() and (forced.order()[1] == small.order()[1]).all()
    _, rep_small = small.footprint(100)
    _, rep_wide = forced.footprint(100)
    assert rep_wide >= rep_small + 3 * 301 * 64
