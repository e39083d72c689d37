"""nmc_anneal_noalloc (thresholds in the library's fixed device array, no
device allocation) against nmc_anneal on twin replica sets: identical states,
energies, best energies, snapshots and first hits, over two calls in a row
where the second has the smaller input; calls past the array's size fail
cleanly and leave the set untouched."""
import numpy as np
import pytest

from paper_2111_13628_amd import instances, nmc

pytestmark = pytest.mark.gpu

SEED = instances.DEFAULT_SEED


def say(msg):
    print(msg, flush=True)


def same(a, b):
    for which in ("current", "best"):
        assert (a.get_state(which) == b.get_state(which)).all(), which
    ea, eb = a.best_energy(), b.best_energy()
    for key in ("energy", "best_per_replica", "first_hit"):
        assert (ea[key] == eb[key]).all(), key
    assert a.sweeps_done() == b.sweeps_done()


def ksat_twins(n, R, seed):
    cp, lits = instances.gen_ksat(n, "9.6", 4, seed)
    inst = nmc.Instance.ksat(n, cp, lits).bind()
    return inst, nmc.Replicas(inst, R, seed), nmc.Replicas(inst, R, seed)


def qap_twins(n, R, seed):
    F, D = instances.gen_qap(n, seed)
    inst = nmc.Instance.qap(F, D).bind()
    return inst, nmc.Replicas(inst, R, seed), nmc.Replicas(inst, R, seed)


def test_noalloc_ksat_two_calls_second_smaller():
    # call 1: N = 700, 72 replicas, 120 sweeps with a 2-class host profile
    say("case: noalloc k-SAT N=700 R=72 120 sweeps, then N=150 R=20 30 sweeps")
    inst, a, b = ksat_twins(700, 72, SEED + 11)
    rng = np.random.Generator(np.random.PCG64(5))
    cls = (rng.random(700) < 0.3).astype(np.uint8)
    prof = instances.profile_schedule(np.full(120, 3.0), instances.linear_schedule(0.5, 3.0, 120))
    a.anneal(instances.linear_schedule(0.1, 2.0, 40)[None, :], target=60)
    b.anneal_noalloc(instances.linear_schedule(0.1, 2.0, 40)[None, :], target=60)
    same(a, b)
    a.anneal(prof, "host", cls, target=20)
    b.anneal_noalloc(prof, "host", cls, target=20)
    same(a, b)
    # call 2: a smaller instance and replica set, fewer sweeps, backbone profile
    inst2, c, d = ksat_twins(150, 20, SEED + 12)
    beta = instances.linear_schedule(0.1, 4.0, 30)[None, :]
    c.anneal(beta, target=0)
    d.anneal_noalloc(beta, target=0)
    same(c, d)
    c.estimate_backbone(9, 10, True)
    d.estimate_backbone(9, 10, True)
    rp = instances.profile_schedule(np.full(10, 4.0), instances.linear_schedule(0.5, 4.0, 10))
    c.reanneal(rp, "backbone", target=0)
    d.anneal_noalloc(rp, "backbone", target=0)
    same(c, d)


def test_noalloc_qap_two_calls_second_smaller():
    say("case: noalloc QAP n=60 R=48 12 sweeps, then n=14 R=16 5 sweeps")
    inst, a, b = qap_twins(60, 48, SEED + 21)
    beta = instances.linear_schedule(2e-5, 4e-3, 12)[None, :]
    a.anneal(beta, target=0)
    b.anneal_noalloc(beta, target=0)
    same(a, b)
    inst2, c, d = qap_twins(14, 16, SEED + 22)
    beta = instances.linear_schedule(1e-4, 4e-3, 5)[None, :]
    c.anneal(beta)
    d.anneal_noalloc(beta)
    same(c, d)


def test_noalloc_rejects_oversized_call():
    say("case: noalloc capacity error")
    cap = nmc.lib().nmc_anneal_noalloc_capacity()
    assert cap >= 1 << 20
    inst, a, b = ksat_twins(200, 8, SEED + 31)
    stride = inst.info.max_degree + 1
    too_many = cap // (4 * stride) + 1
    before = a.get_state()
    with pytest.raises(nmc.NmcError) as e:
        a.anneal_noalloc(np.full((1, too_many), 1.0))
    assert e.value.code == -5 and "allocation-free" in str(e.value)
    assert a.sweeps_done() == 0 and (a.get_state() == before).all()
    # the array is intact for the next call
    beta = instances.linear_schedule(0.1, 4.0, 25)[None, :]
    a.anneal_noalloc(beta)
    b.anneal(beta)
    same(a, b)
