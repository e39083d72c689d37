"""The wide k-SAT layout (spins in device memory, one lane per group of 4
replicas, one launch per colour class) vs the CPU oracle: bit-exact states,
energies, best energies, first hits, best-state snapshots and backbones.
Small instances take the layout through NMC_KSAT_WIDE=1; N = 70,000 takes it
by size."""
import numpy as np
import pytest

from gpu_util import KsatPair, say
from paper_2111_13628_amd import instances, nmc

pytestmark = pytest.mark.gpu

SEED = instances.DEFAULT_SEED


def reanneal_profile(S, beta_hot=0.5, beta_end=4.0):
    return instances.profile_schedule(np.full(S, beta_end), instances.linear_schedule(beta_hot, beta_end, S))


@pytest.mark.parametrize("n,alpha,k,R,cap", [(300, "9.6", 4, 38, 0), (700, "4.15", 3, 21, 64), (200, "9.6", 4, 4, 0),
                                             (500, "9.6", 4, 300, 0), (120, "9.6", 4, 9, 1), (260, "9.6", 4, 1101, 0),
                                             (150, "4.15", 3, 2048, 0)])
def test_wide_nmc_rounds_match_oracle(n, alpha, k, R, cap, monkeypatch):
    """anneal -> backbone -> reanneal, twice, on the wide layout: ragged
    replica counts, more than 64 groups (two lane blocks), rows of 512 groups
    with four groups per lane (R = 1101: a partial last group; R = 2048),
    3-SAT with variables of no clause, and one variable per class (cap 1)."""
    monkeypatch.setenv("NMC_KSAT_WIDE", "1")
    say(f"case: wide nmc rounds n={n} k={k} R={R} cap={cap}")
    cp, lits = instances.gen_ksat(n, alpha, k, SEED + n)
    p = KsatPair(n, cp, lits, R, SEED + 1, cap=cap)
    assert p.inst.info.wide == 1
    p.anneal(instances.linear_schedule(0.1, 4.0, 40)[None, :], target=2)
    p.compare()
    for rnd in range(2):
        cls = p.backbone(9, 10, expand=True)
        say(f"  round {rnd}: hot = {int(cls.sum())}")
        p.anneal(reanneal_profile(15), profile="backbone", class_of=cls, target=1)
        p.compare()


def test_wide_host_profile_and_extremes(monkeypatch):
    """Three host classes, beta = 0 (every flip accepted but for a word of
    2^32 - 1) and beta = 60, and a call of zero sweeps with a target."""
    monkeypatch.setenv("NMC_KSAT_WIDE", "1")
    say("case: wide host profile")
    n = 400
    cp, lits = instances.gen_ksat(n, "9.6", 4, 7)
    p = KsatPair(n, cp, lits, 13, 77)
    rng = np.random.Generator(np.random.PCG64(1))
    cls = rng.integers(0, 3, n).astype(np.uint8)
    beta = np.stack([instances.linear_schedule(0.1, 4.0, 12), np.full(12, 0.0), np.full(12, 60.0)])
    p.anneal(beta, class_of=cls, target=0)
    p.compare()
    p.anneal(np.zeros((1, 0)), target=10 ** 6)
    p.compare()


def test_wide_state_resume_and_noalloc(monkeypatch):
    """A set restored with set_state and annealed on equals the uninterrupted
    run (states and energies; set_state restarts the best-energy tallies);
    the allocation-free anneal equals the plain one."""
    monkeypatch.setenv("NMC_KSAT_WIDE", "1")
    say("case: wide resume / noalloc")
    n = 250
    cp, lits = instances.gen_ksat(n, "9.6", 4, 11)
    beta = instances.linear_schedule(0.2, 3.0, 20)[None, :]
    a = KsatPair(n, cp, lits, 24, 5)
    a.anneal(beta[:, :10])
    x = a.rep.get_state()
    a.anneal(beta[:, 10:])
    a.compare()
    inst = nmc.Instance.ksat(n, cp, lits).bind()
    assert inst.info.wide == 1
    b = nmc.Replicas(inst, 24, 5)
    b.set_state(x, 10)
    assert (b.best_energy()["energy"] == b.recount()).all()
    b.anneal(beta[:, 10:])
    assert (b.get_state() == a.orep.x).all()
    assert (b.best_energy()["energy"] == a.orep.energy).all()
    q = KsatPair(n, cp, lits, 24, 5)
    q.rep.anneal_noalloc(beta)
    q.orep.anneal(beta)
    q.compare()


def test_wide_by_size_n70000():
    """N = 70,000 (above the LDS layout's 65,534): 3-SAT at alpha 4.2, 8
    replicas, a short anneal, the backbone and a short reanneal, bit-exact."""
    say("case: wide by size N=70000 R=8")
    n = 70000
    cp, lits = instances.gen_ksat(n, "4.2", 3, SEED + 3)
    p = KsatPair(n, cp, lits, 8, SEED + 4)
    assert p.inst.info.wide == 1
    p.anneal(instances.linear_schedule(0.5, 3.0, 4)[None, :], target=0)
    p.compare()
    cls = p.backbone(3, 4, expand=False)
    p.anneal(reanneal_profile(3), profile="backbone", class_of=cls)
    p.compare()


def test_wide_unsupported_calls(monkeypatch):
    """Features that keep spin tables in LDS refuse wide instances with
    NMC_ERR_UNSUPPORTED, before any work."""
    monkeypatch.setenv("NMC_KSAT_WIDE", "1")
    say("case: wide unsupported calls")
    n = 100
    cp, lits = instances.gen_ksat(n, "9.6", 4, 3)
    inst = nmc.Instance.ksat(n, cp, lits).bind()
    rep = nmc.Replicas(inst, 8, 1)
    for call in (lambda: rep.pt_run(np.array([1.0, 2.0]), 1),
                 lambda: rep.lbp_backbone(0),
                 lambda: rep.whiten(),
                 lambda: rep.cluster_flip(np.zeros(n, np.int32), 1.0),
                 lambda: nmc.Batch([rep])):
        with pytest.raises(nmc.NmcError) as e:
            call()
        assert e.value.code == -6, e.value
    assert rep.sweeps_done() == 0
