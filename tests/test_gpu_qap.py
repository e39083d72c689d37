"""GPU QAP path vs the CPU oracle: bit-exact permutations, costs, best costs,
first hits, best permutations, assignment frequencies and backbone classes."""
import numpy as np
import pytest

from gpu_util import QapPair, say
from paper_2111_13628_amd import instances, nmc

pytestmark = pytest.mark.gpu

SEED = instances.DEFAULT_SEED


def beta_scale(F, D, seed=1, samples=2000):
    """1 / median positive swap change on random assignments (schedule units)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = F.shape[0]
    F = F.astype(np.int64)
    D = D.astype(np.int64)
    vals = []
    for _ in range(samples):
        p = rng.permutation(n)
        a, b = rng.choice(n, 2, replace=False)
        k = np.array([i for i in range(n) if i not in (a, b)])
        d = 2 * int(((F[a, k] - F[b, k]) * (D[p[b], p[k]] - D[p[a], p[k]])).sum())
        if d > 0:
            vals.append(d)
    return 1.0 / float(np.median(vals))


def reanneal_profile(S, scale, beta_hot=0.5, beta_end=4.0):
    return instances.profile_schedule(np.full(S, beta_end * scale),
                                      instances.linear_schedule(beta_hot * scale, beta_end * scale, S))


@pytest.mark.parametrize("n,R", [(12, 20), (37, 45), (64, 16)])
def test_qap_nmc_rounds(n, R):
    say(f"case: qap n={n} R={R}")
    F, D = instances.gen_qap(n, SEED + n)
    sc = beta_scale(F, D)
    p = QapPair(F, D, R, SEED + 1)
    p.anneal(instances.linear_schedule(0.1 * sc, 4.0 * sc, 20)[None, :], target=0)
    p.compare()
    cls = p.backbone(9, 10)
    p.anneal(reanneal_profile(8, sc), profile="backbone", class_of=cls)
    p.compare()
    cls = p.backbone(1, 2)
    p.anneal(reanneal_profile(5, sc), profile="backbone", class_of=cls, target=int(p.orep.best.min()))
    p.compare()


def test_qap_edges_and_host_profile():
    say("case: qap edges")
    for n in (2, 3):
        F, D = instances.gen_qap(n, 3)
        p = QapPair(F, D, 6, 2)
        p.anneal(np.full((1, 4), 0.01))
        p.compare()
    F, D = instances.gen_qap(20, 4)
    sc = beta_scale(F, D)
    p = QapPair(F, D, 9, 5)
    cls = (np.arange(20) % 3).astype(np.uint8)
    beta = np.stack([np.full(6, 3.0 * sc), np.full(6, 0.3 * sc), np.zeros(6)])
    p.anneal(beta, class_of=cls)
    p.compare()
    p.anneal(np.zeros((1, 0)), target=10**12)
    p.compare()


def test_qap_full_size_n100_r4096_short_schedule():
    """The QAP benchmark's size: n = 100, 4096 replicas, on the first anneal
    sweeps, the frequency backbone and the first reanneal sweep."""
    say("case: qap full size n=100 R=4096")
    F, D = instances.gen_qap(100, SEED)
    sc = beta_scale(F, D)
    p = QapPair(F, D, 4096, SEED)
    p.anneal(instances.linear_schedule(0.1 * sc, 4.0 * sc, 5000)[None, :2])
    say("  anneal done")
    p.compare()
    cls = p.backbone(9, 10)
    p.anneal(reanneal_profile(1000, sc)[:, :1], profile="backbone", class_of=cls)
    p.compare()


@pytest.mark.parametrize("rows", ["1", "4", "8", "2", "3", "0"])
def test_qap_every_step_width_matches_oracle(rows, monkeypatch):
    """The number of proposals a wave evaluates per step (pinned to 1, 4 or 8,
    to the table mode (2), to four replicas per wave (3, whole workgroups of
    16 replicas only), or chosen per sweep from the acceptance rate) never
    changes the result: sizes on each side of the width limits, and a
    schedule that crosses from mostly-accepted to mostly-rejected sweeps
    inside one call."""
    monkeypatch.setenv("NMC_QAP_ROWS", rows)
    for n, R in ((45, 9), (100, 6), (130, 5), (7, 4), (10, 3), (64, 32), (100, 16), (150, 48), (23, 16)):
        say(f"case: qap width={rows} n={n} R={R}")
        F, D = instances.gen_qap(n, SEED + 3 * n)
        sc = beta_scale(F, D)
        p = QapPair(F, D, R, SEED + n)
        p.anneal(np.geomspace(0.05 * sc, 8.0 * sc, 10)[None, :], target=0)
        p.compare()
        cls = p.backbone(2, 3)
        p.anneal(reanneal_profile(4, sc), profile="backbone", class_of=cls)
        p.compare()


def test_qap_largest_n255():
    """n = 255, the largest permutation a byte holds.  With entries up to 99
    one threshold table fits next to F and D in LDS but two do not: the
    backbone profile must then fail cleanly with NMC_ERR_CAPACITY."""
    say("case: qap n=255")
    F, D = instances.gen_qap(255, SEED + 255)
    sc = beta_scale(F, D, samples=300)
    p = QapPair(F, D, 3, SEED)
    p.anneal(np.full((1, 2), 2.0 * sc), target=0)
    p.compare()
    cls = p.backbone(1, 3)
    try:
        p.rep.reanneal(reanneal_profile(1, sc), "backbone")
    except nmc.NmcError as e:
        assert e.code == -5, e
        return
    p.orep.anneal(reanneal_profile(1, sc), class_of=cls)
    p.compare()


def test_accept_count_qap():
    """At beta = 0 every proposal is accepted (threshold 2^32 - 1, which only a
    word of 2^32 - 1 fails), so a sweep counts every pair of every replica; at
    a very large beta only non-increasing swaps are taken and the count never
    exceeds the proposals."""
    say("case: accepted-move counter, QAP")
    n, R = 30, 20
    F, D = instances.gen_qap(n, 93)
    rep = nmc.Replicas(nmc.Instance.qap(F, D).bind(), R, 94)
    rep.anneal(np.zeros((1, 3)))
    assert rep.accept_count(reset=True) == 3 * R * n * (n - 1) // 2
    rep.anneal(np.full((1, 4), 60.0))
    cold = rep.accept_count(reset=True)
    assert 0 <= cold < 4 * R * n * (n - 1) // 2
    rep.anneal(np.full((1, 4), 1e-4))
    assert rep.accept_count() > cold


@pytest.mark.parametrize("n,R", [(31, 17), (100, 20), (150, 6)])
def test_qap_table_mode_switches_match_oracle(n, R, monkeypatch):
    """The per-sweep choice enters the table mode once a sweep accepts fewer
    than 1/128 of the proposals and enough sweeps remain, keeps its table
    across sweeps, leaves it when the acceptance rises again (a hot reanneal
    class) and re-enters later; every launch and mode switch stays bit-exact
    with the oracle, including the best-state snapshots and first hits."""
    say(f"case: qap table-mode switches n={n} R={R}")
    monkeypatch.setenv("NMC_QAP_TAB", "1")  # off by default (slower on MI355X)
    F, D = instances.gen_qap(n, SEED + 7 * n)
    sc = beta_scale(F, D)
    p = QapPair(F, D, R, SEED + 2 * n)
    sched = np.concatenate([np.geomspace(0.05, 6.0, 12), np.full(20, 6.0), np.full(6, 0.3), np.full(14, 8.0)])
    p.anneal(sched[None, :] * sc, target=0)
    p.compare()
    first = int(p.orep.best.min())
    cls = p.backbone(1, 2)
    p.anneal(reanneal_profile(16, sc, beta_hot=0.2, beta_end=7.0), profile="backbone", class_of=cls, target=first)
    p.compare()
    # a one-sweep launch after table-mode sweeps takes another width
    p.anneal(np.full((1, 1), 7.0 * sc))
    p.compare()
    p.anneal(np.full((1, 12), 7.0 * sc))
    p.compare()
    acc = p.rep.accept_count()
    assert 0 < acc < R * n * (n - 1) // 2 * 90


@pytest.mark.parametrize("n,R,rpw", [(40, 32, "2"), (100, 48, "2"), (100, 48, "4"), (130, 16, "2"), (20, 32, "4")])
def test_qap_multi_replica_waves_match_oracle(n, R, rpw, monkeypatch):
    """Two or four replicas per wave, chosen per sweep for whole workgroups
    of hot replicas (NMC_QAP_RPW), switching to one replica per wave as the
    schedule cools and back for a hot reanneal: bit-exact with the oracle."""
    say(f"case: qap {rpw} replicas per wave n={n} R={R}")
    monkeypatch.setenv("NMC_QAP_RPW", rpw)
    F, D = instances.gen_qap(n, SEED + 5 * n)
    sc = beta_scale(F, D)
    p = QapPair(F, D, R, SEED + 3 * n)
    sched = np.concatenate([np.full(4, 0.05), np.geomspace(0.05, 5.0, 10), np.full(3, 0.1), np.full(3, 5.0)])
    p.anneal(sched[None, :] * sc, target=0)
    p.compare()
    cls = p.backbone(1, 2)
    p.anneal(reanneal_profile(6, sc, beta_hot=0.05, beta_end=0.2), profile="backbone", class_of=cls)
    p.compare()


@pytest.mark.parametrize("rows", ["1", "8", "0"])
def test_qap_acceptance_bound_extremes(rows, monkeypatch):
    """The sweeps accept a proposal when its change is below the acceptance
    bound d*(u) of its random word, found by a search that starts from a
    float guess: exact whatever the guess.  Schedules at beta = 0 (every
    threshold 2^32 - 1; the guess is the end of the table), very small and
    very large beta (the guess far from most words' bounds) and two classes
    of different beta in one sweep stay bit-exact with the oracle, which reads
    the thresholds directly."""
    monkeypatch.setenv("NMC_QAP_ROWS", rows)
    F, D = instances.gen_qap(41, SEED + 41)
    sc = beta_scale(F, D)
    for R, betas in ((7, [0.0, 0.0]), (9, [1e-7 * sc, 1e-4 * sc, 3e-3 * sc]), (6, [50.0 * sc, 1e3 * sc, 1e6 * sc]),
                     (16, [0.02 * sc, 0.5 * sc, 2.0 * sc, 12.0 * sc])):
        say(f"case: qap acceptance bound rows={rows} R={R} betas={betas}")
        p = QapPair(F, D, R, SEED + R)
        p.anneal(np.array(betas)[None, :], target=0)
        p.compare()
    p = QapPair(F, D, 12, SEED + 3)
    p.anneal(np.geomspace(0.1 * sc, 4.0 * sc, 6)[None, :])
    cls = (np.arange(41) % 4 == 1).astype(np.uint8)
    beta = np.stack([np.full(5, 6.0 * sc), np.array([0.0, 1e-6, 0.3, 1.0, 30.0]) * sc])
    p.anneal(beta, class_of=cls)
    p.compare()


def test_qap_direct_threshold_reads_match_oracle(monkeypatch):
    """NMC_QAP_DSTAR=0: every proposal reads its two threshold words (the path
    the library takes when a table row's T is not monotone, which the host
    checks per row); the per-sweep width choice then never takes the
    one-proposal path.  Bit-exact with the oracle at the full-size shape's
    width limits and with two classes."""
    monkeypatch.setenv("NMC_QAP_DSTAR", "0")
    for n, R in ((45, 9), (100, 16)):
        say(f"case: qap direct thresholds n={n} R={R}")
        F, D = instances.gen_qap(n, SEED + 11 * n)
        sc = beta_scale(F, D)
        p = QapPair(F, D, R, SEED + n)
        p.anneal(np.geomspace(0.05 * sc, 8.0 * sc, 10)[None, :], target=0)
        p.compare()
        cls = p.backbone(2, 3)
        p.anneal(reanneal_profile(4, sc), profile="backbone", class_of=cls)
        p.compare()
