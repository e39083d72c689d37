"""GPU k-SAT path vs the CPU oracle: bit-exact states, energies, best
energies, first-hit sweeps, best-state snapshots, magnetization counts and
backbone classes."""
import numpy as np
import pytest

import oracle
from gpu_util import KsatPair, say
from paper_2111_13628_amd import instances, nmc

pytestmark = pytest.mark.gpu

SEED = instances.DEFAULT_SEED


def reanneal_profile(S, beta_hot=0.5, beta_end=4.0):
    cold = np.full(S, beta_end)
    hot = instances.linear_schedule(beta_hot, beta_end, S)
    return instances.profile_schedule(cold, hot)


def test_plain_sa_n200_r64_1000_sweeps():
    """Plain simulated annealing: random 4-SAT N=200, M=1920, 64 replicas,
    1000 sweeps with beta 0.1 -> 4.0."""
    say("case: plain SA N=200 R=64 S=1000")
    cp, lits = instances.gen_ksat(200, "9.6", 4, SEED)
    p = KsatPair(200, cp, lits, 64, SEED)
    p.anneal(instances.linear_schedule(0.1, 4.0, 1000)[None, :], target=3)
    p.compare()


@pytest.mark.parametrize("stage,block", [("0", 0), ("1", 0), ("1", 64), ("1", 256)])
def test_staged_instance_kernel(stage, block, monkeypatch):
    """Instances whose records fit in LDS beside the spin tables take the
    staged kernel (records and chunk tables copied into LDS at the start);
    NMC_KSAT_STAGE=0 keeps the streamed kernel.  Both bit-exact vs the oracle
    over an anneal and a backbone reanneal, with a partial replica group, at
    the default workgroup size and at one and four waves per workgroup."""
    monkeypatch.setenv("NMC_KSAT_STAGE", stage)
    say(f"case: staged={stage} block={block} n=150 R=22")
    n = 150
    cp, lits = instances.gen_ksat(n, "9.6", 4, SEED + 5)
    p = KsatPair(n, cp, lits, 22, SEED + 6)
    if block:
        p.rep.set_tuning(block)
    p.anneal(instances.linear_schedule(0.1, 4.0, 60)[None, :], target=2)
    p.compare()
    cls = p.backbone(9, 10, expand=True)
    p.anneal(reanneal_profile(20), profile="backbone", class_of=cls, target=1)
    p.compare()


@pytest.mark.parametrize("n,alpha,k,R,cap", [(300, "9.6", 4, 38, 0), (700, "4.15", 3, 21, 64),
                                             (2100, "9.9", 4, 12, 128), (120, "9.6", 4, 9, 1)])
def test_nmc_rounds_ragged(n, alpha, k, R, cap):
    """anneal -> backbone -> reanneal -> backbone -> reanneal, with replica
    counts that leave a partial group and several tiles per colour class;
    cap = 1 gives one variable per class (the plain index order)."""
    say(f"case: nmc rounds n={n} k={k} R={R} cap={cap}")
    cp, lits = instances.gen_ksat(n, alpha, k, SEED + n)
    p = KsatPair(n, cp, lits, R, SEED + 1, cap=cap)
    p.anneal(instances.linear_schedule(0.1, 4.0, 60)[None, :], target=2)
    p.compare()
    for rnd in range(2):
        cls = p.backbone(9, 10, expand=True)
        say(f"  round {rnd}: hot = {int(cls.sum())}")
        p.anneal(reanneal_profile(25), profile="backbone", class_of=cls, target=1)
        p.compare()


def test_host_profile_three_classes():
    say("case: host profile, 3 classes")
    n = 900
    cp, lits = instances.gen_ksat(n, "9.6", 4, 5)
    p = KsatPair(n, cp, lits, 16, 77)
    rng = np.random.Generator(np.random.PCG64(1))
    cls = rng.integers(0, 3, n).astype(np.uint8)
    beta = np.stack([instances.linear_schedule(0.1, 4.0, 30), np.full(30, 0.7), np.full(30, 9.0)])
    p.anneal(beta, class_of=cls, target=0)
    p.compare()


def test_threshold_without_expansion_and_other_ratio():
    n = 1200
    cp, lits = instances.gen_ksat(n, "9.9", 4, 8)
    p = KsatPair(n, cp, lits, 40, 3)
    p.anneal(instances.linear_schedule(0.5, 5.0, 80)[None, :])
    p.backbone(4, 5, expand=False)
    p.backbone(1, 1, expand=True)
    p.backbone(9, 10, expand=True)


def test_chunked_calls_equal_one_call_and_block_shapes():
    say("case: chunking and block shapes")
    n = 1500
    cp, lits = instances.gen_ksat(n, "9.9", 4, 12)
    beta = instances.linear_schedule(0.1, 4.0, 48)[None, :]
    ref = KsatPair(n, cp, lits, 24, 9)
    ref.anneal(beta, target=5)
    ref.compare()
    for bt in (64, 256, 512):
        inst = nmc.Instance.ksat(n, cp, lits).bind()
        rep = nmc.Replicas(inst, 24, 9)
        rep.set_tuning(bt)
        for s in range(0, 48, 7):
            rep.anneal(beta[:, s:s + 7], target=5)
        assert (rep.get_state() == ref.orep.x).all(), bt
        be = rep.best_energy()
        assert (be["best_per_replica"] == ref.orep.best).all()
        assert (be["first_hit"] == ref.orep.first_hit).all()


def test_edge_cases():
    say("case: edge cases")
    # one variable, no clauses: every move has dE = 0 and is taken
    p = KsatPair(1, np.array([0], np.int32), np.zeros(0, np.int32), 5, 1)
    p.anneal(np.full((1, 3), 1.0))
    p.compare()
    assert (p.orep.x == (p.orep.x * 0 + (p.oinst.init(5, 1) ^ 1))).all()
    # unit clauses and mixed clause lengths, one replica
    cp = np.array([0, 1, 3, 6, 10, 11], np.int32)
    lits = np.array([1, -1, 2, 3, -4, 5, -2, 4, -5, 6, -6], np.int32)
    p = KsatPair(6, cp, lits, 1, 4)
    p.anneal(instances.linear_schedule(0.1, 3.0, 20)[None, :], target=1)
    p.compare()
    # zero-sweep call records a hit at the call's start when the target is easy
    cp2, lits2 = instances.gen_ksat(100, "9.6", 4, 2)
    p = KsatPair(100, cp2, lits2, 7, 2)
    p.anneal(np.zeros((1, 0)), target=10**6)
    p.compare()
    assert (p.orep.first_hit == 0).all()
    # beta = 0 flips everything (all-accept table), huge beta never rises
    p = KsatPair(100, cp2, lits2, 9, 3)
    p.anneal(np.zeros((1, 2)))
    p.anneal(np.full((1, 5), 60.0))
    p.compare()


def test_largest_instance_and_no_clauses():
    """N = 65534, the largest spin table the LDS holds (2N + 2 bytes of 160 KB),
    and an instance without clauses (every move has dE = 0)."""
    say("case: N = 65534, 5 replicas")
    n = 65534
    cp, lits = instances.gen_ksat(n, "9.9", 4, SEED + 7)
    p = KsatPair(n, cp, lits, 5, SEED + 8, cap=1024)
    p.anneal(instances.linear_schedule(0.1, 4.0, 100)[None, :2], target=0)
    p.compare()
    cls = p.backbone(9, 10, True)
    p.anneal(reanneal_profile(2), profile="backbone", class_of=cls)
    p.compare()
    say("case: 300 variables, no clauses")
    p = KsatPair(300, np.zeros(1, np.int32), np.zeros(0, np.int32), 11, 5)
    p.anneal(np.full((1, 3), 2.0), target=0)
    p.compare()
    assert (p.orep.energy == 0).all() and (p.orep.first_hit == 0).all()


def test_set_state_resume_matches_continuation():
    n = 800
    cp, lits = instances.gen_ksat(n, "9.9", 4, 4)
    beta = instances.linear_schedule(0.1, 4.0, 40)[None, :]
    a = KsatPair(n, cp, lits, 20, 6)
    a.anneal(beta[:, :20])
    x = a.rep.get_state()
    a.anneal(beta[:, 20:])
    inst = nmc.Instance.ksat(n, cp, lits).bind()
    b = nmc.Replicas(inst, 20, 6)
    b.set_state(x, 20)
    assert (b.best_energy()["energy"] == b.recount()).all()
    b.anneal(beta[:, 20:])
    assert (b.get_state() == a.orep.x).all()
    assert (b.best_energy()["energy"] == a.orep.energy).all()


def test_full_size_n50000_r1024_short_schedule():
    """The benchmark's instance and launch configuration (N=50,000, M=495,000,
    1024 replicas, colour-class cap 1024) on the first sweeps of the anneal,
    the backbone estimate and the first reanneal sweep, bit-exact on every
    replica."""
    say("case: full size N=50000 R=1024 (2 anneal sweeps, backbone, 1 reanneal sweep)")
    n = 50000
    cp, lits = instances.gen_ksat(n, "9.9", 4, SEED)
    p = KsatPair(n, cp, lits, 1024, SEED, cap=1024)
    p.anneal(instances.linear_schedule(0.1, 4.0, 2000)[None, :2], target=0)
    say("  anneal done")
    p.compare(check_best_state=False)
    cls = p.backbone(9, 10, expand=True)
    say(f"  backbone hot = {int(cls.sum())}")
    p.anneal(reanneal_profile(1000)[:, :1], profile="backbone", class_of=cls)
    p.compare()


def test_layout_schedule_does_not_change_results(monkeypatch):
    """The bank-aware record placement only reorders additions: states and
    energies are identical with and without it."""
    n = 3000
    cp, lits = instances.gen_ksat(n, "9.9", 4, 31)
    beta = instances.linear_schedule(0.1, 4.0, 30)[None, :]
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("NMC_KSAT_BANK_SCHEDULE", flag)
        inst = nmc.Instance.ksat(n, cp, lits, 256).bind()
        rep = nmc.Replicas(inst, 36, 5)
        rep.anneal(beta, target=3)
        out.append((rep.get_state(), rep.best_energy()))
    assert (out[0][0] == out[1][0]).all()
    for key in ("energy", "best_per_replica", "first_hit"):
        assert (out[0][1][key] == out[1][1][key]).all()


@pytest.mark.parametrize("n,cap,R", [(200, 0, 64), (900, 16, 21), (300, 1, 8)])
def test_split_lanes_do_not_change_results(monkeypatch, n, cap, R):
    """Chunks of small colour classes spread each variable's clauses over
    several lanes (NMC_KSAT_SPLIT=0 keeps one lane per variable): the partial
    sums only regroup integer additions, so states, energies, snapshots,
    backbones and whitening are identical, and both equal the oracle."""
    say(f"case: split lanes n={n} cap={cap} R={R}")
    cp, lits = instances.gen_ksat(n, "9.6", 4, 41 + n)
    beta = instances.linear_schedule(0.1, 4.0, 40)[None, :]
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("NMC_KSAT_SPLIT", flag)
        p = KsatPair(n, cp, lits, R, 6, cap=cap)
        p.anneal(beta, target=5)
        cls = p.backbone(9, 10, True)
        p.anneal(reanneal_profile(15), class_of=cls, profile="backbone", target=5)
        p.compare()
        out.append((p.rep.get_state(), p.rep.get_state("best"), p.rep.whiten("best", white=True)))
    assert (out[0][0] == out[1][0]).all() and (out[0][1] == out[1][1]).all()
    w0, w1 = out[0][2], out[1][2]
    assert (w0[0] == w1[0]).all() and (w0[1] == w1[1]).all()


def test_accept_count_equals_flipped_spins():
    """Every variable is visited once per sweep, so the flips a sweep accepts
    are exactly the spins that differ before and after it; the counter of
    accepted moves must equal that Hamming distance, sweep by sweep, over a
    schedule from hot (mostly accepted) to cold."""
    say("case: accepted-move counter, k-SAT")
    n, R = 700, 37
    cp, lits = instances.gen_ksat(n, "9.6", 4, 91)
    rep = nmc.Replicas(nmc.Instance.ksat(n, cp, lits).bind(), R, 92)
    assert rep.accept_count() == 0
    betas = instances.linear_schedule(0.05, 5.0, 12)
    total = 0
    for b in betas:
        x0 = rep.get_state()
        rep.anneal(np.array([[b]]))
        flips = int((rep.get_state() != x0).sum())
        got = rep.accept_count(reset=True)
        assert got == flips, (b, got, flips)
        total += got
    assert total > 0 and rep.accept_count() == 0
    # a multi-sweep call counts its sweeps together
    rep.anneal(np.full((1, 5), 0.3))
    assert rep.accept_count() > 0


@pytest.mark.parametrize("n,alpha,k,R,cap", [(300, "9.6", 4, 37, 0), (1200, "4.15", 3, 6, 64), (500, "9.6", 4, 4, 0),
                                             (2000, "9.9", 4, 64, 0), (160, "9.6", 4, 24, 1), (4096, "9.9", 4, 40, 0)])
def test_eight_replicas_per_workgroup_matches_oracle(n, alpha, k, R, cap):
    """Sweep workgroups of 8 replicas (two groups sharing each spin byte in
    LDS), with ragged and single-group replica counts, split and unsplit
    chunks: anneal, backbone and reanneal bit-exact with the oracle."""
    say(f"case: 8 replicas per workgroup n={n} k={k} R={R} cap={cap}")
    cp, lits = instances.gen_ksat(n, alpha, k, SEED + 3 * n)
    p = KsatPair(n, cp, lits, R, SEED + 4, cap=cap)
    p.rep.set_replicas_per_workgroup(8)
    p.anneal(instances.linear_schedule(0.1, 4.0, 30)[None, :], target=3)
    p.compare()
    cls = p.backbone(9, 10, True)
    p.anneal(reanneal_profile(12), class_of=cls, profile="backbone", target=1)
    p.compare()
    rng = np.random.Generator(np.random.PCG64(n))
    host = rng.integers(0, 3, n).astype(np.uint8)
    beta3 = np.stack([np.full(5, 3.0), np.full(5, 0.7), np.full(5, 1.9)])
    p.anneal(beta3, class_of=host)
    p.compare()


def test_eight_replicas_per_workgroup_full_size():
    """N = 50,000, 2048 replicas: 8 replicas per workgroup equals 4 per
    workgroup bit for bit on every replica, and the first and last groups
    equal the oracle; the single-set tuner's choice changes nothing."""
    say("case: 8 replicas per workgroup, N=50000 R=2048")
    n, R = 50000, 2048
    cp, lits = instances.gen_ksat(n, "9.9", 4, SEED)
    inst = nmc.Instance.ksat(n, cp, lits, 1024).bind()
    beta = instances.linear_schedule(0.1, 4.0, 2000)[None, :3]
    a = nmc.Replicas(inst, R, SEED + 9)
    b = nmc.Replicas(inst, R, SEED + 9)
    c = nmc.Replicas(inst, R, SEED + 9)
    b.set_replicas_per_workgroup(8)
    blk, rpw = c.tune(2)
    assert blk in (64, 128, 256, 512, 1024) and rpw in (4, 8)
    for rep in (a, b, c):
        rep.anneal(beta, target=10000)
    for other in (b, c):
        assert (a.get_state() == other.get_state()).all()
        assert (a.get_state("best") == other.get_state("best")).all()
        ea, eo = a.best_energy(), other.best_energy()
        for key in ("energy", "best_per_replica", "first_hit"):
            assert (ea[key] == eo[key]).all(), key
    ok = oracle.KSat(n, cp, lits)
    _, order, _ = ok.color(1024)
    orep = oracle.KSatReplicas(ok, R, SEED + 9, order, threads=16)
    for lo, hi in ((0, 8), (R - 8, R)):
        orep.anneal(beta, target=10000, r_begin=lo, r_end=hi)
        orep.sweeps_done -= beta.shape[1]
    x = b.get_state()
    be = b.best_energy()
    for lo, hi in ((0, 8), (R - 8, R)):
        assert (x[lo:hi] == orep.x[lo:hi]).all()
        assert (be["energy"][lo:hi] == orep.energy[lo:hi]).all()
        assert (be["first_hit"][lo:hi] == orep.first_hit[lo:hi]).all()
