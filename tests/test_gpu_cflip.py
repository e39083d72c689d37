"""Collective cluster flips on the GPU against the CPU oracle, bit for bit:
states, energies, best energies and snapshots, first hits and flips per
replica, for clusters from the oracle's own LBP backbone and for seeded
synthetic clusters, hot, warm and cold, interleaved with sweeps; and sampled
replicas at N = 50,000."""
import numpy as np
import pytest

from gpu_util import KsatPair, say, threads
from paper_2111_13628_amd import instances, nmc

pytestmark = pytest.mark.gpu


def _random_labels(n, n_clusters, lo, hi, seed):
    """Disjoint clusters of lo..hi variables, each named by its smallest."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lab = np.full(n, -1, np.int32)
    free = rng.permutation(n)
    pos = 0
    for _ in range(n_clusters):
        k = int(rng.integers(lo, hi + 1))
        if pos + k > n:
            break
        vs = free[pos:pos + k]
        pos += k
        lab[vs] = vs.min()
    return lab


def _flip(pair, lab, beta, target=-1):
    acc = pair.rep.cluster_flip(lab, beta, target)
    oacc = pair.orep.cluster_flip(lab, beta, target)
    assert (acc == oacc).all(), (acc, oacc)
    return acc


@pytest.mark.parametrize("n,alpha,k,R,seed", [(400, "9.6", 4, 12, 1), (301, "4.2", 3, 10, 2), (1000, "9.7", 4, 8, 3)])
def test_cluster_flips_match_oracle(n, alpha, k, R, seed):
    say(f"case: cluster flips n={n} R={R}")
    cp, lits = instances.gen_ksat(n, alpha, k, seed)
    pair = KsatPair(n, cp, lits, R, 50 + seed)
    lab = _random_labels(n, 25, 1, 12, seed)
    pair.anneal(instances.linear_schedule(0.3, 2.0, 20)[None, :])
    a0 = _flip(pair, lab, 0.0)
    assert (a0 == len(np.unique(lab[lab >= 0]))).all()
    pair.anneal(np.full((1, 10), 2.5))
    a1 = _flip(pair, lab, 1.5, int(np.median(pair.orep.energy)))
    pair.anneal(np.full((1, 10), 4.0))
    _flip(pair, lab, 60.0)
    say(f"  flips at beta 1.5: {a1.tolist()}")
    pair.compare()


def test_cluster_flips_of_an_lbp_backbone():
    """Clusters from the oracle's LBP backbone around a replica's best state
    (the move the NMC scheme builds from them), then sweeps."""
    say("case: cluster flips of LBP clusters")
    cp, lits = instances.gen_ksat(600, "9.6", 4, 6)
    pair = KsatPair(600, cp, lits, 16, 8)
    pair.anneal(instances.linear_schedule(0.2, 3.0, 60)[None, :])
    o = pair.oinst.lbp(pair.orep.best_x[3], 1.0, 4.0, 0.8, 0.02, 200, 1e-10)
    label, cls, nc = pair.oinst.clusters(o["corr"], 0.95, 0.9)
    assert nc > 0
    for beta in (0.5, 2.0):
        _flip(pair, label, beta)
        pair.anneal(np.full((1, 5), 3.0))
    pair.compare()


def test_full_size_cluster_flips_sampled_replicas():
    """N = 50,000, 1024 replicas, 200 synthetic clusters: replicas 6 and 7,
    followed by the oracle alone through 40 sweeps and one collective sweep,
    match bit for bit."""
    import oracle
    N, R = 50000, 1024
    say("case: cluster flips at N = 50,000, replicas 6 and 7")
    cp, lits = instances.gen_ksat(N, "9.9", 4, instances.DEFAULT_SEED)
    inst = nmc.Instance.ksat(N, cp, lits, 1024).bind()
    rep = nmc.Replicas(inst, R, 4)
    lab = _random_labels(N, 200, 5, 50, 9)
    beta = instances.linear_schedule(0.5, 3.0, 40)[None, :]
    rep.anneal(beta)
    acc = rep.cluster_flip(lab, 2.0)
    be = rep.best_energy()
    assert (rep.recount() == be["energy"]).all()
    ok = oracle.KSat(N, cp, lits)
    _, order, _ = ok.color(1024)
    orep = oracle.KSatReplicas(ok, R, 4, order, threads=threads())
    orep.threads = 2
    orep.anneal(beta, r_begin=6, r_end=8)
    oacc = orep.cluster_flip(lab, 2.0, r_begin=6, r_end=8)
    x = rep.get_state()
    for r in (6, 7):
        assert acc[r] == oacc[r]
        assert (x[r] == orep.x[r]).all() and be["energy"][r] == orep.energy[r]
        assert be["best_per_replica"][r] == orep.best[r]


def test_cluster_flip_errors():
    say("case: cluster flip argument errors")
    cp, lits = instances.gen_ksat(50, "4.2", 3, 1)
    rep = nmc.Replicas(nmc.Instance.ksat(50, cp, lits).bind(), 8, 1)
    bad = np.full(50, -1, np.int32)
    bad[3] = 4  # names a variable that does not label itself
    with pytest.raises(nmc.NmcError):
        rep.cluster_flip(bad, 1.0)
    with pytest.raises(nmc.NmcError):
        rep.cluster_flip(np.full(50, -1, np.int32), -1.0)
    assert rep.sweeps_done() == 0
    assert (rep.cluster_flip(np.full(50, -1, np.int32), 1.0) == 0).all() and rep.sweeps_done() == 1
    F, D = instances.gen_qap(8, 1)
    q = nmc.Replicas(nmc.Instance.qap(F, D).bind(), 16, 1)
    with pytest.raises(nmc.NmcError):
        q.cluster_flip(np.full(8, -1, np.int32), 1.0)
