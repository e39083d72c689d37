"""Parallel tempering on the GPU (appendix A) against the CPU oracle, bit for
bit: replica-exchange rounds (states, energies, best energies and snapshots,
first hits, exchange counts) and the adaptive ladder (every beta and sigma),
for k-SAT and QAP, over ragged sizes, both parities and every spin-row width
the exchange kernel distinguishes; plus the layout and ladder errors."""
import numpy as np
import pytest

from gpu_util import KsatPair, QapPair, say
from paper_2111_13628_amd import instances, nmc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,alpha,k,M,C,seed,step", [
    (301, "9.6", 4, 5, 8, 1, 0.3),     # N % 4 != 0: byte rows
    (1000, "4.2", 3, 4, 12, 2, 0.1),   # N % 4 == 0, N % 16 != 0: word rows
    (2048, "9.7", 4, 3, 4, 3, 0.03),   # N % 16 == 0: 16-byte rows
    (700, "9.6", 4, 7, 4, 4, 0.15),    # odd ladder length
])
def test_ksat_tempering_matches_oracle(n, alpha, k, M, C, seed, step):
    say(f"case: k-SAT tempering n={n} M={M} C={C}")
    cp, lits = instances.gen_ksat(n, alpha, k, seed)
    pair = KsatPair(n, cp, lits, M * C, 40 + seed)
    beta = 1.0 + step * np.arange(M)
    pair.anneal(np.linspace(0.1, 1.0, 6)[None, :])
    acc, att = pair.pt_run(beta, 7, 1, 0)
    assert att.sum() > 0 and acc.sum() > 0
    target = int(np.median(pair.orep.energy))
    pair.pt_run(beta, 4, 3, 1, target)
    pair.compare()


def test_ksat_tempering_with_one_temperature_is_annealing():
    say("case: k-SAT tempering with one ladder position")
    cp, lits = instances.gen_ksat(500, "9.6", 4, 9)
    a = KsatPair(500, cp, lits, 16, 5)
    acc, att = a.pt_run(np.array([1.3]), 5, 2)
    assert acc.size == 0 and att.size == 0
    a.compare()
    b = nmc.Replicas(a.inst, 16, 5)
    b.anneal(np.full((1, 10), 1.3))
    assert (b.get_state() == a.rep.get_state()).all()


@pytest.mark.parametrize("n,M,C,seed,rows", [(19, 3, 16, 1, "0"), (45, 4, 16, 2, "0"), (33, 2, 32, 3, "1"),
                                             (120, 3, 16, 4, "4")])
def test_qap_tempering_matches_oracle(n, M, C, seed, rows, monkeypatch):
    say(f"case: QAP tempering n={n} M={M} C={C} rows={rows}")
    monkeypatch.setenv("NMC_QAP_ROWS", rows)
    F, D = instances.gen_qap(n, seed)
    pair = QapPair(F, D, M * C, 60 + seed)
    beta = np.geomspace(2e-4, 3e-3, M)
    acc, att = pair.pt_run(beta, 6, 1, 1)
    assert att.sum() > 0
    pair.pt_run(beta, 3, 2, 0, int(np.median(pair.orep.cost)))
    pair.compare()


def test_qap_tempering_wide_tables_match_oracle():
    """n = 160 with entries up to 255: one threshold row is 84 KB, so four
    temperatures' rows do not fit one workgroup's LDS and the sweep keeps
    the block-per-temperature mapping; the result is the same."""
    say("case: QAP tempering n=160, entries to 255")
    n = 160
    rng = np.random.default_rng(21)
    F = rng.integers(0, 256, (n, n), dtype=np.int32)
    D = rng.integers(0, 256, (n, n), dtype=np.int32)
    F = np.triu(F, 1) + np.triu(F, 1).T
    D = np.triu(D, 1) + np.triu(D, 1).T
    pair = QapPair(F, D, 32, 22)
    beta = np.array([2e-6, 5e-6])
    pair.pt_run(beta, 3, 1, 0)
    pair.compare()


def test_ksat_adaptive_ladder_matches_oracle():
    say("case: k-SAT adaptive ladder")
    cp, lits = instances.gen_ksat(600, "9.6", 4, 12)
    pair = KsatPair(600, cp, lits, 64, 13)
    b, sg = pair.apt_ladder(0.2, 1.1, 3.0, 4, 3, 9)
    assert len(b) >= 3
    pair.compare()
    # then temper on the first positions of the ladder found
    M = 4 if len(b) >= 4 else 2
    pair.pt_run(b[:M], 5, 1)
    pair.compare()


def test_qap_adaptive_ladder_and_tempering_match_oracle():
    say("case: QAP adaptive ladder")
    F, D = instances.gen_qap(23, 7)
    pair = QapPair(F, D, 64, 14)
    b, sg = pair.apt_ladder(1e-4, 1.1, 300.0, 3, 2, 4)
    assert len(b) >= 2
    pair.compare()
    M = 4 if len(b) >= 4 else 2
    pair.pt_run(b[:M], 4, 1)
    pair.compare()


def test_disjoint_clause_ladder_follows_closed_form():
    """At full replica count the device ladder's sigma follows the binomial
    closed form of a formula with disjoint clauses (property check at a size
    the oracle is not run on)."""
    say("case: disjoint-clause ladder, 4096 replicas")
    M, k = 2000, 3
    cp, lits = instances.gen_ksat_disjoint(M, k, 2)
    inst = nmc.Instance.ksat(M * k, cp, lits).bind()
    rep = nmc.Replicas(inst, 4096, 3)
    b, sg = rep.apt_ladder(0.5, 1.1, 8.0, 100, 4, 16)
    for beta, s in zip(b, sg):
        w = np.exp(-beta)
        p = w / (w + 2**k - 1)
        assert s == pytest.approx(np.sqrt(M * p * (1 - p)), rel=0.04), beta
    assert (rep.recount() == rep.best_energy()["energy"]).all()


def test_layout_and_ladder_errors():
    say("case: tempering argument errors")
    cp, lits = instances.gen_ksat(200, "9.6", 4, 1)
    inst = nmc.Instance.ksat(200, cp, lits).bind()
    rep = nmc.Replicas(inst, 24, 1)
    with pytest.raises(nmc.NmcError):
        rep.pt_run(np.linspace(1, 2, 5), 1)          # 24 replicas on 5 positions
    with pytest.raises(nmc.NmcError):
        rep.pt_run(np.linspace(1, 2, 4), 1)          # 6 chains: not a multiple of 4
    with pytest.raises(nmc.NmcError):
        rep.pt_run(np.array([1.0, 1.0, 2.0]), 1)     # not strictly increasing
    with pytest.raises(nmc.NmcError):
        rep.pt_run(np.array([1.0, 2.0]), 1, 0)       # no sweeps per round
    with pytest.raises(nmc.NmcError):
        rep.apt_ladder(0.1, 0.0)                     # alpha must be positive
    with pytest.raises(nmc.NmcError):
        rep.apt_ladder(0.1, 1.1, -1.0)               # sigma_min must be >= 0
    assert rep.sweeps_done() == 0
    F, D = instances.gen_qap(12, 1)
    q = nmc.Replicas(nmc.Instance.qap(F, D).bind(), 32, 1)
    with pytest.raises(nmc.NmcError):
        q.pt_run(np.array([1e-3, 2e-3, 3e-3, 4e-3]), 1)  # 8 chains: not a multiple of 16
    acc, att = q.pt_run(np.array([1e-3, 2e-3]), 0)
    assert att.tolist() == [0] and q.sweeps_done() == 0


def _slots(M, C, chains):
    return [i * C + c for i in range(M) for c in range(*chains)]


def test_full_size_ksat_tempering_sampled_chains():
    """N = 50,000, alpha = 9.9, 1024 replicas as 64 temperatures x 16 chains
    (the benchmark's launch shape): chains 3 and 4, followed by the oracle
    alone, match the GPU's slots bit for bit; every slot's tracked energy
    equals a recount."""
    from gpu_util import threads
    import oracle
    N, R, M, C = 50000, 1024, 64, 16
    say("case: full-size k-SAT tempering, sampled chains")
    cp, lits = instances.gen_ksat(N, "9.9", 4, instances.DEFAULT_SEED)
    inst = nmc.Instance.ksat(N, cp, lits, 1024).bind()
    rep = nmc.Replicas(inst, R, 5)
    beta = np.linspace(1.5, 2.5, M)
    target = 30000
    acc, att = rep.pt_run(beta, 6, 1, 0, target)
    assert att.tolist() == [3 * C] * (M - 1)
    assert acc.sum() > 0
    be = rep.best_energy()
    assert (rep.recount() == be["energy"]).all()
    ok = oracle.KSat(N, cp, lits)
    _, order, _ = ok.color(1024)
    orep = oracle.KSatReplicas(ok, R, 5, order, threads=threads())
    say("  oracle following chains 3, 4")
    orep.pt_run(beta, 6, 1, 0, target, chains=(3, 5))
    sl = _slots(M, C, (3, 5))
    assert (rep.get_state()[sl] == orep.x[sl]).all()
    assert (rep.get_state("best")[sl] == orep.best_x[sl]).all()
    assert (be["energy"][sl] == orep.energy[sl]).all()
    assert (be["best_per_replica"][sl] == orep.best[sl]).all()
    assert (be["first_hit"][sl] == orep.first_hit[sl]).all()


def test_full_size_qap_tempering_sampled_chains():
    """n = 100, 4096 replicas as 64 temperatures x 64 chains: chains 16..31
    (one sweep workgroup's worth) followed by the oracle match bit for bit."""
    from gpu_util import threads
    import oracle
    n, R, M, C = 100, 4096, 64, 64
    say("case: full-size QAP tempering, sampled chains")
    F, D = instances.gen_qap(n, instances.DEFAULT_SEED)
    rep = nmc.Replicas(nmc.Instance.qap(F, D).bind(), R, 6)
    beta = np.geomspace(2e-5, 1e-3, M)
    rep.pt_run(beta, 4, 1, 1)
    be = rep.best_energy()
    assert (rep.recount() == be["energy"]).all()
    orep = oracle.QapReplicas(oracle.Qap(F, D), R, 6, threads=threads())
    orep.pt_run(beta, 4, 1, 1, chains=(16, 32))
    sl = _slots(M, C, (16, 32))
    assert (rep.get_state()[sl] == orep.perm[sl]).all()
    assert (rep.get_state("best")[sl] == orep.best_perm[sl]).all()
    assert (be["energy"][sl] == orep.cost[sl]).all()
    assert (be["best_per_replica"][sl] == orep.best[sl]).all()
