"""Whitening on the GPU (section "Whitening procedure for low energy
states") against the CPU oracle, bit for bit: frozen counts and white masks
of every replica's current and best state, over ragged replica counts,
clause lengths 2 to 4, states with and without frozen cores, and sampled
replicas of the N = 50,000 instance whose states the oracle computes itself."""
import numpy as np
import pytest

from gpu_util import KsatPair, say, threads
from paper_2111_13628_amd import instances, nmc

pytestmark = pytest.mark.gpu


def _check(pair, which):
    fz, white, passes = pair.rep.whiten(which, white=True)
    xs = pair.orep.best_x if which == "best" else pair.orep.x
    for r in range(pair.rep.R):
        k, star, _ = pair.oinst.whiten(xs[r])
        assert fz[r] == k, (r, fz[r], k)
        assert (white[r] == star).all(), r
    assert passes >= 1
    return fz, passes


def _mixed_formula(n, m, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    cp, lits = [0], []
    for _ in range(m):
        k = int(rng.integers(2, 5))
        vs = rng.choice(n, size=k, replace=False)
        lits += [int(v + 1) * (1 if rng.integers(0, 2) else -1) for v in vs]
        cp.append(len(lits))
    return np.array(cp, np.int32), np.array(lits, np.int32)


@pytest.mark.parametrize("n,alpha,k,R,seed,sweeps", [(400, "9.6", 4, 12, 3, 400), (301, "9.0", 4, 10, 4, 400),
                                                     (1000, "4.2", 3, 8, 5, 300), (400, "9.6", 4, 6, 6, 5)])
def test_whiten_matches_oracle(n, alpha, k, R, seed, sweeps):
    say(f"case: whitening n={n} alpha={alpha} R={R} sweeps={sweeps}")
    cp, lits = instances.gen_ksat(n, alpha, k, seed)
    pair = KsatPair(n, cp, lits, R, 20 + seed)
    pair.anneal(instances.linear_schedule(0.5, 6.0, sweeps)[None, :])
    pair.compare()
    for which in ("current", "best"):
        fz, passes = _check(pair, which)
        say(f"  {which}: frozen {fz.tolist()} passes {passes}")


def test_whiten_mixed_clause_lengths():
    say("case: whitening, clauses of 2 to 4 literals")
    cp, lits = _mixed_formula(300, 900, 7)
    pair = KsatPair(300, cp, lits, 8, 3)
    pair.anneal(instances.linear_schedule(0.5, 6.0, 300)[None, :])
    pair.compare()
    _check(pair, "current")


def test_full_size_whiten_sampled_replicas():
    """N = 50,000, 1024 replicas after 150 anneal sweeps; replicas 4 and 5,
    annealed by the oracle alone, whiten to the same frozen sets."""
    import oracle
    N, R = 50000, 1024
    say("case: whitening at N = 50,000, replicas 4 and 5")
    cp, lits = instances.gen_ksat(N, "9.9", 4, instances.DEFAULT_SEED)
    inst = nmc.Instance.ksat(N, cp, lits, 1024).bind()
    rep = nmc.Replicas(inst, R, 9)
    beta = instances.linear_schedule(0.5, 6.0, 150)[None, :]
    rep.anneal(beta)
    fz, white, passes = rep.whiten("current", white=True)
    say(f"  frozen: min {fz.min()} max {fz.max()} passes {passes}")
    ok = oracle.KSat(N, cp, lits)
    _, order, _ = ok.color(1024)
    orep = oracle.KSatReplicas(ok, R, 9, order, threads=threads(), snapshot=False)
    orep.threads = 2
    orep.anneal(beta, r_begin=4, r_end=6)
    for r in (4, 5):
        k, star, _ = ok.whiten(orep.x[r])
        assert fz[r] == k and (white[r] == star).all(), r


def test_whiten_errors():
    F, D = instances.gen_qap(8, 1)
    q = nmc.Replicas(nmc.Instance.qap(F, D).bind(), 16, 1)
    with pytest.raises(nmc.NmcError):
        q.whiten()
