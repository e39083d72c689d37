"""Pins of the oracle's parallel-tempering pieces (appendix A) against facts
fixed outside the oracle: the exchange probability min{1, exp[dbeta dE]}
measured as a frequency, exact equilibrium averages by enumeration, the
binomial closed form of a formula with disjoint clauses, and exact variance.

Each test names the mistake it is meant to catch.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2111_13628_amd import instances


# ------------------------------------------------------------------ energy spread

def test_sigma_is_exact_population_spread():
    """sigma^2 = <E^2> - <E>^2 (divide by the count, not count - 1), checked
    against exact rational arithmetic; catches a sample (n - 1) variance, a
    dropped square or cancellation at large energies."""
    rng = np.random.Generator(np.random.PCG64(3))
    for base, spread, count in [(0, 30, 7), (5000, 40, 1000), (3_900_000_000, 100_000, 4096), (12, 0, 50)]:
        e = base + rng.integers(0, spread + 1, count)
        s1 = sum(Fraction(int(v)) for v in e)
        s2 = sum(Fraction(int(v) ** 2) for v in e)
        var = s2 / count - (s1 / count) ** 2
        want = math.sqrt(float(var))
        got = oracle.energy_sigma(e)
        assert got == pytest.approx(want, rel=1e-14, abs=1e-300), (base, spread)
    assert oracle.energy_sigma(np.array([0, 2])) == 1.0
    assert oracle.energy_sigma(np.array([7, 7, 7])) == 0.0
    e = rng.integers(0, 1000, 20000)
    assert oracle.energy_sigma(e) == pytest.approx(np.std(e), rel=1e-12)


# ------------------------------------------------------------------ exchange rule

def _exchange_rate(beta, e_hot, e_cold, chains, seed=5):
    rows = np.zeros((2 * chains, 3), np.uint8)
    rows[:chains, 0] = 1  # tag: the hot configuration
    energy = np.concatenate([np.full(chains, e_hot), np.full(chains, e_cold)]).astype(np.int64)
    acc, att = oracle.pt_exchange(np.array(beta), chains, seed, 17, 0, rows, energy)
    moved = rows[chains:, 0] == 1
    # configurations and energies travel together; a swap is all or nothing
    assert ((energy[chains:] == e_hot) == moved).all()
    assert ((energy[:chains] == e_cold) == moved).all()
    assert (rows[:chains, 0] == 0).sum() == moved.sum()
    assert att[0] == chains and acc[0] == moved.sum()
    return moved.mean()


@pytest.mark.parametrize("beta,d", [((0.5, 0.9), 1), ((0.5, 0.9), 3), ((1.0, 1.25), 6), ((2e-4, 1.2e-3), 1500),
                                    ((1e-5, 3e-5), 90_000)])
def test_exchange_frequency_is_min_one_exp(beta, d):
    """With the hot replica above the cold one by d, a swap happens with
    probability exp(-(beta_cold - beta_hot) d); catches a flipped sign
    (always accept), a missing factor or a swapped beta difference.  The last
    two cases need the high digit of the factored threshold."""
    chains = 40000
    rate = _exchange_rate(beta, 100_000 + d, 100_000, chains)
    p = math.exp(-(beta[1] - beta[0]) * d)
    se = math.sqrt(p * (1 - p) / chains)
    assert abs(rate - p) < 5 * se + 1e-9, (rate, p)


@pytest.mark.parametrize("d", [0, -1, -400])
def test_exchange_always_taken_when_hot_is_lower(d):
    """E_hot <= E_cold gives exp(>= 0) >= 1: every pair swaps."""
    assert _exchange_rate((0.3, 2.0), 1000 + d, 1000, 500) == 1.0


def test_exchange_pairs_follow_parity():
    """Parity 0 offers (0,1), (2,3); parity 1 offers (1,2), (3,4); no replica
    is in two pairs of one step."""
    beta = np.array([0.1, 0.2, 0.3, 0.4, 0.5])
    C = 8
    for parity, want in [(0, [C, 0, C, 0]), (1, [0, C, 0, C])]:
        rows = np.arange(5 * C, dtype=np.uint8)[:, None].copy()
        energy = np.arange(5 * C, dtype=np.int64)[::-1].copy()  # hotter holds higher: real draws
        _, att = oracle.pt_exchange(beta, C, 1, 3, parity, rows, energy)
        assert list(att) == want
        moved = np.nonzero(rows[:, 0] != np.arange(5 * C))[0] // C
        offered = {i for i, a in enumerate(want) if a} | {i + 1 for i, a in enumerate(want) if a}
        assert set(moved.tolist()) <= offered


def test_exchange_draw_is_word0_of_pt_stream():
    """The decision uses word 0 of the Philox block at (chain, sweep, position,
    PT_SWAP) against the factored threshold: recomputed from the RNG pin."""
    beta = np.array([0.4, 0.9])
    C, seed, t, d = 64, 99, 41, 2
    rows = np.zeros((2 * C, 1), np.uint8)
    rows[:C] = 1
    energy = np.array([10 + d] * C + [10] * C, np.int64)
    oracle.pt_exchange(beta, C, seed, t, 0, rows, energy)
    thr = oracle.threshold(0.5, d)
    for c in range(C):
        u = int(oracle.philox4x32_10([c, t, 0, oracle.STREAM_PT_SWAP], [seed, 0])[0])
        assert bool(rows[C + c, 0]) == (u < thr), c


# ------------------------------------------------------------------ equilibrium

def _all_states_energy(n, cp, lits):
    s = np.arange(2**n, dtype=np.uint32)
    e = np.zeros(2**n, np.int64)
    for a in range(len(cp) - 1):
        sat = np.zeros(2**n, bool)
        for l in lits[cp[a]:cp[a + 1]]:
            v = abs(int(l)) - 1
            bit = ((s >> np.uint32(v)) & np.uint32(1)).astype(bool)
            sat |= bit if l > 0 else ~bit
        e += ~sat
    return e


def test_pt_keeps_every_temperature_at_equilibrium():
    """Tempering with exchanges every sweep leaves each ladder position at its
    own Boltzmann distribution: the chain-averaged energy at every position
    matches the exact average over all 2^10 states.  A swap rule that breaks
    detailed balance (e.g. accepting every swap) drags the cold positions up
    and the hot ones down."""
    n = 10
    cp, lits = instances.gen_ksat(n, "4.3", 3, 21)
    allE = _all_states_energy(n, cp, lits)
    beta = np.array([0.2, 0.6, 1.1, 1.8])
    exact = [(allE * np.exp(-b * allE)).sum() / np.exp(-b * allE).sum() for b in beta]
    ks = oracle.KSat(n, cp, lits)
    _, order, _ = ks.color(0)
    C = 512
    rep = oracle.KSatReplicas(ks, C * len(beta), 8, order, threads=8, snapshot=False)
    rep.pt_run(beta, 60, 1)  # burn-in
    sums = np.zeros((len(beta), C))
    rounds = 300
    for k in range(rounds):
        rep.pt_run(beta, 1, 1, first_parity=k & 1)
        sums += rep.energy.reshape(len(beta), C)
    per_chain = sums / rounds
    for i in range(len(beta)):
        m = per_chain[i].mean()
        se = per_chain[i].std() / math.sqrt(C)
        assert abs(m - exact[i]) < 5 * se + 1e-3, (i, m, exact[i], se)


def _p_violated(beta, k):
    w = math.exp(-beta)
    return w / (w + 2**k - 1)


def test_pt_acceptance_matches_closed_form_on_disjoint_clauses():
    """With disjoint clauses the energy at beta is Binomial(M, p(beta)),
    p = e^-beta / (e^-beta + 2^k - 1), and replicas at different positions are
    independent at equilibrium, so the mean exchange probability of a pair is
    the double sum of min{1, exp[(b_i - b_j)(E_i - E_j)]} over both binomials."""
    M, k = 40, 3
    cp, lits = instances.gen_ksat_disjoint(M, k, 4)
    ks = oracle.KSat(M * k, cp, lits)
    _, order, _ = ks.color(0)
    beta = np.array([0.5, 0.9, 1.4])
    C = 128
    rep = oracle.KSatReplicas(ks, C * len(beta), 31, order, threads=8, snapshot=False)
    rep.pt_run(beta, 40, 2)
    acc, att = rep.pt_run(beta, 600, 2)
    from scipy.stats import binom
    Es = np.arange(M + 1)
    for i in range(len(beta) - 1):
        pi = binom.pmf(Es, M, _p_violated(beta[i], k))
        pj = binom.pmf(Es, M, _p_violated(beta[i + 1], k))
        ex = np.minimum(1.0, np.exp((beta[i] - beta[i + 1]) * (Es[:, None] - Es[None, :])))
        want = float(pi @ ex @ pj)
        rate = acc[i] / att[i]
        assert att[i] == C * 300
        assert abs(rate - want) < 0.02, (i, rate, want)


def test_ladder_sigma_matches_binomial_closed_form():
    """The adaptive ladder's sigma_i is the equilibrium energy spread at
    beta_i: sqrt(M p (1 - p)) for disjoint clauses; the next position is
    beta_i + alpha / sigma_i and the ladder stops at the first sigma <= sigma_min."""
    M, k = 300, 3
    cp, lits = instances.gen_ksat_disjoint(M, k, 6)
    ks = oracle.KSat(M * k, cp, lits)
    _, order, _ = ks.color(0)
    rep = oracle.KSatReplicas(ks, 512, 12, order, threads=8, snapshot=False)
    alpha, sigma_min = 1.1, 2.5
    # at high temperature most moves have dE = 0 and flip every sweep, so
    # sweep-order Metropolis keeps an even/odd memory of its start for tens of
    # sweeps; pooled samples then overstate the spread until it has decayed
    betas, sigmas = rep.apt_ladder(0.4, alpha, sigma_min, 60, 10, 12)
    assert len(betas) >= 3
    for b, s in zip(betas, sigmas):
        p = _p_violated(b, k)
        assert s == pytest.approx(math.sqrt(M * p * (1 - p)), rel=0.05), b
    for i in range(len(betas) - 1):
        assert betas[i + 1] == betas[i] + alpha / sigmas[i]
        assert sigmas[i] > sigma_min
    assert sigmas[-1] <= sigma_min or len(betas) == 12
    assert rep.sweeps_done == len(betas) * 70


def test_qap_exchange_moves_assignments_with_costs():
    """QAP tempering: assignments stay permutations, tracked costs equal
    recomputed costs after rounds of sweeps and exchanges."""
    F, D = instances.gen_qap(9, 3)
    q = oracle.Qap(F, D)
    beta = np.array([1e-3, 3e-3, 9e-3, 2e-2])
    C = 16
    rep = oracle.QapReplicas(q, C * len(beta), 5, threads=4)
    acc, att = rep.pt_run(beta, 30, 1)
    assert (att == [15 * C, 15 * C, 15 * C]).all() and (acc > 0).all()
    for r in range(rep.R):
        assert sorted(rep.perm[r]) == list(range(9))
        assert rep.cost[r] == q.cost(rep.perm[r])
    assert (rep.best <= rep.cost).all()


def test_following_some_chains_equals_the_full_run():
    """Chains are independent: following chains 1..2 alone reproduces those
    chains' slots of a run over all chains (used to check full-size runs on a
    sample of chains)."""
    cp, lits = instances.gen_ksat(200, "9.6", 4, 8)
    ks = oracle.KSat(200, cp, lits)
    _, order, _ = ks.color(0)
    beta = np.array([0.8, 1.1, 1.5, 2.0])
    C = 4
    full = oracle.KSatReplicas(ks, C * len(beta), 3, order, threads=4)
    part = oracle.KSatReplicas(ks, C * len(beta), 3, order, threads=4)
    full.pt_run(beta, 9, 1, 1, 30)
    part.pt_run(beta, 9, 1, 1, 30, chains=(1, 3))
    slots = [i * C + c for i in range(len(beta)) for c in (1, 2)]
    others = [r for r in range(C * len(beta)) if r not in slots]
    assert (full.x[slots] == part.x[slots]).all()
    for a in ("energy", "best", "first_hit"):
        assert (getattr(full, a)[slots] == getattr(part, a)[slots]).all(), a
    assert (part.x[others] == ks.init(C * len(beta), 3)[others]).all()
