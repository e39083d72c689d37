"""Pins of the oracle's collective cluster flips (the NMC scheme's nonlocal
move) against facts fixed outside it: at beta = 0 every cluster flips once
(a closed form), at a huge beta no flip raises the energy, tracked energies
equal recounts, and alternating Metropolis sweeps with cluster flips keeps
the exact Boltzmann distribution (a flip of a fixed cluster is its own
inverse, so Metropolis acceptance keeps detailed balance).

Each test names the mistake it is meant to catch."""
import math

import numpy as np

import oracle
from paper_2111_13628_amd import instances


def _labels(n, groups):
    lab = np.full(n, -1, np.int32)
    for g in groups:
        lab[list(g)] = min(g)
    return lab


def test_zero_beta_flips_every_cluster_once():
    """Catches skipping clusters, flipping a cluster twice, or flipping
    variables outside it."""
    n = 60
    cp, lits = instances.gen_ksat(n, "4.2", 3, 2)
    ks = oracle.KSat(n, cp, lits)
    _, order, _ = ks.color(0)
    lab = _labels(n, [(3, 7, 9), (10, 11), (20, 30, 40, 50), (59,)])
    rep = oracle.KSatReplicas(ks, 6, 4, order)
    x0 = rep.x.copy()
    acc = rep.cluster_flip(lab, 0.0)
    assert (acc == 4).all()
    want = x0 ^ (lab >= 0).astype(np.uint8)[None, :]
    assert (rep.x == want).all()
    assert all(rep.energy[r] == ks.energy(rep.x[r]) for r in range(6))
    assert rep.sweeps_done == 1


def test_cold_flips_never_raise_the_energy():
    """Catches accepting uphill moves at beta -> infinity and a wrong sign of dE."""
    n = 300
    cp, lits = instances.gen_ksat(n, "9.6", 4, 3)
    ks = oracle.KSat(n, cp, lits)
    _, order, _ = ks.color(0)
    rng = np.random.Generator(np.random.PCG64(5))
    lab = np.full(n, -1, np.int32)
    for c in range(30):
        vs = rng.choice(n, 4, replace=False)
        if (lab[vs] < 0).all():
            lab[vs] = vs.min()
    rep = oracle.KSatReplicas(ks, 16, 8, order)
    rep.anneal(np.full((1, 5), 1.0))
    for _ in range(3):
        e0 = rep.energy.copy()
        rep.cluster_flip(lab, 60.0)
        assert (rep.energy <= e0).all()
        assert all(rep.energy[r] == ks.energy(rep.x[r]) for r in range(16))


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


def test_cluster_flips_keep_boltzmann():
    """Start 200,000 replicas exactly at exp(-beta E) over all 2^10 states
    (drawn with numpy), apply one collective-move sweep and nothing else: the
    distribution must stay put (chi-square).  Accepting every flip, halving
    the exponent or flipping the sign of dE moves it away."""
    n, beta = 10, 0.9
    cp, lits = instances.gen_ksat(n, "4.2", 3, 12)
    ks = oracle.KSat(n, cp, lits)
    _, order, _ = ks.color(0)
    lab = _labels(n, [(0, 4, 5), (2, 7), (1, 3, 8, 9)])
    allE = _all_states_energy(n, cp, lits)
    p = np.exp(-beta * allE)
    p /= p.sum()
    R = 200000
    idx0 = np.random.Generator(np.random.PCG64(3)).choice(2**n, size=R, p=p)
    rep = oracle.KSatReplicas(ks, R, 77, order, threads=8, snapshot=False)
    rep.x[:] = ((idx0[:, None] >> np.arange(n)) & 1).astype(np.uint8)
    rep.energy[:] = allE[idx0]
    acc = rep.cluster_flip(lab, beta)
    assert 0 < acc.mean() < 3
    idx = (rep.x.astype(np.int64) << np.arange(n)).sum(1)
    assert (rep.energy == allE[idx]).all()
    h = np.bincount(idx, minlength=2**n)
    chi2 = ((h - R * p) ** 2 / (R * p)).sum()
    dof = 2**n - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof), chi2
