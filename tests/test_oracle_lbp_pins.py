"""Pins of the oracle's surrogate-Hamiltonian LBP and backbone growth
against facts fixed outside the oracle: on a factor graph without cycles
belief propagation is exact, so magnetizations and clause moments must equal
brute-force averages of the surrogate Boltzmann weight; the beta = 0 and
large-lambda limits have closed forms; the clusters are the connected
components (a library routine) of the rigid clauses that hold a seed.

Each test names the mistake it is meant to catch."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2111_13628_amd import instances


def _tree_formula(seed):
    """Clauses that each share one variable with the clauses before them: the
    factor graph is a tree (13 variables, clause lengths 2 to 4)."""
    vs = [(0, 1, 2), (2, 3, 4), (4, 5, 6), (1, 7, 8), (6, 9), (9, 10, 11, 12)]
    rng = np.random.Generator(np.random.PCG64(seed))
    lits, cp = [], [0]
    for c in vs:
        for v in c:
            lits.append((v + 1) * (1 if rng.integers(0, 2) else -1))
        cp.append(len(lits))
    return 13, np.array(cp, np.int32), np.array(lits, np.int32)


def _exact(n, cp, lits, s, beta, lam):
    """Brute-force <r_i> and <prod_{j in a} r_j> under
    exp(sum_i lam deg_i s_i r_i) * prod_a (exp(-2 beta) if a is violated)."""
    deg = np.zeros(n)
    for l in lits:
        deg[abs(l) - 1] += 1
    states = np.array(list(itertools.product([-1, 1], repeat=n)), np.float64)
    logw = states @ (lam * deg * s)
    for a in range(len(cp) - 1):
        sat = np.zeros(len(states), bool)
        for l in lits[cp[a]:cp[a + 1]]:
            sat |= states[:, abs(l) - 1] == (1 if l > 0 else -1)
        logw += np.where(sat, 0.0, -2.0 * beta)
    w = np.exp(logw - logw.max())
    w /= w.sum()
    mag = w @ states
    corr = np.array([w @ np.prod(states[:, [abs(l) - 1 for l in lits[cp[a]:cp[a + 1]]]], axis=1)
                     for a in range(len(cp) - 1)])
    return mag, corr


@pytest.mark.parametrize("seed,beta,lam", [(1, 0.7, 0.3), (2, 1.5, 0.1), (3, 0.3, 0.6), (4, 2.5, 0.05)])
def test_tree_marginals_are_exact(seed, beta, lam):
    """On a tree LBP is exact: magnetizations and clause moments equal the
    enumeration.  Catches a wrong message frame or sign, a missing cavity
    exclusion, a wrong clause weight and the clause moment without its
    product-of-biases term."""
    n, cp, lits = _tree_formula(seed)
    ks = oracle.KSat(n, cp, lits)
    x = np.random.Generator(np.random.PCG64(seed + 10)).integers(0, 2, n).astype(np.uint8)
    r = ks.lbp(x, beta, lam, 0.5, lam * 0.9, 500, 1e-15)
    assert r["converged"] == 1 and r["steps"] == 1 and r["lambda"] == lam
    mag, corr = _exact(n, cp, lits, 2.0 * x - 1, beta, lam)
    assert np.allclose(r["mag"], mag, atol=1e-12), np.abs(r["mag"] - mag).max()
    assert np.allclose(r["corr"], corr, atol=1e-12), np.abs(r["corr"] - corr).max()
    assert r["overlap"] == pytest.approx(np.mean((2.0 * x - 1) * mag), abs=1e-12)
    assert r["self_overlap"] == pytest.approx(np.mean(mag ** 2), abs=1e-12)


def test_zero_beta_is_free_spins_in_the_field():
    """beta = 0 makes every clause weight 1: u = 0, <r_i> = tanh(lam deg_i s_i)
    and the clause moment is the product of the literal biases."""
    cp, lits = instances.gen_ksat(40, "4.2", 3, 5)
    ks = oracle.KSat(40, cp, lits)
    x = ks.init(1, 2)[0]
    r = ks.lbp(x, 0.0, 0.05, 0.5, 0.04, 50, 1e-14)
    deg = np.bincount(np.abs(lits) - 1, minlength=40)
    s = 2.0 * x - 1
    assert np.abs(r["u"]).max() == 0.0
    assert np.allclose(r["mag"], np.tanh(0.05 * deg * s), atol=1e-15)
    want = [np.prod([math.tanh(0.05 * deg[abs(l) - 1] * s[abs(l) - 1]) for l in lits[cp[a]:cp[a + 1]]])
            for a in range(len(cp) - 1)]
    assert np.allclose(r["corr"], want, atol=1e-15)


def test_large_lambda_pins_to_the_reference():
    """A field far above every clause's pull keeps the surrogate at s*: the
    overlap p and the self-overlap q1 are 1 and every clause moment is the
    product of the reference spins."""
    cp, lits = instances.gen_ksat(200, "9.6", 4, 2)
    ks = oracle.KSat(200, cp, lits)
    x = ks.init(1, 4)[0]
    r = ks.lbp(x, 1.0, 50.0, 0.5, 40.0, 100, 1e-12)
    s = 2.0 * x - 1
    assert r["overlap"] > 1 - 1e-12 and r["self_overlap"] > 1 - 1e-12
    assert np.allclose(r["mag"], s, atol=1e-12)
    want = [np.prod(s[np.abs(lits[cp[a]:cp[a + 1]]) - 1]) for a in range(len(cp) - 1)]
    assert np.allclose(r["corr"], want, atol=1e-9)


def test_adiabatic_steps_and_stop_rule():
    """lambda_k = lambda0 ratio^k while >= lambda_min; a step that does not
    converge is discarded (the kept lambda is the last converged one), and a
    shorter schedule ending at the kept lambda gives the same messages."""
    cp, lits = instances.gen_ksat(300, "9.6", 4, 1)
    ks = oracle.KSat(300, cp, lits)
    x = ks.init(1, 3)[0]
    full = ks.lbp(x, 1.0, 4.0, 0.8, 1e-3, 40, 1e-10)
    assert full["converged"] == 1
    k = full["steps"]
    # the kept lambda is lambda0 ratio^(k-2) when step k-1 failed, else ratio^(k-1)
    last = 4.0 * 0.8 ** (k - 1)
    assert full["lambda"] in (pytest.approx(last), pytest.approx(last / 0.8))
    again = ks.lbp(x, 1.0, 4.0, 0.8, full["lambda"] * 0.9999, 40, 1e-10)
    assert again["lambda"] == full["lambda"]
    assert np.array_equal(again["u"], full["u"]) and np.array_equal(again["mag"], full["mag"])
    # a single step at lambda0 with one iteration cannot meet a tight tolerance
    one = ks.lbp(x, 1.0, 0.3, 0.8, 1e-3, 1, 1e-14)
    assert one["converged"] == 0 and one["steps"] == 1 and one["iterations"] == 1


def test_clusters_are_seeded_components_of_rigid_clauses():
    """Labels equal the connected components (scipy) of the variable graph
    joined by clauses with |corr| >= theta_cut, kept when a clause in them
    has |corr| >= theta_seed, labelled by their smallest variable."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    n = 400
    cp, lits = instances.gen_ksat(n, "4.2", 3, 9)
    m = len(cp) - 1
    corr = np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, m)
    ks = oracle.KSat(n, cp, lits)
    for ts, tc in [(0.99, 0.9), (0.95, 0.95), (0.999, 0.7)]:
        label, cls, k = ks.clusters(corr, ts, tc)
        rows, cols = [], []
        for a in range(m):
            if abs(corr[a]) >= tc:
                vs = np.abs(lits[cp[a]:cp[a + 1]]) - 1
                rows += [vs[0]] * len(vs)
                cols += list(vs)
        g = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
        nc, comp = connected_components(g, directed=False)
        seeded = set()
        for a in range(m):
            if abs(corr[a]) >= ts:
                seeded.add(comp[abs(lits[cp[a]]) - 1])
        want = np.full(n, -1)
        for c in seeded:
            members = np.nonzero(comp == c)[0]
            want[members] = members.min()
        assert (label == want).all()
        assert (cls == (want >= 0)).all()
        assert k == len(seeded)
