"""Pins of the oracle's whitening (section "Whitening procedure for low
energy states") against facts fixed outside it: hand-solved formulas, the
least fixed point found by brute force over every set of white variables,
independence of the inspection order, and the lower-bound property the
section states (whitening never reports a variable frozen that changes
within the solution's cluster), checked by enumerating all solutions.

Each test names the mistake it is meant to catch."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2111_13628_amd import instances


def _formula(clauses):
    cp, lits = [0], []
    for c in clauses:
        lits += list(c)
        cp.append(len(lits))
    return np.array(cp, np.int32), np.array(lits, np.int32)


@pytest.mark.parametrize("clauses,n,x,frozen", [
    ([(1,), (-1, 2), (-2, 3), (-3, 4)], 4, [1, 1, 1, 1], [1, 1, 1, 1]),   # a forced chain
    ([(1,), (-1, 2), (-2, 3), (3, 4)], 4, [1, 1, 1, 0], [1, 1, 1, 0]),     # x4 false in its only clause
    ([(1, 2)], 2, [0, 0], [0, 0]),                                        # violated clause pins nothing
    ([(1, 2), (-1, 3)], 3, [1, 0, 1], [0, 0, 0]),                         # whitening cascades
    ([(1, 2), (1, -2)], 2, [1, 0], [0, 0]),               # x2 is white, then (1, 2) no longer pins x1
    ([(1, 2, 3), (-1, 2), (-2, 3), (-3, -1)], 3, [0, 1, 1], [0, 0, 0]),   # cascade over two passes
    ([(1,), (-1, 2), (2, 3)], 3, [1, 1, 0], [1, 1, 0]),
])
def test_hand_examples(clauses, n, x, frozen):
    """Catches a wrong pin condition (own literal true, every other literal
    false, no other white variable) and violated clauses that pin."""
    cp, lits = _formula(clauses)
    k, star, _ = oracle.KSat(n, cp, lits).whiten(np.array(x, np.uint8))
    assert list(1 - star) == frozen
    assert k == sum(frozen)


def _pins(n, cp, lits, x, star):
    """For each variable: pinned by some clause given the white set `star`."""
    out = np.zeros(n, bool)
    for a in range(len(cp) - 1):
        ls = lits[cp[a]:cp[a + 1]]
        true = [(l > 0) == bool(x[abs(l) - 1]) for l in ls]
        for j, l in enumerate(ls):
            i = abs(l) - 1
            others = [t for q, t in enumerate(true) if q != j]
            ostar = [star[abs(ls[q]) - 1] for q in range(len(ls)) if q != j]
            if true[j] and not any(others) and not any(ostar):
                out[i] = True
    return out


@pytest.mark.parametrize("seed", range(6))
def test_least_fixed_point_by_brute_force(seed):
    """The white set is the smallest set S with S = S u {unpinned given S}:
    found by trying every subset of 10 variables.  Catches stopping early,
    an order-dependent result and whitening pinned variables."""
    n = 10
    cp, lits = instances.gen_ksat(n, "2.5", 3, seed)
    ks = oracle.KSat(n, cp, lits)
    x = np.random.Generator(np.random.PCG64(seed)).integers(0, 2, n).astype(np.uint8)
    k, star, _ = ks.whiten(x)
    closed = []
    for bits in range(2 ** n):
        S = np.array([(bits >> i) & 1 for i in range(n)], bool)
        if ((~_pins(n, cp, lits, x, S)) <= S).all():
            closed.append(S)
    least = np.logical_and.reduce(closed)
    assert ((~_pins(n, cp, lits, x, least)) <= least).all()
    assert (star.astype(bool) == least).all()


def test_order_does_not_change_the_result():
    """Any inspection order reaches the same white set (a frozen core of
    hundreds of variables here)."""
    cp, lits = instances.gen_ksat(400, "9.6", 4, 3)
    ks = oracle.KSat(400, cp, lits)
    _, order, _ = ks.color(0)
    rep = oracle.KSatReplicas(ks, 4, 5, order, threads=4)
    rep.anneal(instances.linear_schedule(0.5, 6.0, 400)[None, :])
    x = rep.x[int(np.argmax([ks.whiten(rep.x[r])[0] for r in range(4)]))]
    ref = ks.whiten(x)
    rng = np.random.Generator(np.random.PCG64(1))
    for _ in range(5):
        o = rng.permutation(400).astype(np.int32)
        got = ks.whiten(x, o)
        assert got[0] == ref[0] and (got[1] == ref[1]).all()
    assert ref[0] > 0


@pytest.mark.parametrize("seed", range(8))
def test_frozen_is_a_lower_bound_on_the_cluster(seed):
    """For a solution, every variable whitening reports frozen keeps its
    value across the solution's cluster (solutions connected by single
    flips), found by enumerating all 2^14 states."""
    n = 14
    cp, lits = instances.gen_ksat(n, "3.8", 3, 100 + seed)
    ks = oracle.KSat(n, cp, lits)
    states = np.array(list(itertools.product([0, 1], repeat=n)), np.uint8)[:, ::-1]
    idx = np.arange(2 ** n)
    energy = np.array([ks.energy(s) for s in states])
    sols = set(idx[energy == 0].tolist())
    if not sols:
        pytest.skip("unsatisfiable draw")
    start = min(sols)
    cluster, todo = {start}, [start]
    while todo:
        s = todo.pop()
        for i in range(n):
            t = s ^ (1 << i)
            if t in sols and t not in cluster:
                cluster.add(t)
                todo.append(t)
    members = states[sorted(cluster)]
    truly_frozen = (members == members[0]).all(0)
    k, star, _ = ks.whiten(states[start])
    assert (truly_frozen | star.astype(bool)).all()  # frozen by whitening => frozen in the cluster
    # and every frozen variable is the only satisfier of some clause: one flip breaks the solution
    for i in np.nonzero(star == 0)[0]:
        assert ks.delta(states[start], i) > 0
