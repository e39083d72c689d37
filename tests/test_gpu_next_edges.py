"""Edge and maximum-size cases of the steps beyond the core path, against
the CPU oracle: the largest instance the spin tables allow (N = 65534) and
an instance without clauses, for the LBP backbone, whitening and collective
cluster flips; tempering with two temperatures and one chain column."""
import numpy as np
import pytest

from gpu_util import KsatPair, say
from paper_2111_13628_amd import instances

pytestmark = pytest.mark.gpu


def test_largest_instance_whiten_cflip_lbp():
    n = 65534
    say("case: N = 65534, 5 replicas: whitening, cluster flips, LBP")
    cp, lits = instances.gen_ksat(n, "9.9", 4, 31)
    p = KsatPair(n, cp, lits, 5, 32, cap=1024)
    p.anneal(instances.linear_schedule(0.5, 3.0, 6)[None, :])
    fz, white, _ = p.rep.whiten("current", white=True)
    for r in (0, 4):
        k, star, _ = p.oinst.whiten(p.orep.x[r])
        assert fz[r] == k and (white[r] == star).all()
    rng = np.random.Generator(np.random.PCG64(2))
    lab = np.full(n, -1, np.int32)
    vs = rng.choice(n, 300, replace=False).reshape(30, 10)
    for row in vs:
        lab[row] = row.min()
    acc = p.rep.cluster_flip(lab, 0.7)
    oacc = p.orep.cluster_flip(lab, 0.7)
    assert (acc == oacc).all()
    p.compare()
    g = p.rep.lbp_backbone(2, "current", beta=1.0, lambda0=4.0, lambda_ratio=0.5, lambda_min=0.5, max_iter=60,
                           tol=1e-9, theta_seed=0.999, theta_cut=0.99)
    o = p.oinst.lbp(p.orep.x[2], 1.0, 4.0, 0.5, 0.5, 60, 1e-9)
    assert g["steps"] == o["steps"] and g["iterations"] == o["iterations"] and g["lambda"] == o["lambda"]
    assert np.abs(g["mag"] - o["mag"]).max() < 1e-9 and np.abs(g["corr"] - o["corr"]).max() < 1e-9


def test_no_clauses():
    say("case: 300 variables, no clauses: whitening, cluster flips, LBP")
    p = KsatPair(300, np.zeros(1, np.int32), np.zeros(0, np.int32), 7, 5)
    p.anneal(np.full((1, 3), 2.0))
    fz, white, passes = p.rep.whiten("best", white=True)
    assert (fz == 0).all() and (white == 1).all() and passes == 2
    lab = np.full(300, -1, np.int32)
    lab[[5, 9, 77]] = 5
    acc = p.rep.cluster_flip(lab, 3.0)
    assert (acc == p.orep.cluster_flip(lab, 3.0)).all() and (acc == 1).all()
    p.compare()
    g = p.rep.lbp_backbone(1, "current", beta=1.0, lambda0=2.0, lambda_ratio=0.5, lambda_min=0.1, max_iter=10,
                           tol=1e-9, theta_seed=0.5, theta_cut=0.5)
    o = p.oinst.lbp(p.orep.x[1], 1.0, 2.0, 0.5, 0.1, 10, 1e-9)
    assert g["converged"] == o["converged"] == 1 and g["steps"] == o["steps"] and g["iterations"] == o["iterations"]
    assert g["backbone_size"] == 0 and np.allclose(g["mag"], 0.0)


def test_tempering_smallest_ladder():
    """Two temperatures and 4 chains (one group column, both parities)."""
    say("case: tempering with 2 temperatures x 4 chains")
    cp, lits = instances.gen_ksat(500, "9.6", 4, 9)
    p = KsatPair(500, cp, lits, 8, 3)
    acc, att = p.pt_run(np.array([1.2, 1.25]), 9, 1, 1)
    assert att.tolist() == [4 * 4]
    p.compare()
