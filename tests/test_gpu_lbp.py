"""Surrogate-Hamiltonian LBP and connected backbone growth on the GPU against
the CPU oracle: the adiabatic schedule's decisions (steps, iterations, kept
lambda) exactly, magnetizations, clause moments and overlaps to 1e-9 (both
sides are IEEE double; their tanh and log differ in the last bits), clusters
and classes exactly; the backbone then drives a reanneal bit for bit; and at
the benchmark size the clusters are the seeded components of the GPU's own
rigid clauses."""
import gc

import numpy as np
import pytest

from gpu_util import KsatPair, say
from paper_2111_13628_amd import instances, nmc

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _mixed_formula(n, m, seed):
    """Clauses of 2, 3 and 4 distinct variables (padding of short clauses)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cp, lits = [0], []
    for _ in range(m):
        k = int(rng.integers(2, 5))
        vs = rng.choice(n, size=k, replace=False)
        lits += [int(v + 1) * (1 if rng.integers(0, 2) else -1) for v in vs]
        cp.append(len(lits))
    return np.array(cp, np.int32), np.array(lits, np.int32)


def _safe_thresholds(corr, seed_thr, cut):
    """Move the thresholds off any |moment| within 1e-7 (the two sides'
    moments agree to ~1e-12, so the rigid and seed sets are then the same)."""
    a = np.abs(corr)
    for _ in range(100):
        if np.abs(a - seed_thr).min() > 1e-7 and np.abs(a - cut).min() > 1e-7:
            break
        seed_thr += 1.3e-7
        cut += 1.1e-7
    return seed_thr, cut


def _compare(pair, replica, which, cfg):
    ks = pair.oinst
    x = (pair.orep.best_x if which == "best" else pair.orep.x)[replica]
    o = ks.lbp(x, cfg["beta"], cfg["lambda0"], cfg["lambda_ratio"], cfg["lambda_min"], cfg["max_iter"], cfg["tol"],
               cfg["p_min"])
    ts, tc = _safe_thresholds(o["corr"], cfg["theta_seed"], cfg["theta_cut"])
    olab, ocls, ok = ks.clusters(o["corr"], ts, tc)
    g = pair.rep.lbp_backbone(replica, which, **dict(cfg, theta_seed=ts, theta_cut=tc))
    say(f"  lambda {g['lambda']:.4g} steps {g['steps']} iters {g['iterations']} p {g['overlap']:.4f} "
        f"q1 {g['self_overlap']:.4f} backbone {g['backbone_size']} clusters {g['n_clusters']}")
    for key in ("steps", "iterations", "converged"):
        assert g[key] == o[key], (key, g[key], o[key])
    assert g["lambda"] == o["lambda"]
    assert np.abs(g["mag"] - o["mag"]).max() < TOL
    assert np.abs(g["corr"] - o["corr"]).max() < TOL
    assert abs(g["overlap"] - o["overlap"]) < TOL and abs(g["self_overlap"] - o["self_overlap"]) < TOL
    assert (g["label"] == olab).all() and (g["cls"] == ocls).all()
    assert g["n_clusters"] == ok and g["backbone_size"] == int(ocls.sum())
    assert g["rigid_clauses"] == int((np.abs(o["corr"]) >= tc).sum())
    assert g["seed_clauses"] == int((np.abs(o["corr"]) >= ts).sum())
    return g, ocls


CFG = dict(beta=1.0, lambda0=4.0, lambda_ratio=0.8, lambda_min=0.02, max_iter=200, tol=1e-10, p_min=-2.0,
           theta_seed=0.995, theta_cut=0.97)


@pytest.mark.parametrize("n,alpha,k,seed,replica,which", [(300, "9.6", 4, 1, 5, "best"), (1000, "4.2", 3, 2, 0, "current"),
                                                          (2000, "9.7", 4, 3, 14, "best")])
def test_lbp_backbone_matches_oracle(n, alpha, k, seed, replica, which):
    say(f"case: LBP n={n} alpha={alpha} replica {replica} ({which})")
    cp, lits = instances.gen_ksat(n, alpha, k, seed)
    pair = KsatPair(n, cp, lits, 16, 30 + seed)
    pair.anneal(instances.linear_schedule(0.2, 3.0, 60)[None, :])
    _compare(pair, replica, which, CFG)


def test_lbp_mixed_lengths_schedule_variants():
    say("case: LBP mixed clause lengths, overlap stop, single step, no convergence")
    cp, lits = _mixed_formula(500, 1800, 4)
    pair = KsatPair(500, cp, lits, 8, 9)
    pair.anneal(instances.linear_schedule(0.2, 3.0, 40)[None, :])
    _compare(pair, 3, "best", CFG)
    _compare(pair, 3, "best", dict(CFG, p_min=0.9))                          # overlap stop
    _compare(pair, 2, "current", dict(CFG, lambda_min=3.5))                  # one step
    _compare(pair, 2, "current", dict(CFG, lambda0=0.3, max_iter=1, tol=1e-14))  # first step fails


def test_lbp_backbone_drives_reanneal():
    """The LBP backbone replaces the device classes: a backbone-profile
    reanneal then equals the oracle's reanneal with the oracle's classes."""
    say("case: LBP backbone -> reanneal")
    cp, lits = instances.gen_ksat(800, "9.6", 4, 5)
    pair = KsatPair(800, cp, lits, 24, 7)
    pair.anneal(instances.linear_schedule(0.2, 3.5, 80)[None, :])
    g, ocls = _compare(pair, 9, "best", dict(CFG, theta_seed=0.99, theta_cut=0.9))
    assert 0 < ocls.sum() < 800
    beta = np.stack([np.full(30, 3.5), np.linspace(0.5, 3.5, 30)])
    pair.anneal(beta, class_of=ocls, profile="backbone")
    pair.compare()


def test_full_size_lbp_properties():
    """N = 50,000, alpha = 9.9 from an annealed replica: converged messages,
    magnetizations in [-1, 1] with p and q1 their averages, and the backbone
    equal to the seeded connected components (scipy) of the GPU's rigid
    clauses, labelled by their smallest variable."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    say("case: LBP at N = 50,000")
    N = 50000
    cp, lits = instances.gen_ksat(N, "9.9", 4, instances.DEFAULT_SEED)
    inst = nmc.Instance.ksat(N, cp, lits, 1024).bind()
    rep = nmc.Replicas(inst, 64, 3)
    rep.anneal(instances.linear_schedule(0.1, 4.0, 300)[None, :])
    g = rep.lbp_backbone(0, "best", **dict(CFG, max_iter=100))
    say(f"  lambda {g['lambda']:.4g} steps {g['steps']} iters {g['iterations']} p {g['overlap']:.4f} "
        f"backbone {g['backbone_size']} clusters {g['n_clusters']} largest {g['largest_cluster']}")
    assert g["converged"] == 1
    x = rep.get_state("best")[0].astype(np.float64)
    s = 2 * x - 1
    assert np.abs(g["mag"]).max() <= 1.0
    assert abs(g["overlap"] - np.mean(s * g["mag"])) < 1e-9
    assert abs(g["self_overlap"] - np.mean(g["mag"] ** 2)) < 1e-9
    ts, tc = CFG["theta_seed"], CFG["theta_cut"]
    a = np.abs(g["corr"])
    rigid = np.nonzero(a >= tc)[0]
    v = np.abs(lits.reshape(-1, 4)) - 1
    rows = np.repeat(v[rigid, 0], 4)
    cols = v[rigid].ravel()
    nc, comp = connected_components(coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(N, N)), directed=False)
    seeded = np.unique(comp[v[np.nonzero(a >= ts)[0], 0]])
    want = np.full(N, -1)
    inb = np.isin(comp, seeded)
    mins = np.full(nc, N)
    np.minimum.at(mins, comp, np.arange(N))
    want[inb] = mins[comp[inb]]
    assert (g["label"] == want).all()
    assert g["backbone_size"] == int(inb.sum()) and g["n_clusters"] == len(seeded)


def test_lbp_errors():
    say("case: LBP argument errors")
    cp, lits = instances.gen_ksat(100, "4.2", 3, 1)
    rep = nmc.Replicas(nmc.Instance.ksat(100, cp, lits).bind(), 8, 1)
    for bad in (dict(lambda_ratio=1.0), dict(lambda0=0.0), dict(max_iter=0), dict(tol=0.0),
                dict(theta_seed=0.5, theta_cut=0.9), dict(beta=-1.0)):
        with pytest.raises(nmc.NmcError):
            rep.lbp_backbone(0, **dict(CFG, **bad))
    with pytest.raises(nmc.NmcError):
        rep.lbp_backbone(8)
    F, D = instances.gen_qap(8, 1)
    q = nmc.Replicas(nmc.Instance.qap(F, D).bind(), 16, 1)
    with pytest.raises(nmc.NmcError) as e:
        q.lbp_backbone(0)
    assert e.value.code == -6


def test_instance_released_before_its_replicas():
    """Releasing the instance first, explicitly or through the cycle
    collector (a frame that holds the exception of pytest.raises(...) as e
    forms a cycle, and the collector finalizes the instance before the
    replica set), must leave the replica set working and free both cleanly."""
    say("case: instance released before its replica set")
    cp, lits = instances.gen_ksat(300, "9.6", 4, 2)
    pair = KsatPair(300, cp, lits, 8, 5)
    pair.inst.free()
    pair.anneal(np.full((1, 20), 1.5))
    pair.compare()
    pair.rep.free()

    def cycle():
        rep = nmc.Replicas(nmc.Instance.ksat(300, cp, lits).bind(), 8, 5)
        with pytest.raises(nmc.NmcError) as e:
            rep.lbp_backbone(8)
        return e.value.code

    for _ in range(5):
        assert cycle() == -1
        gc.collect()


def test_batched_lbp_equals_single_runs_and_oracle():
    """One batched call over three sets of different sizes gives every set
    the result of its own single-set call (bit for bit) and of the oracle,
    and leaves each set's own backbone on the device for its reanneal."""
    say("case: batched LBP over 3 sets")
    specs = [(300, "9.6", 4, 1, 5), (1000, "4.2", 3, 2, 0), (2000, "9.7", 4, 3, 14)]
    pairs, singles, ocorr = [], [], []
    sched = instances.linear_schedule(0.2, 3.0, 60)[None, :]
    for n, alpha, k, seed, replica in specs:
        cp, lits = instances.gen_ksat(n, alpha, k, seed)
        pair = KsatPair(n, cp, lits, 16, 30 + seed)
        pair.anneal(sched)
        single = nmc.Replicas(nmc.Instance.ksat(n, cp, lits).bind(), 16, 30 + seed)
        single.anneal(sched)
        pairs.append(pair)
        singles.append(single)
        o = pair.oinst.lbp(pair.orep.best_x[replica], CFG["beta"], CFG["lambda0"], CFG["lambda_ratio"],
                           CFG["lambda_min"], CFG["max_iter"], CFG["tol"], CFG["p_min"])
        ocorr.append(o)
    ts, tc = CFG["theta_seed"], CFG["theta_cut"]
    for o in ocorr:
        ts, tc = _safe_thresholds(o["corr"], ts, tc)
    for o in ocorr:
        assert _safe_thresholds(o["corr"], ts, tc) == (ts, tc)
    cfg = dict(CFG, theta_seed=ts, theta_cut=tc)
    batch = nmc.Batch([p.rep for p in pairs])
    got = batch.lbp_backbone([sp[4] for sp in specs], "best", **cfg)
    for (n, alpha, k, seed, replica), pair, single, o, g in zip(specs, pairs, singles, ocorr, got):
        one = single.lbp_backbone(replica, "best", **cfg)
        for key in ("lambda", "steps", "iterations", "converged", "delta", "overlap", "self_overlap",
                    "backbone_size", "n_clusters", "largest_cluster", "rigid_clauses", "seed_clauses"):
            assert g[key] == one[key], (n, key, g[key], one[key])
        for key in ("steps", "iterations", "converged"):
            assert g[key] == o[key], (n, key)
        assert g["lambda"] == o["lambda"]
        _, ocls, _ = pair.oinst.clusters(o["corr"], ts, tc)
        assert g["backbone_size"] == int(ocls.sum())
        beta = np.stack([np.full(20, 3.0), np.linspace(0.5, 3.0, 20)])
        pair.anneal(beta, class_of=ocls, profile="backbone")
        pair.compare()
