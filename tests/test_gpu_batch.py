"""Batched launches (many replica sets of different instances in one grid,
optionally one HIP graph for the whole anneal -> backbone -> reanneal plan):
every set's results are bit-identical to running it alone, whatever the
workgroup size the tuner picks."""
import numpy as np
import pytest

import oracle
from gpu_util import say, threads
from paper_2111_13628_amd import instances, nmc

pytestmark = pytest.mark.gpu


def _mix(seed=11):
    specs = [("ksat", 1000, "4.15", 3, 64), ("ksat", 1700, "9.8", 4, 128), ("ksat", 3900, "9.8", 4, 38),
             ("ksat", 700, "4.15", 3, 10), ("qap", 23, None, None, 40), ("ksat", 6000, "9.8", 4, 256),
             ("qap", 57, None, None, 16)]
    out = []
    for i, (kind, n, alpha, k, R) in enumerate(specs):
        if kind == "ksat":
            cp, lits = instances.gen_ksat(n, alpha, k, seed + i)
            out.append(("ksat", (n, cp, lits), R, seed + 100 + i))
        else:
            F, D = instances.gen_qap(n, seed + i)
            out.append(("qap", (F, D), R, seed + 100 + i))
    return out


def _make(mix):
    sets = []
    for kind, data, R, sd in mix:
        inst = nmc.Instance.ksat(*data) if kind == "ksat" else nmc.Instance.qap(*data)
        inst.bind()
        sets.append(nmc.Replicas(inst, R, sd))
    return sets


def _sched():
    a = instances.linear_schedule(0.1, 4.0, 24)
    r = instances.profile_schedule(np.full(10, 4.0), instances.linear_schedule(0.5, 4.0, 10))
    return a, r


def _scale(kind):
    return 1.0 if kind == "ksat" else 2e-4


def _compare(a, b):
    assert (a.get_state() == b.get_state()).all()
    assert (a.get_state("best") == b.get_state("best")).all()
    ea, eb = a.best_energy(), b.best_energy()
    for key in ("energy", "best_per_replica", "first_hit"):
        assert (ea[key] == eb[key]).all(), key
    assert a.sweeps_done() == b.sweeps_done()


def test_batched_calls_equal_individual_calls():
    say("case: batch vs alone, 7 sets (5 k-SAT, 2 QAP)")
    mix = _mix()
    alone = _make(mix)
    batched = _make(mix)
    a_beta, r_beta = _sched()
    # nmc_batch_anneal takes one schedule for every set, so the QAP sets (beta
    # in cost units) get a batch of their own here; one batch with a schedule
    # per set is nmc_batch_run (test_per_set_plans_mixed_batch)
    groups = {"ksat": [i for i, m in enumerate(mix) if m[0] == "ksat"],
              "qap": [i for i, m in enumerate(mix) if m[0] == "qap"]}
    for kind, idx in groups.items():
        sc = _scale(kind)
        targets = [int(i * 3) for i in idx]
        b = nmc.Batch([batched[i] for i in idx])
        b.anneal(a_beta[None, :] * sc, targets=targets)
        b.estimate_backbone(9, 10, True)
        b.anneal(r_beta * sc, profile="backbone", targets=targets)
        for j, i in enumerate(idx):
            s = alone[i]
            s.anneal(a_beta[None, :] * sc, target=targets[j])
            s.estimate_backbone(9, 10, True)
            s.reanneal(r_beta * sc, "backbone", target=targets[j])
    for i in range(len(mix)):
        _compare(alone[i], batched[i])


@pytest.mark.parametrize("use_graph,chunk", [(True, 0), (False, 0), (True, 7)])
def test_plan_equals_call_sequence(use_graph, chunk):
    say(f"case: plan (graph={use_graph}, chunk={chunk})")
    mix = [m for m in _mix(23) if m[0] == "ksat"]
    alone = _make(mix)
    planned = _make(mix)
    a_beta, r_beta = _sched()
    b = nmc.Batch(planned)
    b.run_plan(a_beta, 2, r_beta, 9, 10, True, targets=5, use_graph=use_graph, chunk_sweeps=chunk)
    for s in alone:
        s.anneal(a_beta[None, :], target=5)
        for _ in range(2):
            s.estimate_backbone(9, 10, True)
            s.reanneal(r_beta, "backbone", target=5)
    for x, y in zip(alone, planned):
        _compare(x, y)


def test_qap_plan_in_graph():
    mix = [m for m in _mix(31) if m[0] == "qap"]
    alone = _make(mix)
    planned = _make(mix)
    a_beta, r_beta = _sched()
    sc = _scale("qap")
    nmc.Batch(planned).run_plan(a_beta * sc, 1, r_beta * sc, 9, 10, False, use_graph=True)
    for s in alone:
        s.anneal(a_beta[None, :] * sc)
        s.estimate_backbone(9, 10, False)
        s.reanneal(r_beta * sc, "backbone")
    for x, y in zip(alone, planned):
        _compare(x, y)


def test_tuner_choice_does_not_change_results():
    say("case: tuner invariance")
    mix = [m for m in _mix(41) if m[0] == "ksat"]
    a_beta, _ = _sched()
    ref = None
    for bt in (64, 256, 1024, "tuned"):
        sets = _make(mix)
        b = nmc.Batch(sets)
        if bt == "tuned":
            chosen = b.tune(2)
            assert chosen in (64, 128, 256, 512, 1024)
        else:
            b.set_tuning(bt)
        b.anneal(a_beta[None, :], targets=2)
        got = [(s.get_state(), s.best_energy()["best_per_replica"]) for s in sets]
        if ref is None:
            ref = got
        else:
            for (x0, b0), (x1, b1) in zip(ref, got):
                assert (x0 == x1).all() and (b0 == b1).all()


def test_full_batch_of_256_sampled_against_oracle():
    """The batched benchmark's configuration (256 mixed k-SAT instances, the
    tuner's block size, one HIP graph, lockstep chunks) on a short plan;
    sampled instances, from the smallest to the largest, checked against the
    oracle running them alone."""
    say("case: 256-instance batch, sampled parity")
    mix = instances.batch_mix(256, instances.DEFAULT_SEED)
    data = [instances.gen_ksat(m["n"], m["alpha"], m["k"], m["seed"]) for m in mix]
    sets = []
    for m, (cp, lits) in zip(mix, data):
        inst = nmc.Instance.ksat(m["n"], cp, lits, 0).bind()
        sets.append(nmc.Replicas(inst, m["replicas"], m["seed"]))
    b = nmc.Batch(sets)
    b.tune(2)
    a_beta = instances.linear_schedule(0.1, 4.0, 1000)[:4]
    r_beta = instances.profile_schedule(np.full(500, 4.0), instances.linear_schedule(0.5, 4.0, 500))[:, :3]
    targets = [len(cp) if i % 2 else 0 for i, (cp, _) in enumerate(data)]
    b.run_plan(a_beta, 1, r_beta, 9, 10, True, targets=targets, use_graph=True, chunk_sweeps=2)
    by_size = sorted(range(256), key=lambda i: mix[i]["n"] * mix[i]["replicas"])
    for i in by_size[:3] + by_size[127:129] + by_size[-1:]:
        m, (cp, lits) = mix[i], data[i]
        say(f"  instance {i}: N={m['n']} k={m['k']} R={m['replicas']}")
        ok = oracle.KSat(m["n"], cp, lits)
        _, order, _ = ok.color(0)
        orep = oracle.KSatReplicas(ok, m["replicas"], m["seed"], order, threads=threads())
        orep.anneal(a_beta[None, :], target=targets[i])
        cls, _ = orep.backbone(9, 10, True)
        orep.anneal(r_beta, class_of=cls, target=targets[i])
        s_ = sets[i]
        assert (s_.get_state() == orep.x).all()
        assert (s_.get_state("best") == orep.best_x).all()
        be = s_.best_energy()
        assert (be["energy"] == orep.energy).all()
        assert (be["best_per_replica"] == orep.best).all()
        assert (be["first_hit"] == orep.first_hit).all()
        assert s_.sweeps_done() == orep.sweeps_done


def _own_plans(mix, seed):
    """A different plan for every set of the mix: own anneal length, beta
    units and range, rounds, reanneal length, backbone rule and chunk size."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(24, 2, 10, 0, (9, 10, True)), (17, 1, 6, 7, (3, 4, False)), (30, 0, 0, 5, (9, 10, True)),
              (9, 3, 4, 0, (1, 2, True)), (20, 1, 8, 4, (9, 10, False)), (12, 2, 5, 0, (9, 10, True)),
              (15, 1, 3, 6, (2, 3, False))]
    plans = []
    for (kind, _, _, _), (sa, rounds, sr, chunk, (num, den, ex)) in zip(mix, shapes):
        sc = _scale(kind) * float(rng.uniform(0.7, 1.4))
        b1 = float(rng.uniform(2.5, 4.5))
        a = instances.linear_schedule(0.1, b1, sa) * sc
        r = instances.profile_schedule(np.full(sr, b1), instances.linear_schedule(0.5, b1, sr)) * sc
        plans.append(dict(anneal_beta=a, rounds=rounds, reanneal_beta=r if rounds else None, thr_num=num,
                          thr_den=den, expand=ex, chunk_sweeps=chunk))
    return plans


def _run_alone(s, plan, target):
    s.anneal(plan["anneal_beta"][None, :], target=target)
    for _ in range(plan["rounds"]):
        s.estimate_backbone(plan["thr_num"], plan["thr_den"], plan["expand"])
        if plan["reanneal_beta"].shape[1]:
            s.reanneal(plan["reanneal_beta"], "backbone", target=target)


@pytest.mark.parametrize("use_graph", [True, False])
def test_per_set_plans_mixed_batch(use_graph):
    """k-SAT and QAP sets, each with its own schedule, in one nmc_batch_run
    call (one HIP graph when use_graph): every set equals its own call
    sequence run alone; a second and a third call of the same shape replay
    the kept graph (the third with other betas and targets)."""
    say(f"case: per-set plans, 5 k-SAT + 2 QAP, graph={use_graph}")
    mix = _mix(53)
    alone = _make(mix)
    batched = _make(mix)
    plans = _own_plans(mix, 1)
    targets = [40, 25, 30, 8, 0, 0, 0]
    b = nmc.Batch(batched)
    b.run(plans, targets=targets, use_graph=use_graph)
    for s, p, t in zip(alone, plans, targets):
        _run_alone(s, p, t)
    for x, y in zip(alone, batched):
        _compare(x, y)
    b.run(plans, targets=targets, use_graph=use_graph)
    for s, p, t in zip(alone, plans, targets):
        _run_alone(s, p, t)
    plans2 = _own_plans(mix, 2)
    targets2 = [t + 3 for t in targets]
    b.run(plans2, targets=targets2, use_graph=use_graph)
    for s, p, t in zip(alone, plans2, targets2):
        _run_alone(s, p, t)
    for x, y in zip(alone, batched):
        _compare(x, y)
    assert b.graph_info() == ((1, 2) if use_graph else (0, 0))
    # another shape (one set's plan longer) captures a new graph
    plans2[0]["anneal_beta"] = np.concatenate([plans2[0]["anneal_beta"], [1.0]])
    b.run(plans2, targets=targets2, use_graph=use_graph)
    for s, p, t in zip(alone, plans2, targets2):
        _run_alone(s, p, t)
    for x, y in zip(alone, batched):
        _compare(x, y)
    assert b.graph_info() == ((2, 2) if use_graph else (0, 0))
    b.free()


def test_per_set_plans_against_oracle():
    """One graph over a k-SAT set and a QAP set with different schedules and
    rounds; both followed by the oracle alone, bit for bit."""
    say("case: per-set plans vs oracle")
    n, R = 900, 36
    cp, lits = instances.gen_ksat(n, "9.8", 4, 71)
    F, D = instances.gen_qap(31, 72)
    ks = nmc.Replicas(nmc.Instance.ksat(n, cp, lits).bind(), R, 73)
    qs = nmc.Replicas(nmc.Instance.qap(F, D).bind(), 20, 74)
    kp = dict(anneal_beta=instances.linear_schedule(0.1, 4.0, 30), rounds=2,
              reanneal_beta=instances.profile_schedule(np.full(12, 4.0), instances.linear_schedule(0.5, 4.0, 12)),
              thr_num=9, thr_den=10, expand=True, chunk_sweeps=8)
    sc = 3e-4
    qp = dict(anneal_beta=instances.linear_schedule(0.1, 4.0, 21) * sc, rounds=1,
              reanneal_beta=instances.profile_schedule(np.full(9, 4.0), instances.linear_schedule(0.5, 4.0, 9)) * sc,
              thr_num=3, thr_den=4, expand=False, chunk_sweeps=5)
    b = nmc.Batch([ks, qs])
    b.run([kp, qp], targets=[35, 0], use_graph=True)
    ok = oracle.KSat(n, cp, lits)
    _, order, _ = ok.color(0)
    ko = oracle.KSatReplicas(ok, R, 73, order, threads=threads())
    ko.anneal(kp["anneal_beta"][None, :], target=35)
    for _ in range(2):
        cls, _ = ko.backbone(9, 10, True)
        ko.anneal(kp["reanneal_beta"], class_of=cls, target=35)
    qo = oracle.QapReplicas(oracle.Qap(F, D), 20, 74, threads=threads())
    qo.anneal(qp["anneal_beta"][None, :], target=0)
    cls, _ = qo.backbone(3, 4)
    qo.anneal(qp["reanneal_beta"], class_of=cls, target=0)
    for s, x, best_x, e, best, fh, sw in ((ks, ko.x, ko.best_x, ko.energy, ko.best, ko.first_hit, ko.sweeps_done),
                                          (qs, qo.perm, qo.best_perm, qo.cost, qo.best, qo.first_hit,
                                           qo.sweeps_done)):
        assert (s.get_state() == x).all()
        assert (s.get_state("best") == best_x).all()
        be = s.best_energy()
        assert (be["energy"] == e).all() and (be["best_per_replica"] == best).all()
        assert (be["first_hit"] == fh).all()
        assert s.sweeps_done() == sw
    b.free()


def test_batch_with_eight_replica_workgroups_equals_alone():
    """Sets with 8 replicas per workgroup (forced, and as the tuner picks)
    next to sets with 4, in one batched plan: every set equals its calls run
    alone with 4 replicas per workgroup."""
    say("case: batch with 4- and 8-replica workgroups")
    mix = [m for m in _mix(61) if m[0] == "ksat"]
    alone = _make(mix)
    batched = _make(mix)
    for i, s in enumerate(batched):
        if i % 2 == 0:
            s.set_replicas_per_workgroup(8)
    a_beta, r_beta = _sched()
    b = nmc.Batch(batched)
    b.run_plan(a_beta, 1, r_beta, 9, 10, True, targets=4, use_graph=True, chunk_sweeps=8)
    chosen = b.tune(2)
    assert chosen in (64, 128, 256, 512, 1024)
    b.run_plan(a_beta, 1, r_beta, 9, 10, True, targets=4, use_graph=True, chunk_sweeps=8)
    for s in alone:
        for _ in range(2):
            s.anneal(a_beta[None, :], target=4)
            s.estimate_backbone(9, 10, True)
            s.reanneal(r_beta, "backbone", target=4)
    for x, y in zip(alone, batched):
        _compare(x, y)
