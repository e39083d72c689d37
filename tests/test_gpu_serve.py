"""Serving: a batched step (every set at its own point of its own schedule)
equals the same calls made set by set; the server's piecewise-constant
schedule equals that schedule run directly, and the CPU oracle; a request's
result does not depend on what else is served beside it; admission keeps the
admitted device bytes under the cap; budgets and bad requests retire cleanly."""
import time

import numpy as np
import pytest

from gpu_util import KsatPair, QapPair, say
from paper_2111_13628_amd import instances, nmc

pytestmark = pytest.mark.gpu

QAP_SCALE = 2e-4


def _ksat_set(n, alpha, k, R, seed):
    cp, lits = instances.gen_ksat(n, alpha, k, seed)
    inst = nmc.Instance.ksat(n, cp, lits).bind()
    return nmc.Replicas(inst, R, seed + 1000)


def _qap_set(n, R, seed):
    F, D = instances.gen_qap(n, seed)
    inst = nmc.Instance.qap(F, D).bind()
    return nmc.Replicas(inst, R, seed + 1000)


def _same(a, b):
    assert (a.get_state() == b.get_state()).all()
    assert (a.get_state("best") == b.get_state("best")).all()
    ea, eb = a.best_energy(), b.best_energy()
    for key in ("energy", "best_per_replica", "first_hit"):
        assert (ea[key] == eb[key]).all(), key
    assert a.sweeps_done() == b.sweeps_done()


def _summary(rep):
    be = rep.best_energy()
    fh = be["first_hit"]
    return int(be["best"]), int(be["n_at_zero"]), int(fh[fh >= 0].min()) if (fh >= 0).any() else -1


def test_step_equals_per_set_calls():
    """Four sets, three steps with different betas, profiles, backbone
    estimates and an idle set, against the same calls made set by set."""
    say("case: batched step vs per-set calls")
    mk = [lambda: _ksat_set(900, "9.6", 4, 37, 3), lambda: _ksat_set(1300, "4.15", 3, 64, 4),
          lambda: _qap_set(29, 40, 5), lambda: _ksat_set(500, "9.6", 4, 10, 6)]
    batched = [f() for f in mk]
    alone = [f() for f in mk]
    K = 9
    steps = [
        [(0.5, 0.5, "homogeneous", 0, 3), (1.5, 1.5, "homogeneous", 0, 0), (0.8 * QAP_SCALE, 0, "homogeneous", 0, -1),
         (2.0, 2.0, "homogeneous", 0, 1)],
        [(3.0, 0.7, "backbone", 1, 3), (2.5, 2.5, "homogeneous", 0, 0), (3 * QAP_SCALE, QAP_SCALE, "backbone", 1, -1),
         (0, 0, None, 0, 0)],
        [(3.5, 1.9, "backbone", 0, 3), (3.0, 1.0, "backbone", 1, 0), (4 * QAP_SCALE, 2 * QAP_SCALE, "backbone", 0, -1),
         (3.0, 3.0, "homogeneous", 0, 1)],
    ]
    b = nmc.Batch(batched)
    for segs in steps:
        status = b.step(segs, K, 9, 10, True)
        for s, (b0, b1, prof, bb, tgt) in zip(alone, segs):
            if prof is None:
                continue
            if bb:
                s.estimate_backbone(9, 10, True)
            if prof == "homogeneous":
                s.anneal(np.full((1, K), b0), target=tgt)
            else:
                s.reanneal(np.stack([np.full(K, b0), np.full(K, b1)]), "backbone", target=tgt)
        for s, st in zip(alone, status):
            assert st == _summary(s)
    for x, y in zip(alone, batched):
        _same(x, y)


def _schedule_segments(req, K):
    """The server's documented schedule, round by round."""
    na = req["anneal"] // K
    for c in range(na):
        f = c / (na - 1) if na > 1 else 0.0
        bt = req["beta0"] + (req["beta1"] - req["beta0"]) * f
        yield ("anneal", bt, None, False)
    nr = req["reanneal"] // K
    for _ in range(req["rounds"]):
        for c in range(nr):
            f = c / (nr - 1) if nr > 1 else 0.0
            yield ("reanneal", req["beta1"], req["beta_hot"] + (req["beta1"] - req["beta_hot"]) * f, c == 0)


def _run_direct(pair, req, K, qap):
    """The schedule on a KsatPair / QapPair (GPU and oracle side by side);
    returns what the server should report."""
    done = 0
    status = "exhausted"
    tgt = req.get("target")
    cls = None
    for phase, bc, bh, bb in _schedule_segments(req, K):
        if bb:
            cls = pair.backbone(9, 10) if qap else pair.backbone(9, 10, True)
        t = -1 if tgt is None else tgt
        if phase == "anneal":
            pair.anneal(np.full((1, K), bc), target=t)
        else:
            pair.anneal(np.stack([np.full(K, bc), np.full(K, bh)]), class_of=cls, profile="backbone", target=t)
        done += K
        if tgt is not None and (pair.orep.first_hit >= 0).any():
            status = "solved"
            break
    pair.compare()
    best = pair.orep.best
    fh = pair.orep.first_hit
    return dict(status=status, best=int(best.min()), n_at_zero=int((best == 0).sum()),
                first_hit=int(fh[fh >= 0].min()) if (fh >= 0).any() else -1, sweeps_done=done)


def _check(res, want):
    for key, val in want.items():
        assert res[key] == val, (key, res[key], val, res["message"])


def test_server_schedule_matches_direct_and_oracle():
    say("case: served requests vs direct schedule vs oracle")
    K = 10
    cp, lits = instances.gen_ksat(300, "9.6", 4, 7)
    F, D = instances.gen_qap(19, 8)
    kreq = dict(beta0=0.2, beta1=3.5, beta_hot=0.8, anneal=40, rounds=2, reanneal=20)
    qreq = dict(beta0=0.2 * QAP_SCALE, beta1=3.5 * QAP_SCALE, beta_hot=0.8 * QAP_SCALE, anneal=30, rounds=1,
                reanneal=20)
    ktreq = dict(kreq, target=6)
    srv = nmc.Server(chunk_sweeps=K)
    try:
        ids = [srv.submit_ksat(300, cp, lits, 32, 11, kreq["beta0"], kreq["beta1"], kreq["beta_hot"], 40, 2, 20),
               srv.submit_qap(F, D, 24, 12, qreq["beta0"], qreq["beta1"], qreq["beta_hot"], 30, 1, 20),
               srv.submit_ksat(300, cp, lits, 32, 13, kreq["beta0"], kreq["beta1"], kreq["beta_hot"], 40, 2, 20,
                               target=6)]
        assert srv.wait_idle(300)
        got = [srv.poll(i) for i in ids]
    finally:
        srv.free()
    want = [_run_direct(KsatPair(300, cp, lits, 32, 11), kreq, K, False),
            _run_direct(QapPair(F, D, 24, 12), qreq, K, True),
            _run_direct(KsatPair(300, cp, lits, 32, 13), ktreq, K, False)]
    say(f"  results: {[(g['status'], g['best'], g['sweeps_done']) for g in got]}")
    for g, w in zip(got, want):
        _check(g, w)


def _mix_requests():
    reqs = []
    for i, (n, alpha, k, R) in enumerate([(2000, "9.7", 4, 64), (700, "4.15", 3, 128), (5000, "9.7", 4, 64),
                                          (1200, "9.7", 4, 256), (3100, "4.15", 3, 32)]):
        cp, lits = instances.gen_ksat(n, alpha, k, 50 + i)
        reqs.append(("ksat", (n, cp, lits), R, 70 + i, (0.2, 3.0, 0.9), (60, 2, 30), 0 if i % 2 else 2))
    for i, n in enumerate((31, 60)):
        F, D = instances.gen_qap(n, 90 + i)
        reqs.append(("qap", (F, D), 64, 95 + i, tuple(x * QAP_SCALE for x in (0.2, 3.0, 0.9)), (60, 1, 30), None))
    return reqs


def _submit(srv, q):
    kind, data, R, seed, (b0, b1, bh), (a, rounds, re), tgt = q
    if kind == "ksat":
        return srv.submit_ksat(*data, R, seed, b0, b1, bh, a, rounds, re, target=tgt)
    return srv.submit_qap(*data, R, seed, b0, b1, bh, a, rounds, re, target=tgt)


def test_alone_equals_in_mix():
    """Every request of a mix of 7 (k-SAT and QAP, some with targets) gives
    the same result served alone and served with the others, with at most 3 on
    the GPU at once so that admission is continuous."""
    say("case: alone vs mix")
    reqs = _mix_requests()
    alone = []
    srv = nmc.Server(chunk_sweeps=10)
    try:
        for q in reqs:
            rid = _submit(srv, q)
            assert srv.wait_idle(300)
            alone.append(srv.poll(rid))
    finally:
        srv.free()
    srv = nmc.Server(chunk_sweeps=10, max_active=3)
    try:
        ids = [_submit(srv, q) for q in reqs]
        assert srv.wait_idle(300)
        mixed = [srv.poll(i) for i in ids]
        stats = srv.stats()
    finally:
        srv.free()
    say(f"  alone: {[(r['status'], r['best'], r['sweeps_done']) for r in alone]}")
    assert stats["completed"] == len(reqs) and stats["active"] == 0
    for a, m in zip(alone, mixed):
        assert a["status"] in ("solved", "exhausted"), a["message"]
        for key in ("status", "best", "n_at_zero", "first_hit", "sweeps_done"):
            assert a[key] == m[key], key
    admits = sorted(r["t_admit"] for r in mixed)
    assert admits[-1] > min(r["t_done"] for r in mixed), "admission was not continuous"


def test_admission_respects_cap():
    say("case: admission under a device-byte cap")
    reqs = _mix_requests()[:5]
    sizes = []
    for q in reqs:
        inst = nmc.Instance.ksat(*q[1])
        sizes.append(sum(inst.footprint(q[2])))
        inst.free()
    cap = int(max(sizes) * 1.6)
    srv = nmc.Server(chunk_sweeps=10, hbm_cap_bytes=cap)
    try:
        ids = [_submit(srv, q) for q in reqs]
        assert srv.wait_idle(300)
        res = [srv.poll(i) for i in ids]
        assert srv.stats()["device_bytes_in_use"] == 0
    finally:
        srv.free()
    assert all(r["status"] in ("solved", "exhausted") for r in res)
    assert [r["device_bytes"] for r in res] == sizes
    for r in res:
        live = sum(x["device_bytes"] for x in res if x["t_admit"] <= r["t_admit"] < x["t_done"])
        assert live <= cap
    assert max(r["t_admit"] for r in res) > min(r["t_done"] for r in res), "the cap never held a request back"


def test_budget_and_failed_requests():
    say("case: budgets and bad requests")
    cp, lits = instances.gen_ksat(800, "9.7", 4, 3)
    bad = lits.copy()
    bad[5] = 5000  # variable out of range: the loader rejects the request
    srv = nmc.Server(chunk_sweeps=10)
    try:
        a = srv.submit_ksat(800, cp, lits, 64, 1, 0.2, 3.0, 0.9, 100000, 0, 0, budget_s=1e-3)
        b = srv.submit_ksat(800, cp, bad, 64, 1, 0.2, 3.0, 0.9, 100, 0, 0)
        c = srv.submit_ksat(800, cp, lits, 64, 1, 0.2, 3.0, 0.9, 100, 0, 0)
        with pytest.raises(nmc.NmcError):
            srv.submit_ksat(800, cp, lits, 64, 1, 0.2, 3.0, 0.9, 95, 0, 0)
        assert srv.wait_idle(300)
        ra, rb, rc = srv.poll(a), srv.poll(b), srv.poll(c)
    finally:
        srv.free()
    assert ra["status"] == "timeout" and 10 <= ra["sweeps_done"] < 100000
    assert rb["status"] == "failed" and "load" in rb["message"]
    assert rc["status"] == "exhausted" and rc["sweeps_done"] == 100


def test_poll_snapshots_are_consistent():
    """Polls taken in a tight loop while requests run: whenever a snapshot
    shows a terminal status it also holds the completion time (published
    together under the server's lock), and a running request has an admission
    time at or after its submission."""
    say("case: polls while requests run")
    reqs = _mix_requests()
    srv = nmc.Server(chunk_sweeps=10, max_active=3)
    seen_terminal = 0
    try:
        ids = [_submit(srv, q) for q in reqs]
        deadline = time.monotonic() + 300
        while True:
            assert time.monotonic() < deadline, "requests did not finish"
            snaps = [srv.poll(i) for i in ids]
            for r in snaps:
                if r["status"] in ("solved", "exhausted", "timeout", "failed"):
                    seen_terminal += 1
                    assert r["t_done"] > 0 and r["t_done"] >= r["t_submit"], r
                    if r["status"] != "failed":
                        assert r["t_done"] >= r["t_admit"] >= r["t_submit"], r
                elif r["status"] == "running":
                    assert r["t_admit"] >= r["t_submit"], r
            if all(r["status"] in ("solved", "exhausted", "timeout", "failed") for r in snaps):
                break
        assert srv.wait_idle(300)
    finally:
        srv.free()
    assert seen_terminal >= len(reqs)
