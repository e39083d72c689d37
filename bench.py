#!/usr/bin/env python3
"""Benchmark of the NMC hot path on one MI355X.

One step = the whole path on the random 4-SAT workload N = 50,000 variables,
alpha = 9.9 (M = 495,000 clauses), 1024 replicas: replica init and energy
count, a homogeneous anneal of 2000 sweeps (beta 0.1 -> 4.0), then 3 rounds of
[backbone estimate (|magnetization| >= 0.9, frozen variables and their clause
neighbours hot) -> reanneal of 1000 sweeps (cold at beta 4.0, hot ramped
0.5 -> 4.0)], then the best-energy tally.  The instance is uploaded to HBM
before the timed region.

Prints one JSON line: attempts/s of the whole step, the sweep kernel's
roofline figures (kernel time from HIP events on the launch stream), the
time-to-target against plain simulated annealing on the same GPU, and the CPU
oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2111_13628_amd import instances  # noqa: E402

N, ALPHA, K, R = 50000, "9.9", 4, 1024
S_ANNEAL, ROUNDS, S_RE = 2000, 3, 1000
BETA0, BETA1, BETA_HOT = 0.1, 4.0, 0.5
CLASS_CAP = 1024
BLOCK_THREADS = 0
RPW = 0  # k-SAT replicas per sweep workgroup (0: the library's default, 4)
# VALU lane-operations the sweep kernel issues per (variable, clause slot) for
# its 4 replicas, and per variable for the acceptance step, counted in the
# kernel's instruction stream.
OPS_PER_SLOT = 9.0
OPS_PER_VAR = 62.0
# VALU lane rate behind the published 157.3 TFLOP/s fp32 vector figure (two
# flops per fused multiply-add): 256 CUs x 128 lane-operations x 2.4 GHz
PEAK_LANE_OPS = 157.3e12 / 2
LDS_LANE_READS = 256 * 32 * 2.4e9  # CUs x LDS banks x clock (one lane read per bank per clock)
# LDS byte reads the sweep kernel does per (variable, clause slot) for its 4
# replicas (the clause's three other literals) and per variable (its own spin)
READS_PER_SLOT = 3.0
READS_PER_VAR = 1.0


HBM_PEAK = 8.0e12  # bytes/s, published MI355X HBM3E figure


def ksat_roofline(kt, n_clauses, acceptance, traffic=None):
    """Roofline of ksat_sweep_kernel from its HIP-event time `kt` on the
    N-variable, n_clauses-clause k-SAT instance.  Primary (the scope table's
    measurement model): the per-clause-counter formulation's algorithmic HBM
    bytes, (deg + 1)(1 + a) per attempt with a the measured acceptance rate,
    against 8 TB/s.  Beside it the model of this kernel, which keeps the
    spins in LDS: LDS byte gathers ((3 deg + 1) / 4 per attempt against one
    lane read per bank per clock) and VALU lane operations."""
    deg_mean = K * n_clauses / N
    att_s = kt["attempts"] / (kt["ms"] / 1000.0)
    per_att = (deg_mean + 1.0) * (1.0 + acceptance)
    launches = max(1, kt["launches"])
    reads = att_s * (READS_PER_SLOT * deg_mean + READS_PER_VAR) / 4.0
    ops = att_s * (OPS_PER_SLOT * deg_mean + OPS_PER_VAR) / 4.0
    hbm = att_s * per_att
    return {"bound": "hbm", "achieved": hbm / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": hbm / HBM_PEAK, "survey_frac": hbm / HBM_PEAK, "traffic": traffic,
            "bytes_per_attempt": per_att, "acceptance": acceptance, "mean_degree": deg_mean,
            "algorithmic_bytes_per_launch": per_att * kt["attempts"] / launches,
            "model": "(deg + 1)(1 + a) bytes per attempt (per-clause counters and the spin byte, "
                     "written back on accept) x kernel attempts/s; a = accepted flips / attempts",
            "kernel": "ksat_sweep_kernel", "kernel_ms_per_launch": kt["ms"] / launches,
            "kernel_attempts_per_s": att_s, "launches": kt["launches"],
            "lds": {"achieved": reads / 1e12, "peak": LDS_LANE_READS / 1e12, "unit": "T lane-reads/s",
                    "frac": reads / LDS_LANE_READS},
            "valu": {"achieved": ops / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "T lane-op/s",
                     "frac": ops / PEAK_LANE_OPS}}


def reanneal_profile(S):
    return instances.profile_schedule(np.full(S, BETA1), instances.linear_schedule(BETA_HOT, BETA1, S))


KSAT_PROFILE = os.path.join(ROOT, "profiles", "ksat_sweep_n50000_r1024.md")


def counter_bytes_per_sweep():
    """HBM bytes per sweep of the k-SAT sweep kernel from the committed
    counter passes, or None when the kernel sources changed since then."""
    import hashlib
    try:
        text = open(KSAT_PROFILE).read()
    except OSError:
        return None
    fields = dict(re.findall(r"^(\w+): (.+)$", text, flags=re.M))
    if "counter_bytes_per_sweep" not in fields or "kernel_sources" not in fields:
        return None
    h = hashlib.sha256()
    for f in fields["kernel_sources"].split():
        try:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        except OSError:
            return None
    if h.hexdigest() != fields.get("kernel_sources_sha256", "").strip():
        return None
    return float(fields["counter_bytes_per_sweep"])


def run_path(inst, seed, target, nmc, stream=None, profile=False):
    rep = nmc.Replicas(inst, R, seed, stream)
    if BLOCK_THREADS:
        rep.set_tuning(BLOCK_THREADS)
    if RPW:
        rep.set_replicas_per_workgroup(RPW)
    rep.set_profiling(profile)
    rep.anneal(instances.linear_schedule(BETA0, BETA1, S_ANNEAL)[None, :], target=target, stream=stream)
    for _ in range(ROUNDS):
        rep.estimate_backbone_device(9, 10, True, stream=stream)
        rep.reanneal(reanneal_profile(S_RE), "backbone", target=target, stream=stream)
    be = rep.best_energy(stream=stream)
    return rep, be


def bench_batch(nmc, torch, seed, n_instances=256, tune_sweeps=2):
    """Batched NMC on mixed k-SAT instances (256 by default; k in {3,4}, N
    log-uniform in [1000, 20000], replicas 64..512 by N) in one graph-captured
    plan, against plain simulated annealing launched once per instance."""
    S_A, RND, S_R, CHUNK = 1000, 2, 500, 50
    S_TOT = S_A + RND * S_R
    mix = instances.batch_mix(256, seed)[:n_instances]
    insts = []
    for m in mix:
        cp, lits = instances.gen_ksat(m["n"], m["alpha"], m["k"], m["seed"])
        insts.append(nmc.Instance.ksat(m["n"], cp, lits, 0).bind())
    sa_beta = instances.linear_schedule(BETA0, BETA1, S_TOT)
    a_beta = instances.linear_schedule(BETA0, BETA1, S_A)
    r_beta = instances.profile_schedule(np.full(S_R, BETA1), instances.linear_schedule(BETA_HOT, BETA1, S_R))
    attempts = float(sum(m["replicas"] * m["n"] for m in mix)) * S_TOT

    def make(offset):
        return [nmc.Replicas(inst, m["replicas"], m["seed"] + offset) for inst, m in zip(insts, mix)]

    # targets: 10th percentile of a calibration plain-SA run (other seeds)
    cal = make(7777)
    cb = nmc.Batch(cal)
    cb.tune(tune_sweeps)
    cb.anneal(sa_beta[None, :])
    targets = np.array([int(np.percentile(s.best_energy()["energy"], 10)) for s in cal], np.int64)
    cb.free()
    del cal

    out = {"instances": len(mix), "attempts": attempts, "sweeps": S_TOT, "chunk_sweeps": CHUNK}

    # (1) plain SA, one launch per instance
    sets = make(0)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ttt = []
    for s, tg in zip(sets, targets):
        t0 = time.perf_counter()
        s.anneal(sa_beta[None, :], target=int(tg))
        fh = s.best_energy()["first_hit"]
        t1 = time.perf_counter()
        hit = fh[fh >= 0]
        ttt.append((t0 - t_start) + (float(hit.min()) / S_TOT) * (t1 - t0) if hit.size else None)
    wall = time.perf_counter() - t_start
    out["per_instance_sa"] = summarize(wall, attempts, ttt)
    del sets

    # (2) plain SA, all instances in one batched launch sequence (lockstep chunks)
    sets = make(0)
    bt = nmc.Batch(sets)
    block = bt.tune(tune_sweeps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.run_plan(sa_beta, 0, r_beta, 9, 10, True, targets=targets, use_graph=True, chunk_sweeps=CHUNK)
    wall = time.perf_counter() - t0
    out["batched_sa"] = summarize(wall, attempts, [None if (fh := s.best_energy()["first_hit"])[fh >= 0].size == 0
                                                   else float(fh[fh >= 0].min()) / S_TOT * wall for s in sets])
    out["batched_sa"]["block_threads"] = block
    out["batched_sa"]["sets_with_8_replicas_per_workgroup"] = sum(1 for s in sets if s.replicas_per_workgroup() == 8)
    bt.free()
    del sets

    # (3) NMC, all instances in one graph: anneal -> 2 x (backbone -> reanneal)
    sets = make(0)
    bn = nmc.Batch(sets)
    bn.tune(tune_sweeps)  # workgroup size and, per set, 4 or 8 replicas per workgroup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bn.run_plan(a_beta, RND, r_beta, 9, 10, True, targets=targets, use_graph=True, chunk_sweeps=CHUNK)
    wall = time.perf_counter() - t0
    out["batched_nmc"] = summarize(wall, attempts, [None if (fh := s.best_energy()["first_hit"])[fh >= 0].size == 0
                                                    else float(fh[fh >= 0].min()) / S_TOT * wall for s in sets])
    bn.free()
    per, bnm, bsa = out["per_instance_sa"], out["batched_nmc"], out["batched_sa"]
    out["ttt"] = {"rule": "seconds until every instance has a replica at or below its target (10th percentile of "
                          "a calibration plain-SA run); one launch per instance is plain SA",
                  "per_instance_sa_s": per["ttt_all_s"], "batched_sa_s": bsa["ttt_all_s"],
                  "batched_nmc_s": bnm["ttt_all_s"],
                  "batched_nmc_speedup": (per["ttt_all_s"] / bnm["ttt_all_s"]
                                          if per["ttt_all_s"] and bnm["ttt_all_s"] else None)}
    return out


def qap_beta_scale(F, D, seed, samples=100000):
    """1 / median positive swap cost change over random (assignment, pair)
    samples: the schedule's inverse temperatures are given in these units."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = F.shape[0]
    F = F.astype(np.int64)
    D = D.astype(np.int64)
    p = np.argsort(rng.random((samples, n)), axis=1)
    a = rng.integers(0, n, samples)
    b = (a + 1 + rng.integers(0, n - 1, samples)) % n
    rows = np.arange(samples)[:, None]
    fa, fb = F[a], F[b]
    pa, pb = p[np.arange(samples), a], p[np.arange(samples), b]
    d = 2 * ((fa - fb) * (D[pb[:, None], p] - D[pa[:, None], p])).sum(1)
    d = d[d > 0]
    return 1.0 / float(np.median(d))


def bench_qap(nmc, torch, seed, sweeps_only=0, sweeps_offset=0, curve=0):
    """QAP NMC: n = 100, 4096 replicas, anneal 5000 sweeps of 4950 proposed
    swaps, then 2 x (frequency backbone -> reanneal 1000).  curve > 0: the
    same schedule in launches of `curve` sweeps, each with its acceptance
    rate and kernel rate (the rate-versus-acceptance curve)."""
    n, Rq, S_A, RND, S_R = 100, 4096, 5000, 2, 1000
    F, D = instances.gen_qap(n, seed)
    sc = qap_beta_scale(F, D, seed + 1)
    inst = nmc.Instance.qap(F, D).bind()
    a_beta = instances.linear_schedule(BETA0 * sc, BETA1 * sc, S_A)
    r_beta = instances.profile_schedule(np.full(S_R, BETA1 * sc), instances.linear_schedule(BETA_HOT * sc, BETA1 * sc, S_R))
    rep = nmc.Replicas(inst, Rq, seed)
    rep.set_profiling(True)
    pairs = n * (n - 1) // 2
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    segments = []

    def seg(beta, profile, start):
        # one launch; its acceptance and kernel rate
        rep.kernel_time(reset=True)
        rep.accept_count(reset=True)
        if profile:
            rep.reanneal(beta, "backbone")
        else:
            rep.anneal(beta)
        k = rep.kernel_time()
        segments.append({"sweep": start, "sweeps": beta.shape[-1],
                         "beta_units": float(np.atleast_2d(beta)[-1].mean() / sc),
                         "acceptance": rep.accept_count() / (float(Rq) * pairs * beta.shape[-1]),
                         "kernel_G_per_s": k["attempts"] / (k["ms"] / 1e3) / 1e9, "kernel_ms": k["ms"]})
        return k

    if sweeps_only:
        rep.anneal(a_beta[None, sweeps_offset:sweeps_offset + sweeps_only])
        S_tot = min(sweeps_only, max(0, S_A - sweeps_offset))
    elif curve:
        ms = 0.0
        for s0 in range(0, S_A, curve):
            ms += seg(a_beta[None, s0:s0 + curve], False, s0)["ms"]
        for r in range(RND):
            rep.estimate_backbone_device(9, 10, False)
            for s0 in range(0, S_R, curve):
                ms += seg(r_beta[:, s0:s0 + curve], True, S_A + r * S_R + s0)["ms"]
        S_tot = S_A + RND * S_R
    else:
        rep.anneal(a_beta[None, :])
        for _ in range(RND):
            rep.estimate_backbone_device(9, 10, False)
            rep.reanneal(r_beta, "backbone")
        S_tot = S_A + RND * S_R
    be = rep.best_energy()
    wall = time.perf_counter() - t0
    if curve:
        kt = {"ms": sum(x["kernel_ms"] for x in segments), "launches": len(segments),
              "attempts": float(Rq) * pairs * S_tot}
        accepted = sum(x["acceptance"] * float(Rq) * pairs * x["sweeps"] for x in segments)
    else:
        kt = rep.kernel_time()
        accepted = rep.accept_count()
    props = float(Rq) * pairs * S_tot
    kps = kt["attempts"] / (kt["ms"] / 1000.0)
    # LDS byte reads per proposal: F[b][k] and the gather D[p_b][p_k] for every k
    # but a, b; peak: 32 banks per CU served per clock
    reads = 2.0 * (n - 2)
    achieved = kps * reads
    roofline = {"bound": "lds", "achieved": achieved / 1e12, "peak": LDS_LANE_READS / 1e12,
                "unit": "T lane-reads/s", "frac": achieved / LDS_LANE_READS, "traffic": None,
                "kernel": "qap_sweep_kernel", "kernel_ms_per_launch": kt["ms"] / max(1, kt["launches"]),
                "launches": kt["launches"],
                # the scope table's model: ~3(n - 2) LDS lane-accesses per proposal
                # (98 permutation bytes + 196 distance gathers at n = 100) against
                # one lane access per bank per clock: about 67 G proposals/s
                "survey_bound_proposals_per_s": LDS_LANE_READS / (3.0 * (n - 2)),
                "survey_frac": kps * 3.0 * (n - 2) / LDS_LANE_READS}
    if not sweeps_only:
        peaks = measured_peaks(nmc, torch)
        roofline["frac_of_measured_lds_distinct"] = roofline["achieved"] / peaks["lds_distinct_T_per_s"]
        roofline["frac_of_measured_lds_random"] = roofline["achieved"] / peaks["lds_random_T_per_s"]
        roofline["measured_peaks"] = peaks
    return {"proposals": props, "wall_s": wall, "proposals_per_s": props / wall,
            "kernel_ms": kt["ms"], "kernel_proposals_per_s": kps, "roofline": roofline,
            "acceptance": accepted / props, "beta_unit": sc, "best_cost": be["best"], "sweeps": S_tot,
            "curve": segments or None}


LBP_CFG = dict(beta=1.0, lambda0=4.0, lambda_ratio=0.8, lambda_min=1e-3, max_iter=100, tol=1e-8, p_min=-2.0)
LBP_THRESHOLDS = ((0.8, 0.6), (0.9, 0.8), (0.95, 0.9))  # (seed, cutoff) per round, raised round by round
# bytes one message iteration must move per literal slot (edge): each
# message read by the variable side, read and written by the clause side, the
# field total T gathered by the clause side (8 B each), the edge's
# variable-major position and the clause's literal address (4 B each); per
# variable: clause range, reference spin, T written.  (The library's second,
# variable-major copy of the messages adds an 8-byte scattered write per edge
# that this count leaves out.)
LBP_BYTES_PER_EDGE, LBP_BYTES_PER_VAR = 40, 13


def bench_lbp(nmc, torch, seed):
    """NMC with the paper's backbone estimator on the N = 50,000 instance:
    anneal 2000 sweeps (beta 0.1 -> 4.0), then 3 rounds of [LBP on the
    surrogate Hamiltonian around the best state of the best replica ->
    connected backbone (thresholds raised each round) -> reanneal 1000
    sweeps, backbone hot]."""
    cp, lits = instances.gen_ksat(N, ALPHA, K, seed)
    inst = nmc.Instance.ksat(N, cp, lits, CLASS_CAP).bind()
    M = inst.info.n_clauses

    def path(profile):
        rep = nmc.Replicas(inst, R, seed)
        rep.set_profiling(profile)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep.anneal(instances.linear_schedule(BETA0, BETA1, S_ANNEAL)[None, :])
        rounds, t_lbp = [], 0.0
        for ts, tc in LBP_THRESHOLDS:
            r0 = int(np.argmin(rep.best_energy()["best_per_replica"]))
            t1 = time.perf_counter()
            g = rep.lbp_backbone(r0, "best", **LBP_CFG, theta_seed=ts, theta_cut=tc)
            t_lbp += time.perf_counter() - t1
            rounds.append({k: g[k] for k in ("lambda", "steps", "iterations", "converged", "overlap", "self_overlap",
                                             "backbone_size", "n_clusters", "largest_cluster")})
            rounds[-1]["label"] = g["label"]
            rep.reanneal(reanneal_profile(S_RE), "backbone")
        be = rep.best_energy()
        torch.cuda.synchronize()
        return rep, rounds, be, time.perf_counter() - t0, t_lbp

    path(False)  # warm-up
    rep, rounds, be, wall, t_lbp = path(False)
    # whitening of every replica's best state (section on whitening): frozen
    # cores of the NMC-with-LBP states against plain SA over the same sweeps
    def whiten(r):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fz, _, passes = r.whiten("best")
        torch.cuda.synchronize()
        bpr = r.best_energy()["best_per_replica"]
        top = int(np.argmin(bpr))
        return {"seconds": time.perf_counter() - t0, "passes": passes, "replicas_with_frozen": int((fz > 0).sum()),
                "frozen_max": int(fz.max()), "frozen_mean": float(fz.mean()), "best_replica_energy": int(bpr[top]),
                "best_replica_frozen": int(fz[top])}
    white_nmc = whiten(rep)
    # one collective-move sweep over the last round's clusters (the scheme's
    # nonlocal move), timed on its own, at the cold beta and at beta_hot
    cflip = {}
    for b in (BETA1, BETA_HOT):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        acc = rep.cluster_flip(rounds[-1]["label"], b)
        torch.cuda.synchronize()
        cflip[f"beta_{b:g}"] = {"seconds": time.perf_counter() - t0, "clusters": rounds[-1]["n_clusters"],
                                "flips_mean": float(acc.mean()), "replicas_with_flips": int((acc > 0).sum())}
    for r in rounds:
        r.pop("label")
    sa = nmc.Replicas(inst, R, seed)
    sa.anneal(instances.linear_schedule(BETA0, BETA1, S_ANNEAL + ROUNDS * S_RE)[None, :])
    white_sa = whiten(sa)
    white_sa["best_energy"] = sa.best_energy()["best"]
    del sa
    prep, _, _, _, _ = path(True)
    kt = prep.kernel_time()
    lt = prep.lbp_kernel_time()
    edges, nvar = 4 * M, N
    bytes_it = LBP_BYTES_PER_EDGE * edges + LBP_BYTES_PER_VAR * nvar
    ms_it = lt["ms"] / max(1, lt["iterations"])
    att = float(R) * N * (S_ANNEAL + ROUNDS * S_RE)
    roofline = ksat_roofline(kt, M, prep.accept_count() / att)
    lbp_roofline = {"bound": "hbm", "achieved": bytes_it / (ms_it / 1000.0) / 1e9, "peak": 8000.0, "unit": "GB/s",
                    "frac": bytes_it / (ms_it / 1000.0) / 8e12, "traffic": None,
                    "kernel": "lbp_var_kernel + lbp_clause_kernel (one message iteration)",
                    "ms_per_iteration": ms_it, "bytes_per_iteration": bytes_it, "iterations": lt["iterations"]}
    return {"attempts": att, "wall_s": wall, "attempts_per_s": att / wall, "lbp_s": t_lbp,
            "lbp_share": t_lbp / wall, "rounds": rounds, "best_energy": be["best"], "roofline": roofline,
            "lbp_roofline": lbp_roofline, "whitening_nmc_lbp": white_nmc, "whitening_plain_sa": white_sa,
            "cluster_flip": cflip}


ALG1_BETA_FIRST, ALG1_PT_ROUNDS, ALG1_SEED_REPLICAS = 2.5, 1000, 64
ALG1_THRESHOLDS = ((0.9, 0.8), (0.95, 0.9))
ALG1_RE, ALG1_UNLEARN = 1000, 500


def bench_alg1(nmc, torch, seed):
    """Algorithm 1 end to end on the N = 50,000 instance: adaptive replica
    exchange over the whole problem (64 temperatures x 16 chains: the ladder
    from beta 2.5, then 1000 one-sweep rounds), the coldest replica of every
    chain as a seed, and for each of the 16 seeds a set of 64 replicas
    started at it; per round every set estimates the LBP backbone around its
    best replica (one batched LBP call for all sets), then all sets run one
    batched launch of inhomogeneous MC
    (backbone hot 0.5 -> 4.0, rest at 4.0) and one of homogeneous unlearning
    at 4.0.  Plain SA over the same sweeps per replica is timed beside it."""
    cp, lits = instances.gen_ksat(N, ALPHA, K, seed)
    inst = nmc.Instance.ksat(N, cp, lits, CLASS_CAP).bind()
    Rp = APT_TEMPS * APT_CHAINS

    def run():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        apt = nmc.Replicas(inst, Rp, seed)
        betas, _ = apt.apt_ladder(ALG1_BETA_FIRST, APT_ALPHA, 0.0, APT_EQUIL, APT_MEAS, APT_TEMPS)
        acc, att = apt.pt_run(betas, ALG1_PT_ROUNDS, 1)
        x = apt.get_state("current")
        cold = slice((APT_TEMPS - 1) * APT_CHAINS, APT_TEMPS * APT_CHAINS)
        seeds_e = apt.best_energy()["energy"][cold]
        seeds = x[cold]
        t_apt = time.perf_counter() - t0
        sets = []
        for k in range(APT_CHAINS):
            rs = nmc.Replicas(inst, ALG1_SEED_REPLICAS, seed + 100 + k)
            rs.set_state(np.repeat(seeds[k][None, :], ALG1_SEED_REPLICAS, 0), apt.sweeps_done())
            sets.append(rs)
        del apt
        batch = nmc.Batch(sets)
        rounds, t_lbp = [], 0.0
        for ts, tc in ALG1_THRESHOLDS:
            t1 = time.perf_counter()
            # the seeds' LBP runs advance together: one grid per kernel for all sets
            seeds_r = [int(np.argmin(rs.best_energy()["best_per_replica"])) for rs in sets]
            sizes = [g["backbone_size"] for g in batch.lbp_backbone(seeds_r, "best", **LBP_CFG, theta_seed=ts,
                                                                     theta_cut=tc)]
            t_lbp += time.perf_counter() - t1
            batch.anneal(reanneal_profile(ALG1_RE), "backbone")
            batch.anneal(np.full((1, ALG1_UNLEARN), BETA1))
            rounds.append({"thresholds": [ts, tc], "backbone_min": int(min(sizes)), "backbone_max": int(max(sizes)),
                           "best": int(min(rs.best_energy()["best"] for rs in sets))})
        best = min(rs.best_energy()["best"] for rs in sets)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return {"wall_s": wall, "apt_s": t_apt, "lbp_s": t_lbp, "seed_energies": seeds_e.tolist(),
                "exchange_rate_mean": float((acc / np.maximum(att, 1)).mean()), "ladder_last_beta": float(betas[-1]),
                "rounds": rounds, "best_energy": int(best)}

    run()  # warm-up
    res = run()
    sweeps = APT_TEMPS * (APT_EQUIL + APT_MEAS) + ALG1_PT_ROUNDS + len(ALG1_THRESHOLDS) * (ALG1_RE + ALG1_UNLEARN)
    att = float(Rp) * N * sweeps
    sa = nmc.Replicas(inst, Rp, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sa.anneal(instances.linear_schedule(BETA0, BETA1, sweeps)[None, :])
    sa_best = sa.best_energy()["best"]
    torch.cuda.synchronize()
    res.update({"sweeps_per_replica": sweeps, "attempts": att, "attempts_per_s": att / res["wall_s"],
                "plain_sa": {"best_energy": int(sa_best), "wall_s": time.perf_counter() - t0}})
    return res


APT_TEMPS, APT_CHAINS, APT_BETA_FIRST, APT_ALPHA = 64, 16, 1.5, 1.1
APT_EQUIL, APT_MEAS, APT_ROUNDS = 20, 5, 2000


def bench_apt_qap(nmc, torch, seed, rounds=500):
    """Tempering on the n = 100 QAP: 4096 replicas as 64 temperatures x 64
    chains (a sweep workgroup's 16 replicas share a temperature), the
    adaptive ladder from beta = 1.5 (in units of 1 / median |dC|), then
    `rounds` rounds of one sweep and one exchange step."""
    n = 100
    F, D = instances.gen_qap(n, seed)
    sc = qap_beta_scale(F, D, seed + 1)
    inst = nmc.Instance.qap(F, D).bind()
    chains = 4096 // APT_TEMPS
    rep = nmc.Replicas(inst, APT_TEMPS * chains, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    betas, sigmas = rep.apt_ladder(1.5 * sc, APT_ALPHA, 0.0, APT_EQUIL, APT_MEAS, APT_TEMPS)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    acc, att = rep.pt_run(betas, rounds, 1)
    be = rep.best_energy()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    props = float(APT_TEMPS * chains) * n * (n - 1) / 2
    rate = acc / np.maximum(att, 1)
    return {"replicas": APT_TEMPS * chains, "chains": chains, "ladder_s": t1 - t0, "pt_s": t2 - t1,
            "ladder_proposals_per_s": props * APT_TEMPS * (APT_EQUIL + APT_MEAS) / (t1 - t0),
            "pt_proposals_per_s": props * rounds / (t2 - t1), "rounds": rounds,
            "ladder": {"beta_first_units": 1.5, "beta_last_units": float(betas[-1] / sc),
                       "sigma_first": float(sigmas[0]), "sigma_last": float(sigmas[-1])},
            "exchange_rate": {"min": float(rate.min()), "mean": float(rate.mean()), "max": float(rate.max())},
            "best_cost": int(be["best"])}


def bench_apt(nmc, torch, seed, rounds, sweeps_per_round):
    """Adaptive parallel tempering on the N = 50,000 4-SAT instance: the
    adaptive ladder (64 positions from beta 1.5, alpha 1.1, 20 + 5 sweeps per
    position) built on the 1024 replicas, then `rounds` rounds of
    [sweeps_per_round sweeps at every position -> one exchange step] over 16
    chains."""
    cp, lits = instances.gen_ksat(N, ALPHA, K, seed)
    inst = nmc.Instance.ksat(N, cp, lits, CLASS_CAP).bind()
    M = inst.info.n_clauses
    Rp = APT_TEMPS * APT_CHAINS

    def step(profile):
        rep = nmc.Replicas(inst, Rp, seed)
        rep.set_profiling(profile)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        betas, sigmas = rep.apt_ladder(APT_BETA_FIRST, APT_ALPHA, 0.0, APT_EQUIL, APT_MEAS, APT_TEMPS)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        acc, att = rep.pt_run(betas, rounds, sweeps_per_round)
        be = rep.best_energy()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return rep, betas, sigmas, acc, att, be, t1 - t0, t2 - t1

    step(False)  # warm-up
    rep, betas, sigmas, acc, att, be, t_ladder, t_pt = step(False)
    ladder_sweeps = len(betas) * (APT_EQUIL + APT_MEAS)
    pt_sweeps = rounds * sweeps_per_round
    att_ladder = float(Rp) * N * ladder_sweeps
    att_pt = float(Rp) * N * pt_sweeps
    # sweep-kernel time of the tempering rounds from HIP events (separate pass)
    prep = nmc.Replicas(inst, Rp, seed)
    prep.anneal(np.full((1, 50), betas[0]))
    prep.accept_count(reset=True)
    prep.set_profiling(True)
    prep.pt_run(betas, min(rounds, 500), sweeps_per_round)
    kt = prep.kernel_time()
    rate = acc / np.maximum(att, 1)
    roofline = ksat_roofline(kt, M, prep.accept_count() / (float(Rp) * N * min(rounds, 500) * sweeps_per_round))
    qap = bench_apt_qap(nmc, torch, seed)
    return {"attempts": att_ladder + att_pt, "wall_s": t_ladder + t_pt, "qap": qap,
            "attempts_per_s": (att_ladder + att_pt) / (t_ladder + t_pt),
            "ladder_s": t_ladder, "ladder_attempts_per_s": att_ladder / t_ladder,
            "pt_s": t_pt, "pt_attempts_per_s": att_pt / t_pt, "pt_rounds_per_s": rounds / t_pt,
            "sweep_kernel_share_of_pt": kt["ms"] / 1000.0 * rounds / min(rounds, 500) / t_pt,
            "ladder": {"positions": len(betas), "beta_first": float(betas[0]), "beta_last": float(betas[-1]),
                       "sigma_first": float(sigmas[0]), "sigma_last": float(sigmas[-1])},
            "exchange_rate": {"min": float(rate.min()), "mean": float(rate.mean()), "max": float(rate.max())},
            "best_energy": be["best"], "roofline": roofline, "rounds": rounds,
            "sweeps_per_round": sweeps_per_round, "replicas": Rp, "chains": APT_CHAINS}


SERVE_RATE, SERVE_SECONDS, SERVE_BUDGET_S = 50.0, 60.0, 2.0
# the default run's short versions of the served, batched and C1 workloads
SHORT_SERVE_SECONDS = 8.0
SHORT_BATCH_INSTANCES = 64
C1_REPEATS = 20
SERVE_SCHED = (150, 2, 50)  # anneal sweeps, rounds, reanneal sweeps per request
SERVE_CHUNK = 25
SERVE_KSAT_GRID = (2000, 4500, 10000, 22400, 50000)
SERVE_QAP_GRID = (30, 60, 90, 120, 150)


def _serve_gen(m):
    if m["kind"] == "ksat":
        return instances.gen_ksat(m["n"], m["alpha"], m["k"], m["seed"])
    return instances.gen_qap(m["n"], m["seed"])


def _qap_random_cost(F, D):
    """Mean cost over uniformly random assignments."""
    n = F.shape[0]
    return float(F.astype(np.float64).sum()) * float(D.astype(np.float64).sum()) / (n * (n - 1))


def serve_calibration(nmc, seed):
    """Targets by request size: plain SA over the request's sweep total on one
    calibration instance per grid size; k-SAT keeps the 10th-percentile final
    energy per variable, QAP the 10th-percentile final cost relative to the
    random-assignment mean, and its inverse-temperature scale."""
    S = sum((SERVE_SCHED[0], SERVE_SCHED[1] * SERVE_SCHED[2]))
    sa = instances.linear_schedule(BETA0, BETA1, S)
    sets, kinfo, qinfo = [], [], []
    for i, n in enumerate(SERVE_KSAT_GRID):
        cp, lits = instances.gen_ksat(n, "9.7", 4, seed + 500 + i)
        inst = nmc.Instance.ksat(n, cp, lits).bind()
        sets.append(nmc.Replicas(inst, instances.serve_ksat_replicas(n), seed + 600 + i))
    kb = nmc.Batch(sets)
    kb.anneal(sa[None, :])
    for n, rep in zip(SERVE_KSAT_GRID, sets):
        kinfo.append(float(np.percentile(rep.best_energy()["energy"], 10)) / n)
    kb.free()
    for i, n in enumerate(SERVE_QAP_GRID):
        F, D = instances.gen_qap(n, seed + 700 + i)
        sc = qap_beta_scale(F, D, seed + 800 + i, samples=20000)
        rep = nmc.Replicas(nmc.Instance.qap(F, D).bind(), 256, seed + 900 + i)
        rep.anneal(sa[None, :] * sc)
        qinfo.append((float(np.percentile(rep.best_energy()["energy"], 10)) / _qap_random_cost(F, D), sc))
    return {"ksat_density": kinfo, "qap_ratio": [q[0] for q in qinfo], "qap_beta_scale": [q[1] for q in qinfo]}


def serve_requests(seed, seconds, procs=16):
    """The request stream and its instances, generated by `procs` worker
    processes (in this process when procs <= 1).  The pool must be created
    before anything in the process touches the GPU: a process that has
    initialised HIP must not fork.  Under a profiler, whose library every
    forked child inherits, pass procs = 0."""
    mix = instances.serve_mix(SERVE_RATE, seconds, seed)
    procs = min(procs, os.cpu_count() or 1)
    if procs <= 1:
        return mix, [_serve_gen(m) for m in mix]
    from multiprocessing import get_context

    with get_context("fork").Pool(procs) as pool:
        data = pool.map(_serve_gen, mix, chunksize=8)
    return mix, data


def bench_serve(nmc, torch, seed, seconds, pre, n_cap=400):
    """Served NMC: a Poisson stream of k-SAT and QAP requests (`pre`, from
    serve_requests) into the continuous-batching server; latency from
    submission to the round end where the request reached its target."""
    cal = serve_calibration(nmc, seed)
    mix, data = pre
    lk = np.log(np.asarray(SERVE_KSAT_GRID, np.float64))
    reqs = []
    for m, d in zip(mix, data):
        if m["kind"] == "ksat":
            dens = float(np.interp(np.log(m["n"]), lk, cal["ksat_density"]))
            reqs.append((m, d, int(np.floor(dens * m["n"])), 1.0))
        else:
            F, D = d
            ratio = float(np.interp(m["n"], SERVE_QAP_GRID, cal["qap_ratio"]))
            sc = float(np.interp(m["n"], SERVE_QAP_GRID, cal["qap_beta_scale"]))
            reqs.append((m, d, int(np.floor((1.0 + 1e-2) * ratio * _qap_random_cost(F, D))), sc))
    del data
    a, rounds, re = SERVE_SCHED
    loaders = max(2, min(12, (os.cpu_count() or 8) - 4))

    def submit(srv, m, d, target, sc):
        if m["kind"] == "ksat":
            cp, lits = d
            return srv.submit_ksat(m["n"], cp, lits, m["replicas"], m["seed"], BETA0, BETA1, BETA_HOT, a, rounds,
                                   re, target=target, budget_s=SERVE_BUDGET_S)
        F, D = d
        return srv.submit_qap(F, D, m["replicas"], m["seed"], BETA0 * sc, BETA1 * sc, BETA_HOT * sc, a, rounds, re,
                              target=target, budget_s=SERVE_BUDGET_S)

    # capacity: the first requests of the stream submitted at once (closed loop)
    n_cap = min(len(reqs), n_cap)
    srv = nmc.Server(chunk_sweeps=SERVE_CHUNK, loader_threads=loaders)
    cap_ids = [submit(srv, *q) for q in reqs[:n_cap]]
    srv.wait_idle(300.0)
    cap_res = [srv.poll(i) for i in cap_ids]
    srv.free()
    cap_wall = max(r["t_done"] for r in cap_res) - min(r["t_submit"] for r in cap_res)
    capacity = n_cap / cap_wall
    print(f"# serve: capacity {capacity:.1f} requests/s ({n_cap} at once)", file=sys.stderr, flush=True)

    srv = nmc.Server(chunk_sweeps=SERVE_CHUNK, loader_threads=loaders)
    ids = []
    t_start = time.perf_counter()
    for q in reqs:
        delay = q[0]["arrival"] - (time.perf_counter() - t_start)
        if delay > 0:
            time.sleep(delay)
        ids.append(submit(srv, *q))
        if len(ids) % 500 == 0:
            print(f"# serve: {len(ids)} submitted, {srv.stats()['completed']} completed", file=sys.stderr, flush=True)
    drained = srv.wait_idle(300.0)
    res = [srv.poll(i) for i in ids]
    stats = srv.stats()
    srv.free()
    t0 = min(r["t_submit"] for r in res)
    wall = max(r["t_done"] for r in res) - t0

    def pct(xs):
        return {"p50": float(np.percentile(xs, 50)), "p99": float(np.percentile(xs, 99))} if xs else None

    out = {"requests": len(res), "offered_rate_per_s": SERVE_RATE, "seconds": seconds, "drained": drained,
           "capacity_requests_per_s": capacity, "offered_load": len(res) / seconds / capacity,
           "schedule": {"anneal": a, "rounds": rounds, "reanneal": re, "chunk_sweeps": SERVE_CHUNK,
                        "budget_s": SERVE_BUDGET_S},
           "wall_s": wall, "gpu_busy_s_summed_over_workers": stats["gpu_busy_s"], "rounds": stats["rounds"],
           "calibration": cal}
    attempts = 0.0
    for kind in ("ksat", "qap", "all"):
        sel = [(m, r) for (m, _, _, _), r in zip(reqs, res) if kind == "all" or m["kind"] == kind]
        solved = [r for _, r in sel if r["status"] == "solved"]
        counts = {}
        for _, r in sel:
            counts[r["status"]] = counts.get(r["status"], 0) + 1
        out[kind] = {"requests": len(sel), "status": counts, "solves_per_s": len(solved) / wall,
                     "time_to_target_s": pct([r["t_done"] - r["t_submit"] for r in solved]),
                     "latency_s": pct([r["t_done"] - r["t_submit"] for _, r in sel]),
                     "queueing_s": pct([r["t_admit"] - r["t_submit"] for _, r in sel if r["t_admit"] > 0])}
        if kind != "all":
            for m, r in sel:
                per = m["n"] if kind == "ksat" else m["n"] * (m["n"] - 1) / 2
                attempts += float(m["replicas"]) * per * r["sweeps_done"]
    out["moves_per_s"] = attempts / wall
    return out


def bench_c1(nmc, torch, seed, repeats=1):
    """Plain SA on random 4-SAT N = 200, M = 1920, 64 replicas, 1000 sweeps
    (beta 0.1 -> 4.0): the latency of the whole anneal, and the rate per
    busy CU (16 workgroups of 4 replicas) against one CU's LDS read bound
    ((3 deg + 1) / 4 byte reads per attempt, 32 lane reads per clock)."""
    n, alpha, R, S = 200, "9.6", 64, 1000
    cp, lits = instances.gen_ksat(n, alpha, K, seed)
    inst = nmc.Instance.ksat(n, cp, lits).bind()
    m = len(cp) - 1
    sched = instances.linear_schedule(BETA0, BETA1, S)[None, :]
    warm = nmc.Replicas(inst, R, seed + 1)
    warm.anneal(sched[:, :20])
    walls, kms = [], []
    for k in range(repeats):
        # one solve: fresh replicas (own seed), the whole anneal, the best energy
        rep = nmc.Replicas(inst, R, seed + 10 * k)
        rep.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep.anneal(sched)
        be = rep.best_energy()
        walls.append(time.perf_counter() - t0)
        kms.append(rep.kernel_time()["ms"])
        if k == 0:
            be0, kt = be, rep.kernel_time()
        del rep
    be = be0
    wall = walls[0]
    att = float(R) * n * S
    groups = (R + 3) // 4
    deg = K * m / n
    per_cu = att / (kt["ms"] / 1e3) / groups
    cu_bound = 32 * 2.4e9 / ((3 * deg + 1) / 4)
    return {"n_vars": n, "n_clauses": m, "replicas": R, "sweeps": S, "colors": inst.info.n_colors,
            "latency_ms": kt["ms"], "wall_ms": wall * 1e3, "attempts_per_s": att / (kt["ms"] / 1e3),
            "busy_cus": groups, "per_cu_attempts_per_s": per_cu, "cu_lds_bound_attempts_per_s": cu_bound,
            "frac_of_one_cu": per_cu / cu_bound, "best_energy": int(be["best"]),
            "repeats": repeats,
            "latency_p50_ms": float(np.percentile(kms, 50)), "latency_p99_ms": float(np.percentile(kms, 99)),
            "wall_p50_ms": float(np.percentile(walls, 50)) * 1e3, "wall_p99_ms": float(np.percentile(walls, 99)) * 1e3,
            "latency_rule": "kernel time of one solve's sweep launch (HIP events); wall = call to best energy "
                            "read back, per solve with fresh replicas"}


def bench_wide(nmc, torch, seed):
    """The NMC path on a random 4-SAT instance too large for the LDS layout
    (the wide layout: spins variable-major in device memory, one launch per
    colour class): N = 1,000,000, alpha 9.9 (M = 9.9 M clauses), no class cap,
    1024 replicas, anneal 200 + 2 x (backbone + reanneal 100) sweeps.  Whole
    path by the host clock, sweep launches by HIP events, the energy recount
    (tables packed, then counted) by the host clock."""
    n, S_A, RND, S_RW = 1_000_000, 200, 2, 100
    cp, lits = instances.gen_ksat(n, ALPHA, K, seed)
    inst = nmc.Instance.ksat(n, cp, lits, 0).bind()
    warm = nmc.Replicas(inst, R, seed + 1)
    warm.anneal(instances.linear_schedule(BETA0, BETA1, S_A)[None, :2])
    warm.recount()
    del warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = nmc.Replicas(inst, R, seed)
    rep.set_profiling(True)
    rep.anneal(instances.linear_schedule(BETA0, BETA1, S_A)[None, :])
    for _ in range(RND):
        rep.estimate_backbone_device(9, 10, True)
        rep.reanneal(reanneal_profile(S_RW), "backbone")
    be = rep.best_energy()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = rep.kernel_time()
    t0 = time.perf_counter()
    e = rep.recount()
    rc_s = time.perf_counter() - t0
    att = float(R) * n * (S_A + RND * S_RW)
    return {"n_vars": n, "n_clauses": inst.info.n_clauses, "replicas": R, "colors": inst.info.n_colors,
            "wide": inst.info.wide, "sweeps": S_A + RND * S_RW, "wall_s": wall, "attempts_per_s": att / wall,
            "kernel_ms": kt["ms"], "kernel_attempts_per_s": kt["attempts"] / (kt["ms"] / 1e3),
            "ms_per_sweep": kt["ms"] / (S_A + RND * S_RW), "recount_s": rc_s,
            "recount_equals_tracked_energy": bool((e == be["energy"]).all()),
            "best_energy": int(be["best"]), "accepted": rep.accept_count()}


def measured_peaks(nmc, torch):
    """Rates that simple, fully occupied kernels reach on this GPU, beside the
    published peaks: LDS byte reads (lanes on distinct banks, and random
    addresses in 100 KB), 32-bit integer adds, and a 1 GiB
    device-to-device copy (bytes read + written)."""
    out = {}
    for which, iters, blocks in (("lds_distinct", 16384, 1024), ("lds_random", 4096, 1024),
                                 ("valu_int", 16384, 2048)):
        nmc.probe_peak(which, 64, blocks)  # warm-up
        ms, ops = nmc.probe_peak(which, iters, blocks)
        out[which + "_T_per_s"] = ops / (ms / 1e3) / 1e12
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    out["hbm_copy_TB_per_s"] = 5 * 2 * a.numel() * 4 / (e0.elapsed_time(e1) / 1e3) / 1e12
    del a, b
    return out


def summarize(wall, attempts, ttt):
    hit = [t for t in ttt if t is not None]
    return {"wall_s": wall, "attempts_per_s": attempts / wall, "instances_hit": len(hit),
            "ttt_all_s": max(hit) if len(hit) == len(ttt) else None,
            "ttt_median_s": float(np.median(hit)) if hit else None}


def cpu_baseline(cp, lits, seed):
    import oracle

    threads = max(1, min(16, os.cpu_count() or 1))
    ok = oracle.KSat(N, cp, lits)
    _, order, _ = ok.color(CLASS_CAP)
    Rs = 4 * threads
    rep = oracle.KSatReplicas(ok, Rs, seed, order, threads=threads, snapshot=True)
    sweeps = 48  # about 10-30 s of host work
    t0 = time.perf_counter()
    rep.anneal(instances.linear_schedule(BETA0, BETA1, S_ANNEAL)[None, :sweeps])
    dt = time.perf_counter() - t0
    att = Rs * N * sweeps
    # the same oracle on one thread: 4 replicas (one group), 8 sweeps
    one = oracle.KSatReplicas(ok, 4, seed, order, threads=1, snapshot=True)
    t0 = time.perf_counter()
    one.anneal(instances.linear_schedule(BETA0, BETA1, S_ANNEAL)[None, :8])
    dt1 = time.perf_counter() - t0
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": att / dt, "unit": "attempts/s", "cores": threads, "kind": "oracle",
            "single_thread_value": 4 * N * 8 / dt1, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)), "cpu_model": model,
            "sample": f"{Rs} replicas x {sweeps} anneal sweeps of the N=50000 instance ({att:.3g} attempts, "
                      f"{dt:.1f} s wall on {threads} threads); single thread: 4 replicas x 8 sweeps "
                      f"({dt1:.1f} s)"}


def main():
    global BLOCK_THREADS, CLASS_CAP, R, RPW
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttt", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the C1 latency, short batched and short served sections")
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--replicas", type=int, default=R, help="replicas of the N=50000 workload (default 1024)")
    ap.add_argument("--rpw", type=int, default=0, help="k-SAT replicas per sweep workgroup: 4 or 8 (0: 4)")
    ap.add_argument("--class-cap", type=int, default=CLASS_CAP)
    ap.add_argument("--workload", choices=["nmc", "batch", "qap", "serve", "apt", "lbp", "alg1", "c1", "wide"],
                    default="nmc",
                    help="nmc: the N=50000 NMC path (default); batch: 256 mixed instances, batched vs "
                         "per-instance; qap: the n=100 QAP path; serve: Poisson stream into the server; "
                         "apt: adaptive parallel tempering on the N=50000 instance; lbp: NMC with LBP "
                         "surrogate backbones on the N=50000 instance; alg1: tempering -> seeds -> per-seed "
                         "LBP backbones -> batched inhomogeneous MC and unlearning; wide: the NMC path on a "
                         "N=1,000,000 instance (the wide layout)")
    ap.add_argument("--tune-sweeps", type=int, default=2,
                    help="with --workload batch: sweeps of each autotuner probe launch")
    ap.add_argument("--pt-rounds", type=int, default=APT_ROUNDS)
    ap.add_argument("--pt-sweeps-per-round", type=int, default=1)
    ap.add_argument("--serve-seconds", type=float, default=SERVE_SECONDS)
    ap.add_argument("--serve-procs", type=int, default=16,
                    help="processes generating the served requests' instances (0: in this process, e.g. under "
                         "a profiler)")
    ap.add_argument("--sweeps-only", type=int, default=0,
                    help="only time one homogeneous anneal of this many sweeps (for counter profiles) and exit")
    ap.add_argument("--qap-curve", type=int, default=0,
                    help="with --workload qap: run the schedule in launches of this many sweeps and report "
                         "acceptance and kernel rate per launch")
    ap.add_argument("--sweeps-offset", type=int, default=0,
                    help="with --workload qap --sweeps-only: start that many sweeps into the anneal schedule")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain elementwise copy of this many MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the replica-parallel path "
              f"would shard by replicas, one slice per GPU", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2111_13628_amd import nmc

    BLOCK_THREADS = args.block_threads
    CLASS_CAP = args.class_cap
    R = args.replicas
    RPW = args.rpw

    # the serving stream's instances come from a process pool, created before
    # this process touches the GPU (a HIP-initialised process must not fork)
    pre_serve = None
    if args.workload == "serve":
        pre_serve = serve_requests(instances.DEFAULT_SEED, args.serve_seconds, args.serve_procs)
    elif args.workload == "nmc" and not args.sweeps_only and not args.copy_probe_mib and not args.no_extras:
        pre_serve = serve_requests(instances.DEFAULT_SEED, SHORT_SERVE_SECONDS, args.serve_procs)

    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        # one read + one write of a known byte count, to scale HBM byte counters
        a = torch.ones(args.copy_probe_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 4, "copy_probe_bytes_written": b.numel() * 4}))
        return
    stream = torch.cuda.current_stream()
    seed = instances.DEFAULT_SEED
    if args.workload == "qap":
        res = bench_qap(nmc, torch, seed, args.sweeps_only, args.sweeps_offset, args.qap_curve)
        print(json.dumps({"metric": "QAP swap proposals/s (whole NMC path)", "value": res["proposals_per_s"],
                          "unit": "proposals/s", "n_gpus": 1, "higher_is_better": True, "dtype": "int32",
                          "data": "synthetic",
                          "config": {"workload": "QAP n=100, 4096 replicas, anneal 5000 + 2x(backbone + reanneal 1000)"},
                          "roofline": res["roofline"], "qap": res}), flush=True)
        return
    if args.workload == "c1":
        res = bench_c1(nmc, torch, seed, repeats=C1_REPEATS)
        print(json.dumps({"metric": "latency of plain SA, random 4-SAT N=200 M=1920, 64 replicas, 1000 sweeps",
                          "value": res["latency_ms"], "unit": "ms", "n_gpus": 1, "higher_is_better": False,
                          "dtype": "int32", "data": "synthetic",
                          "config": {"workload": "plain SA, random 4-SAT N=200 alpha=9.6, 64 replicas, 1000 sweeps"},
                          "c1": res}), flush=True)
        return
    if args.workload == "wide":
        res = bench_wide(nmc, torch, seed)
        print(json.dumps({"metric": "spin-flip attempts/s (NMC path, wide layout)", "value": res["attempts_per_s"],
                          "unit": "attempts/s", "n_gpus": 1, "higher_is_better": True, "dtype": "int32",
                          "data": "synthetic",
                          "config": {"workload": f"NMC random 4-SAT N=1000000 alpha=9.9, {R} replicas, anneal 200 + "
                                                 "2x(backbone + reanneal 100)"},
                          "wide": res}), flush=True)
        return
    if args.workload == "alg1":
        res = bench_alg1(nmc, torch, seed)
        print(json.dumps({"metric": "spin-flip attempts/s (Algorithm 1: tempering, seeds, LBP backbones, "
                                    "inhomogeneous MC)", "value": res["attempts_per_s"], "unit": "attempts/s",
                          "n_gpus": 1, "higher_is_better": True, "dtype": "int32", "data": "synthetic",
                          "config": {"workload": "Algorithm 1 on random 4-SAT N=50000 alpha=9.9, 1024 replicas: "
                                                 "APT 64x16 + 16 seeds x 64 replicas x 2 rounds"},
                          "alg1": res}), flush=True)
        return
    if args.workload == "lbp":
        res = bench_lbp(nmc, torch, seed)
        print(json.dumps({"metric": "spin-flip attempts/s (NMC path with LBP surrogate backbones)",
                          "value": res["attempts_per_s"], "unit": "attempts/s", "n_gpus": 1,
                          "higher_is_better": True, "dtype": "int32", "data": "synthetic",
                          "config": {"workload": "NMC random 4-SAT N=50000 alpha=9.9, 1024 replicas, anneal 2000 + "
                                                 "3x(LBP backbone + reanneal 1000)"},
                          "roofline": res["roofline"], "lbp": res}), flush=True)
        return
    if args.workload == "apt":
        res = bench_apt(nmc, torch, seed, args.pt_rounds, args.pt_sweeps_per_round)
        print(json.dumps({"metric": "spin-flip attempts/s (adaptive ladder + parallel tempering)",
                          "value": res["attempts_per_s"], "unit": "attempts/s", "n_gpus": 1,
                          "higher_is_better": True, "dtype": "int32", "data": "synthetic",
                          "config": {"workload": f"APT random 4-SAT N=50000 alpha=9.9, {APT_TEMPS} temperatures x "
                                                 f"{APT_CHAINS} chains, ladder + {args.pt_rounds} rounds of "
                                                 f"{args.pt_sweeps_per_round} sweep(s) + exchange"},
                          "roofline": res["roofline"], "apt": res}), flush=True)
        return
    if args.workload == "serve":
        res = bench_serve(nmc, torch, seed, args.serve_seconds, pre_serve)
        print(json.dumps({"metric": "served NMC: solves/s and p50/p99 time-to-target", "value": res["all"]["solves_per_s"],
                          "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "dtype": "int32",
                          "data": "synthetic",
                          "config": {"workload": f"Poisson {SERVE_RATE:g} req/s for {args.serve_seconds:g} s: 70% 4-SAT "
                                                 "N log-uniform [2000, 50000] alpha 9.7, 30% QAP n in [30, 150]"},
                          "serve": res}), flush=True)
        return
    if args.workload == "batch":
        res = bench_batch(nmc, torch, seed, tune_sweeps=args.tune_sweeps)
        print(json.dumps({"metric": "batched NMC vs one-launch-per-instance plain SA: attempts/s and time-to-target",
                          "value": res["batched_nmc"]["attempts_per_s"], "unit": "attempts/s", "n_gpus": 1,
                          "higher_is_better": True, "dtype": "int32", "data": "synthetic",
                          "config": {"workload": "256 random k-SAT instances, k in {3,4}, N log-uniform "
                                                 "[1000, 20000], 1000 anneal + 2x(backbone + 500 reanneal)"},
                          "batch": res}), flush=True)
        return
    cp, lits = instances.gen_ksat(N, ALPHA, K, seed)
    inst = nmc.Instance.ksat(N, cp, lits, CLASS_CAP).bind()
    M = inst.info.n_clauses
    if args.sweeps_only:
        rep = nmc.Replicas(inst, R, seed)
        if BLOCK_THREADS:
            rep.set_tuning(BLOCK_THREADS)
        if RPW:
            rep.set_replicas_per_workgroup(RPW)
        rep.set_profiling(True)
        rep.anneal(instances.linear_schedule(BETA0, BETA1, S_ANNEAL)[None, :args.sweeps_only])
        kt = rep.kernel_time()
        print(json.dumps({"sweeps": args.sweeps_only, "kernel_ms": kt["ms"],
                          "attempts_per_s": kt["attempts"] / (kt["ms"] / 1000.0)}))
        return
    attempts = float(R) * N * (S_ANNEAL + ROUNDS * S_RE)

    for w in range(args.warmup):
        run_path(inst, seed + 1000 + w, -1, nmc)
    torch.cuda.synchronize()

    times = []
    last = None
    for s in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep, be = run_path(inst, seed + s, -1, nmc)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        last = (rep, be)
    ms_per_step = 1000.0 * float(np.mean(times))

    # sweep-kernel time from HIP events on the launch stream (separate pass)
    prep, _ = run_path(inst, seed, -1, nmc, profile=True)
    kt = prep.kernel_time()
    acceptance = prep.accept_count() / attempts
    bps = counter_bytes_per_sweep()
    sweeps_per_launch = (S_ANNEAL + ROUNDS * S_RE) / (1 + ROUNDS)
    roofline = ksat_roofline(kt, M, acceptance, None if bps is None else bps * sweeps_per_launch)
    roofline["traffic_unit"] = "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    del prep
    # the same rates against what the probe kernels reach on this GPU
    peaks = measured_peaks(nmc, torch)
    roofline["frac_of_measured_hbm_copy"] = roofline["achieved"] / 1e3 / peaks["hbm_copy_TB_per_s"]
    roofline["lds"]["frac_of_measured_random"] = roofline["lds"]["achieved"] / peaks["lds_random_T_per_s"]
    roofline["lds"]["frac_of_measured_distinct"] = roofline["lds"]["achieved"] / peaks["lds_distinct_T_per_s"]
    roofline["valu"]["frac_of_measured"] = roofline["valu"]["achieved"] / peaks["valu_int_T_per_s"]

    out = {
        "metric": "spin-flip attempts/s (whole NMC path) + time-to-target vs plain SA on 1 GPU",
        "value": attempts / (ms_per_step / 1000.0),
        "unit": "attempts/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"NMC random 4-SAT N=50000 alpha=9.9 M=495000, {R} replicas, "
                               "anneal 2000 + 3x(backbone + reanneal 1000)",
                   "n_vars": N, "n_clauses": M, "k": K, "replicas": R, "replicas_per_workgroup": RPW or 4,
                   "sweeps": S_ANNEAL + ROUNDS * S_RE, "class_cap": CLASS_CAP,
                   "colors": inst.info.n_colors, "parallelism": "replicas"},
        "best_energy": last[1]["best"], "replicas_at_zero": last[1]["n_at_zero"],
        "roofline": roofline,
        "measured_peaks": peaks,
    }

    if not args.no_ttt:
        # time-to-target: target = 10th percentile of final energies of a
        # calibration plain-SA run (other seed); plain SA = homogeneous
        # 0.1 -> 4.0 over the same 5000 sweeps and replicas.
        S_tot = S_ANNEAL + ROUNDS * S_RE
        cal = nmc.Replicas(inst, R, seed + 777)
        cal.anneal(instances.linear_schedule(BETA0, BETA1, S_tot)[None, :])
        target = int(np.percentile(cal.best_energy()["energy"], 10))
        del cal
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sa = nmc.Replicas(inst, R, seed)
        sa.set_profiling(True)
        sa.anneal(instances.linear_schedule(BETA0, BETA1, S_tot)[None, :], target=target)
        sbe = sa.best_energy()
        sa_s = time.perf_counter() - t0
        nrep, nbe = run_path(inst, seed, target, nmc)
        torch.cuda.synchronize()
        # the same schedule with the paper's backbone estimator: LBP surrogate
        # backbones (as --workload lbp) in place of the magnetization
        # backbones; the time to the first hit is interpolated inside the
        # phase (anneal, or a round's reanneal after its LBP) that holds it
        t0 = time.perf_counter()
        lr = nmc.Replicas(inst, R, seed)
        lr.anneal(instances.linear_schedule(BETA0, BETA1, S_ANNEAL)[None, :], target=target)
        torch.cuda.synchronize()
        marks = [(0, S_ANNEAL, 0.0, time.perf_counter() - t0)]
        done = S_ANNEAL
        for ts, tc in LBP_THRESHOLDS:
            r0 = int(np.argmin(lr.best_energy()["best_per_replica"]))
            lr.lbp_backbone(r0, "best", **LBP_CFG, theta_seed=ts, theta_cut=tc)
            torch.cuda.synchronize()
            t_s = time.perf_counter() - t0
            lr.reanneal(reanneal_profile(S_RE), "backbone", target=target)
            torch.cuda.synchronize()
            marks.append((done, S_RE, t_s, time.perf_counter() - t0))
            done += S_RE
        lbe = lr.best_energy()
        lhit = lbe["first_hit"][lbe["first_hit"] >= 0]
        lbp_ttt, lbp_h = None, None
        if lhit.size:
            lbp_h = int(lhit.min())
            for s0, ns, ta, tb in marks:
                if s0 <= lbp_h <= s0 + ns:
                    lbp_ttt = ta + (lbp_h - s0) * (tb - ta) / ns
                    break
        del lr
        def ttt(fh, s_per_sweep):
            hit = fh[fh >= 0]
            return None if hit.size == 0 else float(hit.min()) * s_per_sweep
        out["time_to_target"] = {
            "target_energy": target, "target_rule": "10th percentile of calibration plain-SA final energies",
            "nmc_s": ttt(nbe["first_hit"], ms_per_step / 1000.0 / S_tot),
            "plain_sa_s": ttt(sbe["first_hit"], sa_s / S_tot),
            "time_rule": "first sweep boundary with a replica at or below target x measured seconds per sweep",
            "nmc_first_hit_sweep": int(nbe["first_hit"][nbe["first_hit"] >= 0].min()) if (nbe["first_hit"] >= 0).any() else None,
            "sa_first_hit_sweep": int(sbe["first_hit"][sbe["first_hit"] >= 0].min()) if (sbe["first_hit"] >= 0).any() else None,
            "nmc_best": nbe["best"], "plain_sa_best": sbe["best"],
            "nmc_replicas_hit": int((nbe["first_hit"] >= 0).sum()), "sa_replicas_hit": int((sbe["first_hit"] >= 0).sum()),
            "ratio_ref": f"paper target ratio 1e-4 * M = {int(1e-4 * M)} violations",
            "nmc_lbp_s": lbp_ttt, "nmc_lbp_first_hit_sweep": lbp_h, "nmc_lbp_best": lbe["best"],
            "nmc_lbp_replicas_hit": int(lhit.size),
            "nmc_lbp_rule": "LBP surrogate backbones in place of the magnetization backbones, same sweeps; "
                            "time interpolated inside the phase holding the first hit",
        }

    if not args.no_extras:
        # the other workloads of the metric, shortened: C1 solve latency
        # (p50 / p99 over repeated solves), batched NMC vs one launch per
        # instance on a reduced C4 batch, and a short C5 served stream
        c1 = bench_c1(nmc, torch, seed, repeats=C1_REPEATS)
        out["c1"] = c1
        print(f"# c1: p50 {c1['latency_p50_ms']:.1f} ms, p99 {c1['latency_p99_ms']:.1f} ms", file=sys.stderr,
              flush=True)
        bt = bench_batch(nmc, torch, seed, n_instances=SHORT_BATCH_INSTANCES)
        out["batch"] = bt
        print(f"# batch: {bt['ttt']}", file=sys.stderr, flush=True)
        sv = bench_serve(nmc, torch, seed, SHORT_SERVE_SECONDS, pre_serve, n_cap=150)
        allr = sv["all"]
        out["serve"] = {"p50": (allr["time_to_target_s"] or {}).get("p50"),
                        "p99": (allr["time_to_target_s"] or {}).get("p99"),
                        "unit": "s, submission to the round end at or below target, solved requests",
                        "solves_per_s": allr["solves_per_s"], "latency_s": allr["latency_s"],
                        "requests": sv["requests"], "seconds": SHORT_SERVE_SECONDS,
                        "offered_load": sv["offered_load"], "ksat": sv["ksat"], "qap": sv["qap"],
                        "capacity_requests_per_s": sv["capacity_requests_per_s"], "schedule": sv["schedule"]}
        print(f"# serve: p50 {out['serve']['p50']} p99 {out['serve']['p99']}", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cp, lits, seed)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
