"""Helpers shared by the GPU parity tests: run the same call sequence on the
HIP library and on the CPU oracle and compare every observable."""
import os

import numpy as np

import oracle
from paper_2111_13628_amd import nmc


def threads():
    return max(1, min(16, os.cpu_count() or 1))


def say(msg):
    print(msg, flush=True)


class KsatPair:
    """The library's replica set next to an oracle replica set of the same
    instance, seed and sweep order."""

    def __init__(self, n, cp, lits, R, seed, cap=0, block_threads=0):
        self.inst = nmc.Instance.ksat(n, cp, lits, cap).bind()
        self.rep = nmc.Replicas(self.inst, R, seed)
        if block_threads:
            self.rep.set_tuning(block_threads)
        self.oinst = oracle.KSat(n, cp, lits)
        _, order, _ = self.oinst.color(cap)
        self.orep = oracle.KSatReplicas(self.oinst, R, seed, order, threads=threads())

    def anneal(self, beta, class_of=None, target=-1, profile=None):
        beta = np.atleast_2d(beta)
        if profile == "backbone":
            self.rep.reanneal(beta, "backbone", target=target)
        elif class_of is not None:
            self.rep.anneal(beta, "host", class_of, target)
        else:
            self.rep.anneal(beta, target=target)
        self.orep.anneal(beta, class_of=class_of, target=target)

    def pt_run(self, beta, n_rounds, sweeps_per_round, first_parity=0, target=-1):
        acc, att = self.rep.pt_run(beta, n_rounds, sweeps_per_round, first_parity, target)
        oacc, oatt = self.orep.pt_run(beta, n_rounds, sweeps_per_round, first_parity, target)
        assert (att == oatt).all(), (att, oatt)
        assert (acc == oacc).all(), (acc, oacc)
        return acc, att

    def apt_ladder(self, *args):
        b, sg = self.rep.apt_ladder(*args)
        ob, osg = self.orep.apt_ladder(*args)
        assert b.tolist() == ob.tolist(), (b, ob)
        assert sg.tolist() == osg.tolist(), (sg, osg)
        return b, sg

    def backbone(self, num=9, den=10, expand=True):
        cls, counts = self.rep.estimate_backbone(num, den, expand)
        ocls, ocounts = self.orep.backbone(num, den, expand)
        assert (counts == ocounts).all(), "magnetization counts differ"
        assert (cls == ocls).all(), "backbone classes differ"
        return ocls

    def compare(self, check_best_state=True):
        x = self.rep.get_state("current")
        assert (x == self.orep.x).all(), f"states differ in {(x != self.orep.x).sum()} entries"
        be = self.rep.best_energy()
        assert (be["energy"] == self.orep.energy).all(), "energies differ"
        assert (be["best_per_replica"] == self.orep.best).all(), "best energies differ"
        assert (be["first_hit"] == self.orep.first_hit).all(), "first-hit sweeps differ"
        assert be["best"] == int(self.orep.best.min())
        assert be["n_at_zero"] == int((self.orep.best == 0).sum())
        assert (self.rep.recount() == self.orep.energy).all(), "recount differs from tracked energy"
        if check_best_state:
            xb = self.rep.get_state("best")
            assert (xb == self.orep.best_x).all(), "best-state snapshots differ"
        assert self.rep.sweeps_done() == self.orep.sweeps_done


class QapPair:
    def __init__(self, F, D, R, seed):
        self.inst = nmc.Instance.qap(F, D).bind()
        self.rep = nmc.Replicas(self.inst, R, seed)
        self.oinst = oracle.Qap(F, D)
        self.orep = oracle.QapReplicas(self.oinst, R, seed, threads=threads())

    def anneal(self, beta, class_of=None, target=-1, profile=None):
        beta = np.atleast_2d(beta)
        if profile == "backbone":
            self.rep.reanneal(beta, "backbone", target=target)
        elif class_of is not None:
            self.rep.anneal(beta, "host", class_of, target)
        else:
            self.rep.anneal(beta, target=target)
        self.orep.anneal(beta, class_of=class_of, target=target)

    pt_run = KsatPair.pt_run
    apt_ladder = KsatPair.apt_ladder

    def backbone(self, num=9, den=10):
        cls, freq = self.rep.estimate_backbone(num, den)
        ocls, ofreq = self.orep.backbone(num, den)
        assert (freq == ofreq).all(), "assignment frequencies differ"
        assert (cls == ocls).all(), "backbone classes differ"
        return ocls

    def compare(self):
        p = self.rep.get_state("current")
        assert (p == self.orep.perm).all(), f"permutations differ in {(p != self.orep.perm).any(1).sum()} replicas"
        be = self.rep.best_energy()
        assert (be["energy"] == self.orep.cost).all(), "costs differ"
        assert (be["best_per_replica"] == self.orep.best).all(), "best costs differ"
        assert (be["first_hit"] == self.orep.first_hit).all(), "first-hit sweeps differ"
        assert (self.rep.recount() == self.orep.cost).all()
        assert (self.rep.get_state("best") == self.orep.best_perm).all(), "best permutations differ"
