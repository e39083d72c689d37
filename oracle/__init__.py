"""CPU oracle for the NMC hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It wraps ``nmc_oracle.c`` (plain sequential C, built with gcc)
through ctypes; it shares no code with the GPU library.

Array conventions (all numpy, C-contiguous):
  k-SAT spins  x[R][N] uint8 in {0,1};  energies int32[R]
  QAP assignment perm[R][n] uint8 (perm[f] = location of facility f); costs int64[R]
"""
from __future__ import annotations

import ctypes
import os
from concurrent.futures import ThreadPoolExecutor
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nmc_oracle.c")
_LIB = os.path.join(_HERE, "libnmc_oracle.so")

STREAM_SWEEP, STREAM_INIT, STREAM_QAP_SWEEP, STREAM_QAP_INIT, STREAM_PT_SWAP, STREAM_CFLIP = 0, 1, 2, 3, 4, 5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/libnmc_oracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lock = threading.Lock()

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64
_I64 = ctypes.c_int64
_D = ctypes.c_double


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            L = ctypes.CDLL(_LIB)
            L.orc_philox4x32_10.argtypes = [_P, _P, _P]
            L.orc_uniform_u32.argtypes = [_U64, _U32, _U32, _U32, _U32]
            L.orc_uniform_u32.restype = _U32
            L.orc_threshold.argtypes = [_D, _I64]
            L.orc_threshold.restype = _U32
            L.orc_qap_threshold.argtypes = [_D, _I64]
            L.orc_qap_threshold.restype = _U32
            L.orc_ksat_energy.argtypes = [_I32, _I32, _P, _P, _P]
            L.orc_ksat_energy.restype = _I32
            L.orc_ksat_delta.argtypes = [_I32, _I32, _P, _P, _I32, _P]
            L.orc_ksat_delta.restype = _I32
            L.orc_ksat_color.argtypes = [_I32, _I32, _P, _P, _I32, _P, _P, _P]
            L.orc_ksat_color.restype = _I32
            L.orc_ksat_init.argtypes = [_I32, _I32, _I32, _U64, _P]
            L.orc_ksat_anneal.argtypes = [_I32, _I32, _P, _P, _P, _I32, _I32, _U64, _U32, _I32,
                                          _I32, _P, _P, _I64, _P, _P, _P, _P, _P]
            L.orc_ksat_anneal.restype = ctypes.c_int
            L.orc_ksat_backbone.argtypes = [_I32, _I32, _P, _P, _I32, _P, _I32, _I32, _I32, _P, _P]
            L.orc_qap_cost.argtypes = [_I32, _P, _P, _P]
            L.orc_qap_cost.restype = _I64
            L.orc_qap_delta.argtypes = [_I32, _P, _P, _P, _I32, _I32]
            L.orc_qap_delta.restype = _I64
            L.orc_qap_init.argtypes = [_I32, _I32, _I32, _U64, _P]
            L.orc_qap_anneal.argtypes = [_I32, _P, _P, _I32, _I32, _U64, _U32, _I32, _I32, _P, _P,
                                         _I64, _P, _P, _P, _P, _P]
            L.orc_qap_anneal.restype = ctypes.c_int
            L.orc_qap_backbone.argtypes = [_I32, _I32, _P, _I32, _I32, _P, _P]
            L.orc_pt_exchange.argtypes = [_I32, _I32, _I32, _I32, _P, _U64, _U32, _I32, _I32, _P, _P, _P, _P]
            L.orc_energy_sigma.argtypes = [_P, _I64]
            L.orc_energy_sigma.restype = _D
            L.orc_lbp_cnf.argtypes = [_I32, _I32, _P, _P, _P, _D, _D, _D, _D, _I32, _D, _D, _P, _P, _P, _P]
            L.orc_lbp_cnf.restype = ctypes.c_int
            L.orc_cnf_clusters.argtypes = [_I32, _I32, _P, _P, _P, _D, _D, _P, _P]
            L.orc_cnf_clusters.restype = _I32
            L.orc_ksat_whiten.argtypes = [_I32, _I32, _P, _P, _P, _P, _P, _P]
            L.orc_ksat_whiten.restype = _I32
            L.orc_ksat_cluster_flip.argtypes = [_I32, _I32, _P, _P, _P, _I32, _I32, _U64, _U32, _D, _I64, _P, _P,
                                                _P, _P, _P, _P]
            L.orc_ksat_cluster_flip.restype = _I32
            _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _split(r_begin, r_end, threads):
    threads = max(1, min(threads, r_end - r_begin))
    edges = np.linspace(r_begin, r_end, threads + 1).astype(int)
    return [(int(edges[i]), int(edges[i + 1])) for i in range(threads) if edges[i + 1] > edges[i]]


def _run_threads(fn, parts):
    if len(parts) == 1:
        fn(*parts[0])
        return
    ts = [threading.Thread(target=fn, args=p) for p in parts]
    for t in ts:
        t.start()
    for t in ts:
        t.join()


# ---------------------------------------------------------------- RNG / tables

def philox4x32_10(ctr, key):
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def uniform_u32(seed, stream, j, t, replica):
    return int(lib().orc_uniform_u32(seed, stream, j, t, replica))


def threshold(beta, d):
    return int(lib().orc_threshold(float(beta), int(d)))


def qap_threshold(beta, d):
    return int(lib().orc_qap_threshold(float(beta), int(d)))


# ---------------------------------------------------------------- k-SAT

class KSat:
    def __init__(self, n, clause_ptr, lits):
        self.n = int(n)
        self.cptr = _c(clause_ptr, np.int32)
        self.lits = _c(lits, np.int32)
        self.m = len(self.cptr) - 1

    def energy(self, x):
        x = _c(x, np.uint8)
        return int(lib().orc_ksat_energy(self.n, self.m, _p(self.cptr), _p(self.lits), _p(x)))

    def delta(self, x, i):
        x = np.array(x, dtype=np.uint8, copy=True)
        return int(lib().orc_ksat_delta(self.n, self.m, _p(self.cptr), _p(self.lits), int(i), _p(x)))

    def color(self, cap=0):
        color = np.zeros(self.n, np.int32)
        order = np.zeros(self.n, np.int32)
        cptr = np.zeros(self.n + 1, np.int32)
        nc = lib().orc_ksat_color(self.n, self.m, _p(self.cptr), _p(self.lits), int(cap),
                                  _p(color), _p(order), _p(cptr))
        return color, order, cptr[: nc + 1].copy()

    def init(self, R, seed, threads=1):
        x = np.zeros((R, self.n), np.uint8)
        _run_threads(lambda a, b: lib().orc_ksat_init(self.n, a, b, seed, _p(x)), _split(0, R, threads))
        return x


    def lbp(self, x_ref, beta, lambda0, ratio, lambda_min, max_iter, tol, p_min=-2.0):
        """Adiabatic LBP on the surrogate Hamiltonian around the 0/1 state
        x_ref; returns dict(u per literal position, mag, corr per clause,
        lambda, steps, iterations, converged, delta, overlap, self_overlap)."""
        s = (2 * _c(x_ref, np.int8) - 1).astype(np.int8)
        u = np.zeros(max(len(self.lits), 1), np.float64)
        mag = np.zeros(max(self.n, 1), np.float64)
        corr = np.zeros(max(self.m, 1), np.float64)
        st = np.zeros(7, np.float64)
        rc = lib().orc_lbp_cnf(self.n, self.m, _p(self.cptr), _p(self.lits), _p(s), float(beta), float(lambda0),
                               float(ratio), float(lambda_min), int(max_iter), float(tol), float(p_min), _p(u),
                               _p(mag), _p(corr), _p(st))
        assert rc == 0
        return dict(u=u[: len(self.lits)], mag=mag[: self.n], corr=corr[: self.m], **{
            k: (int(v) if k in ("steps", "iterations", "converged") else float(v))
            for k, v in zip(("lambda", "steps", "iterations", "converged", "delta", "overlap", "self_overlap"), st)})

    def whiten(self, x, order=None):
        """Whitening of the 0/1 state x: (frozen count, star mask, passes)."""
        x = _c(x, np.uint8)
        star = np.zeros(max(self.n, 1), np.uint8)
        passes = ctypes.c_int32()
        o = None if order is None else _c(order, np.int32)
        k = lib().orc_ksat_whiten(self.n, self.m, _p(self.cptr), _p(self.lits), _p(x), _p(o), _p(star),
                                  ctypes.byref(passes))
        return int(k), star[: self.n], passes.value

    def clusters(self, corr, theta_seed, theta_cut):
        """Connected backbone growth: (label, cls, n_clusters)."""
        corr = _c(corr, np.float64)
        label = np.zeros(max(self.n, 1), np.int32)
        cls = np.zeros(max(self.n, 1), np.uint8)
        k = lib().orc_cnf_clusters(self.n, self.m, _p(self.cptr), _p(self.lits), _p(corr), float(theta_seed),
                                   float(theta_cut), _p(label), _p(cls))
        return label[: self.n], cls[: self.n], int(k)


class KSatReplicas:
    """Replica set mirroring the library's handle: state, energies, best
    energies, first-hit sweeps, best-state snapshot and the sweep counter."""

    def __init__(self, inst: KSat, R, seed, order, threads=1, snapshot=True):
        self.inst, self.R, self.seed = inst, int(R), int(seed)
        self.order = _c(order, np.int32)
        self.x = inst.init(R, seed, threads)
        self.energy = np.array([inst.energy(self.x[r]) for r in range(R)], np.int32)
        self.best = self.energy.copy()
        self.first_hit = np.full(R, -1, np.int32)
        self.best_x = self.x.copy() if snapshot else None
        self.sweeps_done = 0
        self.threads = threads

    def anneal(self, beta, class_of=None, target=-1, r_begin=0, r_end=None):
        beta = np.atleast_2d(_c(beta, np.float64))
        nc, S = beta.shape
        beta = _c(beta, np.float64)
        cls = None if class_of is None else _c(class_of, np.uint8)
        r_end = self.R if r_end is None else r_end
        _run_threads(lambda a, b: self._sweeps(beta, cls, target, a, b), _split(r_begin, r_end, self.threads))
        self.sweeps_done += S

    def _sweeps(self, beta, cls, target, a, b):
        """Sweeps of replicas a..b-1 from the current sweep counter (not advanced)."""
        inst = self.inst
        nc, S = beta.shape
        lib().orc_ksat_anneal(inst.n, inst.m, _p(inst.cptr), _p(inst.lits), _p(self.order), a, b,
                              self.seed, self.sweeps_done, S, nc, _p(beta), _p(cls), int(target),
                              _p(self.x), _p(self.energy), _p(self.best), _p(self.first_hit),
                              _p(self.best_x))

    def pt_run(self, beta, n_rounds, sweeps_per_round, first_parity=0, target=-1, chains=None):
        return _pt_run(self, self.x, beta, n_rounds, sweeps_per_round, first_parity, target, chains)

    def cluster_flip(self, label, beta, target=-1, r_begin=0, r_end=None):
        """One collective-move sweep over the clusters of `label`; returns the
        clusters flipped per replica."""
        inst = self.inst
        lab = _c(label, np.int32)
        r_end = self.R if r_end is None else r_end
        acc = np.zeros(self.R, np.int32)

        def run(a, b):
            lib().orc_ksat_cluster_flip(inst.n, inst.m, _p(inst.cptr), _p(inst.lits), _p(lab), a, b, self.seed,
                                        self.sweeps_done, float(beta), int(target), _p(self.x), _p(self.energy),
                                        _p(self.best), _p(self.first_hit), _p(self.best_x), _p(acc))

        _run_threads(run, _split(r_begin, r_end, self.threads))
        self.sweeps_done += 1
        return acc

    def apt_ladder(self, beta_first, alpha, sigma_min, equil, meas, max_temps):
        return _apt_ladder(self, beta_first, alpha, sigma_min, equil, meas, max_temps)

    def backbone(self, thr_num=9, thr_den=10, expand=True):
        inst = self.inst
        counts = np.zeros(inst.n, np.int32)
        cls = np.zeros(inst.n, np.uint8)
        lib().orc_ksat_backbone(inst.n, inst.m, _p(inst.cptr), _p(inst.lits), self.R, _p(self.x),
                                thr_num, thr_den, int(bool(expand)), _p(counts), _p(cls))
        return cls, counts


# ---------------------------------------------------------------- QAP

class Qap:
    def __init__(self, F, D):
        self.F = _c(F, np.int32)
        self.D = _c(D, np.int32)
        self.n = self.F.shape[0]

    def cost(self, perm):
        perm = _c(perm, np.uint8)
        return int(lib().orc_qap_cost(self.n, _p(self.F), _p(self.D), _p(perm)))

    def delta(self, perm, r, s):
        perm = _c(perm, np.uint8)
        return int(lib().orc_qap_delta(self.n, _p(self.F), _p(self.D), _p(perm), int(r), int(s)))

    def init(self, R, seed, threads=1):
        p = np.zeros((R, self.n), np.uint8)
        _run_threads(lambda a, b: lib().orc_qap_init(self.n, a, b, seed, _p(p)), _split(0, R, threads))
        return p


class QapReplicas:
    def __init__(self, inst: Qap, R, seed, threads=1, snapshot=True):
        self.inst, self.R, self.seed = inst, int(R), int(seed)
        self.perm = inst.init(R, seed, threads)
        self.cost = np.array([inst.cost(self.perm[r]) for r in range(R)], np.int64)
        self.best = self.cost.copy()
        self.first_hit = np.full(R, -1, np.int32)
        self.best_perm = self.perm.copy() if snapshot else None
        self.sweeps_done = 0
        self.threads = threads

    def anneal(self, beta, class_of=None, target=-1, r_begin=0, r_end=None):
        beta = np.atleast_2d(_c(beta, np.float64))
        nc, S = beta.shape
        beta = _c(beta, np.float64)
        cls = None if class_of is None else _c(class_of, np.uint8)
        r_end = self.R if r_end is None else r_end
        _run_threads(lambda a, b: self._sweeps(beta, cls, target, a, b), _split(r_begin, r_end, self.threads))
        self.sweeps_done += S

    def _sweeps(self, beta, cls, target, a, b):
        inst = self.inst
        nc, S = beta.shape
        lib().orc_qap_anneal(inst.n, _p(inst.F), _p(inst.D), a, b, self.seed, self.sweeps_done, S, nc,
                             _p(beta), _p(cls), int(target), _p(self.perm), _p(self.cost),
                             _p(self.best), _p(self.first_hit), _p(self.best_perm))

    @property
    def energy(self):
        return self.cost

    def pt_run(self, beta, n_rounds, sweeps_per_round, first_parity=0, target=-1, chains=None):
        return _pt_run(self, self.perm, beta, n_rounds, sweeps_per_round, first_parity, target, chains)

    def apt_ladder(self, beta_first, alpha, sigma_min, equil, meas, max_temps):
        return _apt_ladder(self, beta_first, alpha, sigma_min, equil, meas, max_temps)

    def backbone(self, thr_num=9, thr_den=10):
        inst = self.inst
        freq = np.zeros((inst.n, inst.n), np.int32)
        cls = np.zeros(inst.n, np.uint8)
        lib().orc_qap_backbone(inst.n, self.R, _p(self.perm), thr_num, thr_den, _p(freq), _p(cls))
        return cls, freq


# ---------------------------------------------------------------- parallel tempering

def energy_sigma(samples):
    """sigma = sqrt(<E^2> - <E>^2) over the samples (appendix A)."""
    e = _c(samples, np.int64)
    return float(lib().orc_energy_sigma(_p(e), e.size))


def pt_exchange(beta, n_chains, seed, t, parity, rows, energy, chains=None):
    """One exchange step on rows [R][row_len] and energies [R] (both updated
    in place) for chains[0]..chains[1]-1 (default all); returns (accepted,
    attempted) per pair position."""
    beta = _c(beta, np.float64)
    M = beta.size
    acc = np.zeros(max(M - 1, 1), np.int64)
    att = np.zeros(max(M - 1, 1), np.int64)
    e = _c(energy, np.int64)
    c0, c1 = (0, int(n_chains)) if chains is None else chains
    lib().orc_pt_exchange(M, int(n_chains), c0, c1, _p(beta), int(seed), int(t), int(parity), rows.shape[1],
                          _p(rows), _p(e), _p(acc), _p(att))
    energy[:] = e
    return acc[: M - 1], att[: M - 1]


def _pt_run(rep, rows, beta, n_rounds, sweeps_per_round, first_parity, target, chains=None):
    """Parallel tempering rounds (appendix A).  Replica r = i * C + c runs at
    beta[i]; every round is sweeps_per_round Metropolis sweeps of every
    replica at its ladder temperature, then one exchange step with parity
    (first_parity + round) mod 2.  chains = (c0, c1) follows only those
    chains (the other replicas are left untouched).  Returns summed
    (accepted, attempted) of the chains followed."""
    beta = _c(beta, np.float64)
    M = beta.size
    C = rep.R // M
    assert C * M == rep.R
    c0, c1 = (0, C) if chains is None else chains
    S = int(sweeps_per_round)
    acc = np.zeros(max(M - 1, 0), np.int64)
    att = np.zeros(max(M - 1, 0), np.int64)
    tabs = [np.full((1, S), b) for b in beta]
    parts = []
    per = max(1, rep.threads // M) if M else 1
    for i in range(M):
        parts += [(i, a, b) for a, b in _split(i * C + c0, i * C + c1, per)]
    with ThreadPoolExecutor(max_workers=max(1, rep.threads)) as pool:
        for k in range(n_rounds):
            list(pool.map(lambda p: rep._sweeps(tabs[p[0]], None, target, p[1], p[2]), parts))
            rep.sweeps_done += S
            if M > 1:
                a, t = pt_exchange(beta, C, rep.seed, rep.sweeps_done, (first_parity + k) & 1, rows, rep.energy,
                                   (c0, c1))
                acc += a
                att += t
    return acc, att


def _apt_ladder(rep, beta_first, alpha, sigma_min, equil, meas, max_temps):
    """Adaptive ladder (appendix A): at beta_i every replica runs `equil`
    sweeps, then `meas` sweeps after each of which all replica energies are
    sampled; sigma_i is their spread and beta_{i+1} = beta_i + alpha / sigma_i,
    until sigma_i <= sigma_min or max_temps positions exist.  The replicas
    carry their states from one temperature to the next."""
    betas, sigmas = [], []
    b = float(beta_first)
    while True:
        if equil:
            rep.anneal(np.full((1, int(equil)), b))
        samples = []
        for _ in range(int(meas)):
            rep.anneal(np.full((1, 1), b))
            samples.append(np.array(rep.energy, np.int64))
        s = energy_sigma(np.concatenate(samples))
        betas.append(b)
        sigmas.append(s)
        if s <= sigma_min or len(betas) >= max_temps:
            break
        b = b + alpha / s
    return np.array(betas), np.array(sigmas)
