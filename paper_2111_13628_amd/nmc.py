"""ctypes binding of the NMC C ABI (include/nmc.h).

Argument marshalling only: every step of the Monte Carlo path runs in the
HIP kernels of libnmc.so.  PyTorch supplies device memory (uint8 tensors on
cuda:0) and streams.  There is no fallback: if libnmc.so is missing or a
GPU call fails, the call raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnmc.so")
HEADER_PATH = os.path.join(_HERE, "..", "include", "nmc.h")

NMC_OK = 0
KIND_KSAT, KIND_QAP = 1, 2
PROFILE = {"homogeneous": 0, "host": 1, "backbone": 2}
STATE = {"current": 0, "best": 1}
ERRORS = {-1: "INVALID", -2: "SIZE", -3: "DEVICE", -4: "STATE", -5: "CAPACITY", -6: "UNSUPPORTED"}


class NmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"NMC_ERR_{ERRORS.get(code, code)}: {msg}")
        self.code = code


class InstanceInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_items", ctypes.c_int32), ("n_clauses", ctypes.c_int32),
                ("max_clause_len", ctypes.c_int32), ("max_degree", ctypes.c_int32),
                ("n_colors", ctypes.c_int32), ("delta_bound", ctypes.c_int64), ("wide", ctypes.c_int32)]


class LbpConfig(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("lambda0", ctypes.c_double), ("lambda_ratio", ctypes.c_double),
                ("lambda_min", ctypes.c_double), ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double),
                ("p_min", ctypes.c_double), ("theta_seed", ctypes.c_double), ("theta_cut", ctypes.c_double)]


class LbpResult(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("steps", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("delta", ctypes.c_double), ("overlap", ctypes.c_double),
                ("self_overlap", ctypes.c_double), ("backbone_size", ctypes.c_int32),
                ("n_clusters", ctypes.c_int32), ("largest_cluster", ctypes.c_int32),
                ("rigid_clauses", ctypes.c_int32), ("seed_clauses", ctypes.c_int32)]


class Plan(ctypes.Structure):
    _fields_ = [("anneal_beta", ctypes.c_void_p), ("anneal_sweeps", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("reanneal_beta", ctypes.c_void_p), ("reanneal_sweeps", ctypes.c_int32),
                ("thr_num", ctypes.c_int32), ("thr_den", ctypes.c_int32), ("expand", ctypes.c_int32),
                ("chunk_sweeps", ctypes.c_int32)]


class Segment(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double * 2), ("profile", ctypes.c_int32), ("backbone_before", ctypes.c_int32),
                ("target", ctypes.c_int64)]


class SetStatus(ctypes.Structure):
    _fields_ = [("best", ctypes.c_int64), ("n_at_zero", ctypes.c_int32), ("first_hit", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_cap_bytes", ctypes.c_size_t), ("chunk_sweeps", ctypes.c_int32),
                ("max_active", ctypes.c_int32), ("loader_threads", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("thr_num", ctypes.c_int32), ("thr_den", ctypes.c_int32),
                ("expand", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_vars", ctypes.c_int32), ("n_clauses", ctypes.c_int32),
                ("class_cap", ctypes.c_int32), ("clause_ptr", ctypes.c_void_p), ("lits", ctypes.c_void_p),
                ("n", ctypes.c_int32), ("flow", ctypes.c_void_p), ("dist", ctypes.c_void_p),
                ("n_replicas", ctypes.c_int32), ("seed", ctypes.c_uint64), ("beta0", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta_hot", ctypes.c_double), ("anneal_sweeps", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("reanneal_sweeps", ctypes.c_int32), ("target", ctypes.c_int64),
                ("has_target", ctypes.c_int32), ("budget_s", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_at_zero", ctypes.c_int32), ("best", ctypes.c_int64),
                ("first_hit_sweep", ctypes.c_int32), ("sweeps_done", ctypes.c_uint32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("device_bytes", ctypes.c_size_t),
                ("message", ctypes.c_char * 128)]


class ServerStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("active", ctypes.c_int32), ("waiting", ctypes.c_int32), ("device_bytes_in_use", ctypes.c_size_t),
                ("gpu_busy_s", ctypes.c_double)]


REQ_STATUS = {0: "queued", 1: "loaded", 2: "running", 3: "solved", 4: "exhausted", 5: "timeout", 6: "failed"}

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_U32 = ctypes.c_uint32
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t
_PP = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "nmc_last_error": ([], ctypes.c_char_p),
    "nmc_version": ([], _I32),
    "nmc_ksat_load": ([_I32, _I32, _P, _P, _I32, _PP], ctypes.c_int),
    "nmc_qap_load": ([_I32, _P, _P, _PP], ctypes.c_int),
    "nmc_instance_get_info": ([_P, ctypes.POINTER(InstanceInfo)], ctypes.c_int),
    "nmc_instance_order": ([_P, _P, _P, _P], ctypes.c_int),
    "nmc_footprint": ([_P, _I32, ctypes.POINTER(_SZ), ctypes.POINTER(_SZ)], ctypes.c_int),
    "nmc_instance_bind": ([_P, _P, _SZ, _P], ctypes.c_int),
    "nmc_instance_free": ([_P], None),
    "nmc_replicas_create": ([_P, _I32, _U64, _P, _SZ, _P, _PP], ctypes.c_int),
    "nmc_replicas_free": ([_P], None),
    "nmc_anneal": ([_P, _P, _I32, _I32, _I32, _P, _I64, _P], ctypes.c_int),
    "nmc_reanneal": ([_P, _P, _I32, _I32, _I32, _P, _I64, _P], ctypes.c_int),
    "nmc_anneal_noalloc": ([_P, _P, _I32, _I32, _I32, _P, _I64, _P], ctypes.c_int),
    "nmc_anneal_noalloc_capacity": ([], _SZ),
    "nmc_estimate_backbone": ([_P, _I32, _I32, _I32, _P, _P, _P], ctypes.c_int),
    "nmc_best_energy": ([_P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "nmc_recount": ([_P, _P, _P], ctypes.c_int),
    "nmc_get_state": ([_P, _I32, _P, _SZ, _P], ctypes.c_int),
    "nmc_set_state": ([_P, _P, _SZ, _U32, _P], ctypes.c_int),
    "nmc_replicas_info": ([_P, _P, _P, _P], ctypes.c_int),
    "nmc_set_tuning": ([_P, _I32], ctypes.c_int),
    "nmc_set_replicas_per_workgroup": ([_P, _I32], ctypes.c_int),
    "nmc_get_tuning": ([_P, _P, _P], ctypes.c_int),
    "nmc_tune": ([_P, _I32, _P, _P, _P], ctypes.c_int),
    "nmc_set_profiling": ([_P, _I32], ctypes.c_int),
    "nmc_kernel_time": ([_P, _P, _P, _P, _I32], ctypes.c_int),
    "nmc_accept_count": ([_P, _P, _I32, _P], ctypes.c_int),
    "nmc_pt_run": ([_P, _P, _I32, _I32, _I32, _I32, _I64, _P, _P, _P], ctypes.c_int),
    "nmc_cluster_flip": ([_P, _P, ctypes.c_double, _I64, _P, _P], ctypes.c_int),
    "nmc_whiten": ([_P, _I32, _P, _P, _P, _P], ctypes.c_int),
    "nmc_lbp_kernel_time": ([_P, _P, _P, _I32], ctypes.c_int),
    "nmc_probe_peak": ([_I32, _I32, _I32, _P, _P, _P], ctypes.c_int),
    "nmc_lbp_backbone": ([_P, _I32, _I32, ctypes.POINTER(LbpConfig), ctypes.POINTER(LbpResult), _P, _P, _P, _P, _P],
                         ctypes.c_int),
    "nmc_apt_ladder": ([_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _I32, _I32, _I32, _P, _P,
                        ctypes.POINTER(_I32), _P], ctypes.c_int),
    "nmc_batch_create": ([_P, _I32, _PP], ctypes.c_int),
    "nmc_batch_free": ([_P], None),
    "nmc_batch_set_tuning": ([_P, _I32], ctypes.c_int),
    "nmc_batch_tune": ([_P, _I32, _P, _P], ctypes.c_int),
    "nmc_batch_anneal": ([_P, _P, _I32, _I32, _I32, _P, _P], ctypes.c_int),
    "nmc_batch_lbp_backbone": ([_P, _P, _I32, ctypes.POINTER(LbpConfig), _P, _P], ctypes.c_int),
    "nmc_batch_estimate_backbone": ([_P, _I32, _I32, _I32, _P], ctypes.c_int),
    "nmc_batch_run_plan": ([_P, ctypes.POINTER(Plan), _P, _I32, _P], ctypes.c_int),
    "nmc_batch_run": ([_P, _P, _P, _I32, _P], ctypes.c_int),
    "nmc_batch_graph_info": ([_P, _P, _P], ctypes.c_int),
    "nmc_batch_set_members": ([_P, _P, _I32], ctypes.c_int),
    "nmc_batch_step": ([_P, _P, _I32, _I32, _I32, _I32, _P, _P], ctypes.c_int),
    "nmc_batch_set_profiling": ([_P, _I32], ctypes.c_int),
    "nmc_batch_kernel_time": ([_P, _P, _P, _P, _I32], ctypes.c_int),
    "nmc_server_create": ([ctypes.POINTER(ServerConfig), _PP], ctypes.c_int),
    "nmc_server_submit": ([_P, ctypes.POINTER(Request), ctypes.POINTER(_U64)], ctypes.c_int),
    "nmc_server_poll": ([_P, _U64, ctypes.POINTER(Result)], ctypes.c_int),
    "nmc_server_wait_idle": ([_P, ctypes.c_double], ctypes.c_int),
    "nmc_server_get_stats": ([_P, ctypes.POINTER(ServerStats)], ctypes.c_int),
    "nmc_server_now": ([_P], ctypes.c_double),
    "nmc_server_free": ([_P], None),
}

_lib = None


def lib():
    """Load libnmc.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        # torch ships its own HIP runtime with the same soname; loading it first
        # makes libnmc.so bind to that one runtime, so torch streams and device
        # pointers are valid handles inside the library.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        _check_single_hip_runtime()
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check_single_hip_runtime():
    try:
        maps = open("/proc/self/maps").read().split("\n")
    except OSError:
        return
    paths = {os.path.realpath(l.split()[-1]) for l in maps if "libamdhip64" in l and "/" in l}
    if len(paths) > 1:
        raise ImportError("two HIP runtimes are mapped in this process: " + ", ".join(sorted(paths)))


def header_functions():
    """Names of the functions include/nmc.h declares."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nmc_[a-z0-9_]+)\s*\(", text)))


def _check(rc):
    if rc != NMC_OK:
        raise NmcError(rc, lib().nmc_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


PROBE = {"lds_distinct": 0, "lds_random": 1, "valu_int": 2}


def probe_peak(which, iters, blocks, stream=None):
    """One timed launch of a peak-rate probe kernel (measurement helper):
    returns (kernel ms, lane operations done)."""
    ms = ctypes.c_double()
    ops = ctypes.c_double()
    w = PROBE[which] if isinstance(which, str) else int(which)
    _check(lib().nmc_probe_peak(w, int(iters), int(blocks), ctypes.byref(ms), ctypes.byref(ops), _stream(stream)))
    return ms.value, ops.value


def _device_buffer(nbytes: int):
    import torch
    if not torch.cuda.is_available():
        raise NmcError(-3, "no GPU visible to torch")
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


class Instance:
    """A loaded k-SAT or QAP instance.  Host metadata lives in the library;
    the device layout is uploaded into a torch buffer by bind()."""

    def __init__(self, handle, kind):
        self._h = handle
        self.kind = kind
        self._buf = None
        self.info = InstanceInfo()
        _check(lib().nmc_instance_get_info(self._h, ctypes.byref(self.info)))

    @classmethod
    def ksat(cls, n_vars, clause_ptr, lits, class_cap=0):
        cp = np.ascontiguousarray(clause_ptr, np.int32)
        li = np.ascontiguousarray(lits, np.int32)
        h = ctypes.c_void_p()
        _check(lib().nmc_ksat_load(int(n_vars), len(cp) - 1, _ptr(cp), _ptr(li), int(class_cap), ctypes.byref(h)))
        return cls(h, KIND_KSAT)

    @classmethod
    def qap(cls, flow, dist):
        F = np.ascontiguousarray(flow, np.int32)
        D = np.ascontiguousarray(dist, np.int32)
        h = ctypes.c_void_p()
        _check(lib().nmc_qap_load(int(F.shape[0]), _ptr(F), _ptr(D), ctypes.byref(h)))
        return cls(h, KIND_QAP)

    @property
    def n(self):
        return self.info.n_items

    def order(self):
        n = self.info.n_items
        order = np.zeros(n, np.int32)
        cptr = np.zeros(self.info.n_colors + 1, np.int32)
        nc = ctypes.c_int32()
        _check(lib().nmc_instance_order(self._h, _ptr(order), _ptr(cptr), ctypes.byref(nc)))
        return order, cptr

    def footprint(self, n_replicas):
        ib, rb = _SZ(), _SZ()
        _check(lib().nmc_footprint(self._h, int(n_replicas), ctypes.byref(ib), ctypes.byref(rb)))
        return ib.value, rb.value

    def bind(self, stream=None):
        ib, _ = self.footprint(1)
        self._buf = _device_buffer(ib)
        _check(lib().nmc_instance_bind(self._h, ctypes.c_void_p(self._buf.data_ptr()), self._buf.numel(),
                                       _stream(stream)))
        return self

    def free(self):
        if self._h:
            lib().nmc_instance_free(self._h)
            self._h = None
        self._buf = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Replicas:
    """R independent chains of one bound instance (nmc_replicas_create)."""

    def __init__(self, inst: Instance, n_replicas: int, seed: int, stream=None):
        self.inst = inst
        # the instance's device arena must outlive these replicas even when
        # the instance object is released first (explicitly, or by the cycle
        # collector, which finalizes in no fixed order)
        self._inst_buf = inst._buf
        self.R = int(n_replicas)
        self.seed = int(seed)
        _, rb = inst.footprint(self.R)
        self._buf = _device_buffer(rb)
        h = ctypes.c_void_p()
        _check(lib().nmc_replicas_create(inst._h, self.R, ctypes.c_uint64(self.seed),
                                         ctypes.c_void_p(self._buf.data_ptr()), self._buf.numel(),
                                         _stream(stream), ctypes.byref(h)))
        self._h = h

    # -- schedule calls
    def _run(self, fn, beta, profile, class_of, target, stream):
        b = np.atleast_2d(np.ascontiguousarray(beta, np.float64))
        nc, S = b.shape
        b = np.ascontiguousarray(b)
        cls = None if class_of is None else np.ascontiguousarray(class_of, np.uint8)
        if isinstance(profile, str):
            profile = PROFILE[profile]
        if cls is not None and profile == 0:
            profile = PROFILE["host"]
        _check(fn(self._h, _ptr(b), nc, S, int(profile), _ptr(cls), ctypes.c_int64(int(target)), _stream(stream)))

    def anneal(self, beta, profile="homogeneous", class_of=None, target=-1, stream=None):
        self._run(lib().nmc_anneal, beta, profile, class_of, target, stream)

    def reanneal(self, beta, profile="backbone", class_of=None, target=-1, stream=None):
        self._run(lib().nmc_reanneal, beta, profile, class_of, target, stream)

    def anneal_noalloc(self, beta, profile="homogeneous", class_of=None, target=-1, stream=None):
        """nmc_anneal_noalloc: nmc_anneal with the thresholds in the library's
        fixed device array (no device allocation)."""
        self._run(lib().nmc_anneal_noalloc, beta, profile, class_of, target, stream)

    def pt_run(self, beta, n_rounds, sweeps_per_round=1, first_parity=0, target=-1, stream=None):
        """Replica-exchange rounds over the ladder beta (replica r = i * C + c
        at beta[i]); returns (accepted, attempted) per pair position."""
        b = np.ascontiguousarray(beta, np.float64)
        M = b.size
        acc = np.zeros(max(M - 1, 1), np.int64)
        att = np.zeros(max(M - 1, 1), np.int64)
        _check(lib().nmc_pt_run(self._h, _ptr(b), M, int(n_rounds), int(sweeps_per_round), int(first_parity),
                                ctypes.c_int64(int(target)), _ptr(acc), _ptr(att), _stream(stream)))
        return acc[: M - 1], att[: M - 1]

    def apt_ladder(self, beta_first, alpha=1.1, sigma_min=1.0, equil_sweeps=50, meas_sweeps=10, max_temps=256,
                   stream=None):
        """Adaptive ladder: returns (betas, sigmas)."""
        b = np.zeros(int(max_temps), np.float64)
        sg = np.zeros(int(max_temps), np.float64)
        k = _I32()
        _check(lib().nmc_apt_ladder(self._h, float(beta_first), float(alpha), float(sigma_min), int(equil_sweeps),
                                    int(meas_sweeps), int(max_temps), _ptr(b), _ptr(sg), ctypes.byref(k),
                                    _stream(stream)))
        return b[: k.value].copy(), sg[: k.value].copy()

    def lbp_backbone(self, replica, which="best", beta=1.0, lambda0=4.0, lambda_ratio=0.8, lambda_min=0.05,
                     max_iter=200, tol=1e-10, p_min=-2.0, theta_seed=0.99, theta_cut=0.95, stream=None):
        """Surrogate-Hamiltonian LBP around one replica's state and connected
        backbone growth; the backbone becomes the device class array.
        Returns dict(cls, mag, corr, label, lambda, steps, iterations,
        converged, delta, overlap, self_overlap, backbone_size, n_clusters,
        largest_cluster, rigid_clauses, seed_clauses)."""
        n, m = self.inst.n, self.inst.info.n_clauses
        cfg = LbpConfig(float(beta), float(lambda0), float(lambda_ratio), float(lambda_min), int(max_iter),
                        float(tol), float(p_min), float(theta_seed), float(theta_cut))
        res = LbpResult()
        cls = np.zeros(max(n, 1), np.uint8)
        mag = np.zeros(max(n, 1), np.float64)
        corr = np.zeros(max(m, 1), np.float64)
        label = np.zeros(max(n, 1), np.int32)
        _check(lib().nmc_lbp_backbone(self._h, int(replica), STATE[which], ctypes.byref(cfg), ctypes.byref(res),
                                      _ptr(cls), _ptr(mag), _ptr(corr), _ptr(label), _stream(stream)))
        out = {f: getattr(res, f) for f, _ in LbpResult._fields_}
        out["lambda"] = out.pop("lambda_")
        out.update(cls=cls[:n], mag=mag[:n], corr=corr[:m], label=label[:n])
        return out

    def estimate_backbone(self, thr_num=9, thr_den=10, expand=True, stream=None):
        n = self.inst.n
        cls = np.zeros(n, np.uint8)
        counts = np.zeros(n * n if self.inst.kind == KIND_QAP else n, np.int32)
        _check(lib().nmc_estimate_backbone(self._h, int(thr_num), int(thr_den), int(bool(expand)), _ptr(cls),
                                           _ptr(counts), _stream(stream)))
        if self.inst.kind == KIND_QAP:
            counts = counts.reshape(n, n)
        return cls, counts

    def estimate_backbone_device(self, thr_num=9, thr_den=10, expand=True, stream=None):
        """Backbone classes kept on the device only (no host copy, no sync)."""
        _check(lib().nmc_estimate_backbone(self._h, int(thr_num), int(thr_den), int(bool(expand)), None, None,
                                           _stream(stream)))

    def best_energy(self, stream=None):
        R = self.R
        best = ctypes.c_int64()
        nz = ctypes.c_int32()
        bpr = np.zeros(R, np.int64)
        e = np.zeros(R, np.int64)
        fh = np.zeros(R, np.int32)
        _check(lib().nmc_best_energy(self._h, ctypes.byref(best), ctypes.byref(nz), _ptr(bpr), _ptr(e), _ptr(fh),
                                     _stream(stream)))
        return dict(best=best.value, n_at_zero=nz.value, best_per_replica=bpr, energy=e, first_hit=fh)

    def recount(self, stream=None):
        e = np.zeros(self.R, np.int64)
        _check(lib().nmc_recount(self._h, _ptr(e), _stream(stream)))
        return e

    def get_state(self, which="current", stream=None):
        out = np.zeros((self.R, self.inst.n), np.uint8)
        _check(lib().nmc_get_state(self._h, STATE[which], _ptr(out), out.nbytes, _stream(stream)))
        return out

    def set_state(self, x, sweeps_done, stream=None):
        x = np.ascontiguousarray(x, np.uint8)
        _check(lib().nmc_set_state(self._h, _ptr(x), x.nbytes, ctypes.c_uint32(int(sweeps_done)), _stream(stream)))

    def sweeps_done(self):
        r, s, t = _I32(), _U64(), _U32()
        _check(lib().nmc_replicas_info(self._h, ctypes.byref(r), ctypes.byref(s), ctypes.byref(t)))
        return t.value

    def set_tuning(self, block_threads=0):
        _check(lib().nmc_set_tuning(self._h, int(block_threads)))

    def set_replicas_per_workgroup(self, reps=0):
        """k-SAT sweep workgroups of 4 (default) or 8 replicas."""
        _check(lib().nmc_set_replicas_per_workgroup(self._h, int(reps)))

    def replicas_per_workgroup(self):
        r = ctypes.c_int32()
        _check(lib().nmc_get_tuning(self._h, None, ctypes.byref(r)))
        return r.value

    def tune(self, probe_sweeps=3, stream=None):
        """nmc_tune: (workgroup size, replicas per workgroup) chosen and kept."""
        b, r = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().nmc_tune(self._h, int(probe_sweeps), ctypes.byref(b), ctypes.byref(r), _stream(stream)))
        return b.value, r.value

    def set_profiling(self, enable=True):
        _check(lib().nmc_set_profiling(self._h, int(bool(enable))))

    def kernel_time(self, reset=False):
        ms = ctypes.c_double()
        launches = ctypes.c_int64()
        att = ctypes.c_double()
        _check(lib().nmc_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(launches), ctypes.byref(att),
                                     int(bool(reset))))
        return dict(ms=ms.value, launches=launches.value, attempts=att.value)

    def accept_count(self, reset=False, stream=None):
        """Moves accepted by the sweep kernels since creation or the last reset."""
        v = ctypes.c_uint64()
        _check(lib().nmc_accept_count(self._h, ctypes.byref(v), int(bool(reset)), _stream(stream)))
        return v.value

    def cluster_flip(self, label, beta, target=-1, stream=None):
        """One collective-move sweep over the clusters of `label` (e.g. the
        label of lbp_backbone); returns the clusters flipped per replica."""
        lab = np.ascontiguousarray(label, np.int32)
        acc = np.zeros(self.R, np.int32)
        _check(lib().nmc_cluster_flip(self._h, _ptr(lab), float(beta), ctypes.c_int64(int(target)), _ptr(acc),
                                      _stream(stream)))
        return acc

    def whiten(self, which="best", white=False, stream=None):
        """Frozen variables per replica after whitening; with white=True also
        the [R][N] white mask.  Returns (frozen, white_or_None, passes)."""
        fz = np.zeros(self.R, np.int32)
        wm = np.zeros((self.R, self.inst.n), np.uint8) if white else None
        p = _I32()
        _check(lib().nmc_whiten(self._h, STATE[which], _ptr(fz), _ptr(wm), ctypes.byref(p), _stream(stream)))
        return fz, wm, p.value

    def lbp_kernel_time(self, reset=False):
        ms = ctypes.c_double()
        it = ctypes.c_int64()
        _check(lib().nmc_lbp_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(it), int(bool(reset))))
        return dict(ms=ms.value, iterations=it.value)

    def free(self):
        if getattr(self, "_h", None):
            lib().nmc_replicas_free(self._h)
            self._h = None
        self._buf = None
        self._inst_buf = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Batch:
    """Many replica sets run by one launch per kernel kind (nmc_batch_*)."""

    def __init__(self, sets):
        self.sets = list(sets)
        arr = (ctypes.c_void_p * len(self.sets))(*[s._h for s in self.sets])
        h = ctypes.c_void_p()
        _check(lib().nmc_batch_create(arr, len(self.sets), ctypes.byref(h)))
        self._h = h

    def _targets(self, targets):
        if targets is None:
            return None
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(targets, np.int64), (len(self.sets),)))
        return t

    def set_tuning(self, block_threads=0):
        _check(lib().nmc_batch_set_tuning(self._h, int(block_threads)))

    def tune(self, probe_sweeps=3, stream=None):
        chosen = ctypes.c_int32()
        _check(lib().nmc_batch_tune(self._h, int(probe_sweeps), ctypes.byref(chosen), _stream(stream)))
        return chosen.value

    def anneal(self, beta, profile="homogeneous", targets=None, stream=None):
        b = np.ascontiguousarray(np.atleast_2d(np.asarray(beta, np.float64)))
        nc, S = b.shape
        t = self._targets(targets)
        _check(lib().nmc_batch_anneal(self._h, _ptr(b), nc, S, PROFILE[profile] if isinstance(profile, str) else profile,
                                      _ptr(t), _stream(stream)))

    def lbp_backbone(self, replicas, which="best", beta=1.0, lambda0=4.0, lambda_ratio=0.8, lambda_min=0.05,
                     max_iter=200, tol=1e-10, p_min=-2.0, theta_seed=0.99, theta_cut=0.95, stream=None):
        """LBP backbone of every set around replica replicas[i]; returns one
        result dict per set (the fields of Replicas.lbp_backbone without the
        arrays)."""
        reps = np.ascontiguousarray(replicas, np.int32)
        cfg = LbpConfig(float(beta), float(lambda0), float(lambda_ratio), float(lambda_min), int(max_iter),
                        float(tol), float(p_min), float(theta_seed), float(theta_cut))
        res = (LbpResult * max(len(reps), 1))()
        _check(lib().nmc_batch_lbp_backbone(self._h, _ptr(reps), STATE[which], ctypes.byref(cfg),
                                            ctypes.cast(res, ctypes.c_void_p), _stream(stream)))
        out = []
        for k in range(len(reps)):
            d = {f: getattr(res[k], f) for f, _ in LbpResult._fields_}
            d["lambda"] = d.pop("lambda_")
            out.append(d)
        return out

    def estimate_backbone(self, thr_num=9, thr_den=10, expand=True, stream=None):
        _check(lib().nmc_batch_estimate_backbone(self._h, int(thr_num), int(thr_den), int(bool(expand)),
                                                 _stream(stream)))

    def run_plan(self, anneal_beta, rounds, reanneal_beta, thr_num=9, thr_den=10, expand=True, targets=None,
                 use_graph=True, chunk_sweeps=0, stream=None):
        a = np.ascontiguousarray(np.asarray(anneal_beta, np.float64).reshape(-1))
        r = np.ascontiguousarray(np.asarray(reanneal_beta, np.float64).reshape(2, -1))
        plan = Plan(a.ctypes.data, a.size, int(rounds), r.ctypes.data, r.shape[1], int(thr_num), int(thr_den),
                    int(bool(expand)), int(chunk_sweeps))
        t = self._targets(targets)
        _check(lib().nmc_batch_run_plan(self._h, ctypes.byref(plan), _ptr(t), int(bool(use_graph)), _stream(stream)))

    def run(self, plans, targets=None, use_graph=True, stream=None):
        """nmc_batch_run: one plan per member set.  Each plan is a dict with
        anneal_beta (S_a values), rounds, reanneal_beta (2 x S_r: cold row,
        hot row; may be omitted when rounds = 0) and optionally thr_num,
        thr_den, expand, chunk_sweeps."""
        plans = list(plans)
        if len(plans) != len(self.sets):
            raise NmcError(-1, f"{len(plans)} plans for {len(self.sets)} sets")
        keep = []
        arr = (Plan * max(1, len(plans)))()
        for i, p in enumerate(plans):
            a = np.ascontiguousarray(np.asarray(p["anneal_beta"], np.float64).reshape(-1))
            rb = p.get("reanneal_beta")
            r = np.ascontiguousarray(np.asarray(rb if rb is not None else np.zeros((2, 0)), np.float64).reshape(2, -1))
            keep += [a, r]
            arr[i] = Plan(a.ctypes.data, a.size, int(p.get("rounds", 0)), r.ctypes.data, r.shape[1],
                          int(p.get("thr_num", 9)), int(p.get("thr_den", 10)), int(bool(p.get("expand", True))),
                          int(p.get("chunk_sweeps", 0)))
        t = self._targets(targets)
        _check(lib().nmc_batch_run(self._h, ctypes.cast(arr, ctypes.c_void_p), _ptr(t), int(bool(use_graph)),
                                   _stream(stream)))

    def graph_info(self):
        """(graphs captured, calls that replayed the kept graph)."""
        c, r = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().nmc_batch_graph_info(self._h, ctypes.byref(c), ctypes.byref(r)))
        return c.value, r.value

    def set_members(self, sets):
        """Replace the member sets (same rules as the constructor)."""
        sets = list(sets)
        arr = (ctypes.c_void_p * len(sets))(*[x._h for x in sets])
        _check(lib().nmc_batch_set_members(self._h, arr, len(sets)))
        self.sets = sets

    def step(self, segments, n_sweeps, thr_num=9, thr_den=10, expand=True, stream=None):
        """One batched step of n_sweeps sweeps; every set at its own constant
        beta pair.  segments: per set (beta_cold, beta_hot, profile,
        backbone_before, target) with profile a name or None (idle).
        Returns [(best, n_at_zero, first_hit)] per set."""
        segs = (Segment * len(self.sets))()
        for g, (b0, b1, prof, bb, tgt) in zip(segs, segments):
            g.beta[0], g.beta[1] = float(b0), float(b1)
            g.profile = -1 if prof is None else (PROFILE[prof] if isinstance(prof, str) else int(prof))
            g.backbone_before = int(bool(bb))
            g.target = int(tgt)
        st = (SetStatus * len(self.sets))()
        _check(lib().nmc_batch_step(self._h, segs, int(n_sweeps), int(thr_num), int(thr_den), int(bool(expand)), st,
                                    _stream(stream)))
        return [(x.best, x.n_at_zero, x.first_hit) for x in st]

    def set_profiling(self, enable=True):
        _check(lib().nmc_batch_set_profiling(self._h, int(bool(enable))))

    def kernel_time(self, reset=False):
        ms = ctypes.c_double()
        launches = ctypes.c_int64()
        att = ctypes.c_double()
        _check(lib().nmc_batch_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(launches), ctypes.byref(att),
                                           int(bool(reset))))
        return dict(ms=ms.value, launches=launches.value, attempts=att.value)

    def free(self):
        if getattr(self, "_h", None):
            lib().nmc_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Continuous-batching solve server (nmc_server_*): a native worker thread
    advances every admitted request by chunk_sweeps sweeps per round in one
    batched launch per kernel kind."""

    def __init__(self, hbm_cap_bytes=0, chunk_sweeps=0, max_active=0, loader_threads=0, block_threads=0,
                 thr_num=0, thr_den=0, expand=True):
        import torch
        if not torch.cuda.is_available():
            raise NmcError(-3, "no GPU visible to torch")
        torch.cuda.init()
        cfg = ServerConfig(int(hbm_cap_bytes), int(chunk_sweeps), int(max_active), int(loader_threads),
                           int(block_threads), int(thr_num), int(thr_den), int(bool(expand)))
        h = ctypes.c_void_p()
        _check(lib().nmc_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def submit_ksat(self, n_vars, clause_ptr, lits, n_replicas, seed, beta0, beta1, beta_hot, anneal_sweeps,
                    rounds, reanneal_sweeps, target=None, budget_s=0.0, class_cap=0):
        cp = np.ascontiguousarray(clause_ptr, np.int32)
        li = np.ascontiguousarray(lits, np.int32)
        r = Request(kind=KIND_KSAT, n_vars=int(n_vars), n_clauses=cp.size - 1, class_cap=int(class_cap),
                    clause_ptr=cp.ctypes.data, lits=li.ctypes.data)
        return self._submit(r, n_replicas, seed, beta0, beta1, beta_hot, anneal_sweeps, rounds, reanneal_sweeps,
                            target, budget_s)

    def submit_qap(self, flow, dist, n_replicas, seed, beta0, beta1, beta_hot, anneal_sweeps, rounds,
                   reanneal_sweeps, target=None, budget_s=0.0):
        F = np.ascontiguousarray(flow, np.int32)
        D = np.ascontiguousarray(dist, np.int32)
        r = Request(kind=KIND_QAP, n=F.shape[0], flow=F.ctypes.data, dist=D.ctypes.data)
        return self._submit(r, n_replicas, seed, beta0, beta1, beta_hot, anneal_sweeps, rounds, reanneal_sweeps,
                            target, budget_s)

    def _submit(self, r, n_replicas, seed, beta0, beta1, beta_hot, anneal_sweeps, rounds, reanneal_sweeps, target,
                budget_s):
        r.n_replicas, r.seed = int(n_replicas), int(seed)
        r.beta0, r.beta1, r.beta_hot = float(beta0), float(beta1), float(beta_hot)
        r.anneal_sweeps, r.rounds, r.reanneal_sweeps = int(anneal_sweeps), int(rounds), int(reanneal_sweeps)
        r.has_target = int(target is not None)
        r.target = int(target) if target is not None else 0
        r.budget_s = float(budget_s)
        rid = ctypes.c_uint64()
        _check(lib().nmc_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        return rid.value

    def poll(self, rid):
        res = Result()
        _check(lib().nmc_server_poll(self._h, int(rid), ctypes.byref(res)))
        return dict(status=REQ_STATUS[res.status], n_at_zero=res.n_at_zero, best=res.best,
                    first_hit=res.first_hit_sweep, sweeps_done=res.sweeps_done, t_submit=res.t_submit,
                    t_admit=res.t_admit, t_done=res.t_done, device_bytes=res.device_bytes,
                    message=res.message.decode(errors="replace"))

    def wait_idle(self, timeout_s=600.0):
        """True when every submitted request completed within timeout_s."""
        rc = lib().nmc_server_wait_idle(self._h, float(timeout_s))
        if rc == -4:
            return False
        _check(rc)
        return True

    def stats(self):
        st = ServerStats()
        _check(lib().nmc_server_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def now(self):
        return lib().nmc_server_now(self._h)

    def free(self):
        if getattr(self, "_h", None):
            lib().nmc_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
