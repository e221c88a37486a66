"""ctypes binding of libmc3.so with the same names as the C ABI (include/mc3.h).

Marshalling only: the workspace is a torch uint8 CUDA tensor, the stream is torch's
current HIP stream; every computation happens in the library's kernels.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmc3.so")
CEIL_PATH = os.path.join(HERE, "libmc3ceil.so")
CEIL_EXPORTS = ["mc3c_mfma_ceiling", "mc3c_mfma_mix"]
MFMA_MIXES = {0: "none", 1: "split_kernel", 2: "tile_64x128", 3: "lds_reads_32", 4: "lds_reads_16"}

MC3_OK, MC3_E_ARG, MC3_E_DEVICE, MC3_E_STATE = 0, -1, -3, -4
MC3_J_PM1, MC3_J_GAUSS = 0, 1
MC3_E_UNSUPPORTED, MC3_E_NUMERIC, MC3_E_WORKSPACE = -5, -6, -7
MC3_FP64, MC3_SPLIT_BF16 = 0, 1
MC3_RULE_MCMCMC, MC3_RULE_METROPOLIS = 0, 1
MC3_SCORER_GEMM, MC3_SCORER_DELTA, MC3_SCORER_AUTO = 0, 1, 2
MC3_LAW_UNIFORM, MC3_LAW_LINE, MC3_LAW_TABLE, MC3_LAW_BIASED = 0, 1, 2, 3
MC3_ENERGY_EXACT, MC3_ENERGY_SCORED = 0, 1

PRECISIONS = {"fp64": MC3_FP64, "split_bf16": MC3_SPLIT_BF16}
RULES = {"mcmcmc": MC3_RULE_MCMCMC, "metropolis": MC3_RULE_METROPOLIS}
SCORERS = {"gemm": MC3_SCORER_GEMM, "delta": MC3_SCORER_DELTA, "auto": MC3_SCORER_AUTO}
LAWS = {"uniform": MC3_LAW_UNIFORM, "line": MC3_LAW_LINE, "table": MC3_LAW_TABLE, "biased": MC3_LAW_BIASED}
ENERGY_UPDATES = {"exact": MC3_ENERGY_EXACT, "scored": MC3_ENERGY_SCORED}

STATUS_NAMES = {0: "MC3_OK", -1: "MC3_E_ARG", -3: "MC3_E_DEVICE", -4: "MC3_E_STATE",
                -5: "MC3_E_UNSUPPORTED", -6: "MC3_E_NUMERIC", -7: "MC3_E_WORKSPACE"}

# every symbol include/mc3.h declares
EXPORTS = ["mc3_workspace_size", "mc3_create", "mc3_destroy", "mc3_init_couplings", "mc3_init_chains",
           "mc3_propose", "mc3_score_candidates", "mc3_select", "mc3_step_n", "mc3_recompute", "mc3_measure",
           "mc3_read_records", "mc3_read_candidates", "mc3_read_means", "mc3_timing_enable", "mc3_timing_read",
           "mc3_sync", "mc3_last_error", "mc3_version", "mc3_batch_workspace_size", "mc3_batch_create",
           "mc3_init_couplings_instance", "mc3_generate_couplings", "mc3_step_n_per_instance", "mc3_step_n_graph", "mc3_checkpoint_save",
           "mc3_checkpoint_load", "mc3_set_generation", "mc3_select_betas", "mc3_step_n_schedules", "mc3_create_noalloc"]
NOALLOC_BYTES = 16 << 20   # MC3_NOALLOC_BYTES


class Config(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32), ("chains", ctypes.c_int32),
                ("kmin", ctypes.c_int32), ("kmax", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("trace_steps", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("chain_base", ctypes.c_uint32), ("mean_steps", ctypes.c_int32),
                ("near_tie_tol", ctypes.c_double), ("scorer", ctypes.c_int32), ("arity", ctypes.c_int32),
                ("law", ctypes.c_int32), ("law_table", ctypes.POINTER(ctypes.c_double)),
                ("tile_cols", ctypes.c_int32), ("recompute_every", ctypes.c_int32),
                ("energy_update", ctypes.c_int32), ("drift_tol", ctypes.c_double), ("bias", ctypes.c_double)]


class InstanceDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32), ("chains", ctypes.c_int32),
                ("kmin", ctypes.c_int32), ("kmax", ctypes.c_int32)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("n_instances", ctypes.c_int32), ("precision", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("trace_steps", ctypes.c_int32), ("mean_steps", ctypes.c_int32), ("chain_base", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("near_tie_tol", ctypes.c_double),
                ("instances", ctypes.POINTER(InstanceDesc)), ("scorer", ctypes.c_int32), ("arity", ctypes.c_int32),
                ("law", ctypes.c_int32), ("law_table", ctypes.POINTER(ctypes.c_double)),
                ("tile_cols", ctypes.c_int32), ("recompute_every", ctypes.c_int32),
                ("energy_update", ctypes.c_int32), ("drift_tol", ctypes.c_double), ("bias", ctypes.c_double)]


class Schedule(ctypes.Structure):
    _fields_ = [("beta0", ctypes.c_double), ("beta1", ctypes.c_double), ("total", ctypes.c_int64)]


class Summary(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int64), ("moves", ctypes.c_int64), ("near_ties", ctypes.c_int64),
                ("min_margin", ctypes.c_double), ("max_drift", ctypes.c_double),
                ("recomputes", ctypes.c_int64), ("drift_events", ctypes.c_int64)]


RECORD_DTYPE = np.dtype([("r", np.int32), ("vstar", np.int32), ("e_cur", np.float64), ("e_bar", np.float64),
                         ("margin", np.float64), ("flags", np.uint32), ("step", np.uint32)])
assert RECORD_DTYPE.itemsize == 40


class MC3Error(RuntimeError):
    def __init__(self, status: int, what: str, msg: str = ""):
        super().__init__(f"{what} -> {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmc3.so (built by paper_2102_05613_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2102_05613_amd.build.build() first")
    L = ctypes.CDLL(LIB_PATH)
    P, c = ctypes.POINTER, ctypes
    vp = c.c_void_p
    L.mc3_workspace_size.argtypes = [P(Config), P(c.c_size_t)]
    L.mc3_create.argtypes = [P(Config), vp, c.c_size_t, vp, P(vp)]
    L.mc3_create_noalloc.argtypes = [P(Config), vp, P(vp)]
    L.mc3_destroy.argtypes = [vp]
    L.mc3_init_couplings.argtypes = [vp, P(c.c_double), c.c_int64, c.c_double]
    L.mc3_init_chains.argtypes = [vp, vp]
    L.mc3_propose.argtypes = [vp, c.c_uint32]
    L.mc3_score_candidates.argtypes = [vp, vp]
    L.mc3_select.argtypes = [vp, c.c_uint32, c.c_double]
    L.mc3_step_n.argtypes = [vp, c.c_uint32, c.c_int64, c.c_double, c.c_double, c.c_int64]
    L.mc3_recompute.argtypes = [vp]
    L.mc3_measure.argtypes = [vp, vp, vp, P(Summary)]
    L.mc3_read_records.argtypes = [vp, c.c_uint32, c.c_int32, vp]
    L.mc3_read_candidates.argtypes = [vp, vp, vp]
    L.mc3_read_means.argtypes = [vp, c.c_uint32, c.c_int32, vp]
    L.mc3_timing_enable.argtypes = [vp, c.c_int32]
    L.mc3_timing_read.argtypes = [vp, P(c.c_double), P(c.c_int64)]
    L.mc3_sync.argtypes = [vp]
    L.mc3_batch_workspace_size.argtypes = [P(BatchConfig), P(c.c_size_t)]
    L.mc3_batch_create.argtypes = [P(BatchConfig), vp, c.c_size_t, vp, P(vp)]
    L.mc3_init_couplings_instance.argtypes = [vp, c.c_int32, P(c.c_double), c.c_int64, c.c_double]
    L.mc3_step_n_per_instance.argtypes = [vp, c.c_uint32, c.c_int64, c.c_double, c.c_double, c.c_int64]
    L.mc3_step_n_graph.argtypes = [vp, c.c_uint32, c.c_int64, c.c_double, c.c_double, c.c_int64]
    L.mc3_generate_couplings.argtypes = [vp, c.c_int32, c.c_int32, c.c_uint64]
    L.mc3_checkpoint_save.argtypes = [vp, vp, P(c.c_size_t)]
    L.mc3_checkpoint_load.argtypes = [vp, vp, c.c_size_t]
    L.mc3_set_generation.argtypes = [vp, c.c_int32, c.c_int32, vp, vp, vp, vp, vp]
    L.mc3_select_betas.argtypes = [vp, c.c_uint32, P(c.c_double)]
    L.mc3_step_n_schedules.argtypes = [vp, c.c_uint32, c.c_int64, P(Schedule)]
    L.mc3_last_error.argtypes = [vp]
    L.mc3_last_error.restype = c.c_char_p
    L.mc3_version.restype = c.c_char_p
    for name in EXPORTS:
        if name not in ("mc3_last_error", "mc3_version"):
            getattr(L, name).restype = c.c_int
    _lib = L
    return L


def make_config(N: int, M: int, chains: int, kmin: int, kmax: int, precision: str = "split_bf16",
                rule: str = "mcmcmc", trace_steps: int = 0, seed: int = 0, chain_base: int = 0,
                near_tie_tol: float = -1.0, mean_steps: int = 0, scorer: str = "gemm", arity: int = 0,
                law: str = "uniform", law_table=None, tile_cols: int = 0, recompute_every: int = 0,
                energy_update: str = "exact", drift_tol: float = -1.0, bias: float = 0.0) -> Config:
    """arity 0: the M-ary star; law "line" (arity 1): the line-graph addition process;
    law "table": root weights law_table[0..M]; tile_cols 0: the split scoring tile width
    by column count, else 128, 256 or 512; recompute_every K > 0: FP64 recompute of the
    carried energies after every step t with (t+1) % K == 0; energy_update "exact" or
    "scored"."""
    tab = _table(law_table)
    cfg = Config(N, M, chains, kmin, kmax, PRECISIONS[precision], RULES[rule], trace_steps, seed, chain_base,
                 mean_steps, near_tie_tol, SCORERS[scorer], arity, LAWS[law],
                 None if tab is None else tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), tile_cols,
                 recompute_every, ENERGY_UPDATES[energy_update], drift_tol, bias)
    cfg._keep_table = tab   # the table lives as long as the config
    return cfg


def _table(law_table):
    if law_table is None:
        return None
    return np.ascontiguousarray(law_table, dtype=np.float64).ravel().copy()


def make_batch_config(instances, precision: str = "split_bf16", rule: str = "mcmcmc", trace_steps: int = 0,
                      seed: int = 0, chain_base: int = 0, near_tie_tol: float = -1.0,
                      mean_steps: int = 0, scorer: str = "gemm", arity: int = 0, law: str = "uniform",
                      law_table=None, tile_cols: int = 0, recompute_every: int = 0, energy_update: str = "exact",
                      drift_tol: float = -1.0, bias: float = 0.0) -> BatchConfig:
    """instances: sequence of (N, M, chains, kmin, kmax); law "table": law_table holds
    the root weights of every instance, M_i+1 values each, in instance order;
    tile_cols as in make_config."""
    arr = (InstanceDesc * len(instances))(*[InstanceDesc(*map(int, d)) for d in instances])
    tab = _table(law_table)
    cfg = BatchConfig(len(instances), PRECISIONS[precision], RULES[rule], trace_steps, mean_steps, chain_base, seed,
                      near_tie_tol, ctypes.cast(arr, ctypes.POINTER(InstanceDesc)), SCORERS[scorer], arity, LAWS[law],
                      None if tab is None else tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), tile_cols,
                      recompute_every, ENERGY_UPDATES[energy_update], drift_tol, bias)
    cfg._keep = arr   # the descriptor array lives as long as the config
    cfg._keep_table = tab
    return cfg


def workspace_size(cfg) -> int:
    n = ctypes.c_size_t()
    if isinstance(cfg, BatchConfig):
        st = lib().mc3_batch_workspace_size(ctypes.byref(cfg), ctypes.byref(n))
    else:
        st = lib().mc3_workspace_size(ctypes.byref(cfg), ctypes.byref(n))
    if st != MC3_OK:
        raise MC3Error(st, "mc3_workspace_size")
    return int(n.value)


class Context:
    """One SK instance (Config) or a batch of instances (BatchConfig) with their
    chains on the current GPU.  noalloc (a Config only): mc3_create_noalloc, the
    library's fixed device array as the workspace instead of a torch allocation."""

    def __init__(self, cfg, device=None, noalloc: bool = False):
        import torch
        self.cfg = cfg
        if isinstance(cfg, BatchConfig):
            self.instances = [(d.N, d.M, d.chains, d.kmin, d.kmax) for d in cfg.instances[:cfg.n_instances]]
        else:
            self.instances = [(cfg.N, cfg.M, cfg.chains, cfg.kmin, cfg.kmax)]
        self.N, self.M = self.instances[0][0], self.instances[0][1]
        self.chains = sum(d[2] for d in self.instances)
        self.words = max((d[0] + 31) // 32 for d in self.instances)
        h = ctypes.c_void_p()
        if noalloc:
            if isinstance(cfg, BatchConfig):
                raise ValueError("mc3_create_noalloc takes a single-instance Config")
            self.workspace = None
            self.stream = torch.cuda.current_stream(device)
            st = lib().mc3_create_noalloc(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
            if st != MC3_OK:
                raise MC3Error(st, "mc3_create_noalloc")
            self.h = h
            return
        nbytes = workspace_size(cfg)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")
        self.stream = torch.cuda.current_stream(self.workspace.device)
        create = lib().mc3_batch_create if isinstance(cfg, BatchConfig) else lib().mc3_create
        st = create(ctypes.byref(cfg), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != MC3_OK:
            raise MC3Error(st, "mc3_create")
        self.h = h

    def _check(self, st: int, what: str):
        if st != MC3_OK:
            raise MC3Error(st, what, lib().mc3_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().mc3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the ABI calls
    def init_couplings(self, J: np.ndarray, scale: float, instance: int = 0):
        N = self.instances[instance][0]
        J = np.ascontiguousarray(J, dtype=np.float64)
        assert J.shape == (N, N)
        self._check(lib().mc3_init_couplings_instance(self.h, instance,
                                                      J.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), N,
                                                      float(scale)), "mc3_init_couplings_instance")

    def generate_couplings(self, kind: int, seed: int, instance: int = 0) -> float:
        """Seeded couplings generated on the device (kind MC3_J_PM1 or MC3_J_GAUSS);
        returns the energy scale they carry."""
        self._check(lib().mc3_generate_couplings(self.h, instance, int(kind), int(seed)), "mc3_generate_couplings")
        N = self.instances[instance][0]
        return 1.0 / math.sqrt(N) if kind == MC3_J_PM1 else 1.0

    def init_chains(self, spins: Optional[np.ndarray] = None):
        """spins: None, or int8 [chains, N] (one instance) / the instances' blocks
        [chains_i * N_i] one after another (a batch)."""
        p = None
        if spins is not None:
            spins = np.ascontiguousarray(spins, dtype=np.int8)
            assert spins.size == sum(d[0] * d[2] for d in self.instances)
            p = spins.ctypes.data
        self._check(lib().mc3_init_chains(self.h, p), "mc3_init_chains")

    def propose(self, step: int):
        self._check(lib().mc3_propose(self.h, step), "mc3_propose")

    def score_candidates(self, out=None):
        """out: optional torch float64 CUDA tensor [chains*M] receiving the energies."""
        p = None if out is None else ctypes.c_void_p(out.data_ptr())
        self._check(lib().mc3_score_candidates(self.h, p), "mc3_score_candidates")

    def select(self, step: int, beta: float):
        self._check(lib().mc3_select(self.h, step, float(beta)), "mc3_select")

    def select_betas(self, step: int, betas):
        """mc3_select with one inverse temperature per instance."""
        b = np.ascontiguousarray(betas, dtype=np.float64)
        assert b.shape == (len(self.instances),)
        self._check(lib().mc3_select_betas(self.h, step, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    "mc3_select_betas")

    def step_n_schedules(self, step0: int, n: int, schedules):
        """mc3_step_n with one (beta0, beta1, total) schedule per instance."""
        assert len(schedules) == len(self.instances)
        arr = (Schedule * len(schedules))(*[Schedule(float(a), float(b), int(t)) for a, b, t in schedules])
        self._check(lib().mc3_step_n_schedules(self.h, step0, n, ctypes.cast(arr, ctypes.POINTER(Schedule))),
                    "mc3_step_n_schedules")

    def step_n(self, step0: int, n: int, beta0: float, beta1: float, total: int):
        self._check(lib().mc3_step_n(self.h, step0, n, float(beta0), float(beta1), total), "mc3_step_n")

    def step_n_graph(self, step0: int, n: int, beta0: float, beta1: float, total: int):
        self._check(lib().mc3_step_n_graph(self.h, step0, n, float(beta0), float(beta1), total), "mc3_step_n_graph")

    def step_n_per_instance(self, step0: int, n: int, beta0: float, beta1: float, total: int):
        self._check(lib().mc3_step_n_per_instance(self.h, step0, n, float(beta0), float(beta1), total),
                    "mc3_step_n_per_instance")

    def checkpoint_save(self) -> bytes:
        n = ctypes.c_size_t()
        self._check(lib().mc3_checkpoint_save(self.h, None, ctypes.byref(n)), "mc3_checkpoint_save")
        buf = ctypes.create_string_buffer(n.value)
        self._check(lib().mc3_checkpoint_save(self.h, buf, ctypes.byref(n)), "mc3_checkpoint_save")
        return buf.raw[:n.value]

    def checkpoint_load(self, data: bytes):
        buf = ctypes.create_string_buffer(data, len(data))
        self._check(lib().mc3_checkpoint_load(self.h, buf, len(data)), "mc3_checkpoint_load")

    def recompute(self):
        self._check(lib().mc3_recompute(self.h), "mc3_recompute")

    def measure(self):
        e = np.zeros(self.chains, dtype=np.float64)
        bits = np.zeros((self.chains, self.words), dtype=np.uint32)
        s = Summary()
        self._check(lib().mc3_measure(self.h, e.ctypes.data, bits.ctypes.data, ctypes.byref(s)), "mc3_measure")
        summ = {k: getattr(s, k) for k, _ in Summary._fields_}
        return e, bits, summ

    def read_records(self, first: int, n: int) -> np.ndarray:
        out = np.zeros((n, self.chains), dtype=RECORD_DTYPE)
        self._check(lib().mc3_read_records(self.h, first, n, out.ctypes.data), "mc3_read_records")
        return out

    def read_candidates(self):
        bits = np.zeros((self.chains, self.M, self.words), dtype=np.uint32)
        roots = np.zeros(self.chains, dtype=np.int32)
        self._check(lib().mc3_read_candidates(self.h, bits.ctypes.data, roots.ctypes.data), "mc3_read_candidates")
        return bits, roots

    def read_means(self, first: int, n: int) -> np.ndarray:
        out = np.zeros((n, 2), dtype=np.float64)
        self._check(lib().mc3_read_means(self.h, first, n, out.ctypes.data), "mc3_read_means")
        return out

    def timing_enable(self, on: bool = True, every: int = 1):
        """Time every `every`-th scoring launch while on (mc3_timing_enable)."""
        self._check(lib().mc3_timing_enable(self.h, int(every) if on else 0), "mc3_timing_enable")

    def timing_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(lib().mc3_timing_read(self.h, ctypes.byref(ms), ctypes.byref(n)), "mc3_timing_read")
        return ms.value, n.value

    def sync(self):
        self._check(lib().mc3_sync(self.h), "mc3_sync")


def set_generation(G, peq=None):
    """mc3_set_generation on torch tensors: G float64 CUDA [n_sets, n, n] (G[s, e, p] =
    P_gen(e | p)); optional peq [n_sets, 2^n].  Returns out [n_sets, 2^n] and, with peq,
    (out, psub, peq_set); runs on the current stream."""
    import torch
    if G.dtype != torch.float64 or not G.is_cuda or G.dim() != 3 or G.shape[1] != G.shape[2]:
        raise ValueError("G must be a float64 CUDA tensor [n_sets, n, n]")
    G = G.contiguous()
    n_sets, n = G.shape[0], G.shape[1]
    out = torch.empty((n_sets, 1 << n), dtype=torch.float64, device=G.device)
    psub = peq_set = None
    if peq is not None:
        peq = peq.contiguous()
        if peq.dtype != torch.float64 or tuple(peq.shape) != (n_sets, 1 << n) or peq.device != G.device:
            raise ValueError("peq must be a float64 tensor [n_sets, 2^n] on G's device")
        psub = torch.empty_like(out)
        peq_set = torch.empty(n_sets, dtype=torch.float64, device=G.device)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    st = lib().mc3_set_generation(ptr(G), n, n_sets, ptr(out), ptr(peq), ptr(psub), ptr(peq_set),
                                  ctypes.c_void_p(torch.cuda.current_stream(G.device).cuda_stream))
    if st != MC3_OK:
        raise MC3Error(st, "mc3_set_generation")
    return out if peq is None else (out, psub, peq_set)


def bits_to_spins(bits: np.ndarray, N: int) -> np.ndarray:
    """Bitsets [..., words] (set bit = -1) to int8 spins [..., N]."""
    b = np.asarray(bits, dtype=np.uint32)
    idx = np.arange(N)
    v = (b[..., idx // 32] >> (idx % 32).astype(np.uint32)) & 1
    return np.where(v == 1, -1, 1).astype(np.int8)


def spins_to_bits(spins: np.ndarray) -> np.ndarray:
    s = np.asarray(spins)
    N = s.shape[-1]
    words = (N + 31) // 32
    out = np.zeros(s.shape[:-1] + (words,), dtype=np.uint32)
    for i in range(N):
        out[..., i // 32] |= ((s[..., i] < 0).astype(np.uint32) << np.uint32(i % 32))
    return out


_ceil = None


def ceiling_lib() -> ctypes.CDLL:
    """Load libmc3ceil.so (the matrix-core ceiling measurement); raises if it is missing."""
    global _ceil
    if _ceil is not None:
        return _ceil
    if not os.path.exists(CEIL_PATH):
        raise ImportError(f"{CEIL_PATH} is not built; run paper_2102_05613_amd.build.build() first")
    L = ctypes.CDLL(CEIL_PATH)
    c = ctypes
    L.mc3c_mfma_ceiling.argtypes = [c.c_int, c.c_int, c.c_int, c.POINTER(c.c_double), c.POINTER(c.c_double)]
    L.mc3c_mfma_ceiling.restype = c.c_int
    L.mc3c_mfma_mix.argtypes = [c.c_int, c.c_int, c.c_int, c.POINTER(c.c_double)]
    L.mc3c_mfma_mix.restype = c.c_int
    _ceil = L
    return L


def mfma_ceiling(iters: int = 12500, blocks: int = 256, repeats: int = 3) -> dict:
    """The attainable BF16 matrix-core rate (TFLOP/s, best of `repeats` launches) and the
    engine clock (GHz, median over blocks) of a plain loop at the scoring kernel's
    occupancy on the current device."""
    t, g = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = ceiling_lib().mc3c_mfma_ceiling(iters, blocks, repeats, ctypes.byref(t), ctypes.byref(g))
    if rc != 0:
        raise RuntimeError(f"mc3c_mfma_ceiling failed ({rc})")
    return {"tflops": t.value, "clock_ghz": g.value, "iters": iters, "blocks": blocks, "repeats": repeats}


def mfma_mix(mix: int, iters: int = 12500, repeats: int = 3) -> float:
    """TFLOP/s of the matrix-core loop with the traffic mix `mix` (see MFMA_MIXES and
    include/mc3_ceiling.h) per round of 64 MFMAs, best of `repeats` launches."""
    t = ctypes.c_double(0.0)
    rc = ceiling_lib().mc3c_mfma_mix(mix, iters, repeats, ctypes.byref(t))
    if rc != 0:
        raise RuntimeError(f"mc3c_mfma_mix failed ({rc})")
    return t.value
