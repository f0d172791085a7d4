"""Python binding of libfvan (the C ABI in include/fvan.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch supplies device memory and streams.  Importing this
module loads the in-tree libfvan.so and fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfvan.so")

FVAN_FP32, FVAN_BF16_SPLIT = 0, 2
PRECISION_NAMES = {0: "fp32", 2: "bf16split"}
WS_SAMPLER, WS_TEACHER = 1, 2
# bytes of the static KV cache of fvan_sample_noalloc (FVAN_NOALLOC_KV_BYTES), per GPU
NOALLOC_KV_BYTES = 64 << 20
BONDS_PM1, BONDS_F32, BONDS_DENSE = 0, 1, 2
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENONFINITE", -5: "EUNSUPPORTED"}

# Every symbol include/fvan.h declares.
EXPORTS = (
    "fvan_num_params", "fvan_derive_mask", "fvan_create_model", "fvan_destroy_model", "fvan_bind_params",
    "fvan_sync_params", "fvan_sample", "fvan_sample_noalloc", "fvan_sample_tokens", "fvan_log_prob_tokens_backward",
    "fvan_tokens_to_spins", "fvan_train_step_tokens", "fvan_group_launch_shape", "fvan_log_prob", "fvan_log_prob_tokens", "fvan_log_prob_backward", "fvan_energy",
    "fvan_free_energy", "fvan_reinforce_weights", "fvan_adam_step", "fvan_train_step",
    "fvan_newton_schulz", "fvan_muon_step", "fvan_train_step_muon",
    "fvan_lmc_refine", "fvan_distill_weights", "fvan_train_step_distill",
    "fvan_overlap_histogram", "fvan_anneal_temperature",
    "fvan_group_create", "fvan_group_destroy", "fvan_group_run", "fvan_group_run_graph", "fvan_model_status",
    "fvan_last_error",
)


class FvanError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class ModelConfigC(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n_spins", "d_model", "d_token", "n_layers", "n_heads", "vocab",
                                         "window", "prefix", "max_batch", "precision", "workspaces")]


class CouplingsC(C.Structure):
    _fields_ = [("n_spins", C.c_int32), ("kind", C.c_int32), ("degree", C.c_int32),
                ("nbr", C.c_void_p), ("J", C.c_void_p)]


class AdamC(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("weight_decay", C.c_float)]


class MuonC(C.Structure):
    _fields_ = [("lr", C.c_float), ("momentum", C.c_float), ("weight_decay", C.c_float), ("rms_scale", C.c_float),
                ("ns_eps", C.c_float), ("ns_steps", C.c_int32), ("adam", AdamC)]


def muon_struct(lr=1e-3, momentum=0.95, weight_decay=0.0, rms_scale=0.2, ns_eps=1e-7, ns_steps=5, adam_lr=1e-3,
                adam_beta1=0.9, adam_beta2=0.999, adam_eps=1e-8, adam_weight_decay=0.0) -> MuonC:
    return MuonC(lr, momentum, weight_decay, rms_scale, ns_eps, ns_steps,
                 AdamC(adam_lr, adam_beta1, adam_beta2, adam_eps, adam_weight_decay))


class LmcC(C.Structure):
    _fields_ = [("degree", C.c_int32), ("nbr", C.c_void_p), ("J", C.c_void_p), ("colour", C.c_void_p),
                ("sweeps", C.c_int32)]


class GroupUnitC(C.Structure):
    _fields_ = [("model", C.c_void_p), ("couplings", C.c_void_p), ("beta", C.c_double), ("batch", C.c_int32),
                ("seed", C.c_uint64), ("stream_id", C.c_uint64), ("spins", C.c_void_p), ("log_q", C.c_void_p),
                ("energy", C.c_void_p), ("stats", C.c_void_p)]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path) and path == LIB_PATH:
        from .build import build      # nothing built yet: compile it in-tree once
        build()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2606_22984_amd/build.py")
    lib = C.CDLL(path)
    P, I32, I64, U64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    sig = {
        "fvan_num_params": [C.POINTER(ModelConfigC), C.POINTER(C.c_int64)],
        "fvan_derive_mask": [I32, I64, P, P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
        "fvan_create_model": [C.POINTER(ModelConfigC), C.POINTER(C.c_void_p)],
        "fvan_destroy_model": [P],
        "fvan_bind_params": [P, P, P],
        "fvan_sync_params": [P, P],
        "fvan_sample": [P, I32, U64, U64, P, P, P],
        "fvan_log_prob": [P, I32, P, P, P],
        "fvan_log_prob_tokens": [P, I32, P, P, P],
        "fvan_log_prob_backward": [P, I32, P, P, P],
        "fvan_energy": [C.POINTER(CouplingsC), I32, P, P, P],
        "fvan_free_energy": [I32, I32, D, I32, P, P, P, P],
        "fvan_reinforce_weights": [I32, D, I32, P, P, P, P],
        "fvan_adam_step": [P, C.POINTER(AdamC), I64, P],
        "fvan_train_step": [P, C.POINTER(CouplingsC), D, I32, U64, U64, C.POINTER(AdamC), P, P],
        "fvan_newton_schulz": [I32, I32, I32, C.c_float, P, P, P],
        "fvan_muon_step": [P, C.POINTER(MuonC), I64, P],
        "fvan_train_step_muon": [P, C.POINTER(CouplingsC), D, I32, U64, U64, C.POINTER(MuonC), P, P],
        "fvan_overlap_histogram": [I32, I32, P, P, P],
        "fvan_anneal_temperature": [I64, D, I64, I64, I32, C.POINTER(C.c_double)],
        "fvan_lmc_refine": [I32, C.POINTER(LmcC), I32, D, U64, C.c_uint32, P, P, P],
        "fvan_distill_weights": [I32, D, D, I32, P, P, P, P],
        "fvan_train_step_distill": [P, C.POINTER(CouplingsC), C.POINTER(LmcC), D, D, I32, U64, U64,
                                    C.POINTER(MuonC), P, P],
        "fvan_group_create": [C.POINTER(GroupUnitC), I32, I32, C.POINTER(C.c_void_p)],
        "fvan_group_destroy": [P],
        "fvan_group_run": [P, P],
        "fvan_group_run_graph": [P, P],
        "fvan_model_status": [P, P],
        "fvan_sample_noalloc": [P, I32, U64, U64, P, P, P],
        "fvan_sample_tokens": [P, I32, U64, U64, P, P, P],
        "fvan_log_prob_tokens_backward": [P, I32, P, P, P],
        "fvan_tokens_to_spins": [I32, I32, P, I32, I32, P, P, P],
        "fvan_train_step_tokens": [P, C.POINTER(CouplingsC), P, D, I32, U64, U64, C.POINTER(MuonC), P, P],
        "fvan_group_launch_shape": [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.fvan_last_error.argtypes = []
    lib.fvan_last_error.restype = C.c_char_p
    return lib


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(rc: int):
    if rc != 0:
        raise FvanError(rc, lib().fvan_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _require_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("tensors passed to libfvan must be contiguous device tensors")


def _spins_arg(spins, n: int):
    """The C side reads batch x n int8 spins from the pointer: check that much is there."""
    if spins.dtype != torch.int8 or spins.dim() != 2 or spins.shape[1] != n or spins.shape[0] < 1:
        raise ValueError(f"spins must be an int8 [batch, {n}] tensor (got {tuple(spins.shape)}, {spins.dtype})")


def _tokens_arg(t, n: int):
    if t.dtype != torch.uint8 or t.dim() != 2 or not t.is_contiguous() or t.shape[1] != n:
        raise ValueError(f"tokens must be a contiguous uint8 [batch, {n}] tensor")


def patch_sites(L: int, dim: int) -> np.ndarray:
    """Site of every bit of every patch token of a periodic L^dim lattice cut into
    2^dim blocks (patches in raster order of their block coordinates, last
    fastest; the site at offset o in {0,1}^dim of a patch is bit
    sum_k o_k 2^(dim-1-k) of its token): int32 [(L/2)^dim, 2^dim]."""
    if L % 2:
        raise ValueError("patches need an even lattice side")
    half = L // 2
    blocks = np.stack(np.unravel_index(np.arange(half ** dim), (half,) * dim), axis=1)      # [T, dim]
    offs = np.stack(np.unravel_index(np.arange(2 ** dim), (2,) * dim), axis=1)              # [2^dim, dim]
    coords = 2 * blocks[:, None, :] + offs[None, :, :]                                    # [T, 2^dim, dim]
    return np.ravel_multi_index(tuple(np.moveaxis(coords, -1, 0)), (L,) * dim).astype(np.int32)


def tokens_to_spins(sites: torch.Tensor, tokens: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """int8 +-1 spins [batch, n_tokens * bits] of patch tokens (fvan_tokens_to_spins)."""
    _require_cuda(sites, tokens)
    T, bits = sites.shape
    if sites.dtype != torch.int32 or not sites.is_contiguous():
        raise ValueError("sites must be a contiguous int32 [n_tokens, bits] tensor")
    _tokens_arg(tokens, T)
    n = T * bits
    if out is None:
        out = torch.empty(tokens.shape[0], n, dtype=torch.int8, device=tokens.device)
    _spins_arg(out, n)
    _check(lib().fvan_tokens_to_spins(T, bits, _ptr(sites), n, tokens.shape[0], _ptr(tokens), _ptr(out),
                                      _stream(stream)))
    return out


def _vec_arg(t, batch: int, name: str, dtypes=(torch.float32,)):
    if t is not None and (t.dtype not in dtypes or t.numel() < batch):
        raise ValueError(f"{name} must hold at least {batch} values of type {dtypes[0]}")


def _energy_logq_args(energy_t, log_q, out, out_len: int, out_dtype=torch.float32):
    """E [batch] (int32 or float32) and ln q [batch] float32 of one length; out holds out_len values."""
    if log_q.dim() != 1 or log_q.dtype != torch.float32 or log_q.shape[0] < 1:
        raise ValueError("log_q must be a float32 [batch] tensor")
    _vec_arg(energy_t, log_q.shape[0], "energy", (torch.int32, torch.float32))
    _vec_arg(out, out_len, "out", (out_dtype,))


def num_params(cfg) -> int:
    c = config_struct(cfg, max_batch=1)
    out = C.c_int64()
    _check(lib().fvan_num_params(C.byref(c), C.byref(out)))
    return out.value


def derive_mask(n: int, edges_i, edges_j) -> Tuple[int, int]:
    ei = np.ascontiguousarray(edges_i, dtype=np.int32)
    ej = np.ascontiguousarray(edges_j, dtype=np.int32)
    w, p = C.c_int32(), C.c_int32()
    _check(lib().fvan_derive_mask(n, ei.shape[0], ei.ctypes.data_as(C.c_void_p), ej.ctypes.data_as(C.c_void_p),
                                  C.byref(w), C.byref(p)))
    return w.value, p.value


def config_struct(cfg, max_batch: int, precision: int = FVAN_FP32,
                  workspaces: int = WS_SAMPLER | WS_TEACHER) -> ModelConfigC:
    return ModelConfigC(n_spins=cfg.n_spins, d_model=cfg.d_model, d_token=cfg.d_token, n_layers=cfg.n_layers,
                        n_heads=cfg.n_heads, vocab=cfg.vocab, window=cfg.window, prefix=cfg.prefix,
                        max_batch=max_batch, precision=precision, workspaces=workspaces)


@dataclass
class Couplings:
    """Device-resident bonds in the layout fvan_energy reads, and the C struct pointing at them."""
    n: int
    kind: int
    degree: int
    nbr: Optional[torch.Tensor]
    J: torch.Tensor
    c: CouplingsC

    @property
    def energy_is_int(self) -> bool:
        return self.kind == BONDS_PM1

    def empty_energy(self, batch: int, device="cuda") -> torch.Tensor:
        return torch.empty(batch, dtype=torch.int32 if self.energy_is_int else torch.float32, device=device)


@dataclass
class LmcGraph:
    """Device-resident neighbour table (both directions of every pair), bonds and
    checkerboard colours for fvan_lmc_refine, and the C struct pointing at them."""
    n: int
    nbr: torch.Tensor
    J: torch.Tensor
    colour: torch.Tensor
    c: LmcC


def lmc_graph(instance, sweeps: int, device="cuda") -> LmcGraph:
    """Neighbour graph of a lattice instance with its checkerboard colouring
    (sum of the raster coordinates mod 2, last coordinate fastest)."""
    if getattr(instance, "L", None) is None:
        raise ValueError("checkerboard refinement needs a lattice instance")
    n = instance.n
    adj = [[] for _ in range(n)]
    for a, b, w in zip(np.asarray(instance.edges_i).tolist(), np.asarray(instance.edges_j).tolist(),
                       np.asarray(instance.J).tolist()):
        adj[a].append((b, w))
        adj[b].append((a, w))
    deg = max(1, max(len(x) for x in adj))
    nbr = -np.ones((n, deg), dtype=np.int32)
    Jl = np.zeros((n, deg), dtype=np.float32)
    for i, lst in enumerate(adj):
        for k, (j, w) in enumerate(lst):
            nbr[i, k] = j
            Jl[i, k] = w
    idx = np.arange(n)
    col = np.zeros(n, dtype=np.int64)
    for _ in range(instance.dim):
        col += idx % instance.L
        idx //= instance.L
    col %= 2
    ei, ej = np.asarray(instance.edges_i), np.asarray(instance.edges_j)
    if ei.size and np.any(col[ei] == col[ej]):
        # e.g. periodic boundaries with odd L: the sites x = L-1 and x = 0 share a colour, so a
        # half-sweep would update two neighbours from stale fields (not sequential Metropolis)
        raise ValueError("the checkerboard colouring is not proper on this lattice (a bond joins two sites "
                         "of one colour); refinement needs a bipartite lattice, e.g. even L under periodic "
                         "boundaries")
    t_nbr = torch.as_tensor(nbr, device=device)
    t_J = torch.as_tensor(Jl, device=device)
    t_col = torch.as_tensor(col.astype(np.int8), device=device)
    c = LmcC(degree=deg, nbr=t_nbr.data_ptr(), J=t_J.data_ptr(), colour=t_col.data_ptr(), sweeps=sweeps)
    return LmcGraph(n, t_nbr, t_J, t_col, c)


def lmc_refine(graph: LmcGraph, spins: torch.Tensor, beta: float, seed: int, stream_tag: int, accepted=None,
               stream=None):
    """Checkerboard Metropolis sweeps on spins [batch, n] in place (fvan_lmc_refine)."""
    _require_cuda(spins, accepted)
    _spins_arg(spins, graph.n)
    _vec_arg(accepted, spins.shape[0], "accepted", (torch.int32,))
    _check(lib().fvan_lmc_refine(graph.n, C.byref(graph.c), spins.shape[0], beta, seed, stream_tag, _ptr(spins),
                                 _ptr(accepted), _stream(stream)))
    return spins


def overlap_histogram(spins: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """counts[k] = pairs a < b of the batch with k agreeing sites (fvan_overlap_histogram)."""
    _require_cuda(spins)
    if spins.dim() != 2:
        raise ValueError("spins must be an int8 [batch, n] tensor")
    n = spins.shape[1]
    _spins_arg(spins, n)
    if out is None:
        out = torch.empty(n + 1, dtype=torch.int64, device=spins.device)
    _require_cuda(out)
    if out.numel() != n + 1 or out.dtype != torch.int64:
        raise ValueError("out must be int64 [n_spins + 1]")
    _check(lib().fvan_overlap_histogram(spins.shape[0], n, _ptr(spins), _ptr(out), _stream(stream)))
    return out


def anneal_temperature(step: int, T0: float, n_warmup: int, n_eq: int, n_anneal: int) -> float:
    """Temperature of a training step under the annealing schedule (fvan_anneal_temperature)."""
    T = C.c_double()
    _check(lib().fvan_anneal_temperature(step, T0, n_warmup, n_eq, n_anneal, C.byref(T)))
    return T.value


def distill_weights(E: torch.Tensor, log_q: torch.Tensor, beta: float, w: float, out=None, stream=None):
    """Weights of the self-distillation gradient, Eq. (loss2) (fvan_distill_weights)."""
    _require_cuda(E, log_q)
    if out is None:
        out = torch.empty(log_q.shape[0], dtype=torch.float32, device=log_q.device)
    _energy_logq_args(E, log_q, out, log_q.shape[0])
    is_int = 1 if E.dtype == torch.int32 else 0
    _check(lib().fvan_distill_weights(log_q.shape[0], beta, w, is_int, _ptr(E), _ptr(log_q), _ptr(out),
                                      _stream(stream)))
    return out


def couplings(instance, device="cuda", dense: Optional[bool] = None) -> Couplings:
    """Pack an instance's pair list into the ELL rows fvan_energy reads (pair (i, j) stored in row i),
    or its dense matrix for SK."""
    n = instance.n
    use_dense = instance.dense is not None if dense is None else dense
    if use_dense:
        J = torch.as_tensor(np.ascontiguousarray(instance.dense, dtype=np.float32), device=device)
        c = CouplingsC(n_spins=n, kind=BONDS_DENSE, degree=0, nbr=None, J=J.data_ptr())
        return Couplings(n, BONDS_DENSE, 0, None, J, c)
    ei = np.asarray(instance.edges_i)
    ej = np.asarray(instance.edges_j)
    counts = np.bincount(ei, minlength=n)
    deg = max(int(counts.max()) if counts.size else 0, 1)
    nbr = -np.ones((n, deg), dtype=np.int32)
    fill = np.zeros(n, dtype=np.int64)
    pm1 = instance.bonds == "pm1"
    Jl = np.zeros((n, deg), dtype=np.int8 if pm1 else np.float32)
    for a, b, w in zip(ei.tolist(), ej.tolist(), np.asarray(instance.J).tolist()):
        k = fill[a]
        nbr[a, k] = b
        Jl[a, k] = w
        fill[a] += 1
    nbr_t = torch.as_tensor(nbr, device=device)
    J_t = torch.as_tensor(Jl, device=device)
    kind = BONDS_PM1 if pm1 else BONDS_F32
    c = CouplingsC(n_spins=n, kind=kind, degree=deg, nbr=nbr_t.data_ptr(), J=J_t.data_ptr())
    return Couplings(n, kind, deg, nbr_t, J_t, c)


class Model:
    """Owns one fvan_model handle plus the caller-side FP32 parameter and gradient tensors.
    workspaces: WS_SAMPLER (KV cache) and/or WS_TEACHER (teacher-forced passes), allocated at creation."""

    def __init__(self, cfg, max_batch: int, precision: int = FVAN_FP32, params=None, device="cuda",
                 workspaces: int = WS_SAMPLER | WS_TEACHER):
        self.cfg = cfg
        self.precision = precision
        self.max_batch = max_batch
        self._c = config_struct(cfg, max_batch, precision, workspaces)
        h = C.c_void_p()
        _check(lib().fvan_create_model(C.byref(self._c), C.byref(h)))
        self.handle = h
        n = num_params(cfg)
        self.params = torch.zeros(n, dtype=torch.float32, device=device)
        self.grads = torch.zeros(n, dtype=torch.float32, device=device)
        _check(lib().fvan_bind_params(self.handle, _ptr(self.params), _ptr(self.grads)))
        if params is not None:
            self.set_params(params)

    def set_params(self, params):
        self.params.copy_(torch.as_tensor(np.asarray(params, dtype=np.float32)))
        self.sync()

    def sync(self, stream=None):
        _check(lib().fvan_sync_params(self.handle, _stream(stream)))

    def sample(self, batch: int, seed: int, stream_id: int, spins=None, log_q=None, stream=None):
        if spins is None:
            spins = torch.empty(batch, self.cfg.n_spins, dtype=torch.int8, device=self.params.device)
        if log_q is None:
            log_q = torch.empty(batch, dtype=torch.float32, device=self.params.device)
        _require_cuda(spins, log_q)
        _spins_arg(spins, self.cfg.n_spins)
        if spins.shape[0] < batch:
            raise ValueError(f"spins holds {spins.shape[0]} rows, batch is {batch}")
        _vec_arg(log_q, batch, "log_q")
        _check(lib().fvan_sample(self.handle, batch, seed, stream_id, _ptr(spins), _ptr(log_q), _stream(stream)))
        return spins, log_q

    def sample_noalloc(self, batch: int, seed: int, stream_id: int, spins: torch.Tensor, log_q: torch.Tensor,
                       stream=None):
        """fvan_sample with the library's static KV cache (no device allocation in the
        call; the caller passes the output tensors)."""
        _require_cuda(spins, log_q)
        _spins_arg(spins, self.cfg.n_spins)
        if spins.shape[0] < batch:
            raise ValueError(f"spins holds {spins.shape[0]} rows, batch is {batch}")
        _vec_arg(log_q, batch, "log_q")
        _check(lib().fvan_sample_noalloc(self.handle, batch, seed, stream_id, _ptr(spins), _ptr(log_q),
                                         _stream(stream)))
        return spins, log_q

    def log_prob(self, spins: torch.Tensor, log_q=None, stream=None):
        _require_cuda(spins)
        if log_q is None:
            log_q = torch.empty(spins.shape[0], dtype=torch.float32, device=spins.device)
        _spins_arg(spins, self.cfg.n_spins)
        _vec_arg(log_q, spins.shape[0], "log_q")
        _check(lib().fvan_log_prob(self.handle, spins.shape[0], _ptr(spins), _ptr(log_q), _stream(stream)))
        return log_q

    def log_prob_tokens(self, tokens: torch.Tensor, log_q=None, stream=None):
        """Teacher-forced ln q of patch-token sequences (uint8 [batch, n_spins])."""
        _require_cuda(tokens)
        if (tokens.dtype != torch.uint8 or tokens.dim() != 2 or not tokens.is_contiguous()
                or tokens.shape[1] != self.cfg.n_spins):
            raise ValueError("tokens must be a contiguous uint8 [batch, n_spins] tensor")
        if log_q is None:
            log_q = torch.empty(tokens.shape[0], dtype=torch.float32, device=tokens.device)
        _check(lib().fvan_log_prob_tokens(self.handle, tokens.shape[0], _ptr(tokens), _ptr(log_q), _stream(stream)))
        return log_q

    def sample_tokens(self, batch: int, seed: int, stream_id: int, tokens=None, log_q=None, stream=None):
        """Ancestral sampling of patch-token sequences (uint8 [batch, n_spins]) and their ln q."""
        dev = self.params.device
        if tokens is None:
            tokens = torch.empty(batch, self.cfg.n_spins, dtype=torch.uint8, device=dev)
        if log_q is None:
            log_q = torch.empty(batch, dtype=torch.float32, device=dev)
        _require_cuda(tokens, log_q)
        _tokens_arg(tokens, self.cfg.n_spins)
        if tokens.shape[0] < batch:
            raise ValueError(f"tokens holds {tokens.shape[0]} rows, batch is {batch}")
        _vec_arg(log_q, batch, "log_q")
        _check(lib().fvan_sample_tokens(self.handle, batch, seed, stream_id, _ptr(tokens), _ptr(log_q),
                                        _stream(stream)))
        return tokens, log_q

    def log_prob_tokens_backward(self, tokens: torch.Tensor, grad_log_q: torch.Tensor, stream=None):
        _require_cuda(tokens, grad_log_q)
        _tokens_arg(tokens, self.cfg.n_spins)
        _vec_arg(grad_log_q, tokens.shape[0], "grad_log_q")
        _check(lib().fvan_log_prob_tokens_backward(self.handle, tokens.shape[0], _ptr(tokens), _ptr(grad_log_q),
                                                   _stream(stream)))

    def train_step_tokens(self, coup: "Couplings", sites: torch.Tensor, beta: float, batch: int, seed: int,
                          step: int, stats=None, stream=None, **hyper):
        """Training step of a patch-token model (Muon); sites: int32 [n_spins, bits] on the device."""
        if stats is None:
            stats = torch.zeros(4, dtype=torch.float64, device=self.params.device)
        _require_cuda(sites)
        if sites.dtype != torch.int32 or not sites.is_contiguous() or sites.shape[0] != self.cfg.n_spins:
            raise ValueError("sites must be a contiguous int32 [n_tokens, bits] tensor")
        o = muon_struct(**hyper)
        _check(lib().fvan_train_step_tokens(self.handle, C.byref(coup.c), _ptr(sites), beta, batch, seed, step,
                                            C.byref(o), _ptr(stats), _stream(stream)))
        return stats

    def log_prob_backward(self, spins: torch.Tensor, grad_log_q: torch.Tensor, stream=None):
        _require_cuda(spins, grad_log_q)
        _spins_arg(spins, self.cfg.n_spins)
        _vec_arg(grad_log_q, spins.shape[0], "grad_log_q")
        _check(lib().fvan_log_prob_backward(self.handle, spins.shape[0], _ptr(spins), _ptr(grad_log_q),
                                            _stream(stream)))

    def adam_step(self, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, stream=None):
        o = AdamC(lr, beta1, beta2, eps, weight_decay)
        _check(lib().fvan_adam_step(self.handle, C.byref(o), step, _stream(stream)))

    def train_step(self, coup: Couplings, beta: float, batch: int, seed: int, step: int, lr=1e-3, beta1=0.9,
                   beta2=0.999, eps=1e-8, weight_decay=0.0, stats=None, stream=None):
        if stats is None:
            stats = torch.zeros(4, dtype=torch.float64, device=self.params.device)
        o = AdamC(lr, beta1, beta2, eps, weight_decay)
        _check(lib().fvan_train_step(self.handle, C.byref(coup.c), beta, batch, seed, step, C.byref(o),
                                     _ptr(stats), _stream(stream)))
        return stats

    def muon_step(self, step: int, stream=None, **hyper):
        """One Muon step (fvan_muon_step); hyper: the keyword arguments of muon_struct."""
        o = muon_struct(**hyper)
        _check(lib().fvan_muon_step(self.handle, C.byref(o), step, _stream(stream)))

    def train_step_muon(self, coup: Couplings, beta: float, batch: int, seed: int, step: int, stats=None,
                        stream=None, **hyper):
        if stats is None:
            stats = torch.zeros(4, dtype=torch.float64, device=self.params.device)
        o = muon_struct(**hyper)
        _check(lib().fvan_train_step_muon(self.handle, C.byref(coup.c), beta, batch, seed, step, C.byref(o),
                                          _ptr(stats), _stream(stream)))
        return stats

    def train_step_distill(self, coup: Couplings, graph: LmcGraph, beta: float, w: float, batch: int, seed: int,
                           step: int, stats=None, stream=None, **hyper):
        if stats is None:
            stats = torch.zeros(4, dtype=torch.float64, device=self.params.device)
        o = muon_struct(**hyper)
        _check(lib().fvan_train_step_distill(self.handle, C.byref(coup.c), C.byref(graph.c), beta, w, batch, seed,
                                             step, C.byref(o), _ptr(stats), _stream(stream)))
        return stats

    def status(self, stream=None):
        """Synchronise and raise FvanError(ENONFINITE) if a kernel of this model produced a NaN or Inf
        since the last report (fvan_model_status)."""
        _check(lib().fvan_model_status(self.handle, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            lib().fvan_destroy_model(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def newton_schulz(M: torch.Tensor, steps: int = 5, eps: float = 1e-7, out=None, stream=None):
    """O = NewtonSchulz(M) for an FP32 device matrix (fvan_newton_schulz); out may be M."""
    _require_cuda(M)
    if M.dim() != 2 or M.dtype != torch.float32:
        raise ValueError("newton_schulz takes a 2-D float32 matrix")
    if out is None:
        out = torch.empty_like(M)
    _require_cuda(out)
    if out.shape != M.shape or out.dtype != torch.float32:
        raise ValueError("out must match M")
    _check(lib().fvan_newton_schulz(M.shape[0], M.shape[1], steps, eps, _ptr(M), _ptr(out), _stream(stream)))
    return out


def energy(coup: Couplings, spins: torch.Tensor, out=None, stream=None):
    _require_cuda(spins)
    if out is None:
        out = coup.empty_energy(spins.shape[0], spins.device)
    _spins_arg(spins, coup.n)
    _vec_arg(out, spins.shape[0], "out", (torch.int32,) if coup.energy_is_int else (torch.float32,))
    _check(lib().fvan_energy(C.byref(coup.c), spins.shape[0], _ptr(spins), _ptr(out), _stream(stream)))
    return out


def free_energy(energy_t: torch.Tensor, log_q: torch.Tensor, beta: float, n_spins: int, out=None, stream=None):
    _require_cuda(energy_t, log_q)
    if out is None:
        out = torch.zeros(2, dtype=torch.float64, device=log_q.device)
    _energy_logq_args(energy_t, log_q, out, 2, torch.float64)
    is_int = 1 if energy_t.dtype == torch.int32 else 0
    _check(lib().fvan_free_energy(log_q.shape[0], n_spins, beta, is_int, _ptr(energy_t), _ptr(log_q), _ptr(out),
                                  _stream(stream)))
    return out


def reinforce_weights(energy_t: torch.Tensor, log_q: torch.Tensor, beta: float, out=None, stream=None):
    _require_cuda(energy_t, log_q)
    if out is None:
        out = torch.empty_like(log_q)
    _energy_logq_args(energy_t, log_q, out, log_q.shape[0])
    is_int = 1 if energy_t.dtype == torch.int32 else 0
    _check(lib().fvan_reinforce_weights(log_q.shape[0], beta, is_int, _ptr(energy_t), _ptr(log_q), _ptr(out),
                                        _stream(stream)))
    return out


class LogProb(torch.autograd.Function):
    """ln q_theta(sigma) as a differentiable function of the model's parameter tensor.

    forward: fvan_log_prob (teacher forced).  backward: fvan_log_prob_backward with
    grad_output as the per-sample weights; it recomputes the forward pass, attention
    included, and returns the accumulated parameter gradient."""

    @staticmethod
    def forward(ctx, params: torch.Tensor, model: "Model", spins: torch.Tensor):
        ctx.model = model
        ctx.save_for_backward(spins)
        return model.log_prob(spins)

    @staticmethod
    def backward(ctx, grad_out):
        (spins,) = ctx.saved_tensors
        m = ctx.model
        saved = m.grads.clone()
        m.grads.zero_()
        m.log_prob_backward(spins, grad_out.contiguous().float())
        g = m.grads.clone()
        m.grads.copy_(saved)
        return g, None, None


def log_prob_autograd(model: Model, spins: torch.Tensor) -> torch.Tensor:
    return LogProb.apply(model.params, model, spins)


class Group:
    """Many (model, couplings, beta) units sampled in one persistent launch (fvan_group_*).
    Keeps references to every tensor the device tables point at."""

    def __init__(self, units, tile_samples: int = 0):
        self._keep = []
        arr = (GroupUnitC * len(units))()
        self.outputs = []
        for i, u in enumerate(units):
            model, coup, beta, batch, seed, stream_id = (u["model"], u["couplings"], u["beta"], u["batch"],
                                                         u["seed"], u["stream_id"])
            dev = model.params.device
            spins = torch.empty(batch, model.cfg.n_spins, dtype=torch.int8, device=dev)
            lq = torch.empty(batch, dtype=torch.float32, device=dev)
            en = coup.empty_energy(batch, dev)
            st = torch.zeros(2, dtype=torch.float64, device=dev)
            self._keep += [spins, lq, en, st, coup, model]
            self.outputs.append(dict(spins=spins, log_q=lq, energy=en, stats=st))
            arr[i] = GroupUnitC(model=model.handle, couplings=C.cast(C.pointer(coup.c), C.c_void_p), beta=beta,
                                batch=batch, seed=seed, stream_id=stream_id, spins=spins.data_ptr(),
                                log_q=lq.data_ptr(), energy=en.data_ptr(), stats=st.data_ptr())
        self._arr = arr
        h = C.c_void_p()
        _check(lib().fvan_group_create(arr, len(units), tile_samples, C.byref(h)))
        self.handle = h

    def launch_shape(self) -> dict:
        """The autotuned launch shape: tile, grid, whether it came from the persisted store, timed ms."""
        t, g, f, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        _check(lib().fvan_group_launch_shape(self.handle, C.byref(t), C.byref(g), C.byref(f), C.byref(ms)))
        return {"tile": t.value, "grid": g.value, "from_store": bool(f.value), "prefix_ms": ms.value}

    def run(self, stream=None):
        _check(lib().fvan_group_run(self.handle, _stream(stream)))

    def run_graph(self, stream=None):
        _check(lib().fvan_group_run_graph(self.handle, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            lib().fvan_group_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
