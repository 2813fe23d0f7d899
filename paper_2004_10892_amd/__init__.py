"""Python binding of libqbe (include/qbe.h): sliced bucket-elimination
contraction of tensor networks on MI355X.

This module only marshals arguments: every planning step runs in the C++
host planner and every contraction step in the library's HIP kernels.  The
names mirror the C entry points (``qbe_order_min_fill`` ...).  PyTorch is
used only to allocate device workspaces and to obtain the current HIP
stream.  There is no fallback: if ``libqbe.so`` is missing, importing this
package fails.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqbe.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
        "from the repository root")

# torch ships its own HIP and HSA runtimes under sonames equal to ROCm's.
# Loaded first, they satisfy this library's runtime dependency, so that the
# process holds one HIP runtime; loading libqbe first would bring ROCm's
# copies beside torch's, and the second runtime to start sees no device.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

QBE_OK = 0
ERRORS = {-1: "INVALID_ARG", -2: "OOM", -3: "HIP", -4: "MEM_CAP", -5: "INTERNAL", -6: "NO_DEVICE"}
SCORE = {"tree_trimming": 0, "degree": 1, "tw_reduction": 2, "betweenness": 3, "learned": 4}
HEAD = {"slicing": 0, "elimination": 1}
EXEC = {"auto": 0, "per_step": 1, "fused": 2}
PREC = {"fp32": 0, "bf16x3": 1, "bf16x6": 2}

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)
_vp = C.c_void_p


class QbeError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.qbe_last_error().decode(errors="replace")
        super().__init__(f"{where}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


class PlanOpts(C.Structure):
    _fields_ = [("exec", C.c_int32), ("precision", C.c_int32), ("block", C.c_int32),
                ("no_merge", C.c_int32), ("fused_prefix", C.c_int32), ("fused_segments", C.c_int32),
                ("no_fold", C.c_int32), ("max_sums", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_vars", C.c_int32), ("n_tensors", C.c_int32), ("m", C.c_int32), ("width", C.c_int32),
                ("n_steps", C.c_int32), ("n_levels", C.c_int32), ("exec", C.c_int32), ("lds_bytes", C.c_int32),
                ("flops_per_slice", C.c_uint64), ("bytes_per_slice", C.c_uint64),
                ("peak_bytes_per_slice", C.c_uint64), ("ws_bytes_min", C.c_uint64),
                ("ws_bytes_all_slices", C.c_uint64), ("n_mfma_steps", C.c_int32), ("precision", C.c_int32),
                ("fused_levels", C.c_int32), ("n_merged_steps", C.c_int32), ("step_bytes_per_slice", C.c_uint64),
                ("n_launches", C.c_int32), ("prefix_buckets", C.c_int32), ("n_fused_segments", C.c_int32),
                ("fused_buckets", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SliceOpts(C.Structure):
    _fields_ = [("score", C.c_int32), ("m", C.c_int32), ("target_width", C.c_int32),
                ("recompute_every", C.c_int32), ("tries", C.c_int32), ("reserved0", C.c_int32),
                ("seed", C.c_uint64), ("mem_cap", C.c_uint64), ("reserved", C.c_uint64 * 2)]


class LaunchInfo(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_buckets", C.c_int32), ("n_ops", C.c_int32), ("out_rank", C.c_int32),
                ("n_sum", C.c_int32), ("mfma", C.c_int32), ("bytes_per_slice", C.c_uint64),
                ("flops_per_slice", C.c_uint64), ("levels", C.c_int32), ("lds_bytes", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["kind"] = LAUNCH_KINDS[d["kind"]]
        return d


LAUNCH_KINDS = {0: "bucket", 1: "merged", 2: "partial", 3: "group", 4: "finalize", 5: "reduce", 6: "prefix",
                7: "segment"}


_SIGS = {
    "qbe_last_error": (C.c_char_p, []),
    "qbe_version": (C.c_int32, []),
    "qbe_create": (C.c_int, [C.POINTER(_vp), C.c_int32, _vp]),
    "qbe_destroy": (C.c_int, [_vp]),
    "qbe_set_stream": (C.c_int, [_vp, _vp]),
    "qbe_model_create": (C.c_int, [C.c_int32, C.c_int32, _i32p, _i32p, _f64p, C.POINTER(_vp)]),
    "qbe_model_destroy": (C.c_int, [_vp]),
    "qbe_model_set_data": (C.c_int, [_vp, _f64p]),
    "qbe_order_min_fill": (C.c_int, [_vp, _i32p]),
    "qbe_width": (C.c_int, [_vp, _i32p, C.c_int32, _i32p, C.c_int32, _i32p]),
    "qbe_clique_tree": (C.c_int, [_vp, _i32p, C.c_int32, _i32p, _i32p, _i32p, C.c_int64, _i32p]),
    "qbe_slice": (C.c_int, [_vp, _i32p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _i32p, _i32p, _i32p, _i32p]),
    "qbe_schedule_cost": (C.c_int, [_vp, _i32p, C.c_int32, _i32p, C.c_int32, C.POINTER(C.c_uint64)]),
    "qbe_vertex_features": (C.c_int, [_vp, _i32p, C.c_int32, _i32p, C.c_int32, C.POINTER(C.c_float)]),
    "qbe_plan_create": (C.c_int, [_vp, _vp, _i32p, C.c_int32, _i32p, C.c_int32, C.POINTER(PlanOpts), C.POINTER(_vp)]),
    "qbe_plan_destroy": (C.c_int, [_vp]),
    "qbe_plan_update_data": (C.c_int, [_vp, _vp]),
    "qbe_model_create_dims": (C.c_int, [C.c_int32, _i32p, C.c_int32, _i32p, _i32p, _f64p, C.POINTER(_vp)]),
    "qbe_model_var_bits": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "qbe_slice_recompute": (C.c_int, [_vp, _i32p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_int32, C.c_uint64, _i32p, C.POINTER(C.c_int32), _i32p,
                                      C.POINTER(C.c_int32)]),
    "qbe_order_anytime": (C.c_int, [_vp, _i32p, C.c_int32, C.c_int32, C.c_uint64, _i32p, C.POINTER(C.c_int32)]),
    "qbe_order_from_td": (C.c_int, [C.c_int32, C.c_int32, _i32p, _i32p, _i32p, _i32p, C.POINTER(C.c_int32)]),
    "qbe_plan_clone": (C.c_int, [_vp, _vp, C.POINTER(_vp)]),
    "qbe_plan_stats": (C.c_int, [_vp, C.POINTER(Stats)]),
    "qbe_plan_dump": (C.c_int, [_vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "qbe_plan_check": (C.c_int, [_vp]),
    "qbe_plan_autotune": (C.c_int, [_vp, _vp, _vp, C.c_size_t, C.c_int64]),
    "qbe_contract": (C.c_int, [_vp, _vp, _vp, C.c_size_t, _f64p]),
    "qbe_contract_slices": (C.c_int, [_vp, _vp, C.c_int64, C.c_int64, _vp, C.c_size_t, _f64p, _f64p]),
    "qbe_contract_async": (C.c_int, [_vp, _vp, _vp, C.c_size_t, _vp]),
    "qbe_contract_static": (C.c_int, [_vp, _vp, _vp]),
    "qbe_plan_num_launches": (C.c_int, [_vp, C.POINTER(C.c_int32)]),
    "qbe_plan_launch_info": (C.c_int, [_vp, C.c_int32, C.c_void_p]),
    "qbe_plan_profile": (C.c_int, [_vp, _vp, _vp, C.c_size_t, C.POINTER(C.c_float), C.c_int32,
                                   C.POINTER(C.c_int32)]),
    "qbe_static_scratch_bytes": (C.c_size_t, []),
    "qbe_gnn_num_params": (C.c_int32, []),
    "qbe_gnn_create": (C.c_int, [_vp, C.c_uint64, C.POINTER(_vp)]),
    "qbe_gnn_destroy": (C.c_int, [_vp]),
    "qbe_gnn_get_params": (C.c_int, [_vp, C.POINTER(C.c_float)]),
    "qbe_gnn_set_params": (C.c_int, [_vp, C.POINTER(C.c_float)]),
    "qbe_gnn_score": (C.c_int, [_vp, _vp, C.c_int32, _i32p, _i32p, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "qbe_gnn_train_step": (C.c_int, [_vp, _vp, C.c_int32, _i32p, _i32p, C.POINTER(C.c_float), C.c_int32, _i32p,
                                     C.POINTER(C.c_float), C.c_float, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "qbe_graph_csr": (C.c_int, [_vp, _i32p, C.c_int32, _i32p, _i32p, C.c_int64, C.POINTER(C.c_int64)]),
    "qbe_batch_create": (C.c_int, [_vp, C.POINTER(_vp), C.c_int32, C.POINTER(_vp)]),
    "qbe_batch_destroy": (C.c_int, [_vp]),
    "qbe_batch_workspace": (C.c_int, [_vp, C.POINTER(C.c_size_t)]),
    "qbe_batch_contract_async": (C.c_int, [_vp, _vp, _vp, C.c_size_t, _vp]),
    "qbe_permute": (C.c_int, [_vp, _vp, _vp, C.c_int32, _i32p, C.c_int64]),
    "qbe_contract_batch": (C.c_int, [_vp, C.POINTER(_vp), C.c_int32, _vp, C.c_size_t, _f64p,
                                     C.POINTER(C.c_size_t)]),
    "qbe_gnn_save": (C.c_int, [_vp, C.c_char_p]),
    "qbe_slice_ex": (C.c_int, [_vp, _vp, _vp, _i32p, C.c_int32, C.POINTER(SliceOpts), _i32p, _i32p, _i32p, _i32p,
                               _i32p]),
    "qbe_order_learned": (C.c_int, [_vp, _vp, _vp, C.c_int32, _i32p, _i32p, _i32p, C.POINTER(C.c_uint64)]),
    "qbe_learned_sample": (C.c_int, [_vp, C.c_int32, _i32p, C.c_int32, _i32p, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_uint64, _i32p, _i32p, C.c_int64, C.POINTER(C.c_int64),
                                     C.POINTER(C.c_float), _i32p, C.POINTER(C.c_float), _i32p]),
    "qbe_gnn_score_head": (C.c_int, [_vp, _vp, C.c_int32, C.c_int32, _i32p, _i32p, C.POINTER(C.c_float),
                                     C.POINTER(C.c_float)]),
    "qbe_gnn_train_step_head": (C.c_int, [_vp, _vp, C.c_int32, C.c_int32, _i32p, _i32p, C.POINTER(C.c_float),
                                          C.c_int32, _i32p, C.POINTER(C.c_float), C.c_float,
                                          C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "qbe_gnn_load": (C.c_int, [_vp, C.c_char_p]),
    "qbe_ledger_create": (C.c_int, [C.c_int64, C.c_int64, C.c_uint64, C.POINTER(_vp)]),
    "qbe_ledger_destroy": (C.c_int, [_vp]),
    "qbe_ledger_info": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_uint64),
                                  C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "qbe_ledger_next": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "qbe_ledger_record": (C.c_int, [_vp, C.c_int64, _f64p]),
    "qbe_ledger_drop": (C.c_int, [_vp, C.c_int64]),
    "qbe_ledger_get": (C.c_int, [_vp, C.c_int64, C.POINTER(C.c_int32), _f64p]),
    "qbe_ledger_run": (C.c_int, [_vp, _vp, _vp, _vp, C.c_size_t, C.c_int64, C.POINTER(C.c_int64)]),
    "qbe_ledger_sum": (C.c_int, [_vp, _f64p]),
    "qbe_ledger_save": (C.c_int, [_vp, C.c_char_p]),
    "qbe_ledger_load": (C.c_int, [C.c_char_p, C.POINTER(_vp)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_SIGS)


def _check(rc: int, where: str):
    if rc != QBE_OK:
        raise QbeError(rc, where)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _p32(a: np.ndarray):
    return a.ctypes.data_as(_i32p)


def _dev_buffer(ctx, t, name: str, dtype=None, min_numel: int = 0):
    """Device address of a torch tensor handed to the library, after checking
    that it is a contiguous tensor on the context's device (of `dtype` and
    at least `min_numel` elements when given): the library writes through
    the raw address, so a CPU, short or mistyped tensor must not reach it."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.device.type != "cuda" or (t.device.index if t.device.index is not None else 0) != ctx.device:
        raise ValueError(f"{name} must live on cuda:{ctx.device}, not {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, not {t.dtype}")
    if t.numel() < min_numel:
        raise ValueError(f"{name} must hold at least {min_numel} elements, not {t.numel()}")
    return _vp(t.data_ptr())


def _workspace(ctx, ws):
    """(address, bytes) of a device workspace tensor (any dtype)."""
    return _dev_buffer(ctx, ws, "workspace"), ws.numel() * ws.element_size()


def _f64():
    import torch

    return torch.float64


def qbe_version() -> int:
    return int(_lib.qbe_version())


# --------------------------------------------------------------------- ctx --

class Context:
    """A device and a borrowed HIP stream (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch  # device memory and streams only

        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = _vp()
        _check(_lib.qbe_create(C.byref(h), device, _vp(stream.cuda_stream)), "qbe_create")
        self.handle = h

    def set_stream(self, stream):
        self._stream = stream
        _check(_lib.qbe_set_stream(self.handle, _vp(stream.cuda_stream)), "qbe_set_stream")

    def close(self):
        # at interpreter exit the module's globals may already be cleared;
        # the process is ending then and its device memory goes with it
        if getattr(self, "handle", None) and _lib is not None:
            _lib.qbe_destroy(self.handle)
            self.handle = None

    __del__ = close


# ------------------------------------------------------------------- model --

class Model:
    """Graphical model: n_vars binary variables and tensors (vars, data)."""

    def __init__(self, n_vars: int, tensors: Sequence[Tuple[Sequence[int], np.ndarray]]):
        self.n_vars = int(n_vars)
        self.tensor_vars = [tuple(int(v) for v in vs) for vs, _ in tensors]
        rank = _i32([len(v) for v in self.tensor_vars])
        flat = _i32([v for vs in self.tensor_vars for v in vs])
        data = self._data(tensors)
        h = _vp()
        _check(_lib.qbe_model_create(self.n_vars, len(rank), _p32(rank), _p32(flat),
                                     data.ctypes.data_as(_f64p), C.byref(h)), "qbe_model_create")
        self.handle = h

    @staticmethod
    def _data(tensors) -> np.ndarray:
        parts = [np.ascontiguousarray(np.asarray(d, dtype=np.complex128)).reshape(-1) for _, d in tensors]
        if not parts:
            return np.zeros(2)
        return np.ascontiguousarray(np.concatenate(parts).view(np.float64))

    @classmethod
    def from_circuitgen(cls, m) -> "Model":
        return cls(m.n_vars, m.tensors)

    @classmethod
    def from_dims(cls, dims: Sequence[int], tensors: Sequence[Tuple[Sequence[int], np.ndarray]]) -> "Model":
        """A network over variables of any dimensions (qbe_model_create_dims):
        tensor data shaped by its variables' dimensions, row-major.  The
        model's variables are the binary expansion; var_bits(v) maps back."""
        d = _i32(dims)
        tv = [tuple(int(v) for v in vs) for vs, _ in tensors]
        rank = _i32([len(v) for v in tv])
        flat = _i32([v for vs in tv for v in vs])
        data = cls._data(tensors)
        h = _vp()
        _check(_lib.qbe_model_create_dims(len(d), _p32(d), len(rank), _p32(rank), _p32(flat),
                                          data.ctypes.data_as(_f64p), C.byref(h)), "qbe_model_create_dims")
        m = cls.__new__(cls)
        m.handle = h
        m.dims = [int(x) for x in dims]
        m.tensor_vars = None  # binary tensors live in the library
        first, count = m.var_bits(len(d) - 1) if len(d) else (0, 0)
        m.n_vars = first + count
        return m

    def var_bits(self, v: int) -> Tuple[int, int]:
        """(first binary variable, count) of variable v."""
        f, c = C.c_int32(), C.c_int32()
        _check(_lib.qbe_model_var_bits(self.handle, v, C.byref(f), C.byref(c)), "qbe_model_var_bits")
        return f.value, c.value

    def set_data(self, tensors):
        data = self._data(tensors)
        _check(_lib.qbe_model_set_data(self.handle, data.ctypes.data_as(_f64p)), "qbe_model_set_data")

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.qbe_model_destroy(self.handle)
            self.handle = None

    __del__ = close


# ---------------------------------------------------------------- planning --

def qbe_order_min_fill(model: Model) -> List[int]:
    out = np.zeros(model.n_vars, dtype=np.int32)
    _check(_lib.qbe_order_min_fill(model.handle, _p32(out)), "qbe_order_min_fill")
    return out.tolist()


def qbe_width(model: Model, order: Sequence[int], removed: Sequence[int] = ()) -> int:
    o = _i32(order)
    r = _i32(removed)
    tau = C.c_int32()
    _check(_lib.qbe_width(model.handle, _p32(o), len(o), _p32(r), len(r), C.byref(tau)), "qbe_width")
    return tau.value


def qbe_clique_tree(model: Model, order: Sequence[int]):
    o = _i32(order)
    n = len(o)
    nb = C.c_int32()
    offs = np.zeros(n + 1, dtype=np.int32)
    par = np.zeros(max(n, 1), dtype=np.int32)
    cap = max(1, n * 4)
    while True:
        bv = np.zeros(cap, dtype=np.int32)
        rc = _lib.qbe_clique_tree(model.handle, _p32(o), n, C.byref(nb), _p32(offs), _p32(bv), cap, _p32(par))
        if rc == -4:
            cap *= 4
            continue
        _check(rc, "qbe_clique_tree")
        break
    bags = [bv[offs[i]:offs[i + 1]].tolist() for i in range(nb.value)]
    return bags, par[:nb.value].tolist()


def qbe_slice(model: Model, order: Sequence[int], m: int, target_width: int = -1,
              score: str = "tree_trimming", recompute_every: int = 0, tries: int = 8, seed: int = 0,
              net: Optional["Gnn"] = None, mem_cap: int = 0, with_fallback: bool = False):
    """Alg. 2 (with recompute_every > 0: its optional order recomputation
    after every recompute_every-th removal).  score "learned" uses the
    network `net` (qbe_slice_ex); mem_cap > 0 with m < 0 stops once the
    per-slice peak fits.  Returns (mu, reduced_order, tau), plus whether the
    learned result fell back to tree-trimming when with_fallback."""
    o = _i32(order)
    n = len(o)
    mu = np.zeros(max(n, 1), dtype=np.int32)
    red = np.zeros(max(n, 1), dtype=np.int32)
    mo = C.c_int32()
    tau = C.c_int32()
    fb = C.c_int32(0)
    if score == "learned" or mem_cap or with_fallback:
        opts = SliceOpts()
        opts.score = SCORE[score]
        opts.m = m
        opts.target_width = target_width
        opts.recompute_every = recompute_every
        opts.tries = tries
        opts.seed = seed
        opts.mem_cap = mem_cap
        ctx = net.ctx.handle if net is not None else None
        _check(_lib.qbe_slice_ex(ctx, net.handle if net is not None else None, model.handle, _p32(o), n,
                                 C.byref(opts), _p32(mu), C.byref(mo), _p32(red), C.byref(tau), C.byref(fb)),
               "qbe_slice_ex")
    elif recompute_every > 0:
        _check(_lib.qbe_slice_recompute(model.handle, _p32(o), n, m, target_width, SCORE[score],
                                        recompute_every, tries, seed, _p32(mu), C.byref(mo), _p32(red),
                                        C.byref(tau)), "qbe_slice_recompute")
    else:
        _check(_lib.qbe_slice(model.handle, _p32(o), n, m, target_width, SCORE[score], _p32(mu), C.byref(mo),
                              _p32(red), C.byref(tau)), "qbe_slice")
    k = mo.value
    out = (mu[:k].tolist(), red[:n - k].tolist(), tau.value)
    return out + (bool(fb.value),) if with_fallback else out


def qbe_order_learned(model: Model, net: "Gnn", refresh: int = 16):
    """Greedy min-fill with the elimination head breaking fill ties, min-fill
    as fallback.  Returns (order, width, fell_back, (learned FLOPs, min-fill
    FLOPs))."""
    out = np.zeros(max(model.n_vars, 1), dtype=np.int32)
    w = C.c_int32()
    fb = C.c_int32()
    fl = (C.c_uint64 * 2)()
    _check(_lib.qbe_order_learned(net.ctx.handle, net.handle, model.handle, refresh, _p32(out), C.byref(w),
                                  C.byref(fb), fl), "qbe_order_learned")
    return out[:model.n_vars].tolist(), w.value, bool(fb.value), (int(fl[0]), int(fl[1]))


def qbe_learned_sample(model: Model, head: str, order: Sequence[int], mu: Sequence[int] = (), k_elim: int = 0,
                       max_cand: int = 24, seed: int = 0):
    """One labelled state (qbe_learned_sample): (rowptr, col, feats, cand,
    target) or None when the state has fewer than two candidates."""
    o = _i32(order)
    u = _i32(mu)
    nv = model.n_vars
    rp = np.zeros(nv + 1, dtype=np.int32)
    feats = np.zeros((nv, FEATURES), dtype=np.float32)
    cand = np.zeros(max_cand, dtype=np.int32)
    tgt = np.zeros(max_cand, dtype=np.float32)
    nnz = C.c_int64()
    nc = C.c_int32()
    cap = 1 << 16
    while True:
        col = np.zeros(cap, dtype=np.int32)
        rc = _lib.qbe_learned_sample(model.handle, HEAD[head], _p32(o), len(o), _p32(u), len(u), k_elim, max_cand,
                                     seed, _p32(rp), _p32(col), cap, C.byref(nnz),
                                     feats.ctypes.data_as(C.POINTER(C.c_float)), _p32(cand),
                                     tgt.ctypes.data_as(C.POINTER(C.c_float)), C.byref(nc))
        if rc == -4 and nnz.value > cap:
            cap = int(nnz.value)
            continue
        _check(rc, "qbe_learned_sample")
        break
    if nc.value < 2:
        return None
    return rp, col[:nnz.value].copy(), feats, cand[:nc.value].copy(), tgt[:nc.value].copy()


def qbe_order_anytime(model: Model, removed: Sequence[int] = (), tries: int = 8, seed: int = 0):
    """The anytime tree-decomposition heuristic.  Returns (order, width)."""
    r = _i32(removed)
    out = np.zeros(max(model.n_vars, 1), dtype=np.int32)
    w = C.c_int32()
    _check(_lib.qbe_order_anytime(model.handle, _p32(r), len(r), tries, seed, _p32(out), C.byref(w)),
           "qbe_order_anytime")
    return out[:model.n_vars - len(r)].tolist(), w.value


def qbe_order_from_td(n_vars: int, bags: Sequence[Sequence[int]], parent: Sequence[int]) -> List[int]:
    """Alg. 5: an elimination order consistent with a tree decomposition."""
    offs = [0]
    flat: List[int] = []
    for b in bags:
        flat += sorted(b)
        offs.append(len(flat))
    bo, bv, pa = _i32(offs), _i32(flat if flat else [0]), _i32(parent if len(parent) else [0])
    out = np.zeros(max(n_vars, 1), dtype=np.int32)
    k = C.c_int32()
    _check(_lib.qbe_order_from_td(n_vars, len(bags), _p32(bo), _p32(bv), _p32(pa), _p32(out), C.byref(k)),
           "qbe_order_from_td")
    return out[:k.value].tolist()


def qbe_schedule_cost(model: Model, reduced_order: Sequence[int], mu: Sequence[int]) -> dict:
    """Exact per-slice cost of a schedule (no device programs)."""
    o = _i32(reduced_order)
    u = _i32(mu)
    out = (C.c_uint64 * 4)()
    _check(_lib.qbe_schedule_cost(model.handle, _p32(o), len(o), _p32(u), len(u), out), "qbe_schedule_cost")
    return {"flops_per_slice": out[0], "bytes_per_slice": out[1], "peak_bytes_per_slice": out[2],
            "width": int(out[3]), "n_slices": 1 << len(u)}


FEATURES = 8


def qbe_vertex_features(model: Model, order: Sequence[int], removed: Sequence[int] = ()) -> np.ndarray:
    """(n_vars, 8) float32 features of the graph without `removed`."""
    o = _i32(order)
    r = _i32(removed)
    out = np.zeros((model.n_vars, FEATURES), dtype=np.float32)
    _check(_lib.qbe_vertex_features(model.handle, _p32(o), len(o), _p32(r), len(r),
                                    out.ctypes.data_as(C.POINTER(C.c_float))), "qbe_vertex_features")
    return out


# ------------------------------------------------------------------- plans --

class Plan:
    """Compiled schedule (and device programs when a context is given)."""

    def __init__(self, model: Model, reduced_order: Sequence[int], mu: Sequence[int],
                 ctx: Optional[Context] = None, exec: str = "auto", precision: str = "fp32",
                 merge: bool = True, fused_prefix=False, fused_segments: bool = False, fold_inputs: bool = True,
                 max_sums: int = 0):
        o = _i32(reduced_order)
        u = _i32(mu)
        opts = PlanOpts()
        opts.exec = EXEC[exec]
        opts.precision = PREC[precision]
        opts.no_merge = 0 if merge else 1
        # False/True: no prefix / the largest rank bound that fits; an int
        # R >= 2: buckets of at most R + 1 variables
        opts.fused_prefix = int(fused_prefix)
        opts.fused_segments = 1 if fused_segments else 0
        opts.no_fold = 0 if fold_inputs else 1
        # summed variables a merged per-step launch may hold (0: default 4)
        opts.max_sums = int(max_sums)
        h = _vp()
        _check(_lib.qbe_plan_create(ctx.handle if ctx else None, model.handle, _p32(o), len(o), _p32(u), len(u),
                                    C.byref(opts), C.byref(h)), "qbe_plan_create")
        self.handle = h
        self.ctx = ctx
        self.model = model
        self.n_slices = 1 << len(u)

    def stats(self) -> dict:
        s = Stats()
        _check(_lib.qbe_plan_stats(self.handle, C.byref(s)), "qbe_plan_stats")
        return s.as_dict()

    def dump(self) -> str:
        n = C.c_size_t()
        _check(_lib.qbe_plan_dump(self.handle, None, 0, C.byref(n)), "qbe_plan_dump")
        buf = C.create_string_buffer(n.value + 1)
        _check(_lib.qbe_plan_dump(self.handle, buf, n.value + 1, C.byref(n)), "qbe_plan_dump")
        return buf.value.decode()

    def check(self):
        _check(_lib.qbe_plan_check(self.handle), "qbe_plan_check")

    def update_data(self, model: Model):
        _check(_lib.qbe_plan_update_data(self.handle, model.handle), "qbe_plan_update_data")

    def clone(self, model: Model) -> "Plan":
        """A plan for a model of the same structure (e.g. another bitstring of
        the same circuit) that reuses this plan's schedule and programs."""
        h = _vp()
        _check(_lib.qbe_plan_clone(self.handle, model.handle, C.byref(h)), "qbe_plan_clone")
        p = Plan.__new__(Plan)
        p.handle = h
        p.ctx = self.ctx
        p.model = model
        p.n_slices = self.n_slices
        return p

    def autotune(self, ws, min_elems: int = 1 << 20):
        """Times the large per-step launches in each tile shape; keeps the best."""
        w, nb = _workspace(self.ctx, ws)
        _check(_lib.qbe_plan_autotune(self.ctx.handle, self.handle, w, nb, min_elems), "qbe_plan_autotune")

    def launches(self) -> list:
        """Per-launch info of a per-step plan (qbe_plan_launch_info), in
        execution order, then finalize and reduce."""
        n = C.c_int32()
        _check(_lib.qbe_plan_num_launches(self.handle, C.byref(n)), "qbe_plan_num_launches")
        out = []
        for i in range(n.value):
            li = LaunchInfo()
            _check(_lib.qbe_plan_launch_info(self.handle, i, C.byref(li)), "qbe_plan_launch_info")
            out.append(li.as_dict())
        return out

    def profile(self, ws) -> np.ndarray:
        """Milliseconds of each launch of one contraction of all slices
        (qbe_plan_profile), in the order of launches()."""
        n = C.c_int32()
        _check(_lib.qbe_plan_num_launches(self.handle, C.byref(n)), "qbe_plan_num_launches")
        ms = np.zeros(max(n.value, 1), dtype=np.float32)
        w, nb = _workspace(self.ctx, ws)
        got = C.c_int32()
        _check(_lib.qbe_plan_profile(self.ctx.handle, self.handle, w, nb, ms.ctypes.data_as(C.POINTER(C.c_float)),
                                     len(ms), C.byref(got)), "qbe_plan_profile")
        return ms[:got.value].copy()

    def workspace(self, all_slices: bool = True):
        """A device workspace (torch uint8 tensor) of the plan's size."""
        import torch

        st = self.stats()
        n = st["ws_bytes_all_slices"] if all_slices else st["ws_bytes_min"]
        return torch.empty(int(n), dtype=torch.uint8, device=f"cuda:{self.ctx.device}")

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.qbe_plan_destroy(self.handle)
            self.handle = None

    __del__ = close


def qbe_contract(ctx: Context, plan: Plan, ws) -> complex:
    out = np.zeros(2)
    w, nb = _workspace(ctx, ws)
    _check(_lib.qbe_contract(ctx.handle, plan.handle, w, nb, out.ctypes.data_as(_f64p)), "qbe_contract")
    return complex(out[0], out[1])


def qbe_contract_slices(ctx: Context, plan: Plan, s_begin: int, s_end: int, ws):
    """Returns (sum over the range, per-slice values as complex128 array)."""
    part = np.zeros(2)
    per = np.zeros(2 * (s_end - s_begin))
    w, nb = _workspace(ctx, ws)
    _check(_lib.qbe_contract_slices(ctx.handle, plan.handle, s_begin, s_end, w, nb,
                                    part.ctypes.data_as(_f64p), per.ctypes.data_as(_f64p)), "qbe_contract_slices")
    return complex(part[0], part[1]), per.view(np.complex128).copy()


def qbe_contract_async(ctx: Context, plan: Plan, ws, d_out):
    """Enqueues the contraction; d_out is a float64 device tensor of >= 2 entries."""
    w, nb = _workspace(ctx, ws)
    out = _dev_buffer(ctx, d_out, "d_out", _f64(), 2)
    _check(_lib.qbe_contract_async(ctx.handle, plan.handle, w, nb, out), "qbe_contract_async")


def qbe_contract_static(ctx: Context, plan: Plan, d_out):
    """Enqueues the contraction on the library's fixed per-device workspace
    (no allocation anywhere); d_out is a float64 device tensor of >= 2
    entries.  Calls overlapping on one device share that workspace."""
    out = _dev_buffer(ctx, d_out, "d_out", _f64(), 2)
    _check(_lib.qbe_contract_static(ctx.handle, plan.handle, out), "qbe_contract_static")


def qbe_static_scratch_bytes() -> int:
    return int(_lib.qbe_static_scratch_bytes())


def qbe_contract_batch(ctx: Context, plans: Sequence[Plan], ws=None) -> np.ndarray:
    """All plans in one synchronous call; returns their complex128
    amplitudes.  ws: a uint8 device tensor of at least
    qbe_contract_batch_workspace(ctx, plans) bytes (allocated when None)."""
    arr = (_vp * len(plans))(*[p.handle for p in plans])
    if ws is None:
        import torch
        ws = torch.empty(qbe_contract_batch_workspace(ctx, plans), dtype=torch.uint8, device=f"cuda:{ctx.device}")
    amps = np.zeros(2 * len(plans), dtype=np.float64)
    w, nb = _workspace(ctx, ws)
    _check(_lib.qbe_contract_batch(ctx.handle, arr, len(plans), w, nb, amps.ctypes.data_as(_f64p), None),
           "qbe_contract_batch")
    return amps.view(np.complex128)


def qbe_contract_batch_workspace(ctx: Context, plans: Sequence[Plan]) -> int:
    arr = (_vp * len(plans))(*[p.handle for p in plans])
    n = C.c_size_t()
    _check(_lib.qbe_contract_batch(ctx.handle, arr, len(plans), None, 0, None, C.byref(n)), "qbe_contract_batch")
    return n.value


class Batch:
    """Many plans contracted in one persistent fused launch."""

    def __init__(self, ctx: Context, plans: Sequence[Plan]):
        arr = (_vp * len(plans))(*[p.handle for p in plans])
        h = _vp()
        _check(_lib.qbe_batch_create(ctx.handle, arr, len(plans), C.byref(h)), "qbe_batch_create")
        self.handle = h
        self.ctx = ctx
        self.plans = list(plans)
        n = C.c_size_t()
        _check(_lib.qbe_batch_workspace(h, C.byref(n)), "qbe_batch_workspace")
        self.ws_bytes = n.value

    def workspace(self):
        import torch

        return torch.empty(int(self.ws_bytes), dtype=torch.uint8, device=f"cuda:{self.ctx.device}")

    def contract_async(self, ws, d_amps):
        """Enqueues the batch; d_amps: float64 device tensor of >= 2 * n_plans entries."""
        w, nb = _workspace(self.ctx, ws)
        out = _dev_buffer(self.ctx, d_amps, "d_amps", _f64(), 2 * len(self.plans))
        _check(_lib.qbe_batch_contract_async(self.ctx.handle, self.handle, w, nb, out), "qbe_batch_contract_async")

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.qbe_batch_destroy(self.handle)
            self.handle = None

    __del__ = close


# ------------------------------------------------------------ slice ledger --

class Ledger:
    """Which slice ranges of one contraction are done, and their FP64
    partial sums (the slices are independent, Sec. 2.4; their sum is the
    result, Eq. 4): a lost range is contracted again alone, and an
    interrupted job resumes from a saved ledger."""

    def __init__(self, n_slices: int, range_size: int, tag: int = 0, _handle=None):
        h = _handle
        if h is None:
            h = _vp()
            _check(_lib.qbe_ledger_create(int(n_slices), int(range_size), int(tag), C.byref(h)), "qbe_ledger_create")
        self.handle = h

    @classmethod
    def load(cls, path: str) -> "Ledger":
        h = _vp()
        _check(_lib.qbe_ledger_load(os.fsencode(path), C.byref(h)), "qbe_ledger_load")
        return cls(0, 0, _handle=h)

    def save(self, path: str):
        _check(_lib.qbe_ledger_save(self.handle, os.fsencode(path)), "qbe_ledger_save")

    def info(self) -> dict:
        v = [C.c_int64(), C.c_int64(), C.c_uint64(), C.c_int64(), C.c_int64()]
        _check(_lib.qbe_ledger_info(self.handle, *[C.byref(x) for x in v]), "qbe_ledger_info")
        return dict(zip(("n_slices", "range_size", "tag", "n_ranges", "n_done"), (x.value for x in v)))

    def next(self):
        """(index, s_begin, s_end) of the lowest pending range, or None."""
        v = [C.c_int64(), C.c_int64(), C.c_int64()]
        _check(_lib.qbe_ledger_next(self.handle, *[C.byref(x) for x in v]), "qbe_ledger_next")
        return None if v[0].value < 0 else tuple(x.value for x in v)

    def record(self, idx: int, partial: complex):
        p = np.array([partial.real, partial.imag], dtype=np.float64)
        _check(_lib.qbe_ledger_record(self.handle, int(idx), p.ctypes.data_as(_f64p)), "qbe_ledger_record")

    def drop(self, idx: int):
        _check(_lib.qbe_ledger_drop(self.handle, int(idx)), "qbe_ledger_drop")

    def get(self, idx: int):
        """(done, partial sum) of range idx."""
        d = C.c_int32()
        p = np.zeros(2)
        _check(_lib.qbe_ledger_get(self.handle, int(idx), C.byref(d), p.ctypes.data_as(_f64p)), "qbe_ledger_get")
        return bool(d.value), complex(p[0], p[1])

    def run(self, ctx: Context, plan: Plan, ws, max_ranges: int = -1) -> int:
        """Contracts up to max_ranges pending ranges (all if < 0); returns
        how many were recorded."""
        n = C.c_int64()
        w, nb = _workspace(ctx, ws)
        _check(_lib.qbe_ledger_run(ctx.handle, plan.handle, self.handle, w, nb, int(max_ranges), C.byref(n)),
               "qbe_ledger_run")
        return n.value

    def sum(self) -> complex:
        out = np.zeros(2)
        _check(_lib.qbe_ledger_sum(self.handle, out.ctypes.data_as(_f64p)), "qbe_ledger_sum")
        return complex(out[0], out[1])

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.qbe_ledger_destroy(self.handle)
            self.handle = None

    __del__ = close


# ----------------------------------------------------------------- permute --

def qbe_permute(ctx: Context, d_in, d_out, r: int, perm: Sequence[int], batch: int = 1):
    """Enqueues out[b][sum_j x_{perm[j]} 2^j] = in[b][sum_p x_p 2^p] for batch
    tensors of 2^r complex64 entries (d_in, d_out: contiguous device tensors
    of at least batch * 2^r * 8 bytes, not overlapping)."""
    need = int(batch) << int(r) if batch > 0 else 0
    ptrs = []
    for name, t in (("d_in", d_in), ("d_out", d_out)):
        ptrs.append(_dev_buffer(ctx, t, name))
        if t.numel() * t.element_size() < need * 8:
            raise ValueError(f"{name} must hold >= {need * 8} bytes")
    p = _i32(perm)
    _check(_lib.qbe_permute(ctx.handle, ptrs[0], ptrs[1], int(r), _p32(p), int(batch)), "qbe_permute")


# -------------------------------------------------------- learned proposal --

def _fp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def qbe_graph_csr(model: Model, removed: Sequence[int] = ()):
    """(rowptr int32[n_vars + 1], col int32[nnz]) of the graph without `removed`."""
    r = _i32(removed)
    rp = np.zeros(model.n_vars + 1, dtype=np.int32)
    nnz = C.c_int64()
    cap = 1 << 16
    while True:
        col = np.zeros(cap, dtype=np.int32)
        rc = _lib.qbe_graph_csr(model.handle, _p32(r), len(r), _p32(rp), _p32(col), cap, C.byref(nnz))
        if rc == -4:
            cap = int(nnz.value)
            continue
        _check(rc, "qbe_graph_csr")
        return rp, col[:nnz.value].copy()


class Gnn:
    """The learned slicing proposal's network, resident on the device."""

    n_params = int(_lib.qbe_gnn_num_params())

    def __init__(self, ctx: Context, seed: int = 0):
        h = _vp()
        _check(_lib.qbe_gnn_create(ctx.handle, seed, C.byref(h)), "qbe_gnn_create")
        self.handle = h
        self.ctx = ctx

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(_lib.qbe_gnn_get_params(self.handle, _fp(out)), "qbe_gnn_get_params")
        return out

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.shape == (self.n_params,)
        _check(_lib.qbe_gnn_set_params(self.handle, _fp(p)), "qbe_gnn_set_params")

    def save(self, path: str):
        """Checkpoint: parameters, Adam moments and step count."""
        _check(_lib.qbe_gnn_save(self.handle, os.fsencode(path)), "qbe_gnn_save")

    def load(self, path: str):
        _check(_lib.qbe_gnn_load(self.handle, os.fsencode(path)), "qbe_gnn_load")

    def score(self, rowptr, col, feats, head: str = "slicing") -> np.ndarray:
        rp, cl = _i32(rowptr), _i32(col)
        f = np.ascontiguousarray(feats, dtype=np.float32)
        n = len(rp) - 1
        out = np.zeros(n, dtype=np.float32)
        _check(_lib.qbe_gnn_score_head(self.ctx.handle, self.handle, HEAD[head], n, _p32(rp), _p32(cl), _fp(f),
                                       _fp(out)), "qbe_gnn_score_head")
        return out

    def train_step(self, rowptr, col, feats, cand, target, lr: float, want_grads: bool = False,
                   head: str = "slicing"):
        rp, cl, cd = _i32(rowptr), _i32(col), _i32(cand)
        f = np.ascontiguousarray(feats, dtype=np.float32)
        y = np.ascontiguousarray(target, dtype=np.float32)
        n = len(rp) - 1
        loss = np.zeros(1, dtype=np.float32)
        grads = np.zeros(self.n_params, dtype=np.float32) if want_grads else None
        _check(_lib.qbe_gnn_train_step_head(self.ctx.handle, self.handle, HEAD[head], n, _p32(rp), _p32(cl),
                                            _fp(f), len(cd), _p32(cd), _fp(y), lr, _fp(loss),
                                            _fp(grads) if want_grads else None), "qbe_gnn_train_step_head")
        return (float(loss[0]), grads) if want_grads else float(loss[0])

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.qbe_gnn_destroy(self.handle)
            self.handle = None

    __del__ = close


# ------------------------------------------------------------ conveniences --

def plan_circuit(model: Model, m: int = 0, target_width: int = -1, score: str = "tree_trimming"):
    """Host planning of one network: min-fill order, then Alg. 2.
    Returns (order, mu, reduced_order, tau)."""
    order = qbe_order_min_fill(model)
    mu, red, tau = qbe_slice(model, order, m, target_width, score)
    return order, mu, red, tau
