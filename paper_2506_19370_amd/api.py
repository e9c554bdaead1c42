"""Python front end of the MI355X FC-SDNN solver (thin wrapper of the C ABI).

Device memory and streams come from PyTorch; every numerical step runs in
the library's HIP kernels (``libfcsdnn.so``).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


@dataclass
class SolverParams:
    gamma: float = 1.4
    cfl: float = 0.5
    c_mu: float = 1.0
    dt_fixed: float = 0.0
    fc_d: int = 5
    fc_C: int = 27
    n_f: int = 5
    n_v: int = 9
    precision: str = "fp64"
    av: str = "off"
    filter: bool = False
    use_graph: bool = False
    autotune: bool = False
    visc_all_lines: bool = False
    sdnn_weights: np.ndarray | None = None
    vortex: tuple = (5.0, 5.0, 5.0, 1.0, 1.0)
    smear: bool = False


def create_context(specs, prm: SolverParams) -> ctypes.c_void_p:
    """fcs_create for a list of subpatch specs (host only: grids, metrics,
    operators and connectivity; no device memory).  Returns the context
    handle; the caller releases it with fcs_destroy (Solver does)."""
    keep = []
    cp = L.Params()
    cp.gamma, cp.cfl, cp.c_mu, cp.dt_fixed = prm.gamma, prm.cfl, prm.c_mu, prm.dt_fixed
    cp.fc_d, cp.fc_C, cp.n_f, cp.n_v = prm.fc_d, prm.fc_C, prm.n_f, prm.n_v
    cp.precision = L.PREC[prm.precision]
    cp.av_mode = L.AV[prm.av]
    cp.filter = int(bool(prm.filter))
    cp.use_graph = int(bool(prm.use_graph))
    cp.autotune = int(bool(prm.autotune))
    cp.visc_all_lines = int(bool(prm.visc_all_lines))
    cp.smear = int(bool(prm.smear))
    if prm.sdnn_weights is not None:
        w = np.ascontiguousarray(prm.sdnn_weights, dtype=np.float32)
        if w.size != L.SDNN_NPARAM:
            raise ValueError("SDNN weights must hold %d floats" % L.SDNN_NPARAM)
        keep.append(w)
        cp.sdnn_weights = w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    cp.vortex = (ctypes.c_double * 5)(*prm.vortex)
    descs = (L.PatchDesc * len(specs))()
    for q, s in enumerate(specs):
        x = np.ascontiguousarray(s.x, dtype=np.float64)
        y = np.ascontiguousarray(s.y, dtype=np.float64)
        keep += [x, y]
        d = descs[q]
        d.type = L.PATCH.get(getattr(s, "kind", "I"), 0)
        d.n2, d.n1 = x.shape
        d.x = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.y = y.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if s.mask is not None:
            m = np.ascontiguousarray(s.mask, dtype=np.uint8)
            keep.append(m)
            d.mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        for k, side in enumerate("WESN"):
            v = s.sides[side]
            d.side[k] = L.SIDE[v] if isinstance(v, str) else int(v)
        d.notch = L.SIDE[s.notch] if isinstance(s.notch, str) else int(s.notch)
        inflow = s.inflow if s.inflow is not None else (1.0, 0.0, 0.0, 1.0)
        for k in range(4):
            d.inflow[k] = float(inflow[k])
    h = ctypes.c_void_p()
    st = L.fcs_create(ctypes.byref(cp), len(specs), descs, ctypes.byref(h))
    if st != L.FCS_OK:
        msg = L.fcs_last_error(h).decode() if h.value else ""
        if h.value:
            L.fcs_destroy(h)
        raise L.FcsError(st, msg)
    return h


class Solver:
    """Subpatch set + state on one GPU (create / bind / set state / advance /
    query).  ``specs``: objects with x, y (n2, n1), mask, sides (dict W/E/S/N
    of kind names or ints), notch, inflow (primitive) and kind."""

    def __init__(self, specs, prm: SolverParams, device="cuda", stream=None):
        self.prm = prm
        self.specs = list(specs)
        self.device = torch.device(device)
        self.h = None
        h = create_context(self.specs, prm)
        self.h = h
        nbytes = ctypes.c_size_t()
        L.check(L.fcs_workspace_size(h, ctypes.byref(nbytes)), h)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L.check(L.fcs_bind(h, ctypes.c_void_p(self.workspace.data_ptr()), nbytes.value,
                           ctypes.c_void_p(_stream_handle(self.stream))), h)

    def __del__(self):
        if getattr(self, "h", None) and L is not None and L.fcs_destroy is not None:
            L.fcs_destroy(self.h)
            self.h = None

    def set_state(self, p: int, values, prim: bool = True):
        arr = np.ascontiguousarray(values, dtype=np.float64)
        L.check(L.fcs_set_state(self.h, p, 1 if prim else 0, arr.ctypes.data, 0), self.h)

    def set_time(self, t: float):
        L.check(L.fcs_set_time(self.h, t), self.h)

    def set_tau(self, p: int, tau):
        arr = np.ascontiguousarray(tau, dtype=np.uint8)
        L.check(L.fcs_set_tau(self.h, p, arr.ctypes.data), self.h)

    def advance(self, n_stages: int, sync: bool = False):
        t = ctypes.c_double()
        L.check(L.fcs_advance(self.h, int(n_stages), ctypes.byref(t) if sync else None), self.h)
        return t.value if sync else None

    def field(self, p: int, name: str) -> np.ndarray:
        n2, n1 = self.specs[p].x.shape
        out = np.zeros((n2, n1))
        L.check(L.fcs_get_field(self.h, p, L.FIELD[name], out.ctypes.data, 0), self.h)
        return out

    def cons(self, p: int) -> np.ndarray:
        return np.stack([self.field(p, k) for k in ("rho", "mx", "my", "E")])

    def stats(self):
        s = L.Stats()
        L.check(L.fcs_stats(self.h, ctypes.byref(s)), self.h)
        return {k: getattr(s, k) for k, _ in L.Stats._fields_}

    def autotune_times(self):
        """Average launch ms of every stage-contraction candidate (0: not timed)."""
        n = L.fcs_gemm_variant_count(L.PREC[self.prm.precision])
        ms = (ctypes.c_double * n)()
        L.check(L.fcs_autotune_times(self.h, n, ms), self.h)
        return list(ms)

    def set_stage_variant(self, name: str):
        """Pin the stage-contraction tile shape (a name from
        gemm_variant_name for the solver's precision) instead of tuning it."""
        n = L.fcs_gemm_variant_count(L.PREC[self.prm.precision])
        names = [L.gemm_variant_name(self.prm.precision, i) for i in range(n)]
        if name not in names:
            raise ValueError(f"unknown stage variant {name!r}; candidates: {names}")
        L.check(L.fcs_set_stage_variant(self.h, names.index(name)), self.h)

    def retune(self):
        """Tune the contraction tile shape again at the next advance, on the
        current state's work (fcs_retune)."""
        L.check(L.fcs_retune(self.h), self.h)

    def profile(self, on: bool):
        L.check(L.fcs_profile_enable(self.h, int(on)), self.h)

    def profile_stage(self, reps: int = 50):
        """The last step's stage contraction timed alone: average ms of
        `reps` back-to-back launches and the useful flops and bytes of one."""
        ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        L.check(L.fcs_profile_stage(self.h, int(reps), ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by)), self.h)
        return {"avg_ms": ms.value, "flops": fl.value, "bytes": by.value, "launches": int(reps)}

    def profile_read(self):
        ms, fl, by, n, lat = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        L.check(L.fcs_profile_read(self.h, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by), ctypes.byref(n),
                                   ctypes.byref(lat)), self.h)
        return {"avg_ms": ms.value, "flops": fl.value, "bytes": by.value, "launches": n.value,
                "event_latency_ms": lat.value}


class DerivSweep:
    """d/dq^1 and d/dq^2 (index units) of ncomp fields on many rectangular
    patches in one grouped launch."""

    def __init__(self, sizes, ncomp=4, precision="fp64", d=5, C=27, device="cuda", stream=None):
        sz = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32).reshape(-1, 2))
        self.sizes = sz
        self.ncomp = ncomp
        h = ctypes.c_void_p()
        L.check(L.fcs_sweep_create(len(sz), sz.ctypes.data, ncomp, L.PREC[precision], d, C, ctypes.byref(h)))
        self.h = h
        nbytes = ctypes.c_size_t()
        L.check(L.fcs_sweep_workspace_size(h, ctypes.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        L.check(L.fcs_sweep_bind(h, ctypes.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                 ctypes.c_void_p(_stream_handle(self.stream))))
        n = ctypes.c_int64()
        L.check(L.fcs_sweep_points(h, ctypes.byref(n)))
        self.npoints = n.value
        self.total = self.npoints * ncomp

    def __del__(self):
        if getattr(self, "h", None) and L is not None and L.fcs_sweep_destroy is not None:
            L.fcs_sweep_destroy(self.h)
            self.h = None

    def run(self, x: torch.Tensor, d1: torch.Tensor, d2: torch.Tensor):
        for t in (x, d1, d2):
            if t.dtype != torch.float64 or not t.is_cuda or t.numel() != self.total or not t.is_contiguous():
                raise ValueError("sweep arrays must be contiguous FP64 device tensors of the sweep's size")
        L.check(L.fcs_sweep_run(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(d1.data_ptr()),
                                ctypes.c_void_p(d2.data_ptr())))

    def set_variant(self, index: int):
        L.check(L.fcs_sweep_set_variant(self.h, int(index)))

    @staticmethod
    def variant_count(precision: str) -> int:
        return int(L.fcs_gemm_variant_count(L.PREC[precision]))

    def autotune(self, x: torch.Tensor, d1: torch.Tensor, d2: torch.Tensor):
        ms = np.zeros(16)
        L.check(L.fcs_sweep_autotune(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(d1.data_ptr()),
                                     ctypes.c_void_p(d2.data_ptr()), ms.ctypes.data))
        return ms

    def profile(self, on: int):
        ms, fl, by, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        L.check(L.fcs_sweep_profile(self.h, on, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by),
                                    ctypes.byref(n)))
        return {"avg_ms": ms.value, "flops": fl.value, "bytes": by.value, "launches": n.value}


def sdnn_infer(params: torch.Tensor, windows: torch.Tensor, logits: bool = False, stream=None):
    """Classes (uint8) of raw 16-point windows (nwin, 16) FP64 on the device."""
    nwin = windows.shape[0]
    tau = torch.empty(nwin, dtype=torch.uint8, device=windows.device)
    lg = torch.empty((nwin, 3), dtype=torch.float32, device=windows.device) if logits else None
    L.check(L.fcs_sdnn_infer(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(windows.data_ptr()), nwin,
                             ctypes.c_void_p(tau.data_ptr()), ctypes.c_void_p(lg.data_ptr()) if logits else None,
                             ctypes.c_void_p(_stream_handle(stream))))
    return (tau, lg) if logits else tau


def modal_infer(windows: torch.Tensor, stream=None):
    nwin = windows.shape[0]
    tau = torch.empty(nwin, dtype=torch.uint8, device=windows.device)
    L.check(L.fcs_modal_infer(ctypes.c_void_p(windows.data_ptr()), nwin, ctypes.c_void_p(tau.data_ptr()),
                              ctypes.c_void_p(_stream_handle(stream))))
    return tau


class SdnnTrainer:
    """Adam training of the classifier with the library's kernels; the
    parameters are an FP32 device tensor in the C-ABI blob order."""

    def __init__(self, params: torch.Tensor, batch: int, lr: float = 1e-3, fp32_activations: bool = False):
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.t = 0
        self.lr = lr
        self.batch = batch
        self.flags = 1 if fp32_activations else 0
        nb = L.fcs_sdnn_train_workspace(batch)
        self.ws = torch.empty(int(nb), dtype=torch.uint8, device=params.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        self.grads = torch.zeros_like(params)

    def step(self, x: torch.Tensor, labels: torch.Tensor, class_weight: torch.Tensor, stream=None):
        B = x.shape[0]
        if B > self.batch:
            raise ValueError("batch larger than the trainer's workspace")
        self.t += 1
        L.check(L.fcs_sdnn_train_step(
            ctypes.c_void_p(self.params.data_ptr()), ctypes.c_void_p(self.m.data_ptr()),
            ctypes.c_void_p(self.v.data_ptr()), self.t, ctypes.c_float(self.lr), ctypes.c_void_p(x.data_ptr()),
            ctypes.c_void_p(labels.data_ptr()), ctypes.c_void_p(class_weight.data_ptr()), B,
            ctypes.c_void_p(self.loss.data_ptr()), ctypes.c_void_p(self.grads.data_ptr()), self.flags,
            ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), ctypes.c_void_p(_stream_handle(stream))))
        return self.loss


def lines_apply(x: torch.Tensor, kind: str, d: int, C: int, stream=None) -> torch.Tensor:
    """Apply the dense FC operator ``kind`` along the rows of x (nlines, n)."""
    nl, n = x.shape
    out = torch.empty_like(x)
    nb = L.fcs_lines_workspace(n, nl)
    ws = torch.empty(int(nb), dtype=torch.uint8, device=x.device)
    L.check(L.fcs_lines_apply(n, nl, L.OP[kind], d, C, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                              ctypes.c_void_p(ws.data_ptr()), nb, ctypes.c_void_p(_stream_handle(stream))))
    return out
