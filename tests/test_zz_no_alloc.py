"""The allocation-free training step (fcs_sdnn_train_step_noalloc) against
the workspace form (fcs_sdnn_train_step) through the C ABI: two calls in a
row on continuing Adam states, the second with a smaller batch and new data,
must give the same loss, gradients, parameters and moments bit for bit (the
two share their kernels; only the scratch differs).  Sizes beyond the static
scratch are refused."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_2506_19370_amd import _lib as L  # noqa: E402
import workloads as W  # noqa: E402

vp = ctypes.c_void_p


def _p(t):
    return vp(t.data_ptr())


def _stream():
    return vp(torch.cuda.current_stream().cuda_stream)


class _State:
    def __init__(self, blob):
        self.params = torch.tensor(blob, dtype=torch.float32, device="cuda")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.full_like(self.params, float("nan"))
        self.loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")


def _inputs(B, salt):
    g = W.rng(7, salt)
    x = torch.tensor(g.random((B, 16)), dtype=torch.float32, device="cuda")
    lab = torch.tensor(g.integers(0, 3, B), dtype=torch.int32, device="cuda")
    cw = torch.tensor([0.4, 2.0, 5.0], dtype=torch.float32, device="cuda")
    return x, lab, cw


def test_noalloc_train_step_matches_workspace_form():
    blob = W.sdnn_blob(W.sdnn_init(W.rng(4, 60)))
    a, b = _State(blob), _State(blob)
    lr = ctypes.c_float(1e-3)
    for t, (B, salt) in enumerate([(L.SDNN_TRAIN_MAX_BATCH, 61), (1000, 62)], start=1):
        x, lab, cw = _inputs(B, salt)
        nb = L.fcs_sdnn_train_workspace(B)
        ws = torch.full((int(nb) // 4,), float("nan"), dtype=torch.float32, device="cuda")
        L.check(L.fcs_sdnn_train_step(_p(a.params), _p(a.m), _p(a.v), t, lr, _p(x), _p(lab), _p(cw), B,
                                      _p(a.loss), _p(a.grads), 0, _p(ws), nb, _stream()))
        L.check(L.fcs_sdnn_train_step_noalloc(_p(b.params), _p(b.m), _p(b.v), t, lr, _p(x), _p(lab), _p(cw), B,
                                              _p(b.loss), _p(b.grads), 0, _stream()))
        torch.cuda.synchronize()
        assert torch.isfinite(a.loss).all() and torch.isfinite(a.grads).all()
        for name in ("loss", "grads", "params", "m", "v"):
            ta, tb = getattr(a, name), getattr(b, name)
            assert torch.equal(ta, tb), (t, B, name, (ta - tb).abs().max().item())


def test_noalloc_train_step_refuses_batches_beyond_its_scratch():
    s = _State(W.sdnn_blob(W.sdnn_init(W.rng(4, 63))))
    x, lab, cw = _inputs(16, 64)
    before = s.params.clone()
    st = L.fcs_sdnn_train_step_noalloc(_p(s.params), _p(s.m), _p(s.v), 1, ctypes.c_float(1e-3), _p(x), _p(lab),
                                       _p(cw), L.SDNN_TRAIN_MAX_BATCH + 1, _p(s.loss), _p(s.grads), 0, _stream())
    assert st == L.FCS_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(s.params, before)
