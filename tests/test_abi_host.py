"""Host-side checks of the C ABI (no GPU): every symbol the header declares
is exported, the host FC construction agrees with the oracle's independent
construction, and subpatch-set creation validates its input."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fcsdnn.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    names = set()
    for decl in text.split(";"):
        if "typedef" in decl or "enum" in decl or "struct" in decl and "{" in decl:
            continue
        m = re.search(r"\b(fcs_\w+)\s*\(", decl)
        if m:
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = header_functions()
    for required in ("fcs_create", "fcs_bind", "fcs_set_state", "fcs_advance", "fcs_get_field", "fcs_destroy",
                     "fcs_sweep_run", "fcs_sdnn_train_step", "fcs_sdnn_infer"):
        assert required in names
    assert len(names) >= 25


def test_library_exports_every_declared_symbol():
    from paper_2506_19370_amd import _lib as L
    lib = ctypes.CDLL(L.LIBPATH)
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("d", [2, 5])
def test_fc_continuation_matches_oracle(d):
    from oracle import fcgram
    import paper_2506_19370_amd as F
    Q, A = F.fc_continuation(d, 27)
    ref = fcgram.continuation_data(d, 27)
    # Q^T Q = I, and the continuation of raw matching values B = A Q^T is
    # independent of the sign convention of the Gram polynomials.  The
    # continuation points lie between the two fitted intervals, where the
    # least-squares fit is ill-conditioned: the library solves it in 113-bit
    # arithmetic, the oracle in 256-bit, and single entries then agree to
    # about 1e-10 of the largest one (d = 2) while the fits themselves match
    # to 1e-16.
    assert np.abs(Q.T @ Q - np.eye(d)).max() < 1e-13
    B = A @ Q.T
    scale = np.abs(ref["B"]).max()
    assert np.abs(B - ref["B"]).max() < 1e-9 * scale


@pytest.mark.parametrize("n,d,kind", [(12, 2, "d1"), (37, 5, "d1"), (101, 2, "d1"), (101, 5, "d2"),
                                      (64, 2, "filter"), (150, 5, "d1"), (48, 2, "smear"), (230, 2, "smear")])
def test_fc_operator_matches_oracle(n, d, kind):
    from oracle import fcgram
    import paper_2506_19370_amd as F
    got = F.fc_operator(n, d, 27, kind)
    ref = fcgram.dense_operator(n, d, 27, kind)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() < 1e-11 * scale


def test_fc_operator_rejects_bad_arguments():
    from paper_2506_19370_amd import _lib as L
    out = np.zeros(16)
    assert L.fcs_fc_operator(4, 0, 27, 0, out.ctypes.data) == L.FCS_EINVAL
    assert L.fcs_fc_operator(4, 2, 200, 0, out.ctypes.data) == L.FCS_EINVAL
    assert L.fcs_fc_operator(4, 2, 27, 0, None) == L.FCS_EINVAL


def _create(specs, **kw):
    from paper_2506_19370_amd.api import SolverParams, create_context
    return create_context(specs, SolverParams(**kw))


def test_create_step_channel_and_workspace_size():
    from paper_2506_19370_amd import _lib as L
    specs = W.step_channel()
    h = _create(specs, fc_d=2, fc_C=27, av="modal", filter=True)
    try:
        nbytes = ctypes.c_size_t()
        assert L.fcs_workspace_size(h, ctypes.byref(nbytes)) == L.FCS_OK
        npts = sum(s.npoints() for s in specs)
        # at least the three state copies, fluxes and derivatives in FP64
        assert nbytes.value > (3 * 4 + 3 * 8) * 8 * npts
    finally:
        L.fcs_destroy(h)


def test_create_reports_missing_donors():
    from paper_2506_19370_amd import _lib as L
    specs = [s for s in W.step_channel() if s.kind != "C1"]
    with pytest.raises(L.FcsError) as e:
        _create(specs, fc_d=2, fc_C=27)
    assert e.value.status == L.FCS_EOVERLAP


def test_create_rejects_smearing_without_classifier():
    from paper_2506_19370_amd import _lib as L
    specs = W.sod_reflect(200)
    with pytest.raises(L.FcsError) as e:
        _create(specs, fc_d=2, fc_C=27, smear=True)
    assert e.value.status == L.FCS_EINVAL
    h = _create(specs, fc_d=2, fc_C=27, smear=True, av="modal")
    L.fcs_destroy(h)


def test_create_rejects_invalid_parameters():
    from paper_2506_19370_amd import _lib as L
    specs = W.vortex_box(41)
    for bad in ({"fc_d": 0}, {"cfl": -1.0}, {"n_f": 0}):
        with pytest.raises(L.FcsError) as e:
            _create(specs, **bad)
        assert e.value.status == L.FCS_EINVAL


def test_create_rejects_empty_and_out_of_range_patch_sets():
    from paper_2506_19370_amd import _lib as L
    from paper_2506_19370_amd.api import SolverParams
    # no subpatch at all
    with pytest.raises(L.FcsError) as e:
        _create([], fc_d=2, fc_C=27)
    assert e.value.status == L.FCS_EINVAL
    # sides below 2 d points or above 1024 points
    for n1, n2 in ((3, 40), (40, 3), (1025, 12)):
        spec = W.box_patch(0.0, 1.0, 0.0, 1.0, n1, n2, {k: W.SLIP for k in "WESN"})
        with pytest.raises(L.FcsError) as e:
            _create([spec], fc_d=2, fc_C=27)
        assert e.value.status == L.FCS_EINVAL


def test_sweep_create_validates_sizes():
    from paper_2506_19370_amd import _lib as L
    import ctypes
    h = ctypes.c_void_p()
    for sizes, d in (([], 5), ([(9, 40)], 5), ([(40, 1025)], 5), ([(40, 40)], 0)):
        sz = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32).reshape(-1, 2))
        st = L.fcs_sweep_create(len(sz), sz.ctypes.data if len(sz) else None, 4, 0, d, 27, ctypes.byref(h))
        assert st == L.FCS_EINVAL, (sizes, d, st)
    sz = np.array([[10, 1024]], dtype=np.int32)  # the smallest and largest sides for d = 5
    assert L.fcs_sweep_create(1, sz.ctypes.data, 4, 0, 5, 27, ctypes.byref(h)) == L.FCS_OK
    L.fcs_sweep_destroy(h)


def test_tuning_and_profile_controls_need_a_bound_context():
    """fcs_retune, fcs_set_stage_variant and fcs_profile_stage act on a bound
    context; before fcs_bind they report FCS_ESTATE, and bad arguments
    FCS_EINVAL, without touching the device."""
    from paper_2506_19370_amd import _lib as L
    h = _create(W.step_channel(), fc_d=2, fc_C=27, av="modal", filter=True)
    try:
        ms = ctypes.c_double()
        assert L.fcs_retune(h) == L.FCS_ESTATE
        assert L.fcs_set_stage_variant(h, 0) == L.FCS_ESTATE
        assert L.fcs_profile_stage(h, 5, ctypes.byref(ms), None, None) == L.FCS_ESTATE
        assert L.fcs_profile_stage(h, 0, ctypes.byref(ms), None, None) == L.FCS_EINVAL
        assert L.fcs_profile_stage(h, 5, None, None, None) == L.FCS_EINVAL
    finally:
        L.fcs_destroy(h)
    assert L.fcs_retune(None) == L.FCS_EINVAL
    assert L.fcs_set_stage_variant(None, 0) == L.FCS_EINVAL
