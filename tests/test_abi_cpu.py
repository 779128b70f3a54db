"""C-ABI checks that need no GPU: the library loads, exports every function
include/bartlett.h declares, the binding knows the same names, and argument
errors are returned before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2604_19723_amd import bartlett as bb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for f in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:ba_status|const char\s*\*)\s*(ba_\w+)\s*\(", src, flags=re.M)
    return names


def test_header_declares_the_path():
    names = declared_functions()
    for n in ("ba_plan_create", "ba_covariance", "ba_spectrum", "ba_peaks", "ba_run"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = C.CDLL(bb.LIB_PATH)
    for n in declared_functions():
        assert hasattr(L, n), n
    assert sorted(declared_functions()) == sorted(bb.exported_symbols())


def test_status_strings_and_version():
    L = bb.lib()
    assert L.ba_status_string(0) == b"ok"
    assert L.ba_status_string(-1) == b"invalid argument"
    assert b"gfx950" in L.ba_version()


def _create(M=4, kind=bb.BA_GRID_ULA_DEG, G=10, grid=None, s0=None, s1=1, wrap=0, prec=1,
            pos=None):
    L = bb.lib()
    h = C.c_void_p()
    pos = np.zeros((M, 3)) if pos is None else pos
    per = {0: 3, 1: 1, 2: 2}.get(kind, 1)
    grid = np.zeros(max(G, 1) * per) if grid is None else grid
    dp = C.POINTER(C.c_double)
    st = L.ba_plan_create(C.byref(h), M, pos.ctypes.data_as(dp), kind, G, grid.ctypes.data_as(dp),
                          G if s0 is None else s0, s1, wrap, prec)
    return st, h


@pytest.mark.parametrize("kw,msg", [
    (dict(M=0), "n_elem"), (dict(M=257), "n_elem"), (dict(kind=7), "grid_kind"),
    (dict(G=0), "n_grid"), (dict(G=10, s0=3, s1=3), "grid_shape"), (dict(wrap=3), "wrap0"),
    (dict(G=3, wrap=2), "period"), (dict(prec=9), "precision"),
    (dict(pos=np.full((4, 3), np.nan)), "non-finite"),
])
def test_plan_create_rejects_bad_arguments_before_device_work(kw, msg):
    st, h = _create(**kw)
    assert st == bb.BA_ERR_ARG and not h.value
    assert msg in bb.lib().ba_last_error().decode()


def test_null_plan_and_null_out():
    L = bb.lib()
    assert L.ba_plan_create(None, 4, None, 1, 4, None, 4, 1, 0, 1) == bb.BA_ERR_ARG
    sz = C.c_size_t()
    assert L.ba_workspace_size(None, 1, 1, 1, C.byref(sz)) == bb.BA_ERR_ARG
    assert L.ba_run(None, 1, 1, None, 1, None, None, None, None, None, 0, None) == bb.BA_ERR_ARG
    assert L.ba_peaks(None, 1, None, 1, None, None, None, None) == bb.BA_ERR_ARG
    assert L.ba_plan_destroy(None) == bb.BA_OK


def test_new_entry_points_reject_bad_arguments_before_device_work():
    L = bb.lib()
    sz = C.c_size_t()
    assert L.ba_residual_covariance(None, 1, None, 1, None, None, None) == bb.BA_ERR_ARG
    assert L.ba_sequential_workspace_size(None, 1, C.byref(sz)) == bb.BA_ERR_ARG
    assert L.ba_sequential_peaks(None, 1, None, 2, None, None, None, None, 0, None) == bb.BA_ERR_ARG
    assert L.ba_proposal_sample(None, 1, None, 4, None, None, None, None) == bb.BA_ERR_ARG
    h = C.c_void_p()
    pos = np.zeros((4, 3))
    rot = np.tile(np.eye(3), (4, 1, 1))
    mt = np.array([1.0, 2.0, 1.0])
    cand = np.array([[14.0, 0.0, 0.0]])
    vp = lambda a: a.ctypes.data_as(C.c_void_p)
    cases = [
        (0, 4, 4, 10, 3.5e9, 1e8, "n_arrays"),       # no arrays
        (4, 0, 4, 10, 3.5e9, 1e8, "n_y"),            # no elements
        (4, 4, 4, 0, 3.5e9, 1e8, "n_f"),             # no frequencies
        (4, 4, 4, 10, -1.0, 1e8, "fc"),              # negative carrier
        (16, 16, 16, 10, 3.5e9, 1e8, "<= 2048"),     # observation too long
    ]
    for J, ny, nz, nf, fc, bw, msg in cases:
        st = L.ba_coherent_create(C.byref(h), J, vp(pos), vp(rot), ny, nz, nf, C.c_double(fc), C.c_double(bw),
                                  vp(mt), 1, vp(cand))
        assert st == bb.BA_ERR_ARG and not h.value, (J, ny, nz, nf)
        assert msg in L.ba_last_error().decode()
    zero = np.zeros((1, 3))
    st = L.ba_coherent_create(C.byref(h), 4, vp(pos), vp(rot), 4, 4, 10, C.c_double(3.5e9), C.c_double(1e8),
                              vp(mt), 1, vp(zero))
    assert st == bb.BA_ERR_ARG and "nonzero" in L.ba_last_error().decode()
    assert L.ba_coherent_destroy(None) == bb.BA_ERR_ARG


def test_message_entry_points_reject_bad_arguments_before_device_work():
    L = bb.lib()
    sz = C.c_size_t()
    h = C.c_void_p()
    pos = np.zeros((4, 3))
    rot = np.tile(np.eye(3), (4, 1, 1))
    vp = lambda a: a.ctypes.data_as(C.c_void_p)
    cases = [
        (0, 4, 4, 10, 3.5e9, 1e8, "n_arrays"),
        (17, 4, 4, 10, 3.5e9, 1e8, "n_arrays"),
        (4, 4, 0, 10, 3.5e9, 1e8, "n_y"),
        (4, 4, 4, 65, 3.5e9, 1e8, "n_f"),
        (4, 16, 16, 8, 3.5e9, 1e8, "<= 1024"),
        (4, 4, 4, 10, 0.0, 1e8, "fc"),
        (4, 4, 4, 10, 3.5e9, -1.0, "bandwidth"),
    ]
    for J, ny, nz, nf, fc, bw, msg in cases:
        st = L.ba_msgs_create(C.byref(h), J, vp(pos), vp(rot), ny, nz, nf, C.c_double(fc), C.c_double(bw))
        assert st == bb.BA_ERR_ARG and not h.value, (J, ny, nz, nf, fc, bw)
        assert msg in L.ba_last_error().decode()
    assert L.ba_msgs_create(C.byref(h), 4, None, vp(rot), 4, 4, 10, C.c_double(3.5e9), C.c_double(1e8)) == \
        bb.BA_ERR_ARG
    assert L.ba_msgs_destroy(None) == bb.BA_ERR_ARG
    assert L.ba_msgs_workspace_size(None, 6, 100, C.byref(sz)) == bb.BA_ERR_ARG
    mi = bb.MsgInputs(6, 100)
    mo = bb.MsgOutputs()
    assert L.ba_update_messages(None, C.byref(mi), C.byref(mo), None, 0, None) == bb.BA_ERR_ARG


def test_candidate_and_packing_entry_points_reject_bad_arguments_before_device_work():
    L = bb.lib()
    sz = C.c_size_t()
    assert L.ba_candidates_size(None, 1, 4, C.byref(sz)) == bb.BA_ERR_ARG
    assert L.ba_last_error().decode().startswith("ba_candidates_size: plan is NULL")
    # the size check they share reports under the caller's name
    assert L.ba_spectrum_candidates(None, 1, None, 4, None, None, 0, None) == bb.BA_ERR_ARG
    assert L.ba_last_error().decode().startswith("ba_spectrum_candidates: plan is NULL")
    assert L.ba_peaks_merge(None, 1, 4, None, None, None, None, None) == bb.BA_ERR_ARG
    assert L.ba_last_error().decode().startswith("ba_peaks_merge: plan is NULL")
    out = np.zeros(5, np.int32)
    assert L.ba_ragged_packed(None, out.ctypes.data_as(C.c_void_p)) == bb.BA_ERR_ARG
