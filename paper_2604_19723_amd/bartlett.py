"""Python binding of libbartlett.so: the C-ABI calls under the same names.

Argument marshalling only. Device buffers are torch tensors on the HIP device
(their data pointers go through ctypes); host arrays are numpy. Every step of
the computation runs in the library's HIP kernels. Sizes, dtypes and
contiguity of the buffers are checked here against what the call will touch,
so a wrong buffer raises instead of reaching a kernel. If the library is not
built, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbartlett.so")

BA_OK = 0
BA_ERR_ARG = -1
BA_ERR_DEVICE = -2
BA_ERR_NOMEM = -3
BA_ERR_UNSUPPORTED = -4
BA_ERR_STATE = -5

BA_PREC_F32 = 1
BA_PREC_BF16X3 = 2
BA_PREC_BF16 = 3
BA_PREC_F32_VALU = 4

BA_GRID_DIRS = 0
BA_GRID_ULA_DEG = 1
BA_GRID_AZEL_DEG = 2


class BartlettError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__("%s failed: status %d (%s): %s" % (fn, status, _status_text(status), msg))
        self.status = status


_lib = None

_vp = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_sz = C.c_size_t
_dp = C.POINTER(C.c_double)



class MsgInputs(C.Structure):
    """Host layout of ba_msg_inputs (device pointers)."""
    _fields_ = [("n_feat", _i32), ("n_part", _i32), ("z", _vp), ("mt_pos", _vp), ("w_beta", _vp), ("sfv", _vp),
                ("gamma", _vp), ("mu", _vp), ("w_alpha", _vp), ("zeta", _vp), ("eta", _vp), ("w_xi", _vp)]


class MsgOutputs(C.Structure):
    """Host layout of ba_msg_outputs (device pointers, NULL to skip)."""
    _fields_ = [("log_iota", _vp), ("log_nu", _vp), ("log_kappa", _vp), ("log_kappa0", _vp), ("log_omega", _vp)]


# name -> (restype, argtypes)
_SIGS = {
    "ba_status_string": (C.c_char_p, [_i32]),
    "ba_last_error": (C.c_char_p, []),
    "ba_version": (C.c_char_p, []),
    "ba_plan_create": (_i32, [C.POINTER(_vp), _i32, _dp, _i32, _i64, _dp, _i32, _i32, _i32, _i32]),
    "ba_plan_destroy": (_i32, [_vp]),
    "ba_plan_info": (_i32, [_vp, C.POINTER(_i32), C.POINTER(_i64), C.POINTER(_i32)]),
    "ba_workspace_size": (_i32, [_vp, _i32, _i32, _i32, C.POINTER(_sz)]),
    "ba_covariance": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "ba_spectrum_workspace_size": (_i32, [_vp, _i32, C.POINTER(_sz)]),
    "ba_spectrum": (_i32, [_vp, _i32, _vp, _vp, _vp, _sz, _vp]),
    "ba_spectrum_snapshots": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "ba_peaks": (_i32, [_vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp]),
    "ba_candidates_size": (_i32, [_vp, _i32, _i32, C.POINTER(_sz)]),
    "ba_spectrum_candidates": (_i32, [_vp, _i32, _vp, _i32, _vp, _vp, _sz, _vp]),
    "ba_peaks_merge": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "ba_proposal_moments": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "ba_run": (_i32, [_vp, _i32, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "ba_run_noalloc": (_i32, [_vp, _i32, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "ba_ragged_create": (_i32, [C.POINTER(_vp), _vp, _i32, _vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp]),
    "ba_ragged_launch": (_i32, [_vp, _vp]),
    "ba_ragged_bind": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "ba_ragged_autotune": (_i32, [_vp, C.c_char_p, _i32, _i32]),
    "ba_ragged_routes": (_i32, [_vp, _vp]),
    "ba_ragged_config": (_i32, [_vp, _vp]),
    "ba_ragged_packed": (_i32, [_vp, _vp]),
    "ba_ragged_destroy": (_i32, [_vp]),
    "ba_pack_covariance": (_i32, [_i32, _i32, _vp, _vp, _vp]),
    "ba_mlp_create": (_i32, [C.POINTER(_vp), _i32, _i32, _i32, _i32, _i32, _i32, C.c_uint64]),
    "ba_mlp_destroy": (_i32, [_vp]),
    "ba_mlp_num_params": (_i32, [_vp, C.POINTER(_i64)]),
    "ba_mlp_get_weights": (_i32, [_vp, _vp, _i64]),
    "ba_mlp_set_weights": (_i32, [_vp, _vp, _i64]),
    "ba_mlp_forward": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "ba_mlp_gradients": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ba_mlp_train_step": (_i32, [_vp, _i32, _vp, _vp, _vp, C.c_float, _vp, _vp]),
    "ba_mlp_dims": (_i32, [_vp, C.POINTER(_i32), C.POINTER(_i32)]),
    "ba_propose_workspace_size": (_i32, [_vp, _i32, _i32, _i32, C.POINTER(_sz)]),
    "ba_propose_refine": (_i32, [_vp, _vp, _i32, _vp, _i32, _i32, C.c_float, _vp, _vp, _vp, _vp,
                                 _vp, _vp, _sz, _vp]),
    "ba_proposal_sample": (_i32, [_vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp]),
    "ba_coherent_create": (_i32, [C.POINTER(_vp), _i32, _vp, _vp, _i32, _i32, _i32, C.c_double, C.c_double,
                                  _vp, C.c_int64, _vp]),
    "ba_coherent_destroy": (_i32, [_vp]),
    "ba_coherent_info": (_i32, [_vp, C.POINTER(_i32), C.POINTER(C.c_int64)]),
    "ba_coherent_workspace_size": (_i32, [_vp, _i32, C.POINTER(_sz)]),
    "ba_coherent_spectrum": (_i32, [_vp, _i32, _vp, _vp, _vp, _sz, _vp]),
    "ba_coherent_moments": (_i32, [_vp, _i32, _vp, _vp, _vp, _sz, _vp]),
    "ba_coherent_sample": (_i32, [_vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp]),
    "ba_residual_covariance": (_i32, [_vp, _i32, _vp, _i32, _vp, _vp, _vp]),
    "ba_sequential_workspace_size": (_i32, [_vp, _i32, C.POINTER(_sz)]),
    "ba_sequential_peaks": (_i32, [_vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "ba_msgs_create": (_i32, [C.POINTER(_vp), _i32, _vp, _vp, _i32, _i32, _i32, C.c_double, C.c_double]),
    "ba_msgs_destroy": (_i32, [_vp]),
    "ba_msgs_workspace_size": (_i32, [_vp, _i32, _i32, C.POINTER(_sz)]),
    "ba_update_messages": (_i32, [_vp, C.POINTER(MsgInputs), C.POINTER(MsgOutputs), _vp, _sz, _vp]),
}

BA_ROUTE_AUTO = -1
BA_ROUTE_COV = 0
BA_ROUTE_SNAPSHOTS = 1

# host layout of ba_trial
TRIAL_DTYPE = np.dtype([("y_offset", np.int64), ("n_elem", np.int32), ("n_snap", np.int32),
                        ("k", np.int32), ("route", np.int32)])


def lib():
    """Load the library (once). Raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libbartlett.so is not built (%s); run "
                               "`python -m paper_2604_19723_amd.build`" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _status_text(s):
    try:
        return lib().ba_status_string(s).decode()
    except Exception:
        return "?"


def _check(fn, status):
    if status != BA_OK:
        raise BartlettError(fn, status, lib().ba_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


_TORCH_DT = {"c64": ("complex64", 8), "c128": ("complex128", 16), "f32": ("float32", 4), "f64": ("float64", 8),
             "i32": ("int32", 4), "u8": ("uint8", 1), "bf16": ("bfloat16", 2)}


def _dev(t, kind, numel, name, optional=False):
    """Device pointer of a torch tensor after checking dtype, device, contiguity
    and that it holds at least ``numel`` elements."""
    if t is None:
        if optional:
            return None
        raise ValueError("%s is required" % name)
    dt, _ = _TORCH_DT[kind]
    if str(t.dtype).replace("torch.", "") != dt:
        raise TypeError("%s must be %s, got %s" % (name, dt, t.dtype))
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < numel:
        raise ValueError("%s holds %d elements, the call needs %d" % (name, t.numel(), numel))
    return C.c_void_p(t.data_ptr())


def _host_f64(a, shape_numel, name):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.size != shape_numel:
        raise ValueError("%s must have %d values, got %d" % (name, shape_numel, a.size))
    return a


# --------------------------------------------------------------------------- plan

class Plan:
    """Owns a ba_plan handle; holds the facts the binding needs to size buffers."""

    def __init__(self, handle, M, G, ndim, shape, wrap0, grid_kind, precision):
        self.handle = handle
        self.M, self.G, self.ndim = M, G, ndim
        self.shape, self.wrap0, self.grid_kind, self.precision = shape, wrap0, grid_kind, precision

    @property
    def coord_dim(self):
        return {BA_GRID_ULA_DEG: 1, BA_GRID_AZEL_DEG: 2, BA_GRID_DIRS: 3}[self.grid_kind]

    def close(self):
        if self.handle:
            ba_plan_destroy(self)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ba_version():
    return lib().ba_version().decode()


def ba_plan_create(n_elem, elem_pos_wl, grid_kind, n_grid, grid, grid_shape0, grid_shape1, wrap0,
                   precision=BA_PREC_F32) -> Plan:
    pos = _host_f64(elem_pos_wl, 3 * n_elem, "elem_pos_wl")
    per = {BA_GRID_ULA_DEG: 1, BA_GRID_AZEL_DEG: 2, BA_GRID_DIRS: 3}.get(grid_kind, 1)
    g = _host_f64(grid, per * n_grid, "grid")
    h = C.c_void_p()
    _check("ba_plan_create", lib().ba_plan_create(
        C.byref(h), n_elem, pos.ctypes.data_as(_dp), grid_kind, n_grid, g.ctypes.data_as(_dp),
        grid_shape0, grid_shape1, wrap0, precision))
    M, G, nd = _i32(), _i64(), _i32()
    _check("ba_plan_info", lib().ba_plan_info(h, C.byref(M), C.byref(G), C.byref(nd)))
    return Plan(h, M.value, G.value, nd.value, (grid_shape0, max(1, grid_shape1)), wrap0,
                grid_kind, precision)


def ba_plan_destroy(plan: Plan):
    _check("ba_plan_destroy", lib().ba_plan_destroy(plan.handle))


def ba_plan_info(plan: Plan):
    M, G, nd = _i32(), _i64(), _i32()
    _check("ba_plan_info", lib().ba_plan_info(plan.handle, C.byref(M), C.byref(G), C.byref(nd)))
    return M.value, G.value, nd.value


def ba_workspace_size(plan: Plan, n_trials, n_snap, with_spectrum_out=True) -> int:
    b = _sz()
    _check("ba_workspace_size", lib().ba_workspace_size(plan.handle, n_trials, n_snap,
                                                        int(bool(with_spectrum_out)), C.byref(b)))
    return b.value


# --------------------------------------------------------------------------- stages

def ba_covariance(plan: Plan, n_trials, n_snap, Y, R, stream=None):
    M = plan.M
    _check("ba_covariance", lib().ba_covariance(
        plan.handle, n_trials, n_snap, _dev(Y, "c64", n_trials * n_snap * M, "Y"),
        _dev(R, "c64", n_trials * M * M, "R"), _stream(stream)))


def ba_spectrum_workspace_size(plan: Plan, n_trials) -> int:
    b = _sz()
    _check("ba_spectrum_workspace_size",
           lib().ba_spectrum_workspace_size(plan.handle, n_trials, C.byref(b)))
    return b.value


def ba_spectrum(plan: Plan, n_trials, R, P, workspace=None, stream=None):
    M, G = plan.M, plan.G
    need = ba_spectrum_workspace_size(plan, n_trials)
    ws, nbytes = _workspace(workspace, need)
    _check("ba_spectrum", lib().ba_spectrum(
        plan.handle, n_trials, _dev(R, "c64", n_trials * M * M, "R"),
        _dev(P, "f32", n_trials * G, "P"), ws, nbytes, _stream(stream)))


def ba_spectrum_snapshots(plan: Plan, n_trials, n_snap, Y, P, stream=None):
    M, G = plan.M, plan.G
    _check("ba_spectrum_snapshots", lib().ba_spectrum_snapshots(
        plan.handle, n_trials, n_snap, _dev(Y, "c64", n_trials * n_snap * M, "Y"),
        _dev(P, "f32", n_trials * G, "P"), _stream(stream)))


def ba_peaks(plan: Plan, n_trials, P, k, idx, val, refined=None, stream=None):
    G, nd = plan.G, plan.ndim
    _check("ba_peaks", lib().ba_peaks(
        plan.handle, n_trials, _dev(P, "f32", n_trials * G, "P"), k,
        _dev(idx, "i32", n_trials * k, "idx"), _dev(val, "f32", n_trials * k, "val"),
        _dev(refined, "f64", n_trials * k * nd, "refined", optional=True), _stream(stream)))


def ba_candidates_size(plan: Plan, n_trials, k) -> int:
    """Bytes of the candidate records of ba_spectrum_candidates (raises
    BartlettError with BA_ERR_UNSUPPORTED for plans it does not serve)."""
    b = _sz()
    _check("ba_candidates_size", lib().ba_candidates_size(plan.handle, n_trials, k, C.byref(b)))
    return b.value


def ba_spectrum_candidates(plan: Plan, n_trials, R, k, P, cand, stream=None):
    """Spectrum (written only when P is not None) and per-range peak candidates."""
    M, G = plan.M, plan.G
    need = ba_candidates_size(plan, n_trials, k)
    ptr, nbytes = _workspace(cand, need)
    _check("ba_spectrum_candidates", lib().ba_spectrum_candidates(
        plan.handle, n_trials, _dev(R, "c64", n_trials * M * M, "R"), k,
        _dev(P, "f32", n_trials * G, "P", optional=True), ptr, nbytes, _stream(stream)))


def ba_peaks_merge(plan: Plan, n_trials, k, cand, idx, val, refined=None, stream=None):
    """Peaks of each trial from the records of ba_spectrum_candidates (same n_trials and k)."""
    nd = plan.ndim
    ptr, _ = _workspace(cand, ba_candidates_size(plan, n_trials, k))
    _check("ba_peaks_merge", lib().ba_peaks_merge(
        plan.handle, n_trials, k, ptr, _dev(idx, "i32", n_trials * k, "idx"),
        _dev(val, "f32", n_trials * k, "val"),
        _dev(refined, "f64", n_trials * k * nd, "refined", optional=True), _stream(stream)))


def candidates_for(plan: Plan, n_trials, k, device="cuda"):
    """A device buffer for the candidate records of n_trials trials and k peaks."""
    import torch
    n = ba_candidates_size(plan, n_trials, k)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device)


def ba_proposal_moments(plan: Plan, n_trials, P, mu_cov, stream=None):
    d = plan.coord_dim
    _check("ba_proposal_moments", lib().ba_proposal_moments(
        plan.handle, n_trials, _dev(P, "f32", n_trials * plan.G, "P"),
        _dev(mu_cov, "f64", n_trials * (d + d * d), "mu_cov"), _stream(stream)))


def ba_proposal_sample(plan: Plan, n_trials, mu_cov, n_particles, z, particles, weights, stream=None):
    """Particles mu + L z and normalised importance weights per trial."""
    d = plan.coord_dim
    _check("ba_proposal_sample", lib().ba_proposal_sample(
        plan.handle, n_trials, _dev(mu_cov, "f64", n_trials * (d + d * d), "mu_cov"), n_particles,
        _dev(z, "f64", n_trials * n_particles * d, "z"),
        _dev(particles, "f64", n_trials * n_particles * d, "particles"),
        _dev(weights, "f64", n_trials * n_particles, "weights"), _stream(stream)))


def _workspace(workspace, need):
    """(pointer, bytes) of a workspace tensor after checking it holds ``need`` bytes."""
    if workspace is None:
        if need:
            raise ValueError("workspace of %d bytes required" % need)
        return None, 0
    if not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    nbytes = workspace.numel() * workspace.element_size()
    if nbytes < need:
        raise ValueError("workspace needs %d bytes, got %d" % (need, nbytes))
    return C.c_void_p(workspace.data_ptr()), nbytes


def ba_run(plan: Plan, n_trials, n_snap, Y, k, P, idx, val, refined, workspace, stream=None):
    M, G, nd = plan.M, plan.G, plan.ndim
    need = ba_workspace_size(plan, n_trials, n_snap, P is not None)
    if workspace is None or workspace.numel() * workspace.element_size() < need:
        raise ValueError("workspace needs %d bytes" % need)
    if not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    _check("ba_run", lib().ba_run(
        plan.handle, n_trials, n_snap, _dev(Y, "c64", n_trials * n_snap * M, "Y"), k,
        _dev(P, "f32", n_trials * G, "P", optional=True), _dev(idx, "i32", n_trials * k, "idx"),
        _dev(val, "f32", n_trials * k, "val"),
        _dev(refined, "f64", n_trials * k * nd, "refined", optional=True),
        C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
        _stream(stream)))


def ba_run_noalloc(plan: Plan, n_trials, n_snap, Y, k, P, idx, val, refined, stream=None):
    """ba_run with the library's fixed scratch array as the workspace."""
    M, G, nd = plan.M, plan.G, plan.ndim
    _check("ba_run_noalloc", lib().ba_run_noalloc(
        plan.handle, n_trials, n_snap, _dev(Y, "c64", n_trials * n_snap * M, "Y"), k,
        _dev(P, "f32", n_trials * G, "P", optional=True), _dev(idx, "i32", n_trials * k, "idx"),
        _dev(val, "f32", n_trials * k, "val"),
        _dev(refined, "f64", n_trials * k * nd, "refined", optional=True),
        _stream(stream)))


# --------------------------------------------------------------------------- convenience

def plan_for(trialset, precision=BA_PREC_F32) -> Plan:
    """Plan for a workload.TrialSet (geometry + grid + adjacency)."""
    ts = trialset
    return ba_plan_create(ts.pos_wl.shape[0], ts.pos_wl, ts.grid_kind, ts.n_grid, ts.grid,
                          ts.grid_shape[0], ts.grid_shape[1], ts.wrap0, precision)


def workspace_for(plan: Plan, n_trials, n_snap, with_spectrum_out=True, device="cuda"):
    import torch
    n = ba_workspace_size(plan, n_trials, n_snap, with_spectrum_out)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device)


def spectrum_workspace_for(plan: Plan, n_trials, device="cuda"):
    import torch
    n = ba_spectrum_workspace_size(plan, n_trials)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device) if n else None


def run_grid_search(plan: Plan, Y, k, with_spectrum=True, stream=None):
    """Allocate outputs and run the whole path on a device tensor Y [B][T][M] c64.
    Returns a dict of device tensors."""
    import torch
    B, T, M = Y.shape
    dev = Y.device
    P = torch.empty((B, plan.G), dtype=torch.float32, device=dev) if with_spectrum else None
    idx = torch.empty((B, k), dtype=torch.int32, device=dev)
    val = torch.empty((B, k), dtype=torch.float32, device=dev)
    ref = torch.empty((B, k, plan.ndim), dtype=torch.float64, device=dev)
    ws = workspace_for(plan, B, T, with_spectrum, dev)
    ba_run(plan, B, T, Y, k, P, idx, val, ref, ws, stream)
    return dict(P=P, idx=idx, val=val, refined=ref)


# --------------------------------------------------------------------------- ragged batches

class Ragged:
    """Owns a ba_ragged handle and keeps the buffers it is bound to alive."""

    def __init__(self, handle, plan, n_trials, kmax, keep):
        self.handle, self.plan, self.n_trials, self.kmax = handle, plan, n_trials, kmax
        self._keep = keep

    def close(self):
        if self.handle:
            ba_ragged_destroy(self)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ba_ragged_create(plan: Plan, desc, kmax, Y_pool, P, idx, val, refined=None) -> Ragged:
    d = np.ascontiguousarray(np.asarray(desc, dtype=TRIAL_DTYPE))
    B = d.shape[0]
    h = C.c_void_p()
    _check("ba_ragged_create", lib().ba_ragged_create(
        C.byref(h), plan.handle, B, d.ctypes.data_as(_vp), kmax,
        _dev(Y_pool, "c64", 1, "Y_pool"), Y_pool.numel(),
        _dev(P, "f32", B * plan.G, "P", optional=True), _dev(idx, "i32", B * kmax, "idx"),
        _dev(val, "f32", B * kmax, "val"),
        _dev(refined, "f64", B * kmax * plan.ndim, "refined", optional=True)))
    return Ragged(h, plan, B, kmax, (plan, Y_pool, P, idx, val, refined))


def ba_ragged_bind(r: Ragged, Y_pool, P, idx, val, refined=None, stream=None):
    """Retarget the captured launch at other buffers (stream-ordered)."""
    B, G, kmax, nd = r.n_trials, r.plan.G, r.kmax, r.plan.ndim
    _check("ba_ragged_bind", lib().ba_ragged_bind(
        r.handle, _dev(Y_pool, "c64", 1, "Y_pool"), Y_pool.numel(),
        _dev(P, "f32", B * G, "P", optional=True), _dev(idx, "i32", B * kmax, "idx"),
        _dev(val, "f32", B * kmax, "val"), _dev(refined, "f64", B * kmax * nd, "refined", optional=True),
        _stream(stream)))
    r._keep = (r._keep, (Y_pool, P, idx, val, refined))   # earlier buffers may still be in use


def ba_ragged_launch(r: Ragged, stream=None):
    _check("ba_ragged_launch", lib().ba_ragged_launch(r.handle, _stream(stream)))


def ba_ragged_autotune(r: Ragged, cache_path=None, repeats=2, max_probe=512):
    _check("ba_ragged_autotune", lib().ba_ragged_autotune(
        r.handle, cache_path.encode() if cache_path else None, repeats, max_probe))


def ba_ragged_routes(r: Ragged):
    out = np.empty(r.n_trials, np.int32)
    _check("ba_ragged_routes", lib().ba_ragged_routes(r.handle, out.ctypes.data_as(_vp)))
    return out


def ba_ragged_config(r: Ragged):
    out = np.empty(5, np.int32)
    _check("ba_ragged_config", lib().ba_ragged_config(r.handle, out.ctypes.data_as(_vp)))
    return out


def ba_ragged_packed(r: Ragged):
    """Per size class (8..128 elements), 1 where trials run packed, one per wave."""
    out = np.empty(5, np.int32)
    _check("ba_ragged_packed", lib().ba_ragged_packed(r.handle, out.ctypes.data_as(_vp)))
    return out


def ba_ragged_destroy(r: Ragged):
    _check("ba_ragged_destroy", lib().ba_ragged_destroy(r.handle))


def ragged_descriptors(rs, route=BA_ROUTE_AUTO):
    """ba_trial records for a workload.RaggedSet."""
    d = np.zeros(rs.n_trials, TRIAL_DTYPE)
    d["y_offset"] = rs.y_offset
    d["n_elem"] = rs.n_elem
    d["n_snap"] = rs.n_snap
    d["k"] = rs.k
    d["route"] = route
    return d


# --------------------------------------------------------------------------- proposal network

class Mlp:
    """Owns a ba_mlp handle."""

    def __init__(self, handle, dims, max_batch, precision):
        self.handle, self.dims, self.max_batch, self.precision = handle, dims, max_batch, precision
        n = _i64()
        _check("ba_mlp_num_params", lib().ba_mlp_num_params(handle, C.byref(n)))
        self.n_params = n.value

    def close(self):
        if self.handle:
            _check("ba_mlp_destroy", lib().ba_mlp_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ba_pack_covariance(n_elem, n_trials, R, X, stream=None):
    _check("ba_pack_covariance", lib().ba_pack_covariance(
        n_elem, n_trials, _dev(R, "c64", n_trials * n_elem * n_elem, "R"),
        _dev(X, "f32", n_trials * n_elem * n_elem, "X"), _stream(stream)))


def ba_mlp_create(d_in, d_hidden, n_hidden, d_out, max_batch, precision=BA_PREC_BF16, seed=0) -> Mlp:
    h = C.c_void_p()
    _check("ba_mlp_create", lib().ba_mlp_create(C.byref(h), d_in, d_hidden, n_hidden, d_out, max_batch,
                                                precision, seed))
    return Mlp(h, [d_in] + [d_hidden] * n_hidden + [d_out], max_batch, precision)


def ba_mlp_get_weights(net: Mlp) -> np.ndarray:
    w = np.empty(net.n_params, np.float32)
    _check("ba_mlp_get_weights", lib().ba_mlp_get_weights(net.handle, w.ctypes.data_as(_vp), net.n_params))
    return w


def ba_mlp_set_weights(net: Mlp, w):
    w = np.ascontiguousarray(np.asarray(w, np.float32))
    if w.size != net.n_params:
        raise ValueError("need %d parameters" % net.n_params)
    _check("ba_mlp_set_weights", lib().ba_mlp_set_weights(net.handle, w.ctypes.data_as(_vp), net.n_params))


def ba_mlp_forward(net: Mlp, B, X, Y, stream=None):
    _check("ba_mlp_forward", lib().ba_mlp_forward(
        net.handle, B, _dev(X, "f32", B * net.dims[0], "X"), _dev(Y, "f32", B * net.dims[-1], "Y"),
        _stream(stream)))


def ba_mlp_gradients(net: Mlp, B, X, T, mask, grads, loss=None, stream=None):
    _check("ba_mlp_gradients", lib().ba_mlp_gradients(
        net.handle, B, _dev(X, "f32", B * net.dims[0], "X"), _dev(T, "f32", B * net.dims[-1], "T"),
        _dev(mask, "f32", B * net.dims[-1], "mask", optional=True),
        _dev(grads, "f32", net.n_params, "grads"), _dev(loss, "f32", 1, "loss", optional=True),
        _stream(stream)))


def ba_mlp_train_step(net: Mlp, B, X, T, mask, lr, loss=None, stream=None):
    _check("ba_mlp_train_step", lib().ba_mlp_train_step(
        net.handle, B, _dev(X, "f32", B * net.dims[0], "X"), _dev(T, "f32", B * net.dims[-1], "T"),
        _dev(mask, "f32", B * net.dims[-1], "mask", optional=True), float(lr),
        _dev(loss, "f32", 1, "loss", optional=True), _stream(stream)))


def mlp_params_to_list(w, dims):
    """Flat parameter vector -> [(W [out][in], b [out])] (the oracle's layout)."""
    out, o = [], 0
    for i in range(len(dims) - 1):
        n_w = dims[i + 1] * dims[i]
        W = np.asarray(w[o:o + n_w]).reshape(dims[i + 1], dims[i])
        o += n_w
        b = np.asarray(w[o:o + dims[i + 1]])
        o += dims[i + 1]
        out.append((W, b))
    return out


def mlp_list_to_params(params):
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in params])


def ba_mlp_dims(net: Mlp):
    a, b = _i32(), _i32()
    _check("ba_mlp_dims", lib().ba_mlp_dims(net.handle, C.byref(a), C.byref(b)))
    return a.value, b.value


def ba_propose_workspace_size(plan: Plan, n_trials, d_out, k) -> int:
    b = _sz()
    _check("ba_propose_workspace_size", lib().ba_propose_workspace_size(plan.handle, n_trials, d_out, k,
                                                                        C.byref(b)))
    return b.value


def ba_propose_refine(plan: Plan, net: Mlp, n_trials, R, k, half_window, tau, idx, val, refined,
                      fell_back, workspace, stream=None, n_fallback=None):
    """Enqueues the learned-proposal refinement; nothing waits for the device.
    n_fallback: optional device int32 tensor that receives the number of
    trials that fell back to the full grid."""
    M = plan.M
    need = ba_propose_workspace_size(plan, n_trials, net.dims[-1], k)
    ws, nbytes = _workspace(workspace, need)
    _check("ba_propose_refine", lib().ba_propose_refine(
        plan.handle, net.handle, n_trials, _dev(R, "c64", n_trials * M * M, "R"), k, half_window,
        float(tau), _dev(idx, "i32", n_trials * k, "idx"), _dev(val, "f32", n_trials * k, "val"),
        _dev(refined, "f64", n_trials * k, "refined"), _dev(fell_back, "u8", n_trials, "fell_back"),
        _dev(n_fallback, "i32", 1, "n_fallback", optional=True), ws, nbytes, _stream(stream)))


# --------------------------------------------------------------------------- residual projector

def ba_residual_covariance(plan: Plan, n_trials, R, S, Psi, R_out, stream=None):
    """R~ = Pi R Pi, Pi = I - Psi Psi^+; Psi is c64 [B][S][M] (None when S = 0)."""
    M = plan.M
    _check("ba_residual_covariance", lib().ba_residual_covariance(
        plan.handle, n_trials, _dev(R, "c64", n_trials * M * M, "R"), S,
        _dev(Psi, "c64", n_trials * S * M, "Psi", optional=S == 0),
        _dev(R_out, "c64", n_trials * M * M, "R_out"), _stream(stream)))


def ba_sequential_workspace_size(plan: Plan, n_trials) -> int:
    b = _sz()
    _check("ba_sequential_workspace_size", lib().ba_sequential_workspace_size(plan.handle, n_trials, C.byref(b)))
    return b.value


def ba_sequential_peaks(plan: Plan, n_trials, R, k, idx, val, refined=None, workspace=None, stream=None):
    """Project-out-and-rescan detection: k passes, outputs in detection order."""
    M, nd = plan.M, plan.ndim
    ws, nbytes = _workspace(workspace, ba_sequential_workspace_size(plan, n_trials))
    _check("ba_sequential_peaks", lib().ba_sequential_peaks(
        plan.handle, n_trials, _dev(R, "c64", n_trials * M * M, "R"), k,
        _dev(idx, "i32", n_trials * k, "idx"), _dev(val, "f32", n_trials * k, "val"),
        _dev(refined, "f64", n_trials * k * nd, "refined", optional=True), ws, nbytes, _stream(stream)))


def sequential_workspace_for(plan: Plan, n_trials, device):
    import torch
    return torch.empty(max(ba_sequential_workspace_size(plan, n_trials), 1), dtype=torch.uint8, device=device)


# --------------------------------------------------------------------------- coherent multi-array cost

class Coherent:
    """Owns a ba_coherent handle (geometry + device steering table)."""

    def __init__(self, handle, n_obs, n_cand):
        self.handle, self.n_obs, self.n_cand = handle, n_obs, n_cand

    def close(self):
        if self.handle:
            ba_coherent_destroy(self)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ba_coherent_create(pa_pos, pa_rot, n_y, n_z, n_f, fc, bandwidth, p_mt, candidates) -> Coherent:
    pa = np.ascontiguousarray(np.asarray(pa_pos, np.float64).reshape(-1, 3))
    J = pa.shape[0]
    rot = _host_f64(pa_rot, 9 * J, "pa_rot")
    mt = _host_f64(p_mt, 3, "p_mt")
    cand = np.ascontiguousarray(np.asarray(candidates, np.float64).reshape(-1, 3))
    h = C.c_void_p()
    _check("ba_coherent_create", lib().ba_coherent_create(
        C.byref(h), J, pa.ctypes.data_as(_vp), rot.ctypes.data_as(_vp), n_y, n_z, n_f, float(fc),
        float(bandwidth), mt.ctypes.data_as(_vp), cand.shape[0], cand.ctypes.data_as(_vp)))
    n_obs, n_cand = _i32(), C.c_int64()
    _check("ba_coherent_info", lib().ba_coherent_info(h, C.byref(n_obs), C.byref(n_cand)))
    return Coherent(h, n_obs.value, n_cand.value)


def ba_coherent_destroy(h: Coherent):
    _check("ba_coherent_destroy", lib().ba_coherent_destroy(h.handle))


def ba_coherent_workspace_size(h: Coherent, n_trials) -> int:
    b = _sz()
    _check("ba_coherent_workspace_size", lib().ba_coherent_workspace_size(h.handle, n_trials, C.byref(b)))
    return b.value


def ba_coherent_spectrum(h: Coherent, n_trials, Z, P, workspace, stream=None):
    ws, nbytes = _workspace(workspace, ba_coherent_workspace_size(h, n_trials))
    _check("ba_coherent_spectrum", lib().ba_coherent_spectrum(
        h.handle, n_trials, _dev(Z, "c64", n_trials * h.n_obs, "Z"), _dev(P, "f32", n_trials * h.n_cand, "P"),
        ws, nbytes, _stream(stream)))


def ba_coherent_moments(h: Coherent, n_trials, P, mu_cov, workspace, stream=None):
    ws, nbytes = _workspace(workspace, ba_coherent_workspace_size(h, n_trials))
    _check("ba_coherent_moments", lib().ba_coherent_moments(
        h.handle, n_trials, _dev(P, "f32", n_trials * h.n_cand, "P"), _dev(mu_cov, "f64", n_trials * 12, "mu_cov"),
        ws, nbytes, _stream(stream)))


def ba_coherent_sample(h: Coherent, n_trials, mu_cov, n_particles, z, particles, weights, stream=None):
    """Birth particles in the candidates' bounding box from N(mu, C)."""
    N = n_particles
    _check("ba_coherent_sample", lib().ba_coherent_sample(
        h.handle, n_trials, _dev(mu_cov, "f64", n_trials * 12, "mu_cov"), N,
        _dev(z, "f64", n_trials * N * 3, "z"), _dev(particles, "f64", n_trials * N * 3, "particles"),
        _dev(weights, "f64", n_trials * N, "weights"), _stream(stream)))


def coherent_workspace_for(h: Coherent, n_trials, device="cuda"):
    import torch
    return torch.empty(max(ba_coherent_workspace_size(h, n_trials), 256), dtype=torch.uint8, device=device)


# --------------------------------------------------------------------------- particle update messages

class Messages:
    """Owns a ba_msgs handle (array geometry on the device)."""

    def __init__(self, handle, n_arrays, n_obs):
        self.handle, self.J, self.n_obs = handle, n_arrays, n_obs

    def close(self):
        if self.handle:
            ba_msgs_destroy(self)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ba_msgs_create(pa_pos, pa_rot, n_y, n_z, n_f, fc, bandwidth) -> Messages:
    pa = np.ascontiguousarray(np.asarray(pa_pos, np.float64).reshape(-1, 3))
    J = pa.shape[0]
    rot = _host_f64(pa_rot, 9 * J, "pa_rot")
    h = C.c_void_p()
    _check("ba_msgs_create", lib().ba_msgs_create(C.byref(h), J, pa.ctypes.data_as(_vp), rot.ctypes.data_as(_vp),
                                                  n_y, n_z, n_f, float(fc), float(bandwidth)))
    return Messages(h, J, n_f * n_y * n_z)


def ba_msgs_destroy(h: Messages):
    _check("ba_msgs_destroy", lib().ba_msgs_destroy(h.handle))


def ba_msgs_workspace_size(h: Messages, n_feat, n_part) -> int:
    b = _sz()
    _check("ba_msgs_workspace_size", lib().ba_msgs_workspace_size(h.handle, n_feat, n_part, C.byref(b)))
    return b.value


def messages_workspace_for(h: Messages, n_feat, n_part, device="cuda"):
    import torch
    return torch.empty(max(ba_msgs_workspace_size(h, n_feat, n_part), 256), dtype=torch.uint8, device=device)


def ba_update_messages(h: Messages, n_feat, n_part, z, mt_pos, w_beta, sfv, gamma, mu, w_alpha, zeta, eta, w_xi,
                       workspace, log_iota=None, log_nu=None, log_kappa=None, log_kappa0=None, log_omega=None,
                       stream=None):
    """All tensors on the device: z complex128 [J][N_z], mt_pos [P][3], w_beta [P],
    sfv [S][P][3], gamma [S][P], mu complex128 [S][P], w_alpha [S][P], zeta [S][J],
    eta [J][P], w_xi [J][P] (float64); outputs float64 log_iota/log_nu [J][P],
    log_kappa [S][J][P], log_kappa0 [S][J], log_omega [S][J][2] (None skips)."""
    S, P, J = int(n_feat), int(n_part), h.J
    ws, nbytes = _workspace(workspace, ba_msgs_workspace_size(h, S, P))
    mi = MsgInputs(S, P, _dev(z, "c128", J * h.n_obs, "z"), _dev(mt_pos, "f64", 3 * P, "mt_pos"),
                   _dev(w_beta, "f64", P, "w_beta"), _dev(sfv, "f64", 3 * S * P, "sfv"),
                   _dev(gamma, "f64", S * P, "gamma"), _dev(mu, "c128", S * P, "mu"),
                   _dev(w_alpha, "f64", S * P, "w_alpha"), _dev(zeta, "f64", S * J, "zeta"),
                   _dev(eta, "f64", J * P, "eta"), _dev(w_xi, "f64", J * P, "w_xi"))
    mo = MsgOutputs(_dev(log_iota, "f64", J * P, "log_iota", True), _dev(log_nu, "f64", J * P, "log_nu", True),
                    _dev(log_kappa, "f64", S * J * P, "log_kappa", True),
                    _dev(log_kappa0, "f64", S * J, "log_kappa0", True),
                    _dev(log_omega, "f64", 2 * S * J, "log_omega", True))
    _check("ba_update_messages", lib().ba_update_messages(h.handle, C.byref(mi), C.byref(mo), ws, nbytes,
                                                          _stream(stream)))


def message_tensors(ms, device="cuda"):
    """The arrays of a workload.MessageSet as contiguous device tensors, keyed
    by the argument names of ba_update_messages."""
    import torch
    f64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(device)
    c128 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.complex128)).to(device)
    return dict(z=c128(ms.z), mt_pos=f64(ms.mt_pos), w_beta=f64(ms.w_beta), sfv=f64(ms.sfv), gamma=f64(ms.gamma),
                mu=c128(ms.mu), w_alpha=f64(ms.w_alpha), zeta=f64(ms.zeta), eta=f64(ms.eta), w_xi=f64(ms.w_xi))
