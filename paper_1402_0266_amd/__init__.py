"""MI355X stochastic domain-decomposition interface solver (Python binding).

A thin ctypes binding of ``libfk.so`` (C ABI declared in ``include/fk.h``):
the functions here only marshal arguments -- every step of the solve runs in
the library's HIP kernels.  PyTorch supplies device memory and the stream.

The library must be built first (``python paper_1402_0266_amd/build.py`` or
``__graft_entry__.build()``); importing this package without it raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfk.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "fk.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_1402_0266_amd/build.py")

# torch ships its own HIP runtime (soname libamdhip64.so.7).  Loading torch
# first makes libfk.so bind to that same runtime instead of a second copy
# from /opt/rocm, so both see the same device, memory and streams.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

FK_OK = 0
FK_E_INVAL = -1
FK_E_NODEVICE = -2
FK_E_NOMEM = -3
FK_E_DEVICE = -4
FK_E_UNSUPPORTED = -5


class FkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fk error {code}: {msg}")
        self.code = code


class fk_density(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("time_mode", ctypes.c_int32),
                ("amp", ctypes.c_double), ("width2", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("orbit_r", ctypes.c_double), ("omega", ctypes.c_double),
                ("t_freeze", ctypes.c_double), ("grid_n", ctypes.c_int32), ("grid_reserved", ctypes.c_int32),
                ("grid_w", ctypes.c_void_p), ("grid_b", ctypes.c_void_p)]


class fk_data(ctypes.Structure):
    _fields_ = [("init_kind", ctypes.c_int32), ("bdry_kind", ctypes.c_int32),
                ("score_mode", ctypes.c_int32), ("grid_n", ctypes.c_int32),
                ("t_init", ctypes.c_double), ("grid_xi", ctypes.c_void_p), ("grid_eta", ctypes.c_void_p)]


class fk_plan(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("node_tile", ctypes.c_int32)]


class fk_level(ctypes.Structure):
    _fields_ = [("w", fk_density), ("t", ctypes.c_double), ("t_init", ctypes.c_double),
                ("node_offset", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("level_id", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


_P = ctypes.c_void_p
_lib.fk_version.restype = ctypes.c_int
_lib.fk_last_error.restype = ctypes.c_char_p
_lib.fk_interface_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64]
_lib.fk_interface_workspace_bytes.restype = ctypes.c_size_t
_lib.fk_sync.argtypes = [_P]
_lib.fk_sync.restype = ctypes.c_int
_lib.fk_interface_solve.argtypes = [
    ctypes.POINTER(fk_density), ctypes.POINTER(fk_data), _P, _P, ctypes.c_int64,
    ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
    _P, _P, _P, _P, _P, _P, _P, _P,
    ctypes.POINTER(fk_plan), _P, ctypes.c_size_t, _P]
_lib.fk_interface_solve.restype = ctypes.c_int
_lib.fk_interface_noalloc_max_bytes.argtypes = []
_lib.fk_interface_noalloc_max_bytes.restype = ctypes.c_size_t
_lib.fk_interface_solve_noalloc.argtypes = [
    ctypes.POINTER(fk_density), ctypes.POINTER(fk_data), _P, _P, ctypes.c_int64,
    ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
    _P, _P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(fk_plan), _P]
_lib.fk_interface_solve_noalloc.restype = ctypes.c_int
_lib.fk_philox_words.argtypes = [_P, ctypes.c_int64, ctypes.c_uint64, _P, _P]
_lib.fk_philox_words.restype = ctypes.c_int
_lib.fk_normals.argtypes = [_P, _P, ctypes.c_int64, ctypes.c_double, _P, _P]
_lib.fk_normals.restype = ctypes.c_int
_lib.fk_batch_create.argtypes = [ctypes.POINTER(fk_level), ctypes.c_int32, _P, ctypes.c_int64,
                                 ctypes.POINTER(fk_data), ctypes.c_double, ctypes.c_int64, ctypes.c_uint64,
                                 ctypes.POINTER(_P)]
_lib.fk_batch_create.restype = ctypes.c_int
_lib.fk_batch_workspace_bytes.argtypes = [_P]
_lib.fk_batch_workspace_bytes.restype = ctypes.c_size_t
_lib.fk_batch_set_plan.argtypes = [_P, ctypes.POINTER(fk_plan)]
_lib.fk_batch_set_plan.restype = ctypes.c_int
_lib.fk_batch_get_plan.argtypes = [_P, ctypes.POINTER(fk_plan)]
_lib.fk_batch_get_plan.restype = ctypes.c_int
_lib.fk_batch_autotune.argtypes = [_P, ctypes.c_int64, _P, ctypes.c_size_t, _P, ctypes.POINTER(fk_plan)]
_lib.fk_batch_autotune.restype = ctypes.c_int
_lib.fk_batch_run.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
_lib.fk_batch_run.restype = ctypes.c_int
_lib.fk_batch_capture.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
_lib.fk_batch_capture.restype = ctypes.c_int
_lib.fk_batch_replay.argtypes = [_P, _P]
_lib.fk_batch_replay.restype = ctypes.c_int
_lib.fk_batch_destroy.argtypes = [_P]
_lib.fk_batch_destroy.restype = None
_lib.subdomain_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
_lib.subdomain_workspace_bytes.restype = ctypes.c_size_t
_lib.subdomain_solve.argtypes = [ctypes.POINTER(fk_density), ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
_lib.subdomain_solve.restype = ctypes.c_int
_lib.subdomain_workspace_bytes_rect.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
_lib.subdomain_workspace_bytes_rect.restype = ctypes.c_size_t
_lib.subdomain_solve_rect.argtypes = [ctypes.POINTER(fk_density), ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P,
                                      ctypes.c_size_t, _P]
_lib.subdomain_solve_rect.restype = ctypes.c_int
_lib.fk_density_sample.argtypes = [ctypes.POINTER(fk_density), ctypes.c_double, ctypes.c_int32, _P, _P]
_lib.fk_density_sample.restype = ctypes.c_int
_lib.fk_density_grid_drift.argtypes = [_P, ctypes.c_int32, _P, _P]
_lib.fk_density_grid_drift.restype = ctypes.c_int
_lib.fk_boundary_workspace_bytes.argtypes = [ctypes.c_int32]
_lib.fk_boundary_workspace_bytes.restype = ctypes.c_size_t
_lib.fk_boundary_data.argtypes = [ctypes.POINTER(fk_density), ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                  _P, ctypes.c_size_t, _P]
_lib.fk_boundary_data.restype = ctypes.c_int
_lib.fk_key_points.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _P, _P]
_lib.fk_key_points.restype = ctypes.c_int
_lib.fk_interface_interpolate.argtypes = [ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int64, _P, _P, _P, _P, _P, _P,
                                          _P]
_lib.fk_interface_interpolate.restype = ctypes.c_int
_lib.fk_interface_interpolate_mask.argtypes = [ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P, _P]
_lib.fk_interface_interpolate_mask.restype = ctypes.c_int
_lib.fk_mesh_quality.argtypes = [_P, _P, ctypes.c_int32, _P, _P]
_lib.fk_mesh_quality.restype = ctypes.c_int
_lib.fk_cv_create.argtypes = [_P, ctypes.c_double, ctypes.POINTER(_P)]
_lib.fk_cv_create.restype = ctypes.c_int
_lib.fk_cv_set_identity_base.argtypes = [_P, ctypes.c_int32]
_lib.fk_cv_set_identity_base.restype = ctypes.c_int
_lib.fk_cv_set_base.argtypes = [_P, ctypes.c_int32]
_lib.fk_cv_set_base.restype = ctypes.c_int
_lib.fk_cv_destroy.argtypes = [_P]
_lib.fk_cv_destroy.restype = None
_lib.fk_cv_get_params.argtypes = [_P, _P, _P]
_lib.fk_cv_get_params.restype = ctypes.c_int
_lib.fk_cv_set_params.argtypes = [_P, _P]
_lib.fk_cv_set_params.restype = ctypes.c_int
_lib.fk_cv_eval.argtypes = [_P, _P, ctypes.c_int64, _P, _P]
_lib.fk_cv_eval.restype = ctypes.c_int
_lib.fk_cv_set_grad_precision.argtypes = [_P, ctypes.c_int32]
_lib.fk_cv_set_grad_precision.restype = ctypes.c_int
_lib.fk_cv_eval_grad.argtypes = [_P, _P, ctypes.c_int64, _P, _P]
_lib.fk_cv_eval_grad.restype = ctypes.c_int
_lib.fk_cv_grad.argtypes = [_P, _P, _P, ctypes.c_int64, _P, _P, _P]
_lib.fk_cv_grad.restype = ctypes.c_int
_lib.fk_cv_adam_apply.argtypes = [_P, _P, ctypes.c_float, _P]
_lib.fk_cv_adam_apply.restype = ctypes.c_int
_lib.fk_cv_train.argtypes = [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                             ctypes.c_uint64, _P, _P]
_lib.fk_cv_train.restype = ctypes.c_int
_lib.fk_interface_cv_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64]
_lib.fk_interface_cv_workspace_bytes.restype = ctypes.c_size_t
_lib.fk_interface_cv_grid_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]
_lib.fk_interface_cv_grid_workspace_bytes.restype = ctypes.c_size_t
_lib.fk_interface_solve_cv.argtypes = [
    ctypes.POINTER(fk_density), ctypes.POINTER(fk_data), _P, _P, ctypes.c_int64,
    ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, _P, ctypes.c_int32,
    ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(fk_plan), _P, ctypes.c_size_t, _P]
_lib.fk_interface_solve_cv.restype = ctypes.c_int
_lib.fk_timing_enable.argtypes = [ctypes.c_int]
_lib.fk_timing_enable.restype = ctypes.c_int
_lib.fk_timing_last.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.fk_timing_last.restype = ctypes.c_int


def library():
    """The loaded ctypes library handle."""
    return _lib


def declared_functions() -> list[str]:
    """Names of the functions ``include/fk.h`` declares."""
    src = open(HEADER_PATH).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(fk_[a-z0-9_]+|subdomain_[a-z0-9_]+)\s*\(",
                                 src, flags=re.M)))


def _check(rc: int):
    if rc != FK_OK:
        raise FkError(rc, _lib.fk_last_error().decode())


def fk_version() -> int:
    return _lib.fk_version()


def fk_last_error() -> str:
    return _lib.fk_last_error().decode()


FK_DENSITY_GRID = 6


def _density(d) -> fk_density:
    """fk_density of an object with its fields; a grid density (``GridDensity``)
    carries the device samples and drift table."""
    if int(d.kind) == FK_DENSITY_GRID:
        return fk_density(FK_DENSITY_GRID, 0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, int(d.grid_n), 0,
                          d.grid_w.data_ptr(), d.grid_b.data_ptr())
    return fk_density(int(d.kind), int(d.time_mode), float(d.amp), float(d.width2), float(d.cx),
                      float(d.cy), float(d.orbit_r), float(d.omega), float(d.t_freeze))


def fk_density_sample(density, tau: float, n: int, device=None, out=None):
    """w of an analytic density at the nodes of an n-cell grid: device FP64
    [(n+1), (n+1)] indexed [j, i] (x = i/n, y = j/n), into `out` if given."""
    import torch
    if out is None:
        out = torch.empty((n + 1, n + 1), dtype=torch.float64, device=device or "cuda")
    elif out.dtype != torch.float64 or out.shape != (n + 1, n + 1) or not out.is_contiguous():
        raise ValueError("out must be a contiguous [(n+1), (n+1)] FP64 tensor")
    w = _density(density)
    _check(_lib.fk_density_sample(ctypes.byref(w), float(tau), int(n), out.data_ptr(), _stream(torch, out.device)))
    return out


def fk_density_grid_drift(grid_w, out=None):
    """Nodal finite-difference drift table of device samples grid_w
    [(n+1), (n+1)] FP64: device FP32 [(n+1), (n+1), 2], into `out` if given."""
    import torch
    n = grid_w.shape[0] - 1
    if grid_w.dtype != torch.float64 or grid_w.shape != (n + 1, n + 1) or not grid_w.is_contiguous():
        raise ValueError("grid_w must be a contiguous square FP64 tensor")
    if out is None:
        out = torch.empty((n + 1, n + 1, 2), dtype=torch.float32, device=grid_w.device)
    elif out.dtype != torch.float32 or out.shape != (n + 1, n + 1, 2) or not out.is_contiguous():
        raise ValueError("out must be a contiguous [(n+1), (n+1), 2] FP32 tensor")
    _check(_lib.fk_density_grid_drift(grid_w.data_ptr(), int(n), out.data_ptr(), _stream(torch, grid_w.device)))
    return out


def n_interface_nodes(px: int, m: int) -> int:
    """Interface nodes of px x px sub-domains on the (px m)-cell grid."""
    N = px * m
    return 2 * (px - 1) * (N - 1) - (px - 1) ** 2


def fk_boundary_data(density, t_w, n, bdry_kind, xi_out, eta_out, workspace=None):
    """Writes the outer boundary data of one mesh step into the edge nodes of
    the device grids xi_out / eta_out ([(n+1), (n+1)] FP64)."""
    import torch
    need = int(_lib.fk_boundary_workspace_bytes(int(n)))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=xi_out.device)
    w = _density(density)
    _check(_lib.fk_boundary_data(ctypes.byref(w), float(t_w), int(n), int(bdry_kind), xi_out.data_ptr(),
                                 eta_out.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                 _stream(torch, xi_out.device)))
    return workspace


def fk_key_points(grid_w, px, m, tol=1e-2, max_gap=None, out=None):
    """Key-point mask (device uint8 [n_iface], canonical order) from device
    samples grid_w [(px m + 1), (px m + 1)] of w at the step's density time."""
    import torch
    n_if = n_interface_nodes(px, m)
    if out is None:
        out = torch.empty(n_if, dtype=torch.uint8, device=grid_w.device)
    max_gap = max(1, m // 2) if max_gap is None else int(max_gap)
    _check(_lib.fk_key_points(grid_w.data_ptr(), int(px), int(m), float(tol), max_gap, out.data_ptr(),
                              _stream(torch, grid_w.device)))
    return out


def fk_interface_interpolate(px, m, slot, key_xi, key_eta, edge_xi, edge_eta, out=None):
    """Every interface value from the key points' values (device FP64 [n_keys])
    and the boundary data in the edge nodes of edge_xi / edge_eta; ``slot``:
    device int32 [n_iface], the node's index into the key arrays or -1."""
    import torch
    n_if = n_interface_nodes(px, m)
    dev = slot.device
    if out is None:
        out = (torch.empty(n_if, dtype=torch.float64, device=dev), torch.empty(n_if, dtype=torch.float64, device=dev))
    n_keys = int(key_xi.numel())
    _check(_lib.fk_interface_interpolate(int(px), int(m), slot.data_ptr(), n_keys,
                                         key_xi.data_ptr() if n_keys else None, key_eta.data_ptr() if n_keys else None,
                                         edge_xi.data_ptr(), edge_eta.data_ptr(), out[0].data_ptr(), out[1].data_ptr(),
                                         _stream(torch, dev)))
    return out


def fk_interface_interpolate_mask(px, m, mask, edge_xi, edge_eta, iface_xi, iface_eta):
    """In place: the interface nodes with ``mask`` (device uint8 [n_iface])
    zero get the interpolant through the values at the nonzero ones (already
    in ``iface_xi`` / ``iface_eta``) and the line ends in the edge nodes of
    ``edge_xi`` / ``edge_eta``."""
    import torch
    n_if = n_interface_nodes(px, m)
    for name, x, dt in (("mask", mask, torch.uint8), ("iface_xi", iface_xi, torch.float64),
                        ("iface_eta", iface_eta, torch.float64)):
        if x.dtype != dt or x.numel() != n_if or not x.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dt} tensor with one entry per interface node")
    _check(_lib.fk_interface_interpolate_mask(int(px), int(m), mask.data_ptr(), edge_xi.data_ptr(),
                                              edge_eta.data_ptr(), iface_xi.data_ptr(), iface_eta.data_ptr(),
                                              _stream(torch, mask.device)))
    return iface_xi, iface_eta


class GridDensity:
    """A density known only at grid nodes (Sect. 4): device FP64 samples
    ``grid_w`` [(n+1), (n+1)] and their drift table ``grid_b`` (computed here
    by ``fk_density_grid_drift``).  The tensors must outlive the calls that
    use the density."""
    kind = FK_DENSITY_GRID
    time_mode = 0

    def __init__(self, grid_w, grid_b=None):
        import torch
        self.grid_w = grid_w.to(torch.float64).contiguous()
        self.grid_n = int(self.grid_w.shape[0]) - 1
        self.grid_b = fk_density_grid_drift(self.grid_w, out=grid_b)


def _data(d, grids=None) -> fk_data:
    gx = gy = None
    n = 0
    if grids is not None:
        gx, gy = grids
        n = int(round(gx.numel() ** 0.5)) - 1
    return fk_data(int(d.init_kind), int(d.bdry_kind), int(d.score_mode), n, float(d.t_init),
                   None if gx is None else gx.data_ptr(), None if gy is None else gy.data_ptr())


def _device_pts(pts, dev):
    """Node coordinates as a contiguous FP64 [n, 2] device tensor (a device
    tensor is used as it is; host arrays are copied)."""
    import torch
    if isinstance(pts, torch.Tensor):
        if pts.device.type != "cuda" or pts.dtype != torch.float64 or not pts.is_contiguous():
            pts = pts.to(device=dev, dtype=torch.float64).contiguous()
        return pts.reshape(-1, 2)
    a = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    return torch.from_numpy(a).to(dev)


def _device_mask(mask, n, dev):
    if mask is None:
        return None
    import torch
    if not isinstance(mask, torch.Tensor):
        mask = torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8)).to(dev)
    if mask.dtype != torch.uint8 or mask.numel() != n or not mask.is_contiguous():
        raise ValueError("mask must be a contiguous uint8 tensor with one entry per node")
    return mask


def _stream(torch, device):
    # torch's current stream on a GPU device; no stream for host tensors (the
    # library then fails its argument checks or finds no device, and says so)
    if torch.device(device).type != "cuda":
        return None
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def fk_interface_workspace_bytes(n_nodes: int, n_paths: int) -> int:
    return int(_lib.fk_interface_workspace_bytes(n_nodes, n_paths))


def fk_interface_cv_grid_workspace_bytes(n_nodes: int, n_paths: int, grid_n: int) -> int:
    """Workspace of a control-variate solve with the mesh-gradient table."""
    return int(_lib.fk_interface_cv_grid_workspace_bytes(n_nodes, n_paths, grid_n))


def fk_boundary_workspace_bytes(n: int) -> int:
    return int(_lib.fk_boundary_workspace_bytes(int(n)))


def fk_philox_words(ctr, seed: int):
    """Philox4x32-10 words of device counters ctr (int32/uint32 tensor [n, 4])."""
    import torch
    out = torch.empty_like(ctr)
    _check(_lib.fk_philox_words(ctr.data_ptr(), ctr.shape[0], int(seed), out.data_ptr(),
                                _stream(torch, ctr.device)))
    return out


def fk_normals(ra, rb, D: float):
    """FP32 Brownian increments sqrt(2 D) (z0, z1) of word pairs (device tensors [n])."""
    import torch
    out = torch.empty((ra.shape[0], 2), dtype=torch.float32, device=ra.device)
    _check(_lib.fk_normals(ra.data_ptr(), rb.data_ptr(), ra.shape[0], float(D), out.data_ptr(),
                           _stream(torch, ra.device)))
    return out


def fk_timing_enable(enable: bool = True):
    _check(_lib.fk_timing_enable(1 if enable else 0))


def fk_timing_last():
    """(path_kernel_ms, reduce_kernel_ms) of the last solve timed on this thread."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(_lib.fk_timing_last(ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def fk_sync(stream=None):
    import torch
    s = stream if stream is not None else _stream(torch, None)
    _check(_lib.fk_sync(s))


def fk_interface_solve(density, data, pts, t, dt, n_paths, seed=0, level_id=0, *,
                       exit_step=False, scores=False, steps=False, plan=None,
                       device="cuda", workspace=None, grids=None, out=None, mask=None):
    """Monte-Carlo interface solve (C: ``fk_interface_solve``).

    ``density`` / ``data`` are objects with the fields of ``fk_density`` /
    ``fk_data`` (e.g. ``workloads.Density`` / ``workloads.Data``); ``pts`` is
    an [n, 2] array of node coordinates (a device tensor, or a host array that
    is copied to the device); ``mask`` (uint8 [n], device or host) restricts
    the solve to its nonzero nodes and leaves the others' outputs as they
    were.  ``grids`` = (xi, eta) device
    FP64 tensors for grid initial data.  Returns a dict of device tensors:
    ``xi, eta, se_xi, se_eta`` (FP64 [n]), ``total_steps`` (uint64 [1] as
    int64), and on request ``exit_step`` (int32 [n, N]), ``scores`` (FP32
    [n, N, 2]) and ``steps`` (int64 [n]).  Runs asynchronously on torch's
    current stream.
    """
    import torch
    dev = torch.device(device)
    pts = _device_pts(pts, dev)
    n = pts.shape[0]
    mask = _device_mask(mask, n, dev)
    if out is None:
        out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("xi", "eta", "se_xi", "se_eta")}
        out["total_steps"] = torch.zeros(1, dtype=torch.int64, device=dev)
        if exit_step:
            out["exit_step"] = torch.empty((n, n_paths), dtype=torch.int32, device=dev)
        if scores:
            out["scores"] = torch.empty((n, n_paths, 2), dtype=torch.float32, device=dev)
        if steps:
            out["steps"] = torch.empty(n, dtype=torch.int64, device=dev)
    need = _lib.fk_interface_workspace_bytes(n, n_paths)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    pl = _plan_struct(plan)

    def ptr(k):
        v = out.get(k)
        return None if v is None else v.data_ptr()

    rc = _lib.fk_interface_solve(
        ctypes.byref(_density(density)), ctypes.byref(_data(data, grids)),
        pts.data_ptr() if n else None, None if mask is None else mask.data_ptr(), n, float(t), float(dt),
        int(n_paths), int(seed), int(level_id),
        ptr("xi"), ptr("eta"), ptr("se_xi"), ptr("se_eta"), ptr("exit_step"), ptr("scores"), ptr("steps"),
        ptr("total_steps"), None if pl is None else ctypes.byref(pl),
        workspace.data_ptr(), workspace.numel(), _stream(torch, dev))
    _check(rc)
    out["_workspace"] = workspace
    out["_pts"] = pts
    return out


def fk_interface_noalloc_max_bytes() -> int:
    return int(_lib.fk_interface_noalloc_max_bytes())


def fk_interface_solve_noalloc(density, data, pts, t, dt, n_paths, seed=0, level_id=0, *, out, plan=None,
                               device="cuda", grids=None, mask=None):
    """``fk_interface_solve_noalloc``: the interface solve on the library's
    static device scratch (no workspace).  ``out``: dict of caller-allocated
    device tensors -- xi, eta, se_xi, se_eta (FP64 [n]) and optionally
    exit_step, scores, steps, total_steps as in ``fk_interface_solve``."""
    import torch
    dev = torch.device(device)
    pts = _device_pts(pts, dev)
    mask = _device_mask(mask, pts.shape[0], dev)
    pl = _plan_struct(plan)

    def ptr(k):
        v = out.get(k)
        return None if v is None else v.data_ptr()

    rc = _lib.fk_interface_solve_noalloc(
        ctypes.byref(_density(density)), ctypes.byref(_data(data, grids)),
        pts.data_ptr() if pts.shape[0] else None, None if mask is None else mask.data_ptr(), pts.shape[0], float(t),
        float(dt), int(n_paths), int(seed), int(level_id), ptr("xi"), ptr("eta"), ptr("se_xi"), ptr("se_eta"),
        ptr("exit_step"), ptr("scores"), ptr("steps"), ptr("total_steps"), None if pl is None else ctypes.byref(pl),
        _stream(torch, dev))
    _check(rc)
    return out


def _plan_struct(plan):
    if plan is None:
        return None
    if isinstance(plan, FkPlan):
        plan = plan.get()
    return fk_plan(int(plan.get("block", 0)), int(plan.get("blocks_per_cu", 0)), int(plan.get("chunk", 0)),
                   int(plan.get("node_tile", 0)))


def _plan_dict(p: fk_plan) -> dict:
    return {"block": p.block, "blocks_per_cu": p.blocks_per_cu, "chunk": p.chunk, "node_tile": p.node_tile}


_lib.fk_plan_create.argtypes = [ctypes.POINTER(fk_plan), ctypes.POINTER(_P)]
_lib.fk_plan_create.restype = ctypes.c_int
_lib.fk_plan_set.argtypes = [_P, ctypes.POINTER(fk_plan)]
_lib.fk_plan_set.restype = ctypes.c_int
_lib.fk_plan_get.argtypes = [_P, ctypes.POINTER(fk_plan)]
_lib.fk_plan_get.restype = ctypes.c_int
_lib.fk_plan_autotune.argtypes = [_P, ctypes.POINTER(fk_density), ctypes.POINTER(fk_data), _P, _P, ctypes.c_int64,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, _P,
                                  ctypes.c_size_t, _P]
_lib.fk_plan_autotune.restype = ctypes.c_int
for _name in ("fk_plan_capture_begin", "fk_plan_capture_end", "fk_plan_replay"):
    getattr(_lib, _name).argtypes = [_P, _P]
    getattr(_lib, _name).restype = ctypes.c_int
_lib.fk_plan_graph_updates.argtypes = [_P]
_lib.fk_plan_graph_updates.restype = ctypes.c_int
_lib.fk_plan_destroy.argtypes = [_P]
_lib.fk_plan_destroy.restype = None


class FkPlan:
    """A launch plan with its autotune record and a captured HIP graph
    (C: ``fk_plan_*``).  Pass it as ``plan=`` to the solves.  ``capture()``
    is a context manager: the library calls made inside it on torch's
    current stream (a non-default one) are recorded, not run; ``replay()``
    runs them.  Capturing the same sequence again with other arguments
    updates the graph in place (``updates`` counts those)."""

    def __init__(self, plan=None):
        h = _P()
        p = _plan_struct(plan) if plan is not None else None
        _check(_lib.fk_plan_create(None if p is None else ctypes.byref(p), ctypes.byref(h)))
        self.handle = h

    def get(self) -> dict:
        p = fk_plan()
        _check(_lib.fk_plan_get(self.handle, ctypes.byref(p)))
        return _plan_dict(p)

    def set(self, plan):
        _check(_lib.fk_plan_set(self.handle, ctypes.byref(_plan_struct(plan))))

    def autotune(self, density, data, pts, t, dt, probe_paths, seed=0, mask=None, device="cuda", grids=None,
                 workspace=None) -> dict:
        import torch
        dev = torch.device(device)
        pts = _device_pts(pts, dev)
        n = pts.shape[0]
        mask = _device_mask(mask, n, dev)
        need = _lib.fk_interface_workspace_bytes(n, probe_paths)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        _check(_lib.fk_plan_autotune(self.handle, ctypes.byref(_density(density)), ctypes.byref(_data(data, grids)),
                                     pts.data_ptr() if n else None, None if mask is None else mask.data_ptr(), n,
                                     float(t), float(dt), int(probe_paths), int(seed), workspace.data_ptr(),
                                     workspace.numel(), _stream(torch, dev)))
        return self.get()

    class _Capture:
        def __init__(self, plan, device):
            self.plan, self.device = plan, device

        def __enter__(self):
            import torch
            _check(_lib.fk_plan_capture_begin(self.plan.handle, _stream(torch, self.device)))
            return self.plan

        def __exit__(self, exc_type, exc, tb):
            import torch
            rc = _lib.fk_plan_capture_end(self.plan.handle, _stream(torch, self.device))
            if exc_type is None:
                _check(rc)
            return False

    def capture(self, device="cuda"):
        import torch
        return FkPlan._Capture(self, torch.device(device))

    def replay(self, device="cuda"):
        import torch
        _check(_lib.fk_plan_replay(self.handle, _stream(torch, torch.device(device))))

    @property
    def updates(self) -> int:
        return int(_lib.fk_plan_graph_updates(self.handle))

    def close(self):
        if self.handle:
            _lib.fk_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FkBatch:
    """Batched interface solve (C: ``fk_batch_*``).

    ``levels`` is a list of (density, t, t_init, pts[n_l, 2], level_id); the
    node slices are concatenated in that order.  Outputs are device tensors
    over all nodes.
    """

    def __init__(self, levels, data, dt, n_paths, seed=0, device="cuda"):
        import torch
        self.device = torch.device(device)
        pts, arr, off = [], (fk_level * len(levels))(), 0
        for i, (dens, t, t_init, p, level_id) in enumerate(levels):
            p = np.ascontiguousarray(p, dtype=np.float64).reshape(-1, 2)
            arr[i] = fk_level(_density(dens), float(t), float(t_init), off, p.shape[0], int(level_id), 0)
            pts.append(p)
            off += p.shape[0]
        self.pts = np.ascontiguousarray(np.concatenate(pts) if pts else np.zeros((0, 2)))
        self.n_total = off
        self.n_paths = int(n_paths)
        self.offsets = np.cumsum([0] + [len(p) for p in pts])
        self._data = _data(data)
        h = ctypes.c_void_p()
        _check(_lib.fk_batch_create(arr, len(levels), self.pts.ctypes.data_as(ctypes.c_void_p), self.n_total,
                                    ctypes.byref(self._data), float(dt), self.n_paths, int(seed), ctypes.byref(h)))
        self._h = h
        self.workspace = torch.empty(max(int(_lib.fk_batch_workspace_bytes(h)), 256), dtype=torch.uint8,
                                     device=self.device)

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fk_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    @property
    def plan(self) -> dict:
        p = fk_plan()
        _check(_lib.fk_batch_get_plan(self._h, ctypes.byref(p)))
        return _plan_dict(p)

    @plan.setter
    def plan(self, plan: dict):
        _check(_lib.fk_batch_set_plan(self._h, _plan_struct(plan)))

    def autotune(self, probe_paths: int) -> dict:
        import torch
        p = fk_plan()
        _check(_lib.fk_batch_autotune(self._h, int(probe_paths), self.workspace.data_ptr(), self.workspace.numel(),
                                      _stream(torch, self.device), ctypes.byref(p)))
        return _plan_dict(p)

    def outputs(self, exit_step=False, scores=False):
        import torch
        n, dev = self.n_total, self.device
        out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("xi", "eta", "se_xi", "se_eta")}
        out["total_steps"] = torch.zeros(1, dtype=torch.int64, device=dev)
        if exit_step:
            out["exit_step"] = torch.empty((n, self.n_paths), dtype=torch.int32, device=dev)
        if scores:
            out["scores"] = torch.empty((n, self.n_paths, 2), dtype=torch.float32, device=dev)
        return out

    def _args(self, out):
        def ptr(k):
            v = out.get(k)
            return None if v is None else v.data_ptr()
        return (ptr("xi"), ptr("eta"), ptr("se_xi"), ptr("se_eta"), ptr("exit_step"), ptr("scores"),
                ptr("total_steps"), self.workspace.data_ptr(), self.workspace.numel())

    def run(self, out=None, exit_step=False, scores=False):
        import torch
        out = out if out is not None else self.outputs(exit_step, scores)
        _check(_lib.fk_batch_run(self._h, *self._args(out), _stream(torch, self.device)))
        return out

    def capture(self, out, stream):
        """Capture run(out) into a HIP graph on ``stream`` (a torch.cuda.Stream)."""
        _check(_lib.fk_batch_capture(self._h, *self._args(out), ctypes.c_void_p(stream.cuda_stream)))

    def replay(self, stream=None):
        import torch
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream(torch, self.device)
        _check(_lib.fk_batch_replay(self._h, s))


def subdomain_workspace_bytes(px: int, m: int) -> int:
    return int(_lib.subdomain_workspace_bytes(px, m))


def subdomain_solve(density, t_w, dt_mesh, px, m, xi_n, eta_n, iface_xi, iface_eta, bdry_kind=0,
                    out=None, workspace=None):
    """Sub-domain backward-Euler solves (C: ``subdomain_solve``).  Grids are
    device FP64 tensors [(px m + 1)^2] (or 2-D views); returns (xi, eta).
    dt_mesh = inf: the steady solves (xi_n, eta_n may be None)."""
    import torch
    dev = iface_xi.device
    N1 = px * m + 1
    if out is None:
        out = (torch.empty((N1, N1), dtype=torch.float64, device=dev),
               torch.empty((N1, N1), dtype=torch.float64, device=dev))
    need = _lib.subdomain_workspace_bytes(px, m)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    _check(_lib.subdomain_solve(ctypes.byref(_density(density)), float(t_w), float(dt_mesh), int(px), int(m),
                                int(bdry_kind), None if xi_n is None else xi_n.data_ptr(),
                                None if eta_n is None else eta_n.data_ptr(), iface_xi.data_ptr(),
                                iface_eta.data_ptr(), out[0].data_ptr(), out[1].data_ptr(), workspace.data_ptr(),
                                workspace.numel(), _stream(torch, dev)))
    return out


def subdomain_workspace_bytes_rect(px: int, py: int, n_cells: int) -> int:
    return int(_lib.subdomain_workspace_bytes_rect(px, py, n_cells))


def n_interface_nodes_rect(px: int, py: int, n_cells: int) -> int:
    """Interface nodes of a px x py split of an n-cell grid (canonical order:
    vertical lines, then horizontal lines without the crossings)."""
    return (px - 1) * (n_cells - 1) + (py - 1) * (n_cells - px)


def subdomain_solve_rect(density, t_w, dt_mesh, px, py, n_cells, xi_n, eta_n, iface_xi, iface_eta, bdry_kind=0,
                         out=None, workspace=None):
    """``subdomain_solve_rect``: px x py sub-domains of (n/px) x (n/py) cells
    of an n-cell grid; otherwise as ``subdomain_solve``."""
    import torch
    dev = iface_xi.device
    N1 = int(n_cells) + 1
    if out is None:
        out = (torch.empty((N1, N1), dtype=torch.float64, device=dev),
               torch.empty((N1, N1), dtype=torch.float64, device=dev))
    need = _lib.subdomain_workspace_bytes_rect(px, py, n_cells)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    _check(_lib.subdomain_solve_rect(ctypes.byref(_density(density)), float(t_w), float(dt_mesh), int(px), int(py),
                                     int(n_cells), int(bdry_kind), None if xi_n is None else xi_n.data_ptr(),
                                     None if eta_n is None else eta_n.data_ptr(), iface_xi.data_ptr(),
                                     iface_eta.data_ptr(), out[0].data_ptr(), out[1].data_ptr(), workspace.data_ptr(),
                                     workspace.numel(), _stream(torch, dev)))
    return out


def fk_mesh_quality(xi, eta, out=None):
    """(min Jacobian, max skewness) device tensor [2] of a nodal map (into
    ``out``, a contiguous FP64 [2], if given)."""
    import torch
    n = int(round(xi.numel() ** 0.5)) - 1
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=xi.device)
    elif out.numel() != 2 or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous FP64 tensor of 2 elements")
    _check(_lib.fk_mesh_quality(xi.data_ptr(), eta.data_ptr(), n, out.data_ptr(), _stream(torch, xi.device)))
    return out


FK_CV_N_PARAMS = 8706


FK_CV_BASES = {"none": 0, "identity": 1, "grid": 2}
FK_CV_GRAD_PRECISIONS = {"split": 0, "bf16": 1}


class FkCv:
    """The control-variate network (C: ``fk_cv_*``)."""

    def __init__(self, params, t_scale=0.1, identity_base=False, base=None, grad_precision="split"):
        """``base``: None / "none" (the network itself), "identity" (u_hat =
        (x, y) + network; also ``identity_base=True``) or "grid" (u_hat = the
        solve's grid initial data, bilinear, + network; martingale solves).
        ``grad_precision``: "split" (BF16 hi + lo operands) or "bf16"
        (activations rounded to BF16 once) for the martingale forms' gradient."""
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        if p.size != FK_CV_N_PARAMS:
            raise ValueError("need 8706 parameters")
        h = ctypes.c_void_p()
        _check(_lib.fk_cv_create(p.ctypes.data_as(ctypes.c_void_p), float(t_scale), ctypes.byref(h)))
        self._h = h
        self.t_scale = float(t_scale)
        base = base or ("identity" if identity_base else "none")
        if base not in FK_CV_BASES:
            raise ValueError(f"base must be one of {sorted(FK_CV_BASES)}")
        self.base = base
        self.identity_base = base == "identity"
        _check(_lib.fk_cv_set_base(h, FK_CV_BASES[base]))
        self.set_grad_precision(grad_precision)

    def set_grad_precision(self, mode):
        if mode not in FK_CV_GRAD_PRECISIONS:
            raise ValueError(f"grad_precision must be one of {sorted(FK_CV_GRAD_PRECISIONS)}")
        _check(_lib.fk_cv_set_grad_precision(self._h, FK_CV_GRAD_PRECISIONS[mode]))
        self.grad_precision = mode

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fk_cv_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    @property
    def handle(self):
        return self._h

    def params(self):
        """(FP32 master weights, BF16 network as float64) on the host."""
        m = np.zeros(FK_CV_N_PARAMS, dtype=np.float32)
        b = np.zeros(FK_CV_N_PARAMS, dtype=np.uint16)
        _check(_lib.fk_cv_get_params(self._h, m.ctypes.data_as(ctypes.c_void_p), b.ctypes.data_as(ctypes.c_void_p)))
        bf = (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        return m, bf

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        _check(_lib.fk_cv_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p)))

    def eval(self, txy):
        """Forward-mode outputs [n, 2, 5] (value, dx, dy, dt, lap) at device points txy [n, 3] (FP32)."""
        import torch
        out = torch.empty((txy.shape[0], 2, 5), dtype=torch.float32, device=txy.device)
        _check(_lib.fk_cv_eval(self._h, txy.data_ptr(), txy.shape[0], out.data_ptr(), _stream(torch, txy.device)))
        return out

    def eval_grad(self, txy):
        """(x, y) gradient [n, 2, 2] as the martingale path kernels take it, at device points txy [n, 3]."""
        import torch
        out = torch.empty((txy.shape[0], 2, 2), dtype=torch.float32, device=txy.device)
        _check(_lib.fk_cv_eval_grad(self._h, txy.data_ptr(), txy.shape[0], out.data_ptr(),
                                    _stream(torch, txy.device)))
        return out

    def grad(self, txy, target):
        import torch
        g = torch.empty(FK_CV_N_PARAMS, dtype=torch.float32, device=txy.device)
        loss = torch.empty(1, dtype=torch.float32, device=txy.device)
        _check(_lib.fk_cv_grad(self._h, txy.data_ptr(), target.data_ptr(), txy.shape[0], g.data_ptr(),
                               loss.data_ptr(), _stream(torch, txy.device)))
        return g, loss

    def adam_apply(self, grad, lr):
        import torch
        _check(_lib.fk_cv_adam_apply(self._h, grad.data_ptr(), float(lr), _stream(torch, grad.device)))

    def train(self, txy, target, steps, batch, lr=1e-3, seed=0, losses=True):
        import torch
        loss = torch.zeros(max(steps, 1), dtype=torch.float32, device=txy.device) if losses else None
        _check(_lib.fk_cv_train(self._h, txy.data_ptr(), target.data_ptr(), txy.shape[0], int(steps), int(batch),
                                float(lr), int(seed), None if loss is None else loss.data_ptr(),
                                _stream(torch, txy.device)))
        return loss


FK_CV_DYNKIN, FK_CV_MARTINGALE, FK_CV_MARTINGALE_GRID = 0, 1, 2


def fk_interface_solve_cv(density, data, pts, t, dt, n_paths, cv, stride=2, seed=0, level_id=0, *,
                          form=FK_CV_DYNKIN, plain=True, exit_step=False, cv_scores=False, plan=None, device="cuda",
                          workspace=None, grids=None, out=None, grad_table=True, mask=None):
    """Control-variate interface solve (C: ``fk_interface_solve_cv``), Dynkin
    or martingale form; returns a dict of device tensors: xi, eta, se_xi,
    se_eta (CV), plain_* (same paths), total_steps, and on request exit_step,
    cv_scores.  ``out`` may supply some of the FP64 [n] outputs (contiguous
    device tensors, e.g. rows of a history buffer); the rest are allocated.
    ``grad_table``: for FK_CV_MARTINGALE_GRID, size the workspace with room
    for the per-cell gradient table (a smaller one is replaced); False keeps
    a given workspace of the plain size, and the kernel reads the grids."""
    import torch
    dev = torch.device(device)
    pts = _device_pts(pts, dev)
    n = pts.shape[0]
    mask = _device_mask(mask, n, dev)
    keys = ["xi", "eta", "se_xi", "se_eta"] + (["plain_xi", "plain_eta", "plain_se_xi", "plain_se_eta"] if plain else [])
    out = dict(out or {})
    for k in keys:
        if k not in out:
            out[k] = torch.empty(n, dtype=torch.float64, device=dev)
        elif out[k].numel() != n or out[k].dtype != torch.float64 or not out[k].is_contiguous():
            raise ValueError(f"out[{k!r}] must be a contiguous FP64 tensor of {n} elements")
    out.setdefault("total_steps", torch.zeros(1, dtype=torch.int64, device=dev))
    if exit_step and "exit_step" not in out:
        out["exit_step"] = torch.empty((n, n_paths), dtype=torch.int32, device=dev)
    if cv_scores and "cv_scores" not in out:
        out["cv_scores"] = torch.empty((n, n_paths, 2), dtype=torch.float32, device=dev)
    need = _lib.fk_interface_cv_workspace_bytes(n, n_paths)
    mesh_gradient = form == FK_CV_MARTINGALE_GRID or (cv is not None and getattr(cv, "base", None) == "grid")
    if mesh_gradient and grids is not None and grad_table:
        grid_n = int(round(grids[0].numel() ** 0.5)) - 1
        need = _lib.fk_interface_cv_grid_workspace_bytes(n, n_paths, grid_n)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)

    def ptr(k):
        v = out.get(k)
        return None if v is None else v.data_ptr()

    _check(_lib.fk_interface_solve_cv(
        ctypes.byref(_density(density)), ctypes.byref(_data(data, grids)), pts.data_ptr() if n else None,
        None if mask is None else mask.data_ptr(), n,
        float(t), float(dt), int(n_paths), int(seed), int(level_id), None if cv is None else cv.handle, int(stride),
        int(form),
        ptr("xi"), ptr("eta"), ptr("se_xi"), ptr("se_eta"), ptr("plain_xi"), ptr("plain_eta"), ptr("plain_se_xi"),
        ptr("plain_se_eta"), ptr("exit_step"), ptr("cv_scores"), ptr("total_steps"), _plan_struct(plan),
        workspace.data_ptr(), workspace.numel(), _stream(torch, dev)))
    out["_workspace"] = workspace
    out["_pts"] = pts
    return out
