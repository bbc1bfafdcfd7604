"""The C ABI of libfk.so on the CPU: it loads, exports every function the
header declares, and rejects bad arguments before touching a device."""
import ctypes

import numpy as np
import pytest

import workloads as W


def test_exports_every_declared_function(fk):
    names = fk.declared_functions()
    assert "fk_interface_solve" in names
    lib = fk.library()
    for n in names:
        assert hasattr(lib, n), n


def test_version(fk):
    assert fk.fk_version() >= 100


def _call(fk, dens=None, data=None, pts=None, t=0.05, dt=1e-4, n_paths=16, ws_bytes=None, out_ptr=8, plan=None):
    dens = dens or W.static_bump()
    data = data or W.Data()
    n = 1 if pts is None else int(pts)
    need = fk.fk_interface_workspace_bytes(max(n, 0), max(n_paths, 2))
    ws = ws_bytes if ws_bytes is not None else need
    lib = fk.library()
    # Non-null dummies (the node coordinates are device memory, never read
    # here): every call must fail validation before any use.
    return lib.fk_interface_solve(ctypes.byref(fk._density(dens)), ctypes.byref(fk._data(data)),
                                  4096 if n else None, None, n, t, dt, n_paths, 0, 0,
                                  out_ptr, out_ptr, out_ptr, out_ptr, None, None, None, None,
                                  None if plan is None else ctypes.byref(fk._plan_struct(plan)),
                                  4096, ws, None)


@pytest.mark.parametrize("kw,code", [
    (dict(n_paths=1), -1),
    (dict(dt=0.0), -1),
    (dict(dt=float("nan")), -1),
    (dict(t=-1.0), -1),
    (dict(pts=-1), -1),
    (dict(dens=W.Density(kind=9)), -1),
    (dict(dens=W.Density(kind=W.KIND_RING, amp=10.0, width2=50.0)), -1),   # ring needs beta <= 0
    (dict(dens=W.Density(kind=W.KIND_RING, amp=-1.0, width2=-50.0)), -1),  # and alpha >= 0
    (dict(data=W.Data(bdry_kind=W.DATA_GRID)), -1),
    (dict(data=W.Data(init_kind=W.DATA_GRID)), -1),
    (dict(ws_bytes=16), -3),
    (dict(plan={"chunk": 4096}), -1),      # a chunk's sums must fit the 64-bit LDS slots
    (dict(plan={"block": 96}), -1),
    (dict(plan={"node_tile": 3}), -1),     # node tiles are powers of two
    (dict(plan={"node_tile": 512}), -1),
    (dict(out_ptr=None), -1),
])
def test_validation_errors(fk, kw, code):
    rc = _call(fk, **kw)
    assert rc == code
    assert fk.fk_last_error() != ""


def test_empty_solve_is_a_noop(fk):
    assert _call(fk, pts=0) == 0


def test_workspace_size(fk):
    """The estimator is reduced inside the path kernel: the workspace holds
    per-node tables and sums only (no per-path records), whatever n_paths."""
    a = fk.fk_interface_workspace_bytes(1521, 100_000)
    assert a == fk.fk_interface_workspace_bytes(1521, 2)
    assert 1521 * 144 <= a <= 1521 * 160 + 4096
    # the batched workload: 66047 nodes at 2^16 paths in a few MB
    assert fk.fk_interface_workspace_bytes(66047, 1 << 16) < 12 << 20
    assert fk.fk_interface_workspace_bytes(10, 1) == 0


class _Ptr:
    def __init__(self, p):
        self.p = p

    def data_ptr(self):
        return self.p


class _FakeGrid:
    """A grid density with dummy device addresses (never dereferenced: every
    call below fails validation first)."""
    kind = 6
    time_mode = 0

    def __init__(self, n, w_ptr=4096, b_ptr=8192):
        self.grid_n = n
        self.grid_w = _Ptr(w_ptr)
        self.grid_b = _Ptr(b_ptr)


@pytest.mark.parametrize("grid", [_FakeGrid(1), _FakeGrid(16, w_ptr=0), _FakeGrid(16, b_ptr=0),
                                  _FakeGrid(16, b_ptr=8196)])
def test_grid_density_validation(fk, grid):
    assert _call(fk, dens=grid) == -1
    assert "grid" in fk.fk_last_error()


def test_grid_density_entry_points_validate(fk):
    lib = fk.library()
    assert lib.fk_density_sample(ctypes.byref(fk._density(_FakeGrid(8))), 0.0, 8, 4096, None) == -1
    assert lib.fk_density_sample(ctypes.byref(fk._density(W.static_bump())), 0.0, 0, 4096, None) == -1
    assert lib.fk_density_sample(ctypes.byref(fk._density(W.static_bump())), 0.0, 8, None, None) == -1
    assert lib.fk_density_grid_drift(4096, 1, 8192, None) == -1
    assert lib.fk_density_grid_drift(4096, 8, 8196, None) == -1
    assert lib.fk_density_grid_drift(None, 8, 8192, None) == -1
    # sub-domain solves need the density sampled on the mesh grid (N = px m = 16)
    need = lib.subdomain_workspace_bytes(2, 8)
    rc = lib.subdomain_solve(ctypes.byref(fk._density(_FakeGrid(12))), 0.0, 1e-3, 2, 8, 0, 4096, 4096, 4096, 4096,
                             4096, 4096, 4096, need, None)
    assert rc == -1 and "mesh grid" in fk.fk_last_error()


def test_key_point_entry_points_validate(fk):
    lib = fk.library()
    assert lib.fk_key_points(4096, 1, 8, 1e-2, 4, 8192, None) == -1          # px < 2
    assert lib.fk_key_points(4096, 2, 1, 1e-2, 4, 8192, None) == -1          # m < 2
    assert lib.fk_key_points(4096, 2, 8, -1.0, 4, 8192, None) == -1         # tol < 0
    assert lib.fk_key_points(4096, 2, 8, float("nan"), 4, 8192, None) == -1
    assert lib.fk_key_points(4096, 2, 8, 1e-2, 0, 8192, None) == -1          # max_gap < 1
    assert lib.fk_key_points(None, 2, 8, 1e-2, 4, 8192, None) == -1
    assert lib.fk_key_points(4096, 128, 128, 1e-2, 4, 8192, None) == -1      # grid too large
    assert lib.fk_interface_interpolate(1, 8, 4096, 1, 4096, 4096, 4096, 4096, 4096, 4096, None) == -1
    assert lib.fk_interface_interpolate(2, 8, 4096, -1, 4096, 4096, 4096, 4096, 4096, 4096, None) == -1
    assert lib.fk_interface_interpolate(2, 8, None, 1, 4096, 4096, 4096, 4096, 4096, 4096, None) == -1
    assert lib.fk_interface_interpolate(2, 8, 4096, 3, None, 4096, 4096, 4096, 4096, 4096, None) == -1
    d = ctypes.byref(fk._density(W.static_bump()))
    assert lib.fk_boundary_data(d, 0.0, 1, 0, 4096, 4096, None, 0, None) == -1          # n < 2
    assert lib.fk_boundary_data(d, 0.0, 16, 7, 4096, 4096, None, 0, None) == -1         # unknown kind
    assert lib.fk_boundary_data(d, 0.0, 16, 4, 4096, 4096, None, 0, None) == -3         # needs workspace
    assert lib.fk_boundary_data(ctypes.byref(fk._density(_FakeGrid(12))), 0.0, 16, 0, 4096, 4096, None, 0,
                                None) == -1                                             # grid_n != n


def test_bridge_and_grid_boundary_validation(fk):
    # grid boundary data needs grid initial data and a projecting score mode
    assert _call(fk, data=W.Data(bdry_kind=W.DATA_GRID, score_mode=W.SCORE_BRIDGE)) == -1
    assert _call(fk, data=W.Data(score_mode=7)) == -1
    assert fk.library().fk_boundary_workspace_bytes(1) == 0
    assert fk.library().fk_boundary_workspace_bytes(40) >= 4 * 40 * 8


def test_steady_subdomain_validation(fk):
    lib = fk.library()
    d = ctypes.byref(fk._density(W.static_bump()))
    need = lib.subdomain_workspace_bytes(2, 8)
    nan, inf = float("nan"), float("inf")
    assert lib.subdomain_solve(d, 0.0, nan, 2, 8, 0, 4096, 4096, 4096, 4096, 4096, 4096, 4096, need, None) == -1
    assert lib.subdomain_solve(d, 0.0, -inf, 2, 8, 0, 4096, 4096, 4096, 4096, 4096, 4096, 4096, need, None) == -1
    # transient solves need the previous mesh
    assert lib.subdomain_solve(d, 0.0, 1e-3, 2, 8, 0, None, None, 4096, 4096, 4096, 4096, 4096, need, None) == -1


def test_binding_rejects_bad_output_rows(fk):
    """Caller-supplied outputs (history rows of a mesh run) are checked in
    the binding before any call: FP64, contiguous, the right length."""
    import torch
    x = torch.zeros(9, dtype=torch.float64)
    with pytest.raises(ValueError):
        fk.fk_mesh_quality(x, x, out=torch.zeros(3, dtype=torch.float64))
    with pytest.raises(ValueError):
        fk.fk_mesh_quality(x, x, out=torch.zeros(2, dtype=torch.float32))
    with pytest.raises(ValueError):
        fk.fk_interface_solve_cv(W.CONST, W.Data(), np.array([[0.5, 0.5], [0.25, 0.5]]), 0.01, 1e-3, 64, None,
                                 form=fk.FK_CV_MARTINGALE_GRID, device="cpu",
                                 out={"xi": torch.zeros((2, 2), dtype=torch.float64)[:, 0]})


def test_noalloc_rejects_sizes_beyond_its_scratch(fk):
    """fk_interface_solve_noalloc checks the size against its static scratch
    before touching a device."""
    lib = fk.library()
    cap = fk.fk_interface_noalloc_max_bytes()
    assert cap == 8 << 20
    n = 100_000
    assert fk.fk_interface_workspace_bytes(n, 16) > cap
    rc = lib.fk_interface_solve_noalloc(ctypes.byref(fk._density(W.static_bump())), ctypes.byref(fk._data(W.Data())),
                                        4096, None, n, 0.05, 1e-4, 16, 0, 0,
                                        8, 8, 8, 8, None, None, None, None, None, None)
    assert rc == -3
    assert "scratch" in fk.fk_last_error()


def test_subdomain_layout_validation(fk):
    """px x py splits: px and py must divide N, sub-domains need 2 cells a
    side and at most 128 on the shorter one; checked before any device use."""
    lib = fk.library()
    assert fk.subdomain_workspace_bytes_rect(2, 3, 48) > 0
    assert fk.subdomain_workspace_bytes_rect(2, 3, 50) == 0          # 3 does not divide 50
    assert fk.subdomain_workspace_bytes_rect(1, 1, 129) == 0         # 129 cells on the shorter side
    assert fk.subdomain_workspace_bytes_rect(1, 2, 256) > 0          # 256 x 128: the shorter side is 128
    assert fk.subdomain_workspace_bytes_rect(4, 1, 4) == 0           # 1-cell-wide sub-domains
    assert fk.subdomain_workspace_bytes(8, 96) == fk.subdomain_workspace_bytes_rect(8, 8, 768)
    dens = ctypes.byref(fk._density(W.static_bump()))
    for px, py, n, code in ((2, 3, 50, -1), (0, 1, 8, -1), (1, 1, 258, -5), (4, 4, 4, -1)):
        rc = lib.subdomain_solve_rect(dens, 0.0, 0.01, px, py, n, 0, 8, 8, 8, 8, 8, 8, 8, 1 << 30, None)
        assert rc == code, (px, py, n, rc)
        assert fk.fk_last_error() != ""


def test_exponential_steps_only_in_single_solves(fk):
    """Exponential time-stepping is a single-solve mode: the control-variate
    and batched solves reject it before any device use; an unknown mode is
    invalid everywhere."""
    data = W.Data(score_mode=W.SCORE_EXPONENTIAL)
    with pytest.raises(fk.FkError) as e:
        fk.fk_interface_solve_cv(W.CONST, data, np.array([[0.5, 0.5]]), 0.01, 1e-3, 64, None,
                                 form=fk.FK_CV_MARTINGALE_GRID, device="cpu")
    assert e.value.code == -5
    with pytest.raises(fk.FkError) as e:
        fk.FkBatch([(W.CONST, 0.01, 0.0, np.array([[0.5, 0.5]]), 1)], data, 1e-3, 64, device="cpu")
    assert e.value.code == -5
    assert _call(fk, data=W.Data(score_mode=5)) == -1


def test_network_handle_calls_reject_a_null_handle(fk):
    lib = fk.library()
    assert lib.fk_cv_set_grad_precision(None, 0) == -1
    assert lib.fk_cv_set_base(None, 0) == -1
    assert lib.fk_cv_eval_grad(None, None, 4, None, None) == -1
    assert lib.fk_cv_eval(None, None, 4, None, None) == -1
    assert fk.fk_last_error() != ""
