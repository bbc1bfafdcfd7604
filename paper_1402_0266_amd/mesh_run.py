"""Time-dependent mesh generation by stochastic domain decomposition (Sect. 4).

One mesh step advances the nodal map (xi, eta) from t^n to t^{n+1} =
t^n + dt_mesh:

1. the density is frozen at t^n (Sect. 4);
2. the interface values at t^{n+1} come from the Feynman-Kac Monte-Carlo
   solve (Sect. 3), with the current mesh as initial data (bilinear in the
   device grid) and the identity map as outer boundary data; with a trained
   network a control-variate form of the estimator is used (by default the
   martingale form, which stays unbiased when the network's gradient is
   taken only every `cv_stride` steps);
3. every sub-domain takes one implicit backward-Euler step with those
   interface values as Dirichlet data (Sect. 4);
4. the mesh quality (minimum Jacobian, maximum skewness) is recorded.

With `density_data="grid"` the density enters as the paper has it
(Sect. 4): sampled at t^n on the mesh's nodes, the drift from finite
differences at the nodes and bilinear between them, in both the interface
solve and the sub-domain solves.  With `key_points=True` only the key points
of each interface line (near the extrema of the first and second
derivatives of rho = 1/w along it, plus crossings and gap fill) are
simulated, and the other interface nodes follow from the monotone piecewise
cubic Hermite interpolant through the line's boundary data and key values
(Sect. 4, further speed-up; the paper's run, Sect. 5).

With `cv_form="grid"` the control is the mesh's own gradient (bilinear in
the grid, taken every `cv_stride` steps of each path) in the martingale
form: no network.  Otherwise the network is refitted every `refit_every`
steps; by default (`cv_base="mesh"`) the control is the mesh's own
interpolant plus the network, which fits the change of the mesh over one
step (new mesh minus the mesh it started from), so between refits it only
has to carry how the step's change moves, not the moving features
themselves.  The network is trained on labels
the run has produced (at their times t^{n+1}), starting from the initial mesh
at t = 0: either the interface estimates themselves, or (default) the mesh
values at the grid nodes within `band` of an interface line, where the paths
travel -- interface estimates fix the network along the lines only, while the
estimator needs its derivatives across them too.  All arithmetic runs in libfk.so
kernels on one stream; this module sequences the calls and keeps the label
buffers.  The run stays on the device between steps: nothing is copied to
the host until `qualities()` / `mesh()` are called.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import (FK_CV_DYNKIN, FK_CV_MARTINGALE, FK_CV_MARTINGALE_GRID, FkCv, GridDensity, fk_boundary_data,
               fk_density_sample, fk_interface_interpolate_mask, fk_interface_solve, fk_interface_solve_cv, fk_key_points,
               fk_mesh_quality, subdomain_solve, subdomain_workspace_bytes)

DATA_GRID = 3
DATA_IDENTITY = 0
SCORE_BRIDGE = 3
DATA_EQUIDISTRIBUTED = 4
KIND_TWO_BUMPS = 3
KIND_RING = 4
TIME_FROZEN = 1


@dataclass(frozen=True)
class MeshRunConfig:
    px: int = 8                 # px x px sub-domains
    m: int = 96                 # cells per sub-domain side; grid N = px m
    dt_mesh: float = 5e-4
    substeps: int = 20          # Euler-Maruyama steps per mesh step
    n_steps: int = 200
    n_paths: int = 1 << 14
    refit_every: int = 20       # 0: plain Monte Carlo throughout
    cv_form: str = "martingale"  # "dynkin"; or "grid": the martingale form with the mesh's own gradient
                                 # (no network, refit_every ignored)
    cv_base: str = "mesh"       # network forms: "mesh" -- the network fits the step's change of the mesh and
                                 # the control is the mesh's own interpolant plus it (martingale form only);
                                 # "none" -- the network fits the map itself
    cv_stride: int = 20
    train_steps: int = 2000
    train_batch: int = 8192
    lr: float = 1e-3
    t_scale: float = 0.1        # network time input range [0, t_scale]
    score_mode: int = 2         # exits: 2 the mesh extended past the edge; 1 projected; 0 unclamped identity
    labels: str = "band"        # "band": mesh values near the interfaces; "interface": the MC estimates
    band: float = 0.06          # half-width of the label band around each interface line
    band_stride: int = 3        # grid stride of the band samples
    label_levels: int = 40      # most recent label levels kept for training
    bdry: int = DATA_IDENTITY   # outer boundary data of the sub-domain solves (the mesh's edge nodes)
    density_data: str = "analytic"  # "grid": w sampled at t^n on the mesh's nodes only, drift by finite
                                    # differences there and bilinear in between (the paper's data path)
    key_points: bool = False    # simulate only the key points; interpolate the other interface nodes
    key_tol: float = 1e-2       # significance of a derivative extremum, relative to the line's largest
    key_gap: int = 0            # largest gap between knots along a line (0: m // 2)
    graph: bool = False         # record each step's device work as a HIP graph (an FkPlan) and replay it;
                                # plain or mesh-gradient runs (no network), on a stream of the run's own
    seed: int = 0


@dataclass(frozen=True)
class Density:
    """Fields of the C struct fk_density."""
    kind: int
    time_mode: int
    amp: float
    width2: float
    cx: float
    cy: float
    orbit_r: float
    omega: float
    t_freeze: float


@dataclass(frozen=True)
class GridData:
    """Fields of the C struct fk_data for grid initial data and identity
    boundary data (the grid pointers are passed separately).

    Exits are scored with the mesh continued bilinearly past the edge
    (FK_SCORE_EXTEND): the discrete exit test sees a path only after a
    step's overshoot of O(sqrt(dt)) beyond the edge, and scoring there is
    unbiased to first order only if the data are continued with the
    solution's own normal slope.  The identity continued unclamped has slope
    1 where a relaxed mesh meets the boundary at a very different slope, and
    a projected exit point drops the overshoot altogether; both bias the
    interface values next to the boundary -- on a 768-cell grid enough to
    fold the cells where an interface line meets the boundary.  The mesh's
    edge nodes hold the identity boundary data, so its continuation is that
    data extended by the mesh's slope."""
    t_init: float
    init_kind: int = DATA_GRID
    bdry_kind: int = DATA_IDENTITY
    score_mode: int = 2


def two_bump_density(t_freeze: float) -> Density:
    """Two counter-rotating bumps (amplitude 30, width^2 0.003, orbit radius
    1/4 about the centre, one turn per unit time) frozen at t_freeze."""
    return Density(KIND_TWO_BUMPS, TIME_FROZEN, amp=30.0, width2=0.003, cx=0.5, cy=0.5, orbit_r=0.25,
                   omega=2.0 * np.pi, t_freeze=t_freeze)


def paper_ring_density(t_freeze: float) -> Density:
    """The paper's density (Sect. 5): w = 1/rho, rho = 1 + 10 exp(-50 |r^2 - 1/100|),
    r the distance to (1/2 + cos(2 pi t)/4, 1/2 + sin(2 pi t)/4), frozen at t_freeze."""
    return Density(KIND_RING, TIME_FROZEN, amp=10.0, width2=-50.0, cx=0.5, cy=0.5, orbit_r=0.25,
                   omega=2.0 * np.pi, t_freeze=t_freeze)


# The paper's run (Sect. 5): 41 x 41 nodes in 2 x 2 sub-domains, mesh step
# 1e-3 in 20 sub-steps, 10^4 paths, up to t = 0.75, equidistributed edges;
# every interface node is simulated (no key points, no interpolation).
PAPER_RING_RUN = dict(px=2, m=20, dt_mesh=1e-3, substeps=20, n_steps=750, n_paths=10000, refit_every=0,
                      bdry=DATA_EQUIDISTRIBUTED, labels="interface")


def interface_nodes(px: int, m: int) -> np.ndarray:
    """Interface nodes of px x px sub-domains on the (px m)-cell grid, in the
    order the sub-domain solve reads its Dirichlet data (vertical lines, then
    horizontal lines without the crossings)."""
    N = px * m
    pts = [(a / px, j / N) for a in range(1, px) for j in range(1, N)]
    pts += [(i / N, c / px) for c in range(1, px) for i in range(1, N) if i % m]
    return np.array(pts, dtype=np.float64).reshape(-1, 2)


def band_index(px: int, m: int, band: float, stride: int) -> np.ndarray:
    """Flat grid indices j (N+1) + i of the nodes on every stride-th grid line
    that lie within `band` of an interface line x = a/px or y = c/px."""
    N = px * m
    k = np.arange(0, N + 1, stride)
    c = k / N
    lines = np.arange(1, px) / px
    near = np.abs(c[:, None] - lines[None, :]).min(1) <= band + 1e-12
    jj, ii = np.meshgrid(k, k, indexing="ij")
    mask = near[:, None] | near[None, :]
    return (jj[mask] * (N + 1) + ii[mask]).astype(np.int64)


class MeshRun:
    """The mesh-step driver on one GPU.

    `density_fn(t)` returns the density frozen at t (default: the two
    counter-rotating bumps).  `init_params` seeds the network (FP32 [8706]);
    it is required when refit_every > 0.
    """

    def __init__(self, cfg: MeshRunConfig, init_params=None, density_fn=two_bump_density, device="cuda"):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.dev = torch.device(device)
        self.density_fn = density_fn
        self.N = cfg.px * cfg.m
        self.pts_host = interface_nodes(cfg.px, cfg.m)
        self.n_nodes = self.pts_host.shape[0]
        self.pts = torch.tensor(self.pts_host, dtype=torch.float64, device=self.dev)
        x = torch.arange(self.N + 1, dtype=torch.float64, device=self.dev) / self.N
        self.xi = x.repeat(self.N + 1, 1).contiguous()            # [j][i] = x_i
        self.eta = x[:, None].repeat(1, self.N + 1).contiguous()  # [j][i] = y_j
        self.spare = (torch.empty_like(self.xi), torch.empty_like(self.eta))
        self.n = 0
        self._quality = torch.zeros((cfg.n_steps, 2), dtype=torch.float64, device=self.dev)
        # per step: (xi, eta) rows, written in place by the interface solve
        self._iface = torch.zeros((cfg.n_steps, 2, self.n_nodes), dtype=torch.float64, device=self.dev)
        self._se = torch.zeros((cfg.n_steps, 2, self.n_nodes), dtype=torch.float64, device=self.dev)
        self.cv = None
        self.used_cv = np.zeros(cfg.n_steps, dtype=bool)
        self.workspace = None
        self.sub_workspace = torch.empty(max(subdomain_workspace_bytes(cfg.px, cfg.m), 256), dtype=torch.uint8,
                                         device=self.dev)
        # step counts of the interface solves (device; keeps the solves from allocating one)
        self._total_steps = torch.zeros((cfg.n_steps, 1), dtype=torch.int64, device=self.dev)
        self.plan = None
        if cfg.graph:
            if cfg.refit_every > 0 and cfg.cv_form != "grid":
                raise ValueError("graph mode records plain or mesh-gradient steps (no network)")
            from . import FkPlan, fk_interface_cv_grid_workspace_bytes, fk_interface_workspace_bytes
            self.plan = FkPlan()
            self.stream = torch.cuda.Stream(device=self.dev)
            # every buffer a step uses exists before its capture
            need = (fk_interface_cv_grid_workspace_bytes(self.n_nodes, cfg.n_paths, self.N)
                    if cfg.cv_form == "grid" else fk_interface_workspace_bytes(self.n_nodes, cfg.n_paths))
            self.workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=self.dev)
        self.losses = []
        if cfg.density_data not in ("analytic", "grid"):
            raise ValueError("density_data must be 'analytic' or 'grid'")
        if cfg.density_data == "grid" or cfg.key_points:
            self._wg = torch.empty((self.N + 1, self.N + 1), dtype=torch.float64, device=self.dev)
        if cfg.density_data == "grid":
            self._wb = torch.empty((self.N + 1, self.N + 1, 2), dtype=torch.float32, device=self.dev)
        if cfg.key_points:
            # each step's key-point mask; standard errors exist at the key points only
            self._masks = torch.zeros((cfg.n_steps, self.n_nodes), dtype=torch.uint8, device=self.dev)
            self._se.fill_(float("nan"))
            from . import fk_boundary_workspace_bytes
            self._bdry_ws = torch.empty(max(fk_boundary_workspace_bytes(self.N), 256), dtype=torch.uint8,
                                        device=self.dev)
        if cfg.refit_every > 0 and cfg.cv_form != "grid":
            if init_params is None:
                raise ValueError("refit_every > 0 needs initial network parameters")
            if cfg.cv_base not in ("mesh", "none"):
                raise ValueError("cv_base must be 'mesh' or 'none'")
            if cfg.cv_base == "mesh" and cfg.cv_form != "martingale":
                raise ValueError("the mesh base needs the martingale form")
            self._mesh_base = cfg.cv_base == "mesh"
            self.cv = FkCv(init_params, cfg.t_scale, base="grid" if self._mesh_base else "none")
            if cfg.labels == "interface":
                lab_pts = self.pts_host
                self._band_idx = None
                ij = np.rint(self.pts_host * self.N).astype(np.int64)
                self._iface_idx = torch.tensor(ij[:, 1] * (self.N + 1) + ij[:, 0], dtype=torch.int64,
                                               device=self.dev)
            elif cfg.labels == "band":
                idx = band_index(cfg.px, cfg.m, cfg.band, cfg.band_stride)
                lab_pts = np.stack([idx % (self.N + 1), idx // (self.N + 1)], 1) / self.N
                self._band_idx = torch.tensor(idx, dtype=torch.int64, device=self.dev)
            else:
                raise ValueError("labels must be 'band' or 'interface'")
            # label ring: level-major (t, x, y) and (xi, eta); level 0 is the initial mesh
            L, n_lab = cfg.label_levels, lab_pts.shape[0]
            self._lab_txy = torch.zeros((L, n_lab, 3), dtype=torch.float32, device=self.dev)
            self._lab_val = torch.zeros((L, n_lab, 2), dtype=torch.float32, device=self.dev)
            self._lab_count = 0
            p = torch.tensor(lab_pts, dtype=torch.float32, device=self.dev)
            self._lab_pts = p
            if self._mesh_base:
                # the initial mesh does not change before the first step
                self._add_labels(0.0, torch.zeros_like(p[:, 0]), torch.zeros_like(p[:, 1]))
            else:
                self._add_labels(0.0, p[:, 0], p[:, 1])

    @property
    def n_keys(self):
        """Key points simulated in each step taken (a host list; reading it
        synchronises with the device)."""
        if not self.cfg.key_points:
            return []
        return [int(v) for v in self._masks[:self.n].sum(1, dtype=self.torch.int64).cpu()]

    @property
    def _mask(self):
        """The last step's key-point mask."""
        return self._masks[max(self.n - 1, 0)]

    # -- labels ----------------------------------------------------------------
    def _add_labels(self, t, xi, eta):
        L = self.cfg.label_levels
        slot = self._lab_count % L
        self._lab_txy[slot, :, 0] = float(t)
        self._lab_txy[slot, :, 1:] = self._lab_pts
        self._lab_val[slot, :, 0] = xi.to(self.torch.float32)
        self._lab_val[slot, :, 1] = eta.to(self.torch.float32)
        self._lab_count += 1

    def refit(self):
        """Train the network on the label levels held (Adam state carries over)."""
        k = min(self._lab_count, self.cfg.label_levels)
        txy = self._lab_txy[:k].reshape(-1, 3)
        val = self._lab_val[:k].reshape(-1, 2)
        loss = self.cv.train(txy, val, steps=self.cfg.train_steps, batch=self.cfg.train_batch, lr=self.cfg.lr,
                             seed=self.cfg.seed + 7919 * (self.n + 1))
        self.losses.append(loss)

    # -- one mesh step -----------------------------------------------------------
    def step(self):
        cfg = self.cfg
        if self.n >= cfg.n_steps:
            raise RuntimeError("the run has taken all its steps")
        if self.plan is None:
            self._step_body()
        else:
            # record the step's device work (its time level and buffers), run
            # it as a graph, and hand its results to the caller's stream
            torch = self.torch
            caller = torch.cuda.current_stream(self.dev)
            self.stream.wait_stream(caller)
            with torch.cuda.stream(self.stream):
                with self.plan.capture(self.dev):
                    self._step_body(advance=False)
                self.plan.replay(self.dev)
            caller.wait_stream(self.stream)
            self._advance()

    def _step_body(self, advance=True):
        cfg = self.cfg
        tn = self.n * cfg.dt_mesh
        dens = self.density_fn(tn)
        if cfg.density_data == "grid" or cfg.key_points:
            fk_density_sample(dens, tn, self.N, out=self._wg)
        if cfg.density_data == "grid":
            dens = GridDensity(self._wg, grid_b=self._wb)
        data = GridData(t_init=tn, score_mode=cfg.score_mode)
        grids = (self.xi.view(-1), self.eta.view(-1))
        if self.cv is not None and self.n % cfg.refit_every == 0:
            self.refit()
        dt = cfg.dt_mesh / cfg.substeps
        # the solve writes the history rows in place; with key points it
        # simulates the masked nodes only (the mask stays on the device: no
        # host synchronisation in the step)
        rows = {"xi": self._iface[self.n, 0], "eta": self._iface[self.n, 1],
                "se_xi": self._se[self.n, 0], "se_eta": self._se[self.n, 1],
                "total_steps": self._total_steps[self.n]}
        mask = None
        if cfg.key_points:
            mask = self._masks[self.n]
            fk_key_points(self._wg, cfg.px, cfg.m, cfg.key_tol, cfg.key_gap or None, out=mask)
        if cfg.cv_form == "grid":
            out = fk_interface_solve_cv(dens, data, self.pts, cfg.dt_mesh, dt, cfg.n_paths, None,
                                        stride=cfg.cv_stride, seed=cfg.seed, level_id=self.n,
                                        form=FK_CV_MARTINGALE_GRID, plain=False, device=self.dev,
                                        workspace=self.workspace, grids=grids, out=rows, mask=mask)
            self.used_cv[self.n] = True
        elif self.cv is not None:
            form = FK_CV_MARTINGALE if cfg.cv_form == "martingale" else FK_CV_DYNKIN
            out = fk_interface_solve_cv(dens, data, self.pts, cfg.dt_mesh, dt, cfg.n_paths, self.cv,
                                        stride=cfg.cv_stride, seed=cfg.seed, level_id=self.n, form=form,
                                        plain=False, device=self.dev, workspace=self.workspace, grids=grids,
                                        out=rows, mask=mask)
            self.used_cv[self.n] = True
        else:
            out = fk_interface_solve(dens, data, self.pts, cfg.dt_mesh, dt, cfg.n_paths, seed=cfg.seed,
                                     level_id=self.n, device=self.dev, workspace=self.workspace, grids=grids,
                                     out=rows, mask=mask)
        self.workspace = out["_workspace"]
        iface_xi, iface_eta = out["xi"], out["eta"]
        if cfg.key_points:
            # the line ends: this step's outer boundary data, in the grids the
            # sub-domain solve then fills
            self._bdry_ws = fk_boundary_data(dens, tn, self.N, cfg.bdry, self.spare[0], self.spare[1],
                                             workspace=self._bdry_ws)
            fk_interface_interpolate_mask(cfg.px, cfg.m, mask, self.spare[0], self.spare[1], iface_xi, iface_eta)
        xi_new, eta_new = subdomain_solve(dens, tn, cfg.dt_mesh, cfg.px, cfg.m, self.xi, self.eta, iface_xi,
                                          iface_eta, bdry_kind=cfg.bdry, out=self.spare,
                                          workspace=self.sub_workspace)
        fk_mesh_quality(xi_new, eta_new, out=self._quality[self.n])
        if self.cv is not None:
            if self._band_idx is None:
                lx, ly = iface_xi, iface_eta
                if self._mesh_base:
                    # the interface nodes lie on the grid: the step's change there
                    lx = lx - self.xi.view(-1)[self._iface_idx]
                    ly = ly - self.eta.view(-1)[self._iface_idx]
                self._add_labels(tn + cfg.dt_mesh, lx, ly)
            else:
                lx, ly = xi_new.view(-1)[self._band_idx], eta_new.view(-1)[self._band_idx]
                if self._mesh_base:
                    lx = lx - self.xi.view(-1)[self._band_idx]
                    ly = ly - self.eta.view(-1)[self._band_idx]
                self._add_labels(tn + cfg.dt_mesh, lx, ly)
        if advance:
            self._advance()

    def _advance(self):
        # the new mesh becomes the current one; the old one the next output
        self.spare, (self.xi, self.eta) = (self.xi, self.eta), self.spare
        self.n += 1

    def run(self, n_steps=None):
        for _ in range(self.cfg.n_steps - self.n if n_steps is None else n_steps):
            self.step()

    # -- results (these synchronise) ---------------------------------------------
    def qualities(self) -> np.ndarray:
        """[steps taken, 2]: minimum Jacobian and maximum skewness after each step."""
        return self._quality[:self.n].cpu().numpy()

    def interface_values(self):
        """([steps, nodes, 2] interface values, [steps, nodes, 2] standard
        errors; with key points, NaN at the interpolated nodes)."""
        return (self._iface[:self.n].transpose(1, 2).cpu().numpy(),
                self._se[:self.n].transpose(1, 2).cpu().numpy())

    def mesh(self):
        """The current (xi, eta) grids on the host, [N+1, N+1] each, indexed [j][i]."""
        return self.xi.cpu().numpy(), self.eta.cpu().numpy()

    def close(self):
        if self.cv is not None:
            self.cv.close()
            self.cv = None


def steady_mesh(density, px: int, m: int, n_paths: int, dt: float, horizon: float, bdry: int = DATA_IDENTITY,
                seed: int = 0, device="cuda"):
    """The elliptic (steady) stochastic domain decomposition (eq. (2)) for a
    static density: the interface values are Feynman-Kac estimates of the
    steady system -- paths run until they leave the square, found by the
    Brownian-bridge exit test and scored with the outer boundary data at the
    crossing; `horizon` only caps the rare long path, which then scores the
    start grid (the identity map with the boundary data on its edges) --
    then each sub-domain solves the steady system with those values as
    Dirichlet data.  Returns a dict of device tensors: xi, eta (the mesh),
    iface_xi, iface_eta, se_xi, se_eta, and `survivors` (paths capped by the
    horizon)."""
    import torch
    from . import fk_boundary_data
    dev = torch.device(device)
    N = px * m
    x = torch.arange(N + 1, dtype=torch.float64, device=dev) / N
    sx = x.repeat(N + 1, 1).contiguous()
    sy = x[:, None].repeat(1, N + 1).contiguous()
    fk_boundary_data(density, 0.0, N, bdry, sx, sy)          # edge nodes: the boundary data
    data = GridData(t_init=0.0, bdry_kind=DATA_GRID, score_mode=SCORE_BRIDGE)
    out = fk_interface_solve(density, data, interface_nodes(px, m), horizon, dt, n_paths, seed=seed, exit_step=True,
                             device=dev, grids=(sx.view(-1), sy.view(-1)))
    xi, eta = subdomain_solve(density, 0.0, float("inf"), px, m, None, None, out["xi"], out["eta"], bdry_kind=bdry)
    return {"xi": xi, "eta": eta, "iface_xi": out["xi"], "iface_eta": out["eta"], "se_xi": out["se_xi"],
            "se_eta": out["se_eta"], "survivors": (out["exit_step"] < 0).sum(), "start": (sx, sy)}
