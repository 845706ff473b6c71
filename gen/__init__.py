"""Seeded synthetic inputs for the shallow-water step.

This module only draws random numbers and evaluates input fields (bed z, Manning n, initial
depth) at triangle centroids.  It holds none of the solver's arithmetic: no fluxes, no
geometry of the scheme, no time stepping.  Both the product path and the CPU oracle are fed
from here, which is the only code they share.

The paper's own meshes (Table 2: 1,036 to 10,261,932 triangles) and water-drop parameters
(section 3, Fig. 5) are not available, so these generators stand in for them: jittered
split-square triangulations with the same connectivity ratios (E/T ~ 1.5, V/T ~ 0.5) and the
same size range.

Random streams are ``numpy.random.default_rng([config, stream])`` with
stream 0 = diagonals, 1 = jitter, 2 = bed, 3 = Manning n, 4 = gauges, 5 = hidden n,
6 = scenario parameters.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

G = 9.81
COURANT = 0.7          # section 2.2: Courant number of the CFL condition
H_DRY = 1e-6           # dry threshold (m)

STREAM_DIAG, STREAM_JITTER, STREAM_BED, STREAM_N, STREAM_GAUGE, STREAM_HIDDEN, STREAM_SCEN = range(7)


def _rng(cfg, stream, *extra):
    return np.random.default_rng([int(cfg), int(stream), *map(int, extra)])


@dataclasses.dataclass
class Case:
    """One synthetic problem: a raw triangle list plus per-cell fields, all in input order."""
    name: str
    xy: np.ndarray          # float64 [V, 2] node coordinates
    tri: np.ndarray         # int32 [T, 3] node ids, counter-clockwise
    z: np.ndarray           # float64 [T] bed elevation at centroids
    n: np.ndarray           # float64 [T] Manning coefficient
    h: np.ndarray           # float64 [T] initial depth
    hu: np.ndarray          # float64 [T]
    hv: np.ndarray          # float64 [T]
    steps: int              # step count of the configuration
    g: float = G
    courant: float = COURANT
    h_dry: float = H_DRY
    edge_tag: np.ndarray | None = None   # int32 [T, 3]: 0 wall, k>=1 inflow segment k
    inflow_q: np.ndarray | None = None   # float64 [K]: unit discharge of inflow segment k
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])


def split_square_mesh(nx: int, ny: int, lx: float, ly: float, cfg: int, jitter: float = 0.2,
                      x0: float = 0.0, y0: float = 0.0, seed_extra=()):
    """Jittered split-square triangulation of [x0, x0+lx] x [y0, y0+ly].

    nx * ny squares, each split along a random diagonal (p = 1/2), two triangles per square in
    row-major square order.  Interior nodes move by U(-jitter, jitter) of the cell size in x
    and y; boundary nodes stay put.  With jitter <= 0.2 every triangle stays counter-clockwise
    with area >= 0.1 dx dy.
    """
    dx, dy = lx / nx, ly / ny
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    x = x0 + ii * dx
    y = y0 + jj * dy
    rj = _rng(cfg, STREAM_JITTER, *seed_extra)
    jx = rj.uniform(-jitter, jitter, size=x.shape)
    jy = rj.uniform(-jitter, jitter, size=y.shape)
    interior = (ii > 0) & (ii < nx) & (jj > 0) & (jj < ny)
    x = np.where(interior, x + jx * dx, x)
    y = np.where(interior, y + jy * dy, y)
    xy = np.stack([x.ravel(), y.ravel()], axis=1).astype(np.float64)

    si, sj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    a = (sj * (nx + 1) + si).ravel()
    b = a + 1
    c = a + (nx + 1) + 1
    d = a + (nx + 1)
    diag_ac = (_rng(cfg, STREAM_DIAG, *seed_extra).random(nx * ny) < 0.5)
    t0 = np.where(diag_ac[:, None], np.stack([a, b, c], 1), np.stack([a, b, d], 1))
    t1 = np.where(diag_ac[:, None], np.stack([a, c, d], 1), np.stack([b, c, d], 1))
    tri = np.stack([t0, t1], axis=1).reshape(-1, 3).astype(np.int32)
    return xy, tri


def centroids(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Centroid of each triangle, used only to evaluate input fields."""
    return (xy[tri[:, 0]] + xy[tri[:, 1]] + xy[tri[:, 2]]) / 3.0


def gaussian_bumps(cxy: np.ndarray, rng, count: int, lx: float, ly: float, x0=0.0, y0=0.0,
                   amp=(0.5, 3.0), width=(20.0, 150.0)) -> np.ndarray:
    """Sum of `count` bumps A exp(-r^2 / w^2), A ~ U(amp), w ~ U(width), centres ~ U(box)."""
    a = rng.uniform(*amp, size=count)
    w = rng.uniform(*width, size=count)
    bx = rng.uniform(x0, x0 + lx, size=count)
    by = rng.uniform(y0, y0 + ly, size=count)
    z = np.zeros(cxy.shape[0])
    for k in range(count):
        r2 = (cxy[:, 0] - bx[k]) ** 2 + (cxy[:, 1] - by[k]) ** 2
        z += a[k] * np.exp(-r2 / (w[k] * w[k]))
    return z


def dam_break(nx=100, ny=50, lx=20.0, ly=10.0, cfg=1, steps=200, h_left=1.0, h_right=0.1,
              x_dam=None, jitter=0.2) -> Case:
    """Flat-bed frictionless dam break (config 1 at its default sizes: 10,000 triangles)."""
    xy, tri = split_square_mesh(nx, ny, lx, ly, cfg, jitter=jitter)
    c = centroids(xy, tri)
    x_dam = lx / 2 if x_dam is None else x_dam
    t = tri.shape[0]
    h = np.where(c[:, 0] < x_dam, h_left, h_right).astype(np.float64)
    return Case(f"dam_break_{t}", xy, tri, np.zeros(t), np.zeros(t), h, np.zeros(t),
                np.zeros(t), steps, extra={"x_dam": x_dam, "h_left": h_left, "h_right": h_right})


def wetdry(nx=1000, ny=500, lx=2000.0, ly=1000.0, cfg=2, steps=1000, n_bumps=8,
           eta_left=2.0, eta_right=0.5, x_split=None) -> Case:
    """Wet/dry flow with friction over Gaussian bumps (config 2 at its default sizes: 1e6)."""
    xy, tri = split_square_mesh(nx, ny, lx, ly, cfg)
    c = centroids(xy, tri)
    z = gaussian_bumps(c, _rng(cfg, STREAM_BED), n_bumps, lx, ly)
    n = _rng(cfg, STREAM_N).uniform(0.02, 0.05, size=tri.shape[0])
    x_split = lx / 4 if x_split is None else x_split
    eta = np.where(c[:, 0] < x_split, eta_left, eta_right)
    h = np.maximum(eta - z, 0.0)
    t = tri.shape[0]
    return Case(f"wetdry_{t}", xy, tri, z, n, h, np.zeros(t), np.zeros(t), steps)


def water_drop(nx=3125, ny=1600, lx=10000.0, ly=5000.0, cfg=3, steps=500, n_bumps=64,
               slope=1e-3, hump=2.0, hump_w=200.0) -> Case:
    """Gaussian hump of water over a sloping bumpy bed (config 3 at its default sizes: 1e7)."""
    xy, tri = split_square_mesh(nx, ny, lx, ly, cfg)
    c = centroids(xy, tri)
    z = slope * c[:, 0] + gaussian_bumps(c, _rng(cfg, STREAM_BED), n_bumps, lx, ly)
    n = _rng(cfg, STREAM_N).uniform(0.015, 0.06, size=tri.shape[0])
    r2 = (c[:, 0] - lx / 2) ** 2 + (c[:, 1] - ly / 2) ** 2
    h = 1.0 + hump * np.exp(-r2 / (hump_w * hump_w))
    t = tri.shape[0]
    return Case(f"water_drop_{t}", xy, tri, z, n, h, np.zeros(t), np.zeros(t), steps)


def lake_at_rest(nx=120, ny=60, lx=240.0, ly=120.0, cfg=12, eta=1.0, n_bumps=8, steps=1000,
                 with_friction=True) -> Case:
    """Still water at level eta over bumps that rise above it (dry islands)."""
    xy, tri = split_square_mesh(nx, ny, lx, ly, cfg)
    c = centroids(xy, tri)
    z = gaussian_bumps(c, _rng(cfg, STREAM_BED), n_bumps, lx, ly, width=(lx / 40, lx / 8))
    t = tri.shape[0]
    n = (_rng(cfg, STREAM_N).uniform(0.02, 0.05, size=t) if with_friction else np.zeros(t))
    h = np.maximum(eta - z, 0.0)
    return Case(f"lake_at_rest_{t}", xy, tri, z, n, h, np.zeros(t), np.zeros(t), steps,
                extra={"eta": eta})


def config(k: int) -> Case:
    """Configurations 1, 2, 3 and 5 at their full sizes."""
    if k == 1:
        return dam_break()
    if k == 2:
        return wetdry()
    if k == 3:
        return water_drop()
    if k == 5:
        return calibration()
    raise ValueError(f"no single-mesh configuration {k}")


def small(k: int) -> Case:
    """The recipe of configuration k at a size the oracle finishes in seconds.

    Each still spans many 256-cell tiles and ends in a ragged tail.
    """
    if k == 1:
        return dam_break()                                   # 10,000 cells = 39 tiles + 16
    if k == 2:
        return wetdry(nx=90, ny=45, lx=2000.0, ly=1000.0, steps=300)      # 8,100 cells
    if k == 3:
        return water_drop(nx=100, ny=51, lx=2000.0, ly=1020.0, steps=200, n_bumps=16)
    if k == 5:
        return calibration(nx=60, ny=30, steps=200)
    raise ValueError(k)


# ---------------------------------------------------------------- config 5: calibration
def random_fourier_field(cxy: np.ndarray, rng, modes=256, length=150.0) -> np.ndarray:
    """Unit-variance stationary random field sqrt(2/M) sum cos(k.x + phi), k ~ N(0, I/l^2)."""
    k = rng.normal(0.0, 1.0 / length, size=(modes, 2))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    acc = np.zeros(cxy.shape[0])
    for m in range(modes):
        acc += np.cos(cxy[:, 0] * k[m, 0] + cxy[:, 1] * k[m, 1] + phi[m])
    return math.sqrt(2.0 / modes) * acc


def calibration(nx=500, ny=250, lx=2000.0, ly=1000.0, cfg=5, steps=2000, n_gauges=64) -> Case:
    """Config-2-style mesh, bed and initial state with a hidden smooth Manning field.

    extra: 'n_hidden' (the field observations come from), 'gauges' (64 cells wet at t=0),
    'n0' (the uniform first guess 0.03).
    """
    xy, tri = split_square_mesh(nx, ny, lx, ly, cfg)
    c = centroids(xy, tri)
    z = gaussian_bumps(c, _rng(cfg, STREAM_BED), 8, lx, ly)
    eta = np.where(c[:, 0] < lx / 4, 2.0, 0.5)
    h = np.maximum(eta - z, 0.0)
    xi = random_fourier_field(c, _rng(cfg, STREAM_HIDDEN))
    n_hidden = np.clip(0.03 + 0.008 * xi, 0.01, 0.06)
    wet = np.flatnonzero(h > H_DRY)
    gauges = np.sort(_rng(cfg, STREAM_GAUGE).choice(wet, size=min(n_gauges, wet.size),
                                                     replace=False)).astype(np.int32)
    t = tri.shape[0]
    n0 = np.full(t, 0.03)
    return Case(f"calibration_{t}", xy, tri, z, n0, h, np.zeros(t), np.zeros(t), steps,
                extra={"n_hidden": n_hidden, "gauges": gauges, "obs_every": 10, "ckpt_every": 50})


# ---------------------------------------------------------------- config 4: ensemble
def ensemble_scenario(s: int, cfg=4, t_min=5e3, t_max=2e5, steps=2000) -> Case:
    """Scenario s of the batched ensemble: own box, seed, roughness and inflow segment."""
    rp = _rng(cfg, STREAM_SCEN, s)
    t_target = math.exp(rp.uniform(math.log(t_min), math.log(t_max)))
    ny = max(2, int(round(math.sqrt(t_target / 4.0))))
    nx = 2 * ny
    delta = rp.uniform(1.0, 4.0)
    n_val = rp.uniform(0.02, 0.05)
    q_in = rp.uniform(5.0, 50.0)
    lx, ly = nx * delta, ny * delta
    xy, tri = split_square_mesh(nx, ny, lx, ly, cfg, seed_extra=(s,))
    c = centroids(xy, tri)
    scale = lx / 2000.0
    z = gaussian_bumps(c, _rng(cfg, STREAM_BED, s), 8, lx, ly,
                       width=(20.0 * scale, 150.0 * scale))
    h = np.maximum(1.0 - z, 0.0)
    t = tri.shape[0]
    n = np.full(t, n_val)
    # inflow segment: boundary edges on x = 0 whose midpoint lies in the centred tenth of ly
    tag = np.zeros((t, 3), dtype=np.int32)
    for k in range(3):
        a = xy[tri[:, k]]
        b = xy[tri[:, (k + 1) % 3]]
        on_left = (a[:, 0] == 0.0) & (b[:, 0] == 0.0)
        ym = 0.5 * (a[:, 1] + b[:, 1])
        seg = on_left & (np.abs(ym - ly / 2) <= 0.05 * ly)
        tag[seg, k] = 1
    return Case(f"ensemble_{s}_{t}", xy, tri, z, n, h, np.zeros(t), np.zeros(t), steps,
                edge_tag=tag, inflow_q=np.array([q_in]),
                extra={"scenario": s, "q_in": q_in, "delta": delta})


def ensemble(count=256, **kw) -> list[Case]:
    return [ensemble_scenario(s, **kw) for s in range(count)]


def strip(nx: int, lx=20.0, ly=None, ny=2, cfg=21, jitter=0.0, **kw) -> Case:
    """Dam break on a narrow strip mesh (for closed-form 1D solutions)."""
    ly = lx / nx * ny if ly is None else ly
    return dam_break(nx=nx, ny=ny, lx=lx, ly=ly, cfg=cfg, jitter=jitter, **kw)


def three_mounds(nx=120, ny=48, lx=60.0, ly=24.0, cfg=41, steps=600, eta0=1.5, x_dam=12.0,
                 n_manning=0.02) -> Case:
    """Wet/dry validation workload: a reservoir released over a dry floor with three mounds.

    Parameters chosen for this suite (not a published geometry): 60 m x 24 m walled box, still
    water at eta0 = 1.5 m behind x = 12 m, dry beyond; one tall mound (2.5 m high, 8 m wide) at
    (40, 12) whose top never floods early, two low ones (1 m, 5 m) at (25, 6) and (25, 18) that
    the wave overtops; uniform Manning n."""
    xy, tri = split_square_mesh(nx, ny, lx, ly, cfg)
    c = centroids(xy, tri)
    z = np.zeros(tri.shape[0])
    for (bx, by, a, w) in ((40.0, 12.0, 2.5, 8.0), (25.0, 6.0, 1.0, 5.0), (25.0, 18.0, 1.0, 5.0)):
        z = z + a * np.exp(-((c[:, 0] - bx) ** 2 + (c[:, 1] - by) ** 2) / (w * w))
    h = np.where(c[:, 0] < x_dam, np.maximum(eta0 - z, 0.0), 0.0)
    t = tri.shape[0]
    return Case(f"three_mounds_{t}", xy, tri, z, np.full(t, n_manning), h, np.zeros(t),
                np.zeros(t), steps, extra={"eta0": eta0, "x_dam": x_dam})
