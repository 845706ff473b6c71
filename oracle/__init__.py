"""Plain FP64 CPU oracle of the shallow-water step (TEST INFRASTRUCTURE).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The product library never does, and this package imports nothing from
the product.  The arithmetic lives in ``swe_oracle.c`` (plain C, FP64, no contraction); this
module compiles it with gcc and marshals numpy arrays through ctypes.

Oracle functions and the passages of the paper they follow (section 2 of Zaoui 2016):
  ``Mesh``          triangles, interfaces and geometry (section 2.2, eq. 3, Fig. 1)
  ``hllc``          HLLC interface flux (section 2.2, ref. [6])
  ``interface``     hydrostatic reconstruction of the bed around the flux (section 2.2)
  ``wall``          reflective wall as a mirror ghost (section 3)
  ``inflow``        prescribed unit discharge through a boundary edge (not in the paper: the
                    ensemble's inflow segments; boundary state read as critical or deeper flow)
  ``run``           explicit Euler steps of eq. 4 with CFL dt (Courant 0.7), friction
                    (S_f of eq. 1) and the host time loop of section 2.3
  ``run_loss_sig``  the same steps with a replayed dt, the gauge misfit and a signature of
                    the branches taken (finite differences are compared only between runs
                    that took the same branches)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "swe_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, EMESH, ENONFINITE, EDRY = 0, -1, -2, -4, -5

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Params(C.Structure):
    _fields_ = [("g", C.c_double), ("courant", C.c_double), ("h_dry", C.c_double),
                ("n_inflow", C.c_int), ("inflow_q", _dp)]


class _Stats(C.Structure):
    _fields_ = [("t", C.c_double), ("steps", C.c_long), ("clamps", C.c_long),
                ("clamped_mass", C.c_double), ("dt_min", C.c_double), ("dt_max", C.c_double),
                ("dt_sum", C.c_double), ("last_reached", C.c_int)]


def build(src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle: FP64, every operation rounded separately, OpenMP for the loops."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib = None


def lib(path: str | None = None):
    """Load the compiled oracle (building it first if it is missing or older than its source)."""
    global _lib
    if path is not None:
        return _bind(C.CDLL(path))
    if _lib is None:
        alt = os.environ.get("SWE_ORACLE_LIB")   # a planted-mistake build (mutation tests)
        if alt:
            _lib = _bind(C.CDLL(alt))
            return _lib
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = _bind(C.CDLL(LIB))
    return _lib


def _bind(L):
    L.om_mesh_build.argtypes = [_dp, C.c_long, _ip, C.c_long, _ip, C.POINTER(C.c_void_p)]
    L.om_mesh_build.restype = C.c_int
    L.om_mesh_free.argtypes = [C.c_void_p]
    L.om_mesh_counts.argtypes = [C.c_void_p, C.POINTER(C.c_long)]
    L.om_mesh_arrays.argtypes = [C.c_void_p, _ip, _ip, _dp, _dp]
    L.om_cfl_dt.argtypes = [C.c_void_p, _dp, _dp, _dp, C.POINTER(_Params)]
    L.om_cfl_dt.restype = C.c_double
    L.om_run.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, C.POINTER(_Params), C.c_long,
                         C.c_double, _dp, _dp, C.POINTER(_Stats)]
    L.om_run.restype = C.c_int
    L.om_hllc_batch.argtypes = [C.c_long, C.c_double] + [_dp] * 9
    L.om_interface_batch.argtypes = [C.c_long, C.c_double, C.c_double] + [_dp] * 13
    L.om_wall_batch.argtypes = [C.c_long, C.c_double, C.c_double] + [_dp] * 7
    L.om_wave_speeds_batch.argtypes = [C.c_long, C.c_double] + [_dp] * 6
    L.om_inflow_batch.argtypes = [C.c_long, C.c_double] + [_dp] * 6
    L.om_run_tl.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                            C.POINTER(_Params), C.c_long, _dp, _ip, C.c_int, C.c_int, _dp, _dp,
                            _dp]
    L.om_run_tl.restype = C.c_int
    L.om_run_loss.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, C.POINTER(_Params), C.c_long,
                              _dp, _ip, C.c_int, C.c_int, _dp, _dp]
    L.om_run_loss.restype = C.c_int
    L.om_run_loss_sig.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, C.POINTER(_Params),
                                  C.c_long, _dp, _ip, C.c_int, C.c_int, _dp, _dp,
                                  C.POINTER(C.c_ulong)]
    L.om_run_loss_sig.restype = C.c_int
    L.om_set_threads.argtypes = [C.c_int]
    L.om_get_threads.restype = C.c_int
    return L


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def set_threads(n: int) -> None:
    lib().om_set_threads(int(n))


def threads() -> int:
    return int(lib().om_get_threads())


class Mesh:
    """The oracle's own connectivity and geometry (section 2.2, eq. 3, Fig. 1)."""

    def __init__(self, xy, tri, edge_tag=None):
        self.xy = _d(xy).reshape(-1, 2)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
        tags = None if edge_tag is None else np.ascontiguousarray(edge_tag, np.int32).reshape(-1, 3)
        self._tags = tags
        h = C.c_void_p()
        rc = lib().om_mesh_build(self.xy.ctypes.data_as(_dp), self.xy.shape[0],
                                 self.tri.ctypes.data_as(_ip), self.tri.shape[0],
                                 None if tags is None else tags.ctypes.data_as(_ip), C.byref(h))
        if rc != OK:
            raise ValueError(f"oracle mesh build failed: {rc}")
        self._h = h
        cnt = (C.c_long * 4)()
        lib().om_mesh_counts(h, cnt)
        self.n_cells, self.n_nodes, self.n_edges, self.n_boundary = (int(v) for v in cnt)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.om_mesh_free(self._h)
            self._h = None

    def arrays(self):
        """(cell_node [T,3] counter-clockwise, cell_nbr [T,3], area [T], inradius [T])."""
        t = self.n_cells
        cn = np.empty((t, 3), np.int32)
        nb = np.empty((t, 3), np.int32)
        a = np.empty(t)
        r = np.empty(t)
        lib().om_mesh_arrays(self._h, cn.ctypes.data_as(_ip), nb.ctypes.data_as(_ip),
                             a.ctypes.data_as(_dp), r.ctypes.data_as(_dp))
        return cn, nb, a, r


def _params(g, courant, h_dry, inflow_q):
    q = None if inflow_q is None else _d(inflow_q)
    p = _Params(g, courant, h_dry, 0 if q is None else q.size, _ptr(q))
    return p, q


def cfl_dt(mesh: Mesh, h, hu, hv, g=9.81, courant=0.7, h_dry=1e-6, inflow_q=None) -> float:
    h, hu, hv = _d(h), _d(hu), _d(hv)
    p, _keep = _params(g, courant, h_dry, inflow_q)
    return float(lib().om_cfl_dt(mesh._h, _ptr(h), _ptr(hu), _ptr(hv), C.byref(p)))


def run(mesh: Mesh, z, n, h, hu, hv, steps: int, g=9.81, courant=0.7, h_dry=1e-6,
        t0=0.0, t_end=0.0, dt_seq=None, inflow_q=None):
    """Advance (h, hu, hv) by up to `steps` steps; returns (rc, h, hu, hv, dts, stats)."""
    z, n = _d(z), _d(n)
    h, hu, hv = _d(h).copy(), _d(hu).copy(), _d(hv).copy()
    dts = np.zeros(max(int(steps), 1))
    seq = None if dt_seq is None else _d(dt_seq)
    p, _keep = _params(g, courant, h_dry, inflow_q)
    st = _Stats(t0, 0, 0, 0.0, 0.0, 0.0, 0.0, 0)
    rc = lib().om_run(mesh._h, _ptr(z), _ptr(n), _ptr(h), _ptr(hu), _ptr(hv), C.byref(p),
                      int(steps), float(t_end), _ptr(seq), _ptr(dts), C.byref(st))
    stats = {k: getattr(st, k) for k, _ in _Stats._fields_}
    return rc, h, hu, hv, dts[: st.steps], stats


def run_case(case, steps=None, mesh: Mesh | None = None, **kw):
    """Run a `gen.Case` from its initial state; returns the same tuple as `run`."""
    mesh = mesh or Mesh(case.xy, case.tri, case.edge_tag)
    kw.setdefault("g", case.g)
    kw.setdefault("courant", case.courant)
    kw.setdefault("h_dry", case.h_dry)
    kw.setdefault("inflow_q", case.inflow_q)
    return run(mesh, case.z, case.n, case.h, case.hu, case.hv,
               case.steps if steps is None else steps, **kw)


def hllc(hl, ul, vl, hr, ur, vr, nx, ny, g=9.81):
    """Vectorised HLLC flux (x, y components) for already reconstructed depths; [N, 3]."""
    a = [_d(v).ravel() for v in (hl, ul, vl, hr, ur, vr, nx, ny)]
    nn = a[0].size
    f = np.empty((nn, 3))
    lib().om_hllc_batch(nn, g, *[_ptr(v) for v in a], _ptr(f))
    return f


def interface(hl, hul, hvl, zl, hr, hur, hvr, zr, nx, ny, g=9.81, h_dry=1e-6):
    """Flux with hydrostatic reconstruction; returns (F [N,3], p_left [N], p_right [N])."""
    a = [_d(v).ravel() for v in (hl, hul, hvl, zl, hr, hur, hvr, zr, nx, ny)]
    nn = a[0].size
    f = np.empty((nn, 3))
    pl = np.empty(nn)
    pr = np.empty(nn)
    lib().om_interface_batch(nn, g, h_dry, *[_ptr(v) for v in a], _ptr(f), _ptr(pl), _ptr(pr))
    return f, pl, pr


def wall(h, hu, hv, nx, ny, g=9.81, h_dry=1e-6):
    """Flux through a reflective wall and its bed correction; (F [N,3], p [N])."""
    a = [_d(v).ravel() for v in (h, hu, hv, nx, ny)]
    nn = a[0].size
    f = np.empty((nn, 3))
    p = np.empty(nn)
    lib().om_wall_batch(nn, g, h_dry, *[_ptr(v) for v in a], _ptr(f), _ptr(p))
    return f, p


def inflow(q_in, h, nx, ny, g=9.81):
    """Flux through an inflow edge carrying unit discharge q_in into a cell of depth h (outward
    unit normal (nx, ny)) and the boundary wave speed; (F [N,3], speed [N])."""
    a = [_d(v).ravel() for v in (q_in, h, nx, ny)]
    nn = a[0].size
    f = np.empty((nn, 3))
    s = np.empty(nn)
    lib().om_inflow_batch(nn, g, *[_ptr(v) for v in a], _ptr(f), _ptr(s))
    return f, s


def wave_speeds(hl, ql, hr, qr, g=9.81):
    a = [_d(v).ravel() for v in (hl, ql, hr, qr)]
    nn = a[0].size
    sl = np.empty(nn)
    sr = np.empty(nn)
    lib().om_wave_speeds_batch(nn, g, *[_ptr(v) for v in a], _ptr(sl), _ptr(sr))
    return sl, sr


def run_tl(mesh: Mesh, z, n, h, hu, hv, dt_seq, gauges, every, obs, dz=None, dn=None, dh=None,
           dhu=None, dhv=None, g=9.81, h_dry=1e-6, inflow_q=None):
    """Tangent-linear run (dt replayed): returns (J, dJ) for the gauge misfit along the
    direction (dz, dn, dh, dhu, dhv) (None = zero)."""
    z, n = _d(z), _d(n)
    h, hu, hv = _d(h).copy(), _d(hu).copy(), _d(hv).copy()
    dirs = [None if d is None else _d(d).copy() for d in (dz, dn, dh, dhu, dhv)]
    seq = _d(dt_seq)
    gg = np.ascontiguousarray(gauges, dtype=np.int32)
    ob = _d(obs)
    p, _keep = _params(g, 0.7, h_dry, inflow_q)
    J = C.c_double()
    dJ = C.c_double()
    rc = lib().om_run_tl(mesh._h, _ptr(z), _ptr(dirs[0]), _ptr(n), _ptr(dirs[1]), _ptr(h),
                         _ptr(dirs[2]), _ptr(hu), _ptr(dirs[3]), _ptr(hv), _ptr(dirs[4]),
                         C.byref(p), seq.size, _ptr(seq), gg.ctypes.data_as(_ip), gg.size,
                         int(every), _ptr(ob), C.byref(J), C.byref(dJ))
    if rc != OK:
        raise RuntimeError(f"oracle tangent run failed: {rc}")
    return J.value, dJ.value


def run_loss(mesh: Mesh, z, n, h, hu, hv, dt_seq, gauges, every, obs, g=9.81, h_dry=1e-6,
             inflow_q=None) -> float:
    """The gauge misfit of a plain run with the replayed dt sequence."""
    z, n = _d(z), _d(n)
    h, hu, hv = _d(h).copy(), _d(hu).copy(), _d(hv).copy()
    seq = _d(dt_seq)
    gg = np.ascontiguousarray(gauges, dtype=np.int32)
    ob = _d(obs)
    p, _keep = _params(g, 0.7, h_dry, inflow_q)
    J = C.c_double()
    rc = lib().om_run_loss(mesh._h, _ptr(z), _ptr(n), _ptr(h), _ptr(hu), _ptr(hv), C.byref(p),
                           seq.size, _ptr(seq), gg.ctypes.data_as(_ip), gg.size, int(every),
                           _ptr(ob), C.byref(J))
    if rc != OK:
        raise RuntimeError(f"oracle loss run failed: {rc}")
    return J.value


def run_loss_sig(mesh: Mesh, z, n, h, hu, hv, dt_seq, gauges, every, obs, g=9.81, h_dry=1e-6,
                 inflow_q=None) -> tuple[float, int]:
    """The gauge misfit of a plain run with the replayed dt sequence and the run's branch
    signature (a 64-bit hash of every branch every edge and cell took at every step): equal
    signatures mark runs that took the same branches, between which the misfit is smooth."""
    z, n = _d(z), _d(n)
    h, hu, hv = _d(h).copy(), _d(hu).copy(), _d(hv).copy()
    seq = _d(dt_seq)
    gg = np.ascontiguousarray(gauges, dtype=np.int32)
    ob = _d(obs)
    p, _keep = _params(g, 0.7, h_dry, inflow_q)
    J = C.c_double()
    sig = C.c_ulong()
    rc = lib().om_run_loss_sig(mesh._h, _ptr(z), _ptr(n), _ptr(h), _ptr(hu), _ptr(hv),
                               C.byref(p), seq.size, _ptr(seq), gg.ctypes.data_as(_ip), gg.size,
                               int(every), _ptr(ob), C.byref(J), C.byref(sig))
    if rc != OK:
        raise RuntimeError(f"oracle signature run failed: {rc}")
    return J.value, int(sig.value)


def observations(case, mesh: Mesh | None = None, steps=None):
    """Synthetic observations of the calibration setup: a run with the hidden roughness and
    the CFL dt, recording h at the gauges every `obs_every` steps.  Returns (dt_seq, obs)."""
    mesh = mesh or Mesh(case.xy, case.tri, case.edge_tag)
    steps = case.steps if steps is None else steps
    every = case.extra["obs_every"]
    gauges = case.extra["gauges"]
    h, hu, hv = case.h.copy(), case.hu.copy(), case.hv.copy()
    dts, obs = [], []
    t = 0.0
    for s in range(steps):
        rc, h, hu, hv, d, st = run(mesh, case.z, case.extra["n_hidden"], h, hu, hv, 1, t0=t)
        if rc != OK:
            raise RuntimeError(f"observation run failed: {rc}")
        t = st["t"]
        dts.append(d[0])
        if (s + 1) % every == 0:
            obs.append(h[gauges].copy())
    return np.array(dts), np.array(obs)
