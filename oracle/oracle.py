"""Python face of the FP64 CPU oracle (``mdoracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark import this module.  It shares no code with the
HIP library and imports nothing from the product package.

Each function marshals numpy arrays into the plain C routines and returns
numpy arrays.  Positions are SoA ``[3, n]`` float64 arrays in ``[0, L)``;
per-pair tables (eps, sig, rc2) are ``[nt, nt]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdoracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: FP64, OpenMP, no FP contraction."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_lj.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.orc_forces.argtypes = [ctypes.c_int64, _dp, _ip, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_forces_rows.argtypes = [ctypes.c_int64, _dp, _ip, ctypes.c_int, _dp, _dp, _dp, _dp,
                                      ctypes.c_int64, _lp, _dp, _lp]
        L.orc_forces_cells.argtypes = L.orc_forces.argtypes
        L.orc_pairs.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_double, ctypes.c_int64, _lp]
        L.orc_pairs.restype = ctypes.c_int64
        L.orc_neighbor_rows.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_double, ctypes.c_int64,
                                        _lp, ctypes.c_int64, _lp, _lp]
        L.orc_neighbor_rows.restype = ctypes.c_int
        L.orc_cell_dims.argtypes = [_dp, ctypes.c_double, _ip]
        L.orc_cells.argtypes = [ctypes.c_int64, _dp, _dp, _ip, _ip, _ip, _ip]
        L.orc_velocity_verlet.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _ip, ctypes.c_int, _dp, _dp,
                                          _dp, _dp, _dp, ctypes.c_double, ctypes.c_int64, ctypes.c_int,
                                          _dp]
        L.orc_force_matching.argtypes = [ctypes.c_int64, _dp, _ip, ctypes.c_int, _dp, _dp, _dp, _dp,
                                         _dp, _dp, _dp]
        L.orc_force_matching.restype = ctypes.c_double
        L.orc_mix.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp]
        L.orc_live_stats.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_double, _dp]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _l(a):
    return a.ctypes.data_as(_lp)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def lj(r2: float, eps: float = 1.0, sig: float = 1.0):
    """(phi, u) of one pair at squared distance r2; f_ij = phi * d_ij."""
    phi, u = ctypes.c_double(), ctypes.c_double()
    lib().orc_lj(float(r2), float(eps), float(sig), ctypes.byref(phi), ctypes.byref(u))
    return phi.value, u.value


def mix(eps_t, sig_t):
    """Lorentz-Berthelot pair tables [nt, nt] from per-type eps, sig."""
    eps_t = _f64(eps_t)
    sig_t = _f64(sig_t)
    nt = eps_t.size
    e = np.zeros((nt, nt))
    s = np.zeros((nt, nt))
    lib().orc_mix(nt, _d(eps_t), _d(sig_t), _d(e), _d(s))
    return e, s


class Params:
    """Per-pair LJ tables of one system (nt types)."""

    def __init__(self, eps, sig, rc2):
        self.eps = _f64(eps)
        self.sig = _f64(sig)
        self.rc2 = _f64(rc2)
        self.nt = int(round(np.sqrt(self.eps.size)))
        assert self.eps.size == self.nt * self.nt


def single(eps=1.0, sig=1.0, rc=2.5) -> Params:
    return Params([[eps]], [[sig]], [[rc * rc]])


def forces(pos, box, params: Params, types=None, cells: bool = False):
    """Brute-force (or linked-cell) FP64 forces.  Returns (F[3,n], U, W, n_pairs)."""
    pos = _f64(pos)
    n = pos.shape[1]
    types = np.zeros(n, np.int32) if types is None else _i32(types)
    box = _f64(box)
    F = np.zeros((3, n))
    out = np.zeros(3)
    fn = lib().orc_forces_cells if cells else lib().orc_forces
    fn(n, _d(pos), _i(types), params.nt, _d(box), _d(params.eps), _d(params.sig), _d(params.rc2),
       _d(F), _d(out))
    return F, out[0], out[1], int(out[2])


def forces_rows(pos, box, params: Params, rows, types=None):
    """Brute-force FP64 forces of the selected rows only: (F[3,m], n_pairs[m])."""
    pos = _f64(pos)
    n = pos.shape[1]
    types = np.zeros(n, np.int32) if types is None else _i32(types)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    m = rows.size
    box = _f64(box)
    F = np.zeros((3, m))
    cnt = np.zeros(m, np.int64)
    lib().orc_forces_rows(n, _d(pos), _i(types), params.nt, _d(box), _d(params.eps), _d(params.sig),
                          _d(params.rc2), m, _l(rows), _d(F), _l(cnt))
    return F, cnt


def pairs(pos, box, r2cut: float):
    """All unordered pairs (i < j) with r2 < r2cut, brute force; int64 [k, 2]."""
    pos = _f64(pos)
    n = pos.shape[1]
    box = _f64(box)
    cap = 1 << 16
    while True:
        out = np.zeros((cap, 2), np.int64)
        cnt = lib().orc_pairs(n, _d(pos), _d(box), float(r2cut), cap, _l(out))
        if cnt <= cap:
            return out[:cnt].copy()
        cap = int(cnt)


def neighbor_rows(pos, box, r2cut: float, rows, cap_per_row: int = 512):
    """For each row i: sorted array of all j != i with r2 < r2cut."""
    pos = _f64(pos)
    n = pos.shape[1]
    box = _f64(box)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    m = rows.size
    counts = np.zeros(m, np.int64)
    lists = np.zeros((m, cap_per_row), np.int64)
    rc = lib().orc_neighbor_rows(n, _d(pos), _d(box), float(r2cut), m, _l(rows), cap_per_row,
                                 _l(counts), _l(lists))
    if rc != 0:
        return neighbor_rows(pos, box, r2cut, rows, cap_per_row=int(counts.max()))
    return [lists[r, :counts[r]].copy() for r in range(m)]


def cell_dims(box, side_min: float):
    box = _f64(box)
    nc = np.zeros(3, np.int32)
    lib().orc_cell_dims(_d(box), float(side_min), _i(nc))
    return nc


def cells(pos, box, ncell):
    """Linked-cell binning: (cell_of[n], order[n], cell_start[ncells+1])."""
    pos = _f64(pos)
    n = pos.shape[1]
    box = _f64(box)
    ncell = _i32(ncell)
    nc = int(np.prod(ncell.astype(np.int64)))
    cell_of = np.zeros(n, np.int32)
    order = np.zeros(n, np.int32)
    start = np.zeros(nc + 1, np.int32)
    lib().orc_cells(n, _d(pos), _d(box), _i(ncell), _i(cell_of), _i(order), _i(start))
    return cell_of, order, start


def velocity_verlet(pos, vel, box, params: Params, dt: float, nsteps: int, types=None,
                    inv_mass=None, cells_mode: bool = False, force=None):
    """Run nsteps of velocity Verlet.  Returns (pos, vel, force, log[nsteps, 4]={U,K,W,n_pairs})."""
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    n = pos.shape[1]
    types = np.zeros(n, np.int32) if types is None else _i32(types)
    inv_mass = _f64(np.ones(params.nt) if inv_mass is None else inv_mass)
    box = _f64(box)
    if force is None:
        force, _, _, _ = forces(pos, box, params, types, cells=cells_mode)
    force = _f64(force).copy()
    log = np.zeros((nsteps, 4))
    lib().orc_velocity_verlet(n, _d(pos), _d(vel), _d(force), _i(types), params.nt, _d(box),
                              _d(params.eps), _d(params.sig), _d(params.rc2), _d(inv_mass),
                              float(dt), int(nsteps), 1 if cells_mode else 0, _d(log))
    return pos, vel, force, log


def force_matching(pos, box, types, theta, rc2, target):
    """Loss and exact gradients of L = 1/(3n) sum |F(x; theta) - target|^2.

    theta = (eps_0..eps_{nt-1}, sig_0..sig_{nt-1}) per type, Lorentz-Berthelot
    mixed; rc2 [nt, nt] held fixed.  Returns (L, F, dL/dx [3,n], dL/dtheta [2nt]).
    """
    pos = _f64(pos)
    n = pos.shape[1]
    types = _i32(types)
    theta = _f64(theta)
    nt = theta.size // 2
    rc2 = _f64(rc2)
    box = _f64(box)
    target = _f64(target)
    F = np.zeros((3, n))
    gx = np.zeros((3, n))
    gt = np.zeros(2 * nt)
    L = lib().orc_force_matching(n, _d(pos), _i(types), nt, _d(box), _d(theta), _d(rc2),
                                 _d(target), _d(F), _d(gx), _d(gt))
    return L, F, gx, gt


def live_stats(pos, box, bin_side: float):
    """(mean, std/mean, median, max, n_bins, n_empty) over CSF-1 cell bins."""
    pos = _f64(pos)
    n = pos.shape[1]
    box = _f64(box)
    out = np.zeros(6)
    lib().orc_live_stats(n, _d(pos), _d(box), float(bin_side), _d(out))
    return out
