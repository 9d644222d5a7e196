"""Helpers of the GPU tests: put a seeded workload on the device through the
C-ABI binding and map results back to the oracle's particle order."""
import math

import numpy as np
import torch

from paper_2505_03438_amd import mdlj as M


def make_config(n, box, rc=2.5, skin=0.3, csf=1.0, container=M.MD_CONTAINER_VL, newton3=0,
                precision=M.MD_FP32, R=10, max_neighbors=160, n_types=1, rc2=None, layout=0):
    c = M.config_default(n, float(box[0]))
    c.box[0], c.box[1], c.box[2] = (float(b) for b in box)
    c.n_types = n_types
    if rc2 is None:
        for k in range(4):
            c.rc2[k] = rc * rc
    else:
        rc2 = np.asarray(rc2, dtype=np.float64).reshape(-1)
        for k in range(rc2.size):
            c.rc2[k] = float(rc2[k])
    c.skin = skin
    c.csf = csf
    c.container = container
    c.newton3 = newton3
    c.precision = precision
    c.rebuild_interval = R
    c.max_neighbors = max_neighbors
    c.layout = layout
    return c


class DeviceSystem:
    """Particle arrays on the GPU in the library's (cell) order."""

    def __init__(self, cfg, pos, vel=None, types=None, eps=(1.0,), sig=(1.0,)):
        self.h = M.md_create(cfg)
        n = pos.shape[1]
        self.n = n
        real = self.h.real
        dev = "cuda"
        self.pos = torch.tensor(np.ascontiguousarray(pos), dtype=torch.float64, device=dev)
        v = np.zeros((3, n)) if vel is None else vel
        self.vel = torch.tensor(np.ascontiguousarray(v), dtype=real, device=dev)
        self.force = torch.zeros((3, n), dtype=real, device=dev)
        t = np.zeros(n, np.int32) if types is None else types
        self.type = torch.tensor(np.ascontiguousarray(t, dtype=np.int32), device=dev)
        self.ids = torch.arange(n, dtype=torch.int32, device=dev)
        self.lj = torch.tensor(list(eps) + list(sig), dtype=torch.float64, device=dev)
        self.inv_mass = torch.ones(cfg.n_types, dtype=torch.float64, device=dev)

    def build(self):
        M.md_build_cells(self.h, self.pos, self.vel, self.force, self.type, self.ids)
        M.md_build_neighbors(self.h, self.pos, self.type)

    def forces(self, energy=True):
        out = torch.zeros(4, dtype=torch.float64, device="cuda") if energy else None
        M.md_compute_forces(self.h, self.pos, self.type, self.lj, self.force, out)
        torch.cuda.synchronize()
        return out

    def ids_np(self):
        return self.ids.cpu().numpy()

    def by_id(self, t):
        """(3, n) or (n,) device tensor in cell order -> numpy in id order."""
        a = t.detach().cpu().numpy()
        ids = self.ids_np()
        out = np.empty_like(a)
        if a.ndim == 2:
            out[:, ids] = a
        else:
            out[ids] = a
        return out


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = math.sqrt(float((b * b).sum()))
    return math.sqrt(float(((a - b) ** 2).sum())) / (nb if nb > 0 else 1.0)


# Per-particle force bound, relative to the RMS force of the reference: the
# FP32 pair arithmetic carries a relative error of a few 1e-7 per pair force
# (fixed-point displacement 2^-24, r^2 within 7e-7, rcp and the products), so
# a particle's error is at most about 1e-6 of the sum of its pair-force
# magnitudes, which stays below 50 F_rms in the workloads (close contacts of
# a hot liquid); FP64 carries 1e-15 per pair.  Bounds: 1e-4 F_rms (FP32),
# 1e-10 F_rms (FP64), beside the relative L2 bars 1e-5 / 1e-12.
FP32_FMAX, FP64_FMAX = 1e-4, 1e-10


def assert_forces(F, F0, fp64, rel=None, fmax=None, what=""):
    """Relative L2 error over all 3n components and the largest per-particle
    error |F_i - F0_i| / F_rms(F0), both within their bars."""
    F = np.asarray(F, dtype=np.float64)
    F0 = np.asarray(F0, dtype=np.float64)
    rel = (1e-12 if fp64 else 1e-5) if rel is None else rel
    fmax = (FP64_FMAX if fp64 else FP32_FMAX) if fmax is None else fmax
    e = rel_l2(F, F0)
    assert e <= rel, ("rel L2", e, what)
    n = F0.shape[-1]
    if n == 0:
        return
    frms = math.sqrt(float((F0 * F0).sum()) / n)
    if frms == 0.0:
        return
    worst = float(np.sqrt(((F - F0) ** 2).sum(axis=0)).max()) / frms
    assert worst <= fmax, ("max |dF_i|/F_rms", worst, what)
