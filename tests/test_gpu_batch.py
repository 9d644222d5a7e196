"""Batched independent systems through the C-ABI: per-system forces and
energies against the FP64 oracle (linked cells in both precisions, Verlet
lists in FP32), the batched time step against the oracle's trajectories, and
graph replays against eager execution."""
import numpy as np
import pytest

from paper_2505_03438_amd import workloads as W
from tests.gpu_util import assert_forces, make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_03438_amd import mdlj
    mdlj.lib()
    return mdlj


def _systems(n_sys=12, n_max=1500, seed=99):
    syss = W.batched_systems(n_sys=n_sys, n_min=256, n_max=n_max, seed=seed)
    # include the smallest box of the workload family (2 cells per dimension)
    return syss


def _concat(syss):
    offs = np.zeros(len(syss) + 1, np.int64)
    offs[1:] = np.cumsum([s["pos"].shape[1] for s in syss])
    pos = np.concatenate([s["pos"] for s in syss], axis=1)
    vel = np.concatenate([s["vel"] for s in syss], axis=1)
    boxes = np.stack([s["box"] for s in syss])
    return offs, pos, vel, boxes


class Dev:
    def __init__(self, M, syss, prec, R=5, csf=1.0, skin=0.3, container=0, max_neighbors=160):
        import torch
        self.offs, pos, vel, boxes = _concat(syss)
        n = pos.shape[1]
        cfg = make_config(n, boxes[0], container=container, precision=prec, R=R, csf=csf, skin=skin,
                          max_neighbors=max_neighbors)
        self.b = M.md_batch_create(cfg, self.offs, boxes)
        real = self.b.real
        self.pos = torch.tensor(pos, dtype=torch.float64, device="cuda")
        self.vel = torch.tensor(vel, dtype=real, device="cuda")
        self.force = torch.zeros((3, n), dtype=real, device="cuda")
        self.type = torch.zeros(n, dtype=torch.int32, device="cuda")
        self.ids = torch.arange(n, dtype=torch.int32, device="cuda")
        self.lj = torch.tensor([1.0, 1.0], dtype=torch.float64, device="cuda")
        self.im = torch.ones(1, dtype=torch.float64, device="cuda")
        self.n = n

    def by_id(self, t):
        a = t.detach().double().cpu().numpy()
        out = np.empty_like(a)
        out[..., self.ids.cpu().numpy()] = a
        return out


@pytest.mark.parametrize("prec,container", [(1, 0), (0, 0), (0, 1)], ids=["fp64", "fp32", "fp32-vl"])
def test_batched_forces_match_oracle(orc, M, prec, container):
    import torch
    syss = _systems()
    d = Dev(M, syss, prec, container=container)
    M.md_batch_build_cells(d.b, d.pos, d.vel, d.force, d.type, d.ids)
    out = torch.zeros(4 * len(syss), dtype=torch.float64, device="cuda")
    M.md_batch_compute_forces(d.b, d.pos, d.type, d.lj, d.force, out)
    torch.cuda.synchronize()
    F = d.by_id(d.force)
    out = out.cpu().numpy().reshape(-1, 4)
    # systems keep their ranges: ids of system s stay inside its range
    ids = d.ids.cpu().numpy()
    for s in range(len(syss)):
        r = slice(d.offs[s], d.offs[s + 1])
        assert np.array_equal(np.sort(ids[r]), np.arange(d.offs[s], d.offs[s + 1]))
    tolF = 1e-12 if prec == 1 else 1e-5
    tolE = 1e-12 if prec == 1 else 1e-6
    for s, sy in enumerate(syss):
        F0, U0, W0, P0 = orc.forces(sy["pos"], sy["box"], orc.single())
        r = slice(d.offs[s], d.offs[s + 1])
        assert int(out[s, 2]) == P0, s
        assert_forces(F[:, r], F0, prec == 1, rel=tolF, what=s)
        assert abs(out[s, 0] - U0) <= tolE * abs(U0), s
        assert abs(out[s, 1] - W0) <= tolE * abs(W0), s


@pytest.mark.parametrize("container", [0, 1], ids=["lc", "vl"])
@pytest.mark.parametrize("csf", [1.0, 0.5], ids=["csf1", "csf05"])
def test_batched_fp32_slab_items(orc, M, csf, container):
    """FP32 forces of systems the force kernel splits differently: a system
    staged whole in LDS (300 particles), systems cut into z-slabs (4,000 and
    14,000), and a system packed into one corner of its box (6,000 particles in
    an eighth of the volume), whose slabs are sized from the mean density so
    that the dense ones overflow the LDS tile and read global memory.  At
    CSF 1/2 the stencil reaches two cells each way (rows of five cells, halos
    of two layers).  With Verlet lists the lists are built over the same
    items (LDS indices where the item is staged, indices in the system where
    it reads global memory)."""
    import torch
    corner = W.batched_systems(n_sys=1, n_min=6000, n_max=6000, seed=44)[0]
    corner = dict(corner, box=2.0 * corner["box"])
    syss = (W.batched_systems(n_sys=2, n_min=300, n_max=300, seed=41)
            + W.batched_systems(n_sys=2, n_min=4000, n_max=4000, seed=42)
            + W.batched_systems(n_sys=1, n_min=14000, n_max=14000, seed=43) + [corner])
    d = Dev(M, syss, 0, csf=csf, container=container)
    M.md_batch_build_cells(d.b, d.pos, d.vel, d.force, d.type, d.ids)
    out = torch.zeros(4 * len(syss), dtype=torch.float64, device="cuda")
    M.md_batch_compute_forces(d.b, d.pos, d.type, d.lj, d.force, out)
    torch.cuda.synchronize()
    F = d.by_id(d.force)
    out = out.cpu().numpy().reshape(-1, 4)
    for s, sy in enumerate(syss):
        F0, U0, W0, P0 = orc.forces(sy["pos"], sy["box"], orc.single())
        r = slice(d.offs[s], d.offs[s + 1])
        assert int(out[s, 2]) == P0, s
        assert_forces(F[:, r], F0, False, what=s)
        assert abs(out[s, 0] - U0) <= 1e-6 * abs(U0), s
        assert abs(out[s, 1] - W0) <= 1e-6 * abs(W0), s


def test_batched_step_matches_oracle(orc, M):
    import torch
    syss = _systems(n_sys=6, n_max=700, seed=5)
    d = Dev(M, syss, 1, R=5)
    M.md_batch_build_cells(d.b, d.pos, d.vel, d.force, d.type, d.ids)
    M.md_batch_compute_forces(d.b, d.pos, d.type, d.lj, d.force)
    M.md_batch_step(d.b, d.pos, d.vel, d.force, d.type, d.ids, d.im, d.lj, 0.005, 40, use_graph=True)
    torch.cuda.synchronize()
    X = d.by_id(d.pos)
    V = d.by_id(d.vel)
    for s, sy in enumerate(syss):
        p1, v1, _, _ = orc.velocity_verlet(sy["pos"], sy["vel"], sy["box"], orc.single(), 0.005, 40)
        r = slice(d.offs[s], d.offs[s + 1])
        dx = X[:, r] - p1
        dx -= sy["box"][0] * np.rint(dx / sy["box"][0])
        assert np.abs(dx).max() < 1e-9, s
        assert np.abs(V[:, r] - v1).max() < 1e-8, s


@pytest.mark.parametrize("prec,container", [(1, 0), (0, 1)], ids=["fp64", "fp32-vl"])
def test_batched_interval_adapts(orc, M, prec, container):
    """A thin skin (0.1) with a long maximum interval (10): skin violations
    shorten the rebuild interval the batch uses, and the trajectory still
    follows the oracle's.  In FP32 the blocks' force passes also advance the
    particles (all but a block's last), while the steps redone after a
    violation run the separate integrator: both within the FP32 bar."""
    import torch
    syss = _systems(n_sys=4, n_max=700, seed=23)
    d = Dev(M, syss, prec, R=10, skin=0.1, container=container)
    assert M.md_batch_get_counters(d.b) == dict(rebuilds=0, forced_rebuilds=0, steps=0, rebuild_interval=10)
    M.md_batch_build_cells(d.b, d.pos, d.vel, d.force, d.type, d.ids)
    M.md_batch_compute_forces(d.b, d.pos, d.type, d.lj, d.force)
    M.md_batch_step(d.b, d.pos, d.vel, d.force, d.type, d.ids, d.im, d.lj, 0.005, 60, use_graph=True)
    torch.cuda.synchronize()
    cnt = M.md_batch_get_counters(d.b)
    assert 1 <= cnt["rebuild_interval"] < 10
    assert cnt["steps"] == 60 and cnt["forced_rebuilds"] >= 1
    # blocks of at most 10 steps, and the last block of a call is never cut short
    assert cnt["rebuilds"] >= max(6, cnt["forced_rebuilds"] + 1)
    X = d.by_id(d.pos)
    V = d.by_id(d.vel)
    # FP32: pair forces to ~1e-6 relative; over 60 steps their rounding moves
    # positions by well under 1e-5 and velocities by under 1e-4
    tx, tv = (1e-9, 1e-8) if prec == 1 else (1e-5, 1e-4)
    for s, sy in enumerate(syss):
        p1, v1, _, _ = orc.velocity_verlet(sy["pos"], sy["vel"], sy["box"], orc.single(), 0.005, 60)
        rs = slice(d.offs[s], d.offs[s + 1])
        dx = X[:, rs] - p1
        dx -= sy["box"][0] * np.rint(dx / sy["box"][0])
        assert np.abs(dx).max() < tx, s
        assert np.abs(V[:, rs] - v1).max() < tv, s


@pytest.mark.parametrize("container", [0, 1], ids=["lc", "vl"])
def test_graph_replays_equal_eager(M, container):
    """Replays of the captured rebuild interval, with eager work and
    synchronisations in between, against the same steps run eagerly."""
    import torch
    syss = _systems(n_sys=8, n_max=1200, seed=17)
    results = []
    for use_graph in (False, True):
        d = Dev(M, syss, 0, R=4, container=container)
        M.md_batch_build_cells(d.b, d.pos, d.vel, d.force, d.type, d.ids)
        M.md_batch_compute_forces(d.b, d.pos, d.type, d.lj, d.force)
        snaps = []
        for rep in range(4):
            M.md_batch_step(d.b, d.pos, d.vel, d.force, d.type, d.ids, d.im, d.lj, 0.005, 12,
                            use_graph=use_graph)
            torch.cuda.synchronize()
            snaps.append(d.by_id(d.pos).copy())
            # eager work of the program between replays
            M.md_batch_compute_forces(d.b, d.pos, d.type, d.lj, d.force)
            torch.cuda.synchronize()
        results.append(snaps)
    for a, b in zip(*results):
        assert np.array_equal(a, b)


def test_batched_list_overflow_falls_back(orc, M):
    """Verlet lists whose capacity the clumped system outgrows: the batch's
    only system holds 6,000 particles in an eighth of its box, so the capacity
    estimated from its mean density (1.3 times the mean count within the list
    radius plus 8, in whole chunks of 8; max_neighbors 8 is lower) is below
    the partners of a particle inside the clump.  Those particles take their
    forces from the stencil instead; every force and the pair count still
    match the oracle."""
    import torch
    corner = W.batched_systems(n_sys=1, n_min=6000, n_max=6000, seed=44)[0]
    corner = dict(corner, box=2.0 * corner["box"])
    syss = [corner]
    d = Dev(M, syss, 0, container=1, max_neighbors=8)
    M.md_batch_build_cells(d.b, d.pos, d.vel, d.force, d.type, d.ids)
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    M.md_batch_compute_forces(d.b, d.pos, d.type, d.lj, d.force, out)
    torch.cuda.synchronize()
    F = d.by_id(d.force)
    out = out.cpu().numpy()
    F0, U0, W0, P0 = orc.forces(corner["pos"], corner["box"], orc.single())
    # the mean particle has more partners within r_c alone than the capacity
    n = corner["pos"].shape[1]
    rho = n / float(corner["box"][0]) ** 3
    cap = 8 * int(np.ceil(max(8, int(1.3 * rho * 4 / 3 * np.pi * 2.8 ** 3 + 8)) / 8))
    assert 2 * P0 / n > 1.5 * cap
    assert int(out[2]) == P0
    assert_forces(F, F0, False)
    assert abs(out[0] - U0) <= 1e-6 * abs(U0)


def test_batched_lists_step_fp32(orc, M):
    """Forty FP32 steps with Verlet lists, graph-captured after the first
    interval: positions within 1e-6 of the oracle's FP64 trajectories, and the
    same steps with linked cells agree with them as closely."""
    import torch
    syss = _systems(n_sys=6, n_max=900, seed=7)
    X = {}
    for container in (0, 1):
        d = Dev(M, syss, 0, R=5, container=container)
        M.md_batch_build_cells(d.b, d.pos, d.vel, d.force, d.type, d.ids)
        M.md_batch_compute_forces(d.b, d.pos, d.type, d.lj, d.force)
        M.md_batch_step(d.b, d.pos, d.vel, d.force, d.type, d.ids, d.im, d.lj, 0.005, 40, use_graph=True)
        torch.cuda.synchronize()
        X[container] = d.by_id(d.pos)
    for s, sy in enumerate(syss):
        p1, _, _, _ = orc.velocity_verlet(sy["pos"], sy["vel"], sy["box"], orc.single(), 0.005, 40)
        r = slice(d.offs[s], d.offs[s + 1])
        for container in (0, 1):
            dx = X[container][:, r] - p1
            dx -= sy["box"][0] * np.rint(dx / sy["box"][0])
            assert np.abs(dx).max() < 1e-6, (s, container)


def test_batched_lists_rejected_outside_their_range(M):
    """Batched Verlet lists are FP32, gather-only, for systems of at most
    65536 particles (16-bit entries); anything else is refused at creation."""
    syss = _systems(n_sys=2, n_max=400, seed=3)
    offs, pos, vel, boxes = _concat(syss)
    n = pos.shape[1]
    for kw in (dict(precision=1), dict(newton3=1)):
        cfg = make_config(n, boxes[0], container=1, **{"precision": 0, **kw})
        with pytest.raises(RuntimeError):
            M.md_batch_create(cfg, offs, boxes)
    big = np.array([0, 70000], np.int64)
    cfg = make_config(70000, [40.0] * 3, container=1, precision=0)
    with pytest.raises(RuntimeError, match="65536"):
        M.md_batch_create(cfg, big, np.array([[40.0] * 3]))
    cfg = make_config(n, boxes[0], container=2, precision=0)
    with pytest.raises(RuntimeError):
        M.md_batch_create(cfg, offs, boxes)


@pytest.mark.parametrize("prec,container", [(1, 0), (0, 0), (0, 1)], ids=["fp64", "fp32", "fp32-vl"])
def test_batched_empty_and_tiny_systems(orc, M, prec, container):
    """A batch holding an empty system (offsets equal) and a system of two
    particles 1.1 apart (a 6-sigma box: two cells per dimension, every cell in
    every stencil) beside an ordinary one: forces, energies and pair counts of
    every system, and ten steps (graph-captured after the first interval),
    against the oracle."""
    import torch
    big = W.batched_systems(n_sys=1, n_min=500, n_max=500, seed=71)[0]
    pair = dict(pos=np.array([[1.0, 2.1], [3.0, 3.0], [3.0, 3.0]]), vel=np.array([[0.3, -0.2], [0.0, 0.1],
                [0.0, 0.0]], dtype=np.float32), box=np.array([6.0, 6.0, 6.0]))
    empty = dict(pos=np.zeros((3, 0)), vel=np.zeros((3, 0), np.float32), box=np.array([7.0, 7.0, 7.0]))
    syss = [big, empty, pair]
    d = Dev(M, syss, prec, R=3, container=container)
    assert list(d.offs) == [0, 500, 500, 502]
    M.md_batch_build_cells(d.b, d.pos, d.vel, d.force, d.type, d.ids)
    out = torch.zeros(4 * len(syss), dtype=torch.float64, device="cuda")
    M.md_batch_compute_forces(d.b, d.pos, d.type, d.lj, d.force, out)
    torch.cuda.synchronize()
    F = d.by_id(d.force)
    out = out.cpu().numpy().reshape(-1, 4)
    assert out[1, 2] == 0 and out[1, 0] == 0
    for s in (0, 2):
        sy = syss[s]
        F0, U0, W0, P0 = orc.forces(sy["pos"], sy["box"], orc.single())
        r = slice(d.offs[s], d.offs[s + 1])
        assert int(out[s, 2]) == P0, s
        assert_forces(F[:, r], F0, prec == 1, what=s)
        assert abs(out[s, 0] - U0) <= (1e-12 if prec == 1 else 1e-6) * abs(U0), s
    M.md_batch_step(d.b, d.pos, d.vel, d.force, d.type, d.ids, d.im, d.lj, 0.005, 10, use_graph=True)
    torch.cuda.synchronize()
    X = d.by_id(d.pos)
    tol = 1e-9 if prec == 1 else 1e-6
    for s in (0, 2):
        sy = syss[s]
        p1, _, _, _ = orc.velocity_verlet(sy["pos"], sy["vel"].astype(np.float64), sy["box"], orc.single(), 0.005,
                                          10)
        r = slice(d.offs[s], d.offs[s + 1])
        dx = X[:, r] - p1
        dx -= sy["box"][0] * np.rint(dx / sy["box"][0])
        assert np.abs(dx).max() < tol, s
