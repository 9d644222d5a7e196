"""Parity of the HIP path with the FP64 oracle, through the C-ABI.

Bars: integer results (cell contents, neighbour sets, pair counts) bit-exact;
forces within a relative L2 error of 1e-5 (FP32 pair arithmetic) or 1e-12
(FP64); energies and virials within 1e-6 (FP32 with FP64 accumulation) or
1e-12 (FP64)."""
import numpy as np
import pytest

from paper_2505_03438_amd import workloads as W
from tests.gpu_util import DeviceSystem, assert_forces, make_config, rel_l2

pytestmark = pytest.mark.gpu

M = None


@pytest.fixture(scope="module", autouse=True)
def _lib():
    global M
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_03438_amd import mdlj
    mdlj.lib()
    M = mdlj


FP32_F, FP64_F = 1e-5, 1e-12
FP32_E, FP64_E = 1e-6, 1e-12

# (container, newton3, csf); newton3 2 is the C08 traversal of linked cells
CONTAINERS = [(0, 0, 1.0), (0, 1, 1.0), (0, 0, 0.5), (0, 1, 0.5), (1, 0, 1.0), (1, 1, 1.0), (1, 0, 0.5),
              (1, 1, 0.5), (2, 0, 1.0), (2, 0, 0.5), (3, 0, 1.0), (4, 1, 1.0), (0, 2, 1.0)]
CNAMES = ["lc", "lc-n3l", "lc-csf.5", "lc-n3l-csf.5", "vl", "vl-n3l", "vl-csf.5", "vl-n3l-csf.5", "cl", "cl-csf.5",
          "pvl", "vlc", "lc-c08"]


def fp32_only(cont):
    """Cluster-pair lists, pairwise Verlet lists, Verlet list cells and the
    C08 traversal run in FP32 only."""
    return cont[0] in (2, 3, 4) or cont[1] == 2


def _fp32_only(cont, prec, box=None):
    """Skip the FP32-only structures in FP64, and those needing three cells of
    side r_c + skin per dimension (pairwise lists, list cells, C08) on
    smaller boxes."""
    if fp32_only(cont) and prec == 1:
        pytest.skip("cluster lists, pairwise lists, list cells and the C08 traversal are FP32-only")
    if box is not None and not fits(cont, box):
        pytest.skip("pairwise lists, list cells and the C08 traversal need three cells per dimension")


def fits(cont, box, prec=0):
    """Whether container cont runs on this machine and precision."""
    if fp32_only(cont) and prec == 1:
        return False
    return (cont[0] not in (3, 4) and cont[1] != 2) or all(int(b // 2.8) >= 3 for b in box)


def _jittered(ncell, seed, density=0.8, jitter=0.08, shape=None):
    rng = np.random.default_rng(seed)
    pos, box = W.jittered_fcc(shape or ncell, density, jitter, rng)
    return pos, box


# ---------------------------------------------------------------- FCC lattice

@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
@pytest.mark.parametrize("cont", CONTAINERS, ids=CNAMES)
def test_fcc_lattice(orc, prec, cont):
    _fp32_only(cont, prec)
    d = W.plain_fcc_864()
    pos, box = d["pos"], d["box"]
    F0, U0, W0, P0 = orc.forces(pos, box, orc.single())
    cfg = make_config(864, box, container=cont[0], newton3=cont[1], csf=cont[2], precision=prec)
    s = DeviceSystem(cfg, pos)
    s.build()
    out = s.forces().cpu().numpy()
    F = s.by_id(s.force)
    assert out[2] == P0 == 23328
    tolF = 1e-12 if prec == 1 else 1e-6
    assert np.abs(F).max() <= tolF * 24 * 54
    tolE = FP64_E if prec == 1 else FP32_E
    assert abs(out[0] - U0) <= tolE * abs(U0)
    assert abs(out[1] - W0) <= tolE * abs(W0)


# ---------------------------------------------------------------- cells

@pytest.mark.parametrize("csf", [1.0, 0.5])
def test_cell_contents_bit_exact(orc, csf):
    """Every cell holds exactly the oracle's particles (the counting sort),
    and inside a cell they are ordered by their staged x coordinate
    floor(x 2^32 / L_x), then by id: the order the Verlet-list build relies
    on when it bisects a stencil row by x.  (The oracle orders a cell by id;
    the paper leaves the order inside a cell open.)"""
    pos, box = _jittered((7, 6, 9), 3)
    n = pos.shape[1]
    cfg = make_config(n, box, container=0, csf=csf)
    s = DeviceSystem(cfg, pos)
    s.build()
    nc = orc.cell_dims(box, csf * 2.8)
    cell_of, order, start = orc.cells(pos, box, nc)
    ids = s.ids_np()
    qx = np.floor(np.clip(pos[0] * (4294967296.0 / box[0]), 0.0, 4294967295.0))
    for c in range(int(np.prod(nc))):
        got = ids[start[c]:start[c + 1]]
        assert np.array_equal(np.sort(got), np.sort(order[start[c]:start[c + 1]])), c
        assert np.array_equal(np.lexsort((got, qx[got])), np.arange(len(got))), c
    # positions were permuted, not altered
    assert np.array_equal(s.pos.cpu().numpy(), pos[:, ids])


# ---------------------------------------------------------------- forces

SIZES = [(4, 1), (5, 2), (7, 3), ((6, 7, 8), 4)]


@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
@pytest.mark.parametrize("cont", CONTAINERS, ids=CNAMES)
@pytest.mark.parametrize("size", SIZES, ids=["n256", "n500", "n1372", "n1344"])
def test_forces_match_oracle(orc, prec, cont, size):
    _fp32_only(cont, prec)
    ncell, seed = size
    pos, box = _jittered(ncell, seed)
    assert min(box) >= 5.6  # 2 (r_c + skin)
    _fp32_only(cont, prec, box)
    n = pos.shape[1]
    F0, U0, W0, P0 = orc.forces(pos, box, orc.single())
    cfg = make_config(n, box, container=cont[0], newton3=cont[1], csf=cont[2], precision=prec)
    s = DeviceSystem(cfg, pos)
    s.build()
    out = s.forces().cpu().numpy()
    F = s.by_id(s.force)
    assert int(out[2]) == P0
    tolF = FP64_F if prec == 1 else FP32_F
    tolE = FP64_E if prec == 1 else FP32_E
    assert_forces(F, F0, prec == 1, rel=tolF)
    assert abs(out[0] - U0) <= tolE * abs(U0)
    assert abs(out[1] - W0) <= tolE * abs(W0)


@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_anisotropic_box_and_two_types(orc, prec):
    rng = np.random.default_rng(17)
    pos, box = W.jittered_fcc((5, 6, 14), 1.0, 0.05, rng)
    n = pos.shape[1]
    types = (rng.random(n) < 0.3).astype(np.int32)
    eps_t, sig_t = [1.0, 0.5], [1.0, 0.88]
    e, sg = orc.mix(eps_t, sig_t)
    rc2 = (2.5 * sg) ** 2
    p = orc.Params(e, sg, rc2)
    F0, U0, W0, P0 = orc.forces(pos, box, p, types)
    for cont in CONTAINERS:
        if not fits(cont, box, prec):
            continue
        cfg = make_config(n, box, container=cont[0], newton3=cont[1], csf=cont[2], precision=prec,
                          n_types=2, rc2=rc2)
        s = DeviceSystem(cfg, pos, types=types, eps=eps_t, sig=sig_t)
        s.build()
        out = s.forces().cpu().numpy()
        assert int(out[2]) == P0, cont
        assert_forces(s.by_id(s.force), F0, prec == 1, what=cont)
        assert abs(out[0] - U0) <= (FP64_E if prec == 1 else FP32_E) * abs(U0)


def test_small_box_wrapping_stencil(orc):
    # 2 cells per dimension: the periodic stencil visits each neighbour cell once
    rng = np.random.default_rng(5)
    for L, n in ((5.7, 120), (6.6, 150), (8.5, 300)):
        pos, box = W.random_gas(n, L, rng)
        # keep particles apart: drop those closer than 0.8 to an earlier one
        keep = []
        for i in range(n):
            d = pos[:, keep] - pos[:, [i]]
            d -= L * np.rint(d / L)
            if not keep or (d * d).sum(axis=0).min() > 0.64:
                keep.append(i)
        pos = np.ascontiguousarray(pos[:, keep])
        F0, U0, W0, P0 = orc.forces(pos, box, orc.single())
        for cont in CONTAINERS:
            if not fits(cont, box):
                continue
            cfg = make_config(pos.shape[1], box, container=cont[0], newton3=cont[1], csf=cont[2])
            s = DeviceSystem(cfg, pos)
            s.build()
            out = s.forces().cpu().numpy()
            assert int(out[2]) == P0, (L, cont)
            assert_forces(s.by_id(s.force), F0, False, what=(L, cont))


def test_tiny_and_empty_systems(orc):
    import torch
    # two particles at r = 1.5 inside a box: analytic force along x
    pos = np.array([[1.0, 2.5], [3.0, 3.0], [3.0, 3.0]])
    box = np.array([8.0, 8.0, 8.0])
    F0, U0, _, P0 = orc.forces(pos, box, orc.single())
    for cont in CONTAINERS:
        if not fits(cont, box):
            continue
        prec = 0 if fp32_only(cont) else 1
        cfg = make_config(2, box, container=cont[0], newton3=cont[1], csf=cont[2], precision=prec)
        s = DeviceSystem(cfg, pos)
        s.build()
        out = s.forces().cpu().numpy()
        assert int(out[2]) == 1
        tol = 1e-12 if prec == 1 else FP32_F
        assert np.abs(s.by_id(s.force) - F0).max() <= tol * np.abs(F0).max()
    # no particles at all
    cfg = make_config(0, box)
    s = DeviceSystem(cfg, np.zeros((3, 0)))
    s.build()
    out = s.forces().cpu().numpy()
    assert list(out) == [0.0, 0.0, 0.0, 0.0]


def test_forces_need_lists_after_cell_build(orc):
    """A cell build reorders the particles: list containers refuse to compute
    forces until the lists are built again (no stale or unbuilt lists)."""
    pos, box = _jittered(6, 8, jitter=0.1)
    n = pos.shape[1]
    for cont in (1, 2, 3, 4):
        cfg = make_config(n, box, container=cont, newton3=1 if cont == 4 else 0, precision=0)
        s = DeviceSystem(cfg, pos)
        M.md_build_cells(s.h, s.pos, s.vel, s.force, s.type, s.ids)
        with pytest.raises(RuntimeError, match="md_build_neighbors"):
            s.forces()
        M.md_build_neighbors(s.h, s.pos, s.type)
        s.forces()
        M.md_build_cells(s.h, s.pos, s.vel, s.force, s.type, s.ids)
        with pytest.raises(RuntimeError, match="md_build_neighbors"):
            s.forces()


def test_step_reports_position_outside_box(orc):
    """A particle placed far outside the box is binned into an edge cell (no
    access leaves the cell arrays) and flagged: md_step fails with
    MD_ERR_NONFINITE until md_status clears the flag."""
    pos, box = _jittered(6, 8, jitter=0.1)
    n = pos.shape[1]
    pos = pos.copy()
    pos[2, 5] = 2.5 * box[2]
    for cont in (0, 1):
        cfg = make_config(n, box, container=cont, precision=0)
        s = DeviceSystem(cfg, pos)
        s.build()
        s.forces()
        with pytest.raises(RuntimeError, match=r"\(-4\).*outside the box"):
            M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.001, 2)
        assert M.md_status(s.h) & M.MD_FLAG_NONFINITE
        assert not (M.md_status(s.h) & M.MD_FLAG_NONFINITE)
        s.h.close()


# ---------------------------------------------------------------- Verlet sets

@pytest.mark.parametrize("csf", [1.0, 0.5])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("half", [0, 1])
def test_verlet_sets_bit_exact(orc, half, prec, csf):
    """Full lists equal the oracle's rows within r_c + skin.  Half lists (Newton's
    third law) hold every such pair exactly once, in the row of one of its two
    particles."""
    pos, box = _jittered(6, 8, jitter=0.1)
    n = pos.shape[1]
    cfg = make_config(n, box, container=1, newton3=half, precision=prec, csf=csf)
    s = DeviceSystem(cfg, pos)
    s.build()
    counts, rows = M.md_get_neighbors(s.h, 256)
    counts = counts.cpu().numpy()
    rows = rows.cpu().numpy()
    ids = s.ids_np()
    rl2 = (2.5 + 0.3) ** 2
    ref = orc.neighbor_rows(pos, box, rl2, np.arange(n))
    cnt = M.md_get_counters(s.h)
    assert cnt["list_entries"] == int(counts.sum())
    assert cnt["force_family"] in ((0,) if prec == 1 else (0, 1))  # FP64 has no windowed kernels
    if not half:
        for k in range(n):
            got = np.sort(ids[rows[k, :counts[k]]])
            assert np.array_equal(got, ref[ids[k]]), k
        return
    seen = {}
    for k in range(n):
        for j in ids[rows[k, :counts[k]]]:
            key = (min(ids[k], j), max(ids[k], j))
            assert key not in seen, key  # once only
            seen[key] = 1
    want = {(i, j) for i in range(n) for j in ref[i] if i < j}
    assert set(seen) == want


@pytest.mark.parametrize("csf", [1.0, 0.5])
@pytest.mark.parametrize("half", [0, 1])
def test_verlet_sets_long_box(orc, half, csf):
    """A box long enough in x (39 CSF-1 cells, more than a block and its
    reach) for the single-precision build windows, and anisotropic (1:1/8:1/8,
    so y and z are rescaled when staged): the sets still equal the oracle's."""
    pos, box = _jittered(None, 8, jitter=0.1, shape=(64, 8, 8))
    n = pos.shape[1]
    cfg = make_config(n, box, container=1, newton3=half, precision=0, csf=csf)
    s = DeviceSystem(cfg, pos)
    s.build()
    counts, rows = M.md_get_neighbors(s.h, 256)
    counts = counts.cpu().numpy()
    rows = rows.cpu().numpy()
    ids = s.ids_np()
    ref = orc.neighbor_rows(pos, box, (2.5 + 0.3) ** 2, np.arange(n))
    if not half:
        for k in range(n):
            assert np.array_equal(np.sort(ids[rows[k, :counts[k]]]), ref[ids[k]]), k
        return
    seen = set()
    for k in range(n):
        for j in ids[rows[k, :counts[k]]]:
            key = (min(ids[k], j), max(ids[k], j))
            assert key not in seen, key
            seen.add(key)
    assert seen == {(i, j) for i in range(n) for j in ref[i] if i < j}


def test_verlet_sets_large_cubic_box(orc):
    """A cubic box of 36 CSF-1 cells per side (dilute, 108,000 particles):
    rows of 3000 sampled particles equal the oracle's."""
    rng = np.random.default_rng(12)
    pos, box = W.jittered_fcc(30, 0.1, 0.1, rng)
    n = pos.shape[1]
    cfg = make_config(n, box, container=1, precision=0, max_neighbors=64)
    s = DeviceSystem(cfg, pos)
    s.build()
    counts, rows = M.md_get_neighbors(s.h, 64)
    counts = counts.cpu().numpy()
    rows = rows.cpu().numpy()
    ids = s.ids_np()
    pick = rng.choice(n, 3000, replace=False)
    ref = orc.neighbor_rows(pos, box, (2.5 + 0.3) ** 2, ids[pick])
    assert counts.max() <= 64
    for t, k in enumerate(pick):
        assert np.array_equal(np.sort(ids[rows[k, :counts[k]]]), ref[t]), k


@pytest.mark.parametrize("cont", [(1, 0, 1.0), (1, 1, 1.0), (0, 0, 1.0), (0, 1, 1.0)],
                         ids=["vl", "vl-n3l", "lc", "lc-n3l"])
def test_long_cell_rows(orc, cont):
    """Rows of 244 cells (about 4300 particles, 17 blocks of 256): more blocks
    per band than the packer's counting pass stages, so the writing pass
    packs those bands again.  Forces and pair counts against the oracle;
    for Verlet lists also 1500 sampled rows."""
    pos, box = _jittered(None, 8, jitter=0.1, shape=(400, 8, 8))
    n = pos.shape[1]
    F0, U0, W0, P0 = orc.forces(pos, box, orc.single(), cells=True)
    cfg = make_config(n, box, container=cont[0], newton3=cont[1], csf=cont[2], precision=0)
    s = DeviceSystem(cfg, pos)
    s.build()
    out = s.forces().cpu().numpy()
    assert M.md_get_counters(s.h)["force_family"] == 1  # the windowed kernels ran
    assert int(out[2]) == P0
    assert_forces(s.by_id(s.force), F0, False)
    assert abs(out[0] - U0) <= 1e-6 * abs(U0)
    if cont[0] == 1 and not cont[1]:
        counts, rows = M.md_get_neighbors(s.h, 128)
        counts = counts.cpu().numpy()
        rows = rows.cpu().numpy()
        ids = s.ids_np()
        pick = np.random.default_rng(3).choice(n, 1500, replace=False)
        ref = orc.neighbor_rows(pos, box, (2.5 + 0.3) ** 2, ids[pick])
        for t, k in enumerate(pick):
            assert np.array_equal(np.sort(ids[rows[k, :counts[k]]]), ref[t]), k
    s.h.close()


# ---------------------------------------------------------------- integration

def _run_nve(orc, prec, cont, nsteps=100, R=10, dt=0.005, energy_every=1, d=None, layout=0):
    import torch
    d = d or W.plain_fcc_864()
    pos, vel, box = d["pos"], d["vel"], d["box"]
    n = pos.shape[1]
    cfg = make_config(n, box, container=cont[0], newton3=cont[1], csf=cont[2], precision=prec, R=R,
                      layout=layout)
    s = DeviceSystem(cfg, pos, vel)
    s.build()
    s.forces(energy=False)
    log = torch.zeros((nsteps // energy_every, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, dt, nsteps, energy_every, log)
    torch.cuda.synchronize()
    return s, log.cpu().numpy()


@pytest.mark.parametrize("cont", CONTAINERS, ids=CNAMES)
def test_nve_fp64_trajectory(orc, cont):
    _fp32_only(cont, 1)
    d = W.plain_fcc_864()
    p1, v1, f1, log0 = orc.velocity_verlet(d["pos"], d["vel"], d["box"], orc.single(), 0.005, 100)
    s, log = _run_nve(orc, 1, cont)
    assert np.array_equal(log[:, 3], log0[:, 3])  # pair counts per step
    for k in (0, 1, 2):
        assert np.abs(log[:, k] - log0[:, k]).max() <= 1e-10 * np.abs(log0[:, k]).max()
    x = s.by_id(s.pos)
    dx = x - p1
    dx -= d["box"][:, None] * np.rint(dx / d["box"][:, None])
    assert np.abs(dx).max() < 1e-9
    assert np.abs(s.by_id(s.vel) - v1).max() < 1e-9


@pytest.mark.parametrize("cont", [(1, 0, 1.0), (2, 0, 1.0), (0, 0, 0.5), (3, 0, 1.0), (4, 1, 1.0), (0, 2, 1.0)],
                         ids=["vl", "cl", "lc-csf.5", "pvl", "vlc", "lc-c08"])
def test_nve_fp32_energy_conservation(orc, cont):
    s, log = _run_nve(orc, 0, cont, nsteps=400, R=10)
    u_rc = orc.lj(6.25)[1]
    E = (log[:, 0] - log[:, 3] * u_rc + log[:, 1]) / 864
    assert np.abs(E - E[0]).max() < 5e-3
    slope = np.polyfit(np.arange(len(E)) * 0.005, E, 1)[0]
    assert abs(slope) < 1e-2


def test_fused_integration_matches_separate_steps(orc):
    """Within a block of steps the Verlet-list force pass also integrates
    the next step; a run of single-step calls (each its own block) never
    does.  Both run the same arithmetic, so the trajectories agree bit for
    bit."""
    import torch
    d = W.plain_fcc_864()
    out = []
    for split in (False, True):
        cfg = make_config(864, d["box"], container=1, precision=0, R=5)
        s = DeviceSystem(cfg, d["pos"], d["vel"])
        s.build()
        s.forces(energy=False)
        if split:
            for _ in range(20):
                M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, 1)
        else:
            M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, 20)
        torch.cuda.synchronize()
        assert M.md_get_counters(s.h)["forced_rebuilds"] == 0
        out.append((s.by_id(s.pos), s.by_id(s.vel), s.by_id(s.force)))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("csf", [1.0, 0.5])
def test_cluster_lists_cover_verlet_pairs(orc, csf):
    """Every pair within r_c + skin at the build is a candidate of the cluster
    lists, clusters hold at most 8 particles of one cell, and the pair count of
    the first step equals the oracle's."""
    pos, box = _jittered((6, 7, 8), 21, jitter=0.1)
    n = pos.shape[1]
    cfg = make_config(n, box, container=2, csf=csf)
    s = DeviceSystem(cfg, pos)
    s.build()
    counts, rows = M.md_get_neighbors(s.h, 1024)
    counts, rows = counts.cpu().numpy(), rows.cpu().numpy()
    assert counts.max() <= 1024
    cnt = M.md_get_counters(s.h)
    assert cnt["force_family"] == 2
    ncl_min = -(-n // 8)  # at least this many clusters of at most 8
    assert ncl_min <= cnt["list_entries"] and cnt["list_entries"] * 8 >= int(counts.sum()) // 8
    ids = s.ids_np()
    ref = orc.neighbor_rows(pos, box, (2.5 + 0.3) ** 2, np.arange(n))
    for k in range(n):
        got = set(ids[rows[k, :counts[k]]].tolist())
        assert ids[k] not in got
        assert set(ref[ids[k]].tolist()) <= got, k
    # candidates come in whole clusters: the row length is bounded by 8 per
    # listed cluster, and the list is symmetric at the particle level
    pairs = set()
    for k in range(n):
        for j in ids[rows[k, :counts[k]]]:
            pairs.add((ids[k], j))
    assert all((j, i) in pairs for (i, j) in pairs)


@pytest.mark.parametrize("shape", [(6, 7, 8), (12, 12, 12), (5, 6, 14)], ids=["box678", "box12", "aniso"])
def test_pairwise_lists_cover_verlet_pairs(orc, shape):
    """Pairwise Verlet lists: every pair within r_c + skin at the build lies
    in a particle's candidates (its own cell and, per neighbour cell, the
    stored prefix of that cell's order along the pair's direction), every
    candidate is a neighbour-cell particle, and the prefixes prune: fewer
    candidates than the 27-cell stencil.  Forces and pair count exact."""
    pos, box = _jittered(None, 23, jitter=0.1, shape=shape)
    n = pos.shape[1]
    assert fits((3, 0, 1.0), box)
    cfg = make_config(n, box, container=3)
    s = DeviceSystem(cfg, pos)
    s.build()
    counts, rows = M.md_get_neighbors(s.h, 512)
    counts, rows = counts.cpu().numpy(), rows.cpu().numpy()
    assert counts.max() <= 512
    cnt = M.md_get_counters(s.h)
    assert cnt["list_entries"] == int(counts.sum())
    ids = s.ids_np()
    ref = orc.neighbor_rows(pos, box, (2.5 + 0.3) ** 2, np.arange(n))
    nc = np.floor(box / 2.8).astype(int)
    cell_of, order, start = orc.cells(pos, box, nc)
    stencil = 0
    for k in range(n):
        got = ids[rows[k, :counts[k]]]
        assert len(set(got.tolist())) == len(got)  # no candidate twice
        assert ids[k] not in set(got.tolist())
        assert set(ref[ids[k]].tolist()) <= set(got.tolist()), k
        ci = np.array(np.unravel_index(cell_of[ids[k]], nc[::-1])[::-1])
        for j in got:
            cj = np.array(np.unravel_index(cell_of[j], nc[::-1])[::-1])
            dc = (cj - ci + 1) % nc
            assert (dc <= 2).all(), (k, j)
        stencil += sum(start[c + 1] - start[c] for c in _stencil_cells(ci, nc)) - 1
    assert counts.sum() < 0.5 * stencil
    F0, U0, W0, P0 = orc.forces(pos, box, orc.single())
    out = s.forces().cpu().numpy()
    assert int(out[2]) == P0
    assert_forces(s.by_id(s.force), F0, False)


@pytest.mark.parametrize("shape", [(6, 7, 8), (8, 8, 8), (5, 6, 14)], ids=["box678", "box8", "aniso"])
def test_list_cells_hold_each_pair_once(orc, shape):
    """Verlet list cells: every pair within r_c + skin at the build exactly
    once over all lists (each in the row of the particle whose cell comes
    first in the C08 base step that owns the cell pair), and the C08 colour
    passes give the oracle's forces and pair count.  Box 678 has an odd cell
    count in x (three colours there)."""
    pos, box = _jittered(None, 29, jitter=0.1, shape=shape)
    n = pos.shape[1]
    assert fits((4, 1, 1.0), box)
    cfg = make_config(n, box, container=4, newton3=1)
    s = DeviceSystem(cfg, pos)
    s.build()
    counts, rows = M.md_get_neighbors(s.h, 256)
    counts, rows = counts.cpu().numpy(), rows.cpu().numpy()
    assert counts.max() <= 256
    ids = s.ids_np()
    ref = orc.neighbor_rows(pos, box, (2.5 + 0.3) ** 2, np.arange(n))
    seen = set()
    for k in range(n):
        for j in ids[rows[k, :counts[k]]]:
            key = (min(ids[k], j), max(ids[k], j))
            assert key not in seen, key
            seen.add(key)
    assert seen == {(i, j) for i in range(n) for j in ref[i] if i < j}
    assert M.md_get_counters(s.h)["list_entries"] == len(seen)
    F0, U0, W0, P0 = orc.forces(pos, box, orc.single())
    out = s.forces().cpu().numpy()
    assert int(out[2]) == P0
    assert_forces(s.by_id(s.force), F0, False)
    assert abs(out[0] - U0) <= FP32_E * abs(U0)


def _stencil_cells(ci, nc):
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                c = (ci + np.array([dx, dy, dz])) % nc
                out.append(int((c[2] * nc[1] + c[1]) * nc[0] + c[0]))
    return out


def test_skin_violation_forces_rebuild(orc):
    # R = 200 with skin 0.3 at T = 0.722: particles outgrow skin/2 long before
    # the scheduled rebuild; the replayed steps must reproduce the oracle.
    d = W.plain_fcc_864()
    p1, v1, _, log0 = orc.velocity_verlet(d["pos"], d["vel"], d["box"], orc.single(), 0.005, 150)
    for cont in ((1, 0, 1.0), (0, 0, 1.0)):
        s, log = _run_nve(orc, 1, cont, nsteps=150, R=200)
        cnt = M.md_get_counters(s.h)
        assert cnt["forced_rebuilds"] >= 1
        assert M.md_status(s.h) & M.MD_FLAG_SKIN_EXCEEDED
        assert np.array_equal(log[:, 3], log0[:, 3])
        assert np.abs(log[:, 0] - log0[:, 0]).max() <= 1e-10 * np.abs(log0[:, 0]).max()


def test_skin_violation_replay_fp32(orc):
    """FP32 pairs with replays after skin violations: the trajectory stays on
    the FP64 oracle's within FP32 rounding (a replay that used stale staged
    coordinates would leave it by orders of magnitude)."""
    d = W.plain_fcc_864()
    nsteps = 60
    p1, v1, _, log0 = orc.velocity_verlet(d["pos"], d["vel"], d["box"], orc.single(), 0.005, nsteps)
    for cont in ((1, 0, 1.0), (0, 0, 1.0), (2, 0, 1.0), (1, 1, 1.0)):
        s, log = _run_nve(orc, 0, cont, nsteps=nsteps, R=200)
        cnt = M.md_get_counters(s.h)
        assert cnt["forced_rebuilds"] >= 1, cont
        x = s.by_id(s.pos)
        dx = x - p1
        dx -= d["box"][:, None] * np.rint(dx / d["box"][:, None])
        assert np.abs(dx).max() < 1e-5, cont
        assert np.abs(s.by_id(s.vel) - v1).max() < 1e-3, cont
        assert np.array_equal(log[:20, 3], log0[:20, 3]), cont


@pytest.mark.parametrize("cont", [(1, 0, 20, 78), (2, 0, 4, 20), (4, 1, 13, 39)], ids=["vl", "cl", "vlc"])
def test_list_overflow_grows(orc, cont):
    """Lists built with too small a row overflow; md_step grows the row (the
    list cells' row stride, a multiple of 8, with it), rebuilds and keeps the
    trajectory on the oracle's."""
    import torch
    d = W.plain_fcc_864()
    n = 864
    prec = 0 if cont[0] in (2, 4) else 1
    cfg = make_config(n, d["box"], container=cont[0], newton3=cont[1], precision=prec, max_neighbors=cont[2])
    s = DeviceSystem(cfg, d["pos"], d["vel"])
    s.build()
    s.forces(energy=False)  # truncated lists give wrong forces, and a flag
    assert M.md_status(s.h) & M.MD_FLAG_LIST_OVERFLOW
    # md_step knows the lists were truncated: it grows them, rebuilds and
    # recomputes the entry forces, so the trajectory is exact
    p1, v1, _, log0 = orc.velocity_verlet(d["pos"], d["vel"], d["box"], orc.single(), 0.005, 30)
    log = torch.zeros((30, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, 30, 1, log)
    log = log.cpu().numpy()
    assert M.md_get_config(s.h).max_neighbors >= cont[3]
    if prec == 1:
        assert np.array_equal(log[:, 3], log0[:, 3])
        assert np.abs(log[:, 0] - log0[:, 0]).max() <= 1e-10 * np.abs(log0[:, 0]).max()
    else:
        # FP32 pair arithmetic: the first steps still match the FP64 oracle
        assert np.array_equal(log[:5, 3], log0[:5, 3])
        assert np.abs(log[:5, 0] - log0[:5, 0]).max() <= 1e-6 * np.abs(log0[:5, 0]).max()
    assert not (M.md_status(s.h) & M.MD_FLAG_LIST_OVERFLOW)


# ---------------------------------------------------------------- live statistics

def test_live_stats(orc):
    d = W.droplet(n=20000, seed=3)
    cfg = make_config(20000, d["box"], container=0)
    s = DeviceSystem(cfg, d["pos"])
    st = M.md_live_stats(s.h, s.pos)
    ref = orc.live_stats(d["pos"], d["box"], 2.8)
    assert st[0] == pytest.approx(ref[0], rel=1e-14)
    assert st[1] == pytest.approx(ref[1], rel=1e-12)
    assert st[2:6] == list(ref[2:6])
    assert st[6] >= 1 and st[7] == 0.3


# ---------------------------------------------------------------- adjoint

@pytest.mark.parametrize("prec,cont", [(1, (0, 0)), (0, (0, 0)), (0, (1, 0)), (0, (0, 1)), (0, (2, 0))],
                         ids=["fp64", "fp32-lc", "fp32-vl", "fp32-lc-n3l", "fp32-cl"])
def test_adjoint_matches_oracle(orc, prec, cont):
    """dL/dx and dL/d(eps, sigma) of the force-matching loss against the
    oracle: FP32 gather structures run the windowed adjoint (over the Verlet
    lists for Verlet lists, over the cut stencil for linked cells), the others
    (and FP64) the per-particle kernel."""
    import torch
    d = W.binary_mixture(ncell=6, seed=11)
    pos, box, types = d["pos"], d["box"], d["types"]
    n = pos.shape[1]
    theta0 = np.array(d["eps"] + d["sig"])
    e0, s0 = orc.mix(d["eps"], d["sig"])
    rc2 = (2.5 * s0) ** 2
    _, target, _, _ = orc.force_matching(pos, box, types, theta0, rc2, np.zeros((3, n)))
    theta = W.perturb_params(theta0, seed=2)
    L, F, gx, gt = orc.force_matching(pos, box, types, theta, rc2, target)
    cfg = make_config(n, box, container=cont[0], newton3=cont[1], precision=prec, n_types=2, rc2=rc2)
    s = DeviceSystem(cfg, pos, types=types, eps=list(theta[:2]), sig=list(theta[2:]))
    s.build()
    s.forces(energy=False)
    ids = s.ids_np()
    Fd = s.force.to(torch.float64)
    tgt = torch.tensor(target[:, ids], device="cuda")
    g = (2.0 / (3 * n)) * (Fd - tgt)
    g = g.to(s.h.real).contiguous()
    gpos = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    glj = torch.zeros(4, dtype=torch.float64, device="cuda")
    M.md_forces_backward(s.h, s.pos, s.type, s.lj, g, gpos, glj)
    torch.cuda.synchronize()
    tol_x, tol_t = (1e-12, 1e-12) if prec == 1 else (1e-4, 1e-5)
    assert rel_l2(s.by_id(gpos), gx) <= tol_x
    assert rel_l2(glj.cpu().numpy(), gt) <= tol_t


def test_adjoint_over_truncated_lists(orc):
    """Verlet lists built with too small a row (max_neighbors 8, so that the
    build overflows and sets MD_FLAG_LIST_OVERFLOW): the adjoint does not walk
    the truncated lists but the stencil, decided on the device, and still
    matches the oracle.  The loss gradient g is the oracle's (the forward pass
    over the truncated lists is not what is tested here)."""
    import torch
    d = W.binary_mixture(ncell=6, seed=11)
    pos, box, types = d["pos"], d["box"], d["types"]
    n = pos.shape[1]
    theta0 = np.array(d["eps"] + d["sig"])
    e0, s0 = orc.mix(d["eps"], d["sig"])
    rc2 = (2.5 * s0) ** 2
    _, target, _, _ = orc.force_matching(pos, box, types, theta0, rc2, np.zeros((3, n)))
    theta = W.perturb_params(theta0, seed=2)
    L, F, gx, gt = orc.force_matching(pos, box, types, theta, rc2, target)
    cfg = make_config(n, box, container=1, precision=0, n_types=2, rc2=rc2, max_neighbors=8)
    s = DeviceSystem(cfg, pos, types=types, eps=list(theta[:2]), sig=list(theta[2:]))
    s.build()
    torch.cuda.synchronize()
    ids = s.ids_np()
    g = torch.tensor((2.0 / (3 * n)) * (F - target)[:, ids], device="cuda").to(s.h.real).contiguous()
    gpos = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    glj = torch.zeros(4, dtype=torch.float64, device="cuda")
    M.md_forces_backward(s.h, s.pos, s.type, s.lj, g, gpos, glj)
    torch.cuda.synchronize()
    assert M.md_status(s.h) & M.MD_FLAG_LIST_OVERFLOW
    assert rel_l2(s.by_id(gpos), gx) <= 1e-4
    assert rel_l2(glj.cpu().numpy(), gt) <= 1e-5


@pytest.mark.parametrize("cont", [(0, 0, 1.0), (1, 0, 1.0)], ids=["lc", "vl"])
def test_forces_and_adjoint_between_builds(orc, cont):
    """Between builds the particles move by up to half the skin, while the
    stencil rows of the linked-cell force and of the adjoint (ordered by x
    when the cells were built) are cut by x with that motion as margin.  A hot
    binary mixture (T = 3, five cells per dimension, so the rows are cut) is
    stepped one step per call: the FP32 forces after every step, and the
    adjoint at the end (its structure built steps earlier), match the oracle
    at the current positions."""
    import torch
    d = W.binary_mixture(ncell=10, seed=5, T=3.0)
    pos, vel, box, types = d["pos"], d["vel"], d["box"], d["types"]
    n = pos.shape[1]
    theta0 = np.array(d["eps"] + d["sig"])
    e0, s0 = orc.mix(d["eps"], d["sig"])
    rc2 = (2.5 * s0) ** 2
    assert int(box[0] // 2.8) >= 5
    cfg = make_config(n, box, container=cont[0], newton3=cont[1], csf=cont[2], n_types=2, rc2=rc2, R=8)
    s = DeviceSystem(cfg, pos, vel, types=types, eps=d["eps"], sig=d["sig"])
    s.build()
    s.forces(energy=False)
    log = torch.zeros((1, 4), dtype=torch.float64, device="cuda")
    moved = 0.0
    for step in range(12):
        M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, 1, 1, log)
        torch.cuda.synchronize()
        p = s.by_id(s.pos)
        _, F0, _, _ = orc.force_matching(p, box, types, theta0, rc2, np.zeros((3, n)))
        assert_forces(s.by_id(s.force), F0, False, what=step)
        dp = p - pos
        dp -= box[:, None] * np.rint(dp / box[:, None])
        moved = max(moved, float(np.sqrt((dp ** 2).sum(axis=0)).max()))
    cnt = M.md_get_counters(s.h)
    assert cnt["rebuilds"] < 13  # the structure was reused between builds
    assert moved > 0.15  # the run went past half the skin: the skin check rebuilt it
    # the adjoint at the final positions, on the structure as it stands
    p = s.by_id(s.pos)
    _, target, _, _ = orc.force_matching(p, box, types, theta0, rc2, np.zeros((3, n)))
    theta = W.perturb_params(theta0, seed=2)
    _, F, gx, gt = orc.force_matching(p, box, types, theta, rc2, target)
    s.lj.copy_(torch.tensor(theta, dtype=torch.float64))
    s.forces(energy=False)
    assert_forces(s.by_id(s.force), F, False, what="perturbed")
    ids = s.ids_np()
    g = ((2.0 / (3 * n)) * (s.force.to(torch.float64) - torch.tensor(target[:, ids], device="cuda")))
    g = g.to(s.h.real).contiguous()
    gpos = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    glj = torch.zeros(4, dtype=torch.float64, device="cuda")
    M.md_forces_backward(s.h, s.pos, s.type, s.lj, g, gpos, glj)
    torch.cuda.synchronize()
    assert rel_l2(s.by_id(gpos), gx) <= 1e-4
    assert rel_l2(glj.cpu().numpy(), gt) <= 1e-5


@pytest.mark.parametrize("layout", [1, 2], ids=["aligned", "soa"])
def test_window_layouts(orc, layout):
    """The Verlet-list force over LDS windows of 16-byte entries or of one
    plane per coordinate (Sec. 2.2.3's layout choice): the same Verlet sets,
    pair counts and forces as the oracle on jittered lattices of several
    sizes, a long anisotropic box included, and energy conserved over an NVE
    run (the fused integrator reads the same windows)."""
    import torch
    for shape, seed in (((6, 7, 8), 4), ((39, 5, 5), 6), ((8, 8, 8), 9)):
        pos, box = _jittered(None, seed, jitter=0.1, shape=shape)
        n = pos.shape[1]
        F0, U0, W0, P0 = orc.forces(pos, box, orc.single())
        cfg = make_config(n, box, container=1, layout=layout)
        s = DeviceSystem(cfg, pos)
        s.build()
        out = s.forces().cpu().numpy()
        assert int(out[2]) == P0, shape
        assert_forces(s.by_id(s.force), F0, False, what=(shape, layout))
        assert abs(out[0] - U0) <= FP32_E * abs(U0)
        assert M.md_get_counters(s.h)["force_family"] == 1  # the windowed kernels ran
        counts, rows = M.md_get_neighbors(s.h, 160)
        counts, rows = counts.cpu().numpy(), rows.cpu().numpy()
        ids = s.ids_np()
        ref = orc.neighbor_rows(pos, box, (2.5 + 0.3) ** 2, np.arange(n))
        for k in range(0, n, 7):
            assert np.array_equal(np.sort(ids[rows[k, :counts[k]]]), ref[ids[k]]), (shape, k)
    # NVE: fused and plain passes over the layout's windows
    s, log = _run_nve(orc, 0, (1, 0, 1.0), nsteps=200, R=10, layout=layout)
    u_rc = orc.lj(6.25)[1]
    E = (log[:, 0] - log[:, 3] * u_rc + log[:, 1]) / 864
    assert np.abs(E - E[0]).max() < 5e-3
    # other containers and two types refuse the other layouts
    d = W.plain_fcc_864()
    for bad in (dict(container=0), dict(container=1, newton3=1), dict(container=1, precision=1),
                dict(container=1, n_types=2)):
        with pytest.raises(RuntimeError, match="layout"):
            M.md_create(make_config(864, d["box"], layout=layout, **bad))


# ---------------------------------------------------------------- full-size fluid

def test_fluid_1m_full_size(orc):
    """The headline workload at its full size, in the configuration the
    benchmark times: all forces against the oracle's linked-cell FP64 forces
    (same pair set as brute force), pair count exact, sampled Verlet rows exact."""
    d = W.homogeneous_fluid()
    pos, box = d["pos"], d["box"]
    n = pos.shape[1]
    F0, U0, W0, P0 = orc.forces(pos, box, orc.single(), cells=True)
    for cont in ((1, 0, 1.0), (0, 0, 1.0), (2, 0, 1.0), (1, 0, 0.5), (1, 1, 0.5), (0, 1, 0.5)):
        cfg = make_config(n, box, container=cont[0], newton3=cont[1], csf=cont[2])
        s = DeviceSystem(cfg, pos)
        s.build()
        out = s.forces().cpu().numpy()
        assert int(out[2]) == P0
        assert_forces(s.by_id(s.force), F0, False, what=cont)
        assert abs(out[0] - U0) <= FP32_E * abs(U0)
        if cont[0] == 1 and cont[1] == 0:
            counts, rows = M.md_get_neighbors(s.h, 160)
            counts, rows = counts.cpu().numpy(), rows.cpu().numpy()
            ids = s.ids_np()
            pos_of = np.empty(n, np.int64)
            pos_of[ids] = np.arange(n)
            sample = np.random.default_rng(0).choice(n, 256, replace=False)
            ref = orc.neighbor_rows(pos, box, (2.5 + 0.3) ** 2, sample)
            for i, want in zip(sample, ref):
                k = pos_of[i]
                assert np.array_equal(np.sort(ids[rows[k, :counts[k]]]), want)


# ---------------------------------------------------------------- autograd

@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
def test_autograd_function_force_matching(orc, prec):
    """LJForces under torch.autograd: the gradient of the force-matching loss
    with respect to positions and the four (eps, sigma) equals the oracle's
    analytic gradient (itself pinned to central differences)."""
    import torch
    from paper_2505_03438_amd.autograd import lj_forces
    d = W.binary_mixture(ncell=6, seed=13)
    pos, box, types = d["pos"], d["box"], d["types"]
    n = pos.shape[1]
    theta0 = np.array(d["eps"] + d["sig"])
    e0, s0 = orc.mix(d["eps"], d["sig"])
    rc2 = (2.5 * s0) ** 2
    _, target, _, _ = orc.force_matching(pos, box, types, theta0, rc2, np.zeros((3, n)))
    theta = W.perturb_params(theta0, seed=5)
    L0, _, gx, gt = orc.force_matching(pos, box, types, theta, rc2, target)
    cfg = make_config(n, box, container=0, precision=prec, n_types=2, rc2=rc2)
    s = DeviceSystem(cfg, pos, types=types, eps=list(theta[:2]), sig=list(theta[2:]))
    s.build()
    ids = s.ids_np()
    x = s.pos.clone().requires_grad_(True)
    lj = s.lj.clone().requires_grad_(True)
    F = lj_forces(s.h, x, s.type, lj)
    tgt = torch.tensor(target[:, ids], device="cuda")
    loss = ((F.to(torch.float64) - tgt) ** 2).sum() / (3 * n)
    loss.backward()
    torch.cuda.synchronize()
    tol_l, tol_x, tol_t = (1e-12, 1e-12, 1e-12) if prec == 1 else (1e-3, 1e-4, 1e-5)
    assert abs(loss.item() - L0) <= tol_l * abs(L0)
    assert rel_l2(s.by_id(x.grad), gx) <= tol_x
    assert rel_l2(lj.grad.cpu().numpy(), gt) <= tol_t


# ---------------------------------------------------------------- autotuned runs

@pytest.mark.parametrize("strategy", [1, 2], ids=["full", "predictive"])
def test_autotuned_fp64_trajectory(orc, strategy):
    """md_step with the run-time configuration selection: every trial step
    advances the simulation, so the trajectory (pair counts, energies,
    positions) equals the oracle's whatever configurations are chosen."""
    import torch
    d = W.plain_fcc_864()
    nsteps = 150
    p1, v1, _, log0 = orc.velocity_verlet(d["pos"], d["vel"], d["box"], orc.single(), 0.005, nsteps)
    n = 864
    cfg = make_config(n, d["box"], container=0, precision=1, R=10)
    cfg.autotune = strategy
    cfg.tune_interval = 40
    cfg.tune_trial_steps = 3
    cfg.total_steps_hint = nsteps
    s = DeviceSystem(cfg, d["pos"], d["vel"])
    s.build()
    s.forces(energy=False)
    log = torch.zeros((nsteps, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, nsteps, 1, log)
    torch.cuda.synchronize()
    log = log.cpu().numpy()
    cnt = M.md_get_counters(s.h)
    assert cnt["tuning_phases"] >= 3
    assert cnt["trials"] >= 6 * 2  # the first two phases trial every configuration
    assert 1 <= M.md_get_config(s.h).rebuild_interval <= 100
    assert np.array_equal(log[:, 3], log0[:, 3])
    for k in (0, 1, 2):
        assert np.abs(log[:, k] - log0[:, k]).max() <= 1e-10 * np.abs(log0[:, k]).max()
    dx = s.by_id(s.pos) - p1
    dx -= d["box"][:, None] * np.rint(dx / d["box"][:, None])
    assert np.abs(dx).max() < 1e-9


@pytest.mark.parametrize("strategy", [4, 2, 1, 3], ids=["forest", "predictive", "full", "expert"])
def test_short_run_tunes(orc, strategy):
    """A short run (5 warm-up steps, then 20 steps, as the benchmark line is
    run) still holds a tuning phase: the first phase is put at the first step
    after the warm-up (tune_first), and a phase is postponed only when the
    trials the strategy asks for (one for the forest, every structure for
    Full Search and the first Predictive phases) do not fit into the call.
    The trial steps advance the simulation: the FP64 trajectory equals the
    oracle's."""
    import torch
    d = W.plain_fcc_864()
    warm, nsteps = 5, 20
    p1, v1, _, log0 = orc.velocity_verlet(d["pos"], d["vel"], d["box"], orc.single(), 0.005, warm + nsteps)
    n = 864
    cfg = make_config(n, d["box"], container=0, precision=1, R=10)
    cfg.autotune = strategy
    space = 1 if strategy == M.MD_TUNE_RF else 6
    cfg.tune_first = warm
    cfg.tune_interval = nsteps // 2
    cfg.tune_trial_steps = max(2, min(10, nsteps // (2 * space)))
    cfg.total_steps_hint = nsteps
    s = DeviceSystem(cfg, d["pos"], d["vel"])
    s.build()
    s.forces(energy=False)
    log_w = torch.zeros((warm, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, warm, 1, log_w)
    torch.cuda.synchronize()
    assert M.md_get_counters(s.h)["tuning_phases"] == 0  # none during the warm-up
    log = torch.zeros((nsteps, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, nsteps, 1, log)
    torch.cuda.synchronize()
    log = np.concatenate([log_w.cpu().numpy(), log.cpu().numpy()])
    cnt = M.md_get_counters(s.h)
    assert cnt["tuning_phases"] >= 1 and cnt["trials"] >= 1, cnt
    if strategy == M.MD_TUNE_RF:
        assert cnt["tuning_phases"] == 2 and cnt["trials"] == 2, cnt
    if strategy == M.MD_TUNE_FULL:
        assert cnt["trials"] == 6, cnt  # one phase of every structure; the second does not fit
    assert cnt["config_index"] >= 0
    assert np.array_equal(log[:, 3], log0[:, 3])
    for k in (0, 1, 2):
        assert np.abs(log[:, k] - log0[:, k]).max() <= 1e-10 * np.abs(log0[:, k]).max()
    dx = s.by_id(s.pos) - p1
    dx -= d["box"][:, None] * np.rint(dx / d["box"][:, None])
    assert np.abs(dx).max() < 1e-9


INF = float("inf")


@pytest.mark.parametrize("rules", ["builtin", "lc_pair", "histogram"])
def test_expert_strategy_fp64_trajectory(orc, rules):
    """Expert strategy (fuzzy rules over the live statistics): only the
    configurations the rules mark as suited are trialled, the fastest of
    them is kept, and the trajectory equals the oracle's whatever is chosen.
    "histogram": a rule on the spread of the bin counts, so each phase runs
    the bin histogram over the cell arrays before its trials rebuild them."""
    import torch
    d = W.plain_fcc_864()
    nsteps = 150
    p1, v1, _, log0 = orc.velocity_verlet(d["pos"], d["vel"], d["box"], orc.single(), 0.005, nsteps)
    n = 864
    cfg = make_config(n, d["box"], container=0, precision=1, R=10)
    cfg.autotune = M.MD_TUNE_EXPERT
    cfg.tune_interval = 40
    cfg.tune_trial_steps = 3
    cfg.total_steps_hint = nsteps
    s = DeviceSystem(cfg, d["pos"], d["vel"])
    every = (0, (-INF, -INF, INF, INF))
    if rules == "builtin":
        suited = [4]  # 32 particles per bin: dense, Verlet lists gather-only
    elif rules == "lc_pair":
        M.md_set_expert_rules(s.h, [{"if": [every], "config": 0, "then": M.MD_SUIT_GOOD},
                                    {"if": [every], "config": 2, "then": M.MD_SUIT_GOOD},
                                    {"if": [every], "config": 4, "then": M.MD_SUIT_OKAY}])
        suited = [0, 2]
    else:
        M.md_set_expert_rules(s.h, [{"if": [(1, (-INF, -INF, 1.0, 2.0)), (3, (0.0, 1.0, 1e9, 2e9))],
                                     "config": 1, "then": M.MD_SUIT_GOOD}])
        suited = [1]
    s.build()
    s.forces(energy=False)
    log = torch.zeros((nsteps, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, nsteps, 1, log)
    torch.cuda.synchronize()
    log = log.cpu().numpy()
    cnt = M.md_get_counters(s.h)
    assert cnt["tuning_phases"] == 4
    assert cnt["trials"] == 4 * len(suited)
    assert cnt["config_index"] in suited
    scores, cfgs = M.md_get_trial_scores(s.h)
    assert len(scores) == 6  # FP64: no cluster lists
    assert [k for k in range(6) if np.isfinite(scores[k])] == suited
    assert all(scores[k] > 0.0 for k in suited)
    assert int(cfgs[4].container) == M.MD_CONTAINER_VL and int(cfgs[4].newton3) == 0
    assert np.array_equal(log[:, 3], log0[:, 3])
    for k in (0, 1, 2):
        assert np.abs(log[:, k] - log0[:, k]).max() <= 1e-10 * np.abs(log0[:, k]).max()
    dx = s.by_id(s.pos) - p1
    dx -= d["box"][:, None] * np.rint(dx / d["box"][:, None])
    assert np.abs(dx).max() < 1e-9
    s.h.close()


def test_reselection_as_liquid_explodes(orc):
    """Re-selection as the load imbalance changes (the exploding liquid of
    Sec. 6.2): a hot liquid cube (864 particles, T = 4) expands into a box
    27 times its volume.  Expert rules over the relative spread of the bin
    counts (a Sec. 4 statistic) call linked cells at CSF 1/2 suitable while
    the particles are clumped (spread >= 3) and Verlet lists once they have
    spread out; a phase every 60 steps.  The phases choose the first, then
    the second, as the spread falls from 4.0 to 2.1 (the oracle's spread
    crosses 3 between steps 180 and 240), and every step of the FP64
    trajectory equals the oracle's."""
    import torch
    rng = np.random.default_rng(7)
    pos, cube = W.jittered_fcc(6, 0.8, 0.05, rng)
    Lb = 30.0
    pos = pos + (Lb - cube[0]) / 2
    box = np.array([Lb] * 3)
    vel = W.maxwell_boltzmann(pos.shape[1], 4.0, rng)
    n = pos.shape[1]
    nsteps = 600
    p1, v1, _, log0 = orc.velocity_verlet(pos, vel, box, orc.single(), 0.005, nsteps)
    cfg = make_config(n, box, container=0, precision=1, R=10)
    cfg.autotune = M.MD_TUNE_EXPERT
    cfg.tune_interval = 60
    cfg.tune_trial_steps = 3
    cfg.total_steps_hint = nsteps
    s = DeviceSystem(cfg, pos, vel)
    clumped, spread = (1, (3.0, 3.0, INF, INF)), (1, (-INF, -INF, 3.0, 3.0))
    M.md_set_expert_rules(s.h, [{"if": [clumped], "config": 2, "then": M.MD_SUIT_GOOD},
                                {"if": [spread], "config": 2, "then": M.MD_SUIT_BAD},
                                {"if": [spread], "config": 4, "then": M.MD_SUIT_GOOD},
                                {"if": [clumped], "config": 4, "then": M.MD_SUIT_BAD}])
    s.build()
    s.forces(energy=False)
    log = torch.zeros((nsteps, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, nsteps, 1, log)
    torch.cuda.synchronize()
    choices = M.md_get_phase_choices(s.h)
    assert choices == [2, 2, 2, 2, 4, 4, 4, 4, 4, 4], choices
    _, cfgs = M.md_get_trial_scores(s.h)
    assert (int(cfgs[2].container), float(cfgs[2].csf)) == (M.MD_CONTAINER_LC, 0.5)
    assert int(cfgs[4].container) == M.MD_CONTAINER_VL
    log = log.cpu().numpy()
    assert np.array_equal(log[:, 3], log0[:, 3])
    for k in (0, 1, 2):
        assert np.abs(log[:, k] - log0[:, k]).max() <= 1e-10 * np.abs(log0[:, k]).max()
    dx = s.by_id(s.pos) - p1
    dx -= box[:, None] * np.rint(dx / box[:, None])
    assert np.abs(dx).max() < 1e-9
    s.h.close()


def test_skin_tuning_fp64_trajectory(orc):
    """Joint skin / rebuild-interval search: the tuning space gains Verlet
    lists at 2/3, 4/3 and 5/3 of the skin; Full Search trials them all, and
    the trajectory still equals the oracle's (the skin changes the work, not
    the forces)."""
    import torch
    d = W.plain_fcc_864()
    nsteps = 120
    p1, v1, _, log0 = orc.velocity_verlet(d["pos"], d["vel"], d["box"], orc.single(), 0.005, nsteps)
    cfg = make_config(864, d["box"], container=0, precision=1, R=10)
    cfg.autotune = M.MD_TUNE_FULL
    cfg.tune_skin = 1
    cfg.tune_interval = 60
    cfg.tune_trial_steps = 3
    cfg.total_steps_hint = nsteps
    s = DeviceSystem(cfg, d["pos"], d["vel"])
    scores, cfgs = M.md_get_trial_scores(s.h)
    assert len(scores) == 9 and all(np.isnan(scores))
    assert [round(float(c.skin), 12) for c in cfgs[6:]] == [0.2, 0.4, 0.5]
    assert all(int(c.container) == M.MD_CONTAINER_VL for c in cfgs[6:])
    s.build()
    s.forces(energy=False)
    log = torch.zeros((nsteps, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, nsteps, 1, log)
    torch.cuda.synchronize()
    log = log.cpu().numpy()
    cnt = M.md_get_counters(s.h)
    assert cnt["tuning_phases"] == 2 and cnt["trials"] == 18
    scores, _ = M.md_get_trial_scores(s.h)
    assert all(np.isfinite(scores))
    assert abs(float(M.md_get_config(s.h).skin) - float(cfgs[cnt["config_index"]].skin)) < 1e-15
    assert np.array_equal(log[:, 3], log0[:, 3])
    for k in (0, 1, 2):
        assert np.abs(log[:, k] - log0[:, k]).max() <= 1e-10 * np.abs(log0[:, k]).max()
    dx = s.by_id(s.pos) - p1
    dx -= d["box"][:, None] * np.rint(dx / d["box"][:, None])
    assert np.abs(dx).max() < 1e-9
    s.h.close()


@pytest.mark.parametrize("strategy", ["forest", "expert"])
def test_named_structure_trials_its_skins(orc, strategy):
    """With the skin tuned, the structure the forest (or the rules) names is
    trialled at every skin of the space: Verlet lists at 0.3 and at 0.2, 0.4
    and 0.5 in each phase, nothing else for the forest; the trajectory still
    equals the oracle's."""
    import torch
    d = W.plain_fcc_864()
    nsteps = 120
    p1, v1, _, log0 = orc.velocity_verlet(d["pos"], d["vel"], d["box"], orc.single(), 0.005, nsteps)
    cfg = make_config(864, d["box"], container=0, precision=1, R=10)
    cfg.autotune = M.MD_TUNE_RF if strategy == "forest" else M.MD_TUNE_EXPERT
    cfg.tune_skin = 1
    cfg.tune_interval = 60
    cfg.tune_trial_steps = 3
    cfg.total_steps_hint = nsteps
    s = DeviceSystem(cfg, d["pos"], d["vel"])
    s.build()
    s.forces(energy=False)
    log = torch.zeros((nsteps, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, nsteps, 1, log)
    torch.cuda.synchronize()
    log = log.cpu().numpy()
    cnt = M.md_get_counters(s.h)
    scores, cfgs = M.md_get_trial_scores(s.h)
    vl = [k for k, c in enumerate(cfgs) if int(c.container) == M.MD_CONTAINER_VL and int(c.newton3) == 0]
    assert len(vl) == 4
    assert cnt["tuning_phases"] == 2
    assert all(np.isfinite(scores[k]) for k in vl)
    if strategy == "forest":
        assert cnt["trials"] == 8
        assert all(np.isnan(scores[k]) for k in range(len(cfgs)) if k not in vl)
    assert cnt["config_index"] in vl
    assert np.array_equal(log[:, 3], log0[:, 3])
    for k in (0, 1, 2):
        assert np.abs(log[:, k] - log0[:, k]).max() <= 1e-10 * np.abs(log0[:, k]).max()
    dx = s.by_id(s.pos) - p1
    dx -= d["box"][:, None] * np.rint(dx / d["box"][:, None])
    assert np.abs(dx).max() < 1e-9
    s.h.close()


def test_random_forest_strategy_fp64_trajectory(orc):
    """Random Forest strategy: each phase reads the live statistics, the
    forest names one configuration, and that one alone is trialled and kept;
    the trajectory equals the oracle's."""
    import torch
    d = W.plain_fcc_864()
    nsteps = 120
    p1, v1, _, log0 = orc.velocity_verlet(d["pos"], d["vel"], d["box"], orc.single(), 0.005, nsteps)
    cfg = make_config(864, d["box"], container=0, precision=1, R=10)
    cfg.autotune = M.MD_TUNE_RF
    cfg.tune_interval = 40
    cfg.tune_trial_steps = 3
    cfg.total_steps_hint = nsteps
    s = DeviceSystem(cfg, d["pos"], d["vel"])
    st = M.md_live_stats(s.h, s.pos)
    want = M.md_rf_predict(st, 6)
    s.build()
    s.forces(energy=False)
    log = torch.zeros((nsteps, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, nsteps, 1, log)
    torch.cuda.synchronize()
    log = log.cpu().numpy()
    cnt = M.md_get_counters(s.h)
    assert cnt["tuning_phases"] == 3 and cnt["trials"] == 3
    assert cnt["config_index"] == want
    assert np.array_equal(log[:, 3], log0[:, 3])
    for k in (0, 1, 2):
        assert np.abs(log[:, k] - log0[:, k]).max() <= 1e-10 * np.abs(log0[:, k]).max()
    dx = s.by_id(s.pos) - p1
    dx -= d["box"][:, None] * np.rint(dx / d["box"][:, None])
    assert np.abs(dx).max() < 1e-9
    s.h.close()


def test_random_forest_picks_cluster_lists_for_small_sparse_gas(orc):
    """A small dilute system (the family where cluster lists won the
    training trials): the forest picks cluster lists, which then run with
    the energy conserved."""
    import torch
    rng = np.random.default_rng(31)
    pos, box = W.thinned_fcc(16, 1.0, lambda sites, L: np.full(sites.shape[1], 0.1), rng)
    n = pos.shape[1]
    vel = W.maxwell_boltzmann(n, 1.0, rng)
    cfg = make_config(n, box, container=0, precision=0, R=10)
    cfg.autotune = M.MD_TUNE_RF
    cfg.tune_interval = 500  # one phase, at the start
    cfg.tune_trial_steps = 5
    cfg.total_steps_hint = 200
    s = DeviceSystem(cfg, pos, vel)
    st = M.md_live_stats(s.h, s.pos)
    assert M.md_rf_predict(st, 7) == 6
    s.build()
    s.forces(energy=False)
    log = torch.zeros((200, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, 200, 1, log)
    torch.cuda.synchronize()
    log = log.cpu().numpy()
    cnt = M.md_get_counters(s.h)
    assert cnt["config_index"] == 6 and cnt["trials"] == 1 and cnt["force_family"] == 2
    u_rc = orc.lj(6.25)[1]
    E = (log[:, 0] - log[:, 3] * u_rc + log[:, 1]) / n
    assert np.abs(E - E[0]).max() < 5e-3
    s.h.close()


def test_expert_rules_rejected_for_untuned_handle(orc):
    d = W.plain_fcc_864()
    s = DeviceSystem(make_config(864, d["box"], container=0, precision=1), d["pos"])
    with pytest.raises(RuntimeError, match="does not tune"):
        M.md_set_expert_rules(s.h, None)
    with pytest.raises(RuntimeError, match="does not tune"):
        M.md_get_trial_scores(s.h)
    s.h.close()


def test_autotuned_fp32_energy_conservation(orc):
    """FP32 autotuned run over all ten configurations (cluster lists,
    pairwise lists, list cells and the C08 traversal included): the total
    energy stays conserved across configuration switches."""
    import torch
    d = W.plain_fcc_864()
    nsteps = 400
    cfg = make_config(864, d["box"], container=0, precision=0, R=10)
    cfg.autotune = 2
    cfg.tune_interval = 100
    cfg.tune_trial_steps = 4
    cfg.total_steps_hint = nsteps
    s = DeviceSystem(cfg, d["pos"], d["vel"])
    s.build()
    s.forces(energy=False)
    log = torch.zeros((nsteps, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, 0.005, nsteps, 1, log)
    torch.cuda.synchronize()
    log = log.cpu().numpy()
    assert M.md_get_counters(s.h)["trials"] >= 20
    u_rc = orc.lj(6.25)[1]
    E = (log[:, 0] - log[:, 3] * u_rc + log[:, 1]) / 864
    assert np.abs(E - E[0]).max() < 5e-3
