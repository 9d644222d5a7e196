"""Constructed edge cases of the pair decisions, on every container and both
precisions, element by element against the FP64 oracle.

* Pairs at r = r_c exactly (excluded: the cutoff is strict), one ulp inside
  and outside it, and at r^2 = r_c^2 (1 + k 2^-21) for k = -12 .. 12, which
  crosses both edges of the FP32 path's guard band (|r^2 - r_c^2| <=
  2^-19 r_c^2, inside which r^2 is recomputed from the FP64 positions).
* The same around the list radius r_c + skin (the Verlet set, whose build
  decides in FP64 inside a wider band of 2^-15).
* Particles on the box faces: x = 0 and x = nextafter(L, 0) in each
  dimension (the fixed-point staging must wrap x -> L to 0, the cell index
  must clamp to the last cell), and pairs across the periodic boundary.
* A box of exactly 2 (r_c + skin) with a pair at |d| = L/2: the minimum
  image keeps +L/2, and r = r_c + skin is outside the list (strict).

Isolated pairs sit on a grid far apart, so each pair's force is the analytic
one; a liquid background with pairs moved onto the same distances puts the
band candidates among ordinary ones (the kernels test candidates in batches).
Pair counts are exact, the Verlet sets equal the oracle's rows, and forces
meet the relative-L2 and per-particle bars."""
import numpy as np
import pytest

from paper_2505_03438_amd import workloads as W
from tests.gpu_util import DeviceSystem, assert_forces, make_config

M = None


@pytest.fixture(scope="module")
def lib():
    global M
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_03438_amd import mdlj
    mdlj.lib()
    M = mdlj


RC, SKIN = 2.5, 0.3
RL = RC + SKIN

# (container, newton3, csf); newton3 2 is the C08 traversal of linked cells
CONTAINERS = [(0, 0, 1.0), (0, 1, 1.0), (0, 0, 0.5), (0, 1, 0.5), (1, 0, 1.0), (1, 1, 1.0), (1, 0, 0.5),
              (1, 1, 0.5), (2, 0, 1.0), (0, 2, 1.0)]
CNAMES = ["lc", "lc-n3l", "lc-csf.5", "lc-n3l-csf.5", "vl", "vl-n3l", "vl-csf.5", "vl-n3l-csf.5", "cl", "lc-c08"]


def _separations():
    """Distances at and around the cutoff and the list radius."""
    s = [RC, np.nextafter(RC, 0.0), np.nextafter(RC, 9.0), RL, np.nextafter(RL, 0.0), np.nextafter(RL, 9.0)]
    s += [RC * np.sqrt(1.0 + k * 2.0 ** -21) for k in range(-12, 13)]
    s += [RL * np.sqrt(1.0 + k * 2.0 ** -17) for k in range(-6, 7)]
    s += [RC * (1.0 + 2.0 ** -19), RC * (1.0 - 2.0 ** -19), RC * (1.0 + 2.0 ** -20), RC * (1.0 - 2.0 ** -20)]
    return np.array(s)


def isolated_pairs():
    """One pair per separation, far from every other (anchor coordinate 0.5
    on the offset axis, so that anchor + separation is exact: both lie in
    [2, 4)); plus pairs of face particles and pairs across the x face."""
    seps = _separations()
    L = 72.0
    anchors = []
    for j in range(5):  # offset along x
        for k in range(5):
            anchors.append(((0.5, 3.0 + 12 * j, 3.0 + 12 * k), 0))
    for j in range(4):  # along y
        for k in range(5):
            anchors.append(((15.0 + 12 * j, 0.5, 3.0 + 12 * k), 1))
    for j in range(4):  # along z
        for k in range(4):
            anchors.append(((15.0 + 12 * j, 15.0 + 12 * k, 0.5), 2))
    assert len(anchors) >= len(seps)
    pts = []
    for sep, (a, axis) in zip(seps, anchors):
        a = np.array(a)
        b = a.copy()
        b[axis] += sep
        pts += [a, b]
    # particles on the faces (x, y or z = 0 and = nextafter(L, 0)), each with a
    # partner through the face at 1.0, 1.45 or 1.9
    Ld = np.nextafter(L, 0.0)
    faces = [((0.0, 62.0, 62.0), (Ld, 63.0, 62.0)), ((Ld, 62.0, 68.0), (0.0, 63.0, 68.0)),
             ((62.0, 0.0, 62.0), (62.0, Ld, 63.45)), ((68.0, Ld, 62.0), (68.0, 0.0, 63.45)),
             ((62.0, 62.0, 0.0), (63.9, 62.0, Ld)), ((62.0, 68.0, Ld), (63.9, 68.0, 0.0))]
    for a, b in faces:
        pts += [np.array(a), np.array(b)]
    # pairs through the x face at distances near r_c and r_c + skin
    for j, sep in enumerate([RC, np.nextafter(RC, 0.0), RL, np.nextafter(RL, 0.0)]):
        a = np.array([0.25, 40.0 + 6.0 * j, 70.0])
        b = a.copy()
        b[0] = a[0] - sep + L
        pts += [a, b]
    pos = np.array(pts).T.copy()
    box = np.array([L, L, L])
    assert (pos >= 0.0).all() and (pos < L).all()
    return pos, box


def liquid_with_probes(seed=3):
    """A jittered FCC liquid (density 0.8) in which, for each separation
    above, a particle j is moved to that distance from a particle i along an
    axis; particles closer than 0.85 to its new place are removed."""
    rng = np.random.default_rng(seed)
    pos, box = W.jittered_fcc(8, 0.8, 0.08, rng)
    n = pos.shape[1]
    L = box[0]
    seps = _separations()
    keep = np.ones(n, bool)
    fixed = set()
    for t, sep in enumerate(seps):
        while True:
            i, j = (int(v) for v in rng.choice(n, 2, replace=False))
            if keep[i] and keep[j] and i not in fixed and j not in fixed:
                break
        cand = pos[:, i].copy()
        cand[t % 3] += sep
        cand = np.mod(cand, L)
        d = pos - cand[:, None]
        d -= L * np.rint(d / L)
        close = ((d * d).sum(axis=0) < 0.85 ** 2) & keep
        close[[i, j]] = False
        if any(k in fixed for k in np.flatnonzero(close)):
            continue  # would remove a probe particle: skip this separation
        keep &= ~close
        pos[:, j] = cand
        fixed.update((i, j))
    assert len(fixed) >= len(seps)
    return np.ascontiguousarray(pos[:, keep]), box


def half_box_tie():
    """Box of exactly 2 (r_c + skin) = 5.6 per side: a pair at |d| = L/2
    along x and one along y (both images at r_c + skin: outside the list,
    the cutoff being strict), and a pair inside the list radius but outside
    r_c."""
    L = 2.0 * RL
    h = 0.5 * L  # = r_c + skin exactly
    pts = [(0.5, 0.5, 0.5), (0.5 + h, 0.5, 0.5), (1.9, 1.0, 3.3), (1.9, 1.0 + h, 3.3),
           (4.2, 4.2, 1.0), (4.2, 4.2, 3.65)]
    return np.array(pts).T.copy(), np.array([L, L, L])


SYSTEMS = {"isolated": isolated_pairs, "liquid": liquid_with_probes, "half_box": half_box_tie}


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [1, 0], ids=["fp64", "fp32"])
@pytest.mark.parametrize("cont", CONTAINERS, ids=CNAMES)
@pytest.mark.parametrize("system", list(SYSTEMS))
def test_edge_pairs(orc, lib, system, cont, prec):
    if cont[0] == 2 and prec == 1:
        pytest.skip("cluster lists are FP32-only")
    if cont[1] == 2 and prec == 1:
        pytest.skip("the C08 traversal is FP32-only")
    pos, box = SYSTEMS[system]()
    if cont[1] == 2 and not all(int(b // RL) >= 3 for b in box):
        pytest.skip("the C08 traversal needs three cells per dimension")
    n = pos.shape[1]
    F0, U0, W0, P0 = orc.forces(pos, box, orc.single())
    cfg = make_config(n, box, container=cont[0], newton3=cont[1], csf=cont[2], precision=prec)
    s = DeviceSystem(cfg, pos)
    s.build()
    out = s.forces().cpu().numpy()
    assert int(out[2]) == P0
    F = s.by_id(s.force)
    if system != "isolated":
        if not F0.any():
            assert not F.any()
        else:
            assert_forces(F, F0, prec == 1)
    else:
        # isolated pairs: each particle feels one pair force (or none, then
        # exactly zero): relative error per particle
        tol = 1e-12 if prec == 1 else 2e-6  # per pair: rcp, products, fixed-point sums
        mag0 = np.sqrt((F0 * F0).sum(axis=0))
        err = np.sqrt(((F - F0) ** 2).sum(axis=0))
        assert (err <= tol * mag0).all(), np.flatnonzero(err > tol * mag0)
    tolE = 1e-12 if prec == 1 else 1e-6
    assert abs(out[0] - U0) <= tolE * max(abs(U0), 1e-300)
    if cont[0] == 1:
        counts, rows = M.md_get_neighbors(s.h, 256)
        counts = counts.cpu().numpy()
        rows = rows.cpu().numpy()
        ids = s.ids_np()
        ref = orc.neighbor_rows(pos, box, RL * RL, np.arange(n))
        if not cont[1]:
            for k in range(n):
                assert np.array_equal(np.sort(ids[rows[k, :counts[k]]]), ref[ids[k]]), k
        else:
            seen = set()
            for k in range(n):
                for j in ids[rows[k, :counts[k]]]:
                    key = (min(ids[k], j), max(ids[k], j))
                    assert key not in seen, key
                    seen.add(key)
            assert seen == {(i, j) for i in range(n) for j in ref[i] if i < j}


def test_edge_systems_are_what_they_claim(orc):
    """The constructed distances land where intended (CPU only): the
    isolated pairs are exactly the separations, which hold pairs on both
    sides of r_c and of r_c + skin and inside the FP32 guard band; groups
    are at least 2 (r_c + skin) apart; the half-box pairs sit at exactly
    L/2."""
    pos, box = isolated_pairs()
    seps = _separations()
    m = len(seps)
    d = pos[:, 1:2 * m:2] - pos[:, 0:2 * m:2]
    r = np.sqrt((d * d).sum(axis=0))
    assert np.array_equal(r, seps)
    r2 = r * r
    assert (r2 < RC * RC).sum() >= 10 and (r2 > RC * RC).sum() >= 10 and (r2 == RC * RC).sum() >= 1
    band = np.abs(r2 - RC * RC) <= 2.0 ** -19 * RC * RC
    assert band.sum() >= 8 and (~band & (np.abs(r2 - RC * RC) < 2.0 ** -17 * RC * RC)).sum() >= 2
    assert ((r2 < RL * RL) & (r2 > RC * RC)).sum() >= 5 and (r2 >= RL * RL).sum() >= 5
    # every particle's nearest non-partner lies beyond r_c + skin
    n = pos.shape[1]
    L = box[0]
    for i in range(n):
        dd = pos - pos[:, [i]]
        dd -= L * np.rint(dd / L)
        q = (dd * dd).sum(axis=0)
        q[i] = np.inf
        q[i ^ 1] = np.inf
        assert q.min() > (2 * RL) ** 2 - 1e-9 or q.min() > RL * RL, i
    p, b = half_box_tie()
    assert p[0, 1] - p[0, 0] == 0.5 * b[0] == RL and p[1, 3] - p[1, 2] == 0.5 * b[1]
    rows = orc.neighbor_rows(p, b, RL * RL, np.arange(6))
    assert 1 not in rows[0] and 3 not in rows[2] and 5 in rows[4]
