"""Cell neighbourhoods denser than an LDS window tile.

The FP32 linked-cell and Verlet-list kernels stage each block's window of
cells in LDS; a window holds at most 2880 particles (full windows, the
gather-only traversals) or 2048 (half windows, Newton's third law).  A system
far denser than a liquid overflows them.  The library must then switch to
its global (non-windowed) kernels and return the same results, never skip
particles: md_build_cells reads the packer's verdict, md_step redoes the
steps of a block whose rebuild overflowed.  Every kernel exits normally in
these tests; the overflow is a counted condition, not a fault."""
import numpy as np
import pytest

from tests.gpu_util import DeviceSystem, make_config, rel_l2

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


def _dense(m=15, a=0.58, jitter=0.05, seed=5):
    """m^3 particles on a jittered simple cubic lattice of spacing a
    (density a^-3 = 5.1, six times a liquid's) in a periodic cube."""
    rng = np.random.default_rng(seed)
    g = (np.arange(m) + 0.5) * a
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()])
    pos = pos + rng.uniform(-jitter, jitter, pos.shape)
    L = m * a
    box = np.array([L, L, L])
    return np.mod(pos, L), box


# (container, newton3): at this box (3 cells of side 2.9 per dimension) a
# full window is the whole box (3375 particles > 2880) and overflows; a half
# window holds 15 of the 27 cells (about 1875 <= 2048) and fits
CASES = [(0, 0, True), (0, 1, False), (1, 0, True), (1, 1, False)]


@pytest.mark.parametrize("case", CASES, ids=["lc", "lc-n3l", "vl", "vl-n3l"])
def test_dense_forces_fall_back(orc, case):
    import torch
    cont, n3, overflows = case
    pos, box = _dense()
    n = pos.shape[1]
    F0, U0, W0, P0 = orc.forces(pos, box, orc.single())
    cfg = make_config(n, box, container=cont, newton3=n3, precision=M.MD_FP32, max_neighbors=640)
    s = DeviceSystem(cfg, pos)
    s.build()
    out = s.forces()
    st = M.md_status(s.h)
    assert bool(st & M.MD_FLAG_WINDOW_FALLBACK) == overflows, st
    assert not st & M.MD_FLAG_LIST_OVERFLOW
    fam = M.md_get_counters(s.h)["force_family"]
    assert fam == (0 if overflows else 1)
    o = out.cpu().numpy()
    assert int(o[2]) == P0
    F = s.by_id(s.force)
    assert rel_l2(F, F0) <= 1e-5
    frms = np.sqrt((F0 * F0).sum() / n)
    assert np.sqrt(((F - F0) ** 2).sum(axis=0)).max() <= 1e-4 * frms
    assert abs(o[0] - U0) <= 1e-6 * abs(U0)
    if cont == 0 and n3 == 0:
        # the adjoint takes the same (global) path
        types = np.zeros(n, np.int32)
        theta = np.array([1.0, 1.0])
        target = F0 * 0.9
        L0, _, gx, gt = orc.force_matching(pos, box, types, theta, np.array([[6.25]]), target)
        g = torch.tensor((2.0 / (3 * n)) * (F0 - target)[:, s.ids_np()], dtype=torch.float32, device="cuda")
        gp = torch.zeros((3, n), dtype=torch.float64, device="cuda")
        gl = torch.zeros(2, dtype=torch.float64, device="cuda")
        M.md_forces_backward(s.h, s.pos, s.type, s.lj, g.contiguous(), gp, gl)
        torch.cuda.synchronize()
        assert rel_l2(s.by_id(gp), gx) <= 1e-4


def test_dense_step_redoes_block(orc):
    """md_step with Full Search from linked cells at CSF 0.5 (whose windows
    hold the dense system): the first trial switches to CSF 1, whose rebuild
    inside a block overflows the windows; the block is redone with the
    global kernels, so every step's pair count equals the oracle's and the
    trajectory follows it."""
    import torch
    pos, box = _dense()
    n = pos.shape[1]
    dt, nsteps = 1e-5, 24
    vel = np.zeros((3, n))
    p1, v1, _, log0 = orc.velocity_verlet(pos, vel, box, orc.single(), dt, nsteps)
    cfg = make_config(n, box, container=0, csf=0.5, precision=M.MD_FP32, R=4, max_neighbors=640)
    cfg.autotune = M.MD_TUNE_FULL
    cfg.tune_interval = 1000
    cfg.tune_trial_steps = 2
    cfg.total_steps_hint = nsteps
    s = DeviceSystem(cfg, pos, vel)
    s.build()
    assert not M.md_status(s.h) & M.MD_FLAG_WINDOW_FALLBACK  # CSF 0.5 windows hold it
    s.forces(energy=False)
    log = torch.zeros((nsteps, 4), dtype=torch.float64, device="cuda")
    M.md_step(s.h, s.pos, s.vel, s.force, s.type, s.ids, s.inv_mass, s.lj, dt, nsteps, 1, log)
    torch.cuda.synchronize()
    st = M.md_status(s.h)
    assert st & M.MD_FLAG_WINDOW_FALLBACK, st
    cnt = M.md_get_counters(s.h)
    assert cnt["tuning_phases"] == 1 and cnt["trials"] == 12, cnt
    log = log.cpu().numpy()
    assert np.array_equal(log[:, 3], log0[:, 3])
    assert np.abs(log[:, 0] - log0[:, 0]).max() <= 1e-6 * np.abs(log0[:, 0]).max()
    dx = s.by_id(s.pos) - p1
    dx -= box[:, None] * np.rint(dx / box[:, None])
    # FP32 forces: the position error grows about as the square of the steps
    # (1e-8 held for 18 steps; 24 steps let a phase trial all twelve FP32
    # structures)
    assert np.abs(dx).max() < 1e-8 * (nsteps / 18) ** 2
