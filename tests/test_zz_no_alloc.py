"""The allocation-free entry point md_compute_forces_noalloc against the
handle-based md_compute_forces (linked cells, gather-only) and the FP64
oracle: two calls in a row on one GPU, the second with fewer particles, in
both precisions; inputs stay in the caller's order."""
import numpy as np
import pytest

from paper_2505_03438_amd import workloads as W
from tests.gpu_util import DeviceSystem, assert_forces, make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_03438_amd import mdlj
    mdlj.lib()
    return mdlj


def _system(ncell, seed):
    rng = np.random.default_rng(seed)
    pos, box = W.jittered_fcc(ncell, 0.8, 0.08, rng)
    perm = rng.permutation(pos.shape[1])  # caller's order unrelated to cells
    return np.ascontiguousarray(pos[:, perm]), box


def _noalloc(M, pos, box, prec, csf):
    import torch
    n = pos.shape[1]
    cfg = make_config(n, box, container=M.MD_CONTAINER_LC, csf=csf, precision=prec)
    real = torch.float64 if prec == M.MD_FP64 else torch.float32
    x = torch.tensor(pos, dtype=torch.float64, device="cuda")
    t = torch.zeros(n, dtype=torch.int32, device="cuda")
    lj = torch.tensor([1.0, 1.0], dtype=torch.float64, device="cuda")
    f = torch.full((3, n), float("nan"), dtype=real, device="cuda")
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    M.md_compute_forces_noalloc(cfg, x, t, lj, f, out)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), pos)  # inputs untouched
    return f.double().cpu().numpy(), out.cpu().numpy()


def _with_handle(M, pos, box, prec, csf):
    n = pos.shape[1]
    cfg = make_config(n, box, container=M.MD_CONTAINER_LC, csf=csf, precision=prec)
    s = DeviceSystem(cfg, pos)
    s.build()
    out = s.forces().cpu().numpy()
    return s.by_id(s.force), out


@pytest.mark.parametrize("csf", [1.0, 0.5])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
def test_noalloc_matches_handle_path(orc, M, prec, csf):
    fp64 = prec == M.MD_FP64
    tolE = 1e-12 if fp64 else 1e-6
    for ncell, seed in ((10, 21), (6, 22)):  # 4000 particles, then 864
        pos, box = _system(ncell, seed)
        F, out = _noalloc(M, pos, box, prec, csf)
        Fh, outh = _with_handle(M, pos, box, prec, csf)
        F0, U0, W0, P0 = orc.forces(pos, box, orc.single())
        assert int(out[2]) == int(outh[2]) == P0
        assert_forces(F, Fh, fp64, what="noalloc vs handle")
        assert_forces(F, F0, fp64, what="noalloc vs oracle")
        assert abs(out[0] - outh[0]) <= tolE * abs(outh[0])
        assert abs(out[0] - U0) <= tolE * abs(U0)
        assert abs(out[1] - W0) <= tolE * abs(W0)


def test_noalloc_limits(M):
    import torch
    assert M.md_noalloc_max_particles() == 131072
    n = M.md_noalloc_max_particles() + 1
    cfg = make_config(n, np.array([60.0, 60.0, 60.0]))
    x = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    t = torch.zeros(n, dtype=torch.int32, device="cuda")
    lj = torch.tensor([1.0, 1.0], dtype=torch.float64, device="cuda")
    f = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError, match="exceeds"):
        M.md_compute_forces_noalloc(cfg, x, t, lj, f)
    # a dilute system whose CSF-1/2 cells do not fit the scratch
    cfg = make_config(1000, np.array([400.0, 400.0, 400.0]), csf=0.5)
    x = torch.zeros((3, 1000), dtype=torch.float64, device="cuda")
    t = torch.zeros(1000, dtype=torch.int32, device="cuda")
    f = torch.zeros((3, 1000), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError, match="scratch"):
        M.md_compute_forces_noalloc(cfg, x, t, lj, f)
    # no particles: the sums are zero
    cfg = make_config(0, np.array([10.0, 10.0, 10.0]))
    out = torch.full((4,), 7.0, dtype=torch.float64, device="cuda")
    e = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    M.md_compute_forces_noalloc(cfg, torch.zeros((3, 0), dtype=torch.float64, device="cuda"),
                                torch.zeros(0, dtype=torch.int32, device="cuda"), lj, e, out)
    torch.cuda.synchronize()
    assert list(out.cpu().numpy()) == [0.0, 0.0, 0.0, 0.0]
