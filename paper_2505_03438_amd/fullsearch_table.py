"""Full Search trial scores over a range of scenarios: the data from which
Expert rules are written.  Sec. 5.2 designs the rules by running the example
simulations with plain full searches and relating the live statistics to the
configurations found optimal; this tool does that on the GPU at hand.

For every scenario it prints one JSON line: the live statistics of the start
positions (Sec. 4, md_live_stats order) and every configuration's score from
the second of two Full Search phases (ms per step, build time spread over the
rebuild interval; the first phase is a warm-up).

    python -m paper_2505_03438_amd.fullsearch_table [--quick] [--set selection]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from . import mdlj as M
from . import workloads as W

CONTAINER = {M.MD_CONTAINER_LC: "lc", M.MD_CONTAINER_VL: "vl", M.MD_CONTAINER_CL: "cl"}


def scenarios(quick: bool):
    """(name, workload dict) pairs: homogeneous fluids over density and size,
    and the inhomogeneous droplet and slab."""
    dens = (0.1, 0.8) if quick else (0.05, 0.1, 0.2, 0.3, 0.5, 0.7, 0.8, 0.9, 1.0)
    sizes = (32,) if quick else (20, 32, 64)
    for ncell in sizes:
        for rho in dens:
            rng = np.random.default_rng(W.seed_for(1) + 7919 * ncell + int(1000 * rho))
            pos, box = W.jittered_fcc(ncell, rho, 0.06, rng)
            vel = W.maxwell_boltzmann(pos.shape[1], 1.0, rng)
            yield "fluid-%d-rho%.2f" % (pos.shape[1], rho), dict(pos=pos, vel=vel, box=box)
    if not quick:
        for n in (250_000, 2_000_000):
            yield "droplet-%d" % n, W.droplet(n=n)
        yield "slab-2000000", W.slab()


def full_search(d, trial_steps: int = 10, dt: float = 0.005):
    n = d["pos"].shape[1]
    box = d["box"]
    c = M.config_default(n, float(box[0]))
    for k in range(3):
        c.box[k] = float(box[k])
    c.precision = M.MD_FP32
    c.skin = float(d.get("skin", 0.3))
    c.autotune = M.MD_TUNE_FULL
    c.tune_trial_steps = trial_steps
    h = M.md_create(c)
    nspace = len(M.md_get_trial_scores(h)[0])
    phase = nspace * trial_steps + 10
    c.tune_interval = phase
    c.total_steps_hint = 2 * phase
    h.close()
    h = M.md_create(c)
    dev = "cuda"
    pos = torch.tensor(d["pos"], dtype=torch.float64, device=dev)
    vel = torch.tensor(d["vel"], dtype=torch.float32, device=dev)
    force = torch.zeros((3, n), dtype=torch.float32, device=dev)
    typ = torch.zeros(n, dtype=torch.int32, device=dev)
    ids = torch.arange(n, dtype=torch.int32, device=dev)
    lj = torch.tensor([1.0, 1.0], dtype=torch.float64, device=dev)
    im = torch.ones(1, dtype=torch.float64, device=dev)
    stats = M.md_live_stats(h, pos)
    M.md_build_cells(h, pos, vel, force, typ, ids)
    M.md_build_neighbors(h, pos, typ)
    M.md_compute_forces(h, pos, typ, lj, force)
    M.md_step(h, pos, vel, force, typ, ids, im, lj, dt, 2 * phase)
    torch.cuda.synchronize()
    scores, cfgs = M.md_get_trial_scores(h)
    chosen = M.md_get_counters(h)["config_index"]
    h.close()
    names = ["%s-csf%g-%s%s" % (CONTAINER[int(k.container)], float(k.csf), "n3l" if k.newton3 else "gather",
                                "" if k.skin == cfgs[0].skin else "-skin%.3g" % k.skin)
             for k in cfgs]
    return stats, dict(zip(names, scores)), names[chosen], chosen


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="two densities at 32,000 particles only")
    ap.add_argument("--set", default="expert", choices=["expert", "selection"],
                    help="expert: fluids, droplet and slab (the Expert rules' data); selection: the generative "
                         "scenarios the Random Forest is trained on")
    args = ap.parse_args()
    M.lib()
    if not torch.cuda.is_available():
        sys.exit("no GPU")
    gen = W.selection_scenarios() if args.set == "selection" else scenarios(args.quick)
    for name, d in gen:
        stats, scores, chosen, index = full_search(d)
        print(json.dumps({"scenario": name, "n": int(d["pos"].shape[1]),
                          "stats": dict(zip(("mean", "rel_std", "median", "max", "n_bins", "n_empty", "cus",
                                             "skin"), stats)),
                          "features": stats, "scores_ms": scores, "chosen": chosen, "label": index}), flush=True)


if __name__ == "__main__":
    main()
