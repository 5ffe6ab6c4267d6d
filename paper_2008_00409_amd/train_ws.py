"""Training of the learned CG warm start on trajectories the solver generates.

Episodes of the 512 x 512 workload (1 m sheet, top row pinned, eight seeded
Gaussian bumps, h = 1/200 s; seed 4000 + episode) are stepped with the
library's own solver.  At every step the system of Eq. 3 is assembled, the
network takes ``--adam`` Adam steps on the energy loss of that system (the
A-norm error of its start, whose gradient is the start's residual: no stored
solutions are needed), and the solver then advances the cloth from the
learned start.  Every step is a training sample of the network, every
episode a new trajectory; the network is evaluated elsewhere, on the 1.65M
triangle workload (bench.py).

    python -m paper_2008_00409_amd.train_ws --episodes 50 --steps 200 --out ws.npy
    python -m paper_2008_00409_amd.train_ws --init ws.npy --first-episode 50 ...   # continue

Writes the FP32 parameters (flat layout of pc_ws_set_params) to --out and a
JSON record of the run beside it (.json).  --budget-s stops after the
episode that crosses a wall-clock budget.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--episodes", type=int, default=10)
    ap.add_argument("--first-episode", type=int, default=0, help="episode e uses seed 4000 + e")
    ap.add_argument("--steps", type=int, default=200, help="solver steps per episode")
    ap.add_argument("--adam", type=int, default=3, help="Adam steps per solver step")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--n", type=int, default=512, help="vertices per side of the sheet")
    ap.add_argument("--init", default=None, help="parameters to start from (.npy); default: seeded init")
    ap.add_argument("--out", required=True)
    ap.add_argument("--budget-s", type=float, default=0.0)
    ap.add_argument("--blocks", default="bf16", choices=["f32", "bf16", "f16"])
    a = ap.parse_args(argv)

    import torch

    from . import binding, meshgen as mg

    if not torch.cuda.is_available():
        sys.exit("train_ws needs a GPU")
    prev = {}
    if a.init:
        params = np.load(a.init).astype(np.float32)
        jpath = os.path.splitext(a.init)[0] + ".json"
        if os.path.exists(jpath):
            with open(jpath) as fh:
                prev = json.load(fh)
    else:
        params = binding.Context.ws_init_params(0)
    t_start = time.perf_counter()
    episodes = []
    for ep in range(a.first_episode, a.first_episode + a.episodes):
        c = mg.config_grid(a.n, seed=4000 + ep, h=1.0 / 200, name=f"grid-{a.n}x{a.n}")
        ctx = binding.Context.from_cloth(c)
        ctx.ws_set_params(params)
        x = torch.from_numpy(c.x0.copy()).cuda()
        v = torch.zeros_like(x)
        dvp = torch.zeros_like(x)
        pin = torch.from_numpy(c.pinned.astype(bool)).cuda()
        x_pin = x[pin].clone()
        losses, iters = [], []
        failed = None
        t0 = time.perf_counter()
        for k in range(a.steps):
            b = ctx.cloth_assemble(x, v, a.blocks)
            for it in range(a.adam):
                L = ctx.ws_train_step(x, v, b, dvp, lr=a.lr, want_loss=(it == 0))
                if it == 0:
                    losses.append(L)
            dv, info = ctx.cloth_pcg_solve(b, dv=dvp.clone(), tol=c.tol, warm="learned", precond="block",
                                           raise_on_error=False)
            if info["status"] != binding.PC_OK:
                # the trajectory cannot go on from an unconverged step: end the episode here
                failed = {"step": k, "status": binding.STATUS_NAMES.get(info["status"], info["status"]),
                          "iters": info["iters"], "rel_res_true": info["rel_res_true"]}
                break
            iters.append(info["iters"])
            v += dv
            v[pin] = 0
            x += c.h * v
            x[pin] = x_pin
            dvp = dv
        params = ctx.ws_get_params()
        ctx.close()
        rec = {"episode": ep, "seed": 4000 + ep, "steps": len(iters), "seconds": time.perf_counter() - t0,
               "loss_first": losses[0], "loss_last": losses[-1], "loss_mean_last_20": float(np.mean(losses[-20:])),
               "cg_iters_mean": float(np.mean(iters)) if iters else None}
        if failed:
            rec["ended_early"] = failed
        episodes.append(rec)
        print(json.dumps(rec), flush=True)
        np.save(a.out, params)
        if a.budget_s and time.perf_counter() - t_start > a.budget_s:
            break
    steps_here = sum(e["steps"] for e in episodes)
    record = {
        "workload": f"grid-{a.n}x{a.n}, h = 1/200 s, top row pinned, seeded bumps (seed 4000 + episode)",
        "solver": f"{a.blocks} blocks, block Jacobi, learned start, tol 1e-6",
        "adam_per_step": a.adam, "lr": a.lr,
        "episodes_total": prev.get("episodes_total", 0) + len(episodes),
        "steps_total": prev.get("steps_total", 0) + steps_here,
        "adam_steps_total": prev.get("adam_steps_total", 0) + steps_here * a.adam,
        "runs": prev.get("runs", []) + [{"first_episode": a.first_episode, "episodes": len(episodes),
                                         "steps": steps_here, "seconds": time.perf_counter() - t_start,
                                         "per_episode": episodes}],
    }
    with open(os.path.splitext(a.out)[0] + ".json", "w") as fh:
        json.dump(record, fh, indent=1)
    print(f"# trained on {record['steps_total']} steps in {record['episodes_total']} episodes", flush=True)


if __name__ == "__main__":
    main()
