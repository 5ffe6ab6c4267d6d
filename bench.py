"""Benchmark: implicit steps/s and CG iterations to 1e-6 at 1.65M triangles.

One step = dynamic assembly of A and b (pattern rebuild, element evaluation,
block reduce), preconditioned CG to ||b - A dv|| <= 1e-6 ||b|| (true residual
with FP64 blocks) and the state update, on three stacked irregular sheets
(3 x 550,000 triangles, 828,153 vertices, h = 0.01 s), seeded synthetic input
resident in HBM.  Two configurations run on the same workload:

  plain   the paper's solver: FP32 blocks, FP64 vectors, Jacobi, zero start;
          timed again with the previous-step start, and the speedup is
          taken against the faster of the two
  value   the project configuration: FP16 blocks (a power-of-two scale per
          instance and assembly) with FP64 refinement sweeps,
          block-Jacobi, learned warm start (the network trained offline on
          the 512 x 512 solver's trajectories, paper_2008_00409_amd/
          ws_params_512.npy, or online first when that file is absent);
          timed again with the previous-step start, so that the learned
          start's own share of the speedup is a number of its own

After the timed runs an untimed replay of the same trajectory solves every
timed step's system from the zero, previous-step and learned starts to the
same tolerance and reports the iterations per step (paired evaluation).

Both use the autotuned launch schedule.  By default 20 steps are timed after
5 warm-up steps.  Prints one JSON line (stdout); progress goes to stderr.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--blocks f32|bf16|f16|f64]
       [--precond jacobi|block] [--warm zero|prev|learned] [--workload large|medium|batch]
       [--no-plain] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BLOCK_BYTES = {"f64": 72, "f32": 36, "bf16": 18, "f16": 18}
KERNEL_TB = {"f64": "double", "f32": "float", "bf16": "pc::bf16_t", "f16": "pc::f16_t"}
# committed counter summaries (profiles/) giving HBM bytes per launch
TRAFFIC_FILES = {"k_pcg_spmv<pc::bf16_t, true, float>": "k_pcg_spmv_bf16_stacked-3x501x551_traffic.md",
                 "k_pcg_spmv<pc::f16_t, true, float>": "k_pcg_spmv_f16_stacked-3x501x551_traffic.md",
                 "k_pcg_spmv<float, true, double>": "k_pcg_spmv_f32_stacked-3x501x551_traffic.md"}


def spmv_bytes(nv, nblk, blocks, col_bytes=4, q_bytes=24):
    """Algorithmic bytes of one difference-form SpMV in the CG loop: every
    block the solver layout stores (nblk: the pattern's blocks less the
    diagonal blocks it leaves out because they are zero) and its column index
    (16-bit offsets when the SpMV runs with them, else 32-bit columns), the
    input vector once per row (three packed FP32), the output (FP64, or FP32
    inside the BF16 and FP16 refinement sweeps), the FP64 mass, and the row
    pointers."""
    return nblk * (BLOCK_BYTES[blocks] + col_bytes) + nv * (12 + q_bytes + 8) + 4 * (nv + 1)


def solver_blocks(rowptr, colidx, pinned):
    """Blocks the solver layout stores: every block of the pattern except
    the diagonal of rows whose remainder D_i is zero, i.e. of pinned rows and
    of free rows without a pinned column."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx)
    pinned = np.asarray(pinned)
    nv = rowptr.size - 1
    rows = np.repeat(np.arange(nv), np.diff(rowptr))
    offd_pinned = (colidx != rows) & (pinned[colidx] != 0)
    has_pin = np.bincount(rows[offd_pinned], minlength=nv) > 0
    keep = has_pin & (pinned == 0)
    return int(colidx.size - (nv - int(keep.sum())))


def assembly_bytes(nv, nt, nh, nnzb, blocks):
    """Compulsory bytes of one assembly: read x, v (48 B/vertex), topology
    (12 B/triangle, 16 B/hinge), rest data (40 B/triangle, 16 B/hinge), mass
    and pins (9 B/vertex); write blocks and both column-index arrays, row
    pointers, b, diag(A) and D^-1 (24 + 24 + 12 B/vertex)."""
    reads = 48 * nv + 12 * nt + 16 * nh + 40 * nt + 16 * nh + 9 * nv
    writes = nnzb * (BLOCK_BYTES[blocks] + 8) + 4 * (nv + 1) + 60 * nv
    return reads + writes


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(cloth, iters_per_step, iters_source, seconds_budget=25.0, contacts=None):
    """The FP64 oracle on the host: one assembly of the same step and as many
    Jacobi-PCG iterations as fit the time budget (at most 2,000); steps/s
    extrapolated with `iters_per_step`, the Jacobi iteration count per step
    at the same tolerance (its source is recorded in the sample text)."""
    from oracle import oracle
    oracle.build()
    P = oracle.Problem.from_cloth(cloth)
    if contacts is not None:
        P.set_contacts(oracle.Contacts(contacts.verts, contacts.weights, contacts.normals, contacts.eta,
                                       contacts.kc))
    t0 = time.perf_counter()
    A = P.assemble(cloth.x0, cloth.v0)
    t_asm = time.perf_counter() - t0
    iters = 5
    t0 = time.perf_counter()
    P.pcg_fixed(A, iters)
    t_it = (time.perf_counter() - t0) / iters
    n2 = int(max(5, min(2000, (seconds_budget - t_asm) / max(t_it, 1e-6) - iters)))
    t0 = time.perf_counter()
    P.pcg_fixed(A, n2)
    t_it = (time.perf_counter() - t0) / n2
    t_step = t_asm + iters_per_step * t_it
    cores = oracle.num_threads()
    rec = {"value": 1.0 / t_step, "unit": "steps/s", "cores": cores, "kind": "oracle", "cpu_model": host_cpu_model(),
           "iters_per_step": iters_per_step, "iters_source": iters_source,
           "sample": (f"FP64 oracle on {cloth.name}: one assembly ({t_asm:.2f} s) and {n2} Jacobi-PCG "
                      f"iterations ({1e3 * t_it:.1f} ms each) on {cores} threads, steps/s = 1/(assembly + "
                      f"{iters_per_step:.0f} iterations); iterations per step: {iters_source}")}
    # the same on one host thread (one assembly and 10 iterations)
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        A1 = P.assemble(cloth.x0, cloth.v0)
        t_asm1 = time.perf_counter() - t0
        n1 = 10
        t0 = time.perf_counter()
        P.pcg_fixed(A1, n1)
        t_it1 = (time.perf_counter() - t0) / n1
    finally:
        oracle.set_threads(cores)
    rec["single_thread"] = {
        "value": 1.0 / (t_asm1 + iters_per_step * t_it1), "unit": "steps/s", "cores": 1,
        "sample": (f"one assembly ({t_asm1:.2f} s) and {n1} iterations ({1e3 * t_it1:.1f} ms each) on one "
                   f"thread, extrapolated with the same {iters_per_step:.0f} iterations per step")}
    return rec


def time_steps(ctx, x, v, steps, warmup, blocks, tol, warm, prof_every, precond="jacobi", inner_rho=0.0,
               method="cg"):
    """Run warmup then timed steps; returns (elapsed s, infos, profile)."""
    import torch
    kw = dict(dtype=blocks, tol=tol, warm=warm, precond=precond, inner_rho=inner_rho, method=method)
    if warmup:
        ctx.cloth_step(x, v, nsteps=warmup, **kw)
    ctx.profile(prof_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = ctx.cloth_step(x, v, nsteps=steps, **kw)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(0)
    return elapsed, infos, prof


def train_warm_start(binding, meshgen, steps, adam_per_step, lr, log):
    """Online training of the warm-start network on the 512 x 512 workload's
    own trajectory: at every step the current system is assembled, the
    network takes `adam_per_step` Adam steps on its energy loss, and the
    solver advances with the learned start."""
    import torch

    c = meshgen.config_medium()
    ctx = binding.Context.from_cloth(c)
    ctx.ws_set_params(binding.Context.ws_init_params(0))
    x = torch.from_numpy(c.x0.copy()).cuda()
    v = torch.zeros_like(x)
    dvp = torch.zeros_like(x)
    pin = torch.from_numpy(c.pinned.astype(bool)).cuda()
    x_pin = x[pin].clone()
    losses = []
    t0 = time.perf_counter()
    for k in range(steps):
        b = ctx.cloth_assemble(x, v, "f32")
        for it in range(adam_per_step):
            L = ctx.ws_train_step(x, v, b, dvp, lr=lr, want_loss=(it == adam_per_step - 1))
        losses.append(L)
        dv, info = ctx.cloth_pcg_solve(b, dv=dvp.clone(), tol=c.tol, warm="learned")
        v += dv
        v[pin] = 0
        x += c.h * v
        x[pin] = x_pin
        dvp = dv
        if k % 10 == 0:
            log(f"# train step {k}: loss {L:.4f}, iters {info['iters']}, start {info['warm_used']}")
    params = ctx.ws_get_params()
    ctx.close()
    return params, {"steps": steps, "adam_per_step": adam_per_step, "lr": lr,
                    "loss_first": losses[0], "loss_last": losses[-1], "seconds": time.perf_counter() - t0,
                    "workload": c.name}


def read_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when there is none or the SpMV sources changed since it was
    taken (the summary records a hash of them)."""
    import re

    from paper_2008_00409_amd.profile_summary import spmv_source_hash
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES.get(kernel, "-"))
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_b = re.search(r"^traffic_bytes_per_launch: (\d+)", txt, re.M)
    m_k = re.search(r"^kernel: (.+)$", txt, re.M)
    m_h = re.search(r"^spmv_source_hash: (\w+)", txt, re.M)
    if not (m_b and m_k and m_h) or m_k.group(1).strip() != kernel or m_h.group(1) != spmv_source_hash():
        return None
    return int(m_b.group(1))


def make_cloth(meshgen, workload):
    """(cloth, proximity pairs or None)."""
    if workload == "large":
        return meshgen.config_large(), None
    if workload == "medium":
        return meshgen.config_medium(), None
    if workload == "contact":
        return meshgen.config_contact()
    return meshgen.config_batch(), None


def new_context(binding, cloth, contacts=None):
    ctx = binding.Context.from_cloth(cloth)
    if len(cloth.sheet_ranges) > 1 and cloth.name.startswith("batch"):
        # independent cloths: per-instance CG scalars, convergence and sweeps
        ctx.set_instances([r[0] for r in cloth.sheet_ranges] + [cloth.nv])
    if contacts is not None:
        ctx.cloth_set_contacts(contacts.verts, contacts.weights, contacts.normals, contacts.eta, contacts.kc)
    return ctx


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 20 timed steps after 5 warm-up steps: the CG counts fall as the sheets'
    # motion settles, so very short runs see only the first, hardest steps
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--blocks", default=None, choices=["f32", "bf16", "f16", "f64"],
                    help="block storage of the project configuration (default: f16)")
    ap.add_argument("--warm", default="learned", choices=["zero", "prev", "learned"],
                    help="CG start of the project configuration")
    ap.add_argument("--precond", default="block", choices=["jacobi", "block"],
                    help="preconditioner of the project configuration")
    ap.add_argument("--inner-rho", type=float, default=0.0,
                    help="residual reduction per refinement sweep (0: library default)")
    ap.add_argument("--workload", default="large", choices=["large", "medium", "batch", "contact"],
                    help="large: 3 stacked sheets, 1.65M triangles (the headline); batch: 64 uneven "
                         "independent sheets, ~1.5M triangles in one launch; contact: 2 sheets 1.5 mm "
                         "apart with 274K vertex-face proximity pairs in the assembly")
    ap.add_argument("--method", default="cg", choices=["cg", "chronopoulos-gear"],
                    help="CG form of the project configuration: textbook recurrences or single reduction")
    ap.add_argument("--keep-direction", type=int, default=None, choices=[0, 1],
                    help="PC_OPT_KEEP_DIRECTION for the value configuration (default: the library's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 / Jacobi / zero-start run")
    ap.add_argument("--no-value-prev", action="store_true",
                    help="skip the timed run of the project configuration with the previous-step start")
    ap.add_argument("--no-paired", action="store_true",
                    help="skip the untimed replay that solves every timed step's system from each start")
    ap.add_argument("--prof-every", type=int, default=8)
    ap.add_argument("--train-steps", type=int, default=30,
                    help="online training steps when no trained parameters are given")
    ap.add_argument("--ws-params", default=os.path.join(ROOT, "paper_2008_00409_amd", "ws_params_512.npy"),
                    help="trained warm-start parameters (train_ws.py); '' trains online instead")
    ap.add_argument("--autotune", type=int, default=1)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the whole 1.65M-triangle workload fits in one MI355X "
              f"and nothing is sharded (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    if args.blocks is None:
        args.blocks = "f16"

    import torch

    from paper_2008_00409_amd import binding, meshgen

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.perf_counter()
    cloth, contacts = make_cloth(meshgen, args.workload)
    log(f"# workload {cloth.name}: nv={cloth.nv} nt={cloth.nt}"
        f"{'' if contacts is None else f' contacts={contacts.n}'} ({time.perf_counter() - t0:.1f} s)")
    tol = cloth.tol
    rec_plain = None
    if not args.no_plain:
        ctx = new_context(binding, cloth, contacts)
        x = torch.from_numpy(cloth.x0.copy()).cuda()
        v = torch.from_numpy(cloth.v0.copy()).cuda()
        tune_plain = None
        if args.autotune:   # the same launch-schedule search as the project configuration
            tune_plain = ctx.autotune(ctx.cloth_assemble(x, v, "f32"), iters=64, precond="jacobi")
            log(f"# autotune (plain): {tune_plain}")
        el, infos, prof = time_steps(ctx, x, v, args.steps, args.warmup, "f32", tol, "zero", args.prof_every)
        rowptr, colidx = ctx.pattern()
        nnzb = int(colidx.numel())
        nblk = solver_blocks(rowptr.cpu().numpy(), colidx.cpu().numpy(), cloth.pinned)
        sp = prof.get("spmv", {}).get("median_ms", float("nan"))
        cb = 2 if ctx.get_option(binding.PC_OPT_SPMV_NARROW_ACTIVE) else 4
        rec_plain = {"steps_per_s": args.steps / el, "block_storage": "f32", "warm_start": "zero",
                     "preconditioner": "jacobi", "schedule": tune_plain,
                     "cg_iters_per_step": [i["iters"] for i in infos],
                     "rel_res_true_max": max(i["rel_res_true"] for i in infos),
                     "spmv_median_ms": sp, "spmv_GBs": spmv_bytes(ctx.nv, nblk, "f32", cb) / (sp * 1e-3) / 1e9}
        log(f"# plain: {rec_plain['steps_per_s']:.3f} steps/s, iters {rec_plain['cg_iters_per_step']}")
        # the same solver with the previous-step start, from the same initial
        # state on the same schedule; the speedup is taken against the faster
        x.copy_(torch.from_numpy(cloth.x0))
        v.copy_(torch.from_numpy(cloth.v0))
        el_p, infos_p, _ = time_steps(ctx, x, v, args.steps, args.warmup, "f32", tol, "prev", 0)
        rec_plain["prev_start"] = {"steps_per_s": args.steps / el_p, "cg_iters_per_step": [i["iters"] for i in infos_p],
                                   "rel_res_true_max": max(i["rel_res_true"] for i in infos_p)}
        log(f"# plain, previous-step start: {rec_plain['prev_start']['steps_per_s']:.3f} steps/s, "
            f"iters {rec_plain['prev_start']['cg_iters_per_step']}")
        ctx.close()
        del x, v
    train_info = None
    params = None
    if args.warm == "learned":
        if args.ws_params and os.path.exists(args.ws_params):
            # the network trained offline on the 512 x 512 solver's trajectories
            params = np.load(args.ws_params).astype(np.float32)
            train_info = {"source": os.path.relpath(args.ws_params, ROOT)}
            meta = os.path.splitext(args.ws_params)[0] + ".json"
            if os.path.exists(meta):
                with open(meta) as fh:
                    m = json.load(fh)
                train_info.update({k: m[k] for k in ("workload", "solver", "episodes_total", "steps_total",
                                                     "adam_steps_total", "adam_per_step", "lr") if k in m})
            log(f"# warm-start network: {train_info}")
        else:
            params, train_info = train_warm_start(binding, meshgen, args.train_steps, 3, 1e-3, log)
    ctx = new_context(binding, cloth, contacts)
    if params is not None:
        ctx.ws_set_params(params)
    if args.keep_direction is not None:
        ctx.set_option(binding.PC_OPT_KEEP_DIRECTION, args.keep_direction)
    x = torch.from_numpy(cloth.x0.copy()).cuda()
    v = torch.from_numpy(cloth.v0.copy()).cuda()
    tune = None
    if args.autotune:
        b = ctx.cloth_assemble(x, v, args.blocks)
        tune = ctx.autotune(b, iters=64, precond=args.precond)
        log(f"# autotune: {tune}")
    el, infos, prof = time_steps(ctx, x, v, args.steps, args.warmup, args.blocks, tol, args.warm, args.prof_every,
                                 args.precond, args.inner_rho, args.method)
    rowptr, colidx = ctx.pattern()
    nnzb = int(colidx.numel())
    nblk = solver_blocks(rowptr.cpu().numpy(), colidx.cpu().numpy(), cloth.pinned)
    nv, nt, nh = ctx.nv, ctx.nt, ctx.nh
    iters = [i["iters"] for i in infos]
    log(f"# timed: {args.steps} steps in {el:.3f} s, iters {iters}, sweeps {[i['sweeps'] for i in infos]}, "
        f"starts {[i['warm_used'] for i in infos]}, true residuals {[float('%.2e' % i['rel_res_true']) for i in infos]}")
    per_instance = None
    if getattr(ctx, "ninst", 1) > 1:
        ii = [d["iters"] for d in ctx.instance_info()]
        per_instance = {"instances": len(ii), "iters_min": min(ii), "iters_median": float(np.median(ii)),
                        "iters_max": max(ii)}
    # the learned start's own share: the same configuration, schedule and
    # initial state with the previous-step start instead, timed alike
    rec_value_prev = None
    if args.warm == "learned" and not args.no_value_prev:
        x.copy_(torch.from_numpy(cloth.x0))
        v.copy_(torch.from_numpy(cloth.v0))
        el_vp, infos_vp, _ = time_steps(ctx, x, v, args.steps, args.warmup, args.blocks, tol, "prev", 0,
                                        args.precond, args.inner_rho, args.method)
        rec_value_prev = {"steps_per_s": args.steps / el_vp, "warm_start": "prev",
                          "cg_iters_per_step": [i["iters"] for i in infos_vp],
                          "refinement_sweeps": [i["sweeps"] for i in infos_vp],
                          "rel_res_true_max": max(i["rel_res_true"] for i in infos_vp)}
        log(f"# value configuration, previous-step start: {rec_value_prev['steps_per_s']:.3f} steps/s, "
            f"iters {rec_value_prev['cg_iters_per_step']}")
    # paired evaluation (untimed replay): the trajectory of the timed run is
    # replayed from the same initial state, and at every timed step the same
    # system (A, b) is solved from each start to the same tolerance; the
    # trajectory advances with the configured start's solution
    paired = None
    if not args.no_paired:
        modes = ["zero", "prev"] + (["learned"] if params is not None else [])
        x.copy_(torch.from_numpy(cloth.x0))
        v.copy_(torch.from_numpy(cloth.v0))
        kw = dict(tol=tol, precond=args.precond, inner_rho=args.inner_rho, method=args.method)
        dv_prev = torch.zeros_like(x)
        if args.warmup:
            if args.warmup > 1:
                ctx.cloth_step(x, v, nsteps=args.warmup - 1, dtype=args.blocks, warm=args.warm, **kw)
            v_before = v.clone()
            ctx.cloth_step(x, v, nsteps=1, dtype=args.blocks, warm=args.warm, **kw)
            dv_prev = v - v_before
        pin = torch.from_numpy(cloth.pinned.astype(bool)).cuda()
        paired = {m: {"iters": [], "sweeps": [], "start_used": [], "a_err2": []} for m in modes}
        paired["missed"] = 0     # solves that ended above the tolerance (none expected)

        def energy(s, b):
            # 1/2 s.A s - b.s through the FP64 blocks
            return 0.5 * float((s * ctx.cloth_spmv(s, solver_blocks=False)).sum()) - float((b * s).sum())
        t_rep = time.perf_counter()
        for k in range(args.steps):
            b = ctx.cloth_assemble(x, v, args.blocks)
            keep = None
            for mode in modes:
                dv0 = torch.zeros_like(x) if mode == "zero" else dv_prev.clone()
                dv, pinfo = ctx.cloth_pcg_solve(b, dv=dv0, warm=mode, raise_on_error=False, **kw)
                if pinfo["status"] != 0 or not pinfo["rel_res_true"] <= tol:
                    paired["missed"] = paired.get("missed", 0) + 1
                paired[mode]["iters"].append(pinfo["iters"])
                paired[mode]["sweeps"].append(pinfo["sweeps"])
                paired[mode]["start_used"].append(pinfo["warm_used"])
                if mode == args.warm:
                    keep = dv
            # squared A-norm error of each start relative to the solution's:
            # (E(s) - E(dv*)) / -E(dv*), 1 for the zero start
            e_star = energy(keep, b)
            for mode in modes:
                s0 = (torch.zeros_like(x) if mode == "zero" else
                      dv_prev if mode == "prev" else ctx.ws_start(x, v, b, dv_prev)[0])
                paired[mode]["a_err2"].append((energy(s0, b) - e_star) / -e_star if e_star < 0 else None)
            v.add_(keep)
            v[pin] = 0.0
            x.add_(cloth.h * v)
            dv_prev = keep
        for m in modes:
            it = paired[m]["iters"]
            paired[m].update({"mean": float(np.mean(it)), "median": float(np.median(it)), "total": int(sum(it))})
            ae = [e for e in paired[m]["a_err2"] if e is not None]
            paired[m]["a_err2_mean"] = float(np.mean(ae)) if ae else None
        if "learned" in paired:
            paired["learned_over_prev_iters"] = paired["learned"]["total"] / paired["prev"]["total"]
            paired["learned_over_zero_iters"] = paired["learned"]["total"] / paired["zero"]["total"]
            paired["steps_learned_fewer_than_prev"] = int(sum(
                1 for a, b_ in zip(paired["learned"]["iters"], paired["prev"]["iters"]) if a < b_))
        paired["seconds"] = time.perf_counter() - t_rep
        log(f"# paired starts per step: " + ", ".join(f"{m} mean {paired[m]['mean']:.0f}" for m in modes))
        log(f"# paired starts, squared A-norm error / solution's: "
            + ", ".join(f"{m} {paired[m]['a_err2_mean']:.3g}" for m in modes if paired[m]["a_err2_mean"] is not None))
    spmv = prof.get("spmv", {})
    spmv_ms = spmv.get("median_ms", float("nan"))
    narrow = bool(ctx.get_option(binding.PC_OPT_SPMV_NARROW_ACTIVE))
    inner32 = (args.blocks in ("bf16", "f16") and args.method == "cg"
               and bool(ctx.get_option(binding.PC_OPT_INNER_FP32)))
    kname = f"k_pcg_spmv<{KERNEL_TB[args.blocks]}, {'true' if narrow else 'false'}, {'float' if inner32 else 'double'}>"
    alg = spmv_bytes(nv, nblk, args.blocks, 2 if narrow else 4, 12 if inner32 else 24)
    ach = alg / (spmv_ms * 1e-3) / 1e9 if spmv_ms == spmv_ms and spmv_ms > 0 else None
    asm = prof.get("assemble_all", {})
    asm_ms = asm.get("median_ms", float("nan"))
    rec = {
        "metric": "implicit steps/s + CG iters to 1e-6 residual @1.65M tris, learned vs plain",
        "value": args.steps / el,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # arithmetic of the CG inner loop: FP32 row sums and inner vectors with
        # BF16 or FP16 blocks (textbook form), FP64 otherwise; dots, the refinement
        # residual and the state are FP64 in every case
        "dtype": "f32" if inner32 else "f64",
        "precision": (f"{args.blocks} blocks; " + ("FP32 SpMV row sums and inner vectors; " if inner32 else
                                                   "FP64 SpMV row sums and vectors; ")
                      + "FP64 dots, refinement residual and state"),
        "data": "synthetic",
        "config": {
            "workload": f"{cloth.name}: {nt} triangles, {nv} vertices, {nh} hinges, nnzb {nnzb}"
                        + ("" if contacts is None else f", {contacts.n} proximity pairs"),
            "h": cloth.h, "tol": tol, "block_storage": args.blocks, "warm_start": args.warm,
            "refinement_sweeps": [i["sweeps"] for i in infos], "starts_used": [i["warm_used"] for i in infos],
            "fallback_steps": sum(1 for i in infos if i["fallback"]),   # steps that fell back to FP64 blocks
            "preconditioner": args.precond, "inner_rho": args.inner_rho, "cg_form": args.method,
            "cg_iters_per_step": {"mean": float(np.mean(iters)), "median": float(np.median(iters)),
                                  "min": int(min(iters)), "max": int(max(iters))},
            "rel_res_true_max": max(i["rel_res_true"] for i in infos),
            "schedule": tune,
            "per_instance": per_instance,
        },
        "plain": rec_plain,
        "value_prev_start": rec_value_prev,
        # value with the learned start over the same configuration with the
        # previous-step start: the learned network's own share of the speedup
        "learned_share": ((args.steps / el) / rec_value_prev["steps_per_s"]) if rec_value_prev else None,
        "paired_per_step": paired,
        # against the faster of the plain solver's zero and previous-step starts
        "speedup_vs_plain": ((args.steps / el) / max(rec_plain["steps_per_s"], rec_plain["prev_start"]["steps_per_s"])
                             if rec_plain else None),
        "training": train_info,
        "roofline": {
            "bound": "hbm", "kernel": kname,
            "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (ach / HBM_PEAK_GBS) if ach else None, "traffic": read_traffic(kname),
            "median_launch_ms": spmv_ms, "samples": spmv.get("samples", 0),
            "algorithmic_bytes_per_launch": alg, "solver_blocks": nblk, "pattern_blocks": nnzb,
        },
        "kernels": {k: {"median_ms": round(vv["median_ms"], 5), "mean_ms": round(vv["mean_ms"], 5),
                        "samples": vv["samples"]} for k, vv in prof.items()},
        "assembly": {
            "median_ms": asm_ms,
            "compulsory_bytes": assembly_bytes(nv, nt, nh, nnzb, args.blocks),
            "compulsory_GBs": assembly_bytes(nv, nt, nh, nnzb, args.blocks) / (asm_ms * 1e-3) / 1e9
            if asm_ms == asm_ms and asm_ms > 0 else None,
        },
    }
    ctx.close()
    if not args.no_cpu_baseline:
        log("# cpu baseline (oracle)...")
        if rec_plain is not None:
            it_cpu = float(np.mean(rec_plain["cg_iters_per_step"]))
            src = ("mean of the plain run (FP32 blocks, Jacobi, zero start, the oracle's preconditioner and "
                   "start) over the timed steps at the same tolerance")
        else:
            it_cpu = float(np.mean(iters))
            src = "mean of the timed configuration (no plain run in this invocation)"
        rec["cpu_baseline"] = cpu_baseline(cloth, it_cpu, src, contacts=contacts)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
