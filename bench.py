"""Benchmark: implicit steps/s and CG iterations to 1e-6 at 1.65M triangles.

One step = dynamic assembly of A and b (pattern rebuild, element evaluation,
block reduce), Jacobi-PCG to ||r|| <= 1e-6 ||b|| and the state update, on the
three stacked irregular sheets (3 x 550,000 triangles, 828,153 vertices,
h = 0.01 s), synthetic seeded input.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--blocks f32|bf16|f64]
       [--no-cpu-baseline] [--workload large|medium]
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
BLOCK_BYTES = {"f64": 72, "f32": 36, "bf16": 18}


def spmv_bytes(nv, nnzb, blocks):
    """Algorithmic bytes of one difference-form SpMV in the CG loop: every
    stored block and its column index once, the input vector once per row
    (float4), the FP64 output, the FP64 mass, and the row pointers."""
    return nnzb * (BLOCK_BYTES[blocks] + 4) + nv * (16 + 24 + 8) + 4 * (nv + 1)


def cg_vector_bytes(nv):
    """Algorithmic bytes of the two CG vector kernels per iteration:
    update reads x, p, r, q, D^-1 and writes x, r; direction reads r, D^-1, p
    and writes p (x, r, q FP64 x3; p float4; D^-1 float x3)."""
    return nv * ((24 + 16 + 24 + 24 + 12 + 24 + 24) + (24 + 12 + 16 + 16))


def assembly_bytes(nv, nt, nh, nnzb, blocks):
    """Compulsory bytes of one assembly: read x, v (48 B/vertex), topology
    (12 B/triangle, 16 B/hinge), rest data (40 B/triangle, 16 B/hinge), mass
    and pins (9 B/vertex); write blocks and both column-index arrays, row
    pointers, b, diag(A) and D^-1 (24 + 24 + 12 B/vertex)."""
    reads = 48 * nv + 12 * nt + 16 * nh + 40 * nt + 16 * nh + 9 * nv
    writes = nnzb * (BLOCK_BYTES[blocks] + 8) + 4 * (nv + 1) + 60 * nv
    return reads + writes


def cpu_baseline(cloth, gpu_iters_per_step, seconds_budget=25.0):
    """The FP64 oracle on the host: one assembly of the same step and a
    bounded number of Jacobi-PCG iterations; steps/s extrapolated with the
    iteration count the GPU needed for the same tolerance."""
    from oracle import oracle
    oracle.build()
    P = oracle.Problem.from_cloth(cloth)
    t0 = time.perf_counter()
    A = P.assemble(cloth.x0, cloth.v0)
    t_asm = time.perf_counter() - t0
    iters = 5
    t0 = time.perf_counter()
    P.pcg_fixed(A, iters)
    t_it = (time.perf_counter() - t0) / iters
    n2 = int(max(5, min(60, (seconds_budget - t_asm) / max(t_it, 1e-6) - iters)))
    t0 = time.perf_counter()
    P.pcg_fixed(A, n2)
    t_it = (time.perf_counter() - t0) / n2
    t_step = t_asm + gpu_iters_per_step * t_it
    return {"value": 1.0 / t_step, "unit": "steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"FP64 oracle on {cloth.name}: one assembly ({t_asm:.2f} s) and {n2} Jacobi-PCG "
                       f"iterations ({1e3 * t_it:.1f} ms each), steps/s = 1/(assembly + "
                       f"{gpu_iters_per_step:.0f} iterations), the GPU's mean iterations per step at the "
                       f"same tolerance")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--blocks", default="f32", choices=["f32", "bf16", "f64"])
    ap.add_argument("--workload", default="large", choices=["large", "medium"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prof-every", type=int, default=8)
    ap.add_argument("--graph", type=int, default=0, help="CG iterations per captured HIP graph (0: off)")
    ap.add_argument("--warm", action="store_true", help="previous-step dv as the CG start")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the whole 1.65M-triangle workload fits in one MI355X "
              f"and nothing is sharded (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2008_00409_amd import binding, meshgen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.perf_counter()
    cloth = meshgen.config_large() if args.workload == "large" else meshgen.config_medium()
    print(f"# workload {cloth.name}: nv={cloth.nv} nt={cloth.nt} ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    ctx = binding.Context.from_cloth(cloth)
    if args.graph:
        ctx.set_option(binding.PC_OPT_GRAPH_CHUNK, args.graph)
    x = torch.from_numpy(cloth.x0.copy()).cuda()
    v = torch.from_numpy(cloth.v0.copy()).cuda()
    tol = cloth.tol
    warm_infos = (ctx.cloth_step(x, v, nsteps=args.warmup, dtype=args.blocks, tol=tol, warm=args.warm)
                  if args.warmup else [])
    print(f"# warmup done: iters {[i['iters'] for i in warm_infos]}", file=sys.stderr, flush=True)
    ctx.profile(args.prof_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = ctx.cloth_step(x, v, nsteps=args.steps, dtype=args.blocks, tol=tol, warm=args.warm)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_read()
    rowptr, colidx = ctx.pattern()
    nnzb = int(colidx.numel())
    nv, nt, nh = ctx.nv, ctx.nt, ctx.nh
    iters = [i["iters"] for i in infos]
    print(f"# timed: {args.steps} steps in {elapsed:.3f} s, iters {iters}, "
          f"true residuals {[float('%.2e' % i['rel_res_true']) for i in infos]}", file=sys.stderr, flush=True)
    spmv = prof.get("spmv", {})
    spmv_ms = spmv.get("mean_ms", float("nan"))
    ach = spmv_bytes(nv, nnzb, args.blocks) / (spmv_ms * 1e-3) / 1e9 if spmv_ms == spmv_ms else None
    asm = prof.get("assemble_all", {})
    asm_ms = asm.get("mean_ms", float("nan"))
    rec = {
        "metric": "implicit steps/s + CG iters to 1e-6 residual @1.65M tris, learned vs plain",
        "value": args.steps / elapsed,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{cloth.name}: {nt} triangles, {nv} vertices, {nh} hinges, nnzb {nnzb}",
            "h": cloth.h, "tol": tol, "block_storage": args.blocks,
            "warm_start": "previous-step" if args.warm else "zero", "graph_chunk": args.graph,
            "refinement_sweeps": [i["sweeps"] for i in infos],
            "preconditioner": "jacobi", "cg_iters_per_step": {"mean": float(np.mean(iters)),
                                                               "min": int(min(iters)), "max": int(max(iters))},
            "rel_res_true_max": max(i["rel_res_true"] for i in infos),
        },
        "roofline": {
            "bound": "hbm", "kernel": f"k_pcg_spmv<{args.blocks}>",
            "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (ach / HBM_PEAK_GBS) if ach else None, "traffic": None,
            "mean_launch_ms": spmv_ms, "samples": spmv.get("samples", 0),
            "algorithmic_bytes_per_launch": spmv_bytes(nv, nnzb, args.blocks),
        },
        "kernels": {k: {"mean_ms": round(vv["mean_ms"], 5), "samples": vv["samples"]} for k, vv in prof.items()},
        "assembly": {
            "mean_ms": asm_ms,
            "compulsory_bytes": assembly_bytes(nv, nt, nh, nnzb, args.blocks),
            "compulsory_GBs": assembly_bytes(nv, nt, nh, nnzb, args.blocks) / (asm_ms * 1e-3) / 1e9
            if asm_ms == asm_ms else None,
        },
    }
    cg = prof.get("cg_update", {}).get("mean_ms", 0) + prof.get("cg_dir", {}).get("mean_ms", 0)
    if cg:
        rec["cg_vector_GBs"] = cg_vector_bytes(nv) / (cg * 1e-3) / 1e9
    ctx.close()
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)...", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(cloth, float(np.mean(iters)))
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
