"""A/B timing of the paper's matrix filling and BELL SpMV against the
solver's own assembly and sliced-ELL SpMV, on one workload through the C ABI.

Assembly: median wall time of one call (stream synchronised on both sides)
of cloth_assemble (FP32 and BF16 solver blocks; its pattern is rebuilt every
call) and of cloth_assemble_bell (FP32 and FP64 tables; its five steps,
including the two host read-backs that size the tables).
SpMV: the CG's own SpMV (median of event-timed launches inside a capped
solve) against cloth_spmv_bell (HIP events around a run of calls; each call
also rounds x to FP32 in a small kernel, whose time a kernel trace separates).
Algorithmic bytes per SpMV for both: the stored blocks of the block pattern
(nnzb x (9 values + 1 column index)) plus one read of x (16 B per row) and one
write of y (24 B per row); the BELL's padded slots are extra traffic.

    python -m paper_2008_00409_amd.bell_bench --workload large --reps 10
"""
from __future__ import annotations

import argparse
import json
import statistics
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="large", choices=["large", "medium", "contact"])
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--spmv-reps", type=int, default=50)
    ap.add_argument("--cg-iters", type=int, default=200)
    a = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import binding, meshgen as mg

    if not torch.cuda.is_available():
        sys.exit("bell_bench needs a GPU")
    contacts = None
    if a.workload == "contact":
        c, cs = mg.config_contact()
        contacts = (cs.verts, cs.weights, cs.normals, cs.eta, cs.kc)
    else:
        c = {"large": mg.config_large, "medium": mg.config_medium}[a.workload]()
    ctx = binding.Context.from_cloth(c)
    if contacts is not None:
        ctx.cloth_set_contacts(*contacts)
    x = torch.from_numpy(c.x0.copy()).cuda()
    v = 0.05 * torch.from_numpy(np.random.default_rng(5).normal(size=c.x0.shape)).cuda()
    v[torch.from_numpy(c.pinned.astype(bool)).cuda()] = 0.0
    print(f"# bell_bench {c.name}: nv={c.nv} nt={c.nt}", flush=True)

    def wall(fn):
        ts = []
        for _ in range(a.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return statistics.median(ts)

    out = {"workload": c.name, "nv": c.nv, "nt": c.nt}
    for dt in ["f32", "bf16"]:
        ctx.cloth_assemble(x, v, dt)
        out[f"assemble_ms_{dt}"] = wall(lambda: ctx.cloth_assemble(x, v, dt))
        print(f"# solver assembly {dt}: {out[f'assemble_ms_{dt}']:.2f} ms", flush=True)
    for dt in ["f32", "f64"]:
        _b, width = ctx.cloth_assemble_bell(x, v, dt)
        out[f"bell_assemble_ms_{dt}"] = wall(lambda: ctx.cloth_assemble_bell(x, v, dt))
        print(f"# paper-layout assembly {dt}: {out[f'bell_assemble_ms_{dt}']:.2f} ms (width {width})", flush=True)
    out["bell_width"] = width

    # solver SpMV inside CG (FP32 and BF16 blocks)
    rowptr, _colidx = ctx.pattern()
    nnzb = int(rowptr[-1].item())
    out["nnzb"] = nnzb
    bytes_alg = nnzb * (9 * 4 + 4) + c.nv * (16 + 24)
    out["spmv_alg_bytes_f32"] = bytes_alg
    for dt in ["f32", "bf16"]:
        b = ctx.cloth_assemble(x, v, dt)
        ctx.profile(1)
        ctx.cloth_pcg_solve(b, tol=1e-30, maxit=a.cg_iters, raise_on_error=False, max_sweeps=1, precond="block")
        prof = ctx.profile_read()
        ctx.profile(0)
        us = prof["spmv"]["median_ms"] * 1e3
        out[f"cg_spmv_us_{dt}"] = us
        print(f"# CG SpMV {dt} blocks: {us:.1f} us median", flush=True)

    # BELL SpMV (FP32 table)
    ctx.cloth_assemble_bell(x, v, "f32")
    xs = torch.from_numpy(np.random.default_rng(11).normal(size=(c.nv, 3))).cuda()
    y = torch.empty_like(xs)
    ctx.cloth_spmv_bell(xs, y)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(a.spmv_reps):
        ctx.cloth_spmv_bell(xs, y)
    ev1.record()
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) * 1e3 / a.spmv_reps
    out["bell_spmv_us_f32_with_round"] = us
    pad_bytes = (width * c.nv - nnzb) * (9 * 4 + 4)
    out["bell_padded_fraction"] = 1.0 - nnzb / (width * c.nv)
    out["bell_spmv_padding_bytes"] = pad_bytes
    print(f"# paper-layout SpMV f32 (with the x rounding kernel): {us:.1f} us; "
          f"padding {100 * out['bell_padded_fraction']:.1f}% of the slots", flush=True)
    out["gbs_alg_cg_f32"] = bytes_alg / (out["cg_spmv_us_f32"] * 1e3)
    out["gbs_alg_bell_f32"] = bytes_alg / (us * 1e3)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
