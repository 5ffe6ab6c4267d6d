"""Fixed-work kernel driver for hardware-counter runs.

Runs a bounded amount of the solver's work on one workload through the C ABI
(``--assemblies`` assemblies of the initial state, then a CG solve capped
at ``--iters`` iterations) plus a
plain device copy of known size, so that a counter profiler can take the
bytes each kernel fetches and writes per dispatch and scale them against the
copy, whose traffic is exactly 2 x its size.

    python -m paper_2008_00409_amd.kernel_bench --workload large --blocks f32 --iters 50
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="large", choices=["large", "medium", "batch"])
    ap.add_argument("--blocks", default="f32", choices=["f32", "bf16", "f16", "f64"])
    ap.add_argument("--iters", type=int, default=50, help="CG iterations (solve capped, tolerance unreachable)")
    ap.add_argument("--precond", default="jacobi", choices=["jacobi", "block"])
    ap.add_argument("--spb", type=int, default=0, help="slices per SpMV block (0: library default)")
    ap.add_argument("--rpb", type=int, default=0, help="rows per vector block (0: library default)")
    ap.add_argument("--lds-window", type=int, default=1, help="1: stage the SpMV's p window in LDS")
    ap.add_argument("--narrow", type=int, default=1, help="1: 16-bit column offsets when they fit")
    ap.add_argument("--copy-mib", type=int, default=1024, help="size of the calibration copy")
    ap.add_argument("--copies", type=int, default=5)
    ap.add_argument("--assemblies", type=int, default=1, help="assemblies of the initial state before the solve")
    a = ap.parse_args(argv)

    import torch

    from . import binding, meshgen as mg

    if not torch.cuda.is_available():
        sys.exit("kernel_bench needs a GPU")
    c = {"large": mg.config_large, "medium": mg.config_medium, "batch": mg.config_batch}[a.workload]()
    ctx = binding.Context.from_cloth(c)
    if a.workload == "batch":             # many independent cloths: per-instance CG scalars
        ctx.set_instances([r[0] for r in c.sheet_ranges] + [c.nv])
    if a.spb:
        ctx.set_option(binding.PC_OPT_SPMV_SLICES_PER_BLOCK, a.spb)
    if a.rpb:
        ctx.set_option(binding.PC_OPT_VECTOR_ROWS_PER_BLOCK, a.rpb)
    ctx.set_option(binding.PC_OPT_LDS_WINDOW, a.lds_window)
    ctx.set_option(binding.PC_OPT_NARROW_COLUMNS, a.narrow)
    x = torch.from_numpy(c.x0.copy()).cuda()
    v = torch.from_numpy(c.v0.copy()).cuda()
    print(f"# kernel_bench {c.name}: nv={c.nv} nt={c.nt} blocks={a.blocks} precond={a.precond} iters={a.iters}",
          flush=True)
    for _ in range(max(1, a.assemblies)):
        b = ctx.cloth_assemble(x, v, a.blocks)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dv, info = ctx.cloth_pcg_solve(b, tol=1e-30, maxit=a.iters, raise_on_error=False, max_sweeps=1,
                                   precond=a.precond)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    print(f"# solve: {info['iters']} iterations in {t_solve * 1e3:.1f} ms (status {info['status']})", flush=True)

    n = a.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.copies):
        torch.mul(src, 1.0, out=dst)      # elementwise copy kernel: reads and writes copy_mib MiB each
    torch.cuda.synchronize()
    t_copy = (time.perf_counter() - t0) / a.copies
    print(json.dumps({"workload": c.name, "nv": c.nv, "blocks": a.blocks, "cg_iters": info["iters"],
                      "solve_ms": t_solve * 1e3, "copy_bytes_each_way": n * 4,
                      "copy_ms": t_copy * 1e3}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
