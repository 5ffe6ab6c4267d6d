"""Host-side parts of the benchmark's contract (no GPU): a request for more
than one GPU ends with a message and exit status 2 before any device work,
and the SpMV byte model that the roofline divides by the measured launch
time gives the per-launch figures used at 1.65M triangles (828,153 rows,
10,617,589 blocks of the flipped sheets, less the zero diagonal blocks the
solver layout leaves out): per stored block its values plus a 2-byte column
offset, per row the float4 input, the product and the FP64 mass, plus the
row pointers."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr and p.stdout == ""


def test_spmv_byte_model_at_full_size():
    nv, nnzb = 828153, 10617589
    # BF16 blocks (18 B), packed FP32 direction (12 B per row), FP32 product
    # (12 B per row), FP64 mass, per stored block
    assert bench.spmv_bytes(nv, nnzb, "bf16", 2, 12) == nnzb * 20 + nv * 32 + 4 * (nv + 1) == 242165292
    # FP32 blocks (36 B), FP64 product (24 B per row)
    assert bench.spmv_bytes(nv, nnzb, "f32", 2, 24) == nnzb * 38 + nv * 44 + 4 * (nv + 1) == 443219730
    # 32-bit columns add 2 B per block
    assert bench.spmv_bytes(nv, nnzb, "bf16", 4, 12) - bench.spmv_bytes(nv, nnzb, "bf16", 2, 12) == 2 * nnzb


def test_solver_blocks_leave_out_zero_diagonals():
    """The solver layout stores a row's diagonal block only when the row is
    free and has a pinned column (else D_i = 0): counted here row by row."""
    import numpy as np
    rng = np.random.default_rng(4)
    nv = 40
    rows = []
    for i in range(nv):
        cols = sorted(set(rng.choice(nv, size=5, replace=False).tolist()) | {i})
        rows.append(cols)
    rowptr = np.cumsum([0] + [len(r) for r in rows])
    colidx = np.concatenate([np.array(r) for r in rows])
    pinned = (rng.random(nv) < 0.2).astype(np.uint8)
    want = 0
    for i, r in enumerate(rows):
        keep = pinned[i] == 0 and any(pinned[j] for j in r if j != i)
        want += len(r) - (0 if keep else 1)
    assert bench.solver_blocks(rowptr, colidx, pinned) == want
