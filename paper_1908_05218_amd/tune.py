"""Tile autotuner of the batched GEMM.

Runs whole products of the tuning workloads once per workgroup tile (every
launch forced to that tile, each launch timed by itself) and once with the
library's shape heuristic, then writes tiles.txt next to the library: for
every launch key (element types, transposes, m, n, k, log2 output count,
log2 tasks per output) the tile with the least total time, where it beats
the heuristic by more than 2 %.  Each configuration runs in a fresh process
(the library reads its tuning switches once).

    python -m paper_1908_05218_amd.tune            # from the repository root, on the GPU
"""
import collections
import math
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tiles.txt")
TILES = ["32x32", "96x32", "32x96", "96x96", "32x64", "64x32", "64x64", "32x32ws"]

# products timed per configuration: plates64k (C = A A, eps 1e-4) in both
# precisions, and the complex Helmholtz sphere of 32,768 points (eps 1e-3)
RUNNER = r"""
import math, sys
sys.path.insert(0, sys.argv[1])
import paper_1908_05218_amd as h2
from h2inputs import configs, points
ctx = h2.Context(0)
w = configs.plates64k()
A = h2.build(ctx, w.pts, w.leaf_size, w.eta, w.order, w.kernel.self_value)
for prec in ("fp32_bulk", "fp64"):
    for _ in range(2):
        h2.mmp(ctx, A, A, 1e-4, precision=prec).free()
n = 32768
kappa = 2 * math.pi / (10 * math.sqrt(4 * math.pi / n))
rho = 2.0 / math.sqrt(n)
pts = points.fibonacci_sphere(n)
S = h2.build(ctx, pts, 64, 1.0, 3, 1 / (2 * math.pi * rho) - 1j * kappa / (4 * math.pi),
             kernel="helmholtz", wavenumber=kappa)
T = h2.build(ctx, pts, 64, 1.0, 3, 1 / (2 * math.pi * rho) - 1j * kappa / (8 * math.pi),
             kernel="helmholtz", wavenumber=kappa / 2, share_tree_with=S)
for _ in range(2):
    h2.mmp(ctx, S, T, 1e-3).free()
ctx.close()
"""


def run(tile, root):
    fd, log = tempfile.mkstemp(suffix=".tiles")
    os.close(fd)
    env = dict(os.environ, H2_TILE_LOG=log, H2_TILE_TABLE=os.devnull,
               H2_TILE_FORCE=str(tile))
    subprocess.run([sys.executable, "-c", RUNNER, root], env=env, check=True)
    tot = collections.defaultdict(float)
    for line in open(log):
        f = line.split()
        tot[" ".join(f[:11])] += float(f[12])
    os.unlink(log)
    return tot


def main():
    root = os.path.dirname(HERE)
    base = run(-1, root)
    print(f"heuristic: {sum(base.values()):.2f} ms over {len(base)} launch keys", flush=True)
    per = {}
    for t, name in enumerate(TILES):
        per[t] = run(t, root)
        print(f"tile {name}: {sum(per[t].values()):.2f} ms", flush=True)
    rows, gain = [], 0.0
    for key, b in sorted(base.items()):
        best, bt = None, b
        for t in per:
            v = per[t].get(key, math.inf)
            if v < bt:
                best, bt = t, v
        if best is not None and bt < 0.98 * b:
            rows.append(f"{key} {best}")
            gain += b - bt
    total = sum(base.values())
    with open(TABLE, "w") as f:
        f.write("# workgroup tiles of the batched GEMM by launch key, written by\n"
                "# python -m paper_1908_05218_amd.tune (plates64k FP32-bulk and FP64 products,\n"
                "# complex Helmholtz sphere of 32,768 points); key: element bytes, A float,\n"
                "# B float, block-product symbol, transA, transB, m, n, k, log2 outputs,\n"
                "# log2 tasks per output; value: tile id (0 32x32, 1 96x32, 2 32x96, 3 96x96,\n"
                "# 4 32x64, 5 64x32, 6 64x64, 7 32x32 wave-split)\n"
                f"# timed launches: {total:.2f} ms with the heuristic, {total - gain:.2f} ms with this table\n")
        for r in rows:
            f.write(r + "\n")
    print(f"wrote {len(rows)} entries to {TABLE}: {total:.2f} -> {total - gain:.2f} ms", flush=True)


if __name__ == "__main__":
    main()
