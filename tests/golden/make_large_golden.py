"""Writes large_top1000.txt: the exact top-1000 triangles of the 100M-vertex / 2B-edge workload
(graphgen.large(): Chung-Lu, gamma 2.0, Zipf(1.5) weights on [1, 1e6], seed 0) at p = 1 and
p = +inf, computed by the CPU oracle alone on a certified subgraph (tests/certificate.py:
certified_topk; the oracle cannot enumerate the whole graph's triangles within a test).  It
calls only graphgen (inputs), numpy and oracle/.

    ORC_PROGRESS=1 python tests/golden/make_large_golden.py [out_path]

Needs ~100 GB of host memory and 16 cores for a few minutes.
"""
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import graphgen  # noqa: E402
import certificate  # noqa: E402


def main():
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "large_top1000.txt")
    t0 = time.time()
    g = graphgen.large()
    print(f"[golden] graph n={g.n} m={g.m} ({time.time() - t0:.0f}s)", flush=True)
    lines = []
    for p in (1.0, math.inf):
        t = time.time()
        r, desc = certificate.certified_topk(g.n, g.src, g.dst, g.w, 1000, p,
                                             log=lambda s: print(s, flush=True))
        el = time.time() - t
        print(f"[golden] p={p}: {r['n_out']} triangles, form {desc['form']}, {el:.0f}s", flush=True)
        lines.append(f"# p={p} form={desc['form']} subgraph_edges={desc.get('edges')} "
                     f"bound_steps={desc.get('steps')} oracle_wall_s={el:.1f}")
        for rank in range(r["n_out"]):
            lines.append(f"{p} {rank} {r['i'][rank]} {r['j'][rank]} {r['l'][rank]} {r['score'][rank].hex()}")
    with open(out, "w") as f:
        f.write("# Exact top-1000 of graphgen.large() (n=100M, ~2B edges, gamma 2.0, Zipf(1.5), seed 0) by the\n")
        f.write("# CPU oracle on a certified subgraph; written by tests/golden/make_large_golden.py\n")
        f.write("# command: ORC_PROGRESS=1 python tests/golden/make_large_golden.py\n")
        f.write(f"# total wall time {time.time() - t0:.0f}s on {os.cpu_count()} cores\n")
        f.write("# columns: p rank i j l score(float.hex)\n")
        f.write("\n".join(lines) + "\n")
    print(f"[golden] wrote {out} ({time.time() - t0:.0f}s)", flush=True)


if __name__ == "__main__":
    main()
