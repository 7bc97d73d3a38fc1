"""Solve a benchmark file with the multi-start loop and print its history.

    python -m paper_1706_00037_amd.solve FILE [--format orlib|triplets] [--index K]
        [--M 16384] [--H 10] [--lam 1/2] [--G 50] [--seed 1] [--deriv] [--blend] [--target T]

Reads problem K of FILE (ubqp_read_instance), makes it resident and runs G
generations of M candidates on GPU 0; prints one line per generation
(incumbent, passers, flips, ms from the start of the run) and, with --target,
the time to target: the end of the first generation whose incumbent reaches T.
The last line is a JSON summary.
"""
from __future__ import annotations

import argparse
import json
import sys

from . import ubqp


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_1706_00037_amd.solve")
    ap.add_argument("file")
    ap.add_argument("--format", choices=("orlib", "triplets"), default="orlib")
    ap.add_argument("--index", type=int, default=0)
    ap.add_argument("--M", type=int, default=16384)
    ap.add_argument("--H", type=int, default=10)
    ap.add_argument("--lam", default="1/2")
    ap.add_argument("--G", type=int, default=50)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--max-flips", type=int, default=0)
    ap.add_argument("--deriv", action="store_true", help="generation-0 seed 0 is the first-derivative start")
    ap.add_argument("--blend", action="store_true", help="diversify by blending pairs of seeds")
    ap.add_argument("--target", type=int, default=None)
    a = ap.parse_args(argv)
    num, den = (int(v) for v in a.lam.split("/"))
    fmt = ubqp.UBQP_FMT_ORLIB if a.format == "orlib" else ubqp.UBQP_FMT_TRIPLETS
    Q, count = ubqp.read_instance(a.file, fmt, a.index)
    flags = (ubqp.UBQP_DERIV_START if a.deriv else 0) | (ubqp.UBQP_BLEND if a.blend else 0)
    ctx = ubqp.Context(0)
    prob = ctx.problem(Q)
    r = ctx.multistart(prob, M=a.M, H=a.H, lam_num=num, lam_den=den, G=a.G, max_flips=a.max_flips,
                       run_seed=a.seed, flags=flags)
    for g in range(r["generations"]):
        s = r["stats"][g]
        print(f"gen {g:4d}  incumbent {int(s[4]):>14d}  passers {int(s[2]):>7d}  flips {int(s[3]):>10d}  "
              f"{r['gen_ms'][g]:10.3f} ms", file=sys.stderr)
    out = dict(file=a.file, index=a.index, problems_in_file=count, n=int(Q.shape[0]), M=a.M, H=a.H, lam=a.lam,
               G=a.G, best_f=r["best_f"], total_ms=float(r["gen_ms"][-1]) if r["generations"] else 0.0)
    if a.target is not None:
        hit = ubqp.time_to_target(r, a.target)
        out["target"] = a.target
        out["time_to_target_ms"] = None if hit is None else hit[1]
        out["target_generation"] = None if hit is None else hit[0]
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
