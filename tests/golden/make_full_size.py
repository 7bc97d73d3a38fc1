"""Write the expected values of the full-size parity tests, from the CPU oracle only.

Every value written here comes from ``oracle`` (the plain C implementation of the
method) on inputs drawn by ``paper_1706_00037_amd.inputs``; nothing is taken from
the GPU library.  Each case is one JSON file under ``tests/golden/full_size/``:

  eval_n7000_M16384        every objective of 16384 random candidates at n = 7000
                           (density 0.5): SHA-256 of the int64 values, 64 block
                           sums of 256 candidates, the first values
  ms_n2500_M65536_G20      the multi-start loop (Fig. 2) at n = 2500, density 0.1,
                           M = 65536, lambda = 1/2, 20 generations
  ms_n7000_M16384_lam*_G3  the same at n = 7000, density 0.5, M = 16384, three
                           generations, for lambda = 3/10, 1/2 and 4/5
  batch_int16_G10          four int16 instances shaped like the batched workload
                           (n 1000 to 7000, the three densities), M = 4096, G = 10
  serve_first64_G10        the first 64 requests of the serving workload
                           (n ~ U{500..7000}, density ~ U[0.05, 1]), G = 10; the
                           file is rewritten after every request, cheapest first
  serve_small_G10          every other request with n <= 1500 among the 2100 of
                           the serving bench's trace (100 warm-up + 2000 timed)
  ms_n8192_M70000_multichunk  one generation at n = 8192, density 0.05, M = 70000,
                           lambda = 0, ascents capped at 32 flips: more passers than one
                           Delta workspace holds
  ms_n7000_M16384_blend_G3 the headline workload with blending diversification
                           (the bench's blend leg), 3 generations
  seq_n7000_I2500          the loop of Fig. 2 on the headline instance, 2500
                           iterations, Mean over 1000 samples, lambda = 1/2 (the bench's
                           sequential leg): its statistics, replacement history, final
                           solution and the SHA-256 of every iteration's objective

A multi-start case records, per generation, the screen statistics {Sum, Max,
passers, flips, incumbent} and the SHA-256 of every candidate's objective before
and after the ascent, and the final incumbent (value and words).

    python tests/golden/make_full_size.py [case ...] [--threads T]

Run time with 8 threads: minutes per case, about two hours for the serving subset.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1706_00037_amd.inputs import (BATCH_PARAMS, BATCH_SUBSET, SERVE_PARAMS, WORKLOADS,  # noqa: E402
                                         make_instance, random_candidates, serving_requests)

OUT = os.path.join(HERE, "full_size")
EVAL_CAND_SEED = 31
SERVE_COUNT = 64
SERVE_TRACE = 2100      # requests of the serving bench's trace
SERVE_SMALL_N = 1500


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def words_hex(x: np.ndarray) -> list:
    return [f"{int(w):016x}" for w in np.asarray(x, np.uint64)]


def write(name: str, obj: dict):
    os.makedirs(OUT, exist_ok=True)
    tmp = os.path.join(OUT, name + ".json.tmp")
    with open(tmp, "w") as fh:
        json.dump(obj, fh, indent=1)
        fh.write("\n")
    os.replace(tmp, os.path.join(OUT, name + ".json"))


def multistart_record(Q, params: dict, threads: int, dump: bool = True, flags: int = 0) -> dict:
    o = oracle.multistart(Q, threads=threads, dump=dump, flags=flags, **params)
    rec = dict(params=params, best_f=o["best_f"], have_best=o["have_best"],
               best_x=words_hex(o["best_x"]), stats=o["stats"].tolist())
    if dump:
        rec["f_sha256"] = [digest(o["f_all"][g]) for g in range(params["G"])]
        rec["f_after_sha256"] = [digest(o["fa_all"][g]) for g in range(params["G"])]
    return rec


def case_eval(threads: int):
    c = WORKLOADS["n7000_d0.50_M16384"]
    n, M = c["n"], c["M"]
    Q = make_instance(n, c["density"], c["lo"], c["hi"], c["inst_seed"])
    X = random_candidates(M, n, EVAL_CAND_SEED)
    f = oracle.eval_many(Q, X, threads=threads)
    write("eval_n7000_M16384", dict(workload="n7000_d0.50_M16384", cand_seed=EVAL_CAND_SEED, M=M,
                                    f_sha256=digest(f), block=256,
                                    block_sums=[int(s) for s in f.reshape(-1, 256).sum(1)],
                                    head=[int(v) for v in f[:16]]))


def case_multistart(workload: str, G: int, lam, name: str, threads: int):
    c = WORKLOADS[workload]
    Q = make_instance(c["n"], c["density"], c["lo"], c["hi"], c["inst_seed"])
    params = dict(M=c["M"], H=c["H"], lam_num=lam[0], lam_den=lam[1], G=G, run_seed=c["run_seed"])
    rec = multistart_record(Q, params, threads)
    rec["workload"] = workload
    write(name, rec)


def case_batch(threads: int):
    inst = []
    for k, s in enumerate(BATCH_SUBSET):
        Q = make_instance(s["n"], s["density"], -32768, 32767, 4001 + k)
        params = dict(BATCH_PARAMS, run_seed=4000 + k)
        rec = multistart_record(Q, params, threads, dump=False)
        rec.update(n=s["n"], density=s["density"], inst_seed=4001 + k)
        inst.append(rec)
        print(f"  batch instance {k} (n={s['n']}) done", flush=True)
    write("batch_int16_G10", dict(instances=inst))


def serve_requests(name: str, count: int, wanted, threads: int):
    """Oracle results of the requests `wanted` (indices into the first `count` of the
    serving stream), cheapest first; the file is rewritten after each request."""
    reqs = serving_requests(count)
    path = os.path.join(OUT, name + ".json")
    done = {}
    if os.path.exists(path):
        with open(path) as fh:
            done = {int(k): v for k, v in json.load(fh)["requests"].items()}
    for r in sorted(wanted, key=lambda r: reqs[r]["n"]):
        if r in done:
            continue
        q = reqs[r]
        t = time.time()
        Q = make_instance(q["n"], q["density"], -100, 100, q["inst_seed"])
        rec = multistart_record(Q, dict(SERVE_PARAMS, run_seed=q["run_seed"]), threads, dump=False)
        rec.update(q)
        done[r] = rec
        write(name, dict(count=count, requests={str(k): done[k] for k in sorted(done)}))
        print(f"  request {r} (n={q['n']}) done in {time.time() - t:.0f} s; {len(done)} of {len(wanted)}",
              flush=True)


def case_serve(threads: int):
    serve_requests("serve_first64_G10", SERVE_COUNT, range(SERVE_COUNT), threads)


def case_serve_small(threads: int):
    reqs = serving_requests(SERVE_TRACE)
    wanted = [r for r in range(SERVE_COUNT, SERVE_TRACE) if reqs[r]["n"] <= SERVE_SMALL_N]
    serve_requests("serve_small_G10", SERVE_TRACE, wanted, threads)


def case_multichunk(threads: int):
    Q = make_instance(8192, 0.05, -100, 100, 818)
    # capped ascents: the oracle's one-column update walks Q by columns, so ~35000
    # uncapped ascents at n = 8192 take hours; the chunking is the same either way
    params = dict(M=70000, H=10, lam_num=0, lam_den=1, G=1, run_seed=5, max_flips=32)
    rec = multistart_record(Q, params, threads)
    rec.update(n=8192, density=0.05, inst_seed=818)
    write("ms_n8192_M70000_multichunk", rec)


def case_blend7000(threads: int):
    c = WORKLOADS["n7000_d0.50_M16384"]
    Q = make_instance(c["n"], c["density"], c["lo"], c["hi"], c["inst_seed"])
    params = dict(M=c["M"], H=c["H"], lam_num=1, lam_den=2, G=3, run_seed=c["run_seed"])
    rec = multistart_record(Q, params, threads, flags=oracle.FLAG_BLEND)
    rec.update(workload="n7000_d0.50_M16384", blend=True)
    write("ms_n7000_M16384_blend_G3", rec)


def case_seq7000(threads: int):
    c = WORKLOADS["n7000_d0.50_M16384"]
    Q = make_instance(c["n"], c["density"], c["lo"], c["hi"], c["inst_seed"])
    params = dict(iterations=2500, samples=1000, lam_num=1, lam_den=2, run_seed=c["run_seed"])
    o = oracle.sequential(Q, H=c["n"], threads=threads, **params)
    rec = {k: (int(o[k]) if k != "have_best" else bool(o[k]))
           for k in ("best_f", "have_best", "sample_sum", "start_f", "passers", "flips", "improvements")}
    rec.update(workload="n7000_d0.50_M16384", params=params, history=o["history"].tolist(),
               best_x=words_hex(o["best_x"]), f_sha256=digest(o["f_dump"]))
    write("seq_n7000_I2500", rec)


CASES = {
    "eval": case_eval,
    "ms2500": lambda th: case_multistart("n2500_d0.10_M65536", 20, (1, 2), "ms_n2500_M65536_G20", th),
    "ms7000_1_2": lambda th: case_multistart("n7000_d0.50_M16384", 3, (1, 2), "ms_n7000_M16384_lam1_2_G3", th),
    "ms7000_3_10": lambda th: case_multistart("n7000_d0.50_M16384", 3, (3, 10), "ms_n7000_M16384_lam3_10_G3", th),
    "ms7000_4_5": lambda th: case_multistart("n7000_d0.50_M16384", 3, (4, 5), "ms_n7000_M16384_lam4_5_G3", th),
    "batch": case_batch,
    "serve": case_serve,
    "serve_small": case_serve_small,
    "multichunk": case_multichunk,
    "blend7000": case_blend7000,
    "seq7000": case_seq7000,
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=list(CASES))
    # the serving subsets resume from what their files already hold
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    for name in a.cases:
        t = time.time()
        print(f"[golden] {name}", flush=True)
        CASES[name](a.threads)
        print(f"[golden] {name} written in {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    main()
