"""Throughput of the multi-start UBQP hot path on one MI355X.

A step is one generation of the multi-start loop over M candidates:
diversify -> exact evaluation -> T(lambda) screening -> steepest ascent of the
passers -> incumbent update and next seeds, all on the device through the C ABI.

Workload (the configuration the headline metric is quoted on): n = 7000
variables, 50% density, coefficients uniform in [-100, 100] \\ {0}, M = 16384
candidates per generation (S = 820 seeds x 10 Glover steps x {x', x''}),
lambda = 1/2, ascent to a 1-flip local optimum.  Synthetic seeded instance
(stand-in for the Palubeckis n = 7000 problems).

value = candidates evaluated and processed per second over the timed
generations (whole path).  Also reported: the batched evaluation alone, the
paper's Table 1 replica (1000 random solutions, n = 2500..7000), the roofline
of the dominant kernel from stream events recorded around each phase during the
timed generations, the CPU oracle timed on a bounded sample, and the serving
form: solves/s and p50/p99 latency of Poisson-arriving solve requests against
the request server, beside the same server admitting one request at a time.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
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

METRIC = "exact xQx evals/s at n=7000 (vs plain); served solves/s + p50/p99 latency"
HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0      # dense int8 matrix-core peak, TOP/s
VALU_INT32_TOPS = 39.3       # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz: int32 lane-operations/s / 1e12
PAPER_TABLE1_S = {2500: 0.7, 5000: 2.0, 6000: 3.0, 7000: 3.5}   # GPU seconds per 1000 evals
# Per-launch memory traffic of the main kernels at the headline workload comes from
# the two counter passes (FETCH_SIZE, WRITE_SIZE; calibrated against a 1 GiB device
# copy) summarised in this file, together with the SHA-256 of each kernel's source
# at the time; a kernel whose source has changed since gets traffic null.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "counters_n7000_M16384.md")
CSRC = os.path.join(ROOT, "paper_1706_00037_amd", "csrc")


def load_traffic():
    """{kernel: {"gb": fetched + written GB per launch, ...}} for the kernels whose
    source is unchanged since the counters were taken; others map to None."""
    import hashlib
    import re
    out = {}
    try:
        text = open(TRAFFIC_FILE).read()
        block = re.search(r"```json\n(.*?)\n```", text, flags=re.S).group(1)
        table = json.loads(block)
    except (OSError, AttributeError, ValueError):
        return out
    for name, rec in table.items():
        try:
            sha = hashlib.sha256(open(os.path.join(CSRC, rec["source"]), "rb").read()).hexdigest()
        except OSError:
            sha = None
        out[name] = rec if sha == rec.get("source_sha256") else None
    return out


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-e1", action="store_true")
    ap.add_argument("--lam", default="1/2")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-lam-sweep", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-blend", action="store_true")
    ap.add_argument("--no-seq", action="store_true")
    ap.add_argument("--no-relink", action="store_true")
    ap.add_argument("--no-gen0", action="store_true", help="skip the generation-0 leg and the population summary")
    ap.add_argument("--no-peaks", action="store_true", help="skip the MFMA and read-bandwidth measurements")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-active", type=int, default=32)
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy 1 GiB device-to-device, a dispatch of known traffic for counter calibration")
    return ap.parse_args()


def cpu_baseline(Q, n, M, P_per_gen, flips_per_gen, threads):
    """The oracle as it stands, on the host cores, timed on a bounded sample of the
    workload.  Measured: the objective of 96*threads candidates (threads in
    parallel), one closed-form delta vector (the ascent's initialisation) and
    2*threads full ascents from random candidates (threads in parallel).  A
    generation then costs (M t_eval + P t_init + F t_flip) / threads of wall time
    with the timed generations' own passer count P and flip count F."""
    import oracle
    from paper_1706_00037_amd.inputs import random_candidates

    Ne = 96 * threads
    Xs = random_candidates(Ne, n, 99)
    t = time.perf_counter()
    oracle.eval_many(Q, Xs, threads=threads)
    t_eval = (time.perf_counter() - t) * threads / Ne            # serial seconds per candidate
    t = time.perf_counter()
    oracle.delta(Q, Xs[0])
    t_init = time.perf_counter() - t                              # serial seconds per initialisation
    Na = 2 * threads
    Xa = random_candidates(Na, n, 98)
    fa = oracle.eval_many(Q, Xa, threads=threads)
    t = time.perf_counter()
    _, _, fl = oracle.ascent_many(Q, Xa, np.arange(Na, dtype=np.int32), fa, threads=threads)
    t_asc = time.perf_counter() - t
    F = float(fl.sum())
    t_flip = max(0.0, t_asc * threads - Na * t_init) / max(F, 1.0)
    t_gen = (M * t_eval + P_per_gen * t_init + flips_per_gen * t_flip) / threads
    # the oracle's evaluation rate at the three single-instance shapes, one thread and
    # all `threads` (bounded samples: 8 and 8 * threads candidates)
    from paper_1706_00037_amd.inputs import WORKLOADS, make_instance
    rates = {}
    for name in ("n500_d0.10_M1000", "n2500_d0.10_M65536", "n7000_d0.50_M16384"):
        c = WORKLOADS[name]
        Qc = Q if c["n"] == n else make_instance(c["n"], c["density"], c["lo"], c["hi"], c["inst_seed"])
        r = {}
        for th, cnt in ((1, 8), (threads, 8 * threads)):
            Xc = random_candidates(cnt, c["n"], 97)
            t = time.perf_counter()
            oracle.eval_many(Qc, Xc, threads=th)
            r[str(th)] = cnt / (time.perf_counter() - t)
        rates[f"n={c['n']}"] = {"threads": r}
    # the small configuration end to end (n=500, M=1000, 20 generations), whole, one
    # thread and all threads
    c1 = WORKLOADS["n500_d0.10_M1000"]
    Q1 = make_instance(c1["n"], c1["density"], c1["lo"], c1["hi"], c1["inst_seed"])
    e2e = {}
    for th in (1, threads):
        t = time.perf_counter()
        o1 = oracle.multistart(Q1, M=c1["M"], H=c1["H"], lam_num=c1["lam"][0], lam_den=c1["lam"][1], G=c1["G"],
                               run_seed=c1["run_seed"], threads=th)
        e2e[str(th)] = dict(s=time.perf_counter() - t, best_f=o1["best_f"])
    host = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                host = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=M / t_gen, unit="evals/s", cores=threads, kind="oracle",
                sample=f"oracle at n={n}: objective of {Ne} candidates, one delta initialisation and {Na} "
                       f"ascents from random candidates ({int(F)} flips), on {threads} threads; generation time "
                       f"(M t_eval + P t_init + F t_flip)/threads with the timed generations' mean "
                       f"P={P_per_gen:.0f}, F={flips_per_gen:.0f}",
                ms_per_step=t_gen * 1e3, eval_only_evals_per_s=threads / t_eval,
                t_eval_ms=t_eval * 1e3, t_init_ms=t_init * 1e3, t_flip_us=t_flip * 1e6,
                eval_rates_evals_per_s=rates, e2e_n500_M1000_G20_threads=e2e, host_cpu=host,
                host_logical_cpus=os.cpu_count())


def passers_of(f, lam_num, lam_den):
    """Boolean mask of the candidates whose objective clears T(lambda) over the
    population f (exact integers; used only to describe the timed populations)."""
    M = len(f)
    s, mx = int(sum(int(v) for v in f)), int(max(f))
    rhs = (lam_den - lam_num) * s + lam_num * M * mx
    return np.array([lam_den * M * int(v) > rhs for v in f])


def population_summary(ctx, prob, kw, gens):
    """Distinct objective values among all candidates and among the passers of each
    of the generations `gens` of the run kw (a second, identical run with an
    objective dump; distinct values bound the distinct solutions from below)."""
    import torch
    G, M = kw["G"], kw["M"]
    dump = torch.zeros(G * M, dtype=torch.int64, device="cuda")
    ctx.multistart(prob, f_dump=dump, **kw)
    fd = dump.cpu().numpy().reshape(G, M)
    out = []
    for g in gens:
        mask = passers_of(fd[g], kw["lam_num"], kw["lam_den"])
        out.append(dict(generation=int(g), distinct_objectives=int(len(np.unique(fd[g]))),
                        passers=int(mask.sum()), distinct_passer_objectives=int(len(np.unique(fd[g][mask])))))
    return out


def gen0_leg(ctx, ubqp, prob, c, lam_num, lam_den, K):
    """Generation 0 from random seeds, K times with distinct run seeds (1000 + k):
    the population is 820 random seeds x 20 Glover candidates, all distinct, and
    the passers are distinct solutions far from local optima.  Per-phase times from
    stream events, as for the headline."""
    n, M, H = c["n"], c["M"], c["H"]
    gen_ms, phases, st = [], [], []
    for k in range(K):
        r = ctx.run(prob, M=M, H=H, lam_num=lam_num, lam_den=lam_den, G=1, run_seed=1000 + k,
                    flags=ubqp.UBQP_TIMING)
        r.step(1)
        rr = r.result()
        r.close()
        gen_ms.append(float(rr["gen_ms"][0]))
        phases.append(rr["phase_ms"][0])
        st.append(rr["stats"][0])
    ph = np.array(phases)
    st = np.array(st)
    pop = population_summary(ctx, prob, dict(M=M, H=H, lam_num=lam_num, lam_den=lam_den, G=1, run_seed=1000), [0])
    ms = float(np.mean(gen_ms))
    return dict(runs=K, ms_per_generation=ms, evals_per_s=M / (ms * 1e-3),
                phases_ms={name: float(ph[:, i].mean()) for i, name in enumerate(ubqp.PHASES)},
                passers_per_gen=float(st[:, 2].mean()), flips_per_gen=float(st[:, 3].mean()),
                population=pop[0],
                note="generation 0 of K runs with distinct run seeds: random seeds, every candidate and "
                     "passer a distinct solution (stream-event time from the seeds to the end of the "
                     "generation)")


def make_request_instance(torch, n, density, seed, out):
    """Symmetric int8 instance of the serving workload, drawn on the device with
    torch's seeded Philox generator (upper-triangle mask Bernoulli(density),
    diagonal included, values uniform in [-100, 100] \\ {0}, mirrored) and copied
    into the host array `out` (int8 [n, n], page-locked)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    u = torch.randint(0, 200, (n, n), generator=g, device="cuda", dtype=torch.int16)
    v = torch.where(u >= 100, u - 99, u - 100)
    keep = torch.rand((n, n), generator=g, device="cuda") < density
    U = torch.triu(torch.where(keep, v, torch.zeros_like(v)))
    Q = (U + torch.tril(U.t(), -1)).to(torch.int8)
    torch.from_numpy(out).copy_(Q)


class PinnedArena:
    """One page-locked host block (hipHostMalloc of the HIP runtime torch loaded)
    handed out as int8 [n, n] arrays; freed by close()."""

    def __init__(self, nbytes):
        import ctypes
        self.ct = ctypes
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipHostMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, ctypes.c_uint]
        self.hip.hipHostFree.argtypes = [ctypes.c_void_p]
        self.ptr = ctypes.c_void_p()
        rc = self.hip.hipHostMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(nbytes), 0)
        if rc != 0 or not self.ptr.value:
            raise RuntimeError(f"hipHostMalloc of {nbytes} bytes failed ({rc})")
        self.nbytes, self.off = nbytes, 0

    def take(self, n):
        size = n * n
        assert self.off + size <= self.nbytes
        buf = (self.ct.c_int8 * size).from_address(self.ptr.value + self.off)
        self.off += (size + 255) // 256 * 256
        return np.ctypeslib.as_array(buf).reshape(n, n)

    def close(self):
        if self.ptr.value:
            self.hip.hipHostFree(self.ptr)
            self.ptr = self.ct.c_void_p()


def serving_bench(ctx, ubqp, torch, R=300, warm=20, rate=200.0, max_active=32, pool_gib=48, seed=5):
    """Poisson arrivals of multi-start solve requests (the serving request stream:
    request r has n ~ U{500..7000}, density ~ U[0.05, 1], coefficients in
    [-100, 100], M=4096, H=10, lambda=1/2, G=10, a fresh instance drawn with seed
    5000 + r and run seed 5000 + r) against the request server, then against the
    same server admitting one request at a time (the plain one-at-a-time GPU loop),
    on the same trace.  Every instance is drawn before the clock starts into
    page-locked host memory (a request's coefficients are in host memory when it
    arrives); latency = result on the host - scheduled arrival, upload included."""
    import threading
    from paper_1706_00037_amd.inputs import SERVE_PARAMS, serving_requests

    reqs = serving_requests(warm + R, seed=seed)
    total = sum((q["n"] * q["n"] + 255) // 256 * 256 for q in reqs)
    log(f"[serve] drawing {warm + R} fresh instances ({total / 2**30:.1f} GiB) into page-locked memory")
    t0 = time.perf_counter()
    arena = PinnedArena(total)
    inst = []
    for q in reqs:
        a = arena.take(q["n"])
        make_request_instance(torch, q["n"], q["density"], q["inst_seed"], a)
        inst.append(a)
    torch.cuda.synchronize()
    log(f"[serve] instances ready in {time.perf_counter() - t0:.1f} s")
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=R)
    offs = np.cumsum(gaps) - gaps[0]
    pr = lambda r: dict(SERVE_PARAMS, run_seed=reqs[r]["run_seed"])

    def run_trace(active):
        srv = ctx.server(pool_bytes=pool_gib << 30, max_active=active)
        try:
            ids = [srv.submit(inst[r], **pr(r)) for r in range(warm)]
            got = 0
            while got < len(ids):
                got += len(srv.wait(timeout_s=5.0))
            done = {}
            stop = threading.Event()

            def collect():
                while len(done) < R and not stop.is_set():
                    for x in srv.wait(timeout_s=0.5):
                        done[x["id"]] = x
            th = threading.Thread(target=collect)
            th.start()
            t0 = time.monotonic_ns() + 20_000_000
            sched = {}
            for k in range(R):
                at = t0 + int(offs[k] * 1e9)
                while True:
                    dt = at - time.monotonic_ns()
                    if dt <= 0:
                        break
                    time.sleep(min(dt, 2_000_000) / 1e9)
                i = srv.submit(inst[warm + k], **pr(warm + k))
                sched[i] = at
            th.join(timeout=600)
            stop.set()
            st = srv.stats()
        finally:
            srv.close()
        assert len(done) == R, f"{len(done)} of {R} requests finished"
        assert all(x["status"] == ubqp.UBQP_OK for x in done.values())
        lat = np.array([(done[i]["t_done_ns"] - sched[i]) / 1e6 for i in sched])
        end = max(x["t_done_ns"] for x in done.values())
        span = (end - t0) / 1e9
        return dict(solves_per_s=R / span, p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()), span_s=span,
                    max_running=st["max_running"], generations=st["generations"],
                    pool_high_gib=st["pool_high"] / 2**30, max_active=active)

    def run_burst(active, count=120):
        """Capacity: `count` requests (the first timed ones) submitted at once; solves/s over the drain."""
        srv = ctx.server(pool_bytes=pool_gib << 30, max_active=active)
        try:
            t0 = time.monotonic_ns()
            ids = [srv.submit(inst[warm + r], **pr(warm + r)) for r in range(count)]
            done = {}
            while len(done) < count:
                for x in srv.wait(timeout_s=5.0):
                    done[x["id"]] = x
        finally:
            srv.close()
        end = max(x["t_done_ns"] for x in done.values())
        return count / ((end - t0) / 1e9)

    try:
        log(f"[serve] trace: {R} requests at {rate}/s, continuous batching (max_active={max_active})")
        batched = run_trace(max_active)
        log(f"[serve] batched: {batched}")
        log("[serve] same trace, one request at a time")
        plain = run_trace(1)
        log(f"[serve] one at a time: {plain}")
        cap_b, cap_p = run_burst(max_active), run_burst(1)
    finally:
        arena.close()
    log(f"[serve] capacity (120 requests at once): {cap_b:.1f} solves/s batched, {cap_p:.1f} one at a time")
    batched["capacity_solves_per_s"] = cap_b
    plain["capacity_solves_per_s"] = cap_p
    ns = np.array([q["n"] for q in reqs[warm:]])
    return dict(batched=batched, one_at_a_time=plain, requests=R, warmup_requests=warm, rate_per_s=rate,
                distinct_instances=warm + R, mean_n=float(ns.mean()),
                workload=f"Poisson {rate:.0f} req/s; request r: n ~ U{{500..7000}}, density ~ U[0.05,1], "
                         f"[-100,100], M=4096, H=10, lambda=1/2, G=10, a fresh instance (seed 5000+r) and "
                         f"run seed per request, uploaded by the server from page-locked host memory")


def make_wide_instance(torch, n, density, seed):
    """Symmetric int16 instance for the batched workload, drawn on the device with
    torch's seeded Philox generator: upper-triangle mask Bernoulli(density)
    (diagonal included), values uniform in [-32768, 32767] \\\\ {0}, mirrored."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    u = torch.randint(-32768, 32767, (n, n), generator=g, device="cuda", dtype=torch.int32)
    v = torch.where(u >= 0, u + 1, u)
    keep = torch.rand((n, n), generator=g, device="cuda") < density
    U = torch.triu(torch.where(keep, v, torch.zeros_like(v)))
    return (U + torch.tril(U.t(), -1)).to(torch.int16).cpu().numpy()


def batched_bench(ctx, ubqp, torch, count=64, G=6, warm=2, seed=4):
    """64 instances, n ~ U{1000..7000}, density in {0.1, 0.5, 1.0}, int16
    coefficients (two int8 planes each), M = 4096, lambda = 1/2: one batch whose
    generation is one launch per step covering every instance (captured as a HIP
    graph), against the same instances run one after another."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(1000, 7001, size=count)
    ds = rng.choice([0.1, 0.5, 1.0], size=count)
    log(f"[batch] uploading {count} int16 instances")
    probs = [ctx.problem(make_wide_instance(torch, int(ns[k]), float(ds[k]), 4001 + k)) for k in range(count)]
    assert all(p.planes == 2 for p in probs)
    # tiles of the evaluation autotuned per (planes, n_pad, M) key when the batch is created
    params = [dict(M=4096, H=10, lam_num=1, lam_den=2, G=G, run_seed=4000 + k, flags=ubqp.UBQP_AUTOTUNE)
              for k in range(count)]
    ops = sum(2.0 * 4096 * int(n) * int(n) * 2 for n in ns)         # dense xQx work of one generation, 2 planes
    t0 = time.perf_counter()
    b = ctx.batch(probs, params)
    t_tune = time.perf_counter() - t0
    chosen = {}
    for p in probs:
        v, _ = ctx.tune_eval(p, 4096)                                  # cached: the variant in use
        chosen[str(v)] = chosen.get(str(v), 0) + 1
    log(f"[batch] tuned eval variants (instances per variant): {chosen} in {t_tune:.2f} s")
    b.step(warm)
    b.result(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(G - warm)
    res = [b.result(k) for k in range(count)]
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / (G - warm)
    b.close()
    flips = float(sum(r["stats"][warm:, 3].sum() for r in res)) / (G - warm)
    row_bytes = float(sum(r["stats"][warm:, 3].sum() * 2 * int(ns[k]) for k, r in enumerate(res))) / (G - warm)
    log(f"[batch] batched: {t_batch * 1e3:.2f} ms per generation of all {count} instances, "
        f"{flips:.0f} flips per generation")
    # the same batch with stream events around every phase (direct launches): the
    # ascent kernels' share of a generation and their row rate
    bt = ctx.batch(probs, [dict(p, flags=p["flags"] | ubqp.UBQP_TIMING) for p in params])
    bt.step(G)
    rt = bt.result(0)
    bt.close()
    ph_t = rt["phase_ms"][warm:]
    phases_b = {name: float(ph_t[:, i].mean()) for i, name in enumerate(ubqp.PHASES)}
    t_asc = phases_b["ascent_kernel"] * 1e-3
    log(f"[batch] phases with events (direct launches): {phases_b}")
    # the same generations, one instance after another
    t_seq = 0.0
    for k in range(count):
        r = ctx.run(probs[k], **params[k])
        r.step(warm)
        r.result()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r.step(G - warm)
        rr = r.result()
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        r.close()
        assert rr["best_f"] == res[k]["best_f"] and np.array_equal(rr["stats"], res[k]["stats"]), k
    t_seq /= (G - warm)
    log(f"[batch] one instance at a time: {t_seq * 1e3:.2f} ms per generation of all {count}")
    return dict(instances=count, ms_per_generation=t_batch * 1e3, evals_per_s=count * 4096 / t_batch,
                flips_per_generation=flips, phases_ms_direct=phases_b,
                ascent_roofline=dict(kernel="ascent_i16_batched (two int8 planes: int16 rows)", bound="hbm",
                                     algorithmic_gb=row_bytes / 1e9, avg_ms=t_asc * 1e3,
                                     achieved=row_bytes / t_asc / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                                     frac=row_bytes / t_asc / 1e9 / HBM_PEAK_GBS,
                                     note="2 n bytes of the int16 ascent matrix per flip; the 64 matrices "
                                          "(about 2.2 GB) exceed the Infinity Cache, so rows stream from HBM"),
                dense_tops=ops / t_batch / 1e12, sequential_ms_per_generation=t_seq * 1e3,
                speedup_vs_sequential=t_seq / t_batch, timed_generations=G - warm,
                eval_variants=chosen, tuning_s=t_tune,
                workload="64 instances, n ~ U{1000..7000}, density in {0.1,0.5,1.0}, int16 coefficients "
                         "(hi/lo int8 planes), M=4096, H=10, lambda=1/2")


def sequential_bench(ctx, WORKLOADS, make_instance, prob7000, Q7000, c7000):
    """The main loop of Fig. 2 as printed, 2500 iterations and Mean over 1000 random
    solutions, on the paper's two instance shapes: n=2500 at density 0.1 (ORLIB)
    and n=7000 at density 0.5 (Palubeckis p7000).  Reports the whole loop's time,
    iterations per second and the time of each replacement of the incumbent."""
    out = {}
    c2 = WORKLOADS["n2500_d0.10_M65536"]
    shapes = [("n2500_d0.1", make_instance(c2["n"], c2["density"], c2["lo"], c2["hi"], c2["inst_seed"]), None,
               c2["run_seed"]),
              ("n7000_d0.5", Q7000, prob7000, c7000["run_seed"])]
    for name, Q, prob, rs in shapes:
        prob = prob if prob is not None else ctx.problem(Q)
        kw = dict(iterations=2500, samples=1000, H=0, lam_num=1, lam_den=2, run_seed=rs)
        ctx.sequential(prob, **dict(kw, iterations=300))  # warm-up
        t0 = time.perf_counter()
        r = ctx.sequential(prob, **kw)
        wall = (time.perf_counter() - t0) * 1e3
        out[name] = dict(iterations=kw["iterations"], samples=kw["samples"], **{"lambda": "1/2"},
                         ms_loop=r["ms_device"], ms_loop_events=r["ms"], ms_call=wall,
                         iterations_per_s=kw["iterations"] / (r["ms_device"] * 1e-3),
                         best_f=r["best_f"], improvements=r["improvements"], passers=r["passers"],
                         flips=r["flips"], windows=r["windows"], evaluated=r["evaluated"],
                         last_improvement_iteration=int(r["history"][-1, 0]) if len(r["history"]) else None,
                         improvement_ms=[round(float(t), 3) for t in r["history_ms"]],
                         improvement_f=[int(v) for v in r["history"][:, 1]])
        log(f"[seq] {name}: {kw['iterations']} iterations in {r['ms_device']:.2f} ms (stream events "
            f"{r['ms']:.2f} ms, {wall:.2f} ms with set-up), "
            f"{r['improvements']} improvements (last at iteration {out[name]['last_improvement_iteration']}, "
            f"{out[name]['improvement_ms'][-1] if r['improvements'] else 0:.2f} ms), best f {r['best_f']}, "
            f"{r['passers']} passers, {r['windows']} windows, {r['evaluated']} candidates evaluated")
    return out


def relink_bench(ctx, ubqp, torch, prob, n, M, H, lam_num, lam_den, E=16, G=3):
    """The polishing phase: E incumbents of independent short runs (G generations
    each, run seeds 100..100+E-1) form the elite set; every ordered pair is
    relinked and the intermediate ascended.  Walk flips = sum over paths of
    (Hamming distance - 1); each streams one row of the ascent matrix."""
    runs = [ctx.multistart(prob, M=M, H=H, lam_num=lam_num, lam_den=lam_den, G=G, run_seed=100 + k)
            for k in range(E)]
    elite = np.stack([r["best_x"] for r in runs])
    best_elite = max(int(r["best_f"]) for r in runs)
    pairs = np.array([(a, b) for a in range(E) for b in range(E) if a != b], np.int32)
    P = len(pairs)
    ed = torch.from_numpy(elite.view(np.int64)).cuda()
    pd = torch.from_numpy(pairs).cuda()
    X = torch.empty((P, prob.W), dtype=torch.int64, device="cuda")
    fm = torch.empty(P, dtype=torch.int64, device="cuda")
    fo = torch.empty(P, dtype=torch.int64, device="cuda")
    st = torch.empty(P, dtype=torch.int32, device="cuda")
    ctx.relink(prob, ed, pd, X, fm, fo, st)  # warm-up
    ctx.sync()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.relink(prob, ed, pd, X, fm, fo, st)
    e1.record(stream)
    ctx.sync()
    ms = e0.elapsed_time(e1)
    bits = np.unpackbits(elite.view(np.uint8), axis=1, bitorder="little")
    dist = np.array([int((bits[a] != bits[b]).sum()) for a, b in pairs])
    walk = int(np.maximum(dist - 1, 0).sum())
    fo_h = fo.cpu().numpy()
    out = dict(elite=E, generations_per_elite_run=G, paths=P, ms=ms, walk_flips=walk,
               walk_flips_per_s=walk / (ms * 1e-3), walk_gb_per_s=walk * n / (ms * 1e-3) / 1e9,
               mean_distance=float(dist.mean()), best_elite_f=best_elite, best_relinked_f=int(fo_h.max()),
               improved_paths=int((fo_h > best_elite).sum()))
    log(f"[relink] {E} elite solutions (n={n}), {P} paths: {ms:.2f} ms, {walk} walk flips "
        f"({out['walk_gb_per_s']:.0f} GB/s of rows), best elite f {best_elite}, best relinked "
        f"{out['best_relinked_f']} ({out['improved_paths']} paths beat the elite)")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the path is built and measured on one GPU; how it would shard is a design only).",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1706_00037_amd import ubqp
    from paper_1706_00037_amd.inputs import WORKLOADS, make_instance, random_candidates

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 1 GiB read, 1 GiB written")
        del src, dst
    c = WORKLOADS["n7000_d0.50_M16384"]
    n, M, H = c["n"], c["M"], c["H"]
    lam_num, lam_den = (int(t) for t in args.lam.split("/"))
    K, Wm = args.steps, args.warmup
    log(f"[bench] instance n={n} density={c['density']} seed={c['inst_seed']}")
    Q = make_instance(n, c["density"], c["lo"], c["hi"], c["inst_seed"])
    ctx = ubqp.Context(0)
    prob = ctx.problem(Q)

    # ---- whole-path generations ------------------------------------------------
    G = Wm + K
    run = ctx.run(prob, M=M, H=H, lam_num=lam_num, lam_den=lam_den, G=G, run_seed=c["run_seed"],
                  flags=ubqp.UBQP_TIMING)
    log(f"[bench] warmup {Wm} generations")
    run.step(Wm)
    run.result()
    torch.cuda.synchronize()
    log(f"[bench] timing {K} generations")
    t0 = time.perf_counter()
    run.step(K)
    res = run.result()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run.close()
    wall_ms = (t1 - t0) * 1e3 / K
    gen_ms = np.diff(np.concatenate([[res["gen_ms"][Wm - 1] if Wm > 0 else 0.0], res["gen_ms"][Wm:]]))
    ph = res["phase_ms"][Wm:]
    st = res["stats"][Wm:]
    phase_mean = {name: float(ph[:, i].mean()) for i, name in enumerate(ubqp.PHASES)}
    P_mean, flips_mean = float(st[:, 2].mean()), float(st[:, 3].mean())
    log(f"[bench] {wall_ms:.3f} ms/generation; phases {phase_mean}; P={P_mean:.0f} flips={flips_mean:.0f}")
    pop_timed, gen0 = None, None
    if not args.no_gen0:
        kw_head = dict(M=M, H=H, lam_num=lam_num, lam_den=lam_den, G=G, run_seed=c["run_seed"])
        pop_timed = population_summary(ctx, prob, kw_head, range(Wm, G))
        log(f"[bench] timed populations: {pop_timed[0]} (first timed generation)")
        # ---- generation 0 from random seeds: distinct candidates and passers ---------
        gen0 = gen0_leg(ctx, ubqp, prob, c, lam_num, lam_den, max(3, min(K, 10)))
        log(f"[bench] generation 0 from random seeds: {gen0['ms_per_generation']:.3f} ms "
            f"({gen0['evals_per_s']:.3g} evals/s), phases {gen0['phases_ms']}, P={gen0['passers_per_gen']:.0f} "
            f"flips={gen0['flips_per_gen']:.0f}")

    # ---- the other screening thresholds of the headline workload ----------------------
    lam_sweep = {}
    if not args.no_lam_sweep:
        for ln, ld in ((3, 10), (4, 5)):
            if (ln, ld) == (lam_num, lam_den):
                continue
            rl = ctx.run(prob, M=M, H=H, lam_num=ln, lam_den=ld, G=Wm + K, run_seed=c["run_seed"],
                         flags=ubqp.UBQP_TIMING)
            rl.step(Wm)
            rl.result()
            tl0 = time.perf_counter()
            rl.step(K)
            rr = rl.result()
            tl = (time.perf_counter() - tl0) * 1e3 / K
            rl.close()
            stl = rr["stats"][Wm:]
            lam_sweep[f"{ln}/{ld}"] = dict(ms_per_generation=tl, evals_per_s=M / (tl * 1e-3),
                                           passers_per_gen=float(stl[:, 2].mean()),
                                           flips_per_gen=float(stl[:, 3].mean()))
            log(f"[bench] lambda {ln}/{ld}: {tl:.3f} ms/generation, P={stl[:, 2].mean():.0f} "
                f"flips={stl[:, 3].mean():.0f}")

    # ---- the small and the timing-table configurations end to end ------------------------
    # n=500 (M=1000) and n=2500 (M=65536), 20 generations each from generation 0, with
    # the mean phase times of the generations after the first
    small_runs = {}
    if not args.no_configs:
        for name in ("n500_d0.10_M1000", "n2500_d0.10_M65536"):
            cc = WORKLOADS[name]
            Qc = make_instance(cc["n"], cc["density"], cc["lo"], cc["hi"], cc["inst_seed"])
            pc = ctx.problem(Qc)
            kw = dict(M=cc["M"], H=cc["H"], lam_num=cc["lam"][0], lam_den=cc["lam"][1], G=cc["G"],
                      run_seed=cc["run_seed"], flags=ubqp.UBQP_TIMING)
            ctx.multistart(pc, **dict(kw, G=2))   # warm-up (graph capture, workspaces)
            torch.cuda.synchronize()
            tc0 = time.perf_counter()
            rc = ctx.multistart(pc, **kw)
            torch.cuda.synchronize()
            tc = (time.perf_counter() - tc0) * 1e3
            stc = rc["stats"]
            small_runs[name] = dict(n=cc["n"], M=cc["M"], G=cc["G"], ms_total_call=tc,
                                 ms_total_events=float(rc["gen_ms"][-1]),
                                 ms_per_generation=float(rc["gen_ms"][-1]) / cc["G"],
                                 evals_per_s=cc["M"] * cc["G"] / (tc * 1e-3), best_f=rc["best_f"],
                                 passers_per_gen=float(stc[:, 2].mean()), flips_per_gen=float(stc[:, 3].mean()),
                                 phases_ms_after_gen0={ph: float(rc["phase_ms"][1:, i].mean())
                                                       for i, ph in enumerate(ubqp.PHASES)})
            del pc
            log(f"[bench] {name}: {cc['G']} generations in {tc:.2f} ms ({small_runs[name]['evals_per_s']:.3g} evals/s), "
                f"best f {rc['best_f']}, phases after generation 0 "
                f"{ {k: round(v, 4) for k, v in small_runs[name]['phases_ms_after_gen0'].items()} }")

    # ---- the headline workload with blending diversification -------------------------
    blend = None
    if not args.no_blend:
        rb = ctx.run(prob, M=M, H=H, lam_num=lam_num, lam_den=lam_den, G=Wm + K, run_seed=c["run_seed"],
                     flags=ubqp.UBQP_TIMING | ubqp.UBQP_BLEND)
        rb.step(Wm)
        rb.result()
        tb0 = time.perf_counter()
        rb.step(K)
        rbr = rb.result()
        tb = (time.perf_counter() - tb0) * 1e3 / K
        rb.close()
        stb = rbr["stats"][Wm:]
        blend = dict(ms_per_generation=tb, evals_per_s=M / (tb * 1e-3),
                     phases_ms={name: float(rbr["phase_ms"][Wm:, i].mean()) for i, name in enumerate(ubqp.PHASES)},
                     passers_per_gen=float(stb[:, 2].mean()), flips_per_gen=float(stb[:, 3].mean()),
                     best_f=int(rbr["best_f"]), best_f_glover=int(res["best_f"]), generations=Wm + K)
        log(f"[bench] blending: {tb:.3f} ms/generation, diversify {blend['phases_ms']['diversify']:.4f} ms, "
            f"P={stb[:, 2].mean():.0f} flips={stb[:, 3].mean():.0f}, best f {rbr['best_f']} "
            f"(Glover {res['best_f']}) after {Wm + K} generations")

    # ---- the paper's own loop: one candidate per iteration (Fig. 2) ------------------
    seq = None
    if not args.no_seq:
        seq = sequential_bench(ctx, WORKLOADS, make_instance, prob, Q, c)

    # ---- path relinking of an elite set at the headline size -------------------------
    relink = None
    if not args.no_relink:
        relink = relink_bench(ctx, ubqp, torch, prob, n, M, H, lam_num, lam_den)

    # ---- evaluation alone (the batched exact objective) ------------------------
    X = random_candidates(M, n, 5)
    Xd = torch.from_numpy(X.view(np.int64)).cuda()
    fd = torch.empty(M, dtype=torch.int64, device="cuda")
    for _ in range(3):
        ctx.eval(prob, Xd, fd)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    R = 20
    e0.record(stream)
    for _ in range(R):
        ctx.eval(prob, Xd, fd)
    e1.record(stream)
    torch.cuda.synchronize()
    eval_ms = e0.elapsed_time(e1) / R
    exec_ops, useful_ops = ctx.eval_ops(prob, M)      # executed by the kernel / the dense definition 2 n^2 M
    log(f"[bench] eval alone {eval_ms:.3f} ms: {exec_ops / eval_ms / 1e9:.1f} TOP/s executed "
        f"({exec_ops / eval_ms / 1e9 / INT8_PEAK_TOPS:.3f} of the int8 peak), "
        f"{useful_ops / eval_ms / 1e9:.1f} TOP/s dense-equivalent")
    mfma_meas, read_peaks = None, None
    if not args.no_peaks:
        mfma_meas = ctx.mfma_peak()
        log(f"[bench] int8 MFMA rate sustained on this device (registers only): {mfma_meas:.0f} TOP/s; the "
            f"evaluation executes {exec_ops / eval_ms / 1e9 / mfma_meas:.3f} of it")
        # read bandwidth of the memory levels (streaming kernel): a buffer each XCD's
        # L2 holds, one only the Infinity Cache holds, and HBM streaming
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        read_peaks = {"l2_2MiB": ctx.read_peak(2 << 20, 2 << 20, 4 << 20),
                      "infinity_cache_128MiB": ctx.read_peak(128 << 20, 64 << 10, 1 << 20),
                      "hbm_stream": ctx.read_peak(8 * cus * (2 << 20), 2 << 20, 2 << 20)}
        log(f"[bench] measured read bandwidth (GB/s): {read_peaks}")
    traffic = load_traffic()

    # ---- roofline of the dominant phase ------------------------------------------
    dom = max((k for k in phase_mean if k != "ascent_kernel"), key=phase_mean.get)
    if dom == "eval":
        t_ms = phase_mean["eval"]
        ach = exec_ops / (t_ms * 1e-3) / 1e12
        tr = traffic.get("eval_batched<0,128>")
        roof = dict(kernel="eval_batched<0,128> (int8 MFMA, lower triangle, fused row dot)", bound="mfma",
                    achieved=ach, peak=INT8_PEAK_TOPS, unit="TFLOP/s", frac=ach / INT8_PEAK_TOPS,
                    traffic=tr["gb"] if tr else None, traffic_unit="GB per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
                    algorithmic="int8 matrix-core ops the launch executes (lower triangle by column tiles)",
                    avg_launch_ms=t_ms)
    else:
        # The ascent kernel alone (its launches in a generation, bracketed by stream
        # events on the launch stream).  Per flip and variable the method does one
        # update of Delta and one comparison of the argmax: 2 n int32 operations per
        # flip, all on the vector ALUs (the row of Q it reads, n bytes, comes from L2
        # or the Infinity Cache).  The bound is the vector-ALU issue rate.
        t_ms = phase_mean["ascent_kernel"]
        ops = 2.0 * n * flips_mean
        ach = ops / (t_ms * 1e-3) / 1e12
        row_gb = flips_mean * n / 1e9
        tr = traffic.get("ascent_i8_batched<7>")
        mem = dict(algorithmic_row_gb=row_gb, row_gbs=row_gb / (t_ms * 1e-3),
                   read_peak_gbs_measured=read_peaks)
        if tr and read_peaks:
            beyond = tr["fetch_gb"]
            l2 = max(row_gb - beyond, 0.0)
            t_lb = (l2 / read_peaks["l2_2MiB"] + beyond / read_peaks["infinity_cache_128MiB"]) * 1e3
            mem.update(beyond_l2_gb=beyond, l2_served_gb=l2, lower_bound_ms=t_lb, frac=t_lb / t_ms,
                       note="time the rows need at the measured L2 and Infinity Cache read rates, split as the "
                            "counters split them, against the kernel's time")
        roof = dict(kernel="ascent_i8_batched<7> (steepest 1-flip ascent of every passer)",
                    bound="alu", achieved=ach, peak=VALU_INT32_TOPS, unit="TOP/s (int32 lane-operations)",
                    frac=ach / VALU_INT32_TOPS, traffic=tr["gb"] if tr else None,
                    traffic_unit="GB per launch beyond L2 (calibrated FETCH_SIZE + WRITE_SIZE)",
                    algorithmic="2 n int32 operations per flip (Delta update and argmax comparison) x flips of "
                                "the generation",
                    algorithmic_tops_per_launch=ops / 1e12, avg_launch_ms=t_ms,
                    phase_ms_with_delta_init=phase_mean[dom], flips_per_s=flips_mean / (t_ms * 1e-3),
                    memory=mem,
                    note="peak = 256 CU x 4 SIMD x 16 lanes x 2.4 GHz; the kernel issues about 2.5 vector "
                         "instructions per variable and flip (multiply, multiply-add, half a three-input "
                         "maximum) and each wave's flip chain waits on its row read in between")

    # ---- the paper's Table 1 replica: 1000 random solutions --------------------------
    e1_rep = {}
    if not args.no_e1:
        for nn, dens, seed in ((2500, 0.1, 6001), (5000, 0.5, 6002), (6000, 0.5, 6003), (7000, 0.5, 6004)):
            Qe = (Q if nn == n else make_instance(nn, dens, -100, 100, seed)).astype(np.int8)
            torch.cuda.synchronize()
            tu = time.perf_counter()
            pe = ctx.problem(Qe)                        # upload: copy, device check, plane build
            torch.cuda.synchronize()
            upload_ms = (time.perf_counter() - tu) * 1e3
            Xe = torch.from_numpy(random_candidates(1000, nn, seed).view(np.int64)).cuda()
            fe = torch.empty(1000, dtype=torch.int64, device="cuda")
            ctx.eval(pe, Xe, fe)
            e0.record(stream)
            for _ in range(10):
                ctx.eval(pe, Xe, fe)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 10
            e1_rep[str(nn)] = dict(ms_per_1000=ms, paper_gpu_s=PAPER_TABLE1_S[nn],
                                   speedup_vs_paper_gpu=PAPER_TABLE1_S[nn] * 1e3 / ms,
                                   q_upload_ms=upload_ms, ms_per_1000_with_upload=ms + upload_ms)
            log(f"[bench] 1000 evals n={nn}: {ms:.3f} ms, {ms + upload_ms:.2f} ms with the Q upload "
                f"(paper GTX 780 Ti: {PAPER_TABLE1_S[nn]} s)")
            pe.close()

    # ---- batched form: 64 int16 instances per launch ----------------------------------
    batched = None
    if not args.no_batch:
        batched = batched_bench(ctx, ubqp, torch)

    # ---- serving: Poisson arrivals against the request server -------------------------
    serving = None
    if not args.no_serve:
        serving = serving_bench(ctx, ubqp, torch, R=args.serve_requests, warm=args.serve_warmup, rate=args.serve_rate,
                                max_active=args.serve_active)

    # ---- CPU oracle -----------------------------------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        log(f"[bench] cpu baseline with {threads} threads")
        cpu = cpu_baseline(Q, n, M, P_mean, flips_mean, threads)

    out = {
        "metric": METRIC,
        "value": M * K / (t1 - t0),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": wall_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": f"n={n}, density {c['density']}, coefficients in [-100,100], M={M} candidates "
                               f"per generation (H={H}), lambda={lam_num}/{lam_den}, ascent to a local optimum; "
                               f"one step = one generation (diversify, eval, screen, ascent, select)",
                   "population_note": "after the warm-up every seed is the incumbent (the next-seed rule's fixed "
                                      "point), so a timed generation's candidates are the incumbent's 20 Glover "
                                      "variants, each repeated; 'timed_population' gives the distinct objective "
                                      "values, 'generation0' the rate from random seeds (all distinct)",
                   "n": n, "M": M, "H": H, "lambda": f"{lam_num}/{lam_den}", "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "phases_ms": phase_mean,
        "gen_ms_events": float(gen_ms.mean()),
        "passers_per_gen": P_mean,
        "flips_per_gen": flips_mean,
        "eval_only": {"ms": eval_ms, "evals_per_s": M / (eval_ms * 1e-3),
                      "executed_ops": exec_ops, "executed_tops": exec_ops / eval_ms / 1e9,
                      "frac_int8_peak": exec_ops / eval_ms / 1e9 / INT8_PEAK_TOPS,
                      "dense_equivalent_ops": useful_ops, "dense_equivalent_tops": useful_ops / eval_ms / 1e9,
                      "dense_equivalent_frac_int8_peak": useful_ops / eval_ms / 1e9 / INT8_PEAK_TOPS,
                      "mfma_peak_measured_tops": mfma_meas,
                      "frac_measured_peak_executed": exec_ops / eval_ms / 1e9 / mfma_meas if mfma_meas else None,
                      "traffic_gb_per_launch": (traffic.get("eval_kernel<0,128>") or {}).get("gb"),
                      "algorithmic_gb_per_launch": (M * prob.W * 8 + prob.n_pad * prob.n_pad + 8 * M) / 1e9},
        "read_peaks_gbs": read_peaks,
        "generation0": gen0,
        "timed_population": pop_timed,
        "e1_replica": e1_rep,
        "lambda_sweep": lam_sweep,
        "configs": small_runs,
        "blend": blend,
        "sequential": seq,
        "relink": relink,
        "batched": batched,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
