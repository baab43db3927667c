"""Benchmark of the xyz interaction search on one MI355X.

Headline workload (the largest single-GPU configuration): n = 5000 rows,
p = 10^6 Rademacher columns handed over bit-packed (625 MB), one +-1 response
with 20 planted pairs of exact strength s ~ U[0.15, 0.5], kappa = 0.12.  A
step answers the search at >= 95 % predicted recall (eq. (9)) of the weakest
planted pair above kappa.  The candidate plans are xyz with m in {10, 11, 12}
and L from eq. (15) for that pair, and the exact search of eq. (1) on the FP4
(e2m1) matrix cores (recall 1); each is timed once and the fastest runs the
timed steps.  Inputs are resident in HBM before timing; a search includes
packing Y, row sampling, projection, bucket sort, candidate expansion,
verification, merging and the copy of the result to the host.  Pairs screened
per search = p (p - 1) / 2 (the whole search space, as in the paper's
"interactions screened"); recall is measured against the exact truth.

Prints one JSON line.  Beside the timed steps it reports the genotype-shaped
workload (n = 2000, p = 10^5, five data sets), the continuous workload (sign
and unbiased transforms), the serving stream and the CPU oracle's rate on a
bounded sample (one thread and all threads).  Separate modes: --scaling-law
(Section 5.2), --lasso (Section 5.4), --dense (Section 5.1: dense Gaussian
projections against minimal subsampling), --calibrate-copy (the reference for
the HBM byte counters).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_ALU_TOPS = 256 * 64 * 2.4e9 / 1e12   # 32-bit integer VALU lane-ops/s (256 CUs x 64 lanes x 2.4 GHz)
PEAK_HBM_GBS = 8000.0
PEAK_FP4_TFLOPS = 10100.0                  # dense FP4 matrix-core peak (the exact search runs in e2m1)
PEAK_FP64_TFLOPS = 78.6                    # FP64 vector peak (continuous verification: binary64 FMAs)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def find_kappa(ctx, x, Yd, n, p, target=10_000):
    """kappa such that at most `target` pairs have s/n > kappa: the (target+1)-th
    largest s over all pairs, found with the exact (matrix-core) brute force."""
    k0 = 0.25
    while True:
        r = ctx.bruteforce(x, Yd, k0)
        s = np.sort(r["pairs"]["s"])[::-1]
        if len(s) > target or k0 < -0.5:
            break
        k0 -= 0.05
    kappa = float(s[target]) / n
    exact = ctx.bruteforce(x, Yd, kappa)["pairs"]
    return kappa, exact


def measured_traffic(kernel, workload, m, L, share=1.0):
    """HBM bytes of `kernel` in one search (m, L) of `workload`, times `share`,
    from the committed counter profile of that search (FETCH_SIZE and
    WRITE_SIZE summed over the kernel's dispatches, scaled by what the counters
    read for a plain device copy); None when the kernel source changed since
    the counters were taken, no profiled search has this plan, or there is no
    profile."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", f"traffic_{workload}.json")) as f:
            t = json.load(f)
        with open(os.path.join(ROOT, "paper_1610_05108_amd", "csrc", "xyz_kernels.hip"), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()[:16]
    except OSError:
        return None
    srch = [q for q in t.get("searches", []) if q.get("m") == m and q.get("L") == L]
    if sha != t.get("kernels_source_sha256_16") or not srch:
        return None
    k = srch[0].get("kernels", {}).get(kernel)
    if not k:
        return None
    if k.get("fetch_kib") is None or k.get("write_kib") is None:
        return None
    return (k["fetch_kib"] * t["fetch_scale"] + k["write_kib"] * t["write_scale"]) * 1024.0 * share


def gamma_of(stat):
    return 0.5 * (1.0 + stat)


def host_threads():
    """Threads for the CPU baseline: this process's CPU share, at most 16."""
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


def unpack_bits(bits, n):
    """(p, ceil(n/64)) uint64 column bits -> (p, n) int8 +-1 (bit 1 = -1)."""
    u8 = np.ascontiguousarray(bits).view(np.uint8)
    b = np.unpackbits(u8, axis=1, bitorder="little")[:, :n]
    return (1 - 2 * b.astype(np.int8)).astype(np.int8)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plan", choices=["auto", "brute", "xyz"], default="auto",
                    help="auto: time every plan once and keep the fastest")
    ap.add_argument("--ms", type=str, default="10,11,12", help="m of the xyz plans (L from eq. (15))")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true", help="search with the default launch shapes (no xyz_autotune)")
    ap.add_argument("--tune-cache", type=str, default=os.path.join(tempfile.gettempdir(), "xyz_tune_cache.txt"),
                    help="cache file of tuned launch shapes")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--no-genotype", action="store_true", help="skip the genotype-shaped workload")
    ap.add_argument("--no-continuous", action="store_true", help="skip the continuous workload")
    ap.add_argument("--seeds", type=int, default=5, help="data sets of the genotype-shaped workload")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-fresh", type=int, default=32)
    ap.add_argument("--serve-workers", type=int, default=2)
    ap.add_argument("--scaling-law", action="store_true",
                    help="only run the scaling experiment of Section 5.2 (time to discovery against p)")
    ap.add_argument("--scaling-p", type=str, default="10000,30000,100000,300000,1000000")
    ap.add_argument("--scaling-gamma", type=str, default="0.7,0.8,0.9")
    ap.add_argument("--scaling-n", type=int, default=4000)
    ap.add_argument("--scaling-sims", type=int, default=40)
    ap.add_argument("--lasso", action="store_true",
                    help="only run the regression experiment of Section 5.4 (Lasso with all interactions)")
    ap.add_argument("--lasso-p", type=str, default="250,500,750,1000")
    ap.add_argument("--lasso-settings", type=str, default="1,2,3")
    ap.add_argument("--dense", action="store_true",
                    help="only Section 5.1: dense Gaussian projections vs minimal subsampling")
    ap.add_argument("--dense-p", type=str, default="1000,10000,100000,1000000")
    ap.add_argument("--profile-search", action="store_true",
                    help="only the headline data, its exact truth and, per m of --ms, one xyz search (L for 95%% "
                         "recall, default launch shapes) between two marker fill kernels, after a warm-up search: "
                         "the run the HBM byte counters are taken on")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB device buffer 3 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 1 << 30, "copies": 3}), flush=True)
        return
    if args.scaling_law:
        import paper_1610_05108_amd as xyz
        ctx = xyz.Context(0)
        out = scaling_law_leg(ctx, args.scaling_n, [int(v) for v in args.scaling_p.split(",")],
                              [float(v) for v in args.scaling_gamma.split(",")], args.scaling_sims)
        print(json.dumps(out), flush=True)
        return
    if args.dense:
        import paper_1610_05108_amd as xyz
        ctx = xyz.Context(0)
        print(json.dumps(dense_leg(ctx, [int(v) for v in args.dense_p.split(",")])), flush=True)
        return
    if args.lasso:
        import paper_1610_05108_amd as xyz
        ctx = xyz.Context(0)
        print(json.dumps(lasso_leg(ctx, [int(v) for v in args.lasso_p.split(",")],
                                   settings=[int(v) for v in args.lasso_settings.split(",")])), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the search shards over repetitions "
              "and responses; this benchmark measures one GPU.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synthgen
    import paper_1610_05108_amd as xyz

    ctx = xyz.Context(0)
    # ---- the headline workload, resident in HBM
    t0 = time.time()
    d = synthgen.config3(seed=0)
    n, p = d.n, d.p
    kappa = d.params["kappa"]
    x = xyz.xyz_x_create(ctx.h, d.bits, n=n)
    Y = torch.from_numpy(d.Y).cuda()
    torch.cuda.synchronize()
    log(f"data ready ({time.time() - t0:.1f}s): n={n} p={p}, {len(d.planted)} planted pairs, kappa={kappa}")
    truth = ctx.bruteforce(x, Y, kappa)["pairs"]
    ex = {(int(a), int(b)): int(sv) for a, b, sv in zip(truth["j"], truth["k"], truth["s"])}
    above = [pq for pq in d.planted if pq in ex]
    gamma_w = min(gamma_of(ex[pq] / n) for pq in above)
    log(f"exact truth: {len(ex)} pairs above kappa, {len(above)} of them planted; weakest planted gamma {gamma_w:.4f}")

    def run(plan, profile=False):
        if plan[0] == "brute":
            return ctx.bruteforce(x, Y, kappa, profile=profile)
        return ctx.search(x, Y, m=plan[1], L=plan[2], kappa=kappa, seed=1, profile=profile)

    def recall_of(res):
        got = {(int(a), int(b)) for a, b in zip(res["pairs"]["j"], res["pairs"]["k"])}
        return sum(1 for pq in above if pq in got) / len(above), len(got & set(ex)) / max(len(ex), 1)

    ms_list = [int(v) for v in args.ms.split(",") if v]
    xyz_plans = [("xyz", m, xyz.xyz_L_for(0.95, gamma_w ** m)) for m in ms_list]
    if args.profile_search:
        # per plan: a warm-up search (workspaces grow, the first chunk may be redone), a fill kernel
        # that marks where the counted search starts in the profile, the counted search, and a
        # fill kernel that marks its end
        def marker():
            torch.cuda.synchronize()
            torch.full((256,), 7, dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()
        for pl in xyz_plans:
            ctx.search(x, Y, m=pl[1], L=pl[2], kappa=kappa, seed=1)
            marker()
            r = ctx.search(x, Y, m=pl[1], L=pl[2], kappa=kappa, seed=1)
            marker()
            tm = r["timing"]
            print(json.dumps({"profile_search": {"m": pl[1], "L": pl[2], "seed": 1, "n": n, "p": p,
                                                 "candidates": tm["candidates"],
                                                 "big_candidates": tm["big_candidates"],
                                                 "big_launches": tm["big_launches"], "pairs": int(len(r["pairs"]))}}),
                  flush=True)
        return
    plans = {"auto": [("brute", 0, 1)] + xyz_plans, "brute": [("brute", 0, 1)], "xyz": xyz_plans}[args.plan]
    table = []
    for pl in plans:
        tuning = None
        if pl[0] == "xyz" and not args.no_tune:
            # launch shapes timed once per search shape (untimed setup; reused from the cache file)
            tuning = ctx.autotune(x, Y, m=pl[1], L=pl[2], kappa=kappa, seed=1, cache_path=args.tune_cache)
            log(f"tuning {pl}: {tuning}")
        run(pl)
        torch.cuda.synchronize()
        tt = time.perf_counter()
        r = run(pl)
        torch.cuda.synchronize()
        dt = time.perf_counter() - tt
        rec, trec = recall_of(r)
        table.append(dict(kind=pl[0], m=pl[1], L=pl[2], ms_per_search=dt * 1e3, planted_recall=rec,
                          predicted_recall_min=1.0 if pl[0] == "brute" else xyz.xyz_eta(gamma_w, pl[1], pl[2]),
                          tuning=tuning))
        log(f"plan {pl}: {dt * 1e3:.1f} ms, planted recall {rec:.3f}")
    best = min(range(len(plans)), key=lambda q: table[q]["ms_per_search"])
    plan = plans[best]
    log(f"running {plan}")

    for _ in range(args.warmup):
        run(plan)
    torch.cuda.synchronize()
    tt = time.perf_counter()
    out = None
    for _ in range(args.steps):
        out = run(plan)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - tt) * 1e3 / args.steps
    recall, truth_recall = recall_of(out)
    pairs_per_search = p * (p - 1) / 2
    value = pairs_per_search / (ms_per_step * 1e-3)

    # profiled pass: HIP events recorded by the library on the stream the kernels run on
    prof = run(plan, profile=True)
    tm = prof["timing"]
    workload_id = f"rademacher_n{n}_p{p}"
    if plan[0] == "brute":
        flops = 2.0 * n * tm["candidates"]
        k_ms, k_launch = tm["brute_ms"], max(tm["verify_launches"], 1)
        dom = dict(kernel="k_brute", bound="mfma", unit="TFLOP/s", peak=PEAK_FP4_TFLOPS)
        hashr = sortr = None
    else:
        m, L = plan[1], plan[2]
        flops = 2.0 * n * tm["big_candidates"]        # the n-row products of the big tiles' candidates
        k_ms, k_launch = tm["big_ms"], max(tm["big_launches"], 1)
        dom = dict(kernel="k_verify_lds", bound="mfma", unit="TFLOP/s", peak=PEAK_FP4_TFLOPS)
        hb = L * (m * p / 8.0 + 4.0 * p)              # rows of the bit matrix read, keys written
        sb = L * (8.0 * p + 4.0 * ((1 << m) + 1))     # keys read, permutation and bucket offsets written
        hashr = dict(kernel="k_hash", bound="hbm", unit="GB/s", peak=PEAK_HBM_GBS,
                     achieved=hb / (tm["hash_ms"] * 1e-3) / 1e9, bytes_per_search=hb, ms_per_search=tm["hash_ms"])
        hashr["frac"] = hashr["achieved"] / PEAK_HBM_GBS
        hashr["traffic"] = measured_traffic("k_hash", workload_id, m, L)
        sortr = dict(kernel="k_bucket", bound="hbm", unit="GB/s", peak=PEAK_HBM_GBS,
                     achieved=sb / (tm["bucket_ms"] * 1e-3) / 1e9, bytes_per_search=sb, ms_per_search=tm["bucket_ms"])
        sortr["frac"] = sortr["achieved"] / PEAK_HBM_GBS
        sortr["traffic"] = measured_traffic("k_bucket", workload_id, m, L)
    achieved = flops / k_launch / (k_ms / k_launch * 1e-3) / 1e12
    traffic = None
    if plan[0] != "brute":
        traffic = measured_traffic(dom["kernel"], workload_id, plan[1], plan[2], 1.0 / k_launch)
    dom.update(achieved=achieved, frac=achieved / dom["peak"], work_per_launch=flops / k_launch,
               avg_launch_ms=k_ms / k_launch, launches=k_launch, traffic=traffic)
    stages = {k: round(tm[k], 3) for k in ("pack_ms", "sample_ms", "hash_ms", "bucket_ms", "tiles_ms", "verify_ms",
                                           "big_ms", "dedup_ms", "brute_ms", "total_ms")}
    stages["candidates"] = tm["candidates"]
    stages["big_candidates"] = tm["big_candidates"]
    literal = None
    if plan[0] != "brute" or args.plan == "auto":
        # the workload's literal parameters (m = 14, L = 500): a parity run, recall as it comes
        lit = ("xyz", d.params["m"], d.params["L"])
        run(lit)
        torch.cuda.synchronize()
        tt = time.perf_counter()
        r = run(lit)
        torch.cuda.synchronize()
        rec, _ = recall_of(r)
        g = [gamma_of(ex[pq] / n) for pq in above]
        literal = dict(m=lit[1], L=lit[2], ms_per_search=(time.perf_counter() - tt) * 1e3, planted_recall=rec,
                       predicted_recall_mean=float(np.mean([xyz.xyz_eta(gg, lit[1], lit[2]) for gg in g])))
    xyz.xyz_x_destroy(x)
    del Y
    torch.cuda.synchronize()

    genotype = None
    if not args.no_genotype:
        genotype = genotype_leg(ctx, args.seeds)
        log(f"genotype: {genotype}")
    continuous = None
    if not args.no_continuous:
        continuous = continuous_leg(ctx)
        log(f"continuous: {continuous}")
    serving = None
    if not args.no_serve:
        serving = serve_leg(ctx, args.serve_requests, args.serve_fresh, args.serve_workers, seq_sample=32)
        log(f"serving: {serving}")
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(d, plan, kappa)
        log(f"cpu: {cpu}")

    line = {
        "metric": "interaction pairs screened/s at >=95% planted recall; p50/p99 request latency",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp4-e2m1/fp32-acc",
        "data": "synthetic",
        "config": {"workload": f"large binary: Rademacher bits n={n} p={p}, 20 planted pairs of strength "
                               f"U[0.15,0.5], kappa={kappa}, one search per step at >=95% predicted recall "
                               f"of the weakest planted pair",
                   "searches_per_step": 1, "plan": plan[0], "m": plan[1], "L": plan[2], "kappa": kappa},
        "recall": {"planted_predicted_min": table[best]["predicted_recall_min"], "planted_measured": recall,
                   "planted_pairs_above_kappa": len(above), "weakest_planted_gamma": gamma_w,
                   "truth_set_recall": truth_recall, "truth_set_size": len(ex)},
        "plans_ms_per_search": table,
        "stages_ms_per_search": stages,
        "roofline": dom,
        "roofline_hash": hashr,
        "roofline_sort": sortr,
        "literal_parameters": literal,
        "cpu_baseline": cpu,
        "serving": serving,
        "genotype": genotype,
        "continuous": continuous,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def genotype_leg(ctx, seeds, n=2000, p=100_000):
    """The genotype-shaped workload (stands in for the SNP data of Section 5.3):
    `seeds` data sets of n = 2000, p = 10^5, minor-allele frequencies U[0.05,
    0.5], +-1 responses from a logistic model with 10 planted pairs; kappa per
    data set so that about 1e4 pairs exceed it (found exactly on the GPU).  Each
    data set is searched at >= 95 % predicted recall of the weakest planted pair
    above kappa; the plans are the exact search and xyz with m in {8, 10, 12}
    (L from eq. (15)), each timed once on data set 0, and the fastest answers all
    data sets; pairs/s over the data sets, recall against the exact truth."""
    import torch
    import synthgen
    import paper_1610_05108_amd as xyz
    data = []
    for seed in range(seeds):
        d = synthgen.config2(seed=seed, n=n, p=p)
        x = ctx.x_create(torch.from_numpy(d.XT).cuda())
        Yd = torch.from_numpy(d.Y).cuda()
        kappa, exact = find_kappa(ctx, x, Yd, n, p)
        ex = {(int(a), int(b)): int(sv) for a, b, sv in zip(exact["j"], exact["k"], exact["s"])}
        data.append(dict(seed=seed, x=x, Y=Yd, kappa=kappa, ex=ex, planted=[pq for pq in d.planted if pq in ex]))
    gamma_w = min(gamma_of(dd["ex"][pq] / n) for dd in data for pq in dd["planted"])

    def run(plan, dd):
        if plan[0] == "brute":
            return ctx.bruteforce(dd["x"], dd["Y"], dd["kappa"])
        return ctx.search(dd["x"], dd["Y"], m=plan[1], L=plan[2], kappa=dd["kappa"], seed=1000 + dd["seed"])

    plans = [("brute", 0, 1)] + [("xyz", m, xyz.xyz_L_for(0.95, gamma_w ** m)) for m in (8, 10, 12)]
    table = []
    for pl in plans:
        run(pl, data[0])
        torch.cuda.synchronize()
        tt = time.perf_counter()
        run(pl, data[0])
        torch.cuda.synchronize()
        table.append(dict(kind=pl[0], m=pl[1], L=pl[2], ms_per_search=(time.perf_counter() - tt) * 1e3))
    plan = plans[min(range(len(plans)), key=lambda q: table[q]["ms_per_search"])]
    torch.cuda.synchronize()
    tt = time.perf_counter()
    outs = [run(plan, dd) for dd in data]
    torch.cuda.synchronize()
    dt = time.perf_counter() - tt
    found = tot = 0
    for dd, o in zip(data, outs):
        got = {(int(a), int(b)) for a, b in zip(o["pairs"]["j"], o["pairs"]["k"])}
        found += sum(1 for pq in dd["planted"] if pq in got)
        tot += len(dd["planted"])
    for dd in data:
        ctx.x_destroy(dd["x"])
    return {"workload": f"genotype-shaped binary n={n} p={p}, {seeds} data sets, kappa for 1e4 survivors",
            "plan": plan, "plans_ms_per_search": table, "weakest_planted_gamma": gamma_w,
            "ms_per_search": dt * 1e3 / len(data), "pairs_per_s": len(data) * p * (p - 1) / 2 / dt,
            "planted_found": found, "planted_above_kappa": tot}


def pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def serve_leg(ctx, count, fresh_count, workers, seq_sample):
    """The serving workload: a shared genotype-shaped X (n=2000, p=200,000)
    resident on the GPU; `count` +-1 responses arrive as a Poisson stream at
    50/s (1-3 planted pairs of strength 0.2-0.5, L from {50, 200, 500},
    kappa 0.15), mixed with `fresh_count` requests on fresh Rademacher data
    sets (n=1000, p from {1e4, 1e5, 5e5}, handed over bit-packed, made
    resident on arrival and freed after).

    Every request is submitted with XYZ_ROUTE: the library's router answers it
    with xyz at the request's L (m from eq. (9) at gamma = (1 + kappa)/2, rows
    from the shared seed, so that compatible requests share a pass) or with the
    exact search, whichever its cost model predicts faster.  Latency = arrival
    to result.  The stream is replayed twice: at its arrival times (p50/p99
    latency, pairs screened per second of the stream) and, for the shared-X
    requests, all at once (the server's capacity: pairs screened per second
    with the queue full), beside the same requests answered one at a time by
    the reported routes."""
    import threading
    import synthgen
    import paper_1610_05108_amd as xyz
    t0 = time.time()
    XT, _ = synthgen.config5_shared(seed=0)
    ps, ns = XT.shape
    x = xyz.xyz_x_create(ctx.h, XT)
    reqs = synthgen.config5_requests(XT, count=count, seed=0, rate=50.0)
    fresh = synthgen.config5_fresh_bits(count=fresh_count, seed=0) if fresh_count else []
    log(f"serving data ready ({time.time() - t0:.1f}s): {len(reqs)} shared-X requests, {len(fresh)} fresh")

    def replay(realtime, with_fresh=True):
        events = [dict(kind="shared", **q) for q in reqs] + ([dict(kind="fresh", **q) for q in fresh] if with_fresh else [])
        events.sort(key=lambda e: e["t"])
        srv = xyz.xyz_serve_start(ctx.h, 0, workers=workers, max_batch=64)
        pending, done = {}, {}
        lock = threading.Lock()
        finished = threading.Event()

        def collector():
            while not finished.is_set() or pending:
                with lock:
                    items = list(pending.items())
                for tk, e in items:
                    try:
                        o = xyz.xyz_serve_poll(srv, tk)
                    except xyz.XyzError as err:          # failed request: report it, keep collecting
                        e["error"] = str(err)
                        o = {"pairs": np.zeros(0, dtype=[("j", "i4"), ("k", "i4")]), "route": {"method": -1}}
                    if o is not None:
                        e["t_done"] = time.perf_counter()
                        e["out"] = o
                        with lock:
                            del pending[tk]
                            done[tk] = e
                time.sleep(0.0005)

        th = threading.Thread(target=collector)
        th.start()
        start = time.perf_counter()
        try:
            for e in events:
                if realtime:
                    wait = start + e["t"] - time.perf_counter()
                    if wait > 0:
                        time.sleep(wait)
                e["t_arr"] = start + e["t"] if realtime else time.perf_counter()
                if e["kind"] == "fresh":
                    e["x"] = xyz.xyz_x_create(ctx.h, e["bits"], n=e["n"])
                    e.update(p=e["bits"].shape[0], xh=e["x"])
                else:
                    e.update(p=ps, n=ns, xh=x)
                tk = xyz.xyz_serve_submit(srv, e["xh"], e["Y"], L=e["L"], kappa=e["kappa"], route=True)
                with lock:
                    pending[tk] = e
        finally:
            finished.set()
            th.join()
            st = xyz.xyz_serve_stats_get(srv)
            xyz.xyz_serve_stop(srv)
        end = max(e["t_done"] for e in events)
        for e in events:
            if "x" in e:
                xyz.xyz_x_destroy(e.pop("x"))
        lat = [(e["t_done"] - e["t_arr"]) * 1e3 for e in events]
        screened = sum(e["p"] * (e["p"] - 1) / 2 for e in events)
        routes = {"xyz": sum(1 for e in events if e["out"]["route"]["method"] == xyz.XYZ_PLAN_XYZ),
                  "exact": sum(1 for e in events if e["out"]["route"]["method"] == xyz.XYZ_PLAN_BRUTE)}
        found = tot = 0
        for e in events:
            got = {(int(a), int(b)) for a, b in zip(e["out"]["pairs"]["j"], e["out"]["pairs"]["k"])}
            for pq in e["planted"]:
                tot += 1
                found += pq in got
        return events, dict(p50_ms=pct(lat, 50), p99_ms=pct(lat, 99), max_ms=max(lat),
                            server_p50_ms=st["p50_ms"], server_p99_ms=st["p99_ms"], batches=st["batches"],
                            max_batch=st["max_batch"], wall_s=end - start, pairs_screened_per_s=screened / (end - start),
                            routes=routes, failed=sum(1 for e in events if "error" in e), planted_found=found,
                            planted_total=tot)

    ev_rt, realtime = replay(True)
    ev_b, burst = replay(False, with_fresh=False)
    # the shared-X requests one at a time, without the server, by the routes the server reported
    seq = [e for e in ev_b if e["kind"] == "shared"][:seq_sample]
    ts = time.perf_counter()
    for e in seq:
        rt = e["out"]["route"]
        if rt["method"] == xyz.XYZ_PLAN_BRUTE:
            ctx.bruteforce(x, e["Y"], e["kappa"])
        else:
            ctx.search(x, e["Y"], m=rt["m"], L=rt["L"], kappa=e["kappa"], seed=rt["seed"])
    t_seq = time.perf_counter() - ts
    xyz.xyz_x_destroy(x)
    seq_rate = sum(ps * (ps - 1) / 2 for _ in seq) / t_seq if seq else None
    return {
        "workload": f"shared genotype X n={ns} p={ps} resident; {len(reqs)} +-1 requests at 50/s "
                    f"(L in {{50,200,500}}, kappa 0.15) + {len(fresh)} fresh Rademacher data sets "
                    f"(n=1000, p in {{1e4,1e5,5e5}}, bit-packed); routed by the library (XYZ_ROUTE)",
        "requests": len(ev_rt), "workers": workers,
        "realtime": realtime, "burst": burst,
        "sequential_pairs_per_s": seq_rate, "sequential_sample": len(seq),
        "burst_over_sequential": burst["pairs_screened_per_s"] / seq_rate if seq_rate else None,
    }


def scaling_law_leg(ctx, n, ps, gammas, sims, gamma0=0.55):
    """Section 5.2: Rademacher X (n x p), one strong pair (columns 0 and 1) of
    strength gamma, M chosen so that p^(-1/M) is close to gamma0 (0.55: above the
    bulk of the strengths, which sit near 1/2), and the time until the pair is
    found, averaged over `sims` row-sampling seeds.  Repetitions run in chunks
    until the pair appears; its first repetition l* gives (l* + 1) repetitions
    to discovery, whose time is (l* + 1) x the measured GPU time per repetition
    and whose work is the operation count of the complexity bound (terms (ii)
    to (iv): M p + p log2 p + n |E_l| per repetition, |E_l| measured).  Theorem 2
    predicts both to grow as p^(1 + log gamma / log gamma0); the fitted slopes of
    log time and log work against log p are reported beside that exponent, over
    all p and over p >= 1e5 (where fixed per-call costs no longer dominate the
    time).  The bound counts a repetition's candidate set as if the bulk of the
    strengths sat at gamma0, i.e. of order p pairs; with the bulk at 1/2 it holds
    about p^2 2^-M pairs, which gives the sharper exponent
    2 - log 2 / log(1/gamma0) + log gamma / log gamma0 ("predicted_bulk_half").
    Expected repetitions to discovery: 1 / gamma^M (eq. (9) with L = 1).  Every
    (p, gamma, simulation) draws its rows with a seed of its own."""
    import torch
    import synthgen
    import paper_1610_05108_amd as xyz
    pts = []
    for p in ps:
        t0 = time.time()
        bits = synthgen.scaling_x(n, p, seed=p)
        x = xyz.xyz_x_create(ctx.h, bits, n=n)
        M = max(1, int(round(math.log(p) / math.log(1.0 / gamma0))))
        log(f"scaling: p={p} n={n} M={M} data {time.time() - t0:.1f}s")
        for g in gammas:
            agree = int(round(g * n))
            gg = agree / n
            Y = torch.from_numpy(synthgen.scaling_y(bits, n, agree, seed=1)).cuda()
            q = gg ** M
            chunk = int(min(4096, max(4, math.ceil(0.5 / q))))
            kappa = (2 * gg - 1) / 2           # half the pair's s/n: far above the null pairs
            reps, ms, work, cands = [], [], [], []
            t1 = time.time()
            for sim in range(sims):
                off, tot_ms, tot_reps, cand_before, found = 0, 0.0, 0, 0, None
                while found is None and off < 200 * math.ceil(1 / q):
                    seed = (p * 7919 + agree * 104729 + sim * 15485863) % (1 << 31)
                    r = ctx.search(x, Y, m=M, L=chunk, kappa=kappa, seed=seed, rep_offset=off, profile=True)
                    tot_ms += r["timing"]["total_ms"]
                    tot_reps += chunk
                    pr = r["pairs"]
                    hit = (pr["j"] == 0) & (pr["k"] == 1)
                    cand = r["reps"]["candidates"].astype(np.int64)
                    if hit.any():
                        found = int(pr["first_rep"][hit][0])
                        cand_before += int(cand[:found - off + 1].sum())
                    else:
                        cand_before += int(cand.sum())
                        off += chunk
                if found is None:
                    continue
                nrep = found + 1
                reps.append(nrep)
                ms.append(nrep * tot_ms / tot_reps)
                cands.append(cand_before / nrep)
                work.append(nrep * (M * p + p * math.log2(p)) + n * cand_before)
            pt = {"p": p, "gamma": gg, "M": M, "gamma0": p ** (-1.0 / M), "sims": len(reps),
                  "mean_reps": float(np.mean(reps)), "expected_reps": 1.0 / q,
                  "mean_ms": float(np.mean(ms)), "mean_work": float(np.mean(work)),
                  "candidates_per_rep": float(np.mean(cands))}
            log(f"  gamma={gg:.3f}: {pt['mean_reps']:.1f} reps (expected {pt['expected_reps']:.1f}), "
                f"{pt['mean_ms']:.2f} ms, work {pt['mean_work']:.3g}, {time.time() - t1:.1f}s")
            pts.append(pt)
        xyz.xyz_x_destroy(x)
    fits = {}
    for g in sorted({pt["gamma"] for pt in pts}):
        f = {"predicted_bound": 1.0 + math.log(g) / math.log(gamma0),
             "predicted_bulk_half": 2.0 - math.log(2) / math.log(1 / gamma0) + math.log(g) / math.log(gamma0)}
        for tag, lo in (("", 0), ("_large_p", 100_000)):
            sel = [pt for pt in pts if pt["gamma"] == g and pt["p"] >= lo]
            if len(sel) < 2:
                continue
            lp = np.log([pt["p"] for pt in sel])
            f["time_slope" + tag] = float(np.polyfit(lp, np.log([pt["mean_ms"] for pt in sel]), 1)[0])
            f["work_slope" + tag] = float(np.polyfit(lp, np.log([pt["mean_work"] for pt in sel]), 1)[0])
        fits[f"{g:.3f}"] = f
    return {"experiment": "time to discovery against p (Section 5.2, Theorem 2)", "n": n, "gamma0": gamma0,
            "data": "synthetic Rademacher, one pair of strength gamma", "points": pts, "fits": fits}


def continuous_leg(ctx):
    """The continuous workload (X ~ N(0,1) float32, n=1000, p=200,000, real Y with
    five planted pairs and ten main effects) at its configured parameters (m=12,
    L=300, kappa=0.5; signs of X hashed, |Y|-weighted rows), each search timed on
    its second run, and the same search with the unbiased transform of Section
    3.2 (XYZ_UNBIASED).  Recall: planted pairs reported among those whose value
    exceeds kappa (values from a plain float64 product on the device).  Roofline
    of the verification (k_verify_real): candidate pairs x n multiply-adds in
    binary64 over the verification time, against the FP64 vector peak."""
    import torch
    import synthgen
    d = synthgen.config4(seed=0)
    XT = torch.from_numpy(d.XT).cuda()
    x = ctx.x_create(XT)
    Y = torch.from_numpy(d.Y).cuda()
    m, L, kappa = 12, 300, 0.5
    Yd = Y.double()
    vals = {pq: float((Yd * XT[pq[0]].double() * XT[pq[1]].double()).sum()) for pq in d.planted}
    above = [pq for pq in d.planted if vals[pq] / d.n > kappa]
    out = {"workload": f"continuous X n={d.n} p={d.p}, real Y, {len(d.planted)} planted pairs, m={m} L={L} "
                       f"kappa={kappa}", "planted_above_kappa": len(above)}
    for name, unb in (("sign", False), ("unbiased", True)):
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.search(x, Y, m=m, L=L, kappa=kappa, seed=rep, unbiased=unb, profile=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        pr = r["pairs"]
        got = set(zip(pr["j"].tolist(), pr["k"].tolist()))
        tm = r["timing"]
        flops = 2.0 * tm["candidates"] * d.n
        out[name] = {"ms": dt * 1e3, "verify_ms": tm["verify_ms"], "hash_ms": tm["hash_ms"],
                     "candidates": tm["candidates"], "planted_found": sum(1 for pq in above if pq in got),
                     "verify_roofline": {"kernel": "k_verify_real", "bound": "fp64", "unit": "TFLOP/s",
                                         "achieved": flops / (tm["verify_ms"] * 1e-3) / 1e12,
                                         "peak": PEAK_FP64_TFLOPS,
                                         "frac": flops / (tm["verify_ms"] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}}
    ctx.x_destroy(x)
    return out


def dense_leg(ctx, ps, n=1000, gammas=(0.7, 0.8, 0.9), per=300, target_hits=40, max_reps=20000):
    """Section 5.1 on the GPU: dense Gaussian projections (Algorithm 1,
    xyz_dense_search, tau = xyz_tau_dense for a mean |E_1| of p ordered pairs
    when every strength is 1/2) against minimal subsampling (Algorithm 2,
    xyz_search, M = ceil(log2 p)), on +-1 data with `per` planted pairs of each
    strength in `gammas` against one Y (n = 1000 as in Section 5.1).  A
    repetition discovers a pair when its candidates hold it: for dense
    projections either orientation, predicted 1 - (1 - eta_dense)^2; for
    minimal subsampling E_l is symmetric and the rate is gamma^M.  Reports the
    measured and predicted rates, candidates per repetition, GPU time per
    repetition (warm, whole call / L) and the time to discovery, time per
    repetition / rate."""
    import torch
    import synthgen
    import paper_1610_05108_amd as xyz
    out = []
    for p in ps:
        per_p = min(per, p // (4 * len(gammas)))         # planted pairs use at most half of the columns
        XT, Y, pairs = synthgen.strength_pairs(n, p, gammas, per_p, seed=p)
        x = ctx.x_create(XT)
        kappa = 2.0 * min(gammas) - 1.0 - 0.05        # planted pairs pass; random pairs are 11 sd below
        M = int(math.ceil(math.log2(p) - 1e-9))
        g0 = min(gammas)
        row = {"p": p, "n": n, "M": M, "pairs_per_strength": per_p}

        def rates(res, L):
            hits = {(int(a), int(b)): int(h) for a, b, h in zip(res["pairs"]["j"], res["pairs"]["k"],
                                                                   res["pairs"]["hits"])}
            return {str(g): sum(hits.get((j, k), 0) for j, k, gg in pairs if gg == g) / (per_p * L) for g in gammas}

        # dense Gaussian projections
        rate0 = 1.0 - (1.0 - xyz.xyz_eta_dense(g0, p)) ** 2
        L = int(min(max_reps, max(16, math.ceil(target_hits / (per_p * rate0)))))
        R, sd = synthgen.gaussian_projections(n, L, seed=p + 1)
        tau = int(round(xyz.xyz_tau_dense(p, n, sd)))
        ctx.dense_search(x, Y, R[:8], tau, kappa)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.dense_search(x, Y, R, tau, kappa)
        dt = time.perf_counter() - t0
        meas = rates(res, L)
        row["dense"] = {"L": L, "tau": tau, "sd": sd, "ms_per_rep": 1e3 * dt / L,
                        "candidates_per_rep": float(res["reps"]["candidates"].mean()),
                        "rate": meas,
                        "rate_predicted": {str(g): 1.0 - (1.0 - xyz.xyz_eta_dense(g, p)) ** 2 for g in gammas}}
        # minimal subsampling
        L = int(min(max_reps, max(16, math.ceil(target_hits / (per_p * g0 ** M)))))
        ctx.search(x, Y, m=M, L=min(L, 8), kappa=kappa, seed=5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.search(x, Y, m=M, L=L, kappa=kappa, seed=7)
        dt = time.perf_counter() - t0
        row["minimal"] = {"L": L, "ms_per_rep": 1e3 * dt / L,
                          "candidates_per_rep": float(res["reps"]["candidates"].mean()),
                          "rate": rates(res, L), "rate_predicted": {str(g): g ** M for g in gammas}}
        for key in ("dense", "minimal"):
            e = row[key]
            e["ms_to_discovery"] = {g: (e["ms_per_rep"] / r if r > 0 else None) for g, r in e["rate"].items()}
        log(f"dense vs minimal: {row}")
        out.append(row)
        ctx.x_destroy(x)
    return {"experiment": "dense Gaussian projections vs minimal subsampling at equal budget (Section 5.1)",
            "data": "synthetic +-1, planted pairs of exact strength", "points": out}


def lasso_leg(ctx, ps, n=1000, settings=(1, 2, 3), nlam=12):
    """Section 5.4 (settings 1, 2 and 3): the Lasso path over all main effects and
    interactions (Algorithm 3) on a grid of `nlam` lambdas from lambda_max (the
    largest main-effect gradient) down to lambda_max / 50, with the interaction
    KKT check done by (a) the xyz search, L = sqrt(p) as in Section 5.4 and
    m = ceil(log2 p), and (b) the exhaustive check of all pairs on the GPU (m = 0:
    every pair is a candidate).  Reports the wall time of each path and how many
    of the 10 true interactions and 20 main effects the final model holds."""
    import torch
    import synthgen
    from paper_1610_05108_amd.lasso import lasso_interactions, xyz_screen
    out = []
    for setting in settings:
        for p in ps:
            X, Y, mains, inters = synthgen.lasso_setting(n, p, setting, seed=p)
            x = ctx.x_create(np.ascontiguousarray(X.T))
            Xc = X.astype(np.float64) - X.mean(0)
            lam_max = float(np.abs(Xc.T @ (Y - Y.mean())).max() / n)
            lambdas = lam_max * np.logspace(0, -math.log10(50), nlam)
            row = {"setting": setting, "p": p, "n": n}
            for name, screen in (("xyz", xyz_screen(ctx, x, m=int(math.ceil(math.log2(p))),
                                                    L=int(math.ceil(math.sqrt(p))), seed=1)),
                                 ("exhaustive", xyz_screen(ctx, x, m=0, L=1))):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                path = lasso_interactions(X, Y, lambdas, screen)
                dt = time.perf_counter() - t0
                row[name] = {"s": dt, "inter_found": sum(1 for pq in inters if pq in path.inter[-1]),
                             "main_found": sum(1 for j in mains if j in path.main[-1]),
                             "model_size": len(path.main[-1]) + len(path.inter[-1]),
                             "kkt_rounds": int(sum(path.rounds))}
                log(f"lasso: setting {setting} p={p} {name}: {row[name]}")
            log(f"lasso: {row}")
            out.append(row)
            ctx.x_destroy(x)
    return {"experiment": "Lasso with all interactions, KKT screening by xyz (Section 5.4, Algorithm 3)",
            "data": "synthetic, settings 1-3 of Section 5.4 (setting 3: correlated DAG design)", "points": out}


def cpu_baseline(d, plan, kappa, ps=40_000, budget_s=12.0):
    """The CPU oracle on a bounded sample of the headline workload: its first `ps`
    columns (all n rows), run with the timed plan's method -- the oracle's
    Algorithm 2 at the plan's m (repetitions, each screening a 1/L share of the
    sample's pairs), or its brute force of eq. (1) -- on one thread, then on all
    threads of this process's CPU share (independent repetition ranges, or
    column blocks, one oracle call per thread).  Each rate is scaled to the
    pairs screened per second."""
    import concurrent.futures as cf
    import oracle
    XT = unpack_bits(d.bits[:ps], d.n)
    pairs = ps * (ps - 1) / 2
    nth = host_threads()
    out = {"unit": "pairs/s", "kind": "oracle", "threads_available": nth}
    if plan[0] == "brute":
        # brute force over column blocks; one block pair per call
        blk = 4000
        t0 = time.perf_counter()
        oracle.brute(XT[:blk], d.Y, kappa)
        t1 = time.perf_counter() - t0
        rate1 = blk * (blk - 1) / 2 / t1
        parts = [XT[q * blk // 2:(q + 2) * blk // 2] for q in range(nth)]
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(nth) as ex:
            list(ex.map(lambda a: oracle.brute(a, d.Y, kappa), parts))
        tn = time.perf_counter() - t0
        raten = sum(len(a) * (len(a) - 1) / 2 for a in parts) / tn
        out.update(value=rate1, cores=1, value_all_threads=raten, cores_all_threads=nth,
                   sample=f"brute force of eq. (1) over {blk}-column blocks of the first {ps} columns "
                          f"(n={d.n}): 1 thread {t1:.1f} s, {nth} threads {tn:.1f} s")
        return out
    m, L = plan[1], plan[2]
    t0 = time.perf_counter()
    reps = 0
    while time.perf_counter() - t0 < budget_s / 2 or reps == 0:
        oracle.search(XT, d.Y, m, 1, kappa, seed=1, rep_offset=reps)
        reps += 1
    t1 = time.perf_counter() - t0
    rate1 = pairs * (reps / L) / t1
    per = max(1, reps // 2)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(nth) as ex:
        list(ex.map(lambda w: oracle.search(XT, d.Y, m, per, kappa, seed=1, rep_offset=1000 + w * per), range(nth)))
    tn = time.perf_counter() - t0
    raten = pairs * (nth * per / L) / tn
    out.update(value=rate1, cores=1, value_all_threads=raten, cores_all_threads=nth,
               sample=f"the oracle's Algorithm 2 (m={m}, a 1/{L} share of the pairs per repetition) on the first "
                      f"{ps} of {d.p} columns (n={d.n}): {reps} repetitions on 1 thread in {t1:.1f} s, "
                      f"{nth} x {per} repetitions on {nth} threads in {tn:.1f} s")
    return out


if __name__ == "__main__":
    main()
