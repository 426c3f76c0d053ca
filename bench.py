#!/usr/bin/env python
"""Benchmark: whole LSH-MF training job on one MI355X.

One step = one full training pass of the hot path over the Netflix-shaped
workload (480,189 users x 17,770 items, 98,591,605 training ratings, F = 128,
K = 100, 128 hash bits, 20 epochs, FP32):
  ingest + layout -> simLSH neighbours (projection, banding, top-K, neighbour
  codes) -> 20 SGD epochs with the K-neighbour term -> predictions and FP64
  RMSE on the 1,408,395 held-out ratings.
The metric is rating SGD updates per second over the whole step
(epochs * training ratings / step time), inputs already resident in HBM.

Prints ONE JSON line.  Besides the contract fields it carries
  roofline      the dominant kernel (k_sgd_stratum): algorithmic bytes of one
                launch (one stratum) over its mean launch time, against the
                8 TB/s HBM peak; traffic = measured HBM bytes per launch from
                the committed counter summary while the kernel's sources match
  lsh_phases_ms the neighbour search of the last step, by phase
  serving       the serving loop on the MovieLens-10M shaped online stream
                (p50 / p99 latency at offered loads, online updates/s)
  cpu_baseline  the FP64 oracle on a bounded sample, 1 thread and all threads

--mode lsh times the neighbour search alone (the paper's simLSH settings),
--mode serve the serving loop alone.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def sgd_bytes_per_epoch(nnz, nseg, F, K, nstride, u_bytes=4):
    """Algorithmic HBM bytes of one epoch of k_sgd_stratum.

    Per rating: packed (user, code) 4 + hand-over word 4 + neighbour codes
    nstride + u_i read and write 8F + b_i read and write 8 + fixed baseline
    b0_i 4.  Per item segment (a run of one item inside a block): v_j read and
    write 8F, bh_j read and write 8, w_j and c_j read and write 16K, the fixed
    baselines of the K neighbours 4K, segment descriptor 12.  The kernel is
    the same in storage modes FP32 and BF16 (BF16 copies are converted after
    it); in mode BF16_U the user row is 2 bytes a feature (u_bytes = 2).
    """
    per_rating = 4 + 4 + nstride + 2 * u_bytes * F + 8 + 4
    per_seg = 8 * F + 8 + 16 * K + 4 * K + 12
    return nnz * per_rating + nseg * per_seg


SHAPE_NAMES = {"ml10m": "MovieLens-10M", "netflix": "Netflix", "ml100k": "MovieLens-100K"}

KERNEL_SOURCES = ("paper_2111_11682_amd/csrc/sgd.hip", "paper_2111_11682_amd/csrc/wave.hpp",
                  "paper_2111_11682_amd/csrc/common.hpp")


def kernel_fingerprint():
    """sha256 over the sources of the SGD kernel."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def profiled_traffic(workload):
    """HBM bytes per k_sgd_stratum launch from the committed counter summary
    of this workload, or None when the kernel's sources changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_sgd_stratum_%s.md" % workload)
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        line = line.strip()
        if line.startswith("{") and "traffic_bytes_per_launch" in line:
            rec = json.loads(line)
    if rec is None or rec.get("source_sha256") != kernel_fingerprint():
        return None
    return int(rec["traffic_bytes_per_launch"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, d, P, stride=16, target_s=8.0):
    """The FP64 oracle on a bounded sample of the same workload: the ratings of
    every stride-th user (ids are a random permutation, so a random 1/stride
    of the users with their whole rating rows), with the sample's own simLSH
    neighbour lists.  Strata of one epoch run in order, first on one thread,
    then on all threads, each until target_s seconds have passed."""
    import numpy as np
    from oracle import oracle as orc
    sel = d["train_u"] % stride == 0
    u = (d["train_u"][sel] // stride).astype(np.int32)
    it = d["train_i"][sel]
    rc = d["train_rc"][sel]
    Ms = (w.M + stride - 1) // stride
    H = d["H"][::stride]
    t0 = time.perf_counter()
    _, sig = orc.simlsh(Ms, w.N, w.B, u, it, rc, H)
    JK = orc.topk(sig, w.B, w.G, w.p, w.q, w.K, 12345) if w.K > 0 else np.zeros((w.N, 0), np.int32)
    m = orc.Model(Ms, w.N, w.F, w.K, w.rscale, u, it, rc, JK, d["U0"][::stride], d["V0"])
    order, blk = orc.schedule(P, u, it)
    m._sched[P] = (order, blk)
    log("oracle sample: %d users, %d ratings, set up in %.1f s" % (Ms, u.size, time.perf_counter() - t0))
    all_threads = orc.max_threads()
    rates = {}
    s = 0
    for threads in (1, all_threads):
        orc.set_threads(threads)
        done = 0
        t0 = time.perf_counter()
        while s < P and time.perf_counter() - t0 < target_s:
            m.sgd_strata(P, s, s + 1, w.alpha, w.lam, w.beta, 0)
            done += int(blk[(s + 1) * P] - blk[s * P])
            s += 1
        dt = time.perf_counter() - t0
        rates[threads] = (done / dt, done, dt)
    orc.set_threads(all_threads)
    rN, nN, tN = rates[all_threads]
    r1, n1, t1 = rates[1]
    return {"value": round(rN, 1), "unit": "updates/s", "cores": all_threads, "kind": "oracle",
            "value_1thread": round(r1, 1), "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": "FP64 oracle SGD (K-neighbour term, P=%d strata in schedule order) on the ratings of every "
                      "%dth user of the %s-shaped set (%d users, %d ratings, own simLSH lists): %d updates in "
                      "%.1f s on %d threads, %d updates in %.1f s on 1 thread"
                      % (P, stride, SHAPE_NAMES.get(w.name, w.name), Ms, u.size, nN, tN, all_threads, n1, t1)}


def serve_runs(w, d, storage, loads=(0.3, 0.6, 0.9), logs=6, log_fn=log):
    """Serving loop on the online split of the workload: pre-train on 80%,
    stream the rest as update batches (log-uniform 1k-1M ratings) mixed 1:4
    with query requests (log-uniform 1-10k pairs); back to back, then Poisson
    arrivals at fractions of the capacity measured back to back.  `logs`
    request logs (seeded cuts of the same stream into batches) are replayed
    at every setting and their latencies pooled, so that the percentiles
    rest on a few hundred requests."""
    import numpy as np
    import torch
    from paper_2111_11682_amd import lshmf, synth

    sp = synth.online_split(w, d, frac_new=0.01, stream_frac=0.2)
    Ls = [synth.serve_log(sp, w.M, w.N, 1000, 1000000, 1, 10000, seed=synth.MASTER_SEED + k) for k in range(logs)]
    M0, N0 = int(sp["M_old"]), int(sp["N_old"])
    dev = torch.device("cuda:0")
    pin = lambda a: torch.from_numpy(a).pin_memory()
    U0 = torch.from_numpy(d["U0"]).to(dev)
    V0 = torch.from_numpy(d["V0"]).to(dev)
    H = torch.from_numpy(d["H"].view(np.int32)).to(dev)
    pre = [torch.from_numpy(sp[k]).to(dev) for k in ("pretrain_u", "pretrain_i", "pretrain_rc")]
    batch_cap = max(int(L["req"]["n"][L["req"]["kind"] == 0].max()) for L in Ls)
    n_req = sum(L["req"].size for L in Ls)
    log_fn("serve: %d logs, %d requests (%d updates), batch_cap %d" %
           (logs, n_req, sum(int((L["req"]["kind"] == 0).sum()) for L in Ls), batch_cap))

    def run(L, arrival):
        req = L["req"]
        upd = (pin(L["upd_u"]), pin(L["upd_i"]), pin(L["upd_rc"]))
        qry = (pin(L["q_u"]), pin(L["q_i"]))
        m = lshmf.LshMF(M0, N0, w.F, w.K, w.G, w.p, w.q, w.rscale, pre[0].numel(), n_strata=w.n_strata,
                        device=dev, M_cap=w.M, N_cap=w.N, nnz_cap=d["train_u"].size,
                        batch_cap=batch_cap, storage=storage)
        m.ingest(*pre)
        m.set_factors(U0[:M0], V0[:N0])
        m.build_lsh_neighbours(H, 12345)
        for t in range(w.epochs):
            m.sgd_epoch(w.alpha, w.lam, w.beta, t)
        torch.cuda.synchronize()
        r = req.copy()
        r["arrival"] = arrival
        _, start, done, status = m.serve(r, upd, qry, U0, V0, H, 12345, w.alpha, w.lam, w.beta, w.epochs, 1,
                                         max_query_batch=65536)
        m.check()
        m.close()
        return start, done, status

    def pooled(results):
        """results: [(L, arrival, start, done, status)] -> latency summary."""
        out = {}
        for kind, name in ((1, "query"), (0, "update")):
            lat = []
            for L, arr, start, done, status in results:
                sel = (L["req"]["kind"] == kind) & (status == 0)
                lat.append((done - arr)[sel] * 1e3)
            lat = np.concatenate(lat)
            out[name + "_p50_ms"] = round(float(np.percentile(lat, 50)), 3)
            out[name + "_p99_ms"] = round(float(np.percentile(lat, 99)), 3)
            out[name + "_count"] = int(lat.size)
        out["refused"] = int(sum(int((st != 0).sum()) for _, _, _, _, st in results))
        return out

    b2b, makespan, upd_time, upd_n = [], 0.0, 0.0, 0
    for L in Ls:
        zero = np.zeros(L["req"].size)
        start, done, status = run(L, zero)
        b2b.append((L, zero, start, done, status))
        makespan += float(done.max())
        sel = (L["req"]["kind"] == 0) & (status == 0)
        upd_time += float(np.sum(done[sel] - start[sel]))
        upd_n += int(np.sum(L["req"]["n"][sel]))
    capacity = n_req / makespan
    online_rate = upd_n / upd_time if upd_time > 0 else 0.0
    log_fn("back to back: %.3f s for %d requests (%.1f requests/s), online %.0f rating updates/s"
           % (makespan, n_req, capacity, online_rate))
    res = {"back_to_back": dict(pooled(b2b), makespan_s=round(makespan, 4))}
    for rho in loads:
        rs = []
        for k, L in enumerate(Ls):
            arr = synth.poisson_arrivals(L["req"].size, rho * capacity, seed=synth.MASTER_SEED + 100 * k + 1)
            start, done, status = run(L, arr)
            rs.append((L, arr, start, done, status))
        res["load_%.1f" % rho] = pooled(rs)
        log_fn("load %.1f: %s" % (rho, res["load_%.1f" % rho]))
    return {"workload": "%s-shaped online stream (1%% new users and items, 20%% of ratings streamed, %d seeded "
                        "request logs)" % (SHAPE_NAMES.get(w.name, w.name), logs),
            "requests": int(n_req), "update_ratings": int(sum(L["upd_u"].size for L in Ls)),
            "query_pairs": int(sum(L["q_u"].size for L in Ls)),
            "storage": storage, "capacity_requests_per_s": round(capacity, 2),
            "online_updates_per_s": round(online_rate, 1), "loads": res}


def serve_main(args, w, d):
    res = serve_runs(w, d, args.storage)
    out = {"metric": "serving query latency p99 at 0.6 of capacity", "value": res["loads"]["load_0.6"]["query_p99_ms"],
           "unit": "ms", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (%s shape, 1%% new users and items, 20%% of ratings streamed)"
                   % SHAPE_NAMES.get(w.name, w.name),
           "config": dict(res, workload=res["workload"])}
    print(json.dumps(out), flush=True)


def lsh_main(args, w, d):
    """The neighbour search alone at the workload's (G, p, q): time per call
    and by phase, and the space of the hash table as the paper counts it
    (one int32 per G-bit hash: N * p * q * 4 bytes)."""
    import numpy as np
    import torch
    from paper_2111_11682_amd import lshmf, synth
    dev = torch.device("cuda:0")
    R = synth.family_rand(w)
    Rt = torch.from_numpy(R.view(np.int32) if R.dtype == np.uint32 else R).to(dev)
    m = lshmf.LshMF(w.M, w.N, w.F, w.K, w.G, w.p, w.q, w.rscale, d["train_u"].size, n_strata=w.n_strata,
                    device=dev, hash_family=w.family)
    m.ingest(*[torch.from_numpy(d[k]).to(dev) for k in ("train_u", "train_i", "train_rc")])
    m.set_timing(True)
    for _ in range(args.warmup):
        m.build_lsh_neighbours(Rt, 12345)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    phases = []
    e0.record()
    for _ in range(args.steps):
        m.build_lsh_neighbours(Rt, 12345)
        phases.append(m.lsh_phase_ms())
    e1.record()
    torch.cuda.synchronize()
    m.check()
    ms = e0.elapsed_time(e1) / args.steps
    ph = {k: round(float(np.mean([p[k] for p in phases])), 3) for k in phases[0]}
    fam = {0: "simLSH", 1: "RP_cos", 2: "minHash"}[w.family]
    out = {"metric": "top-K neighbour search time (%s, p=%d, q=%d)" % (fam, w.p, w.q), "value": round(ms, 3),
           "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": False,
           "vs_baseline": None, "dtype": "int32" if w.family != 1 else "f32",
           "data": "synthetic (%s shape)" % SHAPE_NAMES.get(w.name.split("_")[0], w.name),
           "config": {"workload": "%s neighbour search on the %s-shaped training set" % (fam, w.name.split("_")[0]),
                      "users": w.M, "items": w.N, "train_ratings": int(d["train_u"].size), "K": w.K, "G": w.G,
                      "p": w.p, "q": w.q, "hash_bits": w.B,
                      "space_mib": round(w.N * w.p * w.q * 4 / 2**20, 3)},
           "lsh_phases_ms": ph}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=None, help="default netflix (train), ml10m (serve), netflix_p3q100 (lsh)")
    ap.add_argument("--epochs", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="leave the serving runs out of the training line")
    ap.add_argument("--mode", choices=("train", "serve", "lsh"), default="train",
                    help="serve: the serving loop alone; lsh: the neighbour search alone")
    ap.add_argument("--storage", choices=("fp32", "bf16", "bf16u"), default=None,
                    help="bf16: BF16 copies of U, V, W, C beside the FP32 masters; bf16u: user rows "
                         "stored in BF16 only (default fp32 for training, bf16 for serving)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy, the reference for HBM byte counters")
    args = ap.parse_args()
    if args.storage is None:
        args.storage = "bf16" if args.mode == "serve" else "fp32"
    if args.workload is None:
        args.workload = {"train": "netflix", "serve": "ml10m", "lsh": "netflix_p3q100"}[args.mode]
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2111_11682_amd import lshmf, synth

    w = synth.WORKLOADS[args.workload]
    epochs = args.epochs or w.epochs
    t0 = time.time()
    d = synth.generate(w, log=log if w.nnz > 200_000_000 else None)
    log("generated %s: %d train / %d test ratings in %.1fs" %
        (w.name, d["train_u"].size, d["test_u"].size, time.time() - t0))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.mode == "serve":
        serve_main(args, w, d)
        return
    if args.mode == "lsh":
        lsh_main(args, w, d)
        return
    g = {k: torch.from_numpy(v).to(dev) for k, v in d.items() if k != "H"}
    if w.family == 0:
        H = torch.from_numpy(d["H"].view(np.int32)).to(dev)
    else:  # the draws of the RP_cos / minHash families
        R = synth.family_rand(w)
        H = torch.from_numpy(R.view(np.int32) if R.dtype == np.uint32 else R).to(dev)
    nnz = d["train_u"].size
    P = w.n_strata
    m = lshmf.LshMF(w.M, w.N, w.F, w.K, w.G, w.p, w.q, w.rscale, nnz, n_strata=P, device=dev,
                    storage=args.storage, hash_family=w.family, model=w.model)
    m.set_timing(True)
    pred = torch.empty(d["test_u"].size, dtype=torch.float32, device=dev)
    rmse = torch.empty(1, dtype=torch.float64, device=dev)
    sgd_events = []

    def step(record):
        m.set_factors(g["U0"], g["V0"])
        m.ingest(g["train_u"], g["train_i"], g["train_rc"])
        m.build_lsh_neighbours(H, 12345)
        for t in range(epochs):
            if record:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
            m.sgd_epoch(w.alpha, w.lam, w.beta, t)
            if record:
                e1.record()
                sgd_events.append((e0, e1))
        m.predict(g["test_u"], g["test_i"], out=pred)
        m.rmse(pred, g["test_rc"], out=rmse)

    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: 1 GiB read + 1 GiB written")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log("warmup done, RMSE %.5f" % rmse.item())
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for k in range(args.steps):
        step(True)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    m.check()
    final_rmse = rmse.item()
    lsh_ms = m.lsh_phase_ms()
    sgd_ms_epoch = sum(a.elapsed_time(b) for a, b in sgd_events) / len(sgd_events)
    log("step %.2f ms, SGD %.3f ms/epoch, RMSE %.5f, LSH phases %s" % (ms, sgd_ms_epoch, final_rmse, lsh_ms))

    lay = m.layout()
    nseg = int(m.arena_view(lay.blk_seg, P * P + 1, torch.int64)[-1].item())
    epoch_bytes = sgd_bytes_per_epoch(nnz, nseg, w.F, w.K, lay.nstride, 2 if args.storage == "bf16u" else 4)
    launch_bytes = epoch_bytes / P
    launch_s = sgd_ms_epoch / 1e3 / P
    achieved = launch_bytes / launch_s / 1e9
    traffic = profiled_traffic(w.name) if args.storage == "fp32" else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": 8000.0, "unit": "GB/s",
                "frac": round(achieved / 8000.0, 5), "traffic": traffic,
                "kernel": "k_sgd_stratum", "launch_bytes": int(launch_bytes),
                "launch_us": round(launch_s * 1e6, 3)}
    m.close()
    del m, g
    torch.cuda.empty_cache()

    serving = None
    if not args.no_serve:
        ws = synth.WORKLOADS["ml10m"]
        serving = serve_runs(ws, synth.generate(ws), "bf16")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a sample")
        cpu = cpu_baseline(w, d, P)
        log("oracle %.0f updates/s on %d threads, %.0f on 1 thread (%s)"
            % (cpu["value"], cpu["cores"], cpu["value_1thread"], cpu["cpu_model"]))

    value = epochs * nnz / (ms / 1e3)
    out = {
        "metric": ("rating SGD updates/sec (K-neighbour term incl.)" if w.K > 0
                   else "rating SGD updates/sec (plain MF, CUSGD++ model)" if w.model == 1
                   else "rating SGD updates/sec (biased MF, K = 0)"),
        "value": round(value, 1),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage != "bf16u" else "f32 (BF16 user rows)",
        "data": "synthetic (seeded Zipf/lognormal ratings with planted structure, %s shape)"
                % SHAPE_NAMES.get(w.name.split("_")[0], w.name),
        "config": {"workload": "%s-shaped LSH-MF training job (ingest, simLSH top-K, %d SGD epochs, held-out "
                               "RMSE)" % (SHAPE_NAMES.get(w.name.split("_")[0], w.name), epochs),
                   "users": w.M, "items": w.N, "train_ratings": int(nnz), "test_ratings": int(d["test_u"].size),
                   "F": w.F, "K": w.K, "hash_bits": w.B, "p": w.p, "q": w.q, "epochs": epochs,
                   "n_strata": P, "storage": args.storage, "heldout_rmse": round(final_rmse, 6),
                   "sgd_ms_per_epoch": round(sgd_ms_epoch, 3),
                   "sgd_updates_per_s": round(nnz / (sgd_ms_epoch / 1e3), 1)},
        "roofline": roofline,
        "lsh_phases_ms": {k: round(v, 3) for k, v in lsh_ms.items()},
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
