#!/usr/bin/env python
"""Benchmark: whole LSH-MF training job on one MI355X.

One step = one full training pass of the hot path over the MovieLens-10M
shaped workload (69,878 users x 10,677 items, 9.9M training ratings, F=64,
K=50, 128 hash bits, 20 epochs):
  ingest + layout -> simLSH neighbours (projection, banding, top-K, neighbour
  codes) -> 20 SGD epochs with the K-neighbour term -> predictions and FP64
  RMSE on the 100,000 held-out ratings.
The metric is rating SGD updates per second over the whole step
(epochs * training ratings / step time), inputs already resident in HBM.

Prints ONE JSON line.  The roofline object covers the dominant kernel
(k_sgd_stratum): algorithmic bytes of one launch (one stratum) over the
measured average launch time, against the 8 TB/s HBM peak.
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


def sgd_bytes_per_epoch(nnz, nseg, F, K, nstride, storage="fp32"):
    """Algorithmic HBM bytes of one epoch of k_sgd_stratum.

    Per rating: packed (user, code) 4 + hand-over word 4 + neighbour codes
    nstride + u_i read and write 8F + b_i read and write 8 + fixed baseline
    b0_i 4.  Per item segment (a run of one item inside a block): v_j read and
    write 8F, bh_j read and write 8, w_j and c_j read and write 16K, the fixed
    baselines of the K neighbours 4K, segment descriptor 12.  The kernel is
    the same in both storage modes (BF16 copies are converted after it).
    """
    per_rating = 4 + 4 + nstride + 8 * F + 8 + 4
    per_seg = 8 * F + 8 + 16 * K + 4 * K + 12
    return nnz * per_rating + nseg * per_seg


SHAPE_NAMES = {"ml10m": "MovieLens-10M", "netflix": "Netflix", "ml100k": "MovieLens-100K",
               "ml10m_k0": "MovieLens-10M", "ml100k_k0": "MovieLens-100K"}

KERNEL_SOURCES = ("paper_2111_11682_amd/csrc/sgd.hip", "paper_2111_11682_amd/csrc/common.hpp",
                  "include/lshmf.h")
PROFILE = os.path.join(ROOT, "profiles", "k_sgd_stratum_ml10m.md")


def kernel_fingerprint():
    """sha256 over the sources of the SGD kernel."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def profiled_traffic():
    """HBM bytes per k_sgd_stratum launch from the committed counter summary,
    or None when the kernel's sources changed since the counters were taken."""
    if not os.path.exists(PROFILE):
        return None
    rec = None
    for line in open(PROFILE):
        line = line.strip()
        if line.startswith("{") and "traffic_bytes_per_launch" in line:
            rec = json.loads(line)
    if rec is None or rec.get("source_sha256") != kernel_fingerprint():
        return None
    return int(rec["traffic_bytes_per_launch"])


def cpu_baseline(w, d, P, epochs=4):
    """The FP64 oracle's SGD on the same training set, a bounded number of epochs."""
    import numpy as np
    from oracle import oracle as orc
    u, it, rc = d["train_u"], d["train_i"], d["train_rc"]
    _, sig = orc.simlsh(w.M, w.N, w.B, u, it, rc, d["H"])
    JK = orc.topk(sig, w.B, w.G, w.p, w.q, w.K, 12345) if w.K > 0 else np.zeros((w.N, 0), np.int32)
    m = orc.Model(w.M, w.N, w.F, w.K, w.rscale, u, it, rc, JK, d["U0"], d["V0"])
    m._sched[P] = orc.schedule(P, u, it)             # the layout, untimed
    t0 = time.perf_counter()
    for t in range(epochs):
        m.sgd_epoch(P, w.alpha, w.lam, w.beta, t)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": float(epochs * u.size / dt), "unit": "updates/s", "cores": cores, "kind": "oracle",
            "sample": "%d FP64 oracle SGD epochs (%s, P=%d strata, OpenMP over the blocks "
                      "of a stratum) over all %d training ratings, %.1f s"
                      % (epochs, "K-neighbour term" if w.K > 0 else "K = 0, no neighbour term", P, u.size, dt)}


def serve_main(args, w, d):
    """Serving loop on the online split of the same workload: pre-train on
    80%, stream the rest as update batches (log-uniform 1k-1M ratings) mixed
    1:4 with query requests (log-uniform 1-10k pairs); Poisson arrivals at
    0.3, 0.6 and 0.9 of the capacity measured back to back."""
    import numpy as np
    import torch
    from paper_2111_11682_amd import lshmf, synth

    sp = synth.online_split(w, d, frac_new=0.01, stream_frac=0.2)
    L = synth.serve_log(sp, w.M, w.N, 1000, 1000000, 1, 10000)
    req = L["req"]
    M0, N0 = int(sp["M_old"]), int(sp["N_old"])
    dev = torch.device("cuda:0")
    pin = lambda a: torch.from_numpy(a).pin_memory()
    upd = (pin(L["upd_u"]), pin(L["upd_i"]), pin(L["upd_rc"]))
    qry = (pin(L["q_u"]), pin(L["q_i"]))
    U0 = torch.from_numpy(d["U0"]).to(dev)
    V0 = torch.from_numpy(d["V0"]).to(dev)
    H = torch.from_numpy(d["H"].view(np.int32)).to(dev)
    pre = [torch.from_numpy(sp[k]).to(dev) for k in ("pretrain_u", "pretrain_i", "pretrain_rc")]
    batch_cap = int(req["n"][req["kind"] == 0].max())
    log("serve: %d requests (%d updates, %d update ratings, %d query pairs), batch_cap %d" %
        (req.size, int((req["kind"] == 0).sum()), L["upd_u"].size, L["q_u"].size, batch_cap))

    def run(arrival):
        m = lshmf.LshMF(M0, N0, w.F, w.K, w.G, w.p, w.q, w.rscale, pre[0].numel(), n_strata=w.n_strata,
                        device=dev, M_cap=w.M, N_cap=w.N, nnz_cap=d["train_u"].size,
                        batch_cap=batch_cap, storage=args.storage)
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
        assert m.device_status() == 0
        m.close()
        return start, done, status

    def summary(arrival, start, done, status):
        out = {}
        for kind, name in ((1, "query"), (0, "update")):
            sel = (req["kind"] == kind) & (status == 0)
            lat = (done - arrival)[sel] * 1e3
            out[name + "_p50_ms"] = round(float(np.percentile(lat, 50)), 3)
            out[name + "_p99_ms"] = round(float(np.percentile(lat, 99)), 3)
        out["refused"] = int((status != 0).sum())
        return out

    zero = np.zeros(req.size)
    start, done, status = run(zero)
    makespan = float(done.max())
    capacity = req.size / makespan
    log("back to back: %.3f s for %d requests (%.1f requests/s)" % (makespan, req.size, capacity))
    loads = {"back_to_back": dict(summary(zero, start, done, status), makespan_s=round(makespan, 4))}
    for rho in (0.3, 0.6, 0.9):
        arr = synth.poisson_arrivals(req.size, rho * capacity)
        start, done, status = run(arr)
        loads["load_%.1f" % rho] = summary(arr, start, done, status)
        log("load %.1f: %s" % (rho, loads["load_%.1f" % rho]))
    out = {"metric": "serving query latency p99 at 0.6 of capacity", "value": loads["load_0.6"]["query_p99_ms"],
           "unit": "ms", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (MovieLens-10M shape, 1% new users and items, 20% of ratings streamed)",
           "config": {"workload": "ml10m-shaped online stream", "requests": int(req.size),
                      "update_ratings": int(L["upd_u"].size), "query_pairs": int(L["q_u"].size),
                      "capacity_requests_per_s": round(capacity, 2), "storage": args.storage, "loads": loads}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ml10m")
    ap.add_argument("--epochs", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=("train", "serve"), default="train",
                    help="serve: the serving loop over an online stream instead of the training job")
    ap.add_argument("--storage", choices=("fp32", "bf16"), default=None,
                    help="bf16: BF16 copies of U, V, W, C beside the FP32 masters "
                         "(default fp32 for training, bf16 for serving)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy, the reference for HBM byte counters")
    args = ap.parse_args()
    if args.storage is None:
        args.storage = "bf16" if args.mode == "serve" else "fp32"
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
    d = synth.generate(w)
    log("generated %s: %d train / %d test ratings in %.1fs" %
        (w.name, d["train_u"].size, d["test_u"].size, time.time() - t0))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.mode == "serve":
        serve_main(args, w, d)
        return
    g = {k: torch.from_numpy(v).to(dev) for k, v in d.items() if k != "H"}
    H = torch.from_numpy(d["H"].view(np.int32)).to(dev)
    nnz = d["train_u"].size
    P = w.n_strata
    m = lshmf.LshMF(w.M, w.N, w.F, w.K, w.G, w.p, w.q, w.rscale, nnz, n_strata=P, device=dev,
                    storage=args.storage)
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
    assert m.device_status() == 0
    final_rmse = rmse.item()
    sgd_ms_epoch = sum(a.elapsed_time(b) for a, b in sgd_events) / len(sgd_events)
    log("step %.2f ms, SGD %.3f ms/epoch, RMSE %.5f" % (ms, sgd_ms_epoch, final_rmse))

    lay = m.layout()
    nseg = int(m.arena_view(lay.blk_seg, P * P + 1, torch.int64)[-1].item())
    epoch_bytes = sgd_bytes_per_epoch(nnz, nseg, w.F, w.K, lay.nstride, args.storage)
    launch_bytes = epoch_bytes / P
    launch_s = sgd_ms_epoch / 1e3 / P
    achieved = launch_bytes / launch_s / 1e9
    traffic = profiled_traffic() if (args.workload == "ml10m" and args.storage == "fp32") else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": 8000.0, "unit": "GB/s",
                "frac": round(achieved / 8000.0, 5), "traffic": traffic,
                "kernel": "k_sgd_stratum", "launch_bytes": int(launch_bytes),
                "launch_us": round(launch_s * 1e6, 3)}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a sample")
        cpu = cpu_baseline(w, d, P)
        log("oracle %.0f updates/s on %d cores" % (cpu["value"], cpu["cores"]))

    value = epochs * nnz / (ms / 1e3)
    out = {
        "metric": ("rating SGD updates/sec (K-neighbour term incl.)" if w.K > 0
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
        "dtype": "f32",
        "data": "synthetic (seeded Zipf/lognormal ratings with planted structure, %s shape)" % SHAPE_NAMES.get(w.name, w.name),
        "config": {"workload": ("%s-shaped LSH-MF training job" % w.name if w.K > 0
                               else "%s-shaped biased-MF training job (K = 0)" % w.name[:-3]), "users": w.M, "items": w.N,
                   "train_ratings": int(nnz), "test_ratings": int(d["test_u"].size), "F": w.F,
                   "K": w.K, "hash_bits": w.B, "p": w.p, "q": w.q, "epochs": epochs,
                   "n_strata": P, "storage": args.storage, "heldout_rmse": round(final_rmse, 6),
                   "sgd_ms_per_epoch": round(sgd_ms_epoch, 3),
                   "sgd_updates_per_s": round(nnz / (sgd_ms_epoch / 1e3), 1)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
