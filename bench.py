"""Benchmark of MPS Pauli-pair feature extraction on one MI355X.

Workload (the headline configuration): 7x7 images -> 49 qubits, batch 1024 synthetic
Gaussian-blob images, L = 4 layers, chi = 16, complex64 contractions with FP64 SVD; 84
horizontal+vertical neighbour pairs x 15 Pauli expectations per image, then the
observable-weighted readout 84 -> 784.  One step = encode + 4 layers + environments + pair
expectations + readout over the whole batch, inputs already resident in HBM.

Prints one JSON line with throughput (images/s, batched), the plain one-image-per-call rate,
per-image latency percentiles, the max abs error of sampled outputs against the FP64 oracle,
the roofline of the dominant kernel (measured with HIP events on the launch stream) and the
CPU oracle baseline on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_FP32_VALU_TFLOPS = 78.6  # FP32 vector with packed FP32 disabled (same lane count and clock)
PEAK_FP32_MFMA_TFLOPS = 157.3  # FP32 matrix cores (dense)
PEAK_FP64_MFMA_TFLOPS = 78.6   # FP64 matrix cores (dense)
PEAK_BF16_MFMA_TFLOPS = 2500.0  # bf16 matrix cores (dense)
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch from two rocprofv3 counter runs (FETCH_SIZE x 2.0 and WRITE_SIZE x 1.0,
# the factors a 1 GiB device copy reads in the same runs), valid only for the kernel source they
# were taken on (and, for the measurement, the default pair-kernel schedule).
MEASURED_TRAFFIC = {
    # one k_layer launch (one layer of the canonical sweep + Jacobi SVD ladder), averaged over
    # the four layers of the headline
    "layers_svd": {"source": "paper_2607_10280_amd/csrc/layer.hip",
                   "sha1": "3b8824bf3b21012db511018fbf8ba81a5c2f76cb",
                   "bytes": (2 * 36810.0 + 73450.0) * 1024},
    # one measurement call: k_env16 + k_pairs16 (complex64, slot 16, blocks of 64 images)
    "measure": {"source": "paper_2607_10280_amd/csrc/measure_mfma.hip",
                "sha1": "e6a3d207a6a8c958fbc5c4e8437ff6e42cdd7f1f",
                "bytes": (2 * (194600.0 + 223460.0) + (204830.0 + 5617.0)) * 1024},
}


def _measured_traffic(kernel):
    import hashlib
    rec = MEASURED_TRAFFIC.get(kernel)
    if rec is None:
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha1(f.read()).hexdigest() != rec["sha1"]:
            return None  # the kernel changed since the counters were taken
    return rec["bytes"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--p", type=int, default=7)
    ap.add_argument("--layers", type=int, default=4)
    ap.add_argument("--chi", type=int, default=16)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "split_bf16"])
    ap.add_argument("--plain-images", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the eager step instead of its HIP-graph replay")
    ap.add_argument("--layers-mode", default="svd", choices=["svd", "qr", "mpo"],
                    help="how layers that keep every singular value are applied in the timed "
                         "step: svd = canonical sweep + Jacobi SVD ladder like every other layer "
                         "(the method; default), qr / mpo = the exact shortcuts")
    ap.add_argument("--no-shortcut", action="store_true",
                    help="skip the extra timing of the exact shortcut (mpo) beside the method")
    ap.add_argument("--tune", action="store_true",
                    help="choose the pair-kernel schedule by measurement before timing (the "
                         "library default is blocks of 64 images, no occupancy cap)")
    ap.add_argument("--no-trunc-cell", action="store_true",
                    help="skip the extra timing of the truncating cell (chi = 8)")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "mixed", "serve", "grid", "paper", "chisweep",
                             "precision"],
                    help="headline: the 7x7 L=4 chi=16 batch; mixed: 4096 requests of mixed size "
                         "and depth through the persistent mixed-table launches; serve: Poisson "
                         "arrivals through the continuous-batching loop; chisweep: feature error "
                         "and cost against chi at 7x7, L=7 (chi=128 is exact); precision: FP32 "
                         "against split-BF16 errors per (L, chi) at 16x16")
    ap.add_argument("--requests", type=int, default=0, help="mixed/serve: number of requests")
    ap.add_argument("--tune-cache", default="", help="mixed/serve: autotuner JSON cache path")
    ap.add_argument("--counters-only", action="store_true",
                    help="headline: run only the copy calibration and --steps eager steps, then "
                         "exit (for counter runs); prints no result line")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a kernel of known "
                         "traffic, to scale hardware byte counters)")
    return ap.parse_args()


LAYER_MODES = {"qr": 0, "svd": 1, "mpo": 2}   # mps_set_exact_layers modes


# ----------------------------------------------------------------------------- CPU baseline
def _single_thread():
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"


def _oracle_worker(args):
    x, th, ph, pairs, chi = args
    from oracle import features as ofeat
    t0 = time.perf_counter()
    f, _, _ = ofeat.truncated_features(x[None], th, ph, pairs, chi)
    return f[0], time.perf_counter() - t0


def _warm_worker():
    """Pool initializer: one BLAS thread, the oracle imported and run once on a tiny input, so
    that neither process start-up nor first-call costs fall inside the timed region."""
    _single_thread()
    from oracle import features as ofeat
    ofeat.truncated_features(np.full((1, 4), 0.5), np.zeros((1, 4)), np.zeros((1, 4)),
                             np.array([[0, 1]], np.int32), 2)


def _ready(_):
    return os.getpid()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x, th, ph, pairs, chi, one_core=16, per_worker=8, max_workers=16):
    """The FP64 oracle (same truncation rule and chi) on the host: `one_core` images serially in
    one process (1-core rate), then `per_worker` images per process over a persistent pool of
    min(os.cpu_count(), max_workers) single-threaded processes (all-core rate).  The pool is
    started and warmed before either timer starts.  Returns (features of the all-core sample,
    record)."""
    workers = max(1, min(os.cpu_count() or 1, max_workers))
    n_all = min(len(x), workers * per_worker)
    n_one = min(len(x), one_core)
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_warm_worker) as pool:
        pool.map(_ready, range(4 * workers), chunksize=1)   # every worker started and warm
        t0 = time.perf_counter()
        for i in range(n_one):
            pool.apply(_oracle_worker, ((x[i], th, ph, pairs, chi),))
        one_s = time.perf_counter() - t0
        jobs = [(x[i], th, ph, pairs, chi) for i in range(n_all)]
        t0 = time.perf_counter()
        res = pool.map(_oracle_worker, jobs, chunksize=1)
        all_s = time.perf_counter() - t0
    feats = np.stack([r[0] for r in res])
    per_image = float(np.mean([r[1] for r in res]))
    rec = {"value": round(n_all / all_s, 3), "unit": "images/s", "cores": workers,
           "kind": "oracle",
           "one_core_images_per_s": round(n_one / one_s, 3),
           "cpu_count": os.cpu_count(), "cpu_model": _cpu_model(),
           "sample": f"FP64 CPU oracle (numpy/LAPACK MPS, same chi and truncation rule) on the "
                     f"batch's first images: {n_one} serially in one process (1-core rate), then "
                     f"{n_all} over a warm pool of {workers} single-threaded processes (all-core "
                     f"rate, {per_worker} per process); {per_image:.3f} s per image per core; "
                     f"the pool is capped at {max_workers} processes, the GPU box's CPU share"}
    return feats, rec


# ----------------------------------------------------------------------------- mixed / serve
def _specs(mix, prec):
    from paper_2607_10280_amd import inputs, mixed
    specs = []
    for q in mix:
        p, L = q["p"], q["layers"]
        x = inputs.blob_image(p, q["image_seed"])
        th, ph = inputs.layer_angles(L, p * p, q["angle_seed"])
        specs.append(mixed.RequestSpec(x, th, ph, inputs.neighbour_pairs(p), q["chi"], prec))
    return specs


def _tune(specs, args):
    from paper_2607_10280_amd import autotune
    if args.tune_cache and autotune.load_and_apply(args.tune_cache):
        return {"source": args.tune_cache}
    sample = specs[: min(len(specs), 2048)]
    choice = autotune.tune(sample)
    if args.tune_cache:
        autotune.save(choice, args.tune_cache)
    return {str(b): {"blocks_per_cu": c[0], "ms": round(c[1], 3)} for b, c in choice.items()}


def run_mixed(args):
    """4096 requests, p in {6,8,10,12}, L in {1,2}, chi = 16, complex64 + FP64 SVD: the whole
    table through init, the layer steps and the measurement, eager and as one HIP graph, against
    one request per call."""
    import torch
    from paper_2607_10280_amd import anomps, inputs, mixed
    from oracle import features as ofeat
    N = args.requests or 4096
    prec = anomps.PRECISIONS[args.precision]
    specs = _specs(inputs.request_mix(N, [6, 8, 10, 12], [1, 2], [16], 4), prec)
    tuning = _tune(specs, args)
    mr = mixed.MixedRequests(specs)
    mr.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        mr.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    outs = mr.outputs()
    # the same sequence captured once and replayed
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            mr.run(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    g.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / args.steps
    graph_same = all(np.array_equal(a, b) for a, b in zip(outs, mr.outputs()))
    # one request per call, and batch invariance on a sample
    rng = np.random.Generator(np.random.PCG64(11))
    sample = rng.choice(N, size=min(N, args.plain_images * 4), replace=False)
    same = 0
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in sample:
        sp = specs[i]
        o, _ = anomps.extract_features(sp.pixels[None], sp.theta, sp.phi, sp.pairs, sp.chi, prec,
                                       per_layer=True)
        same += int(np.array_equal(o.cpu().numpy()[0], outs[i]))
    plain_s = (time.perf_counter() - t) / len(sample)
    small = [i for i in sample if specs[i].n <= 64][:4]
    err = max(float(np.abs(outs[i] - ofeat.exact_features(specs[i].pixels[None], specs[i].theta,
                                                           specs[i].phi, specs[i].pairs)[0]).max())
              for i in small)
    ctrl = mr.ctrl()
    result = {
        "metric": "mixed-request images/sec (4096 requests, p in {6,8,10,12}, L in {1,2}, chi=16)",
        "value": round(N / (ms * 1e-3), 1), "unit": "images/s", "n_gpus": 1,
        "steps": args.steps, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "dtype": "c64+f64svd" if prec == anomps.PREC_FP32 else "f64", "data": "synthetic",
        "config": {"workload": f"{N} mixed requests, Gaussian blobs, p~U{{6,8,10,12}}, "
                               f"L~U{{1,2}}, chi=16, H+V pairs", "requests": N,
                   "layers_mode": args.layers_mode},
        "graph": {"images_per_s": round(N / (ms_graph * 1e-3), 1), "ms_per_step": round(ms_graph, 4),
                  "identical_to_eager": bool(graph_same)},
        "plain": {"images_per_s": round(1.0 / plain_s, 1), "requests_timed": int(len(sample))},
        "batch_invariance": {"checked": int(len(sample)), "identical": int(same)},
        "max_abs_err_vs_oracle": err, "oracle_checked": len(small),
        "status_nonzero": int(np.count_nonzero(ctrl[:, 1])),
        "layers_ok": bool(np.all(ctrl[:, 0] == [sp.layers for sp in specs])),
        "tuning": tuning,
    }
    print(json.dumps(result))


def run_serve(args):
    """Poisson arrivals of single-image requests (p~U{7..16}, L~U{1..4}, chi~U{2,4,8,16,32});
    p = 7 requests also run the readout 84 -> 784.  Saturation throughput first (all requests
    present at t = 0), then traces at 0.5x and 0.9x of it; the same trace through a plain FIFO
    (one request per call) for comparison."""
    import torch
    from paper_2607_10280_amd import anomps, inputs, serving
    prec = anomps.PRECISIONS[args.precision]
    N = args.requests or 11000
    warm = min(1000, N // 11)
    mix = inputs.request_mix(N, list(range(7, 17)), [1, 2, 3, 4], [2, 4, 8, 16, 32], 6)
    specs = _specs(mix, prec)
    tuning = _tune(specs, args)
    m7 = len(inputs.neighbour_pairs(7))
    ra, rb, rd, rw, rbias = inputs.readout_params(m7, 784, 8)
    real = torch.float64 if prec == anomps.PREC_FP64 else torch.float32
    T = lambda v: torch.as_tensor(v, dtype=real, device="cuda").contiguous()
    coeff = torch.empty((m7, 16), dtype=real, device="cuda")
    anomps.ano_coeffs(T(ra), T(rb), T(rd), coeff)
    ro = (coeff, T(rw), T(rbias))
    free, total = torch.cuda.mem_get_info()
    arena = int(min(free * 0.5, 64 << 30))

    def make(arrivals, idx):
        return [serving.Request(k, float(arrivals[j]), specs[k], ro if specs[k].n == 49 else None)
                for j, k in enumerate(idx)]

    srv = serving.Server(arena)
    sat_n = min(N, 4000)
    sat = srv.run(make(np.zeros(sat_n), range(sat_n))).summary()
    qps_sat = sat["throughput_req_per_s"]
    print(f"[serve] saturation {qps_sat} req/s", file=sys.stderr, flush=True)
    runs = {}
    for frac in (0.5, 0.9):
        arr = inputs.poisson_arrivals(N, frac * qps_sat, 6)
        reqs = make(arr, range(N))
        st = srv.run(reqs)
        lat = np.array(st.latencies_ms)
        order = np.argsort([r.arrival for r in reqs])
        lat_after = np.array([(reqs[i].done_time - reqs[i].arrival) * 1e3 for i in order[warm:]])
        print(f"[serve] {frac}x done: p99 {np.percentile(lat_after, 99):.1f} ms", file=sys.stderr,
              flush=True)
        runs[f"{frac}x"] = {"qps": round(frac * qps_sat, 1), "requests": N, "warmup": warm,
                            "latency_ms_p50": round(float(np.percentile(lat_after, 50)), 3),
                            "latency_ms_p99": round(float(np.percentile(lat_after, 99)), 3),
                            "throughput_req_per_s": round(st.completed / st.wall_s, 1),
                            "peak_arena_bytes": st.peak_bytes,
                            "status_nonzero": int(sum(r.status != 0 for r in reqs))}
        del lat
    # plain FIFO on the start of the 0.5x trace (bounded: it cannot keep up with that rate)
    arr = inputs.poisson_arrivals(N, 0.5 * qps_sat, 6)
    plain_n = min(N, args.plain_images)
    pst = serving.serve_plain(make(arr, range(plain_n)))
    # a served request equals the same image run alone
    check = make(np.zeros(8), range(8))
    serving.Server(1 << 30).run(check)
    same = sum(int(np.array_equal(r.features, anomps.extract_features(
        r.spec.pixels[None], r.spec.theta, r.spec.phi, r.spec.pairs, r.spec.chi,
        prec, per_layer=True)[0].cpu().numpy()[0])) for r in check)
    result = {
        "metric": "serving p50/p99 latency and throughput (Poisson arrivals, mixed p/L/chi)",
        "value": runs["0.9x"]["latency_ms_p99"], "unit": "ms (p99 at 0.9x saturation)",
        "n_gpus": 1, "higher_is_better": False,
        "dtype": "c64+f64svd" if prec == anomps.PREC_FP32 else "f64", "data": "synthetic",
        "config": {"workload": "single-image requests, p~U{7..16}, L~U{1..4}, "
                               "chi~U{2,4,8,16,32}, readout 84->784 for p=7",
                   "requests": N, "arena_bytes": arena, "layers_mode": args.layers_mode},
        "saturation": sat, "runs": runs,
        "plain_fifo_0.5x": {**pst.summary(), "requests": plain_n},
        "batch_invariance": {"checked": len(check), "identical": same},
        "tuning": tuning,
    }
    print(json.dumps(result))


def run_grid(args):
    """The 7x7 grid of depths and bond limits at batch 1024: images/s per (L, chi) cell and the
    max error of sampled images against the oracle (exact where chi >= 2^L, the truncated
    oracle otherwise)."""
    import torch
    from paper_2607_10280_amd import anomps, inputs
    from oracle import features as ofeat
    prec = anomps.PRECISIONS[args.precision]
    p, B = args.p, args.batch
    n = p * p
    x = inputs.blob_images(B, p, 2)
    pairs = inputs.neighbour_pairs(p)
    pd = torch.as_tensor(pairs, device="cuda")
    pix = torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    real = torch.float64 if prec == anomps.PREC_FP64 else torch.float32
    cells = []
    for L in (1, 2, 3, 4):
        th, ph = inputs.layer_angles(L, n, 3 + L)
        thd = torch.as_tensor(th, device="cuda").contiguous()
        phd = torch.as_tensor(ph, device="cuda").contiguous()
        for chi in (2, 4, 8, 16):
            b = anomps.new_batch(n, chi, L, B, prec)
            out = torch.empty((B, len(pairs), 15), dtype=real, device="cuda")

            def step():
                anomps.init_batch(b, pix)
                anomps.apply_layers(b, thd, phd)
                anomps.pauli_pair_expect(b, pd, out)
            step()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                step()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            o = out.cpu().numpy()
            sample = [0, B // 2, B - 1]
            if chi >= 2 ** L:
                ref = ofeat.exact_features(x[sample], th, ph, pairs)
                kind = "exact"
            else:
                ref = ofeat.truncated_features(x[sample], th, ph, pairs, chi)[0]
                kind = "truncated"
            print(f"[grid] L={L} chi={chi} {ms:.3f} ms", file=sys.stderr, flush=True)
            cells.append({"L": L, "chi": chi, "images_per_s": round(B / (ms * 1e-3), 1),
                          "ms": round(ms, 4), "max_abs_err": float(np.abs(o[sample] - ref).max()),
                          "oracle": kind, "status_nonzero": int(np.count_nonzero(b.status.cpu()))})
            del b, out
    head = next(c for c in cells if c["L"] == 4 and c["chi"] == 16)
    print(json.dumps({
        "metric": "Pauli-feature images/sec per (L, chi) cell, 7x7, batch 1024",
        "value": head["images_per_s"], "unit": "images/s (L=4, chi=16 cell)", "n_gpus": 1,
        "steps": args.steps, "higher_is_better": True, "data": "synthetic",
        "dtype": "c64+f64svd" if prec == anomps.PREC_FP32 else args.precision,
        "config": {"workload": f"{p}x{p} Gaussian blobs, L in 1..4 x chi in {{2,4,8,16}}",
                   "global_batch": B, "layers_mode": args.layers_mode}, "cells": cells}))


def run_paper(args):
    """The paper's own encoding circuit (H, R_Y(2 pi x - pi), brickwork CNOTs, repeated L times)
    on 7x7 images with its 156 neighbour pairs (horizontal, vertical, diagonal), batch 1024."""
    import torch
    from paper_2607_10280_amd import anomps, inputs
    from oracle import paper_ansatz as opa
    prec = anomps.PRECISIONS[args.precision]
    p, B, L, chi = args.p, args.batch, args.layers, args.chi
    n = p * p
    x = inputs.blob_images(B, p, 2)
    pairs = inputs.neighbour_pairs(p, diagonal=True)
    pix = torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    pd = torch.as_tensor(pairs, device="cuda")
    real = torch.float64 if prec == anomps.PREC_FP64 else torch.float32
    b = anomps.new_batch(n, chi, L, B, prec)
    out = torch.empty((B, len(pairs), 15), dtype=real, device="cuda")

    def step():
        anomps.init_zero(b)
        for _ in range(L):
            anomps.apply_layer_program(b, anomps.LAYER_H_RY_BRICKWORK, pixels=pix)
        anomps.pauli_pair_expect(b, pd, out)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    o = out.cpu().numpy()
    sample = [0, B // 2, B - 1]
    ref = opa.features(x[sample], L, pairs) if chi >= 2 ** L else opa.features(x[sample], L, pairs, chi)
    print(json.dumps({
        "metric": "Pauli-feature images/sec, the paper's encoding circuit, 7x7, 156 pairs",
        "value": round(B / (ms * 1e-3), 1), "unit": "images/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "dtype": "c64+f64svd" if prec == anomps.PREC_FP32 else args.precision, "data": "synthetic",
        "config": {"workload": f"{p}x{p} Gaussian blobs, H + R_Y(2 pi x - pi) + brickwork CNOTs, "
                               f"L={L}, chi={chi}, {len(pairs)} pairs", "global_batch": B,
                   "layers_mode": args.layers_mode},
        "max_abs_err": float(np.abs(o[sample] - ref).max()),
        "status_nonzero": int(np.count_nonzero(b.status.cpu()))}))


def run_chisweep(args):
    """Accuracy and cost against the bond limit (the analogue of the paper's chi study, §III on
    synthetic images): 7x7 blob images, L = 7 layers of the R_Y R_Z + CNOT-ladder circuit, chi in
    2..128.  chi = 128 = 2^L keeps every Schmidt value, so it is the exact result; each cell
    reports the mean and max feature error against it, the mean discarded weight per bond and
    the batch time.  The exact reference is checked against the oracle on one image."""
    import torch
    from paper_2607_10280_amd import anomps, inputs
    from oracle import features as ofeat
    prec = anomps.PRECISIONS[args.precision]
    p, L = args.p, 7
    B = args.batch
    n = p * p
    x = inputs.blob_images(B, p, 2)
    th, ph = inputs.layer_angles(L, n, 11)
    pairs = inputs.neighbour_pairs(p)
    pd = torch.as_tensor(pairs, device="cuda")
    pix = torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    thd = torch.as_tensor(th, device="cuda").contiguous()
    phd = torch.as_tensor(ph, device="cuda").contiguous()
    real = torch.float64 if prec == anomps.PREC_FP64 else torch.float32

    def run(chi, nb):
        b = anomps.new_batch(n, chi, L, nb, prec)
        out = torch.empty((nb, len(pairs), 15), dtype=real, device="cuda")
        te = torch.zeros((L, nb, n - 1), dtype=torch.float64, device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        anomps.init_batch(b, pix[:nb])
        for layer in range(L):
            anomps.apply_layer(b, thd[layer], phd[layer], te[layer])
        anomps.pauli_pair_expect(b, pd, out)
        e1.record()
        torch.cuda.synchronize()
        res = (out.double().cpu().numpy(), te.cpu().numpy(), int(np.count_nonzero(b.status.cpu())),
               e0.elapsed_time(e1))
        del b, out, te
        return res

    chis = (2, 4, 8, 16, 32, 64, 128)
    results = {}
    for chi in chis:
        run(chi, 4)  # code and allocator warm-up
        results[chi] = run(chi, B)
        print(f"[chisweep] chi={chi} {results[chi][3]:.1f} ms", file=sys.stderr, flush=True)
    ref = results[128][0]
    oracle_ref = ofeat.exact_features(x[:1], th, ph, pairs)
    cells = []
    for chi in chis:
        o, te, bad, ms = results[chi]
        err = np.abs(o - ref)
        cells.append({"chi": chi, "slot": anomps.slot_dim(n, chi, L), "ms": round(ms, 2),
                      "images_per_s": round(B / (ms * 1e-3), 1),
                      "mae": float(err.mean()), "max_abs_err": float(err.max()),
                      "mean_discarded_weight_per_bond": float(te.sum(axis=0).mean()),
                      "status_nonzero": bad})
    print(json.dumps({
        "metric": "feature error and cost against chi, 7x7, L=7 (chi=128 exact)",
        "value": cells[-1]["images_per_s"], "unit": "images/s (chi=128 cell)", "n_gpus": 1,
        "steps": 1, "higher_is_better": True, "data": "synthetic",
        "dtype": "c64+f64svd" if prec == anomps.PREC_FP32 else args.precision,
        "config": {"workload": f"{p}x{p} Gaussian blobs, R_Y R_Z + CNOT ladder, L={L}, "
                               f"{len(pairs)} H+V pairs", "global_batch": B,
                   "layers_mode": args.layers_mode},
        "reference_vs_oracle_max_abs_err": float(np.abs(ref[:1] - oracle_ref).max()),
        "cells": cells}))


def run_precision(args):
    """FP32 against split-BF16 contractions on 16x16 images (256 qubits), batch 256: for
    L in {1, 2} x chi in {16, 32, 64} the max abs error of sampled images against the FP64
    untruncated MPS oracle, with the batch time of each precision.  At these depths every bond
    is at most 2^L = 4 wide (the bond rule), so these cells run the vector contractions of
    slot 2 and 4, where the split-BF16 variant does not apply and both precisions give the same
    numbers; one more cell, L = 4 and chi = 16 (slot 16, every bond up to 16 wide), runs the
    matrix-core contractions where the two precisions differ."""
    import torch
    from paper_2607_10280_amd import anomps, inputs
    from oracle import features as ofeat
    p = 16
    B = args.batch if args.batch != 1024 else 256
    n = p * p
    x = inputs.blob_images(B, p, 21)
    pairs = inputs.neighbour_pairs(p)
    pd = torch.as_tensor(pairs, device="cuda")
    pix = torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    sample = [0, B // 3, (2 * B) // 3, B - 1]
    grid = [(L, chi) for L in (1, 2) for chi in (16, 32, 64)] + [(4, 16)]
    refs, angles = {}, {}
    for L in sorted({L for L, _ in grid}):
        th, ph = inputs.layer_angles(L, n, 22 + L)
        angles[L] = (torch.as_tensor(th, device="cuda").contiguous(),
                     torch.as_tensor(ph, device="cuda").contiguous())
        refs[L] = ofeat.exact_features(x[sample], th, ph, pairs)
    cells = []
    for L, chi in grid:
        thd, phd = angles[L]
        cell = {"L": L, "chi": chi, "slot": anomps.slot_dim(n, chi, L),
                "in_configured_grid": L <= 2}
        for name in ("fp32", "split_bf16"):
            prec = anomps.PRECISIONS[name]
            b = anomps.new_batch(n, chi, L, B, prec)
            out = torch.empty((B, len(pairs), 15), dtype=torch.float32, device="cuda")

            def step():
                anomps.init_batch(b, pix)
                anomps.apply_layers(b, thd, phd)
                anomps.pauli_pair_expect(b, pd, out)
            step()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                step()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            o = out.double().cpu().numpy()[sample]
            cell[name] = {"ms": round(ms, 3), "images_per_s": round(B / (ms * 1e-3), 1),
                          "max_abs_err": float(np.abs(o - refs[L]).max()),
                          "status_nonzero": int(np.count_nonzero(b.status.cpu()))}
            del b, out
        cells.append(cell)
        print(f"[precision] L={L} chi={chi} fp32 {cell['fp32']['max_abs_err']:.2e} "
              f"split {cell['split_bf16']['max_abs_err']:.2e}", file=sys.stderr, flush=True)
    worst = max(c["split_bf16"]["max_abs_err"] for c in cells)
    print(json.dumps({
        "metric": "max abs Pauli-expectation error vs the FP64 MPS oracle per (L, chi), FP32 and "
                  "split-BF16 contractions, 16x16",
        "value": worst, "unit": "abs error (split-BF16, worst cell)", "n_gpus": 1,
        "steps": args.steps, "higher_is_better": False, "data": "synthetic",
        "dtype": "c64+f64svd / split_bf16",
        "config": {"workload": f"{p}x{p} Gaussian blobs, L in {{1,2}} x chi in {{16,32,64}} "
                               f"(+ L=4, chi=16), {len(pairs)} H+V pairs", "global_batch": B,
                   "sampled_images": len(sample), "layers_mode": args.layers_mode},
        "cells": cells}))


# ----------------------------------------------------------------------------- main
def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)
    if args.workload != "headline":
        import torch  # the HIP runtime comes up through torch before the library is loaded
        torch.cuda.init()
        from paper_2607_10280_amd import anomps
        anomps.set_exact_layers(LAYER_MODES[args.layers_mode])
    if args.workload == "mixed":
        return run_mixed(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "grid":
        return run_grid(args)
    if args.workload == "paper":
        return run_paper(args)
    if args.workload == "chisweep":
        return run_chisweep(args)
    if args.workload == "precision":
        return run_precision(args)
    import torch
    from paper_2607_10280_amd import anomps, inputs, workload

    torch.cuda.set_device(0)
    dev = torch.device("cuda")
    prec = anomps.PRECISIONS[args.precision]
    p, B, L, chi = args.p, args.batch, args.layers, args.chi
    n = p * p
    x = inputs.blob_images(B, p, 2)
    th, ph = inputs.layer_angles(L, n, 3 + L)
    pairs = inputs.neighbour_pairs(p)
    m = len(pairs)
    out_dim = 784
    ra, rb, rd, rw, rbias = inputs.readout_params(m, out_dim, 8)
    anomps.validate_pairs(pairs, n)
    real = torch.float64 if prec == anomps.PREC_FP64 else torch.float32

    pix_d = torch.as_tensor(x, dtype=torch.float64, device=dev).contiguous()
    th_d = torch.as_tensor(th, dtype=torch.float64, device=dev).contiguous()
    ph_d = torch.as_tensor(ph, dtype=torch.float64, device=dev).contiguous()
    pairs_d = torch.as_tensor(pairs, device=dev).contiguous()
    T = lambda v: torch.as_tensor(v, dtype=real, device=dev).contiguous()
    A_d, B_d, D_d, W_d, bias_d = T(ra), T(rb), T(rd), T(rw), T(rbias)
    coeff_d = torch.empty((m, 16), dtype=real, device=dev)
    out_d = torch.empty((B, m, 15), dtype=real, device=dev)
    y_d = torch.empty((B, out_dim), dtype=real, device=dev)
    batch = anomps.new_batch(n, chi, L, B, prec)
    stream = torch.cuda.current_stream()

    def step(b=batch, pix=pix_d, out=out_d, y=y_d, events=None, th_=th_d, ph_=ph_d):
        def mark(name):
            if events is not None:
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(stream)
                events.append((name, ev))
        mark("start")
        anomps.init_batch(b, pix)
        mark("encode")
        anomps.apply_layers(b, th_, ph_)
        mark("layers")
        anomps.pauli_pair_expect(b, pairs_d, out)
        mark("measure")
        anomps.ano_coeffs(A_d, B_d, D_d, coeff_d)
        anomps.ano_readout(out, coeff_d, W_d, bias_d, y)
        mark("readout")

    if args.calibrate_copy_mb:
        src = torch.empty(args.calibrate_copy_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.counters_only:
        # a short program for rocprofv3 counter passes: the copy above, then K eager steps of
        # the headline batch, nothing else on the GPU
        anomps.set_exact_layers(LAYER_MODES[args.layers_mode])
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        print(f"[counters] {args.steps} steps of {args.layers_mode} layers done", flush=True)
        return

    def per_call(stepf, count):
        """Average duration of each call of the step (HIP events on the launch stream)."""
        per = {}
        for _ in range(count):
            evs = []
            stepf(events=evs)
            torch.cuda.synchronize()
            for (_, a), (name, b) in zip(evs[:-1], evs[1:]):
                per.setdefault(name, []).append(a.elapsed_time(b))
        return {k: float(np.mean(v)) for k, v in per.items()}

    def timed(mode_name, stepf, use_graph):
        """Warm-up, eager timing, then (unless disabled) a HIP-graph capture of the same step
        and its timed replays; returns a dict of timings and the outputs of the timed run."""
        anomps.set_exact_layers(LAYER_MODES[mode_name])
        for _ in range(args.warmup):
            stepf()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            stepf()
        e1.record(stream)
        torch.cuda.synchronize()
        eager_ms = e0.elapsed_time(e1) / args.steps
        eager_out, eager_y = out_d.cpu().numpy(), y_d.cpu().numpy()
        # The same step captured once as a HIP graph and replayed (no host launch gaps between
        # the step's kernels; the library's second stream for layer runs joins the capture
        # through its fork/join events).  Its outputs must equal the eager step's bit for bit.
        graph = None
        if use_graph:
            cs = torch.cuda.Stream()
            cs.wait_stream(stream)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=cs):
                stepf()
            graph.replay()
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            if graph is not None:
                graph.replay()
            else:
                stepf()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1) / args.steps
        outs = out_d.cpu().numpy()
        same = graph is None or (np.array_equal(outs, eager_out)
                                 and np.array_equal(y_d.cpu().numpy(), eager_y))
        avg = per_call(stepf, args.steps)
        del graph
        return {"ms": ms, "eager_ms": eager_ms, "wall": wall, "graph_same": bool(same),
                "graph": use_graph, "avg": avg, "out": outs,
                "status": batch.status.cpu().numpy()}

    # Pair-kernel launch schedule for this batch shape, chosen by measurement (every candidate
    # gives the same results bit for bit).
    tuning = {"pair_block_images": 64, "pair_waves_per_cu": 0, "source": "library default"}
    if anomps.slot_dim(n, chi, L) == 16 and args.tune:
        from paper_2607_10280_amd import autotune
        choice, tms, timings = autotune.tune_measure(n, chi, L, B, prec)
        tuning = {"pair_block_images": choice[0], "pair_waves_per_cu": choice[1],
                  "source": "autotune", "measure_ms": round(tms, 4), "candidates": len(timings)}
    mode = args.layers_mode
    head = timed(mode, step, not args.no_graph)
    avg = head["avg"]
    per_step = {"encode": avg["encode"], "layers": avg["layers"], "measure": avg["measure"],
                "readout": avg["readout"]}
    gpu_out = head["out"]

    # Plain method: one image per call, serial, on the same GPU (same layer mode).
    plain = anomps.new_batch(n, chi, L, 1, prec)
    lat = []
    o1 = torch.empty((1, m, 15), dtype=real, device=dev)
    y1 = torch.empty((1, out_dim), dtype=real, device=dev)
    for i in range(args.plain_images + 2):
        pix1 = pix_d[i % B: i % B + 1]
        torch.cuda.synchronize()
        t = time.perf_counter()
        step(plain, pix1, o1, y1)
        torch.cuda.synchronize()
        if i >= 2:
            lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat)

    def layer_roofline(n_, chi_, L_, B_, lay_ms, mode_name):
        """k_layer family priced against the FP64 vector peak with the algorithmic count of
        workload.layer_flops (nominal R-SVD count per truncating two-site split + Householder
        canonical sweep + contractions), per launch = one layer of the whole batch."""
        fl = sum(workload.layer_flops(n_, chi_, l, mode=mode_name, n_layers=L_)["total_fp64"]
                 for l in range(L_)) * B_
        ach = fl / (lay_ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4),
                "traffic": None, "kernel": "k_layer",
                "what": f"FP64 VALU, one mps_apply_layers call = {L_} k_layer launches (one per "
                        f"layer, one wavefront per image): canonical sweep + CNOT ladder with "
                        f"Jacobi SVD of every two-site matrix",
                "flops_per_launch": fl / L_, "launches": L_,
                "avg_launch_ms": round(lay_ms / L_, 4),
                "algorithmic_bytes_per_launch": round(
                    sum(workload.layer_bytes(n_, chi_, l, 8 if prec == anomps.PREC_FP64 else 4,
                                             mode=mode_name) for l in range(L_)) * B_ / L_)}

    # Measurement call (k_env16 + k_pairs16 at slot 16).
    meas_flops = (workload.env_flops(n, chi, L) + workload.pair_flops(n, chi, L, pairs)) * B
    if anomps.slot_dim(n, chi, L) == 16:
        meas_bound, meas_peak = "mfma", {anomps.PREC_FP64: PEAK_FP64_MFMA_TFLOPS,
                                         anomps.PREC_FP32: PEAK_FP32_MFMA_TFLOPS,
                                         anomps.PREC_SPLIT_BF16: PEAK_BF16_MFMA_TFLOPS}[prec]
    else:
        meas_bound = "alu"
        meas_peak = PEAK_FP64_TFLOPS if prec == anomps.PREC_FP64 else PEAK_FP32_VALU_TFLOPS
    ach_m = meas_flops / (per_step["measure"] * 1e-3) / 1e12
    traffic_m = _measured_traffic("measure")
    if (tuning["pair_block_images"], tuning["pair_waves_per_cu"]) != anomps.DEFAULT_MEASURE_SCHEDULE:
        traffic_m = None  # the counters were taken with the default schedule
    roof_measure = {"bound": meas_bound, "achieved": round(ach_m, 3), "peak": meas_peak,
                    "unit": "TFLOP/s", "frac": round(ach_m / meas_peak, 4),
                    "traffic": None if traffic_m is None else round(traffic_m),
                    "kernel": "k_env16+k_pairs16",
                    "what": "environments + pair contractions, per measurement call",
                    "flops_per_launch": meas_flops, "avg_launch_ms": round(per_step["measure"], 4)}
    if mode == "mpo":
        lay_fl = sum(workload.layer_flops(n, chi, l, n_layers=L)["total_fp64"] for l in range(L)) * B
        ach_l = lay_fl / (per_step["layers"] * 1e-3) / 1e12
        roof_layers = {"bound": "alu", "achieved": round(ach_l, 3), "peak": PEAK_FP64_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(ach_l / PEAK_FP64_TFLOPS, 4),
                       "traffic": None, "kernel": "k_mpo_run_core+k_mpo_run_ends",
                       "flops_per_launch": lay_fl, "avg_launch_ms": round(per_step["layers"], 4)}
    else:
        roof_layers = layer_roofline(n, chi, L, B, per_step["layers"], mode)
        traffic_l = _measured_traffic("layers_" + mode)
        if traffic_l is not None:
            roof_layers["traffic"] = round(traffic_l)
    dom = "layers" if per_step["layers"] >= per_step["measure"] else "measure"
    roofline = roof_layers if dom == "layers" else roof_measure

    result = {
        "metric": "Pauli-feature images/sec, 49q L=4 chi=16, batched vs plain; p99 latency; max abs err",
        "value": round(B / (head["ms"] * 1e-3), 1),
        "unit": "images/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 4),
        "timing": {"mode": "hip_graph" if head["graph"] else "eager",
                   "eager_ms_per_step": round(head["eager_ms"], 4),
                   "eager_images_per_s": round(B / (head["eager_ms"] * 1e-3), 1),
                   "graph_identical_to_eager": head["graph_same"]},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {anomps.PREC_FP32: "c64+f64svd", anomps.PREC_FP64: "f64",
                  anomps.PREC_SPLIT_BF16: "c64(split-bf16 mfma)+f64svd"}[prec],
        "data": "synthetic",
        "config": {"workload": f"{p}x{p} images ({n} qubits), Gaussian blobs, L={L}, chi={chi}, "
                               f"{m} H+V pairs x 15 Paulis, readout {m}->{out_dim}",
                   "global_batch": B, "precision": args.precision,
                   "layers": {"svd": "canonical sweep + CNOT ladder, FP64 Jacobi SVD of every "
                                     "two-site matrix (the method as stated)",
                              "qr": "exact Householder splits where nothing is discarded",
                              "mpo": "exact parity-operator contraction where nothing is "
                                     "discarded (shortcut)"}[mode]},
        "wall_s": round(head["wall"], 3),
        "per_step_ms": {k: round(v, 4) for k, v in per_step.items()},
        "plain": {"images_per_s": round(1e3 / float(np.mean(lat)), 1),
                  "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
                  "latency_ms_p99": round(float(np.percentile(lat, 99)), 4),
                  "images": int(len(lat))},
        "batched_latency_ms": round(head["ms"], 4),
        "status_nonzero": int(np.count_nonzero(head["status"])),
        "roofline": roofline,
        "roofline_layers": roof_layers,
        "roofline_measure": roof_measure,
        "tuning": tuning,
    }

    if mode != "mpo" and not args.no_shortcut:
        # The same batch with the exact shortcut for layers that keep every singular value
        # (chi >= 2^L: nothing is discarded, so the parity product operator gives the same
        # state without any SVD).  Reported beside the method, never as its value.
        sc = timed("mpo", step, not args.no_graph)
        result["exact_shortcut"] = {
            "layers": "parity product operator (site-local, exact) for every layer that keeps "
                      "all singular values; Jacobi SVD ladder elsewhere",
            "images_per_s": round(B / (sc["ms"] * 1e-3), 1), "ms_per_step": round(sc["ms"], 4),
            "per_step_ms": {k: round(v, 4) for k, v in sc["avg"].items()},
            "graph_identical_to_eager": sc["graph_same"],
            "max_abs_diff_vs_value": float(np.abs(sc["out"].astype(np.float64) - gpu_out).max())}

    if not args.no_trunc_cell and (p, L, chi) == (7, 4, 16):
        # A truncating cell of the same grid (chi = 8 < 2^L): the method with real truncation.
        tchi = 8
        tb = anomps.new_batch(n, tchi, L, B, prec)
        tstep = lambda events=None: step(b=tb, events=events)  # noqa: E731
        tc = timed(mode, tstep, False)
        result["truncating_cell"] = {
            "config": f"{p}x{p}, L={L}, chi={tchi}, batch {B}", "layers_mode": mode,
            "images_per_s": round(B / (tc["ms"] * 1e-3), 1), "ms_per_step": round(tc["ms"], 4),
            "per_step_ms": {k: round(v, 4) for k, v in tc["avg"].items()},
            "status_nonzero": int(np.count_nonzero(tb.status.cpu().numpy())),
            "roofline_layers": layer_roofline(n, tchi, L, B, tc["avg"]["layers"], mode)}
        del tb
    anomps.set_exact_layers(LAYER_MODES[mode])

    if not args.no_cpu_baseline:
        ref, cpu = cpu_baseline(x, th, ph, pairs, chi)
        err = np.abs(gpu_out[: len(ref)].astype(np.float64) - ref)
        result["max_abs_err"] = float(err.max())
        result["mae"] = float(err.mean())
        result["oracle_images_checked"] = int(len(ref))
        result["cpu_baseline"] = cpu
    print(json.dumps(result))


if __name__ == "__main__":
    main()
