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
# the factors a 1 GiB device copy reads), valid only for the kernel source they were taken on.
MEASURED_TRAFFIC = {
    # one mps_apply_layers call (all four layers): k_mpo_run_core + k_mpo_run_ends
    "layers": {"source": "paper_2607_10280_amd/csrc/layer.hip",
               "sha1": "0907698710102818f3f2e5ee101d2b7c003502cf",
               "bytes": ((2 * 5316.7 + 167936.0) + (2 * 4974.2 + 6260.0)) * 1024},
    # one measurement call: k_env16 + k_pairs16 (complex64, slot 16)
    "measure": {"source": "paper_2607_10280_amd/csrc/measure_mfma.hip",
                "sha1": "c6c9cc4b97a5bb9efc391a340bbd09b0ba75f440",
                "bytes": (2 * (194730.2 + 439745.1) + (204825.4 + 8715.8)) * 1024},
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
    ap.add_argument("--cpu-sample", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the eager step instead of its HIP-graph replay")
    ap.add_argument("--no-svd-compare", action="store_true",
                    help="skip the extra timing with every layer through the SVD ladder")
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
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a kernel of known "
                         "traffic, to scale hardware byte counters)")
    return ap.parse_args()


class _SkipSvd(Exception):
    pass


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


def cpu_baseline(x, th, ph, pairs, chi, sample):
    """The FP64 oracle (same truncation rule and chi) on `sample` images, one process per core."""
    cores = min(os.cpu_count() or 1, 16, sample)
    jobs = [(x[i], th, ph, pairs, chi) for i in range(sample)]
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores, initializer=_single_thread) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    feats = np.stack([r[0] for r in res])
    per_image = np.mean([r[1] for r in res])
    return feats, {"value": round(sample / wall, 3), "unit": "images/s", "cores": cores,
                   "kind": "oracle",
                   "sample": f"{sample} of the batch's images through the FP64 CPU oracle (numpy/"
                             f"LAPACK MPS, same chi and truncation rule), one process per core; "
                             f"{per_image:.2f} s per image per core"}


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
                               f"L~U{{1,2}}, chi=16, H+V pairs", "requests": N},
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
    runs = {}
    for frac in (0.5, 0.9):
        arr = inputs.poisson_arrivals(N, frac * qps_sat, 6)
        reqs = make(arr, range(N))
        st = srv.run(reqs)
        lat = np.array(st.latencies_ms)
        order = np.argsort([r.arrival for r in reqs])
        lat_after = np.array([(reqs[i].done_time - reqs[i].arrival) * 1e3 for i in order[warm:]])
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
                   "requests": N, "arena_bytes": arena},
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
                   "global_batch": B}, "cells": cells}))


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
                               f"L={L}, chi={chi}, {len(pairs)} pairs", "global_batch": B},
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
                               f"{len(pairs)} H+V pairs", "global_batch": B},
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
                   "sampled_images": len(sample)},
        "cells": cells}))


# ----------------------------------------------------------------------------- main
def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)
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

    def step(b=batch, pix=pix_d, out=out_d, y=y_d, events=None):
        def mark(name):
            if events is not None:
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(stream)
                events.append((name, ev))
        mark("start")
        anomps.init_batch(b, pix)
        mark("encode")
        anomps.apply_layers(b, th_d, ph_d)
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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # Eager: one stream-ordered call per step function.
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / args.steps
    eager_out = out_d.cpu().numpy()
    eager_y = y_d.cpu().numpy()

    # The same step captured once as a HIP graph and replayed (no host launch gaps between the
    # step's kernels; the library's second stream for layer runs joins the capture through its
    # fork/join events).  Its outputs must equal the eager step's bit for bit.
    graph = None
    if not args.no_graph:
        cs = torch.cuda.Stream()
        cs.wait_stream(stream)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=cs):
            step()
        graph.replay()
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        if graph is not None:
            graph.replay()
        else:
            step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = e0.elapsed_time(e1) / args.steps
    status = batch.status.cpu().numpy()
    gpu_out = out_d.cpu().numpy()
    graph_same = graph is None or (np.array_equal(gpu_out, eager_out)
                                   and np.array_equal(y_d.cpu().numpy(), eager_y))

    # Per-call durations (HIP events on the launch stream), same steps again.
    per = {}
    for _ in range(args.steps):
        evs = []
        step(events=evs)
        torch.cuda.synchronize()
        for (_, a), (name, b) in zip(evs[:-1], evs[1:]):
            per.setdefault(name, []).append(a.elapsed_time(b))
    avg = {k: float(np.mean(v)) for k, v in per.items()}   # ms per call
    per_step = {"encode": avg["encode"], "layers": avg["layers"], "measure": avg["measure"],
                "readout": avg["readout"]}

    # Plain method: one image per call, serial, on the same GPU.
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

    # The same batch with every layer through the canonical sweep + Jacobi SVD ladder (by
    # default a layer that keeps every singular value is applied site by site as the parity
    # product operator).
    anomps.set_exact_layers(anomps.EXACT_SVD)
    try:
        if args.no_svd_compare:
            raise _SkipSvd
        step()
        torch.cuda.synchronize()
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record()
        for _ in range(args.steps):
            step()
        s1.record()
        torch.cuda.synchronize()
        svd_ms = s0.elapsed_time(s1) / args.steps
        svd_err = float(np.abs(out_d.cpu().numpy().astype(np.float64) - gpu_out).max())
    except _SkipSvd:
        svd_ms = svd_err = None
    finally:
        anomps.set_exact_layers(anomps.EXACT_MPO)
    exact = [l for l in range(L) if workload.layer_keeps_all(n, chi, l)]

    # Roofline of the dominant kernel family.
    lay_flops = sum(workload.layer_flops(n, chi, l, n_layers=L)["total_fp64"] for l in range(L)) * B
    meas_flops = (workload.env_flops(n, chi, L) + workload.pair_flops(n, chi, L, pairs)) * B
    # Slot-16 measurement runs on matrix cores in every precision (FP64, FP32, or bf16 with
    # three bf16 products per FP32 product: the split variant is priced against the bf16 peak
    # with the algorithmic, FP32-product count); narrower slots on the vector units.
    if anomps.slot_dim(n, chi, L) == 16:
        meas_bound, meas_peak = "mfma", {anomps.PREC_FP64: PEAK_FP64_MFMA_TFLOPS,
                                         anomps.PREC_FP32: PEAK_FP32_MFMA_TFLOPS,
                                         anomps.PREC_SPLIT_BF16: PEAK_BF16_MFMA_TFLOPS}[prec]
    else:
        meas_bound = "alu"
        meas_peak = PEAK_FP64_TFLOPS if prec == anomps.PREC_FP64 else PEAK_FP32_VALU_TFLOPS
    cand = {
        "layers": (lay_flops, avg["layers"], "alu", PEAK_FP64_TFLOPS,
                   "FP64 VALU, per mps_apply_layers call (all L layers): gates + parity-operator "
                   "contraction with exact end carries for layers that keep every singular "
                   "value, else Jacobi SVD (nominal R-SVD count) + canonical sweep"),
        "measure": (meas_flops, avg["measure"], meas_bound, meas_peak,
                    "environments + pair contractions, per measurement call"),
    }
    dom = max(cand, key=lambda k: per_step[k])
    fl, dur_ms, bound, peak, what = cand[dom]
    achieved = fl / (dur_ms * 1e-3) / 1e12
    traffic = _measured_traffic(dom)
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4),
                "traffic": None if traffic is None else round(traffic),
                "kernel": dom, "what": what, "flops_per_launch": fl,
                "avg_launch_ms": round(dur_ms, 4)}
    if dom == "layers":
        alg = sum(workload.layer_bytes(n, chi, l, 8 if prec == anomps.PREC_FP64 else 4)
                  for l in range(L)) * B
        roofline["algorithmic_bytes_per_launch"] = round(alg)

    result = {
        "metric": "Pauli-feature images/sec, 49q L=4 chi=16, batched vs plain; p99 latency; max abs err",
        "value": round(args.steps * B / (ms_per_step * args.steps * 1e-3), 1),
        "unit": "images/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "timing": {"mode": "eager" if graph is None else "hip_graph",
                   "eager_ms_per_step": round(eager_ms, 4),
                   "eager_images_per_s": round(B / (eager_ms * 1e-3), 1),
                   "graph_identical_to_eager": bool(graph_same)},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {anomps.PREC_FP32: "c64+f64svd", anomps.PREC_FP64: "f64",
                  anomps.PREC_SPLIT_BF16: "c64(split-bf16 mfma)+f64svd"}[prec],
        "data": "synthetic",
        "config": {"workload": f"{p}x{p} images ({n} qubits), Gaussian blobs, L={L}, chi={chi}, "
                               f"{m} H+V pairs x 15 Paulis, readout {m}->{out_dim}",
                   "global_batch": B, "precision": args.precision},
        "wall_s": round(wall, 3),
        "per_step_ms": {k: round(v, 4) for k, v in per_step.items()},
        "plain": {"images_per_s": round(1e3 / float(np.mean(lat)), 1),
                  "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
                  "latency_ms_p99": round(float(np.percentile(lat, 99)), 4),
                  "images": int(len(lat))},
        "batched_latency_ms": round(ms_per_step, 4),
        "status_nonzero": int(np.count_nonzero(status)),
        "roofline": roofline,
        "exact_layers": {"site_local_layers": exact, "svd_every_layer": None if svd_ms is None else {
            "images_per_s": round(B / (svd_ms * 1e-3), 1), "ms_per_step": round(svd_ms, 4),
            "max_abs_diff_vs_default": svd_err}},
    }
    if not args.no_cpu_baseline:
        ref, cpu = cpu_baseline(x, th, ph, pairs, chi, min(args.cpu_sample, B))
        err = np.abs(gpu_out[: len(ref)].astype(np.float64) - ref)
        result["max_abs_err"] = float(err.max())
        result["mae"] = float(err.mean())
        result["cpu_baseline"] = cpu
    print(json.dumps(result))


if __name__ == "__main__":
    main()
