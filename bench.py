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
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch from two rocprofv3 counter runs (FETCH_SIZE x 2.0 and WRITE_SIZE x 1.0,
# the factors a 1 GiB device copy reads), valid only for the kernel source they were taken on.
MEASURED_TRAFFIC = {
    "layer": {"source": "paper_2607_10280_amd/csrc/layer.hip",
              "sha1": "cddcf1b8bec629f1e182470fe45463770fe77fda",
              "bytes": (2 * 37032.8 + 73786.8) * 1024},
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
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32"])
    ap.add_argument("--plain-images", type=int, default=64)
    ap.add_argument("--cpu-sample", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a kernel of known "
                         "traffic, to scale hardware byte counters)")
    return ap.parse_args()


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


# ----------------------------------------------------------------------------- main
def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)
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
        for layer in range(L):
            anomps.apply_layer(b, th_d[layer], ph_d[layer])
            mark("layer")
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
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = e0.elapsed_time(e1) / args.steps
    status = batch.status.cpu().numpy()
    gpu_out = out_d.cpu().numpy()

    # Per-call durations (HIP events on the launch stream), same steps again.
    per = {}
    for _ in range(args.steps):
        evs = []
        step(events=evs)
        torch.cuda.synchronize()
        for (_, a), (name, b) in zip(evs[:-1], evs[1:]):
            per.setdefault(name, []).append(a.elapsed_time(b))
    avg = {k: float(np.mean(v)) for k, v in per.items()}   # ms per call (layer: per layer call)
    per_step = {"encode": avg["encode"], "layers": avg["layer"] * L, "measure": avg["measure"],
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

    # Roofline of the dominant kernel family.
    lay_flops = sum(workload.layer_flops(n, chi, l)["total_fp64"] for l in range(L)) * B
    meas_flops = (workload.env_flops(n, chi, L) + workload.pair_flops(n, chi, L, pairs)) * B
    mfma = prec == anomps.PREC_FP32 and anomps.slot_dim(n, chi, L) == 16
    cand = {
        "layer": (lay_flops / L, avg["layer"], "alu", PEAK_FP64_TFLOPS,
                  "FP64 VALU: Jacobi SVD + canonical sweep, per layer launch (nominal R-SVD count)"),
        "measure": (meas_flops, avg["measure"], "mfma" if mfma else "alu",
                    PEAK_FP64_TFLOPS if prec == anomps.PREC_FP64 else
                    (PEAK_FP32_MFMA_TFLOPS if mfma else PEAK_FP32_VALU_TFLOPS),
                    "environments + pair contractions, per measurement call"),
    }
    dom = max(cand, key=lambda k: per_step["layers" if k == "layer" else k])
    fl, dur_ms, bound, peak, what = cand[dom]
    achieved = fl / (dur_ms * 1e-3) / 1e12
    traffic = _measured_traffic(dom)
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4),
                "traffic": None if traffic is None else round(traffic),
                "kernel": dom, "what": what, "flops_per_launch": fl,
                "avg_launch_ms": round(dur_ms, 4)}
    if dom == "layer":
        alg = sum(workload.layer_bytes(n, chi, l, 8 if prec == anomps.PREC_FP64 else 4)
                  for l in range(L)) / L * B
        roofline["algorithmic_bytes_per_launch"] = round(alg)

    result = {
        "metric": "Pauli-feature images/sec, 49q L=4 chi=16, batched vs plain; p99 latency; max abs err",
        "value": round(args.steps * B / (ms_per_step * args.steps * 1e-3), 1),
        "unit": "images/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64+f64svd" if prec == anomps.PREC_FP32 else "f64",
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
