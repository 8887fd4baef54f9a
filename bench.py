#!/usr/bin/env python3
"""Benchmark: batched AMI evaluation of an order-4 Hubbard self-energy on one MI355X.

Workload (one step = one pass of the evaluation path over one batch):
  a seeded random order-4 self-energy topology (4 nested Matsubara sums, 7
  propagators) constructed once by the library (outside the timed region);
  10^6 momentum samples k uniform in the Brillouin zone, resident in HBM;
  energies E_j = 2t(cos K_jx + cos K_jy) + mu computed in the kernel (t = 1,
  mu = 0, q = (pi/2, pi/2)); beta = 5; one external Matsubara frequency i pi/beta.
  The step evaluates out[N_F, N_E] and its Monte-Carlo row sum out_sum[N_F].

Metric: term-evaluations/s = T * N_E * N_F / (seconds per step), T the number
of canonical flat terms.  Also reported: the forward kernel's algorithmic FP64
FLOP rate against the FP64 vector peak, and the oracle timed on host cores.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "term-evaluations/sec (FP64, order-4 self-energy) + % FP64 peak; fwd vs fwd+adjoint"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--diagram", type=int, default=1, help="seed index of the topology")
    ap.add_argument("--n-e", type=int, default=1_000_000)
    ap.add_argument("--beta", type=float, default=5.0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target duration of the oracle CPU baseline (0 disables it)")
    return ap.parse_args()


def cpu_baseline(d, k_all, q, beta, t, mu, w, target_s):
    """The oracle (float64 mode, as it stands) on a bounded slice of the same
    samples, with a process pool over the host cores this process may use."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor

    from oracle.construct import canonical, construct
    terms = canonical(construct(d.alpha, d.eps, d.n_int, d.fermionic))
    cores = min(len(os.sched_getaffinity(0)), 16)
    # calibrate on one chunk in this process
    chunk = 2000
    t0 = time.perf_counter()
    _oracle_chunk((terms, d, k_all[:chunk], q, beta, t, mu, w))
    dt = time.perf_counter() - t0
    per_sample = dt / chunk
    n = int(min(len(k_all), max(chunk, target_s * cores / per_sample)))
    n = (n // chunk) * chunk
    jobs = [(terms, d, k_all[i:i + chunk], q, beta, t, mu, w) for i in range(0, n, chunk)]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores) as ex:
        list(ex.map(_oracle_chunk, jobs))
    el = time.perf_counter() - t0
    return {"value": len(terms) * n * len(w) / el, "unit": "term-evals/s", "cores": cores,
            "kind": "oracle",
            "sample": f"first {n} of the same momentum samples (float64 oracle, "
                      f"{len(jobs)} chunks of {chunk} over {cores} processes), {el:.1f} s"}


def _oracle_chunk(args):
    import numpy as np

    from oracle.evaluate import energies_from_k, evaluate_terms
    terms, d, k, q, beta, t, mu, w = args
    E = energies_from_k(d.alpha, k, q, t, mu, dtype=np.float64)
    return evaluate_terms(terms, d.n_int, E, w, beta, dtype=np.float64)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the evaluation shards over samples with no exchange but the row-sum "
              "all-reduce; that path is not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2311_17189_amd as amd
    from ami_inputs import DEFAULT_Q, k_samples, matsubara_freqs, random_self_energy
    from paper_2311_17189_amd import roofline as rl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d = random_self_energy(args.order, (0, args.order, args.diagram))
    t0 = time.perf_counter()
    terms = amd.Terms.from_diagram(d)
    construct_ms = (time.perf_counter() - t0) * 1e3
    info = terms.info()
    terms.upload()
    st = rl.structure_from_canonical(terms.canonical())

    hop_t, mu = 1.0, 0.0
    q = np.array(DEFAULT_Q)
    n_e = args.n_e
    k_host = k_samples(n_e, d.n_int, seed=(100, args.order, args.diagram))
    k = torch.from_numpy(k_host).to(dev)
    w_host = matsubara_freqs(1, args.beta)
    w = torch.from_numpy(w_host).to(dev)
    n_f = w.shape[0]
    out = torch.empty((n_f, n_e), dtype=torch.complex128, device=dev)
    out_sum = torch.empty((n_f,), dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream()

    def fwd():
        amd.evaluate_hubbard(terms, k, q, hop_t, mu, w, args.beta, want_sum=True,
                             out=out, out_sum=out_sum, stream=stream)

    for _ in range(args.warmup):
        fwd()
    torch.cuda.synchronize()

    # timed region: K steps, with events around every launch on the launch stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for i in range(args.steps):
        ev[i][0].record(stream)
        fwd()
        ev[i][1].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = start.elapsed_time(stop) / args.steps
    fwd_ms = sum(a.elapsed_time(b) for a, b in ev) / args.steps

    te = float(info["T"]) * n_e * n_f
    value = te / (ms_step * 1e-3)
    fl = rl.forward_flops(st, n_e, n_f, d.alpha)
    achieved = fl["total"] / (fwd_ms * 1e-3)
    bytes_fwd = rl.forward_bytes(n_e, n_f, 2 * d.n_int, True)

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "term-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"order-{args.order} Hubbard self-energy (seeded topology {args.diagram}), "
                        f"{n_e} k-samples, beta={args.beta}, 1 Matsubara frequency, energies from "
                        "momenta in-kernel, out[N_F,N_E] + row sum",
            "order": args.order, "terms": info["T"], "distinct_leaves": info["L"],
            "distinct_denominators": info["D"], "groups": info["G"], "n_e": n_e, "n_f": n_f,
            "beta": args.beta, "t": hop_t, "mu": mu, "q": [float(x) for x in q],
            "diagram_seed": [0, args.order, args.diagram],
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": rl.PEAK_FP64_VECTOR / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / rl.PEAK_FP64_VECTOR,
            "traffic": None,
            "kernel": "ami_fwd_kernel<8,true> (+ row-sum kernel in the same interval)",
            "flops_per_launch": fl["total"],
            "flops_per_sample": fl["per_sample"],
            "flops_per_point": fl["per_point"],
            "kernel_ms": fwd_ms,
            "hbm_gbps_compulsory": bytes_fwd / (fwd_ms * 1e-3) / 1e9,
        },
        "construct_ms": construct_ms,
        "wall_s": wall,
    }
    if args.cpu_seconds > 0:
        res["cpu_baseline"] = cpu_baseline(d, k_host, q, args.beta, hop_t, mu, w_host,
                                           args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
