#!/usr/bin/env python3
"""Benchmark: batched AMI evaluation of an order-4 Hubbard self-energy on one MI355X.

Workload (one step = one pass of the evaluation path over one batch):
  a seeded random order-4 self-energy topology (4 nested Matsubara sums, 7
  propagators) constructed once by the library (outside the timed region);
  10^6 momentum samples k uniform in the Brillouin zone, resident in HBM;
  energies E_j = 2t(cos K_jx + cos K_jy) + mu computed in the kernel (t = 1,
  mu = 0, q = (pi/2, pi/2)); beta = 5; one external Matsubara frequency i pi/beta.
  The step evaluates out[N_F, N_E] and its Monte-Carlo row sum out_sum[N_F]
  (forward) and the gradients of the summed integrand with respect to every
  momentum component, mu, t, beta and the external frequency (adjoint), in one
  pass of the adjoint kernel with values.  The kernels are the diagram's own
  specialized ones (generated and compiled at run time, before the timed
  region).  Each timed step is one replay of a HIP graph holding the step's
  launches (captured once after the warm-up; --no-graph times plain
  launches); the same steps as plain launches are reported beside it.

Metric: term-evaluations/s = T * N_E * N_F / (seconds per step), T the number
of canonical flat terms; the forward alone, the table-driven (packed) kernels
and the plain double-table kernel are reported beside it.  Also reported: the
algorithmic FP64 FLOP rate of the dominant kernel (timed alone with HIP events
on its stream) against the FP64 vector peak, and the oracle timed on host
cores.  Prints one JSON line.
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
    ap.add_argument("--no-graph", action="store_true",
                    help="time the steps as plain launches instead of HIP graph replays")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the persistent mixed-diagram batch section")
    ap.add_argument("--batch-n-e", type=int, default=200_000)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (C1-C3, large solutions)")
    ap.add_argument("--sections", default="next,configs,large,batch",
                    help="sections beside the headline step, comma-separated: next (the rows beyond the "
                         "main path), configs (C1-C3), large (the adjoint of large solutions), batch")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB device to device (a plain copy "
                         "kernel of known size, to scale hardware byte counters)")
    return ap.parse_args()


def cpu_baseline(d, k_all, q, beta, t, mu, w, target_s):
    """The oracle, as it stands, on bounded slices of the same samples, over
    the host cores this process may use (a process pool, capped at 16):
    float64 values (its plain evaluation of the flat terms, energies from
    momenta) on all cores -- the reported value -- and on one core, and the
    whole step (float64 values and the analytic gradients of the summed
    integrand with the momentum chain rule, in long double) on all cores;
    each of these about target_s / 3 seconds.  Beside them: the oracle's own
    long-double values on 10^4 samples (one process) and its construction time
    for the diagram."""
    from oracle.construct import canonical, construct
    t0 = time.perf_counter()
    terms = canonical(construct(d.alpha, d.eps, d.n_int, d.fermionic))
    construct_ms = (time.perf_counter() - t0) * 1e3
    cores = min(len(os.sched_getaffinity(0)), 16)
    each = target_s / 3.0
    chunk = 1000
    out = {}
    for key, fn, n_proc in (("values_f64", _oracle_values, cores), ("values_f64_1core", _oracle_values, 1),
                            ("step", _oracle_step, cores)):
        t0 = time.perf_counter()                     # calibrate on one chunk in this process
        fn((terms, d, k_all[:chunk], q, beta, t, mu, w))
        per_sample = (time.perf_counter() - t0) / chunk
        n = int(min(len(k_all), max(chunk, each * n_proc / per_sample)))
        n = (n // chunk) * chunk
        jobs = [(terms, d, k_all[i:i + chunk], q, beta, t, mu, w) for i in range(0, n, chunk)]
        t0 = time.perf_counter()
        if n_proc > 1:
            from concurrent.futures import ProcessPoolExecutor
            with ProcessPoolExecutor(max_workers=n_proc) as ex:
                list(ex.map(fn, jobs))
        else:
            for j in jobs:
                fn(j)
        el = time.perf_counter() - t0
        out[key] = {"term_evals_per_s": len(terms) * n * len(w) / el, "samples": n, "processes": n_proc,
                    "seconds": el}
    # the oracle's own precision (long double) on 10^4 samples, one process
    n_ld = min(len(k_all), 10_000)
    t0 = time.perf_counter()
    for i in range(0, n_ld, chunk):
        _oracle_values_ld((terms, d, k_all[i:i + chunk], q, beta, t, mu, w))
    el = time.perf_counter() - t0
    out["values_longdouble_1core"] = {"term_evals_per_s": len(terms) * n_ld * len(w) / el, "samples": n_ld,
                                      "processes": 1, "seconds": el}
    v = out["values_f64"]
    return {"value": v["term_evals_per_s"], "unit": "term-evals/s", "cores": cores, "kind": "oracle",
            "sample": f"first {v['samples']} of the same momentum samples, float64 values of the flat terms "
                      f"(energies from momenta), {v['samples'] // chunk} chunks of {chunk} over {cores} "
                      f"processes, {v['seconds']:.1f} s",
            "values_f64_1core": out["values_f64_1core"],
            "values_longdouble_1core": out["values_longdouble_1core"],
            "construct_ms": construct_ms,
            "step_values_and_gradients": dict(out["step"], note="float64 values and long-double analytic "
                                                                "gradients w.r.t. k, mu, t, beta, w")}


def _oracle_values(args):
    import numpy as np

    from oracle.evaluate import energies_from_k, evaluate_terms
    terms, d, k, q, beta, t, mu, w = args
    E = energies_from_k(d.alpha, k, q, t, mu, dtype=np.float64)
    return evaluate_terms(terms, d.n_int, E, w, beta, dtype=np.float64).sum(axis=1)


def _oracle_values_ld(args):
    from oracle.evaluate import energies_from_k, evaluate_terms
    terms, d, k, q, beta, t, mu, w = args
    E = energies_from_k(d.alpha, k, q, t, mu)
    return evaluate_terms(terms, d.n_int, E, w, beta).sum(axis=1)


def _oracle_step(args):
    import numpy as np

    from oracle.evaluate import energies_from_k, evaluate_terms, gradients, momentum_gradients
    terms, d, k, q, beta, t, mu, w = args
    E = energies_from_k(d.alpha, k, q, t, mu, dtype=np.float64)
    vals = evaluate_terms(terms, d.n_int, E, w, beta, dtype=np.float64)
    cot = np.ones((len(w), len(k)), dtype=np.complex128)          # row-sum cotangent of the step
    dE, db, dw = gradients(terms, d.n_int, E, w, beta, cot)
    dk, dmu, dt = momentum_gradients(d.alpha, k, q, t, mu, dE)
    return vals.sum(axis=1), dk, dmu, dt, db, dw


def kernel_source_hash() -> str:
    """sha256 over the HIP/C++ sources of the library: hardware byte counters
    recorded for one build are reported only while the sources are unchanged."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2311_17189_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode())
                h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary (profiles/traffic.json), or None when absent or
    taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    entry = rec.get("kernels", {}).get(kernel, {}).get(workload)
    if not entry:
        return None
    return entry["fetch_bytes"] + entry["write_bytes"]


def batch_section(args, torch, dev):
    """Mixed batch: 64 seeded diagrams of orders 2-6 (13/13/13/13/12), 16
    external Matsubara frequencies and N samples each, one graph launch with
    the autotuned choice (the specialized kernels as recorded launches or in
    persistent kernels, or the persistent packed kernels, each with its
    tilings), against the best persistent batches of either kind and 64
    separate launches of the specialized, the packed and the plain kernels."""
    import numpy as np

    import paper_2311_17189_amd as amd
    from ami_inputs import DEFAULT_Q, k_samples, matsubara_freqs, random_self_energy
    from paper_2311_17189_amd.autotune import autotune, time_batch

    orders = [2] * 13 + [3] * 13 + [4] * 13 + [5] * 13 + [6] * 12
    beta, n_f, n_e = 5.0, 16, args.batch_n_e
    w = torch.from_numpy(matsubara_freqs(n_f, beta)).to(dev)
    items, seen = [], {}
    for order in orders:
        i = seen.get(order, 0)
        seen[order] = i + 1
        d = random_self_energy(order, (5, order, i))
        T = amd.Terms.from_diagram(d)
        k = torch.from_numpy(k_samples(n_e, d.n_int, seed=(200, order, i))).to(dev)
        items.append({"terms": T, "k": k, "q": list(DEFAULT_Q), "t": 1.0, "mu": 0.0, "ext_freqs": w,
                      "beta": beta,
                      "out": torch.empty((n_f, n_e), dtype=torch.complex128, device=dev),
                      "out_sum": torch.empty((n_f,), dtype=torch.complex128, device=dev)})
    term_counts = [it["terms"].info()["T"] for it in items]
    te = float(sum(term_counts)) * n_e * n_f
    # compile (or load from the disk cache) every diagram's specialized
    # kernels, several at a time, before tuning
    from concurrent.futures import ThreadPoolExecutor

    def _spec(it):
        try:
            it["terms"].specialize(momentum=True)
        except amd.AmiError:
            pass                               # that item stays on the packed kernels
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=8) as pool:
        list(pool.map(_spec, items))
    specialize_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    best, timings = autotune(items, reps=3)
    tune_s = time.perf_counter() - t0
    b = amd.Batch(items, best)
    batch_ms = time_batch(b, reps=5)
    info = b.info()
    stream = torch.cuda.current_stream()

    def separate():
        for it in items:
            amd.evaluate_hubbard(it["terms"], it["k"], it["q"], it["t"], it["mu"], w, beta,
                                 want_sum=True, out=it["out"], out_sum=it["out_sum"], stream=stream)

    def timed(fn, reps=3):
        _warm(torch, fn)
        ts = []
        for _ in range(reps):
            a0 = torch.cuda.Event(enable_timing=True)
            a1 = torch.cuda.Event(enable_timing=True)
            a0.record(stream)
            fn()
            a1.record(stream)
            torch.cuda.synchronize()
            ts.append(a0.elapsed_time(a1))
        return sorted(ts)[len(ts) // 2]

    auto_ms = timed(separate)               # AUTO: the specialized kernels, one launch after another
    for it in items:
        it["terms"].set_variant(amd.VARIANT_PACKED)
    sep_ms = timed(separate)
    # the persistent packed batch (the kernels every item had before the
    # specialized ones), best of the packed tilings the autotuner timed
    packed_best = min(((v, k) for k, v in timings.items() if '"kernels": 1' in k), default=(None, None))
    # the specialized tile functions inside persistent kernels, best of the tilings timed
    pspec_best = min(((v, k) for k, v in timings.items() if '"kernels": 2' in k), default=(None, None))
    for it in items:
        it["terms"].set_variant(amd.VARIANT_TABLES)
    plain_ms = timed(separate)
    for it in items:
        it["terms"].set_variant(amd.VARIANT_AUTO)
    return {
        "workload": f"64 seeded self-energy diagrams, orders 2-6 (13/13/13/13/12), {n_f} Matsubara "
                    f"frequencies, {n_e} k-samples each, beta={beta}, out[N_F,N_E] + row sums",
        "terms_min": min(term_counts), "terms_max": max(term_counts), "terms_total": sum(term_counts),
        "term_evals": te,
        "batch_ms": batch_ms, "batch_term_evals_per_s": te / (batch_ms * 1e-3),
        "separate_auto_ms": auto_ms, "separate_auto_term_evals_per_s": te / (auto_ms * 1e-3),
        "packed_batch_ms": packed_best[0], "packed_batch_tuning": packed_best[1],
        "persistent_specialized_ms": pspec_best[0], "persistent_specialized_tuning": pspec_best[1],
        "separate_packed_ms": sep_ms, "separate_packed_term_evals_per_s": te / (sep_ms * 1e-3),
        "separate_plain_ms": plain_ms, "separate_plain_term_evals_per_s": te / (plain_ms * 1e-3),
        "tuning": best, "tuning_candidates": len(timings), "tuning_s": tune_s, "info": info,
        "specialize_s": specialize_s,
    }


def _warm(torch, fn, calls=1, seconds=0.1):
    """Untimed calls right before a timed loop: at least `calls` of them and
    at least `seconds` of work, so that timing does not start on a clock still
    ramping up after idle set-up."""
    n, t_end = 0, time.perf_counter() + seconds
    while n < calls or time.perf_counter() < t_end:
        fn()
        n += 1
        if n % 10 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()


def _timed_kernel(torch, amd, stream, fn, reps):
    """(ms per call between stream events, mean kernel ms from the library's
    dispatch events) over `reps` calls after the warm-up of _warm."""
    _warm(torch, fn)
    amd.kernel_timer_start(reps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    ks = amd.kernel_timer_stop()
    return e0.elapsed_time(e1) / reps, sum(ks) / len(ks)


def _median_ms(torch, stream, fn, reps=25):
    """Median over `reps` calls, each bracketed by its own pair of stream
    events, after the warm-up of _warm; also the minimum."""
    _warm(torch, fn)
    ts = []
    for _ in range(reps):
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        fn()
        a1.record(stream)
        a1.synchronize()
        ts.append(a0.elapsed_time(a1))
    ts.sort()
    return ts[len(ts) // 2], ts[0]


def configs_section(args, torch, dev, stream):
    """The workloads beside the headline one, each timed as the median of 25
    individually timed calls: C1, the order-2 self-energy of Sec. 5.1.1 at
    10^4 k-samples (a latency); C2, seeded order-3 and order-4 topologies at
    beta = 2, 5, 10 and 10^6 k-samples (forward, and the value-and-gradient
    step); C3, an order-4 topology on the 256-point real-frequency grid
    omega + 0.05i, omega in [-6, 6], at 10^6 k-samples (out is 4.1 GB: HBM
    rate and FP64 fraction); C4, the C3 topology's adjoint with a per-sample
    cotangent (grad_out) at 10^6 k-samples."""
    import numpy as np

    import paper_2311_17189_amd as amd
    from ami_inputs import DEFAULT_Q, k_samples, matsubara_freqs, order2_example, random_self_energy, real_freqs
    from paper_2311_17189_amd import roofline as rl

    q = np.array(DEFAULT_Q)
    res = {}

    def prepare(d, n_e, seed, freqs):
        T = amd.Terms.from_diagram(d)
        T.upload()
        T.specialize(momentum=True)
        st = rl.structure_from_canonical(T.canonical())
        k = torch.from_numpy(k_samples(n_e, d.n_int, seed=seed)).to(dev)
        w = torch.from_numpy(freqs).to(dev)
        n_f = w.shape[0]
        out = torch.empty((n_f, n_e), dtype=torch.complex128, device=dev)
        osum = torch.empty((n_f,), dtype=torch.complex128, device=dev)
        gs = torch.ones((n_f,), dtype=torch.complex128, device=dev)
        return T, st, k, w, out, osum, gs

    def fwd_and_step(d, n_e, seed, beta, freqs, with_step=True):
        T, st, k, w, out, osum, gs = prepare(d, n_e, seed, freqs)
        n_f = w.shape[0]
        te = float(st.T) * n_e * n_f
        fwd = lambda: amd.evaluate_hubbard(T, k, q, 1.0, 0.0, w, beta, want_sum=True, out=out, out_sum=osum,
                                           stream=stream)
        f_med, f_min = _median_ms(torch, stream, fwd)
        fv = amd.last_variant()
        ffl = rl.specialized_forward_flops(st, n_e, n_f, d.alpha)["total"]
        row = {"terms": st.T, "n_e": n_e, "n_f": n_f, "beta": beta,
               "fwd_ms_median": f_med, "fwd_ms_min": f_min, "fwd_kernel": fv,
               "fwd_term_evals_per_s": te / (f_med * 1e-3),
               "fwd_frac_fp64_peak": ffl / (f_med * 1e-3) / rl.PEAK_FP64_VECTOR}
        if with_step:
            g = [None]

            def step():
                g[0] = amd.evaluate_hubbard_adjoint(T, k, q, 1.0, 0.0, w, beta, grad_sum=gs, out=out,
                                                    out_sum=osum, stream=stream, grads=g[0])
            s_med, s_min = _median_ms(torch, stream, step)
            sfl = rl.specialized_adjoint_flops(st, n_e, n_f, d.alpha, with_values=True)["total"]
            row.update({"step_ms_median": s_med, "step_ms_min": s_min, "step_kernel": amd.last_variant(),
                        "step_term_evals_per_s": te / (s_med * 1e-3),
                        "step_frac_fp64_peak": sfl / (s_med * 1e-3) / rl.PEAK_FP64_VECTOR})
        return row

    # C1: latency of the order-2 example
    try:
        d = order2_example()
        res["C1_order2_latency"] = fwd_and_step(d, 10_000, (110, 2, 0), 5.0, matsubara_freqs(1, 5.0))
        res["C1_order2_latency"]["workload"] = ("order-2 self-energy (R0 of Sec. 5.1.1), 10^4 k-samples, beta=5, "
                                                "i pi/beta; times are latencies (launch-bound)")
    except amd.AmiError as e:
        res["C1_order2_latency"] = f"not run: {e}"
    # C2: orders 3 and 4, two topologies each, three temperatures
    c2 = []
    for order, i in ((3, 0), (3, 1), (4, 1), (4, 3)):
        d = random_self_energy(order, (0, order, i))
        for beta in (2.0, 5.0, 10.0):
            try:
                row = fwd_and_step(d, 1_000_000, (111, order, i), beta, matsubara_freqs(1, beta))
                row.update({"order": order, "topology": [0, order, i]})
                c2.append(row)
            except amd.AmiError as e:
                c2.append({"order": order, "topology": [0, order, i], "beta": beta, "error": str(e)})
    res["C2_orders3_4_betas"] = c2
    # C3: the real-frequency grid, forward (out is 256 x 10^6 complex128)
    try:
        d = random_self_energy(4, (0, 4, 1))
        n_e, beta = 1_000_000, 5.0
        wr = real_freqs(256, -6.0, 6.0, 0.05)
        T, st, k, w, out, osum, _ = prepare(d, n_e, (112, 4, 1), wr)
        fwd = lambda: amd.evaluate_hubbard(T, k, q, 1.0, 0.0, w, beta, want_sum=True, out=out, out_sum=osum,
                                           stream=stream)
        f_med, f_min = _median_ms(torch, stream, fwd, reps=21)
        nbytes = n_e * 2 * d.n_int * 8 + 256 * n_e * 16 + 256 * 16
        fl = rl.specialized_forward_flops(st, n_e, 256, d.alpha)["total"]
        # a plain write kernel of known size on the same buffer (torch's fill of
        # out): the write rate this GPU reaches, beside the vendor figure
        z_med, _ = _median_ms(torch, stream, out.zero_, reps=11)
        zbytes = out.numel() * out.element_size()
        res["C3_real_frequency_grid"] = {
            "workload": "order-4 topology (0, 4, 1), 10^6 k-samples, 256 real frequencies omega + 0.05i, "
                        "omega in [-6, 6], beta=5, out [256, 10^6] complex128 (4.1 GB) + row sums",
            "kernel": amd.last_variant(), "ms_median": f_med, "ms_min": f_min,
            "term_evals_per_s": float(st.T) * n_e * 256 / (f_med * 1e-3),
            "algorithmic_bytes": nbytes, "hbm_gb_per_s": nbytes / (f_med * 1e-3) / 1e9,
            "frac_hbm_peak": nbytes / (f_med * 1e-3) / rl.PEAK_HBM,
            "plain_write_gb_per_s": zbytes / (z_med * 1e-3) / 1e9,
            "frac_of_plain_write": (nbytes / f_med) / (zbytes / z_med),
            "flops": fl, "frac_fp64_peak": fl / (f_med * 1e-3) / rl.PEAK_FP64_VECTOR}
        del out
    except amd.AmiError as e:
        res["C3_real_frequency_grid"] = f"not run: {e}"
    # C4: the C3 topology's adjoint with a per-sample cotangent grad_out (16 MB read)
    try:
        d = random_self_energy(4, (0, 4, 1))
        n_e, beta = 1_000_000, 5.0
        T, st, k, w, out, osum, _ = prepare(d, n_e, (114, 4, 1), matsubara_freqs(1, beta))
        rng = np.random.default_rng(115)
        go = torch.from_numpy(rng.standard_normal((1, n_e)) + 1j * rng.standard_normal((1, n_e))).to(dev)
        g = [None]

        def c4():
            g[0] = amd.evaluate_hubbard_adjoint(T, k, q, 1.0, 0.0, w, beta, grad_out=go, stream=stream, grads=g[0])
        a_med, a_min = _median_ms(torch, stream, c4)
        afl = rl.specialized_adjoint_flops(st, n_e, 1, d.alpha)["total"]
        nbytes = n_e * 2 * d.n_int * 8 + n_e * 16 + n_e * 2 * d.n_int * 8
        res["C4_adjoint_grad_out"] = {
            "workload": "order-4 topology (0, 4, 1), 10^6 k-samples, beta=5, i pi/beta; adjoint with a per-sample "
                        "cotangent grad_out [1, 10^6] complex128 -> grad_k [10^6, 8], grad_mu, grad_t, grad_beta, grad_w",
            "kernel": amd.last_variant(), "ms_median": a_med, "ms_min": a_min,
            "term_evals_per_s": float(st.T) * n_e / (a_med * 1e-3), "algorithmic_bytes": nbytes,
            "flops": afl, "frac_fp64_peak": afl / (a_med * 1e-3) / rl.PEAK_FP64_VECTOR}
    except amd.AmiError as e:
        res["C4_adjoint_grad_out"] = f"not run: {e}"
    return res


def large_section(args, torch, dev, stream):
    """The adjoint of large solutions in passes (order 5 and order 6 at 2 10^5
    k-samples, one Matsubara frequency): forward and value-and-gradient step,
    each the median of 25 individually timed calls."""
    import numpy as np

    import paper_2311_17189_amd as amd
    from ami_inputs import DEFAULT_Q, k_samples, matsubara_freqs, random_self_energy
    from paper_2311_17189_amd import roofline as rl

    q = np.array(DEFAULT_Q)
    res = {}

    def fwd_and_step(d, n_e, seed, beta, freqs):
        T = amd.Terms.from_diagram(d)
        T.upload()
        T.specialize(momentum=True)
        st = rl.structure_from_canonical(T.canonical())
        k = torch.from_numpy(k_samples(n_e, d.n_int, seed=seed)).to(dev)
        w = torch.from_numpy(freqs).to(dev)
        n_f = w.shape[0]
        out = torch.empty((n_f, n_e), dtype=torch.complex128, device=dev)
        osum = torch.empty((n_f,), dtype=torch.complex128, device=dev)
        gs = torch.ones((n_f,), dtype=torch.complex128, device=dev)
        te = float(st.T) * n_e * n_f
        fwd = lambda: amd.evaluate_hubbard(T, k, q, 1.0, 0.0, w, beta, want_sum=True, out=out, out_sum=osum,
                                           stream=stream)
        f_med, f_min = _median_ms(torch, stream, fwd)
        ffl = rl.specialized_forward_flops(st, n_e, n_f, d.alpha)["total"]
        row = {"terms": st.T, "n_e": n_e, "n_f": n_f, "beta": beta, "fwd_ms_median": f_med, "fwd_ms_min": f_min,
               "fwd_kernel": amd.last_variant(), "fwd_term_evals_per_s": te / (f_med * 1e-3),
               "fwd_frac_fp64_peak": ffl / (f_med * 1e-3) / rl.PEAK_FP64_VECTOR}
        g = [None]

        def step():
            g[0] = amd.evaluate_hubbard_adjoint(T, k, q, 1.0, 0.0, w, beta, grad_sum=gs, out=out,
                                                out_sum=osum, stream=stream, grads=g[0])
        s_med, s_min = _median_ms(torch, stream, step)
        sfl = rl.specialized_adjoint_flops(st, n_e, n_f, d.alpha, with_values=True)["total"]
        row.update({"step_ms_median": s_med, "step_ms_min": s_min, "step_kernel": amd.last_variant(),
                    "step_term_evals_per_s": te / (s_med * 1e-3),
                    "step_frac_fp64_peak": sfl / (s_med * 1e-3) / rl.PEAK_FP64_VECTOR})
        return row

    large = []
    for order, seed in ((5, (0, 5, 0)), (6, (0, 6, 0)), (6, (5, 6, 2))):
        try:
            d = random_self_energy(order, seed)
            row = fwd_and_step(d, 200_000, (113,) + seed, 5.0, matsubara_freqs(1, 5.0))
            row.update({"order": order, "topology": list(seed)})
            large.append(row)
        except amd.AmiError as e:
            large.append({"order": order, "topology": list(seed), "error": str(e)})
    return large


def next_rows_section(args, torch, dev, stream):
    """The rows built beyond the main path, each measured on the order-4
    workload: complex energies (forward and value-and-gradient step, energy
    input), poles of higher order (the order-4 topology with one internal line
    taken twice, momentum input, forward and step) and graph input (label +
    construct from the 4-column form); and a large order-6 solution through
    the two-pass forward, at real momenta and at complex energies."""
    import numpy as np

    import paper_2311_17189_amd as amd
    from ami_inputs import DEFAULT_Q, complex_energies, k_samples, matsubara_freqs, random_self_energy
    from paper_2311_17189_amd import roofline as rl

    res = {}
    d = random_self_energy(args.order, (0, args.order, args.diagram))
    n_e, reps = args.n_e, max(5, args.steps // 2)
    w = torch.from_numpy(matsubara_freqs(1, args.beta)).to(dev)
    # complex energies: |beta Im x| below pi/2 for every leaf
    try:
        T = amd.Terms.from_diagram(d)
        st = rl.structure_from_canonical(T.canonical())
        eta = 0.25 / (args.beta * d.n_int)
        E = torch.from_numpy(complex_energies(n_e, d.n_eps, seed=(101, args.order, args.diagram),
                                              a=3.0, eta=eta)).to(dev)
        out = torch.empty((1, n_e), dtype=torch.complex128, device=dev)
        osum = torch.empty((1,), dtype=torch.complex128, device=dev)
        ms, kms = _timed_kernel(torch, amd, stream, lambda: amd.evaluate_complex(
            T, E, w, args.beta, out=out, out_sum=osum, want_sum=True, stream=stream), reps)
        fl = rl.specialized_complex_forward_flops(st, n_e, 1)
        res["complex_energies"] = {
            "workload": f"order-{args.order} topology {args.diagram}, {n_e} complex energy rows "
                        f"(Re uniform in (-3, 3), |Im| < {eta:.3g}), 1 Matsubara frequency, out + row sum",
            "kernel": amd.last_variant(), "ms": ms, "kernel_ms": kms,
            "term_evals_per_s": float(st.T) * n_e / (ms * 1e-3),
            "flops_per_launch": fl["total"], "frac_fp64_peak": fl["total"] / (kms * 1e-3) / rl.PEAK_FP64_VECTOR}
        # its value-and-gradient step: dL/dRe E + i dL/dIm E, dL/dbeta, dL/dw of the summed values
        gs = torch.ones((1,), dtype=torch.complex128, device=dev)
        ms_a, kms_a = _timed_kernel(torch, amd, stream, lambda: amd.evaluate_complex_adjoint(
            T, E, w, args.beta, grad_sum=gs, out=out, out_sum=osum, stream=stream), reps)
        res["complex_adjoint"] = {
            "workload": res["complex_energies"]["workload"] + "; value-and-gradient step (complex energy gradients)",
            "kernel": amd.last_variant(), "ms": ms_a, "kernel_ms": kms_a,
            "term_evals_per_s": float(st.T) * n_e / (ms_a * 1e-3)}
    except amd.AmiError as e:
        res["complex_energies"] = f"not run: {e}"
    # poles of higher order: one internal line repeated, its energy slot unused
    try:
        j = [r for r in range(d.alpha.shape[0]) if np.any(d.alpha[r, :d.n_int])][0]
        ng = d.alpha.shape[0]
        alpha = np.vstack([d.alpha, d.alpha[j:j + 1]])
        eps = np.eye(ng + 1, dtype=np.int8)
        eps[ng] = 0
        eps[ng, j] = 1
        T = amd.Terms(alpha, eps, d.n_int, d.fermionic, multipole=True)
        T.specialize(momentum=True)
        st = rl.structure_from_canonical(T.canonical())
        k = torch.from_numpy(k_samples(n_e, d.n_int, seed=(102, args.order, args.diagram))).to(dev)
        q = np.array(DEFAULT_Q)
        out = torch.empty((1, n_e), dtype=torch.complex128, device=dev)
        osum = torch.empty((1,), dtype=torch.complex128, device=dev)
        ms, kms = _timed_kernel(torch, amd, stream, lambda: amd.evaluate_hubbard(
            T, k, q, 1.0, 0.0, w, args.beta, out=out, out_sum=osum, want_sum=True, stream=stream), reps)
        fl = rl.specialized_forward_flops(st, n_e, 1, alpha)
        orders = sorted({abs(c) - 1 for c, _ in st.leaves})
        res["multipole"] = {
            "workload": f"order-{args.order} topology {args.diagram} with line {j} taken twice (double poles), "
                        f"{n_e} k-samples, 1 Matsubara frequency, out + row sum",
            "terms": st.T, "leaf_orders": orders, "kernel": amd.last_variant(), "ms": ms, "kernel_ms": kms,
            "term_evals_per_s": float(st.T) * n_e / (ms * 1e-3),
            "flops_per_launch": fl["total"], "frac_fp64_peak": fl["total"] / (kms * 1e-3) / rl.PEAK_FP64_VECTOR}
        # its value-and-gradient step (Taylor-coefficient leaves differentiated in the kernel)
        gs = torch.ones((1,), dtype=torch.complex128, device=dev)
        g = [None]

        def mstep():
            g[0] = amd.evaluate_hubbard_adjoint(T, k, q, 1.0, 0.0, w, args.beta, grad_sum=gs, out=out,
                                                out_sum=osum, stream=stream, grads=g[0])
        ms_a, kms_a = _timed_kernel(torch, amd, stream, mstep, reps)
        res["multipole_adjoint"] = {
            "workload": res["multipole"]["workload"] + "; value-and-gradient step",
            "kernel": amd.last_variant(), "ms": ms_a, "kernel_ms": kms_a,
            "term_evals_per_s": float(st.T) * n_e / (ms_a * 1e-3)}
    except amd.AmiError as e:
        res["multipole"] = f"not run: {e}"
    # a large solution through the two-pass forward: order 6, 2804 terms, the
    # batch's frequency count
    try:
        dl = random_self_energy(6, (5, 6, 2))
        T = amd.Terms.from_diagram(dl)
        T.specialize(momentum=True)
        st = rl.structure_from_canonical(T.canonical())
        n_l, n_fl = 200_000, 16
        wl = torch.from_numpy(matsubara_freqs(n_fl, args.beta)).to(dev)
        k = torch.from_numpy(k_samples(n_l, dl.n_int, seed=(103, 6, 2))).to(dev)
        q = np.array(DEFAULT_Q)
        out = torch.empty((n_fl, n_l), dtype=torch.complex128, device=dev)
        osum = torch.empty((n_fl,), dtype=torch.complex128, device=dev)
        ms, _ = _timed_kernel(torch, amd, stream, lambda: amd.evaluate_hubbard(
            T, k, q, 1.0, 0.0, wl, args.beta, out=out, out_sum=osum, want_sum=True, stream=stream), 5)
        fl = rl.specialized_forward_flops(st, n_l, n_fl, dl.alpha)
        res["large_two_pass"] = {
            "workload": f"order-6 topology (5, 6, 2), {st.T} terms, {n_l} k-samples, {n_fl} Matsubara frequencies, "
                        "out + row sums",
            "kernel": amd.last_variant(), "ms": ms,
            "term_evals_per_s": float(st.T) * n_l * n_fl / (ms * 1e-3),
            "flops_per_call": fl["total"], "frac_fp64_peak": fl["total"] / (ms * 1e-3) / rl.PEAK_FP64_VECTOR}
        # the same solution at complex energies (two passes: above the one-pass size)
        eta = 0.25 / (args.beta * dl.n_int)
        Ec = torch.from_numpy(complex_energies(n_l, dl.n_eps, seed=(104, 6, 2), a=3.0, eta=eta)).to(dev)
        ms_c, _ = _timed_kernel(torch, amd, stream, lambda: amd.evaluate_complex(
            T, Ec, wl, args.beta, out=out, out_sum=osum, want_sum=True, stream=stream), 5)
        res["large_complex_two_pass"] = {
            "workload": f"order-6 topology (5, 6, 2), {st.T} terms, {n_l} complex energy rows (|Im| < {eta:.3g}), "
                        f"{n_fl} Matsubara frequencies, out + row sums",
            "kernel": amd.last_variant(), "ms": ms_c,
            "term_evals_per_s": float(st.T) * n_l * n_fl / (ms_c * 1e-3)}
        # the adjoint at complex energies in passes: order 6, 560 terms, one frequency
        dm = random_self_energy(6, (0, 6, 0))
        Tm = amd.Terms.from_diagram(dm)
        Tm.specialize(momentum=False)
        stm = rl.structure_from_canonical(Tm.canonical())
        em = 0.25 / (args.beta * dm.n_int)
        Em = torch.from_numpy(complex_energies(n_l, dm.n_eps, seed=(105, 6, 0), a=3.0, eta=em)).to(dev)
        om = torch.empty((1, n_l), dtype=torch.complex128, device=dev)
        sm = torch.empty((1,), dtype=torch.complex128, device=dev)
        gs = torch.ones((1,), dtype=torch.complex128, device=dev)
        ms_a, _ = _timed_kernel(torch, amd, stream, lambda: amd.evaluate_complex_adjoint(
            Tm, Em, w, args.beta, grad_sum=gs, out=om, out_sum=sm, stream=stream), 5)
        res["large_complex_adjoint"] = {
            "workload": f"order-6 topology (0, 6, 0), {stm.T} terms, {n_l} complex energy rows (|Im| < {em:.3g}), "
                        "1 Matsubara frequency; value-and-gradient step",
            "kernel": amd.last_variant(), "ms": ms_a, "term_evals_per_s": float(stm.T) * n_l / (ms_a * 1e-3)}
    except amd.AmiError as e:
        res["large_two_pass"] = f"not run: {e}"
    # graph input: label and construct, host only
    g = {}
    for order, i in ((args.order, args.diagram), (6, 0)):
        dd = random_self_energy(order, (0, order, i))
        n = 20
        t0 = time.perf_counter()
        for _ in range(n):
            amd.Terms.from_graph(dd.graph).close()
        g[f"order{order}"] = {"construct_ms": (time.perf_counter() - t0) * 1e3 / n,
                              "terms": amd.Terms.from_graph(dd.graph).info()["T"]}
    res["graph_construct"] = g
    return res


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
    # generate and compile (or load from the disk cache) the specialized kernels
    t0 = time.perf_counter()
    try:
        terms.specialize(momentum=True)
        specialize_note = "ok"
    except amd.AmiError as e:          # AUTO then runs the packed kernels; reported below
        specialize_note = str(e)
    specialize_ms = (time.perf_counter() - t0) * 1e3
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
    # cotangent of the row sum: gradients of Re sum_s I(s) (the summed integrand)
    g_sum = torch.ones((n_f,), dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream()

    def fwd():
        amd.evaluate_hubbard(terms, k, q, hop_t, mu, w, args.beta, want_sum=True,
                             out=out, out_sum=out_sum, stream=stream)

    def adj():
        return amd.evaluate_hubbard_adjoint(terms, k, q, hop_t, mu, w, args.beta,
                                            grad_sum=g_sum, stream=stream)

    grads = [None]

    def step():
        # the whole path in one pass: values out[N_F, N_E] and out_sum[N_F] and the
        # gradients of Re sum_s I(s) (the row-sum cotangent is fixed in advance),
        # written into the same output tensors every step
        grads[0] = amd.evaluate_hubbard_adjoint(terms, k, q, hop_t, mu, w, args.beta, grad_sum=g_sum,
                                                out=out, out_sum=out_sum, stream=stream, grads=grads[0])
        return grads[0]

    if args.copy_mib > 0:
        src = torch.empty(args.copy_mib * (1 << 20) // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    step_variant = amd.last_variant()

    # the step as a HIP graph: captured once on a side stream (after the
    # kernels are loaded and the workspace sized there), replayed per step
    graph, gstream, graph_note = None, None, None
    if not args.no_graph:
        try:
            gstream = torch.cuda.Stream()
            gstream.wait_stream(stream)
            with torch.cuda.stream(gstream):
                amd.evaluate_hubbard_adjoint(terms, k, q, hop_t, mu, w, args.beta, grad_sum=g_sum,
                                             out=out, out_sum=out_sum, grads=grads[0])
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=gstream):
                amd.evaluate_hubbard_adjoint(terms, k, q, hop_t, mu, w, args.beta, grad_sum=g_sum,
                                             out=out, out_sum=out_sum, grads=grads[0])
        except Exception as e:            # reported, not fatal: the steps are then plain launches
            graph, graph_note = None, f"not captured: {e}"

    def warm(replay):
        # untimed steps right before the timed loop (at least W of them)
        with torch.cuda.stream(gstream if replay else stream):
            _warm(torch, graph.replay if replay else step, calls=max(args.warmup, 1))

    def timed_steps(replay):
        s_ = gstream if replay else stream
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        with torch.cuda.stream(s_):       # replay() launches on the current stream
            t0.record(s_)
            for _ in range(args.steps):
                if replay:
                    graph.replay()
                else:
                    step()
            t1.record(s_)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / args.steps

    # timed region: K steps, each one graph replay of the whole step (plain
    # launches with --no-graph or when the capture failed)
    warm(graph is not None)
    wall0 = time.perf_counter()
    ms_step = timed_steps(graph is not None)
    wall = time.perf_counter() - wall0
    step_mode = "graph replay" if graph is not None else "launches"
    # the same steps again, each timed alone (max(K, 20) of them): median and minimum
    with torch.cuda.stream(gstream if graph is not None else stream):
        step_median = _median_ms(torch, gstream if graph is not None else stream,
                                 graph.replay if graph is not None else step, reps=max(args.steps, 20))

    # the same K steps as plain launches; the library records HIP events on
    # the launch stream around the main kernel of every step (the roofline's
    # kernel duration)
    warm(False)
    amd.kernel_timer_start(args.steps)
    launch_ms = timed_steps(False)
    kernel_ms = amd.kernel_timer_stop()
    step_kernel_ms = sum(kernel_ms) / len(kernel_ms)
    graph_ms = ms_step if graph is not None else graph_note
    del graph
    # FP64 FMA throughput of this GPU right after the timed steps (clock warm)
    try:
        fma_peak = amd.measure_fp64_peak(1 << 16, stream=stream)
    except amd.AmiError:
        fma_peak = None

    def timed(fn, reps):
        _warm(torch, fn)
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        for _ in range(reps):
            fn()
        a1.record(stream)
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) / reps

    # host time to issue one step (no synchronization inside the loop)
    torch.cuda.synchronize()
    h0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    host_ms = (time.perf_counter() - h0) * 1e3 / args.steps
    torch.cuda.synchronize()

    # beside the step: forward alone and adjoint alone (separate passes)
    reps = max(5, args.steps // 2)
    fwd_ms = timed(fwd, reps)
    fwd_variant = amd.last_variant()
    adj_ms = timed(adj, reps)

    # the table-driven (packed) kernels on the same launches
    terms.set_variant(amd.VARIANT_PACKED)
    packed_fwd_ms = timed(fwd, reps)
    packed_variant = amd.last_variant()
    packed_step_ms = timed(step, reps)
    terms.set_variant(amd.VARIANT_AUTO)

    # the plain per-diagram kernel (double tables) on the same launch, outside the timed region
    terms.set_variant(amd.VARIANT_TABLES)
    _warm(torch, fwd, calls=2)
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    n_plain = max(5, args.steps // 2)
    p0.record(stream)
    for _ in range(n_plain):
        fwd()
    p1.record(stream)
    torch.cuda.synchronize()
    plain_ms = p0.elapsed_time(p1) / n_plain
    plain_variant = amd.last_variant()
    terms.set_variant(amd.VARIANT_AUTO)

    # Monte-Carlo integration of the same diagram with momenta drawn in the
    # kernel (no sample touches HBM): forward values summed over 10 N_E samples
    mc = None
    try:
        n_mc = 10 * n_e
        sums = amd.integrate_hubbard(terms, n_mc, 1234, q, hop_t, mu, w, args.beta, stream=stream)
        _warm(torch, lambda: amd.integrate_hubbard(terms, n_mc, 1234, q, hop_t, mu, w, args.beta, sums=sums,
                                                   stream=stream))
        amd.kernel_timer_start(5)
        m0 = torch.cuda.Event(enable_timing=True)
        m1 = torch.cuda.Event(enable_timing=True)
        m0.record(stream)
        for _ in range(5):
            amd.integrate_hubbard(terms, n_mc, 1234, q, hop_t, mu, w, args.beta, sums=sums, stream=stream)
        m1.record(stream)
        torch.cuda.synchronize()
        mk = amd.kernel_timer_stop()
        mc_ms = m0.elapsed_time(m1) / 5
        mean, err = amd.mc_estimate(sums, n_mc)
        mfl = rl.mc_flops(st, n_mc, n_f, d.alpha)
        mc = {"samples": n_mc, "ms": mc_ms, "kernel_ms": sum(mk) / len(mk),
              "term_evals_per_s": float(info["T"]) * n_mc * n_f / (mc_ms * 1e-3),
              "tflops": mfl["total"] / (sum(mk) / len(mk) * 1e-3) / 1e12,
              "frac_fp64_peak": mfl["total"] / (sum(mk) / len(mk) * 1e-3) / rl.PEAK_FP64_VECTOR,
              "estimate": [[float(z.real), float(z.imag)] for z in mean],
              "stderr": [[float(a), float(b)] for a, b in err]}
    except amd.AmiError as e:
        mc = f"not run: {e}"

    te = float(info["T"]) * n_e * n_f
    value = te / (ms_step * 1e-3)
    spec = step_variant.startswith("specialized")
    if spec:
        fl = rl.specialized_forward_flops(st, n_e, n_f, d.alpha)
        fa = rl.specialized_adjoint_flops(st, n_e, n_f, d.alpha)
        fs = rl.specialized_adjoint_flops(st, n_e, n_f, d.alpha, with_values=True)
        dom, dom_key = "ami_jit_adj (specialized adjoint with values)", "ami_jit_adj"
    else:
        fl = rl.forward_flops(st, n_e, n_f, d.alpha)
        fa = rl.adjoint_flops(st, n_e, n_f, d.alpha)
        fs = rl.adjoint_flops(st, n_e, n_f, d.alpha, with_values=True)
        dom, dom_key = "ami_adj_packed (packed adjoint with values)", "ami_adj_packed"
    pfl = rl.forward_flops(st, n_e, n_f, d.alpha)
    pfs = rl.adjoint_flops(st, n_e, n_f, d.alpha, with_values=True)
    # the step's main kernel: the adjoint with values, timed alone
    dom_ms, dom_fl = step_kernel_ms, fs["total"]
    achieved = dom_fl / (dom_ms * 1e-3)
    workload_key = f"order{args.order}-diagram{args.diagram}-ne{n_e}-nf{n_f}-beta{args.beta:g}"
    traffic = recorded_traffic(dom_key, workload_key)

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
                        f"{n_e} k-samples, beta={args.beta}, 1 Matsubara frequency; step = forward "
                        "(out[N_F,N_E] + row sum, energies from momenta in-kernel) + adjoint "
                        "(d/dk, d/dmu, d/dt, d/dbeta, d/dw of the summed integrand)",
            "order": args.order, "terms": info["T"], "distinct_leaves": info["L"],
            "distinct_denominators": info["D"], "groups": info["G"], "n_e": n_e, "n_f": n_f,
            "beta": args.beta, "t": hop_t, "mu": mu, "q": [float(x) for x in q],
            "diagram_seed": [0, args.order, args.diagram],
            "key": workload_key,
        },
        "fwd": {"ms": fwd_ms, "term_evals_per_s": te / (fwd_ms * 1e-3), "kernel": fwd_variant,
                "flops": fl["total"], "tflops": fl["total"] / (fwd_ms * 1e-3) / 1e12,
                "frac_fp64_peak": fl["total"] / (fwd_ms * 1e-3) / rl.PEAK_FP64_VECTOR},
        "fwd_adjoint": {"step_mode": step_mode, "one_pass_ms": launch_ms, "one_pass_kernel_ms": step_kernel_ms,
                        "host_ms_per_call": host_ms, "graph_ms_per_step": graph_ms,
                        "one_pass_term_evals_per_s": te / (launch_ms * 1e-3), "kernel": step_variant,
                        "separate_ms": fwd_ms + adj_ms, "adjoint_ms": adj_ms,
                        "adjoint_flops": fa["total"],
                        "adjoint_tflops": fa["total"] / (adj_ms * 1e-3) / 1e12},
        "packed_kernels": {"fwd_ms": packed_fwd_ms, "kernel": packed_variant,
                           "fwd_tflops": pfl["total"] / (packed_fwd_ms * 1e-3) / 1e12,
                           "step_ms": packed_step_ms,
                           "step_term_evals_per_s": te / (packed_step_ms * 1e-3),
                           "step_tflops": pfs["total"] / (packed_step_ms * 1e-3) / 1e12,
                           "speedup_of_specialized_step": packed_step_ms / launch_ms},
        "plain_kernel": {"ms": plain_ms, "term_evals_per_s": te / (plain_ms * 1e-3),
                         "kernel": plain_variant, "speedup_of_fwd": plain_ms / fwd_ms},
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": rl.PEAK_FP64_VECTOR / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / rl.PEAK_FP64_VECTOR,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "kernel": dom,
            "flops_per_launch": dom_fl,
            "kernel_ms": dom_ms,
            # FP64 FMA throughput measured on this GPU (eight independent FMA
            # chains per lane, eight waves per SIMD), beside the vendor peak
            "measured_fma_peak": fma_peak,
            "frac_of_measured_fma_peak": (achieved / 1e12 / fma_peak) if fma_peak else None,
        },
        "monte_carlo": mc,
        "construct_ms": construct_ms,
        "specialize_ms": specialize_ms, "specialize": specialize_note,
        "wall_s": wall,
    }
    res["ms_per_step_median"], res["ms_per_step_min"] = step_median
    sections = {x.strip() for x in args.sections.split(",") if x.strip()}
    if args.no_configs:
        sections -= {"configs", "large"}
    if args.no_batch:
        sections.discard("batch")
    if "next" in sections:
        res["next_rows"] = next_rows_section(args, torch, dev, stream)
    if "configs" in sections:
        res["configs"] = configs_section(args, torch, dev, stream)
    if "large" in sections:
        res["large_adjoint_passes"] = large_section(args, torch, dev, stream)
    if "batch" in sections:
        res["batch"] = batch_section(args, torch, dev)
    if args.cpu_seconds > 0:
        res["cpu_baseline"] = cpu_baseline(d, k_host, q, args.beta, hop_t, mu, w_host,
                                           args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
