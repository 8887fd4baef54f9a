"""Mixed-diagram batch (one HIP graph launch over many diagrams), in its
three modes -- every item on its specialized kernels where AUTO would run them
(recorded launches in a child graph), every item's specialized tile functions
in persistent kernels, or every item on the persistent packed kernels:
outputs against the oracle, bitwise equal to the per-diagram
launches of the same kernels, stable across graph replays, row sums
consistent, the autotuner, host-side errors, and the 64-diagram workload at
full size (sampled outputs against the oracle)."""
import numpy as np
import pytest

from ami_inputs import (DEFAULT_Q, k_samples, matsubara_freqs, random_self_energy,
                        uniform_energies)

from parity import NEAR, TOL, TOL_NEAR, check, oracle_terms, reference, reference_hubbard

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amd = pytest.importorskip("paper_2311_17189_amd")

DEV = "cuda"


def _mixed_items(n_per_order=2, orders=(2, 3, 4, 5, 6), n_f=4, beta=5.0, energies=False, seed=0, kernels=1):
    items = []
    for order in orders:
        for i in range(n_per_order):
            d = random_self_energy(order, (seed, order, i))
            T = amd.Terms.from_diagram(d)
            # the per-diagram kernels the batch shares
            T.set_variant(amd.VARIANT_PACKED if kernels == 1 else amd.VARIANT_AUTO)
            n_e = 300 + 517 * i + 131 * order            # ragged sizes
            w = torch.from_numpy(matsubara_freqs(n_f, beta)).to(DEV)
            it = {"terms": T, "ext_freqs": w, "beta": beta, "diagram": d,
                  "out": torch.empty((n_f, n_e), dtype=torch.complex128, device=DEV),
                  "out_sum": torch.empty((n_f,), dtype=torch.complex128, device=DEV)}
            if energies:
                it["energies"] = torch.from_numpy(uniform_energies(n_e, d.n_eps, seed=(30, order, i),
                                                                   a=4.0)).to(DEV)
            else:
                it["k"] = torch.from_numpy(k_samples(n_e, d.n_int, seed=(31, order, i))).to(DEV)
                it.update(q=list(DEFAULT_Q), t=1.0, mu=0.05)
            items.append(it)
    return items


_ORACLE = {}


def _oracle_check(it, idx=None, label=""):
    """The item's out (all samples, or the columns idx) and out_sum against
    the oracle: values by the parity bar, the row sum within the bar summed
    over the samples (only when every sample is compared)."""
    import hashlib
    d = it["diagram"]
    w = it["ext_freqs"].cpu().numpy()
    hub = it.get("k") is not None
    x = (it["k"] if hub else it["energies"]).cpu().numpy()
    x = x if idx is None else x[idx]
    # the cache key is the whole input: labels, samples, frequencies, scalars
    h = hashlib.sha256()
    for a in (d.alpha, d.eps, x, w, np.array([it["beta"], it.get("t", 0.0), it.get("mu", 0.0)])):
        h.update(np.ascontiguousarray(a).tobytes())
    key = (hub, h.hexdigest())
    if key not in _ORACLE:
        terms = oracle_terms(d)
        if hub:
            ref, scale, dist, _ = reference_hubbard(d, x, it["q"], it["t"], it["mu"], w, it["beta"], terms=terms)
        else:
            ref, scale, dist = reference(d, x, w, it["beta"], terms=terms)
        _ORACLE[key] = (ref, scale, dist)
    ref, scale, dist = _ORACLE[key]
    out = it["out"] if idx is None else it["out"][:, torch.from_numpy(np.asarray(idx)).to(DEV)]
    check(out.cpu().numpy(), ref, scale, dist, label=label)
    if idx is None and it.get("out_sum") is not None:
        bound = (np.where(dist >= NEAR, TOL, TOL_NEAR) * scale).sum(axis=1)
        assert np.all(np.abs(it["out_sum"].cpu().numpy() - ref.sum(axis=1)) <= bound), label


def _per_diagram(it):
    if it.get("k") is not None:
        return amd.evaluate_hubbard(it["terms"], it["k"], it["q"], it["t"], it["mu"], it["ext_freqs"],
                                    it["beta"], want_sum=True)
    return amd.evaluate(it["terms"], it["energies"], it["ext_freqs"], it["beta"], want_sum=True)


@pytest.mark.parametrize("energies", [False, True])
@pytest.mark.parametrize("tuning", [None, {"block": 64, "waves_per_cu": 4, "tile_factor": 1, "kernels": 1},
                                    {"block": 128, "waves_per_cu": 16, "tile_factor": 4, "kernels": 1},
                                    {"block": 0, "waves_per_cu": 32, "tile_factor": 2, "kernels": 2},
                                    {"block": 0, "waves_per_cu": 8, "tile_factor": 1, "kernels": 2}])
def test_batch_bitwise_equals_per_diagram(energies, tuning):
    kernels = 0 if tuning is None else tuning["kernels"]
    items = _mixed_items(energies=energies, kernels=kernels)
    b = amd.Batch(items, tuning)
    b.run()
    torch.cuda.synchronize()
    info = b.info()
    assert info["items"] == len(items)
    if kernels == 1:
        assert info["work_items"] >= len(items) and info["specialized_items"] == 0
        assert info["lds_classes"] >= 2          # orders 2..6 span more than one LDS class
    elif kernels == 2:
        # persistent kernels running every item's own tile functions
        assert info["specialized_items"] == len(items) and info["capture_streams"] == 0
        assert info["lds_classes"] >= 1 and info["work_items"] >= len(items)
    else:
        assert info["specialized_items"] == len(items) and info["lds_classes"] == 0
        assert info["capture_streams"] == 4
    for j, it in enumerate(items):
        _oracle_check(it, label=f"batch item {j}")
        ref_out, ref_sum = _per_diagram(it)
        torch.cuda.synchronize()
        assert torch.equal(it["out"], ref_out)
        if kernels in (0, 2):
            assert torch.equal(it["out_sum"], ref_sum)       # the same tile functions and reduction
        else:
            # the row sum runs over the batch's tiles; it equals the per-diagram
            # one bit for bit when the tile size matches, else to rounding
            assert torch.allclose(it["out_sum"], ref_sum, rtol=1e-12, atol=1e-15 * float(ref_out.abs().sum()))


@pytest.mark.parametrize("kernels", [0, 1, 2])
def test_graph_replays_are_identical(kernels):
    """Replay the batch graph several times with other GPU work and
    synchronizations in between; every replay gives the same bits."""
    items = _mixed_items(n_per_order=1, kernels=kernels)
    b = amd.Batch(items, {"block": 64, "waves_per_cu": 8, "tile_factor": 2, "kernels": kernels})
    b.run()
    torch.cuda.synchronize()
    first = [(it["out"].clone(), it["out_sum"].clone()) for it in items]
    scratch = torch.zeros(1 << 20, dtype=torch.float64, device=DEV)
    for rep in range(4):
        for it in items:
            it["out"].fill_(float("nan"))
            it["out_sum"].zero_()
        scratch.add_(1.0)                      # eager work between replays
        torch.cuda.synchronize()
        b.run()
        torch.cuda.synchronize()
        for (o, s), it in zip(first, items):
            assert torch.equal(it["out"], o)
            assert torch.equal(it["out_sum"], s)


@pytest.mark.parametrize("kernels", [0, 1, 2])
def test_batch_outputs_only_sums(kernels):
    items = _mixed_items(n_per_order=1, kernels=kernels)
    for it in items:
        it["out"] = None
    b = amd.Batch(items, {"kernels": kernels})
    b.run()
    torch.cuda.synchronize()
    for it in items:
        _, ref_sum = _per_diagram(it)
        torch.cuda.synchronize()
        assert torch.allclose(it["out_sum"], ref_sum, rtol=1e-11)


def test_autotuner_picks_a_working_tuning(tmp_path):
    from paper_2311_17189_amd.autotune import autotune
    items = _mixed_items(n_per_order=1, orders=(2, 4, 6))
    cands = [{"block": 64, "waves_per_cu": 4, "tile_factor": 1, "kernels": 1},
             {"block": 0, "waves_per_cu": 8, "tile_factor": 4, "kernels": 1}]
    best, timings = autotune(items, cands, reps=2, path=str(tmp_path / "tune.json"))
    assert best in cands and len(timings) == 2
    again, _ = autotune(items, cands, reps=2, path=str(tmp_path / "tune.json"))
    assert again == best                     # served from the cache
    b = amd.Batch(items, best)
    b.run()
    torch.cuda.synchronize()
    for it in items:
        ref_out, _ = _per_diagram(it)
        torch.cuda.synchronize()
        assert torch.equal(it["out"], ref_out)


def test_batch_host_errors():
    items = _mixed_items(n_per_order=1, orders=(2, 3))
    mixed = [items[0], dict(items[1])]
    mixed[1].pop("k")
    mixed[1]["energies"] = torch.zeros((10, mixed[1]["terms"].n_eps), dtype=torch.float64, device=DEV)
    mixed[1]["out"] = torch.empty((4, 10), dtype=torch.complex128, device=DEV)
    with pytest.raises(amd.AmiError):
        amd.Batch(mixed)
    with pytest.raises(amd.AmiError):
        amd.Batch(items, {"block": 96, "waves_per_cu": 8, "tile_factor": 1})
    with pytest.raises(amd.AmiError):
        amd.Batch(items, {"kernels": 3})


@pytest.mark.timeout(900)
def test_full_size_mixed_batch_against_oracle():
    """The 64-diagram workload the benchmark times (orders 2-6, 13/13/13/13/12
    seeded topologies, 16 Matsubara frequencies, 2*10^5 k-samples each), one
    graph launch with the default tuning: 12 sampled samples of every diagram
    (the last one included) at all 16 rows against the oracle, and the row
    sums against sums of the returned rows."""
    from concurrent.futures import ThreadPoolExecutor
    orders = [2] * 13 + [3] * 13 + [4] * 13 + [5] * 13 + [6] * 12
    beta, n_f, n_e = 5.0, 16, 200_000
    w = torch.from_numpy(matsubara_freqs(n_f, beta)).to(DEV)
    items, seen = [], {}
    for order in orders:
        i = seen.get(order, 0)
        seen[order] = i + 1
        d = random_self_energy(order, (5, order, i))
        T = amd.Terms.from_diagram(d)
        k = torch.from_numpy(k_samples(n_e, d.n_int, seed=(200, order, i))).to(DEV)
        items.append({"terms": T, "k": k, "q": list(DEFAULT_Q), "t": 1.0, "mu": 0.0, "ext_freqs": w,
                      "beta": beta, "diagram": d,
                      "out": torch.empty((n_f, n_e), dtype=torch.complex128, device=DEV),
                      "out_sum": torch.empty((n_f,), dtype=torch.complex128, device=DEV)})

    def spec(it):
        try:
            it["terms"].specialize(momentum=True)
        except amd.AmiError:
            pass
    with ThreadPoolExecutor(max_workers=8) as pool:
        list(pool.map(spec, items))
    b = amd.Batch(items)
    for it in items:
        it["out"].fill_(float("nan"))
    b.run()
    torch.cuda.synchronize()
    print(f"batch: {b.info()}", flush=True)
    rng = np.random.default_rng(7)
    for j, it in enumerate(items):
        idx = np.sort(rng.choice(n_e - 1, 11, replace=False)).tolist() + [n_e - 1]
        _oracle_check(it, idx=idx, label=f"full-size batch item {j} (order {orders[j]})")
        rows = it["out"].sum(dim=1)
        torch.cuda.synchronize()
        np.testing.assert_allclose(it["out_sum"].cpu().numpy(), rows.cpu().numpy(), rtol=1e-9,
                                   atol=1e-12 * float(torch.abs(it["out"]).sum()))
