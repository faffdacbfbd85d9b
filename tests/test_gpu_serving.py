"""The serving loop: continuous batching with HBM admission; results alone == results in the mix."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import TOL_F32, compare, make_params, run_gpu, to_device

pytestmark = pytest.mark.gpu

ARRAYS = [(3, 8), (5, 16), (2, 32), (4, 4), (6, 8)]      # (stations, channels)
T, M, N_INT = 1024, 64, 3


def _params(N, C):
    B = N * (N + 1) // 2
    return make_params(B, C, T, M, "cf16", d=2.2, s_low=0.5, s_high=1.6, gamma=0.3,
                       options=oracle.OPT_ADAPTIVE, n_warm=32, kappa_sk=3.0, kappa_ds=3.0)


def _data():
    """Integrations of every array, pre-staged on the device (complex half)."""
    out = {}
    for a, (N, C) in enumerate(ARRAYS):
        for k in range(N_INT):
            env = synth.pulse_train(T, 128, 20, 7 * k + a)
            sc = synth.Scene(N, C, T, seed=1000 * a + k, rho=0.1,
                             rfi=[synth.Rfi([C // 2], 10.0, 0.5, 0.2, env, f0=0.1)])
            vis = synth.to_cf16(synth.correlate(synth.make_voltages(sc)))
            out[a, k] = (vis, to_device(vis, "cf16"))
    return out


def _host(res):
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in res.items()}


def test_results_alone_equal_results_in_the_mix():
    import torch
    from paper_2412_14775_amd import rfi
    data = _data()
    # alone: one array at a time, integrations in order, default stream
    alone = {}
    for a, (N, C) in enumerate(ARRAYS):
        plan = rfi.Plan(_params(N, C)[1])
        for k in range(N_INT):
            out = plan.alloc_outputs(flags=True, stats=True)
            plan.screen(data[a, k][1], out["avg"], out["weight"], out["flags"], out["stats"])
            torch.cuda.synchronize()
            alone[a, k] = _host(out)
        plan.close()
    # in the mix: fresh plans, every request submitted with random arrival times
    plans = [rfi.Plan(_params(N, C)[1]) for (N, C) in ARRAYS]
    srv = rfi.Server(n_slots=4, hbm_budget=1 << 36)
    rng = np.random.default_rng(3)
    t0 = srv.now() + 0.05
    outs = {}
    for k in range(N_INT):
        for a in rng.permutation(len(ARRAYS)):
            outs[a, k] = plans[a].alloc_outputs(flags=True, stats=True)
            srv.submit(plans[a], data[a, k][1], outs[a, k], arrival=t0 + 0.01 * k + rng.uniform(0, 0.01),
                       tag=int(100 * a + k))
    srv.drain(60)
    done = srv.poll(1000)
    st = srv.stats()
    srv.close()
    assert len(done) == len(ARRAYS) * N_INT and all(c["status"] == 0 for c in done)
    assert st["graphs"] == len(done)               # one graph per (plan, buffer set)
    for c in done:
        assert c["arrival"] <= c["admitted"] <= c["done"]
    order = {}
    for c in sorted(done, key=lambda c: c["done"]):
        a, k = divmod(c["tag"], 100)
        assert order.get(a, -1) == k - 1, "integrations of one array completed out of order"
        order[a] = k
    for key, ref in alone.items():
        got = _host(outs[key])
        for name in ("avg", "weight", "flags", "stats"):
            assert np.array_equal(got[name], ref[name], equal_nan=True), (key, name)
    for p in plans:
        p.close()
    # the first integration of one array against the oracle (plan thresholds: state still cold)
    op, _ = _params(*ARRAYS[1])
    gpu = run_gpu_from_host(alone[1, 0])
    compare(gpu, data[1, 0][0], op, TOL_F32, label="served integration vs oracle")


def run_gpu_from_host(h):
    g = {"avg": h["avg"][..., 0].astype(np.float64) + 1j * h["avg"][..., 1], "weight": h["weight"],
         "flags": h["flags"], "stats32": h["stats"]}
    g["tau"], g["r_re"], g["r_im"] = (h["stats"][..., k].astype(np.float64) for k in range(3))
    return g


def test_requests_overlap_in_flight():
    """Requests of different plans run concurrently on the server's slots.  Each (plan, buffer
    set) is served once first, so its graph exists; then all four arrive at the same instant
    and must be in flight together (each screens 1.7 GB, some 250 us, while an admission that
    replays a graph takes a few us).  Results equal those of the first, unhurried pass."""
    import torch
    from paper_2412_14775_amd import rfi
    N, C, Tl = 32, 64, 3072
    B = N * (N + 1) // 2
    dev = torch.device("cuda:0")
    e = synth.device_voltages(synth.Scene(N, C, Tl, seed=77, rho=0.1), dev)
    vis = torch.empty((B, C, Tl, 4, 2), dtype=torch.float16, device=dev)
    synth.correlate_torch(e, vis, "cf16")
    del e
    rp = rfi.rfi_params_default(n_stations=N, n_baselines=B, n_channels=C, n_samples=Tl, block_m=M,
                                vis_format=rfi.RFI_VIS_CF16, sk_d=2.2, sk_low=0.5, sk_high=1.6, ds_gamma=0.3)
    plans = [rfi.Plan(rp) for _ in range(4)]
    outs = [p.alloc_outputs(flags=True, stats=False) for p in plans]
    srv = rfi.Server(n_slots=4)
    for i, p in enumerate(plans):                  # first pass: capture one graph per request
        srv.submit(p, vis, outs[i], tag=i)
        srv.drain(60)
    first = [_host(o) for o in outs]
    t0 = srv.now() + 0.02
    for i, p in enumerate(plans):
        srv.submit(p, vis, outs[i], arrival=t0, tag=10 + i)
    srv.drain(60)
    done = srv.poll(100)
    st = srv.stats()
    srv.close()
    assert len(done) == 8 and all(c["status"] == 0 for c in done)
    assert st["graphs"] == 4, "graphs were not reused"
    assert st["peak_inflight"] > 1, "requests never overlapped"
    second = sorted((c for c in done if c["tag"] >= 10), key=lambda c: c["admitted"])
    assert second[1]["admitted"] < second[0]["done"], "the second request was admitted after the first had finished"
    for i in range(4):
        got = _host(outs[i])
        for name in ("avg", "weight", "flags"):
            assert np.array_equal(got[name], first[i][name], equal_nan=True), (i, name)
    for p in plans:
        p.close()
    del vis
    torch.cuda.empty_cache()


def test_recreated_plan_gets_its_own_graph():
    """A plan is served, destroyed, and another with different thresholds created (the allocator
    usually hands it the same host address) and served into the same buffers: the server must not
    replay the first plan's cached graph, whose kernel arguments hold the old thresholds."""
    import torch
    from paper_2412_14775_amd import rfi
    N, C = 4, 8
    B = N * (N + 1) // 2
    vis = synth.to_cf16(synth.correlate(synth.make_voltages(synth.Scene(N, C, T, seed=11))))
    dev = to_device(vis, "cf16")
    srv = rfi.Server(n_slots=2)
    out, served, addresses = None, [], []
    for s_high in (1.6, 1.05):
        _, rp = make_params(B, C, T, M, "cf16", d=2.2, s_low=0.5, s_high=s_high, gamma=0.3)
        plan = rfi.Plan(rp)
        addresses.append(int(plan.handle))
        if out is None:
            out = plan.alloc_outputs(flags=True, stats=False)
        srv.submit(plan, dev, out, tag=len(served))
        srv.drain(30)
        assert srv.poll(10)[0]["status"] == 0
        served.append(out["flags"].cpu().numpy().copy())
        ref = plan.alloc_outputs(flags=True, stats=False)
        plan.screen(dev, ref["avg"], ref["weight"], ref["flags"], None)
        torch.cuda.synchronize()
        assert np.array_equal(served[-1], ref["flags"].cpu().numpy()), f"served flags differ (s_high={s_high})"
        plan.close()
    st = srv.stats()
    srv.close()
    print("plan addresses", [hex(x) for x in addresses])
    assert st["graphs"] == 2
    assert not np.array_equal(served[0], served[1])


def test_persistent_launch_in_served_graphs():
    """A complex64 array with flags and one wave per stream (32 stations x 64 channels x 256
    samples: 33 792 streams, no segments) takes the persistent tiled launch, whose flags sit in
    dynamic LDS: served twice (graph captured, then replayed) it gives the direct screen's
    results bit for bit."""
    import torch
    from paper_2412_14775_amd import rfi
    N, C, Tl = 32, 64, 256
    B = N * (N + 1) // 2
    g = torch.Generator(device="cuda:0").manual_seed(5)
    vis = torch.randn((B, C, Tl, 4, 2), generator=g, device="cuda:0", dtype=torch.float32)
    vis[:, 7, 64:80] *= 25.0
    rp = rfi.rfi_params_default(n_stations=N, n_baselines=B, n_channels=C, n_samples=Tl, block_m=16,
                                vis_format=rfi.RFI_VIS_CF32, sk_d=2.2, sk_low=0.4, sk_high=1.8, ds_gamma=0.45)
    plan = rfi.Plan(rp)
    ref = plan.alloc_outputs(flags=True, stats=False)
    plan.screen(vis, ref["avg"], ref["weight"], ref["flags"], None)
    torch.cuda.synchronize()
    want = _host(ref)
    assert want["flags"].any() and not want["flags"].all()
    out = plan.alloc_outputs(flags=True, stats=False)
    srv = rfi.Server(n_slots=2)
    try:
        for rep in range(2):
            for t in out.values():
                if t is not None:
                    t.zero_()
            torch.cuda.synchronize()
            srv.submit(plan, vis, out, tag=rep)
            srv.drain(60)
            assert srv.poll(10)[0]["status"] == 0
            got = _host(out)
            for name in ("avg", "weight", "flags"):
                assert np.array_equal(got[name], want[name], equal_nan=True), (rep, name)
        assert srv.stats()["graphs"] == 1
    finally:
        srv.close()
        plan.close()


def test_admission_respects_the_hbm_budget():
    import torch
    from paper_2412_14775_amd import rfi
    N, C = 5, 16
    plans = [rfi.Plan(_params(N, C)[1]) for _ in range(6)]
    fp = plans[0].footprint()
    srv = rfi.Server(n_slots=8, hbm_budget=int(2.5 * fp))
    vis = to_device(np.zeros((N * (N + 1) // 2, C, T, 4, 2), np.float16), "cf16")
    outs = []
    for i, p in enumerate(plans):
        outs.append(p.alloc_outputs())
        srv.submit(p, vis, outs[-1], arrival=0.0, tag=i)
    srv.drain(60)
    st = srv.stats()
    assert st["completed"] == 6 and st["failed"] == 0
    assert st["peak_inflight_bytes"] <= int(2.5 * fp)
    assert st["peak_inflight"] <= 2
    big = rfi.Server(n_slots=2, hbm_budget=fp - 1)
    with pytest.raises(rfi.RfiError):
        big.submit(plans[0], vis, outs[0], tag=99)
    big.close()
    srv.close()
    torch.cuda.synchronize()
    for p in plans:
        p.close()


def test_direct_launch_mode_matches_graph_mode():
    import torch
    from paper_2412_14775_amd import rfi
    N, C = 4, 8
    _, rp = _params(N, C)
    vis = synth.to_cf16(synth.correlate(synth.make_voltages(synth.Scene(N, C, T, seed=5))))
    dev = to_device(vis, "cf16")
    res = []
    for graphs in (True, False):
        plan = rfi.Plan(rp)
        srv = rfi.Server(n_slots=2, use_graphs=graphs)
        out = plan.alloc_outputs(flags=True, stats=True)
        srv.submit(plan, dev, out, tag=1)
        srv.drain(30)
        assert srv.poll(10)[0]["status"] == 0
        srv.close()
        torch.cuda.synchronize()
        res.append(_host(out))
        plan.close()
    for name in ("avg", "weight", "flags", "stats"):
        assert np.array_equal(res[0][name], res[1][name], equal_nan=True), name


def test_server_holds_the_plan_of_a_request_in_flight():
    """A request whose Plan the caller does not keep (``srv.submit(rfi.Plan(p), ...)``) for a
    future arrival: the server holds the plan until its completion is polled, so the scheduler
    thread and the kernel never see a destroyed plan; the result equals a direct screen."""
    import gc
    import torch
    from paper_2412_14775_amd import rfi
    N, C = 4, 8
    _, rp = make_params(N * (N + 1) // 2, C, T, M, "cf16", d=2.2, s_low=0.5, s_high=1.6, gamma=0.3)
    vis = synth.to_cf16(synth.correlate(synth.make_voltages(synth.Scene(N, C, T, seed=21))))
    dev = to_device(vis, "cf16")
    ref_plan = rfi.Plan(rp)
    ref = ref_plan.alloc_outputs(flags=True, stats=True)
    ref_plan.screen(dev, ref["avg"], ref["weight"], ref["flags"], ref["stats"])
    torch.cuda.synchronize()
    out = ref_plan.alloc_outputs(flags=True, stats=True)
    srv = rfi.Server(n_slots=2)
    try:
        srv.submit(rfi.Plan(rp), dev, out, arrival=srv.now() + 0.3, tag=5)
        gc.collect()                               # the caller holds no reference to that plan
        srv.drain(30)
        done = srv.poll(10)
        assert len(done) == 1 and done[0]["status"] == 0
        got, want = _host(out), _host(ref)
        for name in ("avg", "weight", "flags", "stats"):
            assert np.array_equal(got[name], want[name], equal_nan=True), name
    finally:
        srv.close()
        ref_plan.close()


def test_graph_cache_is_bounded():
    """With room for two graphs, five buffer sets of one plan served in turn (twice over) are
    captured again after eviction, the cache never holds more than two graphs, and every
    result equals the direct screen's."""
    import torch
    from paper_2412_14775_amd import rfi
    N, C = 3, 8
    _, rp = make_params(N * (N + 1) // 2, C, T, M, "cf16", d=2.2, s_low=0.5, s_high=1.6, gamma=0.3)
    vis = synth.to_cf16(synth.correlate(synth.make_voltages(synth.Scene(N, C, T, seed=23))))
    dev = to_device(vis, "cf16")
    plan = rfi.Plan(rp)
    ref = plan.alloc_outputs(flags=True, stats=False)
    plan.screen(dev, ref["avg"], ref["weight"], ref["flags"], None)
    torch.cuda.synchronize()
    want = _host(ref)
    outs = [plan.alloc_outputs(flags=True, stats=False) for _ in range(5)]
    srv = rfi.Server(n_slots=2, max_graphs=2)
    try:
        tag = 0
        for rnd in range(2):
            for o in outs:
                for t in o.values():
                    if t is not None:
                        t.zero_()
                torch.cuda.synchronize()
                srv.submit(plan, dev, o, tag=tag)
                tag += 1
                srv.drain(30)
                assert srv.poll(10)[0]["status"] == 0
                got = _host(o)
                for name in ("avg", "weight", "flags"):
                    assert np.array_equal(got[name], want[name], equal_nan=True), (rnd, name)
                assert srv.stats()["graphs_cached"] <= 2
        st = srv.stats()
        assert st["graphs"] == 10, st              # every buffer set captured again after eviction
    finally:
        srv.close()
        plan.close()


def test_admission_counts_the_statistics_output():
    """A request that writes per-window statistics needs [B][C/F][T/M][3] float32 more than the
    plan's footprint: with a budget of the footprint alone it can never be admitted."""
    from paper_2412_14775_amd import rfi
    N, C = 3, 8
    B = N * (N + 1) // 2
    _, rp = make_params(B, C, T, M, "cf16", d=2.2, s_low=0.5, s_high=1.6, gamma=0.3)
    plan = rfi.Plan(rp)
    fp = plan.footprint()
    out = plan.alloc_outputs(flags=True, stats=True)
    dev = to_device(np.zeros((B, C, T, 4, 2), np.float16), "cf16")
    srv = rfi.Server(n_slots=1, hbm_budget=fp + B * C * (T // M) * 12 - 1)
    try:
        with pytest.raises(rfi.RfiError):
            srv.submit(plan, dev, out, tag=1)
        srv.submit(plan, dev, {"avg": out["avg"], "weight": out["weight"], "flags": out["flags"]}, tag=2)
        srv.drain(30)
        assert srv.poll(10)[0]["status"] == 0
    finally:
        srv.close()
        plan.close()
