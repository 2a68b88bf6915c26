"""Serving runtime and its batching primitives on the GPU: the segmented launch
and the device kappa solve equal their single-request forms, every served
result is the same alone and in a mix of concurrent requests (batched and
plain mode), admission respects the arena size and FIFO order, and served
values match the binary128 oracle on a sample."""
import numpy as np
import pytest
import torch

from parity import TOL32, TOL64, cond_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the -m gpu tests need an MI355X")
    import paper_2409_08729_amd as m
    m.lib()
    return m


SIZES = [0, 1, 63, 2047, 2048, 2049, 7000, 100_003]


@pytest.mark.parametrize("inline", [False, True])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", ["I", "K"])
def test_segmented_launch_equals_single_array(lb, kind, dtype, inline):
    from paper_2409_08729_amd import workloads as wl
    v, x = wl.serving_pool(sum(SIZES), seed=11)
    vs, xs, at = [], [], 0
    for n in SIZES:
        vs.append(torch.from_numpy(v[at:at + n]).to("cuda:0", dtype))
        xs.append(torch.from_numpy(x[at:at + n]).to("cuda:0", dtype))
        at += n
    outs = lb.eval_segments(kind, vs, xs, inline=inline)
    f = lb.log_iv if kind == "I" else lb.log_kv
    for vv, xx, o in zip(vs, xs, outs):
        ref = f(vv, xx)
        assert torch.equal(torch.isnan(o), torch.isnan(ref))
        assert torch.equal(torch.nan_to_num(o), torch.nan_to_num(ref)), (kind, dtype, xx.numel())


@pytest.mark.parametrize("p", [3, 2048, 8192])
def test_device_kappa_solve_matches_host_newton(lb, oracle, p):
    import math
    from paper_2409_08729_amd import vmf, workloads as wl
    X = wl.vmf_features(3000, p, seed=p + 1, device="cuda:0")
    k, R, k0, steps = lb.vmf_fit(X)
    _, R_host = vmf.mean_resultant(X)
    assert R == R_host                       # same column-sum kernels, same bits
    ks = vmf.kappa_estimates(R, p)
    assert abs(k0 - ks[0]) <= 1e-13 * ks[0]
    assert 1 <= steps <= 12                  # quadratic convergence, then the noise floor
    # both solves end inside the noise band of the root: A_p(kappa) = R with
    # A_p from log-values of size ~kappa (relative error ~kappa * 1e-16)
    assert abs(k - ks[-1]) <= 1e-9 * ks[-1], (k, ks[-1])
    v = np.array([p / 2 - 1, p / 2])
    hi, lo = oracle.log_iv(v, np.array([k, k]))
    a_ref = math.exp((hi[1] - hi[0]) + (lo[1] - lo[0]))
    s = sum(max(abs(h), 1 + math.hypot(vv, k)) for h, vv in zip(hi, v))
    assert abs(a_ref - R) <= TOL64 * s * a_ref + 1e-15, (p, k, a_ref, R)


def _pinned(a: np.ndarray) -> torch.Tensor:
    t = torch.empty(a.shape, dtype=torch.float64 if a.dtype == np.float64 else torch.float32,
                    pin_memory=True)
    t.copy_(torch.from_numpy(a))
    return t


def _make_requests(count, seed, max_pairs=200_000, vmf_rows=(200, 3000)):
    from paper_2409_08729_amd import workloads as wl
    reqs, _ = wl.serving_requests(count, seed=seed, max_pairs=max_pairs, pool=1 << 20,
                                  vmf_rows=vmf_rows)
    v, x = wl.serving_pool(1 << 20, seed=seed + 1)
    feats = {p: wl.vmf_features(vmf_rows[1], p, seed=p, device="cuda:0")
             for p in wl.SERVE_VMF_DIMS}
    for r in reqs:
        if r["type"] == "eval":
            dt = np.float64 if r["precision"] == 64 else np.float32
            sl = slice(r["offset"], r["offset"] + r["n"])
            r["v"] = _pinned(v[sl].astype(dt))
            r["x"] = _pinned(x[sl].astype(dt))
        else:
            r["X"] = feats[r["p"]][: r["N"]]
    return reqs


def _fresh_outputs(reqs):
    for r in reqs:
        if r["type"] == "eval":
            r["out"] = torch.full_like(r["v"], float("nan")).pin_memory()
        else:
            r["result"] = torch.full((4,), float("nan"), dtype=torch.float64).pin_memory()


def _items(reqs, times):
    out = []
    for r, t in zip(reqs, times):
        it = {"t": t, "type": r["type"]}
        if r["type"] == "eval":
            it.update(kind=r["kind"], v=r["v"], x=r["x"], out=r["out"])
        else:
            it.update(X=r["X"], result=r["result"])
        out.append(it)
    return out


def _snapshot(reqs):
    return [(r["out"] if r["type"] == "eval" else r["result"]).clone() for r in reqs]


def _same_bits(a: torch.Tensor, b: torch.Tensor) -> bool:
    if a.dtype != b.dtype or a.shape != b.shape:
        return False
    if a.numel() == 0:
        return True
    it = torch.int64 if a.dtype == torch.float64 else torch.int32
    return torch.equal(a.contiguous().view(it), b.contiguous().view(it))


def test_results_same_alone_and_in_mix(lb):
    from paper_2409_08729_amd import serve
    reqs = _make_requests(48, seed=5)
    assert any(r["type"] == "vmf" for r in reqs) and any(r["type"] == "eval" for r in reqs)
    # alone: one request at a time through a batched server
    _fresh_outputs(reqs)
    with serve.Server("batched", arena_bytes=1 << 30) as srv:
        for r in reqs:
            t = (srv.submit_eval(r["kind"], r["v"], r["x"], r["out"]) if r["type"] == "eval"
                 else srv.submit_vmf(r["X"], r["result"]))
            info = srv.wait(t, timeout=60)
            assert info["status"] == 0
    alone = _snapshot(reqs)
    # mixed: everything arrives at once; batches form and overlap
    for mode in ("batched", "plain"):
        _fresh_outputs(reqs)
        with serve.Server(mode, arena_bytes=1 << 30, streams=4) as srv:
            infos = srv.replay(_items(reqs, [0.0] * len(reqs)), timeout=120)
            st = srv.stats()
        assert all(i["status"] == 0 and i["state"] == 3 for i in infos)
        assert st["completed"] == len(reqs)
        if mode == "batched":
            assert st["batches"] < len(reqs) and st["max_batch_requests_seen"] > 1, st
        else:
            assert st["batches"] == len(reqs) and st["max_batch_requests_seen"] == 1, st
        for r, a, b in zip(reqs, alone, _snapshot(reqs)):
            assert _same_bits(a, b), (mode, r["type"], r.get("kind"), r.get("n"), r.get("p"))
    # and the served values are what the library gives for the request directly
    for r, a in zip(reqs, alone):
        if r["type"] == "eval":
            f = lb.log_iv if r["kind"] == "I" else lb.log_kv
            ref = f(r["v"].to("cuda:0"), r["x"].to("cuda:0")).cpu()
            assert _same_bits(a, ref)
        else:
            k, R, k0, steps = lb.vmf_fit(r["X"])
            assert a.tolist() == [k, R, k0, float(steps)]


def test_served_values_match_oracle(lb, oracle):
    from paper_2409_08729_amd import serve
    reqs = [r for r in _make_requests(24, seed=9, max_pairs=50_000) if r["type"] == "eval"]
    _fresh_outputs(reqs)
    with serve.Server("batched", arena_bytes=1 << 28) as srv:
        srv.replay(_items(reqs, [0.0] * len(reqs)), timeout=120)
    g = np.random.default_rng(3)
    for r in reqs:
        n = r["n"]
        idx = g.choice(n, size=min(n, 300), replace=False)
        v = r["v"].numpy()[idx].astype(np.float64)
        x = r["x"].numpy()[idx].astype(np.float64)
        got = r["out"].numpy()[idx].astype(np.float64)
        hi, lo = (oracle.log_iv if r["kind"] == "I" else oracle.log_kv)(v, x)
        tol = TOL64 if r["precision"] == 64 else TOL32
        fin = np.isfinite(hi)
        assert np.array_equal(np.isfinite(got), fin), r["kind"]
        err = cond_err(got[fin], hi[fin], lo[fin], v[fin], x[fin])
        assert err.size == 0 or err.max() <= tol, (r["kind"], r["precision"], err.max())


def test_admission_by_memory_is_fifo_and_bounded(lb):
    from paper_2409_08729_amd import serve
    g = np.random.default_rng(17)
    reqs = []
    for i in range(40):
        n = int(g.integers(20_000, 60_000))
        reqs.append({"type": "eval", "kind": "IK"[i % 2], "n": n,
                     "v": _pinned(g.uniform(0, 50, n)), "x": _pinned(g.uniform(0.1, 80, n))})
    _fresh_outputs(reqs)
    arena = 4 << 20                       # room for two or three requests at a time
    with serve.Server("batched", arena_bytes=arena, streams=3) as srv:
        infos = srv.replay(_items(reqs, [0.0] * len(reqs)), timeout=120)
        st = srv.stats()
        with pytest.raises(lb.LbesselError, match="larger than the server arena"):
            big = torch.zeros(1 << 20, dtype=torch.float64)
            srv.submit_eval("I", big, big, big.clone())
    assert all(i["status"] == 0 for i in infos)
    assert st["arena_peak_bytes"] <= arena
    assert st["queue_peak"] > 1                            # requests did wait for memory
    admits = [i["t_admit"] for i in infos]
    assert admits == sorted(admits)                        # FIFO admission
    assert all(i["t_arrival"] <= i["t_submit"] <= i["t_admit"] <= i["t_launch"] <= i["t_done"]
               for i in infos)
    for r in reqs:
        f = lb.log_iv if r["kind"] == "I" else lb.log_kv
        assert _same_bits(r["out"], f(r["v"].to("cuda:0"), r["x"].to("cuda:0")).cpu())


def test_empty_and_tiny_requests(lb):
    from paper_2409_08729_amd import serve
    e = torch.empty(0, dtype=torch.float64).pin_memory()
    one_v = torch.tensor([2.5], dtype=torch.float64).pin_memory()
    one_x = torch.tensor([3.0], dtype=torch.float64).pin_memory()
    out = torch.empty(1, dtype=torch.float64).pin_memory()
    with serve.Server("batched", arena_bytes=1 << 20) as srv:
        t0 = srv.submit_eval("K", e, e, e.clone())
        t1 = srv.submit_eval("I", one_v, one_x, out)
        assert srv.wait(t0, 30)["status"] == 0
        assert srv.wait(t1, 30)["status"] == 0
    assert out.item() == lb.log_iv(one_v.cuda(), one_x.cuda()).item()


def test_large_requests_and_fits_go_out_alone(lb):
    """Evaluation requests of at least solo_elems pairs and vMF fits form a
    batch of their own; smaller evaluation requests still share batches."""
    from paper_2409_08729_amd import serve
    reqs = _make_requests(64, seed=21, max_pairs=300_000)
    _fresh_outputs(reqs)
    solo = 1 << 15
    with serve.Server("batched", arena_bytes=1 << 30, solo_elems=solo) as srv:
        infos = srv.replay(_items(reqs, [0.0] * len(reqs)), timeout=120)
    assert all(i["status"] == 0 for i in infos)
    members = {}
    for r, i in zip(reqs, infos):
        members.setdefault(i["batch"], []).append(r)
    for r, i in zip(reqs, infos):
        if r["type"] == "vmf" or r["n"] >= solo:
            assert len(members[i["batch"]]) == 1, (r["type"], r.get("n"))
    assert any(len(m) > 1 for m in members.values())


def test_device_resident_requests_same_alone_and_in_mix(lb):
    """Evaluation requests whose arrays live on the GPU (no copies): the same
    bits alone, in a batched mix (batches of more and of fewer than 32
    requests: device and inline segment tables) and in plain mode, and the
    same as the single-array entry point."""
    from paper_2409_08729_amd import serve, workloads as wl
    g = np.random.default_rng(31)
    v, x = wl.serving_pool(1 << 20, seed=32)
    reqs = []
    for i in range(80):
        n = int(np.exp(g.uniform(0.0, np.log(20_000))))
        at = int(g.integers(0, v.size - n))
        dt = torch.float64 if i % 3 else torch.float32
        reqs.append({"type": "eval_device", "kind": "IK"[i % 2],
                     "v": torch.from_numpy(v[at:at + n]).to("cuda:0", dt),
                     "x": torch.from_numpy(x[at:at + n]).to("cuda:0", dt)})
    reqs.append({"type": "eval_device", "kind": "K",
                 "v": torch.empty(0, dtype=torch.float64, device="cuda:0"),
                 "x": torch.empty(0, dtype=torch.float64, device="cuda:0")})

    def fresh():
        for r in reqs:
            r["out"] = torch.full_like(r["v"], float("nan"))
        torch.cuda.synchronize()

    fresh()
    with serve.Server("batched", arena_bytes=1 << 20) as srv:
        for r in reqs:
            t = srv.submit_eval_device(r["kind"], r["v"], r["x"], r["out"])
            assert srv.wait(t, timeout=60)["status"] == 0
    alone = [r["out"].clone() for r in reqs]
    for r, a in zip(reqs, alone):
        f = lb.log_iv if r["kind"] == "I" else lb.log_kv
        assert _same_bits(a, f(r["v"], r["x"])), (r["kind"], r["v"].dtype, r["v"].numel())
    for mode, cap in (("batched", 64), ("batched", 8), ("plain", 64)):
        fresh()
        items = [{"t": 0.0, "type": "eval_device", "kind": r["kind"], "v": r["v"], "x": r["x"],
                  "out": r["out"]} for r in reqs]
        # the arena holds no request data: a tiny one admits everything
        with serve.Server(mode, arena_bytes=1 << 16, streams=4,
                          max_batch_requests=cap) as srv:
            infos = srv.replay(items, timeout=120)
            st = srv.stats()
        assert all(i["status"] == 0 and i["state"] == 3 for i in infos)
        if mode == "batched":
            assert st["max_batch_requests_seen"] > 1, st
        for r, a in zip(reqs, alone):
            assert _same_bits(a, r["out"]), (mode, cap, r["kind"], r["v"].numel())
