"""The continuous-batching server on the GPU: every frame's result is the same
alone and in the mix (tolerance 0) and equals the oracle's, batched and plain
modes agree, admission by HBM budget keeps out streams that do not fit, and a
stream kept out at the start is admitted once a departing stream releases its
bytes, with every result still the oracle's."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2003_13493_amd import fastgrid, serve, synth  # noqa: E402


def small_streams():
    sizes = [(320, 240, 3, 16), (640, 480, 4, 32), (376, 240, 5, 16), (752, 480, 3, 64)]
    out = []
    for i, (w, h, L, cell) in enumerate(sizes):
        out.append(synth.StreamSpec(i, w, h, L, synth.BATCH_T[i % 4], synth.BATCH_N[i % 3], cell,
                                    rate_fps=400.0 + 150 * i, seed=7000 + i))
    return out


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = fastgrid.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def alone(ctx, spec, img):
    pyr = fastgrid.Pyramid(spec.width, spec.height, spec.levels)
    pyr.upload(img)
    g = fastgrid.Grid(spec.width, spec.height, spec.cell)
    ctx.detect(pyr, spec.t, spec.n, spec.cell, g)
    torch.cuda.synchronize()
    return g.fetch()


@pytest.mark.parametrize("batched", [True, False], ids=["batched", "plain"])
def test_native_loop_results_are_the_oracles(ctx, batched):
    """fast_pump_run serves the same arrivals with the loop in the library:
    every request is served, no earlier than it arrived, and every result
    slot holds the oracle's answer for the frame of the last request it
    served, both on the device and in its pinned host copy."""
    specs = small_streams()
    srv = serve.Server(ctx, specs, pool_frames=2, slots_per_stream=3, max_batch=16, inflight=3)
    print(f"case native loop batched={batched}", flush=True)
    stats = srv.run_native(0.4, seed=11, batched=batched)
    assert stats["frames"] == stats["offered_frames"] > 50
    assert stats["batches"] >= (1 if batched else stats["frames"])
    assert stats["latency_ms"]["p50"] > 0
    served, slot_of = stats["served"], stats["slot_of"]
    assert (slot_of >= 0).all() and (slot_of < 3).all()
    last = {}
    for r, (_, s, k) in enumerate(served):
        last[(s, int(slot_of[r]))] = k
    assert len(last) >= 8
    for (s, slot), k in sorted(last.items()):
        st, spec = srv.streams[s], srv.specs[s]
        want, _ = oracle.detect_grid(st.host_pool[k % len(st.pool)], spec.width, spec.levels, spec.t, spec.n,
                                     spec.cell)
        sl = st.slots[slot]
        assert np.array_equal(sl.host.numpy().view(fastgrid.FEATURE_DTYPE), want), (s, slot, k)
        assert np.array_equal(sl.grid.cpu().numpy().view(fastgrid.FEATURE_DTYPE), want), (s, slot, k)


def test_native_loop_rejects_bad_arguments(ctx):
    specs = small_streams()[:1]
    srv = serve.Server(ctx, specs, pool_frames=1, slots_per_stream=1, max_batch=4, inflight=1)
    st, spec = srv.streams[0], specs[0]
    pool = (fastgrid.fast_plane * 1)(*st.pool_planes)
    upper = (fastgrid.fast_plane * (spec.levels - 1))(*st.slots[0].planes[1:spec.levels])
    import ctypes
    out = (ctypes.c_void_p * 1)(st.slots[0].grid.data_ptr())
    arr = (fastgrid.fast_pump_stream * 1)(fastgrid.fast_pump_stream(
        spec.levels, spec.t, spec.n, spec.cell, 0, 1, pool, 1, upper, out, None))
    good = (fastgrid.fast_pump_request * 2)(fastgrid.fast_pump_request(0, 0, 0.0),
                                             fastgrid.fast_pump_request(0, 1, 0.001))
    done, slot, nb = fastgrid.fast_pump_run(ctx.handle, arr, 1, good, 2, 1, 4, True, 5.0)
    assert (done > 0).all() and nb == 2
    bad_order = (fastgrid.fast_pump_request * 2)(fastgrid.fast_pump_request(0, 0, 0.01),
                                                  fastgrid.fast_pump_request(0, 1, 0.0))
    bad_stream = (fastgrid.fast_pump_request * 1)(fastgrid.fast_pump_request(1, 0, 0.0))
    for args in ((arr, 1, bad_order, 2, 1, 4), (arr, 1, bad_stream, 1, 1, 4), (arr, 1, good, 2, 9, 4),
                 (arr, 1, good, 2, 0, 4), (arr, 1, good, 2, 1, 0), (arr, 1, good, 0, 1, 4)):
        with pytest.raises(fastgrid.FastError) as ei:
            fastgrid.fast_pump_run(ctx.handle, args[0], args[1], args[2], args[3], args[4], args[5], True, 5.0)
        assert ei.value.code == fastgrid.FAST_EINVAL
    # arrivals later than the run's time limit: the loop gives up, launching nothing
    late = (fastgrid.fast_pump_request * 1)(fastgrid.fast_pump_request(0, 0, 5.0))
    with pytest.raises(fastgrid.FastError) as ei:
        fastgrid.fast_pump_run(ctx.handle, arr, 1, late, 1, 1, 4, True, 0.02)
    assert ei.value.code == fastgrid.FAST_ETIMEDOUT
    torch.cuda.synchronize()


@pytest.mark.parametrize("batched", [True, False], ids=["batched", "plain"])
def test_native_loop_runs_back_to_back(ctx, batched):
    """Several serving-loop runs in a row, each with more launches than the
    context tracks submissions (256), so every run recycles completion events
    of the one before.  The loop's launch streams live as long as the
    context, so each run succeeds and serves every frame."""
    specs = small_streams()[:1]
    srv = serve.Server(ctx, specs, pool_frames=1, slots_per_stream=1, max_batch=1, inflight=1)
    st, spec = srv.streams[0], specs[0]
    pool = (fastgrid.fast_plane * 1)(*st.pool_planes)
    upper = (fastgrid.fast_plane * (spec.levels - 1))(*st.slots[0].planes[1:spec.levels])
    import ctypes
    out = (ctypes.c_void_p * 1)(st.slots[0].grid.data_ptr())
    arr = (fastgrid.fast_pump_stream * 1)(fastgrid.fast_pump_stream(
        spec.levels, spec.t, spec.n, spec.cell, 0, 1, pool, 1, upper, out, None))
    n = 300
    reqs = (fastgrid.fast_pump_request * n)(*[fastgrid.fast_pump_request(0, k, 0.0) for k in range(n)])
    for run in range(3):
        print(f"case native back-to-back batched={batched} run {run}", flush=True)
        done, slot, nb = fastgrid.fast_pump_run(ctx.handle, arr, 1, reqs, n, 1, 1, batched, 30.0)
        assert (done > 0).all() and nb == n
    torch.cuda.synchronize()


@pytest.mark.parametrize("batched,upload", [(True, False), (False, False), (True, True)],
                         ids=["batched", "plain", "batched_upload"])
def test_each_result_same_alone_and_in_mix(ctx, batched, upload):
    specs = small_streams()
    srv = serve.Server(ctx, specs, pool_frames=2, slots_per_stream=3, max_batch=16, inflight=3,
                       keep_results=True, upload=upload)
    print(f"case serve batched={batched} upload={upload}", flush=True)
    stats = srv.run(0.4, seed=11, batched=batched)
    assert stats["frames"] == stats["offered_frames"] > 50
    assert stats["latency_ms"]["p50"] is not None
    if batched:
        assert stats["mean_batch"] >= 1.0
    ref = {}
    for r in stats["requests"]:
        st = srv.streams[r.stream]
        key = (r.stream, r.frame % len(st.pool))
        if key not in ref:
            ref[key] = alone(ctx, st.spec, st.host_pool[key[1]])
        got = srv.results[r.rid].view(fastgrid.FEATURE_DTYPE)
        assert np.array_equal(got, ref[key]), (r.rid, key)
    # and every served (stream, frame) answer is the oracle's
    assert len(ref) == sum(len(st.pool) for st in srv.streams if st is not None)
    for (s, k), want_gpu in ref.items():
        spec = srv.specs[s]
        want, _ = oracle.detect_grid(srv.streams[s].host_pool[k], spec.width, spec.levels, spec.t,
                                     spec.n, spec.cell)
        assert np.array_equal(want_gpu, want)
    srv.close()


def test_admission_by_hbm_budget(ctx):
    specs = small_streams()
    need = [serve.resident_bytes(s, 2, 2) for s in specs]
    budget = need[0] + need[1] + need[2] // 2
    srv = serve.Server(ctx, specs, pool_frames=2, slots_per_stream=2, hbm_budget=budget)
    assert len(srv.admitted) == 2 and len(srv.rejected) == 2
    assert [i for i, st in enumerate(srv.streams) if st is not None] == [0, 1]
    assert srv.resident <= budget
    stats = srv.run(0.2, seed=3)
    assert stats["streams_admitted"] == 2
    # frames of the streams kept out are refused, the rest all served
    assert stats["frames"] + stats["refused_frames"] == stats["offered_frames"]
    assert set(stats["refused_by_stream"]) == {2, 3}
    srv.close()


def test_waiting_stream_admitted_when_another_leaves(ctx):
    """Streams 0 and 1 fit at the start, 2 and 3 wait.  Stream 0 leaves at
    0.15 s; once its last request completes its bytes are released and stream
    2 (which fits in them) is admitted mid-run; 3 never fits.  Every served
    frame, before and after the change, is the oracle's answer."""
    specs = small_streams()
    need = [serve.resident_bytes(s, 2, 2) for s in specs]
    budget = need[1] + need[2]
    assert need[0] <= need[2] and need[0] + need[1] + need[2] > budget and need[1] + need[3] > budget
    srv = serve.Server(ctx, specs, pool_frames=2, slots_per_stream=2, hbm_budget=budget,
                       max_batch=16, inflight=3, keep_results=True)
    assert [i for i, st in enumerate(srv.streams) if st is not None] == [0, 1]
    assert srv.waiting == [2, 3]
    print("case serve join/leave", flush=True)
    trace = []
    stats = srv.run(0.5, seed=21, leave={0: 0.15}, trace=trace)
    log = srv.admission_log
    rel = [t for t, i, what in log if i == 0 and what == "released"]
    adm = [t for t, i, what in log if i == 2 and what == "admitted"]
    assert len(rel) == 1 and len(adm) == 1 and 0.15 <= rel[0] <= adm[0] < 0.5, log
    assert srv.streams[0] is None and srv.streams[2] is not None and srv.streams[3] is None
    assert srv.waiting == [3] and srv.resident == need[1] + need[2] <= budget
    served = {s: [r for r in stats["requests"] if r.stream == s] for s in range(4)}
    assert served[0] and all(r.arrival < 0.15 for r in served[0])
    assert served[2] and all(r.arrival >= adm[0] for r in served[2])
    assert not served[3] and stats["refused_by_stream"].get(3, 0) > 0
    assert stats["refused_by_stream"].get(2, 0) > 0          # sent while still waiting
    assert len(trace) == stats["batches"] and all(b["device_ms"] >= 0 for b in trace)
    want = {}
    for r in stats["requests"]:
        spec = specs[r.stream]
        k = r.frame % 2
        if (r.stream, k) not in want:
            want[(r.stream, k)] = oracle.detect_grid(spec.frame(k), spec.width, spec.levels, spec.t,
                                                     spec.n, spec.cell)[0]
        got = srv.results[r.rid].view(fastgrid.FEATURE_DTYPE)
        assert np.array_equal(got, want[(r.stream, k)]), (r.rid, r.stream, k)
    srv.close()


class TexturedStream:
    """A stream spec whose pool frames are crops of a textured scene along a
    random walk (well-posed tracks, as in the front-end tests)."""

    def __init__(self, index, width, height, levels, t, n, cell, rate_fps, seed):
        from test_gpu_frontend_multi import sequence
        self.index, self.width, self.height, self.levels = index, width, height, levels
        self.t, self.n, self.cell, self.rate_fps = t, n, cell, rate_fps
        self._frames = sequence(width, height, 3, seed)

    def frame(self, k):
        return self._frames[k % 3]


def test_frontend_serving_matches_oracle_loop(ctx):
    """Frontend serving: every stream's frames go through the detect-and-track
    loop in arrival order, batched across streams, with device-resident
    feature lists.  Each served step equals the oracle step applied to the
    feature list the stream held before it (the previous step's result):
    identical counts and decisions, kept positions within the tracker
    tolerance, and exactly the oracle's added features."""
    from test_gpu_frontend_multi import check_step, oracle_step
    specs = [TexturedStream(0, 320, 240, 3, 10, 9, 16, 150.0, 91),
             TexturedStream(1, 640, 480, 4, 8, 10, 32, 200.0, 92),
             TexturedStream(2, 376, 240, 3, 15, 12, 16, 250.0, 93)]
    fp = serve.FrontendParams(target=60, redetect_frac=0.5, mode=3, max_iter=30, eps=1e-3)
    srv = serve.Server(ctx, specs, pool_frames=3, max_batch=16, inflight=3, keep_results=True, frontend=fp)
    print("case serve frontend", flush=True)
    stats = srv.run(0.1, seed=5)
    assert stats["mode"] == "frontend" and stats["frames"] == stats["offered_frames"] > 20
    tracked = 0
    for s, spec in enumerate(specs):
        reqs = sorted((r for r in stats["requests"] if r.stream == s), key=lambda r: r.arrival)
        assert [r.done for r in reqs] == sorted(r.done for r in reqs)          # served in order
        prev, feats_in = None, np.zeros((0, 2))
        for f, r in enumerate(reqs):
            info, feats = srv.results[r.rid]
            info = (int(info[0]), bool(info[1]), int(info[2]))
            feats = feats.astype(np.float64)
            want = oracle_step(prev, spec.frame(r.frame), feats_in, spec.width, spec.levels, spec.t, spec.n,
                               spec.cell, fp.target, fp.redetect_frac, fp.mode, fp.eps, kept_device=feats[:info[0]])
            check_step(f"stream {s} frame {f}", info, feats, want)
            tracked += info[0]
            prev, feats_in = want[4], feats
    assert tracked > 0
    srv.close()


def test_native_frontend_loop_equals_the_python_loop(ctx):
    """fast_pump_run_frontend serves the same arrivals as the Python loop
    (whose steps the test above checks against the oracle).  A stream's
    computation does not depend on which streams share its launches, so every
    stream ends with the same feature list and step summary, bit for bit, and
    its frames are served in order."""
    specs = [TexturedStream(0, 320, 240, 3, 10, 9, 16, 150.0, 91),
             TexturedStream(1, 640, 480, 4, 8, 10, 32, 200.0, 92),
             TexturedStream(2, 376, 240, 3, 15, 12, 16, 250.0, 93)]
    fp = serve.FrontendParams(target=60, redetect_frac=0.5, mode=3, max_iter=30, eps=1e-3)
    print("case serve frontend native", flush=True)
    py = serve.Server(ctx, specs, pool_frames=3, max_batch=16, inflight=3, frontend=fp)
    a = py.run(0.1, seed=5)
    nat = serve.Server(ctx, specs, pool_frames=3, max_batch=16, inflight=3, frontend=fp)
    b = nat.run_native(0.1, seed=5)
    torch.cuda.synchronize()
    assert b["mode"] == "frontend-native" and b["frames"] == a["frames"] > 20
    for s in range(len(specs)):
        fa, fb = py.streams[s].fe, nat.streams[s].fe
        na, nb = int(fa.count.cpu()[0]), int(fb.count.cpu()[0])
        assert na == nb, s
        assert np.array_equal(fa.info.cpu().numpy(), fb.info.cpu().numpy()), s
        assert np.array_equal(fa.info_host.numpy(), fb.info_host.numpy()), s
        assert torch.equal(fa.feats[:na].cpu(), fb.feats[:nb].cpu()), s
        done = [d for d, (_, st, _) in zip(b["done_s"], b["served"]) if st == s]
        assert done == sorted(done), s   # a stream's frames complete in arrival order
    assert b["frames"] == sum(fb.frames for fb in (nat.streams[s].fe for s in range(len(specs))))
    py.close()
    nat.close()
