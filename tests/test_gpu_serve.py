"""The continuous-batching server on the GPU: every frame's result is the same
alone and in the mix (tolerance 0), batched and plain modes agree, and
admission by HBM budget rejects streams that do not fit."""
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
            img = st.pool[key[1]].cpu().numpy()
            ref[key] = alone(ctx, st.spec, img)
        got = srv.results[r.rid].view(fastgrid.FEATURE_DTYPE)
        assert np.array_equal(got, ref[key]), (r.rid, key)
    # and every served (stream, frame) answer is the oracle's
    assert len(ref) == sum(len(st.pool) for st in srv.streams)
    for (s, k), want_gpu in ref.items():
        st = srv.streams[s]
        img = st.pool[k].cpu().numpy()
        want, _ = oracle.detect_grid(img, st.spec.width, st.spec.levels, st.spec.t, st.spec.n,
                                     st.spec.cell)
        assert np.array_equal(want_gpu, want)
    srv.close()


def test_admission_by_hbm_budget(ctx):
    specs = small_streams()
    need = [serve.resident_bytes(s, 2, 2) for s in specs]
    budget = need[0] + need[1] + need[2] // 2
    srv = serve.Server(ctx, specs, pool_frames=2, slots_per_stream=2, hbm_budget=budget)
    assert len(srv.streams) == 2 and len(srv.rejected) == 2
    assert srv.resident <= budget
    stats = srv.run(0.2, seed=3)
    assert stats["streams_admitted"] == 2 and stats["frames"] == stats["offered_frames"]
    srv.close()
