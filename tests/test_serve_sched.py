"""The request loop's scheduling, batching and admission on the CPU: the
server runs with a simulated executor (no device work; a batch occupies one
shared simulated device for fixed + per-megapixel time), so the policy code
is the one the GPU server runs."""
import numpy as np
import pytest
import torch

import synth
from paper_2505_22335_amd import _lib as L
from paper_2505_22335_amd.serve import MAP, TRACK, RequestSpec, Server, latency_summary, poisson_arrivals

A, K = 50_000, 10
FAKE = torch.zeros(16)  # stands for device buffers: the simulated executor never touches them


def _track(cam, arrival=-1.0):
    return RequestSpec(TRACK, [cam], [FAKE], [FAKE], d_pose=FAKE, arrival=arrival)


def _map(cams, arrival=-1.0):
    n = len(cams)
    return RequestSpec(MAP, cams, [FAKE] * n, [FAKE] * n, d_pose=FAKE, d_xyz=FAKE, d_feat=FAKE, d_off=FAKE,
                       d_params=FAKE, arrival=arrival)


def _server(**kw):
    base = dict(n_anchors=A, k=K, n_feat=16, simulate=True, sim_us_fixed=300.0, sim_us_per_mpix=1000.0,
                arena_bytes=64 << 30)
    base.update(kw)
    return Server(None, **base)


def test_all_complete_and_tracking_fuses_under_load():
    cam = synth.camera_c2()
    with _server(n_streams=2, max_batch_views=8) as s:
        specs = [_track(cam, arrival=0.0002 * i) for i in range(40)]
        res = s.replay(specs)
        st = s.stats()
    assert all(r.status == 0 for r in res)
    assert st.completed == 40 and st.failed == 0
    assert st.batches < 40                     # requests arriving together were fused
    assert max(r.batch_views for r in res) <= 8
    assert all(r.done >= r.start >= r.arrival - 1e-4 for r in res)


def test_fifo_runs_one_request_at_a_time():
    cam = synth.camera_c2()
    with _server(n_streams=1, max_batch_views=1, fifo=True) as s:
        res = s.replay([_track(cam, arrival=0.0) for _ in range(10)])
        st = s.stats()
    assert st.max_in_flight == 1 and st.batches == 10
    done = sorted(r.done for r in res)
    svc = (300.0 + 1000.0 * 0.3072) * 1e-6
    # the k-th completion cannot come before k service times
    for i, d in enumerate(done):
        assert d - min(r.arrival for r in res) >= (i + 1) * svc * 0.99


def test_admission_respects_the_arena():
    cam = synth.camera_c2()
    with _server(n_streams=1, max_batch_views=1) as s:     # one request's footprint
        s.replay([_track(cam, arrival=0.0)])
        one = s.stats().arena_peak
    assert one > 0
    with _server(n_streams=4, max_batch_views=1, arena_bytes=int(2.5 * one)) as s:
        res = s.replay([_track(cam, arrival=0.0) for _ in range(12)])
        st = s.stats()
    assert all(r.status == 0 for r in res)
    assert st.arena_peak <= st.arena_bytes
    assert 1 <= st.max_in_flight <= 2           # memory, not streams, bounded the overlap


def test_request_larger_than_arena_fails_cleanly():
    cams = [synth.camera_c2()] * 16
    with _server(n_streams=2, arena_bytes=256 << 20) as s:
        t = s.submit(_map(cams))
        r = s.wait(t)
        t2 = s.submit(_track(synth.camera_half(cams[0].T_wc)))
        r2 = s.wait(t2)
    assert r.status == L.E_CAPACITY
    assert r2.status in (0, L.E_CAPACITY)


def test_invalid_requests_rejected_at_submit():
    cam = synth.camera_c2()
    with _server() as s:
        bad = _track(cam)
        bad.cams = [cam, cam]
        with pytest.raises(L.AsgsError):
            s.submit(bad)
        m = _map([cam, cam])
        m.d_params = None
        with pytest.raises(L.AsgsError):
            s.submit(m)
        mixed = _map([cam, synth.camera_c1()])
        with pytest.raises(L.AsgsError):
            s.submit(mixed)


def test_mixed_trace_and_latency_summary():
    rng = np.random.default_rng(5)
    cam = synth.camera_c2()
    half = synth.camera_half(cam.T_wc)
    tr = poisson_arrivals(rng, 300.0, 0.5)
    mp = poisson_arrivals(rng, 20.0, 0.5)
    ev = sorted([(t, TRACK) for t in tr] + [(t, MAP) for t in mp])
    specs, kinds = [], []
    for t, kind in ev:
        if kind == TRACK:
            specs.append(_track(cam, t))
        else:
            B = int(rng.integers(4, 17))
            specs.append(_map([cam if rng.random() < 0.5 else half] * B, t))
        kinds.append(kind)
    with _server(n_streams=3, max_batch_views=16) as s:
        res = s.replay(specs)
        st = s.stats()
    summ = latency_summary(res, kinds)
    assert summ["failed"] == 0
    assert summ["track"]["p99_ms"] >= summ["track"]["p50_ms"] > 0
    assert st.completed == len(specs)
    # every mapping request ran as its own batch
    assert all(r.batch_views >= 4 for r, k in zip(res, kinds) if k == MAP)
