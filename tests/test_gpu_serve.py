"""Serving loop on the GPU: a request served inside a continuous batch
(several scenes and image sizes in one launch, two streams) gets the image
it gets when rendered alone, bit for bit; the plain one-launch-per-view path
gives the same images; a small HBM budget queues requests without ever
exceeding it and rejects one that can never fit; under-sized capacities are
caught from the status header and the launch is re-run before its requests
complete."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

SIZES = (64, 128, 256)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _registry(margin=1.5):
    from paper_2406_01579_amd.serve import SceneRegistry
    reg = SceneRegistry(margin=margin)
    rng = np.random.default_rng(11)
    for sc in synth.serving_scenes(n_scenes=4, res=(16, 24, 32)):
        probe = np.concatenate([synth.random_orbit_cameras(rng, 2, s) for s in SIZES], 0)
        reg.add(sc, probe)
    return reg


def _trace(n=48, rate=4000.0):
    return synth.serving_requests(n, rate, 4, sizes=SIZES, seed=7)


def _alone(reg, req):
    import torch
    from paper_2406_01579_amd import Renderer
    plan = Renderer(reg.params, check="sync").forward([reg.scenes[req.scene]], req.cams)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in plan.outs]


def _images(req):
    return [o.cpu().numpy() for o in req.outs]


def test_batched_request_equals_request_alone_and_plain_path():
    from paper_2406_01579_amd.serve import Server
    reg = _registry()
    srv = Server(reg, streams=2)
    st = srv.run(_trace())
    print(st)
    assert st["served"] == st["requests"] == 48
    assert st["batches"] < 48 and st["mean_views_per_batch"] > 2.5   # batching happened
    plain = Server(reg, streams=1, batching=False)
    sp = plain.run(_trace())
    print(sp)
    assert sp["launches"] == sum(r.views for r in plain.requests)
    for r, q in zip(srv.requests, plain.requests):
        a = _images(r)
        assert len(a) == r.views
        for x, y, z in zip(a, _alone(reg, r), _images(q)):
            assert np.array_equal(x, y) and np.array_equal(x, z), r.id


def test_small_budget_queues_and_rejects():
    from paper_2406_01579_amd.serve import Server
    reg = _registry()
    probe = Server(reg)
    tr = _trace(24)
    fps = [probe.footprint(sc, cams) for _, sc, cams in tr]
    budget = int(max(fps) * 1.2)
    srv = Server(reg, streams=2, budget_bytes=budget)
    st = srv.run(tr)
    assert st["served"] == 24 and st["max_in_flight_bytes"] <= budget
    assert st["max_queue"] > 1
    big = np.concatenate([synth.random_orbit_cameras(np.random.default_rng(1), 4, 1024)], 0)
    r = srv.submit(0, big)
    srv.drain()
    assert r.error is not None and r.done_at is None
    for q in srv.requests[:24]:
        for x, y in zip(_images(q), _alone(reg, q)):
            assert np.array_equal(x, y)


def test_undersized_capacities_are_rerun():
    from paper_2406_01579_amd.serve import Server
    reg = _registry(margin=0.02)
    srv = Server(reg, streams=2)
    st = srv.run(_trace(16))
    print(st)
    assert st["served"] == 16 and st["reruns"] > 0
    for q in srv.requests:
        for x, y in zip(_images(q), _alone(reg, q)):
            assert np.array_equal(x, y)
