"""Serving admission and batch formation on the host (no GPU): requests over
the budget are rejected, the in-flight bytes never exceed the budget, batches
respect the view and pixel limits, order is FIFO, and without batching every
launch holds one request."""
import numpy as np

from paper_2406_01579_amd.serve import Request, Scheduler


def _req(i, nv=1, size=256, fp=100):
    cams = np.zeros((nv, 22), np.float32)
    cams[:, 0] = cams[:, 1] = size
    return Request(i, 0, cams, float(i), footprint=fp)


def test_over_budget_request_is_rejected():
    s = Scheduler(budget_bytes=1000)
    r = _req(0, fp=1001)
    assert not s.submit(r) and r.error and r.done() and s.rejected == 1 and not s.queue


def test_budget_bounds_in_flight_and_queues_the_rest():
    s = Scheduler(budget_bytes=1000)
    for i in range(10):
        assert s.submit(_req(i, fp=300))
    b1 = s.next_batch()
    assert [r.id for r in b1] == [0, 1, 2] and s.in_flight == 900
    assert s.next_batch() == []              # back-pressure: nothing fits now
    s.release(b1)
    b2 = s.next_batch()
    assert [r.id for r in b2] == [3, 4, 5]
    assert s.max_in_flight <= 1000


def test_view_and_pixel_limits_and_fifo():
    s = Scheduler(budget_bytes=10 ** 12, max_views=5, max_pixels=3 * 512 * 512)
    for i, nv in enumerate([2, 2, 2, 1]):
        s.submit(_req(i, nv=nv, size=256))
    assert [r.id for r in s.next_batch()] == [0, 1]     # 2+2 views; 6 would exceed 5
    assert [r.id for r in s.next_batch()] == [2, 3]
    s2 = Scheduler(budget_bytes=10 ** 12, max_views=64, max_pixels=3 * 512 * 512)
    for i in range(4):
        s2.submit(_req(i, nv=1, size=512))
    assert len(s2.next_batch()) == 3                      # pixel limit
    # a batch always takes at least its head, even one over the pixel limit
    s3 = Scheduler(budget_bytes=10 ** 12, max_views=1, max_pixels=1)
    s3.submit(_req(0, nv=4, size=1024))
    assert len(s3.next_batch()) == 1


def test_without_batching_one_request_per_launch():
    s = Scheduler(budget_bytes=10 ** 12, batching=False)
    for i in range(3):
        s.submit(_req(i, nv=2))
    assert [len(s.next_batch()) for _ in range(3)] == [1, 1, 1]


def test_rerun_growth_is_charged_until_release():
    """A launch re-run with larger capacities charges the extra workspace to
    the in-flight bytes (admission sees it) and gives it back with its batch."""
    s = Scheduler(budget_bytes=1000)
    for i in range(4):
        s.submit(_req(i, fp=300))
    b1 = s.next_batch()
    assert s.in_flight == 900
    s.charge(200)                              # the re-run's larger workspace
    assert s.in_flight == 1100 and s.max_in_flight == 1100
    assert s.next_batch() == []
    s.release(b1, 200)
    assert s.in_flight == 0
    assert [r.id for r in s.next_batch()] == [3]
