"""Host logic of the serving loop: batch admission and arrival generation."""
import collections

import numpy as np
import pytest

from paper_1805_00754_amd import serve


def req(i, n, kq, arrival=0.0):
    return serve.Request(i, 0, n, kq, arrival)


def test_output_bytes():
    # U n x kq, Sigma kq, V c x kq in FP64 plus the int32 rank
    assert serve.output_bytes(100, 4, 10) == 8 * (400 + 4 + 40) + 4
    # FP32-stored factors: U and V in FP32, Sigma still FP64
    assert serve.output_bytes(100, 4, 10, esize=4) == 4 * (400 + 40) + 8 * 4 + 4


def test_budget_counts_the_output_element_size():
    one32 = serve.output_bytes(100, 2, 4, esize=4)
    pol = serve.BatchPolicy(c=4, max_queries=100, budget_bytes=2 * one32, esize=4)
    pending = collections.deque([req(i, 100, 2) for i in range(3)])
    assert [r.idx for r in pol.take(pending)] == [0, 1]
    pol64 = serve.BatchPolicy(c=4, max_queries=100, budget_bytes=2 * one32, esize=8)
    pending = collections.deque([req(i, 100, 2) for i in range(3)])
    assert [r.idx for r in pol64.take(pending)] == [0]


def test_fifo_order_and_query_cap():
    pol = serve.BatchPolicy(c=8, max_queries=3, budget_bytes=1 << 30)
    pending = collections.deque(req(i, 10, 2) for i in range(7))
    sizes = []
    while pending:
        b = pol.take(pending)
        assert [r.idx for r in b] == sorted(r.idx for r in b)
        sizes.append(len(b))
    assert sizes == [3, 3, 1]


def test_byte_budget_stops_at_first_request_that_does_not_fit():
    c = 4
    one = serve.output_bytes(100, 2, c)
    pol = serve.BatchPolicy(c=c, max_queries=100, budget_bytes=3 * one + 10)
    pending = collections.deque([req(0, 100, 2), req(1, 100, 2), req(2, 100, 2), req(3, 100, 2)])
    assert [r.idx for r in pol.take(pending)] == [0, 1, 2]
    assert [r.idx for r in pol.take(pending)] == [3]
    # FIFO: a large request blocks smaller ones behind it rather than being skipped
    big = req(4, 250, 2)
    pending = collections.deque([req(5, 100, 2), big, req(6, 10, 2)])
    assert [r.idx for r in pol.take(pending)] == [5]
    assert pending[0].idx == 4


def test_fits_alone_rejects_oversized():
    pol = serve.BatchPolicy(c=4, max_queries=10, budget_bytes=serve.output_bytes(50, 3, 4))
    assert pol.fits_alone(req(0, 50, 3))
    assert not pol.fits_alone(req(1, 51, 3))


def test_invalid_policy():
    with pytest.raises(ValueError):
        serve.BatchPolicy(c=4, max_queries=0, budget_bytes=10)


def test_poisson_arrivals_rate():
    rng = np.random.Generator(np.random.PCG64(5))
    arr = serve.poisson_arrivals(rng, 2000.0, 20000)
    assert np.all(np.diff(arr) > 0)
    gaps = np.diff(np.concatenate(([0.0], arr)))
    assert abs(gaps.mean() - 1 / 2000.0) < 0.03 / 2000.0
    # exponential: coefficient of variation 1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05


def test_make_requests_ranges():
    rng = np.random.Generator(np.random.PCG64(6))
    rs = serve.make_requests(rng, 1_000_000, 500, 2000.0, 1e4, 3.2e5, [8, 16, 20])
    assert all(0 <= r.t_s < r.t_e <= 1_000_000 for r in rs)
    L = np.array([r.t_e - r.t_s for r in rs])
    assert L.min() >= 1e4 - 1 and L.max() <= 3.2e5 + 1
    assert set(r.k_q for r in rs) <= {8, 16, 20}
    assert [r.idx for r in rs] == list(range(500))


def test_budget_counts_the_scratch():
    c = 4
    one = serve.output_bytes(100, 2, c)
    scratch = lambda r: 1000 * (r.idx + 1)
    pol = serve.BatchPolicy(c=c, max_queries=100, budget_bytes=2 * one + 3000, scratch_fn=scratch)
    assert pol.bytes_of(req(0, 100, 2)) == one + 1000
    pending = collections.deque([req(0, 100, 2), req(1, 100, 2), req(2, 100, 2)])
    # 0 and 1 cost 2 one + 3000: they fit; 2 would add one + 3000 more
    assert [r.idx for r in pol.take(pending)] == [0, 1]
    assert not serve.BatchPolicy(c=c, max_queries=100, budget_bytes=one + 999,
                                 scratch_fn=scratch).fits_alone(req(0, 100, 2))


def test_fifo_replay():
    arrival = np.array([0.0, 0.1, 0.15, 1.0])
    service = np.array([0.2, 0.2, 0.2, 0.05])
    # 0: 0 -> 0.2; 1 waits: 0.2 -> 0.4; 2: 0.4 -> 0.6; 3 arrives after: 1.0 -> 1.05
    np.testing.assert_allclose(serve.fifo_replay(arrival, service), [0.2, 0.4, 0.6, 1.05])
