"""Host logic of the served form (no GPU): the order in which requests are
considered for admission."""
from types import SimpleNamespace

from paper_2506_17357_amd import serve


def req(rid, arrival, n, steps=500):
    return serve.ServeRequest(rid, arrival, SimpleNamespace(n=n), None, steps)


def test_simultaneous_arrivals_largest_first():
    reqs = [req(0, 0.0, 200), req(1, 0.0, 9000), req(2, 0.0, 1000), req(3, 0.0, 9000, steps=100)]
    # (n + 1)^2 x step cap: 4.1e10 (rid 1), 8.1e9 (rid 3), 5.0e8 (rid 2), 2.0e7 (rid 0)
    assert [r.rid for r in serve.admission_order(reqs)] == [1, 3, 2, 0]


def test_arrival_time_comes_first():
    reqs = [req(0, 0.2, 9000), req(1, 0.1, 200), req(2, 0.1, 5000), req(3, 0.0, 100)]
    assert [r.rid for r in serve.admission_order(reqs)] == [3, 2, 1, 0]


def test_equal_size_keeps_request_order():
    reqs = [req(k, 0.0, 700) for k in (4, 2, 9, 0)]
    assert [r.rid for r in serve.admission_order(reqs)] == [0, 2, 4, 9]
