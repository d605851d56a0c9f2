"""Host-side pieces of the serving loop (no GPU): flight bookkeeping and latency percentiles."""
import torch

from paper_1503_00576_amd import serve


def test_flights_compare_by_identity():
    # flights hold tensors of different sizes; removing one from the in-flight list must not
    # compare tensors element-wise
    a = serve._Flight([], [], None, None, 0, None, [torch.zeros(3)], "single")
    b = serve._Flight([], [], None, None, 0, None, [torch.zeros(5)], "batch")
    inflight = [a, b]
    inflight.remove(b)
    assert inflight == [a] and inflight[0] is a
    assert a != serve._Flight([], [], None, None, 0, None, [torch.zeros(3)], "single")


def test_percentile():
    xs = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert serve.percentile(xs, 0) == 1.0
    assert serve.percentile(xs, 50) == 3.0
    assert serve.percentile(xs, 100) == 5.0
    assert serve.percentile([], 50) != serve.percentile([], 50)  # nan
