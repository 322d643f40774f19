"""Host-side pieces of the serving driver."""
from paper_2006_09808_amd.serve import percentile


def test_percentile_interpolates():
    xs = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert percentile(xs, 0) == 1.0
    assert percentile(xs, 50) == 3.0
    assert percentile(xs, 100) == 5.0
    assert abs(percentile(xs, 99) - 4.96) < 1e-12
    assert percentile([7.0], 99) == 7.0
