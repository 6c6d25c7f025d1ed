"""Host logic of bench.py: the algorithmic byte model of the step kernels and
the stream-mix bound (no GPU)."""

import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


@pytest.mark.parametrize("elt", [4, 8])
def test_read_write_split_sums_to_the_byte_model(elt):
    n, M = 256, 16
    N, H = n ** 3, (n // 2 + 1) * n * n
    c, nterm = 2 * elt, 2 * (M + 1)
    # the step kernels' bytes, written out from their loads and stores
    expect = {
        "c2r0_kick": (nterm * H * c + N * 8 + 2 * N * elt, H * c),
        "mid_terms": (nterm * H * c, nterm * H * c),
        "mid_dv": (H * c, H * c),
        "contig_kick": (H * c + 2 * 16 * H, 2 * 16 * H + nterm * H * c),
    }
    for cls, rw in expect.items():
        assert bench.algorithmic_rw(cls, n, M, elt) == rw
        assert bench.algorithmic_bytes(cls, n, M, elt) == sum(rw)
    assert bench.algorithmic_bytes("r2c0", n, M, elt) == 0.0  # not a step kernel class


def test_stream_mix_bound_limits():
    s = {"read_GBps": 7000.0, "write_GBps": 5000.0}
    assert bench.mix_bound((1.0, 0.0), s) == pytest.approx(7000.0)
    assert bench.mix_bound((0.0, 1.0), s) == pytest.approx(5000.0)
    # equal reads and writes: the harmonic mean of the two rates
    assert bench.mix_bound((1.0, 1.0), s) == pytest.approx(2 / (1 / 7000 + 1 / 5000))
    # a mix is bounded by its two streams
    b = bench.mix_bound((3.0, 1.0), s)
    assert 5000.0 < b < 7000.0


def test_kernel_source_hash_covers_the_step_kernels():
    assert set(bench.KERNEL_SOURCES) >= {"kernels.hpp", "fft_engine.hpp", "launch_impl.hpp"}
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash()
