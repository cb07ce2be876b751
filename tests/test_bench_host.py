"""Host logic of bench.py (no GPU): the digest that ties a committed
rocprofv3 counter summary to the step kernel, and the summaries on file."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1411_3133_amd", "csrc")


def _read(fn):
    with open(os.path.join(CSRC, fn)) as f:
        return f.read()


def test_digest_ignores_comments_and_sees_code():
    base = bench.kernel_source_digest(_read)
    commented = bench.kernel_source_digest(
        lambda fn: "// a remark\n" + _read(fn).replace("{\n", "{  /* note */\n\n", 1))
    assert commented == base
    edited = bench.kernel_source_digest(lambda fn: _read(fn) + ("\nint extra;\n" if fn == "step.hip" else ""))
    assert edited != base


@pytest.mark.parametrize("tag", ["uneven_ellipsoid_batch_f32", "cylinder_sweep_64x4x256_f32",
                                 "cylinder_sweep_64x4x256_f64", "cylinder_sweep_64x4x256_f16",
                                 "ellipsoid_96x192x192_f32", "ellipsoid_96x384x192_f16"])
def test_committed_counter_summaries_match_the_kernel(tag):
    """A code change to the step kernel voids the committed summaries; they
    are taken again before such a change is committed."""
    traffic = bench.measured_traffic(tag, bench.kernel_source_digest())
    assert traffic is not None and traffic > 0
