"""The measured-ceiling micro-benchmarks run and lose no update: random FP64
atomics into an array the size of the duct's tally, LDS ds_add_f64 into an
array the size of the hot tile, and the streaming copy."""
import pytest

pytestmark = pytest.mark.gpu


def test_micro_benchmarks_count_every_update():
    from paper_2409_04668_amd import mcdc
    # each helper asserts that the array's total equals the updates made
    assert mcdc.micro_atomic_rate(7_200_000, 10_000_000, run=1, reps=1) > 1e9
    assert mcdc.micro_lds_atomic_rate(18816, 100_000_000, reps=1) > 1e10
    assert mcdc.micro_lds_atomic_rate(7, 1_000_000, reps=1) > 0
    assert mcdc.micro_copy_rate(1 << 26, reps=1) > 1e11
