"""The choice rule of the server tuner and its argument checks (host only)."""
import pytest

from paper_1803_11301_amd import serve_tune as st


def row(slots, sat, p99):
    return {"slots": slots, "batch_limit_bits": 1 << 20, "max_batch": 512, "saturated_per_s": sat, "p99_ms": p99}


def test_fastest_without_a_limit():
    t = [row(4, 100.0, 1.0), row(8, 300.0, 9.0), row(12, 200.0, 2.0)]
    assert st.choose(t)["slots"] == 8


def test_fastest_within_the_limit():
    t = [row(4, 100.0, 1.0), row(8, 300.0, 9.0), row(12, 200.0, 2.0)]
    assert st.choose(t, p99_limit_ms=2.5)["slots"] == 12
    assert st.choose(t, p99_limit_ms=1.0)["slots"] == 4     # the limit itself is met


def test_lowest_p99_when_none_meets_the_limit():
    t = [row(4, 100.0, 3.0), row(8, 300.0, 9.0), row(12, 200.0, 2.5)]
    assert st.choose(t, p99_limit_ms=1.0)["slots"] == 12


def test_no_rows_is_an_error():
    with pytest.raises(ValueError):
        st.choose([])


def test_default_candidates_are_valid_settings():
    # slots 1..64, batch limit <= 2^22 bits, batches of 1..4096 (polymul_server_set_policy)
    for slots, limit, max_batch in st.DEFAULT_CANDIDATES:
        assert 1 <= slots <= 64 and 0 <= limit <= 1 << 22 and 1 <= max_batch <= 4096
    assert (8, 1 << 20, 512) in st.DEFAULT_CANDIDATES   # the server's defaults are among them


@pytest.mark.parametrize("la,lb,rho", [([], [], 0.8), ([10, 20], [10], 0.8), ([0], [5], 0.8), ([5], [5], 1.0)])
def test_bad_arguments_are_refused_before_any_device_work(la, lb, rho):
    with pytest.raises(ValueError):
        st.tune_server(None, la, lb, rho=rho)
