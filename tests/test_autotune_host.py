"""Autotuner search and memory-probe logic on the host (injected timer and
allocator; no GPU)."""

import pytest

from paper_2606_17212_amd.autotune import probe_state_batch, search


def test_search_picks_fastest_and_skips_failures():
    cost = {((16, 16), 2): 5.0, ((16, 16), 4): 3.0, ((16, 16), 8): 2.5, ((16, 16), 16): 2.7,
            ((32, 8), 2): 6.0, ((32, 8), 4): 3.5, ((32, 8), 8): 2.4, ((32, 8), 16): 9.0}

    def timer(tile, S, persistent, B):
        if S == 32:
            raise MemoryError("too big")
        return cost[(tile, S)] - (0.25 if persistent and S == 16 else 0.0) + (0.01 if B != 256 else 0.0)

    r = search(timer, num_states=64)
    assert (r.tile, r.states_per_group, r.persistent, r.lds_batch, r.ms) == ((32, 8), 8, False, 256, 2.4)
    assert r.table["16x16/S32/grid/B256"].startswith("failed")
    assert r.table["16x16/S16/persistent/B256"] == pytest.approx(2.45)
    r = search(timer, num_states=64, tiles=((16, 16),))
    assert (r.states_per_group, r.persistent) == (16, True)


def test_search_covers_lds_batches_for_groups_of_four_or_more():
    seen = set()

    def timer(tile, S, persistent, B):
        seen.add((S, B))
        return 1.0 + S / 100 - (0.5 if (S, B) == (8, 512) else 0.0)

    r = search(timer, num_states=64, tiles=((16, 16),), launches=(False,))
    assert (r.states_per_group, r.lds_batch) == (8, 512)
    # groups of 2 have only the default batch; groups of 4+ are timed with each
    assert {B for S, B in seen if S == 2} == {256}
    assert {B for S, B in seen if S == 8} == {128, 256, 512}
    assert r.as_dict()["lds_batch"] == 512


def test_search_skips_groups_larger_than_the_batch():
    seen = []

    def timer(tile, S, persistent, B):
        seen.append(S)
        return float(S)

    r = search(timer, num_states=3)
    assert max(seen) <= 4 and r.states_per_group == 2


@pytest.mark.parametrize("limit,upper", [(37, 512), (512, 512), (1, 64), (300, 1000)])
def test_probe_finds_largest_batch_under_budget(limit, upper):
    calls = []

    def try_alloc(b):
        calls.append(b)
        if b > limit:
            raise MemoryError
    assert probe_state_batch(try_alloc, upper) == min(limit, upper)
    assert len(calls) <= 2 * upper.bit_length() + 2


def test_probe_zero_when_nothing_fits_and_reraises_other_errors():
    def never(b):
        raise MemoryError
    assert probe_state_batch(never, 64) == 0

    def broken(b):
        raise ValueError("not an allocation failure")
    with pytest.raises(ValueError):
        probe_state_batch(broken, 64)
