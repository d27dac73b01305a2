"""Pins of the delivery-state sampler oracle (Sec. 4's training worlds:
Gilbert-Elliott / IID erasures, playout deadline, dependency closure):
Philox known answers, closed-form special cases, statistical invariants of
the Markov channel, and the counter-based stream's properties."""

import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def channels(W, p_gb=0.0, p_bg=0.0, loss_good=0.0, loss_bad=0.0, p_start_bad=0.0, deadline=-1):
    c = np.zeros(W, dtype=oracle.CHANNEL_DTYPE)
    c["p_gb"], c["p_bg"], c["loss_good"], c["loss_bad"] = p_gb, p_bg, loss_good, loss_bad
    c["p_start_bad"], c["deadline"] = p_start_bad, deadline
    return c


def test_philox_known_answers():
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")) as f:
        kat = json.load(f)
    for v in kat["vectors"]:
        out = oracle.philox4x32_10([int(x, 16) for x in v["counter"]], [int(x, 16) for x in v["key"]])
        assert [int(x) for x in out] == [int(x, 16) for x in v["output"]]


def test_closed_form_special_cases():
    P, L = 37, 4
    assert np.all(oracle.sample_states(channels(5), P, L, 1) == L)                      # lossless
    assert np.all(oracle.sample_states(channels(5, loss_good=1.0), P, L, 1) == 0)       # all erased
    assert np.all(oracle.sample_states(channels(5, deadline=0), P, L, 1) == 0)          # nothing in time
    # layer-major order: a deadline of k P + r slots gives packets p < r k + 1 layers, the rest k
    for k, r in ((0, 5), (1, 0), (2, 11), (3, 36)):
        codes = oracle.sample_states(channels(3, deadline=k * P + r), P, L, 9)
        want = np.where(np.arange(P) < r, k + 1, k)
        assert np.all(codes == want[None, :])
    # a bad channel that never leaves the bad state loses everything it is asked to
    assert np.all(oracle.sample_states(channels(4, p_start_bad=1.0, loss_bad=1.0), P, L, 3) == 0)
    # single layer: codes are 0/1
    c1 = oracle.sample_states(channels(50, loss_good=0.3), P, 1, 4)
    assert set(np.unique(c1)) <= {0, 1}


def test_iid_prefix_closure_distribution():
    """IID erasure e: P(code >= c) = (1 - e)^c (the code counts leading arrived layers)."""
    W, P, L, e = 400, 256, 4, 0.2
    codes = oracle.sample_states(channels(W, loss_good=e), P, L, 12345).astype(np.int64).ravel()
    n = codes.size
    for c in range(1, L + 1):
        p = (1 - e) ** c
        got = np.mean(codes >= c)
        assert abs(got - p) <= 5 * np.sqrt(p * (1 - p) / n), (c, got, p)


def test_gilbert_elliott_sojourns_and_stationary_loss():
    """Single layer: the code sequence over packets is the arrival sequence.
    With loss 1 in bad and 0 in good, losses are exactly the bad sojourns:
    mean run lengths 1/p_bg (losses) and 1/p_gb (arrivals); started in the
    stationary law, the loss rate is p_gb / (p_gb + p_bg)."""
    p_gb, p_bg = 0.05, 0.25
    W, P = 200, 2000
    ch = channels(W, p_gb=p_gb, p_bg=p_bg, loss_good=0.0, loss_bad=1.0, p_start_bad=p_gb / (p_gb + p_bg))
    codes = oracle.sample_states(ch, P, 1, 777)
    lost = 1 - codes.astype(np.int64)
    rate = lost.mean()
    pi_b = p_gb / (p_gb + p_bg)
    assert abs(rate - pi_b) < 0.01, rate
    runs = {0: [], 1: []}
    for row in lost:
        edges = np.flatnonzero(np.diff(row)) + 1
        segs = np.split(row, edges)
        for sgm in segs[1:-1]:  # complete runs only
            runs[int(sgm[0])].append(len(sgm))
    assert abs(np.mean(runs[1]) - 1 / p_bg) < 0.1 * (1 / p_bg)
    assert abs(np.mean(runs[0]) - 1 / p_gb) < 0.1 * (1 / p_gb)


def test_counter_based_stream_properties():
    P, L = 64, 4
    ch = channels(20, p_gb=0.1, p_bg=0.3, loss_good=0.05, loss_bad=0.7, p_start_bad=0.25, deadline=200)
    a = oracle.sample_states(ch, P, L, 2606)
    b = oracle.sample_states(ch, P, L, 2606)
    assert np.array_equal(a, b)                                        # deterministic
    assert np.array_equal(oracle.sample_states(ch[:7], P, L, 2606), a[:7])  # world w independent of W
    assert not np.array_equal(oracle.sample_states(ch, P, L, 2607), a)     # seed matters
    assert a.max() <= L and a.min() >= 0
