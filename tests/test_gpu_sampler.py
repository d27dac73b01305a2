"""Device delivery-state sampler against the oracle: bit-exact codes for
random and edge-case channels, several packet / layer counts."""

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


def _random_channels(W, seed, P, L):
    rng = np.random.default_rng(seed)
    c = np.zeros(W, dtype=oracle.CHANNEL_DTYPE)
    c["p_gb"] = rng.uniform(0, 0.3, W)
    c["p_bg"] = rng.uniform(0, 1, W)
    c["loss_good"] = rng.uniform(0, 0.2, W)
    c["loss_bad"] = rng.uniform(0.3, 1, W)
    c["p_start_bad"] = rng.uniform(0, 1, W)
    c["deadline"] = rng.integers(-1, L * P + 2, W)
    # edge values: probabilities 0 and 1, deadlines 0 and n
    c["loss_good"][:4] = [0.0, 1.0, 0.0, 0.5]
    c["p_gb"][4:8] = [0.0, 1.0, 1.0, 0.0]
    c["p_bg"][4:8] = [0.0, 0.0, 1.0, 1.0]
    c["deadline"][8:11] = [0, L * P, -5]
    return c


@pytest.mark.parametrize("W,P,L", [(257, 1024, 4), (64, 3, 1), (5, 16384, 4), (33, 7, 3), (1, 1, 1)])
def test_sampler_matches_oracle(W, P, L):
    import paper_2606_17212_amd as dgs
    dev = torch.device("cuda:0")
    ch = _random_channels(max(W, 12), 100 + P, P, L)[:W]
    for seed in (0, 2606, 0xFFFFFFFFFFFFFFFF):
        got = dgs.sample_states(dgs.channels_to_device(ch, dev), P, L, seed).cpu().numpy()
        want = oracle.sample_states(ch, P, L, seed)
        assert np.array_equal(got, want), (W, P, L, seed, np.argwhere(got != want)[:5])


def test_sampler_edge_calls():
    import paper_2606_17212_amd as dgs
    dev = torch.device("cuda:0")
    empty = dgs.sample_states(dgs.channels_to_device(np.zeros(0, dtype=oracle.CHANNEL_DTYPE), dev), 8, 2, 1)
    assert empty.shape == (0, 8)
    ch = dgs.channels_to_device(np.zeros(2, dtype=oracle.CHANNEL_DTYPE), dev)
    with pytest.raises(dgs.DgsError):
        dgs.sample_states(ch, 8, 5, 1)
    with pytest.raises(dgs.DgsError):
        dgs.sample_states(ch, 0, 2, 1)
