"""The test-side state conversion (oracle messages <-> signed log2 words)."""
import numpy as np

from tests._msg import from_state, to_state


def test_state_round_trip_and_signed_zero():
    rng = np.random.default_rng(0)
    p = rng.random((3, 5, 8))
    p /= p.sum(-1, keepdims=True)
    w = to_state(p)
    assert not np.any(np.signbit(w[..., 0]))          # P(0) = 1 must not decode as -1
    P = p @ np.array([[(-1) ** bin(z & x).count("1") for x in range(8)] for z in range(8)]).T
    assert np.allclose(from_state(w), P, atol=1e-6)
    delta = np.zeros((1, 1, 4))
    delta[..., 0] = 1.0
    assert np.array_equal(from_state(to_state(delta)), np.ones((1, 1, 4)))
