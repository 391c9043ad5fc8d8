import numpy as np

from oracle import stats


def test_moments_hand_values():
    q = np.array([[1.0, 2.0, 3.0, 4.0], [2.0, 2.0, 2.0, 2.0], [0.0, 0.0, 0.0, 8.0]])
    mean, var = stats.moments(q)
    assert np.allclose(mean, [2.5, 2.0, 2.0])
    assert np.allclose(var, [5.0 / 3.0, 0.0, 16.0])
