"""The CPU oracle against closed forms, invariants and brute force."""
import pytest

import oracle
import pins
import pins_les


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


@pytest.mark.parametrize("pin", pins.PINS + pins_les.PINS, ids=lambda p: p.__name__)
def test_pin(pin, lib):
    pin(lib)


def test_point_evaluation_equals_sweep(lib):
    """ora_point (used for sampled checks of large grids) equals the sweeps."""
    import numpy as np
    g, _ = pins.make_grid(9, 7, 6, 0)
    u, v, w = pins.random_state(g, 31, lib=lib)
    adv, du, dv, dw = pins.tendencies(g, u, v, w, 0.2, lib=lib)
    rng = np.random.default_rng(0)
    for _ in range(40):
        i, j, k = int(rng.integers(1, 10)), int(rng.integers(1, 8)), int(rng.integers(1, 7))
        p = oracle.point(g, 0.2, u, v, w, i, j, k, lib=lib)
        ref = [adv[k - 1, j - 1, i - 1], du[k - 1, j - 1, i - 1], dv[k - 1, j - 1, i - 1],
               dw[k - 1, j - 1, i - 1]]
        assert np.array_equal(p, np.array(ref))
