"""Input generators: the device version of the smoothed random stress follows
the host recipe exactly when given the same random numbers."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W


def test_device_stress_recipe_matches_host_recipe():
    gen = torch.Generator()
    gen.manual_seed(5)
    draws = torch.randn((6, 6, 8, 10), generator=gen, dtype=torch.float64).numpy()
    dev = W.stress_field_device(10, 8, 6, 5, "cpu").numpy()
    # the host recipe (face-mean Jacobi, periodic x/y, linear z ghosts) on the same draws
    s = draws.copy()
    for _ in range(3):
        lo, hi = 2 * s[:, 0] - s[:, 1], 2 * s[:, -1] - s[:, -2]
        zp = np.concatenate([s[:, 1:], hi[:, None]], axis=1)
        zm = np.concatenate([lo[:, None], s[:, :-1]], axis=1)
        s = (np.roll(s, 1, -1) + np.roll(s, -1, -1) + np.roll(s, 1, -2) + np.roll(s, -1, -2)
             + zp + zm) / 6.0
    assert np.abs(dev - s).max() == 0.0
    # and the host generator is that recipe on numpy's draws
    host = W.stress_field(10, 8, 6, 5)
    assert host.shape == dev.shape and np.isfinite(host).all()
    assert abs(host.std() - dev.std()) < 0.2
