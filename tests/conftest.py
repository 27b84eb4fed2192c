import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def c1():
    import synth
    return synth.WORKLOADS[1]


@pytest.fixture(scope="session")
def c1_lib():
    import synth
    return synth.make_library(1)


@pytest.fixture(scope="session")
def c1_olib(c1, c1_lib):
    import oracle
    import synth
    return oracle.OracleLibrary.build(c1_lib, synth.px_per_inv_A(c1), c1.R, c1.n_theta)


def small_library(n_templates=12, seed=0, max_spots=8, g_max=1.0, with_duplicates=True,
                  g_min=0.15):
    """Random CSR library of tiny templates (spots in 1/Angstrom)."""
    rng = np.random.default_rng(seed)
    kx, ky, I, off = [], [], [], [0]
    for t in range(n_templates):
        n = int(rng.integers(1, max_spots + 1))
        r = rng.uniform(g_min, g_max, n)
        a = rng.uniform(0, 2 * np.pi, n)
        x, y = r * np.cos(a), r * np.sin(a)
        w = rng.uniform(0.1, 1.0, n)
        if with_duplicates and n > 1 and t % 3 == 0:
            # a second spot landing on the same polar pixel as the first
            x[1], y[1] = x[0] * (1 + 1e-6), y[0] * (1 + 1e-6)
        kx += list(x)
        ky += list(y)
        I += list(w)
        off.append(off[-1] + n)
    return dict(kx=np.array(kx), ky=np.array(ky), intensity=np.array(I),
                offsets=np.array(off, dtype=np.int64))
