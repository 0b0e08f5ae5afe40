"""Seeded random tiny phantoms (K <= 64, keys colliding on every axis) under
random mixes of every block kind, through all three GPU modes against the
FP64 oracle (|dM| <= 1e-5, relative signal error <= 1e-4).  The same
generators drive the oracle's own property tests."""
import numpy as np
import pytest

import random_cases as rc
from tests.test_gpu_parity import check_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_03960_amd as gb
    return gb


@pytest.mark.parametrize("seed", range(100))
def test_random_case(gb, seed):
    rng = np.random.default_rng(1000 + seed)
    K = int(rng.integers(1, 65))
    kinds = list(rng.choice(rc.KINDS, size=int(rng.integers(1, 7))))
    ph, seq = rc.phantom(rng, K), rc.sequence(rng, kinds)
    # odd seeds start from a random state, so that readouts before any RF see signal
    m_init = rng.uniform(-0.6, 0.6, (3, K)) if seed % 2 else None
    check_case(gb, f"random{seed}:{'+'.join(kinds)}", ph, seq, modes=("plain", "grouped", "cached"),
               axes=31 if seed % 2 == 0 else 7, m_init=m_init)


@pytest.mark.parametrize("seed", range(10))
def test_random_case_large_groups(gb, seed):
    """K from 500 to 5000 on the same few key values: groups of hundreds of
    members that span several tiles, with ragged padding."""
    rng = np.random.default_rng(5000 + seed)
    K = int(rng.integers(500, 5001))
    kinds = list(rng.choice(rc.KINDS, size=int(rng.integers(2, 7))))
    ph, seq = rc.phantom(rng, K), rc.sequence(rng, kinds)
    m_init = rng.uniform(-0.6, 0.6, (3, K)) if seed % 2 else None
    check_case(gb, f"random-large{seed}:{'+'.join(kinds)}", ph, seq, modes=("plain", "grouped", "cached"),
               axes=31, m_init=m_init)


@pytest.mark.parametrize("seed", range(20))
def test_random_case_coils(gb, seed):
    """Random cases with 2 to 4 receive coils of random complex sensitivity,
    from a random initial state: grouped, cached and plain against the
    oracle's coil sums."""
    from tests.test_gpu_coils import check as check_coils
    rng = np.random.default_rng(9000 + seed)
    while True:
        K = int(rng.integers(1, 65))
        kinds = list(rng.choice(rc.KINDS, size=int(rng.integers(1, 7))))
        ph, seq = rc.phantom(rng, K), rc.sequence(rng, kinds)
        if seq.total_samples > 0:
            break
    P = int(rng.integers(2, 5))
    sens = (rng.uniform(0.2, 1.0, (P, K)) * np.exp(1j * rng.uniform(0, 2 * np.pi, (P, K)))).astype(np.complex64)
    m_init = rng.uniform(-0.6, 0.6, (3, K))
    check_coils(gb, f"random{seed}:{'+'.join(kinds)}", ph, seq, sens, m_init=m_init, plain=True)


@pytest.mark.parametrize("seed", range(12))
def test_random_repeated_emissions(gb, seed):
    """relax -> RF -> relax -> ADC -> ADC: the pending map before the RF has a
    y moment, and the two readouts share theirs, so the second emission's y
    phase steps by a zero step after the pre map's y phase was evaluated."""
    rng = np.random.default_rng(7000 + seed)
    K = int(rng.integers(1, 65))
    rf = str(rng.choice(["rf_x", "rf_z", "rf_none"]))
    adc = str(rng.choice(["adc_x", "adc_z"]))
    kinds = ["relax", rf, "relax", adc, adc] * int(rng.integers(1, 3))
    ph, seq = rc.phantom(rng, K), rc.sequence(rng, kinds)
    check_case(gb, f"repeat{seed}:{'+'.join(kinds)}", ph, seq, modes=("grouped",), axes=31 if seed % 2 else 7)
