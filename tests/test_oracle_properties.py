"""Hypothesis-generated tiny phantoms (K <= 64, keys colliding on every axis)
under random mixes of every block kind: the brute-force grouped FP64 method
equals the plain FP64 oracle to rounding (the grouped update re-associates
the same product, Sec. 2.3, Eq. 7-10), and the plain result is invariant
under permutations of the isochromats."""
import numpy as np
from hypothesis import given, settings, strategies as st, HealthCheck

import random_cases as rc

SETTINGS = settings(max_examples=150, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow])


@SETTINGS
@given(seed=st.integers(0, 2**31 - 1), K=st.integers(1, 64),
       kinds=st.lists(st.sampled_from(rc.KINDS), min_size=1, max_size=6))
def test_grouped_equals_plain_on_random_cases(oracle_lib, seed, K, kinds):
    from oracle.grouped import simulate_grouped
    rng = np.random.default_rng(seed)
    ph, seq = rc.phantom(rng, K), rc.sequence(rng, kinds)
    Mp, sp = oracle_lib.simulate(ph, seq)
    Mg, sg = simulate_grouped(ph, seq)
    assert np.max(np.abs(Mp - Mg)) < 1e-11
    assert np.linalg.norm(sp - sg) <= 1e-11 * max(np.linalg.norm(sp), 1.0)


@SETTINGS
@given(seed=st.integers(0, 2**31 - 1), K=st.integers(2, 64),
       kinds=st.lists(st.sampled_from(rc.KINDS), min_size=1, max_size=6))
def test_permutation_invariance_on_random_cases(oracle_lib, seed, K, kinds):
    rng = np.random.default_rng(seed)
    ph, seq = rc.phantom(rng, K), rc.sequence(rng, kinds)
    perm = rng.permutation(K)
    M, s = oracle_lib.simulate(ph, seq)
    Mp, sp = oracle_lib.simulate(ph.subset(perm), seq)
    assert np.array_equal(Mp, M[:, perm])
    assert np.allclose(sp, s, rtol=0, atol=1e-12 * max(np.abs(s).max(initial=0.0), 1.0))
