"""Plant plausible mistakes in copies of the oracle and show the pins catch them.

CPU only.  Each mutant is the oracle source with one textual change (a sign,
a transposed entry, the splitting order, a dropped term, an axis mix-up),
compiled into a temporary directory; at least one pin of oracle_pins.py must
fail against it.  The real oracle is never modified.
"""
import os
import subprocess

import pytest

import oracle
from tests import oracle_pins as pins

MUTANTS = {
    "theta_sign": ("double theta = -OR_TWO_PI", "double theta = OR_TWO_PI"),
    "R_entry_transposed": ("R[0][1] = -uz * s + ux * uy * v;", "R[0][1] = uz * s + ux * uy * v;"),
    "splitting_order_RD": ("matmul4(D, R, U);", "matmul4(R, D, U);"),
    "dropped_M0_recovery": ("D[2][3] = 1.0 - e1;", "D[2][3] = 0.0;"),
    "T1_for_transverse": ("double e1 = exp(-dt / t1), e2 = exp(-dt / t2);",
                          "double e1 = exp(-dt / t1), e2 = exp(-dt / t1);"),
    "missing_offresonance": ("gz[s] * z[k] + bz_off;", "gz[s] * z[k];"),
    "relax_phase_conjugated": ("M[0] = e2 * (mx * c + my * s);", "M[0] = e2 * (mx * c - my * s);"),
    "relax_moment_axis": ("mom[1] * y + mom[2] * z", "mom[1] * x + mom[2] * z"),
    "signal_imag_sign": ("acc[2 * (so + next) + 1] += M[1];", "acc[2 * (so + next) + 1] -= M[1];"),
    "relax_t1_t2_swapped": ("double e2 = exp(-tau / t2), e1 = exp(-tau / t1);",
                            "double e2 = exp(-tau / t1), e1 = exp(-tau / t2);"),
}


@pytest.fixture(scope="module")
def source():
    with open(oracle.SRC_PATH) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) == 1, f"mutation anchor for {name} not unique"
    src = tmp_path / f"{name}.c"
    src.write_text(source.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", str(src), "-o", str(so), "-lm"],
                   check=True)
    lib = oracle.bind(str(so))
    sim = lambda ph, seq, **kw: oracle.simulate(ph, seq, lib=lib, **kw)
    failed = []
    for check in pins.CHECKS:
        try:
            check(sim)
        except AssertionError:
            failed.append(check.__name__)
    assert failed, f"no pin detects mutant {name}"
    os.remove(so)
