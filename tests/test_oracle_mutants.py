"""The pins have teeth: plausible mistakes planted in a copy of the oracle's C
source (on the CPU only) must each make at least one pin fail."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from test_oracle_pins import (test_brute_force_unfold_times_khatri_rao,
                              test_closed_form_full_exact_rank_R,
                              test_gradient_central_differences,
                              test_worked_example_golden)

SRC = os.path.join(os.path.dirname(oracle.__file__), "mttkrp_ref.c")

MUTANTS = {
    # a dropped term: the last input factor is skipped
    "dropped_factor": ("if (w == mode) continue;",
                       "if (w == mode || (w == order - 1 && mode != order - 1)) continue;"),
    # a transposed operand: rank columns read in reverse order
    "reversed_rank": ("prod *= A[w][iw * R + r];\n            }\n            out[",
                      "prod *= A[w][iw * R + (R - 1 - r)];\n            }\n            out["),
    # overwrite instead of accumulate
    "no_accumulate": ("out[i * R + r] += prod;", "out[i * R + r] = prod;"),
    # wrong nonzero's output index
    "wrong_row_index": ("const int64_t i = idx[(int64_t)mode * nnz + k];",
                        "const int64_t i = idx[(int64_t)mode * nnz + (nnz - 1 - k)];"),
    # wrong sign of the residual
    "residual_sign": ("const double e = val[k] - resid[k];", "const double e = resid[k] - val[k];"),
    # model value missing the last rank component
    "model_drops_rank": ("for (int r = 0; r < R; ++r) {\n            double prod = 1.0;",
                         "for (int r = 0; r < R - 1; ++r) {\n            double prod = 1.0;"),
}

PINS = [
    lambda: test_worked_example_golden(),
    lambda: test_brute_force_unfold_times_khatri_rao((5, 4, 3), 23, "cyclic"),
    lambda: test_brute_force_unfold_times_khatri_rao((4, 3, 3, 2), 31, "first_fastest"),
    lambda: test_closed_form_full_exact_rank_R((9, 7, 5), 4),
    lambda: test_gradient_central_differences(),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, "mutation site not found: %s" % name
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    lib_path = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", str(lib_path),
                    str(mpath)], check=True)
    lib = oracle._configure(ctypes.CDLL(str(lib_path)))
    monkeypatch.setattr(oracle, "_lib", lib)
    failures = 0
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failures += 1
    assert failures >= 1, "mutant %s passed every pin" % name
