"""The pins catch plausible mistakes in the oracle: each case plants one
(a flipped sign, a dropped term, a wrong index, a transposed operand) in a
copy of the oracle's C source, builds it on the CPU, and runs a fast subset
of tests/test_oracle_pins.py against it in a child process, which must fail.
The unmodified oracle passes the same subset in the ordinary run of that
file."""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
SRC = os.path.join(REPO, "oracle", "bfsft_oracle.c")
PINS = os.path.join(HERE, "test_oracle_pins.py")
SUBSET = ("direct_matches_mpmath or dft or geometric or brute_force_tiny or operators_equal_literal"
          " or matching_condition or single_source")

MUTANTS = [
    # O1, eq. (1)
    ("O1 exponent sign", "acc += expi_dd_d(dd_div(t, N)) * fc[j];",
     "acc += conj(expi_dd_d(dd_div(t, N))) * fc[j];"),
    ("O1 first source dropped", "for (int64_t j = 0; j < nk; ++j) {\n            const double *kj = k + j * d;",
     "for (int64_t j = 1; j < nk; ++j) {\n            const double *kj = k + j * d;"),
    ("O1 axis index", "t = dd_add(t, two_prod(xi[a], kj[a]));", "t = dd_add(t, two_prod(xi[a], kj[0]));"),
    # O2, Section 2.1 operators
    ("eq. (M1) box index", "m12[l] = expi_rational((uint64_t)iA * (uint64_t)l, (uint64_t)P->q, P->N, P->L);",
     "m12[l] = expi_rational((uint64_t)(iA + 1) * (uint64_t)l, (uint64_t)P->q, P->N, P->L);"),
    ("eq. (E1) child width",
     "e11[l] = expi_rational((uint64_t)(P->q * iA + l) * (uint64_t)ic, (uint64_t)(2 * P->q), P->N, P->L);",
     "e11[l] = expi_rational((uint64_t)(P->q * iA + l) * (uint64_t)ic, (uint64_t)P->q, P->N, P->L);"),
    ("eq. (E1) H taken as G", "P->H[l * p + m] = expi_rational((uint64_t)(l * m), (uint64_t)(2 * q * q), N, P->L);",
     "P->H[l * p + m] = expi_rational((uint64_t)(l * m), (uint64_t)(q * q), N, P->L);"),
    # the solve of M f = u and the per-axis application
    ("back substitution transposed", "for (int j = i + 1; j < p; ++j) b[i * s] -= LU[i * p + j] * b[j * s];",
     "for (int j = i + 1; j < p; ++j) b[i * s] -= LU[j * p + i] * b[j * s];"),
    ("axis operator transposed", "acc += A[l * p + m] * fib[m];", "acc += A[m * p + l] * fib[m];"),
    # steps 2 and 4 of Section 2.2
    ("step 2 axis index", "ph[s][l] = expi_dd(dd_div(two_prod((double)(q * iA[s] + l), kj[s]), qs));",
     "ph[s][l] = expi_dd(dd_div(two_prod((double)(q * iA[s] + l), kj[0]), qs));"),
    ("step 4 axis order", "for (int s = d - 1; s >= 0; --s) { w *= ph[s][r % p]; r /= p; }\n                acc += w;",
     "for (int s = 0; s < d; ++s) { w *= ph[s][r % p]; r /= p; }\n                acc += w;"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of '{name}' not unique"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    so = oracle.build(True, src=str(mutated), out=str(tmp_path / "mutant.so"))
    env = dict(os.environ, BFSFT_ORACLE_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", PINS, "-x", "-q", "-p", "no:cacheprovider",
                        "-k", SUBSET], cwd=REPO, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"'{name}' was not caught:\n{r.stdout[-2000:]}"
