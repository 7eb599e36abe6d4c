"""The pins must catch plausible mistakes in the oracle.

Each case copies the oracle's C source, plants one mistake (a dropped term,
a wrong sign or index, a swapped operand), compiles the copy on the CPU and
runs the pin tests against it: at least one pin has to fail.  The committed
oracle itself is never modified.
"""
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "sfr_oracle.c")

# (name, exact text in the source, replacement)
MUTANTS = [
    ("soft_threshold_sign", "double b = x + t;", "double b = x - t;"),
    ("sym_dropped_in_spd_step", "orc_sym(C, r, B);", "memcpy(B, C, sizeof(double) * (size_t)(r * r));"),
    ("vstep_without_B0", "mm(XtU, Bc, T, n, r, r);", "memcpy(T, XtU, sizeof(double) * (size_t)(n * r));"),
    ("vstep_transposed_operand", "mtm(X, U, XtU, m, n, r);", "mtm(X, U, XtU, m, n, r); for (int64_t z = 0; z < r; ++z) { double tz = XtU[z * r + 0]; XtU[z * r + 0] = XtU[0 * r + z]; XtU[0 * r + z] = tz; }"),
    ("spd_step_reuses_U_product", "mm(X, V, XV, m, n, r);\n    mtm(U, XV, C, m, r, r);", "mm(X, V, XV, m, n, r);\n    mtm(U, XV, C, m, r, r); C[0] *= 1.001;"),
    ("dual_sign", "Y[i] = Y[i] + mk * E;", "Y[i] = Y[i] - mk * E;"),
    ("threshold_drops_lambda", "const double t = lambda / mk;", "const double t = 1.0 / mk;"),
    ("no_continuation", "double nm = rho * mk;", "double nm = mk;"),
    ("Lstep_input_sign", "X[i] = M[i] - S[i] + Y[i] / mk;", "X[i] = M[i] - S[i] - Y[i] / mk;"),
    ("jacobi_rotation_sign", "G[i * k + q] = s * gp + c * gq;", "G[i * k + q] = -s * gp + c * gq;"),
    ("jacobi_accumulator_index", "Z[i * k + q] = s * zp + c * zq;", "Z[i * k + q] = s * zq + c * zp;"),
    ("pinv_keeps_smallest", "while (j > 0 && sig[idx[j - 1]] < sig[v])", "while (j > 0 && sig[idx[j - 1]] > sig[v])"),
    ("nystrom_unshuffle_dropped", "int64_t dst = perm[i];", "int64_t dst = i;"),
    ("residual_uses_old_Y", "double E = M[i] - L[i] - S[i];", "double E = M[i] - L[i] - S[i] + 1e-3 * Y[i];"),
    ("Lstep_input_uses_next_mu", "X[i] = M[i] - S[i] + Y[i] / mk;", "X[i] = M[i] - S[i] + Y[i] / (rho * mk);"),
    ("V0_shifted", "V[i * r + j] = (i == j) ? 1.0 : 0.0;", "V[i * r + j] = (i == j + 1) ? 1.0 : 0.0;"),
    ("B0_not_identity", "B[i * r + j] = (i == j) ? 1.0 : 0.0;", "B[i * r + j] = (i == j) ? 1.0 + (double)i : 0.0;"),
    ("Sstep_uses_next_mu", "const double t = lambda / mk;", "const double t = lambda / (rho * mk);"),
]

PIN_TESTS = [
    pins.test_golden_closed_forms,
    pins.test_soft_threshold_is_prox_bruteforce,
    lambda: pins.test_polar_matches_lapack_svd_and_gram_form(7, 3, 0),
    pins.test_svd_jacobi_reconstructs,
    pins.test_fr_step_invariants_and_lemma1,
    pins.test_fr_step_identity_B0_gives_symmetric_product,
    pins.test_fradm_iteration_identities,
    pins.test_fradm_starts_from_identity_factors,
    pins.test_lambda_mu_equivalence,
    pins.test_nystrom_exact_on_rank_r_and_reading,
    pins.test_nystrom_blocks_matches_full,
    lambda: pins.test_planted_recovery_plain(0),
]


def _run_pins():
    failures = 0
    for t in PIN_TESTS:
        try:
            t()
        except Exception:
            failures += 1
    return failures


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mutated = src.replace(old, new)
    c = tmp_path / "mut.c"
    c.write_text(mutated)
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", str(so), str(c), "-lm"])
    saved = oracle._lib
    oracle._lib = oracle.load(str(so))
    try:
        failures = _run_pins()
    finally:
        oracle._lib = saved
    assert failures >= 1, f"no pin caught mutant {name}"


def test_unmutated_oracle_passes_all_listed_pins():
    assert _run_pins() == 0
