"""The oracle's pins must catch plausible mistakes.

Each case copies oracle.c, plants one mistake (a dropped term, a wrong sign,
a wrong index, a transposed operand, a missing sort, a wrong mask), builds
the copy with gcc and runs the pin tests against it in a child process
(the ORACLE_LIB variable points the oracle at the copy). The pins pass on
the real oracle and must fail on every mutant.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "dropped_term": ("spa[j] += a * b;", "if (q + 1 < brp[k + 1]) spa[j] += a * b;", "test_oracle_spgemm.py"),
    "wrong_sign": ("spa[j] += a * b;", "spa[j] -= a * b;", "test_oracle_spgemm.py"),
    "wrong_index": ("double b = bval[q];", "double b = bval[brp[k]];", "test_oracle_spgemm.py"),
    "no_sort": ("qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);", "", "test_oracle_spgemm.py"),
    "count_skips_first": ("for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {\n                int32_t k = aci[p];\n                for (int32_t q = brp[k]; q < brp[k + 1]; ++q) {\n                    int32_t j = bci[q];\n                    if (mark[j] != t) { mark[j] = t; ++cnt; }",
                          "for (int32_t p = arp[i] + 1; p < arp[i + 1]; ++p) {\n                int32_t k = aci[p];\n                for (int32_t q = brp[k]; q < brp[k + 1]; ++q) {\n                    int32_t j = bci[q];\n                    if (mark[j] != t) { mark[j] = t; ++cnt; }",
                          "test_oracle_spgemm.py"),
    "tc_wrong_row": ("for (int32_t q = lrp[k]; q < lrp[k + 1]; ++q)", "for (int32_t q = lrp[i]; q < lrp[i + 1]; ++q)", "test_oracle_tc.py"),
    "tc_upper_triangle": ("if (j < i) lci[nnz++] = j;", "if (j > i) lci[nnz++] = j;", "test_oracle_tc.py"),
    "tc_ascending_degree": ("return (da < db) - (da > db);", "return (da > db) - (da < db);", "test_oracle_tc.py"),
    "bwd_transposed_operand": ("dA[p] += w[j] * bval[q];", "dA[p] += w[j] * a;", "test_oracle_backward.py"),
    "bwd_dropped_dB": ("dB[q] += a * w[j];", "if (q > brp[k]) dB[q] += a * w[j];", "test_oracle_backward.py"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new, pins = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           str(mutant), "-o", str(lib)])
    env = dict(os.environ, ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", pins)], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"pins in {pins} did not catch mutant {name}:\n{r.stdout[-2000:]}"
