"""The pruning pins catch each wrong reading of the zero-clearing rule.

The oracle source is copied with one planted change, compiled on the CPU, and
the pins of tests/test_oracle_prune.py run against that copy in a child
process (QW_ORACLE_LIB); every planted reading must fail the pins named for
it, while the committed oracle passes them (tests/test_oracle_prune.py)."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "qw_oracle.cpp")

# (name, text in the oracle, planted text, pins that must fail)
MUTANTS = [
    ("modulus",  # remove a branch when |amp| <= tau
     "    if (mx <= o.tau) {\n",
     "    if (std::abs(it->second) <= o.tau) {\n",
     {"test_one_step_survivors_mass_and_margin", "test_prepare_survivors_mass_and_margin"}),
    ("either_part",  # remove when |Re| <= tau or |Im| <= tau
     "    const double mx = std::max(std::fabs(it->second.real()), std::fabs(it->second.imag()));\n",
     "    const double mx = std::min(std::fabs(it->second.real()), std::fabs(it->second.imag()));\n",
     {"test_one_step_survivors_mass_and_margin"}),
    ("every_operation",  # prune after each register-level operation
     "    apply(o.st, *o.m, op);\n    o.max_size",
     "    apply(o.st, *o.m, op);\n    prune(o);\n    o.max_size",
     {"test_one_step_survivors_mass_and_margin", "test_raw_tridiagonal_start_100_steps"}),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new,must_fail", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_pruning_rule_fails_pins(tmp_path, name, old, new, must_fail):
    src = open(SRC).read()
    assert src.count(old) == 1, f"planting site for {name} not found once"
    mutant = tmp_path / "qw_oracle_mutant.cpp"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libqworacle_mutant.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", str(lib), str(mutant)], check=True)
    env = dict(os.environ, QW_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-rf", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_prune.py"), "-k", "not cyclic32"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    failed = set(re.findall(r"FAILED tests/test_oracle_prune\.py::(\w+)", r.stdout))
    assert r.returncode != 0, f"{name}: the pins pass with the planted rule\n{r.stdout[-2000:]}"
    assert must_fail <= failed, f"{name}: failed {sorted(failed)}, expected {sorted(must_fail)}"
