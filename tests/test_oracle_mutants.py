"""The controller pins catch plausible mistakes: each test plants one mistake
in a copy of oracle.c (on the CPU, in a temporary directory), builds it, and
requires that at least one of the pins of tests/test_oracle_controller.py
fails against that build while all of them pass against the real oracle.
"""
import os

import pytest

from tests import test_oracle_controller as P

PINS = [P.pin_initial_step, P.pin_error_estimate, P.pin_neighbour_order_estimates,
        P.pin_order_choice_rules, P.pin_step_counts_vs_scipy_bdf,
        P.pin_order_usage_vs_scipy_kappa0, P.pin_smooth_problem_reaches_order_5]

# (name, text in oracle.c, replacement): each a mistake someone could make
# writing the controller from its description.
MUTANTS = [
    ("order choice reads D_(k+1) for the higher order",
     "D + (k + 2) * n, s2, &factor)", "D + (k + 1) * n, s2, &factor)"),
    ("error constant 1/k instead of 1/(k+1)",
     "tmp[i] = d[i] / (double)(k + 1);", "tmp[i] = d[i] / (double)k;"),
    ("higher-order estimate divided by k+1",
     "tmp[i] = dk2[i] / (double)(k + 2);", "tmp[i] = dk2[i] / (double)(k + 1);"),
    ("lower-order estimate divided by k-1",
     "tmp[i] = dk[i] / (double)k;", "tmp[i] = dk[i] / (double)(k - 1);"),
    ("ties between k and k-1 go to k-1",
     "if (fm > best) { best = fm; dk_ = -1; }", "if (fm >= best) { best = fm; dk_ = -1; }"),
    ("ties between k-1 and k+1 go to k+1",
     "if (fp > best) { best = fp; dk_ = 1; }", "if (fp >= best) { best = fp; dk_ = 1; }"),
    ("starting step without the square root",
     "h1 = sqrt(0.01 / dm);", "h1 = 0.01 / dm;"),
    ("starting step cap 10 h0",
     "double h = 100.0 * h0;", "double h = 10.0 * h0;"),
    ("order-k ratio exponent -1/k",
     "double f0 = pow(err, -1.0 / (double)(k + 1));", "double f0 = pow(err, -1.0 / (double)k);"),
]


def test_pins_pass_on_the_oracle(oracle):
    for pin in PINS:
        pin(oracle)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(oracle, tmp_path, name, old, new):
    with open(oracle.SRC) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site not found once: {old}"
    path = os.path.join(tmp_path, "mutant.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = oracle.compile_source(path, os.path.join(tmp_path, "libmutant.so"))
    failed = []
    with oracle.using_library(so):
        for pin in PINS:
            try:
                pin(oracle)
            except AssertionError:
                failed.append(pin.__name__)
    print(f"{name}: caught by {failed}")
    assert failed, f"no pin catches the mistake: {name}"
