"""The stored oracle digests (tests/golden/oracle_digests.json) agree with the
seeded generator and with the oracle: every case's input images hash as
stored, and the cases the oracle finishes in a few seconds reproduce their
stored output digests exactly."""
import os
import sys

import pytest

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import oracle_digests as od  # noqa: E402


def test_every_case_is_stored_and_inputs_match_the_generator():
    table = od.load()
    assert table["params"] == od.PARAMS
    names = [n for n, _ in od.cases()]
    assert sorted(table["cases"]) == sorted(names)
    for name, spec in od.cases():
        stored = table["cases"][name]
        assert stored["spec"] == spec, name
        left, right = od.case_inputs(spec)
        assert od.digest(left) == stored["inputs"]["left"], name
        assert od.digest(right) == stored["inputs"]["right"], name


@pytest.mark.parametrize("name", ["batch_320x240x64", "batch_320x240x128", "batch_640x512x64",
                                  "serve_640x512x128_0"])
def test_small_cases_reproduce(oracle_lib, name):
    oracle = oracle_lib
    stored = od.load()["cases"][name]
    left, right = od.case_inputs(stored["spec"])
    ref = oracle.run(left, right, oracle.Params(ndisp=stored["spec"]["ndisp"], **od.PARAMS))
    for key, want in stored["outputs"].items():
        assert od.digest(ref[key]) == want, f"{name}: {key}"
