"""The oracle against its stored values (tests/golden/oracle_sphere120.json,
written by tests/golden/make_golden.py, which calls only the oracle): a guard
against unintended drift of the oracle's arithmetic.  The values are the
oracle's own, so this is no pin of it; the pins are the closed forms,
invariants, brute-force cases and the Mie series of the other oracle tests."""
import importlib.util
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _make_golden():
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_oracle_matches_stored_values():
    make_golden = _make_golden()
    with open(os.path.join(HERE, "golden", "oracle_sphere120.json")) as f:
        stored = json.load(f)
    assert stored["case"] == make_golden.CASE
    want = stored["values"]
    got = make_golden.compute()
    assert (got["ne"], got["K"]) == (want["ne"], want["K"])
    np.testing.assert_allclose(got["block_frobenius"], want["block_frobenius"], rtol=1e-11)
    np.testing.assert_allclose(got["cond1_T0"], want["cond1_T0"], rtol=1e-11)
    np.testing.assert_allclose(got["current_peak"], want["current_peak"], rtol=1e-11)
    # currents sampled over the march, to a fraction of the peak current
    np.testing.assert_allclose(got["current"], want["current"], rtol=0, atol=1e-11 * want["current_peak"])
