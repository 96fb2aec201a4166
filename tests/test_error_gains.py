"""The stored error gains (tests/golden/error_gains.json) are what the oracle
computes for the named configurations today: recomputed for a few components of
the small configurations (the script, tests/golden/make_error_gains.py, writes
them from the oracle alone), and every configuration the GPU tests bound has an
entry with one gain per body coordinate."""
import importlib.util
import json
import os

import numpy as np

from tests.parity_configs import gain_configs

HERE = os.path.dirname(os.path.abspath(__file__))


def _script():
    spec = importlib.util.spec_from_file_location("make_error_gains",
                                                  os.path.join(HERE, "golden", "make_error_gains.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_every_configuration_has_gains():
    with open(os.path.join(HERE, "golden", "error_gains.json")) as fh:
        data = json.load(fh)
    for name, w in gain_configs().items():
        assert name in data, name
        assert len(data[name]["gain"]) == 6 * w.nb
        assert list(data[name]["grid"]) == list(w.n) and data[name]["markers"] == w.nm
        assert data[name]["max_oracle_residual"] < 1e-11


def test_stored_gains_match_a_recomputation():
    mod = _script()
    with open(os.path.join(HERE, "golden", "error_gains.json")) as fh:
        data = json.load(fh)
    for name, ks in (("ragged_10x12x14", (0, 4, 11, 17)), ("periodic_x_16x12x12", (2, 9))):
        for k in ks:
            _, _, g, res = mod._gain((name, k))
            assert abs(g - data[name]["gain"][k]) <= 1e-9 * g, (name, k)
            assert res < 1e-11
