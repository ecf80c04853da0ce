"""The oracle still reproduces its frozen regression fixtures."""
import json
import os

import numpy as np
import pytest

import oracle
from tests.golden.make_golden import CASES

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name", sorted(CASES))
def test_oracle_matches_fixture(oracle_lib, name):
    with open(os.path.join(HERE, name)) as f:
        ref = json.load(f)
    sc, idx = CASES[name]()
    assert idx.tolist() == ref["receivers"]
    P, TL = oracle.forward(sc.table, sc.gamma, sc.rcv[idx], sc.freqs, sc.eps, c=sc.c, gate=sc.gate)
    Pref = np.array(ref["P_re"]) + 1j * np.array(ref["P_im"])
    assert np.max(np.abs(P - Pref) / np.abs(Pref)) <= 1e-12
