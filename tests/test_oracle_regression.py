"""The oracle still reproduces its frozen fixtures (tests/golden/make_golden.py)."""
import os

import numpy as np

import importlib.util

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
mg = importlib.util.module_from_spec(spec)
spec.loader.exec_module(mg)


def test_yamaguchi_fixture():
    ref = np.loadtxt(os.path.join(HERE, "yamaguchi_s_sample0.txt"))
    got = mg.yamaguchi_case()
    assert np.allclose(got[:, 0], ref[:, 0], rtol=1e-10, atol=1e-14)
    assert np.abs(got[:, 1] - ref[:, 1]).max() < 1e-8


def test_coupled_fixture():
    ev_ref = np.loadtxt(os.path.join(HERE, "coupled_yukawa_sample0_evals.txt"))
    ph_ref = np.loadtxt(os.path.join(HERE, "coupled_yukawa_sample0_phases.txt"))
    ev, ph = mg.coupled_case()
    assert np.allclose(ev, ev_ref, rtol=1e-10, atol=1e-14)
    assert np.abs(ph - ph_ref).max() < 1e-7
