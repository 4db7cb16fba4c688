"""The stored oracle trajectories (tests/golden/*_trajectory.npz) are the
oracle's: the first two iterations from the cold start, run afresh, give the
stored errors; the stored probe spread comes from a run that does differ;
and the stored error curves rise again after iteration 50 on these Poisson
scans (no consistent fixed point), as the GPU runs do.  CPU only."""
import importlib.util
import os

import numpy as np
import pytest

from oracle import dm_oracle as oracle

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location(
    "make_trajectories", os.path.join(HERE, "golden", "make_trajectories.py"))
golden = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(golden)


@pytest.mark.parametrize("case", ["spiral_300", "flyscan188_40"])
def test_stored_trajectory_starts_as_the_oracle_does(case):
    g = np.load(golden.out_path(case))
    s = golden.CASES[case]()
    psi = oracle.init_views(s.P0, s.O0, s.pos)
    P, O = s.P0.astype(np.complex128), s.O0.astype(np.complex128)
    I = s.I.astype(np.float64)
    for it in range(2):
        psi, P, O, e = oracle.iterate(psi, P, O, s.pos, I, s.beta)
        stored = g["eps"][it]
        assert abs(e["eps_probe"] - stored[0]) <= 1e-10 * stored[0]
        assert abs(e["eps_obj"] - stored[1]) <= 1e-10 * stored[1]
        assert abs(e["eps_psi"] - stored[2]) <= 1e-10 * stored[2]
    assert g["eps"].shape == g["eps_perturbed"].shape == (golden.N_ITER, 3)
    # the perturbation is invisible at first and grows later
    assert abs(g["eps_perturbed"][0, 0] - g["eps"][0, 0]) <= 1e-6 * g["eps"][0, 0]
    assert float(g["P_spread"]) > 0 and float(g["model_spread"]) > 0
    assert g["P"].shape == s.P0.shape
