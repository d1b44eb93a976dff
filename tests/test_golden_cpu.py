"""CPU checks of the stored oracle summaries under tests/golden (no GPU)."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_c2_oracle_reference_runs_are_converged_and_agree():
    """The two independent FP64 oracle runs of the C2 workload (emulator term on) that the
    GPU posterior test compares with: unflagged ESS above 1e5 each, acceptance at the 0.57
    target, and a noise floor (mean difference over sd, variance ratios) far inside the
    0.05 sd / 5% bar."""
    with open(os.path.join(GOLDEN, "c2_posterior_oracle.json")) as f:
        ref = json.load(f)
    for r in ref["runs"]:
        assert all(fl == 0 for fl in r["ess_flags"]) and r["min_ess"] > 1e5
        assert abs(r["accept"] - 0.57) < 0.03
        c = np.array(r["cov"])
        assert np.all(np.linalg.eigvalsh(c) > 0)
    assert max(ref["noise_floor"]["mean_diff_over_sd"]) < 0.01
    assert np.all(np.abs(np.array(ref["noise_floor"]["var_ratio"]) - 1) < 0.02)
