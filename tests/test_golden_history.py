"""The stored laser-heating history (tests/golden/laser_history_8.txt) is the
oracle's: its first 40 steps are recomputed live and must agree to
rounding, so a change in the oracle's arithmetic shows here before the
GPU history test compares against a stale file."""
import numpy as np

from tests.golden import make_laser_history as G


def test_stored_history_is_the_oracle_run():
    hist_ref, T_ref = G.load()
    assert len(hist_ref) == G.N_STEPS and len(T_ref) == G.N_CELLS ** 3
    hist, _ = G.run(40)
    np.testing.assert_allclose(hist, hist_ref[:40], rtol=1e-14, atol=0)
    # the pulse heats the top: the stored run rises and the last field is warmer than the start
    assert hist_ref.max() > 300.01 and np.all(np.isfinite(T_ref)) and T_ref.max() > 300.0
