"""Host-side checks of the Monte Carlo tuning helpers (no GPU)."""
import pytest

from paper_2212_02197_amd import tuning, workloads as W


def test_backoff_tightens_the_nmpc_bounds_only():
    cfg = W.c0_small_nmpc()
    c = tuning._apply(cfg, "backoff", 25.0)
    assert (c["umin"], c["umax"]) == (25.0, 975.0)
    assert (c["pi_umin"], c["pi_umax"]) == (cfg["pi_umin"], cfg["pi_umax"])
    with pytest.raises(ValueError):
        tuning._apply(cfg, "backoff", 500.0)
    with pytest.raises(KeyError):
        tuning._apply(cfg, "kP", 1.0)
    assert tuning._apply(cfg, "N", 7)["N"] == 7
