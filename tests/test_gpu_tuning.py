"""Monte Carlo NMPC tuning on the GPU against the oracle: candidate
back-offs on common random numbers, their mean costs and the central
difference of the mean, at the parity bar."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a HIP device", allow_module_level=True)

import oracle  # noqa: E402
from paper_2212_02197_amd import tuning, workloads as W  # noqa: E402

NTHREADS = min(16, len(os.sched_getaffinity(0)))


def _oracle_phi(cfg, b):
    c = tuning._apply(cfg, "backoff", b)
    return oracle.run(c, ids=np.arange(cfg["n_samples"]), nthreads=NTHREADS)["phi"]


def test_backoff_sweep_and_crn_gradient_match_the_oracle():
    # c0's recipe: 64 NMPC samples at 320 K, SQP tolerance 1e-10
    cfg = W.c0_small_nmpc(sqp_eps=1e-10)
    values = (0.0, 100.0, 300.0)
    res = tuning.sweep(cfg, "backoff", values)
    for r in res:
        ref = _oracle_phi(cfg, r["value"])
        m, v, _ = oracle.stats(ref)
        print("backoff", r["value"], "mean", r["mean"], "oracle", m, "diff to first",
              r["diff_to_first"], "+-", r["diff_stderr"], flush=True)
        assert r["mean"] == pytest.approx(m, rel=1e-8)
        assert r["var"] == pytest.approx(v, rel=1e-8)
    g = tuning.crn_gradient(cfg, "backoff", 300.0, 20.0)
    lo, hi = _oracle_phi(cfg, 280.0), _oracle_phi(cfg, 320.0)
    g_ref = np.mean((hi - lo) / 40.0)
    print("d mean Phi / d backoff at 300", g, "oracle", g_ref, flush=True)
    assert g["gradient"] == pytest.approx(g_ref, rel=1e-6, abs=1e-12)
