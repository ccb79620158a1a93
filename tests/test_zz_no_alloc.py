"""The allocation-free entry point mc_cl_run_static against mc_cl_run.

Both run the same kernels; the launch shape differs (the static run sizes its
wavefront slots to the library's scratch array) and Phi, the counters and the
active-set hashes do not depend on it, so the outputs must agree bit for bit.
Two calls in a row on the shared scratch array, the second smaller.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a HIP device", allow_module_level=True)

from paper_2212_02197_amd import binding, workloads as W  # noqa: E402


def _reference(cfg):
    camp = binding.Campaign(cfg)
    camp.run()
    camp.costs()
    ps = camp.per_sample()
    camp.close()
    return ps


def _static(cfg):
    S = cfg["n_samples"]
    dev = torch.device("cuda", torch.cuda.current_device())
    phi = torch.full((S,), float("nan"), dtype=torch.float64, device=dev)
    cnt = torch.full((binding.NCNT, S), -7, dtype=torch.int32, device=dev)
    hsh = torch.zeros(S, dtype=torch.int64, device=dev)
    binding.run_static(cfg, phi, cnt, hsh)
    torch.cuda.synchronize()
    c = cnt.cpu().numpy()
    out = {n: c[i] for i, n in enumerate(binding.CNT_NAMES)}
    out["phi"] = phi.cpu().numpy()
    out["ashash"] = hsh.cpu().numpy().view("u8")
    return out


def _same(a, b, tag):
    np.testing.assert_array_equal(a["phi"], b["phi"], err_msg=tag)
    np.testing.assert_array_equal(a["ashash"], b["ashash"], err_msg=tag)
    for n in binding.CNT_NAMES:
        np.testing.assert_array_equal(a[n], b[n], err_msg=f"{tag} {n}")


def test_static_run_equals_run_twice_in_a_row():
    # first call: NMPC in all three horizon classes (N 10 / 25 / 60) with
    # ragged lengths, and PI samples; second call: a smaller campaign on the
    # same scratch array (a mixed c4-like split, N = 25)
    big = W.c3_uneven(n_samples=300, L_lo=5, L_hi=14, horizon_choices=(10, 25, 60),
                      kind_split=200, noise_mod=0, sqp_eps=1e-10)
    small = W.c4_mixed(n_samples=70, kind_split=40, noise_mod=40, L=9, sp_step_lo=2,
                       sp_step_hi=6, sqp_eps=1e-10)
    for tag, cfg in (("first", big), ("second", small)):
        ref = _reference(cfg)
        got = _static(cfg)
        print(tag, "classes", sorted(set(ref["N"][ref["kind"] == 0].tolist())),
              "kinds", np.bincount(ref["kind"]).tolist(), flush=True)
        _same(got, ref, tag)
    assert set(_reference(big)["N"][:200].tolist()) == {10, 25, 60}


def test_static_run_without_optional_outputs():
    cfg = W.c0_small_nmpc(n_samples=33, L=6, sqp_eps=1e-10)
    ref = _reference(cfg)
    phi = torch.empty(33, dtype=torch.float64, device="cuda")
    binding.run_static(cfg, phi)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(phi.cpu().numpy(), ref["phi"])
