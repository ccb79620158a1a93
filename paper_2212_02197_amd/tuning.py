"""Monte Carlo based NMPC tuning (the paper's outlook: its performance
quantification suits tuning of the stage cost or of a constraint back-off).

A tuning candidate changes one controller setting of the campaign; every
candidate runs the same sample ids on the same Philox noise (common random
numbers), so differences between candidates are the controller's and not the
noise's.  Each evaluation is one campaign of the HIP library; this module
only chooses the settings and reduces the per-sample costs.

Settings:
  * "backoff" b (mL/min): the NMPC's input bounds become [u_min + b, u_max - b]
    (the plant's flow stays physical; the controller keeps a margin);
  * "Qz": the stage-cost weight.  With the paper's stage cost (the output
    error only) a positive factor scales the OCP's objective without moving
    its minimiser, so Qz moves mean Phi only through the SQP's stopping test
    (its scaled KKT residual grows with Qz): a tuning of the stage cost needs
    a second term the paper does not define;
  * "N": the prediction horizon (a sweep; no derivative).
"""
from __future__ import annotations

import math

import numpy as np

from . import binding

SETTINGS = ("backoff", "Qz", "N")


def _apply(cfg: dict, name: str, value) -> dict:
    c = dict(cfg)
    if name == "backoff":
        b = float(value)
        if not 0.0 <= 2.0 * b < cfg["umax"] - cfg["umin"]:
            raise ValueError("back-off must leave a non-empty input range")
        c["umin"] = cfg["umin"] + b
        c["umax"] = cfg["umax"] - b
    elif name == "Qz":
        if not value > 0:
            raise ValueError("Qz must be positive")
        c["Qz"] = float(value)
    elif name == "N":
        c["N"] = int(value)
    else:
        raise KeyError(f"unknown tuning setting {name!r}; one of {SETTINGS}")
    return c


def evaluate(cfg: dict, name: str, value) -> dict:
    """One candidate: the NMPC samples' Phi (numpy, NaN for a diverged
    closed loop) and their statistics."""
    c = _apply(cfg, name, value)
    camp = binding.Campaign(c)
    camp.run()
    phi, st = camp.costs()
    ps = camp.per_sample()
    camp.close()
    nm = ps["kind"] == 0
    return dict(value=value, phi=phi[nm], mean=st["mean"][0], var=st["var"][0],
                count=st["count"][0], ocp_failed=int(ps["n_ocp_fail"][nm].sum()))


def sweep(cfg: dict, name: str, values) -> list:
    """Mean and variance of Phi for every candidate value (common random
    numbers), and each candidate's mean difference to the first with its
    standard error from the per-sample differences."""
    out = []
    base = None
    for v in values:
        r = evaluate(cfg, name, v)
        if base is None:
            base = r
        d = r["phi"] - base["phi"]
        d = d[np.isfinite(d)]
        out.append(dict(value=v, mean=r["mean"], var=r["var"], count=r["count"],
                        ocp_failed=r["ocp_failed"],
                        diff_to_first=float(d.mean()) if d.size else 0.0,
                        diff_stderr=float(d.std(ddof=1) / math.sqrt(d.size)) if d.size > 1 else 0.0))
    return out


def crn_gradient(cfg: dict, name: str, value, step: float) -> dict:
    """d mean Phi / d setting at `value` by a central difference over common
    random numbers: the mean over samples of (Phi(v + h) - Phi(v - h)) / 2h,
    with its standard error.  The pathwise derivative of each sample's Phi
    has kinks where an active set changes, so h must stay above the scale
    of those kinks; the estimate is of the derivative of the mean."""
    if name == "N":
        raise ValueError("the horizon is an integer: use sweep")
    lo = evaluate(cfg, name, value - step)
    hi = evaluate(cfg, name, value + step)
    d = (hi["phi"] - lo["phi"]) / (2.0 * step)
    d = d[np.isfinite(d)]
    return dict(value=value, step=step, gradient=float(d.mean()),
                stderr=float(d.std(ddof=1) / math.sqrt(d.size)) if d.size > 1 else 0.0,
                samples=int(d.size), mean_minus=lo["mean"], mean_plus=hi["mean"])
