"""The droplet sweep (64 D2Q9 SRT droplets: sides U{64..512}, R, G in
[-5.5, -4.5], tau in {0.8, 1, 1.2} and force order per item; the droplet
test of Sec. 3 repeated over a parameter sweep) against the FP64 oracle's
own runs, stored by tests/golden/make_sweep_64_oracle.py.

early   every item after 2,000 steps, the whole sweep in one batch.  FP64
        state: observables within 1e-9 relative (Laplace jump: 1e-9 of p_in),
        the centre lines within 1e-10.  FP32 state: |u| norms within 1e-3
        relative, Laplace jump within 1e-4 of p_in, density extremes within
        5e-5 relative (the FP32 density drifts by ~1e-5 over 2,000 steps).
        The six items the oracle sees diverge (non-finite)
        are non-finite on the GPU as well.
steady  the 4 smallest items to the steady-state rule (max |u| change below
        1e-10 between checks 100 steps apart):
        - FP64 batch: stops at the oracle's step, or one check from it where
          the change crosses 1e-10 within rounding, and the item the oracle
          sees diverge is quarantined; single FP64 runs to the oracle's stop
          step match its observables to 1e-9 and its centre lines to 1e-10;
        - FP32 batch with its own rules: max |u| within 1e-3 and the Laplace
          jump within 1e-4 of the oracle's steady values, except item 27,
          whose FP64 run develops a slow symmetry-breaking mode over 10^5
          steps (max |u| +8%) that the FP32 state does not resolve: the
          rounding of its stored populations absorbs the mode's per-step
          growth (expected failure);
        - the FP32 batch finished in FP64 (sc_lbm_batch_promote, then the
          literal rule): the observables of the oracle's own run at the step
          where the finish stopped (the stored samples every 500 steps,
          interpolated) to 1e-4 (max |u|), 5e-5 (mean |u|) and 1e-5 (Laplace
          jump, density extremes): the FP32 stage's deviation, decaying in
          the FP64 stage.  The rule can fire at a turning point of
          max |u| while the state still relaxes, so the finish and the
          oracle may stop far apart; item 27's slow mode, which the FP32
          stage does not resolve, develops in the FP64 stage.
"""
import json
import math
import os

import numpy as np
import pytest

from tests.gpu_helpers import say
from workload import droplet_rho

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1906_11027_amd import Batch, Sim  # noqa: E402

with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sweep_64_oracle.json")) as _fh:
    GOLD = json.load(_fh)
ITEMS = GOLD["items"]
OBS = ("max_u", "mean_u", "l2_u", "rho_in", "rho_out", "rho_min", "rho_max", "mass")


def _item(k):
    it = ITEMS[k]
    return {"rho0": droplet_rho((it["side"],) * 2, it["R"], seed=it["seed"]), "order": it["order"], "G": it["G"],
            "tau": it["tau"]}


def _finite(ob):
    return all(math.isfinite(ob[k]) for k in ("max_u", "mass"))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sweep_first_2000_steps(prec):
    say("case sweep of 64 droplets, %d steps, %s" % (GOLD["early_steps"], prec))
    items = [_item(k) for k in range(len(ITEMS))]
    bt = Batch(items, precision=prec)
    bt.step(GOLD["early_steps"])
    worst = {}
    for ref in GOLD["early"]:
        k = ref["item"]
        got = bt.observe(k)
        ob, ro = got["obs"], ref["obs"]
        if not _finite(ro):
            assert ob["nonfinite"] > 0, (k, "oracle diverges, GPU finite")
            continue
        assert ob["nonfinite"] == 0, k
        y = ITEMS[k]["side"] // 2
        if prec == "fp64":
            for key in OBS:
                e = abs(ob[key] - ro[key]) / abs(ro[key])
                worst[key] = max(worst.get(key, 0.0), e)
                assert e <= 1e-9, (k, key, ob[key], ro[key])
            assert abs(ob["dp"] - ro["dp"]) <= 1e-9 * abs(ro["p_in"]), k
            assert np.max(np.abs(got["rho"][:, y] - np.asarray(ref["rho_line"]))) <= 1e-10, k
            assert np.max(np.abs(got["u"][:, :, y] - np.asarray(ref["u_line"]))) <= 1e-10, k
        else:
            errs = {key: abs(ob[key] - ro[key]) / ro[key] for key in ("max_u", "mean_u", "l2_u", "rho_min", "rho_max")}
            errs["dp/p_in"] = abs(ob["dp"] - ro["dp"]) / abs(ro["p_in"])
            for key, e in errs.items():
                worst[key] = max(worst.get(key, 0.0), e)
            say("item %d: %s" % (k, " ".join("%s %.1e" % kv for kv in sorted(errs.items()))))
            for key in ("max_u", "mean_u", "l2_u"):
                assert errs[key] <= 1e-3, (k, key, ob[key], ro[key])
            assert errs["dp/p_in"] <= 1e-4, (k, ob["dp"], ro["dp"])
            # the FP32 state's density drifts by ~1e-5 over 2,000 steps
            # (interface and bulk respond to its rounding; measured up to
            # 1.4e-5 in the largest droplets), hence 5e-5 here
            for key in ("rho_min", "rho_max"):
                assert errs[key] <= 5e-5, (k, key, ob[key], ro[key])
    bt.close()
    say("sweep %s at %d steps, worst relative errors: %s" % (
        prec, GOLD["early_steps"], " ".join("%s %.1e" % kv for kv in sorted(worst.items()))))


STEADY = [s["item"] for s in GOLD["steady"]]


def _steady_ref(k):
    return next(s for s in GOLD["steady"] if s["item"] == k)


def test_sweep_steady_fp64_batch():
    items = [_item(k) for k in STEADY]
    bt = Batch(items, precision="fp64", obs_every=GOLD["every"])
    bt.step(GOLD["max_steps"], tol=GOLD["tol"])
    for j, k in enumerate(STEADY):
        ref = _steady_ref(k)
        steps, by = bt.status(j)
        say("steady item %d: FP64 batch %d steps (by %d), oracle %d (%s)" % (
            k, steps, by, ref["step"], "converged" if ref["converged"] else "not converged"))
        if not _finite(ref["obs"]):
            assert by == -1, k
            continue
        assert by == 1 and abs(steps - ref["step"]) <= GOLD["every"], (k, steps, ref["step"])
        ob = bt.observe(j, fields=False)["obs"]
        assert abs(ob["max_u"] - ref["obs"]["max_u"]) <= 1e-8 * ref["obs"]["max_u"], k
    bt.close()


@pytest.mark.parametrize("k", [s["item"] for s in GOLD["steady"] if s["converged"]])
def test_sweep_steady_fp64_single_at_oracle_step(k):
    ref = _steady_ref(k)
    it = _item(k)
    sim = Sim(it["rho0"], "D2Q9", order=it["order"], G=it["G"], tau=it["tau"], precision="fp64")
    sim.step(ref["step"])
    got = sim.observe()
    sim.close()
    ob, ro = got["obs"], ref["obs"]
    for key in OBS:
        assert abs(ob[key] - ro[key]) <= 1e-9 * abs(ro[key]), (k, key, ob[key], ro[key])
    assert abs(ob["dp"] - ro["dp"]) <= 1e-9 * abs(ro["p_in"])
    y = ITEMS[k]["side"] // 2
    er = float(np.max(np.abs(got["rho"][:, y] - np.asarray(ref["rho_line"]))))
    eu = float(np.max(np.abs(got["u"][:, :, y] - np.asarray(ref["u_line"]))))
    say("item %d at the oracle's stop (%d steps): centre line rho %.1e u %.1e" % (k, ref["step"], er, eu))
    assert er <= 1e-10 and eu <= 1e-10


def _fp32_cases():
    out = []
    for s in GOLD["steady"]:
        if not s["converged"]:
            continue
        k = s["item"]
        marks = [pytest.mark.xfail(strict=True, reason="slow mode below the FP32 state's resolution")] \
            if k == 27 else []
        out.append(pytest.param(k, marks=marks))
    return out


@pytest.fixture(scope="module")
def fp32_sweep():
    items = [_item(k) for k in STEADY]
    bt = Batch(items, precision="fp32", obs_every=GOLD["every"])
    bt.step(GOLD["max_steps"], tol=GOLD["tol"])
    res = {k: (bt.status(j), bt.observe(j, fields=False)["obs"]) for j, k in enumerate(STEADY)}
    bt.promote()
    bt.step(GOLD["max_steps"], tol=GOLD["tol"])
    res64 = {k: (bt.status(j), bt.observe(j, fields=False)["obs"]) for j, k in enumerate(STEADY)}
    bt.close()
    return res, res64


@pytest.mark.parametrize("k", _fp32_cases())
def test_sweep_steady_fp32_batch(fp32_sweep, k):
    (steps, by), ob = fp32_sweep[0][k]
    ro = _steady_ref(k)["obs"]
    e = abs(ob["max_u"] - ro["max_u"]) / ro["max_u"]
    say("item %d FP32 batch: %d steps (by %d), max|u| %.6e vs oracle %.6e (rel %.1e)" % (
        k, steps, by, ob["max_u"], ro["max_u"], e))
    assert by > 0
    assert e <= 1e-3
    assert abs(ob["dp"] - ro["dp"]) <= 1e-4 * abs(ro["dp"])


def _tail_at(k, step):
    """The oracle's observables of item k at `step`, linearly interpolated
    between its samples every `tail_every` steps (the slow relaxation moves
    max|u| by about 1e-9 per 500 steps there)."""
    t = next(r for r in GOLD["tails"] if r["item"] == k)
    at = np.asarray(t["steps"], dtype=float)
    assert at[0] <= step <= at[-1], (k, step, at[-1])
    return {key: float(np.interp(step, at, np.asarray(v))) for key, v in t["obs"].items()}


@pytest.mark.parametrize("k", [s["item"] for s in GOLD["steady"]])
def test_sweep_steady_fp32_then_fp64(fp32_sweep, k):
    ref = _steady_ref(k)
    (steps, by), ob = fp32_sweep[1][k]
    (s32, by32), _ = fp32_sweep[0][k]
    say("item %d FP32 batch %d steps (by %d), promoted, FP64 to %d steps (by %d); oracle %d" % (
        k, s32, by32, steps, by, ref["step"]))
    if not _finite(ref["obs"]):
        assert by32 == -1 and by == -1
        return
    assert by == 1
    # The literal rule stops at the first check whose max|u| differs from the
    # previous one by less than 1e-10.  Near a turning point of max|u| it can
    # fire while the state still relaxes (item 63: the oracle stops at 5,200
    # steps, and its max|u| falls by another 5e-4 of itself over the next
    # 100,000), so the two runs may stop far apart.  The finished state is
    # compared with the oracle's own run at the step where the finish stopped.
    # What remains is the FP32 stage's deviation at the promotion, decaying in
    # the FP64 stage: item 41 is promoted 2.2e-4 (max |u|) from the oracle's
    # run at the same step and stops 1,100 FP64 steps later with 3.2e-5 left.
    ro = _tail_at(k, steps)
    errs = {key: abs(ob[key] - ro[key]) / abs(ro[key]) for key in ("max_u", "mean_u", "dp", "rho_min", "rho_max")}
    say("item %d finished in FP64 vs the oracle at step %d: %s" % (
        k, steps, " ".join("%s %.1e" % kv for kv in sorted(errs.items()))))
    assert errs["max_u"] <= 1e-4, (k, ob["max_u"], ro["max_u"])
    assert errs["mean_u"] <= 5e-5, (k, ob["mean_u"], ro["mean_u"])
    for key in ("dp", "rho_min", "rho_max"):
        assert errs[key] <= 1e-5, (k, key, ob[key], ro[key])
