"""The continuous-batching solve server (GPU): requests admitted by memory,
advanced together, each result identical alone and in the mix and within
its storage format's error of the FP64 oracle run for the same steps;
requests retire when their steady-state residual falls below the tolerance
and waiting requests take the freed memory."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


SERVER_RATES = dict(s_c=1.2, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=0.8)  # the server's defaults

# rel-L2(u) of a served request against the FP64 oracle at the same step
# count: FP64 at the rounding floor (growing as sqrt(steps)), the others at
# their storage rounding (measured on the mix below at 400 steps: f16s at most
# 3.4e-4, f32 6.2e-5, f32s 4.3e-6, f64 6.5e-14)
ORACLE_BOUND = {"f64": 1e-12, "f32s": 1e-4, "f32": 1e-3, "f16s": 5e-3}


def _check_against_oracle(oracle, req, s, precision):
    o = oracle.Oracle(req["L"], req["L"], req["phi"], kappa=0.5, rates=SERVER_RATES,
                      g=(req["g"], 0.0), drag=(req["beta"], (0.0, 0.0))).init_equilibrium()
    o.step(s.steps)
    ref = o.macroscopic()
    e = math.sqrt(np.sum((s.result["ux"] - ref["ux"]) ** 2 + (s.result["uy"] - ref["uy"]) ** 2)
                  / np.sum(ref["ux"] ** 2 + ref["uy"] ** 2))
    bound = ORACLE_BOUND[precision]
    if precision == "f64":
        bound *= math.sqrt(max(s.steps, 1000) / 1000.0)
    _say(f"  request {s.rid} ({s.L}^2, {s.steps} steps, {precision}): rel-L2(u) vs oracle "
         f"{e:.3e} (bound {bound:.1e})")
    assert e <= bound


def small_requests():
    from paper_2409_02964_amd import workloads as W
    rng = np.random.default_rng(7)
    out = []
    for k, (L, t) in enumerate([(40, 0.0), (64, 0.0), (33, 0.02), (80, 0.05), (50, 0.05),
                                (72, 0.3), (45, 0.31)]):
        phi = W.inclusion_phi(L, rng, rmin=3.0, rmax=9.0, fill=0.2)
        out.append(dict(rid=k, L=L, arrival=t, phi=phi, beta=3e-3 + 2e-2 * (1 - phi),
                        g=1e-5 * (1 + 0.1 * k)))
    return out


@pytest.mark.parametrize("precision,steps_per_pass", [("f16s", 1), ("f32", 1), ("f16s", 2)])
def test_served_results_equal_solo_runs(precision, steps_per_pass):
    _torch()
    from paper_2409_02964_amd.serve import SolveServer
    from paper_2409_02964_amd.vanse import workspace_bytes
    reqs = small_requests()
    need = sorted(workspace_bytes(r["L"], r["L"], precision, drag=True) for r in reqs)
    budget = need[-1] + need[-2] + need[0]  # about three requests at a time
    kw = dict(precision=precision, chunk=40, max_steps=400, tol=1e-7, keep_results=True,
              steps_per_pass=steps_per_pass)
    mix = SolveServer(budget, **kw)
    done = {s.rid: s for s in mix.run(reqs)}
    assert sorted(done) == list(range(len(reqs)))
    assert max(a for _, a, _, _ in mix.log) >= 2          # requests overlapped on the GPU
    assert any(p > 0 for _, _, p, _ in mix.log)           # some waited for memory
    assert all(u <= budget for _, _, _, u in mix.log)
    for r in reqs:
        solo = SolveServer(1 << 40, **kw).run([dict(r, arrival=0.0)])[0]
        s = done[r["rid"]]
        assert s.steps == solo.steps and s.converged == solo.converged
        assert np.array_equal(s.populations, solo.populations)
        assert s.history == solo.history
        assert s.latency >= 0 and s.finished >= s.admitted >= s.arrival - 1e-9


@pytest.mark.parametrize("precision,steps_per_pass", [("f16s", 1), ("f32", 1), ("f32s", 1), ("f64", 1),
                                                      ("f16s", 2), ("f64", 2)])
def test_served_results_match_oracle(oracle, precision, steps_per_pass):
    """Every request of a served mix (run to the step cap) against the FP64
    oracle advanced by the same number of steps from the same inputs, with
    one or two time steps per launch."""
    _torch()
    from paper_2409_02964_amd.serve import SolveServer
    from paper_2409_02964_amd.vanse import workspace_bytes
    reqs = small_requests()
    need = sorted(workspace_bytes(r["L"], r["L"], precision, drag=True) for r in reqs)
    srv = SolveServer(need[-1] + need[-2] + need[0], precision=precision, chunk=40,
                      max_steps=400, tol=1e-30, keep_results=True, steps_per_pass=steps_per_pass)
    done = {s.rid: s for s in srv.run(reqs)}
    assert max(a for _, a, _, _ in srv.log) >= 2
    for r in reqs:
        _check_against_oracle(oracle, r, done[r["rid"]], precision)


def converging_requests():
    """Small lattices with a strong drag: they reach a steady state within a
    few hundred steps."""
    from paper_2409_02964_amd import workloads as W
    rng = np.random.default_rng(11)
    out = []
    for k, (L, t) in enumerate([(36, 0.0), (48, 0.0), (40, 0.0), (30, 0.01), (44, 0.02),
                                (34, 0.02)]):
        phi = W.inclusion_phi(L, rng, rmin=3.0, rmax=8.0, fill=0.2)
        out.append(dict(rid=k, L=L, arrival=t, phi=phi, beta=2e-2 + 5e-2 * (1 - phi),
                        g=1e-5 * (1 + 0.2 * k)))
    return out


@pytest.mark.parametrize("precision,tol", [("f64", 1e-9), ("f32s", 1e-5)])
def test_served_requests_retire_on_convergence(oracle, precision, tol):
    """With a tolerance above the storage format's residual floor every
    request retires on its residual before the step cap; the memory it frees
    admits a waiting request; each converged result matches the oracle run
    for the same steps and is bitwise the request served alone."""
    _torch()
    from paper_2409_02964_amd.serve import SolveServer
    from paper_2409_02964_amd.vanse import workspace_bytes
    reqs = converging_requests()
    need = sorted(workspace_bytes(r["L"], r["L"], precision, drag=True) for r in reqs)
    budget = need[-1] + need[-2]  # two requests at a time at most
    kw = dict(precision=precision, chunk=50, max_steps=5000, tol=tol, keep_results=True)
    srv = SolveServer(budget, **kw)
    done = {s.rid: s for s in srv.run(reqs)}
    assert sorted(done) == list(range(len(reqs)))
    for s in done.values():
        _say(f"request {s.rid}: {s.steps} steps, residual {s.residual:.2e}")
        assert s.converged and s.residual < tol and s.steps < kw["max_steps"]
    assert max(a for _, a, _, _ in srv.log) == 2
    # only two fit at a time: the others were admitted as retirements freed
    # memory
    first_retirement = min(s.finished for s in done.values())
    assert sum(s.admitted < first_retirement for s in done.values()) == 2
    for r in reqs:
        s = done[r["rid"]]
        _check_against_oracle(oracle, r, s, precision)
        solo = SolveServer(1 << 40, **kw).run([dict(r, arrival=0.0)])[0]
        assert solo.steps == s.steps and solo.converged
        assert np.array_equal(s.populations, solo.populations)


def test_server_rejects_request_larger_than_budget():
    _torch()
    from paper_2409_02964_amd.serve import SolveServer
    r = small_requests()[0]
    with pytest.raises(ValueError):
        SolveServer(1024, chunk=10, max_steps=20).run([r])
