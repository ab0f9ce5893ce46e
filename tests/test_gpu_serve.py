"""The continuous-batching solve server (GPU): requests admitted by memory,
advanced together, each result identical alone and in the mix."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


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


def test_server_rejects_request_larger_than_budget():
    _torch()
    from paper_2409_02964_amd.serve import SolveServer
    r = small_requests()[0]
    with pytest.raises(ValueError):
        SolveServer(1024, chunk=10, max_steps=20).run([r])
