"""The serving form (paper_2205_00385_amd.serve): a seeded request stream of
uneven grids, 1-4 load cases and perturbed repeat designs, served with
continuous batching.  Each result is the same alone (one worker, no other
request in flight) and in the mix (three workers, requests overlapping on the
GPU) -- bit for bit while no family is evicted -- and matches the CPU FP64
oracle to the 1e-6 compliance bar; under a tight HBM budget (evictions) the
results stay within 1e-6."""

import numpy as np
import pytest

import synth
from oracle import sens

from gpu_util import log, rel, soa

pytestmark = pytest.mark.gpu

SIZES = ((16, 16, 16), (24, 24, 24), (32, 16, 16))


def _trace():
    return synth.serve_trace(14, 0.0, seed=5, sizes=SIZES, repeat_frac=0.6, max_case=4)


def _server(**kw):
    from paper_2205_00385_amd import aarmr, serve

    kw.setdefault("hbm_budget", 8 << 30)
    kw.setdefault("precision", aarmr.FP32_REFINE)
    return serve.AnalysisServer(keep_u=True, **kw)


def test_serve_same_alone_and_in_mix_and_oracle():
    trace = _trace()
    alone = _server(n_workers=1)
    ra = alone.run(trace, realtime=False)
    mix = _server(n_workers=3)
    rb = mix.run(trace, realtime=False)
    log(f"  paths alone {[r.path for r in ra]}")
    log(f"  workers used in the mix: {sorted(set(r.worker for r in rb))}")
    assert len(set(r.worker for r in rb)) > 1
    for a, b in zip(ra, rb):
        assert a.rid == b.rid and a.path == b.path
        assert a.compliance == b.compliance, f"request {a.rid}"
        assert np.array_equal(a.u, b.u), f"request {a.rid}"
        assert a.rel_residual <= 1e-8 or a.path == "ca"
    # oracle: one request per path present (plus the first request)
    from paper_2205_00385_amd import serve

    check = {0}
    for p in ("mgcg", "ca", "fallback"):
        for r in ra:
            if r.path == p:
                check.add(r.rid)
                break
    for rid in sorted(check):
        req = trace[rid]
        prob = serve.family_problem(req)
        us, Cs, _ = sens.analyse(prob, np.asarray(req["rho"]).ravel())
        n3 = 3 * prob.n_node
        r = ra[rid]
        for l in range(req["n_case"]):
            assert abs(r.compliance[l] - Cs[l]) <= 1e-6 * abs(Cs[l]), f"request {rid} ({r.path})"
            if r.path != "ca":
                assert rel(r.u[l * n3:(l + 1) * n3], soa(us[l])) <= 1e-6
        log(f"  request {rid} {r.path}: C={r.compliance[0]:.10g} ref={Cs[0]:.10g}")
    alone.close()
    mix.close()


def test_serve_tight_budget_evicts_and_stays_within_tolerance():
    trace = _trace()
    ref = _server(n_workers=1).run(trace, realtime=False)
    probe = _server(n_workers=1)
    biggest = max(probe.workspace_bytes(r) for r in trace)
    tight = _server(n_workers=3, hbm_budget=int(1.5 * biggest))
    rt = tight.run(trace, realtime=False)
    log(f"  evictions {tight.evictions}, budget {1.5 * biggest / 2**20:.0f} MiB")
    assert tight.evictions > 0
    for a, b in zip(ref, rt):
        for ca, cb in zip(a.compliance, b.compliance):
            assert abs(ca - cb) <= 1e-6 * abs(ca)
    tight.close()
