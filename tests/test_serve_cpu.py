"""Failure handling of the serving loop, on the CPU (no kernel runs): a
request whose workspace can never fit the HBM budget stops every worker and
is raised by run(), which must neither hang nor return partial results."""

import contextlib

import pytest
import torch

from paper_2205_00385_amd import serve


@pytest.mark.timeout(60)
def test_request_above_budget_is_raised_not_hung(monkeypatch):
    # the scheduler fails before any device work; stand-ins for the stream calls
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(torch.cuda, "Stream", lambda *a, **k: None)
    monkeypatch.setattr(torch.cuda, "stream", lambda s: contextlib.nullcontext())
    srv = serve.AnalysisServer(hbm_budget=1 << 20, n_workers=3)
    req = dict(rid=0, family=0, grid=(32, 16, 16), n_case=1, rho=None, arrival=0.0)
    assert srv.workspace_bytes(req) > 1 << 20
    with pytest.raises(RuntimeError, match="budget"):
        srv.run([req, dict(req, rid=1, family=1)], realtime=False)
