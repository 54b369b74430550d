"""Host-side checks of the serving loop (no GPU): a request that can never fit
the budget is refused before anything runs, instead of blocking FIFO admission
for ever."""
import pytest


def test_serve_refuses_request_larger_than_budget():
    from paper_1210_6116_amd.serve import request_bytes, serve
    need = request_bytes(1024)
    assert request_bytes(256) < request_bytes(512) < need
    trace = [dict(arrival=0.0, L=256, sweeps=10, seed=1, beta0=1.0),
             dict(arrival=0.1, L=1024, sweeps=10, seed=2, beta0=1.0)]
    with pytest.raises(ValueError, match="request 1"):
        serve(trace, budget_bytes=need - 1)
