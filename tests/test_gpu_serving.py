"""Continuous-batching server: every request's result equals the same
instance solved alone, whatever else is in flight."""
import pytest

from paper_2305_18575_amd import serving

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("budget,qps", [(64 << 30, 2000.0), (256 << 20, 300.0)])
def test_served_results_equal_alone(rei, budget, qps):
    specs = serving.request_mix(7, 60)
    print(f"\nserving {len(specs)} requests, budget {budget}, qps {qps}", flush=True)
    hs = serving.stage(rei, specs)
    alone = [h.solve() for h in hs]
    arrivals = serving.poisson_arrivals(7, len(hs), qps)
    res, lat, ips = serving.run_served(rei, hs, arrivals, budget)
    for k, (a, b) in enumerate(zip(res, alone)):
        assert serving.same(a, b), (k, specs[k][0], a, b)
    assert all(l > 0 for l in lat)
    for h in hs:
        h.close()
