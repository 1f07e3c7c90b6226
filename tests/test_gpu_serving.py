"""Serving on the GPU: each request's result is the same alone (one slot,
one solve at a time) and in a mix of concurrent solves (4 slots, all
arriving at once), in FP64 and in the mixed arithmetic; every solve
converges.  The library's kernels are
deterministic, so the solutions agree to rounding (checked at 1e-12 on the
full tensors)."""
import numpy as np
import pytest

from paper_2306_00632_amd import serve
from oracle import tucker as T

from gpu_helpers import say

pytestmark = pytest.mark.gpu


def full(sol):
    core, U = sol
    return T.Tucker(core, U).full()


@pytest.mark.parametrize("arith", ["f64", "mixed"])
def test_same_result_alone_and_in_the_mix(arith):
    reqs = serve.mixed_requests(6, 4242, n_els=(16, 32), ps=(2, 3), Rs=(3, 6), ranks=range(1, 5), arith=arith)
    say(f"serving ({arith}): alone")
    alone_srv = serve.Server(slots=1)
    alone = alone_srv.run(reqs, keep_solutions=True)
    alone_srv.close()
    say("serving: mix")
    mix_srv = serve.Server(slots=4)
    mix = mix_srv.run(serve.poisson_arrivals(reqs, 0.0, 1), keep_solutions=True)
    mix_srv.close()
    for a, m in zip(alone, mix):
        assert a.error is None and m.error is None, (a.error, m.error)
        assert a.converged and m.converged
        assert a.iters == m.iters
        assert a.f32_applications == m.f32_applications
        assert (a.f32_applications > 0) == (arith == "mixed")
        xa, xm = full(a.solution), full(m.solution)
        assert np.linalg.norm(xa - xm) <= 1e-12 * np.linalg.norm(xa), a.rid
    s = serve.summarize(mix)
    say(f"mix: {s['solves_per_s']:.2f} solves/s, p50 {s['latency_ms']['p50']:.1f} ms")
