"""cis_iterate_noalloc, the iteration entry point for callers that cannot allocate device memory, against
cis_iterate: the same kernels, so the same residual histories and states, bit for bit, over two calls in a row
(the second on a smaller mesh, a smaller velocity set and fewer iterations, so stale scratch contents of the
first would show), in both precisions."""
import sys

import numpy as np
import pytest

from paper_2303_10846_amd.cases import configs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(case, n, precision, noalloc):
    from paper_2303_10846_amd.binding import Solver
    s = Solver(case, precision=precision)
    s.init_equilibrium(case["W0"])
    hist = s.iterate_noalloc(n) if noalloc else s.iterate(n)
    return hist, s.get_state()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_iterate_matches_iterate_on_two_calls(precision):
    runs = [(configs.cavity_case(n=3, nv_side=6), 100),    # more iterations than cis_iterate's first history buffer
            (configs.cavity_case(n=2, nv_side=4), 7)]      # then a smaller input
    for case, n in runs:
        say(f"case {case['name']} {precision} {n} iterations: cis_iterate vs cis_iterate_noalloc")
        h_ref, st_ref = _run(case, n, precision, noalloc=False)
        h_na, st_na = _run(case, n, precision, noalloc=True)
        assert h_na.shape == (n, 6)
        assert np.array_equal(h_ref, h_na)
        for a, b in zip(st_ref, st_na):
            assert np.array_equal(a, b)
        assert np.all(np.isfinite(h_na)) and h_na[-1].max() < h_na[0].max()


def test_noalloc_iterate_rejects_histories_beyond_its_scratch():
    from paper_2303_10846_amd.binding import CisError, Solver
    c = configs.cavity_case(n=2, nv_side=4)
    s = Solver(c, precision="fp64")
    s.init_equilibrium(c["W0"])
    W0, _ = s.moments()
    with pytest.raises(CisError) as e:
        s.iterate_noalloc(4097)
    assert e.value.status == -1
    W1, _ = s.moments()
    assert np.array_equal(W0, W1)              # rejected before any device work
    assert s.iterate_noalloc(0).shape == (0, 6)
