"""The allocation-free state check (pstd_check_state_noalloc) against the
allocating one (pstd_check_state), through the C ABI: the same kernels on
the same data, so the norms agree bit for bit; two calls in a row, the
second on a smaller grid, then a state holding a NaN."""
import math

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2403_04053_amd as mod
    return mod


def c64(a):
    return np.asarray(a).astype(np.complex64)


def host_norm2(t):
    a = t.cpu().numpy().astype(np.complex128)
    return float(np.sum(a.real ** 2 + a.imag ** 2))


def test_noalloc_matches_allocating_check(P):
    sizes = [((96, 80, 64), 3), ((24, 20, 32), 1)]    # second call: a smaller input
    for k, (n, r) in enumerate(sizes):
        print(f"no-alloc state check: grid {n}", flush=True)
        prob, V = synth.tiny(n=n, P=4, transition=3, v0=0.4, radius_cells=r)
        s = P.Solver(prob)
        s.set_potential(V)
        s.set_state(c64(synth.random_state(prob.n, 40 + k)), c64(synth.random_state(prob.n, 50 + k)), 11)
        s.run(7)
        want = P.pstd_check_state(s.handle)
        got = P.pstd_check_state_noalloc(s.handle)
        assert got == want, (n, got, want)
        ref = host_norm2(s.psi(0))
        assert math.isclose(got, ref, rel_tol=1e-12), (got, ref)
        # the array keeps the last call's partial sums; a repeat gives the same bits
        assert P.pstd_check_state_noalloc(s.handle) == want
        s.close()


def test_noalloc_reports_nonfinite_like_the_allocating_check(P):
    prob, V = synth.tiny(n=(24, 24, 24), P=4, transition=3, v0=0.0, radius_cells=0)
    s = P.Solver(prob)
    cur = c64(synth.random_state(prob.n, 3))
    prev = cur.copy()
    prev[5, 6, 7] = np.nan
    s.set_state(prev, cur, 4)
    for fn in (P.pstd_check_state, P.pstd_check_state_noalloc):
        with pytest.raises(P.PstdError) as e:
            fn(s.handle)
        assert e.value.name == "PSTD_ENONFINITE"
    s.set_state(cur, cur, 4)
    assert P.pstd_check_state_noalloc(s.handle) == P.pstd_check_state(s.handle)
    s.close()
