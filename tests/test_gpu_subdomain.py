"""GPU parity of the overlapping-subdomain mode (Section 2.6) against the
block-by-block FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import pstd as opstd
from oracle import subdomain as osub

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2403_04053_amd as mod
    return mod


def c64(a):
    return np.asarray(a).astype(np.complex64)


def small_problem(steps=80, dft=(40, 80)):
    n = (64, 64, 96)
    prob, V = synth.tiny(n=n, P=6, transition=4, v0=0.5, radius_cells=5, steps=steps, theta=0.6, phi=0.9)
    prob = prob.replace(ramp_periods=0.5, dft_begin=dft[0], dft_end=dft[1],
                        sub_core=(16, 32, 48), sub_halo=8, sub_taper=3)
    V = V.astype(np.float32).astype(np.float64)
    blocks = osub.Blocks(n, prob.sub_core, prob.sub_halo, prob.sub_taper)
    return prob, V, blocks


def test_subdomain_single_step(P):
    prob, V, blocks = small_problem()
    s = P.Solver(prob)
    s.set_potential(V)
    prev = c64(synth.random_state(prob.n, 31))
    cur = c64(synth.random_state(prob.n, 32))
    s.set_state(prev, cur, 13)
    s.run(1)
    got = s.psi(0).cpu().numpy()
    m = opstd.build(prob, V)
    ref = osub.step(m, blocks, prev.astype(np.complex128), cur.astype(np.complex128), 13)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("subdomain single-step max rel err", err)
    assert err < 1e-5


def test_subdomain_run_and_phasors(P):
    prob, V, blocks = small_problem()
    s = P.Solver(prob)
    s.set_potential(V)
    s.run(prob.n_steps)
    got = s.psi(0).cpu().numpy()
    m = opstd.build(prob, V)
    shape = (prob.n[2], prob.n[1], prob.n[0])
    prev = np.zeros(shape, np.complex128)
    cur = np.zeros(shape, np.complex128)
    phi = [None] * 6
    dphi = [None] * 6
    inc = 0.0
    for n in range(prob.n_steps):
        if prob.dft_begin <= n < prob.dft_end:
            w = np.exp(1j * n * m.dtau)
            for f in range(6):
                a, side = opstd.FACES[f]
                idx = prob.surf_lo[a] if side == 0 else prob.surf_hi[a]
                p_ = w * opstd.plane(cur, a, idx)
                d_ = w * osub.derivative(m, blocks, cur, a, idx)
                phi[f] = p_ if phi[f] is None else phi[f] + p_
                dphi[f] = d_ if dphi[f] is None else dphi[f] + d_
            inc += opstd.ramp(n * m.dtau, m.tau_r)
        prev, cur = cur, osub.step(m, blocks, prev, cur, n)
    rel = np.linalg.norm(got - cur) / np.linalg.norm(cur)
    print("subdomain psi rel-L2 after", prob.n_steps, "steps:", rel)
    assert rel < 1e-4
    gphi, gdphi = s.split_phasors(s.phasors().cpu().numpy())
    for f in range(6):
        r1 = np.linalg.norm(gphi[f] - phi[f] / inc) / np.linalg.norm(phi[f] / inc)
        r2 = np.linalg.norm(gdphi[f] - dphi[f] / inc) / np.linalg.norm(dphi[f] / inc)
        assert r1 < 1e-4 and r2 < 1e-4, (f, r1, r2)


def test_subdomain_full_size_sampled(P):
    """The non-central workload at its real size: 288^3 global grid as
    216 subdomains of 64^3 (core 48, halo 8)."""
    prob, V = synth.bumps_288()
    prob = prob.replace(ramp_periods=0.5)
    V = V.astype(np.float32).astype(np.float64)
    s = P.Solver(prob)
    s.set_potential(V)
    prev = c64(synth.random_state(prob.n, 41))
    cur = c64(synth.random_state(prob.n, 42))
    s.set_state(prev, cur, 30)
    s.run(1)
    got = s.psi(0).cpu().numpy()
    m = opstd.build(prob, V)
    blocks = osub.Blocks(prob.n, prob.sub_core, prob.sub_halo, prob.sub_taper)
    rng = np.random.default_rng(7)
    N = prob.n[0]
    pts = [(int(rng.integers(N)), int(rng.integers(N)), int(rng.integers(N))) for _ in range(40)]
    pts += [(47, 48, 95), (48, 47, 96), (0, 287, 144), (143, 144, 145)]
    ref = osub.step_at(m, blocks, prev.astype(np.complex128), cur.astype(np.complex128), 30, pts)
    g = np.array([got[k, j, i] for (i, j, k) in pts])
    err = np.abs(g - ref).max() / np.abs(cur).max()
    print("288^3 subdomain sampled single-step err", err)
    assert err < 1e-5
