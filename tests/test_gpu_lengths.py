"""Single-step parity for every compiled pass length, on each axis."""
import numpy as np
import pytest

import synth
from oracle import pstd as opstd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LENGTHS = [8, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 100, 108, 120, 128, 144, 150, 160, 162, 180, 192, 256, 288]


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2403_04053_amd as mod
    return mod


def geometry(n):
    # absorber 1 cell, taper 1 cell, box one cell outside the taper box
    tf = tuple((2, 3, N - 4, N - 3) for N in n)
    return synth.Problem(n=n, h=(0.1,) * 3, k0=2 * np.pi / 0.8, theta=0.7, phi=1.9, abc_cells=(1, 1, 1),
                         abc_U0=3.0, abc_alpha=1.0, tfsf=tf, v_max=10.0, ramp_periods=0.5,
                         dft_begin=0, dft_end=100, surf_lo=(1, 1, 1), surf_hi=tuple(N - 2 for N in n))


def variants():
    import paper_2403_04053_amd as mod
    out = []
    for L in LENGTHS:
        for (n1, n2, p, m1) in mod.pstd_tile_variants(L):
            out.append((L, n1, p, m1))
    return out


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("L,n1,pencils,m1", variants())
def test_length_single_step(P, L, n1, pencils, m1, axis):
    n = [12, 12, 12]
    n[axis] = L
    prob = geometry(tuple(n))
    V = np.zeros((n[2], n[1], n[0]))
    c = [N // 2 for N in n]
    V[c[2] - 1:c[2] + 1, c[1] - 1:c[1] + 1, c[0] - 1:c[0] + 1] = 5.0
    s = P.Solver(prob)
    s.set_potential(V)
    s.set_tile(axis, n1, pencils, m1)
    assert s.tiles()[axis] == (L, n1, L // n1, pencils, m1)
    prev = synth.random_state(prob.n, 1).astype(np.complex64)
    cur = synth.random_state(prob.n, 2).astype(np.complex64)
    s.set_state(prev, cur, 7)
    s.run(1)
    got = s.psi(0).cpu().numpy()
    m = opstd.build(prob, V)
    ref = opstd.step(m, prev.astype(np.complex128), cur.astype(np.complex128), 7)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < 1e-5, (L, axis, err)
    flat = s.phasors().cpu().numpy()
    gphi, gdphi = s.split_phasors(flat)
    # the surface DFT of that single step: w psi / R on the planes of this axis
    R = opstd.ramp(7 * m.dtau, m.tau_r)
    w = np.exp(1j * 7 * m.dtau) / R
    d = opstd.derivative(m, cur.astype(np.complex128), axis)
    for side in (0, 1):
        idx = prob.surf_lo[axis] if side == 0 else prob.surf_hi[axis]
        f = 2 * axis + side
        rp = w * opstd.plane(cur.astype(np.complex128), axis, idx)
        rd = w * opstd.plane(d, axis, idx)
        assert np.abs(gphi[f] - rp).max() <= 1e-5 * np.abs(rp).max()
        assert np.abs(gdphi[f] - rd).max() <= 1e-5 * np.abs(rd).max()
