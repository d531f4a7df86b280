"""Pins of the overlapping-subdomain oracle (Section 2.6)."""
import math

import numpy as np
import pytest

import synth
from oracle import pstd, subdomain


def test_halo_weights_eq_weight():
    w = subdomain.halo_weights(8, 3)
    assert w[0] == 0.0
    assert np.allclose(w[1:4], [pstd.xi(0.25), 0.5, pstd.xi(0.75)])
    assert np.allclose(w[1:4], [0.0377934092, 0.5, 0.9622065908])
    assert (w[4:] == 1.0).all()
    with pytest.raises(ValueError):
        subdomain.halo_weights(7, 3)
    loc = subdomain.local_weights(48, 8, 3)
    assert len(loc) == 64 and np.allclose(loc, loc[::-1]) and (loc[8:56] == 1).all()


def gaussian_packet(model, n, centre, sigma, kvec):
    X = [pstd._bcast(pstd.coords(n[a], model.dxb[a]), a) for a in range(3)]
    r2 = sum((X[a] - centre[a]) ** 2 for a in range(3))
    ph = sum(kvec[a] * X[a] for a in range(3))
    g = np.exp(-r2 / (2 * sigma ** 2)) * np.exp(1j * ph)
    # -lap of g e^{ik.r} in closed form
    lap = g * (sum((1j * kvec[a] - (X[a] - centre[a]) / sigma ** 2) ** 2 for a in range(3)) - 3 / sigma ** 2)
    return g * np.ones((n[2], n[1], n[0])), -lap


def test_local_basis_kinetic_matches_closed_form():
    """For a smooth packet spread over several blocks the local-basis kinetic
    term approximates -lap to better than the 8th-order stencil would
    (Section 2.6's claim), and the global one to spectral accuracy."""
    n = (48, 40, 56)
    prob, V = synth.tiny(n=n, P=4, transition=3, v0=0.0, radius_cells=0)
    m = pstd.build(prob, V)
    g, ref = gaussian_packet(m, n, (0.7, -1.1, 0.4), 2.0, (0.6, -0.5, 0.55))
    scale = np.abs(ref).max()
    assert np.abs(pstd.kinetic(m, g) - ref).max() < 1e-9 * scale
    # the paper's halo (15 points, 10 tapered): better than the 8th-order stencil
    paper = subdomain.Blocks(n, (16, 20, 14), 15, 10)
    err = np.abs(subdomain.kinetic(m, paper, g) - ref).max()
    assert err < 1e-4 * scale, err
    # a wrong halo weight is visible
    paper.w[1][12] = 0.9
    assert np.abs(subdomain.kinetic(m, paper, g) - ref).max() > 20 * err
    # an 8-point halo with 3 tapered points: about 1e-2 (measured, not a paper number)
    short = subdomain.Blocks(n, (16, 20, 14), 8, 3)
    assert np.abs(subdomain.kinetic(m, short, g) - ref).max() < 2e-2 * scale


def test_local_basis_derivative_on_plane():
    n = (48, 40, 56)
    prob, V = synth.tiny(n=n, P=4, transition=3, v0=0.0, radius_cells=0)
    m = pstd.build(prob, V)
    kv = (0.6, -0.5, 0.55)
    c = (0.7, -1.1, 0.4)
    s = 3.2
    s = 2.0
    g, _ = gaussian_packet(m, n, c, s, kv)
    blocks = subdomain.Blocks(n, (16, 20, 14), 15, 10)
    X = [pstd.coords(n[a], m.dxb[a]) for a in range(3)]
    for a in range(3):
        idx = n[a] // 2 + 3
        d = subdomain.derivative(m, blocks, g, a, idx)
        ref = pstd.plane(g * (1j * kv[a] - (pstd._bcast(X[a], a) - c[a]) / s ** 2), a, idx)
        assert np.abs(d - ref).max() < 1e-4 * np.abs(ref).max()


def test_single_block_is_the_global_step_when_halo_is_zero_padding():
    """With one block per axis the local array is the global one padded by
    the halo; for a field that vanishes near the global edges the local and
    global kinetic terms agree to spectral accuracy."""
    n = (32, 32, 32)
    prob, V = synth.tiny(n=n, P=4, transition=3, v0=0.0, radius_cells=0)
    m = pstd.build(prob, V)
    g, ref = gaussian_packet(m, n, (0.0, 0.0, 0.0), 2.0, (0.4, 0.3, -0.2))
    blocks = subdomain.Blocks(n, (32, 32, 32), 8, 3)
    assert np.abs(subdomain.kinetic(m, blocks, g) - ref).max() < 1e-6 * np.abs(ref).max()


def test_local_array_gather_brute_force():
    n = (24, 16, 20)
    blocks = subdomain.Blocks(n, (8, 8, 10), 6, 1)
    psi = synth.random_state(n, 3)
    for (bx, by, bz) in [(0, 0, 0), (1, 1, 1), (2, 0, 1)]:
        loc = blocks.local(psi, bx, by, bz)
        for kk in range(blocks.nloc[2]):
            for jj in range(blocks.nloc[1]):
                for ii in range(blocks.nloc[0]):
                    gi, gj, gk = bx * 8 - 6 + ii, by * 8 - 6 + jj, bz * 10 - 6 + kk
                    inside = 0 <= gi < 24 and 0 <= gj < 16 and 0 <= gk < 20
                    w = blocks.w[0][ii] * blocks.w[1][jj] * blocks.w[2][kk]
                    ref = w * psi[gk, gj, gi] if inside else 0.0
                    assert abs(loc[kk, jj, ii] - ref) < 1e-15


def test_pencil_evaluation_matches_block_step():
    n = (32, 24, 40)
    prob, V = synth.tiny(n=n, P=4, transition=3, v0=0.5, radius_cells=3)
    prob = prob.replace(theta=0.5, phi=0.3, ramp_periods=0.5)
    m = pstd.build(prob, V)
    blocks = subdomain.Blocks(n, (16, 12, 20), 8, 3)
    prev = synth.random_state(n, 1)
    cur = synth.random_state(n, 2)
    full = subdomain.step(m, blocks, prev, cur, 9)
    rng = np.random.default_rng(0)
    pts = [(int(rng.integers(32)), int(rng.integers(24)), int(rng.integers(40))) for _ in range(25)]
    got = subdomain.step_at(m, blocks, prev, cur, 9, pts)
    ref = np.array([full[k, j, i] for (i, j, k) in pts])
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
