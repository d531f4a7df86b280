"""Pins of the complex absorbing potential in the oracle (Section 2.1: the
absorbing potential may be complex as long as its imaginary part, the mask's
rate, stays non-positive).  The real part w(d) = UR / cosh^2(alphaR d) of
every axis's layer enters the step like V."""
import math

import numpy as np
import pytest

import synth
from oracle import pstd


def layered_problem(n, P, UR, U0=0.0, alphaR=0.5, v_max=0.0, dt=0.0):
    h = 0.1
    k0 = 2 * math.pi / (8 * h)
    E0 = k0 * k0 / 2
    mid = [N // 2 for N in n]
    tf = tuple((m - 2, m - 1, m, m + 1) for m in mid)
    p = synth.Problem(n=n, h=(h, h, h), k0=k0, abc_cells=(P,) * 3, abc_U0=U0, abc_alpha=0.5,
                      abc_UR=UR, abc_alphaR=alphaR, tfsf=tf, v_max=v_max * E0, dt=dt)
    return p, E0


def test_zero_real_part_is_the_mask_alone():
    """UR = 0 leaves the model of the mask-only absorber unchanged."""
    prob, V = synth.tiny(n=(24, 20, 16), P=4, v0=0.5, radius_cells=3)
    a = pstd.build(prob, V)
    b = pstd.build(prob.replace(abc_UR=0.0, abc_alphaR=0.7), V)
    assert a.dtau == b.dtau
    assert np.array_equal(a.v, b.v) and np.array_equal(a.Gamma, b.Gamma)


def test_real_part_profile_and_placement():
    """Inside the layers only, summed over axes, UR at the outermost points,
    falling as 1/cosh^2; the user's potential check ignores it."""
    n = (16, 12, 20)
    p, E0 = layered_problem(n, 3, -2.0, U0=1.0, alphaR=0.4)
    m = pstd.build(p, np.zeros((n[2], n[1], n[0])))
    w = m.v
    assert w[0, 0, 0] == pytest.approx(-6.0, rel=1e-15)             # three layers meet
    assert w[10, 6, 0] == pytest.approx(-2.0, rel=1e-15)            # x layer only
    assert w[10, 6, 2] == pytest.approx(-2.0 / math.cosh(0.8) ** 2, rel=1e-15)
    assert w[10, 6, 3] == 0.0 and w[10, 6, 8] == 0.0                # outside the layer
    assert w[10, 11, 15] == pytest.approx(-4.0, rel=1e-15)          # y and x layers (mirror ends)
    assert pstd.check_potential(m)


def test_leapfrog_invariant_with_real_absorbing_part():
    """The real part is Hermitian: with the mask off and no source the
    leapfrog keeps Re<psi^{n+1}, psi^n> exactly (a factor of i on it would
    break this)."""
    n = (12, 10, 16)
    p, E0 = layered_problem(n, 3, -3.0, U0=0.0, alphaR=0.6)
    m = pstd.build(p, np.zeros((n[2], n[1], n[0])))
    assert np.abs(m.v).max() > 2.0
    prev = synth.random_state(n, 3)
    cur = synth.random_state(n, 4)
    q0 = np.vdot(cur, prev).real
    for s in range(400):
        prev, cur = cur, pstd.step(m, prev, cur, s, with_source=False)
    assert abs(np.vdot(cur, prev).real - q0) <= 1e-12 * np.vdot(cur, cur).real


def test_step_bound_counts_the_real_part():
    """A deep well in the layers (|w| larger than the kinetic spectrum) is
    unstable at the bound that ignores it and stable at the oracle's bound,
    which takes max(v_max / E0, |UR| x axes with a layer)."""
    n = (12, 12, 12)
    UR = -25.0
    p, E0 = layered_problem(n, 3, UR, U0=0.0, alphaR=0.3)
    kin = math.pi ** 2 * float(np.sum(1 / pstd.dxbar(p) ** 2))
    assert pstd.dtau_of(p) == pytest.approx(0.9 / (kin + 75.0), rel=1e-15)
    assert 3 * abs(UR) > kin                                 # the well dominates the spectrum
    V0 = np.zeros((12, 12, 12))

    def growth(prob):
        m = pstd.build(prob, V0)
        prev = synth.random_state(n, 5)
        cur = synth.random_state(n, 6)
        nrm0 = np.abs(cur).max()
        for s in range(300):
            prev, cur = cur, pstd.step(m, prev, cur, s, with_source=False)
        return np.abs(cur).max() / nrm0

    assert growth(p) < 10.0
    unsafe = p.replace(dt=0.9 / kin / E0)                    # the bound without the layers' well
    assert growth(unsafe) > 1e6
