"""Pins of the oracle's discrete adjoint: dot-product tests of each linear
map and of the whole chain (tangent-linear vs adjoint), and central finite
differences of the misfit."""
import numpy as np
import pytest

import synth
from oracle import adjoint, ntdf, pstd


@pytest.fixture(scope="module")
def setup():
    prob, V = synth.tiny(n=(20, 20, 24), P=3, transition=3, v0=0.3, radius_cells=3, steps=60, dft=(20, 60))
    prob = prob.replace(ramp_periods=0.5)
    pts = np.array([[0.1, 0.2, 2.0], [-0.3, 0.1, 2.2], [0.4, -0.2, 1.9], [0.0, 0.0, -2.5]])
    target = adjoint.intensity(prob, 0.5 * V, pts)
    return prob, V, pts, target


def test_projection_dot_product(setup):
    prob, V, pts, _ = setup
    model = pstd.build(prob, V)
    box = ntdf.Box(prob.n, model.dxb, prob.surf_lo, prob.surf_hi)
    G = adjoint.Projection(box, pts * prob.k0)
    rng = np.random.default_rng(0)
    shapes = [(24, 20)] * 4 + [(20, 20)] * 2
    x = [rng.normal(size=s) + 1j * rng.normal(size=s) for s in shapes]
    xd = [rng.normal(size=s) + 1j * rng.normal(size=s) for s in shapes]
    y = rng.normal(size=len(pts)) + 1j * rng.normal(size=len(pts))
    lhs = np.vdot(y, G.apply(x, xd))
    hp, hd = G.adjoint(y)
    rhs = sum(np.vdot(hp[f], x[f]) + np.vdot(hd[f], xd[f]) for f in range(6))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the linear map is the projection of Section 3.2 (Taylor form)
    assert np.allclose(G.apply(x, xd), ntdf.TaylorTables(box, x, xd).project(pts * prob.k0), rtol=1e-12)


def test_surface_adjoint_dot_product(setup):
    prob, V, _, _ = setup
    model = pstd.build(prob, V)
    rng = np.random.default_rng(1)
    x = synth.random_state(prob.n, 5)
    shapes = [(24, 20)] * 4 + [(20, 20)] * 2
    hp = [rng.normal(size=s) + 1j * rng.normal(size=s) for s in shapes]
    hd = [rng.normal(size=s) + 1j * rng.normal(size=s) for s in shapes]
    n, inc = 33, 7.5
    e = adjoint.surface_adjoint(model, n, hp, hd, inc)
    sd = pstd.SurfaceDFT(model)
    sd.accumulate(x, n)
    lhs = sum(np.vdot(hp[f], sd.phi[f] / inc) + np.vdot(hd[f], sd.dphi[f] / inc) for f in range(6))
    rhs = np.vdot(e, x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_tangent_linear_equals_adjoint(setup):
    prob, V, pts, target = setup
    J, grad = adjoint.gradient(prob, V, pts, target)
    rng = np.random.default_rng(2)
    dV = np.zeros_like(V)
    c0, c1 = prob.tfsf[0][1], prob.tfsf[0][2]
    dV[c0:c1 + 1, c0:c1 + 1, c0:c1 + 1] = rng.normal(size=(c1 - c0 + 1,) * 3)
    J2, dJ = adjoint.tangent(prob, V, dV, pts, target)
    assert J == pytest.approx(J2, rel=1e-14)
    assert abs(np.sum(grad * dV) - dJ) <= 1e-9 * abs(dJ)


def test_gradient_matches_finite_differences(setup):
    prob, V, pts, target = setup
    J, grad = adjoint.gradient(prob, V, pts, target)
    rng = np.random.default_rng(3)
    c0, c1 = prob.tfsf[0][1], prob.tfsf[0][2]
    for _ in range(3):
        k, j, i = (int(rng.integers(c0, c1 + 1)) for _ in range(3))
        eps = 1e-3 * prob.k0 ** 2 / 2
        Vp = V.copy()
        Vp[k, j, i] += eps
        Vm = V.copy()
        Vm[k, j, i] -= eps
        fd = (adjoint.misfit(prob, Vp, pts, target)[0] - adjoint.misfit(prob, Vm, pts, target)[0]) / (2 * eps)
        assert abs(grad[k, j, i] - fd) <= 1e-4 * max(abs(fd), 1e-3 * np.abs(grad).max())
