"""The paper's own Section-4 run at its scale on one GPU (next row F4): the
central square potential of radius 4 pi at 20 points per wavelength on a
288^3 grid, against the exact partial-wave solution in the far field, at
r_bar = 2e4 and in the Fresnel region at r_bar = 100 (x-y and y-z planes,
incidence along y)."""
import math

import numpy as np
import pytest

import synth
from oracle import partial_waves as pw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G = np.deg2rad(np.arange(0, 181, 2.0))
DIRS = np.concatenate([np.stack([np.sin(G), np.cos(G), 0 * G], -1), np.stack([0 * G, np.cos(G), np.sin(G)], -1)])
GAM = np.concatenate([G, G])


def _rel(a, b):
    w = np.sin(GAM) + 1e-2
    return math.sqrt(np.sum(w * np.abs(a - b) ** 2) / np.sum(w * np.abs(b) ** 2))


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2403_04053_amd as mod
    return mod


@pytest.mark.parametrize("s,steps", [(0.5, 36000), (-1.0, 60000)])
def test_paper_scale_square_potential(P, s, steps):
    prob, V = synth.x3_square_potential(s, n_steps=steps)
    k, a, E0 = prob.k0, 4 * math.pi / prob.k0, prob.k0 ** 2 / 2
    print(f"paper-scale square potential s={s}: grid {prob.n}, {steps} steps", flush=True)
    sol = P.Solver(prob)
    sol.set_potential(V)
    sol.run(steps)
    err = {"far": _rel(sol.far_field(DIRS).cpu().numpy(), pw.amplitude(k, a, s * E0, GAM))}
    for rb in (2e4, 100.0):
        r = rb / k
        err[rb] = _rel(sol.project(DIRS * r).cpu().numpy(), pw.scattered_wave(k, a, s * E0, r, GAM))
    print("  rel-L2 vs partial waves", err, flush=True)
    sol.close()
    assert max(err.values()) < 0.01
