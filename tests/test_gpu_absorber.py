"""GPU parity of the complex absorbing potential (mask plus a real part in
the layers, Section 2.1) against the FP64 oracle, and its effect on the
plain-method workload's far field."""
import math

import numpy as np
import pytest

import synth
from oracle import partial_waves as pw
from oracle import pstd as opstd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2403_04053_amd as mod
    return mod


@pytest.mark.parametrize("UR,alphaR", [(-2.0, 0.4), (1.5, 0.0), (-30.0, 0.3)])
def test_complex_absorber_run_matches_oracle(P, UR, alphaR):
    """200 steps from rest with the incident wave, a barrier and a complex
    absorber (the deepest case sets the step bound through its real part)."""
    prob, V = synth.tiny(n=(24, 24, 32), P=4, transition=2, v0=0.5, radius_cells=3, steps=200,
                         theta=0.6, phi=2.0, dft=(100, 200))
    prob = prob.replace(abc_U0=3.0, abc_alpha=0.35, abc_UR=UR, abc_alphaR=alphaR, ramp_periods=0.5)
    V = V.astype(np.float32).astype(np.float64)
    print(f"complex absorber UR={UR} alphaR={alphaR}: grid {prob.n}", flush=True)
    s = P.Solver(prob)
    s.set_potential(V)
    s.run(prob.n_steps)
    got = s.psi(0).cpu().numpy()
    _, _, ref, _ = opstd.run(prob, V)
    rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print("  psi rel-L2 vs oracle", rel, flush=True)
    assert rel < 1e-4
    s.close()


TH = np.deg2rad(np.arange(0, 181, 5.0))
PH = np.deg2rad(np.arange(0, 360, 30.0))


def _far(P, prob, V):
    T, F = np.meshgrid(TH, PH, indexing="ij")
    d = np.stack([np.sin(T) * np.cos(F), np.sin(T) * np.sin(F), np.cos(T)], -1).reshape(-1, 3)
    s = P.Solver(prob)
    s.set_potential(V)
    s.run(prob.n_steps)
    f = s.far_field(d).cpu().numpy().reshape(T.shape)
    s.close()
    return f


def _rel(a, b):
    w = np.sin(TH)[:, None] + 1e-3
    return math.sqrt(np.sum(w * np.abs(a - b) ** 2) / np.sum(w * np.abs(b) ** 2))


@pytest.mark.parametrize("case", ["plain", "well"])
def test_tuned_absorbers_cut_the_layer_error(P, case):
    """The far field of the 8-cell-layer problem against the same problem
    with a 32-cell layer on 96^3 (the layer's own error): the tuned mask and
    the tuned complex absorber cut it well below the paper-profile default,
    also on an attractive well that was not used for the tuning."""
    prob, V = synth.plain_barrier()
    if case == "well":
        V = -V
    E0 = prob.k0 ** 2 / 2
    print(f"absorber layer error, {case}: grid {prob.n}, reference 96^3", flush=True)
    fref = _far(P, *synth.wide_layer_reference(prob, V))
    err = {name: _rel(_far(P, prob.replace(**kw), V), fref)
           for name, kw in (("default", {}), ("mask", synth.TUNED_MASK_8), ("complex", synth.TUNED_COMPLEX_8))}
    print("  layer error", err, flush=True)
    assert err["mask"] < 0.45 * err["default"]
    assert err["complex"] < 0.45 * err["default"]
    assert err["complex"] < err["mask"]
    if case == "plain":
        # and the far field moves towards the partial-wave series
        ref = pw.amplitude(prob.k0, 0.6, 0.5 * E0, TH)[:, None] * np.ones((1, PH.size))
        d0 = _rel(_far(P, prob, V), ref)
        d1 = _rel(_far(P, prob.replace(**synth.TUNED_COMPLEX_8), V), ref)
        print("  vs partial waves: default", d0, "tuned complex", d1, flush=True)
        assert d1 < d0
