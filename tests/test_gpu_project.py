"""GPU parity of the NTDF projection (far field and Fresnel points) against
the oracle, on the same phasors (FP64 both: 1e-10) and end to end."""
import math

import numpy as np
import pytest

import synth
from oracle import ntdf as ontdf
from oracle import pstd as opstd
from oracle import partial_waves as pw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2403_04053_amd as mod
    return mod


@pytest.fixture(scope="module")
def run_small(P):
    prob, V = synth.tiny(n=(24, 20, 32), P=3, transition=2, v0=0.5, radius_cells=3, steps=400,
                         theta=0.4, phi=1.0)
    prob = prob.replace(ramp_periods=1.0, dft_begin=200, dft_end=400)
    V = V.astype(np.float32).astype(np.float64)
    s = P.Solver(prob)
    s.set_potential(V)
    s.run(prob.n_steps)
    return prob, V, s


def box_of(prob):
    return ontdf.Box(prob.n, opstd.dxbar(prob), prob.surf_lo, prob.surf_hi)


def test_far_field_same_phasors(P, run_small):
    prob, V, s = run_small
    phi, dphi = s.split_phasors(s.phasors().cpu().numpy())
    rng = np.random.default_rng(0)
    d = rng.normal(size=(300, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d = np.vstack([d, [[0, 0, 1.0], [0, 0, -1.0], [1, 0, 0]]])
    got = s.far_field(d).cpu().numpy()
    ref = ontdf.far_field(box_of(prob), phi, dphi, d) / prob.k0
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
    # the literal cell sums agree as well
    ref2 = ontdf.far_field_direct(box_of(prob), phi, dphi, d[:5]) / prob.k0
    assert np.abs(got[:5] - ref2).max() <= 1e-10 * np.abs(ref).max()


def test_fresnel_points_same_phasors(P, run_small):
    prob, V, s = run_small
    phi, dphi = s.split_phasors(s.phasors().cpu().numpy())
    rng = np.random.default_rng(1)
    pts = rng.normal(size=(40, 3))
    pts = pts / np.linalg.norm(pts, axis=1, keepdims=True) * rng.uniform(1.5, 6.0, size=(40, 1))
    pts = np.vstack([pts, [[0, 0, 3.0], [0.2, -0.1, -2.5]]])
    got = s.project(pts).cpu().numpy()
    box = box_of(prob)
    ref = ontdf.TaylorTables(box, phi, dphi, order=8).project(pts * prob.k0)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
    direct = ontdf.project_direct(box, phi, dphi, pts[:3] * prob.k0)
    assert np.abs(got[:3] - direct).max() <= 1e-8 * np.abs(ref).max()


def test_projection_end_to_end(P, run_small):
    prob, V, s = run_small
    _, _, _, sd = opstd.run(prob, V)
    ophi, odphi = sd.normalized()
    d = np.array([[0, 0, 1.0], [0.6, 0, 0.8], [0, -1, 0], [0.48, 0.6, 0.64]])
    got = s.far_field(d).cpu().numpy()
    ref = ontdf.far_field(box_of(prob), ophi, odphi, d) / prob.k0
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-4


def test_points_inside_box_rejected(P, run_small):
    prob, V, s = run_small
    with pytest.raises(P.PstdError) as e:
        s.project(np.array([[0.0, 0.0, 0.0]]))
    assert e.value.name == "PSTD_EINVAL"


def test_plain_method_against_partial_waves(P):
    """The square barrier of radius 0.6, V0 = E0/2 at 8 points per wavelength
    (FFT grid 48^3): far-field amplitude against the partial-wave series."""
    prob, V = synth.plain_barrier()
    s = P.Solver(prob)
    s.set_potential(V)
    s.run(prob.n_steps)
    th = np.deg2rad(np.arange(0, 181, 5.0))
    ph = np.deg2rad(np.arange(0, 360, 30.0))
    T, F = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(T) * np.cos(F), np.sin(T) * np.sin(F), np.cos(T)], -1).reshape(-1, 3)
    f = s.far_field(d).cpu().numpy().reshape(T.shape)
    ref = pw.amplitude(prob.k0, 0.6, 0.5 * prob.k0 ** 2 / 2, th)[:, None] * np.ones_like(F)
    w = np.sin(T) + 1e-3
    rel = math.sqrt(np.sum(w * np.abs(f - ref) ** 2) / np.sum(w * np.abs(ref) ** 2))
    print("plain method: solid-angle rel-L2 of f vs partial waves", rel)
    print("f(0)", f[0, 0], ref[0, 0], "f(90)", f[18, 0], ref[18, 0], "f(180)", f[-1, 0], ref[-1, 0])
    # measured 3.5 %: TF/SF leakage and absorber reflection of the workload's
    # thin layers plus the discretisation at 8 points per wavelength (the split
    # is tests/test_gpu_accuracy.py's plain-method budget)
    assert rel < 0.04


def test_refined_plain_method_within_one_percent(P):
    """The same barrier at h = 0.05 with a 1.6-wide absorber (FFT grid 128^3,
    26 388 steps): the far-field amplitude converges to the partial-wave
    series, within 1 % (solid-angle weighted rel-L2).  At the 8-points-per-
    wavelength spacing of the plain-method workload the same measure is 3.5 %,
    which is the method's discretisation error at that spacing (the error
    falls by about h^3 once the absorber is wide enough)."""
    prob, V = synth.plain_barrier_refined()
    print(f"refined plain method: grid {prob.n}, {prob.n_steps} steps", flush=True)
    s = P.Solver(prob)
    s.set_potential(V)
    s.run(prob.n_steps)
    th = np.deg2rad(np.arange(0, 181, 5.0))
    ph = np.deg2rad(np.arange(0, 360, 30.0))
    T, F = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(T) * np.cos(F), np.sin(T) * np.sin(F), np.cos(T)], -1).reshape(-1, 3)
    f = s.far_field(d).cpu().numpy().reshape(T.shape)
    ref = pw.amplitude(prob.k0, 0.6, 0.5 * prob.k0 ** 2 / 2, th)[:, None] * np.ones_like(F)
    w = np.sin(T) + 1e-3
    rel = math.sqrt(np.sum(w * np.abs(f - ref) ** 2) / np.sum(w * np.abs(ref) ** 2))
    print("  solid-angle rel-L2 of f vs partial waves", rel, flush=True)
    assert rel < 0.01
    s.close()
