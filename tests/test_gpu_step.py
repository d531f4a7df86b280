"""GPU parity of the PSTD step and the surface DFT against the FP64 oracle,
through the C-ABI library.

Tolerances: one FP32 step differs from FP64 by the FP32 rounding of the FFT
passes (about log2(N) * 6e-8 of the largest term, the kinetic term being at
most 2 eta dtau kbar_max^2 ~ 1.8 |psi|): 1e-5 of max|psi| is used.  Many
steps: the rel-L2 bar of 1e-4 that the FP32 path must meet."""
import math

import numpy as np
import pytest

import synth
from oracle import pstd as opstd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2403_04053_amd as mod
    return mod


def c64(a):
    return np.asarray(a).astype(np.complex64)


def f32(a):
    return np.asarray(a).astype(np.float32).astype(np.float64)


CASES = {
    "cube24": dict(n=(24, 24, 24), P=4, transition=3),
    "aniso": dict(n=(24, 20, 32), P=3, transition=2, theta=0.7, phi=2.1),
    "ragged": dict(n=(48, 40, 32), P=4, transition=4, theta=2.3, phi=4.4),
    # the taper's core covers 40 % of the x rows: the z pass takes the
    # potential term (the other cases: the x pass, V's box being small)
    "widebox": dict(n=(24, 20, 32), P=2, transition=1, theta=1.1, phi=0.3),
}


def make(case, **kw):
    args = dict(CASES[case])
    args.update(kw)
    return synth.tiny(**args)


@pytest.mark.parametrize("case", list(CASES))
def test_single_step_matches_oracle(P, case):
    prob, V = make(case, v0=0.4, radius_cells=3)
    prob = prob.replace(ramp_periods=0.5, dft_begin=0, dft_end=0)
    V = f32(V)
    s = P.Solver(prob)
    s.set_potential(V)
    prev = c64(synth.random_state(prob.n, 11))
    cur = c64(synth.random_state(prob.n, 12))
    n = 37
    s.set_state(prev, cur, n)
    s.run(1)
    got = s.psi(0).cpu().numpy()
    m = opstd.build(prob, V)
    ref = opstd.step(m, prev.astype(np.complex128), cur.astype(np.complex128), n)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(case, "single-step max rel err", err)
    assert err < 1e-5
    # the previous level is the old psi^n
    assert np.array_equal(s.psi(1).cpu().numpy(), cur)
    assert s.step == n + 1


@pytest.mark.parametrize("case", ["cube24", "ragged"])
def test_many_steps_from_rest(P, case):
    prob, V = make(case, v0=0.5, radius_cells=3, steps=300)
    prob = prob.replace(ramp_periods=1.0, dft_begin=200, dft_end=300)
    V = f32(V)
    s = P.Solver(prob)
    s.set_potential(V)
    s.run(prob.n_steps)
    got = s.psi(0).cpu().numpy()
    model, prev, cur, sd = opstd.run(prob, V)
    rel = np.linalg.norm(got - cur) / np.linalg.norm(cur)
    print(case, "psi rel-L2 after", prob.n_steps, "steps:", rel)
    assert rel < 1e-4
    # surface phasors
    flat = s.phasors().cpu().numpy()
    gphi, gdphi = s.split_phasors(flat)
    ophi, odphi = sd.normalized()
    for f in range(6):
        r1 = np.linalg.norm(gphi[f] - ophi[f]) / np.linalg.norm(ophi[f])
        r2 = np.linalg.norm(gdphi[f] - odphi[f]) / np.linalg.norm(odphi[f])
        assert r1 < 1e-4 and r2 < 1e-4, (f, r1, r2)


def test_eta_on_source_flag(P):
    prob, V = make("cube24", v0=0.0, radius_cells=0, steps=60)
    prob = prob.replace(ramp_periods=0.2, eta_on_source=True, dft_begin=0, dft_end=0)
    s = P.Solver(prob)
    s.run(prob.n_steps)
    _, _, cur, _ = opstd.run(prob, V)
    got = s.psi(0).cpu().numpy()
    assert np.linalg.norm(got - cur) / np.linalg.norm(cur) < 1e-4


@pytest.mark.parametrize("n", [(160, 160, 160), (100, 96, 108), (288, 288, 288)])
def test_full_size_single_step_sampled(P, n):
    """At the benchmark size and at the largest compiled length on every
    axis (each in every tile shape the autotuner may pick), one GPU step
    against the oracle evaluated on the three pencils through each sampled
    cell (plus the plane phasors there)."""
    if n[0] in (160, 288):
        prob, V = synth.square_barrier_160(n_fft=n[0])
    else:
        prob, V = synth.tiny(n=n, P=16, transition=4, v0=0.5, radius_cells=10)
    prob = prob.replace(ramp_periods=0.5, dft_begin=0, dft_end=10 ** 9)
    V = f32(V)
    s = P.Solver(prob)
    s.set_potential(V)
    prev = c64(synth.random_state(prob.n, 21))
    cur = c64(synth.random_state(prob.n, 22))
    step = 25
    s.set_state(prev, cur, step)
    s.run(1)
    got = s.psi(0).cpu().numpy()
    m = opstd.build(prob, V)
    rng = np.random.default_rng(5)
    nx, ny, nz = prob.n
    pts = [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(48)]
    pts += [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx // 2, ny // 2, nz // 2)]
    tf = prob.tfsf
    pts += [(tf[0][0] + 1, ny // 2, nz // 2), (nx // 2, tf[1][3] - 1, nz // 2), (nx // 2, ny // 2, tf[2][0] + 2)]
    ref = opstd.step_at(m, prev.astype(np.complex128), cur.astype(np.complex128), step, pts)
    scale = np.abs(cur).max()

    def sampled_err(psi):
        g = np.array([psi[k, j, i] for (i, j, k) in pts])
        return np.abs(g - ref).max() / scale

    err = sampled_err(got)
    print(n, "sampled single-step max err / max|psi|", err, flush=True)
    assert err < 1e-5
    # surface DFT of psi^step: psi on the planes and the spectral normal derivative
    flat = s.phasors().cpu().numpy()
    gphi, gdphi = s.split_phasors(flat)
    R = opstd.ramp(step * m.dtau, m.tau_r)
    w = np.exp(1j * step * m.dtau) / R   # one window step: phasor = w psi / R(tau)
    psi = cur.astype(np.complex128)
    for f in range(6):
        a, side = opstd.FACES[f]
        idx = prob.surf_lo[a] if side == 0 else prob.surf_hi[a]
        for t in range(8):
            u, v = int(rng.integers(gphi[f].shape[1])), int(rng.integers(gphi[f].shape[0]))
            # plane point (v, u) -> 3D pencil along a
            if a == 0:
                pen = psi[v, u, :]
            elif a == 1:
                pen = psi[v, :, u]
            else:
                pen = psi[:, v, u]
            from oracle import fft as offt
            d = offt.ifft(1j * m.kb[a] * offt.fft(pen))[idx]
            assert abs(gphi[f][v, u] - w * pen[idx]) <= 1e-6 * scale / R
            assert abs(gdphi[f][v, u] - w * d) <= 2e-5 * scale * np.abs(m.kb[a]).max() / R
    if n[0] in (160, 288):
        # every compiled tile shape (the autotuner may pick any), on all three axes
        for (n1, n2, pencils, m1) in P.pstd_tile_variants(n[0]):
            for ax in range(3):
                s.set_tile(ax, n1, pencils, m1)
            s.set_state(prev, cur, step)
            s.run(1)
            e = sampled_err(s.psi(0).cpu().numpy())
            print(n, "tile", (n1, n2, pencils, m1), "sampled max err", e, flush=True)
            assert e < 1e-5


def test_potential_validation(P):
    prob, V = make("cube24", v0=0.5, radius_cells=3)
    s = P.Solver(prob)
    bad = V.copy()
    bad[0, 0, 0] = 1.0
    with pytest.raises(P.PstdError) as e:
        s.set_potential(bad)
    assert e.value.name == "PSTD_EINVAL"
    bad = V.copy()
    bad[12, 12, 12] = np.nan
    with pytest.raises(P.PstdError) as e:
        s.set_potential(bad)
    assert e.value.name == "PSTD_ENONFINITE"
    with pytest.raises(P.PstdError) as e:
        s.set_potential(V * 3)
    assert e.value.name == "PSTD_EUNSTABLE"
    with pytest.raises(P.PstdError) as e:
        s.phasors()
    assert e.value.name == "PSTD_ESTATE"


def test_rerun_is_bitwise_deterministic(P):
    prob, V = make("ragged", v0=0.5, radius_cells=3, steps=50)
    prob = prob.replace(dft_begin=10, dft_end=50)
    outs = []
    for _ in range(2):
        s = P.Solver(prob)
        s.set_potential(f32(V))
        s.run(prob.n_steps)
        outs.append((s.psi(0).cpu().numpy(), s.phasors().cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_check_state_norm_and_blow_up(P):
    """pstd_check_state: the FP64 norm of psi^n against the oracle's, and
    ENONFINITE once a run forced above the stability bound of Eq.
    PSTDstability has blown up (forced from the host: dt = 1.2 dt_crit)."""
    prob, V = synth.tiny(n=(24, 24, 24), steps=40)
    s = P.Solver(prob)
    s.set_potential(V)
    s.run(40)
    got = s.check_state()
    _, _, ref, _ = opstd.run(prob, V)
    assert got == pytest.approx(float(np.sum(np.abs(ref) ** 2)), rel=1e-5)
    s.close()
    dt = 1.2 * opstd.critical_dt(prob, prob.v_max)
    bad = P.Solver(prob.replace(dt=dt, force_dt=True))
    bad.set_potential(V)
    bad.set_state(synth.random_state(prob.n, 1).astype(np.complex64),
                  synth.random_state(prob.n, 2).astype(np.complex64), 0)
    norms = []
    for _ in range(40):
        bad.run(50)
        try:
            norms.append(bad.check_state())
        except P.PstdError as e:
            assert e.name == "PSTD_ENONFINITE"
            break
    else:
        pytest.fail(f"no blow-up detected, norms {norms[-3:]}")
    assert len(norms) == 0 or norms[-1] > 1e6 * norms[0]
    bad.close()
