"""GPU parity of pulsed incidence (Section 2.2.3, calculation of the incident
wave; Section 3.3 with several frequencies) against the FP64 oracle
`oracle/pulse.py`, through the C ABI, and the far field of one pulsed run
at several wavenumbers against the partial-wave series."""
import math

import numpy as np
import pytest

import synth
from oracle import ntdf as ontdf
from oracle import partial_waves as pw
from oracle import pstd as opstd
from oracle import pulse as opulse
from oracle import sphere as osph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KB = [0.9, 1.0, 1.1]


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2403_04053_amd as mod
    return mod


def small_problem(steps=300):
    """64^3 (a power of two keeps the oracle's FFTs fast) at 8 points per
    wavelength, taper box 26..38 around a barrier of radius 2 cells, a
    sphere of radius 1.9 (19 cells) whose interpolation shell lies where the
    taper is zero; oblique incidence; the packet's centre starts 12 before
    the corner of the taper box and reaches it at the last step."""
    h = 0.1
    k0 = 2 * math.pi / (8 * h)
    E0 = k0 * k0 / 2
    alpha = 1.0
    n = 64
    prob = synth.Problem(n=(n,) * 3, h=(h,) * 3, k0=k0, theta=0.7, phi=0.9, abc_cells=(4,) * 3,
                         abc_alpha=alpha, abc_U0=synth.paper_u0(alpha, k0 * h, 4), tfsf=((26, 29, 35, 38),) * 3,
                         v_max=E0, n_steps=steps, dft_begin=0, dft_end=steps, surf_lo=(20,) * 3, surf_hi=(44,) * 3,
                         surface_kind=1, sphere_radius=1.9, sphere_nodes=(16, 32))
    V = np.zeros((n,) * 3)
    x = np.arange(n) - n // 2
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    V[X * X + Y * Y + Z * Z <= 4] = E0
    delta = k0 * h
    psi0 = synth.gaussian_pulse_1d(256, delta, 1.0, 4.0, -12.0)
    return prob, V.astype(np.float32).astype(np.float64), psi0, delta


@pytest.fixture(scope="module")
def small(P):
    prob, V, psi0, delta = small_problem()
    print(f"pulse parity: grid {prob.n}, {prob.n_steps} steps", flush=True)
    s = P.Solver(prob)
    s.set_potential(V)
    s.set_pulse(psi0, delta, KB)
    s.run(prob.n_steps)
    sph = osph.Sphere(prob, prob.sphere_radius, n_theta=16, n_phi=32)
    pm, _, ref, sd = opulse.run(prob, V, psi0, delta, sphere=sph, kbars=KB)
    return prob, s, sph, pm, ref, sd


def test_pulse_run_matches_oracle(P, small):
    prob, s, _, _, ref, _ = small
    got = s.psi(0).cpu().numpy()
    rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"  psi rel-L2 {rel:.2e}, max|psi| {np.abs(ref).max():.3f}", flush=True)
    assert np.abs(ref).max() > 0.1
    assert rel < 1e-4


def test_pulse_phasors_match_oracle(P, small):
    prob, s, sph, _, _, sd = small
    for ik in range(len(KB)):
        v, d = (x.cpu().numpy() for x in s.sphere_phasors(ik))
        rv, rd = sph.node_values(sd.normalized(ik))
        ev = np.linalg.norm(v - rv) / np.linalg.norm(rv)
        ed = np.linalg.norm(d - rd) / np.linalg.norm(rd)
        print(f"  k = {KB[ik]}: phasors rel-L2 psi {ev:.2e}, d psi/dn {ed:.2e}", flush=True)
        assert ev < 1e-4 and ed < 1e-4
        dirs = np.random.default_rng(ik).normal(size=(20, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        gf = s.far_field(dirs, ik=ik).cpu().numpy()
        rf = sph.far_field(v, d, dirs, k=KB[ik])
        assert np.abs(gf - rf).max() <= 1e-10 * np.abs(rf).max()


@pytest.mark.parametrize("theta,phi,eta_src", [(2.3, 4.0, 0), (1.2, 5.5, 0), (0.7, 0.9, 1)])
def test_pulse_other_octants_match_oracle(P, theta, phi, eta_src):
    """Incidence from two more octants (the origin corner of Eq. Oinc and
    the axis coordinate change with the signs of k_hat), and the source
    scaled by eta: 150 steps, psi against the oracle."""
    prob, V, psi0, delta = small_problem(steps=150)
    prob = prob.replace(theta=theta, phi=phi, dft_end=0, eta_on_source=eta_src)
    print(f"pulse, theta {theta} phi {phi} eta on source {eta_src}: grid {prob.n}, {prob.n_steps} steps", flush=True)
    s = P.Solver(prob)
    s.set_potential(V)
    s.set_pulse(psi0, delta, KB)
    s.run(prob.n_steps)
    got = s.psi(0).cpu().numpy()
    s.close()
    _, _, ref, _ = opulse.run(prob, V, psi0, delta)
    rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"  psi rel-L2 {rel:.2e}, max|psi| {np.abs(ref).max():.3f}", flush=True)
    assert np.abs(ref).max() > 0.01
    assert rel < 1e-4


def test_pulse_split_runs_are_bit_identical(P):
    prob, V, psi0, delta = small_problem(steps=60)
    out = []
    for split in ((60,), (16, 7, 17, 20), (1, 33, 26)):
        s = P.Solver(prob)
        s.set_potential(V)
        s.set_pulse(psi0, delta, KB)
        for k in split:
            s.run(k)
        out.append((s.psi(0).cpu().numpy(), s.sphere_phasors(1)[0].cpu().numpy()))
        s.close()
    for a, b in out[1:]:
        assert np.array_equal(a, out[0][0]) and np.array_equal(b, out[0][1])


def test_pulse_resumed_from_a_state_is_bit_identical(P):
    """A pulsed run restarted from its own state at step 37 (pstd_set_state
    primes the packet's table of that step) continues bit for bit."""
    prob, V, psi0, delta = small_problem(steps=60)
    prob = prob.replace(dft_end=0)
    a = P.Solver(prob)
    a.set_potential(V)
    a.set_pulse(psi0, delta, KB)
    a.run(37)
    prev, cur = a.psi(1).clone(), a.psi(0).clone()
    a.run(23)
    want = a.psi(0).cpu().numpy()
    a.close()
    b = P.Solver(prob)
    b.set_potential(V)
    b.set_pulse(psi0, delta, KB)
    b.set_state(prev, cur, 37)
    b.run(23)
    got = b.psi(0).cpu().numpy()
    b.close()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("surface_kind", [1, 0])
def test_pulse_checkpoint_resumes_bit_for_bit(P, surface_kind):
    """pstd_save_state at step 150 of a 300-step pulsed run (in the middle of
    a launch group and of the DFT window), loaded into a fresh solver given
    the same pulse and into the saved solver after it has run on: both end
    with the field, the phasors and the far field of every wavenumber of the
    uninterrupted run, bit for bit (sphere and box surfaces)."""
    prob, V, psi0, delta = small_problem()
    prob = prob.replace(surface_kind=surface_kind)
    dirs = np.array([[0.0, 0.0, 1.0], [0.6, 0.0, 0.8], [0.0, -1.0, 0.0]])

    def outputs(s):
        out = [s.psi(0).cpu().numpy(), s.psi(1).cpu().numpy()]
        for ik in range(len(KB)):
            if surface_kind == 1:
                out += [x.cpu().numpy() for x in s.sphere_phasors(ik)]
            else:
                out.append(s.phasors(ik).cpu().numpy())
            out.append(s.far_field(dirs, ik=ik).cpu().numpy())
        return out

    a = P.Solver(prob)
    a.set_potential(V)
    a.set_pulse(psi0, delta, KB)
    a.run(100)
    a.run(50)
    buf = a.save_state()
    a.run(150)
    want = outputs(a)
    a.load_state(buf)
    a.run(150)
    again = outputs(a)
    a.close()
    b = P.Solver(prob)
    b.set_potential(V)
    b.set_pulse(psi0, delta, KB)
    b.load_state(buf)
    b.run(150)
    got = outputs(b)
    b.close()
    for i, (x, y, z) in enumerate(zip(want, again, got)):
        assert np.array_equal(x, y), i
        assert np.array_equal(x, z), i


def test_pulse_validation(P):
    prob, V, psi0, delta = small_problem(steps=20)
    s = P.Solver(prob)
    s.set_potential(V)
    for kw, name in ((dict(psi0=psi0[:200]), "PSTD_EINVAL"), (dict(delta=-1.0), "PSTD_EINVAL"),
                     (dict(kbars=[]), "PSTD_EINVAL"), (dict(kbars=[0.0]), "PSTD_EINVAL"),
                     (dict(kbars=[40.0]), "PSTD_EINVAL"), (dict(psi0=np.zeros(256)), "PSTD_EINVAL")):
        args = dict(psi0=psi0, delta=delta, kbars=KB)
        args.update(kw)
        with pytest.raises(P.PstdError) as e:
            s.set_pulse(args["psi0"], args["delta"], args["kbars"])
        assert e.value.name == name, kw
    s.set_pulse(psi0, delta, KB)
    with pytest.raises(P.PstdError) as e:
        s.far_field(np.array([[0.0, 0.0, 1.0]]), ik=3)
    assert e.value.name == "PSTD_ESTATE"          # no window step yet
    s.run(4)
    with pytest.raises(P.PstdError) as e:
        s.far_field(np.array([[0.0, 0.0, 1.0]]), ik=3)
    assert e.value.name == "PSTD_EINVAL"
    with pytest.raises(P.PstdError) as e:
        s.set_pulse(psi0, delta, KB)
    assert e.value.name == "PSTD_ESTATE"
    buf = s.save_state()
    s.close()
    # a pulsed run's state does not load into a solver without the pulse,
    # nor into one given another number of wavenumbers
    for kbars in (None, KB[:2]):
        s = P.Solver(prob)
        s.set_potential(V)
        if kbars is not None:
            s.set_pulse(psi0, delta, kbars)
        with pytest.raises(P.PstdError) as e:
            s.load_state(buf)
        assert e.value.name == "PSTD_EINVAL", kbars
        s.close()
    for bad, name in ((dict(scheme=1), "PSTD_EUNSUPPORTED"),
                      (dict(sphere_radius=1.2), "PSTD_EINVAL")):  # 1.2: the shell reaches the taper
        s = P.Solver(prob.replace(**bad))
        with pytest.raises(P.PstdError) as e:
            s.set_pulse(psi0, delta, KB)
        assert e.value.name == name, bad
        s.close()
    # the box surface takes a pulse (its faces lie outside the taper box by
    # construction), and the misfit then refuses the solver
    s = P.Solver(prob.replace(surface_kind=0))
    s.set_pulse(psi0, delta, KB)
    with pytest.raises(P.PstdError) as e:
        s.misfit(prob.n_steps, np.array([[0.0, 0.0, 3.0]]), np.ones(1))
    assert e.value.name == "PSTD_EUNSUPPORTED"
    s.close()


def test_pulse_far_field_at_five_wavenumbers(P):
    """One pulsed run of the 160^3 square-barrier grid (sphere of radius 5.6
    outside the taper box) gives the far field at k = 0.8 ... 1.2 k0; each
    against the partial-wave series of the barrier at that wavenumber, and
    k = 1 against the monochromatic run.  The run lasts tau = 160, long
    enough for the slowest of these components (group velocity 2k) to pass
    the sphere (at tau = 110, k = 0.8 was 8.9 % off, at 160 4.7 %, at 220
    4.1 %)."""
    base, V = synth.square_barrier_160(transition=4)   # shell outside the taper box
    sph = dict(surface_kind=1, sphere_radius=5.6, sphere_nodes=(64, 128))
    dtau = opstd.dtau_of(base)
    steps = int(round(160.0 / dtau))
    prob = base.replace(n_steps=steps, dft_begin=0, dft_end=steps, **sph)
    delta = base.k0 * base.h[0]
    psi0 = synth.gaussian_pulse_1d(512, delta, 1.0, 6.0, -30.0)
    kb = [0.8, 0.9, 1.0, 1.1, 1.2]
    print(f"pulsed square barrier: grid {prob.n}, {steps} steps", flush=True)
    s = P.Solver(prob)
    s.set_potential(V)
    s.set_pulse(psi0, delta, kb)
    s.run(steps)
    th = np.deg2rad(np.arange(0, 181, 3.0))
    ph = np.deg2rad(np.arange(0, 360, 30.0))
    T, F = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(T) * np.cos(F), np.sin(T) * np.sin(F), np.cos(T)], -1).reshape(-1, 3)
    w = np.sin(T) + 1e-3

    def rel(a, b):
        return math.sqrt(np.sum(w * np.abs(a - b) ** 2) / np.sum(w * np.abs(b) ** 2))
    errs = []
    for ik, k in enumerate(kb):
        f = s.far_field(d, ik=ik).cpu().numpy().reshape(T.shape)
        ref = pw.amplitude(k * base.k0, 2.4, 0.5 * base.k0 ** 2 / 2, th)[:, None] * np.ones_like(F)
        errs.append(rel(f, ref))
        if k == 1.0:
            f1 = f
    s.close()
    cw = P.Solver(base.replace(**sph))
    cw.set_potential(V)
    cw.run(base.n_steps)
    fc = cw.far_field(d).cpu().numpy().reshape(T.shape)
    cw.close()
    r1 = rel(f1, fc)
    print("  vs partial waves: " + ", ".join(f"k={k}: {e:.4f}" for k, e in zip(kb, errs))
          + f"; k = 1 vs the monochromatic run {r1:.4f}", flush=True)
    assert max(errs) < 0.07
    assert errs[2] < 0.035 and r1 < 0.02


def test_pulse_box_phasors_and_projection_match_oracle(P):
    """The same pulsed run on the box surface (planes 20 and 44, outside the
    taper box): plane phasors and normal derivatives at three wavenumbers
    against the oracle, then the far field and Fresnel points of each
    wavenumber against the oracle's projection at that wavenumber on the
    same phasors (the library rescales the units by k)."""
    prob, V, psi0, delta = small_problem()
    prob = prob.replace(surface_kind=0)
    print(f"pulse on the box: grid {prob.n}, {prob.n_steps} steps", flush=True)
    s = P.Solver(prob)
    s.set_potential(V)
    s.set_pulse(psi0, delta, KB)
    s.run(prob.n_steps)
    _, _, _, sd = opulse.run(prob, V, psi0, delta, kbars=KB, box=True)
    box = ontdf.Box(prob.n, opstd.dxbar(prob), prob.surf_lo, prob.surf_hi)
    rng = np.random.default_rng(8)
    dirs = rng.normal(size=(16, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pts = np.array([[0.3, -0.2, 3.5], [-3.0, 0.4, 0.2], [1.0, 3.2, -0.6]])
    for ik, k in enumerate(KB):
        gp, gd = s.split_phasors(s.phasors(ik).cpu().numpy())
        rp, rd = sd.normalized(ik)
        ep = math.sqrt(sum(np.linalg.norm(gp[f] - rp[f]) ** 2 for f in range(6)) / sum(np.linalg.norm(x) ** 2 for x in rp))
        ed = math.sqrt(sum(np.linalg.norm(gd[f] - rd[f]) ** 2 for f in range(6)) / sum(np.linalg.norm(x) ** 2 for x in rd))
        gf = s.far_field(dirs, ik=ik).cpu().numpy()
        rf = ontdf.far_field(box, gp, gd, dirs, k=k) / prob.k0
        gq = s.project(pts, ik=ik).cpu().numpy()
        rq = ontdf.TaylorTables(box, gp, gd, order=8).project(pts * prob.k0, k=k)
        print(f"  k = {k}: plane phasors rel-L2 {ep:.2e}, derivatives {ed:.2e}; far field "
              f"{np.abs(gf - rf).max() / np.abs(rf).max():.1e}, points {np.abs(gq - rq).max() / np.abs(rq).max():.1e}",
              flush=True)
        assert ep < 1e-4 and ed < 1e-4
        assert np.abs(gf - rf).max() <= 1e-10 * np.abs(rf).max()
        assert np.abs(gq - rq).max() <= 1e-8 * np.abs(rq).max()
    s.close()


def test_pulse_box_far_field_at_five_wavenumbers(P):
    """The pulsed 160^3 run on the box planes 40 and 120: the far field at k
    = 0.8 ... 1.2 k0 against the partial-wave series."""
    base, V = synth.square_barrier_160()
    dtau = opstd.dtau_of(base)
    steps = int(round(160.0 / dtau))
    prob = base.replace(n_steps=steps, dft_begin=0, dft_end=steps)
    delta = base.k0 * base.h[0]
    psi0 = synth.gaussian_pulse_1d(512, delta, 1.0, 6.0, -30.0)
    kb = [0.8, 0.9, 1.0, 1.1, 1.2]
    print(f"pulsed square barrier on the box: grid {prob.n}, {steps} steps", flush=True)
    s = P.Solver(prob)
    s.set_potential(V)
    s.set_pulse(psi0, delta, kb)
    s.run(steps)
    th = np.deg2rad(np.arange(0, 181, 3.0))
    ph = np.deg2rad(np.arange(0, 360, 30.0))
    T, F = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(T) * np.cos(F), np.sin(T) * np.sin(F), np.cos(T)], -1).reshape(-1, 3)
    w = np.sin(T) + 1e-3

    def rel(a, b):
        return math.sqrt(np.sum(w * np.abs(a - b) ** 2) / np.sum(w * np.abs(b) ** 2))
    errs = []
    for ik, k in enumerate(kb):
        f = s.far_field(d, ik=ik).cpu().numpy().reshape(T.shape)
        ref = pw.amplitude(k * base.k0, 2.4, 0.5 * base.k0 ** 2 / 2, th)[:, None] * np.ones_like(F)
        errs.append(rel(f, ref))
    s.close()
    print("  vs partial waves: " + ", ".join(f"k={k}: {e:.4f}" for k, e in zip(kb, errs)), flush=True)
    assert max(errs) < 0.08
