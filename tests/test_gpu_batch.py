"""Batched, graph-replayed solves: every instance of a batch must equal the
same problem solved alone (same kernels: bitwise) and the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import pstd as opstd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2403_04053_amd as mod
    return mod


def small_instances():
    out = []
    specs = [((24, 24, 24), 0.0, 0.0, 8, 0.5), ((32, 24, 40), 0.9, 2.0, 7, -0.4),
             ((48, 40, 32), 2.2, 4.0, 10, 0.3), ((24, 32, 24), 1.4, 0.6, 6, 0.6),
             ((40, 40, 40), 0.4, 5.1, 9, 0.2)]
    for n, th, ph, ppw, v0 in specs:
        prob, V = synth.tiny(n=n, P=4, transition=3, theta=th, phi=ph, k_ppw=ppw, v0=v0, radius_cells=3,
                             steps=60, dft=(30, 60))
        prob = prob.replace(ramp_periods=0.5)
        out.append((prob, V.astype(np.float32).astype(np.float64)))
    return out


def test_graph_replay_equals_plain_launches(P):
    prob, V = synth.tiny(n=(24, 20, 32), P=3, transition=2, v0=0.5, radius_cells=3, steps=40, dft=(10, 40))
    a = P.Solver(prob)
    b = P.Solver(prob)
    for s in (a, b):
        s.set_potential(V)
    a.run(40)              # graph replays of 16 steps + 8 plain steps
    b.run_timed(40)        # plain launches with events
    assert np.array_equal(a.psi(0).cpu().numpy(), b.psi(0).cpu().numpy())
    assert np.array_equal(a.psi(1).cpu().numpy(), b.psi(1).cpu().numpy())
    assert np.array_equal(a.phasors().cpu().numpy(), b.phasors().cpu().numpy())


def test_batch_instances_equal_single_solves(P):
    inst = small_instances()
    batch = P.Batch([p for p, _ in inst])
    for i, (_, V) in enumerate(inst):
        batch.set_potential(i, V)
    steps = [60, 45, 60, 17, 33]
    batch.run(steps)
    for i, (prob, V) in enumerate(inst):
        view = batch.instance(i)
        assert view.step == steps[i]
        alone = P.Solver(prob)
        alone.set_potential(V)
        alone.run(steps[i])
        assert np.array_equal(view.psi(0).cpu().numpy(), alone.psi(0).cpu().numpy()), i
        _, _, ref, sd = opstd.run(prob.replace(n_steps=steps[i]), V)
        got = view.psi(0).cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-4, i
        if steps[i] > prob.dft_begin:
            gphi, gdphi = view.split_phasors(view.phasors().cpu().numpy())
            ophi, odphi = sd.normalized()
            for f in range(6):
                assert np.linalg.norm(gphi[f] - ophi[f]) <= 1e-4 * np.linalg.norm(ophi[f])
    # continue the batch: counters and tables carry over
    batch.run([5, 0, 3, 20, 1])
    assert [batch.instance(i).step for i in range(5)] == [65, 45, 63, 37, 34]


def test_batch_autotune_keeps_results(P):
    inst = small_instances()[:3]
    a = P.Batch([p for p, _ in inst])
    b = P.Batch([p for p, _ in inst])
    for bb in (a, b):
        for i, (_, V) in enumerate(inst):
            bb.set_potential(i, V)
    a.autotune(reps=2)
    a.run(30)
    b.run(30)
    for i in range(3):
        x = a.instance(i).psi(0).cpu().numpy()
        y = b.instance(i).psi(0).cpu().numpy()
        assert np.linalg.norm(x - y) <= 1e-6 * np.linalg.norm(y)


def _sampled_check(prob, V, got, prev, cur, step, seed):
    m = opstd.build(prob, V)
    rng = np.random.default_rng(seed)
    nx, ny, nz = prob.n
    pts = [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(24)]
    ref = opstd.step_at(m, prev.astype(np.complex128), cur.astype(np.complex128), step, pts)
    g = np.array([got[k, j, i_] for (i_, j, k) in pts])
    return np.abs(g - ref).max() / np.abs(cur).max()


@pytest.mark.parametrize("mode", ["single", "single_tuned", "batch_of_one"])
def test_uneven_instance_alone(P, mode):
    prob, V = synth.uneven_batch(count=1)[0]
    Vf = V.astype(np.float32).astype(np.float64)
    prev = synth.random_state(prob.n, 100).astype(np.complex64)
    cur = synth.random_state(prob.n, 200).astype(np.complex64)
    if mode == "batch_of_one":
        b = P.Batch([prob])
        b.set_potential(0, Vf)
        b.instance(0).set_state(prev, cur, 11)
        b.run([1])
        got = b.instance(0).psi(0).cpu().numpy()
    else:
        s = P.Solver(prob)
        s.set_potential(Vf)
        if mode == "single_tuned":
            print("tiles", s.autotune(reps=2))
        s.set_state(prev, cur, 11)
        s.run(1)
        got = s.psi(0).cpu().numpy()
    err = _sampled_check(prob, Vf, got, prev, cur, 11, 5)
    print(mode, prob.n, "sampled err", err)
    assert err < 1e-5


def test_uneven_batch_full_size_sampled(P):
    """The uneven-grid workload at its real size (64 instances, grid lengths
    96..192): three instances start from random states; one batched step is
    checked on sampled cells against the oracle."""
    inst = synth.uneven_batch()
    batch = P.Batch([p for p, _ in inst])
    for i, (_, V) in enumerate(inst):
        batch.set_potential(i, V.astype(np.float32))
    batch.autotune(reps=2)
    chosen = [0, 17, 63]
    states = {}
    for i in chosen:
        prob = inst[i][0]
        prev = synth.random_state(prob.n, 100 + i).astype(np.complex64)
        cur = synth.random_state(prob.n, 200 + i).astype(np.complex64)
        batch.instance(i).set_state(prev, cur, 11)
        states[i] = (prev, cur)
    batch.run([1 if i in chosen else 0 for i in range(len(inst))])
    rng = np.random.default_rng(3)
    for i in chosen:
        prob, V = inst[i]
        Vf = V.astype(np.float32).astype(np.float64)
        got = batch.instance(i).psi(0).cpu().numpy()
        m = opstd.build(prob, Vf)
        prev, cur = states[i]
        nx, ny, nz = prob.n
        pts = [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(24)]
        ref = opstd.step_at(m, prev.astype(np.complex128), cur.astype(np.complex128), 11, pts)
        g = np.array([got[k, j, i_] for (i_, j, k) in pts])
        err = np.abs(g - ref).max() / np.abs(cur).max()
        print("batch instance", i, prob.n, "sampled err", err)
        assert err < 1e-5


def test_non_temporal_z_pass_changes_no_bits(P):
    """A batch whose largest instance outgrows the Infinity Cache runs every
    z pass with non-temporal loads (a cache hint only); its small instance
    must equal the same problem solved alone, which runs without the hint,
    bit for bit, and its large instance the large problem solved alone."""
    big, Vb = synth.square_barrier_160(n_fft=256)
    big = big.replace(n_steps=12, dft_begin=4, dft_end=12)
    small, Vs = synth.tiny(n=(24, 20, 32), P=3, transition=2, v0=0.5, radius_cells=3, steps=12, dft=(4, 12))
    Vb, Vs = Vb.astype(np.float32), Vs.astype(np.float32)
    batch = P.Batch([big, small])
    batch.set_potential(0, Vb)
    batch.set_potential(1, Vs)
    batch.run([12, 12])
    for i, (prob, V) in enumerate(((big, Vb), (small, Vs))):
        alone = P.Solver(prob)
        alone.set_potential(V)
        alone.run(12)
        view = batch.instance(i)
        print(f"instance {prob.n}: batch vs alone", flush=True)
        assert np.array_equal(view.psi(0).cpu().numpy(), alone.psi(0).cpu().numpy()), i
        assert np.array_equal(view.psi(1).cpu().numpy(), alone.psi(1).cpu().numpy()), i
        assert np.array_equal(view.phasors().cpu().numpy(), alone.phasors().cpu().numpy()), i
        alone.close()
    batch.close()
