"""Checkpoint / resume of a solve (pstd_save_state, pstd_load_state): a
resumed run is bit-identical to the uninterrupted one, wave function and
surface phasors alike."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2403_04053_amd as mod
    return mod


def make(P, prob, V):
    s = P.Solver(prob)
    s.set_potential(V)
    return s


def test_resume_is_bit_identical(P):
    prob, V = synth.tiny(n=(24, 20, 32), P=3, transition=2, v0=0.5, radius_cells=3, steps=200,
                         theta=0.4, phi=1.0, dft=(60, 200))
    print(f"state resume: grid {prob.n}", flush=True)
    a = make(P, prob, V)
    a.run(110)
    buf = a.save_state()
    assert buf.numel() == P.pstd_state_size(a.handle)
    a.run(90)
    b = make(P, prob, V)
    b.load_state(buf)
    assert b.step == 110
    b.run(90)
    assert b.step == a.step == 200
    assert torch.equal(a.psi(0), b.psi(0))
    assert torch.equal(a.psi(1), b.psi(1))
    assert torch.equal(a.phasors(), b.phasors())
    # loading into the saved solver itself rewinds it
    a.load_state(buf)
    a.run(90)
    assert torch.equal(a.psi(0), b.psi(0))
    a.close()
    b.close()


def test_state_errors(P):
    prob, V = synth.tiny(n=(24, 24, 24), steps=20)
    s = make(P, prob, V)
    buf = s.save_state()
    with pytest.raises(P.PstdError) as e:
        P.pstd_load_state(s.handle, buf, buf.numel() - 1)
    assert e.value.name == "PSTD_EINVAL"
    with pytest.raises(P.PstdError) as e:
        s.load_state(torch.zeros_like(buf))
    assert e.value.name == "PSTD_EINVAL"
    prob2, V2 = synth.tiny(n=(24, 24, 32), steps=20)
    s2 = make(P, prob2, V2)
    big = s2.save_state()
    with pytest.raises(P.PstdError) as e:
        s.load_state(big)
    assert e.value.name == "PSTD_EINVAL"
    with pytest.raises(P.PstdError) as e:
        P.pstd_save_state(s.handle, buf, buf.numel() - 1)
    assert e.value.name == "PSTD_EINVAL"
    s.close()
    s2.close()
