"""Pins of the oracle's wave actuation (Sec. IV-B, Eqs. 3-5: the worm).

The rest length of a spring is L0 (1 + c sin(omega tau)), tau = (T - t_o)
mod t_p taken in [0, t_p), with offsets t_o = (smaller x of the two ends) -
(smallest x of the body).  Each pin checks the oracle against values worked
out by hand here, or against the phasor mode in the special case where the
two must agree."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_10274_amd import scenes


def one_spring(L0=0.1, k=1.0e4, c=0.2, t_o=0.0):
    """Two masses L0 apart along x; the spring at its base length."""
    return dict(pos=np.array([[0.0, 0.0, 1.0], [L0, 0.0, 1.0]], np.float32),
                vel=np.zeros((2, 3), np.float32), mass=np.full(2, 0.1, np.float32),
                ends=np.array([[0, 1]]), k=np.array([k], np.float32), damping=None,
                amp=np.array([c], np.float32), phase=np.array([t_o], np.float64))


# (T, t_o, tau) with tau = (T - t_o) mod 1 worked out by hand
CASES = [
    (0.10, 0.30, 0.80),  # T < t_o: the modulo is taken non-negative
    (1.25, 0.05, 0.20),  # more than one period after the offset
    (0.40, 0.40, 0.00),  # exactly at a period start: no actuation
    (2.70, 0.20, 0.50),
    (0.00, 2.25, 0.75),  # several periods before the offset
]


@pytest.mark.parametrize("T,t_o,tau", CASES)
def test_wave_rest_length_by_hand(T, t_o, tau):
    L0, k, c, omega = 0.1, 1.0e4, 0.2, 20.0
    sc = one_spring(L0, k, c, t_o)
    sys_ = O.System(sc)
    x = O._d(sc["pos"])
    f = sys_.spring_forces(x, np.zeros_like(x), T, omega, wave=True, period=1.0)
    # the ends sit at the base length: f on the first end = k (l - L) u
    # = -k L0 c sin(omega tau) along +x
    want = -k * float(np.float32(L0)) * float(np.float32(c)) * math.sin(omega * tau)
    assert abs(f[0, 0] - want) <= 1e-9 * k * L0
    assert abs(f[1, 0] + want) <= 1e-9 * k * L0
    assert np.all(f[:, 1:] == 0.0)


def test_wave_period_matches_phasor_when_the_period_is_whole_cycles():
    """With omega t_p a whole number of cycles, sin(omega ((T - t_o) mod t_p))
    = sin(omega T + phase) with phase = -omega t_o: both modes must give the
    same trajectory (to rounding)."""
    w = scenes.worm(7, 3, 2)
    period = 0.5
    omega = 2 * math.pi * 3 / period  # three cycles per period
    t_o = O.wave_offsets(w["pos"], w["ends"], w.get("body"))
    wave_sc = dict(w, phase=t_o)
    phas_sc = dict(w, phase=-omega * t_o)
    p_wave = O.Params(dt=1e-3, omega=omega, wave=True, period=period)
    p_phas = O.Params(dt=1e-3, omega=omega)
    xa, va, _ = O.System(wave_sc).run(p_wave, O._d(w["pos"]), O._d(w["vel"]), 0, 400)
    xb, vb, _ = O.System(phas_sc).run(p_phas, O._d(w["pos"]), O._d(w["vel"]), 0, 400)
    moved = np.abs(xa - O._d(w["pos"]).reshape(-1, 3)).max()
    assert moved > 1e-3  # the worm actually moves
    assert np.abs(xa - xb).max() <= 1e-9
    assert np.abs(va - vb).max() <= 1e-7


def test_wave_offsets_eq5_by_hand():
    """t_o = min(x_a, x_b) - x_min of the body, per body."""
    h = 0.25  # exact in binary
    a = scenes.worm(4, 2, 2, spacing=h, origin=(1.0, 0.0, 0.0))
    b = scenes.worm(3, 2, 2, spacing=h, origin=(-2.0, 5.0, 0.0))
    sc = scenes.concat([a, b])
    t_o = O.wave_offsets(sc["pos"], sc["ends"], sc["body"])
    pos = sc["pos"].astype(np.float64)
    for s, (i, j) in enumerate(sc["ends"]):
        # grid column of the lower end, counted from the body's own first column
        x0 = 1.0 if sc["body"][i] == 0 else -2.0
        col = min(round((pos[i, 0] - x0) / h), round((pos[j, 0] - x0) / h))
        assert t_o[s] == col * h
    # body 1 has three columns (offsets 0, h, 2h): its largest offset is 2h
    assert t_o.min() == 0.0 and t_o[sc["body"][sc["ends"][:, 0]] == 1].max() == 2 * h


def test_wave_momentum_conserved_without_gravity_and_ground():
    w = scenes.worm(9, 3, 2)
    t_o = O.wave_offsets(w["pos"], w["ends"], w.get("body"))
    sys_ = O.System(dict(w, phase=t_o))
    p = O.Params(dt=1e-4, gravity=(0.0, 0.0, 0.0), ground=False, omega=20.0, wave=True, period=1.0)
    x, v, _ = sys_.run(p, O._d(w["pos"]), O._d(w["vel"]), 0, 3000)
    P = (sys_.mass[:, None] * v).sum(axis=0)
    assert np.abs(P).max() <= 1e-10
    assert np.abs(v).max() > 1e-3


def test_wave_adjoint_is_refused():
    w = scenes.worm(4, 2, 2)
    sys_ = O.System(dict(w, phase=O.wave_offsets(w["pos"], w["ends"])))
    with pytest.raises(ValueError):
        sys_.rollout_grad(O.Params(omega=20.0, wave=True), 10)
