"""Oracle pins of the boundary conditions of Sec. 4 beyond periodic and
extrapolated ends: prescribed (inflow) states, the split sides of the double
Mach reflection (Sec. 4.5), the characteristic non-reflecting condition, and
the Woodward-Colella blast wave between reflecting walls (Sec. 4.2).  The
paper prints no values for these cases (figures only); the pins are
invariants, limits that reduce to another boundary condition, and
qualitative properties the paper states."""
import math

import numpy as np
import pytest

import oracle
from paper_1901_00261_amd import workloads as wl


def _run(p, **over):
    return oracle.run(p.dim, p.W, p.Wx, p.Wy, **{**p.oracle_kwargs(), **over})


def test_inflow_of_the_flow_state_keeps_a_free_stream():
    """An inflow side whose state equals a uniform flow leaves the flow
    exactly uniform (1-D and 2-D)."""
    W1 = wl.prim_to_cons(np.full(16, 1.3), 0.7, 2.1, 1.4)
    p1 = wl.Problem(1, 16, 1, 0.0, 1.0, 0.0, 1.0, 1.4, 0.0, 0.3, 0.0, 0.2, 8, 1, (3, 1, 0, 0), W1, np.zeros_like(W1))
    p1.bc_state[0, 0] = [W1[0, 0], W1[0, 1], 0.0, W1[0, 2]]
    W2 = wl.prim_to_cons(np.full((8, 10), 1.3), 0.7, 2.1, 1.4, V=-0.4)
    p2 = wl.Problem(2, 10, 8, 0.0, 1.0, 0.0, 1.0, 1.4, 0.0, 0.3, 0.0, 1.0, 8, 1, (3, 1, 1, 3), W2,
                    np.zeros_like(W2), np.zeros_like(W2))
    p2.bc_state[0, 0] = W2[0, 0]
    p2.bc_state[3, 0] = W2[0, 0]
    for p, steps in ((p1, 0), (p2, 3)):
        W, Wx, Wy, t, n = _run(p, max_steps=steps)
        assert np.array_equal(W, p.W) and not Wx.any() and (Wy is None or not Wy.any())


def test_split_side_reduces_to_inflow_and_to_wall():
    """A split side whose switch point lies beyond the whole side is an
    inflow side; one whose switch point lies before it is a reflecting wall
    (bc_beyond = wall) -- the results equal those runs exactly."""
    base = wl.pulse_box_2d(12, ny=10, bc=(2, 2, 2, 2))
    st = wl.prim_to_cons(1.0, 0.1, 1.0, 1.4, V=0.05)
    ref_in = wl.pulse_box_2d(12, ny=10, bc=(2, 2, 3, 2))
    ref_in.bc_state[2, 0] = st
    got_in = wl.pulse_box_2d(12, ny=10, bc=(2, 2, 4, 2))
    got_in.bc_state[2, 0] = st
    got_in.bc_split[2] = (5.0, 0.0)
    got_wall = wl.pulse_box_2d(12, ny=10, bc=(2, 2, 4, 2))
    got_wall.bc_state[2, 0] = st
    got_wall.bc_split[2] = (-5.0, 0.0)
    a = _run(ref_in, max_steps=3)
    b = _run(got_in, max_steps=3)
    c = _run(base, max_steps=3)
    d = _run(got_wall, max_steps=3)
    for k in range(3):
        assert np.array_equal(a[k], b[k]) and np.array_equal(c[k], d[k])
    assert not np.array_equal(a[0], c[0])


def test_characteristic_boundary_removes_the_shu_osher_end_wave():
    """Sec. 4.2 Shu-Osher problem: with extrapolated ends the non-uniform
    density at x = 10 makes a kink whose free-transport flux starts a
    spurious wave (|U| ~ 0.2 near the right end by t = 1.8); the
    characteristic condition extends the entropy wave linearly and keeps
    the right end quiet (|U| < 2e-3)."""
    p = wl.shu_osher_1d(200)
    p.bc = (5, 5, 0, 0)
    W, _, _, t, n = _run(p)
    q = wl.shu_osher_1d(200)
    W2, _, _, t2, n2 = _run(q)
    U, U2 = W[:, 1] / W[:, 0], W2[:, 1] / W2[:, 0]
    assert t == t2 == 1.8
    assert np.abs(U[-10:]).max() < 2e-3 < 0.05 < np.abs(U2[-10:]).max()
    # the interior away from the right end is the same solution
    assert np.abs(W[:150, 0] - W2[:150, 0]).max() < 1e-2


def test_characteristic_boundary_lets_a_pulse_leave():
    """A right-running acoustic pulse leaves through characteristic ends:
    after it has gone, what remains is below 1e-3 of its amplitude (the
    left-running part of the initial data, O(amp^2), and no reflection),
    and free-stream data stay exactly free-stream."""
    amp = 1e-3
    p = wl.acoustic_pulse_1d(100, bc=(5, 5, 0, 0), t_end=0.8, amp=amp)
    W, _, _, t, n = _run(p)
    assert np.abs(W[:, 0] - 1.0).max() < 1e-3 * amp
    U = wl.prim_to_cons(np.full(12, 0.9), -0.3, 0.8, 1.4)
    q = wl.Problem(1, 12, 1, 0.0, 1.0, 0.0, 1.0, 1.4, 0.0, 0.3, 0.0, 0.1, 6, 1, (5, 5, 0, 0), U, np.zeros_like(U))
    W2, Wx2, _, _, _ = _run(q)
    assert np.array_equal(W2, U) and not Wx2.any()


def test_blast_wave_8th_order_conserves_and_stays_physical():
    """Sec. 4.2 Woodward-Colella blast wave, 200 cells, 8th-order WENO-Z,
    reflecting walls, to t = 3.8: mass and energy are conserved to
    round-off between the walls, the state stays physical, and the density
    peak lies between the pre-shock density and the strong-shock limit
    (gamma + 1)/(gamma - 1) = 6.  The positivity fallback of the
    reconstructed states is taken a few dozen times (reported)."""
    p = wl.blast_wave_1d(200)
    W, _, _, t, n = _run(p)
    assert t == 3.8
    for k in (0, 2):
        assert abs(W[:, k].sum() / p.W[:, k].sum() - 1.0) < 1e-13
    rho = W[:, 0]
    pr = 0.4 * (W[:, 2] - 0.5 * W[:, 1] ** 2 / rho)
    assert rho.min() > 0 and pr.min() > 0
    assert 3.0 < rho.max() < 6.0
    print("blast wave 200: steps", n, "fallbacks", oracle.fallbacks())


def test_blast_wave_6th_order_stops_on_its_first_step():
    """With these readings the 6th-order scheme meets a negative pressure in
    the first step of the blast wave (the cell next to the 1e5 pressure
    jump); the oracle reports it (the paper shows this case running)."""
    p = wl.blast_wave_1d(200, order=6)
    with pytest.raises(oracle.OracleError) as e:
        _run(p)
    assert e.value.nsteps <= 1


def test_double_mach_reflection_boundaries():
    """Sec. 4.5 double Mach reflection on 48 x 12 cells, 4 steps: the state
    stays physical; far ahead of the shock (more than the 4 cells per step
    that the stencils reach) the pre-shock gas is untouched, bit for bit;
    the total mass grows by the post-shock inflow through the left side."""
    p = wl.double_mach_2d(48, 12)
    W, Wx, Wy, t, n = _run(p, max_steps=4)
    assert n == 4
    rho = W[..., 0]
    pr = 0.4 * (W[..., 3] - 0.5 * (W[..., 1] ** 2 + W[..., 2] ** 2) / rho)
    assert rho.min() > 0 and pr.min() > 0
    pre = wl.prim_to_cons(*[wl.DMR_PRE[k] for k in (0, 1, 3)], 1.4, V=wl.DMR_PRE[2])
    # the shock crosses y = 1 at x < 1 (column 12) by then
    assert wl.dmr_shock_x(1.0, t) < 1.0
    np.testing.assert_array_equal(W[:, 30:], np.broadcast_to(pre, W[:, 30:].shape))
    assert not Wx[:, 30:].any() and not Wy[:, 30:].any()
    assert rho.sum() > p.W[..., 0].sum()
    print("double Mach 48x12, 4 steps: fallbacks", oracle.fallbacks())


def test_titarev_toro_initial_data():
    """Sec. 4.2 Titarev-Toro initial data: the cell averages carry the
    closed-form mass and momentum of the two regions (the sine wave has an
    integer number of periods over (-4.5, 5], so it adds no mass), the shock
    sits on face 100 of 2000 cells, and the ends are characteristic (left)
    and extrapolated (right)."""
    p = wl.titarev_toro_1d(2000)
    dx = (p.xhi - p.xlo) / p.nx
    rho_l, u_l = 1.515695, 0.523346
    assert abs(p.W[:, 0].sum() * dx - (0.5 * rho_l + 9.5)) < 1e-12
    assert abs(p.W[:, 1].sum() * dx - 0.5 * rho_l * u_l) < 1e-12
    assert np.all(p.W[:100, 0] == p.W[0, 0]) and abs(p.W[0, 0] - rho_l) < 1e-15
    assert np.all(p.W[100:, 1] == 0.0) and tuple(p.bc[:2]) == (5, 1)


def test_shock_velocity_wave_initial_data():
    """Sec. 4.4 initial data: closed-form mass, momentum and energy of the
    two regions (the velocity wave has whole periods over (1, 10], so its
    momentum integrates to zero and its kinetic energy to 0.2^2/4 per unit
    length times the density), the shock on face 40 of 400 cells, and
    characteristic ends."""
    p = wl.shock_velocity_wave_1d(400)
    dx = (p.xhi - p.xlo) / p.nx
    g = p.gamma
    E_l = 116.5 / (g - 1.0) + 0.5 * 8.0 * 8.25 ** 2
    E_r = 9.0 * (1.0 / (g - 1.0) + 0.5 * 1.4 * 0.2 ** 2 / 2.0)
    assert abs(p.W[:, 0].sum() * dx - (8.0 + 9.0 * 1.4)) < 1e-12
    assert abs(p.W[:, 1].sum() * dx - 8.0 * 8.25) < 1e-12
    assert abs(p.W[:, 2].sum() * dx - (E_l + E_r)) < 1e-11
    assert np.abs(p.W[:40, 0] - 8.0).max() < 1e-14 and np.abs(p.W[40:, 0] - 1.4).max() < 1e-14
    assert tuple(p.bc[:2]) == (5, 5)
