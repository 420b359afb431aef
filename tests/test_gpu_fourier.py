"""The GPU path's semi-discrete symbol against the printed modified
wavenumbers (Sec. 3.2, eqs. wavenumber-6th and wavenumber-8th), in 1-D and
along either axis of the 2-D path (x faces and y faces).

For an entropy wave (density varies, U = 1 and p uniform) with the linear
reconstruction, the left and right states equal the equilibrium state, the
non-equilibrium terms cancel and tau = 0 (Euler), so the mass flux through
a face is U times the reconstructed density there.  The density then obeys
d(rho_i)/dt = -(U/dx)(rho_{i+1/2} - rho_{i-1/2}), whose Fourier symbol for a
mode of scaled wavenumber w = k dx is -i U w'(w)/dx, w' being the printed
modified wavenumber.  One MSMD step with a tiny fixed dt measures the symbol
from the GPU's cell averages: its imaginary part is -w'/dx up to rounding,
its real part is the time-stepping term of order dt |w'/dx|^2.  The same
measurement on the oracle agrees to 1e-10 (imaginary part); replacing w' by
w would be off by up to 22 % at the modes used.
"""
import math

import numpy as np
import pytest

from paper_1901_00261_amd import workloads as wl

pytestmark = pytest.mark.gpu


def modified_wavenumber(order, w):
    """Sec. 3.2, the closed forms for the 6th- and 8th-order compact schemes."""
    if order == 6:
        return (298 * math.sin(w) + math.sin(2 * w) - 114 * w * math.cos(w) + 3 * w * math.cos(2 * w) + 111 * w) / 300
    return (160 * math.sin(w) + 25 * math.sin(2 * w) - 96 * w * math.cos(w) - 6 * w * math.cos(2 * w) + 102 * w) / 210


@pytest.mark.parametrize("order", [6, 8])
def test_symbol_matches_printed_modified_wavenumber(order):
    from paper_1901_00261_amd import gks as g
    n, dt = 32, 1e-7
    dx = 2.0 / n
    for m in (2, 5, 8, 12, 15):  # w = 2 pi m / n from 0.39 to 2.95
        k = math.pi * m          # m periods on [0, 2]
        p = wl.sine_wave_1d(n, order=order, recon=0, dt_fixed=dt, t_end=dt, amp=0.1, k=k)
        S = g.Solver([p], 0)
        S.step(1)
        W1, _, _, t, nsteps = S.state(0)
        S.close()
        assert nsteps == 1 and t == dt
        rho0, rho1 = p.W[:, 0], W1[:, 0]
        ratio = np.fft.fft((rho1 - rho0) / dt)[m] / np.fft.fft(rho0 - rho0.mean())[m]
        lam = modified_wavenumber(order, k * dx) / dx
        print(f"order {order} w={k * dx:.3f}: symbol {ratio:.10g}, -i w'/dx = {-lam:.10g}i")
        assert abs(ratio.imag + lam) <= 1e-7 * lam, (m, ratio, lam)
        assert abs(ratio.real) <= lam * lam * dt, (m, ratio, lam)


@pytest.mark.parametrize("order", [6, 8])
@pytest.mark.parametrize("axis", [0, 1])
def test_symbol_2d_axis_waves(order, axis):
    """A wave along x (U = 1) runs through the x-face kernels only, one along
    y (V = 1) through the y-face kernels; uniform across the other axis, so
    the tangential reconstruction returns the row values and the symbol is
    the 1-D one."""
    from paper_1901_00261_amd import gks as g
    n, dt = 32, 1e-7
    d = 2.0 / n
    for m in (2, 8, 15):
        k = math.pi * m
        p = wl.axis_wave_2d(n, axis, order=order, k=k, dt_fixed=dt)
        S = g.Solver(p, 0)
        S.step(1)
        W1, _, _, t, nsteps = S.state(0)
        S.close()
        assert nsteps == 1 and t == dt
        D = (W1[..., 0] - p.W[..., 0]) / dt
        ref = D[0:1, :] if axis == 0 else D[:, 0:1]
        assert np.abs(D - ref).max() <= 1e-9 * np.abs(D).max()  # uniform across the wave
        line0 = p.W[0, :, 0] if axis == 0 else p.W[:, 0, 0]
        line = D[0, :] if axis == 0 else D[:, 0]
        ratio = np.fft.fft(line)[m] / np.fft.fft(line0 - line0.mean())[m]
        lam = modified_wavenumber(order, k * d) / d
        print(f"2-D axis {axis} order {order} w={k * d:.3f}: symbol {ratio:.10g}, -i w'/dx = {-lam:.10g}i")
        assert abs(ratio.imag + lam) <= 1e-7 * lam, (m, ratio, lam)
        assert abs(ratio.real) <= lam * lam * dt, (m, ratio, lam)
