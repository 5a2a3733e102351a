"""Pins of the oracle's forcing from Fourier modes (orc_forcing; the
driven-turbulence workload's acceleration, sum_m a_m cos(2 pi k_m . x/L +
phi_m) at the cell centres).

The pin is the discrete Fourier transform (numpy's FFT, an independent
library routine): on a periodic grid a cosine mode is two exponentials, so
the transform of the evaluated field has, in the bin of wavevector k, the
sum of (a/2) e^{i(phi + pi s)} over the modes with wavevector k and of
(a/2) e^{-i(phi + pi s)} over those with -k, where s = k_x/n_x + k_y/n_y +
k_z/n_z is the half-cell shift of the cell centres, and nothing anywhere
else.  A swapped axis, a wrong sign of the phase, a missing 2 pi, a cell
corner in place of the centre or a wrong period each move power to another
bin or change the phase.  A window of the grid with its offset evaluates
the same field."""
import numpy as np

from oracle import orc


def _modes(rng, n):
    ks = [(a, b, c) for a in range(-2, 3) for b in range(-2, 3) for c in range(-2, 3)
          if 1 <= a * a + b * b + c * c <= 4]
    idx = rng.choice(len(ks), n, replace=False)
    out = []
    for i in idx:
        k = np.array(ks[i], dtype=float)
        a = rng.normal(size=3)
        a -= k * (k @ a) / (k @ k)
        out.append([*k, *a, rng.uniform(0, 2 * np.pi)])
    return np.array(out)


def test_spectrum_of_the_forcing_is_the_modes():
    rng = np.random.default_rng(17)
    nx, ny, nz = 12, 10, 8
    L = (2.0, 1.5, 0.75)
    p = dict(nx=nx, ny=ny, nz=nz, hi=L)
    modes = _modes(rng, 20)
    f = orc.Oracle(p).forcing_field(modes, (0.0, 0.0, 0.0), L)
    want = np.zeros((3, nz, ny, nx), dtype=complex)
    for m in modes:
        k = m[:3].astype(int)
        s = k[0] / nx + k[1] / ny + k[2] / nz
        for c in range(3):
            e = 0.5 * m[3 + c] * np.exp(1j * (m[6] + np.pi * s))
            want[c][k[2] % nz, k[1] % ny, k[0] % nx] += e
            want[c][(-k[2]) % nz, (-k[1]) % ny, (-k[0]) % nx] += np.conj(e)
    for c in range(3):
        got = np.fft.fftn(f[c]) / f[c].size
        np.testing.assert_allclose(got, want[c], atol=1e-13)


def test_window_evaluates_the_same_field():
    rng = np.random.default_rng(18)
    modes = _modes(rng, 12)
    full = orc.Oracle(dict(nx=16, ny=16, nz=16)).forcing_field(modes, (0, 0, 0), (1, 1, 1))
    # a window of 6 x 5 x 4 cells at cells (11, 3, 13), wrapping in x and z
    d = 1.0 / 16
    win = orc.Oracle(dict(nx=6, ny=5, nz=4, hi=(6 * d, 5 * d, 4 * d))).forcing_field(
        modes, (11 * d, 3 * d, 13 * d), (1, 1, 1))
    ii, jj, kk = (11 + np.arange(6)) % 16, 3 + np.arange(5), (13 + np.arange(4)) % 16
    np.testing.assert_allclose(win, full[:, kk][:, :, jj][:, :, :, ii], atol=1e-13)
