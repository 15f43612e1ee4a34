"""Pins for oracle.dft (Eq. (1)): geometry, FFT route, conjugate symmetry, adjoint."""
import math

import numpy as np

from oracle import dft
from paper_1903_06555_amd import synthetic as syn

FOV = math.radians(10.0)


def test_phase_is_baseline_dot_direction_offset():
    # single pixel source: y = x0 exp(-2 pi i b.(s - s0)) / n with s = (l, m, n)
    n_img = 32
    rng = np.random.default_rng(0)
    uvw = rng.uniform(-50, 50, size=(20, 3))
    for (row, col) in [(16, 16), (3, 29), (30, 1), (0, 0)]:
        x = np.zeros((n_img, n_img))
        x[row, col] = 2.5
        dl = FOV / n_img
        s = np.array([(col - n_img / 2) * dl, (row - n_img / 2) * dl, 0.0])
        s[2] = math.sqrt(1.0 - s[0] ** 2 - s[1] ** 2)
        s0 = np.array([0.0, 0.0, 1.0])
        delay = uvw @ (s - s0)
        ref = 2.5 * np.exp(-2j * np.pi * delay) / s[2]
        got = dft.measure(x, uvw, FOV)
        assert np.max(np.abs(got - ref)) < 1e-12


def test_w0_integer_frequencies_match_numpy_fft():
    n_img = 16
    x = syn.random_image(n_img, seed=3)
    k = np.array([[a, b] for a in range(-3, 4) for b in range(-2, 3)], dtype=np.float64)
    uvw = np.zeros((k.shape[0], 3))
    uvw[:, 0] = k[:, 0] / FOV
    uvw[:, 1] = k[:, 1] / FOV
    got = dft.measure(x, uvw, FOV)
    lcol, mrow = dft.pixel_lm(n_img, FOV)
    L, M = np.meshgrid(lcol, mrow)
    _, n = dft.n_minus_one(L, M)
    F = np.fft.fft2(np.fft.ifftshift(x / n))          # axis 0 = m / v, axis 1 = l / u
    ref = F[k[:, 1].astype(int) % n_img, k[:, 0].astype(int) % n_img]
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))


def test_conjugate_symmetry_eq8():
    n_img = 24
    x = syn.random_image(n_img, seed=4)
    uvw = syn.uniform_box_uvw(50, seed=5)
    y = dft.measure(x, uvw, FOV)
    ym = dft.measure(x, -uvw, FOV)
    assert np.max(np.abs(ym - np.conj(y))) < 1e-12 * np.max(np.abs(y))


def test_adjoint_dot_product():
    n_img = 20
    x = syn.random_image(n_img, seed=6)
    uvw = syn.uniform_box_uvw(80, seed=7)
    wts = syn.random_weights(80, seed=8)
    y = syn.random_vis(80, seed=9)
    lhs = np.real(np.vdot(dft.measure(x, uvw, FOV, wts), y))
    rhs = np.sum(x * dft.measure_adjoint(y, uvw, n_img, FOV, wts))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
