"""Pins for oracle.taper: the closed-form KB pairs against numerical transforms."""
import numpy as np
from scipy import integrate, special

from oracle import taper

J, BETA = 4, 9.36


def _hankel_of_blob(r):
    # 2 pi int_0^{J/2} k(q) J0(2 pi r q) q dq by adaptive quadrature
    f = lambda q: taper.kb_blob(np.array([q]), J, BETA)[0] * special.j0(2 * np.pi * r * q) * q
    val, _ = integrate.quad(f, 0.0, J / 2, epsabs=1e-14, epsrel=1e-13, limit=400)
    return 2 * np.pi * val


def test_blob_ft_matches_numerical_hankel_transform():
    # covers the I1 branch, the z = 0 transition (r ~ 0.745) and the J1 branch
    for r in [0.0, 0.1, 0.25, 0.5, 0.7, 0.744, 0.745, 0.746, 0.8, 1.0, 1.7]:
        ref = _hankel_of_blob(r)
        got = taper.kb_blob_ft(np.array([r]), J, BETA)[0]
        assert abs(got - ref) <= 1e-10 * max(1.0, abs(ref)), (r, got, ref)


def test_blob_ft_other_support():
    for Jx, beta in [(6, 2.34 * 6), (8, 2.34 * 8)]:
        for r in [0.0, 0.3, 0.6]:
            f = lambda q: taper.kb_blob(np.array([q]), Jx, beta)[0] * special.j0(2 * np.pi * r * q) * q
            ref = 2 * np.pi * integrate.quad(f, 0.0, Jx / 2, epsabs=1e-14, epsrel=1e-13, limit=400)[0]
            got = taper.kb_blob_ft(np.array([r]), Jx, beta)[0]
            assert abs(got - ref) <= 1e-10 * max(1.0, abs(ref))


def test_blob_edges():
    q = np.array([0.0, 1.0, 1.999999, 2.0, 2.5])
    k = taper.kb_blob(q, J, BETA)
    assert k[0] == 1.0
    assert k[3] == 0.0 and k[4] == 0.0
    assert abs(k[2] - 1.0 / special.i0(BETA)) < 1e-4


def test_1d_pair_matches_numerical_fourier_transform():
    for r in [0.0, 0.2, 0.5, 0.744, 0.9, 1.3]:
        f = lambda x: taper.kb_1d(np.array([x]), J, BETA)[0] * np.cos(2 * np.pi * r * x)
        ref = integrate.quad(f, -J / 2, J / 2, epsabs=1e-14, epsrel=1e-13, limit=400)[0]
        got = taper.kb_1d_ft(np.array([r]), J, BETA)[0]
        assert abs(got - ref) <= 1e-10 * max(1.0, abs(ref)), (r, got, ref)
