"""Pins for oracle.wkernel (Eq. (6)): closed forms, invariants and brute force."""
import math

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy import integrate, special

from oracle import taper, wkernel

GEOM25 = wkernel.Geometry(n=1024, fov=math.radians(25.0))
GEOM10 = wkernel.Geometry(n=64, fov=math.radians(10.0))


@pytest.mark.parametrize("w", [0.5, 20.0, 150.0, 500.0])
def test_flat_taper_centre_tap_closed_form(w):
    # g = 1, q = 0: 2 pi int_0^R e^{-2 pi i w (n-1)} r dr = 2 pi du^2 int_{n_R}^1 e^{-ik(n-1)} n dn
    g = GEOM25
    R = g.r_max
    n_R = math.sqrt(1.0 - (R / g.du) ** 2)
    k = 2 * math.pi * w
    prim = lambda n: np.exp(-1j * k * n) * (1j * n / k + 1.0 / k ** 2)
    ref = 2 * math.pi * g.du ** 2 * np.exp(1j * k) * (prim(1.0) - prim(n_R))
    got = wkernel.radial_transform(np.array([0.0]), lambda r: wkernel.chirp(r, w, g), R,
                                   wkernel.chirp_half_cycle_radii(w, g))[0]
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (got, ref)


@pytest.mark.parametrize("q", [0.0, 0.3, 5.5, 77.2, 150.0])
def test_flat_taper_w0_closed_form(q):
    R = 1.0
    ref = math.pi * R * R if q == 0 else R * special.j1(2 * math.pi * q * R) / q
    got = wkernel.radial_transform(np.array([q]), lambda r: np.ones_like(r), R)[0]
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("wp", [0.0, 30.0, 200.0])
def test_gaussian_taper_paraxial_chirp_closed_form(wp):
    # 2 pi int_0^inf e^{-c r^2} J0(2 pi q r) r dr = (pi / c) e^{-pi^2 q^2 / c},  c = a - i pi w'
    a = 8.0
    c = a - 1j * math.pi * wp
    R = 6.0 / math.sqrt(a)
    h = lambda r: np.exp(-c * r * r)
    bps = np.sqrt(np.arange(1, int(wp * R * R) + 1) / wp) if wp > 0 else ()
    q = np.array([0.0, 1.3, 4.7, 12.0])
    got = wkernel.radial_transform(q, h, R, bps)
    ref = (math.pi / c) * np.exp(-math.pi ** 2 * q ** 2 / c)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_w0_kernel_reduces_to_kb_blob():
    q = np.linspace(0.0, 2.8, 57)
    K = wkernel.wkernel(q, 0.0, GEOM25)
    assert np.max(np.abs(K.imag)) == 0.0
    # truncation of Eq. (6) at r = alpha/2 leaves an error set by the blob's
    # edge step 1/I0(beta) ~ 8e-4
    assert np.max(np.abs(K - taper.kb_blob(q, 4, 9.36))) < 2e-3


def _blob_conv_disk(qv, R, J=4, beta=9.36, nt=64, nth=512):
    # brute force: (k * D)(q), D(t) = R J1(2 pi R t) / t = inverse FT of the disk r < R.
    # blob radius a, substitution rho = a sqrt(1 - t^2) makes the radial integrand smooth.
    a = J / 2
    t, wt = leggauss(nt)
    t = 0.5 * (t + 1)
    wt = 0.5 * wt
    rho = a * np.sqrt(1 - t * t)
    th = np.arange(nth) * 2 * np.pi / nth
    sx = rho[:, None] * np.cos(th)[None, :]
    sy = rho[:, None] * np.sin(th)[None, :]
    d = np.hypot(qv - sx, sy)
    D = np.where(d > 0, R * special.j1(2 * np.pi * R * d) / np.where(d > 0, d, 1), np.pi * R * R)
    inner = D.mean(axis=1) * 2 * np.pi
    return a * a * np.sum(wt * t * special.i0(beta * t) / special.i0(beta) * inner)


def test_w0_kernel_equals_blob_convolved_with_disk_transform():
    # K(q, 0) = FT^-1[g 1_{r<R}] = k * FT^-1[1_{r<R}] exactly (g is the transform of k)
    for qv in [0.0, 0.7, 1.5, 1.99, 2.4]:
        ref = _blob_conv_disk(qv, GEOM25.r_max)
        got = wkernel.wkernel(np.array([qv]), 0.0, GEOM25)[0]
        assert abs(got - ref) < 1e-10, (qv, got, ref)


@pytest.mark.parametrize("w", [3.0, 77.0, 310.0])
def test_conjugate_in_w(w):
    q = np.array([0.0, 0.9, 4.2, 30.5])
    assert np.max(np.abs(wkernel.wkernel(q, -w, GEOM25) - np.conj(wkernel.wkernel(q, w, GEOM25)))) < 1e-14


@pytest.mark.parametrize("w,q", [(20.0, 1.7), (60.0, 9.3)])
def test_brute_force_2d_fourier_integral(w, q):
    # int_{|r|<R} g(|r|) chirp(|r|) e^{-2 pi i r.s} d^2r, |s| = q, angle integral by trapezoid
    g = GEOM25
    s_ang = 0.37
    sx, sy = q * math.cos(s_ang), q * math.sin(s_ang)
    nth = 512
    th = np.arange(nth) * 2 * np.pi / nth

    def radial(r):
        ang = np.exp(-2j * np.pi * r * (sx * np.cos(th) + sy * np.sin(th))).mean() * 2 * np.pi
        h = taper.kb_blob_ft(np.array([r]), 4, 9.36)[0] * wkernel.chirp(np.array([r]), w, g)[0]
        return h * ang * r

    edges = [0.0] + list(wkernel.chirp_half_cycle_radii(w, g)) + [g.r_max]
    re = im = 0.0
    for a_, b_ in zip(edges[:-1], edges[1:]):
        re += integrate.quad(lambda r: radial(r).real, a_, b_, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
        im += integrate.quad(lambda r: radial(r).imag, a_, b_, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
    got = wkernel.wkernel(np.array([q]), w, g)[0]
    assert abs(got - complex(re, im)) < 1e-11, (got, re, im)


@pytest.mark.parametrize("w", [150.0, 500.0])
def test_panel_refinement_converged(w):
    q = np.array([0.2, 11.0, 45.5, 100.3])
    a = wkernel.wkernel(q, w, GEOM25)
    b = wkernel.wkernel(q, w, GEOM25, refine=2)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_scipy_quad_agrees_at_large_w():
    w, qs = 300.0, [0.0, 2.2, 37.9]
    g = GEOM25
    edges = [0.0] + list(wkernel.chirp_half_cycle_radii(w, g)) + [g.r_max]
    for qv in qs:
        f = lambda r: (2 * np.pi * taper.kb_blob_ft(np.array([r]), 4, 9.36)[0]
                       * wkernel.chirp(np.array([r]), w, g)[0] * special.j0(2 * np.pi * qv * r) * r)
        re = sum(integrate.quad(lambda r: f(r).real, a_, b_, epsabs=1e-15, limit=200)[0]
                 for a_, b_ in zip(edges[:-1], edges[1:]))
        im = sum(integrate.quad(lambda r: f(r).imag, a_, b_, epsabs=1e-15, limit=200)[0]
                 for a_, b_ in zip(edges[:-1], edges[1:]))
        got = wkernel.wkernel(np.array([qv]), w, g)[0]
        assert abs(got - complex(re, im)) < 1e-12


@pytest.mark.parametrize("geom", [GEOM25, GEOM10])
def test_support_rule_is_chirp_bandwidth_at_image_corner(geom):
    # half-width (J_p - J)/2 = ceil(local chirp frequency in cells at the image corner)
    r_c = geom.fov * math.sqrt(0.5) * geom.du
    h = 1e-6
    for w in [0.0, 0.4, 7.0, 150.0, 499.0]:
        ph = np.angle(wkernel.chirp(np.array([r_c + h]), w, geom)[0]
                      / wkernel.chirp(np.array([r_c - h]), w, geom)[0])
        f_local = abs(ph) / (2 * math.pi * 2 * h)
        jp = int(wkernel.support(w, geom))
        assert jp % 2 == 0
        assert (jp - geom.J) // 2 == math.ceil(f_local - 1e-6), (w, jp, f_local)


def test_taps_are_nearest_grid_points():
    rng = np.random.default_rng(1)
    for _ in range(50):
        up, vp = rng.uniform(-300, 300, 2)
        jp = int(rng.choice([4, 6, 10, 32]))
        u0, v0, q = wkernel.tap_geometry(up, vp, jp)
        cand = np.arange(math.floor(up) - 40, math.floor(up) + 40)
        nearest = np.sort(cand[np.argsort(np.abs(cand - up), kind="stable")[:jp]])
        assert np.array_equal(nearest, u0 + np.arange(jp))
        assert abs(q[0, 0] - math.hypot(up - u0, vp - v0)) < 1e-12


def test_horizon_rejected():
    with pytest.raises(ValueError):
        wkernel.Geometry(n=64, fov=0.6)   # alpha^2 fov / 2 = 1.2
