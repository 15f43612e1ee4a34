"""Pins of the oracle's polarised operator (Eq. (9)), CPU only.

The reference is the direct DFT of Eq. (1) applied to the complex image
P = Q + iU at the original (unfolded) coordinates: by linearity its
visibilities are measure(Q) + i measure(U).  The folded operator of Eq. (9)
must reproduce them to the aliasing level, the Stokes I conjugation rule
must not (its error is 2 |y_U| on every folded visibility), U = 0 must give
the Stokes operator, and the adjoint identity must hold.
"""
import math

import numpy as np

from oracle import dft, operator, polar, wkernel
from paper_1903_06555_amd import synthetic as syn

N, FOV = 32, math.radians(10.0)


def setup():
    geom = wkernel.Geometry(n=N, fov=FOV)
    uvw = syn.uniform_box_uvw(400, u_max=25.0, w_max=15.0, seed=61)
    op = operator.StackedOperator(geom, uvw, n_stacks=2, fold=True)
    q = syn.point_source_sky(N, 6, "gaussian", seed=62, margin=3)
    u = syn.point_source_sky(N, 6, "gaussian", seed=63, margin=3)
    return geom, uvw, op, q, u


def test_matches_direct_dft_of_linear_polarisation():
    geom, uvw, op, q, u = setup()
    assert op.flag.any() and not op.flag.all()
    y_ref = dft.measure(q, uvw, FOV) + 1j * dft.measure(u, uvw, FOV)
    y = polar.forward(op, q, u)
    err = np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)
    assert err <= 1e-2, err
    # the Stokes I rule (conjugating y_P) is off by 2|y_U| on the folded rows
    bad = polar.naive_forward(op, q, u)
    f = op.flag
    err_bad = np.linalg.norm(bad[f] - y_ref[f]) / np.linalg.norm(y_ref[f])
    assert err_bad > 0.3, err_bad
    # on the unfolded rows both rules agree
    assert np.array_equal(bad[~f], y[~f])


def test_no_u_reduces_to_stokes_operator():
    geom, uvw, op, q, u = setup()
    y = polar.forward(op, q, np.zeros_like(u))
    assert np.allclose(y, op.forward(q), rtol=0, atol=1e-13 * np.abs(y).max())


def test_pair_adjoint_identity():
    geom, uvw, op, q, u = setup()
    yr = syn.random_vis(op.m, seed=64)
    lhs = float(np.real(np.vdot(polar.forward(op, q, u), yr)))
    qa, ua = polar.adjoint(op, yr)
    rhs = float(np.sum(q * qa) + np.sum(u * ua))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
