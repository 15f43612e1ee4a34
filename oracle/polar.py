"""Linear polarisation under conjugate-symmetry folding (Sec. 3.3, Eq. (9)).  FP64.

Test infrastructure only.

Stokes Q and U are separate real images; the linear polarisation image is
P = Q + iU, and its visibilities are y_P = y_Q + i y_U.  Folding (Eq. (8))
reflects a visibility with w < 0 to (-u, -v, -w) and conjugates it, which is
valid for a real image only.  So the reflection is applied to y_Q and y_U
separately and the two are combined with -i (Eq. (9)):

    y_P(u, v, w) = conj( y_Q(-u, -v, -w) - i y_U(-u, -v, -w) )    for w < 0,
    y_P(u, v, w) = y_Q(u, v, w) + i y_U(u, v, w)                    otherwise,

with y_Q, y_U the (unconjugated) Stokes operators at the folded coordinates.
Conjugating y_P as if P were real (the Stokes I rule) gives
conj(y_Q) + i conj(y_U) wrong by conj(i y_U) - i conj(y_U) = -2i conj(y_U).

The pair operator A(Q, U) = Phi Q + i Phi U is real-linear; under the real
inner product its adjoint is (Re Phi^dagger y, Re Phi^dagger (-i y)).

Pins (tests/test_oracle_polar.py): agreement with the direct DFT of P at the
unfolded coordinates (to the aliasing level), the wrong Stokes I rule failing
that comparison, U = 0 reducing to the Stokes operator, and the adjoint
identity of the pair operator.
"""
from __future__ import annotations

import numpy as np

from .operator import StackedOperator


def folded_stokes(op: StackedOperator, x):
    """Phi x at the folded coordinates, without the Eq. (8) conjugation."""
    y = op.forward(x)
    return np.where(op.flag, np.conj(y), y)


def forward(op: StackedOperator, q_img, u_img):
    """y_P of Eq. (9) for the visibilities of ``op`` (folded or not)."""
    yq = folded_stokes(op, q_img)
    yu = folded_stokes(op, u_img)
    return np.where(op.flag, np.conj(yq - 1j * yu), yq + 1j * yu)


def adjoint(op: StackedOperator, y_p):
    """(Q, U) = (Re Phi^dagger y_P, Re Phi^dagger (-i y_P))."""
    y_p = np.asarray(y_p, dtype=np.complex128)
    return op.adjoint(y_p), op.adjoint(-1j * y_p)


def naive_forward(op: StackedOperator, q_img, u_img):
    """The Stokes I folding rule applied to P (conjugate y_P itself): wrong when U != 0."""
    y = folded_stokes(op, q_img) + 1j * folded_stokes(op, u_img)
    return np.where(op.flag, np.conj(y), y)
