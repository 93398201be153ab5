"""Pade-type high-order absorbing condition used as the transmission condition (paper Sec. 7: the
experiments prescribe it on every interface with N_pade = 8 auxiliary fields and a branch-cut
rotation phi = pi/3).  Test infrastructure: nothing here is used by the GPU path.

The exact one-way condition of an outgoing wave on a straight face is d_n u = i kappa sqrt(1 + Z) u
with Z = d_tau (kappa^-2 d_tau) the tangential operator.  The rotated Pade approximation
(Milinazzo, Zala and Brooke, J. Acoust. Soc. Am. 101, 1997; used as a transmission condition by
Boubendir, Antoine and Geuzaine, J. Comput. Phys. 231, 2012) replaces the square root by

    sqrt(1 + z) ~ C0 + sum_l A_l z / (1 + B_l z),   l = 1..N,

obtained from the standard Pade expansion 1 + sum a_l w / (1 + b_l w) of sqrt(1 + w), with
a_l = 2 sin^2(l pi / (2N+1)) / (2N+1), b_l = cos^2(l pi / (2N+1)), applied after rotating the
branch cut: sqrt(1 + z) = e^{i phi/2} sqrt(1 + w) with w = (1 + z) e^{-i phi} - 1.  Each term is an
auxiliary field phi_l on the face with (1 + B_l Z) phi_l = u.  Without rotation the evanescent
modes (z < -1) are not approximated; with it they are (the branch chosen is the decaying one,
sqrt(1 + z) = i sqrt(-1 - z)).

Discrete reading on the 5-point grid (the paper uses P7 finite elements and gives no discrete
form).  Along a face with positions e = 0..n-1 and face wavenumbers kappa_e (the interface alpha
of the face template), Z becomes the symmetric tridiagonal D with

    (D v)_e = sum_{e' = e +- 1} w_{e,e'} (v_{e'} - v_e),   w_{e,e+1} = 1 / (h^2 kappa_e kappa_{e+1}),

and homogeneous Neumann closure at the two face ends (no corner compatibility relations).
Eliminating the auxiliary fields gives the face operator R(D) = C0 I + sum_l A_l D (I + B_l D)^{-1},
a dense symmetric n x n matrix, and the impedance alpha of the first-order face template becomes
the symmetric matrix X = K^{1/2} R(D) K^{1/2} (K = diag(kappa); X = kappa R(D) for a constant
kappa).  With N = 0 and phi = 0, X = K and the template is the Robin condition exactly.

Pins (tests/test_oracle_habc.py): the rational approximation against the square root on
propagating and evanescent z, with the error decreasing in N; R(D) against the eigen-decomposition
of D; the reduction to the Robin condition; the interface identities of the decomposition.
"""
from __future__ import annotations

import numpy as np

PADE_DEFAULT = (8, np.pi / 3)  # (N_pade, phi) of the paper's experiments


def pade_coefficients(npade, phi):
    """(C0, A[l], B[l]) of sqrt(1 + z) ~ C0 + sum_l A_l z / (1 + B_l z) with branch rotation phi."""
    n = int(npade)
    ell = np.arange(1, n + 1)
    a = 2.0 / (2 * n + 1) * np.sin(ell * np.pi / (2 * n + 1)) ** 2
    b = np.cos(ell * np.pi / (2 * n + 1)) ** 2
    w0 = np.exp(-1j * phi) - 1.0  # w at z = 0
    c0 = np.exp(0.5j * phi) * (1.0 + np.sum(a * w0 / (1.0 + b * w0)))
    A = np.exp(-0.5j * phi) * a / (1.0 + b * w0) ** 2
    B = np.exp(-1j * phi) * b / (1.0 + b * w0)
    return complex(c0), A.astype(np.complex128), B.astype(np.complex128)


def pade_sqrt(z, npade, phi):
    """The rational function C0 + sum_l A_l z / (1 + B_l z) at scalar or array z."""
    c0, A, B = pade_coefficients(npade, phi)
    z = np.asarray(z, dtype=np.complex128)
    r = np.full(z.shape, c0, dtype=np.complex128)
    for al, bl in zip(A, B):
        r = r + al * z / (1.0 + bl * z)
    return r


def tangential_operator(kappa, h):
    """D: the symmetric tridiagonal d_tau (kappa^-2 d_tau) along a face of len(kappa) positions,
    Neumann closure at both ends."""
    kappa = np.asarray(kappa, dtype=np.float64)
    n = kappa.size
    D = np.zeros((n, n), dtype=np.float64)
    if n > 1:
        w = 1.0 / (h * h * kappa[:-1] * kappa[1:])
        e = np.arange(n - 1)
        D[e, e + 1] = w
        D[e + 1, e] = w
        D[e, e] -= w
        D[e + 1, e + 1] -= w
    return D


def face_operator(D, npade, phi):
    """R(D) = C0 I + sum_l A_l D (I + B_l D)^{-1} (dense)."""
    c0, A, B = pade_coefficients(npade, phi)
    n = D.shape[0]
    eye = np.eye(n, dtype=np.complex128)
    R = c0 * eye
    for al, bl in zip(A, B):
        R = R + al * D @ np.linalg.inv(eye + bl * D)
    return R


def face_impedance(kappa, h, npade, phi):
    """X = K^{1/2} R(D) K^{1/2}, the matrix that takes the place of alpha in the face template."""
    kappa = np.asarray(kappa, dtype=np.float64)
    s = np.sqrt(kappa)
    R = face_operator(tangential_operator(kappa, h), npade, phi)
    return s[:, None] * R * s[None, :]


def face_maps(kappa, h, npade, phi):
    """Matrices of the face template (u_q - u_p)/h - (i/2) X (u_p + u_q) = g along one face:

      bm, bp  beta-+ = I/h -+ (i/2) X                 (g = bm u_q - bp u_p)
      Q       bm^{-1}; the ghost values u_q = Q (g + bp u_p)
      rho     bp Q = (2/h) Q - I: the block -rho / h^2 joins the rows of the face nodes
      sigma   bp Q bp - bm = (4/h)(Q/h - I): the data sent across are -rho g - sigma u_p
      inj     Q / h^2: the incoming data enter the right-hand side as inj g
    """
    X = face_impedance(kappa, h, npade, phi)
    n = X.shape[0]
    eye = np.eye(n, dtype=np.complex128)
    bm = eye / h - 0.5j * X
    bp = eye / h + 0.5j * X
    Q = np.linalg.inv(bm)
    return {"X": X, "bm": bm, "bp": bp, "Q": Q, "rho": bp @ Q, "sigma": bp @ Q @ bp - bm, "inj": Q / (h * h)}
