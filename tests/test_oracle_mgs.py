"""Pins of the oracle's modified Gram-Schmidt least squares solver.

References: numpy.linalg.lstsq (FP64), the normal equations solved by mpmath at
400 bits (DD and QD), orthonormality of the computed Q, residual orthogonality
A^H (A dx - b) = 0, and the singular flag on a rank-deficient matrix.
"""
import mpmath
import numpy as np
import pytest

import oracle
from tests.exact import fr


def _cplx_limbs(Z, L, rng):
    """complex array -> [..., 2, L] limbs with random lower limbs."""
    out = np.zeros(Z.shape + (2, L))
    out[..., 0, 0] = Z.real
    out[..., 1, 0] = Z.imag
    for l in range(1, L):
        out[..., :, l] = rng.uniform(-0.5, 0.5, Z.shape + (2,)) * np.spacing(np.abs(out[..., :, l - 1]))
    return out


def _mpf(q):
    return mpmath.mpf(q.numerator) / q.denominator


def _mp_complex(limbs2L):
    return mpmath.mpc(_mpf(fr(limbs2L[0])), _mpf(fr(limbs2L[1])))


@pytest.mark.parametrize("m,n", [(3, 3), (8, 8), (16, 16), (12, 7)])
def test_fp64_against_lstsq(m, n):
    rng = np.random.default_rng(m * 100 + n)
    A = rng.normal(size=(m, n)) + 1j * rng.normal(size=(m, n))
    b = rng.normal(size=m) + 1j * rng.normal(size=m)
    dx, sing, q = oracle.mgs(1, _cplx_limbs(A, 1, rng), _cplx_limbs(b, 1, rng), want_q=True)
    assert not sing
    got = dx[:, 0, 0] + 1j * dx[:, 1, 0]
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(got - ref) <= 1e-14 * kappa * max(1.0, np.linalg.norm(ref)) * n
    # residual orthogonal to the range of A
    r = A @ got - b
    assert np.linalg.norm(A.conj().T @ r) <= 1e-12 * kappa * np.linalg.norm(A) * max(1, np.linalg.norm(b))
    Q = q[..., 0, 0] + 1j * q[..., 1, 0]
    assert np.linalg.norm(Q.conj().T @ Q - np.eye(n)) <= 1e-13 * kappa * n


@pytest.mark.parametrize("L", [2, 4])
@pytest.mark.parametrize("m,n", [(4, 4), (8, 8), (9, 5)])
def test_multilimb_against_mpmath(L, m, n):
    rng = np.random.default_rng(7 * m + n + L)
    A = rng.normal(size=(m, n)) + 1j * rng.normal(size=(m, n))
    b = rng.normal(size=m) + 1j * rng.normal(size=m)
    Al, bl = _cplx_limbs(A, L, rng), _cplx_limbs(b, L, rng)
    dx, sing, q = oracle.mgs(L, Al, bl, want_q=True)
    assert not sing
    with mpmath.workdps(120):
        MA = mpmath.matrix(m, n)
        Mb = mpmath.matrix(m, 1)
        for i in range(m):
            Mb[i] = _mp_complex(bl[i])
            for j in range(n):
                MA[i, j] = _mp_complex(Al[i, j])
        AH = MA.transpose_conj()
        ref = mpmath.lu_solve(AH * MA, AH * Mb)
        kappa = np.linalg.cond(A)
        u = 2.0 ** (-52 * L)
        err = max(abs(_mp_complex(dx[j]) - ref[j]) for j in range(n))
        nrm = max(abs(ref[j]) for j in range(n))
        assert float(err) <= 64 * n * kappa * u * max(1.0, float(nrm))
        # orthonormality of Q in L limbs
        MQ = mpmath.matrix(m, n)
        for i in range(m):
            for j in range(n):
                MQ[i, j] = _mp_complex(q[i, j])
        G = MQ.transpose_conj() * MQ
        dev = max(abs(G[i, j] - (1 if i == j else 0)) for i in range(n) for j in range(n))
        assert float(dev) <= 64 * n * kappa * u


def _hi_only(Z, L):
    """complex array -> [..., 2, L] with zero lower limbs (exact copies)."""
    out = np.zeros(Z.shape + (2, L))
    out[..., 0, 0] = Z.real
    out[..., 1, 0] = Z.imag
    return out


@pytest.mark.parametrize("L", [1, 2, 4])
def test_singular_flag(L):
    rng = np.random.default_rng(99)
    b = rng.normal(size=6) + 1j * rng.normal(size=6)
    # zero matrix
    _, sing0, _ = oracle.mgs(L, _hi_only(np.zeros((6, 4), dtype=complex), L), _hi_only(b, L))
    assert sing0
    # duplicated column: rank deficient
    B = rng.normal(size=(6, 4)) + 1j * rng.normal(size=(6, 4))
    B[:, 2] = B[:, 0]
    _, sing1, _ = oracle.mgs(L, _hi_only(B, L), _hi_only(b, L))
    assert sing1
    # a regular matrix is not flagged
    _, sing2, _ = oracle.mgs(L, _hi_only(B[:, [0, 1, 3]], L), _hi_only(b, L))
    assert not sing2


def test_identity_exact():
    """For A = I the solution is b exactly."""
    rng = np.random.default_rng(5)
    b = rng.normal(size=4) + 1j * rng.normal(size=4)
    for L in (1, 2, 4):
        dx, sing, _ = oracle.mgs(L, _hi_only(np.eye(4) + 0j, L), _hi_only(b, L))
        assert not sing
        assert np.array_equal(dx[:, 0, 0] + 1j * dx[:, 1, 0], b)
