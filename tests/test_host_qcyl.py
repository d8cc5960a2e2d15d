"""The quasi-cylindrical solver's host logic (no GPU): its spectral grid
(zeros of J_m) and its Hankel transform matrices (with the k_r = 0 function
(r/R)^{m-1} as the last order m - 1 column for m >= 1), against mpmath's
arbitrary-precision Bessel functions and zeros and against scipy."""

import mpmath
import numpy as np
import pytest
from scipy import special

from paper_1608_00215_amd import galpic as gp

mpmath.mp.dps = 30


@pytest.mark.parametrize("m", [0, 1, 2, 7])
def test_wavenumbers_are_correctly_rounded_zeros(m):
    nr = 512
    k = gp.qc_wavenumbers(m, nr, 1.0 / nr)  # R = 1: k_i = alpha_{m,i}
    for i in (0, 1, 2, 9, 99, 250, 511):
        exact = mpmath.besseljzero(m, i + 1)
        # the zero rounded to a double, then divided by R = 1 (exact)
        assert abs(k[i] - float(exact)) <= np.spacing(k[i]), (m, i)
    # and within 2 ulp of scipy's zeros everywhere
    a = special.jn_zeros(m, nr)
    assert np.all(np.abs(k - a) <= 2 * np.spacing(a))


@pytest.mark.parametrize("m", [0, 1, 3, 7])
def test_backward_matrix_is_bessel_values(m):
    """Entries against mpmath at sampled points spanning both evaluation
    regimes (small arguments and arguments in the hundreds), with the
    argument formed as the library forms it."""
    nr, dr = 512, 0.1
    k = gp.qc_wavenumbers(m, nr, dr)
    rng = np.random.default_rng(500 + m)
    for p in (m - 1, m, m + 1):
        M = gp.qc_hankel_matrix(p, m, nr, dr)
        # for p = m - 1, m >= 1, the last column is the k_r = 0 function
        # (r_j / R)^{m-1} that completes the order m - 1 set
        cols = nr - 1 if (m >= 1 and p == m - 1) else nr
        if cols < nr:
            r = (np.arange(nr) + 0.5) / nr
            assert np.max(np.abs(M[:, -1] - r ** (m - 1))) <= 1e-15
        for _ in range(40):
            j, i = int(rng.integers(0, nr)), int(rng.integers(0, cols))
            x = k[i] * (j + 0.5) * dr
            ref = float(mpmath.besselj(p, x))
            assert abs(M[j, i] - ref) <= 4e-15, (p, j, i, x)
        # the first rows and columns are the small-argument corner
        for j, i in ((0, 0), (0, 5), (3, 0), (10, 10), (1, 40), (40, 1)):
            x = k[i] * (j + 0.5) * dr
            assert abs(M[j, i] - float(mpmath.besselj(p, x))) <= 4e-15, (p, j, i)


def test_backward_matrix_matches_scipy():
    nr, dr = 300, 0.25
    r = (np.arange(nr) + 0.5) * dr
    for m in (0, 1, 2):
        k = gp.qc_wavenumbers(m, nr, dr)
        for p in (m - 1, m, m + 1):
            ref = special.jv(p, np.outer(r, k))
            if m >= 1 and p == m - 1:
                ref[:, -1] = (r / (nr * dr)) ** (m - 1)
            assert np.max(np.abs(gp.qc_hankel_matrix(p, m, nr, dr) - ref)) <= 1e-14


@pytest.mark.parametrize("m", [0, 1, 2])
def test_forward_matrix_inverts_backward(m):
    nr, dr = 64, 0.5
    for p in (m - 1, m, m + 1):
        M = gp.qc_hankel_matrix(p, m, nr, dr)
        A = gp.qc_hankel_matrix(p, m, nr, dr, forward=True)
        kappa = np.linalg.cond(M)
        err = np.max(np.abs(A @ M - np.eye(nr)))
        assert err <= max(1e-13, 64 * kappa * 2.0 ** -52), (p, err, kappa)


def test_host_calls_reject_bad_arguments():
    for args in ((-1, 8, 0.5), (64, 8, 0.5), (0, 0, 0.5), (0, 513, 0.5), (0, 8, 0.0),
                 (0, 8, float("inf"))):
        with pytest.raises(gp.GalpicError) as e:
            gp.qc_wavenumbers(*args)
        assert e.value.status == gp.GP_ERR_ARG, args
    with pytest.raises(gp.GalpicError):
        gp.qc_hankel_matrix(65, 0, 8, 0.5)
    with pytest.raises(gp.GalpicError):
        gp.qc_hankel_matrix(0, 0, 8, -1.0, forward=True)
