"""The pins catch plausible mistakes: each test plants one mistake in the
oracle (on the CPU, by monkeypatching) and checks that the pin that should
detect it fails."""

import numpy as np
import pytest

from oracle import coefficients as co
from oracle import particles as pt
from oracle import spectral as sp
from tests import test_oracle_coefficients as tc
from tests import test_oracle_particles as tp


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_theta_instead_of_theta_squared_is_caught(monkeypatch):
    orig = co.galilean_psatd_coefficients

    def wrong(k, v, dt, c=1.0, eps0=1.0):
        out = orig(k, v, dt, c, eps0)
        # c_EE = theta C instead of theta^2 C
        out["c_EE"] = out["c_EE"] / out["theta"]
        return out

    monkeypatch.setattr(co, "galilean_psatd_coefficients", wrong)
    _fails(tc.test_update_matches_exact_propagator)


def test_wrong_sign_of_rho_old_term_is_caught(monkeypatch):
    orig = co.galilean_psatd_coefficients

    def wrong(k, v, dt, c=1.0, eps0=1.0):
        out = orig(k, v, dt, c, eps0)
        out["c_R0"] = -out["c_R0"]
        return out

    monkeypatch.setattr(co, "galilean_psatd_coefficients", wrong)
    _fails(tc.test_update_matches_exact_propagator)
    _fails(tc.test_drifting_coulomb_field_is_a_fixed_point)


def test_dropped_current_term_in_b_is_caught(monkeypatch):
    orig = sp.galilean_psatd_update

    def wrong(E, B, J, r0, r1, k, coef, mask, c=1.0):
        coef = dict(coef)
        coef["c_BJ"] = np.zeros_like(coef["c_BJ"])
        return orig(E, B, J, r0, r1, k, coef, mask, c)

    monkeypatch.setattr(sp, "galilean_psatd_update", wrong)
    _fails(tc.test_update_matches_exact_propagator)


def test_transposed_cross_product_is_caught(monkeypatch):
    def wrong(a, b):
        return (a[2] * b[1] - a[1] * b[2], a[0] * b[2] - a[2] * b[0], a[1] * b[0] - a[0] * b[1])

    monkeypatch.setattr(sp, "cross", wrong)
    _fails(tc.test_vacuum_plane_wave_exact_for_any_dt, 1.0)


def test_wrong_quadrature_panel_is_caught(monkeypatch):
    # too coarse a rule (one 2-point panel) loses the integrals' accuracy
    monkeypatch.setattr(co, "GL_POINTS", 2)
    monkeypatch.setattr(co, "PANEL_LENGTH", 100.0)
    orig = co.duhamel_integrals

    def coarse(phi, nu, points=2, panel_length=100.0):
        return orig(phi, nu, points, panel_length)

    monkeypatch.setattr(co, "duhamel_integrals", coarse)
    _fails(tc.test_chis_match_printed_closed_form_random)


def test_swapped_cubic_weights_are_caught(monkeypatch):
    orig = pt.bspline_weights

    def wrong(delta, order):
        w, rel = orig(delta, order)
        if order == 3:
            w = w[:, ::-1].copy()
        return w, rel

    monkeypatch.setattr(pt, "bspline_weights", wrong)
    _fails(tp.test_shape_matches_scipy_cardinal_bspline, 3)


def test_boris_rotation_sign_is_caught(monkeypatch):
    orig = pt.boris_push

    def wrong(u, E, B, q, m, dt, c=1.0):
        return orig(u, E, -B, q, m, dt, c)

    monkeypatch.setattr(pt, "boris_push", wrong)
    _fails(tp.test_boris_uniform_magnetic_field_rotation)


def test_fft_sign_convention_is_caught(monkeypatch):
    monkeypatch.setattr(sp, "forward", lambda f: np.conj(np.fft.fftn(np.asarray(f, float))))
    from tests import test_oracle_spectral as ts

    _fails(ts.test_forward_matches_direct_dft)
