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


def test_half_push_with_full_step_is_caught(monkeypatch):
    """The laser start pushed through dt instead of dt / 2."""
    from oracle import pic
    from tests import test_oracle_step as tst

    def wrong(self, state):
        g, s = self.grid, self.species
        F = pt.gather(list(state.E) + list(state.B), state.x, g.shape, g.spacing, g.order)
        state.u = pt.boris_push(state.u, F[:3].T, F[3:].T, s.q, s.m, g.dt, self.c)
        return state

    monkeypatch.setattr(pic.Simulation, "half_push", wrong)
    _fails(tst.test_half_push_uniform_electric_field, 3)
    _fails(tst.test_half_push_uniform_magnetic_field)


def test_field_energy_without_half_is_caught(monkeypatch):
    from oracle import diagnostics as dg
    from tests import test_oracle_step as tst

    orig = dg.field_energy

    def wrong(E, B, cell_volume):
        we, wb = orig(E, B, cell_volume)
        return 2 * we, 2 * wb

    monkeypatch.setattr(dg, "field_energy", wrong)
    _fails(tst.test_field_energy_closed_form)


def test_field_energy_without_cell_volume_is_caught(monkeypatch):
    from oracle import diagnostics as dg
    from tests import test_oracle_step as tst

    orig = dg.field_energy
    monkeypatch.setattr(dg, "field_energy", lambda E, B, cell_volume: orig(E, B, 1.0))
    _fails(tst.test_field_energy_closed_form)


def test_galilean_phase_with_nyquist_is_caught(monkeypatch):
    """The largest phase taken at the Nyquist index n / 2 instead of n / 2 - 1."""
    def wrong(shape, spacing, v_gal, dt):
        return sum(abs(v) * 2 * np.pi * (n // 2) / (n * d)
                   for n, d, v in zip(shape, spacing, v_gal)) * dt

    monkeypatch.setattr(co, "max_galilean_phase", wrong)
    _fails(tc.test_max_galilean_phase_hand_value)
    _fails(tc.test_max_galilean_phase_brute_force)


def test_slab_window_off_by_one_is_caught(monkeypatch):
    from oracle import local as olc
    from tests import test_oracle_local as tl

    orig = olc.slab_planes
    monkeypatch.setattr(olc, "slab_planes",
                        lambda nz, n, g: [np.mod(p + 1, nz) for p in orig(nz, n, g)])
    _fails(tl.test_full_window_equals_global_solve, 4, 12)


def test_slab_sources_keeping_their_mean_is_caught(monkeypatch):
    from oracle import local as olc
    from tests import test_oracle_local as tl

    orig = olc.SlabSolver._source
    monkeypatch.setattr(olc.SlabSolver, "_source", lambda self, f, s, mean: orig(self, f, s, 0.0))
    _fails(tl.test_full_window_equals_global_solve, 2, 8)
