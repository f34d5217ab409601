"""Plant plausible mistakes in the oracle (on the CPU, via monkeypatch) and
check that the pins catch each one. Guards the pins themselves."""
import numpy as np
import pytest

from oracle import metrics as om
from oracle import tfdp as ot
import tests.test_oracle_pins as pins


def fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_flipped_hx_sign_is_caught(monkeypatch):
    orig = ot.kernel_tables

    def bad(m, s, gamma, tau=1.0):
        k, hx, hy = orig(m, s, gamma, tau)
        return k, -hx, hy
    monkeypatch.setattr(ot, "kernel_tables", bad)
    assert fails(pins.test_on_grid_points_are_exact, 2, "stable")


def test_transposed_hy_is_caught(monkeypatch):
    orig = ot.kernel_tables

    def bad(m, s, gamma, tau=1.0):
        k, hx, hy = orig(m, s, gamma, tau)
        return k, hx, hy.T
    monkeypatch.setattr(ot, "kernel_tables", bad)
    assert fails(pins.test_on_grid_points_are_exact, 1, "stable")


def test_wrong_node_placement_is_caught(monkeypatch):
    monkeypatch.setattr(ot, "node_offsets", lambda k: np.arange(k, dtype=np.float64) / k)
    assert fails(pins.test_on_grid_points_are_exact, 2, "paper")


def test_dropped_spring_term_is_caught(monkeypatch):
    def bad(pos, row_ptr, col_idx, alpha, beta, rows=None, tau=1.0, weights=None):
        x = np.asarray(pos, dtype=np.float64)
        n = x.shape[0]
        src = np.repeat(np.arange(n), np.diff(row_ptr))
        diff = x[src] - x[np.asarray(col_idx)]
        d2 = (diff ** 2).sum(1)
        f = (beta / (1 + d2))[:, None] * diff
        return -alpha * np.stack([np.bincount(src, f[:, 0], n), np.bincount(src, f[:, 1], n)], 1)
    monkeypatch.setattr(ot, "attraction", bad)
    assert fails(pins.test_forces_are_minus_energy_gradient, 2.0)


def test_wrong_exponent_is_caught(monkeypatch):
    monkeypatch.setattr(ot, "kernel", lambda d2, gamma, tau=1.0: (1.0 + tau * np.asarray(d2)) ** (-(gamma - 1)))
    assert fails(pins.test_three_points_hand_computed)
    assert fails(pins.test_forces_are_minus_energy_gradient, 2.0)


def test_uncentred_box_is_caught(monkeypatch):
    def bad(pos):
        x = np.asarray(pos, dtype=np.float64)
        lo = x.min(0)
        w = (x.max(0) - lo).max()
        return (lo[0], lo[1], w)
    monkeypatch.setattr(ot, "square_box", bad)
    assert fails(pins.test_interpolated_invariances) or fails(pins.test_box_and_binning)


def test_missing_gather_offset_term_is_caught(monkeypatch):
    orig = ot.Interp.gather

    def bad(self, grid, combine):
        return orig(self, grid, lambda v, dx, dy: combine(v, 0.0 * dx, 0.0 * dy))
    monkeypatch.setattr(ot.Interp, "gather", bad)
    # on-grid points have delta = 0 at their only tap, so the off-grid
    # agreement of the two formulations is the pin for this term
    assert fails(pins.test_paper_form_equals_stable_form, 2)


def test_wrong_k_schedule_is_caught(monkeypatch):
    monkeypatch.setattr(ot, "k_for_iteration", lambda t, total: 1 if t < 0.9 * total else 3)
    assert fails(pins.test_k_schedule)


def test_kernel_tables_ignoring_tau_are_caught(monkeypatch):
    orig = ot.kernel_tables
    monkeypatch.setattr(ot, "kernel_tables", lambda m, s, gamma, tau=1.0: orig(m, s, gamma))
    assert fails(pins.test_tau_is_a_change_of_length_scale, 1)


def test_one_sided_edge_weights_are_caught(monkeypatch):
    orig = ot.attraction

    def bad(pos, row_ptr, col_idx, alpha, beta, rows=None, tau=1.0, weights=None):
        if weights is None:
            return orig(pos, row_ptr, col_idx, alpha, beta, rows, tau)
        return orig(pos, row_ptr, col_idx, alpha, beta, rows, tau) * np.asarray(weights)[:, None]
    monkeypatch.setattr(ot, "attraction", bad)
    assert fails(pins.test_local_refinement_two_nodes_closed_form)
    assert fails(pins.test_generalised_forces_are_minus_energy_gradient, 1.7, True)


def _sampled_pairs_with(mask_rule, src_rows):
    """stress_pairs with a planted change in how sampled rows are masked or
    where their source positions are read."""
    def bad(pos, row_ptr, col_idx, sources=None):
        x = np.asarray(pos, dtype=np.float64)
        n = x.shape[0]
        src = np.arange(n) if sources is None else np.asarray(sources)
        d = om.graph_distances(n, row_ptr, col_idx, src)
        rows = src_rows(src)
        lay = np.sqrt(((x[rows, None, :] - x[None, :, :]) ** 2).sum(-1))
        mask = np.isfinite(d) & (d > 0)
        mask &= mask_rule(n, src)
        return lay[mask], d[mask]
    return bad


def test_upper_triangle_mask_on_sampled_rows_is_caught(monkeypatch):
    # the all-pairs i < j rule applied to sampled rows, by node index or by
    # row position
    by_node = lambda n, src: np.arange(n)[None, :] > src[:, None]
    by_row = lambda n, src: np.arange(n)[None, :] > np.arange(len(src))[:, None]
    for rule in (by_node, by_row):
        monkeypatch.setattr(om, "stress_pairs", _sampled_pairs_with(rule, lambda src: src))
        assert fails(pins.test_sampled_stress_hand_computed)


def test_sampled_rows_read_by_position_are_caught(monkeypatch):
    monkeypatch.setattr(om, "stress_pairs",
                        _sampled_pairs_with(lambda n, src: True, lambda src: np.arange(len(src))))
    assert fails(pins.test_sampled_stress_hand_computed)
    assert fails(pins.test_sampled_stress_over_all_sources_equals_all_pairs)
