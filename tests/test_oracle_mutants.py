"""Planted mistakes in the oracle (on the CPU) must each fail some pin.

Each mutant is the oracle's source with one plausible slip (a dropped term, a
wrong index or sign, a missing conjugate, an inverted selection).  The pins of
``test_oracle_pins`` are re-run against the mutant; at least one of them has to
fail, which shows the pins constrain that part of the oracle.
"""

import os
import sys
import types

import pytest

import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "gmres_sdr.py")

MUTANTS = {
    "window_one_short": ("range(max(j - t + 1, 1), j + 1)", "range(max(j - t + 2, 1), j + 1)"),
    "no_conjugate": ("np.vdot(V[:, i - 1], w)", "np.dot(V[:, i - 1], w)"),
    "sav_drops_subdiagonal": ("nc = j if breakdown else j + 1", "nc = j"),
    "smallest_mu_selected": ('order = np.argsort(-mod, kind="stable")',
                             'order = np.argsort(mod, kind="stable")'),
    "residual_sign": ("rt = r0 - A @ xt", "rt = r0 + A @ xt"),
    "su_from_saw": ("new = Recycle(Wb @ G, SB @ G, SAW @ G)",
                    "new = Recycle(Wb @ G, SAW @ G, SAW @ G)"),
    "m_without_conjugate": ("M = Uh.conj().T @ SB @ Vh", "M = Uh.T @ SB @ Vh"),
    "safety_inverted": ("safety = res / sres", "safety = sres / res"),
    "sketch_not_of_new_vector": ("SV[:, j] = S @ V[:, j]\n", "SV[:, j] = S @ V[:, j - 1]\n"),
    "rank_loss_keeps_dependent_column": ("        if rank_loss:\n            # a column",
                                         "        if False:\n            # a column"),
    "rank_loss_absolute_distance": ("return not (_norm(a - SAW[:, :-1] @ c) / na > rank_rtol)",
                                    "return not (_norm(a - SAW[:, :-1] @ c) > rank_rtol)"),
}

PINS = [
    lambda: pins.test_truncated_arnoldi_relation_and_band(False),
    lambda: pins.test_truncated_arnoldi_relation_and_band(True),
    pins.test_inner_product_count_is_t_plus_one_per_step,
    pins.test_sketch_of_Av_from_arnoldi_relation,
    pins.test_sketched_residual_nonincreasing_within_cycle,
    pins.test_identity_sketch_full_orthogonalisation_is_gmres_dr,
    lambda: pins.test_exact_eigenspace_is_recovered_for_any_sketch(1),
    pins.test_exact_eigenspace_complex,
    pins.test_recycled_exact_solution_space_converges_in_one_step,
    lambda: pins.test_solution_matches_dense_lu("cd"),
    lambda: pins.test_solution_matches_dense_lu("helmholtz"),
    pins.test_safety_factor_update_rule,
    pins.test_rank_loss_leaves_the_dependent_column_out,
]


def _mutant_module(old, new, path=SRC):
    src = open(path).read()
    assert src.count(old) == 1, old
    src = (src.replace(old, new).replace("from .sketch import", "from oracle.sketch import")
           .replace("from .srdct import", "from oracle.srdct import"))
    name = "oracle_mutant"
    mod = types.ModuleType(name)
    sys.modules[name] = mod  # dataclasses look their module up here
    try:
        exec(compile(src, name, "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    mod = _mutant_module(*MUTANTS[name])
    monkeypatch.setattr(pins, "sdr_solve", mod.sdr_solve)
    monkeypatch.setattr(pins, "harmonic_ritz_update", mod.harmonic_ritz_update)
    monkeypatch.setattr(pins, "Recycle", mod.Recycle)
    caught = []
    for pin in PINS:
        try:
            pin()
        except Exception:  # an assertion or a numerical failure both count
            caught.append(pin)
            break
    assert caught, f"mutant {name} passed every pin"


# Planted mistakes in the right Jacobi preconditioned solve, against its pins.
PRECOND_MUTANTS = {
    "left_scaling": ("Ahat.data = A.data * dinv[A.indices]",
                     "Ahat.data = A.data * dinv[np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))]"),
    "d_not_inverted": ("Ahat.data = A.data * dinv[A.indices]", "Ahat.data = A.data * d[A.indices]"),
    "x_not_back_transformed": ("out.x = out.x / d", "out.x = out.x"),
    "x0_not_transformed": ("u0 = None if x0 is None else d * np.asarray(x0)",
                           "u0 = None if x0 is None else np.asarray(x0)"),
}


@pytest.mark.parametrize("name", sorted(PRECOND_MUTANTS))
def test_precond_mutant_is_caught(name, monkeypatch):
    import test_oracle_precond as ppins
    mod = _mutant_module(*PRECOND_MUTANTS[name])
    monkeypatch.setattr(ppins, "sdr_solve_right_jacobi", mod.sdr_solve_right_jacobi)
    caught = False
    for pin in (lambda: ppins.test_power_of_two_columns_reduce_to_the_unscaled_solve(False),
                ppins.test_diagonal_matrix_is_one_step,
                ppins.test_badly_scaled_columns_converge_as_the_balanced_system,
                ppins.test_exact_initial_guess_and_zero_diagonal):
        try:
            pin()
        except Exception:
            caught = True
            break
    assert caught, f"mutant {name} passed every pin"


# Planted mistakes in the Givens-rotation residual control, against its pins.
GIVENS_MUTANTS = {
    "cosine_for_sine": ("        s_last = abs(b) / r\n", "        s_last = abs(a) / r\n"),
    "rotation_sign": ("G[c0 + 1, c0:] = -np.conj(sn) * rows[0] + cs * rows[1]",
                      "G[c0 + 1, c0:] = np.conj(sn) * rows[0] + cs * rows[1]"),
    "factor_without_sqrt": ("return float(np.sqrt((sine * sine + 2.0 * eps * (1.0 + c)) / (1.0 - eps * eps)))",
                            "return float((sine * sine + 2.0 * eps * (1.0 + c)) / (1.0 - eps * eps))"),
    "eps_not_refitted": ("            self.eps = hi\n", "            self.eps = self.eps\n"),
    "anchor_ignores_recycled_block": ("        if khat == 0:\n            self.anchor = (beta, False)",
                                      "        if True:\n            self.anchor = (beta, False)"),
}


@pytest.mark.parametrize("name", sorted(GIVENS_MUTANTS))
def test_givens_mutant_is_caught(name, monkeypatch):
    import test_oracle_givens as gpins
    mod = _mutant_module(*GIVENS_MUTANTS[name])
    for attr in ("sdr_solve", "givens_sine", "givens_factor", "sketched_least_squares"):
        monkeypatch.setattr(gpins, attr, getattr(mod, attr))
    caught = False
    for pin in (lambda: gpins.test_sketched_residual_is_givens_sine_times_previous(False),
                gpins.test_identity_sketch_estimate_is_the_true_residual,
                gpins.test_eps_refit_reaches_the_observed_residual,
                gpins.test_givens_control_solution_matches_dense_lu,
                gpins.test_givens_factor_special_values):
        try:
            pin()
        except Exception:
            caught = True
            break
    assert caught, f"mutant {name} passed every pin"


# Planted mistakes in the subsampled randomised DCT sketch, against its pins.
SRDCT_SRC = os.path.join(os.path.dirname(SRC), "srdct.py")
SRDCT_MUTANTS = {
    "scale_dropped": ("self.scale = np.sqrt(N / s)", "self.scale = 1.0"),
    "signs_not_applied": ("Y = X.reshape(self.N, -1) * self.signs[:, None]", "Y = X.reshape(self.N, -1) * 1.0"),
    "dct_type_3": ("F = scipy.fft.dct(Y, type=2, norm=\"ortho\", axis=0)",
                   "F = scipy.fft.dct(Y, type=3, norm=\"ortho\", axis=0)"),
    "rows_by_largest_key": ("order = np.lexsort((np.arange(N), k))", "order = np.lexsort((np.arange(N), -k))"),
}


@pytest.mark.parametrize("name", sorted(SRDCT_MUTANTS))
def test_srdct_mutant_is_caught(name, monkeypatch):
    import test_oracle_srdct as spins
    mod = _mutant_module(*SRDCT_MUTANTS[name], path=SRDCT_SRC)
    for attr in ("SRDCT", "srdct_rows", "srdct_signs"):
        monkeypatch.setattr(spins, attr, getattr(mod, attr))
    caught = False
    for pin in (spins.test_columns_follow_the_dct_definition,
                spins.test_signs_and_rows_follow_the_generator,
                lambda: spins.test_all_rows_kept_is_an_isometry(64)):
        try:
            pin()
        except Exception:
            caught = True
            break
    assert caught, f"mutant {name} passed every pin"


# Planted mistakes in the multicolour ILU(0) right preconditioning, against its pins.
ILU_SRC = os.path.join(os.path.dirname(SRC), "ilu.py")
ILU_MUTANTS = {
    "left_preconditioning": ("return A @ M.solve(np.asarray(v).reshape(-1))",
                             "return M.solve(A @ np.asarray(v).reshape(-1))"),
    "no_pivot_division": ("            row[k] = row[k] / piv\n", "            row[k] = row[k]\n"),
    "update_only_right_of_diagonal": ("                if j > k and j in row:", "                if j >= i and j in row:"),
    "colours_from_higher_neighbours": ("used = {int(colours[j]) for j in nb if j < i}",
                                       "used = {int(colours[j]) for j in nb if j > i}"),
    "natural_order": ("    return np.lexsort((np.arange(n), colours))", "    return np.arange(n)"),
}


@pytest.mark.parametrize("name", sorted(ILU_MUTANTS))
def test_ilu_mutant_is_caught(name, monkeypatch):
    import test_oracle_ilu as ipins
    old, new = ILU_MUTANTS[name]
    src = open(ILU_SRC).read()
    assert src.count(old) == 1, old
    src = src.replace(old, new).replace("from .gmres_sdr import", "from oracle.gmres_sdr import")
    mod = types.ModuleType("oracle_ilu_mutant")
    sys.modules["oracle_ilu_mutant"] = mod
    try:
        exec(compile(src, "oracle_ilu_mutant", "exec"), mod.__dict__)
    finally:
        del sys.modules["oracle_ilu_mutant"]
    for attr in ("ILU0", "greedy_colours", "ilu0", "multicolour_order", "sdr_solve_right_ilu0"):
        monkeypatch.setattr(ipins, attr, getattr(mod, attr))
    caught = False
    for pin in (ipins.test_five_point_colouring_is_the_checkerboard,
                ipins.test_colouring_is_proper_and_greedy,
                lambda: ipins.test_ilu0_defining_property_and_column_elimination("general"),
                ipins.test_apply_and_multiply_are_inverse_and_match_dense_factors,
                lambda: ipins.test_preconditioned_solution_matches_dense_solve("cd")):
        try:
            pin()
        except Exception:
            caught = True
            break
    assert caught, f"mutant {name} passed every pin"
