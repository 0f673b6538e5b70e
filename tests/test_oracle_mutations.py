"""Plant plausible mistakes in the oracle (on the CPU) and check that at least
one pin catches each of them.  This guards the pins' strength, not the
oracle's values.

Two kinds of plant: a function of the oracle replaced by a wrong one, and a
source-level edit (one expression of the oracle's text changed, the module
re-executed from the edited text, and every function of the module swapped
for its mutant so that internal calls see the mistake too)."""
import inspect
import sys
import types

import numpy as np
import pytest

from oracle import apg
import test_oracle_extrapolation_pins as xpins
import test_oracle_pins as pins


def _wrong_krp_order(U, n):
    return apg.khatri_rao([U[m] for m in range(len(U)) if m != n])


def _skip_ignored(U, skip=None):
    return _orig_hog(U, None)


_orig_hog = apg.hadamard_of_grams
_orig_sn = apg.spectral_norm


MUTATIONS = {
    # transposed Khatri-Rao order in the MTTKRP
    "krp_order": (("krp_minus", _wrong_krp_order), pins.test_mttkrp_matches_element_sum, (1,)),
    # H_{-n} that forgets to drop mode n (wrong gradient)
    "hadamard_skip": (("hadamard_of_grams", _skip_ignored), pins.test_gradients_match_finite_differences, ()),
    # step twice too long
    "half_lipschitz": (("spectral_norm", lambda A: 0.5 * _orig_sn(A)),
                       pins.test_unextrapolated_sweep_is_exact_block_minimisation_rank1, ((1, 0, 1), None, True)),
    # wrong t recursion
    "t_recursion": (("t_next", lambda t: 0.5 * (1.0 + np.sqrt(1.0 + 2.0 * t * t))),
                    pins.test_t_sequence_closed_forms, ()),
    # extrapolation weight without the Lipschitz-ratio cap
    "weight_cap": (("extrapolation_weight", lambda w, Lp, Lc, d: w if Lp is not None else 0.0),
                   pins.test_extrapolation_weight_rule, ()),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    (attr, fn), pin, args = MUTATIONS[name]
    monkeypatch.setattr(apg, attr, fn)
    with pytest.raises(AssertionError):
        pin(*args)


def test_planted_mistake_ignoring_coupling_groups_is_caught(monkeypatch):
    # flexible coupling that ties the shared columns of every block instead of
    # only the listed ones
    monkeypatch.setattr(apg.Options, "group", lambda self, n, S: list(range(S)) if self.L[n] else [])
    with pytest.raises(AssertionError):
        pins.test_unextrapolated_sweep_is_exact_block_minimisation_rank1((1, 0, 1), ((0, 2), None, (1, 2)), True)


# ---------------------------------------------------------------------------
# source-level plants
# ---------------------------------------------------------------------------

SOURCE_MUTATIONS = {
    # extrapolation in the wrong direction (a wrong sign), core / individual / shared
    "extrap_sign_core": ("lam_hat = st.lam[s] + w * (st.lam[s] - st.lam_prev[s])",
                         "lam_hat = st.lam[s] - w * (st.lam[s] - st.lam_prev[s])"),
    "extrap_sign_individual": ("Uhat.append(st.U[n][s] + w * (st.U[n][s] - st.U_prev[n][s]))",
                               "Uhat.append(st.U[n][s] - w * (st.U[n][s] - st.U_prev[n][s]))"),
    "extrap_sign_shared": ("UC_hat = UC_old + wC * (UC_old - UC_prev)",
                           "UC_hat = UC_old - wC * (UC_old - UC_prev)"),
    # extrapolation from x_{k-2} instead of x_{k-1}
    "extrap_base_individual": ("Uhat.append(st.U[n][s] + w * (st.U[n][s] - st.U_prev[n][s]))",
                               "Uhat.append(st.U_prev[n][s] + w * (st.U[n][s] - st.U_prev[n][s]))"),
    # w_hat = (t_k - 1) / t_k instead of (t_{k-1} - 1) / t_k
    "w_hat_index": ("w_hat = (st.t - 1.0) / t_k", "w_hat = (t_k - 1.0) / t_k"),
    # shared block weighted with block 0's own Lipschitz constants instead of L_C
    "shared_weight_individual_L": (
        "wC = extrapolation_weight(w_hat, st.LC_prev[n], LC, opt.delta_w)",
        "wC = extrapolation_weight(w_hat, st.Lu_prev[n][grp[0]], Lu[grp[0]], opt.delta_w)"),
    # stopping on the objective instead of the RelErr change
    "stop_on_objective": ("abs(st.relerr - prev_rel) < opt.tol", "abs(st.F - prev_rel) < opt.tol"),
    # RelErr as the squared norm ratio
    "relerr_squared": ("float(np.linalg.norm(X - reconstruct(lam[s], Us)) / np.linalg.norm(X))",
                       "float((np.linalg.norm(X - reconstruct(lam[s], Us)) / np.linalg.norm(X)) ** 2)"),
    # no restart
    "no_restart": ("if opt.restart and F >= st.F:", "if False and opt.restart and F >= st.F:"),
    # restart that keeps the rejected extrapolated sweep's point as the start of the redo
    "restart_from_rejected": ("        lam, U, rec = sweep(data, st, w_hat, False, opt)\n",
                              "        st = State(U=U, lam=lam, U_prev=st.U, lam_prev=st.lam, Ld_prev=st.Ld_prev,"
                              " Lu_prev=st.Lu_prev, LC_prev=st.LC_prev, t=st.t, k=st.k, F=st.F)\n"
                              "        lam, U, rec = sweep(data, st, w_hat, False, opt)\n"),
}


def _pins_for_source_mutation(name):
    ext = xpins.test_extrapolated_sweep_from_objective_evaluations
    stop = xpins.test_run_stops_at_first_small_relerr_change_and_at_max_it
    rel = xpins.test_relerr_and_fit_match_element_sum_reconstruction
    table = {
        "extrap_sign_core": [(ext, ("cap_free", 4))],
        "extrap_sign_individual": [(ext, ("cap_free", 4))],
        "extrap_sign_shared": [(ext, ("cap_free", 4))],
        "extrap_base_individual": [(ext, ("cap_free", 4))],
        "w_hat_index": [(ext, ("cap_free", 4))],
        "shared_weight_individual_L": [(ext, ("cap_binds", 4)), (ext, ("group", 4))],
        "stop_on_objective": [(stop, (1e-4,))],
        "relerr_squared": [(rel, ())],
        "no_restart": [(pins.test_forced_overshoot_triggers_restart, ())],
        "restart_from_rejected": [(pins.test_forced_overshoot_triggers_restart, ())],
    }
    return table[name]


def _mutant_module(monkeypatch, old, new):
    src = inspect.getsource(apg)
    assert src.count(old) == 1, f"mutation target not unique: {old!r}"
    mod = types.ModuleType("apg_mutant")
    monkeypatch.setitem(sys.modules, "apg_mutant", mod)   # dataclasses look their module up
    exec(compile(src.replace(old, new), "apg_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(SOURCE_MUTATIONS))
def test_planted_source_mistake_is_caught(name, monkeypatch):
    mod = _mutant_module(monkeypatch, *SOURCE_MUTATIONS[name])
    for attr, val in vars(mod).items():
        if isinstance(val, types.FunctionType) and getattr(apg, attr, None) is not None:
            monkeypatch.setattr(apg, attr, val)
    for pin, args in _pins_for_source_mutation(name):
        with pytest.raises(AssertionError):
            pin(*args)


def test_unmutated_source_module_passes_the_same_pins(monkeypatch):
    # the re-execution machinery itself changes nothing
    mod = _mutant_module(monkeypatch, "w_hat = (st.t - 1.0) / t_k", "w_hat = (st.t - 1.0) / t_k")
    for attr, val in vars(mod).items():
        if isinstance(val, types.FunctionType) and getattr(apg, attr, None) is not None:
            monkeypatch.setattr(apg, attr, val)
    xpins.test_extrapolated_sweep_from_objective_evaluations("cap_binds", 4)
    xpins.test_run_stops_at_first_small_relerr_change_and_at_max_it(1e-4)
    pins.test_forced_overshoot_triggers_restart()
