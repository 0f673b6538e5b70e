"""Plant plausible mistakes in the oracle (on the CPU) and check that at least
one pin catches each of them.  This guards the pins' strength, not the
oracle's values."""
import numpy as np
import pytest

from oracle import apg
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
