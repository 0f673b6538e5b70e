"""The device spectral norms behind the Lipschitz constants of eqs. eqLipsLd /
eqLipsLu, through the C ABI test hook, against the largest eigenvalue from
LAPACK's symmetric eigensolver (numpy.linalg.eigvalsh, FP64).

Every size class of the device code is covered (n <= 16, 24, 32 on the
vector ALU, <= 48 on the FP64 matrix cores, <= 64 by Lanczos), with the
matrices the sweep sees (Hadamard products of Grams, D H D), and the
degenerate cases: zero, rank one, identity (all eigenvalues equal), a
reducible diagonal (the squaring bounds never meet, so the Lanczos path
decides), a zero row, entries near the ends of the FP64 range, a negative
entry (Lanczos) and NaN.  Tolerance: 1e-12 relative; the squaring path stops
once its rigorous bounds agree to 1e-14 and LAPACK's error is a few ulps of
the norm.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lmax_ref(a):
    return np.linalg.eigvalsh(a)[..., -1]


def hadamard_of_grams(rng, count, n, rows=60):
    out = np.empty((count, n, n))
    for c in range(count):
        h = np.ones((n, n))
        for _ in range(3):
            u = rng.random((rows, n))
            h *= u.T @ u
        out[c] = h
    return out


def dhd(rng, count, n):
    h = hadamard_of_grams(rng, count, n)
    d = rng.random((count, n)) * 3.0
    return d[:, :, None] * h * d[:, None, :]


@pytest.mark.parametrize("n", [1, 2, 5, 6, 15, 16, 17, 19, 20, 23, 24, 25, 30, 31, 32, 33, 40, 47, 48, 49, 64])
def test_sweep_matrices_all_size_classes(n):
    from paper_2302_05119_amd import spectral_norm
    rng = np.random.default_rng(1000 + n)
    mats = np.concatenate([hadamard_of_grams(rng, 6, n), dhd(rng, 6, n)])
    say(f"[spectral] n={n} count={len(mats)}")
    got = spectral_norm(mats)
    np.testing.assert_allclose(got, lmax_ref(mats), rtol=RTOL)


@pytest.mark.parametrize("n", [7, 20, 30, 40, 60])
def test_degenerate_cases(n):
    from paper_2302_05119_amd import spectral_norm
    rng = np.random.default_rng(77 + n)
    say(f"[spectral] degenerate n={n}")
    v = rng.random(n) + 0.1
    zero_row = hadamard_of_grams(rng, 1, n)[0]
    zero_row[n // 2, :] = 0.0
    zero_row[:, n // 2] = 0.0
    cases = {
        "zero": np.zeros((n, n)),
        "rank_one": np.outer(v, v),
        "identity": np.eye(n) * 2.5,
        "reducible": np.diag(np.linspace(3.0, 1.0, n)),
        "zero_row": zero_row,
        "huge": hadamard_of_grams(rng, 1, n)[0] * 1e290,
        "tiny": hadamard_of_grams(rng, 1, n)[0] * 1e-290,
    }
    g = rng.standard_normal((2 * n, n))
    cases["negative_entries"] = g.T @ g
    for name, a in cases.items():
        got = spectral_norm(a)
        want = lmax_ref(a)
        say(f"   {name}: gpu={got:.17e} lapack={want:.17e}")
        if want == 0.0:
            assert got == 0.0, name
        else:
            assert abs(got - want) <= RTOL * abs(want), (name, got, want)
    bad = hadamard_of_grams(rng, 1, n)[0]
    bad[1 % n, 0] = bad[0, 1 % n] = np.nan
    assert np.isnan(spectral_norm(bad))


def test_many_matrices_one_launch():
    from paper_2302_05119_amd import spectral_norm
    rng = np.random.default_rng(5)
    mats = dhd(rng, 2000, 20)
    say("[spectral] 2000 matrices n=20")
    np.testing.assert_allclose(spectral_norm(mats), lmax_ref(mats), rtol=RTOL)


def test_rejects_bad_arguments():
    from paper_2302_05119_amd import ConcpdError, spectral_norm
    with pytest.raises(ConcpdError):
        spectral_norm(np.eye(65))
    with pytest.raises(ValueError):
        spectral_norm(np.ones((3, 4)))
