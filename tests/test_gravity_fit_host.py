"""The library's particle-mesh polynomial fit (host code in libcrk.so, no GPU)
against the oracle's fit of the same force."""

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def crk():
    import paper_2310_16122_amd as crk

    crk.load_library()
    return crk


@pytest.mark.parametrize("ratio", [4.0, 5.0, 6.0])
def test_fit_matches_the_oracle(crk, ratio):
    """Same weighted least-squares problem, independent solvers (Householder QR
    in the library, numpy's SVD-based solver in the oracle): the polynomials
    agree to 1e-11 of the force's scale over [0, r_c]."""
    rc = 3.0 / 128
    r_s = rc / ratio
    got = np.array(crk.sr_gravity_fit_poly(r_s, rc))
    ref = oracle.fit_poly(r_s, rc)
    r = np.linspace(0.0, 1.0, 1001) * rc
    pg, pr = np.polyval(got[::-1], r * r), np.polyval(ref[::-1], r * r)
    assert np.abs(pg - pr).max() <= 1e-11 * np.abs(pr).max()
    # and the force it stands for
    g = oracle.long_range_force(r[1:], r_s) / r[1:]
    assert np.abs((pg[1:] - g) * r[1:] ** 3).max() < 1e-2


def test_fit_rejects_bad_arguments(crk):
    for args in ((0.0, 0.02, 256), (0.004, -1.0, 256), (0.004, 0.02, 3), (float("nan"), 0.02, 256)):
        with pytest.raises(crk.CrkError):
            crk.sr_gravity_fit_poly(*args)
