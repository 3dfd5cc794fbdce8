"""The library's choice of the number of filter periods against the oracle's
(host computation, no GPU): the same integer for 2D and 3D boxes, adjusted and
plain frequencies, several wanted counts."""
import pytest

from oracle import discrete as D


def _omega_used(omega, adjust, n_its=10):
    if not adjust:
        return omega
    import math
    s = math.sin(math.pi / n_its)
    return omega * math.pi / n_its * math.sqrt((1 - 2 * s * s) / (s * s))


@pytest.mark.parametrize("length,omega,k,adjust", [
    ((1.0, 1.0), 40.0, 8, True),
    ((1.0, 1.0), 120.0, 16, True),
    ((1.0, 1.0), 90.0, 16, True),
    ((1.3, 0.6), 25.0, 4, False),
    ((1.0, 1.0, 1.0), 40.0, 8, True),
    ((1.0, 0.5, 0.8), 30.0, 12, False),
    ((1.0, 1.0), 5.0, 50, False),
])
def test_library_matches_oracle(length, omega, k, adjust):
    from paper_2507_18282_amd import choose_periods
    got = choose_periods(length, omega, k, adjust_omega=adjust)
    want = D.choose_periods(length, _omega_used(omega, adjust), k)
    assert got == want


def test_invalid_arguments_raise():
    from paper_2507_18282_amd import EigenwaveError, choose_periods
    with pytest.raises(EigenwaveError):
        choose_periods((1.0, 1.0), 40.0, 0)
    with pytest.raises(EigenwaveError):
        choose_periods((1.0, 1.0), 40.0, 4, beta_r=0.3)
