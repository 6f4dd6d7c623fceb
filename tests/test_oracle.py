"""The FP64 oracle against its pins (closed forms, libraries, brute force,
invariants).  CPU only."""
import pytest

import oracle
import oracle_pins as pins


def test_dct_basis():
    pins.check_dct_basis()


def test_dft_basis():
    pins.check_dft_basis()


def test_metrics():
    pins.check_metrics()


@pytest.mark.parametrize("check", pins.ORACLE_CHECKS, ids=lambda f: f.__name__)
def test_oracle_pin(check):
    check(oracle)
