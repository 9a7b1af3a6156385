"""The CPU oracle against values fixed by the paper and by mathematics."""
import pytest

import oracle
import pins


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda f: f.__name__)
def test_pin(check):
    check(oracle)


def test_table1_layout():
    pins.check_table1_layout()
