"""The package's smoke check (one small run of the hot path on cuda:0 against
the oracle: keys after one step, states after twenty) passes."""
import pytest

pytestmark = pytest.mark.gpu


def test_smoke():
    import __graft_entry__
    __graft_entry__.smoke()
