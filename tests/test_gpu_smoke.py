"""The round-trip check of __graft_entry__.smoke(): a fused small-N FP64 run and
an FP32 semi-implicit run on the MFMA stage kernels, each against the oracle."""
import pytest

pytestmark = pytest.mark.gpu


def test_smoke_entry_point():
    import __graft_entry__ as entry
    entry.smoke()
