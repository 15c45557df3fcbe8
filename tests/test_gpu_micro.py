"""The FP64 FMA-chain measurement (a helper beside the published peak)."""
import pytest

pytestmark = pytest.mark.gpu


def test_fma_chain_rate_is_positive_and_below_the_published_peak():
    from paper_2011_01740_amd import ens
    tf, ms = ens.micro_fma(0, 1 << 12)
    assert ms > 0
    assert 5.0 < tf < 78.6 * 1.02, tf
    with pytest.raises(ens.EnsError):
        ens.micro_fma(0, 0)
