"""Host logic of the screening calibration (no GPU)."""
import numpy as np

from paper_2011_01740_amd.surrogate import calibrate


def test_plain_band_when_errors_are_spread():
    rng = np.random.default_rng(0)
    d = rng.uniform(0, 1, 20000)
    wrong = (rng.uniform(0, 1, 20000) < 0.05) & (d < 0.3)
    emap = rng.uniform(0, 1, 20000)           # uninformative
    m0, e, m1 = calibrate(d, wrong, emap, 0.005, d.size)
    res = (d < m0) | ((emap > e) & (d < m1))
    assert (wrong & ~res).sum() <= 0.005 * d.size
    # the search returns the smallest band it finds; an uninformative map
    # cannot beat the plain band by much
    plain = np.sort(d[wrong])[::-1][int(0.005 * d.size)] + 1e-7
    assert res.mean() <= (d < plain).mean() + 1e-12


def test_error_map_narrows_the_band_when_errors_cluster():
    rng = np.random.default_rng(1)
    n = 40000
    d = rng.uniform(0, 1, n)
    rough = rng.uniform(0, 1, n) < 0.1                   # 10% rough region
    emap = np.where(rough, rng.uniform(0.5, 1, n), rng.uniform(0, 0.2, n))
    wrong = (rough & (d < 0.4) & (rng.uniform(0, 1, n) < 0.5)) | (~rough & (d < 0.02))
    m0, e, m1 = calibrate(d, wrong, emap, 0.002, n)
    res = (d < m0) | ((emap > e) & (d < m1))
    assert (wrong & ~res).sum() <= 0.002 * n
    assert np.isfinite(e) and 0.2 <= e < 0.75
    plain = (d < np.sort(d[wrong])[::-1][int(0.002 * n)] + 1e-7).mean()
    assert res.mean() < 0.5 * plain
