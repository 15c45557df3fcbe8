"""Host logic of the screening calibration (no GPU)."""
import numpy as np

from paper_2011_01740_amd.surrogate import calibrate_labels, loo_disagreement


def test_loo_disagreement_counts_axis_neighbours():
    lab = np.zeros((5, 5), np.int8)
    lab[2, 2] = 1            # the node itself never counts
    lab[1, 2] = 1            # one neighbour agrees with label 1
    lab[3, 2] = -1           # unknown label: counts as different
    G = 5
    k = loo_disagreement(lab.ravel(), np.array([2 * G + 2]), np.array([1], np.int8))
    assert k.tolist() == [3]
    k0 = loo_disagreement(lab.ravel(), np.array([2 * G + 2]), np.array([0], np.int8))
    assert k0.tolist() == [2]                # (1,2) = 1 and (3,2) = -1 differ from 0
    # border: neighbours reflect inwards, (0,0) sees (1,0) twice and (0,1) twice
    lab2 = np.zeros((5, 5), np.int8)
    lab2[1, 0] = 1
    k2 = loo_disagreement(lab2.ravel(), np.array([0]), np.array([0], np.int8))
    assert k2.tolist() == [2]


def test_only_contradicted_points_when_errors_sit_there():
    rng = np.random.default_rng(0)
    n = 20000
    d = rng.uniform(0, 1, n)
    k = np.where(rng.uniform(0, 1, n) < 0.02, 4, 0)
    wrong = k == 4
    m0, m1 = calibrate_labels(d, wrong, k, 0.001, n)
    assert m0 == 0.0 and m1 == 0.0


def test_budget_is_met_and_band_beats_the_plain_margin():
    rng = np.random.default_rng(1)
    n = 40000
    d = rng.uniform(0, 1, n)
    k = rng.choice([0, 1, 2, 3, 4], size=n, p=[0.9, 0.03, 0.03, 0.02, 0.02])
    part = (k >= 1) & (k <= 3)
    wrong = (k == 4) | (part & (d < 0.1) & (rng.uniform(0, 1, n) < 0.5)) | \
            ((k == 0) & (d < 0.01) & (rng.uniform(0, 1, n) < 0.2))
    target = 0.003
    m0, m1 = calibrate_labels(d, wrong, k, target, n)
    res = (k == 4) | (part & (d < m1)) | (d < m0)
    assert (wrong & ~res).sum() <= target * n
    plain = (d < np.sort(d[wrong])[::-1][int(target * n)] + 1e-7).mean()
    assert res.mean() < 0.5 * plain
