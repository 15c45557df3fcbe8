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


# ------------------------------------------------ the screen without a network

def test_bilinear_values_reproduce_a_bilinear_function():
    from paper_2011_01740_amd.surrogate import bilinear_values
    Gt, Gs = 7, 25
    x = np.linspace(-1, 1, Gt)
    f = lambda a, b: 0.3 + 1.7 * a - 0.4 * b + 2.2 * a * b  # noqa: E731
    vt = f(x[:, None], x[None, :]).ravel()
    xs = np.linspace(-1, 1, Gs)
    want = f(xs[:, None], xs[None, :]).ravel()
    got = bilinear_values(vt, Gt, Gs)
    assert np.max(np.abs(got - want)) < 1e-13
    # at the nodes the values themselves (the dense grid holds every fourth point)
    assert np.array_equal(got.reshape(Gs, Gs)[::4, ::4], vt.reshape(Gt, Gt))


def test_corner_disagreement_brute_force():
    from paper_2011_01740_amd.surrogate import corner_disagreement
    rng = np.random.default_rng(3)
    Gt, Gs = 6, 17
    nlab = rng.choice([-1, 0, 1], size=Gt * Gt, p=[0.1, 0.5, 0.4]).astype(np.int8)
    lab = rng.integers(0, 2, Gs * Gs).astype(np.int8)
    k = corner_disagreement(nlab, Gt, Gs, lab)
    L = nlab.reshape(Gt, Gt)
    for a in range(Gs):
        for b in range(Gs):
            # the cell [i, i+1] x [j, j+1] that holds the point (the last cell
            # at the upper border)
            u, v = a * (Gt - 1) / (Gs - 1), b * (Gt - 1) / (Gs - 1)
            i, j = min(int(u), Gt - 2), min(int(v), Gt - 2)
            want = sum(int(L[i + di, j + dj] != lab[a * Gs + b]) for di in (0, 1) for dj in (0, 1))
            assert k[a * Gs + b] == want


def test_loo_values_mean_of_the_axis_neighbours():
    from paper_2011_01740_amd.surrogate import loo_values
    G = 6
    x = np.arange(G, dtype=np.float64)
    vt = (2.0 * x[:, None] - 3.0 * x[None, :]).ravel()   # linear: interior mean is exact
    inner = np.array([i * G + j for i in range(1, G - 1) for j in range(1, G - 1)])
    assert np.max(np.abs(loo_values(vt, G, inner) - vt[inner])) < 1e-12
    vt2 = vt.copy()
    vt2[1 * G + 2] = np.nan                               # left out of (2, 2)'s mean
    want = (vt[3 * G + 2] + vt[2 * G + 1] + vt[2 * G + 3]) / 3.0
    assert abs(loo_values(vt2, G, np.array([2 * G + 2]))[0] - want) < 1e-12


def test_band_tradeoff_is_the_optimum_over_all_thresholds():
    from paper_2011_01740_amd.surrogate import band_resolve, band_tradeoff
    rng = np.random.default_rng(5)
    n = 600
    d = np.round(rng.uniform(0, 1, n), 3)
    d[:5] = -1.0                                        # always re-solved
    k = rng.choice([0, 1, 2, 3, 4], size=n, p=[0.7, 0.1, 0.08, 0.07, 0.05])
    jsel = np.sort(rng.choice(n, 300, replace=False))
    wrong_j = (rng.uniform(0, 1, 300) < np.exp(-6 * np.abs(d[jsel]))) & (rng.uniform(0, 1, 300) < 0.4)
    for budget in (0, 2, 5, 20):
        frac, m0, m1 = band_tradeoff(d, k, jsel, wrong_j, budget)
        res = band_resolve(d, k, m0, m1)
        assert abs(res.mean() - frac) < 1e-15
        assert (wrong_j & ~res[jsel]).sum() <= budget
        # brute force over thresholds at every distinct d (and just above)
        cand = np.unique(np.concatenate([[0.0], d[d >= 0], d[d >= 0] + 1e-9, [2.0]]))
        best = 1.0
        for a in cand:
            cov = band_resolve(d, k, a, cand[:, None])      # every m1 at once
            ok = (wrong_j[None, :] & ~cov[:, jsel]).sum(axis=1) <= budget
            if ok.any():
                best = min(best, cov[ok].mean(axis=1).min())
        assert frac <= best + 1e-15
