"""GPU surrogate kernels (BF16 MFMA, FP32 accumulation) against the NumPy
oracle evaluated with the same BF16 rounding points.

Tolerances.  Both sides round the same operands to BF16; they differ in the
accumulation (FP32 on the GPU, FP64 in the oracle) and in the sine and GELU
(on the GPU the hardware sine of an FP32 argument and a rational approximation
of the normal tail with |error| <= 1.5e-7; in the oracle FP64 library
functions), which now and then move an operand across a BF16 rounding
boundary (one BF16 unit, 2^-8 relative, in that one term of a sum).  So:
per tensor the relative Frobenius error is at most 1e-3; element by element,
every entry of at least a tenth of the tensor's RMS is within 10% of its own
value (a weight-gradient entry sums 64 to 4096 row terms; where they cancel
to a tenth of their sizes, one or two flipped terms move it by up to
2 x 2^-8 x 10, about 8%), and the smaller entries within 1% of the RMS.  A
transposed operand, a wrong index, sign or scale moves entries by O(1) of
their value and fails both.
"""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2011_01740_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL_NORM = 1e-3          # per tensor, relative Frobenius
TOL_REL = 0.1            # entries >= 0.1 RMS, relative to themselves
TOL_ABS = 1e-2           # smaller entries, relative to the tensor's RMS


def _sur():
    import torch
    from paper_2011_01740_amd import sur
    assert torch.cuda.is_available()
    return sur


def _data(m, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, size=(m, 2)).astype(np.float32)
    t = rng.normal(size=(m, 64)).astype(np.float32)
    return x, t


def _close(g, o, name):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    if not np.any(o):
        assert not np.any(g), (name, np.abs(g).max())
        return 0.0
    rel = np.linalg.norm(g - o) / np.linalg.norm(o)
    rms = np.sqrt(np.mean(o * o))
    big = np.abs(o) >= 0.1 * rms
    d = np.abs(g - o)
    er_big = (d[big] / np.abs(o[big])).max()
    er_small = d[~big].max() / rms if (~big).any() else 0.0
    print(f"{name}: frobenius {rel:.2e}, large entries {er_big:.2e}, small entries {er_small:.2e}")
    assert rel <= TOL_NORM and er_big <= TOL_REL and er_small <= TOL_ABS, (name, rel, er_big,
                                                                          er_small)
    return rel


def _f32_params(seed):
    return I.mlp_init(seed).astype(np.float32).astype(np.float64)


def test_forward_matches_oracle():
    sur = _sur()
    flat = _f32_params(4)
    x, _ = _data(320, 1)
    with sur.Surrogate(max_batch=512) as s:
        s.set_params(flat)
        out = s.forward(x)
    ref, _ = M.forward(M.unpack(flat), x.astype(np.float64), bf16=True)
    _close(out, ref, "output")


@pytest.mark.parametrize("m", [1, 33, 1000])
def test_forward_ragged_sizes_match_oracle(m):
    """The fused inference kernel takes 32 points per wave and 4 waves per
    block: sizes below one wave, one point past a wave, and a ragged tail."""
    sur = _sur()
    flat = _f32_params(6)
    x, _ = _data(m, 3)
    with sur.Surrogate(max_batch=512) as s:
        s.set_params(flat)
        out = s.forward(x)
    ref, _ = M.forward(M.unpack(flat), x.astype(np.float64), bf16=True)
    _close(out, ref, f"output m={m}")


def test_forward_host_chunks_equal_device_call():
    """From host memory the inputs pass through the handle's staging buffers
    65536 rows at a time; from device memory one launch takes all rows.  Both
    give the same bits, and a seeded sample of rows (both ends of each chunk
    included) matches the oracle."""
    import torch
    sur = _sur()
    flat = _f32_params(7)
    m = 65536 + 1000
    x, _ = _data(m, 4)
    with sur.Surrogate(max_batch=512) as s:
        s.set_params(flat)
        out_h = s.forward(x)
        out_d = s.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.array_equal(out_h, out_d)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([[0, 65535, 65536, m - 1], rng.integers(0, m, 1000)]))
    ref, _ = M.forward(M.unpack(flat), x[idx].astype(np.float64), bf16=True)
    _close(out_h[idx], ref, "output sample")


def test_screen_full_grid_sample_matches_oracle():
    """sur_screen over the whole 4096 x 4096 sweep grid (2^24 points, the
    screening launch of the screened sweep): the predicted maximum at a seeded
    sample of points (the grid's corners included) against the oracle's
    network on the same normalised inputs, and the label wherever the
    oracle's prediction is not within 1e-2 of the threshold."""
    import torch
    sur = _sur()
    G = 4096
    P, _ = I.km_grid(G, G)
    lo = np.array([P[0].min(), np.log(P[1].min())])
    hi = np.array([P[0].max(), np.log(P[1].max())])
    mean = np.linspace(0.2, 0.9, 64)
    std = np.linspace(0.3, 0.6, 64)
    flat = _f32_params(8)
    with sur.Surrogate(max_batch=512) as s:
        s.set_params(flat)
        s.set_norm(lo, hi, mean, std)
        label, resolve, pmax, idx = s.screen(torch.from_numpy(P).cuda(), 0.05, 0.5, 0.1)
        label, resolve, pmax = (v.cpu().numpy() for v in (label, resolve, pmax))
    rng = np.random.default_rng(9)
    k = np.unique(np.concatenate([[0, G - 1, G * (G - 1), G * G - 1],
                                  rng.integers(0, G * G, 4000)]))
    x = np.stack([(P[0, k] - lo[0]) * (2.0 / (hi[0] - lo[0])) - 1.0,
                  (np.log(P[1, k]) - lo[1]) * (2.0 / (hi[1] - lo[1])) - 1.0],
                 axis=1).astype(np.float32)
    ref, _ = M.forward(M.unpack(flat), x.astype(np.float64), bf16=True)
    y = ref * std + mean
    want = y.max(axis=1)
    _close(pmax[k], want, "predicted max")
    far = np.abs(want - np.log(2.0)) > 1e-2
    assert np.array_equal(label[k][far].astype(bool), (want >= np.log(2.0))[far])
    assert idx.numel() == int(resolve.sum())


@pytest.mark.parametrize("m", [64, 128, 4096])
def test_gradients_match_oracle(m):
    sur = _sur()
    flat = _f32_params(5)
    x, t = _data(m, 2)
    with sur.Surrogate(max_batch=4096) as s:
        s.set_params(flat)
        g, loss = s.gradients(x, t)
        g2, loss2 = s.gradients(x, t)
    assert np.array_equal(g, g2) and loss == loss2          # deterministic
    ps = M.unpack(flat)
    out, cache = M.forward(ps, x.astype(np.float64), bf16=True)
    ref = M.backward(ps, cache, out, t.astype(np.float64), bf16=True, w=M.OUT_WEIGHTS)
    assert loss == pytest.approx(M.mse(out, t, M.OUT_WEIGHTS), rel=1e-4)
    gs = M.unpack(g.astype(np.float64))
    names = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    for name, gg, rr in zip(names, gs, ref):
        _close(gg, rr, name)


def test_adam_steps_follow_the_oracle():
    """Five Adam steps on the GPU against five oracle steps (BF16-mode forward
    and backward, the oracle's Adam with its bias corrections, pinned by the
    constant-gradient test): the parameters agree to 1e-3 per tensor, and the
    feature layer never moves.  (Per element, Adam's first steps are about
    lr times the gradient's sign, so an entry whose tiny gradient the two
    sides round to opposite signs moves the other way; the comparison is per
    tensor for that reason.)"""
    sur = _sur()
    flat = _f32_params(13)
    x, t = _data(1024, 14)
    ps = M.unpack(flat)
    mm = [np.zeros_like(p) for p in ps]
    vv = [np.zeros_like(p) for p in ps]
    names = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    with sur.Surrogate(max_batch=1024) as s:
        s.set_params(flat)
        s.set_adam(lr=1e-3)
        for k in range(1, 6):
            s.train_step(x, t)
            out, cache = M.forward(ps, x.astype(np.float64), bf16=True)
            g = M.backward(ps, cache, out, t.astype(np.float64), bf16=True, w=M.OUT_WEIGHTS)
            ps, mm, vv = M.adam_step(ps, g, mm, vv, k, lr=1e-3, fixed=2)
            got = M.unpack(s.get_params())
            for name, a, b in zip(names, got, ps):
                rel = np.linalg.norm(a - b) / np.linalg.norm(b)
                assert rel <= 1e-3, (k, name, rel)
            assert np.array_equal(got[0], M.unpack(flat)[0])
            assert np.array_equal(got[1], M.unpack(flat)[1])


def test_dataset_targets_are_sorted_standardised_maxima():
    """sur_fit_norm and sur_build_dataset take each point's recorded maxima in
    decreasing order: mean / std per rank, targets (ln - mean) / std."""
    import torch
    sur = _sur()
    rng = np.random.default_rng(15)
    n = 1000
    rec = np.exp(rng.normal(size=(64, n)) * 0.3)
    rec[:, 5] = 1.7                                    # ties
    P = np.stack([rng.uniform(0.2e5, 1.2e5, n), np.exp(rng.uniform(np.log(20e3), np.log(1e6), n))])
    lo = np.array([0.2e5, np.log(20e3)])
    hi = np.array([1.2e5, np.log(1e6)])
    srt = -np.sort(-np.log(rec), axis=0)
    with sur.Surrogate(max_batch=64) as s:
        mean = np.empty(64)
        std = np.empty(64)
        rd = torch.from_numpy(rec).cuda()
        sur._check(sur._lib().sur_fit_norm(s.h, sur._dptr(lo), sur._dptr(hi),
                                           sur.ens.C.c_void_p(rd.data_ptr()), n,
                                           sur._dptr(mean), sur._dptr(std)), s.h)
        x, y = s.build_dataset(torch.from_numpy(P).cuda(), rd, n)
        y = y.cpu().numpy()
    assert np.allclose(mean, srt.mean(axis=1), rtol=1e-12, atol=1e-14)
    assert np.allclose(std, srt.std(axis=1), rtol=1e-10)
    want = ((srt - mean[:, None]) / std[:, None]).T
    assert np.allclose(y, want, rtol=1e-6, atol=1e-6)
    assert np.all(np.diff(y * std + mean, axis=1) <= 1e-6)


def test_adam_step_matches_formula():
    sur = _sur()
    flat = _f32_params(6)
    x, t = _data(256, 3)
    with sur.Surrogate(max_batch=256) as s:
        s.set_params(flat)
        s.set_adam(lr=1e-3)
        g, _ = s.gradients(x, t)
        s.train_step(x, t)
        p1 = s.get_params()
    ps = M.unpack(flat)
    zeros = [np.zeros_like(p) for p in ps]
    want, _, _ = M.adam_step(ps, M.unpack(g.astype(np.float64)), zeros, zeros, t=1, lr=1e-3)
    want = M.pack(want)
    assert np.allclose(p1, want, rtol=1e-6, atol=1e-7)


def test_training_reduces_loss_on_a_smooth_target():
    sur = _sur()
    rng = np.random.default_rng(9)
    x = rng.uniform(-1, 1, size=(4096, 2)).astype(np.float32)
    j = np.arange(64) / 64.0
    t = (np.sin(2 * x[:, :1] + j) * np.cos(x[:, 1:] - j)).astype(np.float32)
    with sur.Surrogate(max_batch=4096) as s:
        s.set_params(I.mlp_init(4))
        _, l0 = s.gradients(x, t)
        for _ in range(300):
            s.train_step(x, t)
        _, l1 = s.gradients(x, t)
    assert l1 < 0.05 * l0, (l0, l1)


def test_screen_matches_forward_and_compacts_in_order():
    import torch
    sur = _sur()
    P, _ = I.km_grid(40, 50)
    n = P.shape[1]
    lo = np.array([0.2e5, np.log(20e3)])
    hi = np.array([1.2e5, np.log(1e6)])
    mean = np.linspace(0.1, 0.9, 64)
    std = np.linspace(0.5, 1.5, 64)
    with sur.Surrogate(max_batch=1024) as s:
        s.set_params(I.mlp_init(7))
        s.set_norm(lo, hi, mean, std)
        Pd = torch.from_numpy(P).cuda()
        label, resolve, pmax, idx = s.screen(Pd, margin=0.3, spread=0.5, flag_margin=0.6)
        label, resolve, pmax, idx = (v.cpu().numpy() for v in (label, resolve, pmax, idx))
        x = np.stack([2 * (P[0] - lo[0]) / (hi[0] - lo[0]) - 1,
                      2 * (np.log(P[1]) - lo[1]) / (hi[1] - lo[1]) - 1], axis=1).astype(np.float32)
        out = s.forward(x).astype(np.float64)
    y = out * std + mean
    mx, mn = y.max(axis=1), y.min(axis=1)
    ok = np.abs(mx - pmax) < 1e-4
    assert ok.mean() > 0.999
    d = np.abs(mx - np.log(2))
    want_res = (d < 0.3) | ((mx - mn > 0.5) & (d < 0.6))
    agree = (resolve.astype(bool) == want_res) | (np.abs(d - 0.3) < 1e-4) | (np.abs(d - 0.6) < 1e-4)
    assert agree.all()
    assert np.array_equal(idx, np.nonzero(resolve)[0])
    assert np.array_equal(label.astype(bool)[ok], (pmax >= np.log(2))[ok])


def test_epoch_graph_replays_equal_eager_steps():
    """sur_train_epoch captures an epoch's launches once and replays them with
    the current learning rate, step count and row order: after three epochs
    (with different orders and learning rates, and eager work in between) the
    parameters equal those of the same batches taken one sur_train_step at a
    time, bit for bit."""
    import torch
    sur = _sur()
    from paper_2011_01740_amd import ens
    rows, batch = 1024, 256
    x, t = _data(rows, 7)
    rng = np.random.default_rng(8)
    orders = [rng.permutation(rows)[:768].astype(np.int64) for _ in range(3)]
    lrs = [3e-3, 2e-3, 1e-3]
    flat = _f32_params(10)
    with sur.Surrogate(max_batch=batch) as s:
        s.set_params(flat)
        xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
        perm = torch.empty(768, dtype=torch.int64, device="cuda")
        L = sur._lib()
        for order, lr in zip(orders, lrs):
            s.set_adam(lr=lr)
            perm.copy_(torch.from_numpy(order))
            loss = ens.C.c_float()
            sur._check(L.sur_train_epoch(s.h, ens.C.c_void_p(xd.data_ptr()),
                                         ens.C.c_void_p(td.data_ptr()), 768,
                                         ens.C.c_void_p(perm.data_ptr()), batch,
                                         ens.C.byref(loss)), s.h)
            s.forward(x[:64])                      # eager work between replays
        graph = s.get_params()
    with sur.Surrogate(max_batch=batch) as s:
        s.set_params(flat)
        for order, lr in zip(orders, lrs):
            s.set_adam(lr=lr)
            for b in range(3):
                r = order[b * batch:(b + 1) * batch]
                s.train_step(x[r], t[r])
        eager = s.get_params()
    assert np.array_equal(graph, eager)


def test_label_flag_against_the_training_labels():
    """sur_fit_label_map labels the training nodes from their records, and
    sur_screen flags a point when the four nodes of its cell contradict the
    network's label: all four, or some while the point is within the label
    margin (checked at points inside the cells, away from node lines)."""
    import torch
    sur = _sur()
    G = 9
    lo = np.array([0.2e5, np.log(20e3)])
    hi = np.array([1.2e5, np.log(1e6)])
    rng = np.random.default_rng(12)
    node_max = rng.choice([1.5, 3.0], size=G * G)
    node_max[17] = np.nan                          # unknown label
    rec = np.tile(node_max, (64, 1)) * np.linspace(0.9, 1.0, 64)[:, None]
    want_lab = np.where(np.isnan(rec).any(axis=0), -1, (rec.max(axis=0) >= 2).astype(np.int8))
    # screen points at fractional cell coordinates in [0.2, 0.8]
    m = 40
    uu = rng.integers(0, G - 1, m) + rng.uniform(0.2, 0.8, m)
    vv = rng.integers(0, G - 1, m) + rng.uniform(0.2, 0.8, m)
    P = np.stack([lo[0] + uu / (G - 1) * (hi[0] - lo[0]),
                  np.exp(lo[1] + vv / (G - 1) * (hi[1] - lo[1]))])
    mean = np.full(64, np.log(2.0))
    std = np.full(64, 0.01)
    with sur.Surrogate(max_batch=256) as s:
        s.set_params(I.mlp_init(3))
        s.set_norm(lo, hi, mean, std)
        lab_map = s.fit_label_map(torch.from_numpy(rec).cuda(), G).cpu().numpy()
        Pd = torch.from_numpy(P).cuda()
        lm = 0.02
        label, resolve, pmax, _ = s.screen(Pd, 0.0, 1e30, 0.0, label_margin=lm)
        label, resolve, pmax = (v.cpu().numpy() for v in (label, resolve, pmax))
        _, off, _, _ = s.screen(Pd, 0.0, 1e30, 0.0)          # flag off
    assert np.array_equal(lab_map, want_lab)
    assert not off.any()
    u0, v0 = np.floor(uu).astype(int), np.floor(vv).astype(int)
    L2 = want_lab.reshape(G, G)
    corners = np.stack([L2[u0, v0], L2[u0, v0 + 1], L2[u0 + 1, v0], L2[u0 + 1, v0 + 1]])
    k = (corners != label[None, :]).sum(axis=0)
    d = np.abs(pmax - np.log(2.0))
    want = (k == 4) | ((k >= 1) & (d < lm))
    near = np.abs(d - lm) < 1e-5
    assert np.array_equal(resolve.astype(bool)[~near], want[~near])
    assert want.any() and (~want).any()


def _epoch_order(rows, seed, epoch):
    """The documented order of sur_train_epochs: rows sorted (stably) by the
    SplitMix64 output function of seed + golden * (epoch * n + i + 1)."""
    n = rows.size
    with np.errstate(over="ignore"):
        z = (np.uint64(seed) + np.uint64(0x9E3779B97F4A7C15)
             * (np.uint64(epoch * n) + np.arange(n, dtype=np.uint64) + np.uint64(1)))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return rows[np.argsort(z, kind="stable")]


def test_train_epochs_equals_single_epochs_with_its_orders():
    import torch
    sur = _sur()
    from paper_2011_01740_amd import ens
    rows_total, batch = 1024, 256
    x, t = _data(rows_total, 11)
    rows = np.sort(np.random.default_rng(2).permutation(rows_total)[:800]).astype(np.int64)
    lrs = [3e-3, 1e-3, 2e-3]
    flat = _f32_params(12)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    with sur.Surrogate(max_batch=batch) as s:
        s.set_params(flat)
        losses = s.train_epochs(xd, td, torch.from_numpy(rows).cuda(), batch, lrs, 77)
        multi = s.get_params()
        with pytest.raises(ens.EnsError):
            s.train_epochs(xd, td, torch.from_numpy(rows).cuda(), batch, [1e-3, 0.0], 77)
    single_losses = []
    with sur.Surrogate(max_batch=batch) as s:
        s.set_params(flat)
        perm = torch.empty(rows.size, dtype=torch.int64, device="cuda")
        L = sur._lib()
        for e, lr in enumerate(lrs):
            s.set_adam(lr=lr)
            perm.copy_(torch.from_numpy(_epoch_order(rows, 77, e)))
            loss = ens.C.c_float()
            sur._check(L.sur_train_epoch(s.h, ens.C.c_void_p(xd.data_ptr()),
                                         ens.C.c_void_p(td.data_ptr()), rows.size,
                                         ens.C.c_void_p(perm.data_ptr()), batch,
                                         ens.C.byref(loss)), s.h)
            single_losses.append(loss.value)
        single = s.get_params()
    assert np.array_equal(multi, single)
    assert np.allclose(losses, single_losses, rtol=0, atol=0)
