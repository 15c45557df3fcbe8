"""GPU surrogate kernels (BF16 MFMA, FP32 accumulation) against the NumPy
oracle evaluated with the same BF16 rounding points.

Tolerances.  Both sides round the same operands to BF16; they differ in the
accumulation (FP32 on the GPU, FP64 in the oracle) and in the FP32 versus FP64
GELU, which occasionally moves a value across a BF16 rounding boundary (one
BF16 unit, 2^-8 relative).  Per tensor the relative Frobenius error is held to
2e-3 and every element to 2e-2 of the tensor's largest magnitude.
"""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2011_01740_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL_NORM, TOL_ELEM = 2e-3, 2e-2


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
    rel = np.linalg.norm(g - o) / max(np.linalg.norm(o), 1e-30)
    el = np.abs(g - o).max() / max(np.abs(o).max(), 1e-30)
    assert rel <= TOL_NORM and el <= TOL_ELEM, (name, rel, el)
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
    ref = M.backward(ps, cache, out, t.astype(np.float64), bf16=True)
    assert loss == pytest.approx(M.mse(out, t), rel=1e-4)
    gs = M.unpack(g.astype(np.float64))
    names = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    for name, gg, rr in zip(names, gs, ref):
        _close(gg, rr, name)


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
