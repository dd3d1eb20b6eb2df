"""GPU parity of the learned prescreen (MLP ensemble on the bfloat16 matrix
cores) and of top-k selection against the float64 oracle, through the C ABI.

Bars: member outputs within 2e-3 of the oracle with bfloat16 rounding
emulated at the same points (the device accumulates in float32 in another
order); gradients within 1e-3 relative L2 of the emulated oracle and 2e-2 of
the pure float64 oracle; top-k indices identical to a brute-force sort.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2403_08131_amd import gpbo as G
from paper_2403_08131_amd import inputs as I

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
E, D, H = 5, 20, 256


@pytest.fixture(scope="module")
def ctx():
    c = G.Context(0)
    yield c
    c.close()


def _init(seed=0, E=E, D=D, H=H):
    init = I.mlp_init(np.random.default_rng(seed), members=E, d_in=D, hidden=H)
    flat = O.mlp_pack(**init)  # (E, P) float64 holding float32 values
    return flat


def _data(n, seed=1):
    spec = I.spec_grouped(D, 0.1)
    r = np.random.default_rng(seed)
    X = I.f32r(r.uniform(0, 1, (n, D)))
    y = I.synthetic_f(X, spec)
    yt = (y - y.mean()) / y.std()
    return X, y, yt.astype(np.float32).astype(np.float64)


def _rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def test_topk_matches_brute_force(ctx):
    r = np.random.default_rng(3)
    for m, k in ((1000, 1), (10000, 100), (65536, 4096), (1 << 20, 4096)):
        v = np.round(r.normal(size=m), 2).astype(np.float32)  # many exact ties
        v[r.integers(0, m, 5)] = np.nan
        idx = G.topk(ctx, torch.tensor(v, device=DEV), k).cpu().numpy()
        vv = np.where(np.isnan(v), -np.inf, v.astype(np.float64))
        want = np.lexsort((np.arange(m), -vv))[:k]
        assert np.array_equal(idx, want), (m, k)
    # all-equal scores: the k lowest indices
    v = np.zeros(5000, dtype=np.float32)
    idx = G.topk(ctx, torch.tensor(v, device=DEV), 333).cpu().numpy()
    assert np.array_equal(idx, np.arange(333))


def test_gather_rows(ctx):
    X = torch.rand((1000, 7), device=DEV)
    idx = torch.tensor([5, 0, 999, 5, 321], dtype=torch.int64, device=DEV)
    out = G.gather_rows(ctx, idx, X)
    assert torch.equal(out, X[idx])


def test_mlp_forward_matches_oracle(ctx):
    flat = _init(0)
    net = G.Mlp(ctx, torch.tensor(flat, dtype=torch.float32, device=DEV).contiguous(), E, D, H)
    X, _, _ = _data(300)
    out = net.forward(torch.tensor(X, dtype=torch.float32, device=DEV)).double().cpu().numpy()
    ref_em = O.mlp_forward(flat, D, H, X, bf16=True)
    ref = O.mlp_forward(flat, D, H, X)
    err_em = np.max(np.abs(out - ref_em)) / np.max(np.abs(ref_em))
    err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    print(f"  forward: vs emulated {err_em:.2e}, vs float64 {err:.2e}")
    assert err_em <= 2e-3
    assert err <= 5e-2
    # a persistent grid of one or two workgroups per compute unit computes
    # every tile the same way: identical outputs (5 tiles x 5 members here,
    # and 600 tiles x 5 members, more items than workgroups)
    Xt = torch.tensor(X, dtype=torch.float32, device=DEV)
    Xb = torch.rand((38400, D), generator=torch.Generator(device=DEV).manual_seed(3), device=DEV)
    base_b = net.forward(Xb)
    for k in (1, 2):
        net.set_occupancy(k)
        assert torch.equal(net.forward(Xt), net.forward(Xt)) and torch.equal(
            net.forward(Xt).double().cpu(), torch.tensor(out))
        assert torch.equal(net.forward(Xb), base_b)
    net.set_occupancy(0)
    with pytest.raises(G.GpboError):
        net.set_occupancy(-1)
    net.free()


def test_mlp_gradients_match_oracle(ctx):
    flat = _init(2)
    net = G.Mlp(ctx, torch.tensor(flat, dtype=torch.float32, device=DEV).contiguous(), E, D, H)
    X, _, yt = _data(256, seed=4)
    g, loss = net.grads(torch.tensor(X, dtype=torch.float32, device=DEV),
                        torch.tensor(yt, dtype=torch.float32, device=DEV))
    g = g.double().cpu().numpy()
    loss = loss.double().cpu().numpy()
    l_em, g_em = O.mlp_loss_grad(flat, D, H, X, yt, bf16=True)
    l64, g64 = O.mlp_loss_grad(flat, D, H, X, yt)
    for e in range(E):
        r_em, r64 = _rel_l2(g[e], g_em[e]), _rel_l2(g[e], g64[e])
        print(f"  member {e}: grad rel L2 vs emulated {r_em:.2e}, vs float64 {r64:.2e}")
        assert r_em <= 1e-3 and r64 <= 2e-2
    assert np.allclose(loss, l_em, rtol=1e-3)


def test_mlp_adam_steps_match_oracle(ctx):
    flat = _init(5)
    net = G.Mlp(ctx, torch.tensor(flat, dtype=torch.float32, device=DEV).contiguous(), E, D, H)
    X, _, yt = _data(128, seed=6)
    hist = net.train(torch.tensor(X, dtype=torch.float32, device=DEV),
                     torch.tensor(yt, dtype=torch.float32, device=DEV), steps=1, lr=1e-3)
    w = net.params().double().cpu().numpy()
    ref, ref_hist = O.mlp_train(flat, D, H, X, yt, steps=1, lr=1e-3, bf16=True, master_f32=True)
    _, g_em = O.mlp_loss_grad(flat, D, H, X, yt, bf16=True)
    # The first Adam step moves each weight by about -lr sign(g); where the
    # gradient is nearly zero the sign is decided by rounding, so the moves
    # are compared where |g| is not negligible.
    move, ref_move = w - flat, ref - flat
    for e in range(E):
        sig = np.abs(g_em[e]) > 1e-3 * np.max(np.abs(g_em[e]))
        agree = np.mean(np.sign(move[e][sig]) == np.sign(ref_move[e][sig]))
        assert agree >= 0.99, (e, agree)
        assert _rel_l2(move[e][sig], ref_move[e][sig]) <= 5e-2, e
    assert np.allclose(hist.double().cpu().numpy(), ref_hist, rtol=2e-3)
    net.free()


def test_mlp_training_trajectory_matches_oracle(ctx):
    """Twelve full-batch Adam steps (the first eager, the rest replays of
    the captured step): the loss history follows the oracle's trajectory with
    bfloat16 rounding emulated and float32 master weights."""
    flat = _init(9)
    net = G.Mlp(ctx, torch.tensor(flat, dtype=torch.float32, device=DEV).contiguous(), E, D, H)
    X, _, yt = _data(256, seed=10)
    hist = net.train(torch.tensor(X, dtype=torch.float32, device=DEV),
                     torch.tensor(yt, dtype=torch.float32, device=DEV), steps=12, lr=1e-3)
    hist = hist.double().cpu().numpy()
    _, ref = O.mlp_train(flat, D, H, X, yt, steps=12, lr=1e-3, bf16=True, master_f32=True)
    err = np.max(np.abs(hist - ref) / ref)
    print(f"  12-step loss history: max rel. deviation from oracle {err:.2e}")
    assert err <= 1e-2
    net.free()


def test_mlp_training_reduces_loss_and_graph_replays(ctx):
    # The oracle's trajectory on data of this kind falls by about 1 % per
    # step over the first steps at lr 1e-3 (Adam's first steps may rise by a
    # fraction of a percent for a member); the bar asks for a 20 % drop in
    # 100 steps, no rise above 1 % of the start over the first 20 steps, and
    # further progress when the captured step is replayed by a second call.
    flat = _init(7)
    net = G.Mlp(ctx, torch.tensor(flat, dtype=torch.float32, device=DEV).contiguous(), E, D, H)
    X, _, yt = _data(1024, seed=8)
    Xd = torch.tensor(X, dtype=torch.float32, device=DEV)
    yd = torch.tensor(yt, dtype=torch.float32, device=DEV)
    h1 = net.train(Xd, yd, steps=100, lr=1e-3).cpu().numpy()
    h2 = net.train(Xd, yd, steps=100, lr=1e-3).cpu().numpy()  # replays the captured step
    net.free()
    print(f"  loss: start {h1[0]}, after 100 {h1[-1]}, after 200 {h2[-1]}")
    assert np.all(np.isfinite(h1)) and np.all(np.isfinite(h2))
    assert np.all(h1[-1] < 0.8 * h1[0])
    assert np.all(h2[-1] < h1[-1])
    assert np.all(np.diff(h1[:20], axis=0) < 0.01 * h1[0])
    assert np.all(h1[19] < h1[0])


def test_prescreen_ei_matches_oracle_and_sort(ctx):
    """gpbo_mlp_prescreen: the ensemble EI (member mean, population standard
    deviation, EI against f_best) of every candidate equals the oracle's
    ens_ei on the device's member outputs to the float32 rounding of the
    result (the kernel evaluates in float64), and the top-k indices equal a
    sort of the device's own float32 EI."""
    flat = _init(13)
    net = G.Mlp(ctx, torch.tensor(flat, dtype=torch.float32, device=DEV).contiguous(), E, D, H)
    X, _, _ = _data(30000, seed=14)
    Xd = torch.tensor(X, dtype=torch.float32, device=DEV)
    outs = net.forward(Xd).double().cpu().numpy()
    for fbest, k in ((float(np.quantile(outs.mean(0), 0.01)), 1),
                     (float(np.quantile(outs.mean(0), 0.2)), 999),
                     (float(outs.mean(0).min()) - 0.5, 4096)):
        idx, ei = net.prescreen(Xd, fbest, k, want_ei=True)
        ei = ei.double().cpu().numpy()
        mu_e, sd_e, ref = O.ens_ei(outs, fbest)
        # float64 evaluation on both sides: the float32 result differs by its
        # rounding, 2^-24 relative in float32's normal range and half the
        # subnormal spacing (2^-150) below it
        err = np.abs(ei - ref) - 2.0 ** -23 * np.abs(ref)
        j = int(np.argmax(ref))
        z = (fbest - mu_e[j]) / sd_e[j]
        print(f"  prescreen EI f_best={fbest:.3f}: max |dEI| beyond float32 rounding = "
              f"{np.max(err):.2e} (EI_max {np.max(ref):.2e}, z* {z:.1f})")
        assert np.all(err <= 2.0 ** -149), fbest
        want = np.lexsort((np.arange(ei.size), -ei))[:k]
        assert np.array_equal(idx.cpu().numpy(), want), fbest
    net.free()


def test_ens_select_equals_prescreen(ctx):
    """gpbo_ens_select on the member outputs of gpbo_mlp_forward gives the
    prescreen's indices and scores, both rules, sorted and set selections."""
    flat = _init(17)
    net = G.Mlp(ctx, torch.tensor(flat, dtype=torch.float32, device=DEV).contiguous(), E, D, H)
    X, _, _ = _data(20000, seed=18)
    Xd = torch.tensor(X, dtype=torch.float32, device=DEV)
    outs = net.forward(Xd)
    fbest = float(outs.double().mean(0).quantile(0.05))
    for k in (1, 777, 12000):
        i1, s1 = net.prescreen_lcb(Xd, 0.5, k, want_score=True)
        i2, s2 = G.ens_select(ctx, outs, G.SELECT_LCB, 0.5, k, want_score=True)
        assert torch.equal(i1, i2) and torch.equal(s1, s2), k
        i1, e1 = net.prescreen(Xd, fbest, k, want_ei=True)
        i2, e2 = G.ens_select(ctx, outs, G.SELECT_EI, fbest, k, want_score=True)
        assert torch.equal(i1, i2) and torch.equal(e1, e2), k
    with pytest.raises(G.GpboError):
        G.ens_select(ctx, outs, 7, 0.0, 5)
    net.free()


def test_prescreen_lcb_matches_oracle_and_sort(ctx):
    """The LCB score equals the oracle's on the device's member outputs to
    float32 rounding, and the top-k indices equal a sort of the device's own
    float32 scores by (score descending, index ascending)."""
    flat = _init(11)
    net = G.Mlp(ctx, torch.tensor(flat, dtype=torch.float32, device=DEV).contiguous(), E, D, H)
    X, _, _ = _data(20000, seed=12)
    Xd = torch.tensor(X, dtype=torch.float32, device=DEV)
    outs = net.forward(Xd).double().cpu().numpy()
    for kappa, k in ((0.0, 1), (0.5, 777), (2.0, 4096)):
        idx, sc = net.prescreen_lcb(Xd, kappa, k, want_score=True)
        sc = sc.cpu().numpy()
        ref = O.ens_lcb(outs, kappa)
        assert np.max(np.abs(sc - ref)) <= 1e-5 * np.max(np.abs(ref)), kappa
        want = np.lexsort((np.arange(sc.size), -sc.astype(np.float64)))[:k]
        assert np.array_equal(idx.cpu().numpy(), want), kappa
    with pytest.raises(G.GpboError):
        net.prescreen_lcb(Xd, -1.0, 4)
    net.free()


def test_prescreen_gain_over_random_subset(ctx):
    """The trained network's top-k, re-scored by the exact GP, finds a better
    candidate than a random subset of the same size (same re-score cost)."""
    hits_net = hits_rand = hits_lcb = 0
    ratio_net, ratio_rand, ratio_lcb = [], [], []
    for seed in range(3):
        spec = I.spec_grouped(D, 0.1)
        r = np.random.default_rng(100 + seed)
        Xtr = I.f32r(r.uniform(0, 1, (1024, D)))
        ytr = I.synthetic_f(Xtr, spec) + r.normal(0, 0.01, 1024)
        ls = np.exp(r.uniform(math.log(0.05), math.log(1.0), D)) * math.sqrt(D)
        pool = I.f32r(r.uniform(0, 1, (65536, D)))
        # exact GP on 512 of the evaluations, scoring the whole pool
        model = G.fit(ctx, torch.tensor(Xtr[:512], device=DEV), torch.tensor(ytr[:512], device=DEV), ls)
        pool_d = torch.tensor(pool, dtype=torch.float32, device=DEV)
        full = G.score(ctx, model, pool_d, "fp32")["ei"].double().cpu().numpy()
        a_star = int(np.argmax(full))
        # network on all 1024 evaluations (normalised targets)
        yt = ((ytr - ytr.mean()) / ytr.std()).astype(np.float32)
        init = O.mlp_pack(**I.mlp_init(np.random.default_rng(seed), E, D, H))
        net = G.Mlp(ctx, torch.tensor(init, dtype=torch.float32, device=DEV).contiguous(), E, D, H)
        net.train(torch.tensor(Xtr, dtype=torch.float32, device=DEV),
                  torch.tensor(yt, device=DEV), steps=400, lr=1e-3, history=False)
        fb = float(yt.min())
        k = 2048
        idx, _ = net.prescreen(pool_d, fb, k)
        idx = idx.cpu().numpy()
        sub = G.gather_rows(ctx, torch.tensor(idx, device=DEV), pool_d)
        rs = G.score(ctx, model, sub, "fp32")["ei"].double().cpu().numpy()
        b_star = int(idx[np.argmax(rs)])
        idx_l, _ = net.prescreen_lcb(pool_d, 0.0, k)
        idx_l = idx_l.cpu().numpy()
        sub_l = G.gather_rows(ctx, torch.tensor(idx_l, device=DEV), pool_d)
        rs_l = G.score(ctx, model, sub_l, "fp32")["ei"].double().cpu().numpy()
        l_star = int(idx_l[np.argmax(rs_l)])
        ratio_lcb.append(full[l_star] / full[a_star])
        hits_lcb += l_star == a_star
        rnd = np.random.default_rng(200 + seed).choice(65536, k, replace=False)
        r_star = int(rnd[np.argmax(full[rnd])])
        hits_net += b_star == a_star
        hits_rand += r_star == a_star
        ratio_net.append(full[b_star] / full[a_star])
        ratio_rand.append(full[r_star] / full[a_star])
        print(f"  seed {seed}: net EI {full[b_star] / full[a_star]:.3f} (hit {b_star == a_star}), "
              f"net mean {full[l_star] / full[a_star]:.3f} (hit {l_star == a_star}), "
              f"random {full[r_star] / full[a_star]:.3f} (hit {r_star == a_star})")
        net.free()
        model.free()
    assert hits_net >= hits_rand and hits_lcb >= hits_rand
    assert np.mean(ratio_net) > np.mean(ratio_rand)
    assert np.mean(ratio_lcb) > np.mean(ratio_rand)


def test_context_close_frees_live_objects():
    """Closing a context frees the models and networks still alive on it;
    their Python handles are cleared, so later frees are no-ops."""
    c2 = G.Context(0)
    p = I.make_config("c2-s", n=64, m=8, d=4)
    model = G.fit(c2, torch.tensor(p.X, device=DEV), torch.tensor(p.y, device=DEV), p.lengthscale)
    net = G.Mlp(c2, torch.tensor(_init(1, D=4), dtype=torch.float32, device=DEV).contiguous(), E, 4, H)
    c2.close()
    assert model.h is None and net.h is None
    model.free()
    net.free()


def test_train_on_model_equals_explicit_targets(ctx):
    """gpbo_mlp_train_model trains on a fitted model's own observations: the
    same parameters and loss history, bit for bit, as gpbo_mlp_train on X
    cast to float32 and the fit's z-scored y (checked against the oracle's
    normalisation) passed explicitly."""
    p = I.make_config("c4", n=512, m=16)
    X = torch.tensor(p.X, device=DEV)
    y = torch.tensor(p.y, device=DEV)
    model = G.fit(ctx, X, y, p.lengthscale, p.kernel, p.signal_var, p.noise_var)
    s = model.stats()
    f = O.fit(p.X, p.y, p.lengthscale, O.SE, p.signal_var, p.noise_var)
    assert s["ymean"] == pytest.approx(f.ymean, rel=1e-14)
    assert s["ystd"] == pytest.approx(f.ystd, rel=1e-13)
    # the fit's own statistics, applied as the fit applies them
    yt = ((p.y - s["ymean"]) / s["ystd"]).astype(np.float32)
    flat = torch.tensor(_init(21), dtype=torch.float32, device=DEV).contiguous()
    a = G.Mlp(ctx, flat, E, D, H)
    b = G.Mlp(ctx, flat, E, D, H)
    ha = a.train_on_model(model, steps=30, lr=1e-3)
    hb = b.train(torch.tensor(p.X, dtype=torch.float32, device=DEV).contiguous(),
                 torch.tensor(yt, device=DEV), steps=30, lr=1e-3)
    torch.cuda.synchronize()
    assert torch.equal(ha, hb)
    assert torch.equal(a.params(), b.params())
    with pytest.raises(G.GpboError):  # n must be a multiple of 64
        q = I.make_config("c4", n=500, m=16)
        m2 = G.fit(ctx, torch.tensor(q.X, device=DEV), torch.tensor(q.y, device=DEV), q.lengthscale)
        try:
            a.train_on_model(m2, steps=1)
        finally:
            m2.free()
    a.free()
    b.free()
    model.free()
