"""Boundary behaviour of the scoring entry points through the C ABI: the
float32 path's escalation to float64 arithmetic on an ill-conditioned K
(decided on the host after a synchronous fit, on the device after an
asynchronous one), argmax and EI maximum written to host memory (the call
synchronises), and the GPBO_DEBUG check of candidate pools for non-finite
values.

Bars: float32 path |dmu| / max(|mu|, s_y sf) and |dsigma| / sigma <= 1e-4
(R9) and the argmax per R8, against the float64 oracle; host and device
outputs of the same call identical.
"""
import math
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2403_08131_amd import gpbo as G
from paper_2403_08131_amd import inputs as I

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def ctx():
    c = G.Context(0)
    yield c
    c.close()


def _t(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


def _ill_conditioned():
    # two dimensions, 193 points, literal lengthscales: cond(K) ~ 1.5e6; the
    # float32 path without escalation misses the mean by ~1e-2 here
    return I.make_c3(lam=0.5, replicate=0, scaled=False, B=64, m=8192)[47]


def _errs(ref, out, f, sf2):
    mu = out["mu"].double().cpu().numpy()
    sg = out["sigma"].double().cpu().numpy()
    scale = f.ystd * math.sqrt(sf2)
    e_mu = np.max(np.abs(mu - ref["mu"]) / np.maximum(np.abs(ref["mu"]), scale))
    floor = ref["sigma"] ** 2 >= 1e-2 * scale ** 2
    e_sg = np.max(np.abs(sg - ref["sigma"])[floor] / ref["sigma"][floor]) if floor.any() else 0.0
    return e_mu, e_sg


def _argmax_ok(ref_ei, am, bound=1e-4):
    srt = np.sort(ref_ei)[::-1]
    if srt[0] - srt[1] > bound * srt[0]:
        return am == O.argmax(ref_ei)
    return ref_ei[am] >= srt[0] * (1 - bound)


def test_fp32_escalates_ill_conditioned_model(ctx):
    p = _ill_conditioned()
    f = O.fit(p.X, p.y, p.lengthscale, O.SE, p.signal_var, p.noise_var)
    ref = O.score(f, p.Xc)
    Xc = _t(p.Xc, torch.float32)
    args = (_t(p.X), _t(p.y), p.lengthscale, p.kernel, p.signal_var, p.noise_var)
    m_sync = G.fit(ctx, *args)
    kinv = m_sync.stats()["kinv"]
    K = O.gram(O.SE, p.X, p.lengthscale, p.signal_var, p.noise_var)
    assert kinv == pytest.approx(p.signal_var * np.trace(np.linalg.inv(K)) / p.n, rel=1e-6)
    assert kinv > G.ESCALATE_KINV
    out_h = G.score(ctx, m_sync, Xc, "fp32")          # escalation decided on the host
    m_async = G.fit_async(ctx, *args)
    out_d = G.score(ctx, m_async, Xc, "fp32")         # ... on the device
    m_async.status()
    torch.cuda.synchronize()
    for out in (out_h, out_d):
        e_mu, e_sg = _errs(ref, out, f, p.signal_var)
        print(f"escalated fp32: e_mu={e_mu:.2e} e_sigma={e_sg:.2e}")
        assert e_mu <= 1e-4 and e_sg <= 1e-4
        assert _argmax_ok(ref["ei"], int(out["argmax"].item()))
    for k in ("mu", "sigma", "ei", "argmax", "ei_max"):
        assert torch.equal(out_h[k], out_d[k]), k
    m_sync.free()
    m_async.free()


def test_fp32_well_conditioned_model_stays_float32(ctx):
    """A well-conditioned model (c2-s shape, n = 300) is below the threshold
    on both paths, and the device-side decision gives the host-side result."""
    p = I.make_config("c2-s", n=300, m=3000)
    args = (_t(p.X), _t(p.y), p.lengthscale, p.kernel, p.signal_var, p.noise_var)
    m_sync = G.fit(ctx, *args)
    assert m_sync.stats()["kinv"] < G.ESCALATE_KINV
    Xc = _t(p.Xc, torch.float32)
    out_h = G.score(ctx, m_sync, Xc, "fp32")
    m_async = G.fit_async(ctx, *args)
    out_d = G.score(ctx, m_async, Xc, "fp32")
    m_async.status()
    torch.cuda.synchronize()
    for k in ("mu", "sigma", "ei", "argmax", "ei_max"):
        assert torch.equal(out_h[k], out_d[k]), k
    f = O.fit(p.X, p.y, p.lengthscale, O.SE, p.signal_var, p.noise_var)
    ref = O.score(f, p.Xc)
    e_mu, e_sg = _errs(ref, out_h, f, p.signal_var)
    assert e_mu <= 1e-4 and e_sg <= 1e-4
    m_sync.free()
    m_async.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_score_argmax_to_host_memory(ctx, prec):
    p = I.make_c1(m=3001)
    m = G.fit(ctx, _t(p.X), _t(p.y), p.lengthscale, p.kernel, p.signal_var, p.noise_var)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xc = _t(p.Xc, dt)
    dev = G.score(ctx, m, Xc, prec)
    host = G.score(ctx, m, Xc, prec, host_argmax=True)  # returns after the stream has run
    assert isinstance(host["argmax"], int) and isinstance(host["ei_max"], float)
    assert host["argmax"] == int(dev["argmax"].item())
    assert host["ei_max"] == float(dev["ei_max"].item())
    assert float(host["ei"][host["argmax"]]) == float(host["ei"].max())
    # an empty pool: index -1 and -inf
    empty = G.score(ctx, m, Xc[:0], prec, host_argmax=True)
    assert empty["argmax"] == -1 and empty["ei_max"] == -math.inf
    m.free()


def test_score_batched_argmax_to_host_memory(ctx):
    probs = I.make_c3(lam=0.1, replicate=2, scaled=True, B=5, m=900)
    specs = [dict(X=_t(q.X), y=_t(q.y), lengthscale=q.lengthscale, kernel=q.kernel,
                  signal_var=q.signal_var, noise_var=q.noise_var) for q in probs]
    st, models, _, _ = G.fit_batched(ctx, specs)
    assert st == G.OK
    Xcs = [_t(q.Xc, torch.float32) for q in probs]
    outs_d, am_d, em_d = G.score_batched(ctx, models, Xcs, "fp32")
    outs_h, am_h, em_h = G.score_batched(ctx, models, Xcs, "fp32", host_argmax=True)
    assert isinstance(am_h, np.ndarray)
    assert np.array_equal(am_h, am_d.cpu().numpy())
    assert np.array_equal(em_h, em_d.cpu().numpy())
    for mo in models:
        mo.free()


def test_debug_rejects_non_finite_pool():
    os.environ["GPBO_DEBUG"] = "1"
    try:
        dctx = G.Context(0)
    finally:
        del os.environ["GPBO_DEBUG"]
    p = I.make_c1(m=500)
    m = G.fit(dctx, _t(p.X), _t(p.y), p.lengthscale, p.kernel, p.signal_var, p.noise_var)
    for prec, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        Xc = _t(p.Xc, dt)
        G.score(dctx, m, Xc, prec)  # finite: accepted
        for bad in (float("nan"), float("inf")):
            Xb = Xc.clone()
            Xb[123, 4] = bad
            with pytest.raises(G.GpboError) as e:
                G.score(dctx, m, Xb, prec)
            assert e.value.status == G.E_NONFINITE
    probs = I.make_c3(lam=0.0, replicate=1, scaled=True, B=3, m=300)
    specs = [dict(X=_t(q.X), y=_t(q.y), lengthscale=q.lengthscale, kernel=q.kernel,
                  signal_var=q.signal_var, noise_var=q.noise_var) for q in probs]
    st, models, _, _ = G.fit_batched(dctx, specs)
    Xcs = [_t(q.Xc, torch.float32) for q in probs]
    G.score_batched(dctx, models, Xcs, "bf16")
    Xcs[1][7, 0] = float("nan")
    with pytest.raises(G.GpboError) as e:
        G.score_batched(dctx, models, Xcs, "bf16")
    assert e.value.status == G.E_NONFINITE
    for mo in models + [m]:
        mo.free()
    dctx.close()


def _overwrite_freed_memory():
    # allocations on the current stream of the sizes the freed buffers came
    # in (the caching allocator hands freed blocks out again at once),
    # filled with NaN
    junk = []
    for mb in (16, 8, 4, 2, 1, 0.5, 0.25, 0.125):
        for _ in range(4):
            junk.append(torch.full((int(mb * 262144),), float("nan"), dtype=torch.float32, device=DEV))
    return junk


def _two_streams():
    s1 = torch.cuda.Stream(device=DEV)
    s2 = torch.cuda.Stream(device=DEV)
    return s1, s2


def test_model_freed_after_scoring_on_another_stream():
    """A model fitted and scored on stream S1, scored again on S2 (a
    2^20-candidate pool: milliseconds of work), the context moved back to S1
    and the model freed at once: the free waits for the device, so S2's
    scoring reads intact buffers although the freed memory is handed out
    again on S1 and overwritten straight away.  The S2 outputs equal the S1
    ones bit for bit."""
    s1, s2 = _two_streams()
    prev = torch.cuda.current_stream(DEV)
    torch.cuda.set_stream(s1)
    c = G.Context(0)
    try:
        p = I.make_config("c2", replicate=0)
        rng = np.random.default_rng(31)
        Xc = torch.tensor(rng.uniform(size=(1 << 20, p.d)), dtype=torch.float32, device=DEV)
        m = G.fit(c, _t(p.X), _t(p.y), p.lengthscale, p.kernel, p.signal_var, p.noise_var)
        ref = G.score(c, m, Xc, "fp32")
        torch.cuda.synchronize()
        print("score on S2, free on S1", flush=True)
        with torch.cuda.stream(s2):
            c.sync_stream()
            out = G.score(c, m, Xc, "fp32")
        c.sync_stream()  # back on S1
        m.free()
        junk = _overwrite_freed_memory()
        torch.cuda.synchronize()
        for k in ("mu", "sigma", "ei"):
            assert torch.equal(out[k], ref[k]), k
        assert out["argmax"].item() == ref["argmax"].item()
        del junk
    finally:
        c.close()
        torch.cuda.set_stream(prev)


def test_network_freed_after_forward_on_another_stream():
    """The same for a network: created and run on S1, run again on S2 over
    2^20 candidates, freed on S1 at once; the S2 outputs equal the S1 ones."""
    s1, s2 = _two_streams()
    prev = torch.cuda.current_stream(DEV)
    torch.cuda.set_stream(s1)
    c = G.Context(0)
    try:
        E, D, H = 5, 20, 256
        init = I.mlp_init(np.random.default_rng(33), members=E, d_in=D, hidden=H)
        net = G.Mlp(c, G.Mlp.pack(**init, device=DEV), E, D, H)
        rng = np.random.default_rng(34)
        Xc = torch.tensor(rng.uniform(size=(1 << 20, D)), dtype=torch.float32, device=DEV)
        ref = net.forward(Xc)
        torch.cuda.synchronize()
        print("forward on S2, free on S1", flush=True)
        with torch.cuda.stream(s2):
            c.sync_stream()
            out = net.forward(Xc)
        c.sync_stream()
        net.free()
        junk = _overwrite_freed_memory()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        del junk
    finally:
        c.close()
        torch.cuda.set_stream(prev)
