"""GPU tests of the learned chemical-potential start (network kernels and the batched search).

Kernel parity: forward, backward and Adam of the library against the FP64
oracle in ``oracle/mlp.py`` on the same float32-rounded weights and inputs
(relative 1e-4 per parameter block; float32 accumulation over at most 256
terms bounds the rounding well below that).

Search: the batched run with Newton or with the network's bracket must land
on the same mu as bisection within the electron-count tolerance, every
problem's |t - N_e| must stay <= 1e-8, a useless network must fall back to
bisection and still converge, and a trained network must cut the number of
trace evaluations against plain bisection.
"""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import chebyshev as ch
from oracle import mlp as om

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_12616_amd as chebdm

    chebdm.load_library()
    return chebdm


@pytest.fixture(scope="module")
def handle(cd):
    h = cd.Handle(0)
    yield h
    h.close()


def _blocks(g):
    W1, b1, W2, b2, w3, b3 = om.unpack(g)
    return {"W1": W1, "b1": b1, "W2": W2, "b2": b2, "w3": w3, "b3": b3}


def _params32(seed):
    rng = np.random.default_rng(seed)
    w = om.init_params(seed)
    w[om.H1 * om.IN: om.H1 * om.IN + om.H1] = rng.normal(0, 0.1, om.H1)
    o2 = om.H1 * om.IN + om.H1 + om.H2 * om.H1
    w[o2: o2 + om.H2] = rng.normal(0, 0.1, om.H2)
    w[-1] = 0.05
    return w.astype(np.float32)


@pytest.mark.parametrize("batch", [1, 37, 300])
def test_forward_backward_match_oracle(cd, handle, batch):
    rng = np.random.default_rng(batch)
    w32 = _params32(7)
    X32 = rng.normal(0, 1, (batch, 64)).astype(np.float32)
    T32 = rng.normal(0, 0.2, batch).astype(np.float32)
    W, X, T = (torch.from_numpy(a).cuda() for a in (w32, X32, T32))
    y = cd.chebdm_mlp_forward(handle, W, X).cpu().numpy()
    y_ref, _ = om.forward(w32.astype(np.float64), X32.astype(np.float64))
    scale = max(1.0, float(np.max(np.abs(y_ref))))
    assert np.max(np.abs(y - y_ref)) <= 1e-5 * scale, np.max(np.abs(y - y_ref))
    g, loss = cd.chebdm_mlp_backward(handle, W, X, T)
    L_ref, g_ref = om.backward(w32.astype(np.float64), X32.astype(np.float64), T32.astype(np.float64))
    assert abs(loss - L_ref) <= 1e-5 * max(L_ref, 1e-30), (loss, L_ref)
    gd, gr = _blocks(g.cpu().numpy().astype(np.float64)), _blocks(g_ref)
    for name in gr:
        err = float(np.max(np.abs(gd[name] - gr[name])))
        ref = float(np.max(np.abs(gr[name])))
        _say(f"  batch={batch} {name}: max|g|={ref:.3e} err={err:.2e}")
        assert err <= 1e-4 * ref + 1e-12, (name, err, ref)


def test_adam_matches_oracle(cd, handle):
    rng = np.random.default_rng(3)
    n = cd.chebdm_mlp_num_params()
    w = _params32(1)
    m = (rng.normal(0, 1e-3, n)).astype(np.float32)
    v = (rng.uniform(0, 1e-5, n)).astype(np.float32)
    g = rng.normal(0, 1e-2, n).astype(np.float32)
    W, M, V, G = (torch.from_numpy(a.copy()).cuda() for a in (w, m, v, g))
    cd.chebdm_mlp_adam(handle, W, G, M, V, 3, lr=2e-3, beta1=0.9, beta2=0.99, eps=1e-8)
    w_ref, m_ref, v_ref = om.adam_step(w.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                                       v.astype(np.float64), 3, lr=2e-3, b1=0.9, b2=0.99, eps=1e-8)
    assert np.max(np.abs(M.cpu().numpy() - m_ref)) <= 1e-6 * np.max(np.abs(m_ref))
    assert np.max(np.abs(V.cpu().numpy() - v_ref)) <= 1e-6 * np.max(np.abs(v_ref))
    step = w_ref - w.astype(np.float64)
    assert np.max(np.abs((W.cpu().numpy().astype(np.float64) - w) - step)) <= 1e-3 * np.max(np.abs(step))


def test_training_lowers_loss(cd, handle):
    from paper_2306_12616_amd.learned_mu import MuNet

    rng = np.random.default_rng(11)
    X = rng.uniform(-1, 1, (2048, 64)).astype(np.float32)
    T = (0.3 * X[:, 0] - 0.2 * X[:, 1] * X[:, 2] + 0.1 * np.abs(X[:, 3])).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    net = MuNet(handle, seed=2)
    before = net.loss(Xd, Td)
    hist = net.train(Xd, Td, epochs=30, batch=128, lr=2e-3)
    after = net.loss(Xd, Td)
    _say(f"  loss {before:.3e} -> {after:.3e}")
    assert after < 0.05 * before
    assert hist[-1] < hist[0]


def test_checkpoint_roundtrip(cd, handle, tmp_path):
    from paper_2306_12616_amd.learned_mu import MuNet

    rng = np.random.default_rng(5)
    X = torch.from_numpy(rng.normal(0, 1, (64, 64)).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.normal(0, 1, 64).astype(np.float32)).cuda()
    net = MuNet(handle, seed=4)
    net.train(X, T, epochs=2, batch=16)
    path = str(tmp_path / "net")
    net.save(path, note="test")
    back = MuNet.load(handle, path)
    assert back.step == net.step and back.meta["note"] == "test"
    for a, b in ((net.W, back.W), (net.M, back.M), (net.V, back.V)):
        assert torch.equal(a, b)
    # resuming gives the same next step as continuing
    net.train(X, T, epochs=1, batch=16, seed=9)
    back.train(X, T, epochs=1, batch=16, seed=9)
    assert torch.equal(net.W, back.W)


def test_newton_and_fallback_agree_with_bisection(cd, handle):
    sizes = np.random.default_rng(21).integers(64, 301, size=48)
    Hs, lams, betas, nes = synth.mu_problems(sizes, seed=21)
    batch = cd.Batch(handle, sizes, 128)
    mu0, st0, it0, t0 = batch.mu_only(Hs, betas, nes)
    ev0, *_ = batch.stats()
    batch.set_search("newton")
    mu1, st1, it1, t1 = batch.mu_only(Hs, betas, nes)
    ev1, *_ = batch.stats()
    # a useless network: every guess far off, so every problem takes the fallback
    n = cd.chebdm_mlp_num_params()
    W = torch.zeros(n, dtype=torch.float32, device="cuda")
    W[-1] = 5.0
    batch.set_search("learned", W, delta=0.01)
    mu2, st2, it2, t2 = batch.mu_only(Hs, betas, nes)
    ev2, learned2, *_ = batch.stats()
    assert np.all(st0 == 0) and np.all(st1 == 0) and np.all(st2 == 0)
    # the guess clamps to mu~ = 1, where the Newton step is undefined or leaves [-1, 1]: the
    # fallback bisects on [-1, 1] with t(1) already evaluated, i.e. exactly the plain bisection
    assert not learned2.any()
    assert np.array_equal(mu2, mu0) and np.array_equal(ev2, ev0)
    for mu, t in ((mu0, t0), (mu1, t1), (mu2, t2)):
        assert np.max(np.abs(t - np.array(nes))) <= 1e-8
    _say(f"  evals bisection {ev0.mean():.1f} newton {ev1.mean():.1f} fallback {ev2.mean():.1f}")
    # the same chemical potential to within what the count tolerance allows
    assert np.max(np.abs(mu1 - mu0)) <= 1e-6
    # oracle check of the electron count on three problems
    for p in (0, 17, 47):
        h = Hs[p].cpu().numpy()
        lo, hi = ch.gershgorin_bounds(h)
        cen, a = ch.scaling(lo, hi)
        M = ch.quadrature_size(128, betas[p] * a)
        c = ch.chebyshev_coeffs(128, betas[p] * a, (mu1[p] - cen) / a, M)
        t_or = ch.trace_of_series(c, ch.moments_from_eigs(lams[p], lo, hi, 128))
        assert abs(t_or - nes[p]) <= 1e-8, (p, t_or, nes[p])
    batch.close()


def test_learned_start_beats_newton(cd, handle, tmp_path):
    # training set: method-generated (bisection) targets, N in 64..512, N_e / N in [0.3, 0.7], order 256
    from paper_2306_12616_amd.learned_mu import MuNet, collect_samples, delta_from_residuals, search_report

    t_start = time.time()
    order, chunk, chunks = 256, 1024, 16
    sizes0 = synth.mu_training_sizes(chunk)
    plan = cd.Batch(handle, sizes0, order)

    def draw(c):
        Hs, _, betas, nes = synth.mu_problems(sizes0, seed=200 + c)
        return Hs, betas, nes

    X, T = collect_samples(plan, draw, chunks, log=lambda m: _say(f"  {m}, {time.time() - t_start:.1f} s"))
    plan.close()
    nval = 1024
    net = MuNet(handle, seed=0)
    net.train(X[nval:], T[nval:], epochs=120, batch=256, lr=1e-3)
    res = (net.predict(X[:nval]) - T[:nval]).cpu().numpy()
    delta = delta_from_residuals(res)
    _say(f"  validation rms {np.sqrt(np.mean(res ** 2)):.2e}, delta {delta:.2e}, {time.time() - t_start:.1f} s")
    net.save(str(tmp_path / "mu_net"), delta=delta)

    # evaluation: 1024 problems at N = 500
    count = 1024
    Hs, _, betas, nes = synth.mu_problems([500] * count, seed=7)
    ev = cd.Batch(handle, [500] * count, order)
    rep, mus = {}, {}
    for mode in ("bisection", "newton", "learned"):
        if mode == "learned":
            ev.set_search(mode, net.W, delta)
        else:
            ev.set_search(mode)
        ev.mu_only(Hs, betas, nes, allow_errors=True)                   # captures the graph
        cd.chebdm_profile_enable(handle, True)
        mu, status, iters, t = ev.mu_only(Hs, betas, nes, allow_errors=True)   # eager, launch-timed
        prof = cd.chebdm_profile_read(handle)
        cd.chebdm_profile_enable(handle, False)
        rep[mode] = search_report(ev, status, iters, t, nes)
        rep[mode]["search_ms"] = round(prof["search_ms"], 3)
        mus[mode] = mu
        _say(f"  {mode}: {rep[mode]}")
        assert rep[mode]["converged"] == count
        assert rep[mode]["max_count_err"] <= 1e-8
    # the gain is measured against the best search without the network (safeguarded Newton
    # from mu~ = 0 after the bracket check at -1 and 1), not only against bisection
    assert rep["learned"]["mean_evals"] <= 0.6 * rep["newton"]["mean_evals"]
    # search-phase time: the per-problem DCT-III of the moments, which every mode runs once, and
    # (learned) the network's forward pass take most of it, so the saved evaluations show as
    # parity in milliseconds rather than a gain; the learned start must not cost more than 10 %
    assert rep["learned"]["search_ms"] <= 1.1 * rep["newton"]["search_ms"]
    assert rep["learned"]["learned_share"] >= 0.9
    assert np.max(np.abs(mus["learned"] - mus["bisection"])) <= 1e-6
    ev.close()


def test_batch_features_match_oracle(cd, handle):
    # the network inputs the device assembles (float32) against the oracle's moments
    sizes = [96, 130, 257]
    order, betas, nes = 128, [30.0, 60.0, 90.0], [40.5, 70.5, 120.5]
    probs = [synth.hamiltonian(n, "gaussmix6", seed=70 + i) for i, n in enumerate(sizes)]
    Hs = [torch.from_numpy(h).cuda() for h, _, _ in probs]
    batch = cd.Batch(handle, sizes, order)
    batch.mu_only(Hs, betas, nes)
    X = batch.features().cpu().numpy()
    _, _, _, beta_s = batch.stats()
    for p, n in enumerate(sizes):
        h, q, lam = probs[p]
        lo, hi = ch.gershgorin_bounds(h)
        cen, a = ch.scaling(lo, hi)
        tau = ch.moments_from_eigs(lam, lo, hi, order)
        ref = om.features(tau, [n], [nes[p]], [betas[p] * a])[0]
        assert abs(beta_s[p] - betas[p] * a) <= 1e-12 * betas[p] * a
        assert np.max(np.abs(X[p] - ref)) <= 1e-6 * max(1.0, float(np.max(np.abs(ref)))), (p, np.max(np.abs(X[p] - ref)))
    batch.close()
