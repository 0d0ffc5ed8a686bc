"""GPU parity of the batched form (many uneven-n Hamiltonians, one graph).

Each problem of a batch must match the CPU oracle exactly as a single
problem does: max-abs 1e-10 on D in float64 (1e-5 in float32 / bf16x6) at the
problem's own mu, and the oracle's trace at that mu within tolerance.
Graph replays must reproduce the first run bit for bit, and an eager run
(launch timing on) must agree with the graph.  References take the oracle's
Gershgorin bounds; each problem's beta' = beta (e_b - e_a)/2 reported by the
library is checked against them first.
"""
import os
import sys

import numpy as np
import pytest

import synth
from oracle import chebyshev as ch

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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _check_problem(q, lam, D, mu, order, beta, ne, emin_emax, M, tol_d, tol_t):
    emin, emax = emin_emax
    cen, a = ch.scaling(emin, emax)
    c = ch.chebyshev_coeffs(order, beta * a, (mu - cen) / a, M)
    ref = ch.density_from_eigs(q, lam, c, emin, emax)
    err = float(np.max(np.abs(D.cpu().numpy() - ref)))
    t_err = abs(ch.trace_of_series(c, ch.moments_from_eigs(lam, emin, emax, order)) - ne)
    assert err <= tol_d, err
    assert t_err <= tol_t, t_err
    return err, t_err


def _check_beta_scaled(beta_s, beta, lo, hi):
    # the library's beta' carries its own Gershgorin bounds: they must be the oracle's to rounding
    ref = beta * 0.5 * (hi - lo)
    assert abs(beta_s - ref) <= 1e-13 * beta * max(abs(lo), abs(hi)), (beta_s, ref)


def _make(sizes, seed0, law="uniform"):
    probs = [synth.hamiltonian(n, law, seed=seed0 + i) for i, n in enumerate(sizes)]
    return probs, [_dev(h) for h, _, _ in probs]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("bf16x6", 1e-5)])
def test_batch_matches_oracle(cd, handle, prec, tol):
    sizes = [96, 130, 200, 257, 64, 320, 33]
    order, beta = 100, 40.0
    probs, Hs = _make(sizes, 500)
    betas = [beta + 3 * i for i in range(len(sizes))]
    nes = [0.5 * n + (i % 3) for i, n in enumerate(sizes)]
    batch = cd.Batch(handle, sizes, order, cd.make_opts(prec))
    _say(f"batch {prec}: {batch.info()}")
    mu, Ds, status, iters, trace = batch.mu_search(Hs, betas, nes)
    _, _, _, beta_s = batch.stats()
    for p, n in enumerate(sizes):
        h, q, lam = probs[p]
        lo, hi = ch.gershgorin_bounds(h)
        _check_beta_scaled(beta_s[p], betas[p], lo, hi)
        cen, a = ch.scaling(lo, hi)
        M = ch.quadrature_size(order, betas[p] * a)
        assert status[p] == 0, (p, status[p])
        err, t_err = _check_problem(q, lam, Ds[p], mu[p], order, betas[p], nes[p], (lo, hi), M, tol,
                                    1e-9 if prec == "fp64" else 1e-5 * n)
        _say(f"  n={n} mu={mu[p]:.12f} iters={iters[p]} err={err:.2e} t_err={t_err:.2e}")
        assert abs(trace[p] - nes[p]) <= (1e-9 if prec == "fp64" else 1e-5 * n)
    batch.close()


def test_batch_replay_is_bitwise_and_matches_eager(cd, handle):
    sizes = [150, 90, 260]
    probs, Hs = _make(sizes, 900, "gaussmix6")
    betas, nes = [30.0, 50.0, 70.0], [70.0, 40.0, 131.0]
    batch = cd.Batch(handle, sizes, 80)
    mu1, D1, *_ = batch.mu_search(Hs, betas, nes)
    d1 = [d.clone() for d in D1]
    mu2, D2, *_ = batch.mu_search(Hs, betas, nes)          # graph replay
    assert np.array_equal(mu1, mu2)
    for a, b in zip(d1, D2):
        assert torch.equal(a, b)
    cd.chebdm_profile_enable(handle, True)                  # eager run with launch timing
    mu3, D3, *_ = batch.mu_search(Hs, betas, nes)
    prof = cd.chebdm_profile_read(handle)
    cd.chebdm_profile_enable(handle, False)
    assert np.array_equal(mu1, mu3)
    for a, b in zip(d1, D3):
        assert torch.equal(a, b)
    info = batch.info()
    assert prof["gemm_launches"] == info["products_per_problem"]
    assert abs(prof["gemm_flop"] - info["flop_per_run"]) <= 1e-6 * info["flop_per_run"]
    batch.close()


def test_batch_replay_reads_new_inputs(cd, handle):
    # the graph is reused; new pointers, beta and N_e come from the uploaded table
    sizes = [128, 200]
    probs_a, Ha = _make(sizes, 1300)
    probs_b, Hb = _make(sizes, 1400, "gaussmix6")
    batch = cd.Batch(handle, sizes, 64)
    batch.mu_search(Ha, [20.0, 25.0], [60.0, 100.0])
    mu, Ds, status, *_ = batch.mu_search(Hb, [35.0, 45.0], [70.0, 90.0])
    for p, n in enumerate(sizes):
        single_mu, single_D, info = cd.chebdm_mu_search(handle, Hb[p], [35.0, 45.0][p], [70.0, 90.0][p], 64,
                                                        cd.make_opts(baby="sequential"))
        assert abs(single_mu - mu[p]) <= 1e-12 * max(1.0, abs(mu[p]))
        assert float(torch.max(torch.abs(single_D - Ds[p]))) <= 1e-12
    batch.close()


def test_batch_per_problem_errors(cd, handle):
    sizes = [64, 80, 50]
    probs, Hs = _make(sizes, 1500)
    Hs[2] = _dev(0.25 * np.eye(50))                          # scalar H: closed form
    batch = cd.Batch(handle, sizes, 40)
    mu, Ds, status, iters, trace = batch.mu_search(Hs, [10.0, 10.0, 10.0], [30.0, 80.0, 20.0], allow_errors=True)
    assert status[0] == 0
    assert status[1] == -1                                    # N_e = n is outside (0, n)
    assert status[2] == 0
    occ = 20.0 / 50
    assert np.max(np.abs(Ds[2].cpu().numpy() - occ * np.eye(50))) <= 1e-15
    assert abs(1.0 / (1.0 + np.exp(10.0 * (0.25 - mu[2]))) - occ) <= 1e-14
    batch.close()


def test_batch_tuner_and_cache(cd, handle, tmp_path):
    sizes = [96, 300, 600, 900] * 4
    probs, Hs = _make(sizes, 1600)
    batch = cd.Batch(handle, sizes, 64, cd.make_opts("fp32"))
    cache = str(tmp_path / "tune.txt")
    rep = batch.tune(cache)
    _say("tune: " + rep)
    assert "chose" in rep and os.path.exists(cache)
    mu, Ds, status, *_ = batch.mu_search(Hs, [30.0] * 16, [0.5 * n for n in sizes])
    assert np.all(status == 0)
    batch2 = cd.Batch(handle, sizes, 64, cd.make_opts("fp32"))
    rep2 = batch2.tune(cache)
    assert rep2.startswith("loaded")
    mu2, Ds2, *_ = batch2.mu_search(Hs, [30.0] * 16, [0.5 * n for n in sizes])
    assert np.array_equal(mu, mu2)
    batch.close()
    batch2.close()


def test_batch_schedules_agree_bitwise(cd, handle, tmp_path):
    # the tuner's item orders (by decreasing n, input order) only move tiles between
    # work-groups, and its tile edges (64, 48, 32 per size bucket) only regroup the output
    # elements: every element is still summed over K in the same order, so mu and D agree bit
    # for bit.  n = 1020 has no 48-tile grid inside its workspace (ceil(1020/48)*48 > 1024) and
    # keeps 64-tiles; 1000 and 900 take 48-tiles.
    sizes = [96, 300, 600, 900, 130, 257, 1000, 1020] * 2
    probs, Hs = _make(sizes, 1700)
    betas = [30.0 + i for i in range(len(sizes))]
    nes = [0.5 * n for n in sizes]
    cache = str(tmp_path / "tune.txt")
    b0 = cd.Batch(handle, sizes, 64, cd.make_opts("fp32"))
    _say("tune: " + b0.tune(cache))
    b0.close()
    key = open(cache).read().split()[0]
    out = []
    for tiles, order in (("64,64,64,64", 0), ("64,64,64,64", 1), ("48,48,48,48", 0), ("32,32,32,32", 0),
                         ("48,32,64,48", 1)):
        with open(cache, "w") as f:
            f.write(f"{key} tiles={tiles} order={order}\n")
        b = cd.Batch(handle, sizes, 64, cd.make_opts("fp32"))
        rep = b.tune(cache)
        assert rep.startswith("loaded") and f"tiles={tiles} order={order}" in rep, rep
        mu, Ds, status, *_ = b.mu_search(Hs, betas, nes)
        assert np.all(status == 0)
        out.append((np.array(mu), [d.cpu().numpy() for d in Ds]))
        b.close()
    for mu, Ds in out[1:]:
        assert np.array_equal(mu, out[0][0])
        for a, c in zip(Ds, out[0][1]):
            assert np.array_equal(a, c)


def test_batch_512_uneven_workload(cd, handle):
    # 512 problems, n uniform on {96, 128, ..., 1024}, beta on [30, 200], order 256, float32:
    # every problem's bounds (through beta') and electron count against the oracle, and the
    # whole D of 40 problems (the first and last few, the largest and smallest, and a stride)
    sizes, betas = synth.batch_problems(512, seed=3000)
    order = 256
    _say("generating 512 Hamiltonians")
    probs = [synth.hamiltonian(int(n), "uniform", seed=3000 + i) for i, n in enumerate(sizes)]
    Hs = [_dev(h) for h, _, _ in probs]
    nes = [0.5 * n for n in sizes]
    batch = cd.Batch(handle, sizes, order, cd.make_opts("fp32"))
    _say("tune: " + batch.tune())
    mu, Ds, status, iters, trace = batch.mu_search(Hs, betas, nes)
    assert np.all(status == 0), np.unique(status)
    _, _, _, beta_s = batch.stats()
    full = set([0, 1, 2, 3, 508, 509, 510, 511, int(np.argmax(sizes)), int(np.argmin(sizes))])
    full |= set(range(5, 512, 17))
    worst_d, worst_t = 0.0, 0.0
    for p in range(512):
        h, q, lam = probs[p]
        lo, hi = ch.gershgorin_bounds(h)
        _check_beta_scaled(beta_s[p], betas[p], lo, hi)
        cen, a = ch.scaling(lo, hi)
        M = ch.quadrature_size(order, betas[p] * a)
        c = ch.chebyshev_coeffs(order, betas[p] * a, (mu[p] - cen) / a, M)
        t_err = abs(ch.trace_of_series(c, ch.moments_from_eigs(lam, lo, hi, order)) - nes[p])
        assert t_err <= 1e-5 * sizes[p], (p, t_err)
        worst_t = max(worst_t, t_err / sizes[p])
        if p in full:
            ref = ch.density_from_eigs(q, lam, c, lo, hi)
            err = float(np.max(np.abs(Ds[p].cpu().numpy() - ref)))
            assert err <= 1e-5, (p, sizes[p], err)
            worst_d = max(worst_d, err)
    _say(f"  512 problems: worst |t_oracle - Ne|/n = {worst_t:.2e}; whole D of {len(full)} problems, "
         f"worst max|D - D_oracle| = {worst_d:.2e}")
    batch.close()


BF16X3_N512 = ("the three-term split (hi*hi + hi*lo + lo*hi) carries about 16 bits per product; at n = 512, "
               "order 128 (gaussmix6 spectrum) the batched density ends at 1.02e-5, just above the 1e-5 target; "
               "the six-term split meets it there")

SPLIT_SIZES = [96, 130, 200, 257, 64, 320, 33]


@pytest.mark.parametrize("prec,tol,sizes", [
    ("bf16x3", 1e-5, SPLIT_SIZES),
    ("bf16x6", 1e-5, SPLIT_SIZES + [512]),
    pytest.param("bf16x3", 1e-5, SPLIT_SIZES + [512], id="bf16x3-n512",
                 marks=pytest.mark.xfail(strict=True, reason=BF16X3_N512)),
], ids=["bf16x3", "bf16x6", "bf16x3-n512"])
def test_batch_split_bf16_matches_oracle(cd, handle, prec, tol, sizes):
    # the split forms in batched form: same products as the single-problem kernels' tiles
    order, beta = 128, 60.0
    probs, Hs = _make(sizes, 2600, "gaussmix6")
    betas = [beta + 5 * i for i in range(len(sizes))]
    nes = [0.5 * n + 0.5 for n in sizes]
    batch = cd.Batch(handle, sizes, order, cd.make_opts(prec))
    mu, Ds, status, iters, trace = batch.mu_search(Hs, betas, nes)
    _, _, _, beta_s = batch.stats()
    for p, n in enumerate(sizes):
        h, q, lam = probs[p]
        lo, hi = ch.gershgorin_bounds(h)
        _check_beta_scaled(beta_s[p], betas[p], lo, hi)
        cen, a = ch.scaling(lo, hi)
        M = ch.quadrature_size(order, betas[p] * a)
        assert status[p] == 0, (p, status[p])
        err, t_err = _check_problem(q, lam, Ds[p], mu[p], order, betas[p], nes[p], (lo, hi), M, tol, 1e-5 * n)
        _say(f"  {prec} n={n} err={err:.2e} t_err={t_err:.2e}")
    batch.close()


def test_batch_jackson_damping_matches_oracle(cd, handle):
    sizes = [100, 170]
    order, betas, nes = 96, [40.0, 55.0], [49.5, 80.5]
    probs, Hs = _make(sizes, 2100)
    batch = cd.Batch(handle, sizes, order, cd.make_opts("fp64", damping="jackson"))
    mu, Ds, status, iters, trace = batch.mu_search(Hs, betas, nes)
    for p, n in enumerate(sizes):
        h, q, lam = probs[p]
        lo, hi = ch.gershgorin_bounds(h)
        cen, a = ch.scaling(lo, hi)
        M = ch.quadrature_size(order, betas[p] * a)
        c = ch.chebyshev_coeffs(order, betas[p] * a, (mu[p] - cen) / a, M, "jackson")
        ref = ch.density_from_eigs(q, lam, c, lo, hi)
        assert float(np.max(np.abs(Ds[p].cpu().numpy() - ref))) <= 1e-10
        assert abs(ch.trace_of_series(c, ch.moments_from_eigs(lam, lo, hi, order)) - nes[p]) <= 1e-9
    batch.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_batch_lanczos_bounds_match_single_and_oracle(cd, handle, prec, tol):
    # per-problem Lanczos bounds inside the batch graph: the same kernels as the single-problem
    # call (so the same bounds bit for bit), then every problem held to the oracle at them
    sizes = [33, 96, 257, 600, 130, 5]
    order = 128
    laws = ["uniform", "gaussmix6", "highdos"]
    probs = [synth.hamiltonian(n, laws[i % 3], seed=900 + i) for i, n in enumerate(sizes)]
    Hs = [_dev(h) for h, _, _ in probs]
    betas = [30.0 + 10 * i for i in range(len(sizes))]
    nes = [0.5 * n + 0.5 for n in sizes]
    batch = cd.Batch(handle, sizes, order, cd.make_opts(prec, bounds="lanczos"))
    mu, Ds, status, iters, trace = batch.mu_search(Hs, betas, nes)
    _, _, _, beta_s = batch.stats()
    for p, n in enumerate(sizes):
        h, q, lam = probs[p]
        lo, hi, _, _ = cd.chebdm_bounds_lanczos(handle, Hs[p], 40, 0.01, 0)
        rlo, rhi, _, _ = ch.lanczos_bounds(h, 40, 0.01, 0)
        scale = max(abs(rlo), abs(rhi))
        assert abs(lo - rlo) <= 1e-10 * scale and abs(hi - rhi) <= 1e-10 * scale
        assert beta_s[p] == betas[p] * (0.5 * (hi - lo)), (p, beta_s[p], betas[p] * 0.5 * (hi - lo))
        assert status[p] == 0, (p, status[p])
        cen, a = ch.scaling(rlo, rhi)                       # the reference takes the oracle's bounds
        M = ch.quadrature_size(order, betas[p] * a)
        err, t_err = _check_problem(q, lam, Ds[p], mu[p], order, betas[p], nes[p], (rlo, rhi), M, tol,
                                    1e-9 if prec == "fp64" else 1e-5 * n)
        _say(f"  p={p} n={n} [{lo:.4f}, {hi:.4f}] err={err:.1e} t_err={t_err:.1e}")
    batch.close()


def test_batch_rejects_unsupported_options(cd, handle):
    for kw in ({"giant": "power"}, {"giant": "two_chains"}, {"n_quad": 4096}):
        with pytest.raises(cd.ChebdmError) as e:
            cd.Batch(handle, [64, 80], 32, cd.make_opts("fp64", **kw))
        assert e.value.code == -6, kw
    with pytest.raises(cd.ChebdmError) as e:
        cd.Batch(handle, [64, 80], 32, cd.make_opts("fp64", bounds="lanczos", lanczos_steps=200))
    assert e.value.code == -1
