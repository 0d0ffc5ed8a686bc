#!/usr/bin/env python3
"""Throughput of the dense Chebyshev density-matrix path on one MI355X.

One step = one pass of the whole hot path on a resident Hamiltonian:
Gershgorin bounds -> H~ -> baby steps -> ladder + Gram moments -> mu
bisection -> coefficients -> block sums -> giant steps -> D and tr D
(``chebdm_mu_search`` with a density output).  Default workload: N = 4000,
order 512, beta = 100, N_e = N/2, H = Q diag(lam) Q^T with lam from a
six-Gaussian mixture (synthetic stand-in for the paper's model Hamiltonians).

Prints one JSON line (stdout); progress goes to stderr.  ``roofline`` is the
matrix-product kernel's algorithmic rate from HIP events recorded by the
library on its own stream over the timed steps; ``cpu_baseline`` times the
CPU oracle (LAPACK eigh route) on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "density matrices/s and % MFMA peak at N=1000/4000 vs plain FP64 path"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0}   # dense MFMA peaks of MI355X
PEAK_HBM_GBS = 8000.0
SEEDS = {1000: 2000, 2000: 2001, 4000: 2002}   # gaussmix6 workloads at order 512
ALL_SECTIONS = ("breakdown", "fixed", "config", "lanczos", "accuracy", "diag", "batch", "learned")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class Inputs:
    """Seeded Hamiltonians, drawn once per (n, law, seed): the host copy with the generator's
    eigenpairs (kept for the oracle check after the timed work) and a resident device copy."""

    def __init__(self):
        self.host = {}
        self.dev = {}

    def get(self, n, law, seed):
        import torch

        import synth

        key = (int(n), law, int(seed))
        if key not in self.dev:
            log(f"generating H: n={n} law={law} seed={seed}")
            self.host[key] = synth.hamiltonian(int(n), law, seed=int(seed))
            self.dev[key] = torch.from_numpy(self.host[key][0]).to("cuda:0")
        return self.dev[key]

    def drop_device(self):
        self.dev.clear()


def band_rows(n, band=64):
    """One row per 64-row band (tile row of the product grid), plus the first and last rows."""
    rows = {0, n - 1}
    for b, start in enumerate(range(0, n, band)):
        stop = min(start + band, n)
        rows.add(start + (b % 3) * (stop - 1 - start) // 2)
    return sorted(rows)


def check_record(row, key, order, beta, n_elec, mu, info, D):
    """What the oracle check after the timed region needs: the sampled rows of D (host), mu and
    the library's bounds; the error fields are written into `row` by attach_oracle_errors."""
    rows = band_rows(key[0])
    d_rows = D[rows].cpu().numpy() if D is not None else None
    return {"row": row, "key": key, "order": order, "beta": beta, "n_elec": n_elec, "mu": mu,
            "rows": rows, "d_rows": d_rows, "emin": info["emin"], "emax": info["emax"], "n_quad": info["n_quad"]}


def timed(call, steps, warmup, cd=None, handle=None):
    """Wall time of `steps` calls after `warmup` untimed ones, bracketed by device syncs.

    With cd/handle given, the same number of calls is then repeated with the library's launch
    timing on (HIP events on its stream around every product / block-sum / Gram / search
    launch; that runs each call eagerly instead of replaying its graph) and those per-phase
    timings are returned too.  The throughput comes from the first, uninstrumented pass.
    """
    import torch

    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = call()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = None
    if cd is not None:
        cd.chebdm_profile_enable(handle, True)
        torch.cuda.synchronize()
        for _ in range(steps):
            call()
        prof = cd.chebdm_profile_read(handle)
        cd.chebdm_profile_enable(handle, False)
    return dt, prof, out


def run_steps(cd, handle, H, beta, n_elec, order, opts, steps, warmup, want_density=True, with_out=False):
    import torch

    D = torch.empty_like(H) if want_density else None
    dt, prof, out = timed(lambda: cd.chebdm_mu_search(handle, H, beta, n_elec, order, opts,
                                                      want_density=want_density, D=D),
                          steps, warmup, cd, handle)
    if with_out:
        return dt, prof, out[2], out[0], D
    return dt, prof, out[2]


def mu_search_row(cd, handle, inputs, key, beta, order, prec, search="bisection", steps=5, warmup=2):
    """Timed mu search + density on one resident workload: the row and its oracle-check record."""
    n = key[0]
    H = inputs.get(*key)
    dt, prof, info, mu, D = run_steps(cd, handle, H, beta, n / 2.0, order, cd.make_opts(prec, search=search),
                                      steps, warmup, with_out=True)
    r = roofline_of(prof, prec)
    row = {"dm_per_s": round(steps / dt, 3), "ms_per_step": round(1e3 * dt / steps, 3),
           "gemm_frac_of_peak": r["frac"] if r else None, "gemm_tflops": r["achieved"] if r else None,
           "search_ms": round(prof["search_ms"] / steps, 3), "search_evals": info["iters"],
           "products": info["n_gemm"], "status": info["status"]}
    return row, check_record(row, key, order, beta, n / 2.0, mu, info, D)


# what the product kernels are built from: their code, and the compile flags build.py gives
# k_gemm.hip (without the include paths, which name the checkout)
GEMM_SOURCES = ("paper_2306_12616_amd/csrc/gemm_tile.h", "paper_2306_12616_amd/csrc/gemm_lds.h",
                "paper_2306_12616_amd/csrc/k_gemm.hip")


def gemm_sources_sha256():
    import hashlib

    from paper_2306_12616_amd import build as pkg_build

    h = hashlib.sha256()
    for rel in GEMM_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    flags = [f for i, f in enumerate(pkg_build.FLAGS)
             if f != "-I" and not (i > 0 and pkg_build.FLAGS[i - 1] == "-I")]
    if "k_gemm.hip" not in pkg_build.NO_VGPR_FORM:
        flags += list(pkg_build.VGPR_FORM)
    h.update(" ".join(flags).encode())
    return h.hexdigest()


def traffic_of(prec, n, order):
    """HBM bytes per product-kernel launch from the committed counter summary, if it still applies.

    The summary (``profiles/traffic_k_gemm_<prec>_n<n>_order<order>.txt``) holds a line
    ``traffic-json: {...}`` written from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of
    ``bench.py --copy-probe-mib``; it is used only while the product kernel's sources hash to
    the recorded value (otherwise the counters describe another kernel and traffic is null).
    """
    path = os.path.join(ROOT, "profiles", f"traffic_k_gemm_{prec}_n{n}_order{order}.txt")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic-json:"):
                rec = json.loads(line.split(":", 1)[1])
                if rec.get("kernel_sources_sha256") == gemm_sources_sha256():
                    return rec.get("bytes_per_launch")
    return None


def run_density_steps(cd, handle, H, beta, mu, order, opts, steps, warmup):
    """Density at a given mu (no moments, no search): chebdm_density on a resident H."""
    import torch

    D = torch.empty_like(H)
    dt, prof, _ = timed(lambda: cd.chebdm_density(handle, H, beta, mu, order, opts, D=D), steps, warmup, cd, handle)
    return dt, prof


def roofline_of(prof, prec):
    """Matrix-product kernel: algorithmic flops / summed launch time vs the MFMA peak."""
    if prof["gemm_ms"] <= 0:
        return None
    flop = prof["gemm_flop"] * {"bf16x3": 3.0, "bf16x6": 6.0}.get(prec, 1.0)   # bf16 products per split product
    achieved = flop / (prof["gemm_ms"] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": None,
            "kernel": "k_gemm (symmetric product, fused epilogue)",
            "launches": prof["gemm_launches"], "products": prof["gemm_products"],
            "avg_launch_ms": round(prof["gemm_ms"] / max(1, prof["gemm_launches"]), 4)}


def hbm_of(ms, nbytes):
    if ms <= 0:
        return None
    return round(nbytes / (ms * 1e-3) / 1e9, 1)


def cpu_baseline(h_np, beta, n_elec, order, reps=5, budget_s=30.0):
    """The oracle's whole path on the host cores: one untimed warm-up, then the median of `reps`
    timed runs (fewer if they would exceed the budget)."""
    import statistics

    from oracle import chebyshev as ch

    try:
        from threadpoolctl import threadpool_info

        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    ch.mu_search_density(h_np, beta, n_elec, order)
    t_warm = time.perf_counter() - t0
    times = []
    while len(times) < reps and (not times or t_warm + sum(times) + times[-1] <= budget_s):
        t1 = time.perf_counter()
        ch.mu_search_density(h_np, beta, n_elec, order)
        times.append(time.perf_counter() - t1)
    med = statistics.median(times)
    return {"value": round(1.0 / med, 4), "unit": "density matrices/s", "cores": int(cores), "kind": "oracle",
            "sample": f"median of {len(times)} runs after 1 warm-up: full mu search + density at "
                      f"N={h_np.shape[0]}, order {order} (oracle route: LAPACK eigh of H, moments, bisection, "
                      f"Q p(lam) Q^T); runs {', '.join(f'{t:.2f}' for t in times)} s"}


def attach_oracle_errors(records, inputs):
    """After the timed work: every recorded GPU result against the float64 oracle.

    The oracle takes its own Gershgorin bounds and quadrature size (the library's bounds are
    compared, as a relative difference), forms the sampled rows of D_L at the GPU's mu from the
    generator's eigenpairs, Q[rows] diag(p(lam~)) Q^T, and the trace with the exact moments.
    Writes max_abs_err_vs_oracle (over one row per 64-row band), trace_err_vs_oracle
    (|t_oracle(mu) - N_e|) and bounds_rel_diff into each record's row."""
    import numpy as np

    from oracle import chebyshev as ch

    bounds_cache = {}
    for rec in records:
        h, q, lam = inputs.host[rec["key"]]
        if rec["key"] not in bounds_cache:
            bounds_cache[rec["key"]] = ch.gershgorin_bounds(h)
        lo, hi = bounds_cache[rec["key"]]
        cen, a = ch.scaling(lo, hi)
        M = ch.quadrature_size(rec["order"], rec["beta"] * a)
        c = ch.chebyshev_coeffs(rec["order"], rec["beta"] * a, (rec["mu"] - cen) / a, M)
        row = rec["row"]
        row["bounds_rel_diff"] = float(f"{max(abs(rec['emin'] - lo), abs(rec['emax'] - hi)) / max(abs(lo), abs(hi)):.2e}")
        row["n_quad_matches_oracle"] = bool(rec["n_quad"] == M)
        tau = ch.moments_from_eigs(lam, lo, hi, rec["order"])
        row["trace_err_vs_oracle"] = float(f"{abs(ch.trace_of_series(c, tau) - rec['n_elec']):.3e}")
        if rec["d_rows"] is not None:
            p = ch.cheb_eval(c, (lam - cen) / a)
            ref = (q[rec["rows"]] * p) @ q.T
            row["max_abs_err_vs_oracle"] = float(f"{float(np.max(np.abs(rec['d_rows'] - ref))):.3e}")
            row["err_rows"] = f"{len(rec['rows'])} rows (one per 64-row band)"


def fermi_level(e, beta, n_elec, iters=200):
    """mu with sum_i 1/(1 + exp(beta (e_i - mu))) = n_elec, by bisection on the eigenvalues."""
    import numpy as np

    lo, hi = float(e.min()) - 50.0 / beta, float(e.max()) + 50.0 / beta
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        with np.errstate(over="ignore"):
            cnt = float(np.sum(1.0 / (1.0 + np.exp(beta * (e - mid)))))
        if cnt < n_elec:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 4.0 * np.spacing(max(abs(mid), 1.0)):
            break
    return 0.5 * (lo + hi)


def diag_gpu_rows(inputs, cheb_rows, beta, workloads):
    """On-box diagonalisation comparator (the paper's Sec. II.A / III.A comparison, on MI355X).

    D = V f(E) V^T with E, V from torch.linalg.eigh on the device (the vendor solver, run as a
    library), mu from the eigenvalues (host bisection), and V f(E) V^T as one device product.
    Reports density matrices/s, the Chebyshev path's speed-up over it (mu search + D, float64),
    and the eigensolver / GEMM time ratio (one float64 N x N x N torch.matmul)."""
    import statistics

    import numpy as np
    import torch

    out = {}
    for key in workloads:
        n = key[0]
        H = inputs.get(*key)

        def sync_time(fn, reps):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            return statistics.median(ts)

        def diag_density():
            e, v = torch.linalg.eigh(H)
            e_h = e.cpu().numpy()
            mu = fermi_level(e_h, beta, n / 2.0)
            with np.errstate(over="ignore"):
                occ = torch.from_numpy(1.0 / (1.0 + np.exp(beta * (e_h - mu)))).to(H.device)
            return torch.matmul(v * occ, v.t().contiguous()), mu

        reps = 5 if n <= 2000 else 3
        log(f"diag_gpu: n={n}")
        t_eigh = sync_time(lambda: torch.linalg.eigh(H), reps)
        t_dm = sync_time(diag_density, reps)
        t_gemm = sync_time(lambda: torch.matmul(H, H), 10)
        cheb = cheb_rows.get(f"n{n}_fp64", {}).get("dm_per_s")
        out[f"n{n}"] = {"dm_per_s": round(1.0 / t_dm, 3), "ms_per_dm": round(1e3 * t_dm, 2),
                        "eigh_ms": round(1e3 * t_eigh, 2), "dgemm_ms": round(1e3 * t_gemm, 3),
                        "dgemm_tflops": round(2.0 * n ** 3 / t_gemm / 1e12, 2),
                        "eigh_over_dgemm": round(t_eigh / t_gemm, 1),
                        "chebyshev_fp64_dm_per_s": cheb,
                        "chebyshev_speedup": round(cheb * t_dm, 2) if cheb else None}
        log(f"diag_gpu: {out[f'n{n}']}")
    return {"method": "torch.linalg.eigh (float64, device) -> mu from the eigenvalues -> V f(E) V^T; exact "
                      "Fermi operator, not the order-L expansion",
            **out}


def lanczos_rows(cd, handle, hs, beta, order, reps=10):
    """Bounds by Gershgorin vs 40 Lanczos steps: time of the bounds call, interval, beta', and the
    mu search + density with each (same order; the tighter interval is more accurate, not faster)."""
    import torch

    out = {}
    for nn in sorted(hs):
        H = hs[nn]
        row = {}
        for name in ("gershgorin", "lanczos"):
            call = (lambda: cd.chebdm_bounds(handle, H)) if name == "gershgorin" else \
                (lambda: cd.chebdm_bounds_lanczos(handle, H, 40, 0.01, 0)[:2])
            lo, hi = call()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                call()
            dt = (time.perf_counter() - t0) / reps
            steps = 20 if nn <= 1000 else 5
            d2, _, i2 = run_steps(cd, handle, H, beta, nn / 2.0, order, cd.make_opts("fp64", bounds=name), steps, 2)
            row[name] = {"emin": lo, "emax": hi, "beta_scaled": round(beta * (hi - lo) / 2, 2),
                         "bounds_ms": round(1e3 * dt, 3), "mu_search_dm_per_s": round(steps / d2, 3)}
        out[f"n{nn}"] = row
    return out


def accuracy_rows(cd, handle, n=1000, beta=400.0, mu=0.0, orders=(64, 128, 256, 512, 1024, 2048)):
    """Distance of the float64 expansion D_L to the exact Fermi operator f(H) = Q f(Lambda) Q^T
    against the order L, on the high-density-of-states spectrum (40 % of the levels in a
    Gaussian of width 0.01 at the Fermi level), for three choices of [e_a, e_b]: the spectrum's
    own extremes (passed by the caller), 40 Lanczos steps and Gershgorin's discs.  f(H) comes
    from the generator's eigenpairs (host float64), not from the library."""
    import numpy as np
    import torch
    import synth

    h, q, lam = synth.hamiltonian(n, "highdos", seed=4000)
    with np.errstate(over="ignore"):
        occ = 1.0 / (1.0 + np.exp(beta * (lam - mu)))
    exact = (q * occ) @ q.T
    H = torch.from_numpy(h).to("cuda:0")
    D = torch.empty_like(H)
    lz = cd.chebdm_bounds_lanczos(handle, H, 40, 0.01, 0)[:2]
    bounds = {"spectrum": (float(lam.min()), float(lam.max())), "lanczos": lz, "gershgorin": cd.chebdm_bounds(handle, H)}
    out = {"workload": f"N={n} high-DOS spectrum (seed 4000), beta {beta:g}, mu {mu:g}, float64, max|D_L - f(H)|",
           "beta_scaled": {k: round(beta * (b[1] - b[0]) / 2, 1) for k, b in bounds.items()}, "orders": list(orders)}
    for name, (lo, hi) in bounds.items():
        errs = []
        for L in orders:
            cd.chebdm_density(handle, H, beta, mu, L, cd.make_opts("fp64"), lo, hi, D=D)
            errs.append(float(np.max(np.abs(D.cpu().numpy() - exact))))
        out[name] = [float(f"{e:.3e}") for e in errs]
        log(f"accuracy: {name} {out[name]}")
    return out


def batch_row(cd, handle, torch, prec="fp32", order=256, reps=3):
    """Batched form: 512 Hamiltonians, n uniform on {96..1024}, beta on [30, 200], one graph per batch."""
    import numpy as np

    import synth

    sizes, betas = synth.batch_problems(512, seed=3000)
    log("batch512: generating 512 Hamiltonians on the device")
    Hs = [h for h, _ in synth.hamiltonians_torch(sizes, "uniform", seed=3000, device="cuda:0")]
    nes = [0.5 * n for n in sizes]
    Ds = [torch.empty((int(n), int(n)), dtype=torch.float64, device="cuda:0") for n in sizes]
    b = cd.Batch(handle, sizes, order, cd.make_opts(prec))
    tune = b.tune()
    log("batch512 tune: " + tune)
    b.mu_search(Hs, betas, nes, Ds)                      # captures the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        mu, _, status, iters, trace = b.mu_search(Hs, betas, nes, Ds)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    cd.chebdm_profile_enable(handle, True)
    b.mu_search(Hs, betas, nes, Ds)                      # eager run with launch timing
    prof = cd.chebdm_profile_read(handle)
    cd.chebdm_profile_enable(handle, False)
    info = b.info()
    _, _, _, beta_s = b.stats()
    b.close()
    # the same batch with per-problem Lanczos bounds (40 steps) inside the graph
    bl = cd.Batch(handle, sizes, order, cd.make_opts(prec, bounds="lanczos"))
    bl.tune()
    bl.mu_search(Hs, betas, nes, Ds)
    _, _, _, beta_s_lz = bl.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, _, status_lz, _, _ = bl.mu_search(Hs, betas, nes, Ds)
    torch.cuda.synchronize()
    dt_lz = (time.perf_counter() - t0) / reps
    bl.close()
    r = roofline_of(prof, prec)
    return {"workload": f"512 Hamiltonians, n uniform on {{96..1024}} step 32, beta on [30,200], N_e=n/2, "
                        f"order {order}, {prec}, one graph per batch",
            "batches_per_s": round(1.0 / dt, 3), "dm_per_s": round(512 / dt, 1), "ms_per_batch": round(1e3 * dt, 2),
            "all_ok": bool(np.all(status == 0)), "products_per_problem": info["products_per_problem"],
            "gemm_tflops": r["achieved"] if r else None, "gemm_frac_of_peak": r["frac"] if r else None,
            "phases_ms_eager": {"gemm": round(prof["gemm_ms"], 2), "gram": round(prof["gram_ms"], 2),
                                "combine": round(prof["combine_ms"], 2)},
            "tuner": tune, "median_beta_scaled": round(float(np.median(beta_s)), 1),
            "lanczos_bounds": {"dm_per_s": round(512 / dt_lz, 1), "ms_per_batch": round(1e3 * dt_lz, 2),
                               "all_ok": bool(np.all(status_lz == 0)),
                               "median_beta_scaled": round(float(np.median(beta_s_lz)), 1)}}


def learned_row(cd, handle, torch, order=256, chunks=30, chunk=1024, eval_count=1024, eval_n=500, epochs=120):
    """Learned mu start: train on method-generated data, then compare search modes on 1024 x N=500."""
    import numpy as np

    import synth
    from paper_2306_12616_amd.learned_mu import MuNet, collect_samples, delta_from_residuals, search_report

    t0 = time.perf_counter()
    sizes0 = synth.mu_training_sizes(chunk)
    plan = cd.Batch(handle, sizes0, order)

    def draw(c):
        Hs, _, betas, nes = synth.mu_problems(sizes0, seed=200 + c, device="cuda:0")
        return Hs, betas, nes

    X, T = collect_samples(plan, draw, chunks, log=lambda m: log("learned: " + m))
    plan.close()
    t_data = time.perf_counter() - t0
    nval = 1024
    net = MuNet(handle, seed=0)
    t1 = time.perf_counter()
    net.train(X[nval:], T[nval:], epochs=epochs, batch=256, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    res = (net.predict(X[:nval]) - T[:nval]).cpu().numpy()
    delta = delta_from_residuals(res)
    log(f"learned: {X.shape[0]} samples in {t_data:.1f} s, trained in {t_train:.1f} s, "
        f"validation rms {np.sqrt(np.mean(res ** 2)):.2e}, delta {delta:.2e}")
    Hs, _, betas, nes = synth.mu_problems([eval_n] * eval_count, seed=7, device="cuda:0")
    ev = cd.Batch(handle, [eval_n] * eval_count, order)
    modes = {}
    for mode in ("bisection", "newton", "learned"):
        if mode == "learned":
            ev.set_search(mode, net.W, delta)
        else:
            ev.set_search(mode)
        ev.mu_only(Hs, betas, nes, allow_errors=True)        # capture
        cd.chebdm_profile_enable(handle, True)
        ev.mu_only(Hs, betas, nes, allow_errors=True)        # eager, launch-timed
        prof = cd.chebdm_profile_read(handle)
        cd.chebdm_profile_enable(handle, False)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        mu, status, iters, t = ev.mu_only(Hs, betas, nes, allow_errors=True)
        torch.cuda.synchronize()
        row = search_report(ev, status, iters, t, nes)
        row["ms_per_batch_mu_only"] = round(1e3 * (time.perf_counter() - ta), 2)
        row["search_ms_eager"] = round(prof["search_ms"], 3)
        modes[mode] = row
        log(f"learned: {mode} {row}")
    ev.close()
    return {"workload": f"train: {X.shape[0]} problems (n on {{64..512}} step 16, N_e/n on [0.3,0.7], beta on "
                        f"[30,200], three spectrum laws, order {order}, bisection targets); evaluate: "
                        f"{eval_count} x n={eval_n}",
            "train_samples": int(X.shape[0] - nval), "data_s": round(t_data, 1), "train_s": round(t_train, 1),
            "epochs": epochs, "validation_rms_mu_scaled": float(np.sqrt(np.mean(res ** 2))), "delta": delta,
            "modes": modes,
            "learned_over_newton": {"evals": round(modes["learned"]["mean_evals"] / modes["newton"]["mean_evals"], 3),
                                    "search_ms": round(modes["learned"]["search_ms_eager"]
                                                       / modes["newton"]["search_ms_eager"], 3)}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4000)
    ap.add_argument("--order", type=int, default=512)
    ap.add_argument("--beta", type=float, default=100.0)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16x3", "bf16x6"])
    ap.add_argument("--no-breakdown", action="store_true")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched 512-problem workload (for profiling it) and print its row")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle leg (its timing and the oracle check of every GPU result)")
    ap.add_argument("--sections", default="all",
                    help=f"comma list of the sections after the headline line: {','.join(ALL_SECTIONS)}")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before timing, run one plain device copy of this many MiB (the calibration "
                         "kernel for rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the method has no multi-GPU path here "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2306_12616_amd as cd

    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)
    cd.load_library()
    handle = cd.Handle(0)
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib * (1 << 18), dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst
    if args.batch_only:
        print(json.dumps({"batch512": batch_row(cd, handle, torch)}), flush=True)
        handle.close()
        return

    n, order, beta = args.n, args.order, args.beta
    n_elec = n / 2.0
    sections = set(ALL_SECTIONS if args.sections == "all" else args.sections.split(","))
    unknown = sections - set(ALL_SECTIONS)
    if unknown:
        print(f"unknown sections {sorted(unknown)}; choose from {ALL_SECTIONS}", file=sys.stderr)
        sys.exit(2)
    if args.no_breakdown:
        sections = set()
    inputs = Inputs()
    head_key = (n, "gaussmix6", 2002 if n == 4000 else SEEDS.get(n, 2000))
    H = inputs.get(*head_key)
    opts = cd.make_opts(args.prec)
    log(f"timing {args.steps} steps (warmup {args.warmup}) of mu search + density, prec={args.prec}")
    dt, prof, info, head_mu, head_D = run_steps(cd, handle, H, beta, n_elec, order, opts, args.steps, args.warmup,
                                                with_out=True)
    value = args.steps / dt
    log(f"  {value:.3f} DM/s, {1e3 * dt / args.steps:.2f} ms/step, gemm {prof['gemm_ms'] / args.steps:.2f} ms/step")
    roof = roofline_of(prof, args.prec)
    if roof is not None:
        roof["traffic"] = traffic_of(args.prec, n, order)
    head_check = {}
    records = [check_record(head_check, head_key, order, beta, n_elec, head_mu, info, head_D)]
    del head_D

    result = {
        "metric": METRIC, "value": round(value, 4), "unit": "density matrices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3 (f32 accumulate)",
                  "bf16x6": "bf16x6 (f32 accumulate)"}[args.prec],
        "data": "synthetic",
        "config": {"workload": f"mu search + density matrix, N={n}, order {order}, beta {beta:g}, "
                               f"N_e=N/2, H=Q diag(lam) Q^T with lam from a 6-Gaussian mixture",
                   "n": n, "order": order, "beta": beta, "n_elec": n_elec, "prec": args.prec,
                   "k": info["k"], "m": info["m"], "products_per_step": info["n_gemm"],
                   "n_quad": info["n_quad"], "bisection_sweeps": info["iters"]},
        "roofline": roof,
        "phases_ms_per_step": {"gemm": round(prof["gemm_ms"] / args.steps, 3),
                               "combine": round(prof["combine_ms"] / args.steps, 3),
                               "gram": round(prof["gram_ms"] / args.steps, 3),
                               "search": round(prof["search_ms"] / args.steps, 3),
                               "other": round(1e3 * dt / args.steps - (prof["gemm_ms"] + prof["combine_ms"]
                                                                       + prof["gram_ms"] + prof["search_ms"])
                                              / args.steps, 3)},
        "hbm_GBs": {"combine": hbm_of(prof["combine_ms"], prof["combine_bytes"]),
                    "gram": hbm_of(prof["gram_ms"], prof["gram_bytes"]), "peak": PEAK_HBM_GBS},
        "oracle_check": head_check,
    }

    rows = {}
    if "breakdown" in sections:
        cases = [(1000, "fp64", "bisection"), (1000, "fp64", "newton"), (1000, "fp32", "bisection"),
                 (2000, "fp64", "bisection"), (2000, "fp32", "bisection"), (4000, "fp32", "bisection"),
                 (4000, "bf16x3", "bisection"), (4000, "bf16x6", "bisection"), (1000, "bf16x3", "bisection"),
                 (2000, "bf16x3", "bisection"), (2000, "bf16x6", "bisection"), (4000, "fp64", "newton")]
        if args.prec != "fp64" or n != 4000:
            cases.append((4000, "fp64", "bisection"))
        for nn, pr, se in cases:
            log(f"breakdown n={nn} prec={pr} search={se}")
            steps = 20 if nn <= 1000 else (10 if nn <= 2000 else 5)
            row, rec = mu_search_row(cd, handle, inputs, (nn, "gaussmix6", SEEDS[nn]), beta, order, pr, se, steps)
            rows[f"n{nn}_{pr}" + ("" if se == "bisection" else f"_{se}")] = row
            records.append(rec)
        for key, row in rows.items():
            nn = key.split("_")[0]
            base = value if (nn == f"n{n}" and args.prec == "fp64") else rows.get(f"{nn}_fp64", {}).get("dm_per_s")
            row["speedup_vs_fp64"] = round(row["dm_per_s"] / base, 3) if base else None
        result["breakdown"] = rows

    if "fixed" in sections:
        fixed = {}
        for nn, pr in ((1000, "fp64"), (4000, "fp64"), (4000, "fp32")):
            log(f"fixed mu: n={nn} prec={pr}")
            key = (nn, "gaussmix6", SEEDS[nn])
            hh = inputs.get(*key)
            mu_nn, _, _ = cd.chebdm_mu_search(handle, hh, beta, nn / 2.0, order, cd.make_opts(pr), want_density=False)
            steps = 20 if nn <= 1000 else 5
            D = torch.empty_like(hh)
            d3, p3, (_, i3) = timed(lambda: cd.chebdm_density(handle, hh, beta, mu_nn, order, cd.make_opts(pr), D=D),
                                    steps, 2, cd, handle)
            r3 = roofline_of(p3, pr)
            fixed[f"n{nn}_{pr}"] = row = {"dm_per_s": round(steps / d3, 3), "ms_per_step": round(1e3 * d3 / steps, 3),
                                          "products": p3["gemm_products"] // steps,
                                          "gemm_frac_of_peak": r3["frac"] if r3 else None}
            records.append(check_record(row, key, order, beta, nn / 2.0, mu_nn, i3, D))
        result["fixed_mu"] = fixed

    if "config" in sections:
        # the N = 256 reference workload (order 128, beta 50, N_e = 128, lam uniform on [-1, 1])
        log("config n=256 order=128")
        row, rec = mu_search_row(cd, handle, inputs, (256, "uniform", 1000), 50.0, 128, "fp64", steps=50, warmup=5)
        result["n256_order128"] = {"workload": "mu search + density, N=256, order 128, beta 50, N_e=128, "
                                               "lam uniform on [-1,1] (seed 1000), float64", **row}
        records.append(rec)
        # the hard case: N = 5000, order 2048, beta 400, 40 % of the levels in a Gaussian of width
        # 0.01 at the Fermi level (seed 4000), every precision
        c4 = {"workload": "mu search + density, N=5000, order 2048, beta 400, N_e=N/2, high DOS at the Fermi "
                          "level (40 % of lam ~ N(0, 0.01^2), rest U[-1,1], seed 4000); split-bf16 form for "
                          "the 1e-5 target: bf16x6"}
        for pr in ("fp64", "fp32", "bf16x3", "bf16x6"):
            log(f"config n=5000 order=2048 prec={pr}")
            row, rec = mu_search_row(cd, handle, inputs, (5000, "highdos", 4000), 400.0, 2048, pr, steps=3, warmup=1)
            c4[pr] = row
            records.append(rec)
        for pr in ("fp32", "bf16x3", "bf16x6"):
            c4[pr]["speedup_vs_fp64"] = round(c4[pr]["dm_per_s"] / c4["fp64"]["dm_per_s"], 3)
        result["n5000_order2048_highdos"] = c4

    if "lanczos" in sections:
        result["lanczos_bounds"] = lanczos_rows(cd, handle, {nn: inputs.get(nn, "gaussmix6", SEEDS[nn])
                                                             for nn in (1000, 2000, 4000)}, beta, order)
    if "accuracy" in sections:
        result["accuracy_vs_order"] = accuracy_rows(cd, handle)
    if "diag" in sections:
        cheb_rows = dict(rows)
        if args.prec == "fp64":   # the headline step is the float64 row at its N
            cheb_rows.setdefault(f"n{n}_fp64", {"dm_per_s": round(value, 3)})
        result["diag_gpu"] = diag_gpu_rows(inputs, cheb_rows, beta,
                                           [(nn, "gaussmix6", SEEDS[nn]) for nn in (1000, 2000, 4000)])
    inputs.drop_device()
    del H
    torch.cuda.empty_cache()
    if "batch" in sections:
        result["batch512"] = batch_row(cd, handle, torch)
    if "learned" in sections:
        result["learned_mu"] = learned_row(cd, handle, torch)

    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on host cores")
        result["cpu_baseline"] = cpu_baseline(inputs.host[head_key][0], beta, n_elec, order)
        log("oracle check of every recorded GPU result")
        attach_oracle_errors(records, inputs)
    else:
        result["cpu_baseline"] = None
    handle.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
