"""chebdm_bounds_noalloc (fixed static scratch, no device allocation) against chebdm_bounds.

Both run the same Gershgorin kernels with the same row split, so the bounds must agree bit
for bit; the oracle's bounds pin them independently.  Two calls in a row, the second on a
smaller matrix, check that the shared scratch carries nothing from one call into the next.
"""
import ctypes
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2306_12616_amd as chebdm  # noqa: E402
from paper_2306_12616_amd import _binding  # noqa: E402
import synth  # noqa: E402
from oracle import chebyshev as ch  # noqa: E402


def test_noalloc_rejects_sizes_beyond_its_scratch_on_the_host():
    lib = chebdm.load_library()
    fake = ctypes.c_void_p(8)   # never dereferenced: the size check comes first
    assert lib.chebdm_bounds_noalloc(None, fake, 70000, 70000, fake) == _binding.ERR_ARG
    assert b"65535" in lib.chebdm_last_error()
    assert lib.chebdm_bounds_noalloc(None, fake, 0, 1, fake) == _binding.ERR_ARG
    assert lib.chebdm_bounds_noalloc(None, fake, 10, 9, fake) == _binding.ERR_ARG


@pytest.mark.gpu
def test_noalloc_bounds_match_chebdm_bounds_two_calls_shrinking():
    dev = torch.device("cuda:0")
    h = chebdm.Handle(0)
    out = torch.full((2,), -7.0, dtype=torch.float64, device=dev)
    for n, law, seed, ld in ((1000, "gaussmix6", 2000, 1000), (300, "uniform", 1001, 320)):
        print(f"noalloc bounds: n={n} ld={ld} law={law} seed={seed}", flush=True)
        h_np = synth.hamiltonian(n, law, seed=seed)[0]
        buf = torch.zeros((n, ld), dtype=torch.float64, device=dev)
        buf[:, :n] = torch.from_numpy(h_np).to(dev)
        H = buf[:, :n]
        chebdm.chebdm_bounds_noalloc(h, H, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().copy()
        lo, hi = chebdm.chebdm_bounds(h, H)
        assert got[0] == lo and got[1] == hi, (got, lo, hi)
        e_lo, e_hi = ch.gershgorin_bounds(h_np)
        scale = max(abs(e_lo), abs(e_hi))
        assert abs(got[0] - e_lo) <= 1e-13 * scale and abs(got[1] - e_hi) <= 1e-13 * scale, (got, e_lo, e_hi)
    h.close()


@pytest.mark.gpu
def test_noalloc_bounds_flag_nonfinite_as_nan():
    dev = torch.device("cuda:0")
    h = chebdm.Handle(0)
    h_np = synth.hamiltonian(64, "uniform", seed=1002)[0]
    h_np[5, 9] = h_np[9, 5] = math.nan
    H = torch.from_numpy(h_np).to(dev)
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    chebdm.chebdm_bounds_noalloc(h, H, out)
    torch.cuda.synchronize()
    assert np.isnan(out.cpu().numpy()).all()
    # a clean call afterwards is unaffected by the flagged one
    H2 = torch.from_numpy(synth.hamiltonian(64, "uniform", seed=1003)[0]).to(dev)
    chebdm.chebdm_bounds_noalloc(h, H2, out)
    torch.cuda.synchronize()
    lo, hi = chebdm.chebdm_bounds(h, H2)
    assert tuple(out.cpu().numpy()) == (lo, hi)
    h.close()
