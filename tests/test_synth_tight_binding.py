"""The two-level tight-binding generator (Sec. III.C model Hamiltonians), on the CPU.

It is an input generator, not part of the method: these tests check that it builds
what its docstring states (orbital layout, couplings, decay over site distance,
onsite energies, seeded noise), and two spectral facts that follow from the model
itself: decoupled A and B chains when gamma = 0, and the mirror symmetry of the
accuracy-study case (eps_b = -eps_a, beta = -alpha, gamma = 0 gives a spectrum
symmetric about 0).  Fidelity to the paper's own generator (a PROGRESS module that
is not available) is unpinned: its orbital layout and sign conventions are readings.
"""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("kind", list(synth.TB_KINDS))
@pytest.mark.parametrize("n", [1, 2, 7, 64])
def test_symmetric_and_finite(kind, n):
    h = synth.tight_binding(n, kind, seed=3)
    assert h.shape == (n, n) and np.all(np.isfinite(h))
    assert np.array_equal(h, h.T)


def test_metal_couplings_and_decay():
    p = synth.TB_KINDS["metal"]
    h = synth.tight_binding(12, "metal")
    # A orbitals at even positions, B at odd; site s holds orbitals 2s, 2s+1
    assert h[0, 2] == pytest.approx(p["alpha"] * np.exp(-1.0))      # A0-A1, one site apart
    assert h[1, 3] == pytest.approx(p["beta"] * np.exp(-1.0))       # B0-B1
    assert h[0, 4] / h[0, 2] == pytest.approx(np.exp(-1.0))         # decay per site
    assert h[0, 1] == 0.0 and h[0, 3] == 0.0                         # gamma = 0: no A-B coupling
    assert np.all(np.diag(h) == 0.0)


def test_semiconductor_and_softmatter_parameters():
    h = synth.tight_binding(10, "semiconductor")
    assert h[0, 1] == -2.0                                           # gamma within a site, no decay
    assert h[0, 2] == 0.0                                            # alpha = 0
    assert h[1, 3] == pytest.approx(-np.exp(-0.01))
    base = synth.tight_binding(40, "softmatter", r=0.0)
    noisy = synth.tight_binding(40, "softmatter", seed=5)
    again = synth.tight_binding(40, "softmatter", seed=5)
    assert np.array_equal(noisy, again)
    assert not np.array_equal(noisy, synth.tight_binding(40, "softmatter", seed=6))
    ratio = noisy[base != 0] / base[base != 0]
    assert ratio.min() >= 0.0 and ratio.max() <= 2.0 and ratio.std() > 0.3   # (1 + eta), eta ~ U[-1, 1]
    assert np.all(noisy[base == 0] == 0.0)
    assert np.mean(np.diag(base)[0::2]) == -10.0


def test_gamma_zero_decouples_the_chains():
    h = synth.tight_binding(80, "metal")
    lam = np.linalg.eigvalsh(h)
    la = np.linalg.eigvalsh(h[0::2, 0::2])
    lb = np.linalg.eigvalsh(h[1::2, 1::2])
    assert np.allclose(np.sort(np.concatenate([la, lb])), lam, atol=1e-12)


def test_accuracy_case_spectrum_is_mirror_symmetric():
    h = synth.tight_binding(200, "metal_accuracy")
    lam = np.linalg.eigvalsh(h)
    assert np.allclose(lam, -lam[::-1], atol=1e-12)
