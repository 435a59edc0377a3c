"""The fit's Lanczos steps past the small-basis limit ((j + 1) l > 40,000
values, where the Gram-Schmidt passes run as separate dot, update and
finish launches), against the FP64 oracle through the C ABI (needs a GPU).

Data of rank 60 whose 60 variances are spread evenly over [1, 2]: the ten
largest eigenvalues of Q1 converge slowly, so at l = 1000 the run takes
about 62 steps (a plain Lanczos run on the oracle's Q1 converges at step
62), the last twenty or so past the limit.  Tolerances as in
test_gpu_parity: landmark indices bit for bit, eigenvalues to 1e-12 of the
largest, X1 to 1e-10 of its largest entry, the FP64 embed to 1e-9.
"""

import numpy as np
import pytest

import oracle

from . import tolerance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rankk(n, p, seed, k=60):
    rng = np.random.Generator(np.random.PCG64(seed))
    U, _ = np.linalg.qr(rng.standard_normal((p, k)))
    sd = np.sqrt(np.linspace(2.0, 1.0, k))
    return (rng.standard_normal((n, k)) * sd) @ U.T


def test_large_basis_steps():
    import paper_2007_11919_amd as mds
    X = _rankk(4000, 80, seed=31)
    Xd = torch.from_numpy(X).cuda()
    model = mds.fit_landmarks(Xd, 1000, 10, seed=3)
    stats = model.fit_stats()
    assert stats["lanczos_steps"] > 50, stats
    fit = oracle.fit_landmarks(X, 1000, 10, seed=3)
    assert np.array_equal(model.landmarks(), fit.idx)
    lam = model.eigenvalues()
    assert np.max(np.abs(lam - fit.lam)) <= 1e-12 * fit.lam[0], (lam, fit.lam)
    X1 = model.landmark_coords()
    assert np.max(np.abs(X1 - fit.X1)) <= 1e-10 * np.max(np.abs(fit.X1))
    Y = mds.embed(model, Xd, prec="fp64").cpu().numpy()
    tolerance.check_embed(Y, oracle.interpolate(fit, X), "fp64")
    model.free()


def test_large_basis_steps_repeatable():
    """Two fits of the same data give the same bits (every sum of the
    steps is taken in a fixed order)."""
    import paper_2007_11919_amd as mds
    X = _rankk(4000, 80, seed=32)
    Xd = torch.from_numpy(X).cuda()
    a = mds.fit_landmarks(Xd, 1000, 10, seed=5)
    b = mds.fit_landmarks(Xd, 1000, 10, seed=5)
    assert np.array_equal(a.eigenvalues(), b.eigenvalues())
    assert np.array_equal(a.landmark_coords(), b.landmark_coords())
    assert a.fit_stats() == b.fit_stats()
    a.free()
    b.free()
