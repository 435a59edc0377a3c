"""The FP64 oracle against facts the paper and mathematics fix (CPU only)."""

import json
import os

import numpy as np
import pytest

import oracle
from oracle import mds as om
from synth import generators as gen

from . import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def small():
    return gen.small_gaussian(n=800, seed=21)


@pytest.fixture(scope="module")
def wide():
    return gen.wide_gaussian(n=600, seed=22).astype(np.float64)


def test_self_reproduction(small, wide):
    pins.check_self_reproduction(small, 120, 2, seed=1)
    pins.check_self_reproduction(wide, 200, 10, seed=2)


def test_proposition_1(small, wide):
    pins.check_proposition_1(small, 120, 2, seed=1)
    pins.check_proposition_1(wide, 200, 10, seed=2)


def test_pca_closed_form(small, wide):
    pins.check_pca_closed_form(small, 120, 2, seed=1)
    pins.check_pca_closed_form(wide, 200, 10, seed=2)


def test_exact_recovery():
    pins.check_exact_recovery()


def test_l_equals_n_brute_force():
    pins.check_l_equals_n()


def test_centring(small, wide):
    pins.check_centring(small, 120, seed=1)
    pins.check_centring(wide, 200, seed=2)


def test_eigen(small, wide):
    pins.check_eigen(small, 120, 2, seed=1)
    pins.check_eigen(wide, 200, 10, seed=2)


def test_integer_distances_exact():
    pins.check_integer_distances()


def test_rigid_invariance(small):
    pins.check_rigid_invariance(small[:300], 60, 2, seed=3)


def test_paper_layout_matches_embed_all(small):
    """The paper stacks X1 for the landmarks and eq. (2) for the rest
    (Section 3.1); interpolating every row gives the same matrix."""
    Yp, fit = om.interpolation_mds_paper_layout(small, 120, 2, seed=4)
    Ya = om.interpolate(fit, small)
    assert np.max(np.abs(Yp - Ya)) < 1e-10 * np.max(np.abs(Ya))


def test_block_size_irrelevant(small):
    """Eq. (2) acts row by row, so the block size m changes nothing."""
    fit = om.fit_landmarks(small, 100, 2, seed=5)
    a = om.interpolate(fit, small, block=100)
    b = om.interpolate(fit, small, block=37)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_expanded_distances_match_direct(wide):
    """The expanded FP64 cross distances agree with direct differences."""
    fit = om.fit_landmarks(wide, 200, 10, seed=6)
    a = om.sqdist_rows(wide[:300], fit.M)
    b = om.sqdist_rows_expanded(wide[:300], fit.M)
    assert np.max(np.abs(a - b)) / np.max(np.abs(a)) < 1e-13


def test_rank_deficient_columns_are_zero():
    """Data of rank 3 asked for r = 5: columns 4-5 are dead (zero)."""
    X, _ = gen.low_rank(200, 8, 3, seed=7)
    Y, fit = om.interpolation_mds(X, 50, 5, seed=7)
    assert fit.r_eff == 3
    assert np.all(Y[:, 3:] == 0.0)
    assert np.all(fit.X1[:, 3:] == 0.0)


def test_degenerate_landmarks():
    X = np.ones((20, 4))
    with pytest.raises(om.DegenerateError):
        om.fit_landmarks(X, 10, 2, seed=0)


# ---- sampler -------------------------------------------------------------

def test_splitmix64_published_vector():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.json")) as f:
        ref = json.load(f)
    g = oracle.SplitMix64(ref["seed"])
    assert [str(g.next()) for _ in ref["outputs"]] == ref["outputs"]


def test_lemire_power_of_two():
    pins.check_lemire_power_of_two()


def test_lemire_range_and_rejection():
    g = oracle.SplitMix64(3)
    for k in (1, 2, 3, 7, 1000, (1 << 63) + 1, (1 << 64) - 1):
        for _ in range(200):
            v = oracle.bounded(g, k)
            assert 0 <= v < k


def test_fisher_yates_enumeration():
    pins.check_sampler_enumeration(5, 3)
    pins.check_sampler_enumeration(4, 4)


def test_sampler_basic_properties():
    for n, l, seed in [(10, 10, 1), (1000, 17, 2), (5000, 200, 3), (10**6, 1000, 4)]:
        idx = oracle.sample_landmarks(n, l, seed)
        assert len(idx) == l
        assert idx == sorted(set(idx))
        assert 0 <= idx[0] and idx[-1] < n
        assert idx == oracle.sample_landmarks(n, l, seed)
    assert oracle.sample_landmarks(7, 7, 123) == list(range(7))
    assert oracle.sample_landmarks(10**6, 50, 1) != oracle.sample_landmarks(10**6, 50, 2)


def test_sampler_inclusion_uniform():
    """Inclusion frequencies over many seeds are uniform (chi^2 test)."""
    from scipy import stats
    n, l, seeds = 20, 5, 4000
    counts = np.zeros(n)
    for s in range(seeds):
        counts[oracle.sample_landmarks(n, l, s)] += 1
    expected = seeds * l / n
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    assert stats.chi2.sf(chi2, n - 1) > 1e-4


# ---- the paper's simulation design (statistical sanity) ------------------

@pytest.mark.parametrize("k,h", [(10, 2), (100, 10)])
def test_paper_design_recovers_dominant_directions(k, h):
    """Section 4.1 design: variance 15 on h of k columns.  After Procrustes
    the embedding correlates with the dominant columns (Table 1 reports a
    mean of 0.99949 for interpolation MDS) and lambda/l estimates the
    variance 15 (eq. (1) and Section 3.1)."""
    X = gen.paper_design(5000, k, h, seed=31 + k)
    Y, fit = om.interpolation_mds(X, 250, h, seed=8)
    aligned, _, _ = oracle.procrustes(X[:, :h], Y)
    cors = [np.corrcoef(aligned[:, j], X[:, j])[0, 1] for j in range(h)]
    assert np.mean(cors) > 0.99
    est = fit.lam / 250
    assert 12.0 < np.mean(est) < 19.0
