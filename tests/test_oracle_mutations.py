"""Plant plausible mistakes in the oracle (on the CPU) and require that the
pins catch every one of them.  This shows the pins constrain the oracle's
arithmetic rather than restate it."""

import numpy as np
import pytest

import oracle
from oracle import mds as om
from oracle import sampler as osamp
from synth import generators as gen

from . import pins

X_SMALL = gen.small_gaussian(n=300, seed=41)


def _all_checks():
    return [
        lambda: pins.check_self_reproduction(X_SMALL, 60, 2, seed=1),
        lambda: pins.check_proposition_1(X_SMALL, 60, 2, seed=1),
        lambda: pins.check_pca_closed_form(X_SMALL, 60, 2, seed=1),
        lambda: pins.check_centring(X_SMALL, 60, seed=1),
        lambda: pins.check_eigen(X_SMALL, 60, 2, seed=1),
        lambda: pins.check_exact_recovery(n=120, l=30),
        lambda: pins.check_l_equals_n(n=12),
        lambda: pins.check_sampler_enumeration(4, 2),
        lambda: pins.check_lemire_power_of_two(),
    ]


def _caught():
    for check in _all_checks():
        try:
            check()
        except (AssertionError, ValueError, IndexError, np.linalg.LinAlgError):
            return True
    return False


def test_unmutated_oracle_passes_all_checks():
    assert not _caught()


def _gower_with_V(fit, A2):
    # a plausible misreading of eq. (2): the eigenvectors V in place of X1
    l = fit.M.shape[0]
    s1_inv = np.where(fit.live, l / fit.lam, 0.0)
    return (1.0 / (2.0 * l)) * ((fit.q[None, :] - A2) @ fit.V) * s1_inv[None, :]


def _gower_missing_half(fit, A2):
    l = fit.M.shape[0]
    s1_inv = np.where(fit.live, l / fit.lam, 0.0)
    return (1.0 / l) * ((fit.q[None, :] - A2) @ fit.X1) * s1_inv[None, :]


def _gower_dropped_q(fit, A2):
    l = fit.M.shape[0]
    s1_inv = np.where(fit.live, l / fit.lam, 0.0)
    return (1.0 / (2.0 * l)) * ((-A2) @ fit.X1) * s1_inv[None, :]


def _gower_s1_not_inverted(fit, A2):
    l = fit.M.shape[0]
    s1 = np.where(fit.live, fit.lam / l, 0.0)
    return (1.0 / (2.0 * l)) * ((fit.q[None, :] - A2) @ fit.X1) * s1[None, :]


def _inner_no_half(D):
    P = om.centring_matrix(D.shape[0])
    return -1.0 * (P @ D @ P)


def _inner_wrong_centring(D):
    n = D.shape[0]
    P = np.eye(n) + np.full((n, n), 1.0 / n)
    return -0.5 * (P @ D @ P)


def _inner_one_sided(D):
    P = om.centring_matrix(D.shape[0])
    return -0.5 * (P @ D)


def _eig_ascending(Q, r):
    lam_all, vec_all = np.linalg.eigh(Q)
    return lam_all[:r].copy(), vec_all[:, :r].copy()


def _eig_transposed(Q, r):
    lam_all, vec_all = np.linalg.eigh(Q)
    order = np.argsort(-lam_all)[:r]
    return lam_all[order].copy(), vec_all.T[:, order].copy()


def _sqdist_abs(A, B):
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    return np.array([np.abs(B - a).sum(axis=1) for a in A])


def _sqdist_missing_column(A, B):
    A = np.asarray(A, dtype=np.float64)[:, 1:]
    B = np.asarray(B, dtype=np.float64)[:, 1:]
    return np.array([((B - a) ** 2).sum(axis=1) for a in A])


def _sign_negative(V):
    V = V.copy()
    for k in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, k])))
        if V[i, k] > 0:
            V[:, k] = -V[:, k]
    return V


def _fy_off_by_one(n, l, draw):
    moved = {}
    for i in range(l):
        j = i + draw(max(n - i - 1, 1))
        ai, aj = moved.get(i, i), moved.get(j, j)
        moved[i], moved[j] = aj, ai
    return [moved.get(i, i) for i in range(l)]


def _bounded_modulo(gen_, k):
    return gen_.next() % k


MUTATIONS = [
    ("gower_block", _gower_with_V),
    ("gower_block", _gower_missing_half),
    ("gower_block", _gower_dropped_q),
    ("gower_block", _gower_s1_not_inverted),
    ("inner_products", _inner_no_half),
    ("inner_products", _inner_wrong_centring),
    ("inner_products", _inner_one_sided),
    ("top_eigenpairs", _eig_ascending),
    ("top_eigenpairs", _eig_transposed),
    ("sqdist_rows", _sqdist_abs),
    ("sqdist_rows", _sqdist_missing_column),
    ("sign_convention", _sign_negative),
]


@pytest.mark.parametrize("name,bad", MUTATIONS, ids=[f.__name__ for _, f in MUTATIONS])
def test_mds_mutation_is_caught(monkeypatch, name, bad):
    monkeypatch.setattr(om, name, bad)
    assert _caught(), f"planted mistake {bad.__name__} in {name} went unnoticed"


def test_sampler_off_by_one_is_caught(monkeypatch):
    monkeypatch.setattr(osamp, "fisher_yates_prefix", _fy_off_by_one)
    monkeypatch.setattr(oracle, "fisher_yates_prefix", _fy_off_by_one)
    assert _caught()


def test_sampler_modulo_draw_is_caught(monkeypatch):
    monkeypatch.setattr(osamp, "bounded", _bounded_modulo)
    monkeypatch.setattr(oracle, "bounded", _bounded_modulo)
    assert _caught()
