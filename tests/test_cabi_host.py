"""The C ABI library on the host: it loads, exports every declared symbol,
its sampler matches the oracle's vectors bit for bit, and argument checks
that need no GPU return the documented status codes."""

import ctypes
import json
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mds.h")
GOLDEN = os.path.join(ROOT, "tests", "golden", "sampler_vectors.json")


@pytest.fixture(scope="module")
def L():
    from paper_2007_11919_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2007_11919_amd import build
        build.build()
    return _lib.lib()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mds_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("mds_fit_landmarks", "mds_embed", "mds_free", "mds_sample_landmarks",
                     "mds_serve_create", "mds_serve_submit", "mds_serve_destroy"):
        assert required in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert not missing, f"not exported: {missing}"


def test_sampler_matches_oracle_vectors(L):
    from paper_2007_11919_amd import sample_landmarks
    ref = json.load(open(GOLDEN))
    for case in ref["sample_landmarks"]:
        got = sample_landmarks(case["n"], case["l"], int(case["seed"]))
        assert got.tolist() == case["idx"], case["n"]


def test_bounded_draw_matches_oracle_vectors(L):
    ref = json.load(open(GOLDEN))
    for case in ref["bounded"]:
        out = (ctypes.c_uint64 * 20)()
        L.mds_debug_bounded(int(case["seed"]), int(case["k"]), 20, out)
        assert [str(v) for v in out] == case["draws"]


def test_sampler_against_oracle_random_cases(L):
    import oracle
    from paper_2007_11919_amd import sample_landmarks
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(40):
        n = int(rng.integers(1, 10**7))
        l = int(rng.integers(1, min(n, 3000) + 1))
        seed = int(rng.integers(0, 2**63))
        assert sample_landmarks(n, l, seed).tolist() == oracle.sample_landmarks(n, l, seed)


def test_sampler_argument_errors(L):
    out = np.empty(4, dtype=np.int64)
    P = ctypes.POINTER(ctypes.c_int64)
    assert L.mds_sample_landmarks(10, 0, 1, out.ctypes.data_as(P)) == 1
    assert L.mds_sample_landmarks(3, 4, 1, out.ctypes.data_as(P)) == 1
    assert L.mds_sample_landmarks(10, 2, 1, None) == 1
    assert b"NULL" in L.mds_last_error()


def test_fit_and_embed_argument_errors_need_no_gpu(L):
    model = ctypes.c_void_p()
    # NULL X, bad sizes: rejected before any device work
    assert L.mds_fit_landmarks(None, 0, 100, 4, 4, 10, 2, 0, None, None, ctypes.byref(model)) == 1
    fake = ctypes.c_void_p(16)
    assert L.mds_fit_landmarks(fake, 0, 100, 4, 3, 10, 2, 0, None, None, ctypes.byref(model)) == 1
    assert L.mds_fit_landmarks(fake, 0, 100, 4, 4, 1, 1, 0, None, None, ctypes.byref(model)) == 1
    assert L.mds_fit_landmarks(fake, 0, 100, 4, 4, 10, 10, 0, None, None, ctypes.byref(model)) == 1
    assert L.mds_fit_landmarks(fake, 7, 100, 4, 4, 10, 2, 0, None, None, ctypes.byref(model)) == 1
    assert L.mds_fit_landmarks(fake, 0, 100, 4, 4, 200, 2, 0, None, None, ctypes.byref(model)) == 1
    dup = (ctypes.c_int64 * 3)(1, 5, 5)
    assert L.mds_fit_landmarks(fake, 0, 100, 4, 4, 3, 2, 0, dup, None, ctypes.byref(model)) == 1
    oob = (ctypes.c_int64 * 3)(1, 5, 100)
    assert L.mds_fit_landmarks(fake, 0, 100, 4, 4, 3, 2, 0, oob, None, ctypes.byref(model)) == 1
    assert model.value is None
    assert L.mds_embed(None, fake, 0, 10, 4, 1, fake, 2, None) == 1
    L.mds_free(None)  # no-op


def test_serve_argument_errors_need_no_gpu(L):
    srv = ctypes.c_void_p()
    assert L.mds_serve_create(0, 4, 0, ctypes.byref(srv)) == 1
    assert L.mds_serve_create(1 << 30, 0, 0, ctypes.byref(srv)) == 1
    assert L.mds_serve_create(1 << 30, 4, -1, ctypes.byref(srv)) == 1
    t = ctypes.c_int64()
    assert L.mds_serve_submit(None, 0, None, 0, 0, 1, 1, None, 1, ctypes.byref(t)) == 1
    L.mds_serve_destroy(None)  # no-op


def test_next_row_entry_points_reject_bad_arguments_without_gpu(L):
    fake = ctypes.c_void_p(16)
    P64 = ctypes.POINTER(ctypes.c_int64)
    out = np.empty(8, dtype=np.int64)
    lam = (ctypes.c_double * 4)()
    reff = ctypes.c_int32(0)
    # divide-and-conquer: c < r + 1, l <= c, n <= c, l too large, NULL X
    for n, l, c, r in [(100, 20, 2, 2), (100, 10, 10, 2), (10, 20, 10, 2), (10**5, 4096, 50, 2)]:
        assert L.mds_divide_conquer(fake, 0, n, 4, 4, l, c, r, 0, fake, r, lam, ctypes.byref(reff),
                                    None, None) == 1, (n, l, c, r)
    assert L.mds_divide_conquer(None, 0, 100, 4, 4, 20, 5, 2, 0, fake, 2, lam, None, None, None) == 1
    # MaxMin: l > n, first out of range, NULL output
    assert L.mds_maxmin_landmarks(fake, 0, 10, 4, 4, 11, 0, out.ctypes.data_as(P64), None) == 1
    assert L.mds_maxmin_landmarks(fake, 0, 10, 4, 4, 3, 10, out.ctypes.data_as(P64), None) == 1
    assert L.mds_maxmin_landmarks(fake, 0, 10, 4, 4, 3, 0, None, None) == 1
    # pivot MDS: r >= l, l > n, duplicate pivots, ldy < r
    assert L.mds_pivot_mds(fake, 0, 100, 4, 4, 5, 5, 0, None, fake, 5, lam, None, None) == 1
    assert L.mds_pivot_mds(fake, 0, 100, 4, 4, 101, 2, 0, None, fake, 2, lam, None, None) == 1
    dup = (ctypes.c_int64 * 3)(1, 4, 4)
    assert L.mds_pivot_mds(fake, 0, 100, 4, 4, 3, 2, 0, dup, fake, 2, lam, None, None) == 1
    assert L.mds_pivot_mds(fake, 0, 100, 4, 4, 10, 3, 0, None, fake, 2, lam, None, None) == 1
    # dissimilarity input and affine form: NULL model / matrix
    model = ctypes.c_void_p()
    assert L.mds_fit_from_sqdist(None, 10, 10, 2, None, ctypes.byref(model)) == 1
    assert L.mds_fit_from_sqdist(fake, 10, 9, 2, None, ctypes.byref(model)) == 1
    assert L.mds_embed_from_sqdist(None, fake, 0, 10, 10, 1, fake, 2, None) == 1
    assert L.mds_embed_affine(None, fake, 0, 10, 4, 1, fake, 2, None) == 1


def test_noalloc_maxmin_limits_need_no_gpu(L):
    """The no-allocation MaxMin rejects sizes past its static array before
    any device work, with a message that names the limit."""
    out = (ctypes.c_int64 * 4)()
    fake = ctypes.c_void_p(256)  # never dereferenced: the size checks come first
    assert L.mds_maxmin_landmarks_noalloc(fake, 0, (1 << 20) + 1, 3, 3, 2, 0, out, None) == 1
    assert b"MDS_NOALLOC_MAX_N" in L.mds_last_error()
    assert L.mds_maxmin_landmarks_noalloc(fake, 0, 1 << 20, 3, 3, 16385, 0, out, None) == 1
    assert b"MDS_NOALLOC_MAX_L" in L.mds_last_error()
    assert L.mds_maxmin_landmarks_noalloc(None, 0, 10, 3, 3, 2, 0, out, None) == 1
