"""MaxMin on the library's static scratch array (mds_maxmin_landmarks_noalloc)
against the allocating entry point, through the C ABI (needs a GPU).

Landmark indices are integers: they must agree bit for bit with
mds_maxmin_landmarks, on two calls in a row (the second smaller, so that it
runs on what the first left in the shared array), for FP32 and FP64 input,
and on a small case also with the oracle's MaxMin."""

import numpy as np
import pytest

from oracle import pivot as opv
from synth import generators as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def mds():
    import paper_2007_11919_amd as m
    return m


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["f32", "f64"])
def test_noalloc_matches_allocating_entry_point(dtype):
    # first call: 300,001 rows (a ragged last row block), 64 landmarks
    X = gen.wide_gaussian(300_001, seed=71, dtype=dtype)
    Xd = torch.from_numpy(X).cuda()
    ref1 = mds().maxmin_landmarks(Xd, 64, first=5)
    got1 = mds().maxmin_landmarks_noalloc(Xd, 64, first=5)
    assert np.array_equal(got1, ref1)
    # second call, smaller: 2,000 rows of strided p = 37 input, 40 landmarks
    Xs = gen.gaussian_columns(2000, np.linspace(9.0, 1.0, 40), seed=72, dtype=dtype)
    Xsd = torch.from_numpy(Xs).cuda()[:, :37]
    ref2 = mds().maxmin_landmarks(Xsd, 40, first=1999)
    got2 = mds().maxmin_landmarks_noalloc(Xsd, 40, first=1999)
    assert np.array_equal(got2, ref2)
    assert np.array_equal(got2, opv.maxmin_landmarks(np.ascontiguousarray(Xs[:, :37]).astype(np.float64),
                                                     40, 1999))


def test_noalloc_limits_and_degenerate_input():
    X = torch.zeros((10, 3), dtype=torch.float32, device="cuda")
    X[:4, 0] = torch.arange(4, dtype=torch.float32, device="cuda")
    # four distinct rows: a fifth landmark is an error, as in the allocating call
    with pytest.raises(mds().MDSError):
        mds().maxmin_landmarks(X, 5)
    with pytest.raises(mds().MDSError):
        mds().maxmin_landmarks_noalloc(X, 5)
    # the flag set by the failed call does not leak into the next one
    assert np.array_equal(mds().maxmin_landmarks_noalloc(X, 4), mds().maxmin_landmarks(X, 4))
    big = torch.empty((1 << 20) + 1, 1, dtype=torch.float32, device="cuda")
    with pytest.raises(mds().MDSError, match="MDS_NOALLOC_MAX_N"):
        mds().maxmin_landmarks_noalloc(big, 2)
