"""Error metrics between an embedding and its FP64 reference.

The paper states no tolerance; its quality measures compare configurations
after Procrustes alignment (Section 4.1).  Here both sides use the same
landmarks, eigenvector sign convention and row order, so coordinates are
compared directly, column by column:

* ``rms_rel``    worst column of |Y_k - R_k|_2 / |R_k|_2 (the binding metric)
* ``maxabs_rms`` worst column of max|Y_k - R_k| / rms(R_k)
* ``frob_rel``   |Y - R|_F / |R|_F

A reference column that is exactly zero (a dead eigen-direction) must be
matched by exact zeros; otherwise the column's error is reported as inf.
"""

import numpy as np


def column_errors(Y, R):
    Y = np.asarray(Y, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    if Y.shape != R.shape:
        raise ValueError(f"shape mismatch {Y.shape} vs {R.shape}")
    rms_rel = []
    maxabs_rms = []
    for k in range(R.shape[1]):
        d = Y[:, k] - R[:, k]
        nr = np.linalg.norm(R[:, k])
        if nr == 0.0:
            bad = np.any(Y[:, k] != 0.0)
            rms_rel.append(np.inf if bad else 0.0)
            maxabs_rms.append(np.inf if bad else 0.0)
            continue
        rms = nr / np.sqrt(R.shape[0])
        rms_rel.append(np.linalg.norm(d) / nr)
        maxabs_rms.append(np.max(np.abs(d)) / rms)
    nR = np.linalg.norm(R)
    frob = np.linalg.norm(Y - R) / nR if nR > 0 else float(np.linalg.norm(Y))
    return {
        "rms_rel": float(max(rms_rel)) if rms_rel else 0.0,
        "maxabs_rms": float(max(maxabs_rms)) if maxabs_rms else 0.0,
        "frob_rel": float(frob),
        "per_column_rms_rel": [float(x) for x in rms_rel],
    }
