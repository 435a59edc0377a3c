"""FP64 CPU oracle of interpolation MDS and divide-and-conquer MDS.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import or run anything in this
package.  The HIP library never calls it and shares no code with it; the two
meet only through the seeded input generators of ``synth``.

Pin status (what fixes each part independently of this code):
* sampler       - published SplitMix64 test vector, Lemire power-of-two
                  closed form, exhaustive Fisher-Yates enumeration, chi^2.
* classical MDS - brute-force Jacobi on tiny n, SVD closed form (PCA),
                  double-centring identities, eigen residuals, eq. (1).
* interpolation - landmark self-reproduction, Proposition 1 (eq. (3)),
                  exact recovery of data lying in R^r, l = n reduces to
                  classical MDS, invariance under rigid motions.
* dissimilarity input (fit_from_sqdist, interpolate_sqdist) - equals the
                  vector path on Euclidean input; brute-force Jacobi on a
                  non-Euclidean matrix; self-reproduction and Proposition 1
                  for non-Euclidean input.
* MaxMin and pivot MDS (oracle.pivot, Section 3.1) - MaxMin checked step
                  by step by brute force and on a line whose sequence is
                  known; pivot MDS with every point a pivot is brute-force
                  Jacobi classical MDS; the double-centred block equals the
                  inner products of centred points and pivots; the
                  configuration spans the centred data; Section 4.1
                  eigenvalue estimates and correlations.
No function is left "parity unpinned".
"""

from .mds import (TAU, DegenerateError, Fit, affine_map, classical_mds, fit_from_sqdist, fit_landmarks,
                  gower_block, inner_products, interpolate, interpolate_affine, interpolate_sqdist,
                  interpolation_mds,
                  interpolation_mds_paper_layout, lmds_block, sign_convention,
                  sqdist_rows, sqdist_rows_expanded, top_eigenpairs)
from .sampler import SplitMix64, bounded, fisher_yates_prefix, sample_landmarks
from .linalg_small import jacobi_eigh, procrustes
from . import dc
from . import pivot

__all__ = [
    "TAU", "DegenerateError", "Fit", "affine_map", "classical_mds", "fit_from_sqdist", "fit_landmarks",
    "interpolate_affine",
    "interpolate_sqdist",
    "gower_block", "inner_products", "interpolate", "interpolation_mds",
    "interpolation_mds_paper_layout", "lmds_block", "sign_convention",
    "sqdist_rows", "sqdist_rows_expanded", "top_eigenpairs", "SplitMix64",
    "bounded", "fisher_yates_prefix", "sample_landmarks", "jacobi_eigh",
    "procrustes", "dc", "pivot",
]
