"""Interpolation MDS (Delicado and Pachon-Garcia, Section 3.1) on one MI355X.

The work runs in libmds.so (HIP for gfx950, C ABI in include/mds.h); this
package only marshals arguments.  There is no CPU fallback: if the library
is missing every call raises.
"""

from .api import (F32, F64, PREC, MDSError, Model, divide_conquer, embed, embed_affine, embed_from_sqdist,
                  fit_from_sqdist, fit_landmarks, free, maxmin_landmarks, maxmin_landmarks_noalloc,
                  pivot_mds, sample_landmarks)

__all__ = ["F32", "F64", "PREC", "MDSError", "Model", "divide_conquer", "embed", "embed_affine", "embed_from_sqdist",
           "fit_from_sqdist", "fit_landmarks", "free", "maxmin_landmarks", "maxmin_landmarks_noalloc", "pivot_mds",
           "sample_landmarks"]
