"""Orthonormalisation of new search directions (Sec. 2.1; test infrastructure only).

The paper orthogonalises new directions against the current subspace and each
other with modified Gram-Schmidt before appending them.  The oracle takes one
reading of the details that the paper leaves open: every input direction is
first scaled to unit norm; it is then projected out of the current basis twice
(classical Gram-Schmidt, two passes), then out of the directions already
accepted from the same block twice (modified Gram-Schmidt, two passes); a
direction whose remaining norm is below ``drop_tol`` is discarded.
"""

from __future__ import annotations

import numpy as np


def orthonormalize(w: np.ndarray, v: np.ndarray | None = None, drop_tol: float = 1e-8) -> np.ndarray:
    """Return an orthonormal block spanning the part of w's columns not in v.

    w: (N, nnew); v: (N, m) with orthonormal columns, or None.
    Output: (N, nkept), nkept <= nnew, orthogonal to v.
    """
    n = w.shape[0]
    kept = []
    for j in range(w.shape[1]):
        c = np.array(w[:, j], dtype=np.float64)
        nrm = np.linalg.norm(c)
        if not np.isfinite(nrm) or nrm == 0.0:
            continue
        c /= nrm
        if v is not None and v.shape[1] > 0:
            for _ in range(2):
                c -= v @ (v.T @ c)
        for _ in range(2):
            for q in kept:
                c -= (q @ c) * q
        nrm = np.linalg.norm(c)
        if nrm < drop_tol:
            continue
        kept.append(c / nrm)
    if not kept:
        return np.zeros((n, 0))
    return np.stack(kept, axis=1)
