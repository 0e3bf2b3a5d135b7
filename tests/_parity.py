"""Shared comparison helpers of the GPU parity tests (no method arithmetic).

rel(a, b)   relative L2 error ||a - b|| / ||b||, the stated 1e-5 bar.
elem(a, b)  largest element-wise error relative to the largest reference
            entry, max|a - b| / max|b|: catches an error confined to a tile
            seam or a border pixel that the L2 norm would average away.
oracle_dual(state)  the q plane of a GPU dual state ([2][m][n][4] float32,
            per pixel (r1, s1, r2, s2), zeros where a difference does not
            exist) as the oracle's unpadded (r1, r2, s1, s2) arrays.
"""
import numpy as np

TOL = 1e-5       # relative L2 against the FP64 oracle at equal K
ELEM_TOL = 1e-5  # element-wise: max|x - x_o| <= ELEM_TOL * max|x_o|


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def elem(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)) if np.size(b) else 0.0


def oracle_dual(state):
    q = np.asarray(state, dtype=np.float64)[0]
    return (q[:-1, :, 0], q[:, :-1, 2], q[:-1, :, 1], q[:, :-1, 3])
