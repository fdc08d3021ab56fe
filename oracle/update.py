"""Resampling and updating the sketches (Section 6), FP64 on the CPU.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Section 6 observes that GN keeps no orthogonal basis, so its two sketch products
can be updated in place:
  * resampling r -> r + dr: only the new columns X_new of X and the new columns
    Y_new of Y are drawn; AX gains the columns A X_new and Y^T A the rows
    Y_new^T A (the core is recomputed, O(r^3));
  * appended rows A -> [A; B]: the sketch Y gains the rows Y_B that belong to the
    new rows, AX -> [AX; B X] and Y^T A -> Y^T A + Y_B^T B (the core becomes
    Y^T A X + Y_B^T B X, formed again from the stacked AX);
  * appended columns A -> [A, B]: X gains the rows X_B, AX -> AX + B X_B and
    Y^T A -> [Y^T A, Y^T B];
  * a perturbation A -> A + E: AX -> AX + E X and Y^T A -> Y^T A + Y^T E.
With the counter-based sketches of oracle.philox, "the new columns / rows" are
the entries at the new indices of the same streams, so the updated products are
exactly the products of the enlarged problem.  Pins (tests/test_oracle_update.py):
each update equals a fresh sketch pass over the enlarged or perturbed matrix with
the enlarged sketches, and the sketches are prefix-stable in rows and columns.
"""
from __future__ import annotations

import numpy as np

from . import philox


def gaussian_block(seed: int, stream: int, rows: int, cols: int, row0: int = 0,
                   col0: int = 0) -> np.ndarray:
    return philox.gaussian(seed, stream, rows, cols, row0=row0, col0=col0)


def extend_rank(A, AX, YA, X_new, Y_new):
    """Resampling: [AX, A X_new] and [Y^T A; Y_new^T A]."""
    return np.hstack([AX, A @ X_new]), np.vstack([YA, Y_new.T @ A])


def append_rows(AX, YA, B, X, Y_B):
    """A -> [A; B]: [AX; B X] and Y^T A + Y_B^T B."""
    return np.vstack([AX, B @ X]), YA + Y_B.T @ B


def append_cols(AX, YA, B, X_B, Y):
    """A -> [A, B]: AX + B X_B and [Y^T A, Y^T B]."""
    return AX + B @ X_B, np.hstack([YA, Y.T @ B])


def perturb(AX, YA, E, X, Y):
    """A -> A + E: AX + E X and Y^T A + Y^T E."""
    return AX + E @ X, YA + Y.T @ E
