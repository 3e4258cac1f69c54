"""FP64 reference for the spectral (energy-compacted) filter copy (CPU oracle).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.

The paper prunes with lower bounds computed on a reduced representation of
every series (the iSAX summary of Sec. II) before it computes real distances
(Sec. III).  The spectral copy is another reduced representation with a
lower bound, used by the matrix-core filter:

  * T is the orthonormal DCT-II of length L (rows are the basis vectors), so
    |T v| = |v| for every v and q.x = Tq . Tx.
  * ext_D(x) = (y_0 .. y_{D-2}, |(y_{D-1} .. y_{L-1})|) with y = T x: the first
    D - 1 coefficients and the norm of the rest.  |ext_D(x)| = |x|.
  * Since the dropped part contributes y_t(q).y_t(x) <= |y_t(q)| |y_t(x)|
    (Cauchy-Schwarz), q.x <= ext_D(q).ext_D(x), hence
    ED^2(q, x) >= |q|^2 + |x|^2 - 2 ext_D(q).ext_D(x) = |ext_D(q) - ext_D(x)|^2.
  * The filter quantises ext_D to BF16; the dot-product error identity of
    margin_ref applies to ext_D(q), ext_D(x) and their BF16 copies, with the
    accumulation over D terms.

The DCT matrix comes from scipy's FFT-based DCT; the tests pin it against the
cosine definition and check orthonormality.
"""
from __future__ import annotations

import numpy as np
from scipy.fft import dct

from . import margin_ref


def dct_matrix(L: int) -> np.ndarray:
    """Orthonormal DCT-II matrix T [L, L], FP64: T @ x equals scipy's dct(x, norm='ortho')."""
    return dct(np.eye(L), norm="ortho", axis=0)


def spectral_ext(X: np.ndarray, D: int) -> np.ndarray:
    """ext_D of every row, FP64 [n, D]: D - 1 leading DCT coefficients and the norm of the rest."""
    X = np.asarray(X, dtype=np.float64)
    L = X.shape[1]
    if not 2 <= D <= L:
        raise ValueError("need 2 <= D <= L")
    Y = dct(X, norm="ortho", axis=1)
    return np.concatenate([Y[:, :D - 1], np.linalg.norm(Y[:, D - 1:], axis=1)[:, None]], axis=1)


def spectral_lb_sq(Q: np.ndarray, X: np.ndarray, D: int) -> np.ndarray:
    """|ext_D(q) - ext_D(x)|^2 for all pairs [m, n], FP64: a lower bound on ED^2."""
    eq, ex = spectral_ext(Q, D), spectral_ext(X, D)
    return ((eq[:, None, :] - ex[None, :, :]) ** 2).sum(axis=2)


def spectral_bf16(X: np.ndarray, D: int):
    """(ext_D FP64, its BF16 copy as FP64): each coefficient rounded to FP32, then to BF16."""
    E = spectral_ext(X, D)
    return E, margin_ref.bf16_round(E.astype(np.float32)).astype(np.float64)


def spectral_filter_scores(Q: np.ndarray, X: np.ndarray, D: int):
    """(approx, err) [m, n] of the spectral filter, FP64.

    approx = |q|^2 + |x|^2 - 2 q~.x~ over the BF16 copies of ext_D (dot product exact in FP64),
    err    = 2 (|q| |ext(x) - x~| + |ext(q) - q~| |x~|), so that
    approx - err <= |ext(q) - ext(x)|^2 <= ED^2.
    """
    Q = np.asarray(Q, np.float64)
    X = np.asarray(X, np.float64)
    eq, qt = spectral_bf16(Q, D)
    ex, xt = spectral_bf16(X, D)
    qn = (Q ** 2).sum(axis=1)
    xn = (X ** 2).sum(axis=1)
    approx = qn[:, None] + xn[None, :] - 2.0 * (qt @ xt.T)
    err = 2.0 * margin_ref.dot_error_bound(eq, ex, qt, xt)
    return approx, err
