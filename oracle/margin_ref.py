"""FP64 reference for the reduced-precision dot-product candidate filter (CPU oracle).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.

The paper's systems compute real distances in full precision (Sec. III); a
low-precision pass may only be used as a candidate filter whose error is
bounded rigorously, so that pruning never drops a true answer.  This module
states the quantisers and the bound from their definitions:

  * BF16: round-to-nearest-even of the FP32 value to 8 significant bits.
  * FP8 E4M3 (OCP, max finite 448, subnormal spacing 2^-9): the series is
    divided by a power-of-two scale s = 2^e, the smallest such that
    max|x| / s <= 448, then rounded to nearest-even E4M3; the dequantised
    value is s times the E4M3 value.
  * For q = q~ + e_q and x = x~ + e_x:  q.x - q~.x~ = q.e_x + e_q.x~, hence
    |q.x - q~.x~| <= |q| |e_x| + |e_q| |x~|   (Cauchy-Schwarz).
"""
from __future__ import annotations

import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to nearest-even BF16, returned as FP32 values."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r << 16).astype(np.uint32).view(np.float32)


def pow2_scale_e4m3(x: np.ndarray) -> np.ndarray:
    """Per-row scale 2^e, the smallest power of two with max|x_row| / 2^e <= 448."""
    amax = np.abs(np.asarray(x, np.float64)).max(axis=-1)
    e = np.zeros_like(amax)
    nz = amax > 0
    e[nz] = np.ceil(np.log2(amax[nz] / 448.0))
    # guard the ceil against log2 rounding: make sure amax / 2^e <= 448 and amax / 2^(e-1) > 448
    s = np.exp2(e)
    bump = nz & (amax / s > 448.0)
    e[bump] += 1
    drop = nz & (amax / np.exp2(e - 1) <= 448.0)
    e[drop] -= 1
    return np.exp2(e)


def e4m3_round(y: np.ndarray) -> np.ndarray:
    """Round FP64 values (already scaled into [-448, 448]) to nearest-even E4M3 values."""
    y = np.asarray(y, dtype=np.float64)
    a = np.abs(y)
    with np.errstate(divide="ignore"):
        ex = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    ex = np.maximum(ex, -6.0)                      # subnormal range shares the 2^-6 binade quantum
    quantum = np.exp2(ex - 3.0)
    r = np.round(y / quantum) * quantum            # np.round: ties to even
    return np.clip(r, -448.0, 448.0)


def quantise_rows(X: np.ndarray, kind: str):
    """Dequantised copy x~ (FP64) and per-row scale for kind in {'bf16', 'fp8'}."""
    X = np.asarray(X, dtype=np.float32)
    if kind == "bf16":
        return bf16_round(X).astype(np.float64), np.ones(X.shape[0])
    if kind == "fp8":
        s = pow2_scale_e4m3(X)
        return e4m3_round(X.astype(np.float64) / s[:, None]) * s[:, None], s
    raise ValueError(kind)


def dot_error_bound(q, x, q_t, x_t) -> np.ndarray:
    """|q| |x - x~| + |q - q~| |x~| for all (query, series) pairs, FP64."""
    q = np.asarray(q, np.float64)
    x = np.asarray(x, np.float64)
    nq = np.linalg.norm(q, axis=1)
    neq = np.linalg.norm(q - q_t, axis=1)
    nex = np.linalg.norm(x - x_t, axis=1)
    nxt = np.linalg.norm(x_t, axis=1)
    return nq[:, None] * nex[None, :] + neq[:, None] * nxt[None, :]
