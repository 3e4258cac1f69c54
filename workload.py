"""Seeded synthetic inputs: random-walk collections and query sets.

This module holds no part of the search method; both the HIP path and the
CPU oracle read the FP32 arrays it produces.

Collections stand in for the paper's Synthetic data set (random walks, Sec. IV
setup): every series is the cumulative sum of i.i.d. N(0, 1) steps,
x_t = s_1 + ... + s_t for t = 1..len, then z-normalised in FP64 with the
population standard deviation and rounded once to FP32.

Queries are either fresh random walks (same recipe, another seed) or noisy
copies: a series of the collection chosen uniformly without replacement, plus
N(0, sigma^2) noise per point, re-z-normalised; sigma cycles through
(0.01, 0.1, 1) by query index.

Generation is chunked: chunk c of a collection is drawn from a generator
seeded with (seed, c), so every chunk can be regenerated on its own and the
collection can be produced on the device that will hold it.  Values drawn on a
GPU differ from values drawn on the CPU for the same seed; each run reads one
array, so the oracle and the kernels always see the same numbers.
"""
from __future__ import annotations

import numpy as np
import torch

CHUNK_ROWS = 1 << 20
SIGMAS = (0.01, 0.1, 1.0)


def _chunk_seed(seed: int, chunk: int) -> int:
    return (int(seed) * 1_000_003 + int(chunk) * 7_919 + 12_345) % (2 ** 63 - 1)


def _znorm_rows64(t: torch.Tensor) -> torch.Tensor:
    mu = t.mean(dim=1, keepdim=True)
    sd = t.std(dim=1, unbiased=False, keepdim=True)
    if bool((sd == 0).any()):
        raise RuntimeError("zero-variance series drawn")
    return (t - mu) / sd


def random_walks(n: int, length: int, seed: int, device="cpu", out: torch.Tensor | None = None,
                 chunk_rows: int = CHUNK_ROWS) -> torch.Tensor:
    """FP32 [n, length] z-normalised random walks on `device` (optionally into `out`)."""
    device = torch.device(device)
    if out is None:
        out = torch.empty((n, length), dtype=torch.float32, device=device)
    for c, start in enumerate(range(0, n, chunk_rows)):
        rows = min(chunk_rows, n - start)
        g = torch.Generator(device=device)
        g.manual_seed(_chunk_seed(seed, c))
        steps = torch.randn((rows, length), dtype=torch.float64, device=device, generator=g)
        walk = torch.cumsum(steps, dim=1)
        del steps
        out[start:start + rows].copy_(_znorm_rows64(walk).to(torch.float32))
        del walk
    return out


def fresh_queries(m: int, length: int, seed: int, device="cpu") -> torch.Tensor:
    """FP32 [m, length] random walks that are not in any collection."""
    return random_walks(m, length, seed + 0x5EED, device=device)


def noisy_queries(data: torch.Tensor, m: int, seed: int, sigmas=SIGMAS):
    """Noisy copies of collection series: (queries FP32 [m, len] on data.device, src ids, sigma per query).

    Source ids and noise come from a CPU numpy generator, so they do not depend
    on the device.
    """
    n, length = data.shape
    rng = np.random.default_rng(seed)
    src = np.sort(rng.choice(n, size=m, replace=False)).astype(np.int64)
    rng.shuffle(src)
    sig = np.array([sigmas[i % len(sigmas)] for i in range(m)], dtype=np.float64)
    noise = rng.standard_normal((m, length)) * sig[:, None]
    base = data[torch.as_tensor(src, device=data.device)].to(torch.float64).cpu()
    q = _znorm_rows64(base + torch.from_numpy(noise)).to(torch.float32)
    return q.to(data.device), src, sig


def planted_duplicates(data: torch.Tensor, pairs) -> None:
    """Overwrite rows: for (dst, src) in pairs, data[dst] = data[src] (exact ties)."""
    for dst, src in pairs:
        data[dst].copy_(data[src])
