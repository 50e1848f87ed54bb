"""Shared test helpers: grid conversions and error norms (no method arithmetic)."""
from __future__ import annotations

import numpy as np

from paper_1206_6152_amd import inputs


def oracle_grid(w):
    from oracle import Grid
    return Grid(n=w.n, nv=w.nv, L=w.L, vmin=w.vmin, vmax=w.vmax, G=w.G, bc=w.bc)


def rel_l1(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a - b).sum())


def structured_f(shape, seed: int) -> np.ndarray:
    """Nonnegative test field mixing a smooth bump, noise, plateaus and empty cells."""
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.linspace(-1, 1, s) for s in shape], indexing="ij", sparse=True)
    r2 = sum(g * g for g in grids)
    smooth = np.exp(-2.0 * r2)
    noise = rng.uniform(0, 1, shape)
    mask = rng.uniform(0, 1, shape) < 0.7
    f = (smooth + 0.3 * noise) * mask
    f[tuple(slice(0, max(1, s // 3)) for s in shape)] = 0.0
    return f


def small_workload(bc: int, n=(4, 6, 8), nv=(12, 8, 6)) -> inputs.Workload:
    """Uneven axis lengths, every sweep kernel kind, and equal spacings (isolated)."""
    d = 0.25
    return inputs.Workload(name="small", n=tuple(n), nv=tuple(nv), L=tuple(d * x for x in n),
                           vmin=(-1.0, -2.0, -0.5), vmax=(1.5, 2.0, 0.5), G=1.0, bc=bc)
