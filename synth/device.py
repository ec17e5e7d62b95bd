"""Seeded synthetic inputs generated on the GPU, for workloads too large to
build on the host (the whole-brain case: 15000 x 1.2e6 complex64 = 144 GB).

Like the rest of ``synth`` this holds none of the method's arithmetic: it
makes unit phasors with torch's seeded device generator and hands the tensor
to the caller.  The oracle side never regenerates them; a test copies the rows
it needs to the host.
"""
from __future__ import annotations

import math

import numpy as np


def phasors_planted_device(n: int, t: int, npairs: int, seed: int, jitter: float = 0.1, device="cuda",
                           rows_per_chunk: int = 256):
    """Unit phasors u = exp(i phi) as complex64 [n, t] on `device`, with i.i.d.
    uniform phases phi ~ U[0, 2 pi), plus `npairs` planted pairs (a, b) of
    distinct signals with phi_b(t) = phi_a(t) - lag + eta(t), lag ~ U[0, pi),
    eta ~ N(0, jitter^2).

    Returns (u, pairs [npairs, 2] int64 numpy, lags [npairs] float64 numpy).
    The phases come from torch's device generator seeded with `seed`; the
    choice of pairs and lags from numpy's generator with the same seed.
    """
    import torch

    rng = np.random.default_rng(seed)
    verts = rng.permutation(n)[: 2 * npairs]
    pairs = verts.reshape(npairs, 2).astype(np.int64)
    lags = rng.uniform(0.0, math.pi, size=npairs)

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    u = torch.empty((n, t), dtype=torch.complex64, device=device)
    for r0 in range(0, n, rows_per_chunk):
        r1 = min(n, r0 + rows_per_chunk)
        phi = torch.rand((r1 - r0, t), generator=gen, device=device, dtype=torch.float32) * (2.0 * math.pi)
        u[r0:r1] = torch.complex(torch.cos(phi), torch.sin(phi))
        del phi
    step = 16
    for p0 in range(0, npairs, step):
        p1 = min(npairs, p0 + step)
        a = torch.from_numpy(pairs[p0:p1, 0]).to(device)
        b = torch.from_numpy(pairs[p0:p1, 1]).to(device)
        lag = torch.from_numpy(lags[p0:p1]).to(device=device, dtype=torch.float32)[:, None]
        eta = torch.randn((p1 - p0, t), generator=gen, device=device, dtype=torch.float32) * float(jitter)
        ang = eta - lag
        u[b] = u[a] * torch.complex(torch.cos(ang), torch.sin(ang))
        del eta, ang
    return u, pairs, lags
