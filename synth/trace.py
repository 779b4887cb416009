"""Seeded request trace for the serving loop (no arithmetic of the method).

Poisson arrivals at ``rate`` requests/s; each request draws a square grid
n in {64,128,256,512}, nz in {16,32,64,128}, 20 m cubic cells, h = 10 m,
1..16 density models, forward or adjoint (50/50) and gz-only or the full
tensor set (50/50).
"""

from dataclasses import dataclass

import numpy as np

from .geometry import SERVING_N, SERVING_NZ


@dataclass(frozen=True)
class TraceRequest:
    rid: int
    t_arrival: float      # seconds from the start of the trace
    n: int                # nx = ny
    nz: int
    batch: int
    op: str               # "forward" or "adjoint"
    full_tensor: bool     # False: gz only; True: gz, gxx, gxy, gxz, gyy, gyz
    seed: int


def poisson_trace(n_requests=4000, rate=200.0, seed=500, n_choices=SERVING_N,
                  nz_choices=SERVING_NZ, max_batch=16):
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        out.append(TraceRequest(
            rid=i,
            t_arrival=float(t[i]),
            n=int(rng.choice(n_choices)),
            nz=int(rng.choice(nz_choices)),
            batch=int(rng.integers(1, max_batch + 1)),
            op="forward" if rng.random() < 0.5 else "adjoint",
            full_tensor=bool(rng.random() < 0.5),
            seed=10_000 + i,
        ))
    return out
