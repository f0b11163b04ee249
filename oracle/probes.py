"""Probe vectors for the stochastic trace (oracle; test infrastructure only).

Paper App. B: the moments are estimated as an average of r^dag T_m(h) r over
random vectors with |r_I|^2 = 1, and the estimate is improved by probing with
correlated random vectors.  Three probe kinds (readings of that passage):

* UNIT        -- r = e_I for I = first, first+1, ...; weight 1 each (R = 2N
                 gives the exact trace).
* DENSE_Z4    -- r_I = i^k, k uniform in {0,1,2,3}; weight 1/R.
* COLORED_Z4  -- sites coloured by (x mod px, y mod py); one probe per colour
                 (and per Nambu component if split_nambu), nonzero only on its
                 colour class, with Z4 phases; the probes of one draw partition
                 the identity, so weight 1/ndraw.

The Z4 phase of Nambu index I in draw s is the top two bits of
SplitMix64(seed, counter = s * 2^32 + I), with SplitMix64 as published by
Steele, Lea & Flood (OOPSLA 2014) in the form of Vigna's splitmix64.c:
    z = seed + (counter + 1) * 0x9E3779B97F4A7C15          (mod 2^64)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)
This file is an independent implementation; the GPU library carries its own.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

UNIT, DENSE_Z4, COLORED_Z4 = 0, 1, 2

_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
_C1 = 0xBF58476D1CE4E5B9
_C2 = 0x94D049BB133111EB


def splitmix64(seed: int, counter: int) -> int:
    """One SplitMix64 output for a 64-bit seed and counter (pure Python ints)."""
    z = (seed + (counter + 1) * _GAMMA) & _M64
    z = ((z ^ (z >> 30)) * _C1) & _M64
    z = ((z ^ (z >> 27)) * _C2) & _M64
    return z ^ (z >> 31)


def z4_phase(seed: int, draw: int, index: int) -> complex:
    k = splitmix64(seed, (draw << 32) + index) >> 62
    return (1, 1j, -1, -1j)[k]


@dataclass(frozen=True)
class ProbeGroup:
    kind: int
    count: int           # UNIT: vectors; DENSE_Z4: vectors; COLORED_Z4: draws
    seed: int = 0
    px: int = 1
    py: int = 1
    split_nambu: int = 0
    first: int = 0       # UNIT only: first Nambu index
    weight: float = 1.0

    def nprobes(self) -> int:
        if self.kind == COLORED_Z4:
            return self.count * self.px * self.py * (2 if self.split_nambu else 1)
        return self.count


def probe_vector(g: ProbeGroup, q: int, Lx: int, Ly: int) -> np.ndarray:
    """The q-th probe of group g as a dense complex vector of length 2N."""
    N = Lx * Ly
    r = np.zeros(2 * N, dtype=np.complex128)
    if g.kind == UNIT:
        r[g.first + q] = 1.0
        return r
    if g.kind == DENSE_Z4:
        for I in range(2 * N):
            r[I] = z4_phase(g.seed, q, I)
        return r
    if g.kind == COLORED_Z4:
        per = g.px * g.py * (2 if g.split_nambu else 1)
        draw, c = divmod(q, per)
        comp = None
        if g.split_nambu:
            c, comp = divmod(c, 2)
        for i in range(N):
            x, y = i % Lx, i // Lx
            if (x % g.px) + g.px * (y % g.py) != c:
                continue
            for a in range(2):
                if comp is not None and a != comp:
                    continue
                r[2 * i + a] = z4_phase(g.seed, draw, 2 * i + a)
        return r
    raise ValueError("unknown probe kind")


def probe_set(groups, Lx, Ly):
    """(R x 2N probe matrix, weights[R]) for a list of groups, in group order."""
    vecs, w = [], []
    for g in groups:
        for q in range(g.nprobes()):
            vecs.append(probe_vector(g, q, Lx, Ly))
            w.append(g.weight)
    return np.array(vecs), np.array(w, dtype=np.float64)
