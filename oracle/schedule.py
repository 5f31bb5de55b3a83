"""Oracle block schedule: which row block each step of the solver uses.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper's block selection (Section 5.2, "simplified block memoization";
Algorithm 2 for CD++, Algorithm 5 for Kaczmarz++; the fixed collection of
Algorithm 1) draws random numbers but never looks at the iterate, so the whole
sequence of blocks is a function of the seed alone.  The random numbers come
from SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): a 64-bit Weyl counter followed by a fixed mixing
function.  The GPU library implements the same published generator on its own;
the two schedules are compared bit for bit by the tests.

Derived draws (all integer arithmetic, so both sides agree exactly):
  uniform()   = (next() >> 11) * 2**-53                 in [0, 1)
  bounded(k)  = ((next() >> 11) * k) >> 53               in [0, k)
  subset(N,s) = sorted first s entries of a partial Fisher-Yates shuffle of
                0..N-1, swapping position j with j + bounded(N - j)

Modes
  online : step 0 always draws a new block; step t >= 1 draws u = uniform()
           and takes a new block iff u < B0 / t, where
           B0 = (rate_dim / s) * ln(log_dim); otherwise it reuses block
           bounded(|collection|).  (Section 5.2; Alg. 2 uses n/s log n, Alg. 5
           min(m, n)/s log m.)  A uniform is drawn at step 0 as well.
  fixed  : the collection is drawn up front (Algorithm 1): either a random
           partition of 0..N-1 into ceil(N/s) blocks (full Fisher-Yates, then
           consecutive chunks of s, the last one possibly shorter), or
           num_blocks independent s-subsets.  Step t uses bounded(B).
  off    : a new s-subset at every step ("without memoization", Section 6.2).

Natural logarithm throughout (the paper does not state the base).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


class SplitMix64:
    """SplitMix64 as published: state += golden gamma; output = mix(state)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + GOLDEN) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)

    def bounded(self, k: int) -> int:
        if k <= 0:
            raise ValueError("bounded(k) needs k >= 1")
        return ((self.next() >> 11) * k) >> 53


def _partial_shuffle(g: SplitMix64, N: int, s: int) -> np.ndarray:
    perm = list(range(N))
    for j in range(s):
        k = j + g.bounded(N - j)
        perm[j], perm[k] = perm[k], perm[j]
    return np.asarray(perm, dtype=np.int64)


def random_subset(g: SplitMix64, N: int, s: int) -> np.ndarray:
    """Uniform s-subset of {0..N-1}, sorted ascending."""
    return np.sort(_partial_shuffle(g, N, s)[:s])


@dataclasses.dataclass
class Schedule:
    blocks: List[np.ndarray]      # each a sorted int64 array of row indices
    step_block: np.ndarray        # block id used at each step
    new_block: np.ndarray         # bool per step: first use of its block

    def rows(self, t: int) -> np.ndarray:
        return self.blocks[int(self.step_block[t])]


def online_rate(kind: str, m: int, n: int, s: int) -> float:
    """B0 of the Bernoulli(min(1, B0 / t)) new-block rule."""
    if kind == "psd":
        return (float(n) / float(s)) * math.log(float(n))
    return (float(min(m, n)) / float(s)) * math.log(float(m))


def make_schedule(mode: str, N: int, s: int, T: int, seed: int, *, B0: float = 0.0,
                  num_blocks: int = 0, partition: bool = True) -> Schedule:
    """Block schedule for T steps over row indices 0..N-1 with block size s."""
    if not (1 <= s <= N):
        raise ValueError("block size must satisfy 1 <= s <= N")
    g = SplitMix64(seed)
    blocks: List[np.ndarray] = []
    step_block = np.zeros(T, dtype=np.int64)
    new_block = np.zeros(T, dtype=bool)
    if mode == "fixed":
        if partition:
            perm = _partial_shuffle(g, N, N - 1) if N > 1 else np.zeros(1, np.int64)
            for lo in range(0, N, s):
                blocks.append(np.sort(perm[lo:lo + s]))
        else:
            if num_blocks < 1:
                raise ValueError("fixed collection needs num_blocks >= 1")
            for _ in range(num_blocks):
                blocks.append(random_subset(g, N, s))
        seen = set()
        for t in range(T):
            j = g.bounded(len(blocks))
            step_block[t] = j
            new_block[t] = j not in seen
            seen.add(j)
    elif mode == "online":
        for t in range(T):
            u = g.uniform()
            if t == 0 or u < B0 / float(t):
                blocks.append(random_subset(g, N, s))
                step_block[t] = len(blocks) - 1
                new_block[t] = True
            else:
                step_block[t] = g.bounded(len(blocks))
    elif mode == "off":
        for t in range(T):
            blocks.append(random_subset(g, N, s))
            step_block[t] = t
            new_block[t] = True
    else:
        raise ValueError(f"unknown schedule mode {mode!r}")
    return Schedule(blocks=blocks, step_block=step_block, new_block=new_block)
