"""Seeded synthetic LSAP instances.

This module only draws random numbers and lays them out as benefit
matrices; it holds none of the solver's arithmetic.  Both the CPU oracle
(tests) and the GPU path (tests, bench, smoke) take their inputs from here,
so the two sides always see byte-identical instances.

Random source: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator.  Draw number ``k`` of stream ``t`` under seed ``s`` is

    mix64((s XOR t*GAMMA) + (k + 1)*GAMMA)      (all arithmetic mod 2**64)

with GAMMA = 0x9E3779B97F4A7C15 and mix64 the SplitMix64 output finaliser.
Every draw is therefore addressable by its index, and a matrix is filled in
any order (or in chunks) with the same result.

Derived draws:
  * integer in [0, B):  ((r >> 32) * B) >> 32   (multiply-shift; bias < B / 2**32)
  * real in [0, 1):     (r >> 11) * 2**-53       (53 random mantissa bits)

Workload shapes follow the paper's setting (dense n x n benefit matrices,
each point an average over several seeds, Section 4) with integer benefits:
  * ``uniform_matrix``: iid integers in [lo, hi).
  * ``lowrank_matrix``: peer-to-peer demand x capacity shape,
        a_ij = round_half_away((1000.0 * u_i) * c_j) + noise_ij,
    u_i, c_j ~ U(0.1, 1), noise_ij uniform integer in [0, 100).
    Computed in IEEE binary64 in exactly that operation order.
  * ``geom_matrix``: the paper's GEOM instances (Section 4): n points in a
    [0, C] x [0, C] square, a_ij = Euclidean distance of points i and j,
    rounded half away from zero to an integer.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Stream ids.  Each generator uses its own streams so that changing one
# workload never shifts the draws of another.
S_UNIFORM = 0
S_ROW_SCALE = 1
S_COL_SCALE = 2
S_NOISE = 3
S_PERM = 4
S_SIZES = 5
S_ARRIVALS = 6
S_GEOM_X = 7
S_GEOM_Y = 8

_ROW_CHUNK_ELEMS = 1 << 21


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser, in place on a uint64 array."""
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def draws(seed: int, stream: int, k: np.ndarray) -> np.ndarray:
    """Raw 64-bit draws number ``k`` (array of uint64) of ``stream``."""
    with np.errstate(over="ignore"):
        base = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ (np.uint64(stream) * GAMMA)
        x = k.astype(np.uint64, copy=True)
        x += np.uint64(1)
        x *= GAMMA
        x += base
        return _mix64(x)


def to_int_below(r: np.ndarray, bound: int) -> np.ndarray:
    """Map raw draws to integers in [0, bound) (multiply-shift)."""
    if not (1 <= bound <= 1 << 32):
        raise ValueError("bound must be in [1, 2**32]")
    with np.errstate(over="ignore"):
        return (((r >> np.uint64(32)) * np.uint64(bound)) >> np.uint64(32)).astype(np.int64)


def to_unit(r: np.ndarray) -> np.ndarray:
    """Map raw draws to binary64 reals in [0, 1)."""
    return (r >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def round_half_away(x: np.ndarray) -> np.ndarray:
    """C ``round`` for finite binary64 values: nearest integer, halves away from 0."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    fl = np.floor(a)
    r = np.where(a - fl >= 0.5, fl + 1.0, fl)
    return np.where(x < 0, -r, r)


def _row_chunks(n: int, cols: int = None):
    rows = max(1, _ROW_CHUNK_ELEMS // max(n if cols is None else cols, 1))
    for r0 in range(0, n, rows):
        yield r0, min(n, r0 + rows)


def _fill_rows(n: int, fill, cols: int = None) -> None:
    """Run fill(r0, r1) over the row chunks of an n-row matrix (of `cols`
    columns, default n) on a few threads (numpy releases the GIL in its
    array operations; the chunks write disjoint rows, so the result does not
    depend on the order)."""
    chunks = list(_row_chunks(n, cols))
    workers = min(16, os.cpu_count() or 1, len(chunks))
    if workers <= 1:
        for r0, r1 in chunks:
            fill(r0, r1)
        return
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda c: fill(*c), chunks))


def uniform_matrix(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """n x n int32 matrix, entries iid uniform integers in [lo, hi)."""
    if n < 0 or hi <= lo:
        raise ValueError("need n >= 0 and hi > lo")
    out = np.empty((n, n), dtype=np.int32)

    def fill(r0, r1):
        k = np.arange(r0 * n, r1 * n, dtype=np.uint64)
        vals = lo + to_int_below(draws(seed, S_UNIFORM, k), hi - lo)
        out[r0:r1] = vals.reshape(r1 - r0, n)

    _fill_rows(n, fill)
    return out


def lowrank_factors(n: int, seed: int):
    """Row scales u_i and column scales c_j, both U(0.1, 1) in binary64."""
    idx = np.arange(n, dtype=np.uint64)
    u = 0.1 + (1.0 - 0.1) * to_unit(draws(seed, S_ROW_SCALE, idx))
    c = 0.1 + (1.0 - 0.1) * to_unit(draws(seed, S_COL_SCALE, idx))
    return u, c


def lowrank_matrix(n: int, seed: int, noise: int = 100, scale: float = 1000.0, rows: int = None) -> np.ndarray:
    """n x n int32: round((scale * u_i) * c_j) + noise_ij, noise uniform in [0, noise).
    rows: only the first `rows` rows (identical to slicing the full matrix)."""
    u, c = lowrank_factors(n, seed)
    su = scale * u
    out = np.empty((n if rows is None else rows, n), dtype=np.int32)

    def fill(r0, r1):
        prod = su[r0:r1, None] * c[None, :]
        base = round_half_away(prod).astype(np.int64)
        if noise > 0:
            k = np.arange(r0 * n, r1 * n, dtype=np.uint64)
            base += to_int_below(draws(seed, S_NOISE, k), noise).reshape(r1 - r0, n)
        out[r0:r1] = base

    _fill_rows(out.shape[0], fill, n)
    return out


def geom_matrix(n: int, seed: int, side: float = 1000.0) -> np.ndarray:
    """GEOM instance: rounded Euclidean distances between n random points."""
    idx = np.arange(n, dtype=np.uint64)
    x = side * to_unit(draws(seed, S_GEOM_X, idx))
    y = side * to_unit(draws(seed, S_GEOM_Y, idx))
    dx = x[:, None] - x[None, :]
    dy = y[:, None] - y[None, :]
    return round_half_away(np.sqrt(dx * dx + dy * dy)).astype(np.int32)


def permutation(n: int, seed: int) -> np.ndarray:
    """Uniform random permutation of 0..n-1 (Fisher-Yates, draw k for slot n-1-k)."""
    p = np.arange(n, dtype=np.int32)
    if n <= 1:
        return p
    r = draws(seed, S_PERM, np.arange(n - 1, dtype=np.uint64))
    for k in range(n - 1):
        i = n - 1 - k
        j = int(((int(r[k]) >> 32) * (i + 1)) >> 32)
        p[i], p[j] = p[j], p[i]
    return p


def loguniform_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """``count`` sizes n = clamp(floor(lo * exp(U * ln(hi / lo))), lo, hi)."""
    u = to_unit(draws(seed, S_SIZES, np.arange(count, dtype=np.uint64)))
    n = np.floor(lo * np.exp(u * math.log(hi / lo))).astype(np.int64)
    return np.clip(n, lo, hi).astype(np.int32)


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of ``rate`` per second on [0, duration)."""
    out = []
    t = 0.0
    k = 0
    chunk = max(16, int(rate * duration * 1.5) + 16)
    while True:
        u = to_unit(draws(seed, S_ARRIVALS, np.arange(k, k + chunk, dtype=np.uint64)))
        for x in u:
            t += -math.log(1.0 - float(x)) / rate
            if t >= duration:
                return np.asarray(out, dtype=np.float64)
            out.append(t)
        k += chunk


# The single-instance workloads, keyed by name.  Seeds 1..5 are the
# averaging seeds; each instance is a pure function of (name, seed).
def single_instance(name: str, seed: int) -> np.ndarray:
    if name == "uniform256":
        return uniform_matrix(256, 0, 1000, seed)
    if name == "lowrank4096":
        return lowrank_matrix(4096, seed)
    if name == "lowrank16384":
        return lowrank_matrix(16384, seed)
    if name == "geom4096":
        return geom_matrix(4096, seed)
    if name == "geom16384":
        return geom_matrix(16384, seed)
    raise KeyError(name)


def batch_instances(count: int = 512, lo: int = 64, hi: int = 2048, seed: int = 1,
                    vmax: int = 10000):
    """Batched workload: ``count`` square instances, n log-uniform in [lo, hi],
    iid uniform integer benefits in [0, vmax).  Instance b uses seed
    ``seed * 1_000_003 + b`` for its matrix."""
    ns = loguniform_sizes(count, lo, hi, seed)
    return [uniform_matrix(int(n), 0, vmax, seed * 1_000_003 + b) for b, n in enumerate(ns)]


def serving_trace(duration: float, rate: float = 200.0, lo: int = 128, hi: int = 16384, seed: int = 1,
                  pool: int = 64):
    """Serving workload: Poisson arrivals of ``rate`` per second on [0, duration).

    Request k uses instance ``k % pool`` of a pool whose sizes are drawn
    log-uniform in [lo, hi]; pool instance p is ``lowrank_matrix(ns[p],
    seed * 1_000_003 + p)``.  Returns (arrival times, pool sizes).
    """
    return poisson_arrivals(rate, duration, seed), loguniform_sizes(pool, lo, hi, seed)
