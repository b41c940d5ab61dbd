"""Seeded block-CSR workloads.

Every generator takes a numpy ``Generator`` (PCG64, ``np.random.default_rng``)
or a seed, and draws in a fixed order: A pattern, A values, B pattern, B
values, then the old C.  Patterns with a stated occupancy p hold exactly
``round(p * nbr * nbc)`` blocks chosen uniformly without replacement; values
are drawn block by block in CSR order, column-major inside a block.

The workloads follow the shapes of the paper's benchmarks (square and
tall-and-skinny FP64 products over square blocks, Sec. IV) and of the
block-sparse cases the method targets:

* ``sparse_uniform``   -- 460 x 460 as a 20 x 20 grid of 23-blocks, 10 %;
* ``dense_square``     -- N = 8192 in 32-blocks, every block present;
* ``dense_rect``       -- M = N = 4096, K = 65536 in 32-blocks;
* ``banded_uneven``    -- N ~ 50000 with block sizes drawn from {5,13,23,32},
  occupancy p, magnitudes decaying as exp(-|I-J|/50), blocks whose magnitude
  envelope is below 1e-10 not stored;
* ``wide_range_dense`` / ``wide_range_sparse`` -- entries sign * 10^U(-6,2).
"""
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "BlockCSR", "rng_of", "pattern_random", "pattern_full", "pattern_from_mask", "values_uniform",
    "values_wide_range", "values_integer", "make_matrix", "sparse_uniform", "dense_square",
    "dense_rect", "banded_sizes", "banded_uneven", "wide_range_dense", "wide_range_sparse",
    "block_elems",
]


@dataclass
class BlockCSR:
    """A block-CSR matrix on the host.

    rbs/cbs: int32 block-row / block-column sizes; row_ptr: int64[nbr+1];
    col_ind: int32[nnzb] ascending per row; data: float64 blocks packed in
    CSR order, column-major inside a block (leading dimension = rows).
    """
    rbs: np.ndarray
    cbs: np.ndarray
    row_ptr: np.ndarray
    col_ind: np.ndarray
    data: np.ndarray = field(default=None)

    @property
    def nbr(self):
        return len(self.rbs)

    @property
    def nbc(self):
        return len(self.cbs)

    @property
    def nnzb(self):
        return int(self.row_ptr[-1])

    def shape(self):
        return int(np.sum(self.rbs, dtype=np.int64)), int(np.sum(self.cbs, dtype=np.int64))


def rng_of(seed_or_rng):
    if isinstance(seed_or_rng, np.random.Generator):
        return seed_or_rng
    return np.random.default_rng(seed_or_rng)


def block_elems(rbs, cbs, row_ptr, col_ind):
    rows = np.repeat(np.arange(len(rbs)), np.diff(row_ptr))
    return np.asarray(rbs, dtype=np.int64)[rows] * np.asarray(cbs, dtype=np.int64)[col_ind]


def pattern_from_mask(mask):
    mask = np.asarray(mask, dtype=bool)
    rp = np.zeros(mask.shape[0] + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=rp[1:])
    ci = np.nonzero(mask)[1].astype(np.int32)
    return rp, ci


def pattern_random(rng, nbr, nbc, occupancy=None, nnzb=None):
    """Exactly ``nnzb`` (or round(occupancy*nbr*nbc)) distinct positions."""
    total = int(nbr) * int(nbc)
    if nnzb is None:
        nnzb = int(round(float(occupancy) * total))
    nnzb = int(min(max(nnzb, 0), total))
    flat = np.sort(rng.choice(total, size=nnzb, replace=False)) if nnzb else np.zeros(0, dtype=np.int64)
    rows = flat // nbc
    cols = (flat % nbc).astype(np.int32)
    rp = np.zeros(nbr + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=nbr), out=rp[1:])
    return rp, cols


def pattern_full(nbr, nbc):
    rp = np.arange(nbr + 1, dtype=np.int64) * nbc
    ci = np.tile(np.arange(nbc, dtype=np.int32), nbr)
    return rp, ci


def values_uniform(rng, n):
    return rng.uniform(-1.0, 1.0, size=int(n))


def values_wide_range(rng, n):
    """sign * 10^U(-6, 2): magnitudes spanning 1e-6 .. 1e2, random sign."""
    mag = 10.0 ** rng.uniform(-6.0, 2.0, size=int(n))
    sign = np.where(rng.random(int(n)) < 0.5, -1.0, 1.0)
    return sign * mag


def values_integer(rng, n, lo=-8, hi=8):
    return rng.integers(lo, hi + 1, size=int(n)).astype(np.float64)


def make_matrix(rng, rbs, cbs, occupancy=1.0, values="uniform", nnzb=None, mask=None):
    rbs = np.asarray(rbs, dtype=np.int32)
    cbs = np.asarray(cbs, dtype=np.int32)
    if mask is not None:
        rp, ci = pattern_from_mask(mask)
    elif nnzb is None and occupancy >= 1.0:
        rp, ci = pattern_full(len(rbs), len(cbs))
    else:
        rp, ci = pattern_random(rng, len(rbs), len(cbs), occupancy=occupancy, nnzb=nnzb)
    n = int(block_elems(rbs, cbs, rp, ci).sum())
    if callable(values):
        data = values(rng, n)
    elif values == "uniform":
        data = values_uniform(rng, n)
    elif values == "wide":
        data = values_wide_range(rng, n)
    elif values == "int":
        data = values_integer(rng, n)
    elif values == "zeros":
        data = np.zeros(n)
    else:
        raise ValueError(values)
    return BlockCSR(rbs, cbs, rp, ci, np.ascontiguousarray(data, dtype=np.float64))


def sparse_uniform(seed=0, nb=20, bs=23, occupancy=0.10):
    """460 x 460 as 20 x 20 blocks of 23, 10 % occupancy, U[-1,1]."""
    rng = rng_of(seed)
    sizes = np.full(nb, bs, dtype=np.int32)
    A = make_matrix(rng, sizes, sizes, occupancy)
    B = make_matrix(rng, sizes, sizes, occupancy)
    return A, B


def dense_square(seed=0, n=8192, bs=32):
    rng = rng_of(seed)
    sizes = np.full(n // bs, bs, dtype=np.int32)
    A = make_matrix(rng, sizes, sizes, 1.0)
    B = make_matrix(rng, sizes, sizes, 1.0)
    return A, B


def dense_rect(seed=0, m=4096, n=4096, k=65536, bs=32):
    rng = rng_of(seed)
    ms = np.full(m // bs, bs, dtype=np.int32)
    ns = np.full(n // bs, bs, dtype=np.int32)
    ks = np.full(k // bs, bs, dtype=np.int32)
    A = make_matrix(rng, ms, ks, 1.0)
    B = make_matrix(rng, ks, ns, 1.0)
    return A, B


def banded_sizes(rng, target=50000, choices=(5, 13, 23, 32)):
    """Block sizes drawn i.i.d. from ``choices`` until their sum reaches target."""
    out = []
    s = 0
    while s < target:
        b = int(choices[rng.integers(0, len(choices))])
        out.append(b)
        s += b
    return np.asarray(out, dtype=np.int32)


def _banded_matrix(rng, sizes, occupancy, decay, cutoff):
    nb = len(sizes)
    rp, ci = pattern_random(rng, nb, nb, occupancy=occupancy)
    rows = np.repeat(np.arange(nb), np.diff(rp))
    dist = np.abs(rows - ci.astype(np.int64))
    # Magnitude envelope of a block: exp(-|I-J|/decay) * sqrt(m*n) bounds its
    # Frobenius norm; blocks whose envelope is below the cutoff are not stored.
    env = np.exp(-dist / decay) * np.sqrt(sizes[rows].astype(np.float64) * sizes[ci])
    keep = env >= cutoff
    rows, ci, dist = rows[keep], ci[keep], dist[keep]
    rp = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=nb), out=rp[1:])
    ne = sizes[rows].astype(np.int64) * sizes[ci]
    data = rng.uniform(-1.0, 1.0, size=int(ne.sum())) * np.repeat(np.exp(-dist / decay), ne)
    return BlockCSR(sizes, sizes, rp, ci.astype(np.int32), data)


def banded_uneven(seed=0, occupancy=0.01, target=50000, decay=50.0, cutoff=1e-10,
                  choices=(5, 13, 23, 32)):
    rng = rng_of(seed)
    sizes = banded_sizes(rng, target, choices)
    A = _banded_matrix(rng, sizes, occupancy, decay, cutoff)
    B = _banded_matrix(rng, sizes, occupancy, decay, cutoff)
    return A, B


def wide_range_dense(seed=0, n=16384, bs=32):
    rng = rng_of(seed)
    sizes = np.full(n // bs, bs, dtype=np.int32)
    A = make_matrix(rng, sizes, sizes, 1.0, values="wide")
    B = make_matrix(rng, sizes, sizes, 1.0, values="wide")
    return A, B


def wide_range_sparse(seed=0, nb=1424, bs=23, occupancy=0.20):
    rng = rng_of(seed)
    sizes = np.full(nb, bs, dtype=np.int32)
    A = make_matrix(rng, sizes, sizes, occupancy, values="wide")
    B = make_matrix(rng, sizes, sizes, occupancy, values="wide")
    return A, B
