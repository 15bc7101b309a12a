"""Seeded synthetic graph generators (input side only).

This module builds the weighted undirected loop-free graphs the Fiedler
solver consumes, as symmetric adjacency CSR (both directions stored, no
diagonal, strictly increasing columns per row).  It contains none of the
method's arithmetic: no Laplacian, no coarsening, no iteration.  Both the
CPU oracle (through the tests) and the GPU library consume its output.

All randomness is counter based: the i-th draw of a stream is the SplitMix64
output function (Steele, Lea & Flood, OOPSLA 2014) applied to
``state0 + (i + 1) * GAMMA`` where ``state0`` is derived from (seed, tag).
Identical seeds therefore give byte-identical graphs on every machine.

Workload families (stand-ins for the paper's University of Florida graphs,
Section 4, Table 2, which are mesh-like plus one social network):
  * 2D 5-point and 3D 7-point grid graphs,
  * random geometric graphs (mesh-like, spatially local),
  * Chung-Lu power-law graphs (skewed degrees),
  * closed-form families used as pins (path, cycle, complete, star).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
GAMMA = np.uint64(0x9E3779B97F4A7C15)

# Stream tags (arbitrary distinct constants).
TAG_X = 1
TAG_Y = 2
TAG_W = 3
TAG_CL = 4
TAG_ER = 5
TAG_STREAM = 6


def mix64(z):
    """SplitMix64 output function on a uint64 numpy array (wrapping)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _state0(seed: int, tag: int) -> np.uint64:
    s = np.uint64((int(seed) ^ (int(tag) << 40)) & 0xFFFFFFFFFFFFFFFF)
    return mix64(np.array([s], dtype=np.uint64))[0]


def stream_u64(seed: int, tag: int, idx) -> np.ndarray:
    """i-th 64-bit output of the SplitMix64 stream (seed, tag)."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        st = _state0(seed, tag) + (idx + np.uint64(1)) * GAMMA
    return mix64(st)


def stream_uniform(seed: int, tag: int, idx) -> np.ndarray:
    """Uniform doubles in [0, 1): top 53 bits of the stream output."""
    return (stream_u64(seed, tag, idx) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclasses.dataclass
class CSR:
    """Symmetric adjacency in CSR form (int32 indices)."""

    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray  # int32[nnz]
    w: np.ndarray  # float64[nnz] (or float32)
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def astype(self, dtype) -> "CSR":
        return CSR(self.n, self.row_ptr, self.col, self.w.astype(dtype), self.name)

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        a[rows, self.col] = self.w
        return a

    def edges(self):
        """Undirected edge list (u < v) with weights."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        c = self.col.astype(np.int64)
        keep = rows < c
        return rows[keep], c[keep], self.w[keep]


def from_edges(n: int, u, v, w=None, name: str = "") -> CSR:
    """Build symmetric CSR from an undirected edge list.

    Self-loops are dropped; parallel edges are merged by summing weights.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if w is None:
        w = np.ones(u.shape[0], dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    keep = u != v
    u, v, w = u[keep], v[keep], w[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = a * n + b
    order = np.argsort(key, kind="stable")
    key = key[order]
    w = w[order]
    # key is sorted: runs of equal keys are the parallel edges
    first = np.ones(key.shape[0], dtype=bool)
    first[1:] = key[1:] != key[:-1]
    start = np.nonzero(first)[0]
    uniq = key[start]
    wsum = np.add.reduceat(w, start) if len(key) else w
    a = uniq // n
    b = uniq % n
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    ww = np.concatenate([wsum, wsum])
    k2 = rows * n + cols
    o2 = np.argsort(k2, kind="stable")
    rows, cols, ww = rows[o2], cols[o2], ww[o2]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("nnz does not fit int32")
    return CSR(n, row_ptr.astype(np.int32), cols.astype(np.int32), ww, name)


def hashed_weights(seed: int, a, b, levels: int = 8) -> np.ndarray:
    """Integer weights 1..levels from a hash of the endpoint pair (a < b)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    key = (a << np.uint64(32)) | b
    h = stream_u64(seed, TAG_W, key)
    return (h % np.uint64(levels)).astype(np.float64) + 1.0


def with_int_weights(g: CSR, seed: int, levels: int = 8) -> CSR:
    """Replace weights by symmetric hashed integers in 1..levels."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    c = g.col.astype(np.int64)
    a = np.minimum(rows, c)
    b = np.maximum(rows, c)
    return CSR(g.n, g.row_ptr, g.col, hashed_weights(seed, a, b, levels), g.name + "+w")


# ----------------------------------------------------------------- closed forms

def path(n: int) -> CSR:
    i = np.arange(n - 1)
    return from_edges(n, i, i + 1, name=f"path{n}")


def cycle(n: int) -> CSR:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, name=f"cycle{n}")


def complete(n: int) -> CSR:
    u, v = np.triu_indices(n, 1)
    return from_edges(n, u, v, name=f"K{n}")


def star(n: int) -> CSR:
    """Star K_{1,n-1}: centre 0."""
    i = np.arange(1, n)
    return from_edges(n, np.zeros(n - 1, dtype=np.int64), i, name=f"star{n}")


def grid2d(rows: int, cols: int, wx: float = 1.0, wy: float = 1.0) -> CSR:
    """5-point grid graph; vertex (r, c) has id r*cols + c.

    Horizontal edges (along c) carry weight wx, vertical edges weight wy.
    """
    n = rows * cols
    ids = np.arange(n, dtype=np.int64).reshape(rows, cols)
    hu = ids[:, :-1].ravel()
    vu = ids[:-1, :].ravel()
    u = np.concatenate([hu, vu])
    v = np.concatenate([hu + 1, vu + cols])
    w = np.concatenate([np.full(hu.size, wx), np.full(vu.size, wy)])
    return from_edges(n, u, v, w, name=f"grid{rows}x{cols}")


def mirrored_prism(a: int) -> CSR:
    """Two copies of the a x a five-point grid joined vertex to vertex (unit
    weights).  Copy 0 labels (r, c) as a r + c, copy 1 as 2 a^2 - 1 - (a r + c),
    so the label reversal i -> n-1-i swaps the copies: an automorphism under
    which the ramp i - (n-1)/2 is odd, while every vector that is constant
    across the copies (the whole lambda_2 eigenspace of the grid, for a >= 2)
    is even."""
    m = a * a
    ids = np.arange(m, dtype=np.int64).reshape(a, a)
    hu, vu = ids[:, :-1].ravel(), ids[:-1, :].ravel()
    u0 = np.concatenate([hu, vu])
    v0 = np.concatenate([hu + 1, vu + a])
    mirror = lambda x: 2 * m - 1 - x  # noqa: E731
    u = np.concatenate([u0, mirror(u0), np.arange(m)])
    v = np.concatenate([v0, mirror(v0), mirror(np.arange(m))])
    return from_edges(2 * m, u, v, name=f"prism{a}")


def grid3d(s: int, dtype=np.float64) -> CSR:
    """3D 7-point grid graph s^3; id = (s*z + y)*s + x; unit weights.

    Built directly in CSR (neighbour offsets are already in ascending
    order), so 256^3 needs no global sort.
    """
    n = s * s * s
    idx = np.arange(n, dtype=np.int64)
    x = idx % s
    y = (idx // s) % s
    z = idx // (s * s)
    offs = [(-s * s, z > 0), (-s, y > 0), (-1, x > 0), (1, x < s - 1), (s, y < s - 1), (s * s, z < s - 1)]
    deg = np.zeros(n, dtype=np.int64)
    for _, m in offs:
        deg += m
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    fill = row_ptr[:-1].copy()
    for off, m in offs:
        pos = fill[m]
        col[pos] = (idx[m] + off).astype(np.int32)
        fill += m
    del fill, x, y, z
    w = np.ones(nnz, dtype=dtype)
    return CSR(n, row_ptr.astype(np.int32), col, w, name=f"grid3d_{s}")


# ----------------------------------------------------------------- components

def lcc(g: CSR) -> CSR:
    """Largest connected component, vertex order preserved."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    a = sp.csr_matrix((np.ones(g.nnz, dtype=np.int8), g.col, g.row_ptr), shape=(g.n, g.n))
    ncomp, lab = connected_components(a, directed=False)
    if ncomp == 1:
        return g
    counts = np.bincount(lab)
    big = int(np.argmax(counts))
    keep = lab == big
    newid = np.full(g.n, -1, dtype=np.int64)
    newid[keep] = np.arange(int(keep.sum()))
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    m = keep[rows]
    r2 = newid[rows[m]]
    c2 = newid[g.col[m].astype(np.int64)]
    w2 = g.w[m]
    n2 = int(keep.sum())
    # rows/cols stay sorted because relabelling is monotone
    counts2 = np.bincount(r2, minlength=n2)
    rp = np.zeros(n2 + 1, dtype=np.int64)
    np.cumsum(counts2, out=rp[1:])
    return CSR(n2, rp.astype(np.int32), c2.astype(np.int32), w2, g.name + "_lcc")


def is_connected(g: CSR) -> bool:
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    a = sp.csr_matrix((np.ones(g.nnz, dtype=np.int8), g.col, g.row_ptr), shape=(g.n, g.n))
    return connected_components(a, directed=False)[0] == 1


# ----------------------------------------------------------------- random families

def rgg(npts: int, mean_deg: float = 10.0, seed: int = 14120565, int_weights: bool = True) -> CSR:
    """Random geometric graph in the unit square, largest component.

    Points are hashed uniforms; edges join pairs at distance < r with
    r = sqrt(mean_deg / (pi * npts)).  Vertices are relabelled in cell order
    (cell side ~ r, row-major over cells, original index inside a cell) for
    mesh-like locality; weights are hashed integers 1..8 on final labels.
    """
    from scipy.spatial import cKDTree

    i = np.arange(npts, dtype=np.uint64)
    x = stream_uniform(seed, TAG_X, i)
    y = stream_uniform(seed, TAG_Y, i)
    r = math.sqrt(mean_deg / (math.pi * npts))
    ncell = max(1, int(1.0 / r))
    cr = np.minimum((y * ncell).astype(np.int64), ncell - 1)
    cc = np.minimum((x * ncell).astype(np.int64), ncell - 1)
    order = np.lexsort((np.arange(npts), cc, cr))
    pts = np.stack([x[order], y[order]], axis=1)
    tree = cKDTree(pts)
    pairs = tree.query_pairs(r, output_type="ndarray")
    g = from_edges(npts, pairs[:, 0], pairs[:, 1], name=f"rgg{npts}")
    g = lcc(g)
    if int_weights:
        g = with_int_weights(g, seed)
    g.name = f"rgg{npts}_d{mean_deg:g}"
    return g


def chung_lu_weights(n: int, gamma: float, mean_deg: float, cap: float) -> np.ndarray:
    """Expected degrees w_i = min(cap, c (i+1)^(-1/(gamma-1))), mean = mean_deg."""
    ex = -1.0 / (gamma - 1.0)
    base = (np.arange(1, n + 1, dtype=np.float64)) ** ex
    lo, hi = 0.0, 1.0
    while np.minimum(cap, hi * base).mean() < mean_deg:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.minimum(cap, mid * base).mean() < mean_deg:
            lo = mid
        else:
            hi = mid
    return np.minimum(cap, hi * base)


def chung_lu(n: int, gamma: float = 2.1, mean_deg: float = 16.0, cap: float = 50000.0,
             seed: int = 14120565, int_weights: bool = False) -> CSR:
    """Edge-sampling Chung-Lu graph, largest component (hubs first).

    M = n*mean_deg/2 endpoint pairs are drawn i.i.d. proportional to the
    expected degrees by inverse-CDF sampling; self-loops are dropped and
    duplicates merged to one edge (so realised mean degree < mean_deg).
    """
    w = chung_lu_weights(n, gamma, mean_deg, cap)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m = int(n * mean_deg / 2)
    out_u = []
    out_v = []
    chunk = 1 << 23
    for s0 in range(0, m, chunk):
        cnt = min(chunk, m - s0)
        idx = np.arange(2 * s0, 2 * (s0 + cnt), dtype=np.uint64)
        uu = stream_uniform(seed, TAG_CL, idx)
        # inverse CDF; queries in sorted order (same result, cache-friendly)
        order = np.argsort(uu)
        e = np.empty(uu.shape[0], dtype=np.int64)
        e[order] = np.searchsorted(cdf, uu[order], side="right")
        e = np.minimum(e, n - 1)
        out_u.append(e[0::2])
        out_v.append(e[1::2])
    u = np.concatenate(out_u)
    v = np.concatenate(out_v)
    g = from_edges(n, u, v, np.ones(u.shape[0]), name=f"chunglu{n}")
    # merge duplicates to unit weight
    g = CSR(g.n, g.row_ptr, g.col, np.ones(g.nnz, dtype=np.float64), g.name)
    g = lcc(g)
    if int_weights:
        g = with_int_weights(g, seed)
    g.name = f"chunglu{n}_g{gamma:g}_d{mean_deg:g}"
    return g


def erdos_renyi_connected(n: int, p: float, seed: int, int_weights: bool = True) -> CSR:
    """G(n, p) plus a random spanning path (so it is connected)."""
    iu, iv = np.triu_indices(n, 1)
    r = stream_uniform(seed, TAG_ER, np.arange(iu.size, dtype=np.uint64))
    keep = r < p
    perm = np.argsort(stream_u64(seed, TAG_ER + 100, np.arange(n, dtype=np.uint64)))
    u = np.concatenate([iu[keep], perm[:-1]])
    v = np.concatenate([iv[keep], perm[1:]])
    g = from_edges(n, u, v, name=f"er{n}")
    g = CSR(g.n, g.row_ptr, g.col, np.ones(g.nnz), g.name)
    if int_weights:
        g = with_int_weights(g, seed)
    return g


# ----------------------------------------------------------------- named workloads

def workload(name: str, seed: int = 14120565) -> CSR:
    """Named configurations.

    grid128  : 2D 128x128 5-point grid, unit weights, FP64 (16,384 vertices).
    rgg1m    : random geometric graph, 1M points, mean degree ~10, LCC,
               integer weights 1..8.
    grid3d256: 3D 256^3 7-point grid, unit weights (16.8M vertices).
    chunglu4m: Chung-Lu, 4M vertices, exponent 2.1, mean degree 16, cap 50k.
    Smaller stand-ins used by tests: rgg<k>k, chunglu<k>k, grid3d<s>.
    """
    if name == "grid128":
        return grid2d(128, 128)
    if name == "rgg1m":
        return rgg(1_000_000, 10.0, seed)
    if name == "grid3d256":
        return grid3d(256, dtype=np.float32)
    if name == "chunglu4m":
        g = chung_lu(4_000_000, 2.1, 16.0, 50000.0, seed)
        return g.astype(np.float32)
    if name.startswith("rgg") and name.endswith("k"):
        return rgg(int(name[3:-1]) * 1000, 10.0, seed)
    if name.startswith("chunglu") and name.endswith("k"):
        k = int(name[7:-1]) * 1000
        return chung_lu(k, 2.1, 16.0, min(50000.0, math.sqrt(16.0 * k) * 10), seed)
    if name.startswith("grid3d"):
        return grid3d(int(name[6:]))
    raise KeyError(name)


# ----------------------------------------------------------------- served stream

TAG_POOL = 7


def serve_pool(count: int, seed: int = 14120565, nmin: int = 1000, nmax: int = 1_000_000):
    """Seeded pool of request graphs for the serving workload.

    Sizes are log-uniform in [nmin, nmax]; the family is uniform over
    {2D grid with side round(sqrt(n)), RGG with mean degree 10, Chung-Lu
    with exponent 2.5, mean degree 8 and degree cap sqrt(8 n)}; integer
    weights 1..8.  Returns a list of (graph_id, CSR).
    """
    out = []
    for i in range(count):
        u = float(stream_uniform(seed, TAG_POOL, np.array([2 * i], dtype=np.uint64))[0])
        f = float(stream_uniform(seed, TAG_POOL, np.array([2 * i + 1], dtype=np.uint64))[0])
        n = int(nmin * (nmax / nmin) ** u)
        fam = min(2, int(3 * f))
        gseed = seed + 1000 + i
        if fam == 0:
            side = max(2, int(round(math.sqrt(n))))
            g = with_int_weights(grid2d(side, side), gseed)
        elif fam == 1:
            g = rgg(n, 10.0, gseed)
        else:
            g = chung_lu(n, 2.5, 8.0, math.sqrt(8.0 * n), gseed, int_weights=True)
        g.name = f"pool{i}_{['grid', 'rgg', 'chunglu'][fam]}_{g.n}"
        out.append((g.name, g))
    return out
