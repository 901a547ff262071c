"""The paper's standardized test networks (Section 3.5, Table modelspace),
regenerated from their description: N in {10, 30, 100, 300, 1000} vertices
placed at random in a square or cube with a minimum distance between any
two, numbered from the centre outwards, and connected by one of four
classes at a low and a high edge density -- 80 networks in all.

Placement.  Rejection sampling, as the paper describes it: draw a position
uniformly in the space and accept it only if it is at least d_min from every
vertex accepted so far.  The space is L = 500 units a side (Section 3.5's
example); d_min = PACKING * L * N^(-1/D), the packing distance L N^(-1/D)
reduced "to allow for some variability in placement" (PACKING = 0.5 here).
Units are micrometres, so delays follow from a conduction speed as for the
other workloads.

Classes (edges are directed, i -> j; no self-loops, no duplicates):
* lattice: every vertex receives edges from its k nearest vertices,
  k = 3 (low) or 8 (high): nearest-neighbour connections only;
* small world: the k = 8 lattice with each edge's source replaced, with
  probability 5 % (low) or 15 % (high), by a vertex drawn uniformly (another
  draw if it would make a self-loop or a duplicate): the lattice plus a
  fraction of long-range connections;
* scale free: preferential attachment in the numbering order (centre
  outwards, so hubs sit near the centre and the graph keeps geometric
  locality): vertex v links to m = 2 (low) or 4 (high) distinct earlier
  vertices chosen with probability proportional to their degree + 1, each
  link an edge in both directions; the degree distribution has a power-law
  tail;
* random: round(rho N^2) ordered pairs drawn uniformly without replacement
  among the N (N - 1) possible ones, rho = 10 % (low) or 20 % (high); the
  positions play no part.

Nothing of the simulated method is computed here (no delays, no dynamics).
"""
from __future__ import annotations

import math
from typing import List, Optional, Tuple

import numpy as np

from . import NetSpec, round_fp16

SIZES = (10, 30, 100, 300, 1000)
DIMS = (2, 3)
CLASSES = ("lattice", "small_world", "scale_free", "random")
DENSITIES = ("low", "high")
SPACE = 500.0
PACKING = 0.5
LATTICE_K = {"low": 3, "high": 8}
REWIRE_P = {"low": 0.05, "high": 0.15}
SMALL_WORLD_K = 8
SCALE_FREE_M = {"low": 2, "high": 4}
RANDOM_RHO = {"low": 0.10, "high": 0.20}


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.default_rng([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF, tag])


def min_distance(n: int, dims: int, space: float = SPACE, packing: float = PACKING) -> float:
    """d_min = packing * L * N^(-1/D) (Section 3.5)."""
    return packing * space * n ** (-1.0 / dims)


def place(n: int, dims: int, seed: int, space: float = SPACE, d_min: Optional[float] = None) -> np.ndarray:
    """Random positions at least d_min apart (the paper's rejection loop),
    then sorted by distance from the centre of the space (centre outwards)."""
    d_min = min_distance(n, dims, space) if d_min is None else d_min
    rng = _rng(seed, 1)
    pts = np.empty((n, dims))
    k = 0
    tries = 0
    while k < n:
        batch = rng.random((256, dims)) * space
        for x in batch:
            tries += 1
            if k == 0 or np.min(np.sum((pts[:k] - x) ** 2, axis=1)) >= d_min * d_min:
                pts[k] = x
                k += 1
                if k == n:
                    break
        if tries > 10000 * n:
            raise RuntimeError("placement: no room for %d vertices at d_min %.3g" % (n, d_min))
    centre = np.full(dims, space / 2.0)
    order = np.argsort(np.sum((pts - centre) ** 2, axis=1), kind="stable")
    return np.ascontiguousarray(pts[order])


def _knn_sources(pos: np.ndarray, k: int) -> List[np.ndarray]:
    d2 = np.sum((pos[:, None, :] - pos[None, :, :]) ** 2, axis=2)
    np.fill_diagonal(d2, np.inf)
    k = min(k, pos.shape[0] - 1)
    return [np.argsort(d2[j], kind="stable")[:k] for j in range(pos.shape[0])]


def lattice_edges(pos: np.ndarray, k: int) -> Tuple[np.ndarray, np.ndarray]:
    nb = _knn_sources(pos, k)
    src = np.concatenate(nb) if nb else np.zeros(0, np.int64)
    dst = np.repeat(np.arange(pos.shape[0]), [len(x) for x in nb])
    return src, dst


def small_world_edges(pos: np.ndarray, k: int, p: float, seed: int) -> Tuple[np.ndarray, np.ndarray, int]:
    """The k-nearest lattice with sources rewired with probability p; also
    returns how many edges were rewired."""
    n = pos.shape[0]
    src, dst = lattice_edges(pos, k)
    rng = _rng(seed, 2)
    have = set(zip(src.tolist(), dst.tolist()))
    rewired = 0
    src = src.copy()
    for e in range(src.shape[0]):
        if rng.random() >= p:
            continue
        j = int(dst[e])
        for _ in range(100):
            i = int(rng.integers(0, n))
            if i != j and (i, j) not in have:
                have.discard((int(src[e]), j))
                have.add((i, j))
                src[e] = i
                rewired += 1
                break
    return src, dst, rewired


def scale_free_edges(n: int, m: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Preferential attachment in numbering order; every link in both directions."""
    rng = _rng(seed, 3)
    deg = np.zeros(n)
    links = []
    for v in range(1, n):
        cand = np.arange(v)
        k = min(m, v)
        w = deg[:v] + 1.0
        chosen = rng.choice(cand, size=k, replace=False, p=w / w.sum())
        for u in chosen.tolist():
            links.append((u, v))
            deg[u] += 1
            deg[v] += 1
    if not links:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    a = np.array(links)
    src = np.concatenate([a[:, 0], a[:, 1]])
    dst = np.concatenate([a[:, 1], a[:, 0]])
    return src, dst


def random_edges(n: int, rho: float, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    rng = _rng(seed, 4)
    m = int(round(rho * n * n))
    m = min(m, n * (n - 1))
    flat = rng.choice(n * (n - 1), size=m, replace=False)
    i = flat // (n - 1)
    r = flat % (n - 1)
    j = np.where(r >= i, r + 1, r)             # skip the diagonal
    return i, j


def test_network(n: int, dims: int, cls: str, density: str, seed: Optional[int] = None,
                 weight: float = 1.0) -> NetSpec:
    """One network of the test set; weights U[0.5, 1.5] * weight (FP16),
    to be scaled for the vertex model used."""
    if seed is None:
        seed = (0x5EED7E57 * (1 + SIZES.index(n) if n in SIZES else n) + 97 * dims
                + 7 * CLASSES.index(cls) + DENSITIES.index(density)) & ((1 << 63) - 1)
    pos = place(n, dims, seed)
    meta = {"class": cls, "density": density, "dims": dims, "d_min": min_distance(n, dims), "space": SPACE}
    if cls == "lattice":
        src, dst = lattice_edges(pos, LATTICE_K[density])
        meta["k"] = LATTICE_K[density]
    elif cls == "small_world":
        src, dst, rewired = small_world_edges(pos, SMALL_WORLD_K, REWIRE_P[density], seed)
        meta.update(k=SMALL_WORLD_K, p=REWIRE_P[density], rewired=rewired)
    elif cls == "scale_free":
        src, dst = scale_free_edges(n, SCALE_FREE_M[density], seed)
        meta["m"] = SCALE_FREE_M[density]
    elif cls == "random":
        src, dst = random_edges(n, RANDOM_RHO[density], seed)
        meta["rho"] = RANDOM_RHO[density]
    else:
        raise ValueError("unknown class " + cls)
    order = np.lexsort((src, dst))
    src = np.ascontiguousarray(src[order], dtype=np.int32)
    dst = np.ascontiguousarray(dst[order], dtype=np.int32)
    rng = _rng(seed, 5)
    w = round_fp16((0.5 + rng.random(src.shape[0])) * weight)
    return NetSpec(name="%s-%s-%dD-N%d" % (cls, density, dims, n), pos_um=pos, src=src, dst=dst, weight=w,
                   seed=seed, meta=meta)


def test_set(dims_list=DIMS, sizes=SIZES) -> List[NetSpec]:
    """The 80 networks (or a subset): sizes x dimensions x classes x densities."""
    out = []
    for dims in dims_list:
        for n in sizes:
            for cls in CLASSES:
                for den in DENSITIES:
                    out.append(test_network(n, dims, cls, den))
    return out
