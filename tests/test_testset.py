"""The standardized test networks (Section 3.5, Table modelspace) against
what their description fixes: the minimum distance, d_min = c L N^(-1/D),
numbering from the centre outwards, nearest-neighbour lattices with exactly
k in-edges taken from the k nearest vertices, the rewired fraction of the
small-world class, the exact edge count of the random class, the heavy tail
and symmetry of the scale-free class, 80 networks in all, and determinism."""
import numpy as np
import pytest

from synth import testset as ts


def test_min_distance_rule():
    # the paper's example: L = 100, N = 1000, D = 3 packs at 10 units
    assert ts.min_distance(1000, 3, space=100.0, packing=1.0) == pytest.approx(10.0)
    assert ts.min_distance(100, 2) == pytest.approx(ts.PACKING * 500.0 / 10.0)


@pytest.mark.parametrize("n,dims", [(10, 2), (300, 2), (1000, 3), (1000, 2)])
def test_placement(n, dims):
    pos = ts.place(n, dims, seed=n + dims)
    assert pos.shape == (n, dims)
    assert (pos >= 0).all() and (pos <= ts.SPACE).all()
    d2 = np.sum((pos[:, None, :] - pos[None, :, :]) ** 2, axis=2)
    np.fill_diagonal(d2, np.inf)
    assert np.sqrt(d2.min()) >= ts.min_distance(n, dims) - 1e-9
    r = np.sqrt(np.sum((pos - ts.SPACE / 2) ** 2, axis=1))
    assert (np.diff(r) >= 0).all()                         # centre outwards
    assert np.array_equal(pos, ts.place(n, dims, seed=n + dims))


def _edges(s):
    return set(zip(s.src.tolist(), s.dst.tolist()))


@pytest.mark.parametrize("density", ["low", "high"])
def test_lattice_is_k_nearest(density):
    s = ts.test_network(300, 2, "lattice", density)
    k = ts.LATTICE_K[density]
    indeg = np.bincount(s.dst, minlength=s.n)
    assert (indeg == k).all()
    d = np.sqrt(np.sum((s.pos_um[:, None, :] - s.pos_um[None, :, :]) ** 2, axis=2))
    np.fill_diagonal(d, np.inf)
    for j in range(0, s.n, 17):
        srcs = s.src[s.dst == j]
        kth = np.sort(d[j])[k - 1]
        assert (d[j, srcs] <= kth + 1e-12).all()           # no farther vertex than the k-th nearest


@pytest.mark.parametrize("density", ["low", "high"])
def test_small_world_rewiring(density):
    s = ts.test_network(1000, 2, "small_world", density)
    lat = ts.lattice_edges(s.pos_um, ts.SMALL_WORLD_K)
    lat = set(zip(lat[0].tolist(), lat[1].tolist()))
    e = _edges(s)
    assert len(e) == s.n_edges == s.n * ts.SMALL_WORLD_K          # no duplicates
    frac = 1.0 - len(e & lat) / len(e)
    p = ts.REWIRE_P[density]
    sd = np.sqrt(p * (1 - p) / len(e))
    assert abs(frac - p) <= 5 * sd + 1.0 / len(e)
    assert frac == pytest.approx(s.meta["rewired"] / s.n_edges, abs=2e-3)   # rare rewires land on lattice edges
    assert (np.bincount(s.dst, minlength=s.n) == ts.SMALL_WORLD_K).all()   # targets keep their in-degree


@pytest.mark.parametrize("density", ["low", "high"])
def test_random_edge_count(density):
    s = ts.test_network(300, 3, "random", density)
    assert s.n_edges == round(ts.RANDOM_RHO[density] * 300 * 300)
    assert len(_edges(s)) == s.n_edges
    assert not (s.src == s.dst).any()
    # uniform over pairs: in- and out-degrees binomial around rho * N
    indeg = np.bincount(s.dst, minlength=s.n)
    assert abs(indeg.mean() - ts.RANDOM_RHO[density] * 300) < 1.0
    assert indeg.std() < 3 * np.sqrt(ts.RANDOM_RHO[density] * 300)


@pytest.mark.parametrize("density", ["low", "high"])
def test_scale_free_tail(density):
    s = ts.test_network(1000, 2, "scale_free", density)
    m = ts.SCALE_FREE_M[density]
    e = _edges(s)
    assert all((j, i) in e for (i, j) in e)                        # every link both ways
    deg = np.bincount(s.dst, minlength=s.n)
    assert deg[1:].min() >= m or deg[m:].min() >= m                # each late vertex brought m links
    assert s.n_edges == 2 * sum(min(m, v) for v in range(1, s.n))
    # a power-law tail: hubs far above the mean, many vertices at the minimum
    assert deg.max() > 8 * deg.mean()
    assert (deg == m).mean() > 0.25
    # hubs are early (central) vertices
    assert np.argmax(deg) < 50


def test_full_set_has_80_networks():
    nets = ts.test_set()
    assert len(nets) == 80
    names = {s.name for s in nets}
    assert len(names) == 80
    big_random = [s for s in nets if s.meta["class"] == "random" and s.n == 1000 and s.meta["density"] == "high"]
    assert all(s.n_edges == 200000 for s in big_random)      # ~2e5 edges, the paper's largest networks
    for s in nets:
        assert not (s.src == s.dst).any()
        assert len(_edges(s)) == s.n_edges
        assert (s.weight >= 0.5).all() and (s.weight <= 1.5).all()
