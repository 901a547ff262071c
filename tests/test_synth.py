"""Statistical checks of the seeded input generator (CPU)."""
import math

import numpy as np
import pytest

import synth


def _pairwise(pos):
    d = pos[:, None, :] - pos[None, :, :]
    return np.sqrt((d * d).sum(-1))


def test_step_rule_edge_count_and_invariants():
    spec = synth.config0()
    assert spec.n == 256 and spec.dims == 2
    assert np.all(spec.src != spec.dst)
    key = spec.dst.astype(np.int64) * spec.n + spec.src
    assert np.all(np.diff(key) > 0)                 # sorted by (dst, src), unique
    r = _pairwise(spec.pos_um)
    close = (r < 150.0) & ~np.eye(spec.n, dtype=bool)
    m = close.sum()
    mean, sd = 0.3 * m, math.sqrt(m * 0.3 * 0.7)
    assert abs(spec.n_edges - mean) < 4 * sd
    assert np.all(close[spec.src, spec.dst])         # only pairs inside the radius
    assert np.all(synth.round_fp16(spec.weight) == spec.weight)
    assert spec.weight.min() >= 0.5 * synth.W0 * (1 - 1e-3) and spec.weight.max() <= 1.5 * synth.W0 * (1 + 1e-3)
    assert spec.meta["driven"].sum() == round(0.1 * 256)


def test_expdecay_rule_matches_expectation():
    n = 3000
    ext = [600.0] * 3
    pos = synth.uniform_positions(n, ext, 5)
    src, dst = synth.sample_edges(pos, ext, 1, 0.1, 100.0, 400.0, 100.0, 17)
    r = _pairwise(pos)
    p = np.where((r < 400.0) & ~np.eye(n, dtype=bool), 0.1 * np.exp(-r / 100.0), 0.0)
    mean, sd = p.sum(), math.sqrt((p * (1 - p)).sum())
    assert abs(src.size - mean) < 4 * sd
    rr = r[src, dst]
    assert rr.max() < 400.0
    # distance profile: mean edge length against the expectation
    assert abs(rr.mean() - (p * r).sum() / p.sum()) < 4.0


def test_generator_is_deterministic_and_thread_independent():
    a = synth.config0_like(512, 99)
    b = synth.config0_like(512, 99)
    assert np.array_equal(a.src, b.src) and np.array_equal(a.dst, b.dst) and np.array_equal(a.weight, b.weight)
    c = synth.config0_like(512, 100)
    assert a.n_edges != c.n_edges or not np.array_equal(a.src, c.src)


def test_inhibitory_fraction_exact():
    spec = synth.config2(n=4096)
    assert spec.inhibitory.sum() == round(0.2 * 4096)
    neg = spec.weight < 0
    assert np.array_equal(neg, spec.inhibitory[spec.src])


def test_config3_sizes_log_uniform():
    s = np.array(synth.config3_sizes())
    assert s.size == 512 and s.min() >= 64 and s.max() <= 4096
    # log-uniform: median near sqrt(64*4096) = 512
    assert 380 < np.median(s) < 690


def test_morton_numbering_is_local():
    pos = synth.uniform_positions(4096, [1000.0, 1000.0, 1000.0], 3)
    step = np.sqrt(((pos[1:] - pos[:-1]) ** 2).sum(1))
    assert np.median(step) < 120.0       # random order would give ~ 660 um
