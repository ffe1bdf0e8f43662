"""Seeded input generators: reference values and reproducibility."""
import numpy as np

from workloads import gen


def test_splitmix64_reference_output():
    # SplitMix64 started from state 0 first returns 0xE220A8397B1DCDAF
    # (the published reference implementation); stream 0, seed 0, draw 0
    # is exactly that output in the counter-based form.
    r = gen.draws(0, 0, np.array([0, 1], dtype=np.uint64))
    assert int(r[0]) == 0xE220A8397B1DCDAF
    assert int(r[1]) == 0x6E789E6AA1B965F4


def test_uniform_matrix_range_and_determinism():
    a = gen.uniform_matrix(300, 0, 1000, 7)
    b = gen.uniform_matrix(300, 0, 1000, 7)
    assert a.dtype == np.int32 and (a == b).all()
    assert a.min() >= 0 and a.max() < 1000
    assert not (a == gen.uniform_matrix(300, 0, 1000, 8)).all()
    # chunking does not change values: rows are addressed by draw index
    old = gen._ROW_CHUNK_ELEMS
    try:
        gen._ROW_CHUNK_ELEMS = 1000
        assert (gen.uniform_matrix(300, 0, 1000, 7) == a).all()
    finally:
        gen._ROW_CHUNK_ELEMS = old


def test_lowrank_matrix_shape():
    A = gen.lowrank_matrix(512, 3)
    u, c = gen.lowrank_factors(512, 3)
    assert u.min() >= 0.1 and u.max() < 1.0 and c.min() >= 0.1 and c.max() < 1.0
    base = gen.round_half_away((1000.0 * u)[:, None] * c[None, :])
    noise = A - base
    assert noise.min() >= 0 and noise.max() < 100
    assert A.min() >= 10 and A.max() <= 1000 + 99


def test_round_half_away():
    x = np.array([0.5, 1.5, 2.5, -0.5, -2.5, 2.4999999999999996, 3.0])
    assert list(gen.round_half_away(x)) == [1, 2, 3, -1, -3, 2, 3]


def test_sizes_and_permutation():
    ns = gen.loguniform_sizes(512, 64, 2048, 1)
    assert ns.min() >= 64 and ns.max() <= 2048
    assert 400 < ns.mean() < 800  # E[n] ~ 572 for log-uniform on [64, 2048]
    p = gen.permutation(1000, 5)
    assert sorted(p.tolist()) == list(range(1000))
    t = gen.poisson_arrivals(200.0, 5.0, 1)
    assert (np.diff(t) > 0).all() and 800 < len(t) < 1200


def test_geom_matrix_is_a_rounded_distance_matrix():
    # Section 4's GEOM type: a_ij = Euclidean distance of random points i and j
    # in [0, 1000]^2, rounded to an integer
    A = gen.geom_matrix(400, 2)
    assert A.dtype == np.int32 and (A == A.T).all() and (np.diag(A) == 0).all()
    assert A.min() >= 0 and A.max() <= int(np.ceil(1000 * np.sqrt(2)))
    # rounding keeps the triangle inequality within 1.5 (three roundings of 0.5)
    i, j, k = np.random.default_rng(0).integers(0, 400, (3, 2000))
    assert (A[i, k] <= A[i, j] + A[j, k] + 1.5).all()
    assert (A == gen.geom_matrix(400, 2)).all() and not (A == gen.geom_matrix(400, 3)).all()
    # point i depends on (seed, i) only, so a smaller instance is a leading block
    assert (gen.single_instance("geom4096", 1)[:50, :50] == gen.geom_matrix(50, 1)).all()
