"""Pins of the ensemble (cross-)entropy reference (Fig. 5A, Fig. 6E): closed
forms, Gibbs' inequality and a brute-force count on a tiny ensemble."""
import math

import numpy as np

from oracle import accuracy as acc


def test_half_occupied_is_one_bit():
    p = np.full(10, 0.5)
    assert np.allclose(acc.entropy(p), 1.0)
    assert np.allclose(acc.cross_entropy(p, p, n_par=8), 1.0)


def test_identical_ensembles_give_their_entropy():
    rng = np.random.Generator(np.random.PCG64(1))
    p = rng.uniform(0.1, 0.9, size=50)   # well inside the clipping range at n = 100
    assert np.allclose(acc.cross_entropy(p, p, n_par=100), acc.entropy(p))
    assert np.allclose(acc.entropy([0.25]), [-(0.25 * math.log2(0.25) + 0.75 * math.log2(0.75))])


def test_certain_pixels_and_clipping():
    n = 64
    # both ensembles always occupy the pixel: only the clip costs
    assert np.isclose(acc.cross_entropy([1.0], [1.0], n)[0], -math.log2(1 - 1 / (2 * n)))
    # the reference always, the parallel ensemble never: log2(2n)
    assert np.isclose(acc.cross_entropy([1.0], [0.0], n)[0], math.log2(2 * n))
    assert np.isclose(acc.cross_entropy([0.0], [0.0], n)[0], -math.log2(1 - 1 / (2 * n)))
    assert acc.entropy([0.0])[0] == 0.0 and acc.entropy([1.0])[0] == 0.0


def test_gibbs_inequality():
    rng = np.random.Generator(np.random.PCG64(2))
    p = rng.uniform(0.05, 0.95, size=200)
    q = rng.uniform(0.05, 0.95, size=200)
    ce = acc.cross_entropy(p, q, n_par=1000)
    assert np.all(ce >= acc.entropy(p) - 1e-12)
    assert np.all(ce[np.abs(p - q) > 0.05] > acc.entropy(p)[np.abs(p - q) > 0.05])


def test_brute_force_tiny_ensembles():
    # 3 reference runs and 2 parallel runs of a 2-pixel lattice, by hand:
    # reference occupancy (2/3, 0), parallel (1/2, 1/2)
    ref = np.array([[1, 0], [3, 0], [0, -1]])
    par = np.array([[2, 0], [0, 5]])
    assert np.allclose(acc.occupancy(ref), [2 / 3, 0.0])
    assert np.allclose(acc.occupancy(par), [0.5, 0.5])
    ce0 = -(2 / 3 * math.log2(0.5) + 1 / 3 * math.log2(0.5))
    ce1 = -(0 * math.log2(0.5) + 1 * math.log2(0.5))
    assert np.isclose(acc.accuracy(ref, par), 1 - (ce0 + ce1) / 2)


def test_harness_formula_matches_reference():
    # the library harness scores occupancy counts with its own code: it must
    # agree with the reference definition on random ensembles
    from paper_2312_09317_amd import accuracy as harness
    rng = np.random.Generator(np.random.PCG64(3))
    for n_ref, n_par in ((250, 250), (16, 64), (7, 3)):
        ref = rng.random((n_ref, 300)) < rng.random(300)
        par = rng.random((n_par, 300)) < rng.random(300)
        got = 1.0 - harness.cross_entropy_bits(ref.sum(0), n_ref, par.sum(0), n_par)
        assert np.isclose(got, acc.accuracy(ref.astype(np.int32), par.astype(np.int32)), rtol=0, atol=1e-12)
