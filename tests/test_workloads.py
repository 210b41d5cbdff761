"""The seeded input recipes: sizes and parameters of the model systems, and the
properties the synthetic arrays are built to have (exact symmetry, seeding)."""
import numpy as np

import workloads as W
from oracle import fedvr


def n_b(sysd):
    return (len(sysd.bounds) - 1) * sysd.n_g - 1


def test_model_systems():
    he = W.config_he()
    assert n_b(he) == 19 and he.M == 128 and he.beta == 50.0
    b = W.config_sigma_bench()
    assert n_b(b) == 199 and b.M == 1024 and b.beta == 50.0
    assert b.bounds[0] == -40.0 and b.bounds[-1] == 40.0 and len(b.bounds) == 41
    h = W.config_h3p()
    assert n_b(h) == 359 and h.beta == 100.0 and h.tau_kind == "power"
    assert len(fedvr.tau_power(h.beta, h.u, h.p)) == 2 * h.u * h.p + 1 == 2049
    assert np.allclose(h.centres, [-1.8, 0.0, 1.8]) and h.e_nn == 5.0 / (2 * 1.8)


def test_scan_recipe():
    systems = W.config_scan()
    assert len(systems) == 64
    R = np.array([s.centres[-1] for s in systems])
    assert R[0] == 1.0 and abs(R[-1] - 3.0) < 1e-12 and np.all(np.diff(R) > 0)
    sizes = [n_b(s) for s in systems]
    assert min(sizes) == 149 and max(sizes) == 399 and len(set(sizes)) == 51
    for s, r in zip(systems, R):
        assert abs(s.bounds[-1] - (30.0 + 10.0 * r)) < 1e-12
        assert len(s.bounds) - 1 == int(round(30 + 25 * (r - 1.0)))
        assert s.tau_kind == "uniform" and s.M == 1024 and s.beta == 100.0


def test_small_scan_recipe():
    systems = W.config_scan_small()
    assert len(systems) == 64
    R = np.array([s.centres[-1] for s in systems])
    assert R[0] == 1.0 and abs(R[-1] - 3.0) < 1e-12
    sizes = [n_b(s) for s in systems]
    assert min(sizes) == 29 and max(sizes) == 69 and sizes == sorted(sizes)
    for s, r in zip(systems, R):
        assert abs(s.bounds[-1] - (10.0 + 2.0 * r)) < 1e-12
        assert len(s.bounds) - 1 == int(round(6 + 4 * (r - 1.0)))
        assert s.tau_kind == "uniform" and s.M == 1024 and s.beta == 100.0


def test_random_potentials_are_seeded():
    a, b = W.random_potential_system(100000), W.random_potential_system(100000)
    assert np.array_equal(a.centres, b.centres) and np.array_equal(a.charges, b.charges)
    for seed in range(50):
        s = W.random_potential_system(seed)
        assert 1 <= len(s.centres) <= 3
        assert np.all((s.charges >= 1.0) & (s.charges <= 2.0))
        assert np.all(np.abs(s.centres) <= 3.0)
        assert n_b(s) == 199 and s.M == 1024


def test_synthetic_arrays():
    G = W.synthetic_G(23, 16, 50.0, seed=2)
    assert G.shape == (17, 23, 23)
    assert np.array_equal(G, G.transpose(0, 2, 1))                     # exactly symmetric
    assert np.array_equal(G, W.synthetic_G(23, 16, 50.0, seed=2))      # seeded
    tau = np.arange(17) * 50.0 / 16
    assert np.all(np.abs(G).max(axis=(1, 2)) <= 0.6 * np.exp(-tau))     # |S_q| < 6 sigma
    A = W.random_symmetric_slices(9, 4, 5)
    assert np.array_equal(A, A.transpose(0, 2, 1))
    assert not np.array_equal(A, W.random_symmetric_slices(9, 4, 6))
