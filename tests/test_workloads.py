"""Seeded input generators: sizes, determinism, velocity recipe, unit constant."""
import numpy as np

from workloads import configs


def test_unit_constant():
    # 1 amu * (1 A/fs)^2 = 103.6427 eV, so (eV/A)/amu = 1/103.6427 A/fs^2
    assert abs(1.0 / configs.FTM2V - 103.642697) < 1e-5


def test_sizes_and_vacancies():
    assert configs.config_small().n == 2000
    b = configs.make_box(74, np.random.default_rng(3), vacancy_fraction=0.01, temperature=2500.0)
    assert b.n == 810448 - 8104
    assert np.all((b.x >= 0) & (b.x < b.box))


def test_velocities_zero_momentum_exact_temperature():
    b = configs.small_box(6, seed=3, temperature=450.0)
    assert np.max(np.abs(b.v.sum(0))) < 1e-15
    ke = 0.5 * configs.MASS * np.sum(b.v ** 2) / configs.FTM2V
    assert abs(ke - 0.5 * (3 * b.n - 3) * configs.KBOLTZ * 450.0) < 1e-10


def test_seeded_determinism():
    a, b = configs.config_small(), configs.config_small()
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)


def test_batch_recipe():
    reps = configs.config_batch(16)
    for r in reps:
        n = r.n_cells
        assert 5 <= n <= 20
        assert 2 * n ** 3 - int(0.02 * 2 * n ** 3) <= r.n <= 2 * n ** 3
        assert 300.0 <= r.temperature <= 2000.0


def test_alloy_box_recipe():
    from workloads import configs, potential as P

    b = configs.alloy_box(6, 5, temperature=900.0)
    assert b.types.dtype == np.int32 and set(np.unique(b.types)) == {0, 1}
    assert abs(b.types.mean() - 0.5) < 0.1
    m = np.asarray(P.ALLOY_MASS)[b.types]
    assert np.all(np.abs((m[:, None] * b.v).sum(axis=0)) < 1e-10)
    ke = 0.5 * np.sum(m[:, None] * b.v ** 2) / configs.FTM2V
    assert abs(ke - 0.5 * (3 * b.n - 3) * configs.KBOLTZ * 900.0) < 1e-9 * ke
    assert np.all((b.x >= 0) & (b.x < b.box))
    # the alloy tables: phi[a][b] is phi[b][a], one table per type for rho and F
    phi, rho, emb = P.alloy_tables(n_knots=50)
    assert phi[0][1] is phi[1][0] and len(rho) == len(emb) == 2
