"""The seeded input generators: determinism, value domains, per-column regeneration."""
import numpy as np

import datagen


def test_same_seed_same_bytes_and_column_regeneration():
    a = datagen.genotype_u8(5, 300, 40)
    b = datagen.genotype_u8(5, 300, 40)
    assert a.tobytes() == b.tobytes()
    # columns 10..19 generated alone equal the same columns of the full draw
    part = datagen.genotype_u8(5, 300, 10, j0=10)
    np.testing.assert_array_equal(part, a[10:20])
    g = datagen.gaussian_f64(9, 50, 30)
    np.testing.assert_array_equal(datagen.gaussian_f64(9, 50, 5, j0=7), g[7:12])


def test_genotype_domain_and_frequencies():
    Xt = datagen.genotype_u8(3, 20000, 50)
    assert set(np.unique(Xt)) <= {0, 1, 2}
    maf = datagen.maf(3, 50)
    assert np.all((maf >= 0.05) & (maf <= 0.5))
    np.testing.assert_allclose(Xt.mean(axis=1) / 2, maf, atol=0.02)


def test_gaussian_moments():
    g = datagen.gaussian_f64(1, 200000, 2)
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1) < 0.01


def test_ar1_correlation():
    X = datagen.ar1_f32(2, 20000, 6, 0.5).astype(np.float64)
    r = np.corrcoef(X)
    for j in range(5):
        assert abs(r[j, j + 1] - 0.5) < 0.03
    B = datagen.ar1_f32(2, 20000, 8, 0.7, block=4).astype(np.float64)
    rb = np.corrcoef(B)
    assert abs(rb[2, 3] - 0.7) < 0.03 and abs(rb[3, 4]) < 0.03   # block boundary between 3 and 4


def test_recipes_shapes_and_snr():
    prob = datagen.make("c1", n=500, p=800)
    assert prob.Xt.shape == (800, 500) and prob.y.shape == (1, 500)
    sup, vals = datagen.coefficients(prob.recipe)
    assert sup.size == 20 and np.all(np.abs(vals) >= 0.5) and np.all(np.abs(vals) <= 1.5)
    signal = prob.Xt[sup].T @ vals
    noise = prob.y[0] - signal
    assert 1.5 < np.var(signal) / np.var(noise) < 6.0


def test_cv_masks_uneven_rows():
    rec = datagen.RECIPES["c4"].scaled(n=2000, p=10)
    m = datagen.cv_row_masks(rec)
    assert m.shape == (64, 2000)
    nb = m.sum(axis=1)
    assert nb.min() >= 1600 and nb.max() <= 1800 and len(set(nb)) > 10
