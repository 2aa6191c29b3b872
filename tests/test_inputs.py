"""The seeded input generators: shapes, determinism, and the FR operators they build."""
import numpy as np

from paper_2003_02633_amd import inputs


def test_fr_derivative_exact_on_polynomials():
    for p in (1, 2, 3, 4, 5):
        x = inputs.gauss_legendre_nodes(p + 1)
        d = inputs.fr_derivative_1d(p, h=0.5)
        for deg in range(p + 1):
            f = x ** deg
            df = deg * x ** (deg - 1) if deg else np.zeros_like(x)
            assert np.abs(d.T @ f - 4.0 * df).max() < 1e-11 * max(1.0, 4.0 * np.abs(df).max())


def test_fr_div_operator_structure():
    p, q = 4, 5
    D = inputs.fr_div_operator(p)
    assert D.shape == (3 * q ** 3, q ** 3)
    # each column holds (p + 1) entries per direction (the centre node's own derivative is 0)
    assert (D != 0).sum() == 3 * q ** 3 * q - 3 * q ** 2
    # the divergence of a constant flux is zero
    assert np.abs(D.sum(axis=0)).max() < 1e-12


def test_euler_flux_tgv_shape_and_rows():
    F = inputs.euler_flux_tgv(12, 2, grid=(3, 2, 2))
    assert F.shape == (12, 27, 5, 3) and F.dtype == np.float32
    # the z momentum is zero in the Taylor-Green state; row 4's z entry is the pressure
    assert (F[:, :, 0, 2] == 0).all()
    assert np.allclose(F[:, :, 3, 2], F[:, :, 1, 0] - (F[:, :, 0, 0] ** 2 / (F[:, :, 3, 2] / 100.0)), rtol=1e-3)


def test_generators_deterministic():
    assert np.array_equal(inputs.gaussian(1000, 4), inputs.gaussian(1000, 4))
    assert np.array_equal(inputs.vmf(1000, 10.0, seed=3), inputs.vmf(1000, 10.0, seed=3))
    assert np.array_equal(inputs.euler_flux_tgv(5, 2, grid=(2, 2, 2)), inputs.euler_flux_tgv(5, 2, grid=(2, 2, 2)))
