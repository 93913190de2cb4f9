"""The seeded input generators: SplitMix64 against its published outputs and
the random-sequential-addition placement against its stated constraints."""
import numpy as np
import pytest

import lbm_inputs


def test_splitmix64_published_vectors():
    """Reference outputs of SplitMix64 (Steele, Lea & Flood 2014) for the
    seeds 1234567 and 0."""
    r = lbm_inputs.SplitMix64(1234567)
    assert [r.next_u64() for _ in range(5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]
    assert lbm_inputs.SplitMix64(0).next_u64() == 0xE220A8397B1DCDAF


@pytest.mark.parametrize("nx,ny,n,d,gap,seed", [
    (256, 256, 20, 12, 1.0, 1), (600, 500, 700, 10, 1.0, 3), (128, 256, 60, 8, 2.0, 4)])
def test_rsa_constraints(nx, ny, n, d, gap, seed):
    P = lbm_inputs.rsa_particles(nx, ny, n, d, gap, seed)
    assert P.shape == (n, 7)
    assert (P[:, 0] >= 0).all() and (P[:, 0] < nx).all()
    r = d / 2
    assert (P[:, 1] - r >= -0.5 + 1 - 1e-12).all() and (P[:, 1] + r <= ny - 0.5 - 1 + 1e-12).all()
    dx = P[:, 0][:, None] - P[:, 0][None, :]
    dx = np.where(dx > nx / 2, dx - nx, np.where(dx < -nx / 2, dx + nx, dx))
    dy = P[:, 1][:, None] - P[:, 1][None, :]
    g = np.sqrt(dx * dx + dy * dy) - d
    np.fill_diagonal(g, np.inf)
    assert g.min() >= gap
    assert (P[:, 3:] == 0).all() and (P[:, 2] == r).all()
    np.testing.assert_array_equal(P, lbm_inputs.rsa_particles(nx, ny, n, d, gap, seed))


def test_rsa_infeasible_raises():
    with pytest.raises(lbm_inputs.SeedingError):
        lbm_inputs.rsa_particles(32, 32, 40, 10, 1.0, 1)
