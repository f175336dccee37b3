"""The host energy diagnostic against the oracle's energy density (CPU only)."""
import numpy as np

import oracle
from paper_2412_10399_amd import diagnostics


def test_energies_match_oracle_energy_density():
    rng = np.random.default_rng(3)
    F = np.eye(3)[None] + 0.2 * rng.standard_normal((50, 3, 3))
    F[0] = np.diag([1.0, 1.0, -0.5])          # an inverted element
    v = rng.standard_normal((50, 3))
    E, nu, mass, vol0 = 1e5, 0.3, 2.0, 1e-6
    m = oracle.material(0, E, nu, 1.0, vol0)
    k, e = diagnostics.energies(v, F, mass, vol0, E, nu)
    assert abs(k - 0.5 * mass * (v * v).sum()) <= 1e-12 * k
    ref = vol0 * sum(oracle.energy_density(m, F[p]) for p in range(50))
    assert abs(e - ref) <= 1e-12 * ref
