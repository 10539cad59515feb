"""Pins of the oracle's blocked Hamiltonian terms and closed-form ground energies."""
import numpy as np
import pytest

from oracle import model


def _place(op, sites, nsites, d):
    """Dense operator on a ring of `nsites` sites of dim d with `op` acting on `sites` (in that order)."""
    k = len(sites)
    rest = [s for s in range(nsites) if s not in sites]
    full = np.kron(op, np.eye(d ** len(rest))).reshape((d,) * (2 * nsites))
    order_in = list(sites) + rest
    perm = np.argsort(order_in)
    full = np.transpose(full, list(perm) + [nsites + p for p in perm])
    return full.reshape(d ** nsites, d ** nsites)


@pytest.mark.parametrize("nblocks", [4, 5])
@pytest.mark.parametrize("kind,param", [("tfim", 1.0), ("tfim", 0.7), ("xxz", 0.3), ("xxz", -0.5)])
def test_h3_sums_to_ring_hamiltonian(nblocks, kind, param):
    h3 = model.tfim_h3(param) if kind == "tfim" else model.xxz_h3(param)
    pf = model.tfim_pair_and_field(param) if kind == "tfim" else model.xxz_pair_and_field(param)
    H_blocks = sum(_place(h3, [s, (s + 1) % nblocks, (s + 2) % nblocks], nblocks, 4) for s in range(nblocks))
    H_spins = model.spin_ring_hamiltonian(2 * nblocks, *pf)
    assert np.max(np.abs(H_blocks - H_spins)) < 1e-12


def test_h3_symmetric_real():
    for h3 in (model.tfim_h3(1.0), model.xxz_h3(1.2)):
        assert h3.shape == (64, 64)
        assert np.max(np.abs(h3 - h3.T)) == 0.0


def test_exact_energies_closed_forms():
    assert abs(model.tfim_exact_energy_per_spin(1.0) + 4.0 / np.pi) < 1e-12
    assert abs(model.xxz_exact_energy_per_spin(0.0) + 4.0 / np.pi) < 1e-10
    assert model.xxz_exact_energy_per_spin(1.0) == 1.0 - 4.0 * np.log(2.0)
    # h -> 0: classical Ising ground energy -1 per spin; h -> large: -h per spin plus O(1/h)
    assert abs(model.tfim_exact_energy_per_spin(1e-9) + 1.0) < 1e-8
    # delta = 1/2 (gamma = pi/3): exactly -3/8 per site in spin-1/2 units, i.e. -3/2 in Pauli units
    assert abs(model.xxz_exact_energy_per_spin(0.5) + 1.5) < 1e-10


def test_xxz_integral_continuous_at_isotropic_point():
    # the Bethe-ansatz integral approaches the Hulthen value as delta -> 1 from below
    assert abs(model.xxz_exact_energy_per_spin(0.999999) - (1.0 - 4.0 * np.log(2.0))) < 1e-4


def test_exact_energy_below_finite_ring_ground_state_gap():
    # A 12-spin periodic ring ground energy per spin lies within 1% of the infinite-chain value (TFIM h=1).
    H = model.spin_ring_hamiltonian(12, *model.tfim_pair_and_field(1.0))
    e12 = np.linalg.eigvalsh(H)[0] / 12
    e_inf = model.tfim_exact_energy_per_spin(1.0)
    assert abs(e12 - e_inf) / abs(e_inf) < 1e-2


def test_closed_forms_from_golden_fixture():
    """The oracle's ground-state energy functions against the closed forms stored in tests/golden (with sources)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "closed_form_energies.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for kind, par, val, *_ in rows:
        f = model.tfim_exact_energy_per_spin if kind == "tfim" else model.xxz_exact_energy_per_spin
        assert abs(f(float(par)) - float(val)) < 1e-9, (kind, par)
