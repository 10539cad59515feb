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


@pytest.mark.parametrize("hx", [0.0, 0.3, 0.999, 1.0, 1.001, 1.5, 3.0])
def test_tfim_energy_against_elliptic_closed_form(hx):
    """-(1/2pi) int sqrt(1 + h^2 - 2h cos k) dk = -(2/pi)(1 + h) E(4h/(1 + h)^2), E the complete elliptic integral
    of the second kind in the parameter convention (scipy.special.ellipe)."""
    from scipy import special
    ref = -(2.0 / np.pi) * (1.0 + hx) * special.ellipe(4.0 * hx / (1.0 + hx) ** 2)
    assert abs(model.tfim_exact_energy_per_spin(hx) - ref) < 1e-13


def _total(nspins, op):
    return sum(model._on_spins(nspins, {i: op}) for i in range(nspins))


@pytest.mark.parametrize("delta", [-0.5, 0.0, 0.4, 1.0, 1.3])
def test_xxz_ring_conserves_total_z(delta):
    """XX + YY + delta ZZ conserves the total Z magnetisation for every delta (U(1) symmetry); a wrong sign of the
    YY part (XX - YY flips two spins the same way) breaks it."""
    H = model.spin_ring_hamiltonian(6, *model.xxz_pair_and_field(delta))
    Z = _total(6, model.PZ)
    assert np.max(np.abs(H @ Z - Z @ H)) < 1e-12
    assert np.max(np.abs(H - H.T)) == 0.0


def test_xxz_isotropic_point_is_su2_invariant():
    """At delta = 1 the term is sigma . sigma: it commutes with the total X (and, being real, total iY) as well."""
    H = model.spin_ring_hamiltonian(6, *model.xxz_pair_and_field(1.0))
    for op in (model.PX, model.PIY):
        S = _total(6, op)
        assert np.max(np.abs(H @ S - S @ H)) < 1e-12


def test_xxz_four_spin_heisenberg_ring():
    """4-spin ring at delta = 1: sum_i S_i.S_{i+1} = ((S1+S2+S3+S4)^2 - (S1+S3)^2 - (S2+S4)^2)/2 has ground energy
    (0 - 2 - 2)/2 = -2 in spin-1/2 units, i.e. -8 in Pauli units (sigma = 2S); spectrum {-8, -4 (x3), 0 (x7), 4 (x5)}
    from the total-spin multiplets (S_A, S_B, S)."""
    H = model.spin_ring_hamiltonian(4, *model.xxz_pair_and_field(1.0))
    ev = np.linalg.eigvalsh(H)
    # multiplets: (1,1,0) -> -8; (1,1,1) -> -4 (3); (1,0,1),(0,1,1) -> 0 (6); (0,0,0) -> 0; (1,1,2) -> 4 (5)
    ref = sorted([-8.0] + [-4.0] * 3 + [0.0] * 7 + [4.0] * 5)
    assert np.max(np.abs(ev - np.array(ref))) < 1e-12


def _xx_ring_free_fermion_energy(nspins):
    """Ground energy of sum_i (X_i X_{i+1} + Y_i Y_{i+1}) on a periodic ring from free fermions (Lieb, Schultz and
    Mattis 1961): the term is 2 (s+_i s-_{i+1} + h.c.), the Jordan-Wigner fermions hop with single-particle energies
    4 cos k, k = 2 pi m / N (periodic) when the fermion number is odd and k = 2 pi (m + 1/2) / N (antiperiodic)
    when it is even; the ground energy is the lowest filling over all fermion numbers."""
    m = np.arange(nspins)
    eps_p = np.sort(4.0 * np.cos(2.0 * np.pi * m / nspins))
    eps_a = np.sort(4.0 * np.cos(2.0 * np.pi * (m + 0.5) / nspins))
    best = np.inf
    for nf in range(nspins + 1):
        eps = eps_p if nf % 2 == 1 else eps_a
        best = min(best, float(np.sum(eps[:nf])))
    return best


@pytest.mark.parametrize("nspins", [6, 8, 10])
def test_xx_ring_against_free_fermions(nspins):
    H = model.spin_ring_hamiltonian(nspins, *model.xxz_pair_and_field(0.0))
    assert abs(np.linalg.eigvalsh(H)[0] - _xx_ring_free_fermion_energy(nspins)) < 1e-10
