"""Model Hamiltonians as symmetric 3-site terms on blocked sites (oracle; test infrastructure only).

The paper's benchmark model is the critical transverse-field Ising chain with local term -X_i X_{i+1} - Z_i
(Sec. 4, definition of the cost function), and it mentions the XXZ model as a second test case (Sec. 4,
discussion of Fig. mera_results). Neither the blocking nor the split into 3-site terms is given in the paper;
the reading used here: two spins form one blocked site of dimension d = 4 (basis |s1 s2>, s1 major), the
two-block term hb collects the inter-block bond plus half of each block's internal terms, and the 3-site term is
h3 = (hb (x) 1 + 1 (x) hb) / 2. Summed over all positions of a ring, h3 reproduces H exactly.
"""
import numpy as np
from scipy import integrate

PX = np.array([[0.0, 1.0], [1.0, 0.0]])
PZ = np.array([[1.0, 0.0], [0.0, -1.0]])
PIY = np.array([[0.0, 1.0], [-1.0, 0.0]])  # i*Y is real; Y (x) Y = -(iY) (x) (iY)
I2 = np.eye(2)


def _kron(*ops):
    out = np.ones((1, 1))
    for o in ops:
        out = np.kron(out, o)
    return out


def _on_spins(nspins, placed):
    """Operator on `nspins` spins (spin 0 major) with {position: 2x2 matrix} placed, identity elsewhere."""
    return _kron(*[placed.get(i, I2) for i in range(nspins)])


def tfim_pair_and_field(hx):
    """TFIM pieces: pair term -X X and single-site field -hx Z (Sec. 4 local term, with a field strength)."""
    def pair(n, i, j):
        return -_on_spins(n, {i: PX, j: PX})

    def field(n, i):
        return -hx * _on_spins(n, {i: PZ})
    return pair, field


def xxz_pair_and_field(delta):
    """XXZ pieces in Pauli units: pair term XX + YY + delta ZZ, no field."""
    def pair(n, i, j):
        return (_on_spins(n, {i: PX, j: PX}) - _on_spins(n, {i: PIY, j: PIY})
                + delta * _on_spins(n, {i: PZ, j: PZ}))

    def field(n, i):
        return np.zeros((2 ** n, 2 ** n))
    return pair, field


def two_block_term(pair, field):
    """hb on two blocked sites (4 spins): inter-block bond + half of each block's internal bond and fields."""
    n = 4
    intra0 = pair(n, 0, 1) + field(n, 0) + field(n, 1)
    intra1 = pair(n, 2, 3) + field(n, 2) + field(n, 3)
    return pair(n, 1, 2) + 0.5 * (intra0 + intra1)


def three_site_term(hb):
    """h3 = (hb (x) 1 + 1 (x) hb)/2 on three blocked sites, as a 64x64 matrix, rows = ket (abc), cols = bra."""
    i4 = np.eye(4)
    return 0.5 * (np.kron(hb, i4) + np.kron(i4, hb))


def tfim_h3(hx=1.0):
    return three_site_term(two_block_term(*tfim_pair_and_field(hx)))


def xxz_h3(delta):
    return three_site_term(two_block_term(*xxz_pair_and_field(delta)))


def spin_ring_hamiltonian(nspins, pair, field):
    """Dense periodic spin-chain Hamiltonian sum_i pair(i, i+1) + field(i), built directly from Pauli strings."""
    H = np.zeros((2 ** nspins, 2 ** nspins))
    for i in range(nspins):
        H += pair(nspins, i, (i + 1) % nspins) + field(nspins, i)
    return H


def tfim_exact_energy_per_spin(hx=1.0):
    """Infinite-chain ground energy per spin of -sum X X - hx sum Z (free-fermion closed form); -4/pi at hx=1.

    Sum of the negative single-particle energies, -(1/2pi) int_{-pi}^{pi} eps(k) dk with
    eps(k) = sqrt(1 + hx^2 - 2 hx cos k) = sqrt((1 - hx)^2 + 4 hx sin^2(k/2)). The integrand is even; with
    t = k/2 the integral is (2/pi) int_0^{pi/2} sqrt((1 - hx)^2 + 4 hx sin^2 t) dt, which has no kink in the
    range (at hx = 1 the k-form has one at k = 0).
    """
    val, _ = integrate.quad(lambda t: np.sqrt((1.0 - hx) ** 2 + 4.0 * hx * np.sin(t) ** 2), 0.0, 0.5 * np.pi,
                            epsabs=0.0, epsrel=1e-13, limit=200)
    return -2.0 * val / np.pi


def xxz_exact_energy_per_spin(delta):
    """Infinite-chain ground energy per spin of sum XX + YY + delta ZZ (Pauli units), -1 < delta <= 1.

    Bethe-ansatz integral of Yang & Yang for spin-1/2 operators with delta = cos(gamma), times 4 for Pauli units;
    delta = 1 is the Hulthen value 1 - 4 ln 2.
    """
    if delta == 1.0:
        return 1.0 - 4.0 * np.log(2.0)
    if not (-1.0 < delta < 1.0):
        raise ValueError("closed form implemented for -1 < delta <= 1 only")
    g = np.arccos(delta)

    def f(x):
        # even integrand sinh((pi-g)x) / (sinh(pi x) cosh(g x)), rewritten with decaying exponentials for x > 0
        if x == 0.0:
            return (np.pi - g) / np.pi
        return (2.0 * np.exp(-2.0 * g * x) * -np.expm1(-2.0 * (np.pi - g) * x)
                / (-np.expm1(-2.0 * np.pi * x) * (1.0 + np.exp(-2.0 * g * x))))
    half, _ = integrate.quad(f, 0.0, np.inf, epsabs=1e-14, epsrel=1e-13, limit=400)
    val = 2.0 * half
    return 4.0 * (delta / 4.0 - 0.5 * np.sin(g) * val)
