"""Dense brute-force Wilson-Dirac matrix for tiny lattices (tests only).

Written independently of the oracle: its own site enumeration (a dict from
coordinate tuples to indices), the gamma structure taken from the printed
projector tables in tests/golden, and Kronecker products for spin x colour.
It follows the hopping term of Eq. 1 entry by entry:
  D[x, x+mu] += P^{-mu} (x) U_x^mu,     D[x, x-mu] += P^{+mu} (x) U_{x-mu}^mu^dagger,
with a factor -1 on hops that cross the t boundary of an antiperiodic lattice.
Spinor vector index: 12 * site + 3 * spin + colour.
"""
import itertools

import numpy as np

from golden_io import read_projectors

PROJ = read_projectors("projectors_degrand_rossi.txt")

# Change of basis psi_UK = S psi_DR between the two printed tables of
# Appendix B (checked against both tables by the oracle pins).
UKQCD_S = np.array([[0, 1, 0, 1], [-1, 0, -1, 0], [0, 1, 0, -1], [-1, 0, 1, 0]]) / np.sqrt(2)


def gammas(proj=PROJ):
    """gamma_mu = (P^{+mu} - P^{-mu}) / 2 for mu = 1..4 (list index 0..3)."""
    return [(proj[("+", m)] - proj[("-", m)]) / 2 for m in range(1, 5)]


def enumerate_sites(dims):
    lx, ly, lz, lt = dims
    coords = [(x, y, z, t) for t, z, y, x in itertools.product(range(lt), range(lz), range(ly), range(lx))]
    return coords, {c: i for i, c in enumerate(coords)}


def links_complex(U):
    """[Lt,Lz,Ly,Lx,4,3,3,2] float -> [V,4,3,3] complex (same site order)."""
    V = int(np.prod(U.shape[:4]))
    return (U[..., 0] + 1j * U[..., 1]).reshape(V, 4, 3, 3)


def dense_hopping(dims, U, antiperiodic_t=True, proj=PROJ):
    coords, index = enumerate_sites(dims)
    L = list(dims)
    Uc = links_complex(U)
    V = len(coords)
    D = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    for i, c in enumerate(coords):
        for mu in range(4):
            fwd = list(c)
            fwd[mu] = (c[mu] + 1) % L[mu]
            bwd = list(c)
            bwd[mu] = (c[mu] - 1) % L[mu]
            s_f = -1.0 if (antiperiodic_t and mu == 3 and c[3] == L[3] - 1) else 1.0
            s_b = -1.0 if (antiperiodic_t and mu == 3 and c[3] == 0) else 1.0
            j, k = index[tuple(fwd)], index[tuple(bwd)]
            D[12 * i:12 * i + 12, 12 * j:12 * j + 12] += s_f * np.kron(proj[("-", mu + 1)], Uc[i, mu])
            D[12 * i:12 * i + 12, 12 * k:12 * k + 12] += s_b * np.kron(proj[("+", mu + 1)],
                                                                       Uc[k, mu].conj().T)
    return D


def parity_masks(dims):
    coords, _ = enumerate_sites(dims)
    par = np.array([sum(c) % 2 for c in coords])
    even = np.repeat(par == 0, 12)
    odd = np.repeat(par == 1, 12)
    return even, odd


def to_vec(psi):
    """[..., 4, 3, 2] float -> flat complex vector."""
    return (psi[..., 0] + 1j * psi[..., 1]).reshape(-1)


def from_vec(v):
    """flat complex vector -> [n, 4, 3, 2] float."""
    v = np.asarray(v).reshape(-1, 4, 3)
    return np.stack([v.real, v.imag], axis=-1)
