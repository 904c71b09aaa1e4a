"""Seeded input generators (no solver arithmetic lives here).

Conventions shared by every consumer:

* complex128 NumPy arrays, row-major blocks;
* a block-tridiagonal pair (H, S) with nb diagonal blocks of size s is stored as
  ``Hd[nb, s, s]`` (H_{i,i}), ``Hu[nb-1, s, s]`` (H_{i,i+1}); the lower blocks are the conjugate
  transposes ``H_{i+1,i} = Hu[i]^H`` because H and S are Hermitian (Sec. 2B: H and S are the
  Hamiltonian and overlap of a localized basis; Sec. 3B: A = E*S - H is symmetric/Hermitian);
* a lead is one periodic cell ``(H00, H01, S00, S01)`` repeated to infinity (Sec. 3A, Eq. (bound)
  with a nearest-cell range).

Recipes
-------
``chain_cell``     random 1-D chain cell: H00 Hermitian with entries of variance 1/s, H01 complex
                   normal with E|h|^2 = 0.5/s, S = identity.
``dft_like_cell``  lattice-slab cell that mimics dense DFT blocks: Lx*Ly*Lz orbitals, couplings
                   exp(-d/2)*N(0,1) for 0 < d <= Lx (d = Euclidean distance, periodic in z with Bloch
                   phase k), onsite energies U[-5, 5] eV drawn once per orbital of the cell, overlap
                   c*exp(-d/2) off-diagonal with unit diagonal, c halved until the Bloch overlap is
                   positive definite with margin 0.05.  The cutoff d <= Lx makes the device matrix exactly
                   block-tridiagonal.
"""
from __future__ import annotations

import functools
from dataclasses import dataclass

import numpy as np

# Lattice-slab shapes (Lx, Ly, Lz): x is transport, y confined, z periodic with momentum k.
SLAB_SHAPES = {
    24: (2, 3, 4),
    40: (2, 4, 5),
    48: (3, 4, 4),
    72: (3, 4, 6),
    100: (4, 5, 5),
    128: (4, 4, 8),
    160: (4, 5, 8),
    256: (4, 8, 8),
    384: (6, 8, 8),
    512: (8, 8, 8),
    768: (8, 8, 12),
    1024: (8, 8, 16),
}


@dataclass
class BTDInstance:
    """A device (block-tridiagonal H, S) plus its lead cell."""

    Hd: np.ndarray
    Hu: np.ndarray
    Sd: np.ndarray
    Su: np.ndarray
    H00: np.ndarray
    H01: np.ndarray
    S00: np.ndarray
    S01: np.ndarray

    @property
    def nb(self) -> int:
        return self.Hd.shape[0]

    @property
    def s(self) -> int:
        return self.Hd.shape[1]


def _cnormal(rng, shape):
    """Complex normal with unit variance: (x + i y)/sqrt(2)."""
    x = rng.standard_normal(shape)
    y = rng.standard_normal(shape)
    return (x + 1j * y) / np.sqrt(2.0)


def chain_cell(s: int, seed: int = 0):
    """Random 1-D chain cell (H00, H01, S00, S01); S = identity.

    Draw order from ``default_rng(seed)``: real then imaginary part of G (H00 = (G + G^H)/sqrt(2)/sqrt(s)),
    then real then imaginary part of the coupling (H01 = sqrt(0.5) * (x + i y)/sqrt(2)/sqrt(s)).
    """
    rng = np.random.default_rng(seed)
    g = _cnormal(rng, (s, s))
    h00 = (g + g.conj().T) / np.sqrt(2.0) / np.sqrt(s)
    h01 = np.sqrt(0.5) * _cnormal(rng, (s, s)) / np.sqrt(s)
    s00 = np.eye(s, dtype=np.complex128)
    s01 = np.zeros((s, s), dtype=np.complex128)
    return h00.astype(np.complex128), h01.astype(np.complex128), s00, s01


def scalar_chain_cell(eps0: float, t: float):
    """One-orbital chain with onsite eps0 and hopping -t (S = 1)."""
    h00 = np.array([[eps0]], dtype=np.complex128)
    h01 = np.array([[-t]], dtype=np.complex128)
    return h00, h01, np.eye(1, dtype=np.complex128), np.zeros((1, 1), dtype=np.complex128)


def ladder_cell(eps, t):
    """s decoupled chains: diagonal onsite eps[k] and hopping -t[k] (S = identity)."""
    eps = np.asarray(eps, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    s = eps.size
    h00 = np.diag(eps).astype(np.complex128)
    h01 = np.diag(-t).astype(np.complex128)
    return h00, h01, np.eye(s, dtype=np.complex128), np.zeros((s, s), dtype=np.complex128)


class DFTLikeCell:
    """Real-space pieces of the lattice-slab cell; ``at(k)`` gives the Bloch cell at momentum k."""

    def __init__(self, shape, seed: int):
        lx, ly, lz = shape
        if lz < lx:
            raise ValueError("need Lz >= Lx so that only z-images m in {-1,0,1} are within the cutoff")
        self.shape = (lx, ly, lz)
        s = lx * ly * lz
        self.s = s
        idx = np.arange(s)
        x = idx // (ly * lz)
        y = (idx // lz) % ly
        z = idx % lz
        rc = float(lx)
        rng = np.random.default_rng(seed)
        onsite = rng.uniform(-5.0, 5.0, s)
        g = rng.standard_normal((s, s))
        w_intra0 = (g + g.T) / np.sqrt(2.0)
        w_intra1 = rng.standard_normal((s, s))
        w_inter = {m: rng.standard_normal((s, s)) for m in (-1, 0, 1)}

        def dist(dx_cell, m):
            ddx = x[None, :] + lx * dx_cell - x[:, None]
            ddy = y[None, :] - y[:, None]
            ddz = z[None, :] + lz * m - z[:, None]
            return np.sqrt(ddx * ddx + ddy * ddy + ddz * ddz)

        def decay(d):
            return np.where((d > 0) & (d <= rc), np.exp(-d / 2.0), 0.0)

        d_intra0, d_intra1 = dist(0, 0), dist(0, 1)
        self.h_intra = {
            0: decay(d_intra0) * w_intra0 + np.diag(onsite),
            1: decay(d_intra1) * w_intra1,
        }
        self.h_intra[-1] = self.h_intra[1].T.copy()
        self.h_inter = {m: decay(dist(1, m)) * w_inter[m] for m in (-1, 0, 1)}
        self._s_intra = {0: decay(d_intra0), 1: decay(d_intra1)}
        self._s_intra[-1] = self._s_intra[1].T.copy()
        self._s_inter = {m: decay(dist(1, m)) for m in (-1, 0, 1)}
        self.c = overlap_scale(self.shape)
        self.onsite = onsite

    def s_pieces(self):
        c = self.c
        s_intra = {m: c * v for m, v in self._s_intra.items()}
        s_intra[0] = s_intra[0] + np.eye(self.s)
        s_inter = {m: c * v for m, v in self._s_inter.items()}
        return s_intra, s_inter

    def at(self, k: float):
        """Bloch cell (H00, H01, S00, S01) at transverse momentum k (phase e^{i k m} per z-image m)."""
        ph = {m: np.exp(1j * k * m) for m in (-1, 0, 1)}
        h00 = sum(self.h_intra[m] * ph[m] for m in (-1, 0, 1))
        h01 = sum(self.h_inter[m] * ph[m] for m in (-1, 0, 1))
        s_intra, s_inter = self.s_pieces()
        s00 = sum(s_intra[m] * ph[m] for m in (-1, 0, 1))
        s01 = sum(s_inter[m] * ph[m] for m in (-1, 0, 1))
        return tuple(np.ascontiguousarray(a, dtype=np.complex128) for a in (h00, h01, s00, s01))


@functools.lru_cache(maxsize=None)
def overlap_scale(shape) -> float:
    """Largest c in {1, 1/2, 1/4, ...} whose Bloch overlap S(kx, kz) has lambda_min >= 0.05.

    The Bloch overlap S(kx,kz) = S00(kz) + S01(kz) e^{i kx} + S01(kz)^H e^{-i kx} is checked on a 9 x 5
    grid of (kx, kz) in [0, pi] x [0, pi].  A positive-definite Bloch symbol makes every finite
    block-tridiagonal section SPD.  The overlap has no random part, so c depends on the shape only.
    """
    lx, ly, lz = shape
    s = lx * ly * lz
    idx = np.arange(s)
    x = idx // (ly * lz)
    y = (idx // lz) % ly
    z = idx % lz
    rc = float(lx)

    def decay(dx_cell, m):
        ddx = x[None, :] + lx * dx_cell - x[:, None]
        ddy = y[None, :] - y[:, None]
        ddz = z[None, :] + lz * m - z[:, None]
        d = np.sqrt(ddx * ddx + ddy * ddy + ddz * ddz)
        return np.where((d > 0) & (d <= rc), np.exp(-d / 2.0), 0.0)

    intra = {0: decay(0, 0), 1: decay(0, 1)}
    intra[-1] = intra[1].T
    inter = {m: decay(1, m) for m in (-1, 0, 1)}
    c = 1.0
    for _ in range(40):
        lam = np.inf
        for kz in np.linspace(0.0, np.pi, 5):
            ph = {m: np.exp(1j * kz * m) for m in (-1, 0, 1)}
            s00 = np.eye(s) + c * sum(intra[m] * ph[m] for m in (-1, 0, 1))
            s01 = c * sum(inter[m] * ph[m] for m in (-1, 0, 1))
            for kx in np.linspace(0.0, np.pi, 9):
                sk = s00 + s01 * np.exp(1j * kx) + s01.conj().T * np.exp(-1j * kx)
                lam = min(lam, np.linalg.eigvalsh(sk).min())
        if lam >= 0.05:
            return c
        c *= 0.5
    raise RuntimeError("could not make the overlap positive definite")


def dft_like_cell(s: int, seed: int, k: float):
    """Bloch cell of the lattice-slab recipe for orbital count s (see ``SLAB_SHAPES``)."""
    return DFTLikeCell(SLAB_SHAPES[s], seed).at(k)


def device_from_cell(cell, nb: int, onsite_disorder=None, seed: int | None = None) -> BTDInstance:
    """Device of nb copies of the cell, leads = the same cell (a perfect crystal).

    ``onsite_disorder`` (eV): if given, every device block gets its own extra diagonal drawn
    U[-w/2, w/2] from ``default_rng(seed)``; the leads stay clean.  All nb blocks are materialised.
    """
    h00, h01, s00, s01 = cell
    s = h00.shape[0]
    hd = np.repeat(h00[None], nb, axis=0).copy()
    hu = np.repeat(h01[None], max(nb - 1, 0), axis=0).copy()
    sd = np.repeat(s00[None], nb, axis=0).copy()
    su = np.repeat(s01[None], max(nb - 1, 0), axis=0).copy()
    if onsite_disorder:
        rng = np.random.default_rng(seed)
        w = float(onsite_disorder)
        for i in range(nb):
            hd[i] += np.diag(rng.uniform(-w / 2, w / 2, s))
    return BTDInstance(hd, hu, sd, su, h00.copy(), h01.copy(), s00.copy(), s01.copy())


def random_btd(nb: int, s: int, seed: int, overlap: bool = True, lead_seed: int | None = None) -> BTDInstance:
    """Disordered device: every block drawn independently; lead cell = ``chain_cell`` of its own seed.

    With ``overlap`` the device overlap is S = I + 0.1*(Hermitian random), blocks scaled so S stays SPD.
    """
    rng = np.random.default_rng(seed)
    hd = np.empty((nb, s, s), np.complex128)
    hu = np.empty((max(nb - 1, 0), s, s), np.complex128)
    for i in range(nb):
        g = _cnormal(rng, (s, s))
        hd[i] = (g + g.conj().T) / np.sqrt(2.0) / np.sqrt(s)
    for i in range(nb - 1):
        hu[i] = np.sqrt(0.5) * _cnormal(rng, (s, s)) / np.sqrt(s)
    sd = np.repeat(np.eye(s, dtype=np.complex128)[None], nb, axis=0)
    su = np.zeros((max(nb - 1, 0), s, s), np.complex128)
    lead = chain_cell(s, seed=(seed + 7919) if lead_seed is None else lead_seed)
    if overlap:
        for i in range(nb):
            g = _cnormal(rng, (s, s))
            sd[i] = sd[i] + 0.05 * (g + g.conj().T) / np.sqrt(2.0) / np.sqrt(s)
        for i in range(nb - 1):
            su[i] = 0.05 * _cnormal(rng, (s, s)) / np.sqrt(s)
        h00, h01, _, _ = lead
        lead = (h00, h01, sd[0].copy(), su[0].copy() if nb > 1 else np.zeros((s, s), np.complex128))
    return BTDInstance(hd, hu, sd, su, *lead)


def gauge_rotate(inst: BTDInstance, u: np.ndarray) -> BTDInstance:
    """Apply the same unitary basis change u to every block: X -> u^H X u."""
    uh = u.conj().T

    def rot(a):
        return np.einsum("ij,njk,kl->nil", uh, a, u) if a.ndim == 3 else uh @ a @ u

    return BTDInstance(*(rot(a) for a in (inst.Hd, inst.Hu, inst.Sd, inst.Su, inst.H00, inst.H01, inst.S00, inst.S01)))


def random_unitary(s: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(_cnormal(rng, (s, s)))
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]


def injection_block(s: int, m: int, seed: int) -> np.ndarray:
    """Non-zero rows b' of the injection (2s x m): complex normal, seeded."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(_cnormal(rng, (2 * s, m)))
