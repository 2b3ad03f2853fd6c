"""Brute-force checkers for the oracle (TEST INFRASTRUCTURE ONLY).

Three independent ways to obtain matrix elements of the Hamiltonian:

* ``pauli_matrix``: the Pauli table as a sum of Kronecker products of 2x2
  matrices (no bit tricks), for up to 12 qubits.
* ``fock_matrix``: Eq. 2 applied literally, in its antisymmetrised form
  1/4 sum <pq||rs> a+_p a+_q a_s a_r plus sum h_pq a+_p a_q, to bit strings
  with explicit creation/annihilation operators.
* ``slater_condon``: the Slater-Condon rules for determinants differing by
  0, 1 or 2 spin orbitals (the baseline evaluator named in Sec. III-B).

All share the ONV ordering of Sec. II-A: spin orbital (p, alpha) is qubit 2p,
(p, beta) is qubit 2p+1, and |n> = a+_{j1} a+_{j2} ... |vac> with
j1 < j2 < ..., so a ladder operator on orbital j picks up (-1) to the number
of occupied orbitals below j.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_I2 = np.eye(2)
_X2 = np.array([[0.0, 1.0], [1.0, 0.0]])
_Z2 = np.array([[1.0, 0.0], [0.0, -1.0]])


def _bit(words, j):
    return (int(words[j // 64]) >> (j % 64)) & 1


def pauli_matrix(n_qubits, x, z, c, c_im=None):
    """Sparse 2^n x 2^n matrix of sum_t c_t i^{ny} X^{x_t} Z^{z_t}.

    Basis index b has qubit j in bit j, so the Kronecker factors are ordered
    from qubit n-1 (leftmost) down to qubit 0.
    """
    dim = 1 << n_qubits
    H = sp.csr_matrix((dim, dim), dtype=np.complex128)
    x = np.asarray(x, dtype=np.uint64).reshape(-1, 2)
    z = np.asarray(z, dtype=np.uint64).reshape(-1, 2)
    c = np.asarray(c, dtype=np.float64)
    ci = np.zeros_like(c) if c_im is None else np.asarray(c_im, dtype=np.float64)
    for t in range(c.shape[0]):
        ny = 0
        M = sp.identity(1, dtype=np.complex128, format="csr")
        for j in range(n_qubits - 1, -1, -1):
            xb, zb = _bit(x[t], j), _bit(z[t], j)
            ny += xb & zb
            m = _I2
            if xb:
                m = _X2
            if zb:
                m = m @ _Z2
            M = sp.kron(M, sp.csr_matrix(m), format="csr")
        coef = complex(c[t], ci[t]) * (1j ** ny)
        H = H + coef * M
    return H.tocsr()


# ---------------------------------------------------------------- fermions


def _apply_annihilate(state: int, j: int):
    if not (state >> j) & 1:
        return None, 0
    sign = -1 if bin(state & ((1 << j) - 1)).count("1") & 1 else 1
    return state ^ (1 << j), sign


def _apply_create(state: int, j: int):
    if (state >> j) & 1:
        return None, 0
    sign = -1 if bin(state & ((1 << j) - 1)).count("1") & 1 else 1
    return state | (1 << j), sign


def spin_orbital_integrals(h, eri):
    """Spin-orbital one-electron integrals and antisymmetrised <PQ||RS>.

    Spin orbital P = 2p + sigma.  <PQ|RS> = (pr|qs) delta(sP,sR) delta(sQ,sS)
    from the chemists' (pq|rs); <PQ||RS> = <PQ|RS> - <PQ|SR>.
    """
    K = h.shape[0]
    n = 2 * K
    hs = np.zeros((n, n))
    for P in range(n):
        for Q in range(n):
            if P % 2 == Q % 2:
                hs[P, Q] = h[P // 2, Q // 2]
    sp_ = np.arange(n) % 2
    o = np.arange(n) // 2
    # <PQ|RS> = (pr|qs) * d(sP,sR) d(sQ,sS)
    phys = eri[o[:, None, None, None], o[None, None, :, None], o[None, :, None, None],
               o[None, None, None, :]]
    phys = phys * ((sp_[:, None, None, None] == sp_[None, None, :, None])
                   & (sp_[None, :, None, None] == sp_[None, None, None, :]))
    anti = phys - phys.transpose(0, 1, 3, 2)
    return hs, anti


def fock_apply(hs, anti, state: int):
    """H|state> as a dict {state': amplitude} from Eq. 2 applied literally."""
    n = hs.shape[0]
    out: dict[int, float] = {}
    for p in range(n):
        for q in range(n):
            v = hs[p, q]
            if v == 0.0:
                continue
            s1, g1 = _apply_annihilate(state, q)
            if s1 is None:
                continue
            s2, g2 = _apply_create(s1, p)
            if s2 is None:
                continue
            out[s2] = out.get(s2, 0.0) + v * g1 * g2
    occ = [j for j in range(n) if (state >> j) & 1]
    for r in occ:
        s1, g1 = _apply_annihilate(state, r)
        for s in occ:
            s2, g2 = _apply_annihilate(s1, s)
            if s2 is None:
                continue
            for q in range(n):
                s3, g3 = _apply_create(s2, q)
                if s3 is None:
                    continue
                for p in range(n):
                    v = anti[p, q, r, s]
                    if v == 0.0:
                        continue
                    s4, g4 = _apply_create(s3, p)
                    if s4 is None:
                        continue
                    out[s4] = out.get(s4, 0.0) + 0.25 * v * g1 * g2 * g3 * g4
    return out


def fock_matrix(h, eri, states):
    """Dense <m|H|n> over the listed basis states (integers), from Eq. 2."""
    hs, anti = spin_orbital_integrals(h, eri)
    idx = {int(s): k for k, s in enumerate(states)}
    M = np.zeros((len(states), len(states)))
    for k, s in enumerate(states):
        for t, v in fock_apply(hs, anti, int(s)).items():
            if t in idx:
                M[idx[t], k] += v
    return M


# ---------------------------------------------------------------- Slater-Condon


def _words_to_int(w):
    return int(w[0]) | (int(w[1]) << 64)


def _gamma(ket: int, annihilate, create):
    """Sign of a+_{c1} ... a_{a_k} ... |ket> applied right to left (annihilators
    first, in the listed order, then creators in reverse listed order)."""
    s, g = ket, 1
    for j in annihilate:
        s, gj = _apply_annihilate(s, j)
        g *= gj
    for j in reversed(create):
        s, gj = _apply_create(s, j)
        g *= gj
    return s, g


class SlaterCondon:
    """<bra|H|ket> between determinants from the excitation-level rules.

    Works on spatial integrals directly: <PQ|RS> = (pr|qs) d(sP,sR) d(sQ,sS)
    and <PQ||RS> = <PQ|RS> - <PQ|SR>, evaluated on demand.
    """

    def __init__(self, h, eri):
        self.h = np.asarray(h, dtype=np.float64)
        self.eri = np.asarray(eri, dtype=np.float64)
        self.n = 2 * self.h.shape[0]

    def _phys(self, P, Q, R, S):
        if P % 2 != R % 2 or Q % 2 != S % 2:
            return 0.0
        return self.eri[P // 2, R // 2, Q // 2, S // 2]

    def anti(self, P, Q, R, S):
        return self._phys(P, Q, R, S) - self._phys(P, Q, S, R)

    def _h(self, P, Q):
        return self.h[P // 2, Q // 2] if P % 2 == Q % 2 else 0.0

    def element(self, bra: int, ket: int) -> float:
        diff = bra ^ ket
        nd = bin(diff).count("1")
        if nd == 0:
            occ = np.array([j for j in range(self.n) if (ket >> j) & 1], dtype=np.int64)
            o, sg = occ // 2, occ % 2
            e1 = float(np.sum(self.h[o, o]))
            coul = self.eri[o[:, None], o[:, None], o[None, :], o[None, :]]
            exch = self.eri[o[:, None], o[None, :], o[None, :], o[:, None]] * (sg[:, None] == sg[None, :])
            return e1 + 0.5 * float(np.sum(coul - exch))
        if nd == 2:
            i = (diff & ket).bit_length() - 1            # occupied in ket only
            a = (diff & bra).bit_length() - 1            # occupied in bra only
            s, g = _gamma(ket, [i], [a])
            assert s == bra
            occ = [j for j in range(self.n) if (ket >> j) & 1 and j != i]
            v = self._h(a, i) + sum(self.anti(a, j, i, j) for j in occ)
            return g * v
        if nd == 4:
            ii = [j for j in range(self.n) if (diff & ket) >> j & 1]
            aa = [j for j in range(self.n) if (diff & bra) >> j & 1]
            if len(ii) != 2:
                return 0.0
            i, j = ii
            a, b = aa
            # |bra> = G a+_a a+_b a_j a_i |ket>
            s, g = _gamma(ket, [i, j], [a, b])
            assert s == bra
            return g * self.anti(a, b, i, j)
        return 0.0

    def elements(self, bras, kets):
        return np.array([self.element(_words_to_int(b), _words_to_int(k))
                         for b, k in zip(bras, kets)])


def sector_ground_state(h, eri, states):
    """Lowest eigenpair of Eq. 2 restricted to the listed sector states."""
    M = fock_matrix(h, eri, [_words_to_int(s) for s in states])
    w, v = np.linalg.eigh(M)
    return float(w[0]), v[:, 0], M
