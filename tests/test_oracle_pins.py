"""Pins for the CPU oracle and the input producer, against what mathematics
and textbook closed forms fix (no GPU).

Each pin is chosen so that a plausible slip in the oracle (a dropped i^ny, a
sign taken from the wrong state, an inverted amplitude ratio, a wrong skip
bound, a lost term) or in the Jordan-Wigner producer fails at least one test.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ints(words):
    return [int(w[0]) | (int(w[1]) << 64) for w in words]


def _random_psi(rng, n, sigma=1.0):
    return rng.normal(0.0, sigma, n), rng.uniform(0.0, 2 * math.pi, n)


def _dense_eloc(Hss, la, ph):
    psi = np.exp(la + 1j * ph)
    return (Hss @ psi) / psi


# ---------------------------------------------------------------- producer


@pytest.mark.parametrize("K", [2, 4, 6, 20])
def test_jw_counts_match_closed_form(K):
    """G and T of a dense molecular Hamiltonian follow closed forms (Eq. 2 via JW)."""
    h, eri = W.integrals(np.random.default_rng([0, 0]), K, 4.0)
    x, z, c = W.jw_terms(h, eri)
    G, T, _ = W.closed_form_counts(K, K // 2)
    assert oracle.n_groups(x) == G
    assert len(c) == T


def test_jw_odd_y_strings_cancel():
    """Odd-Y strings of a real Hamiltonian cancel to rounding (kept with no threshold)."""
    h, eri = W.integrals(np.random.default_rng([0, 0]), 6, 4.0)
    x, z, c, ci = W.jw_terms(h, eri, thresh=0.0, keep_odd=True)
    ny = np.array([bin(int(a) & int(b)).count("1") + bin(int(a2) & int(b2)).count("1")
                   for (a, a2), (b, b2) in zip(x, z)])
    odd = ny % 2 == 1
    assert odd.sum() > 0
    assert np.abs(ci[odd]).max() < 1e-15
    assert np.abs(c[odd]).max() == 0.0
    assert np.abs(ci[~odd]).max() == 0.0


def test_pauli_matrix_equals_fock_matrix_full_space():
    """Kronecker-product Pauli H == Eq. 2 applied to bit strings, all 2^8 states."""
    K = 4
    h, eri = W.integrals(np.random.default_rng([7, 0]), K, 4.0)
    x, z, c = W.jw_terms(h, eri, thresh=0.0)
    Hp = dense.pauli_matrix(2 * K, x, z, c).toarray()
    Hf = dense.fock_matrix(h, eri, list(range(1 << (2 * K))))
    assert np.abs(Hp.imag).max() < 1e-14
    assert np.abs(Hp.real - Hf).max() < 1e-12
    # Hermitian and (N_alpha, N_beta)-conserving
    assert np.abs(Hp - Hp.conj().T).max() < 1e-13
    states = np.arange(1 << (2 * K))
    na = np.array([bin(s & 0x55).count("1") for s in states])
    nb = np.array([bin(s & 0xAA).count("1") for s in states])
    nz = np.abs(Hf) > 0
    rows, cols = np.nonzero(nz)
    assert (na[rows] == na[cols]).all() and (nb[rows] == nb[cols]).all()


def test_slater_condon_equals_fock_matrix():
    """Slater-Condon rules == Eq. 2 on every same-sector pair (K = 4)."""
    K = 4
    h, eri = W.integrals(np.random.default_rng([8, 0]), K, 4.0)
    sc = dense.SlaterCondon(h, eri)
    states = list(range(1 << (2 * K)))
    Hf = dense.fock_matrix(h, eri, states)
    for a in states:
        for b in states:
            if bin(a & 0x55).count("1") != bin(b & 0x55).count("1"):
                continue
            if bin(a & 0xAA).count("1") != bin(b & 0xAA).count("1"):
                continue
            assert abs(sc.element(a, b) - Hf[a, b]) < 1e-12, (a, b)


def test_hubbard_dimer_spectrum_golden():
    """JW table of the Hubbard dimer reproduces the textbook spectrum."""
    rows = np.loadtxt(os.path.join(GOLDEN, "hubbard_dimer.txt"))
    for t, U, *E in rows:
        h = np.array([[0.0, -t], [-t, 0.0]])
        eri = np.zeros((2, 2, 2, 2))
        eri[0, 0, 0, 0] = eri[1, 1, 1, 1] = U
        x, z, c = W.jw_terms(h, eri)
        states = W.sector_states(2, 1, 1)
        idx = [int(s[0]) for s in states]
        Hp = dense.pauli_matrix(4, x, z, c).toarray()[np.ix_(idx, idx)]
        w, v = np.linalg.eigh(Hp)
        assert np.allclose(w, E, atol=1e-12)
        # every eigenvector gives a constant local energy equal to its eigenvalue
        for k in range(4):
            vec = v[:, k]
            if np.min(np.abs(vec)) < 1e-6:
                continue
            la = np.log(np.abs(vec))
            ph = np.angle(vec)
            el, _, _ = oracle.eloc(4, x, z, c, states, la, ph)
            assert np.allclose(el, E[k], atol=1e-12), (t, U, k)


# ---------------------------------------------------------------- oracle E_loc


@pytest.fixture(scope="module")
def nq12(workload_cache):
    return workload_cache(("workload", "nq12"))


@pytest.fixture(scope="module")
def nq12_dense(nq12):
    idx = [int(s[0]) for s in nq12.samples]
    Hp = dense.pauli_matrix(12, nq12.x, nq12.z, nq12.c)
    return Hp[idx][:, idx].toarray()


def test_oracle_equals_dense_on_random_subsets(nq12, nq12_dense):
    """E_loc(x) = (H_SS psi_S)_x / psi_x for random S inside the sector (Eq. 5, LUT semantics)."""
    rng = np.random.default_rng(11)
    for size in (1, 7, 64, 250, 400):
        sel = np.sort(rng.choice(400, size=size, replace=False))
        S = nq12.samples[sel]
        la, ph = _random_psi(rng, size)
        el, ab, _ = oracle.eloc(12, nq12.x, nq12.z, nq12.c, S, la, ph)
        ref = _dense_eloc(nq12_dense[np.ix_(sel, sel)], la, ph)
        assert np.all(np.abs(el - ref) <= 1e-12 * ab + 1e-300)


def test_oracle_equals_fock_matrix_from_integrals(nq12):
    """Same check with H built from the integrals by Eq. 2, not from the Pauli table."""
    Hf = dense.fock_matrix(nq12.h, nq12.eri, _ints(nq12.samples))
    el, ab, _ = oracle.eloc(12, nq12.x, nq12.z, nq12.c, nq12.samples, nq12.log_amp, nq12.phase)
    ref = _dense_eloc(Hf, nq12.log_amp, nq12.phase)
    assert np.all(np.abs(el - ref) <= 1e-12 * ab)


def test_oracle_ground_eigenvector_gives_constant_eloc(nq12):
    """With psi the exact sector ground state, E_loc == E0 (zero-variance principle)."""
    E0, v, _ = dense.sector_ground_state(nq12.h, nq12.eri, nq12.samples)
    la = np.log(np.abs(v))
    ph = np.where(v < 0, math.pi, 0.0)
    el, _, _ = oracle.eloc(12, nq12.x, nq12.z, nq12.c, nq12.samples, la, ph)
    keep = np.abs(v) >= 1e-4 * np.abs(v).max()
    print(f"excluded small components: {(~keep).sum()} of {keep.size}")
    assert np.abs(el[keep] - E0).max() <= 1e-10
    # eigen-solver residuals are amplified by max|v| / |v_x| below the cut
    amp = np.abs(v).max() / np.abs(v[~keep])
    assert np.all(np.abs(el[~keep] - E0) <= 1e-14 * amp * abs(E0) + 1e-10)
    mean, var, _ = oracle.energy(np.ones(400, np.int64), el)
    wmean = np.sum(np.abs(v) ** 2 * el.real) / np.sum(np.abs(v) ** 2)
    assert abs(wmean - E0) <= 1e-12 * abs(E0)
    assert var < 1e-18


def test_oracle_unit_psi_gives_row_sums(nq12, nq12_dense):
    """psi == 1 over the whole sector: E_loc is the row sum of H, mean is 1'H1/|S|."""
    n = nq12.n_samples
    el, _, _ = oracle.eloc(12, nq12.x, nq12.z, nq12.c, nq12.samples, np.zeros(n), np.zeros(n))
    rows = nq12_dense.sum(axis=1)
    assert np.abs(el - rows).max() < 1e-12
    mean, _, _ = oracle.energy(np.ones(n, np.int64), el)
    assert abs(mean - nq12_dense.sum() / n) < 1e-12


def test_oracle_connected_count_closed_form(nq12):
    """Every sample connects to all in-sector single/double flips plus itself."""
    _, _, conn = W.closed_form_counts(6, 3)
    _, _, nc = oracle.eloc(12, nq12.x, nq12.z, nq12.c, nq12.samples, nq12.log_amp, nq12.phase)
    assert (nc == conn + 1).all()
    pairs = oracle.connected_pairs(nq12.x, nq12.samples)
    assert pairs.shape[0] == 400 * (conn + 1)


def test_oracle_hermitian_and_permutation(nq12):
    """<x|H|x'> = conj(<x'|H|x>); permuting S permutes E_loc."""
    pairs = oracle.connected_pairs(nq12.x, nq12.samples)
    S = nq12.samples
    a = oracle.hij(nq12.x, nq12.z, nq12.c, S[pairs[:, 0]], S[pairs[:, 1]])
    b = oracle.hij(nq12.x, nq12.z, nq12.c, S[pairs[:, 1]], S[pairs[:, 0]])
    assert np.abs(a - np.conj(b)).max() < 1e-13
    perm = np.random.default_rng(3).permutation(400)
    el, _, _ = oracle.eloc(12, nq12.x, nq12.z, nq12.c, S, nq12.log_amp, nq12.phase)
    elp, _, _ = oracle.eloc(12, nq12.x, nq12.z, nq12.c, S[perm], nq12.log_amp[perm],
                            nq12.phase[perm])
    assert np.abs(elp - el[perm]).max() < 1e-12 * np.abs(el).max()


def test_oracle_general_pauli_sets_against_kronecker():
    """Non-molecular Pauli sets (arbitrary X masks, odd and even #Y, complex
    coefficients) on 10 qubits against Kronecker products."""
    rng = np.random.default_rng(5)
    nq = 10
    T = 300
    bits = rng.random((T, nq)) < 0.3
    zb = rng.random((T, nq)) < 0.4
    x = W.pack_bits(bits)
    z = W.pack_bits(zb)
    c = rng.normal(size=T)
    ci = rng.normal(size=T)
    H = dense.pauli_matrix(nq, x, z, c, ci).toarray()
    S_idx = np.sort(rng.choice(1 << nq, size=300, replace=False))
    S = np.zeros((300, 2), np.uint64)
    S[:, 0] = S_idx
    la, ph = _random_psi(rng, 300)
    el, ab, _ = oracle.eloc(nq, x, z, c, S, la, ph, c_im=ci)
    ref = _dense_eloc(H[np.ix_(S_idx, S_idx)], la, ph)
    assert np.all(np.abs(el - ref) <= 1e-12 * ab)


# ---------------------------------------------------------------- large N_q closure sets


def closure_set(K, n, n_seed_states, n_doubles, seed):
    """A few random sector states, all their single flips and some double flips."""
    rng = np.random.default_rng(seed)
    base = W.sector_samples(rng, K, n, n, n_seed_states)
    out = {tuple(int(v) for v in b) for b in base}
    bits = W.unpack_bits(base, 2 * K)
    for row in bits:
        for spin in (0, 1):
            occ = [2 * p + spin for p in range(K) if row[2 * p + spin]]
            vir = [2 * p + spin for p in range(K) if not row[2 * p + spin]]
            for i in occ:
                for a in vir:
                    r = row.copy()
                    r[i] = False
                    r[a] = True
                    out.add(tuple(int(v) for v in W.pack_bits(r[None])[0]))
        occ = np.nonzero(row)[0]
        vir = np.nonzero(~row)[0]
        added = 0
        while added < n_doubles:
            i, j = rng.choice(occ, 2, replace=False)
            a, b = rng.choice(vir, 2, replace=False)
            r = row.copy()
            r[[i, j]] = False
            r[[a, b]] = True
            if r[0::2].sum() != n or r[1::2].sum() != n:
                continue
            out.add(tuple(int(v) for v in W.pack_bits(r[None])[0]))
            added += 1
    arr = np.array(sorted(out), dtype=np.uint64)
    return arr[rng.permutation(len(arr))]


@pytest.mark.parametrize("K,n,L", [(20, 10, 4.0), (50, 25, 6.0)])
def test_oracle_matches_slater_condon_on_closure_sets(K, n, L, workload_cache):
    """Connected pairs of closure sets (bits on both sides of the 64-bit word
    boundary at 100 qubits) match Slater-Condon to 1e-12."""
    def make():
        h, eri = W.integrals(np.random.default_rng([1 if K == 20 else 2, 0]), K, L)
        x, z, c = W.jw_terms(h, eri)
        return h, eri, x, z, c
    h, eri, x, z, c = workload_cache(("ham", K), make)
    S = closure_set(K, n, 2, 150, seed=K)
    pairs = oracle.connected_pairs(x, S)
    assert pairs.shape[0] > 5 * S.shape[0]
    hs = oracle.hij(x, z, c, S[pairs[:, 0]], S[pairs[:, 1]])
    sc = dense.SlaterCondon(h, eri)
    sel = np.random.default_rng(0).choice(pairs.shape[0], size=min(3000, pairs.shape[0]),
                                          replace=False)
    ref = sc.elements(S[pairs[sel, 0]], S[pairs[sel, 1]])
    assert np.abs(hs[sel].imag).max() == 0.0
    assert np.abs(hs[sel].real - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    if 2 * K > 64:
        lo = (S[pairs[sel, 0], 0] ^ S[pairs[sel, 1], 0]) != 0
        hi = (S[pairs[sel, 0], 1] ^ S[pairs[sel, 1], 1]) != 0
        assert (lo & hi).any()
    # E_loc assembled from Slater-Condon elements, on a subset of rows
    la, ph = _random_psi(np.random.default_rng(1), S.shape[0], 0.5)
    rows = np.sort(np.random.default_rng(2).choice(S.shape[0], size=40, replace=False))
    el, ab, _ = oracle.eloc_rows(2 * K, x, z, c, S, la, ph, rows)
    for k, i in enumerate(rows):
        js = pairs[pairs[:, 0] == i, 1]
        full = sc.elements(np.repeat(S[i:i + 1], len(js), axis=0), S[js])
        ratio = np.exp(la[js] - la[i] + 1j * (ph[js] - ph[i]))
        ref_el = np.sum(full * ratio)
        assert abs(el[k] - ref_el) <= 1e-12 * ab[k]


def _absum_from_terms(x, c, S, la):
    """A(x) written out from its definition, in numpy: the diagonal group's
    sum of |c_t|, plus, for every other x' in S reached by some X_t = x ^ x',
    |psi(x') / psi(x)| = exp(a(x') - a(x)) times the sum of |c_t| over the
    terms with that X."""
    groups = {}
    for (a, b), cc in zip(x.tolist(), np.abs(c).tolist()):
        groups.setdefault((a, b), []).append(cc)
    gsum = {k: math.fsum(v) for k, v in groups.items()}
    maxpop = max(int(np.bitwise_count(np.uint64(a))) + int(np.bitwise_count(np.uint64(b)))
                 for a, b in groups)
    n = S.shape[0]
    A = np.zeros(n)
    for i in range(n):
        d0 = S[i, 0] ^ S[:, 0]
        d1 = S[i, 1] ^ S[:, 1]
        near = np.nonzero(np.bitwise_count(d0).astype(int) + np.bitwise_count(d1) <= maxpop)[0]
        parts = []
        for j in near.tolist():
            g = gsum.get((int(d0[j]), int(d1[j])))
            if g is not None:
                parts.append(math.exp(la[j] - la[i]) * g)
        A[i] = math.fsum(parts)
    return A


@pytest.mark.parametrize("case", ["nq12", "closure100"])
def test_oracle_absum_equals_its_definition(case, nq12, workload_cache):
    """The scale A(x) that every floating-point tolerance is taken against is
    what its definition says: an inflated A(x) (a doubled group, a ratio
    taken the wrong way round) would loosen every parity check silently."""
    if case == "nq12":
        x, z, c, S = nq12.x, nq12.z, nq12.c, nq12.samples
        la, ph = _random_psi(np.random.default_rng(31), S.shape[0], 1.0)
        nq = 12
    else:
        def make():
            h, eri = W.integrals(np.random.default_rng([2, 0]), 50, 6.0)
            x_, z_, c_ = W.jw_terms(h, eri)
            return h, eri, x_, z_, c_
        _, _, x, z, c = workload_cache(("ham", 50), make)
        S = closure_set(50, 25, 2, 150, seed=50)
        la, ph = _random_psi(np.random.default_rng(32), S.shape[0], 1.0)
        nq = 100
    _, ab, nc = oracle.eloc(nq, x, z, c, S, la, ph)
    A = _absum_from_terms(x, c, S, la)
    assert (nc > 1).sum() > S.shape[0] // 2
    assert np.all(np.abs(ab - A) <= 1e-13 * A), np.max(np.abs(ab - A) / A)


# ---------------------------------------------------------------- energy


def test_energy_invariants():
    """Eq. 1: constant E_loc has zero variance; scaling the counts changes nothing;
    a two-sample case matches the definition worked by hand."""
    rng = np.random.default_rng(2)
    w = rng.integers(1, 9, 1000)
    el = np.full(1000, -3.25 + 0.5j)
    m, v, sw = oracle.energy(w, el)
    assert m == -3.25 + 0.5j and v == 0.0 and sw == w.sum()
    el = rng.normal(size=1000) + 1j * rng.normal(size=1000)
    m1, v1, _ = oracle.energy(w, el)
    m3, v3, _ = oracle.energy(3 * w, el)
    assert abs(m1 - m3) < 1e-15 and abs(v1 - v3) < 1e-14
    # w = (1, 3), E = (1, 5): mean 4, var (1*9 + 3*1)/4 = 3
    m, v, sw = oracle.energy([1, 3], [1.0, 5.0])
    assert m == 4.0 and v == 3.0 and sw == 4.0
    # complex: E = (i, -i) with w = (1, 1): mean 0, var 1
    m, v, _ = oracle.energy([1, 1], [1j, -1j])
    assert m == 0 and v == 1.0
