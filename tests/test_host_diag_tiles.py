"""The fixed-point digit tiles of the occupation-form diagonal, built on the
host (nqs_diag_tiles_host), against the diagonal's definition.

The finish kernel evaluates the X = 0 group of a JW molecular table as
d0 + sum_{i <= j} n_i n_j U[j][i] on the matrix cores, from U stored as
fixed point in four base-2^15 digits, each held as two int8 byte planes
(E = a - 128 b).  Here, on the CPU:
  * the planes decode (digit l weighs 2^(15 l); plane a once, plane b
    times -128) to integers Q with |Q| < 2^59, and Q * scale is U rounded to
    the grid, where U is rewritten in this test from the Z strings
    (c Z_i = c (1 - 2 n_i), c Z_i Z_j = c (1 - 2 n_i)(1 - 2 n_j)); zero above
    the diagonal and outside the register; the grid is the finest that
    keeps |Q| below 2^59; every digit lies in [-2^14, 2^14] (so that the
    kernel's 32-bit sums cannot overflow);
  * the exact integer sum over the occupied pairs, scaled once, equals the
    Z-string sum sum_t c_t (-1)^{popc(Z_t & x)} of the X = 0 terms (the
    definition, no rewrite) within 1e-13 of D = sum_t |c_t|.
Tables: the 12-qubit molecule, and diagonal-only tables of random one- and
two-qubit Z strings at 40, 100 and 127 qubits (one and two k-blocks, the
largest register).
"""
import math

import numpy as np
import pytest

import paper_2506_23809_amd as nqs
import workloads as W

DIGITS = 4
PLANES = 2 * DIGITS
GRID_BITS = 59


def _tile_order(jtiles):
    """(jt, kb) of each stored tile, in storage order."""
    return [(jt, kb) for jt in range(jtiles) for kb in range(1 if jt < 4 else 2)]


def _decode(tiles, nq):
    """Q[j][i] (Python ints) from the digit tiles; also checks the plane and
    digit ranges and that every stored entry outside i <= j < nq is zero."""
    jtiles = (nq + 15) // 16
    order = _tile_order(jtiles)
    assert tiles.size == len(order) * PLANES * 64 * 16
    t = tiles.reshape(len(order), DIGITS, 2, 64, 16).astype(np.int64)
    assert t.min() >= -128 and t.max() <= 127
    digits = t[:, :, 0] - 128 * t[:, :, 1]
    assert np.abs(digits).max() <= 2 ** 14
    weights = np.array([2 ** (15 * l) for l in range(DIGITS)], dtype=object)
    Q = {}
    for k, (jt, kb) in enumerate(order):
        for L in range(64):
            for b in range(16):
                j, i = 16 * jt + L % 16, 64 * kb + 16 * (L // 16) + b
                q = int(np.dot(digits[k, :, L, b].astype(object), weights))
                if i > j or j >= nq:
                    assert q == 0, (j, i)
                else:
                    Q[(j, i)] = q
    return Q


def _occupation_form(nq, x, z, c):
    """d0 and U[(j, i)] (i <= j) from the X = 0 group's Z strings."""
    d0 = 0.0
    U = {}
    diag = (x[:, 0] == 0) & (x[:, 1] == 0)
    zb = W.unpack_bits(z[diag], nq)
    for row, ct in zip(zb, c[diag]):
        q = np.nonzero(row)[0]
        assert len(q) <= 2
        d0 += ct
        for i in q:
            U[(i, i)] = U.get((i, i), 0.0) - 2.0 * ct
        if len(q) == 2:
            i, j = sorted(q)
            U[(j, i)] = U.get((j, i), 0.0) + 4.0 * ct
    return d0, U


def _z_string_sum(nq, x, z, c, samples):
    """The definition: sum over the X = 0 terms of c_t (-1)^{popc(Z_t & x)}."""
    diag = (x[:, 0] == 0) & (x[:, 1] == 0)
    zd, cd = z[diag], c[diag]
    out = []
    for s in samples:
        par = (np.bitwise_count(zd[:, 0] & s[0]) + np.bitwise_count(zd[:, 1] & s[1])) & 1
        out.append(math.fsum(np.where(par == 1, -cd, cd)))
    return np.array(out), float(np.sum(np.abs(cd)))


def _diag_only_table(nq, seed):
    """Identity, every Z_i and every Z_i Z_j with random coefficients."""
    rng = np.random.default_rng([77, nq, seed])
    zrows = [np.zeros(nq, bool)]
    for i in range(nq):
        r = np.zeros(nq, bool)
        r[i] = True
        zrows.append(r)
    for i in range(nq):
        for j in range(i + 1, nq):
            r = np.zeros(nq, bool)
            r[[i, j]] = True
            zrows.append(r)
    z = W.pack_bits(np.array(zrows))
    x = np.zeros_like(z)
    c = rng.normal(0.0, 1.0, len(zrows)) * np.exp(rng.uniform(-3, 3, len(zrows)))
    return x, z, c


def _cases():
    yield "nq12-molecule", 12
    for nq in (40, 100, 127):
        yield f"diag-{nq}", nq


@pytest.mark.parametrize("name,nq", list(_cases()))
def test_digit_tiles_decode_to_the_occupation_form(name, nq):
    if name.startswith("nq12"):
        w = W.workload("nq12")
        x, z, c, sm = w.x, w.z, w.c, w.spin_masks
    else:
        x, z, c = _diag_only_table(nq, 0)
        sm = None
    tiles, d0, scale = nqs.diag_tiles_host(nq, x, z, c, sm)
    d0_ref, U = _occupation_form(nq, x, z, c)
    assert abs(d0 - d0_ref) <= 1e-12 * max(1.0, abs(d0_ref))
    Q = _decode(tiles, nq)
    maxq = max(abs(q) for q in Q.values())
    assert maxq < 2 ** GRID_BITS
    assert maxq >= 2 ** (GRID_BITS - 1)  # the finest grid that fits
    # every entry is U on the grid, rounded to nearest (U rewritten in FP64
    # here in another order: allow a few ulps of U beside the half step)
    for (j, i), q in Q.items():
        u = U.get((j, i), 0.0)
        assert abs(q * scale - u) <= 0.5 * scale + 4 * np.spacing(abs(u)) + 1e-300, (j, i)


@pytest.mark.parametrize("name,nq", list(_cases()))
def test_exact_digit_sum_equals_the_z_string_sum(name, nq):
    if name.startswith("nq12"):
        w = W.workload("nq12")
        x, z, c, sm = w.x, w.z, w.c, w.spin_masks
        samples = w.samples
    else:
        x, z, c = _diag_only_table(nq, 1)
        sm = None
        rng = np.random.default_rng([78, nq])
        bits = rng.random((64, nq)) < rng.uniform(0.1, 0.9, (64, 1))
        bits[0] = False          # the empty register
        bits[1] = True           # the full register
        samples = W.pack_bits(bits)
    tiles, d0, scale = nqs.diag_tiles_host(nq, x, z, c, sm)
    Q = _decode(tiles, nq)
    want, D = _z_string_sum(nq, x, z, c, samples)
    occ = W.unpack_bits(samples, nq)
    for s, row, ref in zip(samples, occ, want):
        on = np.nonzero(row)[0]
        total = 0
        for a, j in enumerate(on):
            for i in on[:a + 1]:
                total += Q.get((int(j), int(i)), 0)
        got = d0 + float(total) * scale
        assert abs(got - ref) <= 1e-13 * D, (got, ref, D)


def test_tables_without_the_form_have_no_tiles():
    """A Z string on three qubits keeps the term form: no tiles."""
    nq = 10
    zb = np.zeros((2, nq), bool)
    zb[0, [1, 4, 7]] = True
    zb[1, 2] = True
    z = W.pack_bits(zb)
    x = np.zeros_like(z)
    tiles, d0, scale = nqs.diag_tiles_host(nq, x, z, np.array([0.5, -1.25]))
    assert tiles.size == 0
