"""Oracle pins: spin-weight -2 spherical harmonics.

Pinned to the l = 2 closed forms, to orthonormality of all 21 modes with
l = 2..4 and of every mode with l = 5..8, the largest degree the library
accepts (quadrature on the sphere), to the addition theorem
sum_m |Y_lm|^2 = (2l+1)/4pi, and to the parity relation
Y_{l,-m}(iota, phi) = (-1)^l conj(Y_{l,m}(pi - iota, phi)).
"""
import math

import numpy as np
import pytest

import synth


def closed_l2(m, iota, phi):
    c, s = math.cos(iota), math.sin(iota)
    e = complex(math.cos(m * phi), math.sin(m * phi))
    if m == 2:
        r = math.sqrt(5 / (64 * math.pi)) * (1 + c) ** 2
    elif m == 1:
        r = math.sqrt(5 / (16 * math.pi)) * s * (1 + c)
    elif m == 0:
        r = math.sqrt(15 / (32 * math.pi)) * s * s
    elif m == -1:
        r = math.sqrt(5 / (16 * math.pi)) * s * (1 - c)
    else:
        r = math.sqrt(5 / (64 * math.pi)) * (1 - c) ** 2
    return r * e


def test_l2_closed_forms(orc):
    rng = np.random.default_rng(5)
    for _ in range(100):
        iota, phi = rng.uniform(0, math.pi), rng.uniform(0, 2 * math.pi)
        for m in range(-2, 3):
            assert abs(orc.sylm(2, m, iota, phi) - closed_l2(m, iota, phi)) < 1e-14


@pytest.mark.parametrize("ls", [(2, 3, 4), (5, 6, 7, 8)])
def test_orthonormal_and_addition(orc, ls):
    modes = synth.MODE_SETS[21] if ls == (2, 3, 4) else [(l, m) for l in ls for m in range(-l, l + 1)]
    xg, wg = np.polynomial.legendre.leggauss(60)   # in cos(iota)
    nphi = 64
    phis = 2 * math.pi * np.arange(nphi) / nphi
    Y = np.zeros((len(modes), len(xg), nphi), dtype=np.complex128)
    for a, (l, m) in enumerate(modes):
        for i, x in enumerate(xg):
            io = math.acos(x)
            for j, ph in enumerate(phis):
                Y[a, i, j] = orc.sylm(l, m, io, ph)
    G = np.einsum("aij,bij,i->ab", Y, Y.conj(), wg) * (2 * math.pi / nphi)
    assert np.abs(G - np.eye(len(modes))).max() < 1e-12
    for l in ls:
        idx = [a for a, (ll, _) in enumerate(modes) if ll == l]
        tot = (np.abs(Y[idx]) ** 2).sum(axis=0)
        assert np.abs(tot - (2 * l + 1) / (4 * math.pi)).max() < 1e-12


def test_parity(orc):
    rng = np.random.default_rng(6)
    for _ in range(50):
        iota, phi = rng.uniform(0, math.pi), rng.uniform(0, 2 * math.pi)
        for l, m in synth.MODE_SETS[21]:
            lhs = orc.sylm(l, -m, iota, phi)
            rhs = (-1) ** l * orc.sylm(l, m, math.pi - iota, phi).conjugate()
            assert abs(lhs - rhs) < 1e-14
