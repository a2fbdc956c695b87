"""Oracle pins: antenna patterns, arrival delays, Catmull-Rom weights.

The antenna pattern is pinned to the textbook closed form for an L-shaped
detector at the north pole with arms along x and y; the tensor form with
the basis convention of the oracle equals minus the textbook form evaluated
at -psi (a polarization-angle convention difference, F(psi + pi/2) = -F(psi)).
"""
import math

import numpy as np
import pytest

import synth

POLE_D = 0.5 * (np.diag([1.0, 0, 0]) - np.diag([0, 1.0, 0]))


def textbook(theta, phi, psi):
    c = math.cos(theta)
    fp = 0.5 * (1 + c * c) * math.cos(2 * phi) * math.cos(2 * psi) - c * math.sin(2 * phi) * math.sin(2 * psi)
    fc = 0.5 * (1 + c * c) * math.cos(2 * phi) * math.sin(2 * psi) + c * math.sin(2 * phi) * math.cos(2 * psi)
    return fp, fc


def test_antenna_matches_closed_form(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        alpha, gmst = rng.uniform(0, 2 * math.pi, 2)
        delta = math.asin(rng.uniform(-1, 1))
        psi = rng.uniform(0, math.pi)
        fp, fc = orc.antenna(POLE_D, alpha, delta, psi, gmst)
        theta = math.pi / 2 - delta
        phi = alpha - gmst
        tp, tc = textbook(theta, phi, -psi)
        assert fp == pytest.approx(-tp, abs=1e-14)
        assert fc == pytest.approx(-tc, abs=1e-14)


def test_antenna_bounds_and_psi_rotation(orc):
    rng = np.random.default_rng(2)
    pos, resp = synth.detector_arrays(["H1", "L1", "V1"])
    for _ in range(100):
        alpha, gmst, psi = rng.uniform(0, 2 * math.pi, 3)
        delta = math.asin(rng.uniform(-1, 1))
        for D in list(resp) + [POLE_D]:
            fp, fc = orc.antenna(D, alpha, delta, psi, gmst)
            assert fp * fp + fc * fc <= 1 + 1e-12
            gp, gc = orc.antenna(D, alpha, delta, psi + math.pi / 2, gmst)
            assert gp == pytest.approx(-fp, abs=1e-14) and gc == pytest.approx(-fc, abs=1e-14)
            hp, hc = orc.antenna(D, alpha, delta, psi + math.pi, gmst)
            assert hp == pytest.approx(fp, abs=1e-14) and hc == pytest.approx(fc, abs=1e-14)
    # overhead source for the polar detector: |F| = 1
    fp, fc = orc.antenna(POLE_D, 0.3, math.pi / 2, 0.7, 0.3)
    assert fp * fp + fc * fc == pytest.approx(1.0, abs=1e-14)


def test_detector_arms_orthonormal():
    for name, d in synth.DETECTORS.items():
        x, y = np.array(d["xarm"]), np.array(d["yarm"])
        assert np.linalg.norm(x) == pytest.approx(1, abs=1e-9)
        assert np.linalg.norm(y) == pytest.approx(1, abs=1e-9)
        assert abs(x @ y) < 1e-6  # surveyed arms are orthogonal to the published digits
        # vertex on the Earth's surface
        assert 6.35e6 < np.linalg.norm(d["vertex"]) < 6.39e6


def test_delays(orc):
    pos, _ = synth.detector_arrays(["H1", "L1", "V1"])
    gmst = 1.234
    for r in pos:
        # source straight above the detector: the wave arrives |r|/c early
        n = r / np.linalg.norm(r)
        delta = math.asin(n[2])
        alpha = math.atan2(n[1], n[0]) + gmst
        assert orc.delay(r, alpha, delta, gmst) == pytest.approx(-np.linalg.norm(r) / synth.C_SI, abs=1e-15)
        assert np.allclose(orc.direction(alpha, delta, gmst), n, atol=1e-15)
    # the H1-L1 delay difference peaks at the light travel time along the baseline
    b = pos[0] - pos[1]
    n = -b / np.linalg.norm(b)
    delta = math.asin(n[2]); alpha = math.atan2(n[1], n[0]) + gmst
    d = orc.delay(pos[0], alpha, delta, gmst) - orc.delay(pos[1], alpha, delta, gmst)
    assert d == pytest.approx(np.linalg.norm(b) / synth.C_SI, abs=1e-15)
    assert 0.0099 < d < 0.0101
    rng = np.random.default_rng(3)
    for _ in range(500):
        a = rng.uniform(0, 2 * math.pi); de = math.asin(rng.uniform(-1, 1))
        dd = orc.delay(pos[0], a, de, gmst) - orc.delay(pos[1], a, de, gmst)
        assert abs(dd) <= d + 1e-15


def test_catmull_rom_weights(orc):
    # interpolates at knots, reproduces quadratics exactly, C1 across knots
    w, dw = orc.catmull_rom(0.0)
    assert np.allclose(w, [0, 1, 0, 0], atol=0)
    rng = np.random.default_rng(4)
    for mu in rng.uniform(0, 1, 50):
        w, dw = orc.catmull_rom(mu)
        assert w.sum() == pytest.approx(1.0, abs=1e-15)
        assert dw.sum() == pytest.approx(0.0, abs=1e-15)
        c0, c1, c2 = rng.standard_normal(3)
        f = lambda x: c0 + c1 * x + c2 * x * x
        xs = np.array([-1.0, 0.0, 1.0, 2.0])
        assert w @ f(xs) == pytest.approx(f(mu), abs=1e-13)
        assert dw @ f(xs) == pytest.approx(c1 + 2 * c2 * mu, abs=1e-13)
    # value and slope continuous across a knot: mu -> 1 from below equals mu = 0 shifted by one row
    vals = rng.standard_normal(6)
    w1, d1 = orc.catmull_rom(1.0)
    w0, d0 = orc.catmull_rom(0.0)
    assert w1 @ vals[0:4] == pytest.approx(w0 @ vals[1:5], abs=1e-15)
    assert d1 @ vals[0:4] == pytest.approx(d0 @ vals[1:5], abs=1e-15)
