"""Pins of the oracle's ray directions (Sec. III-E, Eq. 10) against closed forms."""
import json
import math
import os
from fractions import Fraction

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "halton_prefix.json")


def test_radical_inverse_closed_forms():
    g = json.load(open(GOLDEN))
    for i, (p, q) in enumerate(g["H2"]):
        assert oracle.radical_inverse(i, 2) == p / q            # dyadic: exact in float64
    for i, (p, q) in enumerate(g["H3"]):
        assert abs(oracle.radical_inverse(i, 3) - p / q) <= 2 ** -52


def test_radical_inverse_is_digit_mirror():
    # H_b(i) = sum_k digit_k(i) b^-(k+1), checked with exact rationals for many i
    for base in (2, 3):
        for i in list(range(0, 2000)) + [65535, 59049, 12345]:
            j, k, exact = i, 1, Fraction(0)
            while j:
                exact += Fraction(j % base, base ** k)
                j //= base
                k += 1
            assert abs(oracle.radical_inverse(i, base) - float(exact)) <= 4 * 2 ** -53


def test_first_directions_closed_forms():
    r = oracle.directions(5).astype(np.float64)
    s3 = math.sqrt(3.0)
    exp = np.array([
        [0.0, 0.0, 1.0],
        [-0.5, s3 / 2, 0.0],
        [-s3 / 4, -0.75, 0.5],
        [(s3 / 2) * math.cos(2 * math.pi / 9), (s3 / 2) * math.sin(2 * math.pi / 9), -0.5],
        [(math.sqrt(7) / 4) * math.cos(8 * math.pi / 9), (math.sqrt(7) / 4) * math.sin(8 * math.pi / 9), 0.75],
    ])
    assert np.all(np.abs(r - exp) <= np.abs(exp) * 2 ** -24 + 1e-300)
    assert r[0].tolist() == [0.0, 0.0, 1.0]
    assert r[1, 2] == 0.0


def test_directions_match_printed_acos_form():
    # The oracle uses sin(acos z) = sqrt(1 - z^2); the printed form evaluates acos, sin, cos.
    n = 4096
    r = oracle.directions(n).astype(np.float64)
    u = np.array([oracle.radical_inverse(i, 2) for i in range(n)])
    w = np.array([oracle.radical_inverse(i, 3) for i in range(n)])
    phi = np.arccos(1 - 2 * u)
    th = 2 * np.pi * w
    ref = np.stack([np.sin(phi) * np.cos(th), np.sin(phi) * np.sin(th), np.cos(phi)], -1)
    # within one float32 rounding plus float64 noise of the acos route
    assert np.max(np.abs(r - ref)) <= 2 ** -24 + 1e-12


def test_polar_coordinate_is_equal_area_prefix():
    # For N = 2^k the first N base-2 radical inverses are exactly {j / N}: z = 1 - 2u hits
    # N equally spaced levels, so sum z over the prefix is exactly 1 (mean 2^-k).
    for k in range(1, 17):
        n = 2 ** k
        z = oracle.directions(n)[:, 2].astype(np.float64)
        assert math.fsum(z) == 1.0
        u = np.sort((1 - z) / 2)
        assert np.array_equal(u, np.arange(n) / n)


def test_directions_unit_norm_and_prefix_property():
    full = oracle.directions(65536)
    assert np.array_equal(oracle.directions(1000), full[:1000])
    nrm = np.linalg.norm(full.astype(np.float64), axis=1)
    assert np.max(np.abs(nrm - 1.0)) < 2e-7
