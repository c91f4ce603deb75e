"""Literal values of the phase families at points where sin and cos are exact.

Each expected value below is worked out by hand from the family's formula
(the c1/c2 ellipse of the batched workloads, the radial family
rho(x)|xi|, the ellipse phase of eq. (nrphase) with r1, r2 of Section 4, and
the circles of eq. (circlerad)) at x where sin(2 pi x) and cos(2 pi x) take
the values 0 and +-1, and at integer frequencies.  They pin the two oracle
implementations of h (the C one in oracle/direct.c and the NumPy one in
oracle/reference.py) independently of each other, so that a misreading
shared by both (a 9 for a 16, sin for cos, 2 pi for 4 pi, xi1 for xi2)
fails here.  The direct sum itself is pinned through a one-frequency input:
u(x) = exp(2 pi i (x.xi0 + h(x, xi0))) / N (eq. (dfio)).
"""
import math

import numpy as np
import pytest

from oracle import direct as od
from oracle import reference as ref

S145, S73, S45, S13 = math.sqrt(145.0), math.sqrt(73.0), math.sqrt(45.0), math.sqrt(13.0)

# (kind, params, x1, x2, xi1, xi2, h by hand)
CASES = [
    # linear: h = p0 xi1 + p1 xi2
    (0, [0.25, -0.5], 0.3, 0.7, 3, 4, 0.25 * 3 - 0.5 * 4),
    # wave: h = p0 |xi|, |(3, 4)| = 5
    (1, [0.05], 0.3, 0.7, 3, 4, 0.25),
    (1, [-0.08], 0.1, 0.2, -3, 4, -0.4),
    # c1/c2 ellipse, c1 = (2 + sin 2pi x1 sin 2pi x2)/16, c2 = (2 + cos 2pi x1 cos 2pi x2)/16
    #   x = (1/4, 1/4): c1 = 3/16, c2 = 2/16 -> sqrt((9/16)^2 + (8/16)^2) = sqrt(145)/16
    (2, [1.0], 0.25, 0.25, 3, 4, S145 / 16),
    #   same x, xi swapped: sqrt((3/16 * 4)^2 + (1/8 * 3)^2) = sqrt(144 + 36)/16
    (2, [1.0], 0.25, 0.25, 4, 3, math.sqrt(180.0) / 16),
    #   x = (1/4, 3/4): c1 = 1/16, c2 = 2/16 -> sqrt((3/16)^2 + (8/16)^2) = sqrt(73)/16
    (2, [1.0], 0.25, 0.75, 3, 4, S73 / 16),
    #   x = (0, 0): c1 = 2/16, c2 = 3/16 -> sqrt((6/16)^2 + (12/16)^2) = sqrt(45)/8
    (2, [1.0], 0.0, 0.0, 3, 4, S45 / 8),
    #   x = (1/2, 0): c1 = 2/16, c2 = 1/16 -> sqrt((6/16)^2 + (4/16)^2) = sqrt(13)/8
    (2, [1.0], 0.5, 0.0, 3, 4, S13 / 8),
    #   phase scale p0 multiplies h; a pure xi1 frequency gives p0 c1 |xi1|
    (2, [1.5], 0.25, 0.25, -7, 0, 1.5 * 7 * 3 / 16),
    (2, [0.5], 0.0, 0.0, 0, 7, 0.5 * 7 * 3 / 16),
    # radial: rho = p0 (1 + p1 sin 2pi x1), depends on x1 only
    (3, [0.05, 0.5], 0.25, 0.0, 3, 4, 0.075 * 5),
    (3, [0.05, 0.5], 0.75, 0.25, 3, 4, 0.025 * 5),
    (3, [0.05, 0.5], 0.0, 0.25, 3, 4, 0.05 * 5),
    # paper ellipse (eq. (nrphase)): r1 = (2+sin 4pi x1)(2+sin 4pi x2)/9, r2 = (2+cos 4pi x1)(2+cos 4pi x2)/9
    #   x = (1/8, 1/8): r1 = 1, r2 = 4/9 -> sqrt(9 + (16/9)^2) = sqrt(985)/9
    (4, [1.0], 0.125, 0.125, 3, 4, math.sqrt(985.0) / 9),
    #   x = (0, 0): r1 = 4/9, r2 = 1 -> sqrt((4/3)^2 + 16) = sqrt(160)/3
    (4, [1.0], 0.0, 0.0, 3, 4, math.sqrt(160.0) / 3),
    #   x = (3/8, 1/8): r1 = 1/3, r2 = 4/9 -> sqrt(1 + (16/9)^2) = sqrt(337)/9
    (4, [1.0], 0.375, 0.125, 3, 4, math.sqrt(337.0) / 9),
    #   x = (1/4, 0): r1 = 4/9, r2 = 1/3 -> sqrt((4/3)^2 + (4/3)^2) = 4 sqrt(2)/3
    (4, [1.0], 0.25, 0.0, 3, 4, 4 * math.sqrt(2.0) / 3),
    # paper circles (eq. (circlerad)): r = (3+sin 4pi x1)(3+sin 4pi x2)/16, h = p0 r |xi|
    (5, [1.0], 0.125, 0.125, 3, 4, 5.0),
    (5, [1.0], 0.375, 0.125, 3, 4, 2.5),
    (5, [1.0], 0.0, 0.0, 3, 4, 45.0 / 16),
    (5, [1.0], 0.375, 0.375, 3, 4, 1.25),
    (5, [2.0], 0.125, 0.375, -4, 3, 2.0 * 0.5 * 5),
]


@pytest.mark.parametrize("kind,p,x1,x2,k1,k2,expect", CASES)
def test_h_literal_values(kind, p, x1, x2, k1, k2, expect):
    hc = od.h_values(kind, p, [x1], [x2], [k1], [k2])[0]
    hn = float(ref.h(kind, p, np.array([x1]), np.array([x2]), np.array([k1]), np.array([k2]))[0])
    assert abs(hc - expect) < 1e-14 * max(1.0, abs(expect)), (hc, expect)
    assert abs(hn - expect) < 1e-14 * max(1.0, abs(expect)), (hn, expect)


# grad_xi h at exact points: for the ellipse families grad = p0 (a^2 xi1, b^2 xi2)/sqrt(a^2 xi1^2 + b^2 xi2^2)
GRAD_CASES = [
    # c1/c2 at x = (1/4, 1/4): a = 3/16, b = 1/8, xi = (3, 4), sqrt(...) = sqrt(145)/16
    (2, [1.0], 0.25, 0.25, 3, 4, (9 / 256 * 3) / (S145 / 16), (1 / 64 * 4) / (S145 / 16)),
    # paper ellipse at x = (1/8, 1/8): a = 1, b = 4/9, sqrt(...) = sqrt(985)/9
    (4, [1.0], 0.125, 0.125, 3, 4, 3 / (math.sqrt(985.0) / 9), (16 / 81 * 4) / (math.sqrt(985.0) / 9)),
    # circles at x = (3/8, 1/8): r = 1/2, grad = r xi/|xi|
    (5, [1.0], 0.375, 0.125, 3, 4, 0.5 * 3 / 5, 0.5 * 4 / 5),
    # radial at x1 = 1/4: rho = 0.075
    (3, [0.05, 0.5], 0.25, 0.6, -3, 4, -0.075 * 3 / 5, 0.075 * 4 / 5),
]


@pytest.mark.parametrize("kind,p,x1,x2,k1,k2,g1,g2", GRAD_CASES)
def test_grad_h_literal_values(kind, p, x1, x2, k1, k2, g1, g2):
    a1, a2 = ref.grad_h(kind, p, np.array([x1]), np.array([x2]), np.array([float(k1)]), np.array([float(k2)]))
    assert abs(float(a1[0]) - g1) < 1e-14 and abs(float(a2[0]) - g2) < 1e-14


@pytest.mark.parametrize("kind,p,x1,x2,k1,k2,expect", [c for c in CASES if c[0] >= 2])
def test_direct_sum_of_one_frequency(kind, p, x1, x2, k1, k2, expect):
    """fhat = delta at xi0 gives u(x) = exp(2 pi i (x.xi0 + h(x, xi0)))/N, with x.xi0 and h by hand."""
    N = 16
    n1, n2 = int(round(x1 * N)), int(round(x2 * N))
    assert abs(n1 / N - x1) < 1e-15 and abs(n2 / N - x2) < 1e-15
    fh = np.zeros((N, N), complex)
    fh[k1 + N // 2, k2 + N // 2] = 1.0
    u = od.direct(N, kind, p, fh, np.array([n1 * N + n2]))
    ph = (n1 * k1 + n2 * k2) / N + expect
    want = np.exp(2j * math.pi * (ph - round(ph))) / N
    assert abs(complex(np.ravel(u)[0]) - want) < 1e-13


@pytest.mark.parametrize("plant", [4, 5])
def test_planted_family_misreadings_are_caught(plant, tmp_path):
    """sin and cos exchanged in c1/c2, or 2 pi in place of 4 pi in r1/r2, fail the literal values."""
    path = od.build(force=True, plant=plant, out=str(tmp_path / ("plant%d.so" % plant)))
    lib = od._load(path)
    bad = 0
    for kind, p, x1, x2, k1, k2, expect in CASES:
        pa = od._params(p)
        arr = [np.ascontiguousarray(np.array([v], float)) for v in (x1, x2, k1, k2)]
        out = np.empty(1)
        lib.oracle_h_batch(kind, pa.ctypes.data, 1, arr[0].ctypes.data, arr[1].ctypes.data, arr[2].ctypes.data,
                           arr[3].ctypes.data, out.ctypes.data)
        bad += abs(out[0] - expect) > 1e-9
    assert bad > 0
