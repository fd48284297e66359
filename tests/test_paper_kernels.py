"""Pin the oracle's collisions to the cascaded kernels printed in the paper.

The oracle computes every collision from the plain rule "relax each central
moment toward its equilibrium" (generic moments, a dense solve).  The paper
prints the closed-form result of its cascade:
  * flow, D3Q15: kernel g^ of Appendix A and its post-collision expansion;
  * thermal, D3Q15: kernel h^ of Sec. 2.2 and its post-collision expansion;
  * thermal, D3Q7: kernel h^ of Appendix C and its post-collision expansion.
Those printed formulas are transcribed below (with and without the scalar
source R, whose populations are the printed inverse tables of Appendix B and
C) and evaluated on seeded random inputs; the two must agree to rounding.  A dropped term, a
wrong sign, a wrong rate index or a transposed moment anywhere in the oracle's
generic machinery breaks the agreement.

Readings applied to the printed text (each also in the design notes):
  * Appendix C lists the first kernel component twice as h1; the first is h0 = 0.
  * Appendix C's source: S_3 and S_4 use m^s_2 (printed m^s_1), and
    m^s_6 = (7 (ux^2 + uy^2 + uz^2) - 6) R (printed 7 ux^2 + uy^2 + uz^2).
  * eq. (21): the source's raw moments inside eta' are the lattice sums of
    the source populations S^phi.
  * Appendix A: the kinematic-viscosity rates are omega_4..omega_9 (the text
    says 5..9).  Here every rate is drawn independently anyway.
  * Appendix A, g14: the 4th-order equilibrium is kxx~ kyy~ / rho, with kxx~,
    kyy~ the post-collision second-order central moments.
  * The flow source S (deferred by the paper to its earlier flow paper) has
    central moments (0; F; 0 ... 0), so its raw moment of a monomial p is
    grad p(u) . F.
"""
import numpy as np
import pytest

# D3Q15 velocities, Sec. 2.2 eq. (5)
EX15 = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1])
EY15 = np.array([0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1])
EZ15 = np.array([0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1])
# D3Q7 velocities, Appendix C
EX7 = np.array([0, 1, -1, 0, 0, 0, 0])
EY7 = np.array([0, 0, 0, 1, -1, 0, 0])
EZ7 = np.array([0, 0, 0, 0, 0, 1, -1])

# Post-collision expansions (K h^)_alpha as printed: row alpha, column k.
_POST15 = """
0: 0:1 9:-2 14:32
1: 0:1 1:1 7:1 8:1 9:-1 10:-8 14:-8
2: 0:1 1:-1 7:1 8:1 9:-1 10:8 14:-8
3: 0:1 2:1 7:-1 8:1 9:-1 11:-8 14:-8
4: 0:1 2:-1 7:-1 8:1 9:-1 11:8 14:-8
5: 0:1 3:1 8:-2 9:-1 12:-8 14:-8
6: 0:1 3:-1 8:-2 9:-1 12:8 14:-8
7: 0:1 1:1 2:1 3:1 4:1 5:1 6:1 9:1 10:2 11:2 12:2 13:1 14:2
8: 0:1 1:-1 2:1 3:1 4:-1 5:-1 6:1 9:1 10:-2 11:2 12:2 13:-1 14:2
9: 0:1 1:1 2:-1 3:1 4:-1 5:1 6:-1 9:1 10:2 11:-2 12:2 13:-1 14:2
10: 0:1 1:-1 2:-1 3:1 4:1 5:-1 6:-1 9:1 10:-2 11:-2 12:2 13:1 14:2
11: 0:1 1:1 2:1 3:-1 4:1 5:-1 6:-1 9:1 10:2 11:2 12:-2 13:-1 14:2
12: 0:1 1:-1 2:1 3:-1 4:-1 5:1 6:-1 9:1 10:-2 11:2 12:-2 13:1 14:2
13: 0:1 1:1 2:-1 3:-1 4:-1 5:-1 6:1 9:1 10:2 11:-2 12:-2 13:1 14:2
14: 0:1 1:-1 2:-1 3:-1 4:1 5:1 6:1 9:1 10:-2 11:-2 12:-2 13:-1 14:2
"""
_POST7 = """
0: 0:1 6:-6
1: 0:1 1:1 4:1 5:1 6:1
2: 0:1 1:-1 4:1 5:1 6:1
3: 0:1 2:1 4:-1 5:1 6:1
4: 0:1 2:-1 4:-1 5:1 6:1
5: 0:1 3:1 5:-2 6:1
6: 0:1 3:-1 5:-2 6:1
"""


def _table(text, q):
    K = np.zeros((q, q))
    for line in text.strip().splitlines():
        row, rest = line.split(":", 1)
        for tok in rest.split():
            k, v = tok.split(":")
            K[int(row), int(k)] = float(v)
    return K


POST15 = _table(_POST15, 15)
POST7 = _table(_POST7, 7)

# Source populations as printed: S_alpha = (sum_k c_k m^s_k) / d.
# Appendix B (D3Q15): "alpha: d | k:c ...".
_SRC15 = """
0: 45 | 0:3 9:-5 14:1
1: 180 | 0:12 1:18 7:45 8:15 9:-10 10:-9 14:-1
2: 180 | 0:12 1:-18 7:45 8:15 9:-10 10:9 14:-1
3: 180 | 0:12 2:18 7:-45 8:15 9:-10 11:-9 14:-1
4: 180 | 0:12 2:-18 7:-45 8:15 9:-10 11:9 14:-1
5: 180 | 0:12 3:18 8:-30 9:-10 12:-9 14:-1
6: 180 | 0:12 3:-18 8:-30 9:-10 12:9 14:-1
7: 720 | 0:48 1:72 2:72 3:72 4:90 5:90 6:90 9:40 10:9 11:9 12:9 13:90 14:1
8: 720 | 0:48 1:-72 2:72 3:72 4:-90 5:-90 6:90 9:40 10:-9 11:9 12:9 13:-90 14:1
9: 720 | 0:48 1:72 2:-72 3:72 4:-90 5:90 6:-90 9:40 10:9 11:-9 12:9 13:-90 14:1
10: 720 | 0:48 1:-72 2:-72 3:72 4:90 5:-90 6:-90 9:40 10:-9 11:-9 12:9 13:90 14:1
11: 720 | 0:48 1:72 2:72 3:-72 4:90 5:-90 6:-90 9:40 10:9 11:9 12:-9 13:-90 14:1
12: 720 | 0:48 1:-72 2:72 3:-72 4:-90 5:90 6:-90 9:40 10:-9 11:9 12:-9 13:90 14:1
13: 720 | 0:48 1:72 2:-72 3:-72 4:-90 5:-90 6:90 9:40 10:9 11:-9 12:-9 13:90 14:1
14: 720 | 0:48 1:-72 2:-72 3:-72 4:90 5:90 6:90 9:40 10:-9 11:-9 12:-9 13:-90 14:1
"""
# Appendix C (D3Q7), with S_3, S_4 on m^s_2 (reading).
_SRC7 = """
0: 7 | 0:1 6:-1
1: 84 | 0:12 1:42 4:21 5:7 6:2
2: 84 | 0:12 1:-42 4:21 5:7 6:2
3: 84 | 0:12 2:42 4:-21 5:7 6:2
4: 84 | 0:12 2:-42 4:-21 5:7 6:2
5: 42 | 0:6 3:21 5:-7 6:1
6: 42 | 0:6 3:-21 5:-7 6:1
"""


def _src_table(text, q):
    A = np.zeros((q, q))
    for line in text.strip().splitlines():
        row, rest = line.split(":", 1)
        d, terms = rest.split("|")
        for tok in terms.split():
            k, v = tok.split(":")
            A[int(row), int(k)] = float(v) / float(d)
    return A


SRC15 = _src_table(_SRC15, 15)
SRC7 = _src_table(_SRC7, 7)


def source_moments15(R, u):
    """Projections m^s of the scalar source on K, eq. (19), as printed."""
    ux, uy, uz = u
    q2 = ux * ux + uy * uy + uz * uz
    return np.array([
        R, ux * R, uy * R, uz * R, ux * uy * R, ux * uz * R, uy * uz * R, (ux ** 2 - uy ** 2) * R,
        (ux ** 2 + uy ** 2 - 2 * uz ** 2) * R, (q2 - 2) * R,
        5 * (ux ** 3 + ux * uy ** 2 + ux * uz ** 2) * R - 13 * ux * R,
        5 * (ux ** 2 * uy + uy ** 3 + uy * uz ** 2) * R - 13 * uy * R,
        5 * (ux ** 2 * uz + uy ** 2 * uz + uz ** 3) * R - 13 * uz * R,
        ux * uy * uz * R,
        30 * (ux ** 2 * uy ** 2 + ux ** 2 * uz ** 2 + uy ** 2 * uz ** 2) * R - 40 * q2 * R + 32 * R])


def source_moments7(R, u):
    """Projections m^s of Appendix C (last one read as 7 (u.u) - 6)."""
    ux, uy, uz = u
    q2 = ux * ux + uy * uy + uz * uz
    return np.array([R, ux * R, uy * R, uz * R, (ux ** 2 - uy ** 2) * R,
                     (ux ** 2 + uy ** 2 - 2 * uz ** 2) * R, (7 * q2 - 6) * R])


def _kvec15():
    """The orthogonal basis K_0..K_14 of Sec. 2.2 evaluated on D3Q15."""
    x, y, z = EX15, EY15, EZ15
    e2 = x * x + y * y + z * z
    one = np.ones(15)
    return np.stack([
        one, x, y, z, x * y, x * z, y * z, x * x - y * y, e2 - 3 * z * z, e2 - 2 * one,
        5 * x * e2 - 13 * x, 5 * y * e2 - 13 * y, 5 * z * e2 - 13 * z, x * y * z,
        30 * (x * x * y * y + x * x * z * z + y * y * z * z) - 40 * e2 + 32 * one,
    ], axis=1).astype(float)


def _kvec7():
    """The orthogonal basis K_0..K_6 of Appendix C evaluated on D3Q7."""
    x, y, z = EX7, EY7, EZ7
    one = np.ones(7)
    return np.stack([one, x, y, z, x * x - y * y, 2 * (x * x - z * z) - (x * x - y * y),
                     7 * (x * x + y * y + z * z) - 6 * one], axis=1).astype(float)


def test_printed_expansions_are_the_columns_of_K():
    """The printed post-collision tables equal K (Sec. 2.2, Appendix A, C)."""
    assert np.array_equal(POST15, _kvec15())
    assert np.array_equal(POST7, _kvec7())


def test_K_orthogonal_with_known_norms():
    K15 = _kvec15()
    G = K15.T @ K15
    assert np.array_equal(G, np.diag(np.diag(G)))
    assert list(np.diag(G)) == [15, 10, 10, 10, 8, 8, 8, 4, 12, 18, 160, 160, 160, 8, 1440]
    K7 = _kvec7()
    G7 = K7.T @ K7
    assert np.array_equal(G7, np.diag(np.diag(G7)))
    assert list(np.diag(G7)) == [7, 2, 2, 2, 4, 12, 42]


def _raw(f, ex, ey, ez):
    """Raw moments sum_a f_a e^m (eq. 17) keyed by monomial name."""
    r = {}
    names = {"0": (0, 0, 0), "x": (1, 0, 0), "y": (0, 1, 0), "z": (0, 0, 1),
             "xy": (1, 1, 0), "xz": (1, 0, 1), "yz": (0, 1, 1), "xx": (2, 0, 0),
             "yy": (0, 2, 0), "zz": (0, 0, 2), "xyy": (1, 2, 0), "xxy": (2, 1, 0),
             "xxz": (2, 0, 1), "xyz": (1, 1, 1), "xxyy": (2, 2, 0)}
    for k, (a, b, c) in names.items():
        r[k] = float(np.sum(f * ex ** a * ey ** b * ez ** c))
    return r


def paper_thermal15(gbar, u, cs2, w, R=0.0):
    """Sec. 2.2 kernel h^ and post-collision expansion (eq. 13a), source S^phi
    from Appendix B; eta' = kappa' + sigma' (eq. 21), phi = sum gbar + R/2."""
    ux, uy, uz = u
    S = SRC15 @ source_moments15(R, u)
    k = _raw(gbar, EX15, EY15, EZ15)
    sg = _raw(S, EX15, EY15, EZ15)
    n = {m: k[m] + sg[m] for m in k}
    phi = k["0"] + R / 2
    ph = phi + R / 2  # the (phi + R/2) of the printed kernel
    h = np.zeros(15)
    h[1] = w[1] / 10 * (phi * ux - k["x"] - ux * R / 2)
    h[2] = w[2] / 10 * (phi * uy - k["y"] - uy * R / 2)
    h[3] = w[3] / 10 * (phi * uz - k["z"] - uz * R / 2)
    h[4] = w[4] / 8 * (-n["xy"] + uy * n["x"] + ux * n["y"] - ph * ux * uy) + 5 / 4 * (uy * h[1] + ux * h[2])
    h[5] = w[5] / 8 * (-n["xz"] + uz * n["x"] + ux * n["z"] - ph * ux * uz) + 5 / 4 * (uz * h[1] + ux * h[3])
    h[6] = w[6] / 8 * (-n["yz"] + uz * n["y"] + uy * n["z"] - ph * uy * uz) + 5 / 4 * (uz * h[2] + uy * h[3])
    h[7] = (w[7] / 4 * (-(n["xx"] - n["yy"]) + 2 * (ux * n["x"] - uy * n["y"]) - ph * (ux ** 2 - uy ** 2))
            + 5 * (ux * h[1] - uy * h[2]))
    h[8] = (w[8] / 12 * (-(n["xx"] + n["yy"] - 2 * n["zz"]) + 2 * (ux * n["x"] + uy * n["y"] - 2 * uz * n["z"])
                         - ph * (ux ** 2 + uy ** 2 - 2 * uz ** 2))
            + 5 / 3 * (ux * h[1] + uy * h[2] - 2 * uz * h[3]))
    h[9] = (w[9] / 18 * (3 * cs2 * phi - (n["xx"] + n["yy"] + n["zz"]) + 2 * (ux * n["x"] + uy * n["y"] + uz * n["z"])
                         - ph * (ux ** 2 + uy ** 2 + uz ** 2))
            + 10 / 9 * (ux * h[1] + uy * h[2] + uz * h[3]))
    h[10] = (w[10] / 16 * (-n["xyy"] + 2 * uy * n["xy"] - uy ** 2 * n["x"] + ux * n["yy"] - 2 * ux * uy * n["y"]
                           + ph * ux * uy ** 2)
             - (5 / 8 * uy ** 2 + 1 / 2) * h[1] - 5 / 4 * ux * uy * h[2] + uy * h[4]
             + 1 / 8 * ux * (-h[7] + h[8] + 3 * h[9]))
    h[11] = (w[11] / 16 * (-n["xxy"] + 2 * ux * n["xy"] + uy * n["xx"] - ux ** 2 * n["y"] - 2 * ux * uy * n["x"]
                           + ph * ux ** 2 * uy)
             - 5 / 4 * ux * uy * h[1] - (5 / 8 * ux ** 2 + 1 / 2) * h[2] + ux * h[4]
             + 1 / 8 * uy * (h[7] + h[8] + 3 * h[9]))
    h[12] = (w[12] / 16 * (-n["xxz"] + 2 * ux * n["xz"] + uz * n["xx"] - 2 * ux * uz * n["x"] - ux ** 2 * n["z"]
                           + ph * ux ** 2 * uz)
             - 5 / 4 * ux * uz * h[1] - (5 / 8 * ux ** 2 + 1 / 2) * h[3] + ux * h[5]
             + 1 / 8 * uz * (h[7] + h[8] + 3 * h[9]))
    h[13] = (w[13] / 8 * (-n["xyz"] + ux * n["yz"] + uy * n["xz"] + uz * n["xy"] - uy * uz * n["x"]
                          - ux * uz * n["y"] - ux * uy * n["z"] + ph * ux * uy * uz)
             - 5 / 4 * (uy * uz * h[1] + ux * uz * h[2] + ux * uy * h[3]) + uz * h[4] + uy * h[5] + ux * h[6])
    h[14] = (w[14] / 16 * (-n["xxyy"] + 2 * uy * n["xxy"] + 2 * ux * n["xyy"] - uy ** 2 * n["xx"]
                           - ux ** 2 * n["yy"] - 4 * ux * uy * n["xy"] + 2 * ux * uy ** 2 * n["x"]
                           + 2 * ux ** 2 * uy * n["y"] + cs2 ** 2 * phi - ph * ux ** 2 * uy ** 2)
             + 5 / 4 * (ux * uy ** 2 * h[1] + ux ** 2 * uy * h[2]) - 2 * ux * uy * h[4]
             + 1 / 8 * (ux ** 2 - uy ** 2) * h[7] - 1 / 8 * (ux ** 2 + uy ** 2) * h[8]
             - (3 / 8 * (ux ** 2 + uy ** 2) + 1 / 2) * h[9] + 2 * (ux * h[10] + uy * h[11])
             + uy * h[2] + ux * h[1])
    return gbar + POST15 @ h + S


def paper_thermal7(gbar, u, cs2, w, R=0.0):
    """Appendix C kernel h^ and post-collision expansion, with its source
    S^phi; eta' = kappa' + sigma' (eq. 21), phi = sum gbar + R/2."""
    ux, uy, uz = u
    S = SRC7 @ source_moments7(R, u)
    k = _raw(gbar, EX7, EY7, EZ7)
    sg = _raw(S, EX7, EY7, EZ7)
    n = {m: k[m] + sg[m] for m in k}
    phi = k["0"] + R / 2
    ph = phi + R / 2
    h = np.zeros(7)
    h[1] = w[1] / 2 * (phi * ux - k["x"] - ux * R / 2)
    h[2] = w[2] / 2 * (phi * uy - k["y"] - uy * R / 2)
    h[3] = w[3] / 2 * (phi * uz - k["z"] - uz * R / 2)
    h[4] = (w[4] / 4 * (-(n["xx"] - n["yy"]) + 2 * (ux * n["x"] - uy * n["y"]) - ph * (ux ** 2 - uy ** 2))
            + ux * h[1] - uy * h[2])
    h[5] = (w[5] / 12 * (-(n["xx"] + n["yy"] - 2 * n["zz"]) + 2 * (ux * n["x"] + uy * n["y"] - 2 * uz * n["z"])
                         - ph * (ux ** 2 + uy ** 2 - 2 * uz ** 2))
            + 1 / 3 * (ux * h[1] + uy * h[2] - 2 * uz * h[3]))
    h[6] = (w[6] / 6 * (3 * cs2 * phi - (n["xx"] + n["yy"] + n["zz"]) + 2 * (ux * n["x"] + uy * n["y"] + uz * n["z"])
                        - ph * (ux ** 2 + uy ** 2 + uz ** 2))
            + 2 / 3 * (ux * h[1] + uy * h[2] + uz * h[3]))
    return gbar + POST7 @ h + S


def _monomial_matrix():
    x, y, z = EX15, EY15, EZ15
    return np.stack([np.ones(15), x, y, z, x * y, x * z, y * z, x * x, y * y, z * z,
                     x * y * y, x * x * y, x * x * z, x * y * z, x * x * y * y]).astype(float)


def paper_flow(fbar, F, w, literal_g14=False):
    """Appendix A kernel g^ and post-collision expansion, with the source S
    whose raw moment of each monomial p is grad p(u) . F.  literal_g14 uses
    the product kxx~ kyy~ exactly as printed (no 1/rho)."""
    Fx, Fy, Fz = F
    rho = fbar.sum()
    ux = (np.dot(fbar, EX15) + Fx / 2) / rho
    uy = (np.dot(fbar, EY15) + Fy / 2) / rho
    uz = (np.dot(fbar, EZ15) + Fz / 2) / rho
    sig = {
        "0": 0.0, "x": Fx, "y": Fy, "z": Fz,
        "xy": uy * Fx + ux * Fy, "xz": uz * Fx + ux * Fz, "yz": uz * Fy + uy * Fz,
        "xx": 2 * ux * Fx, "yy": 2 * uy * Fy, "zz": 2 * uz * Fz,
        "xyy": uy ** 2 * Fx + 2 * ux * uy * Fy, "xxy": 2 * ux * uy * Fx + ux ** 2 * Fy,
        "xxz": 2 * ux * uz * Fx + ux ** 2 * Fz,
        "xyz": uy * uz * Fx + ux * uz * Fy + ux * uy * Fz,
        "xxyy": 2 * ux * uy ** 2 * Fx + 2 * ux ** 2 * uy * Fy,
    }
    order = ["0", "x", "y", "z", "xy", "xz", "yz", "xx", "yy", "zz", "xyy", "xxy", "xxz", "xyz", "xxyy"]
    S = np.linalg.solve(_monomial_matrix(), np.array([sig[k] for k in order]))
    kb = _raw(fbar, EX15, EY15, EZ15)
    n = {k: kb[k] + sig[k] for k in order}  # eta' = kappa_bar' + sigma'
    sx, sy, sz = Fx, Fy, Fz
    g = np.zeros(15)
    g[4] = w[4] / 8 * (-n["xy"] + rho * ux * uy + 0.5 * (sx * uy + sy * ux))
    g[5] = w[5] / 8 * (-n["xz"] + rho * ux * uz + 0.5 * (sx * uz + sz * ux))
    g[6] = w[6] / 8 * (-n["yz"] + rho * uy * uz + 0.5 * (sy * uz + sz * uy))
    g[7] = w[7] / 4 * (-(n["xx"] - n["yy"]) + rho * (ux ** 2 - uy ** 2) + (sx * ux - sy * uy))
    g[8] = w[8] / 12 * (-(n["xx"] + n["yy"] - 2 * n["zz"]) + rho * (ux ** 2 + uy ** 2 - 2 * uz ** 2)
                        + (sx * ux + sy * uy - 2 * sz * uz))
    g[9] = w[9] / 18 * (-(n["xx"] + n["yy"] + n["zz"]) + rho * (ux ** 2 + uy ** 2 + uz ** 2)
                        + (sx * ux + sy * uy + sz * uz) + rho)
    g[10] = (w[10] / 16 * (-n["xyy"] + 2 * uy * n["xy"] + ux * n["yy"] - 2 * rho * ux * uy ** 2
                           - 0.5 * sx * uy ** 2 - sy * uy * ux)
             + uy * g[4] + 1 / 8 * ux * (-g[7] + g[8] + 3 * g[9]))
    g[11] = (w[11] / 16 * (-n["xxy"] + 2 * ux * n["xy"] + uy * n["xx"] - 2 * rho * ux ** 2 * uy
                           - 0.5 * sy * ux ** 2 - sx * ux * uy)
             + ux * g[4] + 1 / 8 * uy * (g[7] + g[8] + 3 * g[9]))
    g[12] = (w[12] / 16 * (-n["xxz"] + 2 * ux * n["xz"] + uz * n["xx"] - 2 * rho * ux ** 2 * uz
                           - 0.5 * sz * ux ** 2 - sx * ux * uz)
             + ux * g[5] + 1 / 8 * uz * (g[7] + g[8] + 3 * g[9]))
    g[13] = (w[13] / 8 * (-n["xyz"] + ux * n["yz"] + uy * n["xz"] + uz * n["xy"] - 2 * rho * ux * uy * uz
                          - 0.5 * (sx * uy * uz + sy * ux * uz + sz * ux * uy))
             + uz * g[4] + uy * g[5] + ux * g[6])
    # post-collision second-order central moments (reading: kxx~, kyy~)
    cxx = n["xx"] - 2 * ux * n["x"] + ux ** 2 * rho
    cyy = n["yy"] - 2 * uy * n["y"] + uy ** 2 * rho
    czz = n["zz"] - 2 * uz * n["z"] + uz ** 2 * rho
    A, B, C = cxx - cyy, cxx + cyy - 2 * czz, cxx + cyy + czz
    At, Bt, Ct = A - w[7] * A, B - w[8] * B, C + w[9] * (rho - C)
    kxx_t = (3 * At + Bt + 2 * Ct) / 6
    kyy_t = (-3 * At + Bt + 2 * Ct) / 6
    g[14] = (w[14] / 16 * (-n["xxyy"] + 2 * ux * n["xyy"] + 2 * uy * n["xxy"] - ux ** 2 * n["yy"]
                           - uy ** 2 * n["xx"] - 4 * ux * uy * n["xy"]
                           + kxx_t * kyy_t / (1.0 if literal_g14 else rho)
                           + 3 * rho * ux ** 2 * uy ** 2 + sx * ux * uy ** 2 + sy * uy * ux ** 2)
             - 2 * ux * uy * g[4] + 1 / 8 * (ux ** 2 - uy ** 2) * g[7] + 1 / 8 * (-ux ** 2 - uy ** 2) * g[8]
             + (3 / 8 * (-ux ** 2 - uy ** 2) - 1 / 2) * g[9] + 2 * ux * g[10] + 2 * uy * g[11])
    return fbar + POST15 @ g + S, rho, np.array([ux, uy, uz])


W15 = np.array([2 / 9] + [1 / 9] * 6 + [1 / 72] * 8)


def _rand_state(rng, q, base, scale):
    return base + scale * rng.standard_normal(q)


@pytest.mark.parametrize("seed", range(20))
def test_flow_kernel_matches_appendix_A(oracle, seed):
    rng = np.random.default_rng(1000 + seed)
    fbar = W15 * (1 + 0.3 * rng.uniform(-1, 1)) + 0.01 * rng.standard_normal(15)
    F = 0.01 * rng.standard_normal(3)
    w = np.zeros(15)
    w[4:] = rng.uniform(0.3, 1.95, 11)
    ref, rho_r, u_r = paper_flow(fbar, F, w)
    out, rho, u = oracle.collide_flow(fbar, F, w)
    assert abs(rho - rho_r) < 1e-14
    assert np.max(np.abs(u - u_r)) < 1e-14
    assert np.max(np.abs(out - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed", range(20))
def test_thermal15_kernel_matches_section_2_2(oracle, seed):
    rng = np.random.default_rng(2000 + seed)
    gbar = rng.uniform(-0.5, 0.5) * W15 + 0.02 * rng.standard_normal(15)
    u = 0.1 * rng.standard_normal(3)
    cs2 = rng.choice([1 / 3, 0.25, 0.3])
    w = np.zeros(15)
    w[1:] = rng.uniform(0.3, 1.95, 14)
    ref = paper_thermal15(gbar, u, cs2, w)
    out = oracle.collide_thermal(15, gbar, u, cs2, w)
    assert np.max(np.abs(out - ref)) < 1e-13 * max(1e-3, np.max(np.abs(ref)))


@pytest.mark.parametrize("seed", range(20))
def test_thermal7_kernel_matches_appendix_C(oracle, seed):
    rng = np.random.default_rng(3000 + seed)
    gbar = rng.uniform(-0.5, 0.5) * np.array([0] + [1 / 6] * 6) + 0.02 * rng.standard_normal(7)
    u = 0.1 * rng.standard_normal(3)
    cs2 = rng.choice([1 / 3, 0.25, 0.3])
    w = np.zeros(7)
    w[1:] = rng.uniform(0.3, 1.95, 6)
    ref = paper_thermal7(gbar, u, cs2, w)
    out = oracle.collide_thermal(7, gbar, u, cs2, w)
    assert np.max(np.abs(out - ref)) < 1e-13 * max(1e-3, np.max(np.abs(ref)))


def test_literal_fourth_order_equilibrium_moves_a_dense_rest_state(oracle):
    """Reading of g14: with the product kxx~ kyy~ as printed, a fluid at rest
    with rho = 1.1 is not a fixed point; with kxx~ kyy~ / rho it is, and at
    rho = 1 the two forms agree."""
    w = np.zeros(15)
    w[4:] = 1.3
    for rho in (1.0, 1.1):
        f = rho * W15
        out, _, _ = oracle.collide_flow(f, np.zeros(3), w)
        assert np.max(np.abs(out - f)) < 1e-15
        ref, _, _ = paper_flow(f, np.zeros(3), w)
        assert np.max(np.abs(ref - f)) < 1e-15
    lit1, _, _ = paper_flow(1.0 * W15, np.zeros(3), w, literal_g14=True)
    assert np.max(np.abs(lit1 - W15)) < 1e-15
    lit, _, _ = paper_flow(1.1 * W15, np.zeros(3), w, literal_g14=True)
    assert np.max(np.abs(lit - 1.1 * W15)) > 1e-2


def test_source_populations_match_appendices_B_and_C(oracle):
    """The oracle builds S^phi = K^-1 m^s by a dense solve with the basis
    vectors; the paper prints the inverse (Appendix B, C).  They agree, and
    the source carries R at zeroth order and no first-order central moment."""
    rng = np.random.default_rng(4000)
    for _ in range(10):
        u = 0.15 * rng.standard_normal(3)
        R = rng.uniform(-1, 1)
        s15 = oracle.scalar_source(15, R, u)
        s7 = oracle.scalar_source(7, R, u)
        assert np.max(np.abs(s15 - SRC15 @ source_moments15(R, u))) < 1e-15
        assert np.max(np.abs(s7 - SRC7 @ source_moments7(R, u))) < 1e-15
        for S, ex, ey, ez in ((s15, EX15, EY15, EZ15), (s7, EX7, EY7, EZ7)):
            assert abs(S.sum() - R) < 1e-15
            for e, ud in ((ex, u[0]), (ey, u[1]), (ez, u[2])):
                assert abs(S @ e - ud * R) < 1e-15


@pytest.mark.parametrize("seed", range(10))
def test_thermal15_kernel_with_source_matches_section_2_2(oracle, seed):
    rng = np.random.default_rng(5000 + seed)
    gbar = rng.uniform(-0.5, 0.5) * W15 + 0.02 * rng.standard_normal(15)
    u = 0.1 * rng.standard_normal(3)
    cs2 = rng.choice([1 / 3, 0.25, 0.3])
    R = rng.uniform(-0.05, 0.05)
    w = np.zeros(15)
    w[1:] = rng.uniform(0.3, 1.95, 14)
    ref = paper_thermal15(gbar, u, cs2, w, R)
    out = oracle.collide_thermal(15, gbar, u, cs2, w, R)
    assert np.max(np.abs(out - ref)) < 1e-13 * max(1e-3, np.max(np.abs(ref)))
    assert abs(out.sum() - gbar.sum() - R) < 1e-15


@pytest.mark.parametrize("seed", range(10))
def test_thermal7_kernel_with_source_matches_appendix_C(oracle, seed):
    rng = np.random.default_rng(6000 + seed)
    gbar = rng.uniform(-0.5, 0.5) * np.array([0] + [1 / 6] * 6) + 0.02 * rng.standard_normal(7)
    u = 0.1 * rng.standard_normal(3)
    cs2 = rng.choice([1 / 3, 0.25, 0.3])
    R = rng.uniform(-0.05, 0.05)
    w = np.zeros(7)
    w[1:] = rng.uniform(0.3, 1.95, 6)
    ref = paper_thermal7(gbar, u, cs2, w, R)
    out = oracle.collide_thermal(7, gbar, u, cs2, w, R)
    assert np.max(np.abs(out - ref)) < 1e-13 * max(1e-3, np.max(np.abs(ref)))
    assert abs(out.sum() - gbar.sum() - R) < 1e-15
