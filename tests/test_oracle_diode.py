"""Pins of the oracle's single-diode electrical model (CPU only).

The cell voltage is checked against the explicit Lambert-W solution of the
diode equation (Wright omega, a different method from the oracle's Newton
iteration) and against the ideal-diode closed form. The string's maximum power
is checked against a bounded scalar optimiser on uniform strings and against
brute force over a dense current grid on partially shaded strings, including
strings with two competing maxima. The generator-level power of the C1 case is
rebuilt from the cell irradiances. None of these reuses the oracle's search.
"""
import math

import numpy as np
import pytest
from scipy import optimize, special

from paper_1410_5780_amd import workloads as W

D = W.DIODE_CELL


def v_lambert(d, G, I):
    """Cell voltage from the explicit solution: with c = Iph + I0 - I,
    V + I Rs = Rsh c - a w(ln(Rsh I0 / a) + Rsh c / a), w the Wright omega function."""
    isc, gref, i0, a, rs, rsh, _ = d
    I = np.asarray(I, np.float64)
    c = isc * G / gref + i0 - I
    z = math.log(rsh * i0 / a) + rsh * c / a
    return rsh * c - a * special.wrightomega(z) - I * rs


def brute_string(d, subs, n=200001):
    """Maximum of I * V(I) over a dense grid of currents in [0, Imax]; subs: cell irradiances per substring."""
    gmax = max(max(s) for s in subs)
    imax = d[0] * gmax / d[1]
    I = np.linspace(0.0, imax, n)
    cache = {}
    V = np.zeros_like(I)
    for s in subs:
        vs = np.zeros_like(I)
        for G in s:
            if G not in cache:
                cache[G] = v_lambert(d, G, I)
            vs += cache[G]
        V += np.maximum(vs, -d[6])
    P = I * V
    j = int(np.argmax(P))
    # refine the best grid point with a bounded optimiser on the same function
    def negp(i):
        v = 0.0
        for s in subs:
            v += max(sum(float(v_lambert(d, G, i)) for G in s), -d[6])
        return -i * v
    lo, hi = I[max(j - 1, 0)], I[min(j + 1, n - 1)]
    r = optimize.minimize_scalar(negp, bounds=(lo, hi), method="bounded", options={"xatol": 1e-13})
    return max(P[j], -r.fun)


def flat(subs):
    return np.concatenate([np.asarray(s, np.float64) for s in subs]), np.array([len(s) for s in subs], np.int32)


@pytest.mark.parametrize("G", [1000.0, 700.0, 120.0, 15.0, 0.0])
def test_cell_voltage_matches_lambert_w(oracle_lib, G):
    iph = D[0] * G / D[1]
    for I in np.concatenate([np.linspace(0.0, 12.0, 121), [iph, iph * (1 - 1e-9), iph + 1e-7]]):
        got = oracle_lib.cell_voltage(D, G, I)
        want = float(v_lambert(D, G, I))
        assert abs(got - want) <= 1e-9 * max(1.0, abs(want)), (G, I, got, want)


def test_cell_voltage_ideal_diode_closed_form(oracle_lib):
    """No series resistance and no shunt: V = a ln(1 + (Iph - I) / I0)."""
    d = D.copy()
    d[4], d[5] = 0.0, 1e300
    for G in (1000.0, 333.0, 20.0):
        iph = d[0] * G / d[1]
        for I in np.linspace(0.0, iph * 0.999999, 50):
            want = d[3] * math.log1p((iph - I) / d[2])
            assert oracle_lib.cell_voltage(d, G, I) == pytest.approx(want, rel=1e-9, abs=1e-12)


def test_open_circuit_voltage_of_the_cell(oracle_lib):
    """At I = 0 the cell sits at its open-circuit voltage, 0.63 V at 1000 W/m2 by construction."""
    assert oracle_lib.cell_voltage(D, 1000.0, 0.0) == pytest.approx(0.6299, abs=1e-3)


@pytest.mark.parametrize("G", [1000.0, 800.0, 250.0, 40.0])
def test_uniform_string_is_cells_times_cell_maximum(oracle_lib, G):
    """Every cell alike: no bypass diode conducts, so the string's maximum is its number of
    cells times one cell's maximum power."""
    r = optimize.minimize_scalar(lambda i: -i * float(v_lambert(D, G, i)), bounds=(0.0, D[0] * G / D[1]),
                                 method="bounded", options={"xatol": 1e-13})
    cell = -r.fun
    for sub_len in ([20, 20, 20], [20] * 60, [7]):
        g = np.full(int(np.sum(sub_len)), G)
        got = oracle_lib.string_mpp(D, g, sub_len)
        assert got == pytest.approx(len(g) * cell, rel=1e-9)


def test_bypass_diode_holds_the_substring_at_minus_vb(oracle_lib):
    """Above a shaded substring's photocurrent its bypass diode conducts: the string's voltage
    is the other substrings' voltage minus Vb; below it every cell adds its voltage."""
    subs = [[1000.0] * 20, [200.0] * 20, [1000.0] * 20]
    g, sl = flat(subs)
    i_sh = D[0] * 200.0 / D[1]
    for I in (0.5 * i_sh, 3.0, 6.0, 8.0):
        v = oracle_lib.string_voltage(D, g, sl, I)
        lit = 40 * float(v_lambert(D, 1000.0, I))
        dark = 20 * float(v_lambert(D, 200.0, I))
        want = lit + max(dark, -D[6])
        assert v == pytest.approx(want, rel=1e-10, abs=1e-9)
        if I > 1.5 * i_sh:
            assert dark < -D[6] and v == pytest.approx(lit - D[6], rel=1e-10)


@pytest.mark.parametrize("case", [
    "one_shaded_substring", "two_maxima_later_higher", "two_maxima_earlier_higher", "graded", "one_cell_shaded",
    "all_dim"])
def test_partial_shading_matches_brute_force(oracle_lib, case):
    lit = [1000.0] * 20
    subs = {
        "one_shaded_substring": [lit, [300.0] * 20, lit],
        # six lit substrings and three at 40 %: the maximum at high current wins
        "two_maxima_later_higher": [lit] * 6 + [[400.0] * 20] * 3,
        # two lit and seven at 55 %: the maximum at low current wins
        "two_maxima_earlier_higher": [lit] * 2 + [[550.0] * 20] * 7,
        "graded": [[1000.0] * 10 + [1000.0 - 60.0 * j for j in range(10)], [700.0] * 20, [400.0] * 20,
                   [1000.0] * 19 + [100.0]],
        "one_cell_shaded": [[1000.0] * 19 + [130.0], lit, lit],
        "all_dim": [[90.0] * 20, [100.0] * 20],
    }[case]
    g, sl = flat(subs)
    got = oracle_lib.string_mpp(D, g, sl)
    want = brute_string(D, subs)
    assert got == pytest.approx(want, rel=1e-7), (case, got, want)


def test_more_shade_never_raises_power(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(25):
        g = rng.choice([1000.0, 1000.0, 1000.0, 700.0, 300.0, 100.0], size=60)
        sl = np.full(3, 20, np.int32)
        p0 = oracle_lib.string_mpp(D, g, sl)
        g2 = g.copy()
        g2[rng.integers(0, 60)] *= rng.uniform(0.0, 0.9)
        assert oracle_lib.string_mpp(D, g2, sl) <= p0 * (1 + 1e-12)


def test_c1_power_rebuilt_from_cell_irradiances(oracle_lib):
    """The C1 pole case with the diode model: per sun, the reference power is 60 cells at the
    module's unshaded irradiance, and the shaded power is the brute-force maximum of the
    cells' irradiances rebuilt from the (separately pinned) shaded counts."""
    import dataclasses
    w = W.c1_tiny(d_poa=100.0)
    g = dataclasses.replace(w.gen, diode=D)
    r = oracle_lib.evaluate(w.scene, g, w.sweep, w.map_n, w.k)
    n = np.cross(g.edge_u[0], g.edge_v[0])
    n /= np.linalg.norm(n)
    shaded_suns = 0
    for t in range(w.sweep.n):
        s = w.sweep.sun_xyz[t]
        if s[2] <= 0:
            assert r.power[t] == 0.0 and r.power_ref[t] == 0.0
            continue
        beam = w.sweep.dni[t] * max(float(n @ s), 0.0)
        G = beam * (1.0 - r.counts[t] / float(w.k * w.k)) + w.sweep.d_poa[t]
        subs = [[G[c] for c in range(60) if g.cell_substring[c] == q] for q in range(g.n_sub)]
        assert r.power[t] == pytest.approx(brute_string(D, subs), rel=1e-7)
        g0 = beam + w.sweep.d_poa[t]
        assert r.power_ref[t] == pytest.approx(brute_string(D, [[g0] * 20] * 3), rel=1e-7)
        shaded_suns += int(r.counts[t].sum() > 0)
    assert shaded_suns >= 1 and r.energy[0] < r.energy[1]
