"""Pins of the oracle's hydrogen rate coefficients beyond alpha_B (which
test_oracle_chemistry pins against the case-B table).

The paper gives no rate set (Sec. 2.2: hydrogen "with the associated
cooling processes"); the oracle uses Cen (1992) for collisional ionisation,
collisional excitation and free-free cooling and Hui & Gnedin (1997) for
case-B recombination cooling.  Nothing in those fits is re-typed here.
Instead each coefficient is held against physics that does not come from
the fit (tests/golden/hydrogen_rates_physics.txt):

  * thresholds: the Boltzmann factor of collisional ionisation carries the
    H I ionisation energy, that of collisional excitation the Lyman-alpha
    energy (3/4 of it); measured as -d ln r / d(1/T) at 300 K;
  * collisional-ionisation cooling removes the ionisation energy per event;
  * collisional ionisation lies within the spread between fits of the
    independent Voronov (1997) fit;
  * case-B recombination cooling per recombination matches Draine's mean
    recombining-electron energy;
  * free-free cooling implies a Gaunt factor in the textbook range when
    divided by the Rybicki & Lightman prefactor built from CODATA constants;
  * collisional-excitation cooling implies an effective collision strength
    of order unity.

The last test plants plausible typos in copies of the oracle source (a
digit of an exponent, a power of ten of a prefactor) and checks that each
copy fails at least one pin.
"""

import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hydrogen_rates_physics.txt")


def golden():
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if len(line) == 2:
                out[line[0]] = float(line[1])
    return out


G = golden()
KB, EV = G["kB_erg_K"], G["eV_erg"]
CHI = G["chi_H_eV"] * EV


def threshold_kelvin(rates, i, T=300.0):
    """-d ln r_i / d(1/T) by a central difference in 1/T."""
    u = 1.0 / T
    du = u * 1e-6
    lo, hi = rates(1.0 / (u - du))[i], rates(1.0 / (u + du))[i]
    return -(math.log(hi) - math.log(lo)) / (2.0 * du)


def voronov(T):
    U = CHI / (KB * T)
    return (G["voronov_A"] * (1.0 + G["voronov_P"] * math.sqrt(U)) * U ** G["voronov_K"] *
            math.exp(-U) / (G["voronov_X"] + U))


def rybicki_lightman_prefactor():
    h, me, c, e = G["h_erg_s"], G["me_g"], G["c_cm_s"], G["e_esu"]
    return (2.0 ** 5 * math.pi * e ** 6 / (3.0 * h * me * c ** 3) *
            math.sqrt(2.0 * math.pi * KB / (3.0 * me)))


def failed_pins(rates) -> list:
    """Names of the pins that `rates(T) -> [alpha_B, beta, recB cooling,
    colex cooling, colion cooling, free-free cooling]` fails."""
    bad = []
    # thresholds (the sqrt(T) prefactor of beta adds T/2 = 150 K at 300 K)
    if abs(threshold_kelvin(rates, 1) / (CHI / KB) - 1.0) > 2e-3:
        bad.append("beta threshold")
    E12 = G["lya_fraction"] * CHI
    if abs(threshold_kelvin(rates, 3) / (E12 / KB) - 1.0) > 5e-4:
        bad.append("excitation threshold")
    for T in (1e4, 3e4, 1e5):
        r = rates(T)
        if abs(r[4] / r[1] / CHI - 1.0) > 1e-3:
            bad.append("ionisation energy per collisional ionisation")
            break
    for T in np.geomspace(5e3, 1e5, 9):
        q = rates(T)[1] / voronov(T)
        if not 0.4 <= q <= 1.25:
            bad.append(f"beta vs Voronov at {T:.3g} K ({q:.3g})")
            break
    for T in np.geomspace(1e3, 3e4, 8):
        r = rates(T)
        m = r[2] / (r[0] * KB * T)
        ref = G["draine_EB_a"] - G["draine_EB_b"] * math.log(T / 1e4)
        if not (0.5 < m < 1.0 and abs(m / ref - 1.0) <= 0.12):
            bad.append(f"recombination cooling per recombination at {T:.3g} K ({m:.3g} kT)")
            break
    C = rybicki_lightman_prefactor()
    for T in np.geomspace(1e3, 1e8, 11):
        g = rates(T)[5] / (C * math.sqrt(T))
        if not G["gaunt_min"] <= g <= G["gaunt_max"]:
            bad.append(f"free-free Gaunt factor at {T:.3g} K ({g:.3g})")
            break
    h, me = G["h_erg_s"], G["me_g"]
    beta_c = h * h / ((2.0 * math.pi * me) ** 1.5 * math.sqrt(KB))
    for T in np.geomspace(5e3, 5e4, 7):
        q12 = rates(T)[3] / E12
        ups = q12 / (beta_c / math.sqrt(T) / 2.0 * math.exp(-E12 / (KB * T)))
        if not G["upsilon_min"] <= ups <= G["upsilon_max"]:
            bad.append(f"excitation collision strength at {T:.3g} K ({ups:.3g})")
            break
    return bad


def test_prefactors_from_constants():
    # the two textbook prefactors, built from CODATA constants, are the
    # familiar 1.43e-27 (free-free) and 8.63e-6 (collision strengths)
    assert rybicki_lightman_prefactor() == pytest.approx(1.4256e-27, rel=1e-3)
    h, me = G["h_erg_s"], G["me_g"]
    assert h * h / ((2 * math.pi * me) ** 1.5 * math.sqrt(KB)) == pytest.approx(8.629e-6,
                                                                                  rel=1e-3)


def test_oracle_rates_meet_every_pin(orc):
    assert failed_pins(orc.rates) == []


PLANTED = [
    ("157809.1", "175809.1"),                        # beta threshold digits swapped
    ("exp(-118348.0 / T)", "exp(-11834.8 / T)"),     # excitation threshold decade
    ("5.85e-11", "5.85e-10"),                        # beta prefactor decade
    ("3.435e-30", "3.435e-31"),                      # recombination cooling decade
    ("3.720", "3.270"),                              # recombination cooling exponent
    ("1.42e-27", "1.42e-26"),                        # free-free decade
    ("7.5e-19", "7.5e-18"),                          # excitation prefactor decade
    ("r[4] = E_ION_EV * EV * r[1];", "r[4] = EV * r[1];"),   # energy per ionisation
    ("sqrt(T) * exp(-157809.1", "T * exp(-157809.1"),        # beta power of T
]


@pytest.mark.parametrize("old,new", PLANTED)
def test_planted_mistake_fails_a_pin(tmp_path, old, new):
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(path),
                    "-I", os.path.dirname(oracle._SRC), "-lm", "-fopenmp"], check=True, cwd=str(tmp_path))
    L = ctypes.CDLL(str(so))
    L.orc_rates.restype = None
    L.orc_rates.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_double)]

    def rates(T):
        out = np.zeros(6)
        L.orc_rates(float(T), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return out

    assert failed_pins(rates), f"planted mistake {old!r} -> {new!r} passed every pin"
