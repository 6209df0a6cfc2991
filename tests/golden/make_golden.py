"""Writes tests/golden/interfaces.json from the paper's stated material values.

The numbers are closed forms of Eqs. 7-11 at the impedances the paper gives for
its experiment (Sec. 4: bone 7.8 MRayl, water 1.54 MRayl) and the tiny
workload's values (1.5 / 7.8 / 3.0 MRayl); computed here with plain math, not
with the oracle or the HIP library.
"""
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def normal_R(z1, z2):
    return ((z2 - z1) / (z2 + z1)) ** 2


def main():
    cases = []
    for z1, z2, cite in [(1.54, 7.8, "Sec. 4 (water 1.54, bone 7.8 MRayl); Eq. 11 at normal incidence"),
                         (1.5, 7.8, "tiny workload reflector; Eq. 11 at normal incidence"),
                         (1.5, 3.0, "tiny workload sphere; Eq. 11 at normal incidence")]:
        cases.append(dict(z1=z1, z2=z2, R_normal=normal_R(z1, z2), T_normal=1 - normal_R(z1, z2), cite=cite))
    crit = [dict(z1=7.8, z2=1.54, critical_deg=math.degrees(math.asin(1.54 / 7.8)),
                 cite="Sec. 4 impedances; Eq. 8 radicand vanishes at sin(theta) = Z2/Z1 with eta = Z1/Z2"),
            dict(z1=7.8, z2=1.5, critical_deg=math.degrees(math.asin(1.5 / 7.8)),
                 cite="tiny workload impedances; Eq. 8")]
    echo = dict(depth_m=0.02, c=1540.0, fs=40e6, t_echo=2 * 0.02 / 1540.0,
                bin=math.floor(2 * 0.02 / 1540.0 * 40e6),
                alpha_db_cm_mhz=0.5, f_mhz=5.0, round_trip_cm=4.0,
                amplitude_factor=10 ** (-0.5 * 5.0 * 4.0 / 20.0),
                cite="tiny workload: planar reflector at 20 mm, c 1540 m/s, 40 MHz; echo time 2d/c; "
                     "attenuation exp(-alpha f d) as amplitude (dB/20)")
    pulse = dict(f_c=5e6, f_s=40e6, n_cycles=5, fwhm_s=5 / 5e6,
                 sigma_s=5 / 5e6 / (2 * math.sqrt(2 * math.log(2))),
                 half_taps=math.ceil(3 * 5 / 5e6 / (2 * math.sqrt(2 * math.log(2))) * 40e6),
                 cite="Eq. 14 with the paper's 5 cycles at 5 MHz (Sec. 4); 40 MHz sampling")
    out = dict(interfaces=cases, critical=crit, echo=echo, pulse=pulse)
    path = os.path.join(HERE, "interfaces.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
