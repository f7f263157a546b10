"""Writes dambreak_exact.json: the exact solution of the 1D shallow-water
Riemann problem h_L = 2, h_R = 1, u_L = u_R = 0, g = 1 (LeVeque 2002,
Ch. 13: a left-going rarefaction and a right-going shock joined at the
middle state h*, u*).  Computed from the wave relations alone (no oracle
code): across a shock u changes by (h - h_k) sqrt(g/2 (1/h + 1/h_k)), across
a rarefaction by 2 (sqrt(g h) - sqrt(g h_k)); h* is the root of the sum.

Run:  python tests/golden/make_dambreak.py
"""
import json
import math
import os

from scipy.optimize import brentq

G, HL, HR = 1.0, 2.0, 1.0


def wave(h, hk):
    if h > hk:
        return (h - hk) * math.sqrt(0.5 * G * (1.0 / h + 1.0 / hk))
    return 2.0 * (math.sqrt(G * h) - math.sqrt(G * hk))


def main():
    hs = brentq(lambda h: wave(h, HL) + wave(h, HR), 1e-6, 10.0,
                xtol=1e-16, rtol=1e-15)
    us = -wave(hs, HL)
    out = {
        "citation": "1D shallow-water dam break, exact Riemann solution "
                    "(LeVeque 2002, Ch. 13); test case of the wave-"
                    "propagation patch solver cited in Sec. 3 of "
                    "arXiv 1308.1472",
        "g": G, "h_left": HL, "h_right": HR,
        "h_star": hs, "u_star": us,
        "shock_speed": hs * us / (hs - HR),
        "rarefaction_head": -math.sqrt(G * HL),
        "rarefaction_tail": us - math.sqrt(G * hs),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "dambreak_exact.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
