"""Writes the stored reference values under tests/golden/.

Calls only the analytic references in `oracle.closed_forms` (40-digit mpmath):

* eq18_points.json     -- eq. 18 (the paper's exact solution of its worked
                          example, eq. 16 with 2 sqrt(2) theta^2 = 1, rescaled)
                          at points of the paper's display box (+-5, STEP 4)
* feynman_points.json  -- Feynman-parameter form of the subtracted bubble for
                          the real, unequal and conjugate-pair mass cases
                          (principal logs where they give the analytic
                          function), and for the conjugate pair in the wedge
                          where they do not (`feynman_continued`: the a-contour
                          deformed so the roots of Delta keep their side)

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import closed_forms as cf  # noqa: E402

EQ18_POINTS = [1 + 1j, 3 - 2j, -0.2 - 0.1j, -0.2 + 0.1j, -2 - 0.05j, -2 + 0.05j,
               -4 + 3j, -4 - 3j, -0.5 + 0.5j, 4 + 0.1j, -1 - 1j, -4.9 + 4.9j,
               4.9 - 4.9j, 0.3 + 2.2j, 0.3 - 2.2j, -0.05 + 0.3j, 2.5 + 4.5j,
               -3.3 - 0.7j, 0.7 - 0.2j, -1.2 + 0.02j]

FEYNMAN_CASES = {
    "equal_m1_m2_1_mu2_1": dict(m1sq=1.0, m2sq=1.0, mu2=1.0,
                                points=[2 + 3j, -3 + 2j, -6 + 3j, 0.5 + 0.3j, -0.8 + 0.5j,
                                        3 + 0.5j, -7.9 + 3.9j, 1.2 + 1.7j, 3.5 - 2.5j,
                                        -0.3 - 0.9j, -2.5 + 1.5j, 6 + 6j]),
    "unequal_m1_1_m2_0p5_mu2_2": dict(m1sq=1.0, m2sq=0.25, mu2=2.0,
                                      points=[2 + 3j, -3 + 2j, 0.5 + 0.3j, -0.8 - 0.5j,
                                              3 + 0.5j, -5 + 3j, 1.2 - 1.7j, -0.2 + 0.2j]),
    "conjugate_1_pm_0p5i_mu2_1": dict(m1sq=1 + 0.5j, m2sq=1 - 0.5j, mu2=1.0,
                                      points=[2 + 3j, 0.5 + 0.3j, 3 + 0.5j, 1.2 - 1.7j,
                                              -0.5 + 0.2j, 4 - 4j, 0.1 + 2j]),
}


# conjugate pair m^2 = 1 +- 0.5i, mu^2 = 1: points of the complex-mass
# workload's box where Delta(a, x) crosses the negative real axis for some a
# in [0, 1], so the principal-log form is not the analytic function (|x| <= 9,
# where the next cutoff term is below the pin's 5e-11 at Lambda^2 = 1e4)
WEDGE_CASE = ("conjugate_1_pm_0p5i_mu2_1_wedge", 1 + 0.5j, 1 - 0.5j, 1.0,
              [-5 + 0.5j, -5 - 0.5j, -4.5 + 0.2j, -7 + 0.1j, -9 - 1j, -6 + 1.5j, -8 + 0.6j,
               -5.5 - 0.05j, -4.3 + 0.01j])


def main():
    eq18 = {
        "source": "eq. 18 (exact subtracted, rescaled correlator of the worked example, "
                  "eq. 16 with m1^2 = -i/2 on the (p-k) leg, m2^2 = +i/2, subtraction at x = 0)",
        "points": [[x.real, x.imag, cf.eq18(x).real, cf.eq18(x).imag] for x in EQ18_POINTS],
    }
    with open(os.path.join(HERE, "eq18_points.json"), "w") as f:
        json.dump(eq18, f, indent=1)
    fey = {"source": "int_0^1 log(Delta(a, mu^2)/Delta(a, x)) da, Delta(a, s) = a m1^2 + "
                     "(1-a) m2^2 + a(1-a) s (textbook Feynman parametrisation of the "
                     "subtracted bubble of eq. 14, infinite cutoff, principal logs)",
           "cases": {}}
    for name, c in FEYNMAN_CASES.items():
        pts = []
        for x in c["points"]:
            if not cf.feynman_principal_ok(x, c["m1sq"], c["m2sq"], c["mu2"]):
                raise SystemExit(f"{name}: principal form not valid at {x}")
            g = cf.feynman(x, c["m1sq"], c["m2sq"], c["mu2"])
            pts.append([x.real, x.imag, g.real, g.imag])
        m1, m2 = complex(c["m1sq"]), complex(c["m2sq"])
        fey["cases"][name] = {"m1sq": [m1.real, m1.imag], "m2sq": [m2.real, m2.imag],
                              "mu2": c["mu2"], "points": pts}
    name, m1, m2, mu2, points = WEDGE_CASE
    pts = []
    for x in points:
        if cf.feynman_principal_ok(x, m1, m2, mu2):
            raise SystemExit(f"{name}: {x} is not in the wedge")
        g = cf.feynman_continued(x, m1, m2, mu2)
        pts.append([x.real, x.imag, g.real, g.imag])
    fey["cases"][name] = {"m1sq": [m1.real, m1.imag], "m2sq": [m2.real, m2.imag], "mu2": mu2,
                          "form": "continued", "points": pts}
    with open(os.path.join(HERE, "feynman_points.json"), "w") as f:
        json.dump(fey, f, indent=1)


if __name__ == "__main__":
    main()
