"""Central finite differences of the oracle's energy on the 10,000-atom
globule (26 A, the autograd workload) against the oracle's analytic forces.

The energy E = E_C + E_GB is evaluated as the plain definition: Born radii
from the coordinates (HCT descreening sums, OBC formula), then the Coulomb and
GB double sums.  For 64 atoms picked at random and each Cartesian component c,
    dE/dx_c ~ (E(x + h e_c) - E(x - h e_c)) / (x_+ - x_-),   h = 1e-5 A,
with the displaced coordinate's actual FP64 values in the denominator.  The
analytic force includes the Born-radius chain term, so a dropped term, a wrong
sign or a transposed index in any of the three passes shows up here.

Error budget: the truncation error h^2 |d^3E/dx^3| / 6 is below 1e-9
kcal/mol/A for pair distances >= 1 A; rounding of E (|E| ~ 1.5e4 kcal/mol,
row sums of 10^4 terms, 10^4 rows) is a few 1e-11 kcal/mol per evaluation,
i.e. a few 1e-6 kcal/mol/A after division by 2h.  The test allows 1e-4
kcal/mol/A absolute (forces here are 1-100 kcal/mol/A).

About 400 energy evaluations (~0.7 s each on 8 cores): marked slow, run with
GBMC_RUN_SLOW=1.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.slow

H = 1e-5
TOL = 1e-4


def test_globule_10000_central_differences_on_64_atoms(orc):
    s = synth.globule_10000()[0]
    ref = orc.energy_forces(s)
    picks = np.random.default_rng(1803).choice(s.n, 64, replace=False)

    def energy(sys_):
        R = orc.radii(sys_)["R"]
        e = orc.energy_fixedR(sys_, R)
        return e[0] + e[1]

    worst = 0.0
    for a in picks:
        for c, name in enumerate(("x", "y", "z")):
            plus, minus = s.copy(), s.copy()
            getattr(plus, name)[a] += H
            getattr(minus, name)[a] -= H
            den = getattr(plus, name)[a] - getattr(minus, name)[a]
            fd = (energy(plus) - energy(minus)) / den
            err = abs(fd - (-ref["F"][a, c]))
            worst = max(worst, err)
            assert err <= TOL, (int(a), name, fd, -ref["F"][a, c], err)
    print("max |FD - dE/dx| over 64 atoms x 3 components:", worst,
          "max |F|:", float(np.abs(ref["F"][picks]).max()))
