"""The multigrid smoother's two weights (csrc/nf_internal.h, kOmega1 and
kOmega2): the reciprocals of the roots of the degree-2 Chebyshev polynomial
on [2/5, 2], so that two damped-Jacobi sweeps with them
* reduce every eigencomponent of D^-1 A in (0, 2] (the range Gershgorin
  gives for the cut-cell and coarse operators): |(1 - w1 l)(1 - w2 l)| < 1,
  and the first sweep alone does not amplify any (|1 - w1 l| <= 1);
* shrink [2/5, 2] by at most 1 / T_2(3/2) = 2/7, and the high-frequency part
  [1/3, 2] by less than the 0.51 of two sweeps with 6/7."""
import math
import os
import re

import numpy as np

HEADER = os.path.join(os.path.dirname(__file__), "..", "paper_2405_14903_amd", "csrc", "nf_internal.h")


def _weight(name):
    m = re.search(r"constexpr float %s = ([0-9.]+)f;" % name, open(HEADER).read())
    assert m, name
    return float(m.group(1))


def test_weights_are_the_chebyshev_roots_on_two_fifths_to_two():
    w1, w2 = _weight("kOmega1"), _weight("kOmega2")
    c, d = (2 + 0.4) / 2, (2 - 0.4) / 2
    assert abs(w1 - 1 / (c + d * math.cos(math.pi / 4))) < 1e-6
    assert abs(w2 - 1 / (c - d * math.cos(math.pi / 4))) < 1e-6
    # the product's roots are the Chebyshev points of [2/5, 2]
    roots = sorted([1 / w1, 1 / w2])
    cheb = sorted(c + d * math.cos((2 * k - 1) * math.pi / 4) for k in (1, 2))
    assert np.allclose(roots, cheb, rtol=1e-6)


def test_two_sweeps_contract_and_smooth():
    w1, w2 = _weight("kOmega1"), _weight("kOmega2")
    lam = np.linspace(1e-9, 2.0, 200001)
    p = (1 - w1 * lam) * (1 - w2 * lam)
    assert np.abs(p).max() < 1.0
    assert np.abs(1 - w1 * lam).max() <= 1.0
    x = 1.5                                       # (c / d) of [2/5, 2]
    t2 = 2 * x * x - 1
    assert abs(np.abs(p[lam >= 0.4]).max() - 1 / t2) < 1e-5
    jacobi = (1 - 6.0 / 7.0 * lam) ** 2
    hi = lam >= 1.0 / 3.0
    assert np.abs(p[hi]).max() < 0.4 < np.abs(jacobi[hi]).max()
