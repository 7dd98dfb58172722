"""The near-field kernels evaluate h0(x) = sin(x)/x - i cos(x)/x, x = k r, through
polynomials in u = x^2 fitted on the range of u the host guarantees (x <= 1 or
x <= 1/2).  This reads their coefficients out of the kernel source and checks each
polynomial against sin(x)/x and cos x on its whole range (50-digit reference), so a
mistyped or reordered coefficient fails here without a GPU."""
import os
import re

import mpmath as mp
import pytest

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_1902_05132_amd", "csrc", "lfmm_kernels.hip")
NUM = r"[-+]?\d+\.\d+(?:e[-+]?\d+)?f?"
LINE = re.compile(r"\b(ps|pc) = (fmaf?)\((%s|ps|pc), u, (%s)\);" % (NUM, NUM))


def _chains():
    """(variable, precision, coefficients from the highest degree down) of every
    Horner chain that starts from literal coefficients."""
    chains, cur = [], {}
    for line in open(SRC):
        m = LINE.search(line)
        if not m:
            continue
        var, fn, a, b = m.groups()
        if a not in ("ps", "pc"):
            cur[var] = {"var": var, "fp32": fn == "fmaf", "c": [a, b]}
            chains.append(cur[var])
        else:
            cur[var]["c"].append(b)
    return chains


def _value(lit, fp32):
    v = float(lit.rstrip("f"))
    if fp32:
        import numpy as np
        v = float(np.float32(v))
    return mp.mpf(v)


# (precision, degree) -> range of u and the largest error allowed: below one rounding
# of the working precision (FP32 6e-8, FP64 1.1e-16 relative near 1), with margin
BOUND = {(True, 4): (1, 2e-8), (True, 3): (0.25, 2e-8), (False, 7): (1, 1e-16), (False, 5): (0.25, 5e-16)}


def test_every_fitted_polynomial_within_its_bound():
    mp.mp.dps = 50
    chains = _chains()
    seen = {(c["fp32"], len(c["c"]) - 1, c["var"]) for c in chains}
    # both functions in every form: FP32 quartics and cubics, FP64 degree 7 and 5
    assert seen == {(p, d, v) for (p, d) in BOUND for v in ("ps", "pc")}
    for c in chains:
        deg = len(c["c"]) - 1
        umax, tol = BOUND[(c["fp32"], deg)]
        coef = [_value(x, c["fp32"]) for x in c["c"]]
        worst = mp.mpf(0)
        for i in range(801):
            u = mp.mpf(umax) * i / 800
            x = mp.sqrt(u)
            exact = (mp.sin(x) / x if u > 0 else mp.mpf(1)) if c["var"] == "ps" else mp.cos(x)
            worst = max(worst, abs(mp.polyval(coef, u) - exact))
        assert worst < tol, (c["var"], c["fp32"], deg, float(worst))


@pytest.mark.parametrize("var", ["ps", "pc"])
def test_a_wrong_coefficient_is_caught(var):
    """The check bites: one coefficient of the FP32 cubic off in its fourth digit fails it."""
    mp.mp.dps = 30
    c = next(c for c in _chains() if c["fp32"] and len(c["c"]) == 4 and c["var"] == var)
    coef = [_value(x, True) for x in c["c"]]
    coef[1] *= mp.mpf("1.001")
    worst = max(abs(mp.polyval(coef, mp.mpf(i) / 3200) -
                    ((mp.sin(mp.sqrt(mp.mpf(i) / 3200)) / mp.sqrt(mp.mpf(i) / 3200) if i else 1) if var == "ps"
                     else mp.cos(mp.sqrt(mp.mpf(i) / 3200)))) for i in range(801))
    assert worst > BOUND[(True, 3)][1]
