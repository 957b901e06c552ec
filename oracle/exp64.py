"""Own double-precision exponential used for every pruning decision.

The pruning test of Theorem 2 (section 5) compares quantities built from
exp(-delta^2 / 2h^2) and exp(-delta^2 / 4h^2).  To make the test reproducible
bit for bit on any machine, the oracle does not call the platform libm here:
it evaluates exp with the classical Cody-Waite method

    x = k ln2 + r,   k = floor(x log2(e) + 1/2),   |r| <= ln2 / 2,
    r = (x - k*LN2_HI) - k*LN2_LO       (LN2_HI has trailing zero bits, so
                                         k*LN2_HI is exact),
    exp(x) = 2^k * P(r),   P = degree-13 Taylor polynomial of exp,

with P evaluated by Horner's rule, every operation a single IEEE-754
round-to-nearest double operation (no fused multiply-add).  The truncation
error of P on |r| <= ln2/2 is below 4e-18 relative, so the result is within a
few units in the last place of the true exponential.  Arguments below -700
return 0 (the true value is below 1e-304 and the pruning test treats it as a
zero error).

Pinned by tests/test_oracle_exp.py against math.exp and 50-digit mpmath.
"""

import math

LOG2E = 1.4426950408889634          # 1 / ln 2, nearest double
LN2_HI = 6.93147180369123816490e-01  # ln 2 rounded to 32 significant bits
LN2_LO = 1.90821492927058770002e-10  # ln 2 - LN2_HI, nearest double
DEGREE = 13
# Taylor coefficients 1/n!, each a correctly rounded quotient.
COEF = [1.0 / math.factorial(n) for n in range(DEGREE + 1)]
UNDERFLOW_ARG = -700.0


def exp64(x):
    """exp(x) for a double x <= 709, by the method in the module docstring."""
    x = float(x)
    if x < UNDERFLOW_ARG:
        return 0.0
    k = math.floor(x * LOG2E + 0.5)
    r = (x - k * LN2_HI) - k * LN2_LO
    p = COEF[DEGREE]
    for n in range(DEGREE - 1, -1, -1):
        p = p * r + COEF[n]
    return math.ldexp(p, k)
