"""Truncation-error bounds and the pruning arithmetic (sections 4-6).

  E_DH(p)  = W_R e^{-dmin^2/4h^2} C(D+p-1,D-1) r_R^p / sqrt(F(p))          (Lemma 4)
  E_DL(p)  = W_R e^{-dmin^2/4h^2} C(D+p-1,D-1) r_Q^p / sqrt(F(p))          (Lemma 5)
  E_H2L(p) = W_R e^{-dmin^2/4h^2} C(D+p-1,D-1) / sqrt(F(p))
             * ( r_Q^p + (sqrt2 r_R)^p C(D+p-1,D) (sqrt2 r_Q)^{I(sqrt2 r_Q)} ) (Lemma 6)
  E_FD     = W_R (K(dmin) - K(dmax)) / 2                                    (section 5)
  with F(p) = (floor(p/D)!)^{D-p'} (ceil(p/D)!)^{p'},  p' = p mod D,
  r_R = max_{r in R} |x_r - x_R|_inf / h,  r_Q likewise,
  I(x) = 0 for x <= 1, p-1 otherwise.

Lemma 6's printed formula is ambiguous about which bracket term the factor
(sqrt2 r_Q)^I multiplies; the proof attaches it to the E_1 part only, and that
is the reading implemented here.

Every value that decides a pruning is computed in a fixed order of
round-to-nearest double operations with the own exponential of exp64, so the
decisions can be reproduced bit for bit: the product is always
((W_R * g) * c(D,p)) * tail with g = exp64(-dmin^2 * inv_4h2), and powers are
left-to-right repeated products.

Pinned by tests/test_oracle_bounds.py: on random node pairs the true
truncation error of each method (computed with the series of `series`) never
exceeds the bound, and the bound is not vacuous (the worst ratio is within a
modest factor of 1).

O(p^D) expansions (DFTO).  The paper takes their bounds from an earlier paper
that is not available here, so the bounds below are derived afresh, from
Cramer's inequality |h_n(t)| <= K 2^{n/2} sqrt(n!) e^{-t^2/2} (K = 1.0864... in
its classical statement, used rounded up to KC = 1.09; the inequality already
holds with K = 1) and from the product form of the tensor sets:
the truncated D-dimensional series is the product of D one-dimensional
truncated series.

  One dimension, far field (DH): e^{-(t-s)^2} = sum_n s^n/n! h_n(t).  With
  rho = sqrt2 |s| = |x_r - x_R|/h <= r_R, the kept part is at most
  K e^{-t^2/2} a_p(rho) and the dropped part at most K e^{-t^2/2} b_p(rho):
    a_p(rho) = sum_{n<p} rho^n / sqrt(n!),
    b_p(rho) = rho^p / (sqrt(p!) (1 - rho/sqrt(p+1)))   (rho < sqrt(p+1); else inf)
  since n!/p! >= (p+1)^{n-p} bounds the tail by a geometric series.
  Local (DL) is the same with the roles of query and reference exchanged
  (rho = |x_q - x_Q|/h <= r_Q).
  H2L: e^{-(T+u-s)^2} = sum_{m,n} s^m (-u)^n/(m! n!) h_{m+n}(T); with
  (m+n)! <= 2^{m+n} m! n!, every term is at most
  K e^{-T^2/2} rho_R^m rho_Q^n / sqrt(m! n!), rho = sqrt2 r, so the kept part
  (m, n < p) is at most K e^{-T^2/2} a_p(rho_R) a_p(rho_Q) and the dropped part
  at most K e^{-T^2/2} (b_p(rho_R)(a_p(rho_Q) + b_p(rho_Q)) + a_p(rho_R) b_p(rho_Q)).

  D dimensions: with f_d the exact factors and S_d their truncations,
  prod f_d - prod S_d = sum_k (prod_{d<k} S_d)(f_k - S_k)(prod_{d>k} f_d), and
  |f_d| <= 1.  Every factor of every term keeps a Gaussian factor of at
  least e^{-gap_d^2/4h^2} (gap_d = the gap between the two boxes along d), whose
  product is g = e^{-dmin^2/4h^2} with dmin the box distance.  Hence, with
  a_1D and b_1D the kept and dropped bounds above without their Gaussian
  factor,
    E_T = W_R g (KC b_1D) sum_{k<D} (KC a_1D)^k.
  The ball bounds of sphere-rectangle mode do not split by dimension, so these
  bounds use the box distance.
"""

import math

SQRT2 = 1.4142135623730951  # nearest double to sqrt(2)


def powi(x, p):
    """x^p for an integer p >= 0 as the left-to-right product x*x*...*x."""
    v = 1.0
    for _ in range(p):
        v = v * x
    return v


def bound_const(D, p):
    """C(D+p-1, D-1) / sqrt(F(p)), F as in the module docstring (Lemma 4)."""
    q, pp = divmod(p, D)
    ceil_q = q + 1 if pp else q
    F = math.factorial(q) ** (D - pp) * math.factorial(ceil_q) ** pp
    return float(math.comb(D + p - 1, D - 1)) / math.sqrt(float(F))


def e_dh(W_R, g, D, p, r_R):
    """Lemma 4 with g = exp(-dmin^2/4h^2)."""
    return ((W_R * g) * bound_const(D, p)) * powi(r_R, p)


def e_dl(W_R, g, D, p, r_Q):
    """Lemma 5 with g = exp(-dmin^2/4h^2)."""
    return ((W_R * g) * bound_const(D, p)) * powi(r_Q, p)


def e_h2l(W_R, g, D, p, r_Q, r_R):
    """Lemma 6 with g = exp(-dmin^2/4h^2)."""
    sq = SQRT2 * r_Q
    itail = 1.0 if sq <= 1.0 else powi(sq, p - 1)
    second = (powi(SQRT2 * r_R, p) * float(math.comb(D + p - 1, D))) * itail
    return ((W_R * g) * bound_const(D, p)) * (powi(r_Q, p) + second)


KC = 1.09  # Cramer's classical constant 1.086435..., rounded up


def _inv_sqrt_fact(n):
    return 1.0 / math.sqrt(float(math.factorial(n)))


def _inv_sqrt_next(p):
    return 1.0 / math.sqrt(float(p + 1))


def tensor_parts(rho, p):
    """(a_p(rho), b_p(rho)) of the O(p^D) bounds: the one-dimensional kept and
    dropped parts, a = sum_{n<p} rho^n/sqrt(n!) left to right, and
    b = (rho^p/sqrt(p!)) / (1 - rho/sqrt(p+1)), inf when rho/sqrt(p+1) >= 1."""
    a = 0.0
    pw = 1.0
    for n in range(p):
        a = a + pw * _inv_sqrt_fact(n)
        pw = pw * rho
    q = rho * _inv_sqrt_next(p)
    b = (pw * _inv_sqrt_fact(p)) / (1.0 - q) if q < 1.0 else math.inf
    return a, b


def _geometric(x, D):
    """sum_{k<D} x^k, left to right."""
    v = 0.0
    pw = 1.0
    for _ in range(D):
        v = v + pw
        pw = pw * x
    return v


def e_dh_tensor(W_R, g, D, p, r_R):
    """O(p^D) far-field bound (module docstring)."""
    a, b = tensor_parts(r_R, p)
    if b == math.inf:
        return math.inf
    return (W_R * g) * ((KC * b) * _geometric(KC * a, D))


def e_dl_tensor(W_R, g, D, p, r_Q):
    """O(p^D) local bound (module docstring)."""
    return e_dh_tensor(W_R, g, D, p, r_Q)


def e_h2l_tensor(W_R, g, D, p, r_Q, r_R):
    """O(p^D) H2L bound (module docstring)."""
    aR, bR = tensor_parts(SQRT2 * r_R, p)
    aQ, bQ = tensor_parts(SQRT2 * r_Q, p)
    if bR == math.inf or bQ == math.inf:
        return math.inf
    tail = bR * (aQ + bQ) + aR * bQ
    return (W_R * g) * ((KC * tail) * _geometric(KC * (aR * aQ), D))


def e_fd(W_R, kmin, kmax):
    """Section 5: E_FD = W_R (K(dmin) - K(dmax)) / 2."""
    return 0.5 * (W_R * (kmin - kmax))


def need(E, W_R, L, W, eps_alg):
    """Token a pruning with absolute error E costs (section 5):
    W E / (eps L) - W_R.  Negative values are deposits.  E = 0 deposits the
    whole W_R; a zero lower bound L makes any positive error unaffordable."""
    if E == 0.0:
        return -W_R
    if L == 0.0:
        return math.inf
    return (W * E) / (eps_alg * L) - W_R


def sphere_rect_dist2(loQ, hiQ, loR, hiR, cQ, cR, radQ, radR):
    """(dmin^2, dmax^2) from both the bounding boxes and the bounding balls
    about the box centres (radius rad = max |x - c|_2): with
    dc = |c_Q - c_R|_2, every point pair is at least dc - rad_Q - rad_R and at
    most dc + rad_Q + rad_R apart, so the tighter of each pair of bounds
    holds.  Fixed operation order (squares summed in d, sqrt, then
    ((dc - rad_Q) - rad_R) and ((dc + rad_Q) + rad_R)) for bit-exact
    reproduction."""
    smin, smax = box_dist2(loQ, hiQ, loR, hiR)
    d2 = 0.0
    for d in range(len(cQ)):
        diff = cQ[d] - cR[d]
        d2 = d2 + diff * diff
    dc = math.sqrt(d2)
    gap = (dc - radQ) - radR
    if gap > 0.0:
        g2 = gap * gap
        if g2 > smin:
            smin = g2
    far = (dc + radQ) + radR
    f2 = far * far
    if f2 < smax:
        smax = f2
    return smin, smax


def box_dist2(loQ, hiQ, loR, hiR):
    """(dmin^2, dmax^2) between two boxes, summed over d in order (section 5:
    the distance bounds come from the bounding boxes)."""
    smin = 0.0
    smax = 0.0
    for d in range(len(loQ)):
        gap = loQ[d] - hiR[d]
        other = loR[d] - hiQ[d]
        if other > gap:
            gap = other
        if gap < 0.0:
            gap = 0.0
        far = hiQ[d] - loR[d]
        other = hiR[d] - loQ[d]
        if other > far:
            far = other
        smin = smin + gap * gap
        smax = smax + far * far
    return smin, smax


INF_COST = (1 << 63) - 1


def _sat_mul(a, b):
    v = a * b
    return v if v < INF_COST else INF_COST


def _pow_int(D, e):
    v = 1
    for _ in range(e):
        v = _sat_mul(v, D)
    return v


def term_cost(D, p, family="graded"):
    """Per-point cost of an order-p expansion in Figure 6's model: D^{p+1}
    (graded, C(D+p-1,D) ~ D^p terms of D factors) or D p^D (tensor)."""
    if family == "tensor":
        return _sat_mul(D, _pow_int(p, D))
    return _pow_int(D, p + 1)


def h2l_cost(D, p, family="graded"):
    """Cost of one order-p H2L translation: D^{2p+1} or D p^{2D}."""
    if family == "tensor":
        return _sat_mul(D, _pow_int(p, 2 * D))
    return _pow_int(D, 2 * p + 1)


def feasible_orders(D, plimit, maxerr, W_R, g, r_Q, r_R, mask=7, family="graded"):
    """Figure 6, first half: for each series method, the smallest order
    p <= plimit whose bound meets maxerr.  Returns {name: (p, E)} for the
    methods that have one; `mask` restricts the candidates (bit 0 DH, 1 DL,
    2 H2L); `family` selects the O(D^p) ("graded") or O(p^D) ("tensor")
    bounds."""
    found = {}
    if family == "tensor":
        fns = ((1, "DH", lambda p: e_dh_tensor(W_R, g, D, p, r_R)),
               (2, "DL", lambda p: e_dl_tensor(W_R, g, D, p, r_Q)),
               (4, "H2L", lambda p: e_h2l_tensor(W_R, g, D, p, r_Q, r_R)))
    else:
        fns = ((1, "DH", lambda p: e_dh(W_R, g, D, p, r_R)),
               (2, "DL", lambda p: e_dl(W_R, g, D, p, r_Q)),
               (4, "H2L", lambda p: e_h2l(W_R, g, D, p, r_Q, r_R)))
    for bit, name, fn in fns:
        if not mask & bit:
            continue
        for p in range(1, plimit + 1):
            E = fn(p)
            if E <= maxerr:
                found[name] = (p, E)
                break
    return found


def best_method(D, plimit, maxerr, W_R, g, r_Q, r_R, N_Q, N_R, mask=7, family="graded"):
    """Figure 6.  Smallest feasible order per method, cost model
    c_DH = N_Q D^{p+1}, c_DL = N_R D^{p+1}, c_H2L = D^{2p+1} (graded; the
    tensor family uses D p^D and D p^{2D}, term_cost and h2l_cost),
    c_Direct = D N_Q N_R, first minimum in the order DH, DL, H2L, DIRECT.
    `mask` restricts the candidate methods (bit 0 DH, 1 DL, 2 H2L) for
    ablations.  Returns (name, p, E) with name in {"DH","DL","H2L","DIRECT"}."""
    found = feasible_orders(D, plimit, maxerr, W_R, g, r_Q, r_R, mask, family)
    costs = []
    for name in ("DH", "DL", "H2L"):
        if name in found:
            p = found[name][0]
            if name == "DH":
                c = _sat_mul(N_Q, term_cost(D, p, family))
            elif name == "DL":
                c = _sat_mul(N_R, term_cost(D, p, family))
            else:
                c = h2l_cost(D, p, family)
        else:
            c = INF_COST
        costs.append(c)
    costs.append(_sat_mul(D, _sat_mul(N_Q, N_R)))
    best = min(costs)
    for i, name in enumerate(("DH", "DL", "H2L")):
        if costs[i] == best and name in found:
            return name, found[name][0], found[name][1]
    return "DIRECT", 0, math.inf
