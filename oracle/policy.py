"""Training records of the learned pair policy, computed from a decision
trace by their plain definitions.  TEST INFRASTRUCTURE ONLY.

For every node pair where bestMethod (Figure 6) is reached, a record holds
  * features f[16] of the pair (geometry only, no token state):
      0 log2 N_Q, 1 log2 N_R, 2 log2(1 + dmin/h), 3 log2(1 + dmax/h), 4 log2 h,
      5 log2(1 + r_Q), 6 log2(1 + r_R) (r = rinf / h, section 4),
      7 [Q is a leaf], 8 [R is a leaf], 9 D / 16, 10..15 zero;
  * targets t[4] = log2 of the cost, in nanoseconds, of each action:
      DH, DL, H2L at the smallest order their bound admits (mask 0 where no
      order up to PLIMIT is admitted), and "recurse" = the cost-to-go of the
      direct path (base case or split), known only where the run took it;
  * masks m[4] in {0, 1}.
Cost of one decided pair under a cost model cm (ns per unit):
  every pair   cm.pair                        (deciding it)
  FD           nothing more
  DH at p      N_Q C(D+p-1, D) cm.dh
  DL at p      N_R C(D+p-1, D) cm.dl
  H2L at p     C(D+p-1, D)^2 cm.h2l
  base case    N_Q N_R cm.base
  split        the cost-to-go of its child pairs (one level down).
"""

import math

import numpy as np

from .bounds import box_dist2
from .multiindex import num_terms

FD, DH, DL, H2L, BASE, SPLIT = 0, 1, 2, 3, 4, 5


class CostModel:
    def __init__(self, pair, dh, dl, h2l, base):
        self.pair, self.dh, self.dl, self.h2l, self.base = pair, dh, dl, h2l, base


def pair_features(qt, rt, Q, R, h, D):
    dmin2, dmax2 = box_dist2(qt.lo[Q], qt.hi[Q], rt.lo[R], rt.hi[R])
    ih = 1.0 / h
    f = np.zeros(16)
    f[0] = math.log2(int(qt.count[Q]))
    f[1] = math.log2(int(rt.count[R]))
    f[2] = math.log2(1.0 + math.sqrt(dmin2) * ih)
    f[3] = math.log2(1.0 + math.sqrt(dmax2) * ih)
    f[4] = math.log2(h)
    f[5] = math.log2(1.0 + float(qt.rinf[Q]) * ih)
    f[6] = math.log2(1.0 + float(rt.rinf[R]) * ih)
    f[7] = 1.0 if qt.left[Q] < 0 else 0.0
    f[8] = 1.0 if rt.left[R] < 0 else 0.0
    f[9] = D / 16.0
    return f


def action_cost(code, p, NQ, NR, D, cm):
    c = cm.pair
    if code == DH:
        c += NQ * num_terms(D, p) * cm.dh
    elif code == DL:
        c += NR * num_terms(D, p) * cm.dl
    elif code == H2L:
        c += num_terms(D, p) ** 2 * cm.h2l
    elif code == BASE:
        c += NQ * NR * cm.base
    return c


def cost_to_go(trace, qt, rt, D, cm):
    """Cost-to-go of every trace row (h, level, Q, R, code, p), deepest level
    first: a split pair's cost is its own decision plus its children's."""
    rows = [tuple(int(v) for v in r) for r in trace]
    index = {(r[0], r[1], r[2], r[3]): i for i, r in enumerate(rows)}
    cost = np.zeros(len(rows))
    for i in sorted(range(len(rows)), key=lambda i: -rows[i][1]):
        h, lev, Q, R, code, p = rows[i]
        c = action_cost(code, p, int(qt.count[Q]), int(rt.count[R]), D, cm)
        if code == SPLIT:
            qs = [Q] if qt.left[Q] < 0 else [int(qt.left[Q]), int(qt.left[Q]) + 1]
            rs = [R] if rt.left[R] < 0 else [int(rt.left[R]), int(rt.left[R]) + 1]
            for qc in qs:
                for rc in rs:
                    c += cost[index[(h, lev + 1, qc, rc)]]
        cost[i] = c
    return cost


def records(trace, feasible, qt, rt, hs, D, cm):
    """(keys, F[n][16], T[n][4], M[n][4]) for the rows where bestMethod was
    reached (the keys of `feasible`), sorted by (h, level, Q, R)."""
    ctg = cost_to_go(trace, qt, rt, D, cm)
    code_of = {}
    for i, r in enumerate(trace):
        code_of[tuple(int(v) for v in r[:4])] = (int(r[4]), i)
    keys = sorted(feasible)
    F = np.zeros((len(keys), 16))
    T = np.zeros((len(keys), 4))
    Mk = np.zeros((len(keys), 4))
    for n, key in enumerate(keys):
        h, lev, Q, R = key
        F[n] = pair_features(qt, rt, Q, R, float(hs[h]), D)
        NQ, NR = int(qt.count[Q]), int(rt.count[R])
        for k, (name, code) in enumerate((("DH", DH), ("DL", DL), ("H2L", H2L))):
            if name in feasible[key]:
                T[n, k] = math.log2(action_cost(code, feasible[key][name], NQ, NR, D, cm))
                Mk[n, k] = 1.0
        code, i = code_of[key]
        if code in (BASE, SPLIT):
            T[n, 3] = math.log2(ctg[i])
            Mk[n, 3] = 1.0
    return keys, F, T, Mk
