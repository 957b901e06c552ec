"""The dual-tree Gaussian summation with token error control (sections 5-6,
Figures 1, 6, 7, 8), run level by level.

The paper states the recursion depth first (Figure 1) and notes that the order
of the node-pair visits is free (it can also be driven by a priority queue).
This oracle visits the node pairs breadth first: a frontier of (Q, R) pairs is
refined one level at a time, and every pair of the frontier is either resolved
(finite difference, a series expansion, or an exhaustive base case) or split
into child pairs.  It is the schedule the GPU library follows, so the pair
lists it records are the ones the library must reproduce bit for bit.

Per bandwidth h, with W = sum_r w_r and eps_alg = (1 - rho) eps (rho is the
share of eps reserved for floating-point rounding):

  state per query node Q: token budget T_Q (starts at 0, section 5), Lpush_Q
  (lower bound on the contribution of the reference nodes already resolved
  against Q or an ancestor), Gest_Q, local coefficients lco_Q of order pL_Q.

  For each frontier segment (Q; R_1..R_k), the R_j in left-to-right tree order:
   1. lower bound on G over Q (the running G_Q^min of section 5):
        L = Lpush_Q + sum_j W_Rj K(dmax(Q,R_j))        (sequential in j)
      and, when the queries are the references themselves, L = max(L, wmin_Q)
      because every query receives its own term w_q K(0) = w_q.
   2. for j = 1..k, with t the running token (Figure 7):
        FD if need(E_FD) <= t: t -= need, Gest_Q += W_R (K(dmin)+K(dmax))/2;
        else bestMethod(maxerr = eps_alg (W_R + t) L / W) (Figure 6); if it is
        not DIRECT: t -= need(E_A), record (Q, R, p) for DH, DL or H2L;
        else if both are leaves: exhaustive base case, t += W_R (E_EX = 0);
        else split: both internal -> 4 child pairs, otherwise split the
        internal one.
      Every resolved pair adds W_R K(dmax) to Lpush_Q.
      need(E) = W E / (eps_alg L) - W_R (section 5; see bounds.need).
   3. child segments inherit the final t and Lpush_Q by copy: a token is a
      per-query-point budget (proof of Theorem 2), valid for every point of Q.

  After the traversal the recorded work is executed (the contributions are
  additive and no decision depends on them): base cases add exact sums,
  DH adds the Hermite series at each query, DL and H2L add local
  coefficients.  Then the post-pass of Figure 8 runs top down: Gest and L2L
  translated local coefficients are pushed to the children, and at a leaf
  every query receives gx + gdh + Gest_Q + EVALL(lco_Q).

Decisions depend only on the tree geometry, weights, counts and h: they are
computed in IEEE double with the own exponential (exp64) in a fixed operation
order, which is what makes them reproducible bit for bit.  Every query result
satisfies |G~ - G| <= eps_alg G (Theorem 2), plus rounding.

Readings of the paper taken here (each also listed in the design notes):
  * the base case weights each kernel value by w_r (Figure 7 omits it);
  * Figure 8's "G_q^est = EVALL + G_Q^est" adds to the base-case and DH sums;
  * the token update uses W E_A/(eps G_Q^min) - W_R, the dimensionally
    consistent form of section 5 with an absolute E_A;
  * G_Q^min is the box lower bound described in step 1 (the paper does not
    say how it is initialised or propagated in a level-wise traversal);
  * pL_Q is the largest order of any local contribution at Q or above.
"""

import math

import numpy as np

from .bounds import best_method, box_dist2, e_fd, feasible_orders, need, sphere_rect_dist2
from .exp64 import exp64
from .kdtree import attach_moments, build_kdtree
from .multiindex import plimit_for, plimit_tensor, set_size
from .series import direct_local, eval_hermite, eval_local, h2l, l2l, scale_moments

FD, DH, DL, H2L, BASE, SPLIT = 0, 1, 2, 3, 4, 5
CODE = {"DH": DH, "DL": DL, "H2L": H2L}
NAME = {DH: "DH", DL: "DL", H2L: "H2L"}
METHODS = ("dito", "dfto", "dfdo", "dfd")
NODE_BOUNDS = ("box", "sphere_rect")
PAIR_ORDERS = ("tree", "far_first")
TRAVERSALS = ("level", "depth_first")


class Result:
    pass


class CertificationError(AssertionError):
    """A replayed choice that the error bounds do not admit."""


def dualtree(xq, xr, w, hs, eps, leaf_size=64, plimit=None, eps_round_share=0.1,
             method="dito", mono=None, trace=False, fmm_mask=7, replay=None,
             record_feasible=False, node_bounds="box", pair_order="tree", traversal="level",
             ledger=False):
    """G~ of shape (n_h, M) in query order, plus the trees and (optionally) the
    decision trace: a list of (h_index, level, Q, R, code, p) tuples.

    replay: {(h_index, level, Q, R): (code, p)} of another run's decisions.
    Where bestMethod is reached, the recorded choice replaces the cost rule of
    Figure 6, after a check with this oracle's own bounds: a series method
    must be admitted (its bound meets maxerr) at exactly the recorded order,
    the smallest that does; otherwise CertificationError.  The token book is
    kept as for any choice, so the run reproduces the other run's pair lists
    when, and only when, its bookkeeping matches.
    record_feasible: keep {(h_index, level, Q, R): {method: p}} of the
    smallest admitted order of every series method wherever bestMethod is
    reached (res.feasible).
    node_bounds: "box" (section 5: distances between bounding boxes) or
    "sphere_rect" (the tighter of the box and the bounding-ball bounds,
    bounds.sphere_rect_dist2).
    pair_order: the order in which a query node's reference list is walked
    (and its lower bound summed): "tree" (left to right, the order of the
    depth-first recursion of Figure 1) or "far_first" (a best-first order in
    the spirit of the priority-queue traversal the paper mentions: decreasing
    dmin^2, ties by R, so that the cheap far prunings deposit their tokens
    before the near pairs ask for them).
    traversal: "level" (the frontier mode above, which the library follows)
    or "depth_first" (paper mode: the recursion of Figures 1 and 7 in its
    printed order, _depth_first_decisions; no replay, no feasibility log).
    ledger: keep res.ledger, one row (h_index, Q, R, code, E, L, W_R, t) per
    resolved pair: the error bound E its resolution spends (the finite
    difference or series bound; 0 for a base case), the lower bound L on G
    over Q that the decision used, W_R, and the token left at Q afterwards.
    The token rule's soundness is checked from these rows alone: per query
    point and bandwidth, the sum over the pairs covering it of
    W E / (eps_alg L) - W_R is at most 0 (Theorem 2's budget).
    method: "dito" (O(D^p) expansions and tokens), "dfto" (O(p^D) expansions
    and tokens, with the bounds of bounds.e_*_tensor; box bounds only),
    "dfdo" (finite differences and tokens), "dfd" (finite differences, local
    rule)."""
    xr = np.atleast_2d(np.asarray(xr, dtype=np.float64))
    if mono is None:
        mono = xq is xr
    xq = xr if mono else np.atleast_2d(np.asarray(xq, dtype=np.float64))
    w = np.asarray(w, dtype=np.float64)
    hs = np.atleast_1d(np.asarray(hs, dtype=np.float64))
    if method not in METHODS:
        raise ValueError(method)
    if node_bounds not in NODE_BOUNDS:
        raise ValueError(node_bounds)
    if pair_order not in PAIR_ORDERS:
        raise ValueError(pair_order)
    if traversal not in TRAVERSALS:
        raise ValueError(traversal)
    if traversal == "depth_first" and (replay is not None or record_feasible or pair_order != "tree"):
        raise ValueError("depth-first mode keeps the tree order and records no feasibility or replay")
    if method == "dfto" and node_bounds != "box":
        raise ValueError("the O(p^D) bounds need box distances")
    D = xr.shape[1]
    family = "tensor" if method == "dfto" else "graded"
    P = plimit if plimit else (plimit_tensor(D) if family == "tensor" else plimit_for(D))
    rt = build_kdtree(xr, w, leaf_size)
    qt = rt if mono else build_kdtree(xq, None, leaf_size)
    if method in ("dito", "dfto"):
        attach_moments(rt, P, family)
    eps_alg = (1.0 - eps_round_share) * eps
    res = Result()
    res.rtree, res.qtree, res.plimit, res.family = rt, qt, P, family
    res.G = np.zeros((len(hs), xq.shape[0]))
    res.trace = [] if trace else None
    res.counts = np.zeros((len(hs), 6), dtype=np.int64)
    res.fmm_mask = fmm_mask
    res.node_bounds = node_bounds
    res.pair_order = pair_order
    res.traversal = traversal
    res.replay = replay
    res.feasible = {} if record_feasible else None
    res.ledger = [] if ledger else None
    res.eps_alg = eps_alg
    for k, h in enumerate(hs):
        res.G[k] = _one_bandwidth(k, float(h), qt, rt, xq, mono, P, eps_alg, method, res)
    return res


def _one_bandwidth(hk, h, qt, rt, xq, mono, P, eps_alg, method, res):
    D = rt.D
    use_tokens = method in ("dito", "dfto", "dfdo")
    use_fmm = method in ("dito", "dfto")
    fam = res.family
    inv_2h2 = 1.0 / (2.0 * h * h)
    inv_4h2 = 0.5 * inv_2h2
    inv_h = 1.0 / h
    Wtot = float(rt.W[0])
    nQ = qt.n_nodes
    C = set_size(D, P, fam)
    Gest = np.zeros(nQ)
    lco = np.zeros((nQ, C))
    pL = np.zeros(nQ, dtype=np.int64)
    work = []  # (code, Q, R, p) in emission order
    segs = [(0, 0.0, 0.0, [0])]
    level = 0
    if res.traversal == "depth_first":
        work = _depth_first_decisions(hk, h, qt, rt, mono, P, eps_alg, method, res, Gest)
        segs = []
    while segs:
        nxt = []
        for Q, t, Lp, Rs in segs:
            qleaf = qt.left[Q] < 0
            dist = []
            for R in Rs:
                if res.node_bounds == "box":
                    dist.append(box_dist2(qt.lo[Q], qt.hi[Q], rt.lo[R], rt.hi[R]))
                else:
                    dist.append(sphere_rect_dist2(qt.lo[Q], qt.hi[Q], rt.lo[R], rt.hi[R], qt.ctr[Q],
                                                  rt.ctr[R], qt.rad[Q], rt.rad[R]))
            if res.pair_order == "far_first":
                order = sorted(range(len(Rs)), key=lambda j: (-dist[j][0], Rs[j]))
                Rs = [Rs[j] for j in order]
                dist = [dist[j] for j in order]
            geo = []
            L = Lp
            for R, (dmin2, dmax2) in zip(Rs, dist):
                kmax = exp64(-dmax2 * inv_2h2)
                geo.append((dmin2, kmax))
                L = L + float(rt.W[R]) * kmax
            if mono and float(qt.wmin[Q]) > L:
                L = float(qt.wmin[Q])
            split = []
            for j, R in enumerate(Rs):
                WR = float(rt.W[R])
                dmin2, kmax = geo[j]
                kmin = exp64(-dmin2 * inv_2h2)
                efd = e_fd(WR, kmin, kmax)
                nd = need(efd, WR, L, Wtot, eps_alg)
                code, p, spent = None, 0, 0.0
                if nd <= (t if use_tokens else 0.0):
                    if use_tokens:
                        t = t - nd
                    Gest[Q] = Gest[Q] + 0.5 * (WR * (kmin + kmax))
                    code, spent = FD, efd
                elif use_fmm:
                    tt = t if use_tokens else 0.0
                    maxerr = ((eps_alg * (WR + tt)) * L) / Wtot
                    g = exp64(-dmin2 * inv_4h2)
                    rQ, rR = float(qt.rinf[Q]) * inv_h, float(rt.rinf[R]) * inv_h
                    key = (hk, level, Q, R)
                    if res.feasible is not None or res.replay is not None:
                        found = feasible_orders(D, P, maxerr, WR, g, rQ, rR, res.fmm_mask, fam)
                        if res.feasible is not None:
                            res.feasible[key] = {n: found[n][0] for n in found}
                    if res.replay is not None:
                        rc, rp = res.replay[key]
                        if rc in (DH, DL, H2L):
                            name = NAME[rc]
                            if name not in found or found[name][0] != rp:
                                raise CertificationError(
                                    "pair %s: %s at order %d is not admitted (smallest "
                                    "admitted: %s)" % (key, name, rp, found.get(name)))
                            p, E = found[name]
                        elif rc in (BASE, SPLIT):
                            name, p, E = "DIRECT", 0, math.inf
                        else:
                            raise CertificationError("pair %s: code %d at bestMethod" % (key, rc))
                    else:
                        name, p, E = best_method(D, P, maxerr, WR, g, rQ, rR,
                                                 int(qt.count[Q]), int(rt.count[R]),
                                                 mask=res.fmm_mask, family=fam)
                    if name != "DIRECT":
                        if use_tokens:
                            t = t - need(E, WR, L, Wtot, eps_alg)
                        code, spent = CODE[name], E
                    else:
                        p = 0
                if code is None:
                    if qleaf and rt.left[R] < 0:
                        if use_tokens:
                            t = t + WR
                        code = BASE
                    else:
                        code = SPLIT
                if code == SPLIT:
                    split.append(R)
                else:
                    if res.ledger is not None:
                        res.ledger.append((hk, Q, R, code, spent, L, WR, t))
                    Lp = Lp + WR * kmax
                    if code != FD:
                        work.append((code, Q, R, p))
                res.counts[hk, code] += 1
                if res.trace is not None:
                    res.trace.append((hk, level, Q, R, code, p))
            if split:
                newR = []
                for R in split:
                    if rt.left[R] < 0:
                        newR.append(R)
                    else:
                        newR.extend((int(rt.left[R]), int(rt.left[R]) + 1))
                if qleaf:
                    nxt.append((Q, t, Lp, newR))
                else:
                    l = int(qt.left[Q])
                    nxt.append((l, t, Lp, list(newR)))
                    nxt.append((l + 1, t, Lp, list(newR)))
        segs = nxt
        level += 1

    return _execute(h, qt, rt, xq, D, fam, work, Gest, lco, pL)


def _execute(h, qt, rt, xq, D, fam, work, Gest, lco, pL):
    """Runs the recorded work (base cases, DH, DL, H2L), then the post-pass of
    Figure 8; returns G~ for every query in input order."""
    nQ = qt.n_nodes
    # Execute the recorded work.
    M = xq.shape[0]
    gx = np.zeros(M)
    gdh = np.zeros(M)
    xr, w = rt.x, rt.w
    for code, Q, R, p in work:
        qpts = qt.perm[qt.begin[Q]:qt.end[Q]]
        rpts = rt.perm[rt.begin[R]:rt.end[R]]
        if code == BASE:
            d2 = np.zeros((len(qpts), len(rpts)))
            for d in range(D):
                diff = xq[qpts, d][:, None] - xr[rpts, d][None, :]
                d2 += diff * diff
            gx[qpts] += np.exp(-d2 / (2.0 * h * h)) @ w[rpts]
        elif code == DH:
            A = scale_moments(rt.moments[R], D, p, h, fam)
            gdh[qpts] += eval_hermite(A, p, rt.ctr[R], xq[qpts], h, fam)
        elif code == DL:
            lco[Q, :set_size(D, p, fam)] += direct_local(xr[rpts], w[rpts], p, qt.ctr[Q], h, fam)
            pL[Q] = max(pL[Q], p)
        elif code == H2L:
            A = scale_moments(rt.moments[R], D, p, h, fam)
            lco[Q, :set_size(D, p, fam)] += h2l(A, p, rt.ctr[R], qt.ctr[Q], h, fam)
            pL[Q] = max(pL[Q], p)

    # Post-pass (Figure 8), top down in breadth-first node order.
    G = np.zeros(M)
    for Q in range(nQ):
        if qt.left[Q] >= 0:
            for c in (int(qt.left[Q]), int(qt.left[Q]) + 1):
                Gest[c] = Gest[c] + Gest[Q]
                if pL[Q] > 0:
                    n = set_size(D, pL[Q], fam)
                    lco[c, :n] += l2l(lco[Q, :n], pL[Q], qt.ctr[Q], qt.ctr[c], h, fam)
                    pL[c] = max(pL[c], pL[Q])
        else:
            qpts = qt.perm[qt.begin[Q]:qt.end[Q]]
            val = gx[qpts] + gdh[qpts] + Gest[Q]
            if pL[Q] > 0:
                val = val + eval_local(lco[Q], pL[Q], qt.ctr[Q], xq[qpts], h, fam)
            G[qpts] = val
    return G


def _depth_first_decisions(hk, h, qt, rt, mono, P, eps_alg, method, res, Gest):
    """Paper mode: the node pairs in the depth-first order of Figure 1 (for a
    pair that is neither approximated nor a base case: (Q.l,R.l), (Q.l,R.r),
    (Q.r,R.l), (Q.r,R.r), or the two pairs of the internal node when the other
    is a leaf), each decided as in Figure 7.  Returns the work list; fills
    Gest and the trace like the frontier mode.

    Readings (Figure 7 leaves the bookkeeping open):
      * a token is a per-query-point budget (proof of Theorem 2), and Q's slot
        Q.W_T must be what every point of Q can still spend.  Each query node
        keeps the sum of the token changes of its own decisions (deposits
        positive, spendings negative); a point's remaining budget is the sum
        of these over the nodes on its root-to-leaf path.  Q's slot is the
        smallest of these over Q's points: the sum over Q and its ancestors,
        plus the least that the decisions below Q have added on any path
        (a node's value is refreshed as the minimum over its children, so a
        spending in a child is seen by every later decision at its
        ancestors, and a spending at an ancestor by every later decision in
        the child).  Nothing is spent twice;
      * G_Q^min is the sum of W_R K(dmax) over the reference nodes resolved at
        Q or an ancestor and over the pairs still pending (on the recursion
        stack) at Q or an ancestor, each with the query node it was formed
        with, in a fixed order; reference nodes resolved only at descendants
        of Q are left out, so the bound is valid for every point of Q (looser
        than it could be, never above G);
      * monochromatic self bound, tokens, maxerr, costs and ties as in the
        frontier mode.
    The trace's level field holds the recursion depth of the pair."""
    D = rt.D
    use_tokens = method in ("dito", "dfto", "dfdo")
    use_fmm = method in ("dito", "dfto")
    fam = res.family
    inv_2h2 = 1.0 / (2.0 * h * h)
    inv_4h2 = 0.5 * inv_2h2
    inv_h = 1.0 / h
    Wtot = float(rt.W[0])
    parent = {}
    for Q in range(qt.n_nodes):
        if qt.left[Q] >= 0:
            parent[int(qt.left[Q])] = Q
            parent[int(qt.left[Q]) + 1] = Q

    def ancestors(Q):
        out = [Q]
        while out[-1] in parent:
            out.append(parent[out[-1]])
        return out[::-1]  # root first

    def dist2(Q, R):
        if res.node_bounds == "box":
            return box_dist2(qt.lo[Q], qt.hi[Q], rt.lo[R], rt.hi[R])
        return sphere_rect_dist2(qt.lo[Q], qt.hi[Q], rt.lo[R], rt.hi[R], qt.ctr[Q], rt.ctr[R], qt.rad[Q],
                                 rt.rad[R])

    own = {}        # Q -> sum of the token changes of Q's own decisions
    below = {}      # Q -> min over Q's children c of own[c] + below[c]

    def token(Q):
        v = below.get(Q, 0.0)
        for A in ancestors(Q):
            v = v + own.get(A, 0.0)
        return v

    def book(Q, delta):
        own[Q] = own.get(Q, 0.0) + delta
        A = Q
        while A in parent:
            A = parent[A]
            l = int(qt.left[A])
            below[A] = min(own.get(l, 0.0) + below.get(l, 0.0), own.get(l + 1, 0.0) + below.get(l + 1, 0.0))

    resolved = {}   # Q -> list of W_R K(dmax) of pairs resolved at Q, in order
    pending = {}    # Q -> {R: W_R K(dmax)} of pairs on the stack
    work = []

    def push(Q, R, depth, stack):
        dmin2, dmax2 = dist2(Q, R)
        pending.setdefault(Q, {})[R] = float(rt.W[R]) * exp64(-dmax2 * inv_2h2)
        stack.append((Q, R, depth, dmin2, dmax2))

    stack = []
    push(0, 0, 0, stack)
    while stack:
        Q, R, depth, dmin2, dmax2 = stack.pop()
        L = 0.0
        for A in ancestors(Q):
            for v in resolved.get(A, ()):
                L = L + v
            for R2 in sorted(pending.get(A, {})):
                L = L + pending[A][R2]
        if mono and float(qt.wmin[Q]) > L:
            L = float(qt.wmin[Q])
        bound = pending[Q].pop(R)
        t = token(Q)
        WR = float(rt.W[R])
        kmax = exp64(-dmax2 * inv_2h2)
        kmin = exp64(-dmin2 * inv_2h2)
        efd = e_fd(WR, kmin, kmax)
        nd = need(efd, WR, L, Wtot, eps_alg)
        code, p, spent, delta = None, 0, 0.0, 0.0
        if nd <= (t if use_tokens else 0.0):
            delta = -nd
            Gest[Q] = Gest[Q] + 0.5 * (WR * (kmin + kmax))
            code, spent = FD, efd
        elif use_fmm:
            tt = t if use_tokens else 0.0
            maxerr = ((eps_alg * (WR + tt)) * L) / Wtot
            g = exp64(-dmin2 * inv_4h2)
            rQ, rR = float(qt.rinf[Q]) * inv_h, float(rt.rinf[R]) * inv_h
            name, p, E = best_method(D, P, maxerr, WR, g, rQ, rR, int(qt.count[Q]), int(rt.count[R]),
                                     mask=res.fmm_mask, family=fam)
            if name != "DIRECT":
                delta = -need(E, WR, L, Wtot, eps_alg)
                code, spent = CODE[name], E
            else:
                p = 0
        qleaf, rleaf = qt.left[Q] < 0, rt.left[R] < 0
        if code is None:
            if qleaf and rleaf:
                delta = WR
                code = BASE
            else:
                code = SPLIT
        if use_tokens and code != SPLIT:
            book(Q, delta)
            t = token(Q)
        res.counts[hk, code] += 1
        if res.trace is not None:
            res.trace.append((hk, depth, Q, R, code, p))
        if code != SPLIT:
            if res.ledger is not None:
                res.ledger.append((hk, Q, R, code, spent, L, WR, t))
            resolved.setdefault(Q, []).append(bound)
            if code != FD:
                work.append((code, Q, R, p))
            continue
        if qleaf:
            kids = [(Q, int(rt.left[R])), (Q, int(rt.left[R]) + 1)]
        elif rleaf:
            kids = [(int(qt.left[Q]), R), (int(qt.left[Q]) + 1, R)]
        else:
            ql, rl = int(qt.left[Q]), int(rt.left[R])
            kids = [(ql, rl), (ql, rl + 1), (ql + 1, rl), (ql + 1, rl + 1)]
        for Qc, Rc in reversed(kids):
            push(Qc, Rc, depth + 1, stack)
    return work
