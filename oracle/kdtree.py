"""kd-tree with cached sufficient statistics (section 6 and Figure 5).

The paper builds its trees by recursively partitioning a node's points into two
(Figure 5) once a node holds more than a leaf threshold of points, caching
per-node statistics.  It leaves the split rule and the threshold open; this
implementation's reading is:

  * a node with n <= leaf_size points is a leaf;
  * otherwise it is split on the dimension of widest bounding-box extent
    (ties to the smallest dimension index); the node's points are ordered by
    (coordinate in that dimension, original index) and the left child takes
    the first n_left = leaf_size * ceil(n / (2 leaf_size)) (half of n rounded
    up to a multiple of leaf_size), the right child the rest, so that all
    leaves but one hold exactly leaf_size points;
  * nodes are numbered breadth first, level by level, left child before right;
  * the points of every node occupy a contiguous range [begin, end) of the
    permutation `perm`; inside a leaf the points are in increasing original
    index.

Cached per node: the exact bounding box lo/hi, the centre ctr = (lo+hi)/2
(the reading of "centroid" used by the bounds: the box centre minimises the
max-norm radius), rinf = max over points of |x - ctr|_inf, the weight sum W
(leaves: sequential sum in `perm` order; internal: W_left + W_right), the
smallest weight wmin, and the point count.  Raw Hermite moments are attached by
`attach_moments` (Figure 5: buildLeaf computes them from the points,
buildInternal by H2H from the children).

Pinned by tests/test_oracle_tree.py: brute-force box/radius/weight checks,
leaf-aligned split property, permutation invariance of the tree geometry.
"""

import math

import numpy as np

from .multiindex import set_size
from .series import h2h, raw_moments


class KDTree:
    pass


def build_kdtree(x, w, leaf_size):
    x = np.asarray(x, dtype=np.float64)
    n_pts, D = x.shape
    w = np.ones(n_pts) if w is None else np.asarray(w, dtype=np.float64)
    nodes_pts = [np.arange(n_pts)]       # point set per node (original indices)
    begin = [0]
    left = []
    depth = [0]
    level = [0]
    head = 0
    # Breadth-first construction: process nodes in id order; children are
    # appended, which numbers them level by level, left before right.
    while head < len(nodes_pts):
        pts = nodes_pts[head]
        n = len(pts)
        if n <= leaf_size:
            left.append(-1)
        else:
            xs = x[pts]
            ext = xs.max(axis=0) - xs.min(axis=0)
            dstar = int(np.argmax(ext))          # first maximum -> smallest d
            order = np.lexsort((pts, xs[:, dstar]))  # by (x_dstar, index)
            srt = pts[order]
            half = leaf_size * ((n + 2 * leaf_size - 1) // (2 * leaf_size))
            left.append(len(nodes_pts))
            for child, b in ((srt[:half], begin[head]), (srt[half:], begin[head] + half)):
                nodes_pts.append(child)
                begin.append(b)
                depth.append(depth[head] + 1)
        head += 1
    nn = len(nodes_pts)
    t = KDTree()
    t.D = D
    t.n_nodes = nn
    t.leaf_size = leaf_size
    t.begin = np.array(begin, dtype=np.int64)
    t.count = np.array([len(p) for p in nodes_pts], dtype=np.int64)
    t.end = t.begin + t.count
    t.left = np.array(left, dtype=np.int64)
    t.depth = np.array(depth, dtype=np.int64)
    perm = np.empty(n_pts, dtype=np.int64)
    for i in range(nn):
        if t.left[i] < 0:
            perm[t.begin[i]:t.end[i]] = np.sort(nodes_pts[i])
    t.perm = perm
    t.lo = np.empty((nn, D))
    t.hi = np.empty((nn, D))
    t.ctr = np.empty((nn, D))
    t.rinf = np.empty(nn)
    t.rad = np.empty(nn)
    t.W = np.empty(nn)
    t.wmin = np.empty(nn)
    for i in range(nn):
        pts = perm[t.begin[i]:t.end[i]]
        xs = x[pts]
        t.lo[i] = xs.min(axis=0)
        t.hi[i] = xs.max(axis=0)
        t.ctr[i] = 0.5 * (t.lo[i] + t.hi[i])
        t.rinf[i] = float(np.max(np.abs(xs - t.ctr[i])))
        # Euclidean radius about the box centre: squares summed in d order
        s2 = np.zeros(len(pts))
        for d in range(D):
            diff = xs[:, d] - t.ctr[i, d]
            s2 = s2 + diff * diff
        t.rad[i] = math.sqrt(float(np.max(s2)))
        t.wmin[i] = float(np.min(w[pts]))
    for i in range(nn - 1, -1, -1):
        if t.left[i] < 0:
            s = 0.0
            for j in perm[t.begin[i]:t.end[i]]:
                s = s + float(w[j])
            t.W[i] = s
        else:
            t.W[i] = t.W[t.left[i]] + t.W[t.left[i] + 1]
    t.x = x
    t.w = w
    return t


def is_leaf(t, i):
    return t.left[i] < 0


def attach_moments(t, p, family="graded"):
    """Raw Hermite moments of order p for every node (Figure 5): leaves from
    their points, internal nodes by H2H of both children (Lemma 2).  family:
    the index set of the expansions (multiindex.index_set)."""
    C = set_size(t.D, p, family)
    M = np.zeros((t.n_nodes, C))
    for i in range(t.n_nodes - 1, -1, -1):
        if t.left[i] < 0:
            pts = t.perm[t.begin[i]:t.end[i]]
            M[i] = raw_moments(t.x[pts], t.w[pts], t.ctr[i], p, family)
        else:
            l = t.left[i]
            M[i] = (h2h(M[l], t.ctr[l], t.ctr[i], t.D, p, family)
                    + h2h(M[l + 1], t.ctr[l + 1], t.ctr[i], t.D, p, family))
    t.moments = M
    t.moment_order = p
    return M
