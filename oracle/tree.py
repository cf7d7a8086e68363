"""4D space-time box cluster tree and its lists (oracle, test-only).

Algorithm 1 (Section 3.2) with these readings of points the paper leaves open:

* root: the bounding box of the surface made cubic about its centre, closed;
  time interval [t_0, t_E];
* a box is refined iff it holds >= n_max elements and its interval has more
  than one time step (early stop);
* refinement type per level l: temporal iff
      hx(l)^2 / (4 alpha ht(l+1)) <= c_st,   ht(l+1) = T / 2^(l+2),
  with hx(l) the unpadded spatial half-size (eq. rel_h_t_h_x);
* temporal split: the middle time node; for an odd number of steps the two
  nodes around the midpoint tie and the earlier one is taken;
* spatial split: uniform octants; an element belongs to the child containing
  its centroid (triangle centroid, step midpoint), points on a split plane
  going to the lower child;
* padding (Section 3.2, after Algorithm 1): per level, the largest overhang
  of a member triangle beyond its unpadded box, then made monotone from fine
  to coarse; overhangs below 1e-12 of the root half-size count as zero;
* numbering: the index of an interval at level l is 2 * parent + child bit,
  and the spatial grid index of an octant is 2 * parent + octant bit per axis.

Lists (Section 3.3):
* temporal nearfield / interaction list, eq. 03:ILtemp;
* interaction area: grid distance (max norm of index differences) <= n_tr,
  eq. 03:Iarea (n_tr = -1: no spatial cut);
* space-time lists, eqs. def_st_nearfield and def_st_interaction_list.

Parity: pinned by the paper's worked example of the temporal lists, by an
exact coverage check (with n_tr = -1 every causal element pair lies in
exactly one nearfield block or one admissible block) and by invariants of
the padded tree (children inside parents).
"""
import numpy as np


class Box:
    __slots__ = ("id", "level", "ix", "k", "s0", "s1", "tris", "parent", "children", "leaf")

    def __init__(self, level, ix, k, s0, s1, tris, parent):
        self.level, self.ix, self.k, self.s0, self.s1 = level, ix, k, s0, s1
        self.tris, self.parent = tris, parent
        self.children = []
        self.leaf = True
        self.id = -1

    @property
    def n_elements(self):
        return (self.s1 - self.s0) * len(self.tris)


class Tree:
    def __init__(self, verts, tris, time_nodes, alpha=1.0, n_max=64, c_st=0.9, n_tr=5):
        self.verts = np.asarray(verts, dtype=np.float64)
        self.tri = np.asarray(tris, dtype=np.int64)
        self.t = np.asarray(time_nodes, dtype=np.float64)
        self.E_t = len(self.t) - 1
        self.E_x = len(self.tri)
        self.alpha, self.n_max, self.c_st, self.n_tr = alpha, n_max, c_st, n_tr
        P = self.verts[self.tri]
        self.centroids = (P[:, 0] + P[:, 1] + P[:, 2]) / 3.0
        lo, hi = self.verts.min(0), self.verts.max(0)
        self.center = 0.5 * (lo + hi)
        self.h0 = 0.5 * float((hi - lo).max())
        self.lo0 = self.center - self.h0
        self.T = float(self.t[-1] - self.t[0])
        h = np.diff(self.t)
        self.uniform = bool(np.all(np.abs(h - self.T / self.E_t) <= 1e-12 * self.T / self.E_t))
        self._build()
        self._pad()
        self._temporal_tree()

    # ------------------------------------------------------------ Algorithm 1
    def _split(self, s0, s1):
        """Split node of the steps [s0, s1): the node nearest to the time
        midpoint (the midpoint itself when it is a node), the earlier of two
        nodes equally near (within 1e-12 T)."""
        tm = 0.5 * (self.t[s0] + self.t[s1])
        d = np.abs(self.t[s0 + 1:s1] - tm)
        return s0 + 1 + int(np.nonzero(d <= d.min() + 1e-12 * self.T)[0][0])

    def _build(self):
        root = Box(0, (0, 0, 0), 0, 0, self.E_t, np.arange(self.E_x), None)
        self.levels = [[root]]
        self.lx = [0]          # spatial refinements at each level
        self.rtype = []        # refinement type of level l -> l+1
        l = 0
        while True:
            hx = self.h0 / 2 ** self.lx[l]
            ht_next = self.T / 2 ** (l + 2)
            temporal = hx * hx / (4.0 * self.alpha * ht_next) <= self.c_st
            nxt = []
            for b in self.levels[l]:
                if b.n_elements < self.n_max or b.s1 - b.s0 <= 1:
                    continue
                b.leaf = False
                mid = self._split(b.s0, b.s1)
                halves = ((b.s0, mid, 2 * b.k), (mid, b.s1, 2 * b.k + 1))
                if temporal:
                    for s0, s1, k in halves:
                        c = Box(l + 1, b.ix, k, s0, s1, b.tris, b)
                        b.children.append(c)
                        nxt.append(c)
                else:
                    hxc = hx  # half-size of the parent = edge length of a child
                    lo = self.lo0 + np.array(b.ix) * (2.0 * hx)
                    midp = lo + hxc
                    cen = self.centroids[b.tris]
                    bits = (cen > midp[None, :]).astype(np.int64)
                    code = bits[:, 0] * 4 + bits[:, 1] * 2 + bits[:, 2]
                    for s0, s1, k in halves:
                        for oc in range(8):
                            sel = b.tris[code == oc]
                            if len(sel) == 0:
                                continue
                            ob = ((oc >> 2) & 1, (oc >> 1) & 1, oc & 1)
                            ix = tuple(2 * b.ix[j] + ob[j] for j in range(3))
                            c = Box(l + 1, ix, k, s0, s1, sel, b)
                            b.children.append(c)
                            nxt.append(c)
            if not nxt:
                break
            self.rtype.append("t" if temporal else "st")
            self.lx.append(self.lx[l] + (0 if temporal else 1))
            self.levels.append(nxt)
            l += 1
        self.depth = len(self.levels) - 1
        self.boxes = [b for lev in self.levels for b in lev]
        for i, b in enumerate(self.boxes):
            b.id = i
        self.index = [{(b.ix, b.k): b for b in lev} for lev in self.levels]
        self.leaves = [b for b in self.boxes if b.leaf]

    # ------------------------------------------------------------ padding
    def _pad(self):
        P = self.verts[self.tri]
        pad = []
        for l, lev in enumerate(self.levels):
            hx = self.h0 / 2 ** self.lx[l]
            p = 0.0
            for b in lev:
                lo = self.lo0 + np.array(b.ix) * (2.0 * hx)
                hi = lo + 2.0 * hx
                V = P[b.tris].reshape(-1, 3)
                over = np.maximum(np.maximum(lo[None, :] - V, V - hi[None, :]), 0.0)
                p = max(p, float(over.max()) if over.size else 0.0)
            pad.append(p if p >= 1e-12 * self.h0 else 0.0)
        for l in range(len(pad) - 2, -1, -1):
            pad[l] = max(pad[l], pad[l + 1])
        self.pad = pad

    def hx_nominal(self, l):
        return self.h0 / 2 ** self.lx[l]

    def hx_padded(self, l):
        return self.hx_nominal(l) + self.pad[l]

    def box_lower(self, b):
        """Lower corner of the padded spatial box."""
        l = b.level
        return self.lo0 + np.array(b.ix) * (2.0 * self.hx_nominal(l)) - self.pad[l]

    def interval(self, b):
        return self.t[b.s0], self.t[b.s1]

    # ------------------------------------------------------------ temporal tree
    def _temporal_tree(self):
        self.tI = [set(b.k for b in lev) for lev in self.levels]
        self.tI_leaf = []
        for l in range(len(self.levels)):
            nxt = self.tI[l + 1] if l + 1 < len(self.levels) else set()
            self.tI_leaf.append({k for k in self.tI[l] if (2 * k) not in nxt and (2 * k + 1) not in nxt})

    def temporal_nearfield(self, l, k):
        """N(I_k^(l)) as a set of (level, index), eq. 03:ILtemp."""
        if k == 0:
            return {(l, 0)}
        out = {(l, j) for j in (k - 1, k) if j in self.tI[l]}
        par = self.temporal_nearfield(l - 1, k // 2)
        out |= {(lp, kp) for (lp, kp) in par if kp in self.tI_leaf[lp]}
        return out

    def temporal_interaction(self, l, k):
        """I(I_k^(l)) as a set of indices at level l, eq. 03:ILtemp."""
        if k < 2:
            return set()
        cand = (k - 2,) if k % 2 == 0 else (k - 3, k - 2)
        return {j for j in cand if j in self.tI[l]}

    # ------------------------------------------------------------ space-time lists
    def grid_close(self, ix, iy):
        if self.n_tr < 0:
            return True
        return max(abs(ix[j] - iy[j]) for j in range(3)) <= self.n_tr

    def _same_level(self, b, ks):
        out = []
        lev = self.levels[b.level]
        for c in lev:
            if c.k in ks and self.grid_close(b.ix, c.ix):
                out.append(c)
        return out

    def nearfield(self, b, _memo=None):
        """N(Z), eq. def_st_nearfield, as a list of boxes."""
        if _memo is None:
            _memo = {}
        if b.id in _memo:
            return _memo[b.id]
        ks = {k for k in ((b.k - 1, b.k) if b.k > 0 else (0,)) if k in self.tI[b.level]}
        out = self._same_level(b, ks)
        if b.parent is not None:
            ids = {c.id for c in out}
            for c in self.nearfield(b.parent, _memo):
                if c.leaf and c.id not in ids:
                    out.append(c)
                    ids.add(c.id)
        _memo[b.id] = out
        return out

    def interaction(self, b):
        """I(Z), eq. def_st_interaction_list, as a list of boxes."""
        ks = self.temporal_interaction(b.level, b.k)
        if not ks:
            return []
        return self._same_level(b, ks)

    # ------------------------------------------------------------ elements
    def elements(self, b):
        """Natural indices j_t * E_x + j_x of the elements of box b (time-major)."""
        st = np.arange(b.s0, b.s1)
        return (st[:, None] * self.E_x + b.tris[None, :]).ravel()

    def leaf_of_element(self):
        """Map natural element index -> leaf box."""
        out = np.empty(self.E_t * self.E_x, dtype=np.int64)
        for b in self.leaves:
            out[self.elements(b)] = b.id
        return out

    def ancestors(self, b):
        chain = []
        while b is not None:
            chain.append(b)
            b = b.parent
        return chain[::-1]
