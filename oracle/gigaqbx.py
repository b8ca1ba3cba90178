"""Tier B oracle: the GIGAQBX FMM (Algorithm 5) as plain steps.  TEST INFRASTRUCTURE ONLY.

Stage 1 (tree) and the interaction lists are written straight from Section 5.2's
definitions, box by box, with no spatial hashing or recursion tricks shared with the
library.  Readings taken where the paper is silent (each is listed in the design notes):

  * Root box: the smallest cube holding every source, center, target and expansion ball
    (Section 5.2.1), with half-width rounded up to a power of two and center on a multiple
    of it, so that every box center and radius is an exact binary fraction.
  * Particles go to the upper child along an axis when their coordinate is >= the box
    center (half-open cells).
  * Sources, centers and targets all count toward nmax; a box splits while it owns more
    than nmax particles and at least one particle would move; at most 30 levels.
  * A center moves to the child containing it iff its ball fits in that child's target
    confinement region: |c - x_child|_2 + r_c <= sqrt(3)|child|(1 + t_f).
  * a < TCR(b):  |x_a - x_b|_2 - sqrt(3)|b|(1+t_f) >= 3|a|;
    TCR(a) < b:  |x_a - x_b|_inf - |b| >= 3|a|(1+t_f)  (both inclusive, the paper's
    'at least').
  * T_b and k-colleagues exclude b itself; 'descendants' in List 3 are strict.
  * Adjacent: the closed cubes touch and neither contains the other.
  * List entries are restricted to boxes whose subtree holds at least one source (others
    contribute nothing); leaf entries (Lists 1, 3close, 4) must own sources.
  * Targets associated with centers are evaluated only through their centers (Stage 9's
    second loop); a box is a target box when it owns at least one center.
  * Remark 4 (optional, parameter wfar_direct_max, 0 = off): a List 3 far box whose
    subtree holds at most that many sources is removed from List 3 far and its source
    leaves are added to List 3 close.
  * The l_inf target confinement region of the earlier two-dimensional algorithm, used for
    the cost comparison of Section 6 (parameter tcr_norm="linf"): TCR(b) is the closed box
    of half-width |b|(1 + t_f) about x_b; a center moves to a child iff
    |c - x_child|_inf + r_c <= |child|(1 + t_f); and a < TCR(b) iff the l_inf distance from
    x_a to the boundary of TCR(b) is at least 3|a|: |x_a - x_b|_inf - |b|(1+t_f) >= 3|a|.

Numerical steps in the order of Algorithm 5 (all coefficients complex, paper form):
  Stage 2: multipole of every needed box.  M2M of an order-p multipole is exact for the
    degrees it keeps, so the oracle forms each box's multipole directly from the sources of
    its subtree, which equals the leaf P2M + upward M2M chain (a pin test checks the
    oracle's own M2M against this identity).
  Stages 3, 5a, 6a: order-p_qbx local at each center from the sources of U, W-close and
    X-close of its box (direct).
  Stage 4: box local (order p_fmm) from the V list by M2L.
  Stage 5b: QBX local from each W-far multipole by M2L (order p_fmm -> p_qbx).
  Stage 6b: box local from the sources of X-far by direct P2L (order p_fmm).
  Stages 7-8: an order-p L2L is exact for the polynomial it represents, so the downward
    chain followed by the L2QBXL equals the sum over the box and its ancestors a of the
    direct L2L of a's own local (V and X-far parts) to the center (p_fmm -> p_qbx).
  Stage 9: each target evaluates its center's QBX local.
"""

from __future__ import annotations

import math

import numpy as np

from . import KERNELS, _f64, _i64, _p, eval_local, eval_mpole, lib, ncoef, strengths
from . import m2l as _m2l_one

SQRT3 = math.sqrt(3.0)
MAX_LEVEL = 30
LIST_NAMES = ("U", "V", "Wclose", "Wfar", "Xclose", "Xfar")


def _dyadic_root(lo, hi):
    ext = float(np.max(hi - lo))
    k = int(math.ceil(math.log2(max(ext, 1e-300) / 2.0))) - 2
    while True:
        h = 2.0 ** k
        x0 = np.empty(3)
        ok = True
        for a in range(3):
            j = math.floor(lo[a] / h) + 1.0
            if not (hi[a] <= (j + 1.0) * h):
                ok = False
                break
            x0[a] = j * h
        if ok:
            return x0, h
        k += 1


class OracleTree:
    """Stage 1: octree with target-confinement-restricted centers."""

    def __init__(self, src, ctr, crad, tgt, nmax, tcf, tcr_norm="l2", level_restrict=False):
        src, ctr, crad, tgt = _f64(src), _f64(ctr), _f64(crad), _f64(tgt)
        self.tcf = float(tcf)
        if tcr_norm not in ("l2", "linf"):
            raise ValueError(tcr_norm)
        self.linf = tcr_norm == "linf"
        self.nmax = int(nmax)
        lo = np.minimum(np.minimum(src.min(0), tgt.min(0)), (ctr - crad[:, None]).min(0))
        hi = np.maximum(np.maximum(src.max(0), tgt.max(0)), (ctr + crad[:, None]).max(0))
        x0, h0 = _dyadic_root(lo, hi)
        centers, halfw, level, parent, children = [x0], [h0], [0], [-1], [[]]
        own_s = [np.arange(src.shape[0])]
        own_c = [np.arange(ctr.shape[0])]
        own_t = [np.arange(tgt.shape[0])]
        def split(b):
            """Subdivide box b by the Stage 1 rule; returns the new children (none if
            nothing would move)."""
            xb, hb = centers[b], halfw[b]
            hc = hb * 0.5

            def octant(P):
                return ((P[:, 0] >= xb[0]).astype(np.int64)
                        + 2 * (P[:, 1] >= xb[1]).astype(np.int64)
                        + 4 * (P[:, 2] >= xb[2]).astype(np.int64))

            def child_center(o):
                return xb + hc * np.array([1.0 if o & 1 else -1.0,
                                           1.0 if o & 2 else -1.0,
                                           1.0 if o & 4 else -1.0])

            os_ = octant(src[own_s[b]])
            ot_ = octant(tgt[own_t[b]])
            oc_ = octant(ctr[own_c[b]])
            cc = np.array([child_center(o) for o in range(8)])
            cpos = ctr[own_c[b]]
            d = cpos - cc[oc_]
            if self.linf:
                dist = np.max(np.abs(d), axis=1)
                fits = dist + crad[own_c[b]] <= hc * (1.0 + self.tcf)
            else:
                dist = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
                fits = dist + crad[own_c[b]] <= (SQRT3 * hc) * (1.0 + self.tcf)
            if len(own_s[b]) + len(own_t[b]) + int(fits.sum()) == 0:
                return []  # subdividing would only produce empty children
            made = []
            for o in range(8):
                s_o = own_s[b][os_ == o]
                t_o = own_t[b][ot_ == o]
                c_o = own_c[b][(oc_ == o) & fits]
                if len(s_o) + len(t_o) + len(c_o) == 0:
                    continue
                cid = len(centers)
                centers.append(cc[o])
                halfw.append(hc)
                level.append(level[b] + 1)
                parent.append(b)
                children.append([])
                children[b].append(cid)
                own_s.append(s_o)
                own_t.append(t_o)
                own_c.append(c_o)
                made.append(cid)
            own_s[b] = own_s[b][:0]
            own_t[b] = own_t[b][:0]
            own_c[b] = own_c[b][~fits]
            return made

        frontier = [0]
        while frontier:
            nxt = []
            for b in frontier:
                n_own = len(own_s[b]) + len(own_c[b]) + len(own_t[b])
                if n_own <= self.nmax or level[b] >= MAX_LEVEL:
                    continue
                nxt += split(b)
            frontier = nxt
        if level_restrict:
            # Level restriction (the remark on List 3 complexity): adjacent leaves may differ
            # by at most one level.  Every pass checks each leaf against the leaves at least
            # two levels finer; one that touches (closed cubes meet) such a leaf is split.
            # A k-d tree in the max norm only narrows the candidates: its radius h_i + h_max
            # (slightly widened) covers every leaf that can touch leaf i, and the exact
            # test below decides.
            from scipy.spatial import cKDTree

            while True:
                leaves = [b for b in range(len(centers)) if not children[b]]
                C = np.array([centers[b] for b in leaves])
                H = np.array([halfw[b] for b in leaves])
                lev = np.array([level[b] for b in leaves])
                kd = cKDTree(C)
                near = kd.query_ball_point(C, (H + H.max()) * (1.0 + 1e-9), p=np.inf)
                todo = []
                for i, b in enumerate(leaves):
                    if level[b] >= MAX_LEVEL:
                        continue
                    j = np.asarray(near[i], dtype=np.int64)
                    j = j[lev[j] >= lev[i] + 2]
                    touch = np.all(np.abs(C[j] - C[i]) <= (H[j] + H[i])[:, None], axis=1)
                    if np.any(touch):
                        todo.append(b)
                made = [c for b in todo for c in split(b)]
                if not made:
                    break
            # breadth-first renumbering, children in octant order (the plain build's order)
            order = [0]
            for b in order:  # the list grows while it is walked
                order += children[b]  # created in octant order
            new = {b: i for i, b in enumerate(order)}
            centers = [centers[b] for b in order]
            halfw = [halfw[b] for b in order]
            level = [level[b] for b in order]
            parent = [-1 if parent[b] < 0 else new[parent[b]] for b in order]
            children = [[new[c] for c in children[b]] for b in order]
            own_s = [own_s[b] for b in order]
            own_c = [own_c[b] for b in order]
            own_t = [own_t[b] for b in order]
        self.center = np.array(centers)
        self.h = np.array(halfw)
        self.level = np.array(level, dtype=np.int64)
        self.parent = np.array(parent, dtype=np.int64)
        self.children = children
        self.own_src, self.own_ctr, self.own_tgt = own_s, own_c, own_t
        nb = len(centers)
        self.nboxes = nb
        self.is_leaf = np.array([len(c) == 0 for c in children])
        self.n_own_src = np.array([len(s) for s in own_s], dtype=np.int64)
        # preorder numbering for ancestor tests, subtree source counts
        self.tin = np.zeros(nb, dtype=np.int64)
        self.tout = np.zeros(nb, dtype=np.int64)
        sub = self.n_own_src.copy()
        order = []
        stack = [(0, False)]
        t = 0
        while stack:
            b, done = stack.pop()
            if done:
                self.tout[b] = t
                continue
            self.tin[b] = t
            t += 1
            order.append(b)
            stack.append((b, True))
            for c in reversed(children[b]):
                stack.append((c, False))
        for b in reversed(order):
            if self.parent[b] >= 0:
                sub[self.parent[b]] += sub[b]
        self.sub_src = sub
        self.preorder = np.array(order, dtype=np.int64)
        self.nlevels = int(self.level.max()) + 1
        self.ctr_owner = np.empty(ctr.shape[0], dtype=np.int64)
        for b in range(nb):
            self.ctr_owner[own_c[b]] = b

    # --- relations ---------------------------------------------------------------------

    def key(self, b):
        """Identity of a box independent of numbering: (level, center)."""
        return (int(self.level[b]),) + tuple(float(x) for x in self.center[b])

    def ancestors(self, b):
        out = []
        a = self.parent[b]
        while a >= 0:
            out.append(int(a))
            a = self.parent[a]
        return out

    def strict_desc_mask(self, a):
        return (self.tin > self.tin[a]) & (self.tout <= self.tout[a])

    def dinf(self, b):
        return np.max(np.abs(self.center - self.center[b]), axis=1)

    def nested_mask(self, b):
        anc = np.zeros(self.nboxes, dtype=bool)
        anc[self.ancestors(b)] = True
        m = self.strict_desc_mask(b) | anc
        m[b] = True
        return m

    def adjacent_mask(self, b):
        return (self.dinf(b) <= self.h + self.h[b]) & ~self.nested_mask(b)

    def adjacent(self, a, b):
        if a == b:
            return False
        if b in self.ancestors(a) or a in self.ancestors(b):
            return False
        return float(np.max(np.abs(self.center[a] - self.center[b]))) <= self.h[a] + self.h[b]

    def colleagues2_mask(self, b):
        m = (self.level == self.level[b]) & (self.dinf(b) <= 4.0 * self.h[b])
        m[b] = False
        return m

    def prec_tcr(self, a, b):
        """a < TCR(b): l2 distance from x_a to the boundary of TCR(b) is at least 3|a|
        (l_inf distance to the box-shaped TCR in the l_inf variant)."""
        if self.linf:
            dinf = float(np.max(np.abs(self.center[a] - self.center[b])))
            return dinf - self.h[b] * (1.0 + self.tcf) >= 3.0 * self.h[a]
        d = self.center[a] - self.center[b]
        dist = math.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
        return dist - (SQRT3 * self.h[b]) * (1.0 + self.tcf) >= 3.0 * self.h[a]

    def tcr_prec(self, a, d):
        """TCR(a) < d: l_inf distance from x_a to the boundary of d is at least 3|a|(1+t_f)."""
        dinf = float(np.max(np.abs(self.center[a] - self.center[d])))
        return dinf - self.h[d] >= (3.0 * self.h[a]) * (1.0 + self.tcf)

    def subtree(self, a):
        m = self.strict_desc_mask(a)
        m[a] = True
        return np.nonzero(m)[0]

    def subtree_sources(self, a):
        boxes = self.subtree(a)
        parts = [self.own_src[b] for b in boxes if self.n_own_src[b] > 0]
        return np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)


class OracleLists:
    """Interaction lists of Section 5.2.3-5.2.4, evaluated lazily per box."""

    def __init__(self, tree: OracleTree, wfar_direct_max: int = 0):
        self.t = tree
        self.wfar_direct_max = int(wfar_direct_max)
        self._cache = {}

    def _get(self, name, b, fn):
        k = (name, b)
        if k not in self._cache:
            self._cache[k] = fn(b)
        return self._cache[k]

    def T(self, b):
        return self._get("T", b, lambda b: set(np.nonzero(self.t.colleagues2_mask(b))[0].tolist()))

    def U(self, b):
        """List 1: leaves among desc(b) and b, plus leaves adjacent to b."""
        def f(b):
            t = self.t
            ds = t.strict_desc_mask(b)
            ds[b] = True
            m = t.is_leaf & (t.n_own_src > 0) & (ds | t.adjacent_mask(b))
            return set(np.nonzero(m)[0].tolist())
        return self._get("U", b, f)

    def V(self, b):
        """List 2: children of the 2-colleagues of b's parent, 2-well-separated from b."""
        def f(b):
            t = self.t
            pb = t.parent[b]
            if pb < 0:
                return set()
            Tp = self.T(int(pb))
            out = set()
            for d in np.nonzero((t.level == t.level[b]) & (t.sub_src > 0))[0]:
                d = int(d)
                if int(t.parent[d]) in Tp and d != b and d not in self.T(b):
                    out.add(d)
            return out
        return self._get("V", b, f)

    def W(self, b):
        """List 3: d in desc(T_b), not adjacent to b, every ancestor of d inside desc(T_b)
        adjacent to b."""
        def f(b):
            t = self.t
            Tb = self.T(b)
            cand = np.zeros(t.nboxes, dtype=bool)
            for a in Tb:
                cand |= t.strict_desc_mask(a)
            out = set()
            for d in np.nonzero(cand & (t.sub_src > 0))[0]:
                d = int(d)
                if t.adjacent(d, b):
                    continue
                ok = True
                w = int(t.parent[d])
                while w not in Tb:
                    if not t.adjacent(w, b):
                        ok = False
                        break
                    w = int(t.parent[w])
                if ok:
                    out.add(d)
            return out
        return self._get("W", b, f)

    def X(self, b):
        """List 4: source leaves d that are 2-colleagues of an ancestor of b, adjacent to
        parent(b) but not to b; or 2-colleagues of b not adjacent to b."""
        def f(b):
            t = self.t
            anc = t.ancestors(b)
            out = set()
            cand = np.nonzero(t.is_leaf & (t.n_own_src > 0))[0]
            Tb = self.T(b)
            for d in cand:
                d = int(d)
                if d in Tb and not t.adjacent(d, b):
                    out.add(d)
                    continue
                if not anc:
                    continue
                if any(d in self.T(a) for a in anc):
                    if t.adjacent(d, int(t.parent[b])) and not t.adjacent(d, b):
                        out.add(d)
            return out
        return self._get("X", b, f)

    def _w_closure(self, b):
        t = self.t
        s = set()
        for d in self.W(b):
            s.update(int(x) for x in t.subtree(d) if t.sub_src[x] > 0)
        return s

    def Wclose(self, b):
        """List 3 close: source leaves in W_b or below that are not d < TCR(b); with
        Remark 4, also the source leaves of the small List 3 far boxes."""
        def f(b):
            t = self.t
            out = {d for d in self._w_closure(b)
                   if t.is_leaf[d] and t.n_own_src[d] > 0 and not t.prec_tcr(d, b)}
            for d in self._wfar_def(b):
                if self._moved(d):
                    out |= {int(x) for x in t.subtree(d) if t.is_leaf[x] and t.n_own_src[x] > 0}
            return out
        return self._get("Wclose", b, f)

    def _moved(self, d):
        return self.wfar_direct_max > 0 and self.t.sub_src[d] <= self.wfar_direct_max

    def Wfar(self, b):
        """List 3 far (after Remark 4, if enabled)."""
        return self._get("Wfar", b, lambda b: {d for d in self._wfar_def(b) if not self._moved(d)})

    def _wfar_def(self, b):
        """List 3 far: d in W_b or below with d < TCR(b) and no such ancestor in that set."""
        def f(b):
            t = self.t
            clos = self._w_closure(b)
            out = set()
            for d in clos:
                if not t.prec_tcr(d, b):
                    continue
                ok = True
                w = int(t.parent[d])
                while w in clos:
                    if t.prec_tcr(w, b):
                        ok = False
                        break
                    w = int(t.parent[w])
                if ok:
                    out.add(d)
            return out
        return self._get("Wfar_def", b, f)

    def Xclose(self, b):
        """List 4 close: d in X_w for some w in anc(b) or b, with not TCR(b) < d."""
        def f(b):
            t = self.t
            pool = set()
            for w in [b] + t.ancestors(b):
                pool |= self.X(w)
            return {d for d in pool if not t.tcr_prec(b, d)}
        return self._get("Xclose", b, f)

    def Xfar(self, b):
        """List 4 far: d in X_b with TCR(b) < d, plus d in Xclose(parent) with TCR(b) < d."""
        def f(b):
            t = self.t
            out = {d for d in self.X(b) if t.tcr_prec(b, d)}
            pb = int(t.parent[b])
            if pb >= 0:
                out |= {d for d in self.Xclose(pb) if t.tcr_prec(b, d)}
            return out
        return self._get("Xfar", b, f)

    def get(self, name, b):
        return getattr(self, name)(b)


class OracleFMM:
    """Tier B: GIGAQBX evaluation of the S or D layer potential."""

    def __init__(self, w, nmax=None, tcf=None, p_fmm=None, p_qbx=None, nthreads=0,
                 wfar_direct_max=0, tcr_norm="l2", level_restrict=False):
        self.w = w
        self.kernel = w.kernel
        self.p = int(w.p_fmm if p_fmm is None else p_fmm)
        self.q = int(w.p_qbx if p_qbx is None else p_qbx)
        self.nthreads = nthreads
        self.tree = OracleTree(w.src_xyz, w.ctr_xyz, w.ctr_radius, w.tgt_xyz,
                               w.nmax if nmax is None else nmax,
                               w.tcf if tcf is None else tcf, tcr_norm, level_restrict)
        self.lists = OracleLists(self.tree, wfar_direct_max)
        self._mpole = {}

    # --- expansions --------------------------------------------------------------------

    def _multipoles(self, boxes, strength):
        boxes = [b for b in boxes if (b, "M") not in self._mpole]
        if not boxes:
            return
        t, w = self.tree, self.w
        parts = [t.subtree_sources(b) for b in boxes]
        ptr = np.zeros(len(boxes) + 1, dtype=np.int64)
        ptr[1:] = np.cumsum([len(x) for x in parts])
        idx = _i64(np.concatenate(parts) if parts else np.zeros(0))
        cen = _f64(t.center[boxes])
        out = np.zeros((len(boxes), ncoef(self.p)), dtype=np.complex128)
        lib().oq_p2m_csr(KERNELS[self.kernel], self.p, len(boxes), _p(cen), _p(ptr), _p(idx),
                         _p(_f64(w.src_xyz)), _p(_f64(w.src_normal)), _p(strength), _p(out),
                         self.nthreads)
        for i, b in enumerate(boxes):
            self._mpole[(b, "M")] = out[i]

    def _sources_of(self, boxes):
        t = self.tree
        parts = [t.own_src[b] for b in sorted(boxes)]
        return np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)

    def evaluate(self, density_index=0, centers=None, lists=LIST_NAMES):
        """Potentials at the targets of the given centers (default: all).

        Returns (target ids, potential, qbx locals dict center -> coefficients).
        ``lists`` selects which list contributions are included.
        """
        t, L, w = self.tree, self.lists, self.w
        p, q = self.p, self.q
        kern = KERNELS[self.kernel]
        strength = _f64(strengths(w)[density_index])
        self._mpole = {}
        centers = np.arange(w.n_ctr) if centers is None else np.asarray(centers, dtype=np.int64)
        owners = sorted(set(int(t.ctr_owner[c]) for c in centers))
        chain = {}
        for b in owners:
            chain[b] = [b] + t.ancestors(b)
        need_local = sorted(set(a for b in owners for a in chain[b]))
        # Stage 2: multipoles of every box used by V (owners and ancestors) and W-far
        mp_boxes = set()
        for a in need_local:
            if "V" in lists:
                mp_boxes |= L.V(a)
        for b in owners:
            if "Wfar" in lists:
                mp_boxes |= L.Wfar(b)
        mp_boxes = sorted(mp_boxes)
        self._multipoles(mp_boxes, strength)
        np_ = ncoef(p)
        nq = ncoef(q)
        # Stages 4 and 6b: each box's own local (V by M2L, X-far by P2L), order p
        own_local = {a: np.zeros(np_, dtype=np.complex128) for a in need_local}
        if "V" in lists:
            src_boxes = sorted(set(d for a in need_local for d in L.V(a)))
            pos = {d: i for i, d in enumerate(src_boxes)}
            Mb = np.array([self._mpole[(d, "M")] for d in src_boxes]).reshape(-1, np_)
            mcen = _f64(t.center[src_boxes]).reshape(-1, 3)
            ptr = np.zeros(len(need_local) + 1, dtype=np.int64)
            lst = []
            for i, a in enumerate(need_local):
                items = sorted(L.V(a))
                lst += [pos[d] for d in items]
                ptr[i + 1] = len(lst)
            out = np.zeros((len(need_local), np_), dtype=np.complex128)
            lib().oq_m2l_csr(p, p, len(need_local), _p(_f64(t.center[need_local])), _p(ptr),
                             _p(_i64(lst)), _p(np.ascontiguousarray(Mb)), _p(mcen), _p(out),
                             self.nthreads)
            for i, a in enumerate(need_local):
                own_local[a] += out[i]
        if "Xfar" in lists:
            for a in need_local:
                xs = L.Xfar(a)
                if not xs:
                    continue
                idx = _i64(self._sources_of(xs))
                out = np.zeros(np_, dtype=np.complex128)
                lib().oq_p2l_shared(kern, p, 1, _p(_f64(t.center[a])), len(idx), _p(idx),
                                    _p(_f64(w.src_xyz)), _p(_f64(w.src_normal)), _p(strength),
                                    _p(out), self.nthreads)
                own_local[a] += out
        # Per center: Stages 3/5a/6a (direct), 5b (W-far M2L), 7-8 (L2L to the center)
        qloc = {}
        by_owner = {}
        for c in centers:
            by_owner.setdefault(int(t.ctr_owner[c]), []).append(int(c))
        for b, cs in by_owner.items():
            cs = np.array(cs, dtype=np.int64)
            cpos = _f64(w.ctr_xyz[cs])
            acc = np.zeros((len(cs), nq), dtype=np.complex128)
            near = set()
            for nm in ("U", "Wclose", "Xclose"):
                if nm in lists:
                    near |= L.get(nm, b)
            if near:
                idx = _i64(self._sources_of(near))
                out = np.zeros((len(cs), nq), dtype=np.complex128)
                lib().oq_p2l_shared(kern, q, len(cs), _p(cpos), len(idx), _p(idx),
                                    _p(_f64(w.src_xyz)), _p(_f64(w.src_normal)),
                                    _p(strength), _p(out), self.nthreads)
                acc += out
            if "Wfar" in lists and L.Wfar(b):
                wf = sorted(L.Wfar(b))
                Mb = np.ascontiguousarray(np.array([self._mpole[(d, "M")] for d in wf]))
                ptr = np.arange(0, len(cs) + 1, dtype=np.int64) * len(wf)
                lst = np.tile(np.arange(len(wf), dtype=np.int64), len(cs))
                out = np.zeros((len(cs), nq), dtype=np.complex128)
                lib().oq_m2l_csr(p, q, len(cs), _p(cpos), _p(ptr), _p(lst), _p(Mb),
                                 _p(_f64(t.center[wf])), _p(out), self.nthreads)
                acc += out
            if ("V" in lists) or ("Xfar" in lists):
                ch = chain[b]
                Lb = np.ascontiguousarray(np.array([own_local[a] for a in ch]))
                ptr = np.arange(0, len(cs) + 1, dtype=np.int64) * len(ch)
                lst = np.tile(np.arange(len(ch), dtype=np.int64), len(cs))
                out = np.zeros((len(cs), nq), dtype=np.complex128)
                lib().oq_l2l_csr(p, q, len(cs), _p(cpos), _p(ptr), _p(lst), _p(Lb),
                                 _p(_f64(t.center[ch])), _p(out), self.nthreads)
                acc += out
            for i, c in enumerate(cs):
                qloc[int(c)] = acc[i]
        # Stage 9: targets through their centers
        tmask = np.isin(w.tgt_center, centers)
        tids = np.nonzero(tmask)[0]
        cl = np.array(sorted(qloc))
        pos = {c: i for i, c in enumerate(cl)}
        Lmat = np.ascontiguousarray(np.array([qloc[c] for c in cl]).reshape(-1, nq))
        tc = _i64([pos[int(c)] for c in w.tgt_center[tids]])
        out = np.empty(len(tids))
        lib().oq_eval_locals(q, len(tids), _p(_f64(w.tgt_xyz[tids])), _p(tc),
                             _p(_f64(w.ctr_xyz[cl])), _p(Lmat), _p(out), self.nthreads)
        return tids, out, qloc

    def point_target_owner(self):
        """Owning box of every target (targets sit in the boxes that own them after the
        last subdivision, as sources do)."""
        own = np.full(self.w.n_tgt, -1, dtype=np.int64)
        for b, ts in enumerate(self.tree.own_tgt):
            own[ts] = b
        return own

    def evaluate_points(self, density_index=0, targets=None, lists=LIST_NAMES):
        """Conventional targets (no QBX center, tgt_center < 0): the stages of Algorithm 5
        for targets owned by box b.  Direct sums over the sources of List 1, List 3 close
        and List 4 close (Stages 3, 5a, 6a), multipole evaluation of each List 3 far box
        (Stage 5b), and the box local of b evaluated at the target (Stage 9), where the box
        local is the sum over b and its ancestors of their own List 2 (M2L) and List 4 far
        (P2L) locals, each evaluated directly at the target (L2L is exact).

        Returns (target ids, potential)."""
        t, L, w = self.tree, self.lists, self.w
        p = self.p
        kern = KERNELS[self.kernel]
        strength = _f64(strengths(w)[density_index])
        conv = np.nonzero(w.tgt_center < 0)[0]
        tids = conv if targets is None else np.intersect1d(conv, np.asarray(targets))
        owner = self.point_target_owner()
        self._mpole = {}
        boxes = sorted(set(int(owner[i]) for i in tids))
        chain = {b: [b] + t.ancestors(b) for b in boxes}
        need_local = sorted(set(a for b in boxes for a in chain[b]))
        mp = set()
        for a in need_local:
            if "V" in lists:
                mp |= L.V(a)
        for b in boxes:
            if "Wfar" in lists:
                mp |= L.Wfar(b)
        self._multipoles(sorted(mp), strength)
        np_ = ncoef(p)
        own_local = {a: np.zeros(np_, dtype=np.complex128) for a in need_local}
        for a in need_local:
            if "V" in lists:
                for d in L.V(a):
                    own_local[a] += _m2l_one(p, p, self._mpole[(d, "M")], t.center[d],
                                              t.center[a])
            if "Xfar" in lists and L.Xfar(a):
                idx = _i64(self._sources_of(L.Xfar(a)))
                out = np.zeros(np_, dtype=np.complex128)
                lib().oq_p2l_shared(kern, p, 1, _p(_f64(t.center[a])), len(idx), _p(idx),
                                    _p(_f64(w.src_xyz)), _p(_f64(w.src_normal)), _p(strength),
                                    _p(out), self.nthreads)
                own_local[a] += out
        pot = np.zeros(len(tids))
        for i, tg in enumerate(tids):
            b = int(owner[tg])
            x = _f64(w.tgt_xyz[tg])
            near = set()
            for nm in ("U", "Wclose", "Xclose"):
                if nm in lists:
                    near |= L.get(nm, b)
            if near:
                # order-0 QBX coefficient at the target itself is the point sum
                idx = _i64(self._sources_of(near))
                c0 = np.zeros(1, dtype=np.complex128)
                lib().oq_p2l_shared(kern, 0, 1, _p(x), len(idx), _p(idx), _p(_f64(w.src_xyz)),
                                    _p(_f64(w.src_normal)), _p(strength), _p(c0), self.nthreads)
                pot[i] += eval_local(0, c0, x, x)
            if "Wfar" in lists:
                for d in L.Wfar(b):
                    pot[i] += eval_mpole(p, self._mpole[(d, "M")], t.center[d], x)
            if ("V" in lists) or ("Xfar" in lists):
                for a in chain[b]:
                    pot[i] += eval_local(p, own_local[a], t.center[a], x)
        return tids, pot

    # --- diagnostics -------------------------------------------------------------------

    def target_boxes(self):
        """Boxes owning a QBX center or a conventional target."""
        s = set(int(b) for b in self.tree.ctr_owner)
        conv = np.nonzero(self.w.tgt_center < 0)[0]
        if len(conv):
            s |= set(int(b) for b in self.point_target_owner()[conv])
        return sorted(s)

    def list_owner_boxes(self):
        """Target boxes and target-ancestor boxes."""
        t = self.tree
        s = set()
        for b in self.target_boxes():
            s.add(b)
            s.update(t.ancestors(b))
        return sorted(s)

    def partition_check(self, b):
        """Each source leaf must be reached exactly once from a center owned by b."""
        t, L = self.tree, self.lists
        count = {}

        def add(d):
            count[d] = count.get(d, 0) + 1

        for nm in ("U", "Wclose", "Xclose"):
            for d in L.get(nm, b):
                add(d)
        for d in L.Wfar(b):
            for x in t.subtree(d):
                if t.is_leaf[x] and t.n_own_src[x] > 0:
                    add(int(x))
        for a in [b] + t.ancestors(b):
            for d in L.V(a):
                for x in t.subtree(d):
                    if t.is_leaf[x] and t.n_own_src[x] > 0:
                        add(int(x))
            for d in L.Xfar(a):
                add(d)
        leaves = set(int(x) for x in np.nonzero(t.is_leaf & (t.n_own_src > 0))[0])
        missing = leaves - set(count)
        multi = {d: c for d, c in count.items() if c != 1}
        return missing, multi
