"""Plain FP64 KIFMM with the paper's kernel tables -- TEST INFRASTRUCTURE ONLY.

Follows the octree traversal of Sec. II (the KIFMM algorithm graph,
fig:kifmmgraph, and the general kernel table tab:ktabdef):

  upward pass   S->M at leaves, M->M to the root; each box finds equivalent
                sources on its M points by matching the field of what it
                encloses on an outer check surface (inverse problem solved by
                a truncated SVD pseudo-inverse, as the paper says PVFMM does);
  downward pass M->L over the V list, S->L over the X list, L->L from the
                parent, then the L equivalent sources from the inner check
                surface;
  evaluation    L->T, M->T over the W list, S->T direct over the U list.

The kernels used at each stage are the paper's kernel tables:
  Stokeslet   G everywhere                                 (Sec. II.B)
  RPY         G^RPY from S, G on the ML tree, G (+) lap G to T (tab:ktab_rpy)
  LapPGrad    L and L^D from S, L on the ML tree, L (+) grad L to T
                                                           (tab:ktab_lapqdpgradgrad)
  PVel        G^P and the double layer K from S, G^P on the ML tree
                                                           (tab:ktab_stkdlpvelgrad)
  Traction    as PVel, with the traction kernel S at the T side
                                                           (tab:ktab_stkdlstress)

The paper defers the list definitions and the surface geometry to the
KIFMM literature ("we omit those technical details"); the readings used here:
  * box B: centre c, side h = L0 2^-level; tree splits a box while it holds
    more than leaf_cap targets, SL sources or DL sources; empty boxes are not
    created; no 2:1 balance.
  * surface S(c, a): c + a (h/2)(-1 + 2 (i,j,k)/(p-1)), i,j,k in 0..p-1 with at
    least one index in {0, p-1}: M = 6(p-1)^2 + 2 points (Sec. III).
  * radii: upward equivalent and downward check a_in = 1.05; upward check
    and downward equivalent a_out = 2.95.
  * U(B): leaves adjacent to leaf B (B included).  V(B): children of the
    colleagues of B's parent that are not adjacent to B.  W(B): descendants
    of B's colleagues that are not adjacent to B but whose parent is.
    X(B): boxes A with B in W(A).
Open boundary only.  Plain loops and NumPy matrices, no blocking or reuse
beyond grouping identical geometry.
"""
from __future__ import annotations

import numpy as np

from . import direct

A_IN = 1.05
A_OUT = 2.95
PI = np.pi


# --------------------------------------------------------------------------
# ML-tree kernel matrices (dense FP64), block [trg_point * kt + i, src_point * ks + j]
# --------------------------------------------------------------------------
def _diff(X, Y):
    r = X[:, None, :] - Y[None, :, :]
    rr = np.sum(r * r, axis=2)
    with np.errstate(divide="ignore"):
        inv = np.where(rr > 0, 1.0 / np.sqrt(np.where(rr > 0, rr, 1.0)), 0.0)
    return r, inv


def laplace_matrix(X, Y):
    """L(x, y) = 1/(4 pi r)  (Sec. II.A)."""
    _, inv = _diff(X, Y)
    return inv / (4 * PI)


def stokeslet_matrix(X, Y):
    """G_ij = (delta_ij / r + r_i r_j / r^3) / (8 pi)  (Sec. II.B)."""
    r, inv = _diff(X, Y)
    m, n = inv.shape
    K = np.zeros((m, 3, n, 3))
    inv3 = inv ** 3
    for i in range(3):
        for j in range(3):
            K[:, i, :, j] = ((i == j) * inv + r[:, :, i] * r[:, :, j] * inv3) / (8 * PI)
    return K.reshape(3 * m, 3 * n)


def stokes_pvel_matrix(X, Y):
    """G^P: [f, q] -> [p, u]  (Sec. II.C, Eqs. stkslp and stkslvel)."""
    r, inv = _diff(X, Y)
    m, n = inv.shape
    K = np.zeros((m, 4, n, 4))
    inv3 = inv ** 3
    for j in range(3):
        K[:, 0, :, j] = r[:, :, j] * inv3 / (4 * PI)
    for i in range(3):
        for j in range(3):
            K[:, 1 + i, :, j] = ((i == j) * inv + r[:, :, i] * r[:, :, j] * inv3) / (8 * PI)
        K[:, 1 + i, :, 3] = -r[:, :, i] * inv3 / (8 * PI)
    return K.reshape(4 * m, 4 * n)


# --------------------------------------------------------------------------
# Kernel tables
# --------------------------------------------------------------------------
class _Table:
    """One row set of a kernel table: what each stage uses."""

    def __init__(self, name, kml, ml_matrix, s_to_check, eq_to_trg, s_to_trg, kt):
        self.name = name
        self.kml = kml                  # ML-tree kernel value width (check / density)
        self.ml_matrix = ml_matrix      # ML kernel  (M->M, M->L, L->L, pinv)
        self.s_to_check = s_to_check    # S->M and S->L kernel, evaluated to check points
        self.eq_to_trg = eq_to_trg      # M->T and L->T kernel from equivalent densities
        self.s_to_trg = s_to_trg        # S->T kernel
        self.kt = kt


def _tab_stokeslet():
    def s2c(chk, sl, slv, dl, dlv):
        return direct.stokeslet(sl, slv, chk)

    def e2t(trg, eq, dens):
        return direct.stokeslet(eq, dens.reshape(-1, 3), trg)

    def s2t(trg, sl, slv, dl, dlv):
        return direct.stokeslet(sl, slv, trg)

    return _Table("Stokeslet", 3, stokeslet_matrix, s2c, e2t, s2t, 3)


def _tab_rpy():
    def s2c(chk, sl, slv, dl, dlv):          # G^RPY velocity only
        return direct.rpy(sl, slv, chk)[:, :3]

    def e2t(trg, eq, dens):                   # G (+) lap G: RPY with b = 0
        fb = np.concatenate([dens.reshape(-1, 3), np.zeros((len(eq), 1))], axis=1)
        return direct.rpy(eq, fb, trg)

    def s2t(trg, sl, slv, dl, dlv):
        return direct.rpy(sl, slv, trg)

    return _Table("RPY", 3, stokeslet_matrix, s2c, e2t, s2t, 6)


def _tab_lap_pgrad():
    def s2c(chk, sl, slv, dl, dlv):           # L and L^D, potential only
        return direct.laplace(sl, slv, dl, dlv, chk)[:, :1]

    def e2t(trg, eq, dens):                   # L (+) grad L from charges
        return direct.laplace(eq, dens.reshape(-1), None, None, trg)

    def s2t(trg, sl, slv, dl, dlv):
        return direct.laplace(sl, slv, dl, dlv, trg)

    return _Table("LapPGrad", 1, laplace_matrix, s2c, e2t, s2t, 4)


def _tab_pvel():
    def s2c(chk, sl, slv, dl, dlv):           # G^P (SL) and K (DL) -> [p, u]
        return direct.pvel(sl, slv, dl, dlv, chk)

    def e2t(trg, eq, dens):                   # G^P from [f, q]
        return direct.pvel(eq, dens.reshape(-1, 4), None, None, trg)

    def s2t(trg, sl, slv, dl, dlv):
        return direct.pvel(sl, slv, dl, dlv, trg)

    return _Table("PVel", 4, stokes_pvel_matrix, s2c, e2t, s2t, 4)


def _tab_traction():
    def s2c(chk, sl, slv, dl, dlv):
        return direct.pvel(sl, slv, dl, dlv, chk)

    def e2t(trg, eq, dens):                   # S from [f, q]
        return direct.traction(eq, dens.reshape(-1, 4), None, None, trg)

    def s2t(trg, sl, slv, dl, dlv):
        return direct.traction(sl, slv, dl, dlv, trg)

    return _Table("Traction", 4, stokes_pvel_matrix, s2c, e2t, s2t, 9)


TABLES = {
    "Stokeslet": _tab_stokeslet,
    "RPY": _tab_rpy,
    "LapPGrad": _tab_lap_pgrad,
    "PVel": _tab_pvel,
    "Traction": _tab_traction,
}


# --------------------------------------------------------------------------
# Surfaces
# --------------------------------------------------------------------------
def surface_grid(p):
    """Unit-cube surface lattice in [-1, 1]^3: M = 6 (p-1)^2 + 2 points."""
    g = -1.0 + 2.0 * np.arange(p) / (p - 1)
    pts = []
    for i in range(p):
        for j in range(p):
            for k in range(p):
                if i in (0, p - 1) or j in (0, p - 1) or k in (0, p - 1):
                    pts.append((g[i], g[j], g[k]))
    return np.array(pts)


def surface(grid, centre, h, alpha):
    return centre + alpha * (h / 2.0) * grid


def pinv(K, tol):
    """Truncated-SVD pseudo-inverse (backward-stable SVD, Sec. II)."""
    U, s, Vt = np.linalg.svd(K, full_matrices=False)
    keep = s > tol * s[0]
    return (Vt[keep].T / s[keep]) @ U[:, keep].T


# --------------------------------------------------------------------------
# Octree and interaction lists
# --------------------------------------------------------------------------
def morton_order(x, origin, L0, bits=21):
    """Sorted position -> input index of points along the Z-order (Morton)
    curve of the 2^bits grid over [origin, origin + L0)^3: points compare by
    the octant digits of their cells from the root down (within a level the
    x bit is the most significant), ties by input index.  Coordinates on the
    upper face fall into the last cell."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    u = (x - np.asarray(origin, dtype=np.float64)) / L0
    cell = np.clip(np.floor(u * 2.0 ** bits), 0, 2 ** bits - 1).astype(np.int64)
    key = np.zeros(len(x), dtype=np.uint64)
    for lev in range(bits):
        sh = bits - 1 - lev
        digit = ((cell[:, 0] >> sh) & 1) * 4 + ((cell[:, 1] >> sh) & 1) * 2 + ((cell[:, 2] >> sh) & 1)
        key = key * np.uint64(8) + digit.astype(np.uint64)
    return np.lexsort((np.arange(len(x)), key))


class Tree:
    """Adaptive octree over the union of SL, DL and target points."""

    def __init__(self, sl, dl, trg, origin, L0, cap, max_depth=20):
        self.origin = np.asarray(origin, dtype=np.float64)
        self.L0 = float(L0)
        self.cap = cap
        self.level, self.anchor, self.parent, self.children = [], [], [], []
        self.idx = []                      # per box: (sl idx, dl idx, trg idx)
        sets = [np.zeros((0, 3)) if a is None else np.asarray(a, float).reshape(-1, 3)
                for a in (sl, dl, trg)]
        self.sets = sets
        root = tuple(np.arange(len(a)) for a in sets)
        self._add(0, (0, 0, 0), -1, root)
        stack = [0]
        while stack:
            b = stack.pop()
            counts = [len(i) for i in self.idx[b]]
            if max(counts) <= cap or self.level[b] >= max_depth:
                continue
            lev = self.level[b] + 1
            h = self.L0 / 2 ** lev
            parts = []
            for s, ids in zip(sets, self.idx[b]):
                ic = np.floor((s[ids] - self.origin) / h).astype(np.int64)
                parts.append((ids, ic))
            for o in range(8):
                off = ((o >> 0) & 1, (o >> 1) & 1, (o >> 2) & 1)
                anc = tuple(2 * a + c for a, c in zip(self.anchor[b], off))
                sub = []
                for ids, ic in parts:
                    m = np.all(ic == np.array(anc), axis=1)
                    sub.append(ids[m])
                if sum(len(x) for x in sub) == 0:
                    continue
                c = self._add(lev, anc, b, tuple(sub))
                self.children[b].append(c)
                stack.append(c)
        self.nbox = len(self.level)
        self.level = np.array(self.level)
        self.anchor = np.array(self.anchor, dtype=np.int64)
        self.parent = np.array(self.parent)
        self.is_leaf = np.array([len(c) == 0 for c in self.children])
        self._lists()

    def _add(self, lev, anc, parent, idx):
        self.level.append(lev)
        self.anchor.append(tuple(anc))
        self.parent.append(parent)
        self.children.append([])
        self.idx.append(idx)
        return len(self.level) - 1

    def centre(self, b):
        h = self.L0 / 2 ** self.level[b]
        return self.origin + (self.anchor[b] + 0.5) * h

    def side(self, b):
        return self.L0 / 2 ** self.level[b]

    def _lists(self):
        D = int(self.level.max()) + 1
        scale = (2 ** (D - self.level))[:, None]
        lo = self.anchor * scale
        hi = (self.anchor + 1) * scale
        # closed boxes intersect: adjacent, identical, or nested
        adj = np.all((lo[:, None, :] <= hi[None, :, :]) & (lo[None, :, :] <= hi[:, None, :]), axis=2)
        self.adj = adj
        nb, lev, par = self.nbox, self.level, self.parent
        # ancestor at each level
        anc = -np.ones((nb, D + 1), dtype=np.int64)
        for b in range(nb):
            a = b
            while a >= 0:
                anc[b, lev[a]] = a
                a = par[a]
        self.anc = anc
        same = lev[:, None] == lev[None, :]
        coll = adj & same
        leaves = np.nonzero(self.is_leaf)[0]
        self.U = {b: [a for a in leaves if adj[b, a]] for b in leaves}
        self.V = {}
        for b in range(nb):
            if par[b] < 0:
                self.V[b] = []
                continue
            cands = [c for pc in np.nonzero(coll[par[b]])[0] for c in self.children[pc]]
            self.V[b] = [c for c in cands if not adj[b, c]]
        self.W = {}
        for b in leaves:
            lb = lev[b]
            w = []
            for a in range(nb):
                if lev[a] <= lb:
                    continue
                if not coll[b, anc[a, lb]]:
                    continue
                if adj[b, a] or not adj[b, par[a]]:
                    continue
                w.append(a)
            self.W[b] = w
        self.X = {b: [] for b in range(nb)}
        for b in leaves:
            for a in self.W[b]:
                self.X[a].append(b)

    def coverage(self):
        """Count how many routes cover each (target leaf, source leaf) pair.

        Every pair must be covered exactly once: U directly, or through the
        V, W or X list of the target leaf or one of its ancestors."""
        leaves = np.nonzero(self.is_leaf)[0]
        pos = {b: i for i, b in enumerate(leaves)}
        n = len(leaves)
        cnt = np.zeros((n, n), dtype=np.int64)

        def leaves_under(a):
            out, st = [], [a]
            while st:
                x = st.pop()
                if self.is_leaf[x]:
                    out.append(x)
                st.extend(self.children[x])
            return out

        for t in leaves:
            ti = pos[t]
            for s in self.U[t]:
                cnt[ti, pos[s]] += 1
            for a in self.W[t]:
                for s in leaves_under(a):
                    cnt[ti, pos[s]] += 1
            x = t
            while x >= 0:
                for a in self.V[x]:
                    for s in leaves_under(a):
                        cnt[ti, pos[s]] += 1
                for s in self.X[x]:
                    cnt[ti, pos[s]] += 1
                x = self.parent[x]
        return cnt


# --------------------------------------------------------------------------
# KIFMM evaluation
# --------------------------------------------------------------------------
def evaluate(kernel, sl=None, sl_val=None, dl=None, dl_val=None, trg=None,
             p=8, leaf_cap=64, origin=(0.0, 0.0, 0.0), L0=1.0, svd_tol=1e-12,
             tree=None, stats=None):
    """FP64 KIFMM of ``kernel`` at the targets; returns [n_trg, k_t]."""
    tab = TABLES[kernel]()
    if tree is None:
        tree = Tree(sl, dl, trg, origin, L0, leaf_cap)
    T = tree
    sl = T.sets[0]
    dl = T.sets[1]
    trg = T.sets[2]
    slv = None if sl_val is None else np.asarray(sl_val, float).reshape(len(sl), -1)
    dlv = None if dl_val is None else np.asarray(dl_val, float).reshape(len(dl), -1)
    grid = surface_grid(p)
    M = len(grid)
    k = tab.kml
    nb = T.nbox

    def box_sources(b):
        i_sl, i_dl, _ = T.idx[b]
        a = (sl[i_sl], None if slv is None else slv[i_sl])
        d = (dl[i_dl], None if dlv is None else dlv[i_dl])
        return a[0], a[1], d[0], d[1]

    def s2c(chk, b):
        ys, vs, yd, vd = box_sources(b)
        return tab.s_to_check(chk, ys if len(ys) else None, vs if len(ys) else None,
                              yd if len(yd) else None, vd if len(yd) else None)

    # per-level inverse operators (geometry depends only on the level)
    cache = {}

    def ops(level):
        if level not in cache:
            h = T.L0 / 2 ** level
            c0 = np.zeros(3)
            uc = surface(grid, c0, h, A_OUT)
            ue = surface(grid, c0, h, A_IN)
            dc = surface(grid, c0, h, A_IN)
            de = surface(grid, c0, h, A_OUT)
            cache[level] = (pinv(tab.ml_matrix(uc, ue), svd_tol),
                            pinv(tab.ml_matrix(dc, de), svd_tol))
        return cache[level]

    # translation matrices depend only on the level and the relative anchor
    # offset of the two boxes (identical geometry), so they are memoised
    mats = {}

    def trans(kind, b_trg, b_src, a_trg, a_src):
        lt, ls = int(T.level[b_trg]), int(T.level[b_src])
        D = max(lt, ls)
        # lower corners on the finer of the two grids fix the relative geometry
        rel = tuple(T.anchor[b_src] * 2 ** (D - ls) - T.anchor[b_trg] * 2 ** (D - lt))
        key = (kind, lt, ls, rel)
        if key not in mats:
            X = surface(grid, T.centre(b_trg), T.side(b_trg), a_trg)
            Y = surface(grid, T.centre(b_src), T.side(b_src), a_src)
            mats[key] = tab.ml_matrix(X, Y)
        return mats[key]

    # ---- upward pass: S->M at leaves, M->M towards the root
    sigma = np.zeros((nb, M * k))
    order = np.argsort(-T.level, kind="stable")
    for b in order:
        c, h = T.centre(b), T.side(b)
        uc = surface(grid, c, h, A_OUT)
        if T.is_leaf[b]:
            chk = s2c(uc, b).reshape(-1)
        else:
            chk = np.zeros(M * k)
            for ch in T.children[b]:
                chk += trans("m2m", b, ch, A_OUT, A_IN) @ sigma[ch]
        sigma[b] = ops(T.level[b])[0] @ chk

    # ---- downward pass: V (M->L), X (S->L), L->L, then L densities
    tau = np.zeros((nb, M * k))
    has_local = np.zeros(nb, dtype=bool)
    n_v = 0
    for b in np.argsort(T.level, kind="stable"):
        c, h = T.centre(b), T.side(b)
        dc = surface(grid, c, h, A_IN)
        chk = np.zeros(M * k)
        any_ = False
        for a in T.V[b]:
            chk += trans("m2l", b, a, A_IN, A_IN) @ sigma[a]
            any_ = True
            n_v += 1
        for a in T.X[b]:
            chk += s2c(dc, a).reshape(-1)
            any_ = True
        pb = T.parent[b]
        if pb >= 0 and has_local[pb]:
            chk += trans("l2l", b, pb, A_IN, A_OUT) @ tau[pb]
            any_ = True
        if any_:
            tau[b] = ops(T.level[b])[1] @ chk
            has_local[b] = True

    # ---- evaluation at targets: L->T, M->T (W), S->T (U)
    out = np.zeros((len(trg), tab.kt))
    for b in np.nonzero(T.is_leaf)[0]:
        it = T.idx[b][2]
        if len(it) == 0:
            continue
        xt = trg[it]
        g = np.zeros((len(it), tab.kt))
        if has_local[b]:
            de = surface(grid, T.centre(b), T.side(b), A_OUT)
            g += tab.eq_to_trg(xt, de, tau[b])
        for a in T.W[b]:
            ue_a = surface(grid, T.centre(a), T.side(a), A_IN)
            g += tab.eq_to_trg(xt, ue_a, sigma[a])
        for a in T.U[b]:
            ys, vs, yd, vd = box_sources(a)
            if len(ys) + len(yd) == 0:
                continue
            g += tab.s_to_trg(xt, ys if len(ys) else None, vs if len(ys) else None,
                              yd if len(yd) else None, vd if len(yd) else None)
        out[it] = g
    if stats is not None:
        stats.update(nbox=nb, nleaf=int(T.is_leaf.sum()), n_v=n_v,
                     depth=int(T.level.max()), M=M)
    return out
