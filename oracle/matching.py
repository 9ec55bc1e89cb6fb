"""Minimum-weight matching start of every class (Sec. III, Sec. IV).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. III ("enhanced" matching) decodes each anyon type on its own: a matching
of the type's anyons, each pair joined by a string of single-qubit errors of
that type and each unpaired anyon joined to a boundary that absorbs it.  Two
matchings are computed per type, one in each line parity (the paper forces the
second by an extra virtual anyon on the absorbing boundaries), and the 2 x 2
combinations are the four class hypotheses; Sec. IV starts each class's chain
from its hypothesis.  Each hypothesis is the most likely member of its class
when x and z parts are counted independently.

Plain definition used here.  For plaquette anyons (made by x parts) the
lattice graph has one vertex per plaquette plus a LEFT and a RIGHT boundary
vertex, and one edge per qubit (a qubit in an even grid row joins its two
horizontal plaquette neighbours, or one of them and a boundary vertex; a
qubit in an odd row joins its vertical neighbours).  An x part is an edge
set; its anyons are the plaquettes of odd degree and its bx parity is the
degree of LEFT (the qubits of grid column 0).  So the cheapest x part with
the measured anyons A and parity b is a minimum T-join with
T = A + {LEFT if b} + {RIGHT if |A| + b is odd}, which is a minimum-weight
perfect matching of T under shortest-path distances (Edmonds and Johnson):

    d(a, a') = min(|di| + |dj|, near(a) + near(a'), far(a) + far(a'))
    d(a, NEAR) = near(a),  d(a, FAR) = far(a),  d(NEAR, FAR) = L

with near/far = j + 1 / L - 1 - j for plaquettes (left/right) and
i + 1 / L - 1 - i for stars (top/bottom, the z parts on grid row 0 give bz).
This is exact; the paper's graph (a virtual partner on each anyon's nearer
boundary) restricts the same problem.

Ties.  Many matchings can share the minimum weight.  Every matching edge
{u, v} therefore carries the weight W = d 2^53 + 2 t(u, v), where t is the
top 43 bits of the 64-bit product K(u) K(v), K(x) = the splitmix64 output
(Steele, Lea and Flood, OOPSLA 2014) at state id(x); an anyon's id is its
site index, NEAR is 4094 and FAR is 4095.  Over any perfect matching (at most 301 edges at
L = 25) the t terms add up to less than 2^53, so W orders matchings by total
distance first; among equal distances the smallest sum of t wins, which is
unique unless two matchings' t sums collide (probability below
|edges| / 2^43 for random t, by the isolation lemma).  W is even, so the
dual variables below stay integers.

Paths.  A matched pair of anyons a < a' (site order) with
d = |di| + |dj| takes the direct path (plaquettes: along a's grid row to
the column of a', then down that column; stars: down a's grid column to the
row of a', then along that row); otherwise both go to the nearer boundary
of the two options (NEAR on a tie).  An anyon matched to NEAR or FAR takes
the straight string there, and NEAR-FAR is the logical string (X on grid
row 0, Z on grid column 0).  For a minimum matching these paths share no
edge, so the part's weight equals the matching's total distance.

The matching solver is Edmonds' primal-dual blossom algorithm for a
minimum-weight perfect matching (Edmonds 1965, with the dual bookkeeping as
in Galil, ACM Computing Surveys 1986), written plainly: every step rescans
all vertex pairs.  Dual feasibility: slack(i, j) = W_ij - u_i - u_j +
sum of z_B over blossoms B containing both i and j >= 0.
"""

import numpy as np

from . import geometry, init

NEAR_ID, FAR_ID = 4094, 4095
T_BITS = 43
D_SHIFT = 53
_M64 = (1 << 64) - 1


def splitmix64(state):
    """Output of splitmix64 at the given state (Steele, Lea, Flood 2014)."""
    z = (state + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def tie_break(id_a, id_b):
    """Top 43 bits of the 64-bit product of the two ends' splitmix64 keys."""
    return ((splitmix64(id_a) * splitmix64(id_b)) & _M64) >> (64 - T_BITS)


# ---------------------------------------------------------------------------
# Edmonds' blossom algorithm, minimum-weight perfect matching
# ---------------------------------------------------------------------------
class Result:
    """mate[v]: partner of vertex v; u: vertex duals; blossoms: list of
    (vertex set, z) of every blossom alive at the end."""

    def __init__(self, mate, u, blossoms, stats=None):
        self.mate, self.u, self.blossoms = mate, u, blossoms
        self.stats = stats or {}


def min_weight_perfect_matching(W):
    """W: int64 [n, n] symmetric, even off-diagonal entries, n even.  Returns a
    Result whose mate is a minimum-weight perfect matching."""
    W = np.asarray(W, dtype=np.int64)
    n = W.shape[0]
    if n % 2:
        raise ValueError("a perfect matching needs an even number of vertices")
    if n == 0:
        return Result(np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64), [])
    off = ~np.eye(n, dtype=bool)
    if (W[off] % 2).any() or not np.array_equal(W, W.T):
        raise ValueError("weights must be symmetric and even")
    BIG = np.int64(1) << 62
    NB = 2 * n
    mate = [-1] * n
    parent = [-1] * NB                 # enclosing blossom of a node
    children = [None] * NB             # blossom: child nodes around the cycle, [0] = base child
    cedges = [None] * NB               # blossom: (x, y), x in children[k], y in children[k+1]
    base = list(range(n)) + [-1] * n
    z = [0] * NB
    free_ids = list(range(NB - 1, n - 1, -1))
    label = [0] * NB                   # outermost nodes: 0 free, 1 S (even), 2 T (odd)
    tedge = [None] * NB                # T node: (s, t), s in its S parent, t inside it
    u = np.full(n, int(W[off].min()) // 2, dtype=np.int64)
    stats = {"shrink": 0, "expand": 0, "nested": 0, "dual": 0, "rotate_blossom": 0}

    def top(v):
        while parent[v] != -1:
            v = parent[v]
        return v

    def child_of(B, v):
        while parent[v] != B:
            v = parent[v]
        return v

    def leaves(x):
        if x < n:
            return [x]
        out = []
        for c in children[x]:
            out += leaves(c)
        return out

    def rotate(B, v):
        """Make vertex v (inside node B) the base of B: flip the even
        alternating path between v's child and the base child."""
        if B < n:
            return
        stats["rotate_blossom"] += 1
        c = child_of(B, v)
        rotate(c, v)
        ch, ed = children[B], cedges[B]
        k, m = ch.index(c), len(children[B])
        step = -1 if k % 2 == 0 else 1
        pos = k
        while pos != 0:
            a = (pos + step) % m
            b = (a + step) % m
            if step == 1:
                x, y = ed[a]                 # edge a joins children a and a + 1 = b
            else:
                y, x = ed[b]                 # edge b joins children b and b + 1 = a
            rotate(ch[a], x)
            rotate(ch[b], y)
            mate[x], mate[y] = y, x
            pos = b
        children[B] = ch[k:] + ch[:k]
        cedges[B] = ed[k:] + ed[:k]
        base[B] = v

    def s_parent(B):
        """The S node above S node B in its tree, or None for a root."""
        m = mate[base[B]]
        if m == -1:
            return None
        return top(tedge[top(m)][0])

    def up_edge(X):
        """(x in X, y in X's tree parent)."""
        if label[X] == 1:
            b = base[X]
            return (b, mate[b])
        s, t = tedge[X]
        return (t, s)

    def augment_path(v, w):
        while True:
            B = top(v)
            t0 = mate[base[B]]
            rotate(B, v)
            mate[v] = w
            if t0 == -1:
                return
            T = top(t0)
            s, t = tedge[T]
            rotate(T, t)
            mate[t] = s
            v, w = s, t

    def shrink(i, j):
        Bi, Bj = top(i), top(j)
        chain_i, x = [], Bi
        while x is not None:
            chain_i.append(x)
            x = s_parent(x)
        on_i = set(chain_i)
        chain_j, x = [], Bj
        while x not in on_i:
            chain_j.append(x)
            x = s_parent(x)
        A = x

        def path_up(B):                  # S and T nodes from B up to, not including, A
            out = []
            while B != A:
                out.append(B)
                T = top(mate[base[B]])
                out.append(T)
                B = top(tedge[T][0])
            return out

        pi, pj = path_up(Bi), path_up(Bj)
        ch = [A] + pj[::-1] + pi
        ed = []
        for X in pj[::-1]:               # going down from A towards Bj
            x, y = up_edge(X)
            ed.append((y, x))
        ed.append((j, i))                # Bj -> Bi
        for X in pi:                     # going up from Bi to A
            ed.append(up_edge(X))
        stats["shrink"] += 1
        stats["nested"] += int(any(c >= n for c in ch))
        b = free_ids.pop()
        children[b], cedges[b] = ch, ed
        base[b] = base[A]
        z[b] = 0
        for c in ch:
            parent[c] = b
        label[b] = 1
        tedge[b] = None

    def expand_t(B):
        stats["expand"] += 1
        s, t = tedge[B]
        ch, ed, m = children[B], cedges[B], len(children[B])
        c = child_of(B, t)
        k = ch.index(c)
        for x in ch:
            parent[x] = -1
            label[x] = 0
            tedge[x] = None
        label[c] = 2
        tedge[c] = (s, t)
        step = -1 if k % 2 == 0 else 1
        pos = k
        while pos != 0:
            a = (pos + step) % m
            b = (a + step) % m
            x, y = ed[a] if step == 1 else (ed[b][1], ed[b][0])
            label[ch[a]] = 1
            label[ch[b]] = 2
            tedge[ch[b]] = (x, y)
            pos = b
        children[B] = cedges[B] = None
        base[B] = -1
        label[B] = 0
        tedge[B] = None
        z[B] = 0
        free_ids.append(B)

    while True:
        exposed = [v for v in range(n) if mate[v] == -1]
        if not exposed:
            break
        for x in range(NB):
            label[x] = 0
            tedge[x] = None
        for v in exposed:
            label[top(v)] = 1
        done = False
        while not done:
            outer = np.array([top(v) for v in range(n)])
            lab = np.array([label[o] for o in outer])
            S, Tm, F = lab == 1, lab == 2, lab == 0
            slack = W - u[:, None] - u[None, :]
            diff = outer[:, None] != outer[None, :]
            cand = S[:, None] & diff & ~Tm[None, :]
            tight = np.argwhere(cand & (slack == 0))
            if tight.size:
                i, j = int(tight[0][0]), int(tight[0][1])
                Bj = int(outer[j])
                if label[Bj] == 0:
                    label[Bj] = 2
                    tedge[Bj] = (i, j)
                    label[top(mate[base[Bj]])] = 1
                else:
                    ri, rj = top(i), Bj
                    while s_parent(ri) is not None:
                        ri = s_parent(ri)
                    while s_parent(rj) is not None:
                        rj = s_parent(rj)
                    if ri != rj:
                        augment_path(i, j)
                        augment_path(j, i)
                        done = True
                    else:
                        shrink(i, j)
                continue
            d2 = slack[S[:, None] & F[None, :] & diff]
            d3 = slack[S[:, None] & S[None, :] & diff]
            if d3.size and (d3 % 2).any():
                raise AssertionError("odd slack between even vertices")
            tops_t = [b for b in set(outer.tolist()) if b >= n and label[b] == 2]
            cands = []
            if d2.size:
                cands.append(int(d2.min()))
            if d3.size:
                cands.append(int(d3.min()) // 2)
            for b in tops_t:
                cands.append(z[b] // 2)
            if not cands:
                raise AssertionError("no dual change possible")
            delta = min(cands)
            stats["dual"] += 1
            u[S] += delta
            u[Tm] -= delta
            for b in set(outer.tolist()):
                if b >= n:
                    if label[b] == 1:
                        z[b] += 2 * delta
                    elif label[b] == 2:
                        z[b] -= 2 * delta
            if np.abs(u).max() >= BIG or any(abs(v) >= BIG for v in z):
                raise AssertionError("dual variables out of range")
            for b in tops_t:
                if z[b] == 0:
                    expand_t(b)
    blossoms = [(sorted(leaves(b)), z[b]) for b in range(n, NB) if children[b] is not None]
    return Result(np.array(mate, dtype=np.int64), u, blossoms, stats)


def certificate_holds(W, res):
    """Linear-programming optimality of res.mate (Edmonds' perfect matching
    polytope): every slack >= 0 with the blossom duals, matched pairs tight,
    z >= 0, and every blossom with z > 0 full."""
    W = np.asarray(W, dtype=np.int64)
    n = W.shape[0]
    if n == 0:
        return True
    mate = res.mate
    if sorted(mate.tolist()) != list(range(n)) or any(mate[mate[v]] != v or mate[v] == v
                                                      for v in range(n)):
        return False
    slack = (W - res.u[:, None] - res.u[None, :]).astype(object)
    for verts, zb in res.blossoms:
        if zb < 0:
            return False
        inside = np.zeros(n, dtype=bool)
        inside[verts] = True
        slack[np.ix_(inside, inside)] += zb
        if zb > 0 and sum(1 for v in verts if inside[mate[v]]) != len(verts) - 1:
            return False
    off = ~np.eye(n, dtype=bool)
    if min(slack[off]) < 0:
        return False
    return all(slack[v, mate[v]] == 0 for v in range(n))


# ---------------------------------------------------------------------------
# The surface-code problems
# ---------------------------------------------------------------------------
def type_anyons(lat, syn, is_star):
    """[(site, i, j)] of the lit sites of one type, ascending site order."""
    rng = range(0, lat.n_stars) if is_star else range(lat.n_stars, lat.n_stab)
    return [(s, int(lat.site_ij[s][0]), int(lat.site_ij[s][1])) for s in rng if syn[s]]


def _near_far(L, is_star, i, j):
    return (i + 1, L - 1 - i) if is_star else (j + 1, L - 1 - j)


def problem(lat, syn, is_star, parity):
    """Vertices of T (anyons, then NEAR and/or FAR) as (id, i, j), and the
    distance matrix d and matching weight matrix W of the complete graph."""
    L = lat.L
    anyons = type_anyons(lat, syn, is_star)
    nodes = [(s, i, j) for (s, i, j) in anyons]
    if parity:
        nodes.append((NEAR_ID, -1, -1))
    if (len(anyons) + parity) % 2:
        nodes.append((FAR_ID, -1, -1))
    m = len(nodes)
    d = np.zeros((m, m), dtype=np.int64)
    for a in range(m):
        for b in range(a + 1, m):
            ia, ja = nodes[a][1:]
            ib, jb = nodes[b][1:]
            ida, idb = nodes[a][0], nodes[b][0]
            if ida < NEAR_ID and idb < NEAR_ID:
                na, fa = _near_far(L, is_star, ia, ja)
                nb, fb = _near_far(L, is_star, ib, jb)
                v = min(abs(ia - ib) + abs(ja - jb), na + nb, fa + fb)
            elif ida < NEAR_ID:
                na, fa = _near_far(L, is_star, ia, ja)
                v = na if idb == NEAR_ID else fa
            else:
                v = L
            d[a, b] = d[b, a] = v
    W = np.zeros((m, m), dtype=np.int64)
    for a in range(m):
        for b in range(a + 1, m):
            W[a, b] = W[b, a] = (int(d[a, b]) << D_SHIFT) + 2 * tie_break(nodes[a][0], nodes[b][0])
    return nodes, d, W


def type_part(lat, syn, is_star, parity):
    """uint8 [n_q] part of one type (x parts for plaquettes, z for stars) of
    parity `parity`, and its total distance."""
    L = lat.L
    nodes, d, W = problem(lat, syn, is_star, parity)
    res = min_weight_perfect_matching(W)
    anyons = [(i, j) for (s, i, j) in nodes if s < NEAR_ID]
    pairs, bmatch, logical = [], [], False
    total = 0
    for a in range(len(nodes)):
        b = int(res.mate[a])
        if b < a:
            continue
        total += int(d[a, b])
        ida, idb = nodes[a][0], nodes[b][0]
        if ida < NEAR_ID and idb < NEAR_ID:            # a < b: a has the lower site index
            ia, ja = nodes[a][1:]
            ib, jb = nodes[b][1:]
            na, fa = _near_far(L, is_star, ia, ja)
            nb, fb = _near_far(L, is_star, ib, jb)
            direct = abs(ia - ib) + abs(ja - jb)
            if direct <= na + nb and direct <= fa + fb:
                pairs.append((a, b))
            else:
                side = 0 if na + nb <= fa + fb else 1
                bmatch += [(a, side), (b, side)]
        elif ida < NEAR_ID:
            bmatch.append((a, 0 if idb == NEAR_ID else 1))
        else:
            logical = True
    part = np.zeros(lat.n_qubits, dtype=np.uint8)
    init._paint(lat, part, anyons, is_star, pairs, bmatch, logical)
    return part, total


def mwpm_representatives(lat, syn):
    """uint8 [4, n_q]: the minimum-weight matching start of every class.  Class
    c combines the x part of parity c & 1 with the z part of parity c >> 1."""
    syn = (np.asarray(syn) != 0).astype(np.uint8)
    xs = [type_part(lat, syn, False, b)[0] for b in (0, 1)]
    zs = [type_part(lat, syn, True, b)[0] for b in (0, 1)]
    out = np.zeros((4, lat.n_qubits), dtype=np.uint8)
    for c in range(4):
        out[c] = xs[c & 1] | (zs[c >> 1] << 1)
    return out


def type_weights(lat, syn):
    """int64 [2, 2]: minimum total distance of each type (0 plaquettes / x
    parts, 1 stars / z parts) and parity."""
    syn = (np.asarray(syn) != 0).astype(np.uint8)
    return np.array([[type_part(lat, syn, t == 1, b)[1] for b in (0, 1)] for t in (0, 1)],
                    dtype=np.int64)


__all__ = ["splitmix64", "tie_break", "min_weight_perfect_matching", "certificate_holds",
           "problem", "type_part", "mwpm_representatives", "type_weights", "geometry"]
