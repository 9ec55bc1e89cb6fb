// Minimum-weight perfect matching for the class starts of Sec. III (exact
// enhanced matching), written once for a wavefront: every scan over vertices
// runs across the lanes of the wave policy WV, and the tree and blossom
// surgery runs uniformly in every lane.  The kernel instantiates it with the
// 64-lane policy; a host build (one lane, no intrinsics) runs the same code.
//
// MW_FN qualifies device functions and MW_HD functions the host uses too.
// The policy WV provides:
//   int lane; static constexpr int N (lanes);
//   sync()                 order LDS writes of all lanes before later reads
//   argmin(key, idx)       smallest key over the lanes and the idx of a lane
//                          holding it, to every lane
//   any(p)                 p in some lane
//   compact(take, &count)  slot of this lane among the takers; count += takers
//   xor_word(p, v)         *p ^= v (atomically across lanes)
//   uni(x), uni64(x)       x, known to be the same in every lane (kept in
//                          scalar registers, so that branches on it are
//                          scalar)
//
// Problem (one anyon type, one line parity): vertices 0..nv-1 are the lit
// sites in ascending site order (crd = i << 8 | j), then NEAR (crd 0xff00) if
// the parity is odd, then FAR (crd 0xff01) if the number of lit sites plus
// the parity is odd.  Matching weight of a pair (twice the d 2^53 + 2 t of
// the plain definition, which orders matchings the same way):
// W = d 2^54 + 4 t with d the shortest-path distance
//   d(a, a') = min(|di| + |dj|, near(a) + near(a'), far(a) + far(a')),
//   d(a, NEAR) = near(a), d(a, FAR) = far(a), d(NEAR, FAR) = L,
// near/far = j+1 / L-1-j (plaquettes), i+1 / L-1-i (stars), and t the top 43
// bits of the 64-bit product K(a) K(a') of the ends' keys, K = splitmix64
// (Steele, Lea, Flood, OOPSLA 2014) at the site index (NEAR 4094, FAR 4095).
//
// Solver: Edmonds' primal-dual blossom algorithm for a minimum-weight perfect
// matching (dual bookkeeping as in Galil, ACM Computing Surveys 1986).  Node
// ids: vertices 0..cap-1, blossoms cap..cap+cap/2-1 (a laminar family of odd
// sets of at least 3 of nv vertices has fewer than nv/2 members).  Dual feasibility:
// slack(i, j) = W_ij - u_i - u_j + sum of z_B over blossoms holding both >= 0;
// between different outermost blossoms only the u terms remain.  Start: u_v
// = half the lightest pair at v (even, as every W is a multiple of 4) and the
// mutual nearest neighbours matched (their pairs are tight).  Every exposed
// vertex roots an alternating tree (S at even depth, T at odd).  All roots
// take every dual change, and tight edges join equal parities, so all S
// vertices share one parity and every dual change is an integer.  Every
// vertex keeps its least-slack edge (best, bestS) to an S vertex outside its
// own outermost node; each step takes the smallest of a free vertex's best,
// half an S vertex's best and half the dual of an outermost T blossom, and
// either acts on the tight edge or blossom it names (grow, shrink, augment,
// expand) or changes the duals by it.  After an augmentation only the two
// trees it joined dissolve; the others keep growing.
#pragma once

#include <stdint.h>

#ifndef MW_COUNT
#define MW_COUNT(what) ((void)0)
#endif

// A fact the compiler may rely on (the vertex count never exceeds the
// capacity, which the caller guarantees by sizing the state for the larger
// of a type's two problems: with a compile-time capacity of at most one
// wave, every pass over the vertices is a single guarded step); nothing on
// other compilers.
#ifdef __clang__
#define MW_ASSUME(cond) __builtin_assume(cond)
#else
#define MW_ASSUME(cond) ((void)0)
#endif

namespace mcmc {
namespace mw {

constexpr uint16_t NEAR_ID = 4094, FAR_ID = 4095;
constexpr uint16_t CRD_NEAR = 0xff00, CRD_FAR = 0xff01, CRD_DUMMY = 0xff02;
// weight of the dummy vertex's pairs other than the one with FAR: never tight
constexpr int64_t W_NEVER = (int64_t)1 << 61;
constexpr int64_t INF = (int64_t)1 << 62;
constexpr int16_t FREE = 0, S = 1, T = 2;
constexpr int ROWS = 2 * MCMC_L_MAX - 1;

MW_FN uint64_t splitmix64(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// vertex capacity of a problem at distance L (a multiple of 4, so that the
// regions below keep 8-byte alignment)
MW_HD int capacity(int L) { return ((L * (L - 1) + 2) + 3) & ~3; }

// bytes of one problem's state (nodes: nn = cap + cap / 2)
MW_HD size_t region_bytes(int cap) {
  // int64: u, best, key [cap], z [cap/2] (blossom b at z[b - cap])
  // int16: crd, mate, top, bestS, list, slist [cap], freel [cap/2]
  //        par, lab, tS, tT, base, bfirst, cnext, cprev, cex, cey, mark,
  //        tid [nn]
  //        stack [2 nn] ((node, vertex) pairs)
  return (size_t)cap * 83;
}

template <class WV>
struct Solver {
  WV wv;
  int64_t *u, *best, *z;
  uint64_t* key;
  uint16_t* crd;
  int16_t *mate, *top, *bestS, *freel, *list, *slist;
  int16_t *par, *lab, *tS, *tT, *base, *bfirst, *cnext, *cprev, *cex, *cey, *mark, *tid;
  int16_t* stk;
  int nv, cap, nn, L, nfree, k_lit;
  bool star, fail;

  MW_FN void carve(uint8_t* r, int cap_) {
    cap = cap_;
    nn = cap + cap / 2;
    int64_t* p64 = reinterpret_cast<int64_t*>(r);
    u = p64;
    best = p64 + cap;
    key = reinterpret_cast<uint64_t*>(p64 + 2 * cap);
    z = p64 + 3 * cap;
    int16_t* p16 = reinterpret_cast<int16_t*>(p64 + 3 * cap + cap / 2);
    crd = reinterpret_cast<uint16_t*>(p16); p16 += cap;
    mate = p16; p16 += cap;
    top = p16; p16 += cap;
    bestS = p16; p16 += cap;
    list = p16; p16 += cap;
    slist = p16; p16 += cap;
    freel = p16; p16 += cap / 2;
    int16_t** node[12] = {&par, &lab, &tS, &tT, &base, &bfirst, &cnext, &cprev, &cex, &cey,
                          &mark, &tid};
    for (int k = 0; k < 12; ++k) { *node[k] = p16; p16 += nn; }
    stk = p16;
  }
  MW_FN bool is_boundary(int v) const { return crd[v] >= CRD_NEAR; }
  // an element every lane reads at the same index, as a wave-uniform value
  MW_FN int rd(const int16_t* a, int i) const { return wv.uni((int)a[i]); }
  MW_FN int64_t rd(const int64_t* a, int i) const { return wv.uni64(a[i]); }

  // ---------------------------------------------------------------- weights
  MW_FN void near_far(int v, int& nr, int& fr) const {
    const int i = crd[v] >> 8, j = crd[v] & 255;
    if (star) { nr = i + 1; fr = L - 1 - i; } else { nr = j + 1; fr = L - 1 - j; }
  }
  MW_FN int dist(int a, int b) const {
    const bool ba = is_boundary(a), bb = is_boundary(b);
    if (!ba && !bb) {
      int na, fa, nb, fb;
      near_far(a, na, fa);
      near_far(b, nb, fb);
      const int di = (crd[a] >> 8) - (crd[b] >> 8), dj = (crd[a] & 255) - (crd[b] & 255);
      const int man = (di < 0 ? -di : di) + (dj < 0 ? -dj : dj);
      const int via = na + nb < fa + fb ? na + nb : fa + fb;
      return man < via ? man : via;
    }
    if (!ba) { int na, fa; near_far(a, na, fa); return crd[b] == CRD_NEAR ? na : fa; }
    if (!bb) { int nb, fb; near_far(b, nb, fb); return crd[a] == CRD_NEAR ? nb : fb; }
    return L;
  }
  MW_FN int64_t weight(int a, int b) const {
    if ((crd[a] | crd[b]) >= CRD_DUMMY && (crd[a] == CRD_DUMMY || crd[b] == CRD_DUMMY))
      return (crd[a] == CRD_FAR || crd[b] == CRD_FAR) ? 0 : W_NEVER;
    const uint64_t t = (key[a] * key[b]) >> 21;
    return ((int64_t)dist(a, b) << 54) + 4 * (int64_t)t;
  }
  MW_FN int64_t slack(int a, int b) const {
    MW_COUNT(slack);
    return weight(a, b) - u[a] - u[b];
  }

  // ---------------------------------------------------------------- structure
  // the child of node B that holds vertex v
  MW_FN int child_of(int B, int v) {
    int x = v;
    for (int g = 0; g < 2 * cap; ++g) {
      const int p = rd(par, x);
      if (p == B) return x;
      if (p < 0) break;
      x = p;
    }
    fail = true;
    return x;
  }
  // the S node above S node B in its tree, -1 for a root
  MW_FN int s_parent(int B) const {
    const int m = rd(mate, rd(base, B));
    if (m < 0) return -1;
    return rd(top, rd(tS, rd(top, m)));
  }
  // (x in X, y in the tree parent of X)
  MW_FN void up_edge(int X, int& x, int& y) const {
    if (rd(lab, X) == S) { x = rd(base, X); y = rd(mate, x); }
    else { x = rd(tT, X); y = rd(tS, X); }
  }
  // index of child c along B's cycle from its base child
  MW_FN int cycle_index(int B, int c) {
    int k = 0;
    for (int x = rd(bfirst, B); x != c; x = rd(cnext, x)) {
      if (++k > cap) { fail = true; return 0; }
    }
    return k;
  }

  // every vertex y with pred(y) into list; returns the count
  template <class P>
  MW_FN int collect(P pred) {
    int cnt = 0;
    for (int y0 = 0; y0 < nv; y0 += WV::N) {
      const int y = y0 + wv.lane;
      const bool take = y < nv && pred(y);
      const int slot = wv.compact(take, cnt);
      if (take) list[slot] = (int16_t)y;
    }
    wv.sync();
    return cnt;
  }

  // Each vertex x in list[0..cnt) has just become S: offer x to every vertex
  // outside its outermost node.  x keeps the least slack it had as a free or
  // T vertex, which is the same quantity when x had no S vertex in its
  // outermost node before (a grow, or the children of an expanded T
  // blossom): every S vertex was offered to it and every dual change updated
  // it; the new S vertices among themselves are covered by the offers.
  MW_FN void refresh(int cnt) {
    for (int k = 0; k < cnt; ++k) MW_COUNT(refresh_vertex);
    if (cnt == 0) return;
    for (int y = wv.lane; y < nv; y += WV::N) {  // in list order, as one offer after another
      const int ty = top[y];
      int64_t b = best[y];
      int bs = -1;
      for (int k = 0; k < cnt; ++k) {
        const int x = list[k];
        if (top[x] == ty) continue;
        const int64_t sl = slack(x, y);
        if (sl < b) { b = sl; bs = x; }
      }
      if (bs >= 0) { best[y] = b; bestS[y] = (int16_t)bs; }
    }
    wv.sync();
  }

  // Make vertex v the base of node B: at every blossom level, flip the even
  // alternating path between v's child and the base child (explicit stack).
  MW_FN void rotate(int B, int v) {
    int sp = 1;
    stk[0] = (int16_t)B;
    stk[1] = (int16_t)v;
    for (int guard = 0; sp > 0 && !fail; ++guard) {
      if (guard > 8 * cap) { fail = true; return; }
      --sp;
      const int Bn = rd(stk, 2 * sp), vv = rd(stk, 2 * sp + 1);
      if (Bn < cap) continue;  // a vertex is its own base
      const int c = child_of(Bn, vv);
      const int first = rd(bfirst, Bn);
      const int k = cycle_index(Bn, c);
      if (fail || sp + 1 > nn) { fail = true; return; }
      stk[2 * sp] = (int16_t)c;
      stk[2 * sp + 1] = (int16_t)vv;
      ++sp;
      if (k != 0) {
        const bool fwd = (k & 1) != 0;
        int pos = c;
        for (int steps = 0; pos != first; ++steps) {
          if (steps > cap || sp + 2 > nn) { fail = true; return; }
          const int a = rd(fwd ? cnext : cprev, pos);
          const int b = rd(fwd ? cnext : cprev, a);
          int x, y;  // x in a, y in b
          if (fwd) { x = rd(cex, a); y = rd(cey, a); } else { x = rd(cey, b); y = rd(cex, b); }
          mate[x] = (int16_t)y;
          mate[y] = (int16_t)x;
          stk[2 * sp] = (int16_t)a; stk[2 * sp + 1] = (int16_t)x; ++sp;
          stk[2 * sp] = (int16_t)b; stk[2 * sp + 1] = (int16_t)y; ++sp;
          pos = b;
        }
        bfirst[Bn] = (int16_t)c;
      }
      base[Bn] = (int16_t)vv;
    }
  }

  // match v to w and flip the alternating path from v up to its tree's root
  MW_FN void augment_path(int v, int w) {
    for (int g = 0; g <= cap && !fail; ++g) {
      const int B = rd(top, v);
      const int t0 = rd(mate, rd(base, B));
      rotate(B, v);
      mate[v] = (int16_t)w;
      if (t0 < 0) return;
      const int Tn = rd(top, t0);
      const int s = rd(tS, Tn), t = rd(tT, Tn);
      rotate(Tn, t);
      mate[t] = (int16_t)s;
      v = s;
      w = t;
    }
    fail = true;
  }

  // a new blossom from the tight edge (i, j) between two S nodes of one tree
  MW_FN void shrink(int i, int j) {
    const int Bi = rd(top, i), Bj = rd(top, j);
    int A = -1, g = 0;
    for (int x = Bi; x >= 0 && g <= cap; x = s_parent(x), ++g) mark[x] = 1;
    g = 0;
    for (int x = Bj; x >= 0 && g <= cap; x = s_parent(x), ++g)
      if (rd(mark, x)) { A = x; break; }
    g = 0;
    for (int x = Bi; x >= 0 && g <= cap; x = s_parent(x), ++g) mark[x] = 0;
    if (A < 0 || nfree <= 0) { fail = true; return; }
    const int b = rd(freel, --nfree);
    for (int X = Bi, gg = 0; X != A; ++gg) {  // going up from Bi: edge kept at X
      if (gg > 2 * cap) { fail = true; return; }
      int x, y;
      up_edge(X, x, y);
      const int P = rd(top, y);
      cnext[X] = (int16_t)P; cprev[P] = (int16_t)X;
      cex[X] = (int16_t)x; cey[X] = (int16_t)y;
      X = P;
    }
    for (int X = Bj, gg = 0; X != A; ++gg) {  // going down to Bj: edge kept at the parent
      if (gg > 2 * cap) { fail = true; return; }
      int x, y;
      up_edge(X, x, y);
      const int P = rd(top, y);
      cnext[P] = (int16_t)X; cprev[X] = (int16_t)P;
      cex[P] = (int16_t)y; cey[P] = (int16_t)x;
      X = P;
    }
    cnext[Bj] = (int16_t)Bi; cprev[Bi] = (int16_t)Bj;
    cex[Bj] = (int16_t)j; cey[Bj] = (int16_t)i;
    int c = A, gg = 0;
    do {
      par[c] = (int16_t)b;
      c = rd(cnext, c);
      if (++gg > 2 * cap) { fail = true; return; }
    } while (c != A);
    bfirst[b] = (int16_t)A;
    base[b] = (int16_t)rd(base, A);
    z[b - cap] = 0;
    lab[b] = S;
    tid[b] = (int16_t)rd(tid, A);
    par[b] = -1;
    wv.sync();
    // The vertices of b's T children become S: offer them to every vertex
    // outside b (as T vertices they already hold their least slack to the S
    // vertices outside their node).
    const int cnt = collect([&](int y) {
      const int ty = top[y];
      return par[ty] == b && lab[ty] == T;
    });
    for (int v = wv.lane; v < nv; v += WV::N)
      if (par[top[v]] == b) top[v] = (int16_t)b;
    wv.sync();
    refresh(cnt);
    // The S vertices outside b are those outside the old nodes minus b's
    // own, so a vertex of b keeps its least slack unless its partner is now
    // inside b.
    const int cnt2 = collect([&](int y) {
      const int s = bestS[y];
      return top[y] == b && s >= 0 && top[s] == b;
    });
    recompute(cnt2);
  }

  // dissolve the outermost T blossom B (dual zero): its children on the even
  // path from the child holding the label edge to the base child alternate
  // T, S, ..., T; the other children become free
  MW_FN void expand_t(int B) {
    const int s = rd(tS, B), t = rd(tT, B);
    const int c = child_of(B, t);
    const int first = rd(bfirst, B);
    const int k = cycle_index(B, c);
    if (fail) return;
    int x = first, g = 0;
    do {
      par[x] = -1;
      lab[x] = FREE;
      x = rd(cnext, x);
      if (++g > 2 * cap) { fail = true; return; }
    } while (x != first);
    const int16_t tree = (int16_t)rd(tid, B);
    lab[c] = T; tS[c] = (int16_t)s; tT[c] = (int16_t)t; tid[c] = tree;
    const bool fwd = (k & 1) != 0;
    int pos = c;
    for (g = 0; pos != first; ++g) {
      if (g > cap) { fail = true; return; }
      const int a = rd(fwd ? cnext : cprev, pos);
      const int b = rd(fwd ? cnext : cprev, a);
      int ex, ey;  // ex in a, ey in b
      if (fwd) { ex = rd(cex, a); ey = rd(cey, a); } else { ex = rd(cey, b); ey = rd(cex, b); }
      lab[a] = S;
      mark[a] = 1;
      lab[b] = T; tS[b] = (int16_t)ex; tT[b] = (int16_t)ey;
      tid[a] = tid[b] = tree;
      pos = b;
    }
    base[B] = -1;
    lab[B] = FREE;
    freel[nfree++] = (int16_t)B;
    wv.sync();
    for (int v = wv.lane; v < nv; v += WV::N) {
      if (top[v] != B) continue;
      int y = v;
      for (int gg = 0; gg < 2 * cap && par[y] >= 0; ++gg) y = par[y];
      top[v] = (int16_t)y;
    }
    wv.sync();
    const int cnt = collect([&](int y) { return mark[top[y]] != 0; });
    x = first;
    g = 0;
    do {
      mark[x] = 0;
      x = rd(cnext, x);
    } while (x != first && ++g <= 2 * cap);
    wv.sync();
    refresh(cnt);
  }

  // ---------------------------------------------------------------- solve
  // best / bestS of every vertex in list[0..cnt): its least slack to an S
  // vertex outside its outermost node
  MW_FN void recompute(int cnt) {
    if (cnt == 0) return;
    for (int k = 0; k < cnt; ++k) MW_COUNT(recompute_vertex);
    // the S vertices, in ascending order
    int ns = 0;
    for (int x0 = 0; x0 < nv; x0 += WV::N) {
      const int x = x0 + wv.lane;
      const bool take = x < nv && lab[top[x]] == S;
      const int slot = wv.compact(take, ns);
      if (take) slist[slot] = (int16_t)x;
    }
    wv.sync();
    // Each vertex takes an aligned group of 2^lg lanes, lane r of the group
    // scanning S list entries r, r + 2^lg, ..., then a (slack, S vertex)
    // minimum within the group.  lg from a cost estimate: a slack counts 4, a
    // reduction step 1 and a pass over N >> lg vertices 4 on its own.
    int lg = 0, cost = 0x7fffffff;
    for (int l = 0; (1 << l) <= WV::N; ++l) {
      const int per = (ns + (1 << l) - 1) >> l, grp = WV::N >> l;
      const int c = (cnt + grp - 1) / grp * (4 * per + l + 4);
      if (c < cost) { cost = c; lg = l; }
    }
    const int P = 1 << lg, grp = WV::N >> lg, r = wv.lane & (P - 1);
    for (int k0 = 0; k0 < cnt; k0 += grp) {
      const int k = k0 + (wv.lane >> lg);
      int y = 0;
      int64_t b = INF;
      int bs = 0x7fff;
      if (k < cnt) {
        y = list[k];
        const int ty = top[y];
        for (int m = r; m < ns; m += P) {  // ascending x: ties keep the smaller
          const int x = slist[m];
          if (top[x] == ty) continue;
          const int64_t sl = slack(x, y);
          if (sl < b) { b = sl; bs = x; }
        }
      }
      wv.seg_argmin(b, bs, lg);
      if (k < cnt && r == P - 1) {
        best[y] = b;
        bestS[y] = (int16_t)(b < INF ? bs : -1);
      }
    }
    wv.sync();
  }

  // The tree of a labelled outermost node is identified by its exposed
  // vertex (tid), set when the node is labelled: exposed vertices at the
  // start, the tree of the edge's S end on a grow, the tree of the shrunk
  // cycle on a shrink, the expanded blossom's tree on an expand.

  MW_FN void solve() {
    for (int x = wv.lane; x < nn; x += WV::N) {
      par[x] = -1;
      lab[x] = FREE;
      mark[x] = 0;
      bfirst[x] = -1;
      base[x] = (int16_t)(x < cap ? x : -1);
      tS[x] = tT[x] = cnext[x] = cprev[x] = cex[x] = cey[x] = 0;  // always valid indices
    }
    for (int v = wv.lane; v < cap; v += WV::N) {
      mate[v] = -1;
      top[v] = (int16_t)v;
    }
    for (int k = wv.lane; k < cap / 2; k += WV::N) {
      z[k] = 0;
      freel[k] = (int16_t)(nn - 1 - k);
    }
    nfree = cap / 2;
    wv.sync();
    // start: u_v = half the lightest pair at v (W is a multiple of 4, so every
    // u is even and every S vertex keeps the parity of the roots); mutual
    // nearest neighbours are tight and matched
    for (int v = wv.lane; v < nv; v += WV::N) {
      int64_t b = INF;
      int bs = -1;
      for (int x = 0; x < nv; ++x) {
        if (x == v) continue;
        const int64_t w = weight(x, v);
        if (w < b) { b = w; bs = x; }
      }
      u[v] = b >> 1;
      bestS[v] = (int16_t)bs;
    }
    wv.sync();
    int matched = 0;
    for (int v0 = 0; v0 < nv; v0 += WV::N) {
      const int v = v0 + wv.lane;
      bool pair = false;
      if (v < nv) {
        const int w = bestS[v];
        pair = w > v && bestS[w] == v;
        if (pair) { mate[v] = (int16_t)w; mate[w] = (int16_t)v; }
      }
      int dummy = 0;
      wv.compact(pair, dummy);
      matched += 2 * dummy;
    }
    wv.sync();
    // then each exposed vertex in turn raises its dual by its least slack
    // (every slack stays >= 0; slacks are even, so u stays even) and is
    // matched along the edge that became tight when that edge's other end is
    // still exposed (exposed ends first among equal slacks)
    for (int v = 0; v < nv; ++v) {
      if (rd(mate, v) >= 0) continue;
      int64_t key = INF;
      int idx = 0x7fff;
      for (int w = wv.lane; w < nv; w += WV::N) {
        if (w == v) continue;
        const int64_t k = (slack(v, w) << 1) | (mate[w] >= 0 ? 1 : 0);
        if (k < key) { key = k; idx = w; }
      }
      wv.argmin(key, idx);
      wv.sync();
      if (key >= INF) continue;
      u[v] += key >> 1;
      if ((key & 1) == 0) {
        mate[v] = (int16_t)idx;
        mate[idx] = (int16_t)v;
        matched += 2;
      }
      wv.sync();
    }
    for (int v = wv.lane; v < nv; v += WV::N)
      if (mate[v] < 0) { lab[v] = S; tid[v] = (int16_t)v; }
    wv.sync();
    {
      const int cnt = collect([&](int y) { (void)y; return true; });
      recompute(cnt);
    }
    run(matched);
  }

  // The other parity of the type just solved, from its solution: the
  // structure (matching, blossoms, duals) stays and two exposed vertices join.
  // With an even number k of lit sites the solved problem had no boundary
  // vertex and NEAR and FAR join.  With k odd it had FAR; NEAR joins with a
  // dummy vertex whose only pair is with FAR (weight 0), so that a perfect
  // matching matches the dummy to FAR and the rest is a perfect matching of
  // the lit sites and NEAR.  The new vertices' duals are the largest that keep
  // every slack non-negative, with a common parity.
  MW_FN void solve_other_parity(const uint8_t* sy) {
    const int k = k_lit;
    if (fail) { load(sy, L, star, 1); solve(); return; }
    const bool odd = (k & 1) != 0;
    const int va = odd ? k + 1 : k, vb = va + 1;  // the two new vertices
    if (wv.lane == 0) {
      crd[va] = CRD_NEAR; key[va] = splitmix64(NEAR_ID);
      if (odd) { crd[vb] = CRD_DUMMY; key[vb] = 0; }
      else { crd[vb] = CRD_FAR; key[vb] = splitmix64(FAR_ID); }
    }
    for (int v = va + wv.lane; v <= vb; v += WV::N) {
      mate[v] = -1; top[v] = (int16_t)v; par[v] = -1; base[v] = (int16_t)v;
      mark[v] = 0; bfirst[v] = -1;
    }
    const int matched = nv;
    nv = vb + 1;
    wv.sync();
    int64_t ua = new_dual(va, vb, 0), ub = new_dual(vb, va, 0);
    // the pair of the two new vertices: lower the larger dual until its slack
    // is >= 0 (the amount is even)
    const int64_t over = u_parity_floor(weight(va, vb) - ua - ub);
    if (over < 0) { if (ua >= ub) ua += over; else ub += over; }
    if (wv.lane == 0) { u[va] = ua; u[vb] = ub; }
    wv.sync();
    for (int x = wv.lane; x < nn; x += WV::N) lab[x] = FREE;
    wv.sync();
    for (int v = wv.lane; v < nv; v += WV::N)
      if (mate[v] < 0) { lab[top[v]] = S; tid[top[v]] = (int16_t)v; }
    wv.sync();
    const int cnt = collect([&](int y) { (void)y; return true; });
    recompute(cnt);
    run(matched);
  }

  // the largest even number <= x (two's complement)
  MW_FN static int64_t u_parity_floor(int64_t x) { return x - (x & 1); }

  // dual of new vertex v: min over the old vertices w (not v, not `skip`) of
  // W(v, w) - u_w, rounded down to parity `par`
  MW_FN int64_t new_dual(int v, int skip, int64_t par_) {
    int64_t b = INF;
    int bi = 0;
    for (int w = wv.lane; w < nv; w += WV::N) {
      if (w == v || w == skip) continue;
      const int64_t d = weight(v, w) - u[w];
      if (d < b) b = d;
    }
    wv.argmin(b, bi);
    const int64_t down = u_parity_floor(b - par_) + par_;
    return down;
  }

  // The least key over the candidates (a free vertex's best, half an S
  // vertex's best, half the dual of an outermost T blossom) and the index
  // holding it, ties to the lowest index; false if an S vertex holds an odd
  // best, which a correct dual state never has.
  MW_FN bool scan(int64_t& key, int& idx) {
    MW_COUNT(event);
    key = INF;
    idx = 0x7fff;
    bool odd = false;
    for (int j = wv.lane; j < nv; j += WV::N) {
      const int16_t l = lab[top[j]];
      const int64_t b = best[j];
      if (b >= INF || l == T) continue;
      int64_t kk = b;
      if (l == S) {
        odd |= (b & 1) != 0;  // the slack between two S vertices is even
        kk = b >> 1;
      }
      if (kk < key || (kk == key && j < idx)) { key = kk; idx = j; }
    }
    if (nfree < cap / 2) {  // blossoms exist (indices >= cap)
      for (int b = cap + wv.lane; b < nn; b += WV::N) {
        if (base[b] < 0 || par[b] >= 0 || lab[b] != T) continue;
        const int64_t kk = z[b - cap] >> 1;
        if (kk < key || (kk == key && b < idx)) { key = kk; idx = b; }
      }
    }
    wv.argmin(key, idx);
    return !wv.any(odd);
  }

  // the event loop, from `matched` matched vertices and a labelled forest
  MW_FN void run(int matched) {
    const int ev_max = 16 * nv * (nv / 2 + 2) + 64;
    // A dual change by the least key lowers every candidate's key by that
    // amount (both ends of an S-S slack move), so the step after it acts on
    // the same candidate at key 0 without a scan.
    bool rescan = true;
    int64_t key = INF;
    int idx = 0x7fff;
    for (int ev = 0; matched < nv && !fail; ++ev) {
      MW_ASSUME(nv >= 0 && nv <= cap);
      if (ev > ev_max) { fail = true; break; }
      if (!rescan) {
        key = 0;
      } else if (!scan(key, idx)) {
        fail = true;
        break;
      }
      rescan = true;
      if (key == 0 && idx >= cap) {
        MW_COUNT(expand);
        expand_t(idx);
      } else if (key == 0) {
        const int j = idx, i = rd(bestS, j);
        if (i < 0) { fail = true; break; }
        const int Bj = rd(top, j);
        if (rd(lab, Bj) == FREE) {  // grow: Bj becomes T, its mate's node S
          MW_COUNT(grow);
          const int mb = rd(mate, rd(base, Bj));
          if (mb < 0) { fail = true; break; }
          const int16_t tree = (int16_t)rd(tid, rd(top, i));
          lab[Bj] = T;
          tS[Bj] = (int16_t)i;
          tT[Bj] = (int16_t)j;
          tid[Bj] = tree;
          const int Bm = rd(top, mb);
          lab[Bm] = S;
          tid[Bm] = tree;
          wv.sync();
          const int cnt = collect([&](int y) { return top[y] == Bm; });
          refresh(cnt);
        } else {
          const int ri = rd(tid, rd(top, i)), rj = rd(tid, Bj);
          if (ri != rj) {
            MW_COUNT(augment);
            // the two trees dissolve after the augmentation; the others stay
            for (int x = wv.lane; x < nn; x += WV::N) {
              if (par[x] >= 0 || lab[x] == FREE || (x >= cap && base[x] < 0) ||
                  (x < cap && x >= nv))
                continue;
              const int r = tid[x];
              mark[x] = (int16_t)(r == ri || r == rj);
            }
            wv.sync();
            // A least slack to the S vertices outside a node can only rise
            // when some of them stop being S, and then only where it was
            // held by one of them: the others keep theirs, whatever their
            // own label becomes.
            const int cnt = collect([&](int y) {
              return bestS[y] >= 0 && mark[top[bestS[y]]] != 0;
            });
            augment_path(i, j);
            augment_path(j, i);
            matched += 2;
            wv.sync();
            for (int x = wv.lane; x < nn; x += WV::N) {
              if (mark[x]) lab[x] = FREE;
              mark[x] = 0;
            }
            wv.sync();
            recompute(cnt);
          } else {
            MW_COUNT(shrink);
            shrink(i, j);
          }
        }
      } else {
        const int64_t delta = key;
        if (delta >= INF) { fail = true; break; }
        MW_COUNT(dual);
        for (int v = wv.lane; v < nv; v += WV::N) {
          const int16_t l = lab[top[v]];
          const int64_t b = best[v];
          if (l == S) {
            u[v] += delta;
            if (b < INF) best[v] = b - 2 * delta;
          } else if (l == T) {
            u[v] -= delta;
          } else if (b < INF) {
            best[v] = b - delta;
          }
        }
        if (nfree < cap / 2) {
          for (int b = cap + wv.lane; b < nn; b += WV::N) {
            if (base[b] < 0 || par[b] >= 0) continue;
            if (lab[b] == S) z[b - cap] += 2 * delta;
            else if (lab[b] == T) z[b - cap] -= 2 * delta;
          }
        }
        wv.sync();
        rescan = false;
      }
    }
    if (matched < nv) fail = true;
  }

  // ---------------------------------------------------------------- load, paint
  // vertices of type `star` with parity `parity` from a syndrome of distance L
  MW_FN void load(const uint8_t* sy, int L_, bool star_, int parity) {
    L = L_;
    star = star_;
    fail = false;
    const int nsite = L * (L - 1);
    const int first = star ? 0 : nsite, nc = star ? L : L - 1;
    int k = 0;
    for (int s0 = 0; s0 < nsite; s0 += WV::N) {
      const int t = s0 + wv.lane;
      const bool lit = t < nsite && sy[first + t] != 0;
      const int slot = wv.compact(lit, k);
      if (lit) {
        key[slot] = splitmix64((uint64_t)(first + t));
        crd[slot] = (uint16_t)(((t / nc) << 8) | (t % nc));
      }
    }
    k_lit = k;
    int n = k;
    if (wv.lane == 0) {
      if (parity) { key[n] = splitmix64(NEAR_ID); crd[n] = CRD_NEAR; }
      if ((k + parity) & 1) { key[n + parity] = splitmix64(FAR_ID); crd[n + parity] = CRD_FAR; }
    }
    n += parity + ((k + parity) & 1);
    nv = n;
    wv.sync();
  }

  MW_FN void xor_fields(uint32_t* pl, int row, int lo, int hi) {
    // toggle fields lo..hi-1 of grid row `row`
    if (hi > lo) wv.xor_word(&pl[row], ((hi >= 32 ? 0u : (1u << hi)) - 1u) ^ ((1u << lo) - 1u));
  }
  MW_FN void paint_side(uint32_t* pl, int i, int j, int side) {
    if (!star) {
      if (side == 0) xor_fields(pl, 2 * i, 0, j + 1);
      else xor_fields(pl, 2 * i, j + 1, L);
    } else {
      const int r0 = side == 0 ? 0 : i + 1, r1 = side == 0 ? i + 1 : L;
      for (int k = r0; k < r1; ++k) wv.xor_word(&pl[2 * k], 1u << j);
    }
  }
  MW_FN void paint_logical(uint32_t* pl) {
    if (!star) xor_fields(pl, 0, 0, L);
    else for (int k = 0; k < L; ++k) wv.xor_word(&pl[2 * k], 1u);
  }

  // XOR the solved part into plane pl (bit f of word r = field f of grid row
  // r).  A problem that hit a bound gets the canonical part instead (every
  // anyon's string to the near boundary, and the logical if the parity needs
  // it).
  MW_FN void paint(uint32_t* pl, int parity) {
    if (fail) {
      for (int a = wv.lane; a < k_lit; a += WV::N) paint_side(pl, crd[a] >> 8, crd[a] & 255, 0);
      if (wv.lane == 0 && (k_lit & 1) != parity) paint_logical(pl);
      return;
    }
    for (int a = wv.lane; a < nv; a += WV::N) {
      const int b = mate[a];
      if (b < a || crd[a] == CRD_DUMMY || crd[b] == CRD_DUMMY) continue;
      const bool ba = is_boundary(a), bb = is_boundary(b);
      if (!ba && !bb) {
        const int i1 = crd[a] >> 8, j1 = crd[a] & 255, i2 = crd[b] >> 8, j2 = crd[b] & 255;
        int na, fa, nb, fb;
        near_far(a, na, fa);
        near_far(b, nb, fb);
        const int di = i1 - i2, dj = j1 - j2;
        const int man = (di < 0 ? -di : di) + (dj < 0 ? -dj : dj);
        if (man <= na + nb && man <= fa + fb) {
          const int jl = j1 < j2 ? j1 : j2, jh = j1 < j2 ? j2 : j1;
          if (!star) {  // along grid row 2 i1, then down grid column 2 j2 + 1
            xor_fields(pl, 2 * i1, jl + 1, jh + 1);
            for (int i = i1; i < i2; ++i) wv.xor_word(&pl[2 * i + 1], 1u << j2);
          } else {      // down grid column 2 j1, then along grid row 2 i2 + 1
            for (int i = i1; i < i2; ++i) wv.xor_word(&pl[2 * i + 2], 1u << j1);
            xor_fields(pl, 2 * i2 + 1, jl, jh);
          }
        } else {
          const int side = na + nb <= fa + fb ? 0 : 1;
          paint_side(pl, i1, j1, side);
          paint_side(pl, i2, j2, side);
        }
      } else if (!ba) {
        paint_side(pl, crd[a] >> 8, crd[a] & 255, crd[b] == CRD_NEAR ? 0 : 1);
      } else {
        paint_logical(pl);
      }
    }
  }
};

}  // namespace mw
}  // namespace mcmc
