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
//   argmin(key, idx)       smallest (key, idx) over the lanes, to every lane
//   any(p)                 p in some lane
//   compact(take, &count)  slot of this lane among the takers; count += takers
//   xor_word(p, v)         *p ^= v (atomically across lanes)
//
// Problem (one anyon type, one line parity): vertices 0..nv-1 are the lit
// sites in ascending site order (nid = site index, crd = i << 8 | j), then
// NEAR (id 4094) if the parity is odd, then FAR (id 4095) if the number of
// lit sites plus the parity is odd.  Matching weight of a pair:
// W = d 2^53 + 2 t with d the shortest-path distance
//   d(a, a') = min(|di| + |dj|, near(a) + near(a'), far(a) + far(a')),
//   d(a, NEAR) = near(a), d(a, FAR) = far(a), d(NEAR, FAR) = L,
// near/far = j+1 / L-1-j (plaquettes), i+1 / L-1-i (stars), and t the top 43
// bits of splitmix64 (Steele, Lea, Flood, OOPSLA 2014) at state
// (min(id) << 12) | max(id).
//
// Solver: Edmonds' primal-dual blossom algorithm for a minimum-weight perfect
// matching (dual bookkeeping as in Galil, ACM Computing Surveys 1986).  Node
// ids: vertices 0..cap-1, blossoms cap..2cap-1.  Dual feasibility:
// slack(i, j) = W_ij - u_i - u_j + sum of z_B over blossoms holding both >= 0;
// between different outermost blossoms only the u terms remain.  All W are
// even and all u start at 0, so every dual change is an integer.  Each stage
// labels the outermost nodes with an exposed base S and grows alternating
// trees until an augmenting path joins two of them; every vertex keeps its
// least-slack edge (best, bestS) to an S vertex outside its own outermost
// node, and each step takes the smallest of: a free vertex's best, half an S
// vertex's best, half the dual of an outermost T blossom.
#pragma once

#include <stdint.h>

namespace mcmc {
namespace mw {

constexpr uint16_t NEAR = 4094, FAR = 4095;
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

// bytes of one problem's state
MW_HD size_t region_bytes(int cap) {
  // int64: u, best [cap], z [cap] (blossom b at z[b - cap])
  // int16: nid, crd, mate, top, bestS, freel, list [cap]
  //        par, lab, tS, tT, base, bfirst, cnext, cprev, cex, cey, mark [2 cap]
  //        stack [4 cap] ((node, vertex) pairs)
  return (size_t)cap * (3 * 8 + 7 * 2 + 11 * 2 * 2 + 4 * 2);
}

template <class WV>
struct Solver {
  WV wv;
  int64_t *u, *best, *z;
  uint16_t *nid, *crd;
  int16_t *mate, *top, *bestS, *freel, *list;
  int16_t *par, *lab, *tS, *tT, *base, *bfirst, *cnext, *cprev, *cex, *cey, *mark;
  int16_t* stk;
  int nv, cap, L, nfree, k_lit;
  bool star, fail;

  MW_FN void carve(uint8_t* r, int cap_) {
    cap = cap_;
    int64_t* p64 = reinterpret_cast<int64_t*>(r);
    u = p64;
    best = p64 + cap;
    z = p64 + 2 * cap;
    int16_t* p16 = reinterpret_cast<int16_t*>(p64 + 3 * cap);
    nid = reinterpret_cast<uint16_t*>(p16); p16 += cap;
    crd = reinterpret_cast<uint16_t*>(p16); p16 += cap;
    mate = p16; p16 += cap;
    top = p16; p16 += cap;
    bestS = p16; p16 += cap;
    freel = p16; p16 += cap;
    list = p16; p16 += cap;
    par = p16; p16 += 2 * cap;
    lab = p16; p16 += 2 * cap;
    tS = p16; p16 += 2 * cap;
    tT = p16; p16 += 2 * cap;
    base = p16; p16 += 2 * cap;
    bfirst = p16; p16 += 2 * cap;
    cnext = p16; p16 += 2 * cap;
    cprev = p16; p16 += 2 * cap;
    cex = p16; p16 += 2 * cap;
    cey = p16; p16 += 2 * cap;
    mark = p16; p16 += 2 * cap;
    stk = p16;
  }

  // ---------------------------------------------------------------- weights
  MW_FN void near_far(int v, int& nr, int& fr) const {
    const int i = crd[v] >> 8, j = crd[v] & 255;
    if (star) { nr = i + 1; fr = L - 1 - i; } else { nr = j + 1; fr = L - 1 - j; }
  }
  MW_FN int dist(int a, int b) const {
    const int ia = nid[a], ib = nid[b];
    if (ia < NEAR && ib < NEAR) {
      int na, fa, nb, fb;
      near_far(a, na, fa);
      near_far(b, nb, fb);
      const int di = (crd[a] >> 8) - (crd[b] >> 8), dj = (crd[a] & 255) - (crd[b] & 255);
      const int man = (di < 0 ? -di : di) + (dj < 0 ? -dj : dj);
      const int via = na + nb < fa + fb ? na + nb : fa + fb;
      return man < via ? man : via;
    }
    if (ia < NEAR) { int na, fa; near_far(a, na, fa); return ib == NEAR ? na : fa; }
    if (ib < NEAR) { int nb, fb; near_far(b, nb, fb); return ia == NEAR ? nb : fb; }
    return L;
  }
  MW_FN int64_t weight(int a, int b) const {
    const uint32_t ia = nid[a], ib = nid[b];
    const uint32_t lo = ia < ib ? ia : ib, hi = ia < ib ? ib : ia;
    const uint64_t t = splitmix64(((uint64_t)lo << 12) | hi) >> 21;
    return ((int64_t)dist(a, b) << 53) + 2 * (int64_t)t;
  }
  MW_FN int64_t slack(int a, int b) const { return weight(a, b) - u[a] - u[b]; }

  // ---------------------------------------------------------------- structure
  // the child of node B that holds vertex v
  MW_FN int child_of(int B, int v) {
    int x = v;
    for (int g = 0; g < 2 * cap && par[x] != B; ++g) {
      if (par[x] < 0) break;
      x = par[x];
    }
    if (par[x] != B) fail = true;
    return x;
  }
  // the S node above S node B in its tree, -1 for a root
  MW_FN int s_parent(int B) const {
    const int m = mate[base[B]];
    if (m < 0) return -1;
    return top[tS[top[m]]];
  }
  // (x in X, y in the tree parent of X)
  MW_FN void up_edge(int X, int& x, int& y) const {
    if (lab[X] == S) { x = base[X]; y = mate[x]; }
    else { x = tT[X]; y = tS[X]; }
  }
  // index of child c along B's cycle from its base child
  MW_FN int cycle_index(int B, int c) {
    int k = 0;
    for (int x = bfirst[B]; x != c; x = cnext[x]) {
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

  // Each vertex x in list[0..cnt) is S: recompute its least slack to S
  // vertices outside its outermost node, and offer x to every vertex outside
  // that node.
  MW_FN void refresh(int cnt) {
    for (int k = 0; k < cnt; ++k) {
      const int x = list[k];
      const int tx = top[x];
      int64_t bk = INF;
      int bi = 0x7fff;
      for (int y = wv.lane; y < nv; y += WV::N) {
        const int ty = top[y];
        if (ty == tx) continue;
        const int64_t sl = slack(x, y);
        if (sl < best[y]) { best[y] = sl; bestS[y] = (int16_t)x; }
        if (lab[ty] == S && sl < bk) { bk = sl; bi = y; }
      }
      wv.argmin(bk, bi);
      wv.sync();
      best[x] = bk;
      bestS[x] = (int16_t)(bk < INF ? bi : -1);
      wv.sync();
    }
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
      const int Bn = stk[2 * sp], vv = stk[2 * sp + 1];
      if (Bn < cap) continue;  // a vertex is its own base
      const int c = child_of(Bn, vv);
      const int first = bfirst[Bn];
      const int k = cycle_index(Bn, c);
      if (fail || sp + 1 > 2 * cap) { fail = true; return; }
      stk[2 * sp] = (int16_t)c;
      stk[2 * sp + 1] = (int16_t)vv;
      ++sp;
      if (k != 0) {
        const bool fwd = (k & 1) != 0;
        int pos = c;
        for (int steps = 0; pos != first; ++steps) {
          if (steps > cap || sp + 2 > 2 * cap) { fail = true; return; }
          const int a = fwd ? cnext[pos] : cprev[pos];
          const int b = fwd ? cnext[a] : cprev[a];
          int x, y;  // x in a, y in b
          if (fwd) { x = cex[a]; y = cey[a]; } else { x = cey[b]; y = cex[b]; }
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
      const int B = top[v];
      const int t0 = mate[base[B]];
      rotate(B, v);
      mate[v] = (int16_t)w;
      if (t0 < 0) return;
      const int Tn = top[t0];
      const int s = tS[Tn], t = tT[Tn];
      rotate(Tn, t);
      mate[t] = (int16_t)s;
      v = s;
      w = t;
    }
    fail = true;
  }

  // a new blossom from the tight edge (i, j) between two S nodes of one tree
  MW_FN void shrink(int i, int j) {
    const int Bi = top[i], Bj = top[j];
    int A = -1, g = 0;
    for (int x = Bi; x >= 0 && g <= cap; x = s_parent(x), ++g) mark[x] = 1;
    g = 0;
    for (int x = Bj; x >= 0 && g <= cap; x = s_parent(x), ++g)
      if (mark[x]) { A = x; break; }
    g = 0;
    for (int x = Bi; x >= 0 && g <= cap; x = s_parent(x), ++g) mark[x] = 0;
    if (A < 0 || nfree <= 0) { fail = true; return; }
    const int b = freel[--nfree];
    for (int X = Bi, gg = 0; X != A; ++gg) {  // going up from Bi: edge kept at X
      if (gg > 2 * cap) { fail = true; return; }
      int x, y;
      up_edge(X, x, y);
      const int P = top[y];
      cnext[X] = (int16_t)P; cprev[P] = (int16_t)X;
      cex[X] = (int16_t)x; cey[X] = (int16_t)y;
      X = P;
    }
    for (int X = Bj, gg = 0; X != A; ++gg) {  // going down to Bj: edge kept at the parent
      if (gg > 2 * cap) { fail = true; return; }
      int x, y;
      up_edge(X, x, y);
      const int P = top[y];
      cnext[P] = (int16_t)X; cprev[X] = (int16_t)P;
      cex[P] = (int16_t)y; cey[P] = (int16_t)x;
      X = P;
    }
    cnext[Bj] = (int16_t)Bi; cprev[Bi] = (int16_t)Bj;
    cex[Bj] = (int16_t)j; cey[Bj] = (int16_t)i;
    int c = A, gg = 0;
    do {
      par[c] = (int16_t)b;
      c = cnext[c];
      if (++gg > 2 * cap) { fail = true; return; }
    } while (c != A);
    bfirst[b] = (int16_t)A;
    base[b] = base[A];
    z[b - cap] = 0;
    lab[b] = S;
    par[b] = -1;
    wv.sync();
    for (int v = wv.lane; v < nv; v += WV::N)
      if (par[top[v]] == b) top[v] = (int16_t)b;
    wv.sync();
    const int cnt = collect([&](int y) { return top[y] == b; });
    refresh(cnt);
  }

  // dissolve the outermost T blossom B (dual zero): its children on the even
  // path from the child holding the label edge to the base child alternate
  // T, S, ..., T; the other children become free
  MW_FN void expand_t(int B) {
    const int s = tS[B], t = tT[B];
    const int c = child_of(B, t);
    const int first = bfirst[B];
    const int k = cycle_index(B, c);
    if (fail) return;
    int x = first, g = 0;
    do {
      par[x] = -1;
      lab[x] = FREE;
      x = cnext[x];
      if (++g > 2 * cap) { fail = true; return; }
    } while (x != first);
    lab[c] = T; tS[c] = (int16_t)s; tT[c] = (int16_t)t;
    const bool fwd = (k & 1) != 0;
    int pos = c;
    for (g = 0; pos != first; ++g) {
      if (g > cap) { fail = true; return; }
      const int a = fwd ? cnext[pos] : cprev[pos];
      const int b = fwd ? cnext[a] : cprev[a];
      int ex, ey;  // ex in a, ey in b
      if (fwd) { ex = cex[a]; ey = cey[a]; } else { ex = cey[b]; ey = cex[b]; }
      lab[a] = S;
      mark[a] = 1;
      lab[b] = T; tS[b] = (int16_t)ex; tT[b] = (int16_t)ey;
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
      x = cnext[x];
    } while (x != first && ++g <= 2 * cap);
    wv.sync();
    refresh(cnt);
  }

  // ---------------------------------------------------------------- solve
  MW_FN void solve() {
    for (int x = wv.lane; x < 2 * cap; x += WV::N) {
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
      u[v] = 0;
      z[v] = 0;
      freel[v] = (int16_t)(2 * cap - 1 - v);
    }
    nfree = cap;
    wv.sync();
    int matched = 0;
    for (int stage = 0; stage <= nv / 2 && matched < nv && !fail; ++stage) {
      for (int x = wv.lane; x < 2 * cap; x += WV::N) lab[x] = FREE;
      wv.sync();
      for (int v = wv.lane; v < nv; v += WV::N)
        if (mate[v] < 0) lab[top[v]] = S;
      wv.sync();
      for (int y = wv.lane; y < nv; y += WV::N) {
        const int ty = top[y];
        int64_t b = INF;
        int bs = -1;
        for (int x = 0; x < nv; ++x) {
          const int tx = top[x];
          if (tx == ty || lab[tx] != S) continue;
          const int64_t sl = slack(x, y);
          if (sl < b) { b = sl; bs = x; }
        }
        best[y] = b;
        bestS[y] = (int16_t)bs;
      }
      wv.sync();
      bool augmented = false;
      const int ev_max = 8 * nv + 64;
      for (int ev = 0; !augmented && !fail; ++ev) {
        if (ev > ev_max) { fail = true; break; }
        int64_t key = INF;
        int idx = 0x7fff;
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
        wv.argmin(key, idx);
        int64_t bkey = INF;
        int bidx = 0x7fff;
        for (int b = cap + wv.lane; b < 2 * cap; b += WV::N) {
          if (base[b] < 0 || par[b] >= 0 || lab[b] != T) continue;
          const int64_t kk = z[b - cap] >> 1;
          if (kk < bkey || (kk == bkey && b < bidx)) { bkey = kk; bidx = b; }
        }
        wv.argmin(bkey, bidx);
        if (wv.any(odd)) { fail = true; break; }
        if (key == 0) {
          const int j = idx, i = bestS[j];
          if (i < 0) { fail = true; break; }
          const int Bj = top[j];
          if (lab[Bj] == FREE) {  // grow: Bj becomes T, its mate's node S
            const int mb = mate[base[Bj]];
            if (mb < 0) { fail = true; break; }
            lab[Bj] = T;
            tS[Bj] = (int16_t)i;
            tT[Bj] = (int16_t)j;
            const int Bm = top[mb];
            lab[Bm] = S;
            wv.sync();
            const int cnt = collect([&](int y) { return top[y] == Bm; });
            refresh(cnt);
          } else {
            int ri = top[i], rj = Bj, g = 0;
            for (int x = s_parent(ri); x >= 0 && g <= cap; x = s_parent(x), ++g) ri = x;
            g = 0;
            for (int x = s_parent(rj); x >= 0 && g <= cap; x = s_parent(x), ++g) rj = x;
            if (ri != rj) {
              augment_path(i, j);
              augment_path(j, i);
              matched += 2;
              augmented = true;
              wv.sync();
            } else {
              shrink(i, j);
            }
          }
        } else if (bkey == 0) {
          expand_t(bidx);
        } else {
          const int64_t delta = key < bkey ? key : bkey;
          if (delta >= INF) { fail = true; break; }
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
          for (int b = cap + wv.lane; b < 2 * cap; b += WV::N) {
            if (base[b] < 0 || par[b] >= 0) continue;
            if (lab[b] == S) z[b - cap] += 2 * delta;
            else if (lab[b] == T) z[b - cap] -= 2 * delta;
          }
          wv.sync();
        }
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
        nid[slot] = (uint16_t)(first + t);
        crd[slot] = (uint16_t)(((t / nc) << 8) | (t % nc));
      }
    }
    k_lit = k;
    int n = k;
    if (wv.lane == 0) {
      if (parity) { nid[n] = NEAR; crd[n] = 0; }
      if ((k + parity) & 1) { nid[n + parity] = FAR; crd[n + parity] = 0; }
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
      if (b < a) continue;
      const int ida = nid[a], idb = nid[b];
      if (ida < NEAR && idb < NEAR) {
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
      } else if (ida < NEAR) {
        paint_side(pl, crd[a] >> 8, crd[a] & 255, idb == NEAR ? 0 : 1);
      } else {
        paint_logical(pl);
      }
    }
  }
};

}  // namespace mw
}  // namespace mcmc
