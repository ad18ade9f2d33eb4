// Host-side tiling of a mesh for the owner-computes step kernel.
//
// Nodes are split into compact tiles by recursive coordinate bisection (per
// instance of a batched mesh).  A tile owns a contiguous range of internal node
// ids and carries its own copy of every element incident to an owned node, so
// one workgroup can compute all loads of its nodes from LDS without atomics.
// Each element-node pair is tagged with the node-local position of the element
// in the node's incidence list sorted by element id: the kernel writes the
// element's contribution into that slot and sums slots in position order, so
// every nodal sum runs in ascending element order whatever the tiling.
#include <algorithm>
#include <climits>
#include <cmath>
#include <numeric>

#include "fed_internal.h"

namespace fed {

namespace {

struct Builder {
  const TilingInput &in;
  Tiling &out;
  std::vector<int64_t> cptr;   // caller-order incidence CSR
  std::vector<int32_t> celem;
  std::vector<int8_t> ca;
  std::vector<uint16_t> posEA; // [E * ne] position of e in the list of node conn[a,e]
  int32_t stamp = 0;
  int32_t touch_limit = 0;

  explicit Builder(const TilingInput &i, Tiling &o) : in(i), out(o) {}

  const int32_t &node(int64_t e, int a) const { return in.conn[(int64_t)a * in.E + e]; }

  void incidence() {
    const int64_t N = in.N, E = in.E;
    const int ne = in.ne;
    cptr.assign(N + 1, 0);
    for (int64_t e = 0; e < E; e++)
      for (int a = 0; a < ne; a++) cptr[node(e, a) + 1]++;
    for (int64_t k = 0; k < N; k++) cptr[k + 1] += cptr[k];
    celem.resize(cptr[N]);
    ca.resize(cptr[N]);
    posEA.resize((size_t)E * ne);
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t e = 0; e < E; e++)
      for (int a = 0; a < ne; a++) {
        int32_t k = node(e, a);
        int64_t p = fill[k]++;
        celem[p] = (int32_t)e;
        ca[p] = (int8_t)a;
        posEA[e * ne + a] = (uint16_t)(p - cptr[k]);
      }
    int32_t mx = 0;
    for (int64_t k = 0; k < N; k++) mx = std::max<int32_t>(mx, (int32_t)(cptr[k + 1] - cptr[k]));
    out.maxinc = mx;
    int pb = 1;
    while ((1 << pb) < mx) pb++;
    out.pb = pb;
    touch_limit = 1 << (16 - pb);
  }

  // Levels around the candidate owned set ids[b, e): lev[l] receives the nodes
  // (caller ids) of level l = 1..K, found by growing element rings.
  std::vector<int32_t> lev[kMaxDepth + 1];
  std::vector<int32_t> stamp_lvl;
  void levels(const std::vector<int32_t> &ids, size_t b, size_t e) {
    ++stamp;
    lev[0].assign(ids.begin() + b, ids.begin() + e);
    for (int32_t k : lev[0]) stamp_lvl[k] = stamp;
    for (int l = 1; l <= in.depth; l++) {
      lev[l].clear();
      for (int32_t k : lev[l - 1])
        for (int64_t p = cptr[k]; p < cptr[k + 1]; p++) {
          int32_t el = celem[p];
          for (int a = 0; a < in.ne; a++) {
            int32_t j = node(el, a);
            if (stamp_lvl[j] != stamp) {
              stamp_lvl[j] = stamp;
              lev[l].push_back(j);
            }
          }
        }
    }
  }

  bool fits(const std::vector<int32_t> &ids, size_t b, size_t e) {
    levels(ids, b, e);
    int64_t nupd = 0, ntouch = 0;
    for (int l = 0; l <= in.depth; l++) {
      if (l < in.depth) nupd += (int64_t)lev[l].size();
      ntouch += (int64_t)lev[l].size();
    }
    int64_t lds = ((int64_t)in.real_bytes + in.touch_bytes) * ntouch +
                  ((int64_t)in.upd_bytes + (int64_t)in.real_bytes * out.maxinc) * nupd + 8;
    return ntouch <= touch_limit && lds <= in.lds_budget;
  }

  // Smoothed coordinates (each node moved to the mean centroid of its
  // elements, a few times): on a distorted mesh they take the jitter out of
  // the layers of nodes, so the bisection cuts follow mesh layers and the
  // tiles keep compact boundaries (few halo nodes).  The tiling tries the
  // nodes' own coordinates and these, and keeps the tiles with fewer halo
  // nodes; no result depends on the tiling.
  std::vector<double> sc[3];
  void smooth_coordinates(int iterations) {
    const int64_t N = in.N, E = in.E;
    const int ne = in.ne;
    const double *X[3] = {in.x, in.y, in.z};
    for (int d = 0; d < 3; d++) sc[d].assign(X[d], X[d] + N);
    std::vector<double> cen((size_t)E), acc((size_t)N);
    for (int it = 0; it < iterations; it++)
      for (int d = 0; d < 3; d++) {
        for (int64_t e = 0; e < E; e++) {
          double c = 0;
          for (int a = 0; a < ne; a++) c += sc[d][node(e, a)];
          cen[e] = c / ne;
        }
        for (int64_t k = 0; k < N; k++) {
          double c = 0;
          for (int64_t p = cptr[k]; p < cptr[k + 1]; p++) c += cen[celem[p]];
          acc[k] = cptr[k + 1] > cptr[k] ? c / (double)(cptr[k + 1] - cptr[k]) : sc[d][k];
        }
        sc[d].swap(acc);
      }
  }

  // recursive coordinate bisection of ids[b, e) into leaves (DFS order), by
  // the coordinates X
  bool rcb(std::vector<int32_t> &ids, size_t b0, size_t e0,
           std::vector<std::pair<size_t, size_t>> &leaves, const double *const X[3]) {
    std::vector<std::pair<size_t, size_t>> stack{{b0, e0}};
    while (!stack.empty()) {
      auto [b, e] = stack.back();
      stack.pop_back();
      size_t n = e - b;
      if (n == 0) continue;
      if (n <= (size_t)in.target_nodes && fits(ids, b, e)) {
        leaves.push_back({b, e});
        continue;
      }
      if (n == 1) return false;
      size_t L = std::max<size_t>(2, (n + in.target_nodes - 1) / in.target_nodes);
      size_t nl = std::max<size_t>(1, n * (L / 2) / L);
      double lo[3], hi[3];
      for (int d = 0; d < 3; d++) lo[d] = hi[d] = X[d][ids[b]];
      for (size_t i = b; i < e; i++)
        for (int d = 0; d < 3; d++) {
          lo[d] = std::min(lo[d], X[d][ids[i]]);
          hi[d] = std::max(hi[d], X[d][ids[i]]);
        }
      int ax = 0;
      for (int d = 1; d < 3; d++)
        if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
      const double *c = X[ax];
      std::nth_element(ids.begin() + b, ids.begin() + b + nl, ids.begin() + e,
                       [c](int32_t p, int32_t q) { return c[p] < c[q] || (c[p] == c[q] && p < q); });
      stack.push_back({b + nl, e});
      stack.push_back({b, b + nl});
    }
    return true;
  }

  // halo nodes of a tiling, summed over the tiles: the (tile, node) pairs of
  // nodes another tile owns that share an element with a node of the tile
  int64_t halo_count(const std::vector<int32_t> &ids,
                     const std::vector<std::pair<size_t, size_t>> &leaves) {
    const int64_t N = in.N;
    std::vector<int32_t> tile_of(N, -1), seen;
    for (size_t t = 0; t < leaves.size(); t++)
      for (size_t i = leaves[t].first; i < leaves[t].second; i++) tile_of[ids[i]] = (int32_t)t;
    int64_t h = 0;
    for (int64_t k = 0; k < N; k++) {
      seen.clear();
      for (int64_t p = cptr[k]; p < cptr[k + 1]; p++)
        for (int a = 0; a < in.ne; a++) {
          const int32_t tb = tile_of[node(celem[p], a)];
          if (tb != tile_of[k]) seen.push_back(tb);
        }
      std::sort(seen.begin(), seen.end());
      h += std::unique(seen.begin(), seen.end()) - seen.begin();
    }
    return h;
  }

  std::string run() {
    const int64_t N = in.N, E = in.E;
    const int ne = in.ne;
    incidence();
    stamp_lvl.assign(N, 0);
    // groups: one per instance (caller node order inside), or one group
    std::vector<int32_t> ids(N);
    std::iota(ids.begin(), ids.end(), 0);
    std::vector<size_t> gstart{0};
    if (in.node_instance) {
      std::stable_sort(ids.begin(), ids.end(), [&](int32_t p, int32_t q) {
        return in.node_instance[p] < in.node_instance[q];
      });
      for (int64_t i = 1; i < N; i++)
        if (in.node_instance[ids[i]] != in.node_instance[ids[i - 1]]) gstart.push_back(i);
    }
    gstart.push_back(N);
    // bisect by the nodes' coordinates and by the smoothed ones; keep the
    // tiling with fewer halo nodes (the first on a tie)
    std::vector<std::pair<size_t, size_t>> leaves;
    int64_t best_halo = -1;
    const std::vector<int32_t> ids0 = ids;
    for (int pass = 0; pass < 2; pass++) {
      const double *X[3] = {in.x, in.y, in.z};
      if (pass == 1) {
        smooth_coordinates(5);
        for (int d = 0; d < 3; d++) X[d] = sc[d].data();
      }
      std::vector<int32_t> idp = ids0;
      std::vector<std::pair<size_t, size_t>> lp;
      for (size_t g = 0; g + 1 < gstart.size(); g++)
        if (!rcb(idp, gstart[g], gstart[g + 1], lp, X))
          return "a single node touches more nodes or LDS than one tile can hold "
                 "(node incidence too high)";
      const int64_t h = halo_count(idp, lp);
      if (best_halo < 0 || h < best_halo) {
        best_halo = h;
        ids.swap(idp);
        leaves.swap(lp);
      }
    }
    for (int d = 0; d < 3; d++) std::vector<double>().swap(sc[d]);
    // internal order: tile by tile; inside a tile the boundary-record nodes
    // first, then by the sorted list of other tiles that read the node (nodes
    // no other tile reads last), then caller id, so the nodes a tile exports,
    // and the nodes a neighbour reads from it, sit in few contiguous runs
    out.nt = (int32_t)leaves.size();
    out.tiles.resize(out.nt);
    out.perm.assign(N, -1);
    out.iperm.resize(N);
    std::vector<int32_t> tile_of(N, -1);
    for (int32_t t = 0; t < out.nt; t++)
      for (size_t i = leaves[t].first; i < leaves[t].second; i++) tile_of[ids[i]] = t;
    // readers of node k: rd[rptr[k] .. rptr[k + 1]), ascending ({INT32_MAX} if none)
    std::vector<int64_t> rptr(N + 1, 0);
    std::vector<int32_t> rd, buf;
    for (int64_t k = 0; k < N; k++) {
      buf.clear();
      for (int64_t p = cptr[k]; p < cptr[k + 1]; p++)
        for (int a = 0; a < ne; a++) {
          const int32_t tb = tile_of[node(celem[p], a)];
          if (tb != tile_of[k]) buf.push_back(tb);
        }
      std::sort(buf.begin(), buf.end());
      buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
      if (buf.empty()) buf.push_back(INT32_MAX);
      rd.insert(rd.end(), buf.begin(), buf.end());
      rptr[k + 1] = (int64_t)rd.size();
    }
    int32_t next = 0, bnext = 0;
    for (int32_t t = 0; t < out.nt; t++) {
      auto [b, e] = leaves[t];
      std::sort(ids.begin() + b, ids.begin() + e, [&](int32_t p, int32_t q) {
        bool bp = in.has_bnd && in.has_bnd[p], bq = in.has_bnd && in.has_bnd[q];
        if (bp != bq) return bp;
        const int32_t *r0 = rd.data() + rptr[p], *r1 = rd.data() + rptr[p + 1];
        const int32_t *s0 = rd.data() + rptr[q], *s1 = rd.data() + rptr[q + 1];
        if (std::lexicographical_compare(r0, r1, s0, s1)) return true;
        if (std::lexicographical_compare(s0, s1, r0, r1)) return false;
        return p < q;
      });
      TileHdr &th = out.tiles[t];
      th.nstart = next;
      th.nown = (int32_t)(e - b);
      th.nbnd = 0;
      th.bstart = bnext;
      for (size_t i = b; i < e; i++) {
        int32_t k = ids[i];
        if (in.has_bnd && in.has_bnd[k]) th.nbnd++;
        out.perm[k] = next;
        out.iperm[next] = k;
        next++;
      }
      bnext += th.nbnd;
    }
    // per tile: node levels, elements within K - 1 rings, halo, packed entries
    const int K = in.depth;
    out.depth = K;
    std::vector<int32_t> loc(N, -1), estamp(E, -1), minlev(E, 0), maxlev(E, 0);
    std::vector<int32_t> telems;
    out.halo.clear();
    out.ent.clear();
    out.eorig.clear();
    out.eowner.clear();
    out.ntouch_max = out.nown_max = 0;
    int64_t lds_max = 0;
    for (int32_t t = 0; t < out.nt; t++) {
      TileHdr &th = out.tiles[t];
      std::vector<int32_t> owned(th.nown);
      for (int32_t j = 0; j < th.nown; j++) owned[j] = out.iperm[th.nstart + j];
      levels(owned, 0, owned.size());
      // local ids: owned by internal id, halo by (level, internal id)
      for (int32_t j = 0; j < th.nown; j++) loc[owned[j]] = j;
      int32_t next_loc = th.nown;
      th.hstart = (int32_t)out.halo.size();
      th.cum_n[0] = th.nown;
      for (int l = 1; l <= K; l++) {
        std::vector<int32_t> hl;
        for (int32_t k : lev[l]) hl.push_back(out.perm[k]);
        std::sort(hl.begin(), hl.end());
        for (int32_t ki : hl) {
          loc[out.iperm[ki]] = next_loc++;
          out.halo.push_back(ki);
        }
        th.cum_n[l] = next_loc;
      }
      for (int l = K + 1; l <= kMaxDepth; l++) th.cum_n[l] = next_loc;
      th.nhalo = next_loc - th.nown;
      // elements touching a node of level < K, with their lowest node level
      telems.clear();
      for (int l = 0; l < K; l++)
        for (int32_t k : lev[l])
          for (int64_t p = cptr[k]; p < cptr[k + 1]; p++) {
            int32_t el = celem[p];
            if (estamp[el] != t) {
              estamp[el] = t;
              telems.push_back(el);
            }
          }
      // sorted by lowest node level (a K-step launch drops the outer levels
      // step by step), then elements with every node owned first (they need no
      // halo value, so a resident step can run them while it waits for the
      // halo), then id; the order changes no result: every nodal sum runs over
      // the node's elements in ascending element id
      th.nint = 0;
      for (int32_t el : telems) {
        int32_t m = kMaxDepth + 1, mx = 0;
        for (int a = 0; a < ne; a++) {
          int32_t lc = loc[node(el, a)];
          int32_t lv = 0;
          while (lc >= th.cum_n[lv]) lv++;
          m = std::min(m, lv);
          mx = std::max(mx, lv);
        }
        minlev[el] = m;
        maxlev[el] = mx;
        th.nint += mx == 0;
      }
      std::sort(telems.begin(), telems.end(), [&](int32_t p, int32_t q) {
        if (minlev[p] != minlev[q]) return minlev[p] < minlev[q];
        if ((maxlev[p] == 0) != (maxlev[q] == 0)) return maxlev[p] == 0;
        return p < q;
      });
      th.estart = (int32_t)out.eorig.size();
      th.ecount = (int32_t)telems.size();
      for (int l = 0; l < kMaxDepth; l++) {
        int32_t c = 0;
        for (int32_t el : telems) c += minlev[el] <= l;
        th.cum_e[l] = l < K ? c : th.ecount;
      }
      for (int32_t el : telems) {
        out.eorig.push_back(el);
        int32_t k0 = out.perm[node(el, 0)];
        out.eowner.push_back(k0 >= th.nstart && k0 < th.nstart + th.nown ? 1 : 0);
        for (int a = 0; a < ne; a++) {
          int32_t l = loc[node(el, a)];
          out.ent.push_back((uint16_t)(((uint32_t)l << out.pb) | posEA[(size_t)el * ne + a]));
        }
      }
      int32_t ntouch = th.cum_n[K], nupd = th.cum_n[K - 1];
      out.ntouch_max = std::max(out.ntouch_max, ntouch);
      out.nown_max = std::max(out.nown_max, th.nown);
      lds_max = std::max<int64_t>(lds_max, ((int64_t)in.real_bytes + in.touch_bytes) * ntouch +
                                               ((int64_t)in.upd_bytes + (int64_t)in.real_bytes *
                                                out.maxinc) * nupd + 8);
      if (ntouch > touch_limit) return "internal: tile exceeds the local index range";
    }
    out.lds_bytes = (int32_t)lds_max;
    // incidence in internal node order
    out.inc_ptr.assign(N + 1, 0);
    out.inc_elem.resize(cptr[N]);
    out.inc_a.resize(cptr[N]);
    for (int64_t ki = 0; ki < N; ki++) {
      int32_t k = out.iperm[ki];
      int64_t cnt = cptr[k + 1] - cptr[k];
      out.inc_ptr[ki + 1] = out.inc_ptr[ki] + cnt;
      std::copy(celem.begin() + cptr[k], celem.begin() + cptr[k + 1],
                out.inc_elem.begin() + out.inc_ptr[ki]);
      std::copy(ca.begin() + cptr[k], ca.begin() + cptr[k + 1],
                out.inc_a.begin() + out.inc_ptr[ki]);
    }
    (void)E;
    return "";
  }
};

}  // namespace

std::string build_tiling(const TilingInput &in, Tiling &out) {
  if (in.N <= 0 || in.E <= 0) return "empty mesh";
  if (in.target_nodes < 1) return "tile_nodes must be positive";
  if (in.depth < 1 || in.depth > kMaxDepth) return "fused steps out of range";
  Builder b(in, out);
  return b.run();
}

}  // namespace fed
