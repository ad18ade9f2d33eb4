// Host-side invariant checker of the tiler (built with g++ and sanitizers by
// tests/test_host_tiling.py; no HIP).  Usage:
//   tiling_check <hex|tet> nx ny nz target [ninst] [depth]
// Builds a structured box (or ninst disjoint copies), tiles it and checks that
// every packed entry decodes to its node, that every owned node's slot
// positions are 0..count-1 in ascending element order, that each element has
// exactly one owner copy, the node levels (checked against a separate
// breadth-first search), that every sub-step of a k-step launch finds all
// elements of the nodes it updates in its element prefix, and the size limits.
// Prints "OK <tiles>" or fails.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <set>
#include <vector>

#include "../paper_1909_03355_amd/csrc/fed_internal.h"

#define REQUIRE(c)                                                   \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      return 1;                                                      \
    }                                                                \
  } while (0)

int main(int argc, char **argv) {
  if (argc < 6) return 2;
  bool hex = std::strcmp(argv[1], "hex") == 0;
  int nx = std::atoi(argv[2]), ny = std::atoi(argv[3]), nz = std::atoi(argv[4]);
  int target = std::atoi(argv[5]);
  int ninst = argc > 6 ? std::atoi(argv[6]) : 1;
  int depth = argc > 7 ? std::atoi(argv[7]) : 1;
  const int ne = hex ? 8 : 4;
  auto nid = [&](int i, int j, int k) { return i + (nx + 1) * (j + (ny + 1) * k); };
  const int np1 = (nx + 1) * (ny + 1) * (nz + 1);
  std::vector<double> x, y, z;
  std::vector<std::vector<int>> elems;
  std::vector<int32_t> inst;
  static const int S[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                              {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
  static const int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (int c = 0; c < ninst; c++) {
    int base = c * np1;
    for (int k = 0; k <= nz; k++)
      for (int j = 0; j <= ny; j++)
        for (int i = 0; i <= nx; i++) {
          x.push_back(i + 3.0 * c * nx);
          y.push_back(j);
          z.push_back(k);
          inst.push_back(c);
        }
    for (int k = 0; k < nz; k++)
      for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
          if (hex) {
            std::vector<int> e;
            for (auto &s : S) e.push_back(base + nid(i + s[0], j + s[1], k + s[2]));
            elems.push_back(e);
          } else {
            for (auto &p : P) {
              int o[3] = {0, 0, 0};
              std::vector<int> e{base + nid(i, j, k)};
              for (int ax : p) {
                o[ax]++;
                e.push_back(base + nid(i + o[0], j + o[1], k + o[2]));
              }
              elems.push_back(e);
            }
          }
        }
  }
  const int64_t N = (int64_t)x.size(), E = (int64_t)elems.size();
  std::vector<int32_t> conn(ne * E);
  for (int64_t e = 0; e < E; e++)
    for (int a = 0; a < ne; a++) conn[a * E + e] = elems[e][a];
  std::vector<uint8_t> has_bnd(N, 0);
  for (int64_t k = 0; k < N; k += 7) has_bnd[k] = 1;
  fed::TilingInput in;
  in.N = N;
  in.E = E;
  in.ne = ne;
  in.x = x.data();
  in.y = y.data();
  in.z = z.data();
  in.conn = conn.data();
  in.node_instance = ninst > 1 ? inst.data() : nullptr;
  in.has_bnd = has_bnd.data();
  in.target_nodes = target;
  in.depth = depth;
  in.upd_bytes = 16;
  fed::Tiling T;
  std::string err = fed::build_tiling(in, T);
  if (!err.empty()) {
    std::fprintf(stderr, "tiling error: %s\n", err.c_str());
    return 1;
  }
  // permutation and contiguous tiles
  std::vector<int> seen(N, 0);
  for (int64_t k = 0; k < N; k++) {
    REQUIRE(T.perm[k] >= 0 && T.perm[k] < N);
    REQUIRE(T.iperm[T.perm[k]] == k);
    seen[T.perm[k]]++;
  }
  for (int64_t k = 0; k < N; k++) REQUIRE(seen[k] == 1);
  int32_t next = 0, bnext = 0;
  const uint32_t limit = 1u << (16 - T.pb);
  std::vector<int> owners(E, 0);
  for (int t = 0; t < T.nt; t++) {
    const fed::TileHdr &th = T.tiles[t];
    REQUIRE(th.nstart == next && th.nown > 0 && th.nown <= target);
    REQUIRE(th.bstart == bnext);
    next += th.nown;
    bnext += th.nbnd;
    for (int j = 0; j < th.nown; j++) {
      int32_t k = T.iperm[th.nstart + j];
      REQUIRE((j < th.nbnd) == (has_bnd[k] != 0));
      if (ninst > 1) REQUIRE(inst[k] == inst[T.iperm[th.nstart]]);
    }
    const int K = depth;
    REQUIRE(th.cum_n[0] == th.nown && th.cum_n[K] == th.nown + th.nhalo);
    REQUIRE((uint32_t)(th.nown + th.nhalo) <= limit);
    REQUIRE(4LL * th.cum_n[K] + (16LL + 4LL * T.maxinc) * th.cum_n[K - 1] + 8 <= T.lds_bytes);
    // independent BFS levels from the owned set (internal ids), capped at K
    std::vector<int> lvl(N, -1);
    std::vector<int32_t> front, nxt;
    for (int j = 0; j < th.nown; j++) {
      lvl[th.nstart + j] = 0;
      front.push_back(th.nstart + j);
    }
    for (int l = 1; l <= K; l++) {
      nxt.clear();
      for (int32_t ki : front)
        for (int64_t p = T.inc_ptr[ki]; p < T.inc_ptr[ki + 1]; p++) {
          int32_t e = T.inc_elem[p];
          for (int a = 0; a < ne; a++) {
            int32_t kj = T.perm[conn[a * E + e]];
            if (lvl[kj] < 0) {
              lvl[kj] = l;
              nxt.push_back(kj);
            }
          }
        }
      front.swap(nxt);
    }
    auto local_level = [&](int32_t lc) {
      int l = 0;
      while (lc >= th.cum_n[l]) l++;
      return l;
    };
    int64_t nlev = 0;
    for (int64_t ki = 0; ki < N; ki++) nlev += lvl[ki] >= 0;
    REQUIRE(nlev == th.cum_n[K]);
    for (int h = 0; h < th.nhalo; h++) {
      int32_t ki = T.halo[th.hstart + h];
      REQUIRE(lvl[ki] == local_level(th.nown + h));
      if (h && local_level(th.nown + h) == local_level(th.nown + h - 1))
        REQUIRE(ki > T.halo[th.hstart + h - 1]);
    }
    // expected element set: elements touching a node of level < K
    std::set<int32_t> want;
    for (int64_t ki = 0; ki < N; ki++)
      if (lvl[ki] >= 0 && lvl[ki] < K)
        for (int64_t p = T.inc_ptr[ki]; p < T.inc_ptr[ki + 1]; p++) want.insert(T.inc_elem[p]);
    REQUIRE((int)want.size() == th.ecount && th.cum_e[K - 1] == th.ecount);
    std::vector<std::vector<std::pair<int32_t, int>>> got(th.cum_n[K - 1]);  // (elem, pos)
    // order: lowest node level, then all nodes owned first, then id; the
    // first nint elements are exactly those with every node owned
    int prevlev = 0, prevout = 0;
    int32_t prev = -1;
    for (int i = 0; i < th.ecount; i++) {
      int64_t ie = th.estart + i;
      int32_t e = T.eorig[ie];
      REQUIRE(want.count(e));
      int ml = 99, mx = 0;
      for (int a = 0; a < ne; a++) {
        ml = std::min(ml, lvl[T.perm[conn[a * E + e]]]);
        mx = std::max(mx, lvl[T.perm[conn[a * E + e]]]);
      }
      const int out = mx > 0;
      REQUIRE(ml >= prevlev);
      if (ml == prevlev) REQUIRE(out >= prevout && (out > prevout || e > prev));
      REQUIRE((i < th.nint) == (mx == 0));
      for (int l = 0; l < K; l++) REQUIRE((i < th.cum_e[l]) == (ml <= l));
      prevlev = ml;
      prevout = out;
      prev = e;
      owners[e] += T.eowner[ie];
      for (int a = 0; a < ne; a++) {
        uint32_t v = T.ent[ie * ne + a];
        uint32_t loc = v >> T.pb, pos = v & ((1u << T.pb) - 1);
        REQUIRE(loc < (uint32_t)(th.nown + th.nhalo));
        int32_t ki = loc < (uint32_t)th.nown ? th.nstart + loc : T.halo[th.hstart + loc - th.nown];
        REQUIRE(ki == T.perm[conn[a * E + e]]);
        if (loc < (uint32_t)th.cum_n[K - 1]) {
          REQUIRE((int)pos < T.maxinc);
          got[loc].push_back({e, (int)pos});
        }
      }
    }
    // every updated node sees its full incidence, in ascending element order, and
    // in a k-step launch sub-step s finds it within the prefix cum_e[k - s]
    for (int32_t lc = 0; lc < th.cum_n[K - 1]; lc++) {
      int32_t ki = lc < th.nown ? th.nstart + lc : T.halo[th.hstart + lc - th.nown];
      int64_t cnt = T.inc_ptr[ki + 1] - T.inc_ptr[ki];
      std::vector<std::pair<int32_t, int>> g = got[lc];
      std::sort(g.begin(), g.end());
      REQUIRE((int64_t)g.size() == cnt);
      for (size_t q = 0; q < g.size(); q++) {
        REQUIRE(g[q].second == (int)q);
        REQUIRE(g[q].first == T.inc_elem[T.inc_ptr[ki] + q]);
      }
      int l = local_level(lc);
      for (int i = 0; i < th.ecount; i++) {
        int32_t e = T.eorig[th.estart + i];
        bool touches = false;
        for (int a = 0; a < ne; a++) touches |= T.perm[conn[a * E + e]] == ki;
        if (touches) REQUIRE(i < th.cum_e[l]);
      }
    }
  }
  REQUIRE(next == N);
  for (int64_t e = 0; e < E; e++) REQUIRE(owners[e] == 1);
  // tiles whose first halo ring holds a node of tile u: the relation the
  // resident step's neighbour waits are built from must be symmetric
  std::vector<int32_t> owner_of(N);
  for (int t = 0; t < T.nt; t++)
    for (int j = 0; j < T.tiles[t].nown; j++) owner_of[T.tiles[t].nstart + j] = t;
  std::set<std::pair<int32_t, int32_t>> rel;
  for (int t = 0; t < T.nt; t++) {
    const fed::TileHdr &th = T.tiles[t];
    for (int h = 0; h < th.cum_n[1] - th.nown; h++) {
      const int32_t u = owner_of[T.halo[th.hstart + h]];
      REQUIRE(u != t);
      rel.insert({t, u});
    }
  }
  for (const auto &pr : rel) REQUIRE(rel.count({pr.second, pr.first}));
  // inside a tile's boundary-record and other nodes, the nodes another tile
  // reads (in some first halo ring) come first, grouped by the sorted list
  // of their readers
  std::vector<std::vector<int32_t>> readers(N);
  for (int t = 0; t < T.nt; t++) {
    const fed::TileHdr &th = T.tiles[t];
    for (int h = 0; h < th.cum_n[1] - th.nown; h++) readers[T.halo[th.hstart + h]].push_back(t);
  }
  for (auto &v : readers) std::sort(v.begin(), v.end());
  for (int t = 0; t < T.nt; t++) {
    const fed::TileHdr &th = T.tiles[t];
    for (int j = 1; j < th.nown; j++) {
      if (j == th.nbnd) continue;  // a new group starts
      const auto &a = readers[th.nstart + j - 1], &b = readers[th.nstart + j];
      if (a.empty()) REQUIRE(b.empty());
      if (!a.empty() && !b.empty()) REQUIRE(!(b < a));
    }
  }
  // resident LDS placement: per tile a permutation of the touched nodes in
  // caller order, and entries that carry it
  {
    std::vector<int16_t> sigma;
    std::vector<uint16_t> ent2;
    int32_t stride = 0;
    REQUIRE(fed::caller_order_positions(T, ne, sigma, stride, ent2));
    REQUIRE(ent2.size() == T.ent.size());
    for (int t = 0; t < T.nt; t++) {
      const fed::TileHdr &th = T.tiles[t];
      const int nt = th.cum_n[T.depth];
      REQUIRE(nt <= stride);
      const int16_t *sg = sigma.data() + (size_t)t * stride;
      std::vector<int> at(nt, -1);
      for (int l = 0; l < nt; l++) {
        REQUIRE(sg[l] >= 0 && sg[l] < nt);
        REQUIRE(at[sg[l]] < 0);
        at[sg[l]] = l;
      }
      auto caller = [&](int l) {
        return T.iperm[l < th.nown ? th.nstart + l : T.halo[th.hstart + l - th.nown]];
      };
      for (int r = 1; r < nt; r++) REQUIRE(caller(at[r - 1]) < caller(at[r]));
      for (int64_t i = (int64_t)th.estart * ne; i < (int64_t)(th.estart + th.ecount) * ne; i++) {
        const uint32_t w = T.ent[i], w2 = ent2[i];
        REQUIRE((w2 >> T.pb) == (uint32_t)sg[w >> T.pb]);
        REQUIRE((w2 & ((1u << T.pb) - 1u)) == (w & ((1u << T.pb) - 1u)));
      }
    }
  }
  std::printf("OK %d tiles, %zu expanded elements, maxinc %d, pb %d\n", T.nt, T.eorig.size(),
              T.maxinc, T.pb);
  return 0;
}
