// Internal declarations shared by the host tiler, the C-ABI layer and the HIP
// kernels of the FED-FEM library.  Not part of the public ABI.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace fed {

constexpr int kMaxDepth = 4;  // most steps one launch may fuse

// One tile = one workgroup per launch.  A tile owns a contiguous range of
// internal nodes.  Nodes get a level: 0 for owned nodes, l for nodes l element
// rings away (up to the tiling depth K).  The tile holds a copy of every
// element touching a node of level < K, so a launch can advance its nodes k <= K
// steps with no communication between workgroups: sub-step s updates the nodes
// of level <= k - s from the elements whose lowest node level is <= k - s.
// Local node order: owned, then halo nodes by (level, id); elements by
// (lowest level, id), so every sub-step works on a prefix of both.
struct TileHdr {
  int32_t nstart;  // first owned internal node
  int32_t nown;    // owned nodes; the first nbnd carry a boundary record
  int32_t nbnd;
  int32_t bstart;  // index of the tile's first boundary record
  int32_t hstart;  // first entry of the tile's halo list
  int32_t nhalo;   // halo nodes (levels 1..K)
  int32_t estart;  // first expanded element of the tile
  int32_t ecount;  // expanded elements of the tile (= cum_e[K-1])
  int32_t nint;    // elements whose nodes are all owned: the first nint of the list
  int32_t cum_n[kMaxDepth + 1];  // local nodes of level <= l
  int32_t cum_e[kMaxDepth];      // elements of lowest level <= l
};

struct TilingInput {
  int64_t N = 0, E = 0;
  int ne = 8;
  const double *x = nullptr, *y = nullptr, *z = nullptr;
  const int32_t *conn = nullptr;           // [ne * E], caller node ids
  const int32_t *node_instance = nullptr;  // [N] or null
  const uint8_t *has_bnd = nullptr;        // [N] node carries a surface record
  int target_nodes = 512;                  // owned nodes per tile (upper bound)
  int depth = 1;                           // K: steps one launch may fuse
  int lds_budget = 64 * 1024;              // bytes of LDS one workgroup may use
  int real_bytes = 4;                      // sizeof(working real)
  int upd_bytes = 0;                       // LDS bytes per updated node besides its slots
  int touch_bytes = 0;                     // LDS bytes per touched node besides its T
};

struct Tiling {
  int32_t nt = 0;          // tiles
  int32_t pb = 0;          // bits of the incidence position in an entry
  int32_t maxinc = 0;      // largest node incidence (slots per owned node)
  int32_t ntouch_max = 0;  // largest nown + nhalo over tiles
  int32_t nown_max = 0;
  int32_t depth = 1;
  int32_t lds_bytes = 0;   // dynamic LDS per workgroup (launches fusing K steps)
  std::vector<int32_t> perm;   // caller node -> internal node
  std::vector<int32_t> iperm;  // internal node -> caller node
  std::vector<TileHdr> tiles;
  std::vector<int32_t> halo;   // internal node ids
  std::vector<uint16_t> ent;   // [E_exp * ne]: (local node << pb) | position
  std::vector<int32_t> eorig;  // [E_exp] caller element id
  std::vector<uint8_t> eowner; // [E_exp] 1 for exactly one copy of every element
  // node -> (element, local node) incidence in internal node order, elements
  // ascending: the canonical summation order of every per-node sum
  std::vector<int64_t> inc_ptr;
  std::vector<int32_t> inc_elem;
  std::vector<int8_t> inc_a;
};

// Builds the tiling; returns an empty string on success, else the reason.
std::string build_tiling(const TilingInput &in, Tiling &out);

// Resident LDS placement (fed_lds_order.cpp): per tile, the position of each
// touched node (local index l -> sigma[t * stride + l]), the tile's touched
// nodes in caller order, and T.ent with those positions in place of the local
// indices.  Positions are a permutation of the tile's touched nodes.  False
// (and nothing to use) when a tile has more touched nodes than an int16 holds.
bool caller_order_positions(const Tiling &T, int ne, std::vector<int16_t> &sigma, int32_t &stride,
                            std::vector<uint16_t> &ent);

}  // namespace fed
