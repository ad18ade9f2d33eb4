// Internal declarations shared by the host tiler, the C-ABI layer and the HIP
// kernels of the FED-FEM library.  Not part of the public ABI.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace fed {

// One tile = one workgroup per step.  A tile owns a contiguous range of
// internal nodes and holds a copy of every element incident to them, so a step
// needs no communication between workgroups besides the ping-pong T buffers.
struct TileHdr {
  int32_t nstart;  // first owned internal node
  int32_t nown;    // owned nodes; the first nbnd carry a boundary record
  int32_t nbnd;
  int32_t bstart;  // index of the tile's first boundary record
  int32_t hstart;  // first entry of the tile's halo list
  int32_t nhalo;   // halo nodes (touched but owned by other tiles)
  int32_t estart;  // first expanded element of the tile
  int32_t ecount;  // expanded elements of the tile
};

struct TilingInput {
  int64_t N = 0, E = 0;
  int ne = 8;
  const double *x = nullptr, *y = nullptr, *z = nullptr;
  const int32_t *conn = nullptr;           // [ne * E], caller node ids
  const int32_t *node_instance = nullptr;  // [N] or null
  const uint8_t *has_bnd = nullptr;        // [N] node carries a surface record
  int target_nodes = 512;                  // owned nodes per tile (upper bound)
  int lds_budget = 64 * 1024;              // bytes of LDS one workgroup may use
  int real_bytes = 4;                      // sizeof(working real)
};

struct Tiling {
  int32_t nt = 0;          // tiles
  int32_t pb = 0;          // bits of the incidence position in an entry
  int32_t maxinc = 0;      // largest node incidence (slots per owned node)
  int32_t ntouch_max = 0;  // largest nown + nhalo over tiles
  int32_t nown_max = 0;
  int32_t lds_bytes = 0;   // dynamic LDS per workgroup
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

}  // namespace fed
