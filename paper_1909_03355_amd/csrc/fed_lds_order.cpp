// Host-side LDS placement of a tile's touched nodes for the resident step.
//
// The resident kernel keeps each touched node's temperature and its element
// slots in LDS.  By default a node sits at its local index (owned nodes, then
// halo nodes, in the tiler's order, which groups them by the tiles that read
// them).  For FP32 hexahedra the library places them in caller node order
// instead, the order of the tile's elements, so a wave's element gathers and
// scatters touch fewer LDS banks more than once.  The placement changes no
// result: every nodal sum still runs over its slots in position order.
#include <algorithm>
#include <cstdint>
#include <utility>

#include "fed_internal.h"

namespace fed {

bool caller_order_positions(const Tiling &T, int ne, std::vector<int16_t> &sigma, int32_t &stride,
                            std::vector<uint16_t> &ent) {
  stride = 1;
  for (const TileHdr &th : T.tiles) stride = std::max(stride, th.cum_n[T.depth]);
  if (stride > INT16_MAX + 1) return false;  // positions must fit an int16
  sigma.assign((size_t)T.nt * stride, 0);
  std::vector<std::pair<int32_t, int32_t>> key;
  for (int32_t t = 0; t < T.nt; t++) {
    const TileHdr &th = T.tiles[t];
    const int32_t nt = th.cum_n[T.depth];
    key.clear();
    for (int32_t l = 0; l < nt; l++) {
      const int32_t ki = l < th.nown ? th.nstart + l : T.halo[th.hstart + l - th.nown];
      key.emplace_back(T.iperm[ki], l);
    }
    std::sort(key.begin(), key.end());
    int16_t *sg = sigma.data() + (size_t)t * stride;
    for (int32_t r = 0; r < nt; r++) sg[key[r].second] = (int16_t)r;
  }
  // the packed entries with the positions in place of the local indices
  ent = T.ent;
  const uint32_t pm = (1u << T.pb) - 1u;
  for (int32_t t = 0; t < T.nt; t++) {
    const TileHdr &th = T.tiles[t];
    const int16_t *sg = sigma.data() + (size_t)t * stride;
    for (int64_t i = (int64_t)th.estart * ne; i < (int64_t)(th.estart + th.ecount) * ne; i++) {
      const uint32_t w = ent[i];
      ent[i] = (uint16_t)(((uint32_t)sg[w >> T.pb] << T.pb) | (w & pm));
    }
  }
  return true;
}

}  // namespace fed
