// Work split of the split-Gram kernels (host code): lower-triangle tiles of
// kGramTile x kGramTile times column chunks of whole kGramPanel-wide panels,
// enough chunks for about kGramTargetGroups workgroups per launch.
#include <algorithm>
#include <cstddef>
#include <cstdint>

#include "kernels.hpp"

namespace kpp {

void gram_syrk_plan(int32_t s, int64_t n, int32_t nb, int32_t* nchunks, int64_t* chunk, int32_t* ntiles) {
  const int32_t nt = (s + kGramTile - 1) / kGramTile;
  const int32_t tiles = nt * (nt + 1) / 2;
  const int64_t panels = std::max<int64_t>(1, (n + kGramPanel - 1) / kGramPanel);
  const int64_t base = std::max<int64_t>(1, static_cast<int64_t>(nb) * tiles);
  int64_t c = std::min<int64_t>(panels, std::max<int64_t>(1, kGramTargetGroups / base));
  const int64_t per = ((panels + c - 1) / c) * kGramPanel;  // whole panels per chunk
  c = std::max<int64_t>(1, (n + per - 1) / per);
  *nchunks = static_cast<int32_t>(c);
  *chunk = per;
  *ntiles = tiles;
}

void gram_syrk_plan_capped(int32_t s, int64_t n, int32_t nb, size_t max_work, int32_t* nchunks, int64_t* chunk,
                           int32_t* ntiles) {
  gram_syrk_plan(s, n, nb, nchunks, chunk, ntiles);
  const size_t per_chunk = static_cast<size_t>(std::max(nb, 1)) * *ntiles * kGramTile * kGramTile;
  if (static_cast<size_t>(*nchunks) * per_chunk <= max_work) return;
  const int64_t panels = std::max<int64_t>(1, (n + kGramPanel - 1) / kGramPanel);
  const int64_t c = std::max<int64_t>(1, static_cast<int64_t>(max_work / per_chunk));
  const int64_t per = ((panels + c - 1) / c) * kGramPanel;
  *chunk = per;
  *nchunks = static_cast<int32_t>(std::max<int64_t>(1, (n + per - 1) / per));
}

size_t gram_syrk_work(int32_t s, int64_t n, int32_t nb) {
  int32_t nc, nt;
  int64_t chunk;
  gram_syrk_plan(s, n, nb, &nc, &chunk, &nt);
  return static_cast<size_t>(nb) * nt * nc * kGramTile * kGramTile;
}

}  // namespace kpp
